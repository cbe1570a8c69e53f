// Internal declarations shared by the host runtime (bfs_host.cpp) and the
// gfx950 kernels (bfs_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfsi {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64s)
constexpr uint32_t kAllVertices = 0xFFFFFFFFu;
constexpr int kRing = 4;               // per-level counter slots (level k uses k & 3)
constexpr int kBarGroups = 16;         // arrival groups of the persistent kernel's grid barrier
constexpr int kMlpIn = 12, kMlpH = 32, kMlpOut = 3;
constexpr int kMlpParams = kMlpIn * kMlpH + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH * kMlpOut + kMlpOut;
// feature normalisation constants live after the weights: mean[12], inv_std[12]
constexpr int kMlpTotal = kMlpParams + 2 * kMlpIn;

enum Variant : uint32_t { kPush = 0, kPull = 1, kBitmap = 2, kLearned = 3, kHeuristic = 4, kShortCircuit = 5 };

// Device-resident search state (first bytes of every workspace).
struct alignas(256) BfsState {
    uint32_t level;          // current level k
    uint32_t variant;        // variant run at level k
    uint32_t u_buf;          // which unvisited-list buffer is current
    uint32_t u_len;          // its length; kAllVertices = the implicit list 0..n-1
    uint32_t u_wr;           // appends into the other buffer during a pull level
    uint32_t visited_cnt;    // |B_k|
    unsigned long long visited_deg;   // sum of out-degrees over B_k
    uint32_t nf[kRing];                  // |F| (short columns, in the list) per ring slot
    unsigned long long heavy[kRing];     // long columns: (#columns) | (#chunks << 32)
    unsigned long long sdf[kRing];       // sum of out-degrees over F per ring slot
    uint32_t barrier_gen;
    uint32_t pad[7];
    // arrivals at the end of a level (every level launch, and the persistent
    // kernel's grid barrier): one counter per group of blocks, each on its own
    // 64-byte line, then one for the groups
    uint32_t bar_group[kBarGroups * 16];
    uint32_t bar_top;
    uint32_t pad2[15];
    // per-group release generations (one line each): the top release is
    // watched by the groups' last arrivals only, everyone else watches its group
    uint32_t bar_gen_group[kBarGroups * 16];
    unsigned long long atomics;          // parent atomicMin operations issued (when counted)
};
// Per-level record kept on the device (a trace ring of kTraceCap entries).
struct DevLevelRec {
    uint32_t level, variant, nf, nu;
    unsigned long long sdf, sdu;
};
constexpr uint32_t kTraceCap = 1024;

struct HeavyItem {
    int32_t v;
    uint32_t chunk_base;
};

// A frontier-list entry: the vertex and its column bounds, written by the
// lane that reached it, so the next level reads them sequentially.
struct alignas(16) QEnt {
    int32_t v, r0, r1, pad;
};

struct LevelParams {
    int32_t n;
    uint32_t nnz;
    uint32_t words;          // 32-bit words per bitmap
    uint32_t policy;         // Variant requested
    uint32_t heavy_min;      // out-degree from which a column goes to the chunk queue
    uint32_t chunk;          // entries per chunk
    const int32_t *out_ptr, *out_idx, *in_ptr, *in_idx;
    int32_t *level;
    uint32_t *parent;        // uint32 view of the int32 parent array (-1 = 0xFFFFFFFF)
    uint32_t *vb[2];         // visited bitmaps, ping-pong: vb[k&1] = B_k
    uint32_t *fb[3];         // frontier bitmaps, rotating: fb[k%3] = F_k (kept only when maintain_fb)
    QEnt *q[2];              // frontier lists of short columns, ping-pong
    int32_t *ul[2];          // unvisited lists, ping-pong
    HeavyItem *hl[2];        // frontier lists of long (chunked) columns, ping-pong
    uint32_t *cmap[2];       // chunk id -> position of its column in hl, ping-pong
    BfsState *st;
    DevLevelRec *trace;      // kTraceCap records, or nullptr
    const float *mlp;        // selector weights (kMlpTotal floats) or nullptr
    uint32_t *host_status;   // pinned host memory: [0] level, [1] its frontier size
    uint32_t maintain_fb;
    uint32_t stats;
    unsigned long long *atomics;   // count the push's parent atomicMin operations here, or nullptr
    uint32_t no_preread;           // 1: every unmasked pair issues its atomicMin (no pre-read)
};

struct WsLayout {
    size_t state, vb0, vb1, fb0, fb1, fb2, q0, q1, u0, u1, h0, h1, c0, c1, trace, total;
};
WsLayout ws_layout(int32_t n, uint32_t nnz, uint32_t heavy_min_floor);

// ---------------------------------------------------------------------------
// Sliced push (bfs_slice.hip): the push form with the row mask in LDS.
//
// The visited bitmap is cut into S <= kSlMaxSlices slices of sw words
// (<= 128 KiB each).  Workgroup b keeps slice s(b) of B_k in LDS for the whole
// level and expands only the part of each frontier column whose rows fall in
// that slice: the graph stores, per vertex, where each slice starts in its
// sorted out-list.  A reached row is claimed by an OR into the LDS slice; the
// rows claimed by a workgroup are OR-ed into the level's claim bitmap C_{k+1}
// at the end.  The frontier of level k is C_k itself (a bitmap), and a vertex
// of C_k receives its level and parent while level k runs: its parent is the
// first in-neighbour, in ascending order, that lies in C_{k-1}.
// ---------------------------------------------------------------------------
constexpr int kSlThreads = 1024;                // threads per workgroup (16 wave64s)
constexpr int kSlWaves = kSlThreads / 64;
constexpr uint32_t kSlMaxSliceWords = 32768;    // 128 KiB of bitmap in LDS
constexpr uint32_t kSlMaxSlices = 4;            // n <= 4 * 2^20 vertices
constexpr uint32_t kSlLong = 1024;              // a column's slice part this long or longer is chunked
constexpr uint32_t kSlChunk = 1024;             // entries per chunk of such a part
constexpr uint32_t kSlBatch = 128;              // ranges a wave expands together (2 per lane)

// One chunk of a long slice part of a column: out_idx[a, e) of vertex v.
struct alignas(16) SlChunk {
    int32_t v, a, e, pad;
};

struct alignas(256) SlState {
    uint32_t level;                          // current level k
    uint32_t pad0[3];
    uint32_t nclaim[kRing];                  // claim bits the level that built C_k found
                                             // (>= |C_k| since workgroups overlap; 0 iff empty)
    uint32_t nf[kRing];                      // |F_k|, counted as F_k is settled
    unsigned long long sdf[kRing];           // sum of out-degrees over F_k
    uint32_t visited_cnt;                    // |B_k| after level k closes
    uint32_t pad1;
    unsigned long long visited_deg;
    uint32_t pad2[8];
    // the running level's sums, one 64-byte line per group of workgroups:
    // acc[8 g] = claim bits | (settled vertices << 32), acc[8 g + 1] = their degree sum
    unsigned long long acc[kBarGroups * 8];
    uint32_t bar_group[kBarGroups * 16];     // arrivals at the end of a level launch
    uint32_t bar_top;
    uint32_t pad3[15];
};

struct SlParams {
    int32_t n;
    uint32_t nnz;
    uint32_t S;                      // slices
    uint32_t sw;                     // 32-bit words per slice (a multiple of 4)
    uint32_t words;                  // S * sw: words of every bitmap (padded)
    uint32_t streams;                // workgroups per slice
    const int4 *seg;                 // [n + 1]: {out_ptr[v], start of slices 1, 2, 3 in v's out-list}
    const uint32_t *occ;             // [S][words]: bit v of slice s = v's part in slice s is short and
                                     // not empty (the frontier loop's work there)
    const int4 *out_idx4;            // out_idx as 16-byte quads (padded to a multiple of 4 entries)
    const int32_t *in_ptr, *in_idx;  // in-lists (undirected: the out-lists)
    const SlChunk *chunks;           // chunk records, slice s at [chunk_off[s], chunk_off[s + 1])
    uint32_t chunk_off[kSlMaxSlices + 1];
    int32_t *level;
    int32_t *parent;
    uint32_t *vb[2];                 // visited bitmaps: level k reads B_{k-1} = vb[(k+1)&1], writes B_k = vb[k&1]
    uint32_t *cb[4];                 // claim bitmaps: C_k = cb[k&3]
    SlState *st;
    DevLevelRec *trace;              // kTraceCap records, or nullptr
    uint32_t *host_status;           // pinned host: [0] level, [1] claim count of that level (0 = done)
};

struct SlLayout {
    size_t state, vb0, vb1, c0, c1, c2, c3, trace, total;
};
SlLayout sl_layout(uint32_t words);
// The file-scope scratch array behind bfs_run_static (bfs_static.hip): its
// size, and this device's address of it (looked up on the device's first call).
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
hipError_t static_scratch(void **out);

hipError_t launch_sl_init(const SlParams &p, int32_t nroots, const int32_t *roots_dev,
                          int32_t single_root, hipStream_t s);
hipError_t launch_sl_level(const SlParams &p, uint32_t grid, hipStream_t s);

// Multi-source search (64 sources per 64-bit word per vertex).
constexpr uint32_t kMsLong = 512;      // degree from which a multi-source list entry is split
constexpr uint32_t kMsChunk = 512;     // entries per chunk of a split entry
constexpr uint32_t kMsRows = 512;      // most rows per chunk of the multi-source pull's row phase

// A split entry of a multi-source work list: the vertex and the id of its
// first chunk (chunks of one list are numbered consecutively in entry order).
struct MsLong {
    int32_t v;
    uint32_t chunk_base;
};

struct MsLevel {
    int32_t n;
    uint32_t W;                    // 64-bit words per vertex mask = ceil(nq / 64)
    uint32_t nq;                   // number of sources
    const int32_t *out_ptr, *out_idx, *in_ptr, *in_idx;
    unsigned long long *vis;       // [n][W]: sources that reached v through level k
    unsigned long long *m[3];      // [n][W] rotating: level-k frontier masks in m[k % 3]
    int32_t *fq[3];                // rotating lists of vertices with a nonzero frontier mask
    uint32_t *flag;                // [n]: last level (+1) a vertex was listed for
    uint32_t *cnt;                 // list sizes per slot
    // the graph's split entries (fixed per graph, built at creation): columns
    // with out-degree >= kMsLong (the push form's chunks) and rows with
    // in-degree >= kMsLong (the settle and pull chunks); chunk id -> entry
    const MsLong *lo, *li;
    const uint32_t *lomap, *limap;
    uint32_t nlo_chunks, nli, nli_chunks;
    const uint32_t *lirest;        // the long rows' chunks but their first, by position in the row, then row
    // the graph's degree-ordered copy (all null: the caller's order): the lists
    // above then hold search labels, orig maps a label to the caller's id, pos
    // the caller's id to its label, ent[e] is the caller's id of entry e; the
    // masks, vis, flags and lists use labels, the staged results and every
    // parent value the caller's ids
    const int32_t *orig, *pos, *ent, *out_ent;   // ent: in-list entries, out_ent: out-list entries
    // the pull's row chunks: row_chunks[c] .. row_chunks[c + 1] - 1, at most
    // kMsRows rows each (null: chunks of kMsRows consecutive rows)
    const int32_t *row_chunks;
    uint32_t nrow_chunks;
    uint32_t stage_labels;         // staged rows by label (the library's own staging with a degree order)
    // results staged vertex-major while the search runs, [n][W * 64]: row v
    // holds every source's level / parent of v (valid where vis has the bit),
    // so the writes of one row share its 256-byte lines; k_ms_out transposes
    // them into the callers' per-source arrays at the end (with stage_labels
    // the row of a vertex is its label, else its caller id; parents are
    // caller ids either way)
    int32_t *slev;
    uint32_t *spar;
    int32_t *const *level;         // device array of nq device pointers
    int32_t *const *parent;
    const int32_t *sources;        // device, nq
    uint32_t *host_status;         // pinned host: [0] level, [1] next frontier size
    uint32_t fill_levels;          // slev / spar are the caller's vertex-major outputs:
                                   // every level starts at -1 (no transpose at the end)
    // union-frontier bitmap of the level a pull runs on (bit v = some source
    // has v in its frontier), [ceil(n / 64)] words, built by k_ms_fbits when
    // use_fbits is set: the pull tests it before gathering a frontier mask
    unsigned long long *fbits;
    uint32_t use_fbits;
    uint32_t wide_steps;           // push: 64 frontier columns per wave step always
                                   // (average degree below 8), else sized to the list
    uint32_t long_split;           // pull: long rows' first chunks, then the later ones
                                   // in a second launch (k_ms_pull_rest)
    // level statistics for the learned direction (layout below), accumulated
    // as each level's list is settled or reported
    unsigned long long *mstat;
    const float *mlp;              // selector weights for the learned direction, or nullptr
    // range-ordered pull (dense levels, one mask word): the rows still open
    // after a pass (two lists, pass r writes list r & 1), their counts (pass
    // r appends to rcnt[r % 3]) and each open row's next in-list entry
    int32_t *rlist[2];
    uint32_t *rcnt;
    int32_t *rcur;
    uint32_t rp_ranges;            // vertex ranges of the pass order (1 = not used)
};

// Layout of mstat: 64-byte group lines ms_line(t, g) for g < kMsDegGroups
// (the blocks' atomics spread over 16 lines).  Slots t < 3 hold the list of
// level k with t = k % 3: word 0 = the out-degree sum of that union frontier,
// word 1 = the (vertex, source) pairs it newly reaches (the popcount of its
// masks).  Slot 3 holds the running totals through the last list built: word 0
// = the summed union-frontier sizes, word 1 = the pairs reached.
constexpr int kMsDegGroups = 16;
constexpr int kMsCumSlot = 3;
constexpr int kMsStatWords = 4 * kMsDegGroups * 8;
__host__ __device__ constexpr int ms_line(int t, int g) { return (t * kMsDegGroups + g) * 8; }

struct MsLayout {
    size_t vis, m0, m1, m2, f0, f1, f2, flag, cnt, mstat, fbits, rl0, rl1, rcnt, rcur, slev, spar, lptr, pptr,
        src, total;
};
// staged = false: the results go straight to the caller's vertex-major
// arrays, so the layout holds no staging (slev / spar are 0)
MsLayout ms_layout(int32_t n, int32_t nq, bool staged = true);

// launches (bfs_kernels.hip)
hipError_t launch_init(const LevelParams &p, int32_t nroots, const int32_t *roots_dev,
                       int32_t single_root, hipStream_t s);
hipError_t launch_level(const LevelParams &p, uint32_t grid, hipStream_t s);
hipError_t launch_parents(const LevelParams &p, uint32_t grid, hipStream_t s);
hipError_t launch_persistent(const LevelParams &p, uint32_t grid, hipStream_t s);
uint32_t persistent_max_grid(int device);

hipError_t launch_ms(const MsLevel &p, int phase, uint32_t k, uint32_t grid, hipStream_t s);
hipError_t launch_ms_rpull(const MsLevel &p, uint32_t k, uint32_t r, uint32_t grid, hipStream_t s);

// ---------------------------------------------------------------------------
// The claim-word push (bfs_claim.hip).  Every vertex of every query holds one
// 64-bit word, (level << 32) | parent, ~0 while unreached; frontier vertex u of
// level k offers ((k + 1) << 32) | u to each out-neighbour by atomicMin, so
// one atomic both masks the visited rows (their words are smaller) and
// selects the smallest frontier in-neighbour; the atomic that finds ~0 lists
// the vertex for the next level.  Several queries (on different graphs) run
// together in one virtual vertex space: query q owns ids [base_q, base_q + n_q).
// ---------------------------------------------------------------------------
constexpr int kCwBlock = 256;                 // threads per workgroup of the wide level
constexpr int kCwNarrowThreads = 1024;        // the narrow kernel's one workgroup
constexpr uint32_t kCwCap = 8192;             // narrow: frontier entries held in LDS
constexpr uint32_t kCwPer = kCwCap / kCwNarrowThreads;
constexpr uint32_t kCwLongCap = 2048;         // narrow: entries with more than 4 out-edges
constexpr uint32_t kCwNarrowEdges = 1u << 16; // narrow: out-edges of a level at most
constexpr uint32_t kCwLong = 256;             // wide: a column this long is split into chunks
constexpr uint32_t kCwChunk = 1024;           // wide: entries per chunk
constexpr uint32_t kCwPrecheck = 1u << 16;    // wide: frontier entries from which a word is read first
constexpr uint32_t kCwMaxQueries = 4096;

struct CwQuery {
    const int32_t *out_ptr, *out_idx;
    int32_t *level, *parent;                  // the query's outputs (n each)
    uint32_t base, n;                         // virtual ids [base, base + n)
    int32_t source;
    uint32_t pad;
};

struct CwLists {                              // one level's frontier
    uint32_t *s;                              // short columns (virtual ids)
    uint32_t *l;                              // long columns (virtual ids)
    uint32_t *lbase;                          // long column i's first chunk
    uint32_t *cmap;                           // chunk -> long column
};

struct alignas(256) CwState {
    uint32_t level;                           // the level whose frontier is listed
    uint32_t done;                            // the last search level ended (narrow)
    uint32_t last;                            // wide: the deepest level launched with a frontier
    uint32_t pad;
    uint32_t cnt[3][4];                       // level k: cnt[k % 3] = short, long, chunks
};

struct CwParams {
    const CwQuery *q;                         // device, nq
    const uint32_t *bases;                    // device, nq + 1: base_q, then V
    uint32_t nq;
    uint32_t V;                               // virtual vertices (sum of n)
    uint32_t max_n;                           // largest n_q
    unsigned long long *cw;                   // [V]
    CwLists lists[2];                         // level k lists in lists[k & 1]
    uint32_t *spill;                          // narrow: next-frontier entries beyond the LDS
    CwState *st;
};

struct CwLayout {
    size_t q, bases, st, cw, s0, l0, b0, c0, s1, l1, b1, c1, spill, total;
};
CwLayout cw_layout(uint64_t V, uint64_t nnz, uint32_t nq);

hipError_t launch_cw_init(const CwParams &p, hipStream_t s);
hipError_t launch_cw_wide(const CwParams &p, uint32_t k, uint32_t grid, hipStream_t s);
hipError_t launch_cw_narrow(const CwParams &p, uint32_t k, uint32_t max_levels, uint32_t max_next,
                            uint32_t max_edges, hipStream_t s);
hipError_t launch_cw_out(const CwParams &p, hipStream_t s);

// Queries on different graphs searched as one block-diagonal graph by the
// list form: the library packs the graphs' out-lists (vertex ids offset by
// each query's base) and splits the packed results back (bfs_claim.hip).
struct PackQuery {
    const int32_t *ptr, *idx;                 // the query's graph (out-lists)
    int32_t *level, *parent;                  // the caller's outputs
    uint32_t base, n;                         // first packed vertex, vertices
    uint32_t ebase, nnz;                      // first packed entry, entries
};
struct PackParams {
    const PackQuery *q;                       // device, nq
    uint32_t nq;
    uint32_t max_n, max_nnz;
    uint32_t E, pad_end;                      // packed entries; idx is zero-filled in [E, pad_end)
    int32_t *ptr, *idx;                       // packed CSR: V + 1 offsets, pad_end entries
    const int32_t *level, *parent;            // packed results [V]
};
hipError_t launch_pack(const PackParams &p, hipStream_t s);
hipError_t launch_unpack(const PackParams &p, hipStream_t s);

// The comparison searches of the Experiments section (bfs_compare.hip).
enum CmpMethod : uint32_t { kCmpSpmv = 0, kCmpSpmspv = 1, kCmpSpmmspv = 2 };

struct alignas(256) CmpState {
    uint32_t k;                    // step
    uint32_t nlist;                // entries of the step's vector list
    uint32_t ntouched;             // rows first touched by the step's product
    uint32_t nnext;                // rows reached by the step
    uint32_t done;                 // set once a step reaches nothing
    uint32_t pad;
    unsigned long long ops;        // algebraic operations so far (two per nonzero multiplied)
};

struct CmpParams {
    int32_t n;
    uint32_t words;                // 32-bit words per bitmap
    uint32_t method;               // CmpMethod
    const int32_t *out_ptr, *out_idx, *in_ptr, *in_idx;
    const MsLong *lo, *li;         // the graph's split long columns / rows
    const uint32_t *lomap, *limap;
    uint32_t nlo_chunks, nli_chunks;
    int32_t *level, *parent;
    unsigned long long *y;         // [n] the product, step-keyed (see bfs_compare.hip)
    int32_t *list[2];              // vector lists, step k reads list[k & 1]
    int32_t *touched;              // the product's support (SpMmSpV, SpMV long rows)
    uint32_t *xb[2];               // vector membership bitmaps, step k reads xb[k & 1]
    CmpState *st;
    uint32_t *host_status;         // pinned: [0] steps done, [1] rows reached by the last step
};

struct CmpLayout {
    size_t state, y, l0, l1, touched, x0, x1, total;
};
CmpLayout cmp_layout(int32_t n);

// One masked sparse-matrix x sparse-vector product over a semiring
// (bfs_spmspv.hip).
enum Semiring : uint32_t { kSrBoolean = 0, kSrArithmetic = 1, kSrMinPlus = 2, kSrMinSelect = 3 };
constexpr uint32_t kSpLong = 512;      // column length from which a vector entry's column is split
constexpr uint32_t kSpChunk = 1024;    // entries per chunk of a split column
constexpr uint32_t kSpOutWords = 256;  // bitmap words per workgroup of the output passes

struct alignas(256) SpState {
    uint32_t nitems;               // split columns listed by the product pass
    uint32_t bad;                  // a vector index outside [0, n)
    unsigned long long nchunks;    // chunks over all split columns
};

struct SpItem {                    // a vector entry whose column is split
    int32_t j;
    uint32_t nch;                  // its chunks
    unsigned long long v;          // its value
    unsigned long long base;       // its first chunk (exclusive prefix of nch)
};

struct SpParams {
    int32_t n;
    uint32_t words;
    uint32_t semiring;
    const int32_t *out_ptr, *out_idx;
    const int32_t *x_idx;
    const unsigned long long *x_val;
    int32_t nx;
    const uint32_t *row_mask, *col_mask;   // nullptr: no mask
    uint32_t row_comp, col_comp;
    unsigned long long *acc;               // [n] the product, zero between calls (min semirings store ~value)
    uint32_t *touched;                     // [words] the product's support, zero between calls
    SpItem *items;                         // [nx]
    uint32_t *block_off;                   // [ceil(words / kSpOutWords)]
    SpState *st;
    int32_t *y_idx;
    unsigned long long *y_val;
    int32_t *ny;                           // device: the output's length
};

struct SpLayout {
    size_t state, acc, touched, items, block_off, ny, total;
};
SpLayout sp_layout(int32_t n, int32_t max_nx);
hipError_t launch_spmspv(const SpParams &p, uint32_t grid, hipStream_t s);
hipError_t launch_cmp_init(const CmpParams &p, int32_t source, hipStream_t s);
hipError_t launch_cmp_step(const CmpParams &p, uint32_t grid, hipStream_t s);

hipError_t launch_mlp_forward(const float *w, const float *x, float *y, int32_t rows, hipStream_t s);
hipError_t launch_mlp_grad(const float *w, const float *x, const float *t, const float *mask,
                           int32_t rows, float inv_norm, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *w, float *grad, float *m, float *v, int32_t step, float lr,
                           hipStream_t s);

}  // namespace bfsi

// Host runtime behind include/bfs.h: graph objects, validation, workspace
// layout and the level loop (host-driven, graph-replayed or persistent).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bfs.h"
#include "bfs_internal.h"

using namespace bfsi;

// What a captured level loop depends on: any difference means a new capture.
struct LoopKey {
    uint32_t kind = 0;                 // 0: list-form level kernel, 1: sliced push
    const void *ws = nullptr, *level = nullptr, *parent = nullptr;
    uint32_t policy = 0, grid = 0, heavy = 0, chunk = 0, levels = 0, fb = 0, stats = 0;
    const float *sel = nullptr;
    const void *trace = nullptr, *slot = nullptr;
    bool operator==(const LoopKey &o) const {
        return kind == o.kind && ws == o.ws && level == o.level && parent == o.parent &&
               policy == o.policy && grid == o.grid && heavy == o.heavy && chunk == o.chunk &&
               levels == o.levels && fb == o.fb && stats == o.stats && sel == o.sel &&
               trace == o.trace && slot == o.slot;
    }
};

struct GraphExecCache {
    bool valid = false;
    LoopKey key;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

struct bfs_graph {
    int32_t n = 0;
    uint32_t nnz = 0;
    uint32_t max_deg = 0;             // largest out-degree (after duplicates and self-loops are removed)
    bool directed = false;
    int device = 0;
    int cus = 0;
    int32_t *out_ptr = nullptr, *out_idx = nullptr, *in_ptr = nullptr, *in_idx = nullptr;
    size_t bytes = 0;
    // split entries for the multi-source kernels (see MsLevel): long columns
    // and long rows; for an undirected graph the two are the same arrays
    bfsi::MsLong *lo = nullptr, *li = nullptr;
    uint32_t *lomap = nullptr, *limap = nullptr;
    uint32_t nlo = 0, nlo_chunks = 0, nli = 0, nli_chunks = 0;
    uint32_t *lirest = nullptr;       // the long rows' later chunks, by position in the row, then row
    // the multi-source search's degree-ordered copy of the graph (null when
    // not kept): search label x = rank of the vertex by descending
    // out-degree; x's in-list (an undirected graph's only list) holds its
    // neighbours' labels in the order of their caller ids, with those ids
    // beside them; its split entries as above
    int32_t *do_ptr = nullptr, *do_idx = nullptr, *do_ent = nullptr;
    int32_t *do_orig = nullptr, *do_pos = nullptr;   // label -> caller id, caller id -> label
    bfsi::MsLong *do_long = nullptr;
    uint32_t *do_map = nullptr, *do_rest = nullptr;
    uint32_t do_nlong = 0, do_nchunks = 0;
    int32_t *do_rows = nullptr;       // the pull's row chunk bounds over the labels
    uint32_t do_nrows = 0;
    // a directed graph's out-lists over the same labels (the lists above are
    // then its in-lists), with their caller ids and long columns
    int32_t *do_optr = nullptr, *do_oidx = nullptr, *do_oent = nullptr;
    bfsi::MsLong *do_olong = nullptr;
    uint32_t *do_omap = nullptr;
    uint32_t do_onlong = 0, do_onchunks = 0;
    // sliced push (bfs_slice.hip): per-vertex slice starts in the sorted
    // out-lists and the chunks of long slice parts; sl_S = 0 when the graph's
    // bitmap needs more than kSlMaxSlices slices
    int4 *sl_seg = nullptr;
    uint32_t *sl_occ = nullptr;       // per slice, the vertices whose part there is short and not empty
    bfsi::SlChunk *sl_chunks = nullptr;
    uint32_t sl_S = 0, sl_sw = 0;
    uint32_t sl_chunk_off[bfsi::kSlMaxSlices + 1] = {};
    std::mutex mu;
    GraphExecCache gcache;
    std::vector<hipEvent_t> events;   // pool for per-launch timing
    hipEvent_t init_ev[2] = {nullptr, nullptr};   // around the init launch (time_kernels)
};

namespace {

thread_local std::string g_detail;

bfs_status fail(bfs_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_detail = buf;
    return s;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(BFS_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                        __FILE__, __LINE__);                                          \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bfs_status validate_csr(int32_t n, const int32_t *ptr, const int32_t *idx, const char *what) {
    if (ptr[0] != 0) return fail(BFS_ECSR, "%s: ptr[0] = %d, expected 0", what, ptr[0]);
    for (int32_t v = 0; v < n; ++v)
        if (ptr[v + 1] < ptr[v])
            return fail(BFS_ECSR, "%s: ptr decreases at %d (%d > %d)", what, v, ptr[v], ptr[v + 1]);
    const int64_t nnz = ptr[n];
    for (int64_t e = 0; e < nnz; ++e)
        if (idx[e] < 0 || idx[e] >= n)
            return fail(BFS_ECSR, "%s: idx[%lld] = %d outside [0, %d)", what, (long long)e, idx[e], n);
    return BFS_OK;
}

// sort each list ascending (pull scans in-neighbours in ascending order)
void sort_rows(int32_t n, const std::vector<int32_t> &ptr, std::vector<int32_t> &idx) {
    for (int32_t v = 0; v < n; ++v) {
        auto b = idx.begin() + ptr[v], e = idx.begin() + ptr[v + 1];
        if (!std::is_sorted(b, e)) std::sort(b, e);
    }
}

void transpose(int32_t n, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
               std::vector<int32_t> &tptr, std::vector<int32_t> &tidx) {
    tptr.assign((size_t)n + 1, 0);
    for (int32_t c : idx) tptr[(size_t)c + 1]++;
    for (int32_t v = 0; v < n; ++v) tptr[(size_t)v + 1] += tptr[v];
    tidx.resize(idx.size());
    std::vector<int32_t> pos(tptr.begin(), tptr.end() - 1);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t e = ptr[r]; e < ptr[r + 1]; ++e) tidx[pos[idx[e]]++] = r;   // rows ascending
}

template <class T>
bfs_status upload(T **dst, const T *src, size_t count, size_t &bytes) {
    size_t b = count * sizeof(T);
    if (b == 0) b = sizeof(T);
    if (hipMalloc((void **)dst, b) != hipSuccess) return fail(BFS_ENOMEM, "hipMalloc(%zu) failed", b);
    bytes += b;
    if (count) HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return BFS_OK;
}

void free_graph(bfs_graph *g) {
    if (!g) return;
    // teardown: errors here have nowhere to go, the memory is released either way
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->init_ev)
        if (e) (void)hipEventDestroy(e);
    if (g->gcache.exec) (void)hipGraphExecDestroy(g->gcache.exec);
    if (g->gcache.graph) (void)hipGraphDestroy(g->gcache.graph);
    if (g->li && g->li != g->lo) (void)hipFree(g->li);
    if (g->limap && g->limap != g->lomap) (void)hipFree(g->limap);
    if (g->lo) (void)hipFree(g->lo);
    if (g->lomap) (void)hipFree(g->lomap);
    if (g->lirest) (void)hipFree(g->lirest);
    for (int32_t *a : {g->do_ptr, g->do_idx, g->do_ent, g->do_orig, g->do_pos, g->do_rows, g->do_optr,
                       g->do_oidx, g->do_oent})
        if (a) (void)hipFree(a);
    if (g->do_olong) (void)hipFree(g->do_olong);
    if (g->do_omap) (void)hipFree(g->do_omap);
    if (g->do_long) (void)hipFree(g->do_long);
    if (g->do_map) (void)hipFree(g->do_map);
    if (g->do_rest) (void)hipFree(g->do_rest);
    if (g->in_ptr && g->in_ptr != g->out_ptr) (void)hipFree(g->in_ptr);
    if (g->in_idx && g->in_idx != g->out_idx) (void)hipFree(g->in_idx);
    if (g->out_ptr) (void)hipFree(g->out_ptr);
    if (g->out_idx) (void)hipFree(g->out_idx);
    if (g->sl_seg) (void)hipFree(g->sl_seg);
    if (g->sl_occ) (void)hipFree(g->sl_occ);
    if (g->sl_chunks) (void)hipFree(g->sl_chunks);
    delete g;
}

// Entries of ptr with at least kMsLong positions, each split into chunks of
// kMsChunk numbered consecutively; uploads the entries and chunk -> entry map.
bfs_status build_long(int32_t n, const std::vector<int32_t> &ptr, bfsi::MsLong **ents, uint32_t **map,
                      uint32_t &count, uint32_t &chunks, size_t &bytes) {
    std::vector<bfsi::MsLong> e;
    std::vector<uint32_t> m;
    for (int32_t v = 0; v < n; ++v) {
        const uint32_t deg = (uint32_t)(ptr[v + 1] - ptr[v]);
        if (deg < bfsi::kMsLong) continue;
        e.push_back(bfsi::MsLong{v, (uint32_t)m.size()});
        const uint32_t nch = (deg + bfsi::kMsChunk - 1) / bfsi::kMsChunk;
        for (uint32_t c = 0; c < nch; ++c) m.push_back((uint32_t)(e.size() - 1));
    }
    count = (uint32_t)e.size();
    chunks = (uint32_t)m.size();
    bfs_status st = upload(ents, e.data(), e.size(), bytes);
    if (st == BFS_OK) st = upload(map, m.data(), m.size(), bytes);
    return st;
}

// The chunk ids of every long row's chunks but its first, ordered by the
// chunk's position in its row (1, 2, ...) and then by row: the pull's later
// chunks run in this order, so that a row's earlier chunks have mostly
// finished (and settled their sources) when its later ones start.
bfs_status build_rest(int32_t n, const std::vector<int32_t> &ptr, uint32_t **out, size_t &bytes) {
    std::vector<std::vector<uint32_t>> by_pos;
    uint32_t base = 0;
    for (int32_t v = 0; v < n; ++v) {
        const uint32_t deg = (uint32_t)(ptr[v + 1] - ptr[v]);
        if (deg < bfsi::kMsLong) continue;
        const uint32_t nch = (deg + bfsi::kMsChunk - 1) / bfsi::kMsChunk;
        if (by_pos.size() < nch) by_pos.resize(nch);
        for (uint32_t j = 1; j < nch; ++j) by_pos[j].push_back(base + j);
        base += nch;
    }
    std::vector<uint32_t> order;
    for (const auto &b : by_pos) order.insert(order.end(), b.begin(), b.end());
    return upload(out, order.data(), order.size(), bytes);
}

// The degree-ordered copy of a graph for the multi-source search.
// Its frontier masks are gathered once per scanned list entry; with the
// vertices ranked by descending degree the masks most entries point to share
// a few megabytes (R-MAT s22: 85% of the entries point to the 262,144 vertices
// of largest degree, 2 MB of 8-byte masks) instead of one line each across the
// whole array.  Each list keeps the order of the caller's ids, and the
// caller's ids sit beside the labels, so that the first frontier neighbour
// found in list order is still the one of smallest caller id (the parent).
// Lists of the caller's CSR (ptr, idx) over labels: row x = the list of
// vertex orig[x] in its own order, entries as labels (dptr, didx) and as the
// caller's ids (dent).
static void relabel_lists(int32_t n, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                          const std::vector<int32_t> &orig, const std::vector<int32_t> &pos,
                          std::vector<int32_t> &dptr, std::vector<int32_t> &didx, std::vector<int32_t> &dent) {
    dptr.assign((size_t)n + 1, 0);
    didx.resize(idx.size());
    dent.resize(idx.size());
    for (int32_t x = 0; x < n; ++x) {
        const int32_t v = orig[(size_t)x];
        int32_t o = dptr[(size_t)x];
        for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e, ++o) {
            dent[(size_t)o] = idx[(size_t)e];
            didx[(size_t)o] = pos[(size_t)idx[(size_t)e]];
        }
        dptr[(size_t)x + 1] = o;
    }
}

// ptr / idx: the out-lists; iptr / iidx: the in-lists (the same arrays for an
// undirected graph).  Labels rank the vertices by descending out-degree (how
// often a vertex's mask is gathered by the pull's scans of in-lists).
bfs_status build_degree_order(bfs_graph *g, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                              const std::vector<int32_t> &iptr, const std::vector<int32_t> &iidx) {
    const int32_t n = g->n;
    std::vector<int32_t> orig((size_t)n), pos((size_t)n);
    for (int32_t v = 0; v < n; ++v) orig[(size_t)v] = v;
    std::stable_sort(orig.begin(), orig.end(), [&](int32_t a, int32_t b) {
        return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b];
    });
    for (int32_t x = 0; x < n; ++x) pos[(size_t)orig[(size_t)x]] = x;
    std::vector<int32_t> dptr, didx, dent;
    relabel_lists(n, iptr, iidx, orig, pos, dptr, didx, dent);
    bfs_status st = BFS_OK;
    if (g->directed) {
        std::vector<int32_t> optr, oidx, oent;
        relabel_lists(n, ptr, idx, orig, pos, optr, oidx, oent);
        st = upload(&g->do_optr, optr.data(), optr.size(), g->bytes);
        if (st == BFS_OK) st = upload(&g->do_oidx, oidx.data(), oidx.size(), g->bytes);
        if (st == BFS_OK) st = upload(&g->do_oent, oent.data(), oent.size(), g->bytes);
        if (st == BFS_OK) st = build_long(n, optr, &g->do_olong, &g->do_omap, g->do_onlong, g->do_onchunks, g->bytes);
    }
    if (st == BFS_OK) st = upload(&g->do_ptr, dptr.data(), dptr.size(), g->bytes);
    if (st == BFS_OK) st = upload(&g->do_idx, didx.data(), didx.size(), g->bytes);
    if (st == BFS_OK) st = upload(&g->do_ent, dent.data(), dent.size(), g->bytes);
    if (st == BFS_OK) st = upload(&g->do_orig, orig.data(), orig.size(), g->bytes);
    if (st == BFS_OK) st = upload(&g->do_pos, pos.data(), pos.size(), g->bytes);
    if (st == BFS_OK) st = build_long(n, dptr, &g->do_long, &g->do_map, g->do_nlong, g->do_nchunks, g->bytes);
    if (st == BFS_OK) st = build_rest(n, dptr, &g->do_rest, g->bytes);
    // the pull's row chunks: runs of at most kMsRows labels holding about the
    // entries kMsRows rows hold on average (rows of kMsLong+ entries count
    // nothing: their chunks are dealt apart), so that the heaviest rows,
    // which now lie side by side, spread over many workgroups
    uint64_t short_entries = 0;
    for (int32_t x = 0; x < n; ++x) {
        const uint32_t d = (uint32_t)(dptr[(size_t)x + 1] - dptr[(size_t)x]);
        if (d < bfsi::kMsLong) short_entries += d;
    }
    const uint64_t target = std::max<uint64_t>(1, short_entries * bfsi::kMsRows / (uint64_t)n);
    std::vector<int32_t> rows{0};
    uint64_t acc = 0;
    uint32_t cnt = 0;
    for (int32_t x = 0; x < n; ++x) {
        const uint32_t d = (uint32_t)(dptr[(size_t)x + 1] - dptr[(size_t)x]);
        const uint64_t wgt = d < bfsi::kMsLong ? d : 0;
        if (cnt > 0 && (cnt == bfsi::kMsRows || acc + wgt > target)) {
            rows.push_back(x);
            acc = 0;
            cnt = 0;
        }
        acc += wgt;
        ++cnt;
    }
    rows.push_back(n);
    g->do_nrows = (uint32_t)(rows.size() - 1);
    if (st == BFS_OK) st = upload(&g->do_rows, rows.data(), rows.size(), g->bytes);
    return st;
}

// The out-lists, padded with zeros to a multiple of four entries plus four, so
// that the sliced push may read any list in aligned 16-byte quads.
bfs_status upload_padded(int32_t **dst, const std::vector<int32_t> &idx, size_t &bytes) {
    const size_t cnt = ((idx.size() + 3) & ~size_t(3)) + 4;
    if (hipMalloc((void **)dst, cnt * 4) != hipSuccess) return fail(BFS_ENOMEM, "hipMalloc(%zu) failed", cnt * 4);
    bytes += cnt * 4;
    HIP_TRY(hipMemset(*dst, 0, cnt * 4));
    if (!idx.empty()) HIP_TRY(hipMemcpy(*dst, idx.data(), idx.size() * 4, hipMemcpyHostToDevice));
    return BFS_OK;
}

// The sliced push's graph data: S slices of sw words (sw a multiple of 4, at
// most kSlMaxSliceWords); seg[v] = {ptr[v], first entry of v's sorted list in
// slice 1, 2, 3} (ptr[v + 1] for slices past the last); and every slice part
// of at least kSlLong entries cut into chunks of kSlChunk, grouped by slice.
bfs_status build_slices(bfs_graph *g, const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                        uint32_t max_words = bfsi::kSlMaxSliceWords) {
    const int32_t n = g->n;
    const uint64_t words = ((uint64_t)n + 31) / 32;
    const uint64_t S = (words + max_words - 1) / max_words;
    if (S == 0 || S > bfsi::kSlMaxSlices) return BFS_OK;          // not eligible: g->sl_S stays 0
    const uint32_t sw = (uint32_t)(((words + S - 1) / S + 3) & ~uint64_t(3));
    const int64_t sv = (int64_t)sw * 32;
    std::vector<int4> seg((size_t)n + 1);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t *b = idx.data() + ptr[v], *e = idx.data() + ptr[v + 1];
        int32_t st[4];
        st[0] = ptr[v];
        for (int t = 1; t < 4; ++t) {
            const int64_t bound = (int64_t)t * sv;
            st[t] = bound >= n ? ptr[v + 1]
                               : (int32_t)(std::lower_bound(b, e, (int32_t)bound) - idx.data());
        }
        seg[v] = make_int4(st[0], st[1], st[2], st[3]);
    }
    const int32_t nnz = ptr[n];
    seg[n] = make_int4(nnz, nnz, nnz, nnz);
    // per slice, a bit for each vertex whose part there the frontier loop
    // expands (short, not empty); long parts go by chunks
    const uint64_t allw = (uint64_t)S * sw;
    std::vector<uint32_t> occ((size_t)(S * allw), 0u);
    for (int32_t v = 0; v < n; ++v) {
        const int4 q = seg[v];
        for (uint32_t s = 0; s < S; ++s) {
            const int32_t a = s == 0 ? q.x : (s == 1 ? q.y : (s == 2 ? q.z : q.w));
            const int32_t e = s == 3 ? seg[v + 1].x : (s == 0 ? q.y : (s == 1 ? q.z : q.w));
            if (e > a && e - a < (int32_t)bfsi::kSlLong) occ[(size_t)(s * allw) + ((uint32_t)v >> 5)] |= 1u << (v & 31);
        }
    }
    std::vector<bfsi::SlChunk> ch;
    uint32_t off[bfsi::kSlMaxSlices + 1] = {};
    for (uint32_t s = 0; s < bfsi::kSlMaxSlices; ++s) {
        off[s] = (uint32_t)ch.size();
        if (s >= S) continue;
        for (int32_t v = 0; v < n; ++v) {
            const int4 q = seg[v];
            const int32_t a = s == 0 ? q.x : (s == 1 ? q.y : (s == 2 ? q.z : q.w));
            const int32_t e = s == 3 ? seg[v + 1].x : (s == 0 ? q.y : (s == 1 ? q.z : q.w));
            if (e - a < (int32_t)bfsi::kSlLong) continue;
            for (int32_t c = a; c < e; c += (int32_t)bfsi::kSlChunk)
                ch.push_back(bfsi::SlChunk{v, c, std::min<int32_t>(e, c + (int32_t)bfsi::kSlChunk), 0});
        }
    }
    off[bfsi::kSlMaxSlices] = (uint32_t)ch.size();
    bfs_status st = upload(&g->sl_seg, seg.data(), seg.size(), g->bytes);
    if (st == BFS_OK) st = upload(&g->sl_chunks, ch.data(), ch.size(), g->bytes);
    if (st == BFS_OK) st = upload(&g->sl_occ, occ.data(), occ.size(), g->bytes);
    if (st != BFS_OK) return st;
    g->sl_S = (uint32_t)S;
    g->sl_sw = sw;
    for (uint32_t s = 0; s <= bfsi::kSlMaxSlices; ++s) g->sl_chunk_off[s] = off[s];
    return BFS_OK;
}

}  // namespace

namespace bfsi {
constexpr uint32_t kChunkFloor = 64;
WsLayout ws_layout(int32_t n, uint32_t nnz, uint32_t heavy_min_floor) {
    WsLayout L{};
    const size_t words = ((size_t)n + 31) / 32;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.state = take(sizeof(BfsState));
    L.vb0 = take(words * 4);
    L.vb1 = take(words * 4);
    L.fb0 = take(words * 4);
    L.fb1 = take(words * 4);
    L.fb2 = take(words * 4);
    L.q0 = take((size_t)n * sizeof(QEnt));
    L.q1 = take((size_t)n * sizeof(QEnt));
    L.u0 = take((size_t)n * 4);
    L.u1 = take((size_t)n * 4);
    // long columns in one frontier: at most nnz / heavy_min of them
    size_t hcap = (size_t)nnz / heavy_min_floor + 1;
    if (hcap > (size_t)n) hcap = (size_t)n;
    L.h0 = take(hcap * sizeof(HeavyItem));
    L.h1 = take(hcap * sizeof(HeavyItem));
    // chunks in one frontier: at most nnz / chunk_floor + (number of long columns)
    const size_t ccap = (size_t)nnz / kChunkFloor + hcap + 1;
    L.c0 = take(ccap * 4);
    L.c1 = take(ccap * 4);
    L.trace = take((size_t)kTraceCap * sizeof(DevLevelRec));
    L.total = off;
    return L;
}
}  // namespace bfsi

namespace bfsi {
MsLayout ms_layout(int32_t n, int32_t nq, bool staged) {
    MsLayout L{};
    const size_t W = ((size_t)nq + 63) / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.vis = take((size_t)n * W * 8);
    L.m0 = take((size_t)n * W * 8);
    L.m1 = take((size_t)n * W * 8);
    L.m2 = take((size_t)n * W * 8);
    L.f0 = take((size_t)n * 4);
    L.f1 = take((size_t)n * 4);
    L.f2 = take((size_t)n * 4);
    L.flag = take((size_t)n * 4);
    L.cnt = take(64);
    L.mstat = take(kMsStatWords * 8);
    L.fbits = take(((size_t)n + 63) / 64 * 8);
    L.rl0 = take((size_t)n * 4);
    L.rl1 = take((size_t)n * 4);
    L.rcnt = take(64);
    L.rcur = take((size_t)n * 4);
    L.slev = staged ? take((size_t)n * W * 64 * 4) : 0;
    L.spar = staged ? take((size_t)n * W * 64 * 4) : 0;
    L.lptr = take((size_t)nq * 8);
    L.pptr = take((size_t)nq * 8);
    L.src = take((size_t)nq * 4);
    L.total = off;
    return L;
}

CwLayout cw_layout(uint64_t V, uint64_t nnz, uint32_t nq) {
    CwLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    // chunks of one level: every long column (at least kCwLong entries) has
    // ceil(deg / kCwChunk) <= deg / kCwChunk + 1 of them
    const size_t chunks = (size_t)(nnz / kCwChunk + nnz / kCwLong + 1);
    L.q = take((size_t)nq * sizeof(CwQuery));
    L.bases = take(((size_t)nq + 1) * 4);
    L.st = take(sizeof(CwState));
    L.cw = take((size_t)V * 8);
    L.s0 = take((size_t)V * 4);
    L.l0 = take((size_t)V * 4);
    L.b0 = take((size_t)V * 4);
    L.c0 = take(chunks * 4);
    L.s1 = take((size_t)V * 4);
    L.l1 = take((size_t)V * 4);
    L.b1 = take((size_t)V * 4);
    L.c1 = take(chunks * 4);
    L.spill = take((size_t)V * 4);
    L.total = off;
    return L;
}
}  // namespace bfsi

namespace {

constexpr uint32_t kHeavyFloor = 32;

struct RunCfg {
    uint32_t policy, loop, per_sync, grid, heavy, chunk;
    const float *sel;
};

bfs_status make_params(bfs_graph *g, int32_t *level, int32_t *parent, const RunCfg &c,
                       void *ws, bool trace, LevelParams &P) {
    const WsLayout L = ws_layout(g->n, g->nnz, kHeavyFloor);
    char *b = (char *)ws;
    P = LevelParams{};
    P.n = g->n;
    P.nnz = g->nnz;
    P.words = (uint32_t)(((size_t)g->n + 31) / 32);
    P.policy = c.policy;
    P.heavy_min = c.heavy;
    P.chunk = c.chunk;
    P.out_ptr = g->out_ptr;
    P.out_idx = g->out_idx;
    P.in_ptr = g->in_ptr;
    P.in_idx = g->in_idx;
    P.level = level;
    P.parent = (uint32_t *)parent;
    P.vb[0] = (uint32_t *)(b + L.vb0);
    P.vb[1] = (uint32_t *)(b + L.vb1);
    P.fb[0] = (uint32_t *)(b + L.fb0);
    P.fb[1] = (uint32_t *)(b + L.fb1);
    P.fb[2] = (uint32_t *)(b + L.fb2);
    P.q[0] = (QEnt *)(b + L.q0);
    P.q[1] = (QEnt *)(b + L.q1);
    P.ul[0] = (int32_t *)(b + L.u0);
    P.ul[1] = (int32_t *)(b + L.u1);
    P.hl[0] = (HeavyItem *)(b + L.h0);
    P.hl[1] = (HeavyItem *)(b + L.h1);
    P.cmap[0] = (uint32_t *)(b + L.c0);
    P.cmap[1] = (uint32_t *)(b + L.c1);
    P.st = (BfsState *)(b + L.state);
    P.trace = trace ? (DevLevelRec *)(b + L.trace) : nullptr;
    P.mlp = c.sel;
    P.maintain_fb = (c.policy == kBitmap || c.policy == kLearned || c.policy == kHeuristic) ? 1u : 0u;
    // the level sums also pick the short-circuit levels
    P.stats = (c.policy == kLearned || c.policy == kHeuristic || c.policy == kShortCircuit || trace) ? 1u : 0u;
    return BFS_OK;
}

bfs_status resolve_cfg(bfs_graph *g, const bfs_run_options *opt, RunCfg &c) {
    c.policy = opt ? opt->variant : kPush;
    c.loop = opt ? opt->loop_mode : BFS_LOOP_HOST;
    c.per_sync = (opt && opt->levels_per_sync) ? opt->levels_per_sync : 4u;
    c.grid = (opt && opt->grid_blocks) ? opt->grid_blocks : (uint32_t)(8 * (g->cus > 0 ? g->cus : 256));
    c.heavy = (opt && opt->heavy_degree) ? opt->heavy_degree : 512u;
    c.chunk = (opt && opt->chunk_edges) ? opt->chunk_edges : 1024u;
    c.sel = opt ? opt->selector : nullptr;
    if (c.policy > kShortCircuit) return fail(BFS_EINVAL, "unknown variant %u", c.policy);
    if (c.loop > BFS_LOOP_PERSISTENT) return fail(BFS_EINVAL, "unknown loop mode %u", c.loop);
    if (c.heavy < kHeavyFloor) return fail(BFS_EINVAL, "heavy_degree %u below %u", c.heavy, kHeavyFloor);
    if (c.chunk < kChunkFloor || c.chunk > (1u << 20))
        return fail(BFS_EINVAL, "chunk_edges %u outside [%u, 2^20]", c.chunk, kChunkFloor);
    if (c.grid == 0 || c.grid > 65535) return fail(BFS_EINVAL, "grid_blocks %u outside [1, 65535]", c.grid);
    if (c.per_sync > 4096) return fail(BFS_EINVAL, "levels_per_sync %u above 4096", c.per_sync);
    return BFS_OK;
}

// Where the level kernels report progress to the host: a small pinned,
// coherent host buffer per host thread, written by the device after every
// level ([0] = current level, [1] = its frontier size).  Allocated on the
// thread's first search and kept for the life of the process, so searches
// themselves allocate nothing.
struct HostSlot {
    volatile uint32_t *h = nullptr;
    uint32_t *d = nullptr;
};

bfs_status host_slot(HostSlot *&out) {
    thread_local HostSlot slot;
    if (!slot.h) {
        void *p = nullptr;
        if (hipHostMalloc(&p, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
            return fail(BFS_ENOMEM, "hipHostMalloc of the progress slot failed");
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess)
            return fail(BFS_EHIP, "hipHostGetDevicePointer of the progress slot failed");
        slot.h = (volatile uint32_t *)p;
        slot.d = (uint32_t *)dp;
    }
    out = &slot;
    return BFS_OK;
}

// wait for the stream, then read the progress the device left in the slot
bfs_status wait_progress(const HostSlot *hs, hipStream_t s, bool &done, uint32_t &level) {
    HIP_TRY(hipStreamSynchronize(s));
    level = hs->h[0];
    done = (hs->h[1] == 0);
    return BFS_OK;
}

// The host loop and the captured-graph loop around a level launch: `launch`
// issues one level on a stream; levels are issued `per_sync` at a time
// between two reads of the progress slot (launches past the end return at
// once).  The captured graph is cached per bfs_graph under `key`.  With
// opt->time_kernels (host loop) every launch is bracketed by HIP events and
// `times` receives the launches' device times.
template <class Launch>
bfs_status level_loop(bfs_graph *g, const LoopKey &key, uint32_t loop, hipStream_t s, HostSlot *hs,
                      Launch launch, uint32_t &level, std::vector<float> &times, bfs_run_options *opt) {
    const uint64_t max_levels = (uint64_t)g->n + 2;
    const uint32_t L = key.levels;
    bool done = false;
    std::unique_lock<std::mutex> lock(g->mu, std::defer_lock);
    if (loop == BFS_LOOP_GRAPH) {
        lock.lock();                  // the captured graph is cached per bfs_graph
        GraphExecCache &gc = g->gcache;
        if (!(gc.valid && gc.key == key)) {
            if (gc.exec) { (void)hipGraphExecDestroy(gc.exec); gc.exec = nullptr; }
            if (gc.graph) { (void)hipGraphDestroy(gc.graph); gc.graph = nullptr; }
            gc.valid = false;
            hipStream_t cap;
            HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            for (uint32_t l = 0; l < L && e == hipSuccess; ++l) e = launch(cap);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(cap, &graph);
            (void)hipStreamDestroy(cap);
            if (e != hipSuccess || e2 != hipSuccess)
                return fail(BFS_EHIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return fail(BFS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
            gc.graph = graph;
            gc.exec = exec;
            gc.key = key;
            gc.valid = true;
        }
        for (uint64_t issued = 0; !done; issued += L) {
            if (issued > max_levels) return fail(BFS_EHIP, "level loop did not terminate");
            HIP_TRY(hipGraphLaunch(gc.exec, s));
            bfs_status st = wait_progress(hs, s, done, level);
            if (st != BFS_OK) return st;
        }
        return BFS_OK;
    }
    const bool tk = opt && opt->time_kernels;
    if (tk) lock.lock();              // the event pool is per bfs_graph
    uint32_t launched = 0;
    auto ev = [&](uint32_t i, hipEvent_t &out) -> bfs_status {
        while (g->events.size() <= i) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            g->events.push_back(e);
        }
        out = g->events[i];
        return BFS_OK;
    };
    for (uint64_t issued = 0; !done; issued += L) {
        if (issued > max_levels) return fail(BFS_EHIP, "level loop did not terminate");
        for (uint32_t l = 0; l < L; ++l) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (tk) {
                bfs_status st = ev(2 * launched, e0);
                if (st == BFS_OK) st = ev(2 * launched + 1, e1);
                if (st != BFS_OK) return st;
                HIP_TRY(hipEventRecord(e0, s));
            }
            HIP_TRY(launch(s));
            if (tk) HIP_TRY(hipEventRecord(e1, s));
            ++launched;
        }
        bfs_status st = wait_progress(hs, s, done, level);
        if (st != BFS_OK) return st;
    }
    if (tk) {
        float total = 0.f;
        for (uint32_t i = 0; i < launched; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, g->events[2 * i], g->events[2 * i + 1]));
            total += ms * 1000.f;
            times.push_back(ms * 1000.f);
        }
        opt->launches = launched;
        opt->kernel_us = total;
    }
    return BFS_OK;
}

// Issue a search's init launch(es); with opt->time_kernels, bracket them with
// the graph's init events and report their device time in opt->init_us.
template <class Launch>
bfs_status timed_init(bfs_graph *g, bfs_run_options *opt, hipStream_t s, Launch launch) {
    const bool tk = opt && opt->time_kernels;
    if (!tk) {
        HIP_TRY(launch());
        return BFS_OK;
    }
    std::lock_guard<std::mutex> lock(g->mu);
    for (hipEvent_t &e : g->init_ev)
        if (!e) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(g->init_ev[0], s));
    HIP_TRY(launch());
    HIP_TRY(hipEventRecord(g->init_ev[1], s));
    HIP_TRY(hipEventSynchronize(g->init_ev[1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, g->init_ev[0], g->init_ev[1]));
    opt->init_us = ms * 1000.f;
    return BFS_OK;
}

// Copy the device's per-level records into opt->trace (host), with the
// launches' device times when they were taken.
bfs_status read_trace(const DevLevelRec *dtrace, uint32_t levels, const std::vector<float> &times,
                      bfs_run_options *opt, hipStream_t s) {
    if (!opt) return BFS_OK;
    if (!(opt->trace && dtrace)) {
        opt->trace_count = 0;
        return BFS_OK;
    }
    const uint32_t nrec = std::min<uint32_t>(std::min<uint32_t>(levels, kTraceCap), opt->trace_capacity);
    std::vector<DevLevelRec> recs(nrec ? nrec : 1);
    if (nrec) {
        HIP_TRY(hipMemcpyAsync(recs.data(), dtrace, nrec * sizeof(DevLevelRec), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    for (uint32_t r = 0; r < nrec; ++r) {
        bfs_level_record &o = opt->trace[r];
        o.level = (int32_t)recs[r].level;
        o.variant = (int32_t)recs[r].variant;
        o.frontier = recs[r].nf;
        o.unvisited = recs[r].nu;
        o.frontier_edges = recs[r].sdf;
        o.unvisited_edges = recs[r].sdu;
        o.time_us = (r < times.size()) ? times[r] : 0.f;
        o.reserved = 0.f;
    }
    opt->trace_count = nrec;
    return BFS_OK;
}

bfs_status run_levels(bfs_graph *g, LevelParams &P, const RunCfg &c, hipStream_t s,
                      uint32_t &levels_out, bfs_run_options *opt) {
    HostSlot *hs = nullptr;
    bfs_status st0 = host_slot(hs);
    if (st0 != BFS_OK) return st0;
    P.host_status = hs->d;
    hs->h[0] = 0;
    hs->h[1] = 1;
    bool done = false;
    uint32_t level = 0;
    std::vector<float> times;
    if (c.loop == BFS_LOOP_PERSISTENT) {
        uint32_t maxg = persistent_max_grid(g->device);
        if (maxg == 0) return fail(BFS_EHIP, "occupancy query for the persistent kernel failed");
        uint32_t grid = std::min(c.grid, maxg);
        HIP_TRY(launch_persistent(P, grid, s));
        bfs_status st = wait_progress(hs, s, done, level);
        if (st != BFS_OK) return st;
        if (!done) return fail(BFS_EHIP, "persistent search stopped at level %u with a nonempty frontier "
                                         "(grid barrier spin limit)", level);
    } else {
        LoopKey key;
        key.kind = 0;
        key.ws = P.st; key.level = P.level; key.parent = P.parent; key.policy = c.policy;
        key.grid = c.grid; key.heavy = c.heavy; key.chunk = c.chunk; key.levels = c.per_sync;
        key.sel = c.sel; key.fb = P.maintain_fb; key.stats = P.stats;
        key.trace = (const void *)P.trace; key.slot = (const void *)P.host_status;
        const LevelParams Pc = P;
        const uint32_t grid = c.grid;
        bfs_status st = level_loop(g, key, c.loop, s, hs,
                                   [&Pc, grid](hipStream_t st_) { return launch_level(Pc, grid, st_); },
                                   level, times, opt);
        if (st != BFS_OK) return st;
    }
    levels_out = level;
    if (c.policy == kShortCircuit) HIP_TRY(launch_parents(P, c.grid, s));     // the parents, after the levels
    return read_trace(P.trace, levels_out, times, opt, s);
}

// Workspace of one search, whichever form runs it.
size_t ws_single(const bfs_graph *g) {
    const size_t list = ws_layout(g->n, g->nnz, kHeavyFloor).total;
    const size_t sliced = g->sl_S ? sl_layout(g->sl_S * g->sl_sw).total : 0;
    const size_t claim = cw_layout((uint64_t)g->n, g->nnz, 1).total;
    return std::max(std::max(list, sliced), claim);
}

// ---------------------------------------------------------------------------
// The claim-word push (bfs_claim.hip): one query, or many on any graphs
// ---------------------------------------------------------------------------

constexpr uint32_t kCwLevelsPerLaunch = 4096;    // narrow: levels per launch at most
// The narrow kernel runs from a frontier of at most kCwNarrowEnter columns
// until the next one holds more than kCwNarrowExit columns or a level more than
// kCwNarrowEdgesMax entries: one workgroup issues about one memory request per
// cycle, so beyond a few thousand requests per level the grid-wide launch
// (about 14 us of dependent memory round trips per level) is faster.
constexpr uint32_t kCwNarrowEnter = 128;
constexpr uint32_t kCwNarrowExit = 512;
constexpr uint32_t kCwNarrowEdgesMax = 4096;
constexpr uint32_t kCwWidePerSync = 32;          // wide levels between two reads of the counts, at most
constexpr uint32_t kCwWideMinGrid = 64;          // workgroups of a wide launch at least

struct ClaimQuery {
    const bfs_graph *g;
    int32_t source;
    int32_t *level, *parent;
};

uint64_t claim_vertices(const ClaimQuery *qs, int32_t nq, uint64_t *nnz) {
    uint64_t V = 0, E = 0;
    for (int32_t q = 0; q < nq; ++q) {
        V += (uint64_t)qs[q].g->n;
        E += qs[q].g->nnz;
    }
    if (nnz) *nnz = E;
    return V;
}

size_t claim_workspace(const ClaimQuery *qs, int32_t nq) {
    uint64_t E = 0;
    const uint64_t V = claim_vertices(qs, nq, &E);
    return cw_layout(V, E, (uint32_t)nq).total;
}

// The searches of qs together: the narrow kernel while a level fits one
// workgroup, the wide one otherwise (a level it hands back unexpanded runs
// wide), the frontier counts read back after every launch.
bfs_status run_claim(const ClaimQuery *qs, int32_t nq, void *workspace, size_t ws_bytes, hipStream_t s,
                     int cus, bfs_run_options *opt) {
    uint64_t E = 0;
    const uint64_t V = claim_vertices(qs, nq, &E);
    if (V >= 0xFFFFFFFFull) return fail(BFS_EINVAL, "the queries hold %llu vertices (at most 2^32 - 2)",
                                        (unsigned long long)V);
    if ((uint32_t)nq > kCwMaxQueries) return fail(BFS_EINVAL, "%d queries (at most %u)", nq, kCwMaxQueries);
    const CwLayout L = cw_layout(V, E, (uint32_t)nq);
    if (ws_bytes < L.total) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    char *b = (char *)workspace;
    std::vector<CwQuery> hq((size_t)nq);
    std::vector<uint32_t> hb((size_t)nq + 1);
    uint32_t base = 0, max_n = 0;
    for (int32_t q = 0; q < nq; ++q) {
        CwQuery &d = hq[(size_t)q];
        d.out_ptr = qs[q].g->out_ptr;
        d.out_idx = qs[q].g->out_idx;
        d.level = qs[q].level;
        d.parent = qs[q].parent;
        d.base = base;
        d.n = (uint32_t)qs[q].g->n;
        d.source = qs[q].source;
        d.pad = 0;
        hb[(size_t)q] = base;
        base += d.n;
        max_n = std::max(max_n, d.n);
    }
    hb[(size_t)nq] = base;
    CwParams P{};
    P.q = (const CwQuery *)(b + L.q);
    P.bases = (const uint32_t *)(b + L.bases);
    P.nq = (uint32_t)nq;
    P.V = (uint32_t)V;
    P.max_n = max_n;
    P.cw = (unsigned long long *)(b + L.cw);
    P.lists[0] = CwLists{(uint32_t *)(b + L.s0), (uint32_t *)(b + L.l0), (uint32_t *)(b + L.b0),
                         (uint32_t *)(b + L.c0)};
    P.lists[1] = CwLists{(uint32_t *)(b + L.s1), (uint32_t *)(b + L.l1), (uint32_t *)(b + L.b1),
                         (uint32_t *)(b + L.c1)};
    P.spill = (uint32_t *)(b + L.spill);
    P.st = (CwState *)(b + L.st);
    HIP_TRY(hipMemcpyAsync(b + L.q, hq.data(), hq.size() * sizeof(CwQuery), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b + L.bases, hb.data(), hb.size() * 4, hipMemcpyHostToDevice, s));
    const bool tk = opt && opt->time_kernels;
    std::vector<hipEvent_t> evs;
    auto free_events = [&]() {
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    };
    // every launch, bracketed by two events when timing
    auto launch = [&](auto &&fn) -> hipError_t {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tk) {
            hipError_t e = hipEventCreate(&e0);
            if (e != hipSuccess) return e;
            evs.push_back(e0);
            if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
            evs.push_back(e1);
            if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
        }
        hipError_t e = fn();
        if (e == hipSuccess && tk) e = hipEventRecord(e1, s);
        return e;
    };
    auto run = [&](uint32_t &levels, uint32_t &launches) -> bfs_status {
        HIP_TRY(launch_cw_init(P, s));
        CwState hst;
        auto read_state = [&]() -> hipError_t {
            hipError_t e = hipMemcpyAsync(&hst, P.st, sizeof hst, hipMemcpyDeviceToHost, s);
            return e == hipSuccess ? hipStreamSynchronize(s) : e;
        };
        HIP_TRY(read_state());
        uint32_t k = 0;
        bool narrow_refused = false;          // the narrow kernel handed level k back
        const uint32_t wide_max = 8u * (uint32_t)(cus > 0 ? cus : 256);
        // wide levels between two reads of the counts: as given, else 2, 4,
        // ... up to kCwWidePerSync as the search goes on (a shallow search
        // launches few levels past its end, a deep one syncs rarely)
        const uint32_t fixed_sync = opt ? opt->levels_per_sync : 0u;
        uint32_t per_sync = fixed_sync ? fixed_sync : 2u;
        for (uint64_t guard = 0;; ++guard) {
            if (guard > V + 4) return fail(BFS_EHIP, "claim-word loop did not terminate");
            const uint32_t *c = hst.cnt[k % 3];
            const uint32_t nf = c[0] + c[1];
            if (nf == 0) break;
            if (nf <= kCwNarrowEnter && !narrow_refused) {
                HIP_TRY(launch([&]() {
                    return launch_cw_narrow(P, k, kCwLevelsPerLaunch, kCwNarrowExit, kCwNarrowEdgesMax, s);
                }));
                ++launches;
                HIP_TRY(read_state());
                if (hst.level == k) {
                    narrow_refused = true;
                    continue;
                }
                k = hst.level;
                if (hst.done) break;
                continue;
            }
            // per_sync wide levels back to back, sized for twice this level's
            // frontier; levels launched past the end of the search find no
            // frontier and change nothing
            const uint32_t waves = (c[0] + 63) / 64 + c[2];
            const uint32_t grid = std::min(wide_max, std::max(kCwWideMinGrid, (2 * waves + 3) / 4));
            for (uint32_t i = 0; i < per_sync; ++i) {
                HIP_TRY(launch([&]() { return launch_cw_wide(P, k + i, grid, s); }));
                ++launches;
            }
            HIP_TRY(read_state());
            const uint32_t *cn = hst.cnt[(k + per_sync) % 3];
            if (cn[0] + cn[1] == 0) {
                k = hst.last + 1;              // the level after the deepest frontier
                break;
            }
            k += per_sync;
            if (!fixed_sync) per_sync = std::min(2 * per_sync, kCwWidePerSync);
            narrow_refused = false;
        }
        levels = k;
        HIP_TRY(launch_cw_out(P, s));
        return BFS_OK;
    };
    uint32_t levels = 0, launches = 0;
    bfs_status st = run(levels, launches);
    if (st == BFS_OK && tk) {
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(BFS_EHIP, "stream synchronise failed");
        float total = 0.f;
        for (size_t i = 0; st == BFS_OK && i + 1 < evs.size(); i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, evs[i], evs[i + 1]) != hipSuccess) st = fail(BFS_EHIP, "event time failed");
            total += ms * 1000.f;
        }
        if (st == BFS_OK) {
            opt->kernel_us = total;
            opt->launches = launches;
        }
    }
    free_events();
    if (st != BFS_OK) return st;
    if (opt) {
        opt->levels = levels;
        opt->trace_count = 0;
    }
    return BFS_OK;
}

// The sliced push's launch size: 8 * S * R workgroups, R = compute units per
// (8 * S) (at least one), one workgroup per compute unit.
uint32_t sl_grid(const bfs_graph *g) {
    const uint32_t cus = (uint32_t)(g->cus > 0 ? g->cus : 256);
    const uint32_t per = 8u * g->sl_S;
    const uint32_t r = std::max<uint32_t>(1u, cus / per);
    return per * r;
}

// The automatic choice of the push's form, from the degree distribution
// (measured, one search each: R-MAT s18 / s20 / s22, Erdos-Renyi 2^18 x 16 and
// 2^20 x 8, 1024^2 / 2048^2 / 4096^2 grids, a pack of 64 ER graphs):
//   - bounded small degree (every out-degree <= kClaimMaxDeg: grids,
//     road-like graphs, thousands of thin levels): the claim-word form (grid
//     2048^2: 25.9 ms, list 57.4, sliced 122.9);
//   - skewed degrees (the largest out-degree at least kSlSkew x the average:
//     hubs) on 2^17 <= n <= 2^22: the sliced form (R-MAT s20: 0.42 ms, list
//     0.72);
//   - otherwise the list form (ER 2^18 x 16: 0.29 ms, sliced 0.57; the ER
//     pack: 1.00 ms, sliced 2.74).
constexpr int32_t kSlMinAuto = 1 << 17;
constexpr uint32_t kClaimMaxDeg = 8;
constexpr uint64_t kSlSkew = 16;

// Thin: every out-degree at most kClaimMaxDeg.
bool thin_graph(const bfs_graph *g) { return g->max_deg <= kClaimMaxDeg; }

bool skewed_graph(const bfs_graph *g) {
    return (uint64_t)g->max_deg * (uint64_t)g->n >= kSlSkew * (uint64_t)g->nnz;
}

bool sliced_applies(const bfs_graph *g, const RunCfg &c, const bfs_run_options *opt) {
    const uint32_t impl = opt ? opt->push_impl : BFS_PUSH_AUTO;
    if (c.policy != kPush || g->sl_S == 0 || c.loop == BFS_LOOP_PERSISTENT) return false;
    return impl == BFS_PUSH_SLICED ||
           (impl == BFS_PUSH_AUTO && g->n >= kSlMinAuto && skewed_graph(g) && !thin_graph(g));
}

bool claim_applies(const bfs_graph *g, const RunCfg &c, const bfs_run_options *opt) {
    const uint32_t impl = opt ? opt->push_impl : BFS_PUSH_AUTO;
    if (impl == BFS_PUSH_CLAIM) return true;
    return impl == BFS_PUSH_AUTO && c.policy == kPush && c.loop == BFS_LOOP_HOST && thin_graph(g);
}

// Many sources on one graph as claim-word searches (each source its own
// words, all in lockstep) instead of the 64-per-word multi-source kernels:
// asked for (push_impl CLAIM), or the automatic choice for the push on a thin
// graph beyond the sliced form's size limit - its levels are too small for
// the multi-source kernels' two grid-wide launches per level (4096^2 grid, 16
// sources: 33 us per level there).
bool claim_batch_applies(const bfs_graph *g, const bfs_run_options *opt) {
    const uint32_t impl = opt ? opt->push_impl : BFS_PUSH_AUTO;
    const uint32_t pol = opt ? opt->variant : kPush;
    const uint32_t loop = opt ? opt->loop_mode : BFS_LOOP_HOST;
    if (impl == BFS_PUSH_CLAIM) return true;
    return impl == BFS_PUSH_AUTO && pol == kPush && loop == BFS_LOOP_HOST && thin_graph(g) && g->sl_S == 0;
}

// Queries on different graphs: the list form over the graphs packed into one
// block-diagonal graph (one search from one root per block), unless a graph
// is thin (its many thin levels suit the claim-word form) or the claim-word
// form is asked for.  Measured on 64 Erdos-Renyi graphs (2^10-2^18 vertices,
// 44.8 M entries): the claim-word call 1.51 ms, the same graphs packed by the
// caller and searched from 64 roots by the list form 1.01 ms.
struct PackLayout {
    size_t q, ptr, idx, level, parent, roots, ws, total;
    uint64_t V, E, pad_end;
};

PackLayout pack_layout(const ClaimQuery *qs, int32_t nq) {
    PackLayout L{};
    for (int32_t q = 0; q < nq; ++q) {
        L.V += (uint64_t)qs[q].g->n;
        L.E += qs[q].g->nnz;
    }
    L.pad_end = ((L.E + 3) & ~uint64_t(3)) + 4;           // as the graphs' own padded lists
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.q = take((size_t)nq * sizeof(PackQuery));
    L.ptr = take((size_t)(L.V + 1) * 4);
    L.idx = take((size_t)L.pad_end * 4);
    L.level = take((size_t)L.V * 4);
    L.parent = take((size_t)L.V * 4);
    L.roots = take((size_t)nq * 4);
    L.ws = off;
    off += ws_layout((int32_t)std::min<uint64_t>(L.V, 0x7FFFFFFFull),
                     (uint32_t)std::min<uint64_t>(L.E, 0xFFFFFFFFull), kHeavyFloor).total;
    L.total = align256(off);
    return L;
}

bool packed_list_applies(const ClaimQuery *qs, int32_t nq, const bfs_run_options *opt) {
    const uint32_t impl = opt ? opt->push_impl : BFS_PUSH_AUTO;
    if (impl == BFS_PUSH_LIST) return true;
    if (impl != BFS_PUSH_AUTO) return false;
    for (int32_t q = 0; q < nq; ++q)
        if (thin_graph(qs[q].g)) return false;
    return true;
}

bfs_status run_packed_list(const ClaimQuery *qs, int32_t nq, void *workspace, size_t ws_bytes, hipStream_t s,
                           int cus, bfs_run_options *opt) {
    const PackLayout L = pack_layout(qs, nq);
    if (L.V > 0x7FFFFFFFull || L.E > 0xFFFFFFF0ull)
        return fail(BFS_EINVAL, "the queries hold %llu vertices and %llu entries (at most 2^31 - 1 and 2^32 - 16)",
                    (unsigned long long)L.V, (unsigned long long)L.E);
    if (ws_bytes < L.total) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    char *b = (char *)workspace;
    std::vector<PackQuery> hq((size_t)nq);
    std::vector<int32_t> roots((size_t)nq);
    uint32_t base = 0, ebase = 0, max_n = 0, max_nnz = 0, max_deg = 0;
    for (int32_t q = 0; q < nq; ++q) {
        const bfs_graph *g = qs[q].g;
        hq[(size_t)q] = PackQuery{g->out_ptr, g->out_idx, qs[q].level, qs[q].parent, base, (uint32_t)g->n, ebase,
                                  g->nnz};
        roots[(size_t)q] = (int32_t)base + qs[q].source;
        base += (uint32_t)g->n;
        ebase += g->nnz;
        max_n = std::max(max_n, (uint32_t)g->n);
        max_nnz = std::max(max_nnz, g->nnz);
        max_deg = std::max(max_deg, g->max_deg);
    }
    PackParams PP{};
    PP.q = (const PackQuery *)(b + L.q);
    PP.nq = (uint32_t)nq;
    PP.max_n = max_n;
    PP.max_nnz = max_nnz;
    PP.E = (uint32_t)L.E;
    PP.pad_end = (uint32_t)L.pad_end;
    PP.ptr = (int32_t *)(b + L.ptr);
    PP.idx = (int32_t *)(b + L.idx);
    PP.level = (const int32_t *)(b + L.level);
    PP.parent = (const int32_t *)(b + L.parent);
    int32_t *roots_dev = (int32_t *)(b + L.roots);
    HIP_TRY(hipMemcpyAsync(b + L.q, hq.data(), hq.size() * sizeof(PackQuery), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(roots_dev, roots.data(), roots.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_pack(PP, s));
    // the packed graph for the list form's kernels (push only: no CSC)
    bfs_graph T;
    T.n = (int32_t)L.V;
    T.nnz = (uint32_t)L.E;
    T.max_deg = max_deg;
    T.directed = true;
    T.device = qs[0].g->device;
    T.cus = cus;
    T.out_ptr = PP.ptr;
    T.out_idx = PP.idx;
    RunCfg c{};
    bfs_status st = resolve_cfg(&T, opt, c);
    LevelParams P;
    uint32_t levels = 0;
    if (st == BFS_OK) st = make_params(&T, (int32_t *)PP.level, (int32_t *)PP.parent, c, b + L.ws, false, P);
    if (st == BFS_OK && launch_init(P, nq, roots_dev, -1, s) != hipSuccess) st = fail(BFS_EHIP, "init launch failed");
    if (st == BFS_OK) st = run_levels(&T, P, c, s, levels, opt);
    if (st == BFS_OK && launch_unpack(PP, s) != hipSuccess) st = fail(BFS_EHIP, "unpack launch failed");
    for (hipEvent_t e : T.events) (void)hipEventDestroy(e);   // per-launch timing, if it ran
    if (st != BFS_OK) return st;
    if (opt) {
        opt->levels = levels;
        opt->push_used = BFS_PUSH_LIST;
    }
    return BFS_OK;
}

bfs_status check_push_impl(const bfs_graph *g, const RunCfg &c, const bfs_run_options *opt) {
    const uint32_t impl = opt ? opt->push_impl : BFS_PUSH_AUTO;
    if (impl > BFS_PUSH_CLAIM) return fail(BFS_EINVAL, "unknown push_impl %u", impl);
    if (impl == BFS_PUSH_CLAIM && (c.policy != kPush || c.loop != BFS_LOOP_HOST))
        return fail(BFS_EINVAL, "the claim-word push needs variant PUSH and the host loop");
    if (impl == BFS_PUSH_SLICED && !sliced_applies(g, c, opt))
        return fail(BFS_EINVAL, "the sliced push needs variant PUSH, the host or graph loop and "
                                "n <= %u (n = %d)", bfsi::kSlMaxSlices * bfsi::kSlMaxSliceWords * 32u, g->n);
    return BFS_OK;
}

SlParams make_sl_params(bfs_graph *g, int32_t *level, int32_t *parent, void *ws, bool trace) {
    const SlLayout L = sl_layout(g->sl_S * g->sl_sw);
    char *b = (char *)ws;
    SlParams P{};
    P.n = g->n;
    P.nnz = g->nnz;
    P.S = g->sl_S;
    P.sw = g->sl_sw;
    P.words = g->sl_S * g->sl_sw;
    P.streams = sl_grid(g) / g->sl_S;
    P.seg = g->sl_seg;
    P.occ = g->sl_occ;
    P.out_idx4 = (const int4 *)g->out_idx;
    P.in_ptr = g->directed ? g->in_ptr : nullptr;
    P.in_idx = g->in_idx;
    P.chunks = g->sl_chunks;
    for (uint32_t i = 0; i <= bfsi::kSlMaxSlices; ++i) P.chunk_off[i] = g->sl_chunk_off[i];
    P.level = level;
    P.parent = parent;
    P.vb[0] = (uint32_t *)(b + L.vb0);
    P.vb[1] = (uint32_t *)(b + L.vb1);
    P.cb[0] = (uint32_t *)(b + L.c0);
    P.cb[1] = (uint32_t *)(b + L.c1);
    P.cb[2] = (uint32_t *)(b + L.c2);
    P.cb[3] = (uint32_t *)(b + L.c3);
    P.st = (SlState *)(b + L.state);
    P.trace = trace ? (DevLevelRec *)(b + L.trace) : nullptr;
    return P;
}

// A search (single root, or roots_dev with nroots) by the sliced push.
bfs_status run_sliced(bfs_graph *g, int32_t source, int32_t nroots, const int32_t *roots_dev,
                      int32_t *level, int32_t *parent, const RunCfg &c, void *ws, hipStream_t s,
                      bfs_run_options *opt) {
    HostSlot *hs = nullptr;
    bfs_status st = host_slot(hs);
    if (st != BFS_OK) return st;
    SlParams P = make_sl_params(g, level, parent, ws, opt && opt->trace != nullptr);
    P.host_status = hs->d;
    hs->h[0] = 0;
    hs->h[1] = 1;
    st = timed_init(g, opt, s, [&]() { return launch_sl_init(P, nroots, roots_dev, source, s); });
    if (st != BFS_OK) return st;
    const uint32_t grid = sl_grid(g);
    LoopKey key;
    key.kind = 1;
    key.ws = P.st; key.level = level; key.parent = parent; key.grid = grid;
    key.levels = c.per_sync; key.trace = (const void *)P.trace; key.slot = (const void *)P.host_status;
    uint32_t levels = 0;
    std::vector<float> times;
    const SlParams Pc = P;
    st = level_loop(g, key, c.loop, s, hs, [&Pc, grid](hipStream_t st_) { return launch_sl_level(Pc, grid, st_); },
                    levels, times, opt);
    if (st != BFS_OK) return st;
    if (opt) opt->levels = levels;
    return read_trace(P.trace, levels, times, opt, s);
}

}  // namespace

extern "C" {

const char *bfs_status_string(bfs_status s) {
    switch (s) {
        case BFS_OK: return "ok";
        case BFS_EINVAL: return "invalid argument";
        case BFS_ERANGE: return "source vertex out of range";
        case BFS_ECSR: return "malformed CSR/CSC input";
        case BFS_ENOMEM: return "out of memory";
        case BFS_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *bfs_last_error_detail(void) { return g_detail.c_str(); }

bfs_status bfs_graph_create(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                            const int32_t *in_ptr, const int32_t *in_idx, uint32_t flags,
                            void *hip_stream, bfs_graph **out) {
    (void)hip_stream;
    if (!out) return fail(BFS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n <= 0) return fail(BFS_EINVAL, "n = %d must be positive", n);
    if (!out_ptr || !out_idx) return fail(BFS_EINVAL, "out_ptr/out_idx is NULL");
    if ((in_ptr == nullptr) != (in_idx == nullptr))
        return fail(BFS_EINVAL, "in_ptr and in_idx must both be given or both be NULL");
    if (flags & ~(uint32_t)(BFS_DIRECTED | BFS_INPUT_ON_DEVICE | BFS_VALIDATE_TRANSPOSE |
                            BFS_MS_DEGREE_ORDER | BFS_MS_NO_DEGREE_ORDER))
        return fail(BFS_EINVAL, "unknown flags 0x%x", flags);
    if ((flags & BFS_MS_DEGREE_ORDER) && (flags & BFS_MS_NO_DEGREE_ORDER))
        return fail(BFS_EINVAL, "BFS_MS_DEGREE_ORDER and BFS_MS_NO_DEGREE_ORDER together");
    const bool directed = (flags & BFS_DIRECTED) != 0;
    const bool on_dev = (flags & BFS_INPUT_ON_DEVICE) != 0;
    if (!directed && in_ptr) return fail(BFS_EINVAL, "a CSC is only accepted with BFS_DIRECTED");

    std::vector<int32_t> ptr, idx, iptr, iidx;
    try {
        ptr.resize((size_t)n + 1);
        if (on_dev) {
            HIP_TRY(hipMemcpy(ptr.data(), out_ptr, ptr.size() * 4, hipMemcpyDeviceToHost));
        } else {
            std::memcpy(ptr.data(), out_ptr, ptr.size() * 4);
        }
        if (ptr[0] != 0) return fail(BFS_ECSR, "CSR: ptr[0] = %d, expected 0", ptr[0]);
        for (int32_t v = 0; v < n; ++v)
            if (ptr[v + 1] < ptr[v]) return fail(BFS_ECSR, "CSR: ptr decreases at %d", v);
        idx.resize((size_t)ptr[n]);
        if (on_dev) {
            if (!idx.empty()) HIP_TRY(hipMemcpy(idx.data(), out_idx, idx.size() * 4, hipMemcpyDeviceToHost));
        } else if (!idx.empty()) {
            std::memcpy(idx.data(), out_idx, idx.size() * 4);
        }
        bfs_status st = validate_csr(n, ptr.data(), idx.data(), "CSR");
        if (st != BFS_OK) return st;
        sort_rows(n, ptr, idx);
        if (directed) {
            if (in_ptr) {
                iptr.resize((size_t)n + 1);
                if (on_dev) HIP_TRY(hipMemcpy(iptr.data(), in_ptr, iptr.size() * 4, hipMemcpyDeviceToHost));
                else std::memcpy(iptr.data(), in_ptr, iptr.size() * 4);
                if (iptr[0] != 0) return fail(BFS_ECSR, "CSC: ptr[0] = %d, expected 0", iptr[0]);
                for (int32_t v = 0; v < n; ++v)
                    if (iptr[v + 1] < iptr[v]) return fail(BFS_ECSR, "CSC: ptr decreases at %d", v);
                if (iptr[n] != ptr[n])
                    return fail(BFS_ECSR, "CSC has %d entries, CSR has %d", iptr[n], ptr[n]);
                iidx.resize((size_t)iptr[n]);
                if (on_dev) {
                    if (!iidx.empty()) HIP_TRY(hipMemcpy(iidx.data(), in_idx, iidx.size() * 4, hipMemcpyDeviceToHost));
                } else if (!iidx.empty()) {
                    std::memcpy(iidx.data(), in_idx, iidx.size() * 4);
                }
                st = validate_csr(n, iptr.data(), iidx.data(), "CSC");
                if (st != BFS_OK) return st;
                sort_rows(n, iptr, iidx);
                if (flags & BFS_VALIDATE_TRANSPOSE) {
                    std::vector<int32_t> tp, ti;
                    transpose(n, ptr, idx, tp, ti);
                    if (tp != iptr || ti != iidx) return fail(BFS_ECSR, "CSC is not the transpose of the CSR");
                }
            } else {
                transpose(n, ptr, idx, iptr, iidx);
            }
        }
    } catch (const std::bad_alloc &) {
        return fail(BFS_ENOMEM, "host allocation failed");
    }

    bfs_graph *g = new (std::nothrow) bfs_graph();
    if (!g) return fail(BFS_ENOMEM, "host allocation failed");
    g->n = n;
    g->nnz = (uint32_t)ptr[n];
    for (int32_t v = 0; v < n; ++v) g->max_deg = std::max<uint32_t>(g->max_deg, (uint32_t)(ptr[v + 1] - ptr[v]));
    g->directed = directed;
    if (hipGetDevice(&g->device) != hipSuccess) { delete g; return fail(BFS_EHIP, "hipGetDevice failed"); }
    if (hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess)
        g->cus = 0;                           // launch sizes then assume 256 compute units
    bfs_status st = upload(&g->out_ptr, ptr.data(), ptr.size(), g->bytes);
    if (st == BFS_OK) st = upload_padded(&g->out_idx, idx, g->bytes);
    if (st == BFS_OK && directed) {
        st = upload(&g->in_ptr, iptr.data(), iptr.size(), g->bytes);
        if (st == BFS_OK) st = upload(&g->in_idx, iidx.data(), iidx.size(), g->bytes);
    } else if (st == BFS_OK) {
        g->in_ptr = g->out_ptr;
        g->in_idx = g->out_idx;
    }
    try {
        if (st == BFS_OK) st = build_long(n, ptr, &g->lo, &g->lomap, g->nlo, g->nlo_chunks, g->bytes);
        if (st == BFS_OK) st = build_slices(g, ptr, idx);
        if (st == BFS_OK && directed) {
            st = build_long(n, iptr, &g->li, &g->limap, g->nli, g->nli_chunks, g->bytes);
        } else if (st == BFS_OK) {
            g->li = g->lo;
            g->limap = g->lomap;
            g->nli = g->nlo;
            g->nli_chunks = g->nlo_chunks;
        }
        if (st == BFS_OK) st = build_rest(n, directed ? iptr : ptr, &g->lirest, g->bytes);
        // automatic: graphs whose masks outgrow an XCD's L2 (2^19+ vertices)
        // and whose degrees are skewed (no locality of their own to lose)
        const bool keep_order = (flags & BFS_MS_DEGREE_ORDER) ||
                                (!(flags & BFS_MS_NO_DEGREE_ORDER) && n >= (1 << 19) && skewed_graph(g));
        if (st == BFS_OK && keep_order)
            st = directed ? build_degree_order(g, ptr, idx, iptr, iidx) : build_degree_order(g, ptr, idx, ptr, idx);
    } catch (const std::bad_alloc &) {
        st = fail(BFS_ENOMEM, "host allocation failed");
    }
    if (st != BFS_OK) {
        std::string keep = g_detail;
        free_graph(g);
        g_detail = keep;
        return st;
    }
    *out = g;
    return BFS_OK;
}

bfs_status bfs_graph_destroy(bfs_graph *g) {
    free_graph(g);
    return BFS_OK;
}

bfs_status bfs_graph_info(const bfs_graph *g, int32_t *n, int64_t *nnz, int32_t *directed,
                          size_t *device_bytes) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (directed) *directed = g->directed ? 1 : 0;
    if (device_bytes) *device_bytes = g->bytes;
    return BFS_OK;
}

size_t bfs_workspace_size(const bfs_graph *g, int32_t num_queries, uint32_t run_flags) {
    if (!g || num_queries <= 0 || (run_flags & ~(uint32_t)BFS_WS_CLAIM) != 0) return 0;
    const size_t single = ws_single(g);
    if (num_queries == 1) return single;
    size_t need = std::max(single, ms_layout(g->n, num_queries).total);
    // thin graphs (or when asked): room for the claim-word batch too (see
    // claim_batch_applies)
    if ((thin_graph(g) && g->sl_S == 0) || (run_flags & BFS_WS_CLAIM))
        need = std::max(need, cw_layout((uint64_t)g->n * (uint64_t)num_queries,
                                        (uint64_t)g->nnz * (uint64_t)num_queries, (uint32_t)num_queries).total);
    return need;
}

bfs_status bfs_run(bfs_graph *g, int32_t source, int32_t *level, int32_t *parent,
                   bfs_run_options *opt, void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (!level || !parent || !workspace) return fail(BFS_EINVAL, "level/parent/workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(BFS_EINVAL, "workspace must be 256-byte aligned");
    if (source < 0 || source >= g->n) return fail(BFS_ERANGE, "source %d outside [0, %d)", source, g->n);
    const size_t need = bfs_workspace_size(g, 1, 0);
    if (ws_bytes < need) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    RunCfg c{};
    bfs_status st = resolve_cfg(g, opt, c);
    if (st != BFS_OK) return st;
    if (c.policy == kPull || c.policy == kHeuristic || c.policy == kLearned) {
        if (!g->in_ptr) return fail(BFS_EINVAL, "pull needs the CSC");
    }
    st = check_push_impl(g, c, opt);
    if (st != BFS_OK) return st;
    const uint32_t count = opt ? opt->count_atomics : 0u;
    if (count > 2u) return fail(BFS_EINVAL, "count_atomics = %u (0, 1 or 2)", count);
    if (count && (claim_applies(g, c, opt) || sliced_applies(g, c, opt)))
        return fail(BFS_EINVAL, "count_atomics needs the list form of the push (push_impl LIST)");
    hipStream_t s = (hipStream_t)hip_stream;
    if (claim_applies(g, c, opt)) {
        if (opt) opt->push_used = BFS_PUSH_CLAIM;
        const ClaimQuery q{g, source, level, parent};
        return run_claim(&q, 1, workspace, ws_bytes, s, g->cus, opt);
    }
    const bool sliced = sliced_applies(g, c, opt);
    if (opt) opt->push_used = sliced ? BFS_PUSH_SLICED : BFS_PUSH_LIST;
    if (sliced)
        return run_sliced(g, source, 1, nullptr, level, parent, c, workspace, s, opt);
    LevelParams P;
    make_params(g, level, parent, c, workspace, opt && opt->trace != nullptr, P);
    if (count) {                                    // zeroed by the init launch
        P.atomics = &P.st->atomics;
        P.no_preread = count == 2u ? 1u : 0u;
    }
    st = timed_init(g, opt, s, [&]() { return launch_init(P, 1, nullptr, source, s); });
    if (st != BFS_OK) return st;
    uint32_t levels = 0;
    st = run_levels(g, P, c, s, levels, opt);
    if (st != BFS_OK) return st;
    if (opt) opt->levels = levels;
    if (count) {
        unsigned long long a = 0;
        HIP_TRY(hipMemcpyAsync(&a, P.atomics, sizeof(a), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        opt->atomics = a;
    }
    return BFS_OK;
}

}  // extern "C"

// Multi-root search used by the batch entry point for block-diagonal packs and
// by the serving loop: roots must lie in distinct components.
extern "C" bfs_status bfs_run_roots(bfs_graph *g, int32_t nroots, const int32_t *roots_host,
                                    int32_t *level, int32_t *parent, bfs_run_options *opt,
                                    void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (!level || !parent || !workspace || !roots_host) return fail(BFS_EINVAL, "NULL argument");
    if (nroots <= 0 || nroots > g->n) return fail(BFS_EINVAL, "nroots = %d outside [1, n]", nroots);
    if (((uintptr_t)workspace & 255) != 0) return fail(BFS_EINVAL, "workspace must be 256-byte aligned");
    const size_t base = ws_single(g);
    const size_t need = base + align256((size_t)nroots * 4);
    if (ws_bytes < need) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    std::vector<char> seen((size_t)g->n, 0);
    for (int32_t r = 0; r < nroots; ++r) {
        const int32_t v = roots_host[r];
        if (v < 0 || v >= g->n) return fail(BFS_ERANGE, "root %d outside [0, %d)", v, g->n);
        if (seen[v]) return fail(BFS_EINVAL, "root %d given twice", v);
        seen[v] = 1;
    }
    RunCfg c{};
    bfs_status st = resolve_cfg(g, opt, c);
    if (st != BFS_OK) return st;
    st = check_push_impl(g, c, opt);
    if (st != BFS_OK) return st;
    if (opt && opt->push_impl == BFS_PUSH_CLAIM)
        return fail(BFS_EINVAL, "the claim-word push runs single searches and bfs_run_batch, not several roots");
    if (opt && opt->count_atomics) return fail(BFS_EINVAL, "count_atomics is for bfs_run");
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t *roots_dev = (int32_t *)((char *)workspace + base);
    HIP_TRY(hipMemcpyAsync(roots_dev, roots_host, (size_t)nroots * 4, hipMemcpyHostToDevice, s));
    const bool sliced = sliced_applies(g, c, opt);
    if (opt) opt->push_used = sliced ? BFS_PUSH_SLICED : BFS_PUSH_LIST;
    if (sliced)
        return run_sliced(g, -1, nroots, roots_dev, level, parent, c, workspace, s, opt);
    LevelParams P;
    make_params(g, level, parent, c, workspace, opt && opt->trace != nullptr, P);
    HIP_TRY(launch_init(P, nroots, roots_dev, -1, s));
    uint32_t levels = 0;
    st = run_levels(g, P, c, s, levels, opt);
    if (st != BFS_OK) return st;
    if (opt) opt->levels = levels;
    return BFS_OK;
}

extern "C" size_t bfs_roots_workspace_size(const bfs_graph *g, int32_t nroots) {
    if (!g || nroots <= 0) return 0;
    return ws_single(g) + align256((size_t)nroots * 4);
}

// A multi-source pull level tests the union-frontier bitmap before each mask
// gather when the frontier holds at most n >> kMsFbitsShift vertices (on
// denser frontiers the extra dependent load costs more than it skips).
constexpr uint32_t kMsFbitsShift = 6;

// From level kMsGroupFrom on, push levels are launched kMsGroupLevels at a
// time between two reads of the progress report (deep graphs: the round trip
// per level would otherwise dominate); levels launched past the end of the
// search find an empty frontier and change nothing.
constexpr uint32_t kMsGroupFrom = 16;
constexpr uint32_t kMsGroupLevels = 8;

// A multi-source level's record when tracing: the direction it ran in and,
// where the host read it before the level, the union frontier's size.
static void ms_note(bfs_run_options *opt, uint32_t k, int32_t variant, uint32_t frontier) {
    if (!opt || !opt->trace || k >= opt->trace_capacity) return;
    bfs_level_record &r = opt->trace[k];
    r = bfs_level_record{};
    r.level = (int32_t)k;
    r.variant = variant;
    r.frontier = frontier;
}

// The range-ordered pull runs on pull levels whose union frontier holds more
// than n >> kMsRangeShift vertices, when a caller asks for it (ms_ranges > 1,
// one mask word).  It is off by default: on R-MAT s22 with 64 sources the
// batch took 6.14 ms in one pass over the lists and 6.52 / 7.73 / 9.20 /
// 12.27 ms in 2 / 4 / 8 / 16 ranges - each pass's per-row work (the row's
// pointers, cursor and visited word, its step through the wave's write loop)
// costs more than the L2-resident gathers save.
constexpr uint32_t kMsRangeShift = 4;

static uint32_t ms_ranges(int32_t, uint32_t) { return 1; }

// The multi-source parameter block over `workspace` (layout ms_layout), the
// per-source output pointers and the sources uploaded on s.  level / parent:
// per-source arrays (staged results), or with vm_level / vm_parent set, the
// caller's vertex-major arrays, written in place.
static bfs_status ms_prepare(bfs_graph *g, int32_t nq, const int32_t *sources,
                             int32_t *const *level, int32_t *const *parent, void *workspace,
                             hipStream_t s, int32_t *vm_level, int32_t *vm_parent, uint32_t grid,
                             MsLevel &p, HostSlot *&hs) {
    const bool vm = vm_level != nullptr;
    const MsLayout L = ms_layout(g->n, nq, !vm);
    char *b = (char *)workspace;
    p = MsLevel{};
    p.n = g->n;
    p.W = (uint32_t)(((size_t)nq + 63) / 64);
    p.nq = (uint32_t)nq;
    p.out_ptr = g->out_ptr;
    p.out_idx = g->out_idx;
    p.in_ptr = g->in_ptr;
    p.in_idx = g->in_idx;
    p.vis = (unsigned long long *)(b + L.vis);
    p.m[0] = (unsigned long long *)(b + L.m0);
    p.m[1] = (unsigned long long *)(b + L.m1);
    p.m[2] = (unsigned long long *)(b + L.m2);
    p.fq[0] = (int32_t *)(b + L.f0);
    p.fq[1] = (int32_t *)(b + L.f1);
    p.fq[2] = (int32_t *)(b + L.f2);
    p.flag = (uint32_t *)(b + L.flag);
    p.cnt = (uint32_t *)(b + L.cnt);
    p.mstat = (unsigned long long *)(b + L.mstat);
    p.fbits = (unsigned long long *)(b + L.fbits);
    p.rlist[0] = (int32_t *)(b + L.rl0);
    p.rlist[1] = (int32_t *)(b + L.rl1);
    p.rcnt = (uint32_t *)(b + L.rcnt);
    p.rcur = (int32_t *)(b + L.rcur);
    p.rp_ranges = ms_ranges(g->n, p.W);
    p.wide_steps = ((uint64_t)g->nnz < 8ull * (uint64_t)g->n) ? 1u : 0u;
    p.lo = g->lo;
    p.li = g->li;
    p.lomap = g->lomap;
    p.limap = g->limap;
    p.nlo_chunks = g->nlo_chunks;
    p.nli = g->nli;
    p.nli_chunks = g->nli_chunks;
    p.lirest = g->lirest;
    p.orig = p.pos = p.ent = nullptr;
    // the degree-ordered copy (undirected: one list set serves both ways); a
    // directed graph's only for batches of more than one mask word (directed
    // R-MAT s20: 16 sources 1.08 ms with it, 0.92 without; 256 sources 4.35
    // against 4.62 ms)
    if (g->do_ptr && (!g->directed || p.W > 1)) {
        p.out_ptr = p.in_ptr = g->do_ptr;
        p.out_idx = p.in_idx = g->do_idx;
        p.ent = p.out_ent = g->do_ent;
        p.orig = g->do_orig;
        p.pos = g->do_pos;
        p.lo = p.li = g->do_long;
        p.lomap = p.limap = g->do_map;
        p.nlo_chunks = p.nli_chunks = g->do_nchunks;
        p.nli = g->do_nlong;
        p.lirest = g->do_rest;
        p.row_chunks = g->do_rows;
        p.nrow_chunks = g->do_nrows;
        if (g->directed) {            // the out-lists for the push
            p.out_ptr = g->do_optr;
            p.out_idx = g->do_oidx;
            p.out_ent = g->do_oent;
            p.lo = g->do_olong;
            p.lomap = g->do_omap;
            p.nlo_chunks = g->do_onchunks;
        }
        // the library's staged rows by label (written in label order, k_ms_out
        // maps them back); the caller's vertex-major arrays by caller id
        p.stage_labels = vm ? 0u : 1u;
    }
    p.slev = vm ? vm_level : (int32_t *)(b + L.slev);
    p.spar = vm ? (uint32_t *)vm_parent : (uint32_t *)(b + L.spar);
    p.fill_levels = vm ? 1u : 0u;
    p.level = (int32_t *const *)(b + L.lptr);
    p.parent = (int32_t *const *)(b + L.pptr);
    p.sources = (const int32_t *)(b + L.src);
    bfs_status st = host_slot(hs);
    if (st != BFS_OK) return st;
    p.host_status = hs->d;
    if (!vm) {
        HIP_TRY(hipMemcpyAsync(b + L.lptr, level, (size_t)nq * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b + L.pptr, parent, (size_t)nq * 8, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(b + L.src, sources, (size_t)nq * 4, hipMemcpyHostToDevice, s));
    // the long rows' later chunks in a launch of their own once they outnumber
    // the grid's waves twice over (then skipping those a row's first chunk
    // has settled saves whole rounds; below that the extra launch costs more)
    p.long_split = ((uint64_t)(g->nli_chunks - g->nli) > 2ull * grid * 4u) ? 1u : 0u;
    return BFS_OK;
}

// One multi-source level k in the pull form (frontier = the union frontier's
// size, which decides whether the pull tests the frontier bitmap first) or in
// the push form.
static hipError_t ms_level(MsLevel &p, uint32_t k, bool pull, uint32_t frontier, uint32_t grid,
                           hipStream_t s) {
    hipError_t e;
    if (pull && p.rp_ranges > 1 && ((uint64_t)frontier << kMsRangeShift) > (uint64_t)p.n) {
        // a dense union frontier: the rows' in-lists one vertex range at a
        // time, each range's masks resident in the XCDs' L2
        for (uint32_t r = 0; r < p.rp_ranges; ++r)
            if ((e = launch_ms_rpull(p, k, r, grid, s)) != hipSuccess) return e;
        return launch_ms(p, 5, k, grid, s);
    }
    if (pull) {
        // a sparse union frontier: the pull tests its bitmap before each
        // mask gather (most in-neighbours are then skipped on chip)
        p.use_fbits = ((uint64_t)frontier << kMsFbitsShift) <= (uint64_t)p.n ? 1u : 0u;
        if (p.use_fbits && (e = launch_ms(p, 8, k, grid, s)) != hipSuccess) return e;
        if ((e = launch_ms(p, 4, k, grid, s)) != hipSuccess) return e;
        if (p.long_split && (e = launch_ms(p, 9, k, grid, s)) != hipSuccess) return e;
        if ((e = launch_ms(p, 6, k, grid, s)) != hipSuccess) return e;
        return launch_ms(p, 5, k, grid, s);
    }
    if ((e = launch_ms(p, 2, k, grid, s)) != hipSuccess) return e;
    return launch_ms(p, 3, k, grid, s);
}

// The multi-source parameters over the caller's vertex order instead of the
// degree-ordered copy.
static void ms_caller_order(const bfs_graph *g, MsLevel &p) {
    p.out_ptr = g->out_ptr;
    p.out_idx = g->out_idx;
    p.in_ptr = g->in_ptr;
    p.in_idx = g->in_idx;
    p.orig = p.pos = p.ent = p.out_ent = nullptr;
    p.row_chunks = nullptr;
    p.nrow_chunks = 0;
    p.stage_labels = 0;
    p.lo = g->lo;
    p.li = g->li;
    p.lomap = g->lomap;
    p.limap = g->limap;
    p.nlo_chunks = g->nlo_chunks;
    p.nli = g->nli;
    p.nli_chunks = g->nli_chunks;
    p.lirest = g->lirest;
}

// Multi-source launch size: 8 workgroups per compute unit, up to 48 on graphs
// of more than 2,730 vertices per compute unit (three workgroups per 1,024
// vertices: R-MAT s22, 64 sources, with the degree-ordered copy 4.99 ms at 48
// per compute unit, 5.00 at 24, 5.08 at 32, 5.11 at 64; 6.25 ms at 8 before
// that copy), except on thin graphs, whose thousands of small levels pay for
// every workgroup of every launch (4096^2 grid, 16 sources: 239 ms at 8 per
// compute unit, 272 ms at 32).
static uint32_t ms_grid(const bfs_graph *g, const bfs_run_options *opt) {
    if (opt && opt->grid_blocks) return opt->grid_blocks;
    const uint32_t cus = (uint32_t)(g->cus > 0 ? g->cus : 256);
    if (thin_graph(g)) return 8u * cus;
    const uint32_t want = (uint32_t)std::min<int64_t>((int64_t)g->n * 3 / 1024, (int64_t)48 * cus);
    return std::max<uint32_t>(8u * cus, want);
}

// All queries on one graph: the multi-source kernels (outputs as ms_prepare).
static bfs_status run_multi_source(bfs_graph *g, int32_t nq, const int32_t *sources,
                                   int32_t *const *level, int32_t *const *parent,
                                   bfs_run_options *opt, void *workspace, hipStream_t s,
                                   int32_t *vm_level = nullptr, int32_t *vm_parent = nullptr) {
    const uint32_t pull_shift = (opt && opt->ms_pull_shift) ? opt->ms_pull_shift : 5u;
    if (pull_shift > 31) return fail(BFS_EINVAL, "ms_pull_shift %u above 31", pull_shift);
    if (opt && opt->variant > kShortCircuit) return fail(BFS_EINVAL, "unknown variant %u", opt->variant);
    const uint32_t grid = ms_grid(g, opt);
    if (grid == 0 || grid > 65535) return fail(BFS_EINVAL, "grid_blocks %u outside [1, 65535]", grid);
    if (opt && opt->ms_ranges > 64) return fail(BFS_EINVAL, "ms_ranges %u above 64", opt->ms_ranges);
    MsLevel p;
    HostSlot *hs = nullptr;
    bfs_status st = ms_prepare(g, nq, sources, level, parent, workspace, s, vm_level, vm_parent, grid, p, hs);
    if (st != BFS_OK) return st;
    if (opt && opt->ms_ranges && p.W == 1) p.rp_ranges = opt->ms_ranges;
    if (p.rp_ranges > 1) ms_caller_order(g, p);       // its passes walk lists sorted by label
    // direction per level: HEURISTIC pushes while the union frontier is
    // small and pulls (no atomics) once it holds more than n >> pull_shift
    // vertices; LEARNED takes the network's argmin over push and pull, which
    // a one-wave launch after each level's list leaves in the progress slot
    // (push on every level without a network); PUSH / PULL as forced
    const uint32_t pol = opt ? opt->variant : kPush;
    const bool learned = pol == kLearned && opt->selector != nullptr;
    p.mlp = learned ? opt->selector : nullptr;
    HIP_TRY(launch_ms(p, 0, 0, grid, s));
    HIP_TRY(launch_ms(p, 1, 0, grid, s));
    uint32_t k = 0, frontier = 1, dir = 0;
    if (learned) {
        HIP_TRY(launch_ms(p, 10, 0, grid, s));
        HIP_TRY(hipStreamSynchronize(s));
        dir = hs->h[2];
    }
    for (;; ++k) {
        if ((uint64_t)k > (uint64_t)g->n + 2) return fail(BFS_EHIP, "multi-source loop did not terminate");
        const bool pull = learned ? dir == 1u
                                  : (pol == kPull) || (pol == kHeuristic &&
                                                       ((uint64_t)frontier << pull_shift) > (uint64_t)g->n);
        if (pull) {
            HIP_TRY(ms_level(p, k, true, frontier, grid, s));
            ms_note(opt, k, 1, frontier);
        } else {
            const uint32_t group = (k >= kMsGroupFrom) ? kMsGroupLevels : 1u;
            for (uint32_t i = 0; i < group; ++i) {
                HIP_TRY(ms_level(p, k + i, false, 0, grid, s));
                ms_note(opt, k + i, 0, i == 0 ? frontier : 0u);
            }
            k += group - 1;
        }
        if (learned) HIP_TRY(launch_ms(p, 10, k + 1, grid, s));   // the next level's direction
        bool done = false;
        uint32_t lv = 0;
        st = wait_progress(hs, s, done, lv);
        if (st != BFS_OK) return st;
        if (done) {
            k = lv - 1;                       // the level whose step found nothing
            break;
        }
        frontier = hs->h[1];
        dir = hs->h[2];
    }
    if (vm_level == nullptr) HIP_TRY(launch_ms(p, 7, k, grid, s));   // staged results -> per-source arrays
    if (opt) {
        opt->levels = k + 1;
        opt->trace_count = opt->trace ? std::min<uint32_t>(k + 1, opt->trace_capacity) : 0u;
    }
    return BFS_OK;
}

extern "C" bfs_status bfs_run_batch(int32_t num_queries, bfs_graph *const *graphs,
                                    const int32_t *sources, int32_t *const *level,
                                    int32_t *const *parent, bfs_run_options *opt,
                                    void *workspace, size_t ws_bytes, void *hip_stream) {
    if (num_queries <= 0) return fail(BFS_EINVAL, "num_queries = %d", num_queries);
    if (!graphs || !sources || !level || !parent || !workspace) return fail(BFS_EINVAL, "NULL argument");
    if (((uintptr_t)workspace & 255) != 0) return fail(BFS_EINVAL, "workspace must be 256-byte aligned");
    bool same = true;
    for (int32_t q = 0; q < num_queries; ++q) {
        if (!graphs[q] || !level[q] || !parent[q]) return fail(BFS_EINVAL, "query %d has a NULL pointer", q);
        if (sources[q] < 0 || sources[q] >= graphs[q]->n)
            return fail(BFS_ERANGE, "query %d: source %d outside [0, %d)", q, sources[q], graphs[q]->n);
        same = same && graphs[q] == graphs[0];
    }
    if (same && num_queries > 1 && !claim_batch_applies(graphs[0], opt)) {
        const size_t need = bfs_workspace_size(graphs[0], num_queries, 0);
        if (ws_bytes < need) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return run_multi_source(graphs[0], num_queries, sources, level, parent, opt, workspace,
                                (hipStream_t)hip_stream);
    }
    if (num_queries == 1)
        return bfs_run(graphs[0], sources[0], level[0], parent[0], opt, workspace, ws_bytes, hip_stream);
    // queries on different graphs, or (claim_batch_applies) many on one thin
    // graph: every search at once through the claim-word push, one launch per
    // level (or one narrow launch for many levels) for all of them
    if (opt && opt->variant != kPush) return fail(BFS_EINVAL, "queries on different graphs run the push only");
    if (opt && opt->loop_mode != BFS_LOOP_HOST) return fail(BFS_EINVAL, "queries on different graphs run the host loop");
    std::vector<ClaimQuery> qs((size_t)num_queries);
    int cus = 0;
    for (int32_t q = 0; q < num_queries; ++q) {
        qs[(size_t)q] = ClaimQuery{graphs[q], sources[q], level[q], parent[q]};
        cus = std::max(cus, graphs[q]->cus);
    }
    if (opt && opt->push_impl == BFS_PUSH_SLICED)
        return fail(BFS_EINVAL, "queries on different graphs run the list or the claim-word form");
    if (!same && packed_list_applies(qs.data(), num_queries, opt))
        return run_packed_list(qs.data(), num_queries, workspace, ws_bytes, (hipStream_t)hip_stream, cus, opt);
    if (opt) opt->push_used = BFS_PUSH_CLAIM;
    return run_claim(qs.data(), num_queries, workspace, ws_bytes, (hipStream_t)hip_stream, cus, opt);
}

extern "C" size_t bfs_batch_workspace_size(int32_t num_queries, bfs_graph *const *graphs) {
    if (num_queries <= 0 || !graphs) return 0;
    bool same = true;
    for (int32_t q = 0; q < num_queries; ++q) {
        if (!graphs[q]) return 0;
        same = same && graphs[q] == graphs[0];
    }
    if (same) return bfs_workspace_size(graphs[0], num_queries, 0);   // one query: bfs_run's
    std::vector<ClaimQuery> qs((size_t)num_queries);
    for (int32_t q = 0; q < num_queries; ++q) qs[(size_t)q] = ClaimQuery{graphs[q], 0, nullptr, nullptr};
    // room for either form (push_impl may ask for the other)
    return std::max(claim_workspace(qs.data(), num_queries), pack_layout(qs.data(), num_queries).total);
}

// ---------------------------------------------------------------------------
// selector network and its training data
// ---------------------------------------------------------------------------

extern "C" int32_t bfs_selector_param_count(void) { return kMlpTotal; }

extern "C" bfs_status bfs_selector_forward(const float *weights, const float *features, float *out,
                                           int32_t rows, void *hip_stream) {
    if (!weights || !features || !out || rows < 0) return fail(BFS_EINVAL, "bad selector_forward arguments");
    HIP_TRY(launch_mlp_forward(weights, features, out, rows, (hipStream_t)hip_stream));
    return BFS_OK;
}

extern "C" bfs_status bfs_selector_grad(const float *weights, const float *features, const float *targets,
                                        const float *mask, int32_t rows, float inv_norm, float *grad,
                                        float *loss, void *hip_stream) {
    if (!weights || !features || !targets || !mask || !grad || !loss || rows < 0)
        return fail(BFS_EINVAL, "bad selector_grad arguments");
    HIP_TRY(launch_mlp_grad(weights, features, targets, mask, rows, inv_norm, grad, loss,
                            (hipStream_t)hip_stream));
    return BFS_OK;
}

extern "C" bfs_status bfs_selector_adam(float *weights, float *grad, float *m, float *v, int32_t step,
                                        float lr, void *hip_stream) {
    if (!weights || !grad || !m || !v || step < 1) return fail(BFS_EINVAL, "bad selector_adam arguments");
    HIP_TRY(launch_mlp_adam(weights, grad, m, v, step, lr, (hipStream_t)hip_stream));
    return BFS_OK;
}

extern "C" size_t bfs_profile_snapshot_size(const bfs_graph *g) {
    if (!g) return 0;
    return ws_layout(g->n, g->nnz, kHeavyFloor).total + 2 * align256((size_t)g->n * 4);
}

extern "C" bfs_status bfs_profile_levels(bfs_graph *g, int32_t source, int32_t *level, int32_t *parent,
                                         void *workspace, size_t ws_bytes, void *snapshot,
                                         size_t snap_bytes, int32_t reps, bfs_level_record *records,
                                         uint32_t capacity, uint32_t *count, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (!level || !parent || !workspace || !snapshot || !records || !count)
        return fail(BFS_EINVAL, "NULL argument");
    if (source < 0 || source >= g->n) return fail(BFS_ERANGE, "source %d outside [0, %d)", source, g->n);
    if (((uintptr_t)workspace & 255) != 0 || ((uintptr_t)snapshot & 255) != 0)
        return fail(BFS_EINVAL, "workspace and snapshot must be 256-byte aligned");
    const size_t wsz = ws_layout(g->n, g->nnz, kHeavyFloor).total;
    if (ws_bytes < wsz) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, wsz);
    if (snap_bytes < bfs_profile_snapshot_size(g)) return fail(BFS_EINVAL, "snapshot too small");
    if (reps < 1 || reps > 100) return fail(BFS_EINVAL, "reps %d outside [1, 100]", reps);
    if (!g->in_ptr) return fail(BFS_EINVAL, "pull needs the CSC");
    hipStream_t s = (hipStream_t)hip_stream;
    RunCfg c{};
    bfs_status st = resolve_cfg(g, nullptr, c);
    if (st != BFS_OK) return st;
    c.policy = kPush;
    LevelParams P;
    make_params(g, level, parent, c, workspace, false, P);
    P.maintain_fb = 1;
    P.stats = 1;
    HostSlot *hs = nullptr;
    st = host_slot(hs);
    if (st != BFS_OK) return st;
    P.host_status = hs->d;
    char *snap = (char *)snapshot;
    const size_t nb = (size_t)g->n * 4;
    char *snap_level = snap + wsz;
    char *snap_parent = snap_level + align256(nb);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } guard{e0, e1};
    auto save = [&]() -> bfs_status {
        HIP_TRY(hipMemcpyAsync(snap, workspace, wsz, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(snap_level, level, nb, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(snap_parent, parent, nb, hipMemcpyDeviceToDevice, s));
        return BFS_OK;
    };
    auto restore = [&]() -> bfs_status {
        HIP_TRY(hipMemcpyAsync(workspace, snap, wsz, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(level, snap_level, nb, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(parent, snap_parent, nb, hipMemcpyDeviceToDevice, s));
        return BFS_OK;
    };
    HIP_TRY(launch_init(P, 1, nullptr, source, s));
    BfsState hst;
    uint32_t n_out = 0;
    for (uint32_t k = 0;; ++k) {
        if ((uint64_t)k > (uint64_t)g->n + 2) return fail(BFS_EHIP, "profiling loop did not terminate");
        HIP_TRY(hipMemcpyAsync(&hst, P.st, sizeof(BfsState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const uint32_t slot = hst.level & 3;
        const uint32_t nf = hst.nf[slot] + (uint32_t)hst.heavy[slot];
        if (nf == 0) break;
        st = save();
        if (st != BFS_OK) return st;
        uint32_t fastest = 0;
        float fastest_us = 1e30f;
        for (uint32_t v = 0; v < 3; ++v) {
            float best = 1e30f;
            for (int32_t r = 0; r < reps; ++r) {
                st = restore();
                if (st != BFS_OK) return st;
                LevelParams Pv = P;
                Pv.policy = v;
                HIP_TRY(hipEventRecord(e0, s));
                HIP_TRY(launch_level(Pv, c.grid, s));
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                best = std::min(best, ms * 1000.f);
            }
            if (n_out < capacity) {
                bfs_level_record &o = records[n_out++];
                o.level = (int32_t)k;
                o.variant = (int32_t)v;
                o.frontier = nf;
                o.unvisited = (uint32_t)g->n - hst.visited_cnt;
                o.frontier_edges = hst.sdf[slot];
                o.unvisited_edges = (uint64_t)g->nnz - hst.visited_deg;
                o.time_us = best;
                o.reserved = 0.f;
            }
            if (best < fastest_us) {
                fastest_us = best;
                fastest = v;
            }
        }
        // the search goes on with the fastest form, so that the state later
        // levels start from (e.g. the unvisited list a pull level compacts)
        // is the one a good per-level choice produces
        st = restore();
        if (st != BFS_OK) return st;
        LevelParams Pc = P;
        Pc.policy = fastest;
        HIP_TRY(launch_level(Pc, c.grid, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    *count = n_out;
    return BFS_OK;
}

// ---------------------------------------------------------------------------
// The comparison searches of the Experiments section
// ---------------------------------------------------------------------------

extern "C" size_t bfs_compare_workspace_size(const bfs_graph *g) {
    if (!g) return 0;
    return cmp_layout(g->n).total;
}

extern "C" bfs_status bfs_run_compare(bfs_graph *g, int32_t source, uint32_t method, int32_t *level,
                                      int32_t *parent, void *workspace, size_t ws_bytes,
                                      uint64_t *ops, uint32_t *steps, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (!level || !parent || !workspace) return fail(BFS_EINVAL, "level/parent/workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(BFS_EINVAL, "workspace must be 256-byte aligned");
    if (method > kCmpSpmmspv) return fail(BFS_EINVAL, "unknown comparison method %u", method);
    if (source < 0 || source >= g->n) return fail(BFS_ERANGE, "source %d outside [0, %d)", source, g->n);
    const CmpLayout L = cmp_layout(g->n);
    if (ws_bytes < L.total) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    HostSlot *hs = nullptr;
    bfs_status st0 = host_slot(hs);
    if (st0 != BFS_OK) return st0;
    hipStream_t s = (hipStream_t)hip_stream;
    char *b = (char *)workspace;
    CmpParams P{};
    P.n = g->n;
    P.words = (uint32_t)(((size_t)g->n + 31) / 32);
    P.method = method;
    P.out_ptr = g->out_ptr;
    P.out_idx = g->out_idx;
    P.in_ptr = g->in_ptr;
    P.in_idx = g->in_idx;
    P.lo = g->lo;
    P.li = g->li;
    P.lomap = g->lomap;
    P.limap = g->limap;
    P.nlo_chunks = g->nlo_chunks;
    P.nli_chunks = g->nli_chunks;
    P.level = level;
    P.parent = parent;
    P.y = (unsigned long long *)(b + L.y);
    P.list[0] = (int32_t *)(b + L.l0);
    P.list[1] = (int32_t *)(b + L.l1);
    P.touched = (int32_t *)(b + L.touched);
    P.xb[0] = (uint32_t *)(b + L.x0);
    P.xb[1] = (uint32_t *)(b + L.x1);
    P.st = (CmpState *)(b + L.state);
    P.host_status = hs->d;
    hs->h[0] = 0;
    hs->h[1] = 1;
    const uint32_t grid = (uint32_t)(8 * (g->cus > 0 ? g->cus : 256));
    HIP_TRY(launch_cmp_init(P, source, s));
    // steps are launched eight at a time between progress checks; steps after
    // the one that reaches nothing return at once
    const uint64_t max_steps = (uint64_t)g->n + 2;
    bool done = false;
    for (uint64_t issued = 0; !done; issued += 8) {
        if (issued > max_steps) return fail(BFS_EHIP, "comparison search did not terminate");
        for (int l = 0; l < 8; ++l) HIP_TRY(launch_cmp_step(P, grid, s));
        uint32_t lv = 0;
        bfs_status st = wait_progress(hs, s, done, lv);
        if (st != BFS_OK) return st;
    }
    CmpState hst;
    HIP_TRY(hipMemcpyAsync(&hst, P.st, sizeof hst, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ops) *ops = (uint64_t)hst.ops;
    if (steps) *steps = hst.k;
    return BFS_OK;
}

// ---------------------------------------------------------------------------
// One masked SpMSpV product over a semiring
// ---------------------------------------------------------------------------

extern "C" size_t bfs_spmspv_workspace_size(const bfs_graph *g, int32_t max_nx) {
    if (!g || max_nx < 0) return 0;
    return sp_layout(g->n, max_nx).total;
}

extern "C" bfs_status bfs_masked_spmspv(bfs_graph *g, uint32_t semiring, const int32_t *x_idx,
                                        const uint64_t *x_val, int32_t nx, const uint32_t *row_mask,
                                        const uint32_t *col_mask, uint32_t mask_flags, int32_t *y_idx,
                                        uint64_t *y_val, int32_t *ny, void *workspace, size_t ws_bytes,
                                        void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (semiring > kSrMinSelect) return fail(BFS_EINVAL, "unknown semiring %u", semiring);
    if (nx < 0) return fail(BFS_EINVAL, "nx = %d", nx);
    if (nx > 0 && (!x_idx || !x_val)) return fail(BFS_EINVAL, "x_idx / x_val is NULL");
    if (!y_idx || !y_val || !ny || !workspace) return fail(BFS_EINVAL, "y_idx / y_val / ny / workspace is NULL");
    if (mask_flags & ~3u) return fail(BFS_EINVAL, "unknown mask flags 0x%x", mask_flags);
    if (((uintptr_t)workspace & 255) != 0) return fail(BFS_EINVAL, "workspace must be 256-byte aligned");
    const SpLayout L = sp_layout(g->n, nx);
    if (ws_bytes < L.total) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)hip_stream;
    char *b = (char *)workspace;
    SpParams P{};
    P.n = g->n;
    P.words = (uint32_t)(((size_t)g->n + 31) / 32);
    P.semiring = semiring;
    P.out_ptr = g->out_ptr;
    P.out_idx = g->out_idx;
    P.x_idx = x_idx;
    P.x_val = (const unsigned long long *)x_val;
    P.nx = nx;
    P.row_mask = row_mask;
    P.col_mask = col_mask;
    P.row_comp = (mask_flags & 1u) ? 1u : 0u;
    P.col_comp = (mask_flags & 2u) ? 1u : 0u;
    P.acc = (unsigned long long *)(b + L.acc);
    P.touched = (uint32_t *)(b + L.touched);
    P.items = (SpItem *)(b + L.items);
    P.block_off = (uint32_t *)(b + L.block_off);
    P.st = (SpState *)(b + L.state);
    P.y_idx = y_idx;
    P.y_val = (unsigned long long *)y_val;
    P.ny = (int32_t *)(b + L.ny);
    const uint32_t grid = (uint32_t)(8 * (g->cus > 0 ? g->cus : 256));
    HIP_TRY(launch_spmspv(P, grid, s));
    SpState hst;
    int32_t hny = 0;
    HIP_TRY(hipMemcpyAsync(&hst, P.st, sizeof hst, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hny, P.ny, sizeof hny, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hst.bad) return fail(BFS_ERANGE, "a vector index lies outside [0, %d)", g->n);
    *ny = hny;
    return BFS_OK;
}

// ---------------------------------------------------------------------------
// Many sources with vertex-major outputs
// ---------------------------------------------------------------------------

extern "C" size_t bfs_batch_vm_workspace_size(const bfs_graph *g, int32_t num_sources) {
    if (!g || num_sources <= 0) return 0;
    return ms_layout(g->n, num_sources, false).total;
}

extern "C" bfs_status bfs_run_batch_vm(bfs_graph *g, int32_t num_sources, const int32_t *sources,
                                       int32_t *level, int32_t *parent, bfs_run_options *opt,
                                       void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (num_sources <= 0) return fail(BFS_EINVAL, "num_sources = %d", num_sources);
    if (!sources || !level || !parent || !workspace) return fail(BFS_EINVAL, "NULL argument");
    if (((uintptr_t)workspace & 255) != 0) return fail(BFS_EINVAL, "workspace must be 256-byte aligned");
    if (((uintptr_t)level & 15) != 0 || ((uintptr_t)parent & 15) != 0)
        return fail(BFS_EINVAL, "level / parent must be 16-byte aligned");
    for (int32_t q = 0; q < num_sources; ++q)
        if (sources[q] < 0 || sources[q] >= g->n)
            return fail(BFS_ERANGE, "source %d (%d) outside [0, %d)", q, sources[q], g->n);
    const size_t need = bfs_batch_vm_workspace_size(g, num_sources);
    if (ws_bytes < need) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    if (opt && opt->variant > kShortCircuit) return fail(BFS_EINVAL, "unknown variant %u", opt->variant);
    return run_multi_source(g, num_sources, sources, nullptr, nullptr, opt, workspace,
                            (hipStream_t)hip_stream, level, parent);
}

// ---------------------------------------------------------------------------
// Exhaustive per-level timing of the multi-source directions
// ---------------------------------------------------------------------------

static size_t ms_vm_bytes(const bfs_graph *g, int32_t nq) {
    const size_t ld = 64 * (((size_t)nq + 63) / 64);
    return (size_t)g->n * ld * 4;
}

extern "C" size_t bfs_ms_profile_snapshot_size(const bfs_graph *g, int32_t num_sources) {
    if (!g || num_sources <= 0) return 0;
    return align256(ms_layout(g->n, num_sources, false).total) + 2 * align256(ms_vm_bytes(g, num_sources));
}

extern "C" bfs_status bfs_ms_profile_levels(bfs_graph *g, int32_t num_sources, const int32_t *sources,
                                            int32_t *level, int32_t *parent, void *workspace,
                                            size_t ws_bytes, void *snapshot, size_t snap_bytes,
                                            int32_t reps, bfs_level_record *records, uint32_t capacity,
                                            uint32_t *count, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (num_sources <= 0) return fail(BFS_EINVAL, "num_sources = %d", num_sources);
    if (!sources || !level || !parent || !workspace || !snapshot || !count)
        return fail(BFS_EINVAL, "NULL argument");
    if (capacity > 0 && !records) return fail(BFS_EINVAL, "records is NULL");
    if (((uintptr_t)workspace & 255) != 0 || ((uintptr_t)snapshot & 255) != 0)
        return fail(BFS_EINVAL, "workspace and snapshot must be 256-byte aligned");
    if (((uintptr_t)level & 15) != 0 || ((uintptr_t)parent & 15) != 0)
        return fail(BFS_EINVAL, "level / parent must be 16-byte aligned");
    if (reps < 1 || reps > 1000) return fail(BFS_EINVAL, "reps %d outside [1, 1000]", reps);
    for (int32_t q = 0; q < num_sources; ++q)
        if (sources[q] < 0 || sources[q] >= g->n)
            return fail(BFS_ERANGE, "source %d (%d) outside [0, %d)", q, sources[q], g->n);
    const size_t wsb = ms_layout(g->n, num_sources, false).total;
    if (ws_bytes < wsb) return fail(BFS_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, wsb);
    const size_t snap_need = bfs_ms_profile_snapshot_size(g, num_sources);
    if (snap_bytes < snap_need) return fail(BFS_EINVAL, "snapshot has %zu bytes, needs %zu", snap_bytes, snap_need);
    *count = 0;
    hipStream_t s = (hipStream_t)hip_stream;
    const uint32_t grid = ms_grid(g, nullptr);
    MsLevel p;
    HostSlot *hs = nullptr;
    bfs_status st = ms_prepare(g, num_sources, sources, nullptr, nullptr, workspace, s, level, parent,
                               grid, p, hs);
    if (st != BFS_OK) return st;
    const size_t outb = ms_vm_bytes(g, num_sources);
    char *snap = (char *)snapshot;
    char *snap_lv = snap + align256(wsb), *snap_pa = snap_lv + align256(outb);
    auto copy_state = [&](bool save) -> hipError_t {
        hipError_t e;
        if ((e = hipMemcpyAsync(save ? snap : (char *)workspace, save ? (char *)workspace : snap, wsb,
                                hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(save ? snap_lv : (char *)level, save ? (char *)level : snap_lv, outb,
                                hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
        return hipMemcpyAsync(save ? snap_pa : (char *)parent, save ? (char *)parent : snap_pa, outb,
                              hipMemcpyDeviceToDevice, s);
    };
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto done_events = [&]() {
        for (hipEvent_t &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    HIP_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        done_events();
        return fail(BFS_EHIP, "hipEventCreate failed");
    }
    bfs_status result = BFS_OK;
    auto run = [&]() -> hipError_t {
        hipError_t e;
        if ((e = launch_ms(p, 0, 0, grid, s)) != hipSuccess) return e;
        if ((e = launch_ms(p, 1, 0, grid, s)) != hipSuccess) return e;
        uint32_t cnt[4];
        std::vector<unsigned long long> stat(kMsStatWords);
        for (uint32_t k = 0;; ++k) {
            if ((uint64_t)k > (uint64_t)g->n + 2) {
                result = fail(BFS_EHIP, "multi-source profile loop did not terminate");
                return hipSuccess;
            }
            if ((e = hipMemcpyAsync(cnt, p.cnt, sizeof cnt, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(stat.data(), p.mstat, stat.size() * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            const uint32_t t = k % 3, f = cnt[t];
            if (f == 0) return hipSuccess;
            unsigned long long sd = 0, listed = 0, reached = 0;
            for (int gi = 0; gi < kMsDegGroups; ++gi) {
                sd += stat[ms_line((int)t, gi)];
                listed += stat[ms_line(kMsCumSlot, gi)];
                reached += stat[ms_line(kMsCumSlot, gi) + 1];
            }
            const unsigned long long pairs = (unsigned long long)g->n * (unsigned long long)num_sources;
            if ((e = copy_state(true)) != hipSuccess) return e;
            float best[2] = {0.f, 0.f};
            for (int form = 0; form < 2; ++form) {
                for (int32_t r = 0; r < reps; ++r) {
                    if ((e = copy_state(false)) != hipSuccess) return e;
                    if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
                    if ((e = ms_level(p, k, form == 1, f, grid, s)) != hipSuccess) return e;
                    if ((e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
                    if ((e = hipEventSynchronize(ev[1])) != hipSuccess) return e;
                    float ms = 0.f;
                    if ((e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) return e;
                    if (r == 0 || ms * 1e3f < best[form]) best[form] = ms * 1e3f;
                }
            }
            for (int form = 0; form < 2; ++form) {
                if (*count >= capacity) break;
                bfs_level_record &rec = records[(*count)++];
                rec = bfs_level_record{};
                rec.level = (int32_t)k;
                rec.variant = form;
                rec.frontier = f;
                rec.unvisited = (uint32_t)std::min<unsigned long long>(listed, 0xffffffffull);
                rec.frontier_edges = sd;
                rec.unvisited_edges = pairs > reached ? pairs - reached : 0ull;
                rec.time_us = best[form];
            }
            // advance with the faster direction, from the saved state
            if ((e = copy_state(false)) != hipSuccess) return e;
            if ((e = ms_level(p, k, best[1] < best[0], f, grid, s)) != hipSuccess) return e;
        }
    };
    const hipError_t e = run();
    done_events();
    if (e != hipSuccess) return fail(BFS_EHIP, "HIP error %s", hipGetErrorString(e));
    return result;
}

// ---------------------------------------------------------------------------
// Re-cut the sliced push's bitmap slices (tuning and testing)
// ---------------------------------------------------------------------------

extern "C" bfs_status bfs_graph_set_slice_words(bfs_graph *g, uint32_t max_words) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (max_words < 4 || max_words > kSlMaxSliceWords || (max_words & 3u))
        return fail(BFS_EINVAL, "slice words %u: a multiple of 4 in [4, %u]", max_words, kSlMaxSliceWords);
    const uint64_t words = ((uint64_t)g->n + 31) / 32;
    if ((words + max_words - 1) / max_words > kSlMaxSlices)
        return fail(BFS_EINVAL, "%u words per slice cut n = %d into more than %u slices", max_words, g->n,
                    kSlMaxSlices);
    std::lock_guard<std::mutex> lock(g->mu);
    std::vector<int32_t> ptr, idx;
    try {
        ptr.resize((size_t)g->n + 1);
        HIP_TRY(hipMemcpy(ptr.data(), g->out_ptr, ptr.size() * 4, hipMemcpyDeviceToHost));
        idx.resize((size_t)ptr[g->n]);
        if (!idx.empty()) HIP_TRY(hipMemcpy(idx.data(), g->out_idx, idx.size() * 4, hipMemcpyDeviceToHost));
    } catch (const std::bad_alloc &) {
        return fail(BFS_ENOMEM, "host allocation failed");
    }
    int4 *old_seg = g->sl_seg;
    uint32_t *old_occ = g->sl_occ;
    SlChunk *old_ch = g->sl_chunks;
    const uint32_t old_S = g->sl_S, old_sw = g->sl_sw;
    uint32_t old_off[kSlMaxSlices + 1];
    for (uint32_t i = 0; i <= kSlMaxSlices; ++i) old_off[i] = g->sl_chunk_off[i];
    const size_t old_bytes = g->bytes;
    g->sl_seg = nullptr;
    g->sl_occ = nullptr;
    g->sl_chunks = nullptr;
    g->sl_S = 0;
    bfs_status st;
    try {
        st = build_slices(g, ptr, idx, max_words);
    } catch (const std::bad_alloc &) {
        st = fail(BFS_ENOMEM, "host allocation failed");
    }
    if (st != BFS_OK) {                       // keep the old cut
        if (g->sl_seg) (void)hipFree(g->sl_seg);
        if (g->sl_occ) (void)hipFree(g->sl_occ);
        if (g->sl_chunks) (void)hipFree(g->sl_chunks);
        g->sl_seg = old_seg;
        g->sl_occ = old_occ;
        g->sl_chunks = old_ch;
        g->sl_S = old_S;
        g->sl_sw = old_sw;
        for (uint32_t i = 0; i <= kSlMaxSlices; ++i) g->sl_chunk_off[i] = old_off[i];
        g->bytes = old_bytes;
        return st;
    }
    size_t freed = 0;
    if (old_seg) { (void)hipFree(old_seg); freed += ((size_t)g->n + 1) * sizeof(int4); }
    if (old_occ) { (void)hipFree(old_occ); freed += (size_t)old_S * old_S * old_sw * 4; }
    if (old_ch) {
        (void)hipFree(old_ch);
        const size_t nch = old_off[kSlMaxSlices];
        freed += (nch ? nch : 1) * sizeof(SlChunk);
    }
    g->bytes -= std::min(freed, g->bytes);
    g->gcache.valid = false;                  // captured launches hold the old slice parameters
    return BFS_OK;
}

// ---------------------------------------------------------------------------
// One search that allocates nothing: the sliced push on the library's
// file-scope scratch array
// ---------------------------------------------------------------------------

extern "C" bfs_status bfs_run_static(bfs_graph *g, int32_t source, int32_t *level, int32_t *parent,
                                     uint32_t levels_per_sync, void *hip_stream) {
    if (!g) return fail(BFS_EINVAL, "graph is NULL");
    if (!level || !parent) return fail(BFS_EINVAL, "level/parent is NULL");
    if (source < 0 || source >= g->n) return fail(BFS_ERANGE, "source %d outside [0, %d)", source, g->n);
    if (levels_per_sync > 4096) return fail(BFS_EINVAL, "levels_per_sync %u above 4096", levels_per_sync);
    if (g->sl_S == 0)
        return fail(BFS_EINVAL, "n = %d: the allocation-free search serves graphs of at most %u vertices",
                    g->n, kSlMaxSlices * kSlMaxSliceWords * 32u);
    const SlLayout L = sl_layout(g->sl_S * g->sl_sw);
    const size_t need = L.total + 256;                    // + the progress words
    if (need > kStaticScratchBytes)
        return fail(BFS_EINVAL, "the search needs %zu bytes of scratch; the library's array holds %zu",
                    need, kStaticScratchBytes);
    void *base = nullptr;
    HIP_TRY(static_scratch(&base));
    hipStream_t s = (hipStream_t)hip_stream;
    SlParams P = make_sl_params(g, level, parent, base, false);
    uint32_t *status = (uint32_t *)((char *)base + L.total);
    P.host_status = status;                             // device words here, read back by copy
    HIP_TRY(launch_sl_init(P, 1, nullptr, source, s));
    const uint32_t grid = sl_grid(g);
    const uint32_t per = levels_per_sync ? levels_per_sync : 4u;
    for (uint64_t issued = 0;; issued += per) {
        if (issued > (uint64_t)g->n + 2) return fail(BFS_EHIP, "level loop did not terminate");
        for (uint32_t l = 0; l < per; ++l) HIP_TRY(launch_sl_level(P, grid, s));
        uint32_t prog[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(prog, status, sizeof prog, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (prog[1] == 0) break;                        // the last level found nothing
    }
    return BFS_OK;
}

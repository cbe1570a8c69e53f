// gfx950 kernels of the sliced push: the push (column) form of
// x_{k+1} = A^T[V_{k+1}, V_k] x_k (Theorem 1) with the row mask held in LDS.
//
// Level k reads the columns of F_k = supp(x_k) and keeps the entries whose row
// is not in V_k's complement, i.e. not visited through level k (Definition 1).
// The mask test is one bit of B_k = B_{k-1} | C_k.  A random 4-byte test
// against a bitmap in L2 is what bounds a column gather on this chip (one L2
// request per entry), so the bitmap is cut into slices of at most 128 KiB and
// each workgroup holds one slice in LDS for the whole level: it expands only
// the part of every frontier column whose rows fall in its slice (the graph
// stores where each slice starts in each sorted out-list), tests the rows in
// LDS and claims a reached row by setting its LDS bit.  A row claimed once is
// masked for the rest of the level, as Algorithm 1 removes it from V' as soon
// as it is reached.
//
// The Boolean product gives the level sets; the parent is the (min, select)
// value of the same product.  A level runs in one of two modes, chosen from
// the size of its frontier:
//  * lazy (large frontier): the claims go into the LDS slice as above; the
//    parent of a claimed row is found one level later, row-wise (Claim 1's
//    inner-product form): when v in F_k is expanded, its parent is the first
//    of its in-neighbours, in ascending order, that lies in F_{k-1} = C_{k-1}.
//    A large F_{k-1} makes that first hit come early in the list.
//  * eager (small frontier, few pairs): every unmasked pair (j, i) takes part
//    in a min-select of parent[i] by atomicMin (Lemma 1's form: all unmasked
//    pairs contribute), the atomic that finds the slot empty claims i, and the
//    mask is read from B_k in L2; there is no slice to load or flush, and the
//    next level has nothing left to settle.
// Either way parent[v] is the smallest frontier in-neighbour of v, the value
// every other form of the search produces.
//
// Grid: 8 * S * R workgroups of kSlThreads threads, one per compute unit
// (the slice takes most of the LDS).  Workgroup b = xcd + 8 (s + S r) works on
// slice s for stream q = xcd + 8 r: the S workgroups of a stream sit on one
// XCD (blocks are dealt to the XCDs round-robin) and read the same frontier
// words and the same column lines, so the XCD's L2 serves the other slices.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_device.h"
#include "bfs_internal.h"

namespace bfsi {

namespace {

// One wave's batch of ranges of out_idx, flattened: range j covers entries
// [a[j], e[j]) and quads pre[j] .. pre[j+1]-1 of the batch (pre[na] = total).
struct WaveTab {
    int32_t a[kSlBatch];
    int32_t e[kSlBatch];
    uint32_t pre[kSlBatch + 1];
};

struct SlLds {
    // lazy level: slice s of the visited bitmap, claims OR-ed in;
    // eager level: the first kSlWaves * kSlBatch words hold each wave's column ids
    uint32_t slice[kSlMaxSliceWords];
    uint32_t dirty[kSlMaxSliceWords / 128];   // lazy: a bit per 4 slice words that took a claim
    WaveTab tab[kSlWaves];
    unsigned long long red[kSlWaves][3];      // per-wave sums for the block reduction
};

// A level with at most this many frontier vertices (an upper bound: the claim
// count of the level that built it) runs eager.
__device__ __forceinline__ bool eager_level(uint32_t nclaim, int32_t n) {
    const uint32_t lim = ((uint32_t)n >> 9) > 256u ? ((uint32_t)n >> 9) : 256u;
    return nclaim <= lim;
}

// Orders a wave's LDS writes before the same wave's later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T pick4(T a, T b, T c, T d, uint32_t i) {
    return i == 0 ? a : (i == 1 ? b : (i == 2 ? c : d));
}

__device__ __forceinline__ int32_t comp4(const int4 &v, uint32_t i) {
    return pick4(v.x, v.y, v.z, v.w, i);
}

__device__ __forceinline__ bool test_bit(const uint32_t *bm, int32_t v) {
    return (bm[(uint32_t)v >> 5] >> (v & 31)) & 1u;
}

// What an eager level needs besides the parameters.
struct Eager {
    uint32_t k;
    const uint32_t *bprev, *cur;     // B_k = bprev | cur
    uint32_t *nxt;                   // C_{k+1}
};

constexpr uint32_t kCols = kSlBatch / 64;          // frontier columns per lane in a batch
constexpr uint32_t kQuadsPerLane = 4;    // quads a lane loads together in one round
constexpr uint32_t kMarkQuads = 1;       // quads whose entries are tested together

// The entries of a lane's quads: entry x of quad i is out_idx[eb[i] + x],
// counted when it lies in [ca[i], ce[i]).
__device__ __forceinline__ int32_t quad_at(const int4 &q, uint32_t x) {
    return x == 0 ? q.x : (x == 1 ? q.y : (x == 2 ? q.z : q.w));
}

// Lazy: claim every reached row in the slice (a part's rows all lie in it).
// All the words are read first, then a row whose bit is clear (not visited,
// not yet claimed by this workgroup) is set and its 4-word group flagged for
// the flush.
__device__ __forceinline__ void mark_lazy4(SlLds &L, uint32_t sbase, uint32_t sv,
                                           const int4 (&d)[kQuadsPerLane], const int32_t (&eb)[kQuadsPerLane],
                                           const int32_t (&ca)[kQuadsPerLane],
                                           const int32_t (&ce)[kQuadsPerLane]) {
#pragma unroll
    for (uint32_t h = 0; h < kQuadsPerLane; h += kMarkQuads) {
        uint32_t w[4 * kMarkQuads], m[4 * kMarkQuads];
        bool on[4 * kMarkQuads];
#pragma unroll
        for (uint32_t i = 0; i < kMarkQuads; ++i) {
            // entry eb + x counts when it lies in [ca, ce): one unsigned compare
            const uint32_t off = (uint32_t)(eb[h + i] - ca[h + i]), len = (uint32_t)(ce[h + i] - ca[h + i]);
#pragma unroll
            for (uint32_t x = 0; x < 4; ++x) {
                // a part's rows lie in its slice (the slice starts split each
                // sorted list at the slice bounds): li < sv needs no test
                const uint32_t li = (uint32_t)quad_at(d[h + i], x) - sbase;
                const bool ok = off + x < len;
                on[4 * i + x] = ok;
                w[4 * i + x] = ok ? li >> 5 : 0u;
                m[4 * i + x] = 1u << (li & 31);
            }
        }
        uint32_t cur[4 * kMarkQuads];
#pragma unroll
        for (uint32_t u = 0; u < 4 * kMarkQuads; ++u) cur[u] = L.slice[w[u]];
#pragma unroll
        for (uint32_t u = 0; u < 4 * kMarkQuads; ++u) {
            if (on[u] && !(cur[u] & m[u])) {
                atomicOr(&L.slice[w[u]], m[u]);
                atomicOr(&L.dirty[w[u] >> 7], 1u << ((w[u] >> 2) & 31));
            }
        }
    }
}

// Eager: the pairs (j, i) of a lane's quads.  For a row i not visited
// through level k (B_k read from L2, all the lane's words loaded together),
// j competes for parent[i] by atomicMin (Lemma 1's form: every such pair
// contributes, so the result is the smallest) and i joins C_{k+1} (its level
// is written when level k + 1 scans C_{k+1}).  None of these waits for an
// answer: the atomics return nothing.  A quad's four mask words are loaded
// together.  Returns the pairs
// (an upper bound of the rows claimed, 0 iff none).
__device__ __forceinline__ uint32_t mark_eager4(const SlParams &P, const Eager &E,
                                                const int4 (&d)[kQuadsPerLane],
                                                const int32_t (&eb)[kQuadsPerLane],
                                                const int32_t (&ca)[kQuadsPerLane],
                                                const int32_t (&ce)[kQuadsPerLane],
                                                const int32_t (&cj)[kQuadsPerLane]) {
    uint32_t pairs = 0;
    uint32_t *par = (uint32_t *)P.parent;
#pragma unroll
    for (uint32_t i = 0; i < kQuadsPerLane; ++i) {
        int32_t r[4];
        bool on[4];
        uint32_t mw[4];
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) {
            const int32_t e = eb[i] + (int32_t)x;
            on[x] = e >= ca[i] && e < ce[i];
            r[x] = on[x] ? quad_at(d[i], x) : 0;
        }
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) mw[x] = E.bprev[(uint32_t)r[x] >> 5] | E.cur[(uint32_t)r[x] >> 5];
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) {
            if (on[x] && !((mw[x] >> (r[x] & 31)) & 1u)) {
                atomicMin(&par[r[x]], (uint32_t)cj[i]);
                atomicOr(&E.nxt[(uint32_t)r[x] >> 5], 1u << (r[x] & 31));
                ++pairs;
            }
        }
    }
    return pairs;
}

// Expand up to kCols ranges per lane with the whole wave: the ranges' quads
// are numbered consecutively across the wave (a prefix sum over the lanes),
// lane t of a round takes quads t, t + 64, ... and finds its range by binary
// search, so consecutive lanes read consecutive quads of a range (coalesced).
// Range p of a lane belongs to column j_p (used by an eager level only).
// Called by every lane of the wave; ranges with e <= a are empty.  Returns the
// lane's eager claims.
__device__ __forceinline__ uint32_t expand(const SlParams &P, SlLds &L, uint32_t wave, uint32_t sbase,
                                           uint32_t sv, const Eager *E, const int32_t (&ra)[kCols],
                                           const int32_t (&re)[kCols], const int32_t (&rj)[kCols]) {
    WaveTab &T = L.tab[wave];
    uint32_t *tj = &L.slice[wave * kSlBatch];        // eager only: the slice is not in use
    const uint32_t lane = lane_id();
    uint32_t nr[kCols], cnt = 0, tot = 0;
#pragma unroll
    for (uint32_t c = 0; c < kCols; ++c) {
        nr[c] = re[c] > ra[c] ? (uint32_t)(((re[c] + 3) >> 2) - (ra[c] >> 2)) : 0u;
        cnt += nr[c] != 0u;
        tot += nr[c];
    }
    // ranges (high bits) and quads (low 20 bits) before this lane, in one scan:
    // at most kSlBatch ranges of at most 257 quads each (parts are < kSlLong entries)
    const uint32_t mine = (cnt << 20) | tot;
    const uint32_t incl = wave_incl_scan(mine);
    const uint32_t total = __shfl(incl, 63, 64);
    const uint32_t nq = total & 0xFFFFFu;
    if (nq == 0u) return 0u;
    const uint32_t na = total >> 20;
    uint32_t slot = (incl - mine) >> 20;
    uint32_t pre = (incl - mine) & 0xFFFFFu;
    const bool eg = E != nullptr;
#pragma unroll
    for (uint32_t c = 0; c < kCols; ++c) {
        if (nr[c]) {
            T.a[slot] = ra[c];
            T.e[slot] = re[c];
            T.pre[slot] = pre;
            if (eg) tj[slot] = (uint32_t)rj[c];
            ++slot;
            pre += nr[c];
        }
    }
    if (lane == 0) T.pre[na] = nq;
    wave_lds_sync();
    uint32_t claims = 0;
    for (uint32_t rb = 0; rb < nq; rb += 64 * kQuadsPerLane) {
        // each quad's range by binary lifting over pre[], the lane's quads
        // interleaved so that their LDS reads are in flight together; quads
        // past the end repeat the last one and are then disabled
        uint32_t t[kQuadsPerLane], c[kQuadsPerLane], pv[kQuadsPerLane];
#pragma unroll
        for (uint32_t i = 0; i < kQuadsPerLane; ++i) {
            const uint32_t ti = rb + lane + 64u * i;
            t[i] = ti < nq ? ti : nq - 1u;
            c[i] = 0;
            pv[i] = 0;
        }
#pragma unroll
        for (uint32_t step = kSlBatch / 2; step >= 1; step >>= 1) {
#pragma unroll
            for (uint32_t i = 0; i < kQuadsPerLane; ++i) {
                const uint32_t m = (c[i] + step < na) ? c[i] + step : na;   // pre[na] = nq > t
                const uint32_t pm = T.pre[m];
                if (pm <= t[i]) {
                    c[i] = m;
                    pv[i] = pm;
                }
            }
        }
        int4 d[kQuadsPerLane];
        int32_t ca[kQuadsPerLane], ce[kQuadsPerLane], eb[kQuadsPerLane], cj[kQuadsPerLane];
#pragma unroll
        for (uint32_t i = 0; i < kQuadsPerLane; ++i) {
            const bool live = rb + lane + 64u * i < nq;
            ca[i] = T.a[c[i]];
            ce[i] = live ? T.e[c[i]] : ca[i];          // an empty window: nothing in it counts
            cj[i] = eg ? (int32_t)tj[c[i]] : 0;
            const int32_t qi = (ca[i] >> 2) + (int32_t)(t[i] - pv[i]);
            eb[i] = qi * 4;
            d[i] = P.out_idx4[qi];
        }
        if (eg) {
            claims += mark_eager4(P, *E, d, eb, ca, ce, cj);
        } else {
            mark_lazy4(L, sbase, sv, d, eb, ca, ce);
        }
    }
    wave_lds_sync();                                   // the table is rewritten by the next batch
    return claims;
}

// Parent of the frontier vertices of F_k a lane settles (up to kCols;
// pending[p] set for each; their level is written by the scan of C_k).  At
// level 0 they are roots.  Otherwise the
// parent is the first in-neighbour, in ascending order, in C_{k-1}.  The
// first kSettleFirst entries of every pending vertex are loaded in
// settle_issue (before the batch's expansion, so that their latency overlaps
// it; positions past a list's end repeat its last entry, which cannot change
// the first hit) and tested in settle_finish; vertices with no hit go on in
// steps of kSettleNext entries, every pending vertex of the wave at once,
// for up to kSettleRounds steps in all; a vertex still pending after those
// is finished by the whole wave, 256 entries per step.  The first step is
// short because the first entry is the hit for almost every vertex of a big
// level (on R-MAT the smallest in-neighbour of a vertex reached from the hub
// level lies in it): each entry tested is a random read of the C_{k-1}
// bitmap, the settle's whole cost.
constexpr int kSettleFirst = 2;
constexpr int kSettleNext = 8;
constexpr int kSettleRounds = 4;

template <int N>
__device__ __forceinline__ void settle_issue(const SlParams &P, const bool (&pending)[kCols],
                                             const int32_t (&pos)[kCols], const int32_t (&end)[kCols],
                                             int32_t (&u)[kCols * N]) {
#pragma unroll
    for (int p = 0; p < (int)kCols; ++p) {
        const int32_t last = pending[p] ? end[p] - 1 : 0;
#pragma unroll
        for (int t = 0; t < N; ++t) {
            const int32_t e = pending[p] ? pos[p] + t : 0;
            u[N * p + t] = P.in_idx[e < last ? e : last];
        }
    }
}

// The C_{k-1} words of the N entries u of each pending vertex.
template <int N>
__device__ __forceinline__ void settle_probe(const uint32_t *prev, const bool (&pending)[kCols],
                                             const int32_t (&u)[kCols * N], uint32_t (&wv)[kCols * N]) {
#pragma unroll
    for (int x = 0; x < (int)kCols * N; ++x) {
        wv[x] = 0u;
        if (pending[x / N]) wv[x] = prev[(uint32_t)u[x] >> 5];
    }
}

// One step: the N entries u (loaded from positions from[p] ..) with their
// C_{k-1} words wv; a hit settles the vertex, otherwise it stays pending
// while entries remain.
template <int N>
__device__ __forceinline__ void settle_test(const SlParams &P, uint32_t k, const int32_t (&v)[kCols],
                                            bool (&pending)[kCols], int32_t (&from)[kCols],
                                            const int32_t (&end)[kCols], const int32_t (&u)[kCols * N],
                                            const uint32_t (&wv)[kCols * N]) {
#pragma unroll
    for (int p = 0; p < (int)kCols; ++p) {
        int32_t hit = -1;
#pragma unroll
        for (int t = N - 1; t >= 0; --t)
            if ((wv[N * p + t] >> (u[N * p + t] & 31)) & 1u) hit = u[N * p + t];
        from[p] += N;
        if (pending[p]) {
            if (hit >= 0) {
                P.parent[v[p]] = hit;
                pending[p] = false;
            } else {
                pending[p] = from[p] < end[p];
            }
        }
    }
}

__device__ __forceinline__ void settle_finish(const SlParams &P, const uint32_t *prev, uint32_t k,
                                              const int32_t (&v)[kCols], bool (&pending)[kCols],
                                              const int32_t (&pos)[kCols], const int32_t (&end)[kCols],
                                              const int32_t (&u)[kCols * kSettleFirst],
                                              const uint32_t (&wv)[kCols * kSettleFirst]) {
    const uint32_t lane = lane_id();
    if (k == 0) {
#pragma unroll
        for (int p = 0; p < (int)kCols; ++p)
            if (pending[p]) {
                P.parent[v[p]] = v[p];
                pending[p] = false;
            }
        return;
    }
    int32_t from[kCols];
#pragma unroll
    for (int p = 0; p < (int)kCols; ++p) from[p] = pos[p];
    settle_test<kSettleFirst>(P, k, v, pending, from, end, u, wv);
    for (int r = 1; r < kSettleRounds; ++r) {
        bool any = false;
#pragma unroll
        for (int p = 0; p < (int)kCols; ++p) any = any || pending[p];
        if (!__ballot(any)) break;                     // uniform
        int32_t u2[kCols * kSettleNext];
        uint32_t w2[kCols * kSettleNext];
        settle_issue<kSettleNext>(P, pending, from, end, u2);
        settle_probe<kSettleNext>(prev, pending, u2, w2);
        settle_test<kSettleNext>(P, k, v, pending, from, end, u2, w2);
    }
    for (int p = 0; p < (int)kCols; ++p) {
        unsigned long long hm = __ballot(pending[p]);
        while (hm) {
            const int l = __ffsll((long long)hm) - 1;
            hm &= hm - 1ull;
            const int32_t hv = __shfl(v[p], l, 64);
            const int32_t hb = __shfl(from[p], l, 64);
            const int32_t he = __shfl(end[p], l, 64);
            int32_t found = -1;
            for (int32_t eb = hb; eb < he && found < 0; eb += 256) {    // uniform
                int32_t w[4];
                uint32_t ww[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int32_t e = eb + 64 * t + (int32_t)lane;
                    w[t] = P.in_idx[e < he ? e : he - 1];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) ww[t] = prev[(uint32_t)w[t] >> 5];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int32_t e = eb + 64 * t + (int32_t)lane;
                    const bool h = (e < he) && ((ww[t] >> (w[t] & 31)) & 1u);
                    const unsigned long long m = __ballot(h);
                    if (found < 0 && m) found = __shfl(w[t], __ffsll((long long)m) - 1, 64);
                }
            }
            if (lane == 0 && found >= 0) P.parent[hv] = found;
        }
    }
}

// The last workgroup of a level launch to finish (see bfs_kernels.hip's
// last_to_arrive: each wave drains its memory operations before the block
// barrier, so everything this workgroup did is performed when it arrives).
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ bool sl_last_to_arrive(SlState *st, uint32_t nblocks) {
    __shared__ uint32_t s_last;
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t groups = nblocks < (uint32_t)kBarGroups ? nblocks : (uint32_t)kBarGroups;
        const uint32_t g = blockIdx.x % groups;
        const uint32_t in_group = (nblocks - g + groups - 1) / groups;
        uint32_t last = 0;
        if (atomicAdd(&st->bar_group[g * 16], 1u) == in_group - 1) {
            __hip_atomic_store(&st->bar_group[g * 16], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (atomicAdd(&st->bar_top, 1u) == groups - 1) {
                __hip_atomic_store(&st->bar_top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = 1;
            }
        }
        s_last = last;
    }
    __syncthreads();
    return s_last != 0;
}

// Close level k (one thread, every workgroup done): collect and reset the
// grouped sums, record the level, advance, report.
__device__ __forceinline__ void sl_close(const SlParams &P, uint32_t k) {
    SlState *st = P.st;
    unsigned long long cn = 0, deg = 0;
    for (int g = 0; g < kBarGroups; ++g) {
        cn += atomicExch(&st->acc[8 * g], 0ull);
        deg += atomicExch(&st->acc[8 * g + 1], 0ull);
    }
    const uint32_t claims = (uint32_t)cn;
    const uint32_t nf = (uint32_t)(cn >> 32);
    const uint32_t vc = st->visited_cnt + nf;
    const unsigned long long vd = st->visited_deg + deg;
    st->nclaim[(k + 1) & 3] = claims;
    st->nf[k & 3] = nf;
    st->sdf[k & 3] = deg;
    st->visited_cnt = vc;
    st->visited_deg = vd;
    if (P.trace) {
        DevLevelRec r;
        r.level = k;
        r.variant = kPush;
        r.nf = nf;
        r.nu = (uint32_t)P.n - vc;
        r.sdf = deg;
        r.sdu = (unsigned long long)P.nnz - vd;
        P.trace[k % kTraceCap] = r;
    }
    st->level = k + 1;
    P.host_status[0] = k + 1;
    P.host_status[1] = claims;
}

}  // namespace

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Outputs to -1, B_{-1} and C_1 empty, C_0 = the root (single_root >= 0) or
// empty (roots set by k_sl_roots), the state at level 0.
__global__ __launch_bounds__(256) void k_sl_init(SlParams P, int32_t single_root, uint32_t nroots) {
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    const uint32_t stride = gridDim.x * 256;
    for (uint32_t v = gid; v < (uint32_t)P.n; v += stride) {
        P.level[v] = -1;
        P.parent[v] = -1;
    }
    for (uint32_t w = gid; w < P.words; w += stride) {
        uint32_t bits = 0;
        if (single_root >= 0 && ((uint32_t)single_root >> 5) == w) bits = 1u << (single_root & 31);
        P.vb[1][w] = 0u;
        P.cb[0][w] = bits;
        P.cb[1][w] = 0u;
    }
    if (gid == 0) {
        SlState *st = P.st;
        st->level = 0;
        for (int r = 0; r < kRing; ++r) {
            st->nclaim[r] = 0;
            st->nf[r] = 0;
            st->sdf[r] = 0ull;
        }
        st->nclaim[0] = nroots;
        st->visited_cnt = 0;
        st->visited_deg = 0ull;
        for (int g = 0; g < kBarGroups; ++g) {
            st->acc[8 * g] = 0ull;
            st->acc[8 * g + 1] = 0ull;
            st->bar_group[g * 16] = 0;
        }
        st->bar_top = 0;
    }
}

// Several roots (after k_sl_init with single_root = -1): their bits in C_0.
__global__ __launch_bounds__(256) void k_sl_roots(SlParams P, int32_t nroots, const int32_t *roots) {
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    if (gid < (uint32_t)nroots) {
        const int32_t r = roots[gid];
        atomicOr(&P.cb[0][(uint32_t)r >> 5], 1u << (r & 31));
    }
}

// The frontier-slice owner of vertex v: v mod S from the low two bits (S <= 4).
__device__ __forceinline__ uint32_t owner(int32_t v, uint32_t S) {
    uint32_t o = (uint32_t)v & 3u;
    if (o >= S) o -= S;
    if (o >= S) o -= S;
    if (o >= S) o -= S;
    return o;
}

// A batch of the segment's frontier vertices, compacted over the wave: the
// vertex of rank b0 + 64 p + lane among the segment's set bits (ascending),
// v[p] = -1 past the last.  Lane j holds word sw0 + j of the segment, with
// excl_j of the segment's bits before it.  (Popping each lane's own word
// instead leaves a batch's lanes idle once their words run out: on a dense
// level the fullest of 64 words sets the number of batches.)
__device__ __forceinline__ void select_batch(uint32_t fw, uint32_t excl, uint32_t total, uint32_t b0,
                                             uint32_t sw0, int32_t (&v)[kCols]) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int p = 0; p < (int)kCols; ++p) {
        const uint32_t r = b0 + (uint32_t)p * 64u + lane;
        // the last lane j with excl_j <= r (the word holding rank r)
        uint32_t j = 0;
#pragma unroll
        for (uint32_t step = 32; step; step >>= 1) {
            const uint32_t e = (uint32_t)__shfl((int)excl, (int)(j + step), 64);
            if (e <= r) j += step;
        }
        uint32_t w = (uint32_t)__shfl((int)fw, (int)j, 64);
        uint32_t kk = r - (uint32_t)__shfl((int)excl, (int)j, 64);
        // the kk-th set bit of w: halve the window, skipping halves whose
        // bits come before it
        uint32_t bit = 0;
#pragma unroll
        for (uint32_t h = 16; h; h >>= 1) {
            const uint32_t lo = (uint32_t)__popc(w & ((1u << h) - 1u));
            if (kk >= lo) {
                kk -= lo;
                w >>= h;
                bit += h;
            }
        }
        v[p] = r < total ? (int32_t)((sw0 + j) * 32u + bit) : -1;
    }
}

// The slice starts of each vertex's out-list and the list's end (for v < 0
// the loads read vertex 0: valid addresses, results unused).
__device__ __forceinline__ void load_starts(const SlParams &P, const int32_t (&v)[kCols],
                                            int4 (&sg)[kCols], int32_t (&vend)[kCols]) {
#pragma unroll
    for (int p = 0; p < (int)kCols; ++p) {
        const int32_t vc = v[p] >= 0 ? v[p] : 0;
        sg[p] = P.seg[vc];
        vend[p] = P.seg[vc + 1].x;
    }
}

constexpr uint32_t kCopyUnroll = 4;      // 16-byte groups a thread moves per step of a bitmap pass

// One level k.  Launches after the end of the search (C_k empty) return.
__global__ __launch_bounds__(kSlThreads) void k_sl_level(SlParams P) {
    __shared__ SlLds L;
    SlState *st = P.st;
    const uint32_t k = st->level;
    const uint32_t nck = st->nclaim[k & 3];
    if (nck == 0u) return;
    const bool eager = eager_level(nck, P.n);
    // F_k was settled by level k - 1 when that level ran eager
    const bool settle_now = (k == 0) || !eager_level(st->nclaim[(k + 3) & 3], P.n);
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t b = blockIdx.x;
    const uint32_t S = P.S;
    const uint32_t s = (b >> 3) % S;                         // slice
    const uint32_t q = (b & 7u) + 8u * ((b >> 3) / S);        // stream
    const uint32_t sbase = s * P.sw * 32u;                   // first vertex of the slice
    const uint32_t sv = P.sw * 32u;
    const uint32_t w0 = s * P.sw;

    // selects, not runtime indexing of the parameter arrays (which would put
    // the kernel arguments in scratch memory)
    const uint32_t *cur = pick4<const uint32_t *>(P.cb[0], P.cb[1], P.cb[2], P.cb[3], k & 3);
    const uint32_t *prev = pick4<const uint32_t *>(P.cb[0], P.cb[1], P.cb[2], P.cb[3], (k + 3) & 3);
    uint32_t *nxt = pick4<uint32_t *>(P.cb[0], P.cb[1], P.cb[2], P.cb[3], (k + 1) & 3);
    uint32_t *clr = pick4<uint32_t *>(P.cb[0], P.cb[1], P.cb[2], P.cb[3], (k + 2) & 3);
    const uint32_t *bprev = (k & 1) ? P.vb[0] : P.vb[1];     // B_{k-1}
    uint32_t *bcur = (k & 1) ? P.vb[1] : P.vb[0];            // B_k

    // every workgroup a share: B_k = B_{k-1} | C_k stored for the next level,
    // and C_{k-2} (read by nobody now) cleared for the claims of level k + 1
    for (uint32_t w = (b * kSlThreads + tid) * 4u; w < P.words; w += gridDim.x * kSlThreads * 4u) {
        uint4 x = *(const uint4 *)(bprev + w);
        const uint4 c = *(const uint4 *)(cur + w);
        x.x |= c.x;
        x.y |= c.y;
        x.z |= c.z;
        x.w |= c.w;
        *(uint4 *)(bcur + w) = x;
        *(uint4 *)(clr + w) = make_uint4(0u, 0u, 0u, 0u);
    }

    // lazy: slice s of B_k into LDS, kCopyUnroll groups of 16 bytes per thread
    // in flight at a time; the dirty flags cleared
    if (!eager) {
        for (uint32_t w = tid; w < P.sw / 128u; w += kSlThreads) L.dirty[w] = 0u;
        constexpr uint32_t step = kSlThreads * 4u;
        for (uint32_t base = tid * 4u; base < P.sw; base += step * kCopyUnroll) {
            uint4 x[kCopyUnroll], c[kCopyUnroll];
#pragma unroll
            for (uint32_t u = 0; u < kCopyUnroll; ++u) {
                const uint32_t w = base + u * step;
                if (w < P.sw) {
                    x[u] = *(const uint4 *)(bprev + w0 + w);
                    c[u] = *(const uint4 *)(cur + w0 + w);
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kCopyUnroll; ++u) {
                const uint32_t w = base + u * step;
                if (w < P.sw) {
                    x[u].x |= c[u].x;
                    x[u].y |= c[u].y;
                    x[u].z |= c[u].z;
                    x[u].w |= c[u].w;
                    *(uint4 *)(&L.slice[w]) = x[u];
                }
            }
        }
    }
    __syncthreads();

    Eager E{k, bprev, cur, nxt};
    const Eager *ep = eager ? &E : nullptr;
    unsigned long long n_settled = 0, deg_settled = 0, claims = 0;

    // long parts of frontier columns in slice s, as chunks: wave gw of the
    // slice takes records c0 + gw, c0 + gw + nw, ... (64 per step, one per
    // lane).  Consecutive gw lie in different workgroups (a column's chunks
    // are consecutive records: a hub's chunks spread over the compute units
    // instead of filling one workgroup's waves, whose random memory
    // operations would queue on one unit)
    {
        const uint32_t c0 = pick4(P.chunk_off[0], P.chunk_off[1], P.chunk_off[2], P.chunk_off[3], s);
        const uint32_t c1 = pick4(P.chunk_off[1], P.chunk_off[2], P.chunk_off[3], P.chunk_off[4], s);
        const uint64_t gw = (uint64_t)wave * P.streams + q, nw = (uint64_t)P.streams * kSlWaves;
        for (uint64_t jb = 0; c0 + gw + jb * nw < c1; jb += 64) {
            const uint64_t r = c0 + gw + (jb + lane) * nw;
            const SlChunk ch = P.chunks[r < c1 ? r : c1 - 1];     // c1 > c0 here
            const bool on = (r < c1) && test_bit(cur, ch.v);
            const int32_t a = on ? ch.a : 0, e = on ? ch.e : 0, j = ch.v;
            int32_t ca[kCols], ce[kCols], cj[kCols];
#pragma unroll
            for (uint32_t c = 0; c < kCols; ++c) {
                ca[c] = c == 0 ? a : 0;
                ce[c] = c == 0 ? e : 0;
                cj[c] = j;
            }
            claims += expand(P, L, wave, sbase, sv, ep, ca, ce, cj);
        }
    }

    // every frontier vertex: settle it (if this slice owns it and level k - 1
    // left it unsettled) and expand its short part in slice s.  The stream's
    // words are cut into 64-word segments (2048 vertices) dealt to the waves; a
    // batch takes the segment's next 64 kCols frontier vertices, kCols per lane.
    {
        // bits j of a word whose vertex 32 w + j this workgroup owns (owner
        // depends on v mod 4 only, and 32 w is a multiple of 4)
        uint32_t own_bits = 0;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
            if (owner((int32_t)j, S) == s) own_bits |= 0x11111111u << j;
        const uint32_t wps = (((P.words + P.streams - 1u) / P.streams) + 63u) & ~63u;
        const uint32_t ws0 = q * wps;
        const uint32_t ws1 = (ws0 + wps < P.words) ? ws0 + wps : P.words;
        for (uint32_t sw0 = ws0 + wave * 64u; sw0 < ws1; sw0 += kSlWaves * 64u) {
            const uint32_t wi = sw0 + lane;
            uint32_t fw = (wi < ws1) ? cur[wi] : 0u;
            // level k for every vertex of the segment in C_k, by one of the
            // stream's S workgroups: for each pair of words 2j, 2j + 1 with a
            // bit, lane t writes vertex t of the pair, so each store covers
            // 64 consecutive vertices (two lines) instead of one line per
            // vertex
            const unsigned long long nzw = __ballot(fw != 0u);
            if ((sw0 >> 6) % S == s) {
                unsigned long long pairs = (nzw | (nzw >> 1)) & 0x5555555555555555ull;
                while (pairs) {                                      // uniform
                    const uint32_t j2 = (uint32_t)__ffsll((long long)pairs) - 1u;
                    pairs &= pairs - 1ull;
                    const uint32_t w = (uint32_t)__shfl((int)fw, (int)(j2 + (lane >> 5)), 64);
                    if ((w >> (lane & 31u)) & 1u) P.level[(sw0 + j2) * 32u + lane] = (int32_t)k;
                }
            }
            // this workgroup's vertices of the segment: those whose part in
            // slice s is short and not empty (P.occ), and the ones it settles
            // and counts (owner s) whatever their part
            const uint32_t fo = fw & (((wi < ws1) ? P.occ[s * P.words + wi] : 0u) | own_bits);
            const uint32_t cnt = (uint32_t)__popc(fo);
            const uint32_t incl = wave_incl_scan(cnt);
            const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
            const uint32_t excl = incl - cnt;
            for (uint32_t b0 = 0; b0 < total; b0 += 64u * kCols) {          // uniform
                int32_t v[kCols], vend[kCols];
                int4 sg[kCols];
                select_batch(fo, excl, total, b0, sw0, v);
                load_starts(P, v, sg, vend);
                int32_t ra[kCols], re[kCols], pos[kCols], end[kCols];
                bool pend[kCols];
#pragma unroll
                for (int p = 0; p < (int)kCols; ++p) {
                    ra[p] = 0;
                    re[p] = 0;
                    pos[p] = 0;
                    end[p] = 0;
                    pend[p] = false;
                    if (v[p] >= 0) {
                        const bool own = owner(v[p], S) == s;
                        const int32_t a = comp4(sg[p], s);
                        const int32_t e = (s == 3u) ? vend[p] : comp4(sg[p], s + 1u);
                        if (e - a < (int32_t)kSlLong) {   // longer parts go by chunks
                            ra[p] = a;
                            re[p] = e;
                        }
                        if (own) {
                            n_settled += 1ull;
                            deg_settled += (unsigned long long)(vend[p] - sg[p].x);
                            if (settle_now) {
                                pend[p] = true;
                                pos[p] = sg[p].x;
                                end[p] = vend[p];
                            }
                        }
                    }
                }
                if (P.in_ptr && settle_now) {             // directed: the in-lists
#pragma unroll
                    for (int p = 0; p < (int)kCols; ++p) {
                        const int32_t vc = v[p] >= 0 ? v[p] : 0;
                        const int32_t i0 = P.in_ptr[vc], i1 = P.in_ptr[vc + 1];
                        if (pend[p]) {
                            pos[p] = i0;
                            end[p] = i1;
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < (int)kCols; ++p) pend[p] = pend[p] && (k == 0 || pos[p] < end[p]);
                // the first settle step's loads are in flight during the expansion
                int32_t su[kCols * kSettleFirst];
                uint32_t sw[kCols * kSettleFirst];
                if (k != 0) {
                    settle_issue<kSettleFirst>(P, pend, pos, end, su);
                    settle_probe<kSettleFirst>(prev, pend, su, sw);
                }
                claims += expand(P, L, wave, sbase, sv, ep, ra, re, v);
                settle_finish(P, prev, k, v, pend, pos, end, su, sw);
            }
        }
    }
    __syncthreads();

    // lazy: the rows this workgroup claimed (its slice minus B_k) into
    // C_{k+1}, only the 4-word groups flagged dirty
    if (!eager) {
        constexpr uint32_t step = kSlThreads * 4u;
        for (uint32_t base = tid * 4u; base < P.sw; base += step * kCopyUnroll) {
            uint4 x[kCopyUnroll], bp[kCopyUnroll], c[kCopyUnroll];
            bool dz[kCopyUnroll];
#pragma unroll
            for (uint32_t u = 0; u < kCopyUnroll; ++u) {
                const uint32_t w = base + u * step;
                dz[u] = (w < P.sw) && ((L.dirty[w >> 7] >> ((w >> 2) & 31)) & 1u);
                if (dz[u]) {
                    x[u] = *(const uint4 *)(&L.slice[w]);
                    bp[u] = *(const uint4 *)(bprev + w0 + w);
                    c[u] = *(const uint4 *)(cur + w0 + w);
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kCopyUnroll; ++u) {
                if (!dz[u]) continue;
                const uint32_t w = base + u * step;
                const uint32_t y0 = x[u].x & ~(bp[u].x | c[u].x), y1 = x[u].y & ~(bp[u].y | c[u].y);
                const uint32_t y2 = x[u].z & ~(bp[u].z | c[u].z), y3 = x[u].w & ~(bp[u].w | c[u].w);
                unsigned long long *n2 = (unsigned long long *)(nxt + w0 + w);
                if (y0 | y1) atomicOr(&n2[0], (unsigned long long)y0 | ((unsigned long long)y1 << 32));
                if (y2 | y3) atomicOr(&n2[1], (unsigned long long)y2 | ((unsigned long long)y3 << 32));
                claims += (unsigned long long)(__popc(y0) + __popc(y1) + __popc(y2) + __popc(y3));
            }
        }
    }
    // the workgroup's sums, one atomic each into its group's line
    claims = wave_sum64(claims);
    n_settled = wave_sum64(n_settled);
    deg_settled = wave_sum64(deg_settled);
    if (lane == 0) {
        L.red[wave][0] = claims;
        L.red[wave][1] = n_settled;
        L.red[wave][2] = deg_settled;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long c = 0, nfs = 0, d = 0;
        for (int w = 0; w < kSlWaves; ++w) {
            c += L.red[w][0];
            nfs += L.red[w][1];
            d += L.red[w][2];
        }
        const uint32_t g = b % (uint32_t)kBarGroups;
        if (c | nfs) atomicAdd(&st->acc[8 * g], c | (nfs << 32));
        if (d) atomicAdd(&st->acc[8 * g + 1], d);
    }
    if (sl_last_to_arrive(st, gridDim.x) && tid == 0) sl_close(P, k);
}

// ---------------------------------------------------------------------------
// layout and launch wrappers
// ---------------------------------------------------------------------------

SlLayout sl_layout(uint32_t words) {
    SlLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t wb = (size_t)words * 4;
    L.state = take(sizeof(SlState));
    L.vb0 = take(wb);
    L.vb1 = take(wb);
    L.c0 = take(wb);
    L.c1 = take(wb);
    L.c2 = take(wb);
    L.c3 = take(wb);
    L.trace = take((size_t)kTraceCap * sizeof(DevLevelRec));
    L.total = off;
    return L;
}

hipError_t launch_sl_init(const SlParams &p, int32_t nroots, const int32_t *roots_dev,
                          int32_t single_root, hipStream_t s) {
    const uint32_t work = (uint32_t)p.n > p.words ? (uint32_t)p.n : p.words;
    uint32_t grid = (work + 255u) / 256u;
    if (grid > 4096u) grid = 4096u;
    if (grid == 0u) grid = 1u;
    hipLaunchKernelGGL(k_sl_init, dim3(grid), dim3(256), 0, s, p, single_root,
                       (uint32_t)(single_root >= 0 ? 1 : nroots));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || single_root >= 0) return e;
    const uint32_t g2 = ((uint32_t)nroots + 255u) / 256u;
    hipLaunchKernelGGL(k_sl_roots, dim3(g2 ? g2 : 1u), dim3(256), 0, s, p, nroots, roots_dev);
    return hipGetLastError();
}

hipError_t launch_sl_level(const SlParams &p, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_sl_level, dim3(grid), dim3(kSlThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace bfsi

// The claim-word push: the masked product x_{k+1} = A^T[V_{k+1}, V_k] x_k of
// Theorem 1 with the visited mask and the parent select folded into one
// 64-bit word per vertex.
//
// Word w(v) = (level << 32) | parent; while v is unreached its top bit is set
// (above every offer).  At level k, frontier column u offers the key
// ((k + 1) << 32) | u to every row v it holds, by atomicMin on w(v):
//   - a row visited at level <= k has a smaller word: the offer changes nothing
//     (the mask V_{k+1} of the product);
//   - an unreached row keeps the smallest key offered during the level, i.e.
//     the smallest frontier in-neighbour (the min-parent reading of the
//     paper's Algorithm 3 parent array);
//   - the one atomic that finds the top bit set lists v for the next level, so every
//     reached vertex is listed once (Theorem 2's single claim per row).
// Nothing else needs a barrier inside a level, and the level and parent of a
// vertex are never written before its final value is known: a pass at the
// end splits the words into the callers' level and parent arrays.
//
// Two forms of a level:
//   - narrow: one workgroup of 1024 threads runs level after level with the
//     frontier in LDS (up to 8192 columns and 2^16 entries per level), so a
//     level costs a few dependent memory round trips and a workgroup barrier
//     instead of a grid-wide launch (deep, thin searches: grids, road-like
//     graphs);
//   - wide: a launch per level over the frontier lists in global memory
//     (short columns a lane each, long ones in chunks of 1024 entries a wave
//     each, as the paper's work-splitting of long columns suggests).
// Several queries on different graphs share the launches: query q owns the
// virtual ids [base_q, base_q + n_q), its words, and its graph's arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_device.h"
#include "bfs_internal.h"

namespace bfsi {

namespace {

// Unreached words have the top bit set (no offer has it: levels stay below
// 2^31); bit 62 is clear for the rows of kCwLong entries or more, so the offer
// that reaches a row learns its class without reading its column pointers.
constexpr unsigned long long kUnreached = ~0ull;
constexpr unsigned long long kUnreachedLong = ~0ull ^ (1ull << 62);
__device__ __forceinline__ bool unreached(unsigned long long w) { return (w >> 63) != 0ull; }
__device__ __forceinline__ bool long_row(unsigned long long w) { return ((w >> 62) & 1ull) == 0ull; }
constexpr uint32_t kCwGroup = 4;               // narrow: columns a thread expands at once
constexpr uint32_t kCwUnroll = 4;              // wide: entries a lane offers at once
constexpr uint32_t kCwStage = 512;             // wide: a wave's staged appends (LDS entries)

__device__ __forceinline__ unsigned long long offer_key(uint32_t level, uint32_t u) {
    return ((unsigned long long)level << 32) | u;
}

// The query owning virtual id x: the last q with bases[q] <= x.
__device__ __forceinline__ uint32_t query_of(const CwParams &P, uint32_t x) {
    if (P.nq == 1) return 0;
    uint32_t lo = 0, hi = P.nq;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (P.bases[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct Col {                                   // a frontier column
    const int32_t *ptr, *idx;                  // its graph
    uint32_t base;                             // its query's first virtual id
    uint32_t u;                                // its vertex (graph-local)
    int32_t r0;                                // its first entry
    uint32_t deg;                              // its entries
};

__device__ __forceinline__ Col column(const CwParams &P, uint32_t x) {
    const CwQuery &Q = P.q[query_of(P, x)];
    Col c;
    c.ptr = Q.out_ptr;
    c.idx = Q.out_idx;
    c.base = Q.base;
    c.u = x - Q.base;
    c.r0 = c.ptr[c.u];
    c.deg = (uint32_t)(c.ptr[c.u + 1] - c.r0);
    return c;
}

// Append x (with deg out-entries) to the level list of count slot t, called
// by every lane of the wave (own = lane has a vertex); short columns through
// one atomic per wave, long ones (with their chunk map) per lane.
__device__ __forceinline__ void append_wide(const CwParams &P, const CwLists &L, uint32_t t, bool own,
                                            uint32_t x, uint32_t deg) {
    CwState *st = P.st;
    const bool sh = own && deg < kCwLong;
    const unsigned long long bm = __ballot(sh);
    if (bm) {
        const uint32_t leader = (uint32_t)__ffsll((long long)bm) - 1u;
        uint32_t base = 0;
        if (lane_id() == leader) base = atomicAdd(&st->cnt[t][0], (uint32_t)__popcll(bm));
        base = __shfl(base, (int)leader, 64);
        if (sh) L.s[base + lanes_below(bm)] = x;
    }
    if (own && deg >= kCwLong) {
        const uint32_t nch = (deg + kCwChunk - 1) / kCwChunk;
        const uint32_t li = atomicAdd(&st->cnt[t][1], 1u);
        const uint32_t cb = atomicAdd(&st->cnt[t][2], nch);
        L.l[li] = x;
        L.lbase[li] = cb;
        for (uint32_t c = 0; c < nch; ++c) L.cmap[cb + c] = li;
    }
}

struct Ref {                                   // a column's graph and query
    const int32_t *ptr, *idx;
    uint32_t base;
};

template <bool kSingle>
__device__ __forceinline__ Ref ref_of(const CwParams &P, const Ref &one, uint32_t x) {
    if (kSingle) return one;
    const CwQuery &Q = P.q[query_of(P, x)];
    return Ref{Q.out_ptr, Q.out_idx, Q.base};
}

// An empty statement that takes x as read and rewritten: the results of a
// batch of atomics issued under each lane's own condition are first examined
// after every atomic of the batch is in flight (the compiler would otherwise
// examine each result inside its condition, right after its atomic, waiting
// for it there).  It emits no instruction.
__device__ __forceinline__ void settle_after_issue(unsigned long long &x) {
    asm volatile("" : "+v"(x));
}
__device__ __forceinline__ void settle_after_issue32(uint32_t &x) {
    asm volatile("" : "+v"(x));
}

// A wave's staging of the next level's short columns in LDS: appends are
// gathered here (a ballot and an LDS write per batch) and go to the global
// list kCwStage - 64 at a time, one counter atomic each (a per-append
// counter atomic would serialise every append of the level on one word).
struct Stage {
    uint32_t *buf;                             // the wave's kCwStage LDS entries
    uint32_t n;                                // entries held (uniform in the wave)
};

__device__ __forceinline__ void stage_flush(const CwParams &P, const CwLists &N, uint32_t t, Stage &S) {
    if (S.n == 0) return;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&P.st->cnt[t][0], S.n);
    base = __shfl(base, 0, 64);
    for (uint32_t i = lane_id(); i < S.n; i += 64) N.s[base + i] = S.buf[i];
    S.n = 0;
}

// After an offer to row v (of column c's graph) that found word `old`: if
// the offer reached v first, list it for the next level (its class from the
// word; the entry count read only for the long ones).  Every lane calls it.
__device__ __forceinline__ void reach(const CwParams &P, const CwLists &N, uint32_t t, const Col &c, int32_t v,
                                      unsigned long long old, Stage &S) {
    const bool own = unreached(old);
    const bool lg = own && long_row(old);
    uint32_t deg = 0;
    if (lg) deg = (uint32_t)(c.ptr[v + 1] - c.ptr[v]);
    append_wide(P, N, t, lg, c.base + (uint32_t)v, deg);           // long rows (with their chunks)
    const bool sh = own && !lg;
    const unsigned long long bm = __ballot(sh);
    if (bm) {
        if (sh) S.buf[S.n + lanes_below(bm)] = c.base + (uint32_t)v;
        S.n += (uint32_t)__popcll(bm);
        if (S.n > kCwStage - 64) stage_flush(P, N, t, S);
    }
}

// kCwUnroll offers of one lane's column c at once: entries e0 + q * stride
// (those with ok[q]); their entry loads, word tests and atomics are each
// issued for the whole batch before the first result is used.  Every lane
// calls it.
__device__ __forceinline__ void offer_batch(const CwParams &P, const CwLists &N, uint32_t t, const Col &c,
                                            unsigned long long key, bool pre, const bool *ok, int32_t e0,
                                            int32_t stride, Stage &S) {
    int32_t v[kCwUnroll];
    unsigned long long old[kCwUnroll];
#pragma unroll
    for (uint32_t q = 0; q < kCwUnroll; ++q) {
        v[q] = 0;
        if (ok[q]) v[q] = c.idx[e0 + (int32_t)q * stride];
    }
    bool go[kCwUnroll];
#pragma unroll
    for (uint32_t q = 0; q < kCwUnroll; ++q) go[q] = ok[q];
    if (pre) {
        unsigned long long w[kCwUnroll];
#pragma unroll
        for (uint32_t q = 0; q < kCwUnroll; ++q) {
            w[q] = 0ull;
            if (ok[q]) w[q] = P.cw[c.base + (uint32_t)v[q]];
        }
#pragma unroll
        for (uint32_t q = 0; q < kCwUnroll; ++q) settle_after_issue(w[q]);
        // the words only decrease, so a stale copy is never below the true value
#pragma unroll
        for (uint32_t q = 0; q < kCwUnroll; ++q) go[q] = ok[q] && w[q] > key;
    }
#pragma unroll
    for (uint32_t q = 0; q < kCwUnroll; ++q) {
        old[q] = 0ull;
        if (go[q]) old[q] = atomicMin(&P.cw[c.base + (uint32_t)v[q]], key);
    }
#pragma unroll
    for (uint32_t q = 0; q < kCwUnroll; ++q) settle_after_issue(old[q]);
#pragma unroll
    for (uint32_t q = 0; q < kCwUnroll; ++q) reach(P, N, t, c, v[q], old[q], S);
}

// Exclusive prefix sum over the 1024 threads of the narrow workgroup; *total
// receives the sum.  Every thread calls it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *s_w, uint32_t *total) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const uint32_t v = lane < kCwNarrowThreads / 64 ? s_w[lane] : 0u;
        const uint32_t vi = wave_incl_scan(v);
        if (lane < kCwNarrowThreads / 64) s_w[lane] = vi - v;
        if (lane == kCwNarrowThreads / 64 - 1) s_w[kCwNarrowThreads / 64] = vi;
    }
    __syncthreads();
    const uint32_t r = s_w[wave] + inc - x;
    *total = s_w[kCwNarrowThreads / 64];
    __syncthreads();
    return r;
}

}  // namespace

// Words to unreached (with the row class), every count zero, then the
// sources: word (0, s) and the level-0 lists.  A block row per query.
__global__ __launch_bounds__(kCwBlock) void k_cw_fill(CwParams P) {
    const CwQuery &Q = P.q[blockIdx.y];
    for (uint32_t v = blockIdx.x * kCwBlock + threadIdx.x; v < Q.n; v += gridDim.x * kCwBlock) {
        const uint32_t deg = (uint32_t)(Q.out_ptr[v + 1] - Q.out_ptr[v]);
        P.cw[Q.base + v] = deg >= kCwLong ? kUnreachedLong : kUnreached;
    }
    const uint32_t gid = (blockIdx.y == 0) ? blockIdx.x * kCwBlock + threadIdx.x : 0xFFFFFFFFu;
    if (gid < 12) P.st->cnt[gid / 4][gid % 4] = 0u;
    if (gid == 0) {
        P.st->level = 0u;
        P.st->done = 0u;
        P.st->last = 0u;
    }
}

__global__ __launch_bounds__(kCwBlock) void k_cw_roots(CwParams P) {
    const uint32_t q = blockIdx.x * kCwBlock + threadIdx.x;
    bool own = false;
    uint32_t x = 0, deg = 0;
    if (q < P.nq) {
        const CwQuery &Q = P.q[q];
        x = Q.base + (uint32_t)Q.source;
        P.cw[x] = offer_key(0u, (uint32_t)Q.source);
        deg = (uint32_t)(Q.out_ptr[Q.source + 1] - Q.out_ptr[Q.source]);
        own = true;
    }
    append_wide(P, P.lists[0], 0u, own, x, deg);
}

// Level k, wide form.  Items: the short columns, 64 to a wave (a lane each,
// entries taken in lockstep rounds so that the next level's appends gather
// per wave), then the chunks of the long columns (a wave each).  The atomic
// is skipped where the row's word is already at or below the offer.
__global__ __launch_bounds__(kCwBlock) void k_cw_wide(CwParams P, uint32_t k) {
    __shared__ uint32_t s_stage[kCwBlock / 64][kCwStage];
    CwState *st = P.st;
    const uint32_t t0 = k % 3, t1 = (k + 1) % 3, t2 = (k + 2) % 3;
    const CwLists C = P.lists[k & 1], N = P.lists[(k + 1) & 1];
    const uint32_t lane = lane_id();
    const uint32_t gw = blockIdx.x * (kCwBlock / 64) + (threadIdx.x >> 6);
    const uint32_t nw = gridDim.x * (kCwBlock / 64);
    // the lane's entry of the wave's first step, read together with the
    // counts (before it is known to exist: the list has room for V entries)
    // instead of one round trip after them
    const uint32_t i_first = gw * 64u + lane;
    uint32_t x_first = C.s[i_first < P.V ? i_first : 0u];
    const uint32_t ns = st->cnt[t0][0], nc = st->cnt[t0][2];
    settle_after_issue32(x_first);
    if (blockIdx.x == 0 && threadIdx.x < 4) st->cnt[t2][threadIdx.x] = 0u;   // level k+2's lists
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->level = k + 1;
        if (ns + nc != 0) st->last = k;                          // the deepest level with a frontier
    }
    const uint32_t sw = (ns + 63) / 64;
    // test the row's word before the atomic on wide levels (most rows are
    // settled there; the test saves their atomics), not on thin ones (where a
    // level's cost is its chain of dependent round trips)
    const bool pre = ns + 64u * nc >= kCwPrecheck;
    Stage S{s_stage[threadIdx.x >> 6], 0u};
    for (uint32_t it = gw; it < sw + nc; it += nw) {             // uniform per wave
        if (it < sw) {
            const uint32_t i = it * 64 + lane;
            Col c{};
            if (i < ns) c = column(P, it == gw ? x_first : C.s[i]);
            const unsigned long long key = offer_key(k + 1, c.u);
            const uint32_t rounds = (uint32_t)wave_max((int32_t)c.deg);
            for (uint32_t r = 0; r < rounds; r += kCwUnroll) {
                bool ok[kCwUnroll];
#pragma unroll
                for (uint32_t q = 0; q < kCwUnroll; ++q) ok[q] = r + q < c.deg;
                offer_batch(P, N, t1, c, key, pre, ok, c.r0 + (int32_t)r, 1, S);
            }
        } else {
            const uint32_t ch = it - sw;
            const uint32_t li = C.cmap[ch];
            const Col c = column(P, C.l[li]);
            const int32_t e0 = c.r0 + (int32_t)((ch - C.lbase[li]) * kCwChunk);
            const int32_t end = c.r0 + (int32_t)c.deg;
            const int32_t e1 = (e0 + (int32_t)kCwChunk < end) ? e0 + (int32_t)kCwChunk : end;
            const unsigned long long key = offer_key(k + 1, c.u);
            for (int32_t eb = e0; eb < e1; eb += 64 * (int32_t)kCwUnroll) {
                bool ok[kCwUnroll];
#pragma unroll
                for (uint32_t q = 0; q < kCwUnroll; ++q) ok[q] = eb + (int32_t)(q * 64u + lane) < e1;
                offer_batch(P, N, t1, c, key, pre, ok, eb + (int32_t)lane, 64, S);
            }
        }
    }
    stage_flush(P, N, t1, S);
}

// Levels in one workgroup, the frontier in LDS, from level k0 (listed in the
// global lists) until the search ends, a level is too wide (more than
// kCwCap columns, kCwLongCap columns of more than four entries or
// kCwNarrowEdges entries: its frontier goes back to the global lists
// unexpanded), or max_levels levels are done.  Per level: each thread takes
// up to kCwPer columns, kCwGroup at a time, reading their first four entries
// and making their offers with every load and atomic of the group in flight;
// the rest of the longer columns follow in 256-entry pieces, a wave each.
template <bool kSingle>
__global__ __launch_bounds__(kCwNarrowThreads) void k_cw_narrow(CwParams P, uint32_t k0, uint32_t max_levels,
                                                                uint32_t max_next, uint32_t max_edges) {
    __shared__ uint32_t s_f[2][kCwCap];        // frontier, next frontier (virtual ids)
    __shared__ uint32_t s_lx[kCwLongCap];      // columns of more than four entries
    __shared__ int32_t s_lr0[kCwLongCap];      //   their entries after the first four
    __shared__ uint32_t s_ldeg[kCwLongCap];
    __shared__ uint32_t s_lpre[kCwLongCap + 1];   // 256-entry pieces before each
    __shared__ uint32_t s_scan[kCwNarrowThreads / 64 + 1];
    __shared__ uint32_t s_n[2], s_nl, s_edges;
    __shared__ uint32_t s_cs, s_cl, s_cc;
    CwState *st = P.st;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const Ref one = Ref{P.q[0].out_ptr, P.q[0].out_idx, P.q[0].base};   // the query, when there is one
    uint32_t k = k0;
    {
        const uint32_t t0 = k % 3, ns = st->cnt[t0][0], nl = st->cnt[t0][1];
        if (ns + nl > kCwCap) return;                             // the host checks this first
        const CwLists C = P.lists[k & 1];
        for (uint32_t i = tid; i < ns + nl; i += kCwNarrowThreads) s_f[0][i] = i < ns ? C.s[i] : C.l[i - ns];
        if (tid == 0) s_n[0] = ns + nl;
    }
    __syncthreads();
    uint32_t cur = 0;
    // Hand frontier f (n columns: the first min(n, kCwCap) in LDS array
    // `lds`, the rest in P.spill) to the global lists of level `lv`.
    auto to_global = [&](const uint32_t *lds, uint32_t n, uint32_t lv) {
        const uint32_t t = lv % 3;
        const CwLists L = P.lists[lv & 1];
        if (tid == 0) {
            s_cs = 0;
            s_cl = 0;
            s_cc = 0;
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kCwNarrowThreads) {
            const uint32_t x = i < kCwCap ? lds[i] : P.spill[i - kCwCap];
            const Col c = column(P, x);
            if (c.deg < kCwLong) {
                L.s[atomicAdd(&s_cs, 1u)] = x;
            } else {
                const uint32_t nch = (c.deg + kCwChunk - 1) / kCwChunk;
                const uint32_t li = atomicAdd(&s_cl, 1u);
                const uint32_t cb = atomicAdd(&s_cc, nch);
                L.l[li] = x;
                L.lbase[li] = cb;
                for (uint32_t j = 0; j < nch; ++j) L.cmap[cb + j] = li;
            }
        }
        __syncthreads();
        if (tid == 0) {
            st->cnt[t][0] = s_cs;
            st->cnt[t][1] = s_cl;
            st->cnt[t][2] = s_cc;
            for (int j = 0; j < 3; ++j) {
                st->cnt[(lv + 1) % 3][j] = 0u;
                st->cnt[(lv + 2) % 3][j] = 0u;
            }
            st->level = lv;
        }
    };
    for (uint32_t done = 0;; ++done, ++k) {
        const uint32_t nf = s_n[cur];
        if (nf == 0) {
            if (tid == 0) {
                for (int t = 0; t < 3; ++t)
                    for (int j = 0; j < 3; ++j) st->cnt[t][j] = 0u;
                st->level = k;
                st->done = 1u;
            }
            return;
        }
        if (done == max_levels) {
            to_global(s_f[cur], nf, k);
            return;
        }
        if (tid == 0) {
            s_nl = 0;
            s_edges = 0;
            s_n[cur ^ 1] = 0;
        }
        __syncthreads();
        // The level's columns: extents, width.  Loads are issued under a
        // lane's own condition with the result left in place otherwise, and
        // nothing reads a result before every load of the batch is issued, so
        // the batch's loads are in flight together.
        uint32_t xs[kCwPer];
        int32_t r0s[kCwPer];
        uint32_t degs[kCwPer];
        Ref refs[kCwPer];
        uint32_t my_edges = 0;
#pragma unroll
        for (uint32_t j = 0; j < kCwPer; ++j) {
            const uint32_t i = tid + j * kCwNarrowThreads;
            xs[j] = s_f[cur][i < nf ? i : 0u];
            refs[j] = ref_of<kSingle>(P, one, xs[j]);
        }
        int32_t pa[kCwPer], pb[kCwPer];
#pragma unroll
        for (uint32_t j = 0; j < kCwPer; ++j) {
            pa[j] = 0;
            pb[j] = 0;
            if (tid + j * kCwNarrowThreads < nf) {
                const uint32_t u = xs[j] - refs[j].base;
                pa[j] = refs[j].ptr[u];
                pb[j] = refs[j].ptr[u + 1];
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kCwPer; ++j) {
            r0s[j] = pa[j];
            degs[j] = (uint32_t)(pb[j] - pa[j]);
            my_edges += degs[j];
            if (my_edges > kCwNarrowEdges) my_edges = kCwNarrowEdges + 1u;   // saturate
            if (degs[j] > 4u) {
                const uint32_t li = atomicAdd(&s_nl, 1u);
                if (li < kCwLongCap) {
                    s_lx[li] = xs[j];
                    s_lr0[li] = r0s[j] + 4;
                    s_ldeg[li] = degs[j] - 4u;
                }
            }
        }
        if (my_edges) atomicAdd(&s_edges, my_edges);
        __syncthreads();
        if (s_edges > max_edges || s_nl > kCwLongCap) {            // too wide: back to the lists
            to_global(s_f[cur], nf, k);
            return;
        }
        const uint32_t nl = s_nl;
        uint32_t *nxt = s_f[cur ^ 1];
        // the first four entries of every column, kCwGroup columns at a time
#pragma unroll
        for (uint32_t g0 = 0; g0 < kCwPer; g0 += kCwGroup) {
            int32_t v[kCwGroup][4];
            unsigned long long old[kCwGroup][4];
#pragma unroll
            for (uint32_t j = 0; j < kCwGroup; ++j)
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) {
                    v[j][e] = -1;
                    if (e < degs[g0 + j]) v[j][e] = refs[g0 + j].idx[r0s[g0 + j] + (int32_t)e];
                }
#pragma unroll
            for (uint32_t j = 0; j < kCwGroup; ++j) {
                const unsigned long long key = offer_key(k + 1, xs[g0 + j] - refs[g0 + j].base);
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) {
                    old[j][e] = 0ull;
                    if (e < degs[g0 + j])
                        old[j][e] = atomicMin(&P.cw[refs[g0 + j].base + (uint32_t)v[j][e]], key);
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kCwGroup; ++j)
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) settle_after_issue(old[j][e]);
#pragma unroll
            for (uint32_t j = 0; j < kCwGroup; ++j)
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e)
                    if (unreached(old[j][e])) {
                        const uint32_t pos = atomicAdd(&s_n[cur ^ 1], 1u);
                        const uint32_t x = refs[g0 + j].base + (uint32_t)v[j][e];
                        if (pos < kCwCap) nxt[pos] = x;
                        else P.spill[pos - kCwCap] = x;
                    }
        }
        // the rest of the longer columns: 256-entry pieces, a wave each
        if (nl) {
            uint32_t total = 0;
            // nl <= 2048: two columns per thread
            const uint32_t i0 = 2 * tid, i1 = 2 * tid + 1;
            const uint32_t p0 = i0 < nl ? (s_ldeg[i0] + 255u) / 256u : 0u;
            const uint32_t p1 = i1 < nl ? (s_ldeg[i1] + 255u) / 256u : 0u;
            const uint32_t ex = block_excl_scan(p0 + p1, s_scan, &total);
            if (i0 < nl) s_lpre[i0] = ex;
            if (i1 < nl) s_lpre[i1] = ex + p0;
            if (tid == 0) s_lpre[nl] = total;
            __syncthreads();
            for (uint32_t it = wave; it < total; it += kCwNarrowThreads / 64) {
                uint32_t lo = 0, hi = nl;                  // s_lpre[lo] <= it < s_lpre[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_lpre[mid] <= it) lo = mid;
                    else hi = mid;
                }
                const uint32_t x = s_lx[lo];
                const Ref r = ref_of<kSingle>(P, one, x);
                const int32_t e0 = s_lr0[lo] + (int32_t)((it - s_lpre[lo]) * 256u);
                const int32_t end = s_lr0[lo] + (int32_t)s_ldeg[lo];
                const unsigned long long key = offer_key(k + 1, x - r.base);
                int32_t vv[4];
                unsigned long long oo[4];
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) {
                    const int32_t ei = e0 + (int32_t)(e * 64u + lane);
                    vv[e] = -1;
                    if (ei < end) vv[e] = r.idx[ei];
                }
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) {
                    oo[e] = 0ull;
                    if (e0 + (int32_t)(e * 64u + lane) < end) oo[e] = atomicMin(&P.cw[r.base + (uint32_t)vv[e]], key);
                }
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e) settle_after_issue(oo[e]);
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e)
                    if (unreached(oo[e])) {
                        const uint32_t pos = atomicAdd(&s_n[cur ^ 1], 1u);
                        const uint32_t y = r.base + (uint32_t)vv[e];
                        if (pos < kCwCap) nxt[pos] = y;
                        else P.spill[pos - kCwCap] = y;
                    }
            }
        }
        __syncthreads();
        if (s_n[cur ^ 1] > max_next) {                     // the next frontier is too wide
            to_global(nxt, s_n[cur ^ 1], k + 1);
            return;
        }
        cur ^= 1;
    }
}

// The words into the callers' arrays: a block row per query.
__global__ __launch_bounds__(kCwBlock) void k_cw_out(CwParams P) {
    const CwQuery &Q = P.q[blockIdx.y];
    for (uint32_t v = blockIdx.x * kCwBlock + threadIdx.x; v < Q.n; v += gridDim.x * kCwBlock) {
        const unsigned long long w = P.cw[Q.base + v];
        const bool r = !unreached(w);
        Q.level[v] = r ? (int32_t)(w >> 32) : -1;
        Q.parent[v] = r ? (int32_t)(uint32_t)w : -1;
    }
}

hipError_t launch_cw_init(const CwParams &p, hipStream_t s) {
    uint32_t g = (p.max_n + kCwBlock - 1) / kCwBlock;
    g = g < 2048u ? (g ? g : 1u) : 2048u;
    hipLaunchKernelGGL(k_cw_fill, dim3(g, p.nq), dim3(kCwBlock), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cw_roots, dim3((p.nq + kCwBlock - 1) / kCwBlock), dim3(kCwBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_cw_wide(const CwParams &p, uint32_t k, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_cw_wide, dim3(grid), dim3(kCwBlock), 0, s, p, k);
    return hipGetLastError();
}

hipError_t launch_cw_narrow(const CwParams &p, uint32_t k, uint32_t max_levels, uint32_t max_next,
                            uint32_t max_edges, hipStream_t s) {
    max_next = max_next < kCwCap ? max_next : kCwCap;
    max_edges = max_edges < kCwNarrowEdges ? max_edges : kCwNarrowEdges;
    if (p.nq == 1)
        hipLaunchKernelGGL(k_cw_narrow<true>, dim3(1), dim3(kCwNarrowThreads), 0, s, p, k, max_levels, max_next,
                           max_edges);
    else
        hipLaunchKernelGGL(k_cw_narrow<false>, dim3(1), dim3(kCwNarrowThreads), 0, s, p, k, max_levels, max_next,
                           max_edges);
    return hipGetLastError();
}

// The queries' out-lists into one block-diagonal CSR: row base_q + v holds
// query q's row v with every entry offset by base_q (a block row of the grid
// per query; the packed offsets of a query's last row and the next query's
// first are the same number, written by both).
__global__ __launch_bounds__(kCwBlock) void k_pack(PackParams P) {
    const PackQuery &Q = P.q[blockIdx.y];
    const uint32_t t0 = blockIdx.x * kCwBlock + threadIdx.x, ts = gridDim.x * kCwBlock;
    for (uint32_t v = t0; v <= Q.n; v += ts) P.ptr[Q.base + v] = Q.ptr[v] + (int32_t)Q.ebase;
    for (uint32_t e = t0; e < Q.nnz; e += ts) P.idx[Q.ebase + e] = Q.idx[e] + (int32_t)Q.base;
    if (blockIdx.y == 0)
        for (uint32_t e = P.E + t0; e < P.pad_end; e += ts) P.idx[e] = 0;
}

// The packed results into the callers' arrays (parents back to the query's ids).
__global__ __launch_bounds__(kCwBlock) void k_unpack(PackParams P) {
    const PackQuery &Q = P.q[blockIdx.y];
    for (uint32_t v = blockIdx.x * kCwBlock + threadIdx.x; v < Q.n; v += gridDim.x * kCwBlock) {
        const int32_t l = P.level[Q.base + v], p = P.parent[Q.base + v];
        Q.level[v] = l;
        Q.parent[v] = p >= 0 ? p - (int32_t)Q.base : -1;
    }
}

hipError_t launch_pack(const PackParams &p, hipStream_t s) {
    const uint32_t work = p.max_nnz > p.max_n + 1u ? p.max_nnz : p.max_n + 1u;
    uint32_t gx = (work + kCwBlock - 1) / kCwBlock;
    gx = gx < 1024u ? (gx ? gx : 1u) : 1024u;
    hipLaunchKernelGGL(k_pack, dim3(gx, p.nq), dim3(kCwBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_unpack(const PackParams &p, hipStream_t s) {
    uint32_t gx = (p.max_n + kCwBlock - 1) / kCwBlock;
    gx = gx < 1024u ? (gx ? gx : 1u) : 1024u;
    hipLaunchKernelGGL(k_unpack, dim3(gx, p.nq), dim3(kCwBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_cw_out(const CwParams &p, hipStream_t s) {
    uint32_t gx = (p.max_n + kCwBlock - 1) / kCwBlock;
    gx = gx < 1024u ? (gx ? gx : 1u) : 1024u;
    hipLaunchKernelGGL(k_cw_out, dim3(gx, p.nq), dim3(kCwBlock), 0, s, p);
    return hipGetLastError();
}

}  // namespace bfsi

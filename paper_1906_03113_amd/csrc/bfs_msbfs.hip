// Many searches on one graph at once: the masked product of Theorem 1 applied
// to Q sources side by side, 64 sources per 64-bit word per vertex.
//
// For source q, row v and level k the recurrence is the single-source one:
// v joins source q's frontier at level k+1 when some frontier vertex u of
// source q has an edge u -> v and v was not reached by q through level k.  So
// with cur[u] = the sources whose level-k frontier holds u and vis[v] = the
// sources that reached v through level k, one pass over the frontier's columns
// computes, for every entry (u, v),
//     new = cur[u] & ~vis[v]      and      nxt[v] |= new,
// i.e. one read of each column serves every source whose frontier holds it.
//
// The parent of v for source q is, as everywhere in this library, the
// smallest frontier in-neighbour; the settle pass finds it by scanning v's
// in-neighbours in ascending order and giving each still-unassigned source
// bit to the first u whose cur[u] holds it.  A wave scans 64 entries per
// step, and an OR prefix across its lanes gives each bit to the lowest lane
// that holds it.  Long lists (>= kMsLong entries) are split into chunks of
// kMsChunk entries scanned by different waves, which combine with atomicMin
// on the parent (the same minimum).  The push form splits long columns the
// same way.  Level k's mask buffers rotate over three slots so the one that
// held F_{k-1} can be cleared while level k runs.  Results are bit-identical
// to single-source searches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_internal.h"

namespace bfsi {

namespace {

__device__ __forceinline__ const unsigned long long *row(const unsigned long long *m, int32_t v,
                                                         uint32_t W) {
    return m + (size_t)v * W;
}
__device__ __forceinline__ unsigned long long *row(unsigned long long *m, int32_t v, uint32_t W) {
    return m + (size_t)v * W;
}

// selects instead of indexing the parameter arrays with a runtime index
template <typename T>
__device__ __forceinline__ T pick3(T a, T b, T c, uint32_t s) {
    return s == 0 ? a : (s == 1 ? b : c);
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return (uint32_t)__popcll(m & ((1ull << __lane_id()) - 1ull));
}

// OR of x over lanes 0..lane (inclusive), every lane of the wave taking part
__device__ __forceinline__ unsigned long long wave_or_incl(unsigned long long x, uint32_t lane) {
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const unsigned long long t = __shfl_up(x, d, 64);
        if (lane >= d) x |= t;
    }
    return x;
}

// Append vertex v with `deg` entries to a split list: one packed atomic gives
// its entry index and first chunk id; its chunks map back to the entry.
__device__ __forceinline__ void add_long(MsLong *ents, uint32_t *map, unsigned long long *ctr, int32_t v,
                                         uint32_t deg) {
    const uint32_t nch = (deg + kMsChunk - 1u) / kMsChunk;
    const unsigned long long old = atomicAdd(ctr, 1ull | ((unsigned long long)nch << 32));
    const uint32_t idx = (uint32_t)old, base = (uint32_t)(old >> 32);
    MsLong e;
    e.v = v;
    e.chunk_base = base;
    ents[idx] = e;
    for (uint32_t c = 0; c < nch; ++c) map[base + c] = idx;
}

// One step of the settle scan over in_idx[eb + lane] (lanes past e1 hold
// nothing): each bit of rem held by some lane's cur mask goes to the lowest
// such lane, i.e. to the smallest in-neighbour of the step.  Returns the bits
// found (the same in every lane).
__device__ __forceinline__ unsigned long long settle_step(const MsLevel &p, const unsigned long long *cur,
                                                          int32_t v, uint32_t w, int32_t eb, int32_t e1,
                                                          unsigned long long rem, uint32_t lk,
                                                          bool owner_alone) {
    const uint32_t lane = __lane_id();
    const int32_t e = eb + (int32_t)lane;
    int32_t u = -1;
    unsigned long long hit = 0ull;
    if (e < e1) {
        u = p.in_idx[e];
        hit = row(cur, u, p.W)[w] & rem;
    }
    const unsigned long long incl = wave_or_incl(hit, lane);
    unsigned long long below = __shfl_up(incl, 1u, 64);
    if (lane == 0) below = 0ull;
    unsigned long long own = hit & ~below;
    while (own) {
        const uint32_t b = (uint32_t)__ffsll((long long)own) - 1u;
        own &= own - 1ull;
        const uint32_t q = w * 64u + b;
        p.level[q][v] = (int32_t)lk;
        if (owner_alone) p.parent[q][v] = u;
        else atomicMin((uint32_t *)&p.parent[q][v], (uint32_t)u);
    }
    return __shfl(incl, 63, 64);
}

}  // namespace

// Outputs to -1 (every source, every vertex) and every mask to zero.
__global__ __launch_bounds__(kBlock) void k_ms_clear(MsLevel p) {
    const size_t gid = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * kBlock;
    const size_t nw = (size_t)p.n * p.W;
    for (size_t i = gid; i < nw; i += stride) {
        p.vis[i] = 0ull;
        p.m[0][i] = 0ull;
        p.m[1][i] = 0ull;
        p.m[2][i] = 0ull;
    }
    for (size_t v = gid; v < (size_t)p.n; v += stride) p.flag[v] = 0u;
    const size_t tot = (size_t)p.n * p.nq;
    for (size_t i = gid; i < tot; i += stride) {
        const uint32_t q = (uint32_t)(i / (size_t)p.n);
        const size_t v = i - (size_t)q * p.n;
        p.level[q][v] = -1;
        p.parent[q][v] = -1;
    }
    if (gid < 4) p.cnt[gid] = 0u;
    if (gid < 6) p.lcnt[gid] = 0ull;
}

// Sources: bit q set in cur and vis of its vertex, level 0, parent itself; each
// distinct source vertex enters the level-0 list once (and the split list of
// long columns when its out-degree is long).
__global__ __launch_bounds__(kBlock) void k_ms_roots(MsLevel p) {
    const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= p.nq) return;
    const int32_t s = p.sources[q];
    const unsigned long long bit = 1ull << (q & 63);
    atomicOr(&row(p.m[0], s, p.W)[q >> 6], bit);
    atomicOr(&row(p.vis, s, p.W)[q >> 6], bit);
    p.level[q][s] = 0;
    p.parent[q][s] = s;
    if (atomicMax(&p.flag[s], 1u) < 1u) {
        p.fq[0][atomicAdd(&p.cnt[0], 1u)] = s;
        const uint32_t od = (uint32_t)(p.out_ptr[s + 1] - p.out_ptr[s]);
        if (od >= kMsLong) add_long(p.pl[0], p.pmap[0], &p.lcnt[0], s, od);
    }
}

// Level k, push half.  Work items, one wave each: the frontier columns with
// fewer than kMsLong entries (lanes over the entries), then the chunks of the
// long ones.  Per entry (u, v): new = cur[u] & ~vis[v] is ORed into nxt[v], and
// v is listed for level k+1 once (and split for the settle pass when its
// in-list is long).  Also clears the masks of F_{k-1} (slot (k+2) % 3).
__global__ __launch_bounds__(kBlock) void k_ms_push(MsLevel p, uint32_t k) {
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s0);
    unsigned long long *nxt = pick3(p.m[0], p.m[1], p.m[2], s1);
    unsigned long long *old = pick3(p.m[0], p.m[1], p.m[2], s2);
    const int32_t *fcur = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s0);
    int32_t *fnxt = pick3(p.fq[0], p.fq[1], p.fq[2], s1);
    const int32_t *fold = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s2);
    const MsLong *lcur = pick3<const MsLong *>(p.pl[0], p.pl[1], p.pl[2], s0);
    const uint32_t *lmap = pick3<const uint32_t *>(p.pmap[0], p.pmap[1], p.pmap[2], s0);
    MsLong *snew = pick3(p.sl[0], p.sl[1], p.sl[2], s1);
    uint32_t *smap = pick3(p.smap[0], p.smap[1], p.smap[2], s1);
    unsigned long long *sctr = p.lcnt + 3 + s1;
    const uint32_t ncur = p.cnt[s0], nold = p.cnt[s2];
    const uint32_t nchunks = (uint32_t)(p.lcnt[s0] >> 32);
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    for (uint32_t t = gt; t < nold * W; t += gs) {
        const uint32_t u = (uint32_t)fold[t / W];
        old[(size_t)u * W + (t % W)] = 0ull;
    }
    const uint32_t lane = __lane_id();
    const uint32_t wave = gt >> 6;
    const uint32_t nwaves = gs >> 6;
    const uint32_t tag = k + 2;          // "listed for level k+1"
    for (uint32_t it = wave; it < ncur + nchunks; it += nwaves) {
        int32_t u, e0, e1;
        if (it < ncur) {
            u = fcur[it];
            e0 = p.out_ptr[u];
            e1 = p.out_ptr[u + 1];
            if ((uint32_t)(e1 - e0) >= kMsLong) continue;        // done by its chunks
        } else {
            const uint32_t c = it - ncur;
            const MsLong L = lcur[lmap[c]];
            u = L.v;
            const int32_t r1 = p.out_ptr[u + 1];
            e0 = p.out_ptr[u] + (int32_t)((c - L.chunk_base) * kMsChunk);
            e1 = (e0 + (int32_t)kMsChunk < r1) ? e0 + (int32_t)kMsChunk : r1;
        }
        const unsigned long long *cu = row(cur, u, W);
        for (int32_t e = e0 + (int32_t)lane; e < e1; e += 64) {
            const int32_t v = p.out_idx[e];
            const unsigned long long *vv = row(p.vis, v, W);
            unsigned long long *nv = row(nxt, v, W);
            bool any = false;
            for (uint32_t w = 0; w < W; ++w) {
                const unsigned long long nb = cu[w] & ~vv[w];
                if (nb) {
                    atomicOr(&nv[w], nb);
                    any = true;
                }
            }
            const bool listed = any && atomicMax(&p.flag[v], tag) < tag;
            const unsigned long long bm = __ballot(listed);
            if (bm) {
                const uint32_t leader = (uint32_t)__ffsll((long long)bm) - 1u;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&p.cnt[s1], (uint32_t)__popcll(bm));
                base = __shfl(base, (int)leader, 64);
                if (listed) {
                    fnxt[base + lanes_below(bm)] = v;
                    const uint32_t id = (uint32_t)(p.in_ptr[v + 1] - p.in_ptr[v]);
                    if (id >= kMsLong) add_long(snew, smap, sctr, v, id);
                }
            }
        }
    }
}

// Level k, settle half: one wave per newly listed vertex v with a short
// in-list, one wave per chunk of a long one.  The new bits join vis (by the
// vertex's own item); each gets level k+1 and its parent = the first
// in-neighbour (ascending) whose level-k frontier mask holds it.  Every
// listed vertex with a long out-list is split for the next push.
__global__ __launch_bounds__(kBlock) void k_ms_settle(MsLevel p, uint32_t k) {
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s0);
    const unsigned long long *nxt = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s1);
    const int32_t *fnxt = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s1);
    const MsLong *lst = pick3<const MsLong *>(p.sl[0], p.sl[1], p.sl[2], s1);
    const uint32_t *lmap = pick3<const uint32_t *>(p.smap[0], p.smap[1], p.smap[2], s1);
    MsLong *pnew = pick3(p.pl[0], p.pl[1], p.pl[2], s1);
    uint32_t *pmap = pick3(p.pmap[0], p.pmap[1], p.pmap[2], s1);
    unsigned long long *pctr = p.lcnt + s1;
    const uint32_t nnext = p.cnt[s1];
    const uint32_t nchunks = (uint32_t)(p.lcnt[3 + s1] >> 32);
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    const uint32_t lane = __lane_id();
    if (gt == 0) {
        p.cnt[s2] = 0u;                       // the lists of level k+2 start empty
        p.lcnt[s2] = 0ull;
        p.lcnt[3 + s2] = 0ull;
        p.host_status[0] = k + 1;
        p.host_status[1] = nnext;
        __threadfence_system();
    }
    for (uint32_t it = gt >> 6; it < nnext + nchunks; it += gs >> 6) {
        int32_t v, e0, e1;
        bool alone;
        if (it < nnext) {
            v = fnxt[it];
            if (lane == 0) {
                const uint32_t od = (uint32_t)(p.out_ptr[v + 1] - p.out_ptr[v]);
                if (od >= kMsLong) add_long(pnew, pmap, pctr, v, od);
            }
            e0 = p.in_ptr[v];
            e1 = p.in_ptr[v + 1];
            if ((uint32_t)(e1 - e0) >= kMsLong) {      // parents by the chunks
                for (uint32_t w = lane; w < W; w += 64) row(p.vis, v, W)[w] |= row(nxt, v, W)[w];
                continue;
            }
            alone = true;
        } else {
            const uint32_t c = it - nnext;
            const MsLong L = lst[lmap[c]];
            v = L.v;
            const int32_t r1 = p.in_ptr[v + 1];
            e0 = p.in_ptr[v] + (int32_t)((c - L.chunk_base) * kMsChunk);
            e1 = (e0 + (int32_t)kMsChunk < r1) ? e0 + (int32_t)kMsChunk : r1;
            alone = false;
        }
        for (uint32_t w = 0; w < W; ++w) {
            const unsigned long long nb = row(nxt, v, W)[w];
            if (!nb) continue;
            if (alone && lane == 0) row(p.vis, v, W)[w] |= nb;      // one writer per (v, w)
            unsigned long long rem = nb;
            for (int32_t eb = e0; eb < e1 && rem; eb += 64)
                rem &= ~settle_step(p, cur, v, w, eb, e1, rem, k + 1, alone);
        }
    }
}

// Level k, pull form (for large frontiers): every vertex v whose sources are
// not all settled ORs, in ascending in-neighbour order, the frontier masks of
// its in-neighbours restricted to the sources that have not reached it; each
// source bit found first at u gets parent u (the smallest frontier
// in-neighbour for that source) and level k+1.  Rows of up to kMsSerial
// entries are scanned by one lane, longer ones by a wave (settle_step).  The
// owner of v writes vis and the next mask without atomics; vertices with new
// bits are listed (one atomicAdd per block chunk) and split for the next push
// when their out-list is long.  Also clears F_{k-1}'s masks.
constexpr uint32_t kMsRows = 2048;       // rows per block chunk
constexpr int32_t kMsSerial = 16;        // longest row one lane scans alone

__global__ __launch_bounds__(kBlock) void k_ms_pull(MsLevel p, uint32_t k) {
    __shared__ int32_t s_list[kMsRows];
    __shared__ int32_t s_long[kMsRows];
    __shared__ uint32_t s_n, s_nl, s_base;
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s0);
    unsigned long long *nxt = pick3(p.m[0], p.m[1], p.m[2], s1);
    unsigned long long *old = pick3(p.m[0], p.m[1], p.m[2], s2);
    int32_t *fnxt = pick3(p.fq[0], p.fq[1], p.fq[2], s1);
    const int32_t *fold = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s2);
    MsLong *pnew = pick3(p.pl[0], p.pl[1], p.pl[2], s1);
    uint32_t *pmap = pick3(p.pmap[0], p.pmap[1], p.pmap[2], s1);
    unsigned long long *pctr = p.lcnt + s1;
    const uint32_t nold = p.cnt[s2];
    const uint32_t W = p.W;
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const uint32_t gt = blockIdx.x * kBlock + tid, gs = gridDim.x * kBlock;
    for (uint32_t t = gt; t < nold * W; t += gs) {
        const uint32_t u = (uint32_t)fold[t / W];
        old[(size_t)u * W + (t % W)] = 0ull;
    }
    const uint32_t tail = p.nq & 63u;
    const uint32_t lk = k + 1;
    for (uint32_t c0 = blockIdx.x * kMsRows; c0 < (uint32_t)p.n; c0 += gridDim.x * kMsRows) {
        if (tid == 0) {
            s_n = 0;
            s_nl = 0;
        }
        __syncthreads();
        const uint32_t c1 = (c0 + kMsRows < (uint32_t)p.n) ? c0 + kMsRows : (uint32_t)p.n;
        for (uint32_t vv = c0 + tid; vv < c1; vv += kBlock) {
            const int32_t v = (int32_t)vv;
            const int32_t e0 = p.in_ptr[v], e1 = p.in_ptr[v + 1];
            if (e1 == e0) continue;
            unsigned long long *vis = row(p.vis, v, W);
            bool open = false;
            for (uint32_t w = 0; w < W && !open; ++w) {
                const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                open = (full & ~vis[w]) != 0ull;
            }
            if (!open) continue;                         // every source has reached v
            if (e1 - e0 > kMsSerial) {
                s_long[atomicAdd(&s_nl, 1u)] = v;
                continue;
            }
            unsigned long long *nv = row(nxt, v, W);
            bool any = false;
            for (uint32_t w = 0; w < W; ++w) {
                const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                const unsigned long long sv = vis[w];
                unsigned long long rem = full & ~sv, found = 0ull;
                for (int32_t e = e0; e < e1 && rem; ++e) {
                    const int32_t u = p.in_idx[e];
                    unsigned long long hit = row(cur, u, W)[w] & rem;
                    if (!hit) continue;
                    rem &= ~hit;
                    found |= hit;
                    while (hit) {
                        const uint32_t b = (uint32_t)__ffsll((long long)hit) - 1u;
                        hit &= hit - 1ull;
                        const uint32_t q = w * 64u + b;
                        p.level[q][v] = (int32_t)lk;
                        p.parent[q][v] = u;
                    }
                }
                if (found) {
                    nv[w] = found;
                    vis[w] = sv | found;
                    any = true;
                }
            }
            if (any) {
                s_list[atomicAdd(&s_n, 1u)] = v;
                const uint32_t od = (uint32_t)(p.out_ptr[v + 1] - p.out_ptr[v]);
                if (od >= kMsLong) add_long(pnew, pmap, pctr, v, od);
            }
        }
        __syncthreads();
        const uint32_t nl = s_nl;
        for (uint32_t i = wave; i < nl; i += kBlock / 64) {           // long rows: a wave each
            const int32_t v = s_long[i];
            const int32_t e0 = p.in_ptr[v], e1 = p.in_ptr[v + 1];
            unsigned long long *vis = row(p.vis, v, W);
            unsigned long long *nv = row(nxt, v, W);
            bool any = false;
            for (uint32_t w = 0; w < W; ++w) {
                const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                const unsigned long long sv = vis[w];
                unsigned long long rem = full & ~sv, found = 0ull;
                for (int32_t eb = e0; eb < e1 && rem; eb += 64) {
                    const unsigned long long f = settle_step(p, cur, v, w, eb, e1, rem, lk, true);
                    rem &= ~f;
                    found |= f;
                }
                if (found) {
                    if (lane == 0) {
                        nv[w] = found;
                        vis[w] = sv | found;
                    }
                    any = true;
                }
            }
            if (any && lane == 0) {
                s_list[atomicAdd(&s_n, 1u)] = v;
                const uint32_t od = (uint32_t)(p.out_ptr[v + 1] - p.out_ptr[v]);
                if (od >= kMsLong) add_long(pnew, pmap, pctr, v, od);
            }
        }
        __syncthreads();
        if (tid == 0 && s_n) s_base = atomicAdd(&p.cnt[s1], s_n);
        __syncthreads();
        for (uint32_t i = tid; i < s_n; i += kBlock) fnxt[s_base + i] = s_list[i];
        __syncthreads();
    }
}

// After a pull level: the lists of level k+2 start empty; report to the host.
__global__ void k_ms_report(MsLevel p, uint32_t k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t s2 = (k + 2) % 3;
    p.cnt[s2] = 0u;
    p.lcnt[s2] = 0ull;
    p.lcnt[3 + s2] = 0ull;
    p.host_status[0] = k + 1;
    p.host_status[1] = p.cnt[(k + 1) % 3];
    __threadfence_system();
}

hipError_t launch_ms(const MsLevel &p, int phase, uint32_t k, uint32_t grid, hipStream_t s) {
    switch (phase) {
        case 0: hipLaunchKernelGGL(k_ms_clear, dim3(grid), dim3(kBlock), 0, s, p); break;
        case 1: hipLaunchKernelGGL(k_ms_roots, dim3((p.nq + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p); break;
        case 2: hipLaunchKernelGGL(k_ms_push, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        case 3: hipLaunchKernelGGL(k_ms_settle, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        case 4: hipLaunchKernelGGL(k_ms_pull, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        default: hipLaunchKernelGGL(k_ms_report, dim3(1), dim3(64), 0, s, p, k); break;
    }
    return hipGetLastError();
}

}  // namespace bfsi

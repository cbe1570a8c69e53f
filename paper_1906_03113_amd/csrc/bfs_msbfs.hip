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
// bit to the first u whose cur[u] holds it.  Level k's mask buffers rotate
// over three slots so the one that held F_{k-1} can be cleared while level k
// runs.  Results are bit-identical to single-source searches.
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
}

// Sources: bit q set in cur and vis of its vertex, level 0, parent itself; each
// distinct source vertex enters the level-0 list once.
__global__ __launch_bounds__(kBlock) void k_ms_roots(MsLevel p) {
    const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= p.nq) return;
    const int32_t s = p.sources[q];
    const unsigned long long bit = 1ull << (q & 63);
    atomicOr(&row(p.m[0], s, p.W)[q >> 6], bit);
    atomicOr(&row(p.vis, s, p.W)[q >> 6], bit);
    p.level[q][s] = 0;
    p.parent[q][s] = s;
    if (atomicMax(&p.flag[s], 1u) < 1u) p.fq[0][atomicAdd(&p.cnt[0], 1u)] = s;
}

// Level k, push half: one wave per frontier column, lanes over its entries.
// Also clears the masks of F_{k-1} (slot (k+2) % 3), which nobody reads now.
__global__ __launch_bounds__(kBlock) void k_ms_push(MsLevel p, uint32_t k) {
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = s0 == 0 ? p.m[0] : (s0 == 1 ? p.m[1] : p.m[2]);
    unsigned long long *nxt = s1 == 0 ? p.m[0] : (s1 == 1 ? p.m[1] : p.m[2]);
    unsigned long long *old = s2 == 0 ? p.m[0] : (s2 == 1 ? p.m[1] : p.m[2]);
    const int32_t *fcur = s0 == 0 ? p.fq[0] : (s0 == 1 ? p.fq[1] : p.fq[2]);
    int32_t *fnxt = s1 == 0 ? p.fq[0] : (s1 == 1 ? p.fq[1] : p.fq[2]);
    const int32_t *fold = s2 == 0 ? p.fq[0] : (s2 == 1 ? p.fq[1] : p.fq[2]);
    const uint32_t ncur = p.cnt[s0], nold = p.cnt[s2];
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    for (uint32_t t = gt; t < nold * W; t += gs) {
        const uint32_t u = (uint32_t)fold[t / W];
        old[(size_t)u * W + (t % W)] = 0ull;
    }
    const uint32_t lane = __lane_id();
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * kBlock) >> 6;
    const uint32_t tag = k + 2;          // "queued for level k+1"
    for (uint32_t f = wave; f < ncur; f += nwaves) {
        const int32_t u = fcur[f];
        const unsigned long long *cu = row(cur, u, W);
        const int32_t e1 = p.out_ptr[u + 1];
        for (int32_t e = p.out_ptr[u] + (int32_t)lane; e < e1; e += 64) {
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
            if (any && atomicMax(&p.flag[v], tag) < tag) fnxt[atomicAdd(&p.cnt[s1], 1u)] = v;
        }
    }
}

// Level k, settle half: one thread per (new frontier vertex, word).  The new
// bits join vis; each gets level k+1 and its parent = the first in-neighbour
// (ascending) whose level-k frontier mask holds it.
__global__ __launch_bounds__(kBlock) void k_ms_settle(MsLevel p, uint32_t k) {
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = s0 == 0 ? p.m[0] : (s0 == 1 ? p.m[1] : p.m[2]);
    const unsigned long long *nxt = s1 == 0 ? p.m[0] : (s1 == 1 ? p.m[1] : p.m[2]);
    const int32_t *fnxt = s1 == 0 ? p.fq[0] : (s1 == 1 ? p.fq[1] : p.fq[2]);
    const uint32_t nnext = p.cnt[s1];
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    for (uint32_t t = gt; t < nnext * W; t += gs) {
        const int32_t v = fnxt[t / W];
        const uint32_t w = t % W;
        const unsigned long long nb = row(nxt, v, W)[w];
        if (!nb) continue;
        row(p.vis, v, W)[w] |= nb;            // one thread per (v, w): no race
        unsigned long long rem = nb;
        const int32_t e1 = p.in_ptr[v + 1];
        for (int32_t e = p.in_ptr[v]; e < e1 && rem; ++e) {
            const int32_t u = p.in_idx[e];
            unsigned long long hit = row(cur, u, W)[w] & rem;
            rem &= ~hit;
            while (hit) {
                const uint32_t b = (uint32_t)__ffsll((long long)hit) - 1u;
                hit &= hit - 1ull;
                const uint32_t q = w * 64u + b;
                p.level[q][v] = (int32_t)(k + 1);
                p.parent[q][v] = u;
            }
        }
    }
    if (gt == 0) {
        p.cnt[s2] = 0u;                       // the list of level k+2 starts empty
        p.host_status[0] = k + 1;
        p.host_status[1] = nnext;
        __threadfence_system();
    }
}

// Level k, pull form (for large frontiers): every vertex v whose sources are
// not all settled ORs, in ascending in-neighbour order, the frontier masks of
// its in-neighbours restricted to the sources that have not reached it; each
// source bit found first at u gets parent u (the smallest frontier
// in-neighbour for that source) and level k+1.  One thread owns v, so vis and
// the next mask are written without atomics; vertices with new bits are
// listed (one atomicAdd per block chunk).  Also clears F_{k-1}'s masks.
constexpr uint32_t kMsChunk = 2048;

__global__ __launch_bounds__(kBlock) void k_ms_pull(MsLevel p, uint32_t k) {
    __shared__ int32_t s_list[kMsChunk];
    __shared__ uint32_t s_n, s_base;
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = s0 == 0 ? p.m[0] : (s0 == 1 ? p.m[1] : p.m[2]);
    unsigned long long *nxt = s1 == 0 ? p.m[0] : (s1 == 1 ? p.m[1] : p.m[2]);
    unsigned long long *old = s2 == 0 ? p.m[0] : (s2 == 1 ? p.m[1] : p.m[2]);
    int32_t *fnxt = s1 == 0 ? p.fq[0] : (s1 == 1 ? p.fq[1] : p.fq[2]);
    const int32_t *fold = s2 == 0 ? p.fq[0] : (s2 == 1 ? p.fq[1] : p.fq[2]);
    const uint32_t nold = p.cnt[s2];
    const uint32_t W = p.W;
    const uint32_t tid = threadIdx.x;
    const uint32_t gt = blockIdx.x * kBlock + tid, gs = gridDim.x * kBlock;
    for (uint32_t t = gt; t < nold * W; t += gs) {
        const uint32_t u = (uint32_t)fold[t / W];
        old[(size_t)u * W + (t % W)] = 0ull;
    }
    const uint32_t tail = p.nq & 63u;
    for (uint32_t c0 = blockIdx.x * kMsChunk; c0 < (uint32_t)p.n; c0 += gridDim.x * kMsChunk) {
        if (tid == 0) s_n = 0;
        __syncthreads();
        const uint32_t c1 = (c0 + kMsChunk < (uint32_t)p.n) ? c0 + kMsChunk : (uint32_t)p.n;
        for (uint32_t vv = c0 + tid; vv < c1; vv += kBlock) {
            const int32_t v = (int32_t)vv;
            const int32_t e0 = p.in_ptr[v], e1 = p.in_ptr[v + 1];
            unsigned long long *vis = row(p.vis, v, W);
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
                        p.level[q][v] = (int32_t)(k + 1);
                        p.parent[q][v] = u;
                    }
                }
                nv[w] = found;
                if (found) {
                    vis[w] = sv | found;
                    any = true;
                }
            }
            if (any) s_list[atomicAdd(&s_n, 1u)] = v;
        }
        __syncthreads();
        if (tid == 0 && s_n) s_base = atomicAdd(&p.cnt[s1], s_n);
        __syncthreads();
        for (uint32_t i = tid; i < s_n; i += kBlock) fnxt[s_base + i] = s_list[i];
        __syncthreads();
    }
}

// After a pull level: the list of level k+2 starts empty; report to the host.
__global__ void k_ms_report(MsLevel p, uint32_t k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    p.cnt[(k + 2) % 3] = 0u;
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

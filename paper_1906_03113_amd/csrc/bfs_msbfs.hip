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
// smallest frontier in-neighbour.  The push form takes it with atomicMin over
// the entries it visits; the pull form scans v's in-neighbours in ascending
// order and gives each still-unassigned source bit to the first u whose
// cur[u] holds it (a wave scans 64 entries per step, and an OR prefix across
// its lanes gives each bit to the lowest lane that holds it).  Lists of
// kMsLong entries or more are split into chunks of kMsChunk entries handled
// by different waves, which combine with atomicMin (the same minimum).
// Results are staged vertex-major and written to the callers' per-source
// arrays at the end.  Level k's mask buffers rotate over three slots so the
// one that held F_{k-1} can be cleared while level k runs.  Results are
// bit-identical to single-source searches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_device.h"
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

__device__ __forceinline__ size_t stage(const MsLevel &p, int32_t v, uint32_t q) {
    return (size_t)v * (p.W * 64u) + q;
}

// Whether u may hold frontier bits at this level (always, without the bitmap).
__device__ __forceinline__ bool in_frontier(const MsLevel &p, int32_t u) {
    return !p.use_fbits || ((p.fbits[(uint32_t)u >> 6] >> ((uint32_t)u & 63u)) & 1ull) != 0ull;
}

// With the graph's degree-ordered copy the kernels walk search labels: the
// caller's id of label x and the label of the caller's vertex v (identities
// in the caller's order).
__device__ __forceinline__ int32_t caller_id(const MsLevel &p, int32_t x) {
    return p.orig ? p.orig[x] : x;
}
__device__ __forceinline__ int32_t label_of(const MsLevel &p, int32_t v) {
    return p.pos ? p.pos[v] : v;
}
// The staged row of label x: the label itself when the staged results are
// the library's own (k_ms_out maps them back), else the caller's id.
__device__ __forceinline__ int32_t srow(const MsLevel &p, int32_t x) {
    return p.stage_labels ? x : caller_id(p, x);
}

// One step of the settle scan by a group of G lanes (G = 16 or 64, aligned
// within the wave) over in_idx[eb + lane-in-group] (lanes past e1 hold
// nothing): each bit of rem held by some lane's cur mask goes to the lowest
// such lane, i.e. to the smallest in-neighbour of the step.  Returns the bits
// found (the same in every lane of the group).  vo is the row's caller id
// (its staged results), parents are written as the entries' caller ids.
// scan_resolve is the second half, given each lane's entry (its caller id uc)
// and its mask bits already restricted to rem.
template <uint32_t G>
__device__ __forceinline__ unsigned long long scan_resolve(const MsLevel &p, int32_t vo, uint32_t w,
                                                           int32_t uc, unsigned long long hit,
                                                           uint32_t lk, bool owner_alone);

template <uint32_t G>
__device__ __forceinline__ unsigned long long scan_step(const MsLevel &p, const unsigned long long *cur,
                                                        int32_t vo, uint32_t w, int32_t eb, int32_t e1,
                                                        unsigned long long rem, uint32_t lk,
                                                        bool owner_alone) {
    const uint32_t li = __lane_id() & (G - 1u);
    const int32_t e = eb + (int32_t)li;
    int32_t uc = -1;
    unsigned long long hit = 0ull;
    if (e < e1) {
        const int32_t u = p.in_idx[e];
        if (in_frontier(p, u)) hit = row(cur, u, p.W)[w] & rem;
        if (hit) uc = caller_id(p, u);                  // only an entry that may give a parent
    }
    return scan_resolve<G>(p, vo, w, uc, hit, lk, owner_alone);
}

template <uint32_t G>
__device__ __forceinline__ unsigned long long scan_resolve(const MsLevel &p, int32_t vo, uint32_t w,
                                                           int32_t uc, unsigned long long hit,
                                                           uint32_t lk, bool owner_alone) {
    const uint32_t li = __lane_id() & (G - 1u);
    if (__ballot(hit != 0ull) == 0ull) return 0ull;        // (uniform) nothing found in the wave
    unsigned long long incl = hit;
#pragma unroll
    for (uint32_t d = 1; d < G; d <<= 1) {
        const unsigned long long t = __shfl_up(incl, d, (int)G);
        if (li >= d) incl |= t;
    }
    unsigned long long below = __shfl_up(incl, 1u, (int)G);
    if (li == 0) below = 0ull;
    unsigned long long own = hit & ~below;
    const unsigned long long found = __shfl(incl, (int)(G - 1u), (int)G);
    // each found bit's parent (the entry of the lane that owns it) through the
    // group's row of 64 LDS slots, then written by source: lane li takes
    // sources li, li + G, ..., so the staged row goes out in 64 / G stores
    // of consecutive entries instead of one store per bit
    __shared__ uint32_t s_par[kBlock / 64][(64 / G) * 64];   // a row per group of the wave
    uint32_t *slot = &s_par[threadIdx.x >> 6][(__lane_id() / G) * 64u];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (own) {
        const uint32_t b = (uint32_t)__ffsll((long long)own) - 1u;
        own &= own - 1ull;
        slot[b] = (uint32_t)uc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t b = li; b < 64u; b += G) {
        if ((found >> b) & 1ull) {
            const size_t at = stage(p, vo, w * 64u + b);
            const uint32_t pu = slot[b];
            p.slev[at] = (int32_t)lk;
            if (owner_alone) p.spar[at] = pu;
            else atomicMin(&p.spar[at], pu);
        }
    }
    return found;
}

}  // namespace

// Every mask to zero and every staged parent to 0xFFFFFFFF (parents are
// combined with atomicMin).  Staged levels are written before they are read
// (k_ms_out reads only entries whose vis bit is set), and k_ms_out writes
// every output; when the staged arrays are the caller's vertex-major outputs
// the levels start at -1 too (there is no k_ms_out).
typedef int32_t v4i __attribute__((ext_vector_type(4)));

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
    // staged parents, 16 bytes at a time, streaming stores (not read by
    // this kernel, and far larger than the caches)
    const size_t ns = (size_t)p.n * p.W * 16u;
    const v4i ones = {-1, -1, -1, -1};
    for (size_t i = gid; i < ns; i += stride) __builtin_nontemporal_store(ones, reinterpret_cast<v4i *>(p.spar) + i);
    if (p.fill_levels)                                  // the caller's arrays: unreached = -1
        for (size_t i = gid; i < ns; i += stride) __builtin_nontemporal_store(ones, reinterpret_cast<v4i *>(p.slev) + i);
    if (gid < 4) p.cnt[gid] = 0u;
    if (gid < 3) p.rcnt[gid] = 0u;
    if (gid < (size_t)kMsStatWords) p.mstat[gid] = 0ull;
}

// Sources: bit q set in cur and vis of its vertex, level 0, parent itself; each
// distinct source vertex enters the level-0 list once.
__global__ __launch_bounds__(kBlock) void k_ms_roots(MsLevel p) {
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    for (uint32_t q = gid; q < p.nq; q += gs) {
        const int32_t s = p.sources[q];                       // the caller's id
        const int32_t x = label_of(p, s);
        const unsigned long long bit = 1ull << (q & 63);
        atomicOr(&row(p.m[0], x, p.W)[q >> 6], bit);
        atomicOr(&row(p.vis, x, p.W)[q >> 6], bit);
        p.slev[stage(p, srow(p, x), q)] = 0;
        p.spar[stage(p, srow(p, x), q)] = (uint32_t)s;
        const int g = (int)(q % kMsDegGroups);
        atomicAdd(&p.mstat[ms_line(0, g) + 1], 1ull);              // one pair per source
        atomicAdd(&p.mstat[ms_line(kMsCumSlot, g) + 1], 1ull);
        if (atomicMax(&p.flag[x], 1u) < 1u) {
            p.fq[0][atomicAdd(&p.cnt[0], 1u)] = x;
            atomicAdd(&p.mstat[ms_line(0, g)], (unsigned long long)(p.out_ptr[x + 1] - p.out_ptr[x]));
            atomicAdd(&p.mstat[ms_line(kMsCumSlot, g)], 1ull);
        }
    }
}

// Level k, push half.  Work items: the frontier list, up to 64 columns per
// wave step - the entries of those with at most kMsShort entries dealt out one per
// lane, each longer one below kMsLong entries taken by the whole wave - then
// the chunks of the graph's long columns, a wave each, skipped unless the
// column is in some frontier.  Per
// entry (u, v): new = cur[u] & ~vis[v] is ORed into nxt[v], each of its bits q
// takes atomicMin(parent_q(v), u) - over all the entries this is the smallest
// frontier in-neighbour of v for q - and v is listed for level k+1 once,
// through a per-wave LDS buffer flushed with one atomic per kMsFlush entries.
// Also clears the masks of F_{k-1} (slot (k+2) % 3).
constexpr uint32_t kMsWaveBuf = 256;
constexpr int32_t kMsShort = 16;         // longest column a group of lanes takes
constexpr uint32_t kMsFlush = kMsWaveBuf - 64;

__global__ __launch_bounds__(kBlock) void k_ms_push(MsLevel p, uint32_t k) {
    __shared__ int32_t s_buf[kBlock / 64][kMsWaveBuf];
    __shared__ int32_t s_pre[kBlock / 64][64];         // per wave: short columns' entry offsets
    __shared__ int32_t s_col[kBlock / 64][64];         // ... their column ids
    __shared__ int32_t s_e0[kBlock / 64][64];          // ... and first entries
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s0);
    unsigned long long *nxt = pick3(p.m[0], p.m[1], p.m[2], s1);
    unsigned long long *old = pick3(p.m[0], p.m[1], p.m[2], s2);
    const int32_t *fcur = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s0);
    int32_t *fnxt = pick3(p.fq[0], p.fq[1], p.fq[2], s1);
    const int32_t *fold = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s2);
    const uint32_t ncur = p.cnt[s0], nold = p.cnt[s2];
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    for (uint32_t t = gt; t < nold * W; t += gs) {
        const uint32_t u = (uint32_t)fold[t / W];
        old[(size_t)u * W + (t % W)] = 0ull;
    }
    const uint32_t lane = __lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    int32_t *buf = s_buf[wid];
    uint32_t nbuf = 0;                    // the same in every lane
    const uint32_t tag = k + 2;           // "listed for level k+1"
    auto flush = [&]() {
        __builtin_amdgcn_wave_barrier();
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&p.cnt[s1], nbuf);
        base = __shfl(base, 0, 64);
        for (uint32_t i = lane; i < nbuf; i += 64) fnxt[base + i] = buf[i];
        __builtin_amdgcn_wave_barrier();
        nbuf = 0;
    };
    // one entry (u, v): the new bits of u's mask for v, their parents, the OR
    // into nxt[v]; true if this lane lists v for level k+1
    auto entry = [&](int32_t u, int32_t e, int32_t &v) -> bool {
        const unsigned long long *cu = row(cur, u, W);
        v = p.out_idx[e];
        const unsigned long long *vv = row(p.vis, v, W);
        unsigned long long *nv = row(nxt, v, W);
        bool listed = false, any = false;
        for (uint32_t w = 0; w < W; ++w) {
            const unsigned long long nb = cu[w] & ~vv[w];
            if (!nb) continue;
            // parents only decrease, so a stale pre-read can only let
            // an atomic through that was not needed (staged rows and parent
            // values in the caller's ids)
            const int32_t vo = p.stage_labels ? v : (p.out_ent ? p.out_ent[e] : v);
            const uint32_t uo = (uint32_t)caller_id(p, u);
            for (unsigned long long b = nb; b; b &= b - 1ull) {
                uint32_t *at = &p.spar[stage(p, vo, w * 64u + (uint32_t)__ffsll((long long)b) - 1u)];
                if (*at > uo) atomicMin(at, uo);
            }
            if (W == 1) {
                // the lane whose OR turns nxt[v] nonzero lists v; a
                // pre-read (possibly stale: bits are only ever added)
                // skips ORs that would add nothing
                if (nb & ~nv[0]) listed = atomicOr(&nv[0], nb) == 0ull;
            } else {
                atomicOr(&nv[w], nb);
                any = true;
            }
        }
        if (W != 1) listed = any && atomicMax(&p.flag[v], tag) < tag;
        return listed;
    };
    // the wave's listed vertices into its LDS buffer (called by whole waves)
    auto emit = [&](bool listed, int32_t v) {
        const unsigned long long bm = __ballot(listed);
        if (bm) {
            if (listed) buf[nbuf + lanes_below(bm)] = v;
            nbuf += (uint32_t)__popcll(bm);
            if (nbuf > kMsFlush) flush();
        }
    };
    // the frontier list C columns per wave step, a lane per column: the
    // entries of the short columns (at most kMsShort) are dealt out over the
    // wave's lanes, one entry each, through an exclusive prefix sum of their
    // lengths in LDS; then each longer column below kMsLong, the whole wave
    // over its entries
    int32_t *pre = s_pre[wid];
    int32_t *cu_of = s_col[wid];
    int32_t *e0_of = s_e0[wid];
    // columns per wave step: 64 on graphs of low average degree (short
    // columns only: fewer, fuller steps), else a power of two up to 64 such
    // that the list spans about one step per wave (a short list of longer
    // columns then keeps every wave busy)
    const uint32_t nwaves = gs >> 6;
    const uint32_t want = (ncur + nwaves - 1) / nwaves;
    const uint32_t C = (p.wide_steps || want >= 64u) ? 64u
                     : (want <= 1u ? 1u : 1u << (32 - __clz((int)(want - 1u))));
    for (uint32_t b0 = (gt >> 6) * C; b0 < ncur; b0 += nwaves * C) {   // uniform per wave
        const uint32_t it = b0 + lane;
        int32_t u = -1, e0 = 0, d = 0;
        if (lane < C && it < ncur) {
            u = fcur[it];
            e0 = p.out_ptr[u];
            d = p.out_ptr[u + 1] - e0;
        }
        const int32_t ds = (d <= kMsShort) ? d : 0;
        int32_t inc = ds;
#pragma unroll
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        const int32_t total = __shfl(inc, 63, 64);
        pre[lane] = inc - ds;
        cu_of[lane] = u;
        e0_of[lane] = e0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int32_t j0 = 0; j0 < total; j0 += 64) {                 // uniform
            const int32_t j = j0 + (int32_t)lane;
            int32_t v = -1;
            bool listed = false;
            if (j < total) {
                // the column holding entry j: the last one whose prefix is <= j
                uint32_t c = 0;
#pragma unroll
                for (uint32_t step = 32; step; step >>= 1)
                    if (c + step < 64u && pre[c + step] <= j) c += step;
                listed = entry(cu_of[c], e0_of[c] + (j - pre[c]), v);
            }
            emit(listed, v);
        }
        for (unsigned long long mm = __ballot(d > kMsShort && (uint32_t)d < kMsLong); mm; mm &= mm - 1ull) {
            const int src = (int)__ffsll((long long)mm) - 1;
            const int32_t mu = __shfl(u, src, 64), me0 = __shfl(e0, src, 64), md = __shfl(d, src, 64);
            for (int32_t eb = 0; eb < md; eb += 64) {               // uniform
                int32_t v = -1;
                const bool listed = (eb + (int32_t)lane < md) ? entry(mu, me0 + eb + (int32_t)lane, v) : false;
                emit(listed, v);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();                           // LDS reused by the next step
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the chunks of the graph's long columns, a wave each
    for (uint32_t c = gt >> 6; c < p.nlo_chunks; c += gs >> 6) {
        const MsLong L = p.lo[p.lomap[c]];
        const int32_t u = L.v;
        bool in_f = false;
        for (uint32_t w = 0; w < W; ++w) in_f = in_f || row(cur, u, W)[w] != 0ull;
        if (!in_f) continue;
        const int32_t r1 = p.out_ptr[u + 1];
        const int32_t e0 = p.out_ptr[u] + (int32_t)((c - L.chunk_base) * kMsChunk);
        const int32_t e1 = (e0 + (int32_t)kMsChunk < r1) ? e0 + (int32_t)kMsChunk : r1;
        for (int32_t eb = e0; eb < e1; eb += 64) {       // uniform: whole waves step together
            const int32_t e = eb + (int32_t)lane;
            int32_t v = -1;
            const bool listed = (e < e1) ? entry(u, e, v) : false;
            emit(listed, v);
        }
    }
    if (nbuf) flush();
}

// The calling block's share of list slot t's statistics (out-degree sum d,
// new pairs c) into the block's group lines of mstat, slot t and the running
// totals (one atomic per word per block).  Every thread calls it.
__device__ __forceinline__ void add_stats(const MsLevel &p, uint32_t t, unsigned long long d,
                                          unsigned long long c) {
    __shared__ unsigned long long s_d[kBlock / 64][2];
    d = wave_sum64(d);
    c = wave_sum64(c);
    if (__lane_id() == 0) {
        s_d[threadIdx.x >> 6][0] = d;
        s_d[threadIdx.x >> 6][1] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sd = 0, sc = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            sd += s_d[w][0];
            sc += s_d[w][1];
        }
        const int g = (int)(blockIdx.x % kMsDegGroups);
        if (sd) atomicAdd(&p.mstat[ms_line((int)t, g)], sd);
        if (sc) {
            atomicAdd(&p.mstat[ms_line((int)t, g) + 1], sc);
            atomicAdd(&p.mstat[ms_line(kMsCumSlot, g) + 1], sc);
        }
    }
}

// List slot t's statistics to zero and the list's size into the running
// total (called by one thread, before the list's statistics are added).
__device__ __forceinline__ void start_stats(const MsLevel &p, uint32_t t_clear, uint32_t listed) {
    for (int g = 0; g < kMsDegGroups; ++g) {
        p.mstat[ms_line((int)t_clear, g)] = 0ull;
        p.mstat[ms_line((int)t_clear, g) + 1] = 0ull;
    }
    atomicAdd(&p.mstat[ms_line(kMsCumSlot, 0)], (unsigned long long)listed);
}

// Level k, settle half, one lane per newly listed vertex v: the new bits
// (nxt[v]) join vis and get level k+1 (their parents were set by the push).
// The progress report is written only for a level that had a frontier, so
// levels launched past the end of the search (an empty frontier: push and
// settle then change nothing) leave the last level's report in place.
__global__ __launch_bounds__(kBlock) void k_ms_settle(MsLevel p, uint32_t k) {
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *nxt = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s1);
    const int32_t *fnxt = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s1);
    const uint32_t nnext = p.cnt[s1];
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    if (gt == 0) {
        p.cnt[s2] = 0u;                       // the list of level k+2 starts empty
        start_stats(p, s2, nnext);
        if (p.cnt[s0] != 0u) {
            p.host_status[0] = k + 1;
            p.host_status[1] = nnext;
            __threadfence_system();
        }
    }
    unsigned long long deg = 0, pairs = 0;
    for (uint32_t i = gt; i < nnext; i += gs) {
        const int32_t v = fnxt[i];
        deg += (unsigned long long)(p.out_ptr[v + 1] - p.out_ptr[v]);
        for (uint32_t w = 0; w < W; ++w) {
            const unsigned long long nb = row(nxt, v, W)[w];
            if (!nb) continue;
            pairs += (unsigned long long)__popcll(nb);
            row(p.vis, v, W)[w] |= nb;
            const int32_t vo = srow(p, v);
            for (unsigned long long b = nb; b; b &= b - 1ull)
                p.slev[stage(p, vo, w * 64u + (uint32_t)__ffsll((long long)b) - 1u)] = (int32_t)(k + 1);
        }
    }
    add_stats(p, s1, deg, pairs);
}

// The union-frontier bitmap of level k: bit v of fbits = some word of v's
// level-k mask is nonzero.  A wave per 64 consecutive vertices (one lane
// each), whose ballot is the word; every word is rewritten, so nothing needs
// clearing.
__global__ __launch_bounds__(kBlock) void k_ms_fbits(MsLevel p, uint32_t k) {
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], k % 3);
    const uint32_t W = p.W, lane = __lane_id();
    const uint32_t nw = (uint32_t)(((size_t)p.n + 63) / 64);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6, nwaves = (gridDim.x * kBlock) >> 6;
    for (uint32_t i = wave; i < nw; i += nwaves) {           // uniform per wave
        const uint32_t v = i * 64u + lane;
        bool nz = false;
        if (v < (uint32_t)p.n)
            for (uint32_t w = 0; w < W; ++w) nz = nz || row(cur, (int32_t)v, W)[w] != 0ull;
        const unsigned long long bm = __ballot(nz);
        if (lane == 0) p.fbits[i] = bm;
    }
}

// Entries [e0, e1) of row v scanned by the whole wave for the sources in rem
// until every one is found; returns the bits found.  The first batch is one
// step of 64 entries (on a dense frontier most rows end there), every later
// one four steps: their index loads, then their bitmap tests, then their mask
// gathers, each four deep in flight.  With prune (a long row's
// chunk after its first), each batch first drops the sources that an earlier
// chunk of the row has settled at an in-neighbour below the batch's first
// entry: staged parents only decrease within the level, so a stale read only
// keeps a source longer.
__device__ __forceinline__ unsigned long long scan_wave4(const MsLevel &p, const unsigned long long *cur,
                                                         int32_t vo, uint32_t w, int32_t e0, int32_t e1,
                                                         unsigned long long rem, uint32_t lk,
                                                         bool owner_alone, bool prune) {
    const uint32_t W = p.W;
    const int32_t lane = (int32_t)__lane_id();
    unsigned long long found = 0ull;
    int32_t nst = 1;                                                    // steps in this batch
    for (int32_t eb = e0; eb < e1 && rem; eb += nst * 64, nst = 4) {
        int32_t uu[4], oo[4];                                           // labels, caller ids
        bool ok[4];
        unsigned long long mm[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int32_t e = eb + t * 64 + lane;
            const bool in = t < nst && e < e1;
            uu[t] = in ? p.in_idx[e] : -1;
        }
        if (prune) {
            const uint32_t first = (uint32_t)(p.ent ? p.ent[eb] : __shfl(uu[0], 0, 64));
            const uint32_t sp = p.spar[stage(p, vo, w * 64u + (uint32_t)lane)];
            rem &= ~__ballot(sp < first);
            if (!rem) break;                                            // uniform
        }
        if (p.use_fbits) {
            unsigned long long fb[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) fb[t] = uu[t] >= 0 ? p.fbits[(uint32_t)uu[t] >> 6] : 0ull;
#pragma unroll
            for (int t = 0; t < 4; ++t) ok[t] = ((fb[t] >> ((uint32_t)uu[t] & 63u)) & 1ull) != 0ull;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) ok[t] = uu[t] >= 0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) mm[t] = ok[t] ? row(cur, uu[t], W)[w] : 0ull;
        // the caller's ids of the entries that may give a parent (with the
        // degree-ordered copy a lookup, mostly in the few megabytes of the
        // labels of largest degree; streaming every entry's id cost more)
#pragma unroll
        for (int t = 0; t < 4; ++t) oo[t] = (mm[t] & rem) ? caller_id(p, uu[t]) : -1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (rem) {                                                  // uniform
                const unsigned long long f = scan_resolve<64>(p, vo, w, oo[t], mm[t] & rem, lk, owner_alone);
                rem &= ~f;
                found |= f;
            }
        }
    }
    return found;
}

// Level k, pull form (for large frontiers): every vertex v whose sources are
// not all settled ORs, in ascending in-neighbour order, the frontier masks of
// its in-neighbours restricted to the sources that have not reached it; each
// source bit found first at u gets parent u (the smallest frontier
// in-neighbour for that source) and level k+1.  Rows of up to kMsSerial
// entries are scanned by one lane, longer ones by a wave (scan_step); the
// owner of such a row writes vis and the next mask without atomics, and rows
// with new bits are listed (one atomicAdd per block chunk).  The graph's long
// rows (kMsLong entries or more) are scanned in chunks by waves across the
// grid: each chunk gives its first hits (atomicMin on the staged parent) and
// ORs its bits into the next mask; k_ms_fixup then folds those into vis and
// lists the rows.  Also clears F_{k-1}'s masks.
// Chunk j (kMsChunk entries) of long row v, scanned by one wave in ascending
// order until every unsettled source is found: first hits go to the staged
// parents by atomicMin, the bits found are ORed into the next mask and, for
// the row's first chunk (first = true), into vis as well.
__device__ __forceinline__ void long_chunk(const MsLevel &p, const unsigned long long *cur,
                                           unsigned long long *nxt, int32_t v, uint32_t j,
                                           uint32_t k, bool first) {
    const uint32_t W = p.W, tail = p.nq & 63u;
    const int32_t r1 = p.in_ptr[v + 1];
    const int32_t e0 = p.in_ptr[v] + (int32_t)(j * kMsChunk);
    const int32_t e1 = (e0 + (int32_t)kMsChunk < r1) ? e0 + (int32_t)kMsChunk : r1;
    unsigned long long *vis = row(p.vis, v, W);
    for (uint32_t w = 0; w < W; ++w) {
        const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
        const unsigned long long found = scan_wave4(p, cur, srow(p, v), w, e0, e1, full & ~vis[w], k + 1,
                                                    false, j != 0);
        if (found && __lane_id() == 0) {
            atomicOr(&row(nxt, v, W)[w], found);
            if (first) vis[w] |= found;
        }
    }
}

constexpr int32_t kMsSerial = 16;        // longest row one lane scans alone
constexpr uint32_t kMsGroupRow = 64;     // longest row a group of 16 lanes scans

__global__ __launch_bounds__(kBlock) void k_ms_pull(MsLevel p, uint32_t k) {
    __shared__ int32_t s_list[kMsRows];
    __shared__ int32_t s_long[kMsRows];
    __shared__ uint32_t s_off[kBlock][9];          // a row's found bits: entry offset, 4 bits each
    __shared__ unsigned long long s_fnd[kBlock];   // a row's found bits (one word)
    __shared__ int32_t s_e0[kBlock];
    __shared__ uint32_t s_n, s_nl, s_base;
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s0);
    unsigned long long *nxt = pick3(p.m[0], p.m[1], p.m[2], s1);
    unsigned long long *old = pick3(p.m[0], p.m[1], p.m[2], s2);
    int32_t *fnxt = pick3(p.fq[0], p.fq[1], p.fq[2], s1);
    const int32_t *fold = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s2);
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
    // row chunks of kMsRows rows, or the graph's own chunk bounds (at most
    // kMsRows rows and about the same number of list entries each: the
    // degree-ordered copy puts its heaviest rows side by side)
    const uint32_t nrc = p.row_chunks ? p.nrow_chunks : (uint32_t)(((size_t)p.n + kMsRows - 1) / kMsRows);
    for (uint32_t c = blockIdx.x; c < nrc; c += gridDim.x) {
        if (tid == 0) {
            s_n = 0;
            s_nl = 0;
        }
        __syncthreads();
        const uint32_t c0 = p.row_chunks ? (uint32_t)p.row_chunks[c] : c * kMsRows;
        const uint32_t c1 = p.row_chunks ? (uint32_t)p.row_chunks[c + 1]
                                         : ((c0 + kMsRows < (uint32_t)p.n) ? c0 + kMsRows : (uint32_t)p.n);
        // Rows of up to kMsSerial entries, one lane each, 256 at a time.  A
        // lane records, per found bit, the offset of the entry that gave it
        // (LDS); then each wave writes its lanes' rows, one row at a time
        // with the 64 sources of the word on the 64 lanes, so the staged
        // results of a row go out as one 256-byte store.
        for (uint32_t r0 = c0; r0 < c1; r0 += kBlock) {
            const uint32_t vv = r0 + tid;
            const int32_t v = (int32_t)vv;
            int32_t e0 = 0, e1 = 0;
            bool mine = false;
            if (vv < c1) {
                e0 = p.in_ptr[v];
                e1 = p.in_ptr[v + 1];
                if (e1 > e0 && (uint32_t)(e1 - e0) < kMsLong) {        // long rows: chunks below
                    const unsigned long long *vis = row(p.vis, v, W);
                    bool open = false;
                    for (uint32_t w = 0; w < W && !open; ++w) {
                        const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                        open = (full & ~vis[w]) != 0ull;
                    }
                    if (open) {                      // else every source has reached v
                        if (e1 - e0 > kMsSerial) s_long[atomicAdd(&s_nl, 1u)] = v;
                        else mine = true;
                    }
                }
            }
            s_e0[tid] = e0;
            bool any = false;
            for (uint32_t w = 0; w < W; ++w) {
                unsigned long long found = 0ull;
#pragma unroll
                for (int i = 0; i < 8; ++i) s_off[tid][i] = 0u;
                if (mine) {
                    unsigned long long *vis = row(p.vis, v, W);
                    const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                    const unsigned long long sv = vis[w];
                    unsigned long long rem = full & ~sv;
                    // four entries at a time: their index and mask loads are
                    // all issued before the first is used; positions past e1
                    // repeat the last entry, whose bits are then already taken
                    for (int32_t e = e0; e < e1 && rem; e += 4) {
                        int32_t uu[4];
                        unsigned long long mm[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) uu[j] = p.in_idx[e + j < e1 ? e + j : e1 - 1];
#pragma unroll
                        for (int j = 0; j < 4; ++j) mm[j] = in_frontier(p, uu[j]) ? row(cur, uu[j], W)[w] : 0ull;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            unsigned long long hit = mm[j] & rem;
                            rem &= ~hit;
                            found |= hit;
                            const uint32_t off = (uint32_t)(e - e0 + j);
                            while (hit) {
                                const uint32_t b = (uint32_t)__ffsll((long long)hit) - 1u;
                                hit &= hit - 1ull;
                                s_off[tid][b >> 3] |= off << ((b & 7u) * 4u);
                            }
                        }
                    }
                    if (found) {
                        row(nxt, v, W)[w] = found;
                        vis[w] = sv | found;
                        any = true;
                    }
                }
                s_fnd[tid] = found;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // this wave's lanes' rows that found something, one at a time
                for (unsigned long long rows = __ballot(found != 0ull); rows; rows &= rows - 1ull) {
                    const uint32_t rr = (tid & ~63u) + (uint32_t)__ffsll((long long)rows) - 1u;
                    const unsigned long long fm = s_fnd[rr];
                    if ((fm >> lane) & 1ull) {
                        const uint32_t j = (s_off[rr][lane >> 3] >> ((lane & 7u) * 4u)) & 15u;
                        const size_t at = stage(p, srow(p, (int32_t)(r0 + rr)), w * 64u + lane);
                        const int32_t e = s_e0[rr] + (int32_t)j;
                        p.slev[at] = (int32_t)lk;
                        p.spar[at] = (uint32_t)(p.ent ? p.ent[e] : p.in_idx[e]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (any) s_list[atomicAdd(&s_n, 1u)] = v;
        }
        __syncthreads();
        // rows longer than kMsSerial: four at a time per wave, a group of 16
        // lanes each for rows of up to kMsGroupRow entries, then the longer
        // ones of the four by the whole wave
        const uint32_t nl = s_nl;
        for (uint32_t i0 = wave * 4u; i0 < nl; i0 += (kBlock / 64) * 4u) {
            const uint32_t gi = i0 + (lane >> 4), gl = lane & 15u;
            int32_t v = -1, e0 = 0, e1 = 0;
            bool wide = false;
            if (gi < nl) {                                   // uniform in the group
                v = s_long[gi];
                e0 = p.in_ptr[v];
                e1 = p.in_ptr[v + 1];
                wide = (uint32_t)(e1 - e0) > kMsGroupRow;
                if (!wide) {
                    unsigned long long *vis = row(p.vis, v, W);
                    bool any = false;
                    for (uint32_t w = 0; w < W; ++w) {
                        const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                        const unsigned long long sv = vis[w];
                        unsigned long long rem = full & ~sv, found = 0ull;
                        for (int32_t eb = e0; eb < e1 && rem; eb += 16) {
                            const unsigned long long f = scan_step<16>(p, cur, srow(p, v), w, eb, e1, rem,
                                                                       lk, true);
                            rem &= ~f;
                            found |= f;
                        }
                        if (found) {
                            if (gl == 0) {
                                row(nxt, v, W)[w] = found;
                                vis[w] = sv | found;
                            }
                            any = true;
                        }
                    }
                    if (any && gl == 0) s_list[atomicAdd(&s_n, 1u)] = v;
                }
            }
            for (unsigned long long wm = __ballot(wide && gl == 0); wm; wm &= wm - 1ull) {   // uniform
                const int src = (int)__ffsll((long long)wm) - 1;
                const int32_t wv = __shfl(v, src, 64), we0 = __shfl(e0, src, 64), we1 = __shfl(e1, src, 64);
                unsigned long long *vis = row(p.vis, wv, W);
                bool any = false;
                for (uint32_t w = 0; w < W; ++w) {
                    const unsigned long long full = (w == W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
                    const unsigned long long sv = vis[w];
                    const unsigned long long found = scan_wave4(p, cur, srow(p, wv), w, we0, we1, full & ~sv,
                                                                lk, true, false);
                    if (found) {
                        if (lane == 0) {
                            row(nxt, wv, W)[w] = found;
                            vis[w] = sv | found;
                        }
                        any = true;
                    }
                }
                if (any && lane == 0) s_list[atomicAdd(&s_n, 1u)] = wv;
            }
        }
        __syncthreads();
        if (tid == 0 && s_n) s_base = atomicAdd(&p.cnt[s1], s_n);
        __syncthreads();
        for (uint32_t i = tid; i < s_n; i += kBlock) fnxt[s_base + i] = s_list[i];
        __syncthreads();
    }
    // The long rows, one wave per chunk.  With long_split, only each row's
    // first chunk here: it holds the row's smallest in-neighbours, so what
    // it finds is final - those bits go into vis now (no other wave touches
    // this row's vis in this kernel) and k_ms_pull_rest then scans the later
    // chunks for the other sources only.  Without it, every chunk here, all
    // looking for the same unsettled sources (vis is not written).
    const uint32_t nitems = p.long_split ? p.nli : p.nli_chunks;
    for (uint32_t c = gt >> 6; c < nitems; c += gs >> 6) {           // uniform per wave
        int32_t v;
        uint32_t j = 0;
        if (p.long_split) {
            v = p.li[c].v;
        } else {
            const MsLong L = p.li[p.limap[c]];
            v = L.v;
            j = c - L.chunk_base;
        }
        long_chunk(p, cur, nxt, v, j, k, p.long_split != 0u);
    }
}

// Level k, pull form, the later chunks of the long rows (after k_ms_pull):
// each looks only for the sources the row's first chunk left unsettled (vis
// holds those found there), gives its first hits to the staged parents by
// atomicMin (the smallest over the chunks) and ORs its bits into the next
// mask; k_ms_fixup then folds those into vis and lists the rows.  The chunks
// are taken every row's second chunk first, then the third, ..., so that
// most chunks find their row's earlier chunks done and skip the sources
// those settled.
__global__ __launch_bounds__(kBlock) void k_ms_pull_rest(MsLevel p, uint32_t k) {
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], k % 3);
    unsigned long long *nxt = pick3(p.m[0], p.m[1], p.m[2], (k + 1) % 3);
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    const uint32_t nrest = p.nli_chunks - p.nli;
    for (uint32_t i = gt >> 6; i < nrest; i += gs >> 6) {                // uniform per wave
        const uint32_t c = p.lirest[i];
        const MsLong L = p.li[p.limap[c]];
        long_chunk(p, cur, nxt, L.v, c - L.chunk_base, k, false);
    }
}

// After a pull level, the long rows: bits their chunks found join vis, and
// rows with any are listed.
__global__ __launch_bounds__(kBlock) void k_ms_fixup(MsLevel p, uint32_t k) {
    const uint32_t s1 = (k + 1) % 3;
    const unsigned long long *nxt = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s1);
    int32_t *fnxt = pick3(p.fq[0], p.fq[1], p.fq[2], s1);
    const uint32_t W = p.W;
    const uint32_t lane = __lane_id();
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    for (uint32_t base_i = gt - lane; base_i < p.nli; base_i += gs) {     // whole waves iterate
        const uint32_t i = base_i + lane;
        bool any = false;
        int32_t v = -1;
        if (i < p.nli) {
            v = p.li[i].v;
            for (uint32_t w = 0; w < W; ++w) {
                const unsigned long long f = row(nxt, v, W)[w];
                if (f) {
                    row(p.vis, v, W)[w] |= f;
                    any = true;
                }
            }
        }
        const unsigned long long bm = __ballot(any);
        if (bm) {
            const uint32_t leader = (uint32_t)__ffsll((long long)bm) - 1u;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&p.cnt[s1], (uint32_t)__popcll(bm));
            base = __shfl(base, (int)leader, 64);
            if (any) fnxt[base + lanes_below(bm)] = v;
        }
    }
}

// The staged results into the callers' arrays: a block per 64 vertices and 64
// sources, through an LDS tile, so that both the staged rows and the
// per-source output rows move in whole lines; each lane reads 4 sources of a
// staged row and writes 4 vertices of an output row (16 bytes, or 4 scalar
// stores where the caller's array is not 16-byte aligned or at the tail).
// Entries whose vis bit is clear (never reached) become -1.
__global__ __launch_bounds__(kBlock) void k_ms_out(MsLevel p) {
    // one 64 x 64 tile (+1 column against bank conflicts), used for the
    // levels and then for the parents: 16.6 KB per block, so that more blocks
    // share a compute unit and keep more loads in flight
    __shared__ int32_t t_x[64][65];
    const uint32_t W = p.W, S = W * 64u, tid = threadIdx.x;
    const uint32_t ntiles = (uint32_t)(((size_t)p.n + 63) / 64);
    const uint32_t g4 = (tid & 15u) * 4u;          // first of this lane's 4 columns
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int32_t v0 = (int32_t)(tile * 64u);
        for (uint32_t w = 0; w < W; ++w) {
            int4 lv[4], pa[4];
            uint32_t bits[4];
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {            // this lane's 4 sources of 4 staged rows
                const int32_t v = v0 + (int32_t)((tid >> 4) + 16u * r);
                lv[r] = make_int4(-1, -1, -1, -1);
                pa[r] = lv[r];
                bits[r] = 0;
                const int32_t x = v < p.n ? label_of(p, v) : 0;
                if (v < p.n) bits[r] = (uint32_t)(row(p.vis, x, W)[w] >> g4) & 15u;
                if (bits[r]) {                          // read once: streaming loads
                    const size_t at = (size_t)(p.stage_labels ? x : v) * S + w * 64u + g4;
                    const v4i a = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p.slev + at));
                    const v4i b = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p.spar + at));
                    lv[r] = make_int4(a.x, a.y, a.z, a.w);
                    pa[r] = make_int4(b.x, b.y, b.z, b.w);
                }
            }
            int4 out_l[4], out_p[4];
            for (int half = 0; half < 2; ++half) {         // levels, then parents
#pragma unroll
                for (uint32_t r = 0; r < 4; ++r) {        // staged rows -> tile[source][vertex]
                    const uint32_t vi = (tid >> 4) + 16u * r;
                    const int4 x = half ? pa[r] : lv[r];
                    t_x[g4 + 0][vi] = (bits[r] & 1u) ? x.x : -1;
                    t_x[g4 + 1][vi] = (bits[r] & 2u) ? x.y : -1;
                    t_x[g4 + 2][vi] = (bits[r] & 4u) ? x.z : -1;
                    t_x[g4 + 3][vi] = (bits[r] & 8u) ? x.w : -1;
                }
                __syncthreads();
#pragma unroll
                for (uint32_t r = 0; r < 4; ++r) {        // tile rows, 4 vertices per lane
                    const uint32_t qi = (tid >> 4) + 16u * r;
                    const int4 y = make_int4(t_x[qi][g4], t_x[qi][g4 + 1], t_x[qi][g4 + 2], t_x[qi][g4 + 3]);
                    if (half) out_p[r] = y;
                    else out_l[r] = y;
                }
                __syncthreads();
            }
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {            // output rows
                const uint32_t qi = (tid >> 4) + 16u * r;
                const uint32_t q = w * 64u + qi;
                if (q >= p.nq) continue;
                int32_t *lo = p.level[q] + v0 + g4;
                int32_t *po = p.parent[q] + v0 + g4;
                const int4 a = out_l[r], b = out_p[r];
                const bool full = v0 + (int32_t)g4 + 3 < p.n;
                if (full && ((reinterpret_cast<uintptr_t>(lo) | reinterpret_cast<uintptr_t>(po)) & 15u) == 0) {
                    // written once and not read here again: streaming stores
                    const v4i av = {a.x, a.y, a.z, a.w}, bv = {b.x, b.y, b.z, b.w};
                    __builtin_nontemporal_store(av, reinterpret_cast<v4i *>(lo));
                    __builtin_nontemporal_store(bv, reinterpret_cast<v4i *>(po));
                } else {
                    const int32_t av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (v0 + (int32_t)g4 + j < p.n) {
                            lo[j] = av[j];
                            po[j] = bv[j];
                        }
                }
            }
        }
    }
}

// Level k, pull form, pass r of the range order (dense levels, one mask
// word).  The in-neighbours are visited one vertex range at a time, in
// ascending order of ranges: pass r looks only at the in-list entries whose
// in-neighbour lies in [r n / R, (r + 1) n / R), so the frontier masks it
// gathers (2 MB) stay in the XCDs' L2.  A row's lists are sorted, so each
// pass continues where the row's previous pass stopped (rcur); a source found
// in an earlier range has its smallest frontier in-neighbour there, so what a
// pass finds is final - written at once, with no atomics between passes.
// Pass 0 looks at every row; a row still open after a pass (sources unfound,
// entries left) goes on the list of the next pass.  Rows of at most kRpShort
// entries are scanned by one lane (16 entries per step, then the wave writes
// the staged results of its lanes' rows one row at a time); longer rows by a
// whole wave, 64 entries per step.  Also clears F_{k-1}'s masks (pass 0).
constexpr int32_t kRpShort = 64;

// One wave, one row: its entries from e with in-neighbour below rend, 64 a
// step, until rem is empty.  Stages the first hits; returns the bits found and
// leaves e at the first entry not scanned.
__device__ __forceinline__ unsigned long long rp_wave_row(const MsLevel &p, const unsigned long long *cur,
                                                          int32_t v, int32_t &e, int32_t e1, uint32_t rend,
                                                          unsigned long long rem, uint32_t lk) {
    const uint32_t lane = __lane_id();
    unsigned long long found = 0ull;
    while (e < e1 && rem) {                                    // uniform
        const int32_t ei = e + (int32_t)lane;
        int32_t u = 0;
        bool in = false;
        if (ei < e1) {
            u = p.in_idx[ei];
            in = (uint32_t)u < rend;
        }
        unsigned long long hit = 0ull;
        if (in) hit = cur[u] & rem;
        // the step's entries in the range are a prefix of its lanes (sorted list)
        const uint32_t cnt = (uint32_t)__popcll(__ballot(in));
        if (__ballot(hit != 0ull)) {
            unsigned long long incl = hit;
#pragma unroll
            for (uint32_t d = 1; d < 64; d <<= 1) {
                const unsigned long long t = __shfl_up(incl, d, 64);
                if (lane >= d) incl |= t;
            }
            unsigned long long below = __shfl_up(incl, 1u, 64);
            if (lane == 0) below = 0ull;
            unsigned long long own = hit & ~below;
            while (own) {
                const uint32_t b = (uint32_t)__ffsll((long long)own) - 1u;
                own &= own - 1ull;
                const size_t at = stage(p, v, b);
                p.slev[at] = (int32_t)lk;
                p.spar[at] = (uint32_t)u;
            }
            const unsigned long long f = __shfl(incl, 63, 64);
            rem &= ~f;
            found |= f;
        }
        e += (int32_t)cnt;
        if (cnt < 64u) break;                                 // the range or the row ended here
    }
    return found;
}

__global__ __launch_bounds__(kBlock) void k_ms_rpull(MsLevel p, uint32_t k, uint32_t r) {
    __shared__ int32_t s_list[kMsRows];                 // rows the level lists
    __shared__ int32_t s_wide[kMsRows];                 // rows for a whole wave
    __shared__ int32_t s_open[kMsRows];                 // rows open after this pass
    __shared__ int32_t s_ocur[kMsRows];                 //   and their next entries
    __shared__ uint32_t s_off[kBlock][9];               // a row's found bits: entry offset, 4 bits each
    __shared__ unsigned long long s_fnd[kBlock];
    __shared__ int32_t s_e0[kBlock];
    __shared__ uint32_t s_n, s_nw, s_no, s_base, s_obase;
    const uint32_t s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const unsigned long long *cur = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s0);
    unsigned long long *nxt = pick3(p.m[0], p.m[1], p.m[2], s1);
    int32_t *fnxt = pick3(p.fq[0], p.fq[1], p.fq[2], s1);
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const uint32_t gt = blockIdx.x * kBlock + tid, gs = gridDim.x * kBlock;
    const uint32_t R = p.rp_ranges;
    const uint32_t rend = (r + 1 == R) ? (uint32_t)p.n : (uint32_t)(((uint64_t)(r + 1) * (uint64_t)p.n) / R);
    const unsigned long long full = (p.nq & 63u) ? ((1ull << (p.nq & 63u)) - 1ull) : ~0ull;
    const uint32_t lk = k + 1;
    if (r == 0) {
        unsigned long long *old = pick3(p.m[0], p.m[1], p.m[2], s2);
        const int32_t *fold = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s2);
        const uint32_t nold = p.cnt[s2];
        for (uint32_t t = gt; t < nold; t += gs) old[fold[t]] = 0ull;
    }
    if (gt == 0) p.rcnt[(r + 1) % 3] = 0u;                     // the next pass's open rows
    const bool all = (r == 0);
    const uint32_t nin = all ? (uint32_t)p.n : p.rcnt[(r + 2) % 3];   // pass r-1's open rows
    const int32_t *lin = p.rlist[(r + 1) & 1];
    int32_t *lout = p.rlist[r & 1];
    for (uint32_t c0 = blockIdx.x * kMsRows; c0 < nin; c0 += gridDim.x * kMsRows) {
        if (tid == 0) {
            s_n = 0;
            s_nw = 0;
            s_no = 0;
        }
        __syncthreads();
        const uint32_t c1 = (c0 + kMsRows < nin) ? c0 + kMsRows : nin;
        for (uint32_t r0 = c0; r0 < c1; r0 += kBlock) {
            const uint32_t i = r0 + tid;
            int32_t v = -1, e = 0, e1 = 0;
            unsigned long long sv = 0ull, rem = 0ull;
            bool act = false;
            if (i < c1) {
                v = all ? (int32_t)i : lin[i];
                const int32_t b0 = p.in_ptr[v];
                e1 = p.in_ptr[v + 1];
                e = all ? b0 : p.rcur[v];
                if (e < e1) {
                    sv = p.vis[v];
                    rem = full & ~sv;
                    if (rem) {
                        if (e1 - b0 > kRpShort) s_wide[atomicAdd(&s_nw, 1u)] = v;
                        else act = true;
                    }
                }
            }
            unsigned long long got = 0ull;
            const bool mine = act;
            // steps of up to 16 entries; after each, the wave writes its
            // lanes' staged results one row at a time
            while (__ballot(act)) {                               // uniform
                unsigned long long found = 0ull;
#pragma unroll
                for (int j = 0; j < 9; ++j) s_off[tid][j] = 0u;
                s_e0[tid] = e;
                if (act) {
                    const int32_t es = e;
                    bool more = true;
                    for (int bt = 0; bt < 4 && more && rem; ++bt) {
                        int32_t uu[4];
                        unsigned long long mm[4];
                        bool in[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) uu[j] = p.in_idx[e + j < e1 ? e + j : e1 - 1];
#pragma unroll
                        for (int j = 0; j < 4; ++j) in[j] = (e + j < e1) && (uint32_t)uu[j] < rend;
#pragma unroll
                        for (int j = 0; j < 4; ++j) mm[j] = in[j] ? cur[uu[j]] : 0ull;
                        int nin4 = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            nin4 += in[j] ? 1 : 0;
                            unsigned long long hit = mm[j] & rem;
                            rem &= ~hit;
                            found |= hit;
                            const uint32_t off = (uint32_t)(e - es + j);
                            while (hit) {
                                const uint32_t b = (uint32_t)__ffsll((long long)hit) - 1u;
                                hit &= hit - 1ull;
                                s_off[tid][b >> 3] |= off << ((b & 7u) * 4u);
                            }
                        }
                        e += nin4;
                        more = (nin4 == 4);
                    }
                    // open while sources are unfound and this range may hold more
                    act = more && rem && e < e1;
                }
                got |= found;
                s_fnd[tid] = found;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (unsigned long long rows = __ballot(found != 0ull); rows; rows &= rows - 1ull) {
                    const uint32_t rr = (tid & ~63u) + (uint32_t)__ffsll((long long)rows) - 1u;
                    const unsigned long long fm = s_fnd[rr];
                    if ((fm >> lane) & 1ull) {
                        const uint32_t j = (s_off[rr][lane >> 3] >> ((lane & 7u) * 4u)) & 15u;
                        const int32_t rv = all ? (int32_t)(r0 + rr) : lin[r0 + rr];
                        const size_t at = stage(p, rv, lane);
                        p.slev[at] = (int32_t)lk;
                        p.spar[at] = (uint32_t)p.in_idx[s_e0[rr] + (int32_t)j];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (mine) {
                if (got) {
                    const unsigned long long before = nxt[v];
                    nxt[v] = before | got;
                    p.vis[v] = sv | got;
                    if (!before) s_list[atomicAdd(&s_n, 1u)] = v;
                }
                if (rem && e < e1) {                               // the next range continues here
                    const uint32_t o = atomicAdd(&s_no, 1u);
                    s_open[o] = v;
                    s_ocur[o] = e;
                }
            }
        }
        __syncthreads();
        // the longer rows: a wave each
        for (uint32_t wi = wave; wi < s_nw; wi += kBlock / 64) {
            const int32_t v = s_wide[wi];
            const int32_t b0 = p.in_ptr[v], e1 = p.in_ptr[v + 1];
            int32_t e = all ? b0 : p.rcur[v];
            const unsigned long long sv = p.vis[v];
            const unsigned long long rem = full & ~sv;
            const unsigned long long got = rp_wave_row(p, cur, v, e, e1, rend, rem, lk);
            if (lane == 0) {
                if (got) {
                    const unsigned long long before = nxt[v];
                    nxt[v] = before | got;
                    p.vis[v] = sv | got;
                    if (!before) s_list[atomicAdd(&s_n, 1u)] = v;
                }
                if ((rem & ~got) && e < e1) {
                    const uint32_t o = atomicAdd(&s_no, 1u);
                    s_open[o] = v;
                    s_ocur[o] = e;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            if (s_n) s_base = atomicAdd(&p.cnt[s1], s_n);
            if (s_no) s_obase = atomicAdd(&p.rcnt[r % 3], s_no);
        }
        __syncthreads();
        for (uint32_t i = tid; i < s_n; i += kBlock) fnxt[s_base + i] = s_list[i];
        for (uint32_t i = tid; i < s_no; i += kBlock) {
            lout[s_obase + i] = s_open[i];
            p.rcur[s_open[i]] = s_ocur[i];
        }
        __syncthreads();
    }
}

// After a pull level: the lists of level k+2 start empty; report to the host;
// the statistics of the level-(k+1) list.
__global__ __launch_bounds__(kBlock) void k_ms_report(MsLevel p, uint32_t k) {
    const uint32_t s1 = (k + 1) % 3, s2 = (k + 2) % 3;
    const uint32_t nnext = p.cnt[s1];
    const int32_t *fnxt = pick3<const int32_t *>(p.fq[0], p.fq[1], p.fq[2], s1);
    const unsigned long long *nxt = pick3<const unsigned long long *>(p.m[0], p.m[1], p.m[2], s1);
    const uint32_t W = p.W;
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
    if (gt == 0) {
        p.cnt[s2] = 0u;
        for (int t = 0; t < 3; ++t) p.rcnt[t] = 0u;           // the range passes' open rows
        start_stats(p, s2, nnext);
        p.host_status[0] = k + 1;
        p.host_status[1] = nnext;
        __threadfence_system();
    }
    unsigned long long deg = 0, pairs = 0;
    for (uint32_t i = gt; i < nnext; i += gs) {
        const int32_t v = fnxt[i];
        deg += (unsigned long long)(p.out_ptr[v + 1] - p.out_ptr[v]);
        for (uint32_t w = 0; w < W; ++w) pairs += (unsigned long long)__popcll(row(nxt, v, W)[w]);
    }
    add_stats(p, s1, deg, pairs);
}

// The direction of level k (one wave): the network's argmin between push (0)
// and pull (1) over the level's twelve features, push when an output is not
// finite (or without a network); written to host_status[2].  Features, from
// f = |F_k| (the union frontier), d = its out-degree sum, c = the summed union
// frontier sizes of levels 0..k, u = the (vertex, source) pairs not reached
// through level k, q sources, k, n and nnz.
__device__ __forceinline__ float ms_feature(uint32_t i, float f, float d, float c, float u, float q,
                                            float k, float n, float nnz) {
    switch (i) {
        case 0: return logf(1.f + f);
        case 1: return logf(1.f + d);
        case 2: return logf(1.f + c);
        case 3: return logf(1.f + q);
        case 4: return logf(1.f + k);
        case 5: return nnz / n;
        case 6: return logf((f + 1.f) / n);
        case 7: return logf((d + 1.f) / (nnz + 1.f));
        case 8: return logf((u + 1.f) / (n * q));
        case 9: return logf((d + 1.f) / (f + 1.f));
        case 10: return logf((f + 1.f) * q / n);
        case 11: return logf((d + 1.f) / (nnz - d + 1.f));
        default: return 0.f;
    }
}

__global__ void k_ms_decide(MsLevel p, uint32_t k) {
    const uint32_t t = k % 3;
    const uint32_t f = p.cnt[t];
    unsigned long long d = 0, c = 0, r = 0;
    for (int g = 0; g < kMsDegGroups; ++g) {
        d += p.mstat[ms_line((int)t, g)];
        c += p.mstat[ms_line(kMsCumSlot, g)];
        r += p.mstat[ms_line(kMsCumSlot, g) + 1];
    }
    const unsigned long long pairs = (unsigned long long)p.n * p.nq;
    const unsigned long long u = pairs > r ? pairs - r : 0ull;
    uint32_t v = 0;
    if (p.mlp != nullptr) {
        const float feat = ms_feature(__lane_id(), (float)f, (float)d, (float)c, (float)u, (float)p.nq,
                                      (float)k, (float)p.n, (float)p.out_ptr[p.n]);
        const int b = mlp_argmin(p.mlp, feat, 2);
        v = b < 0 ? 0u : (uint32_t)b;
    }
    if (threadIdx.x == 0) {
        p.host_status[2] = v;
        __threadfence_system();
    }
}

hipError_t launch_ms_rpull(const MsLevel &p, uint32_t k, uint32_t r, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_ms_rpull, dim3(grid), dim3(kBlock), 0, s, p, k, r);
    return hipGetLastError();
}

hipError_t launch_ms(const MsLevel &p, int phase, uint32_t k, uint32_t grid, hipStream_t s) {
    // the list walks after a level (settle, fixup, report) end in one pair of
    // counter atomics per workgroup on the same two words: at most 2,048
    // workgroups for them (R-MAT s22: the report 25-31 us at 8,192, 17-22 us
    // at 1,024-2,048)
    const uint32_t small = grid < 2048u ? grid : 2048u;
    switch (phase) {
        case 0: hipLaunchKernelGGL(k_ms_clear, dim3(grid), dim3(kBlock), 0, s, p); break;
        case 1: hipLaunchKernelGGL(k_ms_roots, dim3(grid), dim3(kBlock), 0, s, p); break;
        case 2: hipLaunchKernelGGL(k_ms_push, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        case 3: hipLaunchKernelGGL(k_ms_settle, dim3(small), dim3(kBlock), 0, s, p, k); break;
        case 4: hipLaunchKernelGGL(k_ms_pull, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        case 6: hipLaunchKernelGGL(k_ms_fixup, dim3(small), dim3(kBlock), 0, s, p, k); break;
        case 7: hipLaunchKernelGGL(k_ms_out, dim3(grid), dim3(kBlock), 0, s, p); break;
        case 8: hipLaunchKernelGGL(k_ms_fbits, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        case 9: hipLaunchKernelGGL(k_ms_pull_rest, dim3(grid), dim3(kBlock), 0, s, p, k); break;
        case 10: hipLaunchKernelGGL(k_ms_decide, dim3(1), dim3(64), 0, s, p, k); break;
        default: hipLaunchKernelGGL(k_ms_report, dim3(small), dim3(kBlock), 0, s, p, k); break;
    }
    return hipGetLastError();
}

}  // namespace bfsi

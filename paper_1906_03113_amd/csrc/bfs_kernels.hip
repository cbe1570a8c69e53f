// gfx950 kernels of the masked sparse-matrix x sparse-vector BFS.
//
// Level k evaluates x_{k+1} = A^T[V_{k+1}, V_k] x_k (Theorem 1): only the
// columns of the current frontier F_k = supp(x_k) are read, and only rows not
// yet visited (V_{k+1}) are accepted.  Three forms of that product exist here:
//
//  * push         - gather the frontier's columns from a compacted list
//                   (Algorithm 3's "for all" over the frontier and its column
//                   entries, mapped to lanes);
//  * push-bitmap  - the same gather, the frontier read from a bitmap;
//  * pull         - the row-wise (inner-product) form of Claim 1, evaluated
//                   over the shrinking list of unvisited rows: scan a row's
//                   in-neighbours in ascending order and stop at the first
//                   frontier vertex.
//
// Every form yields the same (level, parent): parent[i] is the smallest
// frontier vertex j with A(j, i) = 1 (push: atomicMin over every unmasked pair
// of the level - the Lemma 1 form; pull: first hit of an ascending scan).
//
// Mask: the visited bitmap B_k used during level k is read-only during that
// level; B_{k+1} is built in the other buffer of a ping-pong pair, which holds
// B_{k-1} on entry and receives F_k and F_{k+1}.  So the test is stable and
// the result does not depend on scheduling.
//
// Level k's counters live in ring slot k & 3; its kernels read k from the
// device state, so the same launches can be issued from a host loop, replayed
// from a captured graph, or run inside one persistent kernel.
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
#include <stdint.h>

#include "bfs_internal.h"

namespace bfsi {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += t;
    }
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// variant choice (uniform across the grid: every block computes it from the
// same device counters)
// ---------------------------------------------------------------------------

__device__ float mlp_logtime(const float *w, const float f[kMlpIn], int out_unit) {
    // 12 -> 32 (ReLU) -> 32 (ReLU) -> 3, row-major weights [out][in]
    const float *W1 = w, *b1 = W1 + kMlpIn * kMlpH, *W2 = b1 + kMlpH,
                *b2 = W2 + kMlpH * kMlpH, *W3 = b2 + kMlpH, *b3 = W3 + kMlpH * kMlpOut;
    float h1[kMlpH];
    for (int o = 0; o < kMlpH; ++o) {
        float a = b1[o];
        for (int i = 0; i < kMlpIn; ++i) a = fmaf(W1[o * kMlpIn + i], f[i], a);
        h1[o] = a > 0.f ? a : 0.f;
    }
    float y = b3[out_unit];
    for (int o = 0; o < kMlpH; ++o) {
        float a = b2[o];
        for (int i = 0; i < kMlpH; ++i) a = fmaf(W2[o * kMlpH + i], h1[i], a);
        a = a > 0.f ? a : 0.f;
        y = fmaf(W3[out_unit * kMlpH + o], a, y);
    }
    return y;
}

__device__ void level_features(float f[kMlpIn], float nf, float sdf, float nu, float sdu,
                               float k, float n, float nnz) {
    f[0] = logf(1.f + nf);
    f[1] = logf(1.f + sdf);
    f[2] = logf(1.f + nu);
    f[3] = logf(1.f + sdu);
    f[4] = k;
    f[5] = nnz / n;
    f[6] = logf((nf + 1.f) / n);
    f[7] = logf((sdf + 1.f) / (nnz + 1.f));
    f[8] = logf((nu + 1.f) / n);
    f[9] = logf((sdu + 1.f) / (nnz + 1.f));
    f[10] = logf((sdf + 1.f) / (sdu + 1.f));
    f[11] = logf((nf + 1.f) / (nu + 1.f));
}

// Called by every thread; thread 0 computes, the block shares through LDS.
__device__ uint32_t choose_variant(const LevelParams &P, uint32_t k, uint32_t nf) {
    if (P.policy == kPush || P.policy == kPull || P.policy == kBitmap) return P.policy;
    __shared__ uint32_t s_var;
    if (threadIdx.x == 0) {
        const BfsState *st = P.st;
        const uint32_t cs = k & 3;
        const float fnf = (float)nf;
        const float fsdf = (float)st->sdf[cs];
        const float fnu = (float)((uint32_t)P.n - st->visited_cnt);
        const float fsdu = (float)((unsigned long long)P.nnz - st->visited_deg);
        uint32_t v = kPush;
        if (P.policy == kHeuristic) {
            // pull when the frontier's edges outweigh a fraction of the
            // unvisited edges and the frontier is not tiny
            if (fsdf * 14.f > fsdu && fnf * 24.f > (float)P.n) v = kPull;
        } else if (P.mlp != nullptr) {
            float f[kMlpIn];
            level_features(f, fnf, fsdf, fnu, fsdu, (float)k, (float)P.n, (float)P.nnz);
            const float *mean = P.mlp + kMlpParams, *istd = mean + kMlpIn;
            for (int i = 0; i < kMlpIn; ++i) f[i] = (f[i] - mean[i]) * istd[i];
            float best = 0.f;
            bool ok = true;
            for (int o = 0; o < kMlpOut; ++o) {
                float y = mlp_logtime(P.mlp, f, o);
                if (!(y == y) || y > 1e30f || y < -1e30f) ok = false;   // NaN / inf -> fallback
                if (o == 0 || y < best) { best = y; v = (uint32_t)o; }
            }
            if (!ok) v = kPush;
            if (v == kBitmap && !P.maintain_fb) v = kPush;
        }
        s_var = v;
    }
    __syncthreads();
    return s_var;
}

// ---------------------------------------------------------------------------
// the per-entry step: test the row mask, min-select the parent, claim
// ---------------------------------------------------------------------------

// Returns true for exactly one (j, i) pair per newly reached i: the one whose
// atomicMin found the parent slot still empty.  Every unmasked pair reaches
// the atomicMin unless the slot already holds a smaller or equal vertex, so
// the final parent is the minimum over the level's frontier in-neighbours.
__device__ __forceinline__ bool visit(const LevelParams &P, const uint32_t *vb_cur,
                                      int32_t i, int32_t j, uint32_t k) {
    const uint32_t w = vb_cur[(uint32_t)i >> 5];
    if ((w >> (i & 31)) & 1u) return false;            // row i masked (visited through level k)
    const uint32_t p = P.parent[i];                    // may be stale: only used to skip
    if (p <= (uint32_t)j) return false;
    const uint32_t old = atomicMin(&P.parent[i], (uint32_t)j);
    if (old != 0xFFFFFFFFu) return false;
    P.level[i] = (int32_t)(k + 1);
    return true;
}

// Wave-aggregated append of newly reached vertices to the next frontier: one
// atomicAdd per wave, lane offsets from the ballot mask.  Must be called by
// every lane of the wave.
__device__ __forceinline__ void append_next(const LevelParams &P, bool owner, int32_t i,
                                            uint32_t ns, int32_t *q_nxt, uint32_t *vb_nxt,
                                            uint32_t *fb_nxt) {
    const unsigned long long m = __ballot(owner);
    if (m == 0ull) return;
    const uint32_t lane = lane_id();
    const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&P.st->nf[ns], (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader, 64);
    unsigned long long d = 0;
    if (owner) {
        q_nxt[base + lanes_below(m)] = i;
        const uint32_t bit = 1u << (i & 31);
        atomicOr(&vb_nxt[(uint32_t)i >> 5], bit);
        if (P.maintain_fb) atomicOr(&fb_nxt[(uint32_t)i >> 5], bit);
        if (P.stats) d = (unsigned long long)(P.out_ptr[i + 1] - P.out_ptr[i]);
    }
    if (P.stats) {
        d = wave_sum64(d);
        if (lane == leader) atomicAdd(&P.st->sdf[ns], d);
    }
}

struct TileLds {
    uint32_t pre[kBlock];
    int32_t r0[kBlock];
    int32_t j[kBlock];
    uint32_t wsum[kBlock / 64];
};

// Expand one tile of up to kBlock frontier columns (one per thread: j >= 0
// with entries [r0, r0 + deg)) with every lane of the block: an exclusive scan
// of the degrees places the tile's entries on one line, lane t takes entries
// t, t + 256, ... and finds its column by binary search over the prefix.
// Consecutive lanes read consecutive entries of a column: coalesced.
__device__ void expand_tile(const LevelParams &P, TileLds &L, int32_t j, int32_t r0,
                            uint32_t deg, uint32_t k, uint32_t ns, const uint32_t *vb_cur,
                            int32_t *q_nxt, uint32_t *vb_nxt, uint32_t *fb_nxt) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t incl = wave_incl_scan(deg);
    if (lane == 63) L.wsum[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kBlock / 64; ++w) {
        const uint32_t s = L.wsum[w];
        woff += (w < wave) ? s : 0u;
        total += s;
    }
    L.pre[tid] = woff + incl - deg;
    L.j[tid] = j;
    L.r0[tid] = r0;
    __syncthreads();
    uint32_t lo = 0;
    for (uint32_t base = 0; base < total; base += kBlock) {
        const uint32_t e = base + tid;
        bool owner = false;
        int32_t i = -1;
        if (e < total) {
            uint32_t hi = kBlock - 1;                  // last slot with pre <= e
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (L.pre[mid] <= e) lo = mid; else hi = mid - 1;
            }
            i = P.out_idx[L.r0[lo] + (int32_t)(e - L.pre[lo])];
            owner = visit(P, vb_cur, i, L.j[lo], k);
        }
        append_next(P, owner, i, ns, q_nxt, vb_nxt, fb_nxt);
    }
    __syncthreads();   // L is reused by the next tile
}

// A frontier column j with out-degree >= heavy_min is not expanded in its
// tile: it is queued with its chunk count, and the tail kernel spreads its
// chunks over the whole grid.  One 64-bit atomic gives both the queue slot and
// the first chunk id, so chunk ids grow with queue position (binary search).
__device__ __forceinline__ void queue_heavy(const LevelParams &P, uint32_t cs, int32_t j,
                                            uint32_t deg) {
    const uint32_t nch = (deg + P.chunk - 1u) / P.chunk;
    const unsigned long long old =
        atomicAdd(&P.st->heavy[cs], 1ull | ((unsigned long long)nch << 32));
    HeavyItem it;
    it.v = j;
    it.chunk_base = (uint32_t)(old >> 32);
    P.heavy[(uint32_t)old] = it;
}

// ---------------------------------------------------------------------------
// the three forms of one level
// ---------------------------------------------------------------------------

__device__ void push_level(const LevelParams &P, TileLds &L, uint32_t k, uint32_t nf,
                           uint32_t bid, uint32_t nblocks) {
    const uint32_t cs = k & 3, ns = (k + 1) & 3;
    const uint32_t *vb_cur = P.vb[k & 1];
    uint32_t *vb_nxt = P.vb[(k + 1) & 1];
    uint32_t *fb_cur = P.fb[k & 1];
    uint32_t *fb_nxt = P.fb[(k + 1) & 1];
    const int32_t *q_cur = P.q[k & 1];
    int32_t *q_nxt = P.q[(k + 1) & 1];
    for (uint32_t tile = bid; tile * kBlock < nf; tile += nblocks) {
        const uint32_t pos = tile * kBlock + threadIdx.x;
        int32_t j = -1, r0 = 0;
        uint32_t deg = 0;
        if (pos < nf) {
            j = q_cur[pos];
            r0 = P.out_ptr[j];
            deg = (uint32_t)(P.out_ptr[j + 1] - r0);
            atomicOr(&vb_nxt[(uint32_t)j >> 5], 1u << (j & 31));   // F_k joins B_{k+1}
            if (P.maintain_fb) fb_cur[(uint32_t)j >> 5] = 0u;      // every bit there is in F_k
            if (deg >= P.heavy_min) {
                queue_heavy(P, cs, j, deg);
                deg = 0;
            }
        }
        expand_tile(P, L, j, r0, deg, k, ns, vb_cur, q_nxt, vb_nxt, fb_nxt);
    }
}

__device__ void bitmap_level(const LevelParams &P, TileLds &L, uint32_t k, uint32_t bid,
                             uint32_t nblocks) {
    const uint32_t cs = k & 3, ns = (k + 1) & 3;
    const uint32_t *vb_cur = P.vb[k & 1];
    uint32_t *vb_nxt = P.vb[(k + 1) & 1];
    uint32_t *fb_cur = P.fb[k & 1];
    uint32_t *fb_nxt = P.fb[(k + 1) & 1];
    int32_t *q_nxt = P.q[(k + 1) & 1];
    for (uint32_t wbase = bid * kBlock; wbase < P.words; wbase += nblocks * kBlock) {
        const uint32_t w = wbase + threadIdx.x;
        uint32_t bits = (w < P.words) ? fb_cur[w] : 0u;
        if (bits) {
            fb_cur[w] = 0u;
            atomicOr(&vb_nxt[w], bits);
        }
        // one frontier column per thread per round, lowest bit first
        while (__syncthreads_or(bits != 0u)) {
            int32_t j = -1, r0 = 0;
            uint32_t deg = 0;
            if (bits) {
                const uint32_t b = (uint32_t)__ffs((int)bits) - 1u;
                bits &= bits - 1u;
                j = (int32_t)(w * 32u + b);
                r0 = P.out_ptr[j];
                deg = (uint32_t)(P.out_ptr[j + 1] - r0);
                if (deg >= P.heavy_min) {
                    queue_heavy(P, cs, j, deg);
                    deg = 0;
                }
            }
            expand_tile(P, L, j, r0, deg, k, ns, vb_cur, q_nxt, vb_nxt, fb_nxt);
        }
    }
}

constexpr uint32_t kPullSerial = 32;     // in-neighbours a lane scans before handing off

struct PullLds {
    int32_t lng[kBlock];
    uint32_t nlong;
};

// Row-wise form over the unvisited list U (or all vertices the first time):
// for u not visited through level k, scan its in-neighbours in ascending order
// and stop at the first w with level[w] = k - the smallest frontier
// in-neighbour, i.e. the same min-parent the push form produces.  Rows with
// long in-lists that are not settled by their first kPullSerial entries are
// finished one wave per row (64 entries per step, ballot for the first hit).
__device__ void pull_level(const LevelParams &P, PullLds &L, uint32_t k, uint32_t nf,
                           uint32_t bid, uint32_t nblocks) {
    const uint32_t ns = (k + 1) & 3;
    const uint32_t *vb_cur = P.vb[k & 1];
    uint32_t *vb_nxt = P.vb[(k + 1) & 1];
    uint32_t *fb_cur = P.fb[k & 1];
    uint32_t *fb_nxt = P.fb[(k + 1) & 1];
    const int32_t *q_cur = P.q[k & 1];
    int32_t *q_nxt = P.q[(k + 1) & 1];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    // F_k joins B_{k+1}; its frontier bits are cleared
    for (uint32_t pos = bid * kBlock + tid; pos < nf; pos += nblocks * kBlock) {
        const int32_t j = q_cur[pos];
        atomicOr(&vb_nxt[(uint32_t)j >> 5], 1u << (j & 31));
        if (P.maintain_fb) fb_cur[(uint32_t)j >> 5] = 0u;
    }
    const uint32_t ub = P.st->u_buf;
    const uint32_t ulen = P.st->u_len;
    const bool all = (ulen == kAllVertices);
    const uint32_t len = all ? (uint32_t)P.n : ulen;
    const int32_t *U = P.ul[ub];
    int32_t *Un = P.ul[ub ^ 1u];
    const int32_t lk = (int32_t)k;
    for (uint32_t tile = bid; tile * kBlock < len; tile += nblocks) {
        if (tid == 0) L.nlong = 0;
        __syncthreads();
        const uint32_t pos = tile * kBlock + tid;
        int32_t u = -1, found = -1;
        bool keep = false;
        if (pos < len) {
            u = all ? (int32_t)pos : U[pos];
            if (!((vb_cur[(uint32_t)u >> 5] >> (u & 31)) & 1u)) {
                const int32_t e0 = P.in_ptr[u], e1 = P.in_ptr[u + 1];
                const int32_t lim = (e1 - e0 > (int32_t)kPullSerial) ? e0 + (int32_t)kPullSerial : e1;
                for (int32_t e = e0; e < lim; ++e) {
                    const int32_t w = P.in_idx[e];
                    if (P.level[w] == lk) { found = w; break; }
                }
                if (found < 0) {
                    if (lim < e1) {
                        const uint32_t slot = atomicAdd(&L.nlong, 1u);
                        L.lng[slot] = u;
                    } else {
                        keep = true;
                    }
                }
            }
        }
        const bool owner = found >= 0;
        if (owner) {
            P.parent[u] = (uint32_t)found;
            P.level[u] = lk + 1;
        }
        append_next(P, owner, u, ns, q_nxt, vb_nxt, fb_nxt);
        {   // survivors stay on the unvisited list
            const unsigned long long m = __ballot(keep);
            if (m) {
                const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&P.st->u_wr, (uint32_t)__popcll(m));
                base = __shfl(base, (int)leader, 64);
                if (keep) Un[base + lanes_below(m)] = u;
            }
        }
        __syncthreads();
        const uint32_t nlong = L.nlong;
        for (uint32_t t = wave; t < nlong; t += kBlock / 64) {
            const int32_t v = L.lng[t];
            const int32_t e1 = P.in_ptr[v + 1];
            int32_t hit = -1;
            for (int32_t eb = P.in_ptr[v] + (int32_t)kPullSerial; eb < e1; eb += 64) {
                const int32_t e = eb + (int32_t)lane;
                int32_t w = -1;
                bool f = false;
                if (e < e1) {
                    w = P.in_idx[e];
                    f = (P.level[w] == lk);
                }
                const unsigned long long m = __ballot(f);
                if (m) {
                    hit = __shfl(w, __ffsll((long long)m) - 1, 64);
                    break;
                }
            }
            const bool own = (hit >= 0) && lane == 0;
            if (own) {
                P.parent[v] = (uint32_t)hit;
                P.level[v] = lk + 1;
            }
            append_next(P, own, v, ns, q_nxt, vb_nxt, fb_nxt);
            if (hit < 0 && lane == 0) Un[atomicAdd(&P.st->u_wr, 1u)] = v;
        }
        __syncthreads();
    }
}

// Chunks of the columns queued by queue_heavy, spread over the grid.
__device__ void heavy_chunks(const LevelParams &P, uint32_t k, uint32_t bid, uint32_t nblocks) {
    const uint32_t cs = k & 3, ns = (k + 1) & 3;
    const uint32_t *vb_cur = P.vb[k & 1];
    uint32_t *vb_nxt = P.vb[(k + 1) & 1];
    uint32_t *fb_nxt = P.fb[(k + 1) & 1];
    int32_t *q_nxt = P.q[(k + 1) & 1];
    const unsigned long long packed = P.st->heavy[cs];
    const uint32_t count = (uint32_t)packed, chunks = (uint32_t)(packed >> 32);
    for (uint32_t c = bid; c < chunks; c += nblocks) {
        uint32_t lo = 0, hi = count - 1;               // last item with chunk_base <= c
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (P.heavy[mid].chunk_base <= c) lo = mid; else hi = mid - 1;
        }
        const HeavyItem it = P.heavy[lo];
        const int32_t j = it.v;
        const int32_t r1 = P.out_ptr[j + 1];
        const int32_t e0 = P.out_ptr[j] + (int32_t)((c - it.chunk_base) * P.chunk);
        const int32_t e1 = (r1 - e0 > (int32_t)P.chunk) ? e0 + (int32_t)P.chunk : r1;
        for (int32_t eb = e0; eb < e1; eb += kBlock) {
            const int32_t e = eb + (int32_t)threadIdx.x;
            bool owner = false;
            int32_t i = -1;
            if (e < e1) {
                i = P.out_idx[e];
                owner = visit(P, vb_cur, i, j, k);
            }
            append_next(P, owner, i, ns, q_nxt, vb_nxt, fb_nxt);
        }
    }
}

// End of level k, one thread: fold the level's counters into the state and
// advance (only if F_k was nonempty, so extra launches after the end are no-ops).
__device__ void finish_level(const LevelParams &P, uint32_t k, uint32_t nf) {
    BfsState *st = P.st;
    const uint32_t cs = k & 3, ns = (k + 1) & 3;
    if (nf == 0) return;
    const uint32_t nf_next = ld_agent(&st->nf[ns]);
    const unsigned long long sdf_next = ld_agent64(&st->sdf[ns]);
    const uint32_t variant = ld_agent(&st->variant);
    if (P.trace) {
        DevLevelRec r;
        r.level = k;
        r.variant = variant;
        r.nf = nf;
        r.nu = (uint32_t)P.n - st->visited_cnt;
        r.sdf = st->sdf[cs];
        r.sdu = (unsigned long long)P.nnz - st->visited_deg;
        P.trace[k % kTraceCap] = r;
    }
    st->visited_cnt += nf_next;
    st->visited_deg += sdf_next;
    if (variant == kPull) {
        st->u_buf ^= 1u;
        st->u_len = ld_agent(&st->u_wr);
    }
    st->u_wr = 0;
    __threadfence();
    st->level = k + 1;
}

__device__ void level_body(const LevelParams &P, uint32_t k, uint32_t nf, uint32_t bid,
                           uint32_t nblocks) {
    __shared__ TileLds tl;
    __shared__ PullLds pl;
    const uint32_t v = choose_variant(P, k, nf);
    if (bid == 0 && threadIdx.x == 0) {
        BfsState *st = P.st;
        const uint32_t fs = (k + 2) & 3;     // slot of level k+2: free since level k-2
        st->variant = v;
        st->nf[fs] = 0;
        st->heavy[fs] = 0ull;
        st->sdf[fs] = 0ull;
    }
    if (v == kPull) pull_level(P, pl, k, nf, bid, nblocks);
    else if (v == kBitmap) bitmap_level(P, tl, k, bid, nblocks);
    else push_level(P, tl, k, nf, bid, nblocks);
}

}  // namespace

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Initialise outputs and state for a search from one root (single_root >= 0)
// or from a list of roots in distinct components (multi-root: each root's
// component gets exactly the result of a search from that root alone).
__global__ __launch_bounds__(kBlock) void k_init(LevelParams P, int32_t nroots,
                                                 const int32_t *roots, int32_t single_root) {
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t v = gid; v < (uint32_t)P.n; v += stride) {
        P.level[v] = (single_root == (int32_t)v) ? 0 : -1;
        P.parent[v] = (single_root == (int32_t)v) ? (uint32_t)v : 0xFFFFFFFFu;
    }
    for (uint32_t w = gid; w < P.words; w += stride) {
        uint32_t bits = 0;
        if (single_root >= 0 && ((uint32_t)single_root >> 5) == w) bits = 1u << (single_root & 31);
        P.vb[0][w] = bits;
        P.vb[1][w] = 0u;
        if (P.maintain_fb) {
            P.fb[0][w] = bits;
            P.fb[1][w] = 0u;
        }
    }
    if (gid == 0) {
        BfsState *st = P.st;
        st->level = 0;
        st->done = 0;
        st->variant = 0;
        st->u_buf = 0;
        st->u_len = kAllVertices;
        st->u_wr = 0;
        st->barrier = 0;
        st->barrier_gen = 0;
        for (int r = 0; r < kRing; ++r) {
            st->nf[r] = 0;
            st->heavy[r] = 0ull;
            st->sdf[r] = 0ull;
        }
        if (single_root >= 0) {
            P.q[0][0] = single_root;
            st->nf[0] = 1;
            const unsigned long long d =
                (unsigned long long)(P.out_ptr[single_root + 1] - P.out_ptr[single_root]);
            st->sdf[0] = d;
            st->visited_cnt = 1;
            st->visited_deg = d;
        } else {
            st->nf[0] = (uint32_t)nroots;
            st->visited_cnt = (uint32_t)nroots;
            st->visited_deg = 0ull;   // completed by k_init_roots
        }
    }
}

// second init pass for multi-root searches (after k_init has cleared everything)
__global__ __launch_bounds__(kBlock) void k_init_roots(LevelParams P, int32_t nroots,
                                                       const int32_t *roots) {
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    unsigned long long d = 0;
    if (gid < (uint32_t)nroots) {
        const int32_t r = roots[gid];
        P.level[r] = 0;
        P.parent[r] = (uint32_t)r;
        atomicOr(&P.vb[0][(uint32_t)r >> 5], 1u << (r & 31));
        if (P.maintain_fb) atomicOr(&P.fb[0][(uint32_t)r >> 5], 1u << (r & 31));
        P.q[0][gid] = r;
        d = (unsigned long long)(P.out_ptr[r + 1] - P.out_ptr[r]);
    }
    d = wave_sum64(d);
    if (lane_id() == 0 && d) {
        atomicAdd(&P.st->sdf[0], d);
        atomicAdd(&P.st->visited_deg, d);
    }
}

__global__ __launch_bounds__(kBlock) void k_level(LevelParams P) {
    const uint32_t k = P.st->level;
    const uint32_t nf = P.st->nf[k & 3];
    if (nf == 0) return;
    level_body(P, k, nf, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_tail(LevelParams P) {
    BfsState *st = P.st;
    const uint32_t k = st->level;
    const uint32_t nf = st->nf[k & 3];
    if (nf != 0) heavy_chunks(P, k, blockIdx.x, gridDim.x);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&st->done, 1u);
        if (prev == gridDim.x - 1) {
            __threadfence();
            st->done = 0;
            finish_level(P, k, nf);
        }
    }
}

// Grid barrier for the cooperative kernel.  Returns false (and raises the
// error flag through `barrier_gen` staying put) only if the spin limit runs
// out, which cannot happen when every block is resident.
__device__ bool grid_sync(BfsState *st, uint32_t nblocks, uint32_t *s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        const uint32_t gen = ld_agent(&st->barrier_gen);
        __threadfence();
        const uint32_t arrived = atomicAdd(&st->barrier, 1u);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&st->barrier, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&st->barrier_gen, 1u);
        } else {
            uint32_t spins = 0;
            while (ld_agent(&st->barrier_gen) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 26)) { ok = 0; break; }
            }
        }
        __threadfence();
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Every level in one launch: level body, barrier, split-column chunks,
// barrier, block 0 finishes the level, barrier.  The loop ends when the
// frontier is empty (every block reads the same counters after a barrier).
__global__ __launch_bounds__(kBlock) void k_persistent(LevelParams P) {
    __shared__ uint32_t s_ok;
    BfsState *st = P.st;
    const uint32_t nb = gridDim.x;
    for (;;) {
        const uint32_t k = ld_agent(&st->level);
        const uint32_t nf = ld_agent(&st->nf[k & 3]);
        if (nf == 0) break;
        level_body(P, k, nf, blockIdx.x, nb);
        if (!grid_sync(st, nb, &s_ok)) break;
        heavy_chunks(P, k, blockIdx.x, nb);
        if (!grid_sync(st, nb, &s_ok)) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) finish_level(P, k, nf);
        if (!grid_sync(st, nb, &s_ok)) break;
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

hipError_t launch_init(const LevelParams &p, int32_t nroots, const int32_t *roots_dev,
                       int32_t single_root, hipStream_t s) {
    const uint32_t work = (uint32_t)p.n > p.words ? (uint32_t)p.n : p.words;
    uint32_t grid = (work + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, p, nroots, roots_dev, single_root);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || single_root >= 0) return e;
    const uint32_t g2 = ((uint32_t)nroots + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_init_roots, dim3(g2 ? g2 : 1), dim3(kBlock), 0, s, p, nroots, roots_dev);
    return hipGetLastError();
}

hipError_t launch_level(const LevelParams &p, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_level, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_tail(const LevelParams &p, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_tail, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

uint32_t persistent_max_grid(int device) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kBlock, 0) != hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return (uint32_t)(per_cu * cus);
}

hipError_t launch_persistent(const LevelParams &p, uint32_t grid, hipStream_t s) {
    LevelParams pc = p;
    void *args[] = {&pc};
    return hipLaunchCooperativeKernel((const void *)k_persistent, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace bfsi

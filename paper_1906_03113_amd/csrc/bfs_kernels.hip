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

#include "bfs_device.h"
#include "bfs_internal.h"

namespace bfsi {

namespace {

// ---------------------------------------------------------------------------
// variant choice (uniform across the grid: every block computes it from the
// same device counters)
// ---------------------------------------------------------------------------

// Feature i of a level (lane i of the calling wave computes feature i; the
// selector's training code computes the same twelve numbers in float64):
// log sizes of the frontier and of the unvisited remainder, in vertices and in
// column entries, the level, the mean degree, and their log-ratios.
__device__ __forceinline__ float level_feature(uint32_t i, float nf, float sdf, float nu,
                                               float sdu, float k, float n, float nnz) {
    switch (i) {
        case 0: return logf(1.f + nf);
        case 1: return logf(1.f + sdf);
        case 2: return logf(1.f + nu);
        case 3: return logf(1.f + sdu);
        case 4: return logf(1.f + k);
        case 5: return nnz / n;
        case 6: return logf((nf + 1.f) / n);
        case 7: return logf((sdf + 1.f) / (nnz + 1.f));
        case 8: return logf((nu + 1.f) / n);
        case 9: return logf((sdu + 1.f) / (nnz + 1.f));
        case 10: return logf((sdf + 1.f) / (sdu + 1.f));
        case 11: return logf((nf + 1.f) / (nu + 1.f));
        default: return 0.f;
    }
}

// The form level k runs, decided once per level by one full wave (all 64
// lanes call it with the same counters) before the level's launch: the
// forced form, the edge-ratio rule, or the network's argmin.
__device__ __forceinline__ uint32_t decide_wave(const LevelParams &P, const float *w, uint32_t k,
                                                float fnf, float fsdf, float fnu, float fsdu) {
    if (P.policy == kPush || P.policy == kPull || P.policy == kBitmap) return P.policy;
    if (P.policy == kShortCircuit) return kPush;
    uint32_t v = kPush;
    if (P.policy == kHeuristic) {
        // pull when the frontier's edges outweigh 1/14 of the unvisited edges
        if (fsdf * 14.f > fsdu) v = kPull;
    } else if (P.mlp != nullptr) {
        const float f = level_feature(lane_id(), fnf, fsdf, fnu, fsdu, (float)k, (float)P.n,
                                      (float)P.nnz);
        const int b = mlp_argmin(w, f);
        v = (b < 0) ? (uint32_t)kPush : (uint32_t)b;
        if (v == kBitmap && !P.maintain_fb) v = kPush;
    }
    return v;
}

struct LevelStats {
    float nf, sdf, nu, sdu;
};

// The counters of the level about to run, read by one thread (coherent loads).
__device__ __forceinline__ LevelStats level_stats(const LevelParams &P, uint32_t k) {
    const BfsState *st = P.st;
    const uint32_t cs = k & 3;
    LevelStats L;
    L.nf = (float)(ld_agent(&st->nf[cs]) + (uint32_t)ld_agent64(&st->heavy[cs]));
    L.sdf = (float)ld_agent64(&st->sdf[cs]);
    L.nu = (float)((uint32_t)P.n - ld_agent(&st->visited_cnt));
    L.sdu = (float)((unsigned long long)P.nnz - ld_agent64(&st->visited_deg));
    return L;
}

// The form of level k from its counters L, by the first wave of the calling
// block (every thread of the block calls it), recorded in the state.  The
// network's weights are first staged in the LDS buffer s_w (kMlpTotal floats)
// with coalesced loads by the whole block; its evaluation then reads LDS only.
__device__ __forceinline__ void decide_level(const LevelParams &P, uint32_t k, const LevelStats &L,
                                             float *s_w) {
    const bool net = (P.policy == kLearned) && P.mlp != nullptr;
    if (net)
        for (uint32_t i = threadIdx.x; i < (uint32_t)kMlpTotal; i += blockDim.x) s_w[i] = P.mlp[i];
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t v = decide_wave(P, s_w, k, L.nf, L.sdf, L.nu, L.sdu);
        if (threadIdx.x == 0) P.st->variant = v;
    }
    __syncthreads();
}

// The form level k runs: the forced one, or the one decided before it.
__device__ __forceinline__ uint32_t level_form(const LevelParams &P, uint32_t decided) {
    if (P.policy == kShortCircuit) return kPush;
    if (P.policy == kPush || P.policy == kPull || P.policy == kBitmap) return P.policy;
    return decided;
}

// ---------------------------------------------------------------------------
// per-block staging of the level's output
// ---------------------------------------------------------------------------
//
// Newly reached vertices are first collected in LDS and written out in
// batches: one global atomicAdd per batch reserves room in the next frontier
// list, instead of one per wave (a single counter hit by every wave of the grid
// serialises at the memory-side atomic unit).

// Each round adds at most one entry per thread to each buffer, so a buffer
// flushed once it holds more than (cap - kBlock) entries never overflows.
constexpr uint32_t kIlp = 4;           // column entries per lane per round
constexpr uint32_t kOutCap = 512;      // short-column entries staged per block
constexpr uint32_t kOutFlush = kOutCap - kBlock;
constexpr uint32_t kLongCap = 320;     // long-column entries staged per block
constexpr uint32_t kLongFlush = kLongCap - kBlock;
constexpr uint32_t kUCap = 384;        // unvisited-list survivors staged per block (pull)
constexpr uint32_t kUFlush = kUCap - kBlock;

struct OutLds {
    QEnt q[kOutCap];
    int32_t lv[kLongCap];
    uint32_t lch[kLongCap];
    int32_t u[kUCap];
    uint32_t qn, ln, un;
    uint32_t qbase, lpos, lcb, ltot, ubase;
    unsigned long long sdf;
};

struct LevelPtrs {
    uint32_t k, cs, ns;
    bool sc;                  // this level claims rows short-circuit (parents set afterwards)
    bool pre;                 // pre-read the parent before its atomicMin
    const uint32_t *vb_cur;
    uint32_t *vb_nxt;
    const uint32_t *fb_cur;
    uint32_t *fb_nxt, *fb_old;
    const QEnt *q_cur;
    QEnt *q_nxt;
    const HeavyItem *h_cur;
    HeavyItem *h_nxt;
    const uint32_t *c_cur;
    uint32_t *c_nxt;
    int32_t *u_nxt;
};

__device__ __forceinline__ LevelPtrs level_ptrs(const LevelParams &P, uint32_t k) {
    LevelPtrs L;
    L.k = k;
    L.cs = k & 3;
    L.ns = (k + 1) & 3;
    // selects instead of indexing the parameter arrays with a runtime index
    // (which would force the kernel-argument struct into scratch memory)
    const bool odd = k & 1;
    const uint32_t r3 = k % 3;
    L.vb_cur = odd ? P.vb[1] : P.vb[0];
    L.vb_nxt = odd ? P.vb[0] : P.vb[1];
    L.fb_cur = r3 == 0 ? P.fb[0] : (r3 == 1 ? P.fb[1] : P.fb[2]);
    L.fb_nxt = r3 == 0 ? P.fb[1] : (r3 == 1 ? P.fb[2] : P.fb[0]);
    L.fb_old = r3 == 0 ? P.fb[2] : (r3 == 1 ? P.fb[0] : P.fb[1]);
    L.q_cur = odd ? P.q[1] : P.q[0];
    L.q_nxt = odd ? P.q[0] : P.q[1];
    L.h_cur = odd ? P.hl[1] : P.hl[0];
    L.h_nxt = odd ? P.hl[0] : P.hl[1];
    L.c_cur = odd ? P.cmap[1] : P.cmap[0];
    L.c_nxt = odd ? P.cmap[0] : P.cmap[1];
    L.u_nxt = nullptr;
    L.sc = false;
    L.pre = true;
    return L;
}

__device__ __forceinline__ void out_init(OutLds &O) {
    if (threadIdx.x == 0) {
        O.qn = 0;
        O.ln = 0;
        O.un = 0;
        O.sdf = 0ull;
    }
    __syncthreads();
}

// Write the staged entries out.  Called by every thread of the block; `final`
// also folds the block's degree sum into the level's counter.
__device__ __forceinline__ void out_flush(const LevelParams &P, const LevelPtrs &L, OutLds &O, bool final) {
    __syncthreads();
    const uint32_t tid = threadIdx.x;
    const uint32_t qn = O.qn, ln = O.ln, un = O.un;
    const bool need = final || qn > kOutFlush || ln > kLongFlush || un > kUFlush;
    if (!need) return;                                   // uniform: everyone read the same counters
    if (ln) {                                            // chunk offsets within the batch
        const uint32_t a0 = (2 * tid < ln) ? O.lch[2 * tid] : 0u;
        const uint32_t a1 = (2 * tid + 1 < ln) ? O.lch[2 * tid + 1] : 0u;
        const uint32_t lane = lane_id(), wave = tid >> 6;
        const uint32_t incl = wave_incl_scan(a0 + a1);
        __shared__ uint32_t s_w[kBlock / 64];
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (uint32_t w = 0; w < kBlock / 64; ++w) {
            off += (w < wave) ? s_w[w] : 0u;
            tot += s_w[w];
        }
        const uint32_t ex = off + incl - (a0 + a1);
        if (2 * tid < ln) O.lch[2 * tid] = ex;
        if (2 * tid + 1 < ln) O.lch[2 * tid + 1] = ex + a0;
        if (tid == 0) O.ltot = tot;
        __syncthreads();
    }
    if (tid == 0) {
        if (qn) O.qbase = atomicAdd(&P.st->nf[L.ns], qn);
        if (ln) {
            const unsigned long long old = atomicAdd(
                &P.st->heavy[L.ns], (unsigned long long)ln | ((unsigned long long)O.ltot << 32));
            O.lpos = (uint32_t)old;
            O.lcb = (uint32_t)(old >> 32);
        }
        if (un) O.ubase = atomicAdd(&P.st->u_wr, un);
        if (final && P.stats && O.sdf) atomicAdd(&P.st->sdf[L.ns], O.sdf);
    }
    __syncthreads();
    for (uint32_t t = tid; t < qn; t += kBlock) L.q_nxt[O.qbase + t] = O.q[t];
    for (uint32_t t = tid; t < ln; t += kBlock) {
        HeavyItem it;
        it.v = O.lv[t];
        it.chunk_base = O.lcb + O.lch[t];
        L.h_nxt[O.lpos + t] = it;
        const uint32_t c1 = (t + 1 < ln) ? O.lch[t + 1] : O.ltot;
        for (uint32_t c = O.lch[t]; c < c1; ++c) L.c_nxt[O.lcb + c] = O.lpos + t;   // chunk -> column
    }
    for (uint32_t t = tid; t < un; t += kBlock) L.u_nxt[O.ubase + t] = O.u[t];
    __syncthreads();
    if (tid == 0) {
        O.qn = 0;
        O.ln = 0;
        O.un = 0;
        if (final) O.sdf = 0ull;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the per-entry step: test the row mask, min-select the parent, claim
// ---------------------------------------------------------------------------

// The claim of an unmasked pair (j, i) (row i not visited through level k):
// exactly one such pair per newly reached i wins, the one whose atomicMin
// found the parent slot still empty.  Every unmasked pair reaches the
// atomicMin unless the slot already holds a smaller or equal vertex, so the
// final parent is the minimum over the level's frontier in-neighbours.  The
// pre-read is a coherent (agent-scope) load, so it sees the other lanes'
// atomics and most pairs that cannot lower the parent skip the atomic.
//
// On a short-circuit level (Theorem 2) the first frontier column to reach row
// i claims it by turning level[i] from -1 to k + 1, so each reached vertex
// takes exactly one claim and no parent atomic; k_parents sets those parents
// after the search.  The coherent pre-read of level[i] sees other XCDs'
// claims, so most losing pairs skip the atomic.  (settle4 below.)
// Set one bit per active lane in a bitmap.  Lanes holding vertices of the
// same 32-bit word are combined into one atomicOr (wave-contiguous atomics are
// an order of magnitude cheaper than ones that collide on a word); after a few
// distinct words the remaining lanes fall back to one atomic each.
__device__ __forceinline__ void or_bits_grouped(uint32_t *bm, bool on, int32_t v) {
    unsigned long long act = __ballot(on);
    const uint32_t lane = lane_id();
    const uint32_t myw = (uint32_t)v >> 5;
    for (int round = 0; act; ++round) {
        if (round == 4) {
            if (on && ((act >> lane) & 1ull)) atomicOr(&bm[myw], 1u << (v & 31));
            break;
        }
        const uint32_t leader = (uint32_t)__ffsll((long long)act) - 1u;
        const uint32_t w = __shfl(myw, (int)leader, 64);
        const bool mine = on && myw == w;
        const unsigned long long grp = __ballot(mine);
        uint32_t bits = mine ? (1u << (v & 31)) : 0u;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) bits |= __shfl_xor(bits, d, 64);
        if (lane == leader) atomicOr(&bm[w], bits);
        act &= ~grp;
    }
}

// A newly reached vertex joins F_{k+1}: its column bounds are read once here
// (or passed in when the caller already has them), its bit goes into B_{k+1},
// and it is staged for the next frontier list (short column) or for the next
// level's chunk queue (long column).  `grouped` combines the bitmap updates of
// lanes that hold vertices of the same word (the pull form reaches vertices in
// ascending order).
__device__ __forceinline__ void append_next(const LevelParams &P, const LevelPtrs &L, OutLds &O,
                                            bool owner, int32_t i, bool grouped = false,
                                            int32_t kr0 = -1, int32_t kr1 = -1) {
    const unsigned long long any = __ballot(owner);
    if (any == 0ull) return;
    int32_t r0 = 0, r1 = 0;
    if (owner) {
        if (kr0 >= 0) {
            r0 = kr0;
            r1 = kr1;
        } else {
            r0 = P.out_ptr[i];
            r1 = P.out_ptr[i + 1];
        }
    }
    if (grouped) {
        or_bits_grouped(L.vb_nxt, owner, i);
        if (P.maintain_fb) or_bits_grouped(L.fb_nxt, owner, i);
    } else if (owner) {
        const uint32_t bit = 1u << (i & 31);
        atomicOr(&L.vb_nxt[(uint32_t)i >> 5], bit);
        if (P.maintain_fb) atomicOr(&L.fb_nxt[(uint32_t)i >> 5], bit);
    }
    const uint32_t deg = (uint32_t)(r1 - r0);
    const bool longcol = owner && deg >= P.heavy_min;
    const bool shortcol = owner && !longcol;
    const uint32_t lane = lane_id();
    const unsigned long long m = __ballot(shortcol);
    if (m) {
        const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&O.qn, (uint32_t)__popcll(m));
        base = __shfl(base, (int)leader, 64);
        if (shortcol) {
            QEnt e;
            e.v = i;
            e.r0 = r0;
            e.r1 = r1;
            e.pad = 0;
            O.q[base + lanes_below(m)] = e;
        }
    }
    if (longcol) {
        const uint32_t slot = atomicAdd(&O.ln, 1u);
        O.lv[slot] = i;
        O.lch[slot] = (deg + P.chunk - 1u) / P.chunk;
    }
    if (P.stats) {
        const unsigned long long d = wave_sum64(owner ? (unsigned long long)deg : 0ull);
        if (lane == 0) atomicAdd(&O.sdf, d);
    }
}

struct TileLds {
    uint32_t pre[kBlock];
    int32_t r0[kBlock];
    int32_t j[kBlock];
    uint32_t wsum[kBlock / 64];
};

// Entry e of the tile's concatenated columns: its row index and its column.
// `lo` only moves forward (entries are visited in increasing e).
__device__ __forceinline__ void tile_entry(const LevelParams &P, const TileLds &T, uint32_t total,
                                           uint32_t e, uint32_t &lo, int32_t &i, int32_t &j) {
    if (e >= total) return;
    uint32_t hi = kBlock - 1;                          // last slot with pre <= e
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (T.pre[mid] <= e) lo = mid; else hi = mid - 1;
    }
    i = P.out_idx[T.r0[lo] + (int32_t)(e - T.pre[lo])];
    j = T.j[lo];
}

// The word of B_k holding row i (all ones for "no entry": masked).
__device__ __forceinline__ uint32_t mask_word(const LevelPtrs &L, int32_t i) {
    return (i >= 0) ? L.vb_cur[(uint32_t)i >> 5] : 0xFFFFFFFFu;
}

// Mask test, parent min-select and claim for one pair (j, i), then the
// block-wide append of the vertices claimed.  Called by every thread.
// The claims of a lane's four entries of one round, with the memory
// operations of the four in flight together: the coherent pre-reads, then the
// atomics, then the column bounds of the rows it won (a row reached through
// two of the four entries is won by the atomic performed first).  Then each
// winner joins F_{k+1} (LDS staging, with a flush check after each of the
// four appends so the staging buffers never overflow).
__device__ __forceinline__ bool unmasked(int32_t i, uint32_t mw) {
    return (i >= 0) && !((mw >> (i & 31)) & 1u);
}

__device__ __forceinline__ void settle4(const LevelParams &P, const LevelPtrs &L, OutLds &O,
                                        int32_t i0, int32_t j0, uint32_t m0, int32_t i1, int32_t j1,
                                        uint32_t m1, int32_t i2, int32_t j2, uint32_t m2, int32_t i3,
                                        int32_t j3, uint32_t m3) {
    const bool u0 = unmasked(i0, m0), u1 = unmasked(i1, m1);
    const bool u2 = unmasked(i2, m2), u3 = unmasked(i3, m3);
    bool o0, o1, o2, o3;
    const int32_t nk = (int32_t)(L.k + 1);
    if (L.sc) {
        // short circuit: the first column to turn level[i] from -1 claims i
        const int32_t v0 = u0 ? __hip_atomic_load(&P.level[i0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const int32_t v1 = u1 ? __hip_atomic_load(&P.level[i1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const int32_t v2 = u2 ? __hip_atomic_load(&P.level[i2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const int32_t v3 = u3 ? __hip_atomic_load(&P.level[i3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const bool t0 = u0 && v0 == -1, t1 = u1 && v1 == -1, t2 = u2 && v2 == -1, t3 = u3 && v3 == -1;
        const int32_t c0 = t0 ? atomicCAS(&P.level[i0], -1, nk) : 0;
        const int32_t c1 = t1 ? atomicCAS(&P.level[i1], -1, nk) : 0;
        const int32_t c2 = t2 ? atomicCAS(&P.level[i2], -1, nk) : 0;
        const int32_t c3 = t3 ? atomicCAS(&P.level[i3], -1, nk) : 0;
        o0 = t0 && c0 == -1;
        o1 = t1 && c1 == -1;
        o2 = t2 && c2 == -1;
        o3 = t3 && c3 == -1;
    } else {
        // min-select: pairs that cannot lower the parent skip the atomic (on a
        // small level the pre-read is skipped: its latency costs more than
        // the few atomics it would save); the atomic that found the slot
        // empty claims the row
        const bool pre = L.pre && !P.no_preread;
        const uint32_t p0 = (u0 && pre) ? ld_agent(&P.parent[i0]) : 0xFFFFFFFFu;
        const uint32_t p1 = (u1 && pre) ? ld_agent(&P.parent[i1]) : 0xFFFFFFFFu;
        const uint32_t p2 = (u2 && pre) ? ld_agent(&P.parent[i2]) : 0xFFFFFFFFu;
        const uint32_t p3 = (u3 && pre) ? ld_agent(&P.parent[i3]) : 0xFFFFFFFFu;
        const bool t0 = u0 && p0 > (uint32_t)j0, t1 = u1 && p1 > (uint32_t)j1;
        const bool t2 = u2 && p2 > (uint32_t)j2, t3 = u3 && p3 > (uint32_t)j3;
        const uint32_t a0 = t0 ? atomicMin(&P.parent[i0], (uint32_t)j0) : 0u;
        const uint32_t a1 = t1 ? atomicMin(&P.parent[i1], (uint32_t)j1) : 0u;
        const uint32_t a2 = t2 ? atomicMin(&P.parent[i2], (uint32_t)j2) : 0u;
        const uint32_t a3 = t3 ? atomicMin(&P.parent[i3], (uint32_t)j3) : 0u;
        o0 = t0 && a0 == 0xFFFFFFFFu;
        o1 = t1 && a1 == 0xFFFFFFFFu;
        o2 = t2 && a2 == 0xFFFFFFFFu;
        o3 = t3 && a3 == 0xFFFFFFFFu;
        if (P.atomics) {                                 // counted: one add per wave
            const unsigned long long act = __ballot(true);
            const uint32_t na = (uint32_t)(__popcll(__ballot(t0)) + __popcll(__ballot(t1)) +
                                           __popcll(__ballot(t2)) + __popcll(__ballot(t3)));
            if (lane_id() == (uint32_t)__ffsll((long long)act) - 1u && na)
                atomicAdd(P.atomics, (unsigned long long)na);
        }
        if (o0) P.level[i0] = nk;
        if (o1) P.level[i1] = nk;
        if (o2) P.level[i2] = nk;
        if (o3) P.level[i3] = nk;
    }
    const int32_t a00 = o0 ? P.out_ptr[i0] : 0, a01 = o0 ? P.out_ptr[i0 + 1] : 0;
    const int32_t a10 = o1 ? P.out_ptr[i1] : 0, a11 = o1 ? P.out_ptr[i1 + 1] : 0;
    const int32_t a20 = o2 ? P.out_ptr[i2] : 0, a21 = o2 ? P.out_ptr[i2 + 1] : 0;
    const int32_t a30 = o3 ? P.out_ptr[i3] : 0, a31 = o3 ? P.out_ptr[i3 + 1] : 0;
    append_next(P, L, O, o0, i0, false, a00, a01);
    out_flush(P, L, O, false);
    append_next(P, L, O, o1, i1, false, a10, a11);
    out_flush(P, L, O, false);
    append_next(P, L, O, o2, i2, false, a20, a21);
    out_flush(P, L, O, false);
    append_next(P, L, O, o3, i3, false, a30, a31);
    out_flush(P, L, O, false);
}

// Expand one tile of up to kBlock short frontier columns (one per thread: j >= 0
// with entries [r0, r0 + deg)) with every lane of the block: an exclusive scan
// of the degrees places the tile's entries on one line, lane t takes entries
// t, t + 256, ... and finds its column by binary search over the prefix.
// Consecutive lanes read consecutive entries of a column: coalesced.
__device__ __forceinline__ void expand_tile(const LevelParams &P, const LevelPtrs &L, TileLds &T, OutLds &O,
                            int32_t j, int32_t r0, uint32_t deg) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t incl = wave_incl_scan(deg);
    if (lane == 63) T.wsum[wave] = incl;
    __syncthreads();
    uint32_t woff = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kBlock / 64; ++w) {
        const uint32_t s = T.wsum[w];
        woff += (w < wave) ? s : 0u;
        total += s;
    }
    T.pre[tid] = woff + incl - deg;
    T.j[tid] = j;
    T.r0[tid] = r0;
    __syncthreads();
    // kIlp (= 4) entries per lane per round, their loads issued together; the
    // four are kept in scalars so nothing is indexed dynamically
    uint32_t lo = 0;
    for (uint32_t base = 0; base < total; base += kBlock * kIlp) {
        int32_t i0 = -1, i1 = -1, i2 = -1, i3 = -1, j0 = 0, j1 = 0, j2 = 0, j3 = 0;
        tile_entry(P, T, total, base + 0 * kBlock + tid, lo, i0, j0);
        tile_entry(P, T, total, base + 1 * kBlock + tid, lo, i1, j1);
        tile_entry(P, T, total, base + 2 * kBlock + tid, lo, i2, j2);
        tile_entry(P, T, total, base + 3 * kBlock + tid, lo, i3, j3);
        const uint32_t m0 = mask_word(L, i0), m1 = mask_word(L, i1);
        const uint32_t m2 = mask_word(L, i2), m3 = mask_word(L, i3);
        settle4(P, L, O, i0, j0, m0, i1, j1, m1, i2, j2, m2, i3, j3, m3);
    }
    __syncthreads();   // T is reused by the next tile
}

// One chunk of a long frontier column: every lane of the block takes entries
// of the chunk in turn.  Chunk 0 of a column also moves the column into B_{k+1}
// (unless the level copies B_k word by word).
__device__ __forceinline__ void expand_chunk(const LevelParams &P, const LevelPtrs &L, OutLds &O, uint32_t c,
                             uint32_t nlong, bool carry) {
    __shared__ HeavyItem s_it;
    (void)nlong;
    if (threadIdx.x == 0) s_it = L.h_cur[L.c_cur[c]];
    __syncthreads();
    const HeavyItem it = s_it;
    __syncthreads();
    const int32_t j = it.v;
    const uint32_t part = c - it.chunk_base;
    if (carry && part == 0 && threadIdx.x == 0) {
        atomicOr(&L.vb_nxt[(uint32_t)j >> 5], 1u << (j & 31));
    }
    const int32_t r1 = P.out_ptr[j + 1];
    const int32_t e0 = P.out_ptr[j] + (int32_t)(part * P.chunk);
    const int32_t e1 = (r1 - e0 > (int32_t)P.chunk) ? e0 + (int32_t)P.chunk : r1;
    for (int32_t eb = e0; eb < e1; eb += kBlock * kIlp) {
        const int32_t e = eb + (int32_t)threadIdx.x;
        const int32_t i0 = (e < e1) ? P.out_idx[e] : -1;
        const int32_t i1 = (e + kBlock < e1) ? P.out_idx[e + kBlock] : -1;
        const int32_t i2 = (e + 2 * kBlock < e1) ? P.out_idx[e + 2 * kBlock] : -1;
        const int32_t i3 = (e + 3 * kBlock < e1) ? P.out_idx[e + 3 * kBlock] : -1;
        const uint32_t m0 = mask_word(L, i0), m1 = mask_word(L, i1);
        const uint32_t m2 = mask_word(L, i2), m3 = mask_word(L, i3);
        settle4(P, L, O, i0, j, m0, i1, j, m1, i2, j, m2, i3, j, m3);
    }
}

// ---------------------------------------------------------------------------
// the three forms of one level
// ---------------------------------------------------------------------------

// B_{k+1} must contain B_k.  For a large frontier it is cheaper to OR B_k into
// the other buffer word by word (words / 32 of the vertex count) than to set
// one bit per frontier vertex with an atomic.
__device__ __forceinline__ bool word_carry(const LevelParams &P, uint32_t nf) {
    return nf > P.words;
}

__device__ __forceinline__ void carry_words(const LevelParams &P, const LevelPtrs &L, uint32_t bid,
                            uint32_t nblocks) {
    for (uint32_t w = bid * kBlock + threadIdx.x; w < P.words; w += nblocks * kBlock) {
        const uint32_t b = L.vb_cur[w];
        if (b) atomicOr(&L.vb_nxt[w], b);
    }
}

// Push: work items are the tiles of the short-column list followed by the
// chunks of the long columns, dealt round-robin to the blocks.
__device__ __forceinline__ void push_level(const LevelParams &P, const LevelPtrs &L, TileLds &T, OutLds &O,
                           uint32_t nreg, uint32_t nlong, uint32_t nchunks, uint32_t bid,
                           uint32_t nblocks) {
    const bool wc = word_carry(P, nreg + nlong);
    if (wc) carry_words(P, L, bid, nblocks);
    const uint32_t ntiles = (nreg + kBlock - 1) / kBlock;
    const uint32_t items = ntiles + nchunks;
    for (uint32_t it = bid; it < items; it += nblocks) {
        if (it < ntiles) {
            const uint32_t pos = it * kBlock + threadIdx.x;
            int32_t j = -1, r0 = 0;
            uint32_t deg = 0;
            if (pos < nreg) {
                const QEnt e = L.q_cur[pos];
                j = e.v;
                r0 = e.r0;
                deg = (uint32_t)(e.r1 - e.r0);
                if (!wc) atomicOr(&L.vb_nxt[(uint32_t)j >> 5], 1u << (j & 31));   // F_k joins B_{k+1}
            }
            expand_tile(P, L, T, O, j, r0, deg);
        } else {
            expand_chunk(P, L, O, it - ntiles, nlong, !wc);
        }
    }
}

// Push with the frontier read from the bitmap: items are 256-word groups of
// the frontier bitmap (one frontier column per thread per round, lowest bit
// first) followed by the chunks of the long columns.
__device__ __forceinline__ void bitmap_level(const LevelParams &P, const LevelPtrs &L, TileLds &T, OutLds &O,
                             uint32_t nlong, uint32_t nchunks, uint32_t bid, uint32_t nblocks) {
    const uint32_t ngroups = (P.words + kBlock - 1) / kBlock;
    const uint32_t items = ngroups + nchunks;
    for (uint32_t it = bid; it < items; it += nblocks) {
        if (it >= ngroups) {
            expand_chunk(P, L, O, it - ngroups, nlong, false);
            continue;
        }
        const uint32_t w = it * kBlock + threadIdx.x;
        uint32_t bits = (w < P.words) ? L.fb_cur[w] : 0u;
        if (bits) atomicOr(&L.vb_nxt[w], bits);         // F_k joins B_{k+1}
        while (__syncthreads_or(bits != 0u)) {
            int32_t j = -1, r0 = 0;
            uint32_t deg = 0;
            if (bits) {
                const uint32_t b = (uint32_t)__ffs((int)bits) - 1u;
                bits &= bits - 1u;
                j = (int32_t)(w * 32u + b);
                r0 = P.out_ptr[j];
                deg = (uint32_t)(P.out_ptr[j + 1] - r0);
                if (deg >= P.heavy_min) {             // a long column: done by its chunks
                    j = -1;
                    deg = 0;
                }
            }
            expand_tile(P, L, T, O, j, r0, deg);
        }
    }
}

constexpr uint32_t kPullSerial = 4;      // in-neighbours a lane scans before handing off

// w in F_k: the frontier bitmap when it is kept (L2-resident), else level[w] = k
__device__ __forceinline__ bool in_frontier(const LevelParams &P, const LevelPtrs &L, int32_t w,
                                            int32_t lk) {
    if (P.maintain_fb) return (L.fb_cur[(uint32_t)w >> 5] >> (w & 31)) & 1u;
    return P.level[w] == lk;
}

constexpr uint32_t kPullStep = 8;        // entries per unsettled row per round afterwards
constexpr uint32_t kRoundIlp = 4;        // entries a lane tests at once in those rounds
static_assert(kPullSerial == 4, "first_hit4 covers the serial window");

// The first in-neighbour, in ascending order, among in_idx[e0, e0 + cnt)
// (1 <= cnt <= 4) that is in F_k, else -1.  The window's index loads are all
// issued before the first frontier test, and the tests before the first use,
// so a row costs two memory latencies instead of up to eight; positions past
// cnt repeat the last entry, which cannot change the first hit.
__device__ __forceinline__ int32_t first_hit4(const LevelParams &P, const LevelPtrs &L, int32_t e0,
                                              int32_t cnt, int32_t lk) {
    const int32_t last = e0 + cnt - 1;
    const int32_t w0 = P.in_idx[e0];
    const int32_t w1 = P.in_idx[e0 + 1 < last ? e0 + 1 : last];
    const int32_t w2 = P.in_idx[e0 + 2 < last ? e0 + 2 : last];
    const int32_t w3 = P.in_idx[last < e0 + 3 ? last : e0 + 3];
    const bool h0 = in_frontier(P, L, w0, lk), h1 = in_frontier(P, L, w1, lk);
    const bool h2 = in_frontier(P, L, w2, lk), h3 = in_frontier(P, L, w3, lk);
    return h0 ? w0 : (h1 ? w1 : (h2 ? w2 : (h3 ? w3 : -1)));
}

struct PullLds {
    int32_t lng[kBlock];                  // rows not settled by their first kPullSerial entries
    int32_t cur[kBlock], end[kBlock];     // their next entry and one past the last
    int32_t hit[kBlock];                  // smallest frontier in-neighbour found this round
    uint32_t pre[kBlock + 1];
    uint32_t wsum[kBlock / 64];
    uint32_t nlong, nnext;
};

// Row-wise form over the unvisited list U (or all vertices the first time):
// for u not visited through level k, scan its in-neighbours in ascending order
// and stop at the first w with level[w] = k - the smallest frontier
// in-neighbour, i.e. the same min-parent the push form produces.  Rows with
// long in-lists that are not settled by their first kPullSerial entries are
// finished one wave per row (64 entries per step, ballot for the first hit).
// A row with no in-neighbour can never be reached and leaves the list.
__device__ __forceinline__ void pull_level(const LevelParams &P, LevelPtrs &L, PullLds &S, OutLds &O,
                           uint32_t nreg, uint32_t nlong, uint32_t bid, uint32_t nblocks) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    // F_k joins B_{k+1}; its frontier bits are cleared
    const bool wc = word_carry(P, nreg + nlong);
    if (wc) carry_words(P, L, bid, nblocks);
    if (!wc) {
        for (uint32_t pos = bid * kBlock + tid; pos < nreg + nlong; pos += nblocks * kBlock) {
            const int32_t j = (pos < nreg) ? L.q_cur[pos].v : L.h_cur[pos - nreg].v;
            atomicOr(&L.vb_nxt[(uint32_t)j >> 5], 1u << (j & 31));
        }
    }
    const uint32_t ub = P.st->u_buf;
    const uint32_t ulen = P.st->u_len;
    const bool all = (ulen == kAllVertices);
    const uint32_t len = all ? (uint32_t)P.n : ulen;
    const int32_t *U = ub ? P.ul[1] : P.ul[0];
    L.u_nxt = ub ? P.ul[0] : P.ul[1];
    const int32_t lk = (int32_t)L.k;
    const bool undirected = (P.in_ptr == P.out_ptr);
    for (uint32_t tile = bid; tile * kBlock < len; tile += nblocks) {
        if (tid == 0) S.nlong = 0;
        __syncthreads();
        const uint32_t pos = tile * kBlock + tid;
        int32_t u = -1, found = -1, ue0 = 0, ue1 = 0;
        bool keep = false;
        if (pos < len) {
            u = all ? (int32_t)pos : U[pos];
            // the mask word and the row bounds are loaded together
            const uint32_t mw = L.vb_cur[(uint32_t)u >> 5];
            const int32_t e0 = P.in_ptr[u], e1 = P.in_ptr[u + 1];
            if (!((mw >> (u & 31)) & 1u)) {
                ue0 = e0;
                ue1 = e1;
                const int32_t lim = (e1 - e0 > (int32_t)kPullSerial) ? e0 + (int32_t)kPullSerial : e1;
                if (lim > e0) found = first_hit4(P, L, e0, lim - e0, lk);
                if (found < 0) {
                    if (lim < e1) {
                        const uint32_t slot = atomicAdd(&S.nlong, 1u);
                        S.lng[slot] = u;
                    } else {
                        keep = e1 > e0;
                    }
                }
            }
        }
        const bool owner = found >= 0;
        if (owner) {
            P.parent[u] = (uint32_t)found;
            P.level[u] = lk + 1;
        }
        if (undirected) append_next(P, L, O, owner, u, true, ue0, ue1);
        else append_next(P, L, O, owner, u, true);
        {   // survivors stay on the unvisited list
            const unsigned long long m = __ballot(keep);
            if (m) {
                const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&O.un, (uint32_t)__popcll(m));
                base = __shfl(base, (int)leader, 64);
                if (keep) O.u[base + lanes_below(m)] = u;
            }
        }
        out_flush(P, L, O, false);
        // Rows still open after their first entries: all of them advance
        // together, kPullStep entries per row per round, the entries of the
        // round laid out on one line (prefix scan) and shared by every lane;
        // the smallest frontier in-neighbour of a row in the first window that
        // has one is its first in ascending order, i.e. the min-parent.
        uint32_t nl = S.nlong;
        if (tid < nl) {
            const int32_t v = S.lng[tid];
            S.cur[tid] = P.in_ptr[v] + (int32_t)kPullSerial;
            S.end[tid] = P.in_ptr[v + 1];
        }
        __syncthreads();
        while (nl > 0) {                               // uniform: nl is read from LDS by all
            uint32_t cnt = 0;
            if (tid < nl) {
                const int32_t r = S.end[tid] - S.cur[tid];
                cnt = r < (int32_t)kPullStep ? (uint32_t)r : kPullStep;
                S.hit[tid] = 0x7fffffff;
            }
            const uint32_t incl = wave_incl_scan(cnt);
            if (lane == 63) S.wsum[wave] = incl;
            __syncthreads();
            uint32_t woff = 0, total = 0;
            for (uint32_t w = 0; w < kBlock / 64; ++w) {
                woff += (w < wave) ? S.wsum[w] : 0u;
                total += S.wsum[w];
            }
            S.pre[tid] = woff + incl - cnt;
            __syncthreads();
            // up to kRoundIlp entries per lane per pass, all loads issued first
            uint32_t lo = 0;
            for (uint32_t e = tid; e < total; e += kRoundIlp * kBlock) {
                uint32_t slot[kRoundIlp];
                int32_t w[kRoundIlp];
#pragma unroll
                for (uint32_t t = 0; t < kRoundIlp; ++t) {
                    const uint32_t et = e + t * kBlock;
                    const uint32_t ec = et < total ? et : total - 1u;   // in range, ignored below
                    uint32_t hi = nl - 1;              // last row slot with pre <= ec
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi + 1) >> 1;
                        if (S.pre[mid] <= ec) lo = mid; else hi = mid - 1;
                    }
                    slot[t] = lo;
                    w[t] = P.in_idx[S.cur[lo] + (int32_t)(ec - S.pre[lo])];
                }
                bool h[kRoundIlp];
#pragma unroll
                for (uint32_t t = 0; t < kRoundIlp; ++t) h[t] = in_frontier(P, L, w[t], lk);
#pragma unroll
                for (uint32_t t = 0; t < kRoundIlp; ++t)
                    if (h[t] && e + t * kBlock < total) atomicMin(&S.hit[slot[t]], w[t]);
            }
            if (tid == 0) S.nnext = 0;
            __syncthreads();
            // settle rows with a hit; rows with entries left go round again
            bool own = false, keep = false, again = false;
            int32_t v = -1, h = -1, ncur = 0, nend = 0;
            if (tid < nl) {
                v = S.lng[tid];
                h = S.hit[tid];
                ncur = S.cur[tid] + (int32_t)cnt;
                nend = S.end[tid];
                if (h != 0x7fffffff) {
                    own = true;
                    P.parent[v] = (uint32_t)h;
                    P.level[v] = lk + 1;
                } else if (ncur < nend) {
                    again = true;
                } else {
                    keep = true;
                }
            }
            __syncthreads();                           // rows are read: compact in place
            if (again) {
                const uint32_t slot = atomicAdd(&S.nnext, 1u);
                S.lng[slot] = v;
                S.cur[slot] = ncur;
                S.end[slot] = nend;
            }
            append_next(P, L, O, own, v, true);
            {
                const unsigned long long m = __ballot(keep);
                if (m) {
                    const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
                    uint32_t base = 0;
                    if (lane == leader) base = atomicAdd(&O.un, (uint32_t)__popcll(m));
                    base = __shfl(base, (int)leader, 64);
                    if (keep) O.u[base + lanes_below(m)] = v;
                }
            }
            out_flush(P, L, O, false);                 // (has a barrier: nnext is final)
            nl = S.nnext;
            __syncthreads();
        }
        __syncthreads();
    }
}

// The counters of level k + 1 as the close of level k leaves them.
struct Closed {
    LevelStats s;
    uint32_t nf;              // |F_{k+1}| (list entries plus long columns)
};

// End of level k, one thread: fold the level's counters into the state,
// advance, and return the next level's counters.  Only called when F_k was
// nonempty, so launches after the end of the search change nothing.
__device__ __forceinline__ Closed finish_level(const LevelParams &P, uint32_t k, uint32_t nf) {
    BfsState *st = P.st;
    const uint32_t cs = k & 3, ns = (k + 1) & 3;
    const uint32_t nf_next = ld_agent(&st->nf[ns]) + (uint32_t)ld_agent64(&st->heavy[ns]);
    const unsigned long long sdf_next = ld_agent64(&st->sdf[ns]);
    const uint32_t variant = level_form(P, ld_agent(&st->variant));
    const uint32_t vc = ld_agent(&st->visited_cnt);
    const unsigned long long vd = ld_agent64(&st->visited_deg);
    if (P.trace) {
        DevLevelRec r;
        r.level = k;
        r.variant = variant;
        r.nf = nf;
        r.nu = (uint32_t)P.n - vc;
        r.sdf = ld_agent64(&st->sdf[cs]);
        r.sdu = (unsigned long long)P.nnz - vd;
        P.trace[k % kTraceCap] = r;
    }
    st->visited_cnt = vc + nf_next;
    st->visited_deg = vd + sdf_next;
    if (variant == kPull) {
        st->u_buf ^= 1u;
        st->u_len = ld_agent(&st->u_wr);
    }
    st->u_wr = 0;
    st->level = k + 1;        // published by the launch's end, or the barrier's release
    Closed c;
    c.nf = nf_next;
    c.s.nf = (float)nf_next;
    c.s.sdf = (float)sdf_next;
    c.s.nu = (float)((uint32_t)P.n - (vc + nf_next));
    c.s.sdu = (float)((unsigned long long)P.nnz - (vd + sdf_next));
    return c;
}

__device__ __forceinline__ uint32_t frontier_size(const BfsState *st, uint32_t slot) {
    return st->nf[slot] + (uint32_t)st->heavy[slot];
}

// The level kernels' LDS: one level's tiles, or, once the level is done, the
// network's weights for the next level's decision.
union LevelLds {
    TileLds t;                                // push / push-bitmap
    PullLds p;                                // pull
    float w[kMlpTotal];                       // decision of the next level's form
};

__device__ __forceinline__ void level_body(const LevelParams &P, uint32_t k, uint32_t bid, uint32_t nblocks,
                                           LevelLds &lds) {
    TileLds &tl = lds.t;
    PullLds &pl = lds.p;
    __shared__ OutLds ol;
    const BfsState *st = P.st;
    LevelPtrs L = level_ptrs(P, k);
    // short-circuit claims on the levels whose frontier columns hold at least
    // n / 8 entries (there atomics bound the level, and the rows they reach
    // find their parent one level up quickly); the min-select elsewhere
    L.sc = (P.policy == kShortCircuit) && st->sdf[L.cs] * 8ull >= (unsigned long long)P.n;
    const uint32_t nreg = st->nf[L.cs];
    const unsigned long long hp = st->heavy[L.cs];
    const uint32_t nlong = (uint32_t)hp, nchunks = (uint32_t)(hp >> 32);
    // small level: fewer than 8192 short columns and under 2^20 entries in long ones
    L.pre = !(nreg < 8192u && (unsigned long long)nchunks * P.chunk < (1ull << 20));
    const uint32_t v = level_form(P, st->variant);     // decided before the launch
    if (bid == 0 && threadIdx.x == 0) {
        BfsState *w = P.st;
        const uint32_t fs = (k + 2) & 3;     // slot of level k+2: free since level k-2
        w->nf[fs] = 0;
        w->heavy[fs] = 0ull;
        w->sdf[fs] = 0ull;
    }
    out_init(ol);
    if (P.maintain_fb) {          // fb[(k+2)%3] held F_{k-1}: nobody reads or writes it now
        for (uint32_t w = bid * kBlock + threadIdx.x; w < P.words; w += nblocks * kBlock)
            L.fb_old[w] = 0u;
    }
    if (v == kPull) pull_level(P, L, pl, ol, nreg, nlong, bid, nblocks);
    else if (v == kBitmap) bitmap_level(P, L, tl, ol, nlong, nchunks, bid, nblocks);
    else push_level(P, L, tl, ol, nreg, nlong, nchunks, bid, nblocks);
    out_flush(P, L, ol, true);
}

}  // namespace

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Initialise outputs and state for a search from one root (single_root >= 0)
// or from a list of roots (multi-root, completed by k_init_roots).
__global__ __launch_bounds__(kBlock) void k_init(LevelParams P, int32_t single_root) {
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
            P.fb[2][w] = 0u;
        }
    }
    if (gid == 0) {
        BfsState *st = P.st;
        st->level = 0;
        st->variant = 0;
        st->u_buf = 0;
        st->u_len = kAllVertices;
        st->u_wr = 0;
        st->barrier_gen = 0;
        for (int g = 0; g < kBarGroups; ++g) st->bar_group[g * 16] = 0;
        st->bar_top = 0;
        st->visited_cnt = 0;
        st->visited_deg = 0ull;
        st->atomics = 0ull;
        for (int r = 0; r < kRing; ++r) {
            st->nf[r] = 0;
            st->heavy[r] = 0ull;
            st->sdf[r] = 0ull;
        }
        if (single_root >= 0) {
            const int32_t r0 = P.out_ptr[single_root], r1 = P.out_ptr[single_root + 1];
            const uint32_t deg = (uint32_t)(r1 - r0);
            if (deg >= P.heavy_min) {
                HeavyItem it;
                it.v = single_root;
                it.chunk_base = 0;
                P.hl[0][0] = it;
                const uint32_t nch = (deg + P.chunk - 1u) / P.chunk;
                for (uint32_t c = 0; c < nch; ++c) P.cmap[0][c] = 0;
                st->heavy[0] = 1ull | ((unsigned long long)nch << 32);
            } else {
                QEnt e;
                e.v = single_root;
                e.r0 = r0;
                e.r1 = r1;
                e.pad = 0;
                P.q[0][0] = e;
                st->nf[0] = 1;
            }
            st->sdf[0] = deg;
            st->visited_cnt = 1;
            st->visited_deg = deg;
        }
    }
}

// second init pass for multi-root searches (after k_init has cleared everything):
// the roots are appended to the level-0 frontier exactly as a level appends
__global__ __launch_bounds__(kBlock) void k_init_roots(LevelParams P, int32_t nroots,
                                                       const int32_t *roots) {
    __shared__ OutLds ol;
    LevelPtrs L = level_ptrs(P, 0u);
    L.vb_nxt = P.vb[0];
    L.fb_nxt = P.fb[0];
    L.q_nxt = P.q[0];
    L.h_nxt = P.hl[0];
    L.c_nxt = P.cmap[0];
    L.ns = 0;
    out_init(ol);
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    bool own = false;
    int32_t r = -1;
    if (gid < (uint32_t)nroots) {
        r = roots[gid];
        P.level[r] = 0;
        P.parent[r] = (uint32_t)r;
        own = true;
    }
    append_next(P, L, ol, own, r);
    unsigned long long d = 0;
    if (own) d = (unsigned long long)(P.out_ptr[r + 1] - P.out_ptr[r]);
    d = wave_sum64(d);
    const unsigned long long c = wave_sum64(own ? 1ull : 0ull);
    if (lane_id() == 0 && c) {
        atomicAdd(&P.st->visited_deg, d);
        atomicAdd(&P.st->visited_cnt, (uint32_t)c);
        if (!P.stats) atomicAdd(&P.st->sdf[0], d);
    }
    out_flush(P, L, ol, true);
}

// s_waitcnt immediate (gfx9 encoding) that waits for vmcnt = 0 only:
// vmcnt bits [3:0] and [15:14] zero, expcnt [6:4] = 7 and lgkmcnt [11:8] = 15
// (no wait on those).
constexpr int kWaitVmcnt0 = 0x0F70;

// The block that arrives last at the end of a level launch.  Blocks arrive
// on one of kBarGroups counters (block b on b % kBarGroups, each counter on its
// own line), the last of each group on the top counter; the block completing
// the top counter has seen every block of the launch finish its part of the
// level.  Nobody waits, and every counter is back at zero afterwards.
// What the closing block reads are counters that the level's blocks changed
// with atomics, so an arrival only has to come after its block's atomics have
// been performed: every wave drains its outstanding memory operations
// (s_waitcnt vmcnt(0)) before the block barrier, and no cache fence is needed
// on the way in (a device-scope fence per block would write back and
// invalidate the L2 under every other block still running).  The level's
// other writes reach the next level at the launch boundary.
__device__ __forceinline__ bool last_to_arrive(BfsState *st, uint32_t nblocks) {
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

// Progress for the host: the level the search stands at and its frontier
// size (0 once the search is over).
__device__ __forceinline__ void report_status(const LevelParams &P, uint32_t level, uint32_t nf) {
    P.host_status[0] = level;
    P.host_status[1] = nf;
}

// Close level k (every block of the level is done): fold the counters, decide
// the next level's form, report.  Called by every thread of one block; s_w is
// that block's LDS (kMlpTotal floats), free by now.  Everything it reads that
// other blocks changed during the level it reads with coherent loads; the
// persistent kernel also acquires (`acquire`) the state that an earlier
// level's close wrote in the same launch.
__device__ __forceinline__ void close_level(const LevelParams &P, uint32_t k, uint32_t nf, float *s_w,
                                            bool acquire) {
    __shared__ Closed s_c;
    if (threadIdx.x == 0) {
        if (acquire) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_c = finish_level(P, k, nf);
    }
    __syncthreads();
    const Closed c = s_c;
    if (c.nf != 0 && (P.policy == kLearned || P.policy == kHeuristic)) decide_level(P, k + 1, c.s, s_w);
    if (threadIdx.x == 0) report_status(P, k + 1, c.nf);
}

// One level: the level body on every block, then the last block to finish
// closes the level, so a level is one launch.  Launches after the end of the
// search (empty frontier) return at once.
__global__ __launch_bounds__(kBlock, 8) void k_level(LevelParams P) {
    __shared__ LevelLds lds;
    BfsState *st = P.st;
    const uint32_t k = st->level;
    const uint32_t nf = frontier_size(st, k & 3);
    if (nf == 0) return;
    level_body(P, k, blockIdx.x, gridDim.x, lds);
    if (last_to_arrive(st, gridDim.x)) close_level(P, k, nf, lds.w, false);
}

// The form of level 0 (after the init kernels).
__global__ void k_decide(LevelParams P) {
    __shared__ LevelStats s_ls;
    __shared__ float s_w[kMlpTotal];
    if (threadIdx.x == 0) s_ls = level_stats(P, 0);
    __syncthreads();
    const LevelStats L = s_ls;
    decide_level(P, 0, L, s_w);
}

// Grid barrier for the cooperative kernel, with the level's closing work done
// inside it.  Blocks arrive on one of kBarGroups counters (block b on group
// b % kBarGroups, each counter on its own line); the last arrival of a group
// arrives on the top counter.  The block of the very last arrival closes level
// k (finish_level, then the next level's form) and bumps the top generation;
// the other groups' last arrivals wait for that and each then releases its
// group by bumping the group's own generation, which the rest of the group
// watches.  Arrivals serialise on kBarGroups + nblocks / kBarGroups atomics
// instead of nblocks, and at most nblocks / kBarGroups blocks poll any one
// line.  Arrivals and releases are release fences (L2 write-back only) and the
// way out is an acquire fence (invalidate only): a full fence at arrival would
// also invalidate the L2 under the blocks still working on the level.  Returns false only if a spin limit runs out, which cannot happen when
// every block is resident.
__device__ __forceinline__ bool level_barrier(const LevelParams &P, uint32_t k, uint32_t nf, uint32_t nblocks,
                              uint32_t *s_role, float *s_w) {
    BfsState *st = P.st;
    const uint32_t groups = nblocks < (uint32_t)kBarGroups ? nblocks : (uint32_t)kBarGroups;
    const uint32_t g = blockIdx.x % groups;
    const uint32_t in_group = (nblocks - g + groups - 1) / groups;
    uint32_t *ggen = &st->bar_gen_group[g * 16];
    uint32_t gen = 0, tgen = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t role = 0;                                   // 0 member, 1 group's last, 2 very last
        gen = ld_agent(ggen);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this block's part of level k
        if (atomicAdd(&st->bar_group[g * 16], 1u) == in_group - 1) {
            __hip_atomic_store(&st->bar_group[g * 16], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tgen = ld_agent(&st->barrier_gen);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            role = 1;
            if (atomicAdd(&st->bar_top, 1u) == groups - 1) {
                __hip_atomic_store(&st->bar_top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                role = 2;
            }
        }
        *s_role = role;
    }
    __syncthreads();
    const uint32_t role = *s_role;
    if (role == 2) close_level(P, k, nf, s_w, true);               // every block is done with level k
    __syncthreads();
    uint32_t ok = 1;
    if (threadIdx.x == 0) {
        if (role == 2) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the level's close
            atomicAdd(&st->barrier_gen, 1u);
        } else if (role == 1) {
            uint32_t spins = 0;
            while (ld_agent(&st->barrier_gen) == tgen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1u << 26)) { ok = 0; break; }
            }
        }
        if (role != 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(ggen, 1u);                             // release this group
        } else {
            uint32_t spins = 0;
            while (ld_agent(ggen) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 26)) { ok = 0; break; }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see every block's level k
        *s_role = ok;
    }
    __syncthreads();
    return *s_role != 0;
}

// Every level in one launch: level body, then the level barrier (whose last
// arrival closes the level).  The loop ends when the frontier is empty (every
// block reads the same counters after a barrier).
__global__ __launch_bounds__(kBlock) void k_persistent(LevelParams P) {
    __shared__ uint32_t s_role;
    __shared__ LevelLds lds;
    BfsState *st = P.st;
    const uint32_t nb = gridDim.x;
    for (;;) {
        const uint32_t k = ld_agent(&st->level);
        const uint32_t nf = ld_agent(&st->nf[k & 3]) + (uint32_t)ld_agent64(&st->heavy[k & 3]);
        if (nf == 0) break;
        level_body(P, k, blockIdx.x, nb, lds);
        if (!level_barrier(P, k, nf, nb, &s_role, lds.w)) break;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t k = ld_agent(&st->level);
        report_status(P, k, ld_agent(&st->nf[k & 3]) + (uint32_t)ld_agent64(&st->heavy[k & 3]));
    }
}

// After a short-circuit search: every reached vertex v whose parent is still
// empty (claimed on a short-circuit level) gets its smallest in-neighbour one
// level up - the first, in ascending order, with level[u] = level[v] - 1 (one
// exists: the column that claimed v).  A lane scans the first kParentSerial
// entries (four loads in flight at a time, positions past the end repeating
// the last entry); rows not settled by then go to a wave, 64 entries a step,
// the lowest lane with a hit giving the first.
constexpr int32_t kParentSerial = 16;

__global__ __launch_bounds__(kBlock) void k_parents(LevelParams P) {
    __shared__ int32_t s_v[kBlock];
    __shared__ uint32_t s_n;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    for (uint32_t base = blockIdx.x * kBlock; base < (uint32_t)P.n; base += gridDim.x * kBlock) {
        if (tid == 0) s_n = 0;
        __syncthreads();
        const uint32_t v = base + tid;
        if (v < (uint32_t)P.n) {
            const int32_t lv = P.level[v];
            if (lv > 0 && P.parent[v] == 0xFFFFFFFFu) {
                const int32_t e0 = P.in_ptr[v], e1 = P.in_ptr[v + 1];
                const int32_t lim = (e1 - e0 > kParentSerial) ? e0 + kParentSerial : e1;
                int32_t found = -1;
                for (int32_t e = e0; e < lim && found < 0; e += 4) {
                    const int32_t last = lim - 1;
                    int32_t u[4], l[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) u[t] = P.in_idx[e + t < last ? e + t : last];
#pragma unroll
                    for (int t = 0; t < 4; ++t) l[t] = P.level[u[t]];
#pragma unroll
                    for (int t = 3; t >= 0; --t)
                        if (l[t] == lv - 1) found = u[t];    // the lowest position wins
                }
                if (found >= 0) P.parent[v] = (uint32_t)found;
                else s_v[atomicAdd(&s_n, 1u)] = (int32_t)v;
            }
        }
        __syncthreads();
        const uint32_t nl = s_n;
        for (uint32_t i = wave; i < nl; i += kBlock / 64) {
            const int32_t w = s_v[i];
            const int32_t lv = P.level[w];
            const int32_t e1 = P.in_ptr[w + 1];
            for (int32_t eb = P.in_ptr[w] + kParentSerial; eb < e1; eb += 64) {   // uniform
                const int32_t e = eb + (int32_t)lane;
                int32_t u = -1;
                bool hit = false;
                if (e < e1) {
                    u = P.in_idx[e];
                    hit = P.level[u] == lv - 1;
                }
                const unsigned long long m = __ballot(hit);
                if (m) {
                    const int first = (int)__ffsll((long long)m) - 1;
                    const int32_t uf = __shfl(u, first, 64);
                    if (lane == 0) P.parent[w] = (uint32_t)uf;
                    break;
                }
            }
        }
        __syncthreads();
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
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, p, single_root);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (single_root < 0) {
        const uint32_t g2 = ((uint32_t)nroots + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_init_roots, dim3(g2 ? g2 : 1), dim3(kBlock), 0, s, p, nroots, roots_dev);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p.policy == kLearned || p.policy == kHeuristic) {
        hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, s, p);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_level(const LevelParams &p, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_level, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_parents(const LevelParams &p, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_parents, dim3(grid), dim3(kBlock), 0, s, p);
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

// The searches the Experiments section measures the method against, built as
// that section describes them, with a device count of their algebraic
// operations (two per nonzero multiplied, Table 2's convention):
//
//  * SpMV-BFS: every nonzero of A^T is multiplied at every step.  The vector
//    is dense (the frontier's indicator, read from a bitmap), so a row's value
//    is the minimum over all of its in-neighbours that the vector holds; the
//    row form scans every entry of every row.  Rows of at most kCmpSerial
//    entries go to one lane, longer ones below kMsLong to a whole wave, and the
//    graph's split long rows to one wave per chunk (combined with atomicMin).
//  * SpMSpV-BFS: x_{k+1} = A^T x_k over the whole support of x_k, which is not
//    masked: from x_0 = e_s it is the set of vertices that a walk of exactly k
//    edges reaches from s.  Column form, every entry of every vector column.
//  * SpMmSpV-BFS: the vector is the frontier, every nonzero of its columns is
//    multiplied, and the visited test comes after the product.
//
// In the column forms the product lives in a step-keyed 64-bit value per row,
// key(k, j) = ((2^32 - 2 - k) << 32) | j: an atomicMin with step k's key
// always replaces an older step's value (and the initial all-ones), so the
// lane whose atomic replaced an older value made the row's first touch of
// the step and lists the row in the product's support; the low half ends as
// the smallest column that reached the row.  After the product a row of the
// support that is still unvisited gets level k + 1 and that column as parent:
// a vector column with an edge to an unvisited row lies at distance exactly k,
// so it is the smallest frontier in-neighbour, and results are bit-identical
// to the method's.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_device.h"
#include "bfs_internal.h"

namespace bfsi {

namespace {

constexpr int32_t kCmpSerial = 16;     // entries a lane multiplies alone
constexpr uint32_t kCmpBuf = 256;      // per-wave staging of listed rows
constexpr uint32_t kCmpFlush = kCmpBuf - 64;
constexpr uint32_t kWaves = kBlock / 64;

__device__ __forceinline__ unsigned long long key_hi(uint32_t k) {
    return (unsigned long long)(0xFFFFFFFEu - k) << 32;
}

__device__ __forceinline__ bool in_bitmap(const uint32_t *b, int32_t v) {
    return (b[(uint32_t)v >> 5] >> (v & 31)) & 1u;
}

// Rows listed by one wave, staged in LDS and appended to a global list in
// batches (one atomicAdd on the list's counter per batch).  `n` is uniform
// across the wave.
struct WaveList {
    int32_t *buf;          // kCmpBuf entries of this wave's LDS
    uint32_t n;
};

__device__ __forceinline__ void wl_flush(WaveList &W, uint32_t *counter, int32_t *out) {
    if (W.n == 0) return;
    __builtin_amdgcn_wave_barrier();
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, W.n);
    base = __shfl(base, 0, 64);
    for (uint32_t t = lane_id(); t < W.n; t += 64) out[base + t] = W.buf[t];
    __builtin_amdgcn_wave_barrier();
    W.n = 0;
}

__device__ __forceinline__ void wl_add(WaveList &W, bool on, int32_t v, uint32_t *counter, int32_t *out) {
    const unsigned long long m = __ballot(on);
    if (m == 0ull) return;
    if (on) W.buf[W.n + lanes_below(m)] = v;
    W.n += (uint32_t)__popcll(m);
    if (W.n > kCmpFlush) wl_flush(W, counter, out);
}

// One column entry of the product: row i gets column j under step k's key.
// True for the lane whose atomic made the row's first touch of the step.
__device__ __forceinline__ bool touch(unsigned long long *y, int32_t i, int32_t j, unsigned long long hi) {
    const unsigned long long old = atomicMin(&y[i], hi | (uint32_t)j);
    return (old & 0xFFFFFFFF00000000ull) != hi;
}

}  // namespace

// Outputs and product cleared, bitmaps zeroed.
__global__ __launch_bounds__(kBlock) void k_cmp_init(CmpParams P) {
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x, stride = gridDim.x * kBlock;
    for (uint32_t v = gid; v < (uint32_t)P.n; v += stride) {
        P.level[v] = -1;
        P.parent[v] = -1;
        P.y[v] = ~0ull;
    }
    for (uint32_t w = gid; w < P.words; w += stride) {
        P.xb[0][w] = 0u;
        P.xb[1][w] = 0u;
    }
}

// x_0 = e_s (after k_cmp_init).
__global__ void k_cmp_seed(CmpParams P, int32_t s) {
    if (threadIdx.x != 0) return;
    P.level[s] = 0;
    P.parent[s] = s;
    P.list[0][0] = s;
    P.xb[0][(uint32_t)s >> 5] = 1u << (s & 31);
    CmpState *st = P.st;
    st->k = 0;
    st->nlist = 1;
    st->ntouched = 0;
    st->nnext = 0;
    st->done = 0;
    st->ops = 0ull;
}

// Column form of step k (SpMSpV-BFS, SpMmSpV-BFS): every entry of every
// column in the vector list is multiplied.  Work items are groups of 64 list
// entries (a lane per column of at most kCmpSerial entries, the wave for
// columns below kMsLong) and then the chunks of the graph's long columns,
// taken when the column is in the vector.
__global__ __launch_bounds__(kBlock) void k_cmp_push(CmpParams P) {
    __shared__ int32_t s_buf[kWaves][kCmpBuf];
    CmpState *st = P.st;
    if (st->done) return;
    const uint32_t k = st->k, cur = k & 1u;
    const uint32_t nlist = st->nlist;
    const int32_t *list = cur ? P.list[1] : P.list[0];
    const uint32_t *xb = cur ? P.xb[1] : P.xb[0];
    int32_t *T = (P.method == kCmpSpmspv) ? (cur ? P.list[0] : P.list[1]) : P.touched;
    const unsigned long long hi = key_hi(k);
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    WaveList W{s_buf[wave], 0u};
    unsigned long long ops = 0;
    const uint32_t ngroups = (nlist + 63u) / 64u;
    const uint32_t nitems = ngroups + P.nlo_chunks;
    const uint32_t nwaves = gridDim.x * kWaves;
    for (uint32_t it = blockIdx.x * kWaves + wave; it < nitems; it += nwaves) {
        if (it < ngroups) {
            const uint32_t x = it * 64u + lane;
            int32_t j = -1, r0 = 0, deg = 0;
            if (x < nlist) {
                j = list[x];
                r0 = P.out_ptr[j];
                deg = P.out_ptr[j + 1] - r0;
            }
            ops += (unsigned long long)deg;
            const int32_t dl = deg <= kCmpSerial ? deg : 0;
            const int32_t dmax = wave_max(dl);
            for (int32_t t = 0; t < dmax; ++t) {
                bool first = false;
                int32_t i = -1;
                if (t < dl) {
                    i = P.out_idx[r0 + t];
                    first = touch(P.y, i, j, hi);
                }
                wl_add(W, first, i, &st->ntouched, T);
            }
            unsigned long long mid = __ballot(deg > kCmpSerial && deg < (int32_t)kMsLong);
            while (mid) {
                const int leader = __ffsll((long long)mid) - 1;
                mid &= mid - 1ull;
                const int32_t jj = __shfl(j, leader, 64), rr = __shfl(r0, leader, 64);
                const int32_t dd = __shfl(deg, leader, 64);
                for (int32_t eb = 0; eb < dd; eb += 64) {
                    bool first = false;
                    int32_t i = -1;
                    if (eb + (int32_t)lane < dd) {
                        i = P.out_idx[rr + eb + (int32_t)lane];
                        first = touch(P.y, i, jj, hi);
                    }
                    wl_add(W, first, i, &st->ntouched, T);
                }
            }
        } else {
            const uint32_t c = it - ngroups;
            const MsLong L = P.lo[P.lomap[c]];
            const int32_t j = L.v;
            if (!in_bitmap(xb, j)) continue;                 // the same for the whole wave
            const int32_t r1 = P.out_ptr[j + 1];
            const int32_t e0 = P.out_ptr[j] + (int32_t)((c - L.chunk_base) * kMsChunk);
            const int32_t e1 = (e0 + (int32_t)kMsChunk < r1) ? e0 + (int32_t)kMsChunk : r1;
            for (int32_t eb = e0; eb < e1; eb += 64) {
                bool first = false;
                int32_t i = -1;
                if (eb + (int32_t)lane < e1) {
                    i = P.out_idx[eb + (int32_t)lane];
                    first = touch(P.y, i, j, hi);
                }
                wl_add(W, first, i, &st->ntouched, T);
            }
        }
    }
    wl_flush(W, &st->ntouched, T);
    ops = wave_sum64(ops);
    if (lane == 0 && ops) atomicAdd(&st->ops, 2ull * ops);
}

// Row form of step k (SpMV-BFS): every entry of every row is multiplied with
// the dense vector.  A row below kMsLong entries is finished here (a lane, or
// the wave for rows above kCmpSerial entries): if the vector reaches it and it
// is unvisited it is claimed at once.  Long rows are multiplied by chunks into
// the step-keyed product and claimed by k_cmp_extract.
__global__ __launch_bounds__(kBlock) void k_cmp_spmv(CmpParams P) {
    __shared__ int32_t s_buf[kWaves][kCmpBuf];       // rows reached
    __shared__ int32_t s_long[kWaves][kCmpBuf];      // long rows touched
    CmpState *st = P.st;
    if (st->done) return;
    const uint32_t k = st->k, cur = k & 1u;
    const uint32_t *xb = cur ? P.xb[1] : P.xb[0];
    uint32_t *xn = cur ? P.xb[0] : P.xb[1];
    int32_t *lnext = cur ? P.list[0] : P.list[1];
    const unsigned long long hi = key_hi(k);
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    WaveList W{s_buf[wave], 0u}, WL{s_long[wave], 0u};
    unsigned long long ops = 0;
    const uint32_t ngroups = ((uint32_t)P.n + 63u) / 64u;
    const uint32_t nitems = ngroups + P.nli_chunks;
    const uint32_t nwaves = gridDim.x * kWaves;
    for (uint32_t it = blockIdx.x * kWaves + wave; it < nitems; it += nwaves) {
        if (it < ngroups) {
            const int32_t i = (int32_t)(it * 64u + lane);
            int32_t r0 = 0, deg = 0;
            if (i < P.n) {
                r0 = P.in_ptr[i];
                deg = P.in_ptr[i + 1] - r0;
            }
            ops += (unsigned long long)deg;
            uint32_t best = 0xFFFFFFFFu;
            const int32_t dl = deg <= kCmpSerial ? deg : 0;
            for (int32_t t = 0; t < dl; ++t) {               // every entry, no early exit
                const int32_t j = P.in_idx[r0 + t];
                if (in_bitmap(xb, j) && (uint32_t)j < best) best = (uint32_t)j;
            }
            unsigned long long mid = __ballot(deg > kCmpSerial && deg < (int32_t)kMsLong);
            while (mid) {
                const int leader = __ffsll((long long)mid) - 1;
                mid &= mid - 1ull;
                const int32_t rr = __shfl(r0, leader, 64), dd = __shfl(deg, leader, 64);
                uint32_t b = 0xFFFFFFFFu;
                for (int32_t eb = (int32_t)lane; eb < dd; eb += 64) {
                    const int32_t j = P.in_idx[rr + eb];
                    if (in_bitmap(xb, j) && (uint32_t)j < b) b = (uint32_t)j;
                }
                b = wave_min(b);
                if ((int)lane == leader) best = b;
            }
            const bool reach = i < P.n && deg < (int32_t)kMsLong && best != 0xFFFFFFFFu && P.level[i] == -1;
            if (reach) {
                P.level[i] = (int32_t)(k + 1);
                P.parent[i] = (int32_t)best;
            }
            // this wave alone writes the two bitmap words of its 64 rows in this kernel
            const unsigned long long m = __ballot(reach);
            if (m && lane == 0) {
                const uint32_t w0 = it * 2u;
                if ((uint32_t)m) xn[w0] = (uint32_t)m;
                if ((uint32_t)(m >> 32) && w0 + 1u < P.words) xn[w0 + 1u] = (uint32_t)(m >> 32);
            }
            wl_add(W, reach, i, &st->nnext, lnext);
        } else {
            const uint32_t c = it - ngroups;
            const MsLong L = P.li[P.limap[c]];
            const int32_t i = L.v;
            const int32_t r1 = P.in_ptr[i + 1];
            const int32_t e0 = P.in_ptr[i] + (int32_t)((c - L.chunk_base) * kMsChunk);
            const int32_t e1 = (e0 + (int32_t)kMsChunk < r1) ? e0 + (int32_t)kMsChunk : r1;
            uint32_t b = 0xFFFFFFFFu;
            for (int32_t e = e0 + (int32_t)lane; e < e1; e += 64) {
                const int32_t j = P.in_idx[e];
                if (in_bitmap(xb, j) && (uint32_t)j < b) b = (uint32_t)j;
            }
            b = wave_min(b);
            bool first = false;
            if (lane == 0 && b != 0xFFFFFFFFu) first = touch(P.y, i, (int32_t)b, hi);
            wl_add(WL, first, i, &st->ntouched, P.touched);
        }
    }
    wl_flush(W, &st->nnext, lnext);
    wl_flush(WL, &st->ntouched, P.touched);
    ops = wave_sum64(ops);
    if (lane == 0 && ops) atomicAdd(&st->ops, 2ull * ops);
}

// After step k's product: the support's unvisited rows are claimed (level
// k + 1, parent = the product's column), the next vector's list and bitmap
// are written, and the current vector's bitmap bits are cleared.
__global__ __launch_bounds__(kBlock) void k_cmp_extract(CmpParams P) {
    __shared__ int32_t s_buf[kWaves][kCmpBuf];
    CmpState *st = P.st;
    if (st->done) return;
    const uint32_t k = st->k, cur = k & 1u, nx = cur ^ 1u;
    const bool walk = P.method == kCmpSpmspv;
    const int32_t *T = walk ? (nx ? P.list[1] : P.list[0]) : P.touched;
    const uint32_t nt = st->ntouched, nl = st->nlist;
    const int32_t *lcur = cur ? P.list[1] : P.list[0];
    int32_t *lnext = nx ? P.list[1] : P.list[0];
    uint32_t *xc = cur ? P.xb[1] : P.xb[0];
    uint32_t *xn = nx ? P.xb[1] : P.xb[0];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    WaveList W{s_buf[wave], 0u};
    uint32_t reached_walk = 0;
    const uint32_t total = nt + nl;
    const uint32_t stride = gridDim.x * kBlock;
    // uniform trip count per wave so that every lane takes part in the ballots
    for (uint32_t base = blockIdx.x * kBlock + wave * 64u; base < total; base += stride) {
        const uint32_t t = base + lane;
        bool reach = false;
        int32_t i = -1;
        if (t < nt) {
            i = T[t];
            const uint32_t bit = 1u << (i & 31);
            if (walk) atomicOr(&xn[(uint32_t)i >> 5], bit);            // W_{k+1}
            if (P.level[i] == -1) {
                P.level[i] = (int32_t)(k + 1);
                P.parent[i] = (int32_t)(uint32_t)P.y[i];
                reach = true;
                if (!walk) atomicOr(&xn[(uint32_t)i >> 5], bit);       // F_{k+1}
            }
        } else if (t < total) {
            const int32_t v = lcur[t - nt];
            atomicAnd(&xc[(uint32_t)v >> 5], ~(1u << (v & 31)));
        }
        if (walk) reached_walk += (uint32_t)__popcll(__ballot(reach));
        else wl_add(W, reach, i, &st->nnext, lnext);
    }
    if (walk) {
        if (lane == 0 && reached_walk) atomicAdd(&st->nnext, reached_walk);
    } else {
        wl_flush(W, &st->nnext, lnext);
    }
}

// Close step k: the next vector list, progress for the host, the stop flag.
__global__ void k_cmp_advance(CmpParams P) {
    if (threadIdx.x != 0) return;
    CmpState *st = P.st;
    if (st->done) return;
    const uint32_t nnext = st->nnext;
    st->nlist = (P.method == kCmpSpmspv) ? st->ntouched : nnext;
    st->ntouched = 0;
    st->nnext = 0;
    st->k = st->k + 1;
    if (nnext == 0) st->done = 1;
    P.host_status[0] = st->k;
    P.host_status[1] = nnext;
}

CmpLayout cmp_layout(int32_t n) {
    CmpLayout L{};
    const size_t words = ((size_t)n + 31) / 32;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~(size_t)255; return o; };
    L.state = take(sizeof(CmpState));
    L.y = take((size_t)n * 8);
    L.l0 = take((size_t)n * 4);
    L.l1 = take((size_t)n * 4);
    L.touched = take((size_t)n * 4);
    L.x0 = take(words * 4);
    L.x1 = take(words * 4);
    L.total = off;
    return L;
}

hipError_t launch_cmp_init(const CmpParams &p, int32_t source, hipStream_t s) {
    uint32_t grid = ((uint32_t)p.n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_cmp_init, dim3(grid), dim3(kBlock), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cmp_seed, dim3(1), dim3(64), 0, s, p, source);
    return hipGetLastError();
}

// One step: the product, the claims, the close.  Steps launched after the
// search has ended return at once.
hipError_t launch_cmp_step(const CmpParams &p, uint32_t grid, hipStream_t s) {
    if (p.method == kCmpSpmv) hipLaunchKernelGGL(k_cmp_spmv, dim3(grid), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL(k_cmp_push, dim3(grid), dim3(kBlock), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cmp_extract, dim3(grid), dim3(kBlock), 0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cmp_advance, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace bfsi

// One masked sparse-matrix x sparse-vector product y = A^T[R, C] x over a
// chosen semiring: the operation the method is built from (Definition 1's
// submatrix A^T[V_{k+1}, V_k] is a row mask over the unvisited rows), offered
// as a primitive the way masked-algebra libraries offer it.  The semirings are
// those the Notation section names - Boolean (OR, AND), arithmetic (+, x),
// tropical (min, +) - plus (min, select), which gives the smallest column.
// A is pattern-only (entries 1); values are unsigned 64-bit, arithmetic wraps
// modulo 2^64, and min-plus adds 1 with saturation at 2^64 - 1.
//
// Passes (one stream, the host waits at the end):
//   k_sp_begin    counters to zero
//   k_sp_check    every vector index in [0, n) (else nothing else runs)
//   k_sp_product  vector entries 64 at a time: a lane per column of at most
//                 kSpSerial entries, the wave for columns below kSpLong;
//                 longer columns are listed for the chunk pass
//   k_sp_items    chunk offsets of the listed columns (one workgroup scan)
//   k_sp_long     chunks of kSpChunk entries, a wave each
//   k_sp_count / k_sp_scan / k_sp_write
//                 the support bitmap compacted in ascending order with the
//                 values, resetting the accumulator and bitmap as it goes
// Every product is an atomic on the row's accumulator (OR, add, or max of
// the complement for the min semirings, so that every identity is zero) and
// the row's support bit; products equal to the identity skip the value atomic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_device.h"
#include "bfs_internal.h"

namespace bfsi {

namespace {

constexpr int32_t kSpSerial = 16;
constexpr uint32_t kWaves = kBlock / 64;
constexpr int kScanBlock = 1024;

__device__ __forceinline__ bool allowed(const uint32_t *mask, uint32_t comp, int32_t v) {
    if (mask == nullptr) return true;
    return (((mask[(uint32_t)v >> 5] >> (v & 31)) & 1u) ^ comp) != 0u;
}

// 1 (x) v for the semiring (A's entries are 1)
__device__ __forceinline__ unsigned long long mul(uint32_t sr, unsigned long long v) {
    if (sr == kSrBoolean) return v != 0ull ? 1ull : 0ull;
    if (sr == kSrMinPlus) return v == ~0ull ? v : v + 1ull;
    return v;
}

// y(i) (+)= p, and i joins the support
__device__ __forceinline__ void accumulate(const SpParams &P, int32_t i, unsigned long long p) {
    const uint32_t bit = 1u << (i & 31);
    if ((P.touched[(uint32_t)i >> 5] & bit) == 0u) atomicOr(&P.touched[(uint32_t)i >> 5], bit);
    if (P.semiring == kSrBoolean) {
        if (p) atomicOr(&P.acc[i], 1ull);
    } else if (P.semiring == kSrArithmetic) {
        if (p) atomicAdd(&P.acc[i], p);
    } else {
        const unsigned long long c = ~p;                 // min of p == max of ~p
        if (c != 0ull && P.acc[i] < c) atomicMax(&P.acc[i], c);
    }
}

// Exclusive prefix sum over a workgroup of kScanBlock threads (LDS), and the
// total.
__device__ __forceinline__ unsigned long long block_scan(unsigned long long v, unsigned long long *s,
                                                         unsigned long long &total) {
    const uint32_t t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
        const unsigned long long o = (t >= d) ? s[t - d] : 0ull;
        __syncthreads();
        s[t] += o;
        __syncthreads();
    }
    total = s[blockDim.x - 1];
    const unsigned long long ex = s[t] - v;
    __syncthreads();
    return ex;
}

}  // namespace

__global__ void k_sp_begin(SpParams P) {
    if (threadIdx.x == 0) {
        P.st->nitems = 0;
        P.st->bad = 0;
        P.st->nchunks = 0ull;
    }
}

__global__ __launch_bounds__(kBlock) void k_sp_check(SpParams P) {
    bool bad = false;
    for (uint32_t x = blockIdx.x * kBlock + threadIdx.x; x < (uint32_t)P.nx; x += gridDim.x * kBlock) {
        const int32_t j = P.x_idx[x];
        bad = bad || j < 0 || j >= P.n;
    }
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&P.st->bad, 1u);
}

__global__ __launch_bounds__(kBlock) void k_sp_product(SpParams P) {
    if (P.st->bad) return;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t ngroups = ((uint32_t)P.nx + 63u) / 64u;
    for (uint32_t it = blockIdx.x * kWaves + wave; it < ngroups; it += gridDim.x * kWaves) {
        const uint32_t x = it * 64u + lane;
        int32_t j = -1, r0 = 0, deg = 0;
        unsigned long long p = 0ull;
        if (x < (uint32_t)P.nx) {
            j = P.x_idx[x];
            if (allowed(P.col_mask, P.col_comp, j)) {
                r0 = P.out_ptr[j];
                deg = P.out_ptr[j + 1] - r0;
                p = mul(P.semiring, P.x_val[x]);
            }
        }
        const int32_t dl = deg <= kSpSerial ? deg : 0;
        const int32_t dmax = wave_max(dl);
        for (int32_t t = 0; t < dmax; ++t) {
            if (t < dl) {
                const int32_t i = P.out_idx[r0 + t];
                if (allowed(P.row_mask, P.row_comp, i)) accumulate(P, i, p);
            }
        }
        unsigned long long mid = __ballot(deg > kSpSerial && deg < (int32_t)kSpLong);
        while (mid) {
            const int leader = __ffsll((long long)mid) - 1;
            mid &= mid - 1ull;
            const int32_t rr = __shfl(r0, leader, 64), dd = __shfl(deg, leader, 64);
            const unsigned long long pp = __shfl(p, leader, 64);
            for (int32_t e = (int32_t)lane; e < dd; e += 64) {
                const int32_t i = P.out_idx[rr + e];
                if (allowed(P.row_mask, P.row_comp, i)) accumulate(P, i, pp);
            }
        }
        if (deg >= (int32_t)kSpLong) {
            const uint32_t slot = atomicAdd(&P.st->nitems, 1u);
            SpItem it2;
            it2.j = j;
            it2.nch = ((uint32_t)deg + kSpChunk - 1u) / kSpChunk;
            it2.v = p;
            it2.base = 0ull;
            P.items[slot] = it2;
        }
    }
}

// Chunk offsets of the listed columns: one workgroup of kScanBlock threads.
__global__ __launch_bounds__(kScanBlock) void k_sp_items(SpParams P) {
    __shared__ unsigned long long s[kScanBlock];
    if (P.st->bad) return;
    const uint32_t m = P.st->nitems;
    unsigned long long run = 0ull;
    for (uint32_t b = 0; b < m; b += kScanBlock) {
        const uint32_t t = b + threadIdx.x;
        const unsigned long long c = t < m ? (unsigned long long)P.items[t].nch : 0ull;
        unsigned long long total;
        const unsigned long long ex = block_scan(c, s, total);
        if (t < m) P.items[t].base = run + ex;
        run += total;
    }
    if (threadIdx.x == 0) P.st->nchunks = run;
}

__global__ __launch_bounds__(kBlock) void k_sp_long(SpParams P) {
    if (P.st->bad) return;
    const unsigned long long nch = P.st->nchunks;
    const uint32_t m = P.st->nitems;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (unsigned long long c = (unsigned long long)blockIdx.x * kWaves + wave; c < nch;
         c += (unsigned long long)gridDim.x * kWaves) {
        uint32_t lo = 0, hi = m - 1;                      // last item with base <= c
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1u) >> 1;
            if (P.items[mid].base <= c) lo = mid; else hi = mid - 1u;
        }
        const SpItem it = P.items[lo];
        const int32_t r1 = P.out_ptr[it.j + 1];
        const int32_t e0 = P.out_ptr[it.j] + (int32_t)((c - it.base) * kSpChunk);
        const int32_t e1 = (e0 + (int32_t)kSpChunk < r1) ? e0 + (int32_t)kSpChunk : r1;
        for (int32_t e = e0 + (int32_t)lane; e < e1; e += 64) {
            const int32_t i = P.out_idx[e];
            if (allowed(P.row_mask, P.row_comp, i)) accumulate(P, i, it.v);
        }
    }
}

// Output pass 1: set bits per workgroup of kSpOutWords words.
__global__ __launch_bounds__(kSpOutWords) void k_sp_count(SpParams P) {
    __shared__ uint32_t s[kSpOutWords / 64];
    if (P.st->bad) return;
    const uint32_t w = blockIdx.x * kSpOutWords + threadIdx.x;
    uint32_t c = w < P.words ? (uint32_t)__popc(P.touched[w]) : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane_id() == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t k = 0; k < kSpOutWords / 64; ++k) t += s[k];
        P.block_off[blockIdx.x] = t;
    }
}

// Output pass 2: exclusive offsets of the workgroups (one workgroup of
// kScanBlock threads) and the output length.
__global__ __launch_bounds__(kScanBlock) void k_sp_scan(SpParams P, uint32_t nblocks) {
    __shared__ unsigned long long s[kScanBlock];
    if (P.st->bad) return;
    unsigned long long run = 0ull;
    for (uint32_t b = 0; b < nblocks; b += kScanBlock) {
        const uint32_t t = b + threadIdx.x;
        const unsigned long long c = t < nblocks ? (unsigned long long)P.block_off[t] : 0ull;
        unsigned long long total;
        const unsigned long long ex = block_scan(c, s, total);
        if (t < nblocks) P.block_off[t] = (uint32_t)(run + ex);
        run += total;
    }
    if (threadIdx.x == 0) *P.ny = (int32_t)run;
}

// Output pass 3: each word's rows in ascending order with their values; the
// accumulator entries and the words go back to zero.
__global__ __launch_bounds__(kSpOutWords) void k_sp_write(SpParams P) {
    __shared__ uint32_t s[kSpOutWords];
    if (P.st->bad) return;
    const uint32_t w = blockIdx.x * kSpOutWords + threadIdx.x;
    uint32_t bits = w < P.words ? P.touched[w] : 0u;
    const uint32_t c = (uint32_t)__popc(bits);
    s[threadIdx.x] = c;
    __syncthreads();
    for (uint32_t d = 1; d < kSpOutWords; d <<= 1) {   // inclusive scan
        const uint32_t o = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += o;
        __syncthreads();
    }
    uint32_t pos = P.block_off[blockIdx.x] + s[threadIdx.x] - c;
    const bool min_sr = P.semiring == kSrMinPlus || P.semiring == kSrMinSelect;
    while (bits) {
        const int b = __ffs(bits) - 1;
        bits &= bits - 1u;
        const int32_t i = (int32_t)(w * 32u + (uint32_t)b);
        const unsigned long long a = P.acc[i];
        P.y_idx[pos] = i;
        P.y_val[pos] = min_sr ? ~a : a;
        P.acc[i] = 0ull;
        ++pos;
    }
    if (c) P.touched[w] = 0u;
}

SpLayout sp_layout(int32_t n, int32_t max_nx) {
    SpLayout L{};
    const size_t words = ((size_t)n + 31) / 32;
    const size_t nblocks = (words + kSpOutWords - 1) / kSpOutWords;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~(size_t)255; return o; };
    L.state = take(sizeof(SpState));
    L.acc = take((size_t)n * 8);
    L.touched = take(words * 4);
    L.items = take((size_t)(max_nx > 0 ? max_nx : 1) * sizeof(SpItem));
    L.block_off = take(nblocks * 4);
    L.ny = take(4);
    L.total = off;
    return L;
}

hipError_t launch_spmspv(const SpParams &p, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_sp_begin, dim3(1), dim3(64), 0, s, p);
    uint32_t cg = ((uint32_t)p.nx + kBlock - 1) / kBlock;
    if (cg > 1024) cg = 1024;
    if (cg == 0) cg = 1;
    hipLaunchKernelGGL(k_sp_check, dim3(cg), dim3(kBlock), 0, s, p);
    hipLaunchKernelGGL(k_sp_product, dim3(grid), dim3(kBlock), 0, s, p);
    hipLaunchKernelGGL(k_sp_items, dim3(1), dim3(kScanBlock), 0, s, p);
    hipLaunchKernelGGL(k_sp_long, dim3(grid), dim3(kBlock), 0, s, p);
    const uint32_t nb = (p.words + kSpOutWords - 1) / kSpOutWords;
    hipLaunchKernelGGL(k_sp_count, dim3(nb), dim3(kSpOutWords), 0, s, p);
    hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(kScanBlock), 0, s, p, nb);
    hipLaunchKernelGGL(k_sp_write, dim3(nb), dim3(kSpOutWords), 0, s, p);
    return hipGetLastError();
}

}  // namespace bfsi

// Wave64 and memory-scope helpers shared by every gfx950 kernel file of the
// library.  Device code only; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_internal.h"

namespace bfsi {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of lanes below the calling lane whose bit is set in m.
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += t;
    }
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(v, d, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int32_t o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Loads that see other compute units' atomics (coherent across the XCDs' L2s).
__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The selector network 12 -> 32 (ReLU) -> 32 (ReLU) -> 3, row-major weights
// [out][in] followed by the biases, then the feature mean and inverse std.
// Evaluated by one wave: lane o < 32 holds hidden unit o, inputs are passed
// between lanes with shuffles (no arrays, so nothing spills).  Returns, in
// every lane, the argmin of the first `nout` predicted log-times, or -1 when
// one of them is not finite.
__device__ __forceinline__ int mlp_argmin(const float *w, float feat, int nout = kMlpOut) {
    const float *W1 = w, *b1 = W1 + kMlpIn * kMlpH, *W2 = b1 + kMlpH,
                *b2 = W2 + kMlpH * kMlpH, *W3 = b2 + kMlpH, *b3 = W3 + kMlpH * kMlpOut;
    const float *mean = w + kMlpParams, *istd = mean + kMlpIn;
    const uint32_t lane = lane_id();
    const uint32_t li = lane < (uint32_t)kMlpIn ? lane : 0u;
    const float x = (lane < (uint32_t)kMlpIn) ? (feat - mean[li]) * istd[li] : 0.f;
    const uint32_t o = lane & (kMlpH - 1);
    float a = b1[o];
    for (int i = 0; i < kMlpIn; ++i) a = fmaf(W1[o * kMlpIn + i], __shfl(x, i, 64), a);
    const float h1 = a > 0.f ? a : 0.f;
    float c = b2[o];
    for (int i = 0; i < kMlpH; ++i) c = fmaf(W2[o * kMlpH + i], __shfl(h1, i, 64), c);
    const float h2 = (c > 0.f ? c : 0.f) * (lane < (uint32_t)kMlpH ? 1.f : 0.f);
    int best = 0;
    float bestv = 0.f;
    bool ok = true;
    for (int u = 0; u < nout; ++u) {
        float y = W3[u * kMlpH + o] * h2;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d, 64);
        y += b3[u];
        if (!(y == y) || y > 1e30f || y < -1e30f) ok = false;
        if (u == 0 || y < bestv) { bestv = y; best = u; }
    }
    return ok ? best : -1;
}

}  // namespace bfsi

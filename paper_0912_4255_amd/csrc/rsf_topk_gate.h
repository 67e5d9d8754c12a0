// Candidate gate of the per-segment top-k (the k loudest 2F values over all
// templates and bins of one search, paper Sec. IV.A).  Order: 2F descending,
// ties by the lower (sky, fdot, bin) key; NaN never enters.
//
// Producers (the second FFT pass, or a scan over a 2F map) read a threshold
// t from the gate: at least k values of the search are known to be >= t, so
// a value below t cannot be among the k best.  A producer unit (a block of
// the second pass, a wave of the scan) with at most kGateFast values >= t
// appends them all; with more, it appends only its own k best and raises t
// to the k-th of them.  After each launch a merge folds the appended
// candidates into the running k best and sets t to the k-th of those.  No
// value of the k best is ever dropped, whatever the order of the units.
#pragma once

#include <math.h>

#include "rsf_params.h"

namespace rsf {

__device__ __forceinline__ bool topk_better(float va, unsigned long long ka, float vb, unsigned long long kb) {
    return va > vb || (va == vb && ka < kb);
}
// The same order on keys that share their upper part (one template row).
__device__ __forceinline__ bool topk_better(float va, unsigned ka, float vb, unsigned kb) {
    return va > vb || (va == vb && ka < kb);
}

__device__ __forceinline__ TopkItem topk_empty() {
    TopkItem e;
    e.v = -INFINITY;
    e.pad = 0;
    e.key = ~0ull;
    return e;
}

// A value enters when it is a number (not NaN, not -inf) at or above t.
__device__ __forceinline__ bool gate_pass(float x, float t) { return x > -INFINITY && x >= t; }

__device__ __forceinline__ float gate_threshold(TopkGate* g) {
    return __uint_as_float(__hip_atomic_load(&g->thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// t = max(t, v)
__device__ __forceinline__ void gate_raise(TopkGate* g, float v) {
    unsigned old = __hip_atomic_load(&g->thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (__uint_as_float(old) < v) {
        const unsigned prev = atomicCAS(&g->thr, old, __float_as_uint(v));
        if (prev == old) break;
        old = prev;
    }
}

// Wave-wide exclusive prefix sum of c (every lane active); total = the sum.
__device__ __forceinline__ int wave_prefix(int c, int lane, int& total) {
    int x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    total = __shfl(x, 63);
    return x - c;
}

// First of n slots of partition part reserved by the wave (every lane active).
__device__ __forceinline__ unsigned gate_reserve(TopkGate* g, int part, int n, int lane) {
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(&g->count[part * kGateStride], (unsigned)n);
    return (unsigned)__shfl((int)base, 0);
}

// Block-wide best of (v, key) over NT threads; every thread gets the result.
// sv, sk: NT / 64 slots of LDS.
template <int NT, typename K>
__device__ __forceinline__ void block_best(float& v, K& key, float* sv, K* sk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const K ok = __shfl_xor(key, off);
        if (topk_better(ov, ok, v, key)) {
            v = ov;
            key = ok;
        }
    }
    if (lane == 0) {
        sv[wave] = v;
        sk[wave] = key;
    }
    __syncthreads();
    v = sv[0];
    key = sk[0];
    for (int i = 1; i < NT / 64; ++i)
        if (topk_better(sv[i], sk[i], v, key)) {
            v = sv[i];
            key = sk[i];
        }
    __syncthreads();
}

}  // namespace rsf

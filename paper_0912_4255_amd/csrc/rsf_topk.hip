// Top-k selection over 2F maps (per-segment candidate lists of a batched
// search).  Order: 2F descending, ties by the lower (sky, fdot, bin) key;
// NaN never enters.  Both kernels select by k rounds of a block-wide argmax
// restricted to items strictly after the previous pick in that order, so the
// result does not depend on the launch geometry.
#include <math.h>

#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanPer = 64;                      // map values per thread
constexpr int kScanChunk = kScanThreads * kScanPer;
constexpr int kMergeThreads = 1024;

__device__ __forceinline__ bool better(float va, unsigned long long ka, float vb, unsigned long long kb) {
    return va > vb || (va == vb && ka < kb);
}

__device__ __forceinline__ TopkItem empty_item() {
    TopkItem e;
    e.v = -INFINITY;
    e.pad = 0;
    e.key = ~0ull;
    return e;
}

// block-wide best of (v, key); every thread gets the result
template <int NT>
__device__ __forceinline__ void block_best(float& v, unsigned long long& key, float* sv, unsigned long long* sk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const unsigned long long ok = __shfl_xor(key, off);
        if (better(ov, ok, v, key)) {
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
        if (better(sv[i], sk[i], v, key)) {
            v = sv[i];
            key = sk[i];
        }
    __syncthreads();
}
}  // namespace

__global__ __launch_bounds__(kScanThreads) void rsf_topk_scan_k(TopkScanArgs A) {
    __shared__ float vals[kScanChunk];
    __shared__ float sv[kScanThreads / 64];
    __shared__ unsigned long long sk[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    for (int i = threadIdx.x; i < kScanChunk; i += kScanThreads) {
        const int64_t m = base + i;
        float v = -INFINITY;
        if (m < A.n_vals) {
            v = A.map[m];
            if (v != v) v = -INFINITY;  // NaN never enters
        }
        vals[i] = v;
    }
    __syncthreads();
    float pv = INFINITY;
    unsigned long long pk = 0ull;
    bool first = true;
    for (int r = 0; r < A.k; ++r) {
        float bv = -INFINITY;
        unsigned long long bk = ~0ull;
        for (int i = threadIdx.x; i < kScanChunk; i += kScanThreads) {
            const float v = vals[i];
            if (v == -INFINITY) continue;
            const int64_t m = base + i;
            const int64_t row = m / A.n_out;
            const int64_t bin = m - row * A.n_out;
            const int64_t s_l = row / A.nf_l;
            const int64_t f = row - s_l * A.nf_l;
            const unsigned long long key =
                (unsigned long long)(((A.sky0 + s_l) * A.n_fdot + A.f0 + f) * A.n_out + bin);
            const bool after = first || better(pv, pk, v, key);
            if (after && better(v, key, bv, bk)) {
                bv = v;
                bk = key;
            }
        }
        block_best<kScanThreads>(bv, bk, sv, sk);
        if (threadIdx.x == 0) {
            TopkItem it;
            it.v = bv;
            it.pad = 0;
            it.key = bk;
            A.cand[(int64_t)blockIdx.x * A.k + r] = it;
        }
        pv = bv;
        pk = bk;
        first = false;
    }
}

__global__ __launch_bounds__(kMergeThreads) void rsf_topk_merge_k(TopkMergeArgs A) {
    __shared__ float sv[kMergeThreads / 64];
    __shared__ unsigned long long sk[kMergeThreads / 64];
    __shared__ TopkItem res[kTopkMax];
    const int64_t total = A.n_cand + (A.run_in ? A.k : 0);
    float pv = INFINITY;
    unsigned long long pk = 0ull;
    bool first = true;
    for (int r = 0; r < A.k; ++r) {
        float bv = -INFINITY;
        unsigned long long bk = ~0ull;
        for (int64_t i = threadIdx.x; i < total; i += kMergeThreads) {
            const TopkItem it = (i < A.n_cand) ? A.cand[i] : A.run_in[i - A.n_cand];
            if (it.v == -INFINITY) continue;
            const bool after = first || better(pv, pk, it.v, it.key);
            if (after && better(it.v, it.key, bv, bk)) {
                bv = it.v;
                bk = it.key;
            }
        }
        block_best<kMergeThreads>(bv, bk, sv, sk);
        if (threadIdx.x == 0) {
            res[r].v = bv;
            res[r].pad = 0;
            res[r].key = bk;
        }
        pv = bv;
        pk = bk;
        first = false;
    }
    __syncthreads();
    if (threadIdx.x < A.k) {
        const TopkItem it = res[threadIdx.x];
        A.run_out[threadIdx.x] = it;
        if (A.entries) {
            // rsf_topk_entry {float twoF; int32 sky, fdot, bin}
            float* e = (float*)A.entries + 4 * threadIdx.x;
            int* ei = (int*)e;
            e[0] = it.v;
            if (it.v == -INFINITY) {
                ei[1] = ei[2] = ei[3] = -1;
            } else {
                const unsigned long long bin = it.key % (unsigned long long)A.n_out;
                const unsigned long long tf = it.key / (unsigned long long)A.n_out;
                ei[1] = (int)(tf / (unsigned long long)A.n_fdot);
                ei[2] = (int)(tf % (unsigned long long)A.n_fdot);
                ei[3] = (int)bin;
            }
        }
    }
}

__global__ void rsf_fill_u32_k(unsigned int* p, int n, unsigned int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int topk_scan_blocks(int64_t n_vals) { return (int)((n_vals + kScanChunk - 1) / kScanChunk); }

hipError_t launch_topk_scan(const TopkScanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(rsf_topk_scan_k, dim3((unsigned)topk_scan_blocks(a.n_vals)), dim3(kScanThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_topk_merge(const TopkMergeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(rsf_topk_merge_k, dim3(1), dim3(kMergeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t s) {
    hipLaunchKernelGGL(rsf_fill_u32_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace rsf

// Top-k selection over 2F maps (per-segment candidate lists of a batched
// search).  Order: 2F descending, ties by the lower (sky, fdot, bin) key;
// NaN never enters.  Both kernels select by k rounds of a block-wide argmax
// restricted to items strictly after the previous pick in that order, so the
// result does not depend on the launch geometry.
#include <math.h>

#include <algorithm>

#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanWaveVals = 64;                 // map values per lane
constexpr int kScanChunk = 64 * kScanWaveVals;    // map values per wave
constexpr int kMergeThreads = 1024;
constexpr int kMergeItems = 4;                    // candidates per merge thread (in registers)
constexpr int kMergePer = kMergeThreads * kMergeItems;

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
template <int NT, typename K>
__device__ __forceinline__ void block_best(float& v, K& key, float* sv, K* sk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const K ok = __shfl_xor(key, off);
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

// Each wave takes a chunk of kScanWaveVals x 64 consecutive map values into
// registers (value q of lane l is chunk element 64 q + l) and selects its k
// best by k rounds of a wave-wide argmax restricted to values strictly after
// the previous pick; no LDS and no barriers.  Within one scan the map index
// m = row n_out + bin orders candidates as the (sky, fdot, bin) key does
// (rows are in template order), so the rounds rank by (2F, index in the
// chunk) and only the k winners get their key.
__global__ __launch_bounds__(kScanThreads) void rsf_topk_scan_k(TopkScanArgs A) {
    const int lane = threadIdx.x & 63;
    const int64_t chunk = (int64_t)blockIdx.x * (kScanThreads / 64) + (threadIdx.x >> 6);
    const int64_t base = chunk * kScanChunk;
    if (base >= A.n_vals) return;  // whole wave: no barrier below
    float v[kScanWaveVals];
#pragma unroll
    for (int q = 0; q < kScanWaveVals; ++q) {
        const int64_t m = base + q * 64 + lane;
        float x = (m < A.n_vals) ? A.map[m] : -INFINITY;
        if (x != x) x = -INFINITY;  // NaN never enters
        v[q] = x;
    }
    float pv = INFINITY;
    unsigned pi = 0u;
    bool first = true;
    for (int r = 0; r < A.k; ++r) {
        float bv = -INFINITY;
        unsigned bi = 0xffffffffu;
        // opaque per round: the 64 indices are recomputed instead of kept live
        unsigned ln = (unsigned)lane;
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int q = 0; q < kScanWaveVals; ++q) {
            const unsigned ii = (unsigned)(q * 64) + ln;
            const float x = v[q];
            if (x != -INFINITY && (first || better(pv, pi, x, ii)) && better(x, ii, bv, bi)) {
                bv = x;
                bi = ii;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(bv, off);
            const unsigned oi = __shfl_xor(bi, off);
            if (better(ov, oi, bv, bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            TopkItem it = empty_item();
            if (bv != -INFINITY) {
                const int64_t m = base + (int64_t)bi;
                const int64_t row = m / A.n_out;
                const int64_t bin = m - row * A.n_out;
                const int64_t s_l = row / A.nf_l;
                const int64_t f = row - s_l * A.nf_l;
                it.v = bv;
                it.key = (unsigned long long)(((A.sky0 + s_l) * A.n_fdot + A.f0 + f) * A.n_out + bin);
            }
            A.cand[chunk * A.k + r] = it;
        }
        pv = bv;
        pi = bi;
        first = false;
    }
}

// Block b ranks items [b kMergePer, (b + 1) kMergePer) of cand ++ run_in
// (each thread holds up to kMergeItems of them in registers) and writes its
// k best: to run_out (and entries) when the grid is one block, else to
// out_blocks[b k ...].
__global__ __launch_bounds__(kMergeThreads) void rsf_topk_merge_k(TopkMergeArgs A) {
    __shared__ float sv[kMergeThreads / 64];
    __shared__ unsigned long long sk[kMergeThreads / 64];
    __shared__ TopkItem res[kTopkMax];
    const int64_t total = A.n_cand + (A.run_in ? A.k : 0);
    const int64_t lo = (int64_t)blockIdx.x * kMergePer;
    TopkItem it[kMergeItems];
#pragma unroll
    for (int q = 0; q < kMergeItems; ++q) {
        const int64_t i = lo + threadIdx.x + (int64_t)q * kMergeThreads;
        it[q] = (i < total) ? ((i < A.n_cand) ? A.cand[i] : A.run_in[i - A.n_cand]) : empty_item();
    }
    float pv = INFINITY;
    unsigned long long pk = 0ull;
    bool first = true;
    for (int r = 0; r < A.k; ++r) {
        float bv = -INFINITY;
        unsigned long long bk = ~0ull;
#pragma unroll
        for (int q = 0; q < kMergeItems; ++q) {
            if (it[q].v == -INFINITY) continue;
            if ((first || better(pv, pk, it[q].v, it[q].key)) && better(it[q].v, it[q].key, bv, bk)) {
                bv = it[q].v;
                bk = it[q].key;
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
        const TopkItem r = res[threadIdx.x];
        if (gridDim.x > 1) {
            A.out_blocks[(int64_t)blockIdx.x * A.k + threadIdx.x] = r;
            return;
        }
        A.run_out[threadIdx.x] = r;
        if (A.entries) {
            // rsf_topk_entry {float twoF; int32 sky, fdot, bin}
            float* e = (float*)A.entries + 4 * threadIdx.x;
            int* ei = (int*)e;
            e[0] = r.v;
            if (r.v == -INFINITY) {
                ei[1] = ei[2] = ei[3] = -1;
            } else {
                const unsigned long long bin = r.key % (unsigned long long)A.n_out;
                const unsigned long long tf = r.key / (unsigned long long)A.n_out;
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

int64_t topk_scan_chunks(int64_t n_vals) { return (n_vals + kScanChunk - 1) / kScanChunk; }

static int topk_scan_blocks(int64_t n_vals) {
    const int waves = kScanThreads / 64;
    return (int)((topk_scan_chunks(n_vals) + waves - 1) / waves);
}

hipError_t launch_topk_scan(const TopkScanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(rsf_topk_scan_k, dim3((unsigned)topk_scan_blocks(a.n_vals)), dim3(kScanThreads), 0, s, a);
    return hipGetLastError();
}

int topk_merge_per_block() { return kMergePer; }

hipError_t launch_topk_merge(const TopkMergeArgs& a, hipStream_t s) {
    const int64_t total = a.n_cand + (a.run_in ? a.k : 0);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, (total + kMergePer - 1) / kMergePer);
    if (blocks > 1 && !a.out_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rsf_topk_merge_k, dim3(blocks), dim3(kMergeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t s) {
    hipLaunchKernelGGL(rsf_fill_u32_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace rsf

// Top-k selection over 2F maps (per-segment candidate lists of a batched
// search) and the merge of gate candidates into the running k best.  Order:
// 2F descending, ties by the lower (sky, fdot, bin) key; NaN never enters.
// Selections take k rounds of an argmax restricted to items strictly after
// the previous pick in that order, so results do not depend on the launch
// geometry or on the order in which candidates were appended.
#include <math.h>

#include <algorithm>

#include "rsf_device.h"
#include "rsf_launch.h"
#include "rsf_topk_gate.h"

namespace rsf {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanWaveVals = 64;                 // map values per lane
constexpr int kScanChunk = 64 * kScanWaveVals;    // map values per wave
constexpr int kMergeThreads = 1024;
constexpr int kMergeItems = 4;                    // candidates per merge thread (in registers)
constexpr int kMergePer = kMergeThreads * kMergeItems;
}  // namespace

// Each wave takes a chunk of kScanWaveVals x 64 consecutive map values into
// registers (value q of lane l is chunk element 64 q + l) and passes them
// through the gate: with at most kGateFast values at or above the threshold
// the wave appends them all; with more, it selects its k best by k rounds of
// a wave-wide argmax (no LDS, no barriers), appends those and raises the
// threshold.  Within one scan the map index m = row n_out + bin orders
// candidates as the (sky, fdot, bin) key does (rows are in template order),
// so the rounds rank by (2F, index in the chunk) and only winners get a key.
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
    auto key_of = [&](int64_t m) {
        const int64_t row = m / A.n_out;
        const int64_t bin = m - row * A.n_out;
        const int64_t s_l = row / A.nf_l;
        const int64_t f = row - s_l * A.nf_l;
        return (unsigned long long)(((A.sky0 + s_l) * A.n_fdot + A.f0 + f) * A.n_out + bin);
    };
    const float thr = gate_threshold(A.gate);
    const int part = (int)(blockIdx.x % (unsigned)A.n_part);
    TopkItem* pc = A.cand + (int64_t)part * A.part_cap;
    int c = 0;
#pragma unroll
    for (int q = 0; q < kScanWaveVals; ++q) c += gate_pass(v[q], thr) ? 1 : 0;
    int total;
    const int pre = wave_prefix(c, lane, total);
    if (total == 0) return;
    if (total <= kGateFast) {
        unsigned slot = gate_reserve(A.gate, part, total, lane) + (unsigned)pre;
#pragma unroll
        for (int q = 0; q < kScanWaveVals; ++q)
            if (gate_pass(v[q], thr)) {
                if ((int64_t)slot < A.part_cap) {
                    TopkItem it;
                    it.v = v[q];
                    it.pad = 0;
                    it.key = key_of(base + q * 64 + lane);
                    pc[slot] = it;
                }
                ++slot;
            }
        return;
    }
    const unsigned first_slot = gate_reserve(A.gate, part, A.k, lane);
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
            if (gate_pass(x, thr) && (first || topk_better(pv, pi, x, ii)) && topk_better(x, ii, bv, bi)) {
                bv = x;
                bi = ii;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(bv, off);
            const unsigned oi = __shfl_xor(bi, off);
            if (topk_better(ov, oi, bv, bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0 && (int64_t)(first_slot + r) < A.part_cap) {
            TopkItem it = topk_empty();
            if (bv != -INFINITY) {
                it.v = bv;
                it.key = key_of(base + (int64_t)bi);
            }
            pc[first_slot + r] = it;
        }
        pv = bv;
        pi = bi;
        first = false;
    }
    // pv is the k-th best (or -inf when fewer than k values passed: no raise)
    if (lane == 0) gate_raise(A.gate, pv);
}

// Block b ranks items [b kMergePer, (b + 1) kMergePer) of cand ++ run_in
// (each thread holds up to kMergeItems of them in registers) and writes its
// k best: to run_out (and entries) when the grid is one block, else to
// out_blocks[b k ...].  With n_gate, cand is the gate's partitions of
// part_cap slots, of which the first count[p] of partition p are filled (the
// rest read as empty).  The one-block level, given a gate, sets its
// threshold to the k-th result (when there are k) and clears its counts.
__global__ __launch_bounds__(kMergeThreads) void rsf_topk_merge_k(TopkMergeArgs A) {
    __shared__ float sv[kMergeThreads / 64];
    __shared__ unsigned long long sk[kMergeThreads / 64];
    __shared__ TopkItem res[kTopkMax];
    const int64_t total = A.n_cand + (A.run_in ? A.k : 0);
    const int64_t lo = (int64_t)blockIdx.x * kMergePer;
    TopkItem it[kMergeItems];
    bool any = false;
#pragma unroll
    for (int q = 0; q < kMergeItems; ++q) {
        const int64_t i = lo + threadIdx.x + (int64_t)q * kMergeThreads;
        bool real = i < total;
        if (real && A.n_gate && i < A.n_cand) {
            const int64_t pt = i / A.part_cap;
            real = i - pt * A.part_cap < (int64_t)A.gate->count[pt * kGateStride];
        }
        it[q] = real ? ((i < A.n_cand) ? A.cand[i] : A.run_in[i - A.n_cand]) : topk_empty();
        if (it[q].v != it[q].v) it[q] = topk_empty();
        any |= it[q].v != -INFINITY;
    }
    if (gridDim.x > 1 && !__syncthreads_or(any)) {
        // nothing but empty slots: k empty results
        if (threadIdx.x < A.k) A.out_blocks[(int64_t)blockIdx.x * A.k + threadIdx.x] = topk_empty();
        return;
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
            if ((first || topk_better(pv, pk, it[q].v, it[q].key)) && topk_better(it[q].v, it[q].key, bv, bk)) {
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
    if (gridDim.x == 1 && A.gate) {
        if (threadIdx.x == 0 && res[A.k - 1].v != -INFINITY) A.gate->thr = __float_as_uint(res[A.k - 1].v);
        for (int i = threadIdx.x; i < kGateParts; i += kMergeThreads) A.gate->count[i * kGateStride] = 0u;
    }
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

// Gate partitions of a scan over n_vals map values and their capacity.
int topk_scan_parts(int64_t n_vals, int64_t* part_cap) {
    const int blocks = topk_scan_blocks(n_vals);
    const int parts = std::max(1, std::min(blocks, kGateParts));
    *part_cap = (int64_t)((blocks + parts - 1) / parts) * (kScanThreads / 64) * kGateItemsPerUnit;
    return parts;
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

// Time-domain front end (paper Sec. III.A.1, eqs. eq14-eq16): heterodyne a
// real high-rate series, low-pass filter it at the new Nyquist frequency and
// keep every D-th sample.  The heterodyne factor of raw sample
// m = j D + c - i splits into exp(-2 pi i f_h j D dt) exp(-2 pi i f_h (c - i) dt),
// so the filter runs with complex taps g[i] = h[i] exp(-2 pi i f_h (c - i) dt)
// on the real series and each output takes one FP64 phase factor.
//
// Two forms: for D = 64 and K = 8, 12 or 16 a product on the FP32 matrix
// cores (rsf_hetdec_mfma_k, below); for every other D and K a direct sum
// (rsf_hetdec_k): one workgroup per 64 outputs, the raw samples its outputs
// touch and the taps in LDS, each wave computing four outputs at a time with
// its lanes striding over the taps (consecutive lanes read consecutive
// samples and taps), then summing across the wave.
#include <algorithm>

#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kHdThreads = 256;
constexpr int kHdOut = 64;     // outputs per workgroup
constexpr int kHdIlp = 4;      // outputs per wave pass
}  // namespace

__global__ __launch_bounds__(kHdThreads) void rsf_hetdec_k(HetdecArgs a) {
    extern __shared__ float sm[];
    float2* g = reinterpret_cast<float2*>(sm);      // L taps
    float* xs = sm + 2 * a.L;                         // raw window
    const int64_t j0 = (int64_t)blockIdx.x * kHdOut;
    const int nj = (int)min((int64_t)kHdOut, a.n_out - j0);
    const int64_t m0 = j0 * a.D + a.c - (a.L - 1);    // first raw sample touched
    const int span = (nj - 1) * a.D + a.L;
    for (int i = threadIdx.x; i < a.L; i += kHdThreads) g[i] = a.g[i];
    for (int i = threadIdx.x; i < span; i += kHdThreads) {
        const int64_t m = m0 + i;
        xs[i] = (m >= 0 && m < a.n_raw) ? a.x[m] : 0.f;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int jb = wave * kHdIlp; jb < nj; jb += 4 * kHdIlp) {
        float re[kHdIlp], im[kHdIlp];
#pragma unroll
        for (int q = 0; q < kHdIlp; ++q) re[q] = im[q] = 0.f;
        // output jb + q reads window index (jb + q) D + (L - 1) - i for tap i
        const int base = jb * a.D + (a.L - 1);
        for (int i = lane; i < a.L; i += 64) {
            const float2 t = g[i];
#pragma unroll
            for (int q = 0; q < kHdIlp; ++q) {
                if (jb + q < nj) {
                    const float v = xs[base + q * a.D - i];
                    re[q] += t.x * v;
                    im[q] += t.y * v;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kHdIlp; ++q) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                re[q] += __shfl_xor(re[q], off);
                im[q] += __shfl_xor(im[q], off);
            }
        }
        if (lane < kHdIlp && jb + lane < nj) {
            float r = re[0], m = im[0];
#pragma unroll
            for (int q = 1; q < kHdIlp; ++q)
                if (lane == q) {
                    r = re[q];
                    m = im[q];
                }
            const int64_t j = j0 + jb + lane;
            const double cyc = a.cyc_per_out * (double)j;
            float s, c;
            sincospif(-2.0f * (float)(cyc - rint(cyc)), &s, &c);
            a.out[j] = make_float2(r * c - m * s, r * s + m * c);
        }
    }
}

// Matrix-core form for D = 64.  With raw rows X[q][p] = x[64 q + p], output j
// is sum_i g[i] x[64 j + c - i], c = 64 K; writing the raw index as 64 q + p
// gives i = 64 (j - q + K) - p, so with m = j - q
//   y_j = sum_{m=-K+1}^{K} Z[j - m][m] + g[0] X[j + K][0],
//   Z[q][m] = sum_p X[q][p] G[m][p],  G[m][p] = g[64 (m + K) - p]
// (m = -K leaves only the tap g[0]).  Z is a real product of the rows
// (64 columns) with the 64 x 4K matrix B[p][c] = Re G[m][p] (c = m + K - 1
// < 2K) or Im G[m][p] (c = m + 3K - 1): FP32 MFMA 16x16x4 tiles, B held in
// registers, A read from rows staged in LDS.  A block is 256 rows: its
// J = 256 - 2K outputs and a halo of K rows on each side.  Persistent
// workgroups (one per CU) walk the blocks with two row buffers: the next
// block's rows arrive by DMA (global -> LDS) while the current block's Z is
// computed in place of its rows (each wave owns one 16-row tile), then one
// thread per output adds the 2K diagonal terms and applies the output phase.
namespace {
constexpr int kMmRows = 256;     // raw rows per block, halo included
constexpr int kMmStride = 66;    // LDS row stride in floats: A reads, Z writes and diagonal reads at most 2-way
constexpr int kMmThreads = 1024;  // 4 waves per SIMD
constexpr int kMmBuf = kMmRows * kMmStride;
typedef float mm_v4f __attribute__((ext_vector_type(4)));
}  // namespace

template <int K>
__global__ __launch_bounds__(kMmThreads) void rsf_hetdec_mfma_k(HetdecArgs a) {
    constexpr int NTL = K / 4;               // 16-column tiles of the 4K columns
    constexpr int J = kMmRows - 2 * K;       // outputs per block
    extern __shared__ float xz[];             // two buffers [kMmRows][kMmStride]: raw rows, then Z
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n_blk = (a.n_out + J - 1) / J;
    // B operand of k step s and column tile n: lane holds B[4 s + lane / 16][16 n + lane % 16]
    float bop[16][NTL];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int pp = 4 * s + (lane >> 4);
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
            const int col = 16 * n + (lane & 15);
            const int mk = col < 2 * K ? col : col - 2 * K;   // m + K - 1
            const float2 gv = a.g[64 * (mk + 1) - pp];
            bop[s][n] = col < 2 * K ? gv.x : gv.y;
        }
    }
    const float2 g0 = a.g[0];
    // rows of block b by DMA, one row of 64 samples per wave instruction;
    // samples outside the series are zero
    auto stage = [&](int64_t b, float* buf) {
        const int64_t r0 = b * J - K;
        for (int row = wave; row < kMmRows; row += kMmThreads / 64) {
            const int64_t m = (r0 + row) * 64 + lane;
            if (m >= 0 && m < a.n_raw)
                __builtin_amdgcn_global_load_lds((const void*)(a.x + m),
                                                 (__attribute__((address_space(3))) void*)(buf + row * kMmStride), 4, 0,
                                                 0);
            else
                buf[row * kMmStride + lane] = 0.f;
        }
    };
    int64_t b = blockIdx.x;
    if (b < n_blk) stage(b, xz);
    for (int it = 0; b < n_blk; ++it, b += gridDim.x) {
        float* buf = xz + (it & 1) * kMmBuf;
        // this thread's DMA for block b (and its earlier stores) have landed;
        // after the barrier, everyone's, and the other buffer's last block is
        // fully consumed
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (b + gridDim.x < n_blk) stage(b + gridDim.x, xz + ((it + 1) & 1) * kMmBuf);
        // X[j + K][0], the sample of the tap g[0], from global memory (the rows
        // in LDS are overwritten by Z below)
        const int64_t m0 = (b * J + tid + K) * 64;
        const float x0 = (tid < J && m0 < a.n_raw) ? a.x[m0] : 0.f;
        for (int rt = wave; rt < kMmRows / 16; rt += kMmThreads / 64) {
            mm_v4f acc[NTL];
#pragma unroll
            for (int n = 0; n < NTL; ++n) acc[n] = mm_v4f{0.f, 0.f, 0.f, 0.f};
            // A operand: lane holds X[16 rt + lane % 16][4 s + lane / 16]
            const float* arow = buf + (16 * rt + (lane & 15)) * kMmStride + (lane >> 4);
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const float av = arow[4 * s];
#pragma unroll
                for (int n = 0; n < NTL; ++n)
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bop[s][n], acc[n], 0, 0, 0);
            }
            // D layout: lane holds Z[16 rt + 4 (lane / 16) + v][16 n + lane % 16];
            // the tile's rows were read only by this wave, above
#pragma unroll
            for (int n = 0; n < NTL; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    buf[(16 * rt + 4 * (lane >> 4) + v) * kMmStride + 16 * n + (lane & 15)] = acc[n][v];
        }
        __syncthreads();
        const int64_t j = b * J + tid;
        if (tid < J && j < a.n_out) {
            float re = g0.x * x0, im = g0.y * x0;
#pragma unroll
            for (int mk = 0; mk < 2 * K; ++mk) {
                const float* z = buf + (tid + 2 * K - 1 - mk) * kMmStride;  // row of q = j - m, m = mk - K + 1
                re += z[mk];
                im += z[2 * K + mk];
            }
            const double cyc = a.cyc_per_out * (double)j;
            float sn, cs;
            sincospif(-2.0f * (float)(cyc - rint(cyc)), &sn, &cs);
            a.out[j] = make_float2(re * cs - im * sn, re * sn + im * cs);
        }
    }
}

namespace {
bool hetdec_mfma_form(int L, int D) {
    const int K = D > 0 ? (L - 1) / (2 * D) : 0;
    return D == 64 && (K == 8 || K == 12 || K == 16);
}
}  // namespace

size_t hetdec_lds(int L, int D) {
    if (hetdec_mfma_form(L, D)) return (size_t)2 * kMmBuf * sizeof(float);
    return (size_t)2 * L * sizeof(float) + (size_t)((kHdOut - 1) * D + L) * sizeof(float);
}

hipError_t launch_hetdec(const HetdecArgs& a, int n_cu, hipStream_t s) {
    if (hetdec_mfma_form(a.L, a.D)) {
        const int K = a.c / a.D;
        const size_t lds = hetdec_lds(a.L, a.D);
        const int64_t n_blk = (a.n_out + (kMmRows - 2 * K) - 1) / (kMmRows - 2 * K);
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_blk, n_cu));
        switch (K) {
            case 8: hipLaunchKernelGGL(rsf_hetdec_mfma_k<8>, dim3(grid), dim3(kMmThreads), lds, s, a); break;
            case 12: hipLaunchKernelGGL(rsf_hetdec_mfma_k<12>, dim3(grid), dim3(kMmThreads), lds, s, a); break;
            default: hipLaunchKernelGGL(rsf_hetdec_mfma_k<16>, dim3(grid), dim3(kMmThreads), lds, s, a); break;
        }
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)((a.n_out + kHdOut - 1) / kHdOut);
    hipLaunchKernelGGL(rsf_hetdec_k, dim3(grid), dim3(kHdThreads), hetdec_lds(a.L, a.D), s, a);
    return hipGetLastError();
}

hipError_t hetdec_set_lds_limit(size_t bytes) {
    static size_t granted = 0;  // only grows
    if (bytes <= granted) return hipSuccess;
    const void* fns[] = {(const void*)rsf_hetdec_k, (const void*)rsf_hetdec_mfma_k<8>,
                         (const void*)rsf_hetdec_mfma_k<12>, (const void*)rsf_hetdec_mfma_k<16>};
    hipError_t out = hipSuccess;
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (out == hipSuccess) out = e;
    }
    if (out == hipSuccess) granted = bytes;
    return out;
}

}  // namespace rsf

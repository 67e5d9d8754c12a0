// Time-domain front end (paper Sec. III.A.1, eqs. eq14-eq16): heterodyne a
// real high-rate series, low-pass filter it at the new Nyquist frequency and
// keep every D-th sample.  The heterodyne factor of raw sample
// m = j D + c - i splits into exp(-2 pi i f_h j D dt) exp(-2 pi i f_h (c - i) dt),
// so the filter runs with complex taps g[i] = h[i] exp(-2 pi i f_h (c - i) dt)
// on the real series and each output takes one FP64 phase factor.
//
// One workgroup per 64 outputs: the raw samples its outputs touch and the
// taps sit in LDS; each wave computes four outputs at a time, its lanes
// striding over the taps (consecutive lanes read consecutive samples and
// taps), then sums across the wave.
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

// Polyphase form for D = 64 (one lane per tap phase p): output j is
//   sum_p sum_k g[p + 64 k] s_p[j + K - k],  s_p[m] = x[64 m - p],
// a (2K+1)-tap convolution per phase.  Lane p keeps its 2K+1 taps and a ring
// of the last 2K+1 samples s_p in registers (slot of m: (m - m0) mod (2K+1)),
// so each output costs one coalesced load per lane (the wave reads 64
// consecutive raw samples) and 2 (2K+1) multiply-adds; the 64 phase sums of
// 2K+1 consecutive outputs are added through a transposed LDS buffer.  One
// wave per workgroup, kPolyChunks runs of 2K+1 outputs per wave.
namespace {
constexpr int kPolyChunks = 16;
}

template <int K>
__global__ __launch_bounds__(64) void rsf_hetdec_poly_k(HetdecArgs a) {
    constexpr int NT = 2 * K + 1;
    __shared__ float stage[2][NT][64];  // the samples of a chunk, one row per output step
    __shared__ float2 red[64][NT + 1];
    const int p = threadIdx.x;
    float2 g[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int i = p + 64 * k;
        g[k] = i < a.L ? a.g[i] : make_float2(0.f, 0.f);
    }
    const int64_t jw = (int64_t)blockIdx.x * kPolyChunks * NT;  // first output of this wave
    if (jw >= a.n_out) return;
    const int64_t m0 = jw - K;                                    // sample in ring slot 0
    const int n_ch = (int)min((int64_t)kPolyChunks, (a.n_out - jw + NT - 1) / NT);
    // chunk ch brings s_p[m] for m = jw + ch NT + K + u, u < NT, by DMA (global -> LDS);
    // samples outside the series are zero
    auto dma = [&](int ch, int buf) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int64_t idx = 64 * (jw + (int64_t)ch * NT + K + u) - p;
            if (idx >= 0 && idx < a.n_raw)
                __builtin_amdgcn_global_load_lds((const void*)(a.x + idx),
                                                 (__attribute__((address_space(3))) void*)&stage[buf][u][0], 4, 0, 0);
            else
                stage[buf][u][p] = 0.f;
        }
    };
    float r[NT];
#pragma unroll
    for (int t = 0; t < NT - 1; ++t) {
        const int64_t idx = 64 * (m0 + t) - p;
        r[t] = (idx >= 0 && idx < a.n_raw) ? a.x[idx] : 0.f;
    }
    dma(0, 0);
    for (int ch = 0; ch < n_ch; ++ch) {
        const int buf = ch & 1;
        // this chunk's DMA (and the previous chunk's stores) have landed; the
        // other buffer was last read by the previous chunk
        __builtin_amdgcn_s_waitcnt(0);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        if (ch + 1 < n_ch) dma(ch + 1, buf ^ 1);
        const int64_t jc = jw + (int64_t)ch * NT;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            // output jc + u needs s_p[jc + u + K - k]; the newest, m = jc + u + K,
            // goes to slot (u + 2K) mod NT (NT divides the chunk stride)
            r[(u + NT - 1) % NT] = stage[buf][u][p];
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                const float v = r[(u + 2 * K - k) % NT];
                re += g[k].x * v;
                im += g[k].y * v;
            }
            red[p][u] = make_float2(re, im);
        }
        // red is this wave's own: its LDS operations run in order, so ordering
        // the compiler's memory operations is enough
        asm volatile("" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        if (p < NT) {
            const int64_t j = jc + p;
            float re = 0.f, im = 0.f;
            for (int q = 0; q < 64; ++q) {
                const float2 v = red[q][p];
                re += v.x;
                im += v.y;
            }
            if (j < a.n_out) {
                const double cyc = a.cyc_per_out * (double)j;
                float sn, cs;
                sincospif(-2.0f * (float)(cyc - rint(cyc)), &sn, &cs);
                a.out[j] = make_float2(re * cs - im * sn, re * sn + im * cs);
            }
        }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_wave_barrier();  // the next chunk rewrites red
    }
}

size_t hetdec_lds(int L, int D) { return (size_t)2 * L * sizeof(float) + (size_t)((kHdOut - 1) * D + L) * sizeof(float); }

hipError_t launch_hetdec(const HetdecArgs& a, hipStream_t s) {
    const int K = a.D > 0 ? a.c / a.D : 0;
    if (a.D == 64 && (K == 8 || K == 12 || K == 16)) {
        const int nt = 2 * K + 1;
        const unsigned grid = (unsigned)((a.n_out + (int64_t)kPolyChunks * nt - 1) / ((int64_t)kPolyChunks * nt));
        switch (K) {
            case 8: hipLaunchKernelGGL(rsf_hetdec_poly_k<8>, dim3(grid), dim3(64), 0, s, a); break;
            case 12: hipLaunchKernelGGL(rsf_hetdec_poly_k<12>, dim3(grid), dim3(64), 0, s, a); break;
            default: hipLaunchKernelGGL(rsf_hetdec_poly_k<16>, dim3(grid), dim3(64), 0, s, a); break;
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
    const hipError_t e = hipFuncSetAttribute((const void*)rsf_hetdec_k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)bytes);
    if (e == hipSuccess) granted = bytes;
    return e;
}

}  // namespace rsf

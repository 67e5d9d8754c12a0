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

size_t hetdec_lds(int L, int D) { return (size_t)2 * L * sizeof(float) + (size_t)((kHdOut - 1) * D + L) * sizeof(float); }

hipError_t launch_hetdec(const HetdecArgs& a, hipStream_t s) {
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

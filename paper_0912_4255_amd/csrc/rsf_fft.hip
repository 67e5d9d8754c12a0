// Zero-padded FFTs of F_a and F_b and the F-statistic (paper Sec. III.A.2,
// steps 6-7; eqs. eq19, eq20, eq6) as a two-pass four-step transform.
//
// N_fft = LA * LB.  With input index n = LB n_a + n_b and output index
// k = k_a + LA k_b:
//   X[k_a + LA k_b] = sum_{n_b} W_LB^{n_b k_b} W_N^{n_b k_a}
//                     sum_{n_a} x[LB n_a + n_b] W_LA^{n_a k_a}.
// Pass A: one workgroup per row n_b.  It forms the integrands
//   y^a = sum_X w_X a z~ exp(-i Phi_s),  y^b likewise  (eq. eq4pt1, FP64 phase)
// from the resampled series (stored transposed, so the row is contiguous),
// transforms the row in LDS (both spectra in one float4 per element), applies
// W_N^{n_b k_a} and spills in blocks of 8 consecutive k_a (128 B).
// Pass B: one workgroup per 8 consecutive k_a.  It reads its contiguous
// block, transforms the 8 columns over n_b in LDS and reduces every bin to
// 2F = cA |f_a|^2 + cB |f_b|^2 + cC Re(f_a f_b^*), writing the reported band
// in ascending frequency.
#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kNT = kFftThreads;
constexpr int kEPT = kFftEPT;  // max LA (pass A) or 8 LB (pass B) = kNT * kEPT = 10240
}  // namespace

__global__ __launch_bounds__(kNT) void rsf_fft_pass_a_k(PassAArgs A) {
    extern __shared__ float4 lds[];
    const int n_b = blockIdx.x;
    const int t0 = blockIdx.y * A.fb;
    const int t1 = min(t0 + A.fb, A.n_tmpl);
    const int tid = threadIdx.x;
    const int64_t row = (int64_t)n_b * A.P;

    for (int t = t0; t < t1; ++t) {
        const double fd = A.fdot[t];
        for (int n_a = tid; n_a < A.LA; n_a += kNT) {
            cp y = make_float4(0.f, 0.f, 0.f, 0.f);
            const int64_t k = (int64_t)A.LB * n_a + n_b;
            if (n_a < A.P && k < A.n) {
                const double tb = (double)k * A.dt;
                for (int X = 0; X < A.n_det; ++X) {
                    const float4 m = A.rs_main[X][row + n_a];
                    float zr, zi, av, bv, tmf;
                    if (A.f16) {
                        const uint32_t bits = __float_as_uint(m.x);
                        const __half2 h = *reinterpret_cast<const __half2*>(&bits);
                        const float2 z = __half22float2(h);
                        zr = z.x;
                        zi = z.y;
                        av = m.y;
                        bv = m.z;
                        tmf = m.w;
                    } else {
                        zr = m.x;
                        zi = m.y;
                        av = m.z;
                        bv = m.w;
                        tmf = A.rs_tm[X][row + n_a];
                    }
                    // Phi_s = 2 pi fdot (T^2/2 + t_m T) = 2 pi fdot (t_b^2 - t_m^2)/2, T = t_b - t_m
                    const double tm = (double)tmf;
                    const double cyc = fd * 0.5 * (tb * tb - tm * tm);
                    const float ph = (float)(cyc - rint(cyc));
                    float s, c;
                    sincospif(2.f * ph, &s, &c);
                    const float er = zr * c + zi * s;  // z exp(-i Phi_s)
                    const float ei = zi * c - zr * s;
                    const float wa = (float)A.w[X] * av, wb = (float)A.w[X] * bv;
                    y.x += wa * er;
                    y.y += wa * ei;
                    y.z += wb * er;
                    y.w += wb * ei;
                }
            }
            lds[n_a] = y;
        }
        __syncthreads();
        lds_fft<kNT, kEPT, 1>(lds, A.st, A.tw);
        float4* out = A.spill + (int64_t)t * A.spill_tmpl_stride;
        for (int ka = tid; ka < A.LA; ka += kNT) {
            cp v = lds[ka];
            const int64_t m = ((int64_t)n_b * ka) % A.n_fft;
            const float2 w = c_mul(A.tw_hi[m >> kTwSplitBits], A.tw_lo[m & ((1 << kTwSplitBits) - 1)]);
            v = cp_rot(v, w);
            out[((int64_t)(ka >> 3) * A.LB + n_b) * kPassBCols + (ka & 7)] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kNT) void rsf_fft_pass_b_k(PassBArgs B) {
    extern __shared__ float4 lds[];
    const int c = blockIdx.x;
    const int t = blockIdx.y;
    const int tid = threadIdx.x;
    const float4* in = B.spill + (int64_t)t * B.spill_tmpl_stride + (int64_t)c * B.LB * kPassBCols;
    const int tot = B.LB * kPassBCols;
    for (int e = tid; e < tot; e += kNT) lds[e] = in[e];
    __syncthreads();
    lds_fft<kNT, kEPT, kPassBCols>(lds, B.st, B.tw);
    const float cA = B.coef[0], cB = B.coef[1], cC = B.coef[2];
    float* out = B.twoF + (B.out_row0 + t) * B.n_out;
    for (int e = tid; e < tot; e += kNT) {
        const int kb = e >> 3;
        const int ka = c * kPassBCols + (e & 7);
        if (ka < B.LA) {
            const int64_t k = (int64_t)ka + (int64_t)B.LA * kb;
            const int64_t s = (2 * k < B.n_fft) ? k : k - B.n_fft;
            const int64_t o = s - B.s_lo;
            if (o >= 0 && o < B.n_out) {
                const cp v = lds[e];
                out[o] = cA * (v.x * v.x + v.y * v.y) + cB * (v.z * v.z + v.w * v.w) +
                         cC * (v.x * v.z + v.y * v.w);
            }
        }
    }
}

int fft_pass_max_elems() { return kNT * kEPT; }

hipError_t launch_fft_pass_a(const PassAArgs& a, hipStream_t s) {
    const size_t lds = (size_t)a.LA * sizeof(float4);
    const unsigned gy = (unsigned)((a.n_tmpl + a.fb - 1) / a.fb);
    hipLaunchKernelGGL(rsf_fft_pass_a_k, dim3((unsigned)a.LB, gy), dim3(kNT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_fft_pass_b(const PassBArgs& b, hipStream_t s) {
    const size_t lds = (size_t)b.LB * kPassBCols * sizeof(float4);
    hipLaunchKernelGGL(rsf_fft_pass_b_k, dim3((unsigned)b.n_groups, (unsigned)b.n_tmpl), dim3(kNT), lds, s, b);
    return hipGetLastError();
}

hipError_t fft_set_lds_limits(size_t bytes) {
    hipError_t e1 = hipFuncSetAttribute((const void*)rsf_fft_pass_a_k,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipError_t e2 = hipFuncSetAttribute((const void*)rsf_fft_pass_b_k,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e1 != hipSuccess ? e1 : e2;
}

}  // namespace rsf

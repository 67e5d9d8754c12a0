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

// Integrand of one detector for one sample (see the header comment).
__device__ __forceinline__ void accumulate_integrand(cp& y, float4 m, float tmf, bool f16, double tb, double fd,
                                                     float w) {
    float zr, zi, av, bv;
    if (f16) {
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
    }
    // Phi_s = 2 pi fdot (T^2/2 + t_m T) = 2 pi fdot (t_b^2 - t_m^2)/2 with T = t_b - t_m
    const double tm = (double)tmf;
    const double cyc = fd * 0.5 * (tb * tb - tm * tm);
    const float ph = (float)(cyc - rint(cyc));
    float s, c;
    sincospif(2.f * ph, &s, &c);
    const float er = zr * c + zi * s;  // z exp(-i Phi_s)
    const float ei = zi * c - zr * s;
    const float wa = w * av, wb = w * bv;
    y.x += wa * er;
    y.y += wa * ei;
    y.z += wb * er;
    y.w += wb * ei;
}

// Inputs of one row held per thread: n_a = tid + q * kNT, q < kInPer (P <= LA/2 <= 5120).
constexpr int kInPer = (kNT * kEPT / 2 + kNT - 1) / kNT;

__global__ __launch_bounds__(kNT) void rsf_fft_pass_a_k(PassAArgs A) {
    extern __shared__ float4 lds[];
    const int n_b = blockIdx.x;
    const int gpf = (A.nf_l + A.fb - 1) / A.fb;       // spindown groups per sky
    const int s_l = blockIdx.y / gpf;
    const int f_lo = (blockIdx.y - s_l * gpf) * A.fb;
    const int f_hi = min(f_lo + A.fb, A.nf_l);
    const int tid = threadIdx.x;
    const int64_t row = (int64_t)s_l * A.rs_sky_stride + (int64_t)n_b * A.P;

    // first detector's row: all loads issued before any is used, kept for every spindown
    float4 m0[kInPer];
    float tm0[kInPer];
#pragma unroll
    for (int q = 0; q < kInPer; ++q) {
        const int n_a = tid + q * kNT;
        const int64_t k = (int64_t)A.LB * n_a + n_b;
        if (n_a < A.P && k < A.n) {
            m0[q] = A.rs_main[0][row + n_a];
            tm0[q] = A.f16 ? 0.f : A.rs_tm[0][row + n_a];
        } else {
            m0[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            tm0[q] = 0.f;
        }
    }

    // inter-pass twiddle W_N^{n_b k_a} for k_a = tid + q kNT: base W^{n_b tid}, step W^{n_b kNT}
    const int64_t mb = ((int64_t)n_b * tid) % A.n_fft;
    const int64_t ms = ((int64_t)n_b * kNT) % A.n_fft;
    const int msk = (1 << kTwSplitBits) - 1;
    const float2 w_base = c_mul(A.tw_hi[mb >> kTwSplitBits], A.tw_lo[mb & msk]);
    const float2 w_step = c_mul(A.tw_hi[ms >> kTwSplitBits], A.tw_lo[ms & msk]);

    for (int f = f_lo; f < f_hi; ++f) {
        const int t = s_l * A.nf_l + f;
        const double fd = A.fdot[f];
#pragma unroll
        for (int q = 0; q < kInPer; ++q) {
            const int n_a = tid + q * kNT;
            if (n_a < A.LA) {
                cp y = make_float4(0.f, 0.f, 0.f, 0.f);
                const int64_t k = (int64_t)A.LB * n_a + n_b;
                if (n_a < A.P && k < A.n) {
                    const double tb = (double)k * A.dt;
                    accumulate_integrand(y, m0[q], tm0[q], A.f16, tb, fd, (float)A.w[0]);
                    for (int X = 1; X < A.n_det; ++X)
                        accumulate_integrand(y, A.rs_main[X][row + n_a], A.f16 ? 0.f : A.rs_tm[X][row + n_a],
                                             A.f16, tb, fd, (float)A.w[X]);
                }
                lds[n_a] = y;
            }
        }
        for (int n_a = tid + kInPer * kNT; n_a < A.LA; n_a += kNT) lds[n_a] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        lds_fft<kNT, kEPT, 1>(lds, A.st, A.tw);
        float4* out = A.spill + (int64_t)t * A.spill_tmpl_stride;
        float2 w = w_base;
        for (int ka = tid; ka < A.LA; ka += kNT) {
            const cp v = cp_rot(lds[ka], w);
            out[((int64_t)(ka >> 3) * A.LB + n_b) * kPassBCols + (ka & 7)] = v;
            w = c_mul(w, w_step);
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
    // loads issued in batches of kEPT/2 before their LDS stores
#pragma unroll
    for (int q0 = 0; q0 < kEPT; q0 += kEPT / 2) {
        float4 v[kEPT / 2];
#pragma unroll
        for (int q = 0; q < kEPT / 2; ++q) {
            const int e = tid + (q0 + q) * kNT;
            v[q] = in[e < tot ? e : 0];
        }
#pragma unroll
        for (int q = 0; q < kEPT / 2; ++q) {
            const int e = tid + (q0 + q) * kNT;
            if (e < tot) lds[e] = v[q];
        }
    }
    __syncthreads();
    lds_fft<kNT, kEPT, kPassBCols>(lds, B.st, B.tw);
    const int s_l = t / B.nf_l;
    const int f = t - s_l * B.nf_l;
    const float* cf = B.coef + 4 * s_l;
    const float cA = cf[0], cB = cf[1], cC = cf[2];
    const int64_t out_row = B.map_rows ? (int64_t)t : (B.sky0 + s_l) * B.n_fdot + B.f0 + f;
    float* out = B.twoF + out_row * B.n_out;
    // 32-bit bin arithmetic (n_fft < 2^31)
    const int nf = (int)B.n_fft, s_lo = (int)B.s_lo, n_out = (int)B.n_out;
    for (int e = tid; e < tot; e += kNT) {
        const int kb = e >> 3;
        const int ka = c * kPassBCols + (e & 7);
        if (ka < B.LA) {
            const int k = ka + B.LA * kb;
            const int s = (2 * k < nf) ? k : k - nf;
            const int o = s - s_lo;
            if (o >= 0 && o < n_out) {
                const cp u = lds[e];
                out[o] = cA * (u.x * u.x + u.y * u.y) + cB * (u.z * u.z + u.w * u.w) +
                         cC * (u.x * u.z + u.y * u.w);
            }
        }
    }
}

int fft_pass_max_elems() { return kNT * kEPT; }

hipError_t launch_fft_pass_a(const PassAArgs& a, hipStream_t s) {
    const size_t lds = (size_t)a.LA * sizeof(float4);
    const unsigned gy = (unsigned)(a.n_sky_l * ((a.nf_l + a.fb - 1) / a.fb));
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

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
#include <algorithm>

#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kNT = kFftThreads;
constexpr int kEPT = kFftEPT;
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
constexpr int kInPer = (kFftMaxLen / 2 + kNT - 1) / kNT;

__global__ __launch_bounds__(kNT) void rsf_fft_pass_a_k(PassAArgs A) {
    extern __shared__ float4 lds[];
    // stage twiddles in LDS after the row: no global load inside the stages,
    // so the spill stores of one spindown stay in flight during the next FFT
    float2* twl = reinterpret_cast<float2*>(lds + A.LA);
    const int n_hi = (A.LA + 31) >> kTwLoBits;
    for (int i = threadIdx.x; i < 32 + n_hi; i += kNT) twl[i] = (i < 32) ? A.tws_lo[i] : A.tws_hi[i - 32];
    const TwLds tws{twl, twl + 32};
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
        lds_fft<kNT, kEPT, 1>(lds, A.st, tws);
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

// Second pass, persistent and software-pipelined.  Workgroup g handles the
// spill blocks g, g + grid, ... (block = template * n_groups + group of 8
// columns), each as two 4-column halves.  Halves go through two LDS buffers:
// while one half is transformed, the next half is copied global -> LDS by
// the DMA loads (no registers involved), so memory traffic overlaps the
// FFT.  The two halves of a 128 B spill row and of a 2F output line are
// handled back to back by the same workgroup and meet in its L2.
constexpr int kHalfCols = kPassBCols / 2;

__device__ __forceinline__ void passb_dma(const PassBArgs& B, int unit, int h, float4* dst) {
    const int t = unit / B.n_groups;
    const int c = unit - t * B.n_groups;
    const float4* base = B.spill + (int64_t)t * B.spill_tmpl_stride + (int64_t)c * B.LB * kPassBCols + h * kHalfCols;
    const int half = B.LB * kHalfCols;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int e0 = wave * 64; e0 < half; e0 += kNT) {
        const int e = e0 + lane;
        if (e < half) {
            const float4* src = base + (e / kHalfCols) * kPassBCols + (e % kHalfCols);
            __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)(dst + e0),
                                             16, 0, 0);
        }
    }
}

__global__ __launch_bounds__(kNT) void rsf_fft_pass_b_k(PassBArgs B) {
    extern __shared__ float4 lds[];
    const int half = B.LB * kHalfCols;
    const int buf_elems = ((half + 63) / 64) * 64;
    float2* twl = reinterpret_cast<float2*>(lds + 2 * buf_elems);
    const int n_hi = (B.LB + 31) >> kTwLoBits;
    float* cfl = reinterpret_cast<float*>(twl + 32 + n_hi);
    const int tid = threadIdx.x;
    for (int i = tid; i < 32 + n_hi; i += kNT) twl[i] = (i < 32) ? B.tw_lo[i] : B.tw_hi[i - 32];
    for (int i = tid; i < 4 * B.n_sky_l; i += kNT) cfl[i] = B.coef[i];
    const TwLds tw{twl, twl + 32};
    const int n_units = B.n_tmpl * B.n_groups;
    const int nf = (int)B.n_fft, s_lo = (int)B.s_lo, n_out = (int)B.n_out;

    int unit = blockIdx.x, h = 0, cur = 0;
    if (unit < n_units) passb_dma(B, unit, 0, lds);
    while (unit < n_units) {
        __builtin_amdgcn_s_waitcnt(0);  // this thread's DMA loads and stores are complete
        __syncthreads();                // ... and everyone's: buffer cur is filled, buffer cur^1 is free
        const int nunit = h ? unit + (int)gridDim.x : unit;
        const int nh = h ^ 1;
        if (nunit < n_units) passb_dma(B, nunit, nh, lds + (cur ^ 1) * buf_elems);
        cp* x = lds + cur * buf_elems;
        lds_fft<kNT, kPassBEPT, kHalfCols>(x, B.st, tw);
        const int t = unit / B.n_groups;
        const int c = unit - t * B.n_groups;
        const int s_l = t / B.nf_l;
        const int f = t - s_l * B.nf_l;
        const float cA = cfl[4 * s_l], cB = cfl[4 * s_l + 1], cC = cfl[4 * s_l + 2];
        const int64_t out_row = B.map_rows ? (int64_t)t : (B.sky0 + s_l) * B.n_fdot + B.f0 + f;
        float* out = B.twoF + out_row * B.n_out;
        for (int e = tid; e < half; e += kNT) {
            const int kb = e >> 2;
            const int ka = c * kPassBCols + h * kHalfCols + (e & 3);
            if (ka < B.LA) {
                const int k = ka + B.LA * kb;
                const int s = (2 * k < nf) ? k : k - nf;
                const int o = s - s_lo;
                if (o >= 0 && o < n_out) {
                    const cp u = x[e];
                    out[o] = cA * (u.x * u.x + u.y * u.y) + cB * (u.z * u.z + u.w * u.w) +
                             cC * (u.x * u.z + u.y * u.w);
                }
            }
        }
        unit = nunit;
        h = nh;
        cur ^= 1;
    }
}

int fft_pass_max_elems() { return kFftMaxLen < kNT * kEPT ? kFftMaxLen : kNT * kEPT; }

size_t fft_pass_a_lds(int LA) { return (size_t)LA * sizeof(float4) + (32 + (LA + 31) / 32) * sizeof(float2); }

hipError_t launch_fft_pass_a(const PassAArgs& a, hipStream_t s) {
    const size_t lds = fft_pass_a_lds(a.LA);
    const unsigned gy = (unsigned)(a.n_sky_l * ((a.nf_l + a.fb - 1) / a.fb));
    hipLaunchKernelGGL(rsf_fft_pass_a_k, dim3((unsigned)a.LB, gy), dim3(kNT), lds, s, a);
    return hipGetLastError();
}

size_t fft_pass_b_lds(int LB, int n_sky_l) {
    const size_t buf = (size_t)((LB * kHalfCols + 63) / 64) * 64;
    return 2 * buf * sizeof(float4) + (32 + (LB + 31) / 32) * sizeof(float2) + (size_t)4 * n_sky_l * sizeof(float);
}

hipError_t launch_fft_pass_b(const PassBArgs& b, int n_cu, hipStream_t s) {
    const size_t lds = fft_pass_b_lds(b.LB, b.n_sky_l);
    const int n_items = b.n_tmpl * b.n_groups;
    const unsigned grid = (unsigned)std::max(1, std::min(n_items, n_cu));
    hipLaunchKernelGGL(rsf_fft_pass_b_k, dim3(grid), dim3(kNT), lds, s, b);
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

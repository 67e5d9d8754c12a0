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
// W_N^{n_b k_a} and spills in groups of 4 consecutive k_a (64-B rows).
// Pass B: persistent workgroups over blocks of 8 consecutive k_a (two
// adjacent spill groups, one contiguous run).  Each block is transformed
// over n_b in LDS and every bin reduced to
// 2F = cA |f_a|^2 + cB |f_b|^2 + cC Re(f_a f_b^*), written in ascending
// frequency over the reported band.
#include <algorithm>

#include "rsf_device.h"
#include "rsf_launch.h"
#include "rsf_spill.h"

namespace rsf {

namespace {
constexpr int kNT = kFftThreads;
constexpr int kNTB = kPassBThreads;
constexpr int kEPT = kFftEPT;
}  // namespace

// One resampled sample of one detector, unpacked for the integrand: z~,
// the noise-weighted beam patterns w a, w b, and the spindown coefficients
// u_j of eq. eq4pt1 in FP64, Phi_s = 2 pi sum_j f^(j) u_j with
// u_j = T^{j+1}/(j+1)! + t_m T^j/j!, T = t_b - t_m; they do not depend on the
// template.  u_1 = (t_b^2 - t_m^2) / 2.
template <int ORDER>
struct Sample {
    float zr, zi, wa, wb;
    double u[ORDER];
};

template <int ORDER>
__device__ __forceinline__ Sample<ORDER> unpack_sample(float4 m, float tmf, bool f16, double tb, float w) {
    Sample<ORDER> r;
    if (f16) {
        const uint32_t bits = __float_as_uint(m.x);
        const __half2 h = *reinterpret_cast<const __half2*>(&bits);
        const float2 z = __half22float2(h);
        r.zr = z.x;
        r.zi = z.y;
        r.wa = w * m.y;
        r.wb = w * m.z;
        tmf = m.w;
    } else {
        r.zr = m.x;
        r.zi = m.y;
        r.wa = w * m.z;
        r.wb = w * m.w;
    }
    const double tm = (double)tmf;
    r.u[0] = 0.5 * (tb * tb - tm * tm);
    if constexpr (ORDER >= 2) {
        const double T = tb - tm;
        const double T2 = T * T;
        r.u[1] = T2 * (T * (1.0 / 6.0) + 0.5 * tm);
        if constexpr (ORDER >= 3) r.u[2] = T2 * T * (T * (1.0 / 24.0) + tm * (1.0 / 6.0));
    }
    return r;
}

// Spindown parameters (f^(1) .. f^(ORDER)) of one template.
template <int ORDER>
struct Spin {
    double f[ORDER];
};

// y += (w a, w b) z~ exp(-i Phi_s) for one detector (eqs. eq19, eq20).
template <int ORDER>
__device__ __forceinline__ void accumulate_integrand(cp& y, const Sample<ORDER>& p, const Spin<ORDER>& sp) {
    double cyc = sp.f[0] * p.u[0];
#pragma unroll
    for (int j = 1; j < ORDER; ++j) cyc = fma(sp.f[j], p.u[j], cyc);
    // reduced to [-1/2, 1/2] cycle; v_sin_f32 / v_cos_f32 take revolutions
    const float ph = (float)(cyc - rint(cyc));
    const float s = __builtin_amdgcn_sinf(ph);
    const float c = __builtin_amdgcn_cosf(ph);
    const float er = p.zr * c + p.zi * s;  // z exp(-i Phi_s)
    const float ei = p.zi * c - p.zr * s;
    y.x += p.wa * er;
    y.y += p.wa * ei;
    y.z += p.wb * er;
    y.w += p.wb * ei;
}

// Inputs of one row held per thread: n_a = tid + q * kNT, q < kInPer (P <= LA/2 <= 5120).
constexpr int kInPer = (kFftMaxLen / 2 + kNT - 1) / kNT;

// NT: the launch's spill is larger than the last-level cache (non-temporal stores)
template <int ORDER, bool NT>
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

    // first detector's row: all loads issued before any is used, kept
    // (unpacked, with u) for every spindown
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
    Sample<ORDER> p0[kInPer];
#pragma unroll
    for (int q = 0; q < kInPer; ++q) {
        const int64_t k = (int64_t)A.LB * (tid + q * kNT) + n_b;
        p0[q] = unpack_sample<ORDER>(m0[q], tm0[q], A.f16, (double)k * A.dt, (float)A.w[0]);
    }
    // the upper half of the row is zero padding when P <= LA/2: it is
    // neither written nor read (pruned first stage)
    const bool prune = 2 * A.P <= A.LA && A.st.n_stages > 1 && (A.st.radix[0] & 1) == 0;
    const int zlim = prune ? A.LA / 2 : A.LA;

    // inter-pass twiddle W_N^{n_b k_a} for k_a = tid + q kNT: base W^{n_b tid}, step W^{n_b kNT}
    const int64_t mb = ((int64_t)n_b * tid) % A.n_fft;
    const int64_t ms = ((int64_t)n_b * kNT) % A.n_fft;
    const int msk = (1 << kTwSplitBits) - 1;
    const float2 w_base = c_mul(A.tw_hi[mb >> kTwSplitBits], A.tw_lo[mb & msk]);
    const float2 w_step = c_mul(A.tw_hi[ms >> kTwSplitBits], A.tw_lo[ms & msk]);
    const int r_last = A.st.n_stages ? A.st.radix[A.st.n_stages - 1] : 1;
    const int lr = A.LA / r_last;
    const int64_t ml = ((int64_t)n_b * lr) % A.n_fft;
    const float2 w_lr = c_mul(A.tw_hi[ml >> kTwSplitBits], A.tw_lo[ml & msk]);

    for (int f = f_lo; f < f_hi; ++f) {
        const int t = s_l * A.nf_l + f;
        Spin<ORDER> fd;
#pragma unroll
        for (int j = 0; j < ORDER; ++j) fd.f[j] = A.fdot[(int64_t)f * ORDER + j];
#pragma unroll
        for (int q = 0; q < kInPer; ++q) {
            const int n_a = tid + q * kNT;
            if (n_a < zlim) {
                cp y = make_float4(0.f, 0.f, 0.f, 0.f);
                const int64_t k = (int64_t)A.LB * n_a + n_b;
                if (n_a < A.P && k < A.n) {
                    accumulate_integrand(y, p0[q], fd);
                    for (int X = 1; X < A.n_det; ++X)
                        accumulate_integrand(y,
                                             unpack_sample<ORDER>(A.rs_main[X][row + n_a],
                                                                  A.f16 ? 0.f : A.rs_tm[X][row + n_a],
                                                           A.f16, (double)k * A.dt, (float)A.w[X]),
                                             fd);
                }
                lds[n_a] = y;
            }
        }
        for (int n_a = tid + kInPer * kNT; n_a < zlim; n_a += kNT) lds[n_a] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        SpillSink<NT> sink{reinterpret_cast<char*>(A.spill + (int64_t)t * A.spill_tmpl_stride), A.LB, n_b, lr,
                           w_base, w_step, w_lr};
        lds_fft_into<kNT, kEPT, 1, false>(lds, A.st, tws, Interleaved<1>{}, sink, NoMid{}, prune);
        __syncthreads();
    }
}

// Second pass, persistent.  Workgroup g handles the spill blocks g, g +
// grid, ... (block = template * n_groups + group of 8 columns k_a): the two
// 4-column groups of a block come into one LDS buffer by DMA loads (global
// -> LDS, no registers), kept as two contiguous [LB][4] groups; the block is
// transformed over n_b as 8 columns.  In the last stage every thread reads
// its inputs, the workgroup synchronises, the DMA of the next block is
// issued into the same buffer, and the last butterflies, the 2F reduction
// (eq. eq6 with the noise-weighted A', B', C') and the stores run while it
// is in flight.  Eight consecutive lanes hold the eight columns of one row,
// so each store covers 32 contiguous bytes of the output.

template <bool NT>
__device__ __forceinline__ void passb_dma(const PassBArgs& B, int unit, float4* dst) {
    const int t = unit / B.n_groups;
    const int c = unit - t * B.n_groups;
    const int blk = B.LB * kPassBCols;  // both groups of the block, contiguous in the spill
    const float4* base = B.spill + (int64_t)t * B.spill_tmpl_stride + (int64_t)c * blk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int e0 = wave * 64; e0 < blk; e0 += kNTB) {
        const int e = e0 + lane;
        if (e < blk) {
            // the spill is read once: non-temporal (cache policy nt) when it
            // was written so, else from the cache
            __builtin_amdgcn_global_load_lds((const void*)(base + e), (__attribute__((address_space(3))) void*)(dst + e0),
                                             16, 0, NT ? 2 : 0);
        }
    }
}

// 2F of the last stage's outputs: row k_b = j + r LB/R of column b of the
// block, bin k = 8c + b + LA k_b, reordered to the ascending band.
struct TwoFSink {
    float* out;
    int LA, LR, ka0, nf, s_lo, n_out;
    float cA, cB, cC;
    template <int R>
    __device__ __forceinline__ void put(int, int j, int b, cp (&v)[R]) {
        const int ka = ka0 + b;
        if (ka >= LA) return;
        const int hnf = (nf + 1) >> 1;  // k < hnf: non-negative signed bin
        const int kst = LA * LR;
        int k = ka + LA * j;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int o = ((k < hnf) ? k : k - nf) - s_lo;
            if ((unsigned)o < (unsigned)n_out) {
                const cp u = v[r];
                out[(unsigned)o] =
                    cA * (u.x * u.x + u.y * u.y) + cB * (u.z * u.z + u.w * u.w) + cC * (u.x * u.z + u.y * u.w);
            }
            k += kst;
        }
    }
};

template <bool NT>
struct PassBMid {
    const PassBArgs* B;
    int next;
    float4* buf;
    __device__ __forceinline__ void operator()() const {
        __syncthreads();  // every thread holds its last-stage inputs: the buffer is free
        if (next >= 0) passb_dma<NT>(*B, next, buf);
    }
};

template <bool NT>
__global__ __launch_bounds__(kNTB) void rsf_fft_pass_b_k(PassBArgs B) {
    extern __shared__ float4 lds[];
    const int blk = B.LB * kPassBCols;
    const int buf_elems = ((blk + 63) / 64) * 64;
    float2* twl = reinterpret_cast<float2*>(lds + buf_elems);
    const int n_hi = (B.LB + 31) >> kTwLoBits;
    float* cfl = reinterpret_cast<float*>(twl + 32 + n_hi);
    const int tid = threadIdx.x;
    for (int i = tid; i < 32 + n_hi; i += kNTB) twl[i] = (i < 32) ? B.tw_lo[i] : B.tw_hi[i - 32];
    for (int i = tid; i < 4 * B.n_sky_l; i += kNTB) cfl[i] = B.coef[i];
    const TwLds tw{twl, twl + 32};
    const Grouped4 lay{B.LB * kGroupCols};
    const int n_units = B.n_tmpl * B.n_groups;
    const int r_last = B.st.n_stages ? B.st.radix[B.st.n_stages - 1] : 1;

    int unit = blockIdx.x;
    if (unit < n_units) passb_dma<NT>(B, unit, lds);
    while (unit < n_units) {
        // this thread's DMA loads (and last block's stores) are complete;
        // after the barrier, everyone's
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int nunit = unit + (int)gridDim.x;
        const int t = unit / B.n_groups;
        const int c = unit - t * B.n_groups;
        const int s_l = t / B.nf_l;
        const int f = t - s_l * B.nf_l;
        const int64_t out_row = B.map_rows ? (int64_t)t : (B.sky0 + s_l) * B.n_fdot + B.f0 + f;
        TwoFSink sink{B.twoF + out_row * B.n_out, B.LA, B.LB / r_last, c * kPassBCols, (int)B.n_fft, (int)B.s_lo,
                      (int)B.n_out, cfl[4 * s_l], cfl[4 * s_l + 1], cfl[4 * s_l + 2]};
        const PassBMid<NT> mid{&B, nunit < n_units ? nunit : -1, lds};
        lds_fft_into<kNTB, kPassBEPT, kPassBCols, true>(lds, B.st, tw, lay, sink, mid);
        unit = nunit;
    }
}

int fft_pass_max_elems() { return kFftMaxLen < kNT * kEPT ? kFftMaxLen : kNT * kEPT; }

size_t fft_pass_a_lds(int LA) { return (size_t)LA * sizeof(float4) + (32 + (LA + 31) / 32) * sizeof(float2); }

hipError_t launch_fft_pass_a(const PassAArgs& a, hipStream_t s) {
    const size_t lds = fft_pass_a_lds(a.LA);
    const unsigned gy = (unsigned)(a.n_sky_l * ((a.nf_l + a.fb - 1) / a.fb));
    const dim3 grid((unsigned)a.LB, gy);
#define RSF_PASS_A(ORD)                                                              \
    if (a.nt_spill)                                                                  \
        hipLaunchKernelGGL((rsf_fft_pass_a_k<ORD, true>), grid, dim3(kNT), lds, s, a); \
    else                                                                             \
        hipLaunchKernelGGL((rsf_fft_pass_a_k<ORD, false>), grid, dim3(kNT), lds, s, a)
    switch (a.spin_order) {
        case 1: RSF_PASS_A(1); break;
        case 2: RSF_PASS_A(2); break;
        case 3: RSF_PASS_A(3); break;
        default: return hipErrorInvalidValue;
    }
#undef RSF_PASS_A
    return hipGetLastError();
}

size_t fft_pass_b_lds(int LB, int n_sky_l) {
    const size_t buf = (size_t)((LB * kPassBCols + 63) / 64) * 64;
    return buf * sizeof(float4) + (32 + (LB + 31) / 32) * sizeof(float2) + (size_t)4 * n_sky_l * sizeof(float);
}

hipError_t launch_fft_pass_b(const PassBArgs& b, int n_cu, hipStream_t s) {
    const size_t lds = fft_pass_b_lds(b.LB, b.n_sky_l);
    const int n_items = b.n_tmpl * b.n_groups;
    const unsigned grid = (unsigned)std::max(1, std::min(n_items, n_cu));
    if (b.nt_spill)
        hipLaunchKernelGGL(rsf_fft_pass_b_k<true>, dim3(grid), dim3(kNTB), lds, s, b);
    else
        hipLaunchKernelGGL(rsf_fft_pass_b_k<false>, dim3(grid), dim3(kNTB), lds, s, b);
    return hipGetLastError();
}

hipError_t fft_set_lds_limits(size_t bytes) {
    // the limit only ever grows: a smaller request from another plan must not
    // undo a larger one
    static size_t granted = 0;
    if (bytes <= granted) return hipSuccess;
    const void* fns[] = {(const void*)rsf_fft_pass_a_k<1, false>, (const void*)rsf_fft_pass_a_k<2, false>,
                         (const void*)rsf_fft_pass_a_k<3, false>, (const void*)rsf_fft_pass_a_k<1, true>,
                         (const void*)rsf_fft_pass_a_k<2, true>,  (const void*)rsf_fft_pass_a_k<3, true>,
                         (const void*)rsf_fft_pass_b_k<false>,    (const void*)rsf_fft_pass_b_k<true>};
    hipError_t out = hipSuccess;
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (out == hipSuccess) out = e;
    }
    if (out == hipSuccess) granted = bytes;
    return out;
}

}  // namespace rsf

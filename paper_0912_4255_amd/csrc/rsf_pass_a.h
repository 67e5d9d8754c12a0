// First pass of the two-pass FFT (paper Sec. III.A.2, steps 6-7; eqs.
// eq19, eq20): one workgroup per row n_b forms the integrands of F_a and F_b
// from the resampled series, transforms the row in LDS, applies the
// inter-pass twiddle and spills in 8-column groups.  Header-only so that the
// same kernel template serves the library's compiled-in plans and row plans
// compiled at run time for other radix sequences.
#pragma once

#include "rsf_device.h"
#include "rsf_spill.h"

namespace rsf {

constexpr int kRowThreads = kFftThreads;

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

// Inputs of one row held per thread: n_a = tid + q * kRowThreads, q < kInPer (P <= LA/2 <= 5120).
constexpr int kInPer = (kFftMaxLen / 2 + kRowThreads - 1) / kRowThreads;

// ---------------------------------------------------------------------------
// First-pass rows with the radix sequence fixed at compile time (RowPlan<R...>,
// radices in stage order, the upper half of the row zero).  Stage sizes are
// constants, so the butterfly index arithmetic and the LDS offsets fold into
// the instructions, and only the radices of the plan are compiled in.  The
// base twiddle W_{Ns R}^k of a middle-stage butterfly comes from a small
// per-stage table in LDS, its powers from complex products.  The plans in
// kFixedRows are compiled in; any other row runs the general stages.
// ---------------------------------------------------------------------------

// One middle (or first) stage of length L after Ns points, radix R; table
// tab = W_{Ns R}^k for k < Ns (unused when Ns = 1).  HZ: the upper half of
// the input is zero.
template <int L, int Ns, int R, bool HZ>
__device__ __forceinline__ void row_stage(cp* __restrict__ s, const float2* __restrict__ tab) {
    constexpr int LR = L / R;
    constexpr int MAXB = (LR + kRowThreads - 1) / kRowThreads;
    cp v[MAXB][R];
    const int tid = opaque_tid();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int j = tid + q * kRowThreads;
        if (q + 1 < MAXB || j < LR) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = (HZ && 2 * r >= R) ? make_float4(0.f, 0.f, 0.f, 0.f) : s[j + r * LR];
            if constexpr (Ns > 1) {
                const float2 w1 = tab[j % Ns];
                float2 w = w1;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    v[q][r] = cp_rot(v[q][r], w);
                    if (r + 1 < R) w = c_mul(w, w1);
                }
            }
            Dft<R>::run(v[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int j = tid + q * kRowThreads;
        if (q + 1 < MAXB || j < LR) {
            const int jq = j / Ns, k = j - jq * Ns;
            cp* p = s + (jq * Ns * R + k);
#pragma unroll
            for (int r = 0; r < R; ++r) p[r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// The last stage (Ns R = L): butterfly j reads x[j + r Ns], rotates input r
// by W_L^{j r} and hands its R outputs to the sink, in q order.
template <int L, int R, typename Sink>
__device__ __forceinline__ void row_last(const cp* __restrict__ s, const TwLds& tw, Sink& sink) {
    constexpr int LR = L / R;
    constexpr int MAXB = (LR + kRowThreads - 1) / kRowThreads;
    const int tid = opaque_tid();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int j = tid + q * kRowThreads;
        if (q + 1 < MAXB || j < LR) {
            cp v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = s[j + r * LR];
            bfly_dft<R, TwLds>(j, LR, 1, tw, v);
            sink.template put<R>(q, j, 0, v);
        }
    }
}

template <int L, int Ns, bool HZ, int R, int... Rest>
struct RowStages {
    template <typename Sink>
    __device__ __forceinline__ static void run(cp* __restrict__ s, const float2* __restrict__ tab, const TwLds& tw,
                                               Sink& sink) {
        if constexpr (sizeof...(Rest) == 0) {
            row_last<L, R>(s, tw, sink);
        } else {
            row_stage<L, Ns, R, HZ>(s, tab);
            RowStages<L, Ns * R, false, Rest...>::run(s, Ns > 1 ? tab + Ns : tab, tw, sink);
        }
    }
};

template <int... R>
struct RowPlan {
    static constexpr int kStages = sizeof...(R);
    static constexpr int kLen = (R * ...);
    // entries of the middle stages' base-twiddle tables (Ns of each)
    static constexpr int tab_entries() {
        constexpr int r[] = {R...};
        int ns = r[0], t = 0;
        for (int i = 1; i + 1 < kStages; ++i) {
            t += ns;
            ns *= r[i];
        }
        return t;
    }
    // table of middle stage i (Ns = r_0 .. r_(i-1)): W_{Ns r_i}^k, k < Ns,
    // from the two-level table
    __device__ __forceinline__ static void tables(float2* tab, const TwLds& tw) {
        constexpr int r[] = {R...};
        int off = 0, ns = r[0];
#pragma unroll
        for (int i = 1; i + 1 < kStages; ++i) {
            const int step = kLen / (ns * r[i]);
            for (int k = threadIdx.x; k < ns; k += kRowThreads) tab[off + k] = tw(k * step);
            off += ns;
            ns *= r[i];
        }
    }
    template <typename Sink>
    __device__ __forceinline__ static void fft(cp* __restrict__ s, const float2* __restrict__ tab, const TwLds& tw,
                                               Sink& sink) {
        RowStages<kLen, 1, true, R...>::run(s, tab, tw, sink);
    }
};

// The general stages, EPT complex pairs per thread.
template <int EPT>
struct GeneralStages {
    static constexpr int kFftEPT = EPT;
};

template <typename T>
struct IsRowPlan {
    static constexpr bool value = false;
};
template <int... R>
struct IsRowPlan<RowPlan<R...>> {
    static constexpr bool value = true;
};

// NT: the launch's spill is larger than the last-level cache (non-temporal stores)
// PLAN: a fixed row plan (RowPlan), or the planned stages of A.st
// (GeneralStages with kFftEPT or kFftEPTWide complex pairs per thread).
template <int ORDER, bool NT, typename PLAN>
__global__ __launch_bounds__(kRowThreads) void rsf_fft_pass_a_k(PassAArgs A) {
    extern __shared__ float4 lds[];
    // stage twiddles in LDS after the row: no global load inside the stages,
    // so the spill stores of one spindown stay in flight during the next FFT
    float2* twl = reinterpret_cast<float2*>(lds + A.LA);
    const int n_hi = (A.LA + 31) >> kTwLoBits;
    for (int i = threadIdx.x; i < 32 + n_hi; i += kRowThreads) twl[i] = (i < 32) ? A.tws_lo[i] : A.tws_hi[i - 32];
    const TwLds tws{twl, twl + 32};
    float2* tab = twl + 32 + n_hi;
    if constexpr (IsRowPlan<PLAN>::value) {
        __syncthreads();  // the two-level table is complete
        PLAN::tables(tab, tws);
    }
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
        const int n_a = tid + q * kRowThreads;
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
        const int64_t k = (int64_t)A.LB * (tid + q * kRowThreads) + n_b;
        p0[q] = unpack_sample<ORDER>(m0[q], tm0[q], A.f16, (double)k * A.dt, (float)A.w[0]);
    }
    // the upper half of the row is zero padding when P <= LA/2: the pruned
    // first stage reads only the rows below pruned_first_reach (LA/2 for an
    // even first radix), and only those are written
    const bool prune = 2 * A.P <= A.LA && A.st.n_stages > 1;
    const int zlim = prune ? pruned_first_reach(A.LA, A.st.radix[0]) : A.LA;

    // inter-pass twiddle W_N^{n_b k_a} for k_a = tid + q kRowThreads: base W^{n_b tid}, step W^{n_b kRowThreads}
    const int64_t mb = ((int64_t)n_b * tid) % A.n_fft;
    const int64_t ms = ((int64_t)n_b * kRowThreads) % A.n_fft;
    const int msk = (1 << kTwSplitBits) - 1;
    const float2 w_base = c_mul(A.tw_hi[mb >> kTwSplitBits], A.tw_lo[mb & msk]);
    const float2 w_step = c_mul(A.tw_hi[ms >> kTwSplitBits], A.tw_lo[ms & msk]);
    const int r_last = A.st.n_stages ? A.st.radix[A.st.n_stages - 1] : 1;
    const int lr = A.LA / r_last;
    const int64_t ml = ((int64_t)n_b * lr) % A.n_fft;
    const float2 w_lr = c_mul(A.tw_hi[ml >> kTwSplitBits], A.tw_lo[ml & msk]);

    // The spindowns are read as uniform values through the constant address
    // space (scalar loads, counted apart from the vector memory operations):
    // a vector load here would make the next template's first wait for it
    // also wait for every spill store of the template before.
    const __attribute__((address_space(4))) double* fdot_c =
        (const __attribute__((address_space(4))) double*)A.fdot;
    for (int f = f_lo; f < f_hi; ++f) {
        const int t = s_l * A.nf_l + f;
        Spin<ORDER> fd;
#pragma unroll
        for (int j = 0; j < ORDER; ++j) fd.f[j] = fdot_c[(int64_t)f * ORDER + j];
#pragma unroll
        for (int q = 0; q < kInPer; ++q) {
            const int n_a = tid + q * kRowThreads;
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
        for (int n_a = tid + kInPer * kRowThreads; n_a < zlim; n_a += kRowThreads) lds[n_a] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        SpillSink<NT> sink{reinterpret_cast<char*>(A.spill + (int64_t)t * A.spill_tmpl_stride), A.LB, n_b, lr,
                           w_base, w_step, w_lr};
        if constexpr (IsRowPlan<PLAN>::value)
            PLAN::fft(lds, tab, tws, sink);
        else
            lds_fft_into<kRowThreads, PLAN::kFftEPT, 1, false>(lds, A.st, tws, Interleaved<1>{}, sink, NoMid{}, prune);
        __syncthreads();
    }
}

}  // namespace rsf

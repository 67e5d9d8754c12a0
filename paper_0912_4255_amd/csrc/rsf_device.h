// Device helpers for librsfstat (gfx950): complex-pair arithmetic, small
// DFT butterflies with compile-time constants, and the analytic timing model.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsf_params.h"

namespace rsf {

// ---------------------------------------------------------------------------
// Compile-time sin/cos of 2 pi m / R (for butterfly constants).  Range
// reduction to [-pi/2, pi/2] and a Taylor series accurate to double precision.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_sin_series(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int n = 1; n < 14; ++n) {
        term *= -x2 / double((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double cx_sin(double x) {  // x in [-pi, pi]
    if (x > kPi / 2) x = kPi - x;
    else if (x < -kPi / 2) x = -kPi - x;
    return cx_sin_series(x);
}
constexpr double cx_wrap(double x) {  // to [-pi, pi]
    while (x > kPi) x -= 2 * kPi;
    while (x < -kPi) x += 2 * kPi;
    return x;
}
constexpr double cx_cos(double x) { return cx_sin(cx_wrap(x + kPi / 2)); }
constexpr double cx_angle(int m, int R) {  // 2 pi m / R reduced to (-pi, pi]
    int r = ((m % R) + R) % R;
    double f = double(r) / double(R);
    if (f > 0.5) f -= 1.0;
    return 2 * kPi * f;
}

// Forward roots W_R^m = exp(-2 pi i m / R): re = cos, im = -sin.
template <int R>
struct Roots {
    float re[R];
    float im[R];
    constexpr Roots() : re(), im() {
        for (int m = 0; m < R; ++m) {
            double a = cx_angle(m, R);
            double c = cx_cos(a), s = cx_sin(a);
            // exact values on the axes
            if (4 * m % R == 0) {
                int q = (4 * m / R) % 4;
                c = (q == 0) ? 1.0 : (q == 2 ? -1.0 : 0.0);
                s = (q == 1) ? 1.0 : (q == 3 ? -1.0 : 0.0);
            }
            re[m] = float(c);
            im[m] = float(-s);
        }
    }
};

// ---------------------------------------------------------------------------
// A complex pair (f_a, f_b) in one float4: (a.re, a.im, b.re, b.im).  Every
// butterfly of the FFT acts on both spectra with the same index arithmetic.
// ---------------------------------------------------------------------------
typedef float4 cp;

__device__ __forceinline__ cp cp_add(cp a, cp b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ __forceinline__ cp cp_sub(cp a, cp b) { return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }
__device__ __forceinline__ cp cp_scale(cp a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, a.w * s); }
// multiply both members by (c + i s)
__device__ __forceinline__ cp cp_rot(cp a, float c, float s) {
    return make_float4(a.x * c - a.y * s, a.x * s + a.y * c, a.z * c - a.w * s, a.z * s + a.w * c);
}
__device__ __forceinline__ cp cp_rot(cp a, float2 w) { return cp_rot(a, w.x, w.y); }
// multiply by -i
__device__ __forceinline__ cp cp_mul_mi(cp a) { return make_float4(a.y, -a.x, a.w, -a.z); }
// multiply by +i
__device__ __forceinline__ cp cp_mul_pi(cp a) { return make_float4(-a.y, a.x, -a.w, a.z); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Small forward DFTs, in place, natural order: y_k = sum_n x_n W_R^{nk}.
// ---------------------------------------------------------------------------
template <int R>
struct Dft;

template <>
struct Dft<1> {
    __device__ __forceinline__ static void run(cp*) {}
};

template <>
struct Dft<2> {
    __device__ __forceinline__ static void run(cp* x) {
        cp a = x[0], b = x[1];
        x[0] = cp_add(a, b);
        x[1] = cp_sub(a, b);
    }
};

template <>
struct Dft<3> {
    __device__ __forceinline__ static void run(cp* x) {
        constexpr float s3 = 0.866025403784438646763723170752936183f;  // sin(2 pi / 3)
        cp t1 = cp_add(x[1], x[2]);
        cp t2 = cp_sub(x[0], cp_scale(t1, 0.5f));
        cp t3 = cp_scale(cp_sub(x[1], x[2]), s3);
        x[0] = cp_add(x[0], t1);
        x[1] = cp_add(t2, cp_mul_mi(t3));
        x[2] = cp_sub(t2, cp_mul_mi(t3));
    }
};

template <>
struct Dft<4> {
    __device__ __forceinline__ static void run(cp* x) {
        cp s02 = cp_add(x[0], x[2]), d02 = cp_sub(x[0], x[2]);
        cp s13 = cp_add(x[1], x[3]), d13 = cp_mul_mi(cp_sub(x[1], x[3]));
        x[0] = cp_add(s02, s13);
        x[2] = cp_sub(s02, s13);
        x[1] = cp_add(d02, d13);
        x[3] = cp_sub(d02, d13);
    }
};

template <>
struct Dft<5> {
    __device__ __forceinline__ static void run(cp* x) {
        constexpr float c1 = float(cx_cos(2 * kPi / 5)), c2 = float(cx_cos(4 * kPi / 5));
        constexpr float s1 = float(cx_sin(2 * kPi / 5)), s2 = float(cx_sin(4 * kPi / 5));
        cp t1 = cp_add(x[1], x[4]), t2 = cp_add(x[2], x[3]);
        cp t3 = cp_sub(x[1], x[4]), t4 = cp_sub(x[2], x[3]);
        cp a1 = cp_add(x[0], cp_add(cp_scale(t1, c1), cp_scale(t2, c2)));
        cp a2 = cp_add(x[0], cp_add(cp_scale(t1, c2), cp_scale(t2, c1)));
        cp b1 = cp_add(cp_scale(t3, s1), cp_scale(t4, s2));
        cp b2 = cp_sub(cp_scale(t3, s2), cp_scale(t4, s1));
        x[0] = cp_add(x[0], cp_add(t1, t2));
        x[1] = cp_add(a1, cp_mul_mi(b1));
        x[4] = cp_sub(a1, cp_mul_mi(b1));
        x[2] = cp_add(a2, cp_mul_mi(b2));
        x[3] = cp_sub(a2, cp_mul_mi(b2));
    }
};

template <>
struct Dft<7> {
    __device__ __forceinline__ static void run(cp* x) {
        constexpr float c1 = float(cx_cos(2 * kPi / 7)), c2 = float(cx_cos(4 * kPi / 7)),
                        c3 = float(cx_cos(6 * kPi / 7));
        constexpr float s1 = float(cx_sin(2 * kPi / 7)), s2 = float(cx_sin(4 * kPi / 7)),
                        s3 = float(cx_sin(6 * kPi / 7));
        cp p1 = cp_add(x[1], x[6]), p2 = cp_add(x[2], x[5]), p3 = cp_add(x[3], x[4]);
        cp m1 = cp_sub(x[1], x[6]), m2 = cp_sub(x[2], x[5]), m3 = cp_sub(x[3], x[4]);
        // y_m = x0 + sum_k cos(2 pi k m/7) p_k - i sum_k sin(2 pi k m/7) m_k
        cp a1 = cp_add(x[0], cp_add(cp_scale(p1, c1), cp_add(cp_scale(p2, c2), cp_scale(p3, c3))));
        cp a2 = cp_add(x[0], cp_add(cp_scale(p1, c2), cp_add(cp_scale(p2, c3), cp_scale(p3, c1))));
        cp a3 = cp_add(x[0], cp_add(cp_scale(p1, c3), cp_add(cp_scale(p2, c1), cp_scale(p3, c2))));
        // sin(2 pi k m / 7) for (m, k): m=1: s1 s2 s3; m=2: s2 -s3 -s1; m=3: s3 -s1 s2
        cp b1 = cp_add(cp_scale(m1, s1), cp_add(cp_scale(m2, s2), cp_scale(m3, s3)));
        cp b2 = cp_sub(cp_scale(m1, s2), cp_add(cp_scale(m2, s3), cp_scale(m3, s1)));
        cp b3 = cp_add(cp_sub(cp_scale(m1, s3), cp_scale(m2, s1)), cp_scale(m3, s2));
        x[0] = cp_add(x[0], cp_add(p1, cp_add(p2, p3)));
        x[1] = cp_add(a1, cp_mul_mi(b1));
        x[6] = cp_sub(a1, cp_mul_mi(b1));
        x[2] = cp_add(a2, cp_mul_mi(b2));
        x[5] = cp_sub(a2, cp_mul_mi(b2));
        x[3] = cp_add(a3, cp_mul_mi(b3));
        x[4] = cp_sub(a3, cp_mul_mi(b3));
    }
};

// Composite radix R = P * Q in registers (Cooley-Tukey), in place: with
// n = Q n1 + n2 and k = k1 + P k2, P-point DFTs over n1 are written back to
// x[Q k1 + n2] times W_R^{n2 k1}; Q-point DFTs then run on the contiguous
// runs x[Q k1 .. Q k1 + Q-1], leaving y[k1 + P k2] at x[Q k1 + k2]; a final
// register permutation restores natural order.  Peak liveness R + P values.
template <int P, int Q>
struct DftCT {
    __device__ __forceinline__ static void run(cp* x) {
        constexpr int R = P * Q;
        constexpr Roots<R> w{};
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
            cp t[P];
#pragma unroll
            for (int n1 = 0; n1 < P; ++n1) t[n1] = x[Q * n1 + n2];
            Dft<P>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) {
                const int m = (n2 * k1) % R;
                x[Q * k1 + n2] = (m == 0) ? t[k1] : cp_rot(t[k1], w.re[m], w.im[m]);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) Dft<Q>::run(x + Q * k1);
        cp y[R];
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) y[k1 + P * k2] = x[Q * k1 + k2];
#pragma unroll
        for (int i = 0; i < R; ++i) x[i] = y[i];
    }
};

// x with x a = 1 (mod m), for a coprime to m
constexpr int inv_mod(int a, int m) {
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

// Composite radix R = P * Q with P, Q coprime (prime-factor algorithm), in
// place: with input index n = (Q n1 + P n2) mod R and output index
// k = (eP k1 + eQ k2) mod R, where eP = 1 (mod P), 0 (mod Q) and eQ = 0
// (mod P), 1 (mod Q), the kernel factors as W_R^{nk} = W_P^{n1 k1} W_Q^{n2 k2}:
// P-point DFTs over n1, then Q-point DFTs over n2, and no twiddle factors
// between them.  Both index maps are register permutations.
template <int P, int Q>
struct DftPFA {
    __device__ __forceinline__ static void run(cp* x) {
        constexpr int R = P * Q;
        constexpr int eP = Q * inv_mod(Q % P, P);
        constexpr int eQ = P * inv_mod(P % Q, Q);
        static_assert(eP % P == 1 % P && eP % Q == 0 && eQ % P == 0 && eQ % Q == 1 % Q, "P, Q not coprime");
        cp u[P][Q];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
            cp t[P];
#pragma unroll
            for (int n1 = 0; n1 < P; ++n1) t[n1] = x[(Q * n1 + P * n2) % R];
            Dft<P>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) u[k1][n2] = t[k1];
        }
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            Dft<Q>::run(u[k1]);
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) x[(eP * k1 + eQ * k2) % R] = u[k1][k2];
        }
    }
};

template <> struct Dft<6> : DftPFA<2, 3> {};
template <> struct Dft<8> : DftCT<2, 4> {};
template <> struct Dft<9> : DftCT<3, 3> {};
template <> struct Dft<10> : DftPFA<2, 5> {};
template <> struct Dft<12> : DftPFA<3, 4> {};
template <> struct Dft<14> : DftPFA<2, 7> {};
template <> struct Dft<15> : DftPFA<3, 5> {};
template <> struct Dft<16> : DftCT<4, 4> {};

// ---------------------------------------------------------------------------
// One Stockham stage of a batch of B transforms of length L kept in LDS
// (element (n, b) placed by a layout policy: interleaved columns, or groups
// of four).  Stage with radix R after Ns points have been combined:
// butterfly j reads n = j + r L/R, multiplies input r by
// W_{Ns R}^{r (j mod Ns)}, takes the R-point DFT and writes output r to
// (j div Ns) Ns R + (j mod Ns) + r Ns.  In place: all butterflies of the
// thread are read into registers, the block synchronises, then they are
// written.  tw(m) = W_L^m, and W_{Ns R}^{x} = W_L^{x L/(Ns R)}.
// ---------------------------------------------------------------------------
// q = j / d and r = j % d for 0 <= j < 2^22 from a float reciprocal: the
// product is off by at most one, which the correction step removes.
__device__ __forceinline__ void divmod_small(int j, int d, float inv_d, int& q, int& r) {
    q = (int)((float)j * inv_d);
    r = j - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
}

// Stage twiddles from a two-level table in LDS, W_L^m = lo[m % 32] * hi[m / 32].
struct TwLds {
    const float2* lo;  // 32 entries
    const float2* hi;  // ceil(L / 32) entries
    __device__ __forceinline__ float2 operator()(int m) const { return c_mul(lo[m & 31], hi[m >> 5]); }
};

// threadIdx.x behind an empty asm: offsets derived from it are recomputed
// at each use instead of being hoisted out of the callers' loops for every
// stage variant (where they would be spilled)
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Butterflies of radix R a thread holds in one stage (at least one); the
// planner keeps L * B / R <= stage_bfly(R, EPT) * NT.
template <int R, int EPT>
struct StageShape {
    static constexpr int MAXB = (EPT / R) > 0 ? (EPT / R) : 1;
};

// Element (row, column b) of a batch of B columns held in LDS: interleaved
// (row B + b), or in groups of four columns, group g a contiguous [row][4]
// block starting at g gs.
// Element index = row * rowstride() + col(b).
template <int B>
struct Interleaved {
    __device__ __forceinline__ static constexpr int rowstride() { return B; }
    __device__ __forceinline__ int col(int b) const { return b; }
    __device__ __forceinline__ int operator()(int row, int b) const { return row * B + b; }
};
struct Grouped8 {
    int gs;
    __device__ __forceinline__ static constexpr int rowstride() { return 8; }
    __device__ __forceinline__ int col(int b) const { return (b >> 3) * gs + (b & 7); }
    __device__ __forceinline__ int operator()(int row, int b) const { return row * 8 + col(b); }
};

// One butterfly of a Stockham stage: x[j + r L/R] of column b, r < R ...
// HZ: the upper half r >= R/2 is known to be zero (first stage of a
// zero-padded transform); it is not read, and the DFT folds it away.
template <int R, typename LAY, bool HZ = false>
__device__ __forceinline__ void bfly_load(const cp* __restrict__ s, int j, int b, int LR, const LAY& lay,
                                          cp (&v)[R]) {
    // element j + r LR of column b: one base and a uniform stride
    const cp* p = s + (j * LAY::rowstride() + lay.col(b));
    const int st = LR * LAY::rowstride();
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (HZ && 2 * r >= R) ? make_float4(0.f, 0.f, 0.f, 0.f) : p[r * st];
}
// ... times the stage twiddles W_{Ns R}^{k r} (k = j mod Ns), then the radix-R DFT.
template <int R, typename TW>
__device__ __forceinline__ void bfly_dft(int k, int Ns, int tstride, const TW& tw, cp (&v)[R]) {
    if (Ns > 1) {
        const float2 w1 = tw(k * tstride);
        float2 w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
            v[r] = cp_rot(v[r], w);
            if (r + 1 < R) w = c_mul(w, w1);
        }
    }
    Dft<R>::run(v);
}

// Read half of a Stockham stage: butterfly bf = tid + q NT (j = bf / B,
// column b = bf % B) leaves its R outputs in v[q] when bf < L B / R.
template <int R, int NT, int EPT, int B, typename TW, typename LAY, bool HZ = false>
__device__ __forceinline__ void stage_compute(const cp* __restrict__ s, int L, int Ns, const TW& tw, const LAY& lay,
                                              cp (&v)[StageShape<R, EPT>::MAXB][R]) {
    constexpr int MAXB = StageShape<R, EPT>::MAXB;
    const int tid = opaque_tid();
    const int LR = L / R;
    const int nb = LR * B;
    const int tstride = L / (Ns * R);
    const float inv_ns = 1.0f / (float)Ns;
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int bf = tid + q * NT;
        if (bf < nb) {
            const int j = (unsigned)bf / B, b = (unsigned)bf % B;
            int jq, k;
            divmod_small(j, Ns, inv_ns, jq, k);
            bfly_load<R, LAY, HZ>(s, j, b, LR, lay, v[q]);
            bfly_dft<R, TW>(k, Ns, tstride, tw, v[q]);
        }
    }
}

// One Stockham stage in place: all reads, a barrier, then the outputs of
// butterfly (j = jq Ns + k) go to x[jq Ns R + k + r Ns].
template <int R, int NT, int EPT, int B, typename TW, typename LAY, bool HZ = false>
__device__ __forceinline__ void stockham_stage(cp* __restrict__ s, int L, int Ns, const TW& tw, const LAY& lay) {
    constexpr int MAXB = StageShape<R, EPT>::MAXB;
    cp v[MAXB][R];
    stage_compute<R, NT, EPT, B, TW, LAY, HZ>(s, L, Ns, tw, lay, v);
    __syncthreads();
    const int tid = opaque_tid();
    const int nb = (L / R) * B;
    const float inv_ns = 1.0f / (float)Ns;
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int bf = tid + q * NT;
        if (bf < nb) {
            const int j = (unsigned)bf / B, b = (unsigned)bf % B;
            int jq, k;
            divmod_small(j, Ns, inv_ns, jq, k);
            const int base = jq * Ns * R + k;
            cp* p = s + (base * LAY::rowstride() + lay.col(b));
            const int st = Ns * LAY::rowstride();
#pragma unroll
            for (int r = 0; r < R; ++r) p[r * st] = v[q][r];
        }
    }
    __syncthreads();
}

// The last stage (Ns R = L) without the write back: output r of butterfly
// (j, b) is element j + r L/R of column b, and sink.put<R>(q, j, b, v)
// receives the R outputs of each valid butterfly, q in increasing order.
// SPLIT = false: one butterfly at a time (only R outputs live); the caller
// synchronises before the buffer is rewritten.  SPLIT = true: every input
// is read first, then mid() runs (all threads; it may synchronise and
// reuse the buffer), then the butterflies are computed and sunk.
template <int R, int NT, int EPT, int B, bool SPLIT, typename TW, typename LAY, typename Sink, typename Mid>
__device__ __forceinline__ void stockham_last(const cp* __restrict__ s, int L, int Ns, const TW& tw, const LAY& lay,
                                              Sink& sink, const Mid& mid) {
    constexpr int MAXB = StageShape<R, EPT>::MAXB;
    const int tid = opaque_tid();
    const int LR = L / R;
    const int nb = LR * B;
    const int tstride = L / (Ns * R);
    const float inv_ns = 1.0f / (float)Ns;
    if constexpr (SPLIT) {
        cp v[MAXB][R];
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int bf = tid + q * NT;
            if (bf < nb) {
                const int j = (unsigned)bf / B, b = (unsigned)bf % B;
                bfly_load<R, LAY>(s, j, b, LR, lay, v[q]);
            }
        }
        mid();
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int bf = tid + q * NT;
            if (bf < nb) {
                const int j = (unsigned)bf / B, b = (unsigned)bf % B;
                int jq, k;
                divmod_small(j, Ns, inv_ns, jq, k);
                bfly_dft<R, TW>(k, Ns, tstride, tw, v[q]);
                sink.template put<R>(q, j, b, v[q]);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int bf = tid + q * NT;
            if (bf < nb) {
                const int j = (unsigned)bf / B, b = (unsigned)bf % B;
                cp v[R];
                int jq, k;
                divmod_small(j, Ns, inv_ns, jq, k);
                bfly_load<R, LAY>(s, j, b, LR, lay, v);
                bfly_dft<R, TW>(k, Ns, tstride, tw, v);
                sink.template put<R>(q, j, b, v);
            }
        }
        mid();
    }
}

#define RSF_RADIX_CASES(M) \
    M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(12) M(14) M(15) M(16)

struct NoMid {
    __device__ __forceinline__ void operator()() const {}
};

// Rows of the input a pruned first stage of radix R reads: x[j + r L/R] for
// r < ceil(R/2) (the rest lie in the zero upper half).
__host__ __device__ inline int pruned_first_reach(int L, int R) { return (L / R) * ((R + 1) / 2); }

// Run all stages but the last of a planned transform in LDS, then the last
// one through sink (see stockham_last).  first_half_zero: every input at or
// above L/2 is zero; inputs at or above pruned_first_reach(L, radix[0]) are
// neither written nor read (pruned first stage, when there is more than one
// stage: input r of a radix-R butterfly, j + r L/R, lies at or above L/2
// for 2 r >= R).
template <int NT, int EPT, int B, bool SPLIT, typename TW, typename LAY, typename Sink, typename Mid>
__device__ __forceinline__ void lds_fft_into(cp* __restrict__ s, const FftStages& st, const TW& tw, const LAY& lay,
                                             Sink& sink, const Mid& mid, bool first_half_zero = false) {
    if (st.n_stages == 0) {  // length 1: the identity
        stockham_last<1, NT, EPT, B, SPLIT, TW, LAY, Sink, Mid>(s, st.len, 1, tw, lay, sink, mid);
        return;
    }
    int Ns = 1;
    int i0 = 0;
    if (first_half_zero && st.n_stages > 1) {
        switch (st.radix[0]) {
#define RSF_STAGE_HZ_CASE(RR) \
    case RR: stockham_stage<RR, NT, EPT, B, TW, LAY, true>(s, st.len, 1, tw, lay); break;
            RSF_RADIX_CASES(RSF_STAGE_HZ_CASE)
#undef RSF_STAGE_HZ_CASE
            default: break;
        }
        Ns = st.radix[0];
        i0 = 1;
    }
    for (int i = i0; i + 1 < st.n_stages; ++i) {
        const int R = st.radix[i];
        switch (R) {
#define RSF_STAGE_CASE(RR) \
    case RR: stockham_stage<RR, NT, EPT, B, TW, LAY>(s, st.len, Ns, tw, lay); break;
            RSF_RADIX_CASES(RSF_STAGE_CASE)
#undef RSF_STAGE_CASE
            default: break;
        }
        Ns *= R;
    }
    switch (st.radix[st.n_stages - 1]) {
#define RSF_LAST_CASE(RR) \
    case RR: stockham_last<RR, NT, EPT, B, SPLIT, TW, LAY, Sink, Mid>(s, st.len, Ns, tw, lay, sink, mid); break;
        RSF_RADIX_CASES(RSF_LAST_CASE)
#undef RSF_LAST_CASE
        default: break;
    }
}

// ---------------------------------------------------------------------------
// Analytic timing model (FP64).  Angles are 2 pi times the fractional number
// of revolutions, so large epochs keep full precision.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double frac_rev(double x) { return x - floor(x); }

struct SiteAngles {
    double sth, cth;  // local sidereal angle
};

// t_m(tau) = n0 . r_d(tau) / c; also returns sin/cos of the local sidereal angle.
__device__ __forceinline__ double roemer(double tau, const double3 n0, const EphDev& e, const DetDev& d,
                                         SiteAngles* ang) {
    const double lam = e.lambda0 + 2.0 * kPi * frac_rev(tau * e.inv_p_orb);
    const double th = e.theta0 + 2.0 * kPi * frac_rev(tau * e.inv_p_sid) + d.lon;
    double sl, cl, st, ct;
    sincos(lam, &sl, &cl);
    sincos(th, &st, &ct);
    ang->sth = st;
    ang->cth = ct;
    const double x = e.au_c * cl + e.re_c * d.clat * ct;
    const double y = e.au_c * e.ceps * sl + e.re_c * d.clat * st;
    const double z = e.au_c * e.seps * sl + e.re_c * d.slat;
    return n0.x * x + n0.y * y + n0.z * z;
}

// t_m(tau) with its first three time derivatives.  Both parts of r_d move
// on circles at uniform rates w, so per part the second derivative is
// -w^2 times the position and the third -w^2 times the velocity.
struct RoemerD {
    double tm, d1, d2, d3;
    SiteAngles ang;
};
__device__ __forceinline__ RoemerD roemer_d(double tau, const double3 n0, const EphDev& e, const DetDev& d) {
    const double lam = e.lambda0 + 2.0 * kPi * frac_rev(tau * e.inv_p_orb);
    const double th = e.theta0 + 2.0 * kPi * frac_rev(tau * e.inv_p_sid) + d.lon;
    double sl, cl, st, ct;
    sincos(lam, &sl, &cl);
    sincos(th, &st, &ct);
    const double wo = 2.0 * kPi * e.inv_p_orb, ws = 2.0 * kPi * e.inv_p_sid;
    const double po = e.au_c * (n0.x * cl + (n0.y * e.ceps + n0.z * e.seps) * sl);        // n0 . r_orb
    const double vo = wo * e.au_c * (-n0.x * sl + (n0.y * e.ceps + n0.z * e.seps) * cl);  // its rate
    const double rc = e.re_c * d.clat;
    const double pr = rc * (n0.x * ct + n0.y * st);  // rotating part in the equatorial plane
    const double vr = ws * rc * (-n0.x * st + n0.y * ct);
    RoemerD o;
    o.tm = po + pr + n0.z * e.re_c * d.slat;
    o.d1 = vo + vr;
    o.d2 = -wo * wo * po - ws * ws * pr;
    o.d3 = -wo * wo * vo - ws * ws * vr;
    o.ang.sth = st;
    o.ang.cth = ct;
    return o;
}

// Solution T of T + t_m(T) = t_b (eq. eq21): one fixed-point step from
// T = t_b, then one Newton step, T <- T - (T + t_m(T) - t_b) / (1 + t_m'(T)).
// The fixed-point step leaves |dT| <= |t_m'| |t_m| (about 0.05 s); the Newton
// step leaves about t_m'' dT^2 / 2, below 1e-12 s.  Also returns the
// expansion point (T1, t_m and derivatives there) and the sidereal angle
// carried to T.
struct Inversion {
    double T, T1;
    RoemerD r1;
    SiteAngles ang;
};
__device__ __forceinline__ Inversion invert_ssb(double t_start, double tb, const double3 n0, const EphDev& e,
                                                const DetDev& d) {
    SiteAngles g0;
    Inversion v;
    v.T1 = tb - roemer(t_start + tb, n0, e, d, &g0);
    v.r1 = roemer_d(t_start + v.T1, n0, e, d);
    const double dT = -(v.T1 + v.r1.tm - tb) / (1.0 + v.r1.d1);
    v.T = v.T1 + dT;
    // rotate the sidereal angle by w_sid dT (|w_sid dT| < 1e-5)
    const double a = 2.0 * kPi * e.inv_p_sid * dT;
    const double sa = a * (1.0 - a * a / 6.0), ca = 1.0 - 0.5 * a * a;
    v.ang.sth = v.r1.ang.sth * ca + v.r1.ang.cth * sa;
    v.ang.cth = v.r1.ang.cth * ca - v.r1.ang.sth * sa;
    return v;
}

// Circular binary orbit of the source: a wavefront emitted at tau_e reaches
// the SSB at tau_e + R(tau_e), R = a_p sin(2 pi (tau_e - t_asc) / P_b).
struct BinaryOrbit {
    double a_p, p_orb, t_asc;
};
// Orbits the timing code is built for: 0 <= a_p <= 100 light-s, finite
// P_b > 0 with 2 pi a_p / P_b <= 1e-2 (the contraction of the emission-time
// iteration), finite t_asc.  NaN fails every comparison and is refused.
__device__ __forceinline__ bool orbit_admitted(const BinaryOrbit& b) {
    return b.a_p >= 0.0 && b.a_p <= 100.0 && b.p_orb > 0.0 && b.p_orb < 1e300 &&
           2.0 * kPi * b.a_p <= 1e-2 * b.p_orb && fabs(b.t_asc) < 1e300;
}
// A refused orbit is replaced by this one (no delay) so that every loop and
// index stays well defined; the caller then writes NaN outputs.
__device__ __forceinline__ BinaryOrbit orbit_or_none(const BinaryOrbit& b) {
    return orbit_admitted(b) ? b : BinaryOrbit{0.0, 1.0, 0.0};
}
__device__ __forceinline__ double binary_delay(const BinaryOrbit& b, double tau_e) {
    const double cyc = (tau_e - b.t_asc) / b.p_orb;
    return b.a_p * sin(2.0 * kPi * (cyc - floor(cyc)));
}
// tau_e with tau_e + R(tau_e) = tau_ssb by the fixed point tau_e <- tau_ssb - R(tau_e):
// contraction 2 pi a_p / P_b (<= 1e-2 is required), at most 8 steps, stopping
// once a step changes nothing.
__device__ __forceinline__ double emission_time(const BinaryOrbit& b, double tau_ssb) {
    double te = tau_ssb;
    for (int it = 0; it < 8; ++it) {
        const double tn = tau_ssb - binary_delay(b, te);
        const bool done = tn == te;
        te = tn;
        if (done) break;
    }
    return te;
}

// Lane l's double, read into scalar registers (l must be wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ RoemerD readlane_rd(const RoemerD& q, int l) {
    RoemerD o;
    o.tm = readlane_d(q.tm, l);
    o.d1 = readlane_d(q.d1, l);
    o.d2 = readlane_d(q.d2, l);
    o.d3 = readlane_d(q.d3, l);
    return o;
}

// t_m at T1 + delta from the expansion at T1 (third order; the remainder is
// about w_sid^4 (R_E/c) delta^4 / 24, 3e-10 s for |delta| = 320 s).
__device__ __forceinline__ double tm_expand(const RoemerD& r, double delta) {
    return r.tm + delta * (r.d1 + delta * (0.5 * r.d2 + delta * (r.d3 * (1.0 / 6.0))));
}

__device__ __forceinline__ double3 sky_unit(double alpha, double delta) {
    double sa, ca, sd, cd;
    sincos(alpha, &sa, &ca);
    sincos(delta, &sd, &cd);
    return make_double3(cd * ca, cd * sa, sd);
}

// Beam patterns a = d:e+, b = d:ex from the local sidereal angle, using
// u^T e+ u = (u.p)^2 - (u.q)^2 and u^T ex u = 2 (u.p)(u.q).
struct SkyFrame {
    double3 p, q;
};
__device__ __forceinline__ SkyFrame sky_frame(double alpha, double delta) {
    double sa, ca, sd, cd;
    sincos(alpha, &sa, &ca);
    sincos(delta, &sd, &cd);
    SkyFrame f;
    f.p = make_double3(-sa, ca, 0.0);
    f.q = make_double3(-sd * ca, -sd * sa, cd);
    return f;
}
__device__ __forceinline__ void beam_ab(const SiteAngles& g, const DetDev& d, const SkyFrame& f,
                                        double* a, double* b) {
    const double3 eE = make_double3(-g.sth, g.cth, 0.0);
    const double3 eN = make_double3(-d.slat * g.cth, -d.slat * g.sth, d.clat);
    const double3 u = make_double3(d.cgu * eE.x + d.sgu * eN.x, d.cgu * eE.y + d.sgu * eN.y,
                                   d.cgu * eE.z + d.sgu * eN.z);
    const double3 v = make_double3(d.cgv * eE.x + d.sgv * eN.x, d.cgv * eE.y + d.sgv * eN.y,
                                   d.cgv * eE.z + d.sgv * eN.z);
    const double up = u.x * f.p.x + u.y * f.p.y + u.z * f.p.z;
    const double uq = u.x * f.q.x + u.y * f.q.y + u.z * f.q.z;
    const double vp = v.x * f.p.x + v.y * f.p.y + v.z * f.p.z;
    const double vq = v.x * f.q.x + v.y * f.q.y + v.z * f.q.z;
    *a = 0.5 * (up * up - uq * uq - vp * vp + vq * vq);
    *b = up * uq - vp * vq;
}

}  // namespace rsf

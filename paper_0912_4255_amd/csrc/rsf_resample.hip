// Barycentric resampling (paper Sec. III.A.2, steps 1-5) for gfx950.
//
// One workgroup (4 waves) resamples a 16 x 64 tile of the SSB grid
// k = LB * n_a + n_b (n_a = tile row, n_b = lane).  Each wave handles four
// runs of 64 consecutive k:
//   1. every lane inverts eq. eq21 for its k in FP64 (one fixed-point step
//      and one Newton step, residual below 1e-12 s).  For sampling intervals
//      short against a sidereal day (63 dt w_sid <= 4e-3, no orbit) the wave
//      instead inverts only lanes 0, 32 and 63 of its four runs, all twelve
//      at once, and every lane takes t_m, a and b from the quadratic through
//      its run's three: t_m, a and b are sums of circular motions with rates
//      up to 2 w_sid, so the remainder is at most 0.008 A (2 w_sid 63 dt)^3,
//      below 2e-11 s for t_m and 1e-9 for a and b;
//   2. the wave loads the detector-grid window its 64 outputs need into LDS,
//      applying the heterodyne correction z = x_h exp(-2 pi i f_h t_m) on the
//      way (eqs. absorb/Fa3; t_m at the detector samples from a third-order
//      expansion about the first lane's inversion, the phase f_h t_m reduced
//      mod 1 in FP64);
//   3. every lane interpolates z at T^k with the W-tap kernel in FP32;
//   4. a(T^k), b(T^k) come from the detector tensor in FP64, and the masked
//      antenna sums A', B', C' (eqs. eq9/eq10) accumulate in FP64.
// The tile is then written either in natural order (API outputs) or
// transposed to row n_b (the layout the first FFT pass reads contiguously).
#include <climits>

#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kTileB = 64;
constexpr int kTileA = 16;
constexpr int kThreads = 256;
constexpr int kWinMax = kTileB + kMaxTaps + 8;
constexpr float kPiF = 3.14159265358979323846f;

__device__ __forceinline__ bool in_gap(const int64_t* __restrict__ gaps, int n_gaps, int64_t j) {
    int lo = 0, hi = n_gaps - 1, best = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (gaps[2 * mid] <= j) {
            best = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    return best >= 0 && j < gaps[2 * best + 1];
}

__device__ __forceinline__ uint32_t pack_half2(float re, float im) {
    const __half2 h = __floats2half2_rn(re, im);
    return *reinterpret_cast<const uint32_t*>(&h);
}
}  // namespace

// BIN: the source is in a circular binary orbit; the grid is regular in
// emission time (target t_b + R(t_s + t_b) of the inversion) and the delay
// used by the correction and stored for the spindown phase is the total
// d = t_m - R(tau_e), tau_e from tau_e + R(tau_e) = tau + t_m(tau).
template <bool BIN>
__global__ __launch_bounds__(kThreads) void rsf_resample_k(ResampleArgs A) {
    __shared__ float2 win[4][kWinMax];
    __shared__ float4 tile_main[kTileA][kTileB + 1];
    __shared__ double tile_tm[kTileA][kTileB + 1];
    __shared__ uint32_t tile_mask[kTileA][2];
    __shared__ double red[4][3];
    // interpolated timing chain: per wave and run, t_m, a, b at lanes 0, 32, 63,
    // and lane 0's expansion point of t_m (the window's heterodyne correction)
    constexpr int kRuns = kTileA / 4;
    __shared__ double node_v[4][3][3 * kRuns];
    __shared__ RoemerD node_r1[4][kRuns];
    __shared__ double node_t1[4][kRuns];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int b0 = blockIdx.x * kTileB;
    const int64_t a0 = (int64_t)blockIdx.y * kTileA;
    const int sky = blockIdx.z;
    const double* srow = A.sky + (int64_t)A.sky_stride * sky;
    const double alpha = srow[0], delta = srow[1];
    BinaryOrbit bo{};
    bool orbit_ok = true;
    if constexpr (BIN) {
        const BinaryOrbit given{srow[2], srow[3], srow[4]};
        orbit_ok = orbit_admitted(given);
        bo = orbit_or_none(given);
    }
    const double3 n0 = sky_unit(alpha, delta);
    const SkyFrame fr = sky_frame(alpha, delta);
    const int W = A.ip.taps;
    const int hw = W / 2;
    const float pin = kPiF / (float)A.ip.n;  // pi / n of the Dirichlet kernel
    // Dirichlet kernel of a long series: |y| = pi |x| / n < pi (hw + 1) / n
    // keeps y / tan(y) (or y / sin(y)) within 1 + 3e-8, so in FP32 every
    // weight is sin(pi x) / (pi x) = (-1)^m sin(pi frac) / (pi x), m = hw - i
    const bool flat = A.ip.kernel == 1 && pin * (float)(hw + 1) < 2.9e-4f;
    double sA = 0.0, sB = 0.0, sC = 0.0;
    bool window_overflow = false;
    const bool fast = !BIN && A.fast_chain;
    if (fast) {
        // node m of run m / 3 sits at lane 0, 32 or 63 of that run
        if (lane < 3 * kRuns) {
            const int rr = lane / 3, which = lane - 3 * rr;
            const int64_t k = (int64_t)A.LB * (a0 + wave + 4 * rr) + b0 + (which == 0 ? 0 : which == 1 ? 32 : 63);
            const double tb = (double)k * A.dt;
            const Inversion inv = invert_ssb(A.t_start, tb, n0, A.eph, A.det);
            double av = 0.0, bv = 0.0;
            beam_ab(inv.ang, A.det, fr, &av, &bv);
            node_v[wave][0][lane] = tb - inv.T;
            node_v[wave][1][lane] = av;
            node_v[wave][2][lane] = bv;
            if (which == 0) {
                node_r1[wave][rr] = inv.r1;
                node_t1[wave][rr] = inv.T1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // value at lane l of the quadratic through (0, f0), (32, f32), (63, f63)
    auto quad = [lane](const double* f) {
        const double d1 = (f[1] - f[0]) * (1.0 / 32.0);
        const double d2 = ((f[2] - f[1]) * (1.0 / 31.0) - d1) * (1.0 / 63.0);
        const double l = (double)lane;
        return f[0] + l * d1 + l * (l - 32.0) * d2;
    };

    for (int r = 0; r < kTileA / 4; ++r) {
        const int ia = wave + 4 * r;
        const int64_t n_a = a0 + ia;
        const int n_b = b0 + lane;
        const int64_t k = (int64_t)A.LB * n_a + n_b;
        const bool valid = (n_b < A.LB) && (n_a < A.P) && (k < A.n);

        int j = 0;
        float frac = 0.f;
        double tm = 0.0, av = 0.0, bv = 0.0;
        bool mk = false;
        Inversion inv{};
        if (valid) {
            const double tb = (double)k * A.dt;
            double T;
            if (fast) {
                tm = quad(&node_v[wave][0][3 * r]);
                av = quad(&node_v[wave][1][3 * r]);
                bv = quad(&node_v[wave][2][3 * r]);
                T = tb - tm;
            } else {
                double target = tb;
                if constexpr (BIN) target = tb + binary_delay(bo, A.t_start + tb);
                inv = invert_ssb(A.t_start, target, n0, A.eph, A.det);
                T = inv.T;
                tm = tb - T;
                beam_ab(inv.ang, A.det, fr, &av, &bv);
            }
            const double u = T / A.dt;
            const double fl = floor(u);
            j = (int)fl;
            frac = (float)(u - fl);
            const int64_t jn = (int64_t)floor(u + 0.5);
            mk = (jn >= 0) && (jn < A.n) && !in_gap(A.gaps, A.n_gaps, jn);
        }
        // expansion point of t_m for this run's window: the first valid lane
        // (lane 0 whenever any lane is valid: it has the run's smallest k)
        const uint64_t vmask = __ballot(valid);
        const int src = vmask ? __ffsll((long long)vmask) - 1 : 0;
        const RoemerD rref = fast ? node_r1[wave][r] : readlane_rd(inv.r1, src);
        const double t_ref = fast ? node_t1[wave][r] : readlane_d(inv.T1, src);

        // window of detector samples needed by this run
        int jmin = valid ? j : INT_MAX;
        int jmax = valid ? j : INT_MIN;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            jmin = min(jmin, __shfl_xor(jmin, off));
            jmax = max(jmax, __shfl_xor(jmax, off));
        }
        const bool any = jmin != INT_MAX;
        const int w0 = any ? jmin - hw + 1 : 0;
        const int wlen = any ? (jmax - jmin + W) : 0;
        const bool ok = wlen <= kWinMax;
        if (any && ok) {
            for (int p = lane; p < wlen; p += 64) {
                const int64_t jj = (int64_t)w0 + p;
                float2 z = make_float2(0.f, 0.f);
                if (jj >= 0 && jj < A.n) {
                    const float2 xv = A.x[jj];
                    double tmj = tm_expand(rref, (double)jj * A.dt - t_ref);
                    if constexpr (BIN)
                        tmj -= binary_delay(bo, emission_time(bo, A.t_start + (double)jj * A.dt + tmj));
                    const double cyc = A.f_het * tmj;
                    const float ph = (float)(cyc - rint(cyc));
                    const float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);  // revolutions
                    z = make_float2(xv.x * c + xv.y * s, xv.y * c - xv.x * s);  // x * (c - i s)
                }
                win[wave][p] = z;
            }
        }
        if (any && !ok) window_overflow = true;
        // the window is this wave's own: its LDS operations complete in order,
        // so a wave-level barrier (no workgroup synchronisation) suffices
        __builtin_amdgcn_wave_barrier();

        float2 zt = make_float2(0.f, 0.f);
        if (valid) {
            if (ok && flat) {
                const int base = j - hw + 1 - w0;
                if (frac == 0.f || frac == 1.f) {
                    // x = 0 at one tap (the centre, or the next one when the
                    // fraction rounded up to 1 in FP32), sin(pi x) = 0 at the others
                    zt = win[wave][base + hw - 1 + (frac == 1.f ? 1 : 0)];
                } else {
                    // sum of (-1)^m z / x, then the common factor sin(pi frac) / pi
                    float ax = 0.f, ay = 0.f;
                    for (int i = 1; i <= W; ++i) {
                        const float x = frac + (float)(hw - i);
                        float r = __builtin_amdgcn_rcpf(x);
                        if ((hw - i) & 1) r = -r;
                        const float2 zz = win[wave][base + i - 1];
                        ax += r * zz.x;
                        ay += r * zz.y;
                    }
                    const float sc = sinpif(frac) * (1.0f / kPiF);
                    zt = make_float2(ax * sc, ay * sc);
                }
            } else if (ok) {
                const float sf = sinpif(frac);
                const int base = j - hw + 1 - w0;
                for (int i = 1; i <= W; ++i) {
                    const float x = frac + (float)(hw - i);
                    float w;
                    if (x == 0.f) {
                        w = 1.f;
                    } else {
                        const float sx = ((hw - i) & 1) ? -sf : sf;  // sin(pi x)
                        const float rx = __builtin_amdgcn_rcpf(kPiF * x);       // 1 / (pi x)
                        if (A.ip.kernel == 0) {
                            // sin(2 pi x / W) straight from x: x is exact (frac + integer) and
                            // an angle-addition form would cancel when x -> 0 off the centre tap
                            const float s2 = sinpif(2.f * x / (float)W);
                            w = sx * s2 * (0.5f * (float)W) * rx * rx;
                        } else {
                            // sin(pi x) / (n tan(pi x / n)) = sinc(x) g(y), y = pi x / n, with
                            // g = y / tan(y) (n even) or y / sin(y) (n odd), a series when small
                            const float y = x * pin;
                            float g;
                            if (fabsf(y) < 0.01f) {
                                const float y2 = y * y;
                                g = A.ip.n_odd ? 1.f + y2 * (1.f / 6.f + y2 * (7.f / 360.f))
                                               : 1.f - y2 * (1.f / 3.f + y2 * (1.f / 45.f));
                            } else {
                                g = A.ip.n_odd ? y / sinf(y) : y / tanf(y);
                            }
                            w = sx * rx * g;
                        }
                    }
                    const float2 zz = win[wave][base + i - 1];
                    zt.x += w * zz.x;
                    zt.y += w * zz.y;
                }
            } else {
                zt = make_float2(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000));
            }
            if (!orbit_ok) zt = make_float2(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000));
            if (mk) {
                sA += av * av;
                sB += bv * bv;
                sC += av * bv;
            }
        }
        if (A.f16) {
            tile_main[ia][lane] = valid ? make_float4(__uint_as_float(pack_half2(zt.x, zt.y)), (float)av,
                                                      (float)bv, (float)tm)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            tile_main[ia][lane] = valid ? make_float4(zt.x, zt.y, (float)av, (float)bv)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        tile_tm[ia][lane] = valid ? tm : 0.0;
        const uint64_t bal = __ballot(valid && mk);
        if (lane == 0) {
            tile_mask[ia][0] = (uint32_t)bal;
            tile_mask[ia][1] = (uint32_t)(bal >> 32);
        }
        __builtin_amdgcn_wave_barrier();  // the next run rewrites this wave's window
    }
    __syncthreads();  // the tile rows of all waves are complete

    if (window_overflow && lane == 0) atomicOr(A.flags, 2u);
    if (!orbit_ok && threadIdx.x == 0) atomicOr(A.flags, 4u);

    // write the tile
    if (A.layout == 1) {
        const int64_t sky_off = (int64_t)sky * A.rs_sky_stride;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nb_off = (threadIdx.x >> 4) + 16 * q;
            const int na_off = threadIdx.x & 15;
            const int n_b = b0 + nb_off;
            const int64_t n_a = a0 + na_off;
            if (n_b < A.LB && n_a < A.P) {
                const int64_t idx = sky_off + (int64_t)n_b * A.P + n_a;
                A.rs_main[idx] = tile_main[na_off][nb_off];
                if (!A.f16) A.rs_tm[idx] = (float)tile_tm[na_off][nb_off];
            }
        }
    } else {
        const int64_t sky_off = (int64_t)sky * A.n;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ia = (threadIdx.x >> 6) + 4 * q;
            const int64_t k = (int64_t)A.LB * (a0 + ia) + b0 + lane;
            if (b0 + lane < A.LB && a0 + ia < A.P && k < A.n) {
                const float4 m = tile_main[ia][lane];
                if (A.out_z) A.out_z[sky_off + k] = A.f16 ? make_float2(0.f, 0.f) : make_float2(m.x, m.y);
                if (A.out_zh) A.out_zh[sky_off + k] = __float_as_uint(m.x);
                if (A.out_a) A.out_a[sky_off + k] = A.f16 ? m.y : m.z;
                if (A.out_b) A.out_b[sky_off + k] = A.f16 ? m.z : m.w;
                if (A.out_tm) A.out_tm[sky_off + k] = tile_tm[ia][lane];
                if (A.out_u) A.out_u[sky_off + k] = ((double)k * A.dt - tile_tm[ia][lane]) / A.dt;
            }
        }
        if (A.out_mask && threadIdx.x < kTileA && A.LB == 64) {
            const int ia = threadIdx.x;
            const int64_t word = ((a0 + ia) * 64) / 32;
            const int64_t moff = (int64_t)sky * A.n_words;
            if (a0 + ia < A.P) {
                if (word < A.n_words) A.out_mask[moff + word] = tile_mask[ia][0];
                if (word + 1 < A.n_words) A.out_mask[moff + word + 1] = tile_mask[ia][1];
            }
        }
    }

    // antenna-sum partials, fixed reduction order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sA += __shfl_xor(sA, off);
        sB += __shfl_xor(sB, off);
        sC += __shfl_xor(sC, off);
    }
    if (lane == 0) {
        red[wave][0] = sA;
        red[wave][1] = sB;
        red[wave][2] = sC;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        const double tot = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        A.partials[((int64_t)sky * A.n_blocks + blk) * 3 + c] = tot;
    }
}

// One workgroup per sky: sums the block partials of every detector in a
// fixed order and forms the F-statistic coefficients 2B'/D', 2A'/D', -4C'/D'
// (eq. eq6 with noise-weighted sums) in FP64.
__global__ __launch_bounds__(256) void rsf_antenna_reduce_k(ReduceArgs R) {
    __shared__ double red[256][3];
    const int sky = blockIdx.x;
    double wsum[3] = {0.0, 0.0, 0.0};
    for (int X = 0; X < R.n_det; ++X) {
        double s[3] = {0.0, 0.0, 0.0};
        const double* p = R.partials + ((int64_t)X * R.n_sky + sky) * (int64_t)R.n_blocks * 3;
        for (int i = threadIdx.x; i < R.n_blocks; i += 256) {
            s[0] += p[3 * i + 0];
            s[1] += p[3 * i + 1];
            s[2] += p[3 * i + 2];
        }
        red[threadIdx.x][0] = s[0];
        red[threadIdx.x][1] = s[1];
        red[threadIdx.x][2] = s[2];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                red[threadIdx.x][0] += red[threadIdx.x + h][0];
                red[threadIdx.x][1] += red[threadIdx.x + h][1];
                red[threadIdx.x][2] += red[threadIdx.x + h][2];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (R.abc_det[X]) {
                double* o = R.abc_det[X] + (int64_t)sky * 3;
                o[0] = red[0][0];
                o[1] = red[0][1];
                o[2] = red[0][2];
            }
            wsum[0] += R.w[X] * red[0][0];
            wsum[1] += R.w[X] * red[0][1];
            wsum[2] += R.w[X] * red[0][2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double A = wsum[0], B = wsum[1], C = wsum[2];
        const double D = A * B - C * C;
        if (R.abc_w) {
            R.abc_w[3 * sky + 0] = A;
            R.abc_w[3 * sky + 1] = B;
            R.abc_w[3 * sky + 2] = C;
        }
        float* cf = R.coef + 4 * sky;
        if (D > 0.0 && A > 0.0 && B > 0.0) {
            cf[0] = (float)(2.0 * B / D);
            cf[1] = (float)(2.0 * A / D);
            cf[2] = (float)(-4.0 * C / D);
            cf[3] = 0.f;
        } else {
            const float nan = __int_as_float(0x7fc00000);
            cf[0] = cf[1] = cf[2] = nan;
            cf[3] = 1.f;
            atomicOr(R.flags, 1u);
        }
    }
}

hipError_t launch_resample(const ResampleArgs& a, int n_sky, hipStream_t s) {
    const unsigned gx = (unsigned)((a.LB + kTileB - 1) / kTileB);
    const unsigned gy = (unsigned)((a.P + kTileA - 1) / kTileA);
    if (a.binary)
        hipLaunchKernelGGL(rsf_resample_k<true>, dim3(gx, gy, (unsigned)n_sky), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(rsf_resample_k<false>, dim3(gx, gy, (unsigned)n_sky), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

int resample_blocks(int LB, int64_t P) {
    return ((LB + kTileB - 1) / kTileB) * (int)((P + kTileA - 1) / kTileA);
}

hipError_t launch_antenna_reduce(const ReduceArgs& r, hipStream_t s) {
    hipLaunchKernelGGL(rsf_antenna_reduce_k, dim3((unsigned)r.n_sky), dim3(256), 0, s, r);
    return hipGetLastError();
}

}  // namespace rsf

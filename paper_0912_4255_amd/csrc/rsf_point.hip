// 2F at continuous parameters and its gradient (project addition on top of
// paper Sec. III.A.2): for every candidate theta = (f, f^(1), ..., f^(s),
// alpha, delta) at spindown order s = 1..3 (followed by the orbit (a_p, P_b,
// t_asc) for a source in a circular binary orbit) the resampled series of the
// candidate's own sky is recomputed on the fly
// (never stored) and reduced to
//   F_a = sum_k y^a_k exp(-2 pi i (f - f_het) t_b^k),   F_b likewise,
//   A', B', C'  (masked antenna sums),
// plus, for the gradient, the derivatives of all five with respect to
// theta, following every dependence of the resampling chain:
//   * f:     d/df exp(-2 pi i (f - f_het) t_b) = -2 pi i t_b (...);
//   * f^(j): Phi_s = 2 pi sum_j f^(j) (T^(j+1)/(j+1)! + t_m T^j/j!)  (eq. eq4pt1),
//            which at s = 1 is pi fdot (t_b^2 - t_m^2) with T = t_b - t_m;
//   * sky:   t_m(tau) = n0 . r_d(tau) (eq. eq4pt2); the inversion of eq. eq21
//            gives dT/dtheta = -(dt_m/dtheta)/(1 + dt_m/dt); the
//            interpolated series changes through the kernel derivative
//            w'(u - p) dT/dtheta / dt and through the heterodyne correction
//            dz_p/dtheta = -2 pi i f_het (dt_m/dtheta)(t_p) z_p (eq. absorb);
//            the beam patterns change through p, q(alpha, delta) and T; the
//            spindown phase through T at fixed t_b:
//            dPhi_s/dT = 2 pi t_m sum_j f^(j) T^(j-1)/(j-1)!;
//   * orbit: the inversion targets t_b + R(tau_e) (tau_e = t_start + t_b on
//            the emission grid), so dT/dtheta_o = (dR/dtheta_o)/(1 + dt_m/dt);
//            t_m is replaced by the total delay d = t_m - R(tau_e) (equal to
//            t_b - T), and at a detector sample p the correction's delay
//            d_p = t_m(t_p) - R(tau_e,p) with tau_e,p + R(tau_e,p) = tau_p +
//            t_m(t_p) changes by -(dR/dtheta_o)/(1 + R') for the orbit and by
//            (dt_m/dtheta)/(1 + R') for the sky, R' = dR/dtau at tau_e,p.
// Each block accumulates FP64 partial sums over 8 tiles of 1024 samples;
// rsf_point_reduce_k sums the blocks of a candidate in a fixed order and
// forms 2F (eq. eq6) and the vector-Jacobian product g * d2F/dtheta.
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

// partial-sum slots at spindown order ORDER: NP = 1 + ORDER + NS parameters,
// the last NS of which (alpha, delta, and a_p, P_b, t_asc for a binary
// source) move the resampled times and hence also A', B', C'
template <int ORDER, bool BIN>
struct Slots {
    static constexpr int NS = BIN ? 5 : 2;
    static constexpr int NP = 1 + ORDER + NS;
    static constexpr int FA = 0, FB = 2, A = 4, B = 5, C = 6;
    static constexpr int DFA = 7;             // NP parameters x (re, im)
    static constexpr int DFB = DFA + 2 * NP;
    static constexpr int DA = DFB + 2 * NP;   // NS parameters each
    static constexpr int DB = DA + NS;
    static constexpr int DC = DB + NS;
    static constexpr int USED = DC + NS;
};
static_assert(Slots<3, true>::USED <= kPointSums, "partial-sum stride too small");

// R(tau_e) of a circular orbit, with cos of its angle for the derivatives
__device__ __forceinline__ double orbit_delay(const BinaryOrbit& b, double tau_e, double& s_phi, double& c_phi) {
    const double cyc = (tau_e - b.t_asc) / b.p_orb;
    sincos(2.0 * kPi * (cyc - floor(cyc)), &s_phi, &c_phi);
    return b.a_p * s_phi;
}

// tau_e with tau_e + R(tau_e) = tau by two Newton steps from tau - R(tau):
// the start is off by at most max R' times max R (at most 1e-2 a_p), and each
// step squares the error times (2 pi / P_b)^2 a_p / 2, so two steps reach
// rounding for every admitted orbit.  The angle's sin and cos at the result
// come from those of the last evaluation turned by the last step (first order).
__device__ __forceinline__ double emission_newton(const BinaryOrbit& b, double tau, double& s_phi, double& c_phi) {
    const double w = 2.0 * kPi / b.p_orb;
    double te = tau - orbit_delay(b, tau, s_phi, c_phi);
    double r = orbit_delay(b, te, s_phi, c_phi);
    te -= (te + r - tau) / (1.0 + b.a_p * w * c_phi);
    r = orbit_delay(b, te, s_phi, c_phi);
    const double d = (te + r - tau) / (1.0 + b.a_p * w * c_phi);
    te -= d;
    const double s = s_phi - c_phi * (w * d), c = c_phi + s_phi * (w * d);
    s_phi = s;
    c_phi = c;
    return te;
}

// dR/d(a_p, P_b, t_asc) at tau_e from the angle's sin and cos
__device__ __forceinline__ void orbit_partials(const BinaryOrbit& b, double tau_e, double s_phi, double c_phi,
                                               double* dR) {
    const double w = 2.0 * kPi / b.p_orb;
    dR[0] = s_phi;
    dR[1] = -b.a_p * c_phi * w * (tau_e - b.t_asc) / b.p_orb;
    dR[2] = -b.a_p * c_phi * w;
}

// 1/j! for the spindown terms
__device__ constexpr double kInvFact[5] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};

struct Orbit {
    double3 r;       // r_d / c (s)
    double3 v;       // v_d / c
    double sl, cl;   // orbital angle (the orbital part of r is AU/c (cl, ceps sl, seps sl))
    double sth, cth;
};

__device__ __forceinline__ Orbit orbit_at(double tau, const EphDev& e, const DetDev& d) {
    const double lam = e.lambda0 + 2.0 * kPi * frac_rev(tau * e.inv_p_orb);
    const double th = e.theta0 + 2.0 * kPi * frac_rev(tau * e.inv_p_sid) + d.lon;
    double sl, cl, st, ct;
    sincos(lam, &sl, &cl);
    sincos(th, &st, &ct);
    const double wo = 2.0 * kPi * e.inv_p_orb, ws = 2.0 * kPi * e.inv_p_sid;
    Orbit o;
    o.r = make_double3(e.au_c * cl + e.re_c * d.clat * ct, e.au_c * e.ceps * sl + e.re_c * d.clat * st,
                       e.au_c * e.seps * sl + e.re_c * d.slat);
    o.v = make_double3(-e.au_c * wo * sl - e.re_c * ws * d.clat * st, e.au_c * wo * e.ceps * cl + e.re_c * ws * d.clat * ct,
                       e.au_c * wo * e.seps * cl);
    o.sl = sl;
    o.cl = cl;
    o.sth = st;
    o.cth = ct;
    return o;
}

__device__ __forceinline__ double dot3(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// sin and cos of a small angle by their Taylor series through a^11 and
// a^10; for |a| <= 0.3 the first omitted terms are below 2e-15.
__device__ __forceinline__ void small_sincos(double a, double& s, double& c) {
    const double a2 = a * a;
    s = a * (1.0 - a2 * (1.0 / 6.0) *
                       (1.0 - a2 * (1.0 / 20.0) *
                                  (1.0 - a2 * (1.0 / 42.0) * (1.0 - a2 * (1.0 / 72.0) * (1.0 - a2 * (1.0 / 110.0))))));
    c = 1.0 - a2 * 0.5 *
                  (1.0 - a2 * (1.0 / 12.0) *
                             (1.0 - a2 * (1.0 / 30.0) * (1.0 - a2 * (1.0 / 56.0) * (1.0 - a2 * (1.0 / 90.0)))));
}

// (sin, cos) of x + a from those of x and a
__device__ __forceinline__ void rot_add(double sx, double cx, double sa, double ca, double& s, double& c) {
    s = sx * ca + cx * sa;
    c = cx * ca - sx * sa;
}

// Orbital and Greenwich sidereal angles at the first sample of the current
// run of a wave, as (sin, cos) pairs.  A wave's runs start 256 samples apart,
// so the pairs advance by a fixed rotation; a sample at tau_run + delta turns
// them by the small angles w delta, with |delta| <= 63 dt + max|t_m| (the
// host admits dt up to 55 s, which keeps w_sid |delta| below 0.3).
struct RunAngles {
    double sl, cl, sg, cg;
};

// The orbit of detector d at tau_run + delta.
__device__ __forceinline__ Orbit orbit_from(const RunAngles& ra, double delta, const EphDev& e, const DetDev& d,
                                            double wo, double ws) {
    double sa, ca, sb, cb, sl, cl, sg, cg, st, ct;
    small_sincos(wo * delta, sa, ca);
    small_sincos(ws * delta, sb, cb);
    rot_add(ra.sl, ra.cl, sa, ca, sl, cl);
    rot_add(ra.sg, ra.cg, sb, cb, sg, cg);
    rot_add(sg, cg, d.slon, d.clon, st, ct);  // local sidereal angle
    Orbit o;
    o.r = make_double3(e.au_c * cl + e.re_c * d.clat * ct, e.au_c * e.ceps * sl + e.re_c * d.clat * st,
                       e.au_c * e.seps * sl + e.re_c * d.slat);
    o.v = make_double3(-e.au_c * wo * sl - e.re_c * ws * d.clat * st, e.au_c * wo * e.ceps * cl + e.re_c * ws * d.clat * ct,
                       e.au_c * wo * e.seps * cl);
    o.sl = sl;
    o.cl = cl;
    o.sth = st;
    o.cth = ct;
    return o;
}

// m . r_d / c and its first three time derivatives at the orbit o (each
// part moves on a circle, so its second derivative is -w^2 times the
// position and the third -w^2 times the velocity); rez = R_E sin(lat) / c.
__device__ __forceinline__ RoemerD project(const Orbit& o, double3 m, const EphDev& e, double wo2, double ws2,
                                           double rez) {
    RoemerD q;
    q.tm = dot3(m, o.r);
    q.d1 = dot3(m, o.v);
    const double my = m.y * e.ceps + m.z * e.seps;
    const double pro = e.au_c * (m.x * o.cl + my * o.sl);
    const double pvo = sqrt(wo2) * e.au_c * (-m.x * o.sl + my * o.cl);
    const double prr = q.tm - pro - m.z * rez, pvr = q.d1 - pvo;
    q.d2 = -wo2 * pro - ws2 * prr;
    q.d3 = -wo2 * pvo - ws2 * pvr;
    return q;
}



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

// sinc(x) = sin(pi x)/(pi x) and its derivative from accurate sin(pi x), cos(pi x);
// a series near 0 avoids the cancellation in (cos(pi x) - sinc(x)) / x.
__device__ __forceinline__ void sinc_d(float x, float sx, float cx, float& s, float& ds) {
    if (fabsf(x) < 0.05f) {
        const float p2 = kPiF * kPiF * x * x;
        s = 1.f - p2 / 6.f + p2 * p2 / 120.f - p2 * p2 * p2 / 5040.f;
        ds = -(kPiF * kPiF * x / 3.f) * (1.f - p2 / 10.f + p2 * p2 / 280.f);
    } else {
        const float rx = __builtin_amdgcn_rcpf(x);
        s = sx * rx * (1.f / kPiF);
        ds = (cx - s) * rx;
    }
}

// Interpolation weight w(x) and w'(x) (Lanczos-W or the periodic Dirichlet
// kernel of length n written as sinc(x) g(pi x / n)); sx, cx = sin/cos(pi x).
template <bool GRAD>
__device__ __forceinline__ void kernel_w(const InterpDev& ip, float x, float sx, float cx, float& w, float& dw) {
    const int W = ip.taps;
    float s0, ds0;
    sinc_d(x, sx, cx, s0, ds0);
    if (ip.kernel == 0) {
        if (fabsf(x) >= 0.5f * (float)W) {
            w = 0.f;
            dw = 0.f;
            return;
        }
        const float v = 2.f * x / (float)W;
        float s1, ds1;
        const float sv = __builtin_amdgcn_sinf(0.5f * v), cv = __builtin_amdgcn_cosf(0.5f * v);  // revolutions
        sinc_d(v, sv, cv, s1, ds1);
        w = s0 * s1;
        if (GRAD) dw = ds0 * s1 + s0 * ds1 * (2.f / (float)W);
    } else {
        const float y = x * (kPiF / (float)ip.n);
        float g, dg;
        if (fabsf(y) < 0.01f) {
            const float y2 = y * y;
            if (ip.n_odd) {  // y / sin(y)
                g = 1.f + y2 / 6.f + 7.f * y2 * y2 / 360.f;
                dg = y / 3.f + 7.f * y * y2 / 90.f;
            } else {         // y / tan(y)
                g = 1.f - y2 / 3.f - y2 * y2 / 45.f;
                dg = -2.f * y / 3.f - 4.f * y * y2 / 45.f;
            }
        } else {
            float sy, cy;
            sincosf(y, &sy, &cy);
            if (ip.n_odd) {
                g = y / sy;
                dg = 1.f / sy - y * cy / (sy * sy);
            } else {
                g = y * cy / sy;
                dg = cy / sy - y / (sy * sy);
            }
        }
        w = s0 * g;
        if (GRAD) dw = ds0 * g + s0 * dg * (kPiF / (float)ip.n);
    }
}

// The sky's unit vector n0, its derivatives, and the polarisation basis
// (p, q) with the derivatives the gradient needs.
struct SkyGeom {
    double3 n0, n0a, n0d, pp, qq, pa, qa, qd;
};

// The timing chain of one resampled sample (eqs. eq4pt2, eq21 and the beam
// patterns of eq2, eq3), and for the gradient its sky (and orbit)
// derivatives.
struct ChainOut {
    double T1;                   // fixed-point iterate of T, the window's expansion point
    RoemerD x0, xa, xd;          // n0.r, n0_alpha.r, n0_delta.r and their time derivatives at T1
    double T, av, bv, dTa, dTd, daa, dad, dba, dbd;
    double dTo[3], dao[3], dbo[3];
};

// The chain at t_b = tb, a sample dl0 seconds after the first sample of its
// run (whose orbital and sidereal angles are ra): one fixed-point step and one
// Newton step of the inversion (residual below 1e-12 s), then the beam
// patterns at T.
template <bool GRAD, bool BIN>
__device__ __forceinline__ ChainOut chain_at(const PointArgs& A, const DetDev& D, const RunAngles& ra, double dl0,
                                             double tb, const SkyGeom& g, const BinaryOrbit& bo, double wo,
                                             double w_sid) {
    const double3 n0 = g.n0, n0a = g.n0a, n0d = g.n0d, pp = g.pp, qq = g.qq, pa = g.pa, qa = g.qa, qd = g.qd;
    ChainOut c{};
    // eq. eq21: one fixed-point step and one Newton step (residual below 1e-12 s)
    // a binary source's grid is regular in emission time: the
    // target is t_b + R(t_start + t_b)
    double tgt = tb, dRk[3] = {0.0, 0.0, 0.0};
    if constexpr (BIN) {
        double sp, cp;
        const double te = A.t_start + tb;
        tgt = tb + orbit_delay(bo, te, sp, cp);
        if (GRAD) orbit_partials(bo, te, sp, cp, dRk);
    }
    const double dl = dl0 + (BIN ? tgt - tb : 0.0);  // offset from the run's first sample
    const double tm0 = dot3(n0, orbit_from(ra, dl, A.eph, D, wo, w_sid).r);
    c.T1 = tgt - tm0;
    const Orbit o1 = orbit_from(ra, dl - tm0, A.eph, D, wo, w_sid);
    {
        const double wo2 = 4.0 * kPi * kPi * A.eph.inv_p_orb * A.eph.inv_p_orb;
        const double ws2 = w_sid * w_sid;
        const double rez = A.eph.re_c * D.slat;
        c.x0 = project(o1, n0, A.eph, wo2, ws2, rez);
        if (GRAD) {
            c.xa = project(o1, n0a, A.eph, wo2, ws2, rez);
            c.xd = project(o1, n0d, A.eph, wo2, ws2, rez);
        }
    }
    const double dT = -(c.T1 + dot3(n0, o1.r) - tgt) / (1.0 + dot3(n0, o1.v));
    c.T = c.T1 + dT;
    // the orbit at T: positions moved by v dT, the sidereal angle turned by w_sid dT
    Orbit o = o1;
    o.r = make_double3(o1.r.x + o1.v.x * dT, o1.r.y + o1.v.y * dT, o1.r.z + o1.v.z * dT);
    {
        const double a = w_sid * dT;
        const double sa = a * (1.0 - a * a / 6.0), ca = 1.0 - 0.5 * a * a;
        o.sth = o1.sth * ca + o1.cth * sa;
        o.cth = o1.cth * ca - o1.sth * sa;
    }
    // arms at the local sidereal angle, and their rate of change
    const double3 eE = make_double3(-o.sth, o.cth, 0.0);
    const double3 eN = make_double3(-D.slat * o.cth, -D.slat * o.sth, D.clat);
    const double3 eEt = make_double3(-o.cth, -o.sth, 0.0);
    const double3 eNt = make_double3(D.slat * o.sth, -D.slat * o.cth, 0.0);
    const double3 uu = make_double3(D.cgu * eE.x + D.sgu * eN.x, D.cgu * eE.y + D.sgu * eN.y,
                                    D.cgu * eE.z + D.sgu * eN.z);
    const double3 vv = make_double3(D.cgv * eE.x + D.sgv * eN.x, D.cgv * eE.y + D.sgv * eN.y,
                                    D.cgv * eE.z + D.sgv * eN.z);
    const double up = dot3(uu, pp), uq = dot3(uu, qq), vp = dot3(vv, pp), vq = dot3(vv, qq);
    c.av = 0.5 * (up * up - uq * uq - vp * vp + vq * vq);
    c.bv = up * uq - vp * vq;
    if (GRAD) {
        const double tmdot = dot3(n0, o.v);
        c.dTa = -dot3(n0a, o.r) / (1.0 + tmdot);
        c.dTd = -dot3(n0d, o.r) / (1.0 + tmdot);
        const double3 ut = make_double3(D.cgu * eEt.x + D.sgu * eNt.x, D.cgu * eEt.y + D.sgu * eNt.y, 0.0);
        const double3 vt = make_double3(D.cgv * eEt.x + D.sgv * eNt.x, D.cgv * eEt.y + D.sgv * eNt.y, 0.0);
        // d/dT through the sidereal rotation (per second)
        const double upt = dot3(ut, pp) * w_sid, uqt = dot3(ut, qq) * w_sid;
        const double vpt = dot3(vt, pp) * w_sid, vqt = dot3(vt, qq) * w_sid;
        const double adT = up * upt - uq * uqt - vp * vpt + vq * vqt;
        const double bdT = upt * uq + up * uqt - vpt * vq - vp * vqt;
        // d/dalpha, d/ddelta at fixed T through p and q
        const double upa = dot3(uu, pa), uqa = dot3(uu, qa), vpa = dot3(vv, pa), vqa = dot3(vv, qa);
        const double uqd = dot3(uu, qd), vqd = dot3(vv, qd);
        c.daa = up * upa - uq * uqa - vp * vpa + vq * vqa + adT * c.dTa;
        c.dba = upa * uq + up * uqa - vpa * vq - vp * vqa + bdT * c.dTa;
        c.dad = -uq * uqd + vq * vqd + adT * c.dTd;
        c.dbd = up * uqd - vp * vqd + bdT * c.dTd;
        if constexpr (BIN) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                c.dTo[i] = dRk[i] / (1.0 + tmdot);
                c.dao[i] = adT * c.dTo[i];
                c.dbo[i] = bdT * c.dTo[i];
            }
        }
    }
    return c;
}

// Per-run interpolation of the chain (used when the run is short against a
// sidereal day): the quantities that vary along a run of 64 samples (t_m,
// a, b and, for the gradient, dT/dalpha, dT/ddelta and the sky derivatives of
// a and b) are evaluated exactly at lanes 0, 32 and 63 and every lane takes
// the quadratic through them, q(l) = q_0 + l d_1 + l (l - 32) d_2.  Each
// quantity is a sum of circular motions with rate w <= 2 w_sid (the orbital
// rate is 366 times smaller), so the remainder is at most 0.008 times the
// third derivative's bound times (63 dt)^3, i.e. 0.008 A (2 w_sid 63 dt)^3
// with A the amplitude: for 63 dt w_sid <= 4e-3 that is below 2e-11 s for
// t_m (A = R_E / c) and below 5e-9 for a, b and their derivatives.
constexpr int kChainQ = 9;                         // interpolated quantities
constexpr int kChainRef = 13;                      // T1 and the three expansions of lane 0
constexpr int kRunVals = 3 * kChainQ + kChainRef;  // per run: q_0, d_1, d_2, then the reference
constexpr int kWaveRuns = kPointTiles * (kTileA / 4);

}  // namespace

// The binary gradient's 50 to 58 FP64 partial sums do not fit beside the rest
// at two waves per SIMD; at one wave per SIMD its spills go to the
// accumulation registers instead of scratch memory.
// FAST: one detector, no orbit, runs short against a sidereal day: the
// chain of each run is interpolated from three exact nodes.
template <bool GRAD, int ORDER, bool BIN, bool FAST>
__global__ __launch_bounds__(kThreads, (BIN && GRAD) ? 1 : 2) void rsf_point_k(PointArgs A) {
    using SL = Slots<ORDER, BIN>;
    constexpr int NP = SL::NP;
    constexpr int S_FA = SL::FA, S_FB = SL::FB, S_A = SL::A, S_B = SL::B, S_C = SL::C;
    constexpr int S_DFA = SL::DFA, S_DFB = SL::DFB, S_DA = SL::DA, S_DB = SL::DB, S_DC = SL::DC;
    constexpr int S_USED = SL::USED;
    constexpr int S_SKY = 2 * (1 + ORDER);  // offset of (alpha, delta) within S_DFA / S_DFB
    __shared__ float4 win[4][kWinMax];  // z (re, im), 2 pi f_het dd_p/dalpha, 2 pi f_het dd_p/ddelta
    __shared__ float4 wino[4][(BIN && GRAD) ? kWinMax : 1];  // 2 pi f_het dd_p/d(a_p, P_b, t_asc)
    __shared__ double red[4][kPointSums];
    __shared__ double runs[4][FAST ? kWaveRuns : 1][FAST ? kRunVals : 1];
    static_assert(!(FAST && BIN), "the interpolated chain is for isolated sources");

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int cand = blockIdx.y;
    const double* th = A.theta + (int64_t)NP * cand;
    const double f = th[0], al = th[1 + ORDER], de = th[2 + ORDER];
    double fs[ORDER];  // f^(1) .. f^(ORDER)
#pragma unroll
    for (int i = 0; i < ORDER; ++i) fs[i] = th[1 + i];
    const double fd = fs[0];
    BinaryOrbit bo{};
    bool orbit_ok = true;
    if constexpr (BIN) {
        const BinaryOrbit given{th[3 + ORDER], th[4 + ORDER], th[5 + ORDER]};
        orbit_ok = orbit_admitted(given);
        bo = orbit_or_none(given);
    }
    double sa, ca, sd, cd;
    sincos(al, &sa, &ca);
    sincos(de, &sd, &cd);
    const double3 n0 = make_double3(cd * ca, cd * sa, sd);
    const double3 n0a = make_double3(-cd * sa, cd * ca, 0.0);
    const double3 n0d = make_double3(-sd * ca, -sd * sa, cd);
    const double3 pp = make_double3(-sa, ca, 0.0);
    const double3 qq = make_double3(-sd * ca, -sd * sa, cd);
    const double3 pa = make_double3(-ca, -sa, 0.0);          // dp/dalpha (dp/ddelta = 0)
    const double3 qa = make_double3(sd * sa, -sd * ca, 0.0);  // dq/dalpha
    const double3 qd = make_double3(-cd * ca, -cd * sa, -sd); // dq/ddelta
    const SkyGeom geo{n0, n0a, n0d, pp, qq, pa, qa, qd};
    const double w_sid = 2.0 * kPi * A.eph.inv_p_sid;
    const int W = A.ip.taps;
    const int hw = W / 2;
    // Dirichlet weights by their small-argument series when pi x / n < 0.01 on every tap
    const float pin = kPiF / (float)A.ip.n;
    const bool dir_series = A.ip.kernel == 1 && pin * (float)(hw + 1) < 0.01f;
    // ... and when pi x / n < 2.9e-4 on every tap, g = 1 and g' pi / n = 0 to
    // FP32 precision: the weights are sinc(x) and its derivative
    const bool dir_flat = A.ip.kernel == 1 && pin * (float)(hw + 1) < 2.9e-4f;

    double acc[S_USED];
#pragma unroll
    for (int i = 0; i < S_USED; ++i) acc[i] = 0.0;
    bool overflow = false;

    // angles at this wave's first run, and the rotation to the next run
    const double wo = 2.0 * kPi * A.eph.inv_p_orb;
    RunAngles ra;
    double s_dl, c_dl, s_dg, c_dg;
    {
        const int64_t k_first = ((int64_t)blockIdx.x * kPointTiles * kTileA + wave) * kTileB;
        const double tau0 = A.t_start + (double)k_first * A.dt;
        sincos(A.eph.lambda0 + 2.0 * kPi * frac_rev(tau0 * A.eph.inv_p_orb), &ra.sl, &ra.cl);
        sincos(A.eph.theta0 + 2.0 * kPi * frac_rev(tau0 * A.eph.inv_p_sid), &ra.sg, &ra.cg);
        const double dtau = 4.0 * kTileB * A.dt;
        sincos(wo * dtau, &s_dl, &c_dl);
        sincos(w_sid * dtau, &s_dg, &c_dg);
    }

    if constexpr (FAST) {
        // nodes: lanes 0, 32, 63 of each of this wave's runs (run rr is row
        // wave + 4 (rr % 4) of tile rr / 4), the chain evaluated exactly
        const DetDev& D = A.det[0];
        for (int nd = lane; nd < 3 * kWaveRuns; nd += 64) {
            const int rr = nd / 3, m = nd - 3 * (nd / 3);
            const int off = m == 0 ? 0 : (m == 1 ? 32 : 63);
            const int64_t row = ((int64_t)blockIdx.x * kPointTiles + rr / 4) * kTileA + wave + 4 * (rr % 4);
            const double tau_run = A.t_start + (double)(row * kTileB) * A.dt;
            RunAngles rn;
            sincos(A.eph.lambda0 + 2.0 * kPi * frac_rev(tau_run * A.eph.inv_p_orb), &rn.sl, &rn.cl);
            sincos(A.eph.theta0 + 2.0 * kPi * frac_rev(tau_run * A.eph.inv_p_sid), &rn.sg, &rn.cg);
            const double tb = (double)(row * kTileB + off) * A.dt;
            const ChainOut c = chain_at<GRAD, false>(A, D, rn, (double)off * A.dt, tb, geo, bo, wo, w_sid);
            double* v = runs[wave][rr] + m * kChainQ;
            v[0] = tb - c.T;
            v[1] = c.av;
            v[2] = c.bv;
            v[3] = c.dTa;
            v[4] = c.dTd;
            v[5] = c.daa;
            v[6] = c.dad;
            v[7] = c.dba;
            v[8] = c.dbd;
            if (m == 0) {
                double* rf = runs[wave][rr] + 3 * kChainQ;
                rf[0] = c.T1;
                rf[1] = c.x0.tm;
                rf[2] = c.x0.d1;
                rf[3] = c.x0.d2;
                rf[4] = c.x0.d3;
                rf[5] = c.xa.tm;
                rf[6] = c.xa.d1;
                rf[7] = c.xa.d2;
                rf[8] = c.xa.d3;
                rf[9] = c.xd.tm;
                rf[10] = c.xd.d1;
                rf[11] = c.xd.d2;
                rf[12] = c.xd.d3;
            }
        }
        __syncthreads();
        // node values (q_0, q_32, q_63) to Newton coefficients (q_0, d_1, d_2)
        if (lane < kWaveRuns) {
            double* v = runs[wave][lane];
#pragma unroll
            for (int i = 0; i < kChainQ; ++i) {
                const double q0 = v[i], q32 = v[kChainQ + i], q63 = v[2 * kChainQ + i];
                const double d1 = (q32 - q0) * (1.0 / 32.0);
                v[kChainQ + i] = d1;
                v[2 * kChainQ + i] = ((q63 - q32) * (1.0 / 31.0) - d1) * (1.0 / 63.0);
            }
        }
        __syncthreads();
    }

    for (int tile = 0; tile < kPointTiles; ++tile) {
        const int64_t a0 = ((int64_t)blockIdx.x * kPointTiles + tile) * kTileA;
        for (int r = 0; r < kTileA / 4; ++r) {
            const int64_t row = a0 + wave + 4 * r;
            const int64_t k = row * kTileB + lane;
            const bool valid = (row < A.P) && (k < A.n);
            const double tb = (double)k * A.dt;
            for (int X = 0; X < A.n_det; ++X) {
                const DetDev& D = A.det[X];
                int j = 0;
                float frac = 0.f;
                double T = tb, tm = 0.0;
                bool mk = false;
                ChainOut c{};
                double t_ref;
                RoemerD q0, qa{}, qd{};
                if constexpr (FAST) {
                    // the run's quadratic through its nodes at lanes 0, 32, 63
                    const double* nd = runs[wave][tile * (kTileA / 4) + r];
                    const double l = (double)lane, b = l * (l - 32.0);
                    auto at = [&](int i) { return nd[i] + l * nd[kChainQ + i] + b * nd[2 * kChainQ + i]; };
                    tm = at(0);
                    c.av = at(1);
                    c.bv = at(2);
                    if (GRAD) {
                        c.dTa = at(3);
                        c.dTd = at(4);
                        c.daa = at(5);
                        c.dad = at(6);
                        c.dba = at(7);
                        c.dbd = at(8);
                    }
                    const double* rf = nd + 3 * kChainQ;
                    t_ref = rf[0];
                    q0 = RoemerD{rf[1], rf[2], rf[3], rf[4]};
                    if (GRAD) {
                        qa = RoemerD{rf[5], rf[6], rf[7], rf[8]};
                        qd = RoemerD{rf[9], rf[10], rf[11], rf[12]};
                    }
                    T = tb - tm;
                } else {
                    if (valid) {
                        c = chain_at<GRAD, BIN>(A, D, ra, (double)lane * A.dt, tb, geo, bo, wo, w_sid);
                        T = c.T;
                        tm = tb - T;
                    }
                    // expansion point of t_m (and of its sky derivatives) for the
                    // window: the first valid lane's fixed-point iterate
                    const uint64_t vmask = __ballot(valid);
                    const int src = vmask ? __ffsll((long long)vmask) - 1 : 0;
                    t_ref = readlane_d(c.T1, src);
                    q0 = readlane_rd(c.x0, src);
                    if (GRAD) {
                        qa = readlane_rd(c.xa, src);
                        qd = readlane_rd(c.xd, src);
                    }
                }
                if (valid) {
                    const double u = T / A.dt;
                    const double fl = floor(u);
                    j = (int)fl;
                    frac = (float)(u - fl);
                    const int64_t jn = (int64_t)floor(u + 0.5);
                    mk = (jn >= 0) && (jn < A.n) && !in_gap(A.gaps[X], A.n_gaps[X], jn);
                }
                const double av = c.av, bv = c.bv, dTa = c.dTa, dTd = c.dTd;
                const double daa = c.daa, dad = c.dad, dba = c.dba, dbd = c.dbd;
                const double* dTo = c.dTo;
                const double* dao = c.dao;
                const double* dbo = c.dbo;
                // detector-grid window of this run, heterodyne-corrected
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
                        float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
                        float4 eo = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (jj >= 0 && jj < A.n) {
                            const float2 xv = A.x[X][jj];
                            const double dl = (double)jj * A.dt - t_ref;
                            double tmj = tm_expand(q0, dl);
                            double inv1r = 1.0;  // 1 / (1 + R') at this sample's emission time
                            if constexpr (BIN) {
                                // total delay d_p = t_m - R(tau_e), tau_e + R(tau_e) = tau_p + t_m
                                double sp, cp;
                                const double te = emission_newton(bo, A.t_start + (double)jj * A.dt + tmj, sp, cp);
                                tmj -= bo.a_p * sp;
                                if (GRAD) {
                                    inv1r = 1.0 / (1.0 + bo.a_p * cp * (2.0 * kPi / bo.p_orb));
                                    double dR[3];
                                    orbit_partials(bo, te, sp, cp, dR);
                                    const double k = -2.0 * kPi * A.f_het * inv1r;
                                    eo = make_float4((float)(k * dR[0]), (float)(k * dR[1]), (float)(k * dR[2]), 0.f);
                                }
                            }
                            const double cyc = A.f_het * tmj;
                            const float ph = (float)(cyc - rint(cyc));
                            const float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);  // revolutions
                            e.x = xv.x * c + xv.y * s;
                            e.y = xv.y * c - xv.x * s;
                            if (GRAD) {
                                e.z = (float)(2.0 * kPi * A.f_het * tm_expand(qa, dl) * inv1r);
                                e.w = (float)(2.0 * kPi * A.f_het * tm_expand(qd, dl) * inv1r);
                            }
                        }
                        win[wave][p] = e;
                        if constexpr (BIN && GRAD) wino[wave][p] = eo;
                    }
                }
                if (any && !ok) overflow = true;
                // the window is this wave's own: its LDS operations complete in
                // order, so a wave-level barrier suffices
                __builtin_amdgcn_wave_barrier();
                if (valid && ok) {
                    // interpolation (and derivative pieces)
                    const float sf = __builtin_amdgcn_sinf(0.5f * frac), cf = __builtin_amdgcn_cosf(0.5f * frac);
                    float2 zt = make_float2(0.f, 0.f), s1 = zt, sza = zt, szd = zt;
                    float2 szo[3] = {zt, zt, zt};
                    const int base = j - hw + 1 - w0;
                    for (int i = 1; i <= W; ++i) {
                        const float x = frac + (float)(hw - i);
                        const bool odd = (hw - i) & 1;
                        const float sx = odd ? -sf : sf, cx = odd ? -cf : cf;  // sin, cos of pi x
                        float w, dw = 0.f;
                        if (x == 0.f) {
                            w = 1.f;
                            dw = 0.f;
                        } else if (dir_flat) {
                            sinc_d(x, sx, cx, w, dw);
                        } else if (dir_series) {
                            // Dirichlet kernel of a long series: sinc(x) g(y), y = pi x / n
                            // small, g = y / tan(y) (n even) or y / sin(y) (n odd) as a series
                            float s0, ds0;
                            sinc_d(x, sx, cx, s0, ds0);
                            const float y = x * pin, y2 = y * y;
                            const float g = A.ip.n_odd ? 1.f + y2 * (1.f / 6.f + y2 * (7.f / 360.f))
                                                       : 1.f - y2 * (1.f / 3.f + y2 * (1.f / 45.f));
                            w = s0 * g;
                            if (GRAD) {
                                const float dg = A.ip.n_odd ? y * (1.f / 3.f + y2 * (7.f / 90.f))
                                                            : -y * (2.f / 3.f + y2 * (4.f / 45.f));
                                dw = ds0 * g + s0 * dg * pin;
                            }
                        } else {
                            kernel_w<GRAD>(A.ip, x, sx, cx, w, dw);
                        }
                        const float4 zz = win[wave][base + i - 1];
                        zt.x += w * zz.x;
                        zt.y += w * zz.y;
                        if (GRAD) {
                            s1.x += dw * zz.x;
                            s1.y += dw * zz.y;
                            sza.x += w * zz.z * zz.x;
                            sza.y += w * zz.z * zz.y;
                            szd.x += w * zz.w * zz.x;
                            szd.y += w * zz.w * zz.y;
                            if constexpr (BIN) {
                                const float4 oo = wino[wave][base + i - 1];
                                szo[0].x += w * oo.x * zz.x;
                                szo[0].y += w * oo.x * zz.y;
                                szo[1].x += w * oo.y * zz.x;
                                szo[1].y += w * oo.y * zz.y;
                                szo[2].x += w * oo.z * zz.x;
                                szo[2].y += w * oo.z * zz.y;
                            }
                        }
                    }
                    // total phase: spindown Phi_s and the Fourier kernel at f;
                    // us[j] = T^(j+2)/(j+2)! + t_m T^(j+1)/(j+1)! (cycles per unit f^(j+1))
                    double us[ORDER];
                    double cyc;
                    if constexpr (ORDER == 1) {
                        cyc = fd * 0.5 * (tb * tb - tm * tm) + (f - A.f_het) * tb;
                    } else {
                        double Tj = T;  // T^(j+1)
                        cyc = (f - A.f_het) * tb;
#pragma unroll
                        for (int i = 0; i < ORDER; ++i) {
                            us[i] = Tj * T * kInvFact[i + 2] + tm * Tj * kInvFact[i + 1];
                            cyc += fs[i] * us[i];
                            Tj *= T;
                        }
                    }
                    const float ph = (float)(cyc - rint(cyc));
                    const float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);  // revolutions
                    // ze = z~ exp(-2 pi i cyc)
                    const float zer = zt.x * c + zt.y * s, zei = zt.y * c - zt.x * s;
                    const double w = D.w;
                    acc[S_FA + 0] += w * av * zer;
                    acc[S_FA + 1] += w * av * zei;
                    acc[S_FB + 0] += w * bv * zer;
                    acc[S_FB + 1] += w * bv * zei;
                    if (mk) {
                        acc[S_A] += w * av * av;
                        acc[S_B] += w * bv * bv;
                        acc[S_C] += w * av * bv;
                    }
                    if (GRAD) {
                        // d/df: -2 pi i t_b ; d/df^(j): -2 pi i us[j-1]
                        // (at order 1: -i pi (t_b^2 - t_m^2))
                        const double cf_ = 2.0 * kPi * tb;
                        // (-i c) (x + i y) = c y - i c x
                        acc[S_DFA + 0] += w * av * cf_ * zei;
                        acc[S_DFA + 1] -= w * av * cf_ * zer;
                        acc[S_DFB + 0] += w * bv * cf_ * zei;
                        acc[S_DFB + 1] -= w * bv * cf_ * zer;
                        // dPhi_s/dT / (2 pi t_m) = sum_j f^(j) T^(j-1)/(j-1)!
                        double rate;
                        if constexpr (ORDER == 1) {
                            const double cfd = kPi * (tb * tb - tm * tm);
                            acc[S_DFA + 2] += w * av * cfd * zei;
                            acc[S_DFA + 3] -= w * av * cfd * zer;
                            acc[S_DFB + 2] += w * bv * cfd * zei;
                            acc[S_DFB + 3] -= w * bv * cfd * zer;
                            rate = fd;
                        } else {
                            double Tj = 1.0;
                            rate = 0.0;
#pragma unroll
                            for (int i = 0; i < ORDER; ++i) {
                                const double cu = 2.0 * kPi * us[i];
                                acc[S_DFA + 2 + 2 * i] += w * av * cu * zei;
                                acc[S_DFA + 3 + 2 * i] -= w * av * cu * zer;
                                acc[S_DFB + 2 + 2 * i] += w * bv * cu * zei;
                                acc[S_DFB + 3 + 2 * i] -= w * bv * cu * zer;
                                rate += fs[i] * Tj * kInvFact[i];
                                Tj *= T;
                            }
                        }
                        // sky: dz~/dth = s1 dT/dth / dt - i sz_th ; dPhi/dth = dPhi_s/dT dT/dth
                        const float dTa_u = (float)(dTa / A.dt), dTd_u = (float)(dTd / A.dt);
                        const float dpa = (float)(2.0 * kPi * rate * tm * dTa);
                        const float dpd = (float)(2.0 * kPi * rate * tm * dTd);
                        // dz~_alpha = (s1.x dTa_u + sza.y, s1.y dTa_u - sza.x)
                        const float dza_r = s1.x * dTa_u + sza.y, dza_i = s1.y * dTa_u - sza.x;
                        const float dzd_r = s1.x * dTd_u + szd.y, dzd_i = s1.y * dTd_u - szd.x;
                        // rotate by exp(-2 pi i cyc)
                        const float ea_r = dza_r * c + dza_i * s, ea_i = dza_i * c - dza_r * s;
                        const float ed_r = dzd_r * c + dzd_i * s, ed_i = dzd_i * c - dzd_r * s;
                        // d(a ze)/dth = da ze + a (dz~ e) + a ze (-i dPhi)
                        acc[S_DFA + S_SKY + 0] += w * (daa * zer + av * ea_r + av * dpa * zei);
                        acc[S_DFA + S_SKY + 1] += w * (daa * zei + av * ea_i - av * dpa * zer);
                        acc[S_DFA + S_SKY + 2] += w * (dad * zer + av * ed_r + av * dpd * zei);
                        acc[S_DFA + S_SKY + 3] += w * (dad * zei + av * ed_i - av * dpd * zer);
                        acc[S_DFB + S_SKY + 0] += w * (dba * zer + bv * ea_r + bv * dpa * zei);
                        acc[S_DFB + S_SKY + 1] += w * (dba * zei + bv * ea_i - bv * dpa * zer);
                        acc[S_DFB + S_SKY + 2] += w * (dbd * zer + bv * ed_r + bv * dpd * zei);
                        acc[S_DFB + S_SKY + 3] += w * (dbd * zei + bv * ed_i - bv * dpd * zer);
                        if (mk) {
                            acc[S_DA + 0] += w * 2.0 * av * daa;
                            acc[S_DA + 1] += w * 2.0 * av * dad;
                            acc[S_DB + 0] += w * 2.0 * bv * dba;
                            acc[S_DB + 1] += w * 2.0 * bv * dbd;
                            acc[S_DC + 0] += w * (daa * bv + av * dba);
                            acc[S_DC + 1] += w * (dad * bv + av * dbd);
                        }
                        if constexpr (BIN) {
                            // the orbit moves T like the sky does, through dT/dtheta_o
#pragma unroll
                            for (int i = 0; i < 3; ++i) {
                                const float dTo_u = (float)(dTo[i] / A.dt);
                                const float dpo = (float)(2.0 * kPi * rate * tm * dTo[i]);
                                const float dz_r = s1.x * dTo_u + szo[i].y, dz_i = s1.y * dTo_u - szo[i].x;
                                const float eo_r = dz_r * c + dz_i * s, eo_i = dz_i * c - dz_r * s;
                                acc[S_DFA + S_SKY + 4 + 2 * i] += w * (dao[i] * zer + av * eo_r + av * dpo * zei);
                                acc[S_DFA + S_SKY + 5 + 2 * i] += w * (dao[i] * zei + av * eo_i - av * dpo * zer);
                                acc[S_DFB + S_SKY + 4 + 2 * i] += w * (dbo[i] * zer + bv * eo_r + bv * dpo * zei);
                                acc[S_DFB + S_SKY + 5 + 2 * i] += w * (dbo[i] * zei + bv * eo_i - bv * dpo * zer);
                                if (mk) {
                                    acc[S_DA + 2 + i] += w * 2.0 * av * dao[i];
                                    acc[S_DB + 2 + i] += w * 2.0 * bv * dbo[i];
                                    acc[S_DC + 2 + i] += w * (dao[i] * bv + av * dbo[i]);
                                }
                            }
                        }
                    }
                } else if (valid && !ok) {
                    acc[S_FA] = __longlong_as_double(0x7ff8000000000000LL);
                }
                __builtin_amdgcn_wave_barrier();  // the next run rewrites this wave's window
            }
            rot_add(ra.sl, ra.cl, s_dl, c_dl, ra.sl, ra.cl);
            rot_add(ra.sg, ra.cg, s_dg, c_dg, ra.sg, ra.cg);
        }
    }
    if (overflow && lane == 0) atomicOr(A.flags, 2u);
    if (!orbit_ok) {
        // a refused orbit: NaN 2F and gradient for this candidate
        acc[S_FA] = __longlong_as_double(0x7ff8000000000000LL);
        if (threadIdx.x == 0) atomicOr(A.flags, 4u);
    }

    // block reduction in a fixed order
    // unrolled: a loop-indexed acc would live in scratch memory
    constexpr int nsum = GRAD ? S_USED : S_DFA;
#pragma unroll
    for (int i = 0; i < nsum; ++i) {
        double v = acc[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < nsum) {
        const int i = threadIdx.x;
        const double t = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
        A.partials[((int64_t)cand * A.n_blocks + blockIdx.x) * kPointSums + i] = t;
    }
}

// One workgroup per candidate: fixed-order sum of the block partials, then
// 2F = 2Q/D with Q = B|Fa|^2 + A|Fb|^2 - 2C Re(Fa Fb^*), D = AB - C^2, and
// d2F = 2 (dQ D - Q dD) / D^2.
template <int ORDER, bool BIN>
__global__ __launch_bounds__(256) void rsf_point_reduce_k(PointReduceArgs R) {
    using SL = Slots<ORDER, BIN>;
    constexpr int NP = SL::NP;
    constexpr int S_FA = SL::FA, S_FB = SL::FB, S_A = SL::A, S_B = SL::B, S_C = SL::C;
    constexpr int S_DFA = SL::DFA, S_DFB = SL::DFB, S_DA = SL::DA, S_DB = SL::DB, S_DC = SL::DC;
    __shared__ double red[256];
    __shared__ double tot[kPointSums];
    const int cand = blockIdx.x;
    const int nsum = R.grad ? SL::USED : S_DFA;
    const double* p = R.partials + (int64_t)cand * R.n_blocks * kPointSums;
    for (int i = 0; i < nsum; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < R.n_blocks; b += 256) s += p[(int64_t)b * kPointSums + i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot[i] = red[0];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double Far = tot[S_FA], Fai = tot[S_FA + 1], Fbr = tot[S_FB], Fbi = tot[S_FB + 1];
    const double Aa = tot[S_A], Bb = tot[S_B], Cc = tot[S_C];
    const double D = Aa * Bb - Cc * Cc;
    const double fa2 = Far * Far + Fai * Fai, fb2 = Fbr * Fbr + Fbi * Fbi;
    const double reab = Far * Fbr + Fai * Fbi;
    const double Q = Bb * fa2 + Aa * fb2 - 2.0 * Cc * reab;
    const bool degenerate = !(D > 0.0);
    const double F2 = degenerate ? __longlong_as_double(0x7ff8000000000000LL) : 2.0 * Q / D;
    if (degenerate) atomicOr(R.flags, 1u);
    if (R.twoF) R.twoF[cand] = (float)F2;
    if (!R.grad) return;
    const double g = (double)R.g_twoF[cand];
    for (int i = 0; i < NP; ++i) {
        const double dar = tot[S_DFA + 2 * i], dai = tot[S_DFA + 2 * i + 1];
        const double dbr = tot[S_DFB + 2 * i], dbi = tot[S_DFB + 2 * i + 1];
        // the antenna sums depend only on the parameters that move T (the last NS)
        const int k = i - (NP - SL::NS);
        const double dA = (k >= 0) ? tot[S_DA + k] : 0.0;
        const double dB = (k >= 0) ? tot[S_DB + k] : 0.0;
        const double dC = (k >= 0) ? tot[S_DC + k] : 0.0;
        const double dQ = dB * fa2 + 2.0 * Bb * (Far * dar + Fai * dai) + dA * fb2 +
                          2.0 * Aa * (Fbr * dbr + Fbi * dbi) - 2.0 * dC * reab -
                          2.0 * Cc * (dar * Fbr + dai * Fbi + Far * dbr + Fai * dbi);
        const double dD = dA * Bb + Aa * dB - 2.0 * Cc * dC;
        const double d2F = degenerate ? F2 : 2.0 * (dQ * D - Q * dD) / (D * D);
        R.g_theta[(int64_t)NP * cand + i] = g * d2F;
    }
}

int point_blocks(int64_t P) { return (int)((P + kTileA * kPointTiles - 1) / (kTileA * kPointTiles)); }

hipError_t launch_point(const PointArgs& a, bool grad, hipStream_t s) {
    const dim3 grid((unsigned)a.n_blocks, (unsigned)a.n_cand);
#define RSF_POINT(G, O, B, F) hipLaunchKernelGGL((rsf_point_k<G, O, B, F>), grid, dim3(kThreads), 0, s, a)
    const bool fast = a.fast && !a.binary && a.n_det == 1;
    switch (a.order * 8 + (a.binary ? 4 : 0) + (fast ? 2 : 0) + (grad ? 1 : 0)) {
        case 8: RSF_POINT(false, 1, false, false); break;
        case 9: RSF_POINT(true, 1, false, false); break;
        case 10: RSF_POINT(false, 1, false, true); break;
        case 11: RSF_POINT(true, 1, false, true); break;
        case 12: RSF_POINT(false, 1, true, false); break;
        case 13: RSF_POINT(true, 1, true, false); break;
        case 16: RSF_POINT(false, 2, false, false); break;
        case 17: RSF_POINT(true, 2, false, false); break;
        case 18: RSF_POINT(false, 2, false, true); break;
        case 19: RSF_POINT(true, 2, false, true); break;
        case 20: RSF_POINT(false, 2, true, false); break;
        case 21: RSF_POINT(true, 2, true, false); break;
        case 24: RSF_POINT(false, 3, false, false); break;
        case 25: RSF_POINT(true, 3, false, false); break;
        case 26: RSF_POINT(false, 3, false, true); break;
        case 27: RSF_POINT(true, 3, false, true); break;
        case 28: RSF_POINT(false, 3, true, false); break;
        case 29: RSF_POINT(true, 3, true, false); break;
        default: return hipErrorInvalidValue;
    }
#undef RSF_POINT
    return hipGetLastError();
}

hipError_t launch_point_reduce(const PointReduceArgs& r, hipStream_t s) {
    const dim3 grid((unsigned)r.n_cand);
#define RSF_POINT_REDUCE(O, B) hipLaunchKernelGGL((rsf_point_reduce_k<O, B>), grid, dim3(256), 0, s, r)
    switch (r.order * 2 + (r.binary ? 1 : 0)) {
        case 2: RSF_POINT_REDUCE(1, false); break;
        case 3: RSF_POINT_REDUCE(1, true); break;
        case 4: RSF_POINT_REDUCE(2, false); break;
        case 5: RSF_POINT_REDUCE(2, true); break;
        case 6: RSF_POINT_REDUCE(3, false); break;
        case 7: RSF_POINT_REDUCE(3, true); break;
        default: return hipErrorInvalidValue;
    }
#undef RSF_POINT_REDUCE
    return hipGetLastError();
}

}  // namespace rsf

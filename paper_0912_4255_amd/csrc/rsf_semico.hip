// Semi-coherent combination of per-segment F-statistics: the hierarchical
// "stack-slide" scheme the paper's introduction names, as a plain sum of
// 2F along each template's frequency track.  Template (sky, f0, f^(1..s)),
// all at t_ref, sees f = f0 + sum_k f^(k) D^k / k! (D = t_seg - t_ref, the
// Taylor series of the frequency, eq. eq4) in a segment starting at t_seg
// (the segment's phase reference) and takes that segment's 2F at the nearest
// bin, floor((f - f_het) / df + 1/2), evaluated in FP64; bins outside the
// segment's band add nothing.  The segment demodulates with the spindowns
// moved to its start, f^(j)(t_seg) = sum_{k >= j} f^(k) D^(k-j) / (k-j)!
// (rsf_spin_translate_k).  One thread per (template, common-grid bin): each
// S element has one writer per call, and calls on one stream add in order.
#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kSemicoThreads = 256;
}

__global__ __launch_bounds__(kSemicoThreads) void rsf_semico_k(SemicoArgs a) {
    // separately rounded products and sums (no fused multiply-add), so that
    // the bin decision matches the same expression evaluated on the host
#pragma clang fp contract(off)
    const int64_t j = (int64_t)blockIdx.x * kSemicoThreads + threadIdx.x;
    const int t = blockIdx.y;
    if (j >= a.n_c) return;
    const int s_l = t / a.nf_l;
    const int f = t - s_l * a.nf_l;
    // the frequency's move from t_ref to t_seg, term by term in order of k
    const double* sp = a.fdot + (a.f0 + f) * a.order;
    const double D = a.t_seg - a.t_ref;
    double shift = sp[0] * D;
    if (a.order > 1) shift = shift + sp[1] * ((D * D) * 0.5);
    if (a.order > 2) shift = shift + sp[2] * (((D * D) * D) * (1.0 / 6.0));
    const double fj = (a.f_lo + (double)j * a.df_c) + shift;
    const int64_t s = (int64_t)floor((fj - a.f_het) / a.df + 0.5);
    const int64_t i = s - a.s_lo;
    if (i < 0 || i >= a.n_out) return;
    const int64_t row = (a.sky0 + s_l) * a.n_fdot + a.f0 + f;
    a.S[row * a.n_c + j] += a.map[(int64_t)t * a.n_out + i];
}

// One thread per template: (f^(1), ..., f^(order)) at t moved to t + D.
__global__ __launch_bounds__(kSemicoThreads) void rsf_spin_translate_k(const double* in, double* out, int64_t n,
                                                                       int order, double D) {
    const int64_t t = (int64_t)blockIdx.x * kSemicoThreads + threadIdx.x;
    if (t >= n) return;
    const double* f = in + t * order;
    for (int j = 0; j < order; ++j) {
        double acc = 0.0, p = 1.0;  // p = D^(k-j) / (k-j)!
        for (int k = j; k < order; ++k) {
            acc += f[k] * p;
            p *= D / (double)(k - j + 1);
        }
        out[t * order + j] = acc;
    }
}

hipError_t launch_spin_translate(const double* in, double* out, int64_t n, int order, double D, hipStream_t s) {
    const unsigned gx = (unsigned)((n + kSemicoThreads - 1) / kSemicoThreads);
    hipLaunchKernelGGL(rsf_spin_translate_k, dim3(gx), dim3(kSemicoThreads), 0, s, in, out, n, order, D);
    return hipGetLastError();
}

hipError_t launch_semico(const SemicoArgs& a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.n_c + kSemicoThreads - 1) / kSemicoThreads);
    hipLaunchKernelGGL(rsf_semico_k, dim3(gx, (unsigned)a.n_tmpl), dim3(kSemicoThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace rsf

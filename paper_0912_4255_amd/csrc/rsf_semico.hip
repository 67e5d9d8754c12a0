// Semi-coherent combination of per-segment F-statistics: the hierarchical
// "stack-slide" scheme the paper's introduction names, as a plain sum of
// 2F along each template's frequency track.  Template (sky, f0, fdot), f0 at
// t_ref, sees f = f0 + fdot (t_seg - t_ref) in a segment starting at t_seg
// (the segment's phase reference) and takes that segment's 2F at the nearest
// bin, floor((f - f_het) / df + 1/2), evaluated in FP64; bins outside the
// segment's band add nothing.  One thread per (template, common-grid bin):
// each S element has one writer per call, and calls on one stream add in
// order.
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
    const double shift = a.fdot[a.f0 + f] * (a.t_seg - a.t_ref);
    const double fj = (a.f_lo + (double)j * a.df_c) + shift;
    const int64_t s = (int64_t)floor((fj - a.f_het) / a.df + 0.5);
    const int64_t i = s - a.s_lo;
    if (i < 0 || i >= a.n_out) return;
    const int64_t row = (a.sky0 + s_l) * a.n_fdot + a.f0 + f;
    a.S[row * a.n_c + j] += a.map[(int64_t)t * a.n_out + i];
}

hipError_t launch_semico(const SemicoArgs& a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.n_c + kSemicoThreads - 1) / kSemicoThreads);
    hipLaunchKernelGGL(rsf_semico_k, dim3(gx, (unsigned)a.n_tmpl), dim3(kSemicoThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace rsf

// Launch parameters of the semi-coherent sum over segments.  Kept apart from
// the search's parameters.
#pragma once

#include "rsf_params.h"

namespace rsf {

// Semi-coherent sum: template t = s nf_l + f of a launch adds its 2F at the
// bin nearest f_lo + j df_c + sum_k f^(k) D^k / k! (D = t_seg - t_ref) to
// S[row][j].
struct SemicoArgs {
    const float* map;         // [n_tmpl][n_out] rows of the launch
    int64_t n_out, s_lo;
    double f_het, df;         // segment grid: bin s at f_het + s df
    double t_seg, t_ref;
    double f_lo, df_c;        // common grid
    int64_t n_c;
    const double* fdot;       // the call's spindowns at t_ref, [n_fdot][order]
    int order;                // spindown order s, 1..3
    int64_t sky0, n_fdot, f0;
    int nf_l, n_tmpl;
    float* S;                 // [n_sky * n_fdot][n_c], accumulated
};

}  // namespace rsf

// Launch parameters of the continuous-parameter 2F and its gradient (one
// detector set, a batch of candidates theta = (f, f^(1), ..., f^(s), alpha,
// delta) at spindown order s, followed by (a_p, P_b, t_asc) for a source in a
// circular binary orbit).  Kept apart from the search's parameters.
#pragma once

#include "rsf_params.h"

namespace rsf {

constexpr int kPointSums = 64;      // FP64 partial-sum stride per (block, candidate); at most 58 used
constexpr int kPointTiles = 8;      // 1024-sample tiles per block

struct PointArgs {
    int64_t n;
    double dt, t_start, f_het;
    EphDev eph;
    int n_det;
    DetDev det[kMaxDet];
    InterpDev ip;
    const float2* x[kMaxDet];
    const int64_t* gaps[kMaxDet];
    int n_gaps[kMaxDet];
    const double* theta;      // [n_cand][3 + order (+ 3 when binary)]
    int order;                // spindown order s, 1..3
    int binary;               // theta ends with a circular orbit (a_p, P_b, t_asc)
    int fast;                 // one detector, no orbit, 63 dt w_sid <= 4e-3: per-run interpolated chain
    int n_cand;
    int64_t P;                // 64-sample rows: ceil(n / 64)
    int n_blocks;             // blocks per candidate
    double* partials;         // [n_cand][n_blocks][kPointSums]
    unsigned int* flags;
};

struct PointReduceArgs {
    const double* partials;
    int n_blocks;
    int n_cand;
    int order;
    int binary;
    int grad;
    const float* g_twoF;      // [n_cand] (grad)
    float* twoF;              // [n_cand] (may be null)
    double* g_theta;          // [n_cand][3 + order (+ 3 when binary)] (grad)
    unsigned int* flags;
};

}  // namespace rsf

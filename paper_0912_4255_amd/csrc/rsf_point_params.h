// Launch parameters of the continuous-parameter 2F and its gradient (one
// detector set, a batch of candidates theta = (f, f^(1), ..., f^(s), alpha,
// delta) at spindown order s).  Kept apart from the search's parameters.
#pragma once

#include "rsf_params.h"

namespace rsf {

constexpr int kPointSums = 40;      // FP64 partial-sum stride per (block, candidate); 13 + 4 (3 + s) used
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
    const double* theta;      // [n_cand][3 + order]
    int order;                // spindown order s, 1..3
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
    int grad;
    const float* g_twoF;      // [n_cand] (grad)
    float* twoF;              // [n_cand] (may be null)
    double* g_theta;          // [n_cand][3 + order] (grad)
    unsigned int* flags;
};

}  // namespace rsf

// Launch parameters of the two front ends that produce the heterodyned,
// downsampled series: the time-domain one (filter and decimate a raw series)
// and the SFT one.  Kept apart from the search's parameters.
#pragma once

#include "rsf_params.h"

namespace rsf {

// Time-domain front end: x_h[j] = P_j sum_i g[i] x[j D + c - i], g the
// heterodyned low-pass taps, P_j = exp(-2 pi i f_h j D dt_raw).
struct HetdecArgs {
    const float* x;           // real raw series [n_raw]
    int64_t n_raw;
    const float2* g;          // [L] complex taps
    int L, c, D;
    double cyc_per_out;       // f_h D dt_raw (cycles per output sample)
    float2* out;              // [n_out]
    int64_t n_out;
};

// ---------------------------------------------------------------------------
// SFT front end (paper Sec. III.B)
// ---------------------------------------------------------------------------
constexpr int kSftMaxWindow = 511;  // longest running-median window
constexpr int kSftMaxTerms = 33;    // 2 dk + 1 Dirichlet terms at most
constexpr int kSftMaxGrid = 8192;   // SFTs of one chunk's transform grid M' (its roots sit in LDS)

// Running-median normalisation of SFT bands (eq. dimlessSFTs1).
struct SftNormArgs {
    const float2* in;   // [n_sft][K]
    float2* out;        // [n_sft][K]
    int K, w;           // bins per SFT, window (odd, <= K)
};

// One contiguous chunk of SFTs and its transform (device table).
struct SftChunkDev {
    int a0, M, Mp;        // first SFT, count, 7-smooth grid M' >= M
    int n;                // transform length B T_sft M'
    int64_t b0;           // long-baseline bin of relabelled bin 0: f_h T_sft M'
    int64_t y_off;        // first element of the chunk's band bins in y
    int64_t spill_off;    // first float4 of its spill
    int64_t j0, n_keep;   // output offset and kept samples
    int64_t blk0;         // first merge workgroup of the chunk
    int64_t dft_off;      // first element of its table Y[K][M'] in the DFT buffer
    int64_t dft_blk0;     // first workgroup of the chunk in the DFT launch
    int64_t fblk0;        // first workgroup of the chunk in the fused DFT and merge launch
    float scale;          // 1 / sqrt(n M)
    float2 corr;          // exp(-2 pi i f_h (t_c - t_s))
};

// Per chunk (one launch over all chunks), for every stored bin k and every
// r < M': Y[k][r] = sum_{alpha < M} X^_{a0+alpha, k} W_{M'}^{r alpha}, the
// M'-point DFT over the chunk's SFTs (missing ones zero) of each bin.
struct SftDftArgs {
    const float2* xh;     // normalised SFT bands [n_sft][K]
    int K;
    const SftChunkDev* chunks;
    int n_chunks;
    float2* Y;            // per chunk [K][M'] at dft_off
};

// Band bins of every chunk (one launch): bin m of chunk c is the
// long-baseline transform (eqs. e9/e91, kernel of eq. e75) at
// b = b0 + q (q = m below n/2, m - n above), times the Tukey window and the
// scale, conjugated (the inverse transform runs as a forward one on
// conjugates), at y[y_off + m].  With b = k* M' + r, the sum over SFTs and
// Dirichlet terms is taken as sum_d P_d(r) Y[k* + d][r].
struct SftMergeArgs {
    const float2* xh;     // normalised SFT bands [n_sft][K] (the fused DFT and merge)
    const float2* Y;      // the DFT tables of SftDftArgs (the separate merge)
    int K;
    int64_t k_lo;
    int dk;
    float taper;          // Tukey fraction over the band
    const SftChunkDev* chunks;
    int n_chunks;
    float2* y;
};

// One chunk transform length n = LA LB of the SFT front end.  Its chunks are
// ids[id0 .. id0 + nc), transformed in pairs (chunks 2i and 2i + 1 as the two
// complex halves of each float4; the last alone when nc is odd).  With R rows
// and C columns per workgroup (the same for every length of a plan), its
// workgroups in the single rows launch are rows_blk0 + i ceil(LB / R) + g
// (rows g R .. g R + R - 1 of its i-th pair), in the single columns launch
// cols_blk0 + i n_groups + g (columns g C .. g C + C - 1, n_groups =
// ceil(LA / C)); st1 and st2 are planned for R and C interleaved transforms.
struct SftLenDev {
    int64_t n;
    int LA, LB, n_groups, nc, id0;
    int64_t rows_blk0, cols_blk0;
    FftStages st1, st2;
    const float2* t1;       // W_LA^m = t1[m % 32] * t1_hi[m / 32]
    const float2* t1_hi;
    const float2* t2;       // W_LB^m = t2[m % 32] * t2_hi[m / 32]
    const float2* t2_hi;
    const float2* tw_lo;    // W_n^m = tw_hi[m >> 12] * tw_lo[m & 4095]
    const float2* tw_hi;
};

// Rows pass over every chunk (one launch): workgroup -> (length, chunk, n_b)
// through the length table; row n_b (elements m = LB n_a + n_b) is
// transformed over n_a and spilled with the inter-pass twiddle.
struct SftRowsArgs {
    const SftLenDev* lens;
    int n_lens;
    const SftChunkDev* chunks;
    const int* ids;
    const float2* y;
    float4* spill;
};

// Columns pass over every chunk (one launch): output j = k_a + LA k_b of a
// chunk; the first n_keep samples, conjugated, times the chunk's phase
// correction and the edge taper, go to x[j0 + j].
struct SftColsArgs {
    const SftLenDev* lens;
    int n_lens;
    const SftChunkDev* chunks;
    const int* ids;
    const float4* spill;
    float2* x;
    int64_t n_out;
    int n_edge;
};

}  // namespace rsf

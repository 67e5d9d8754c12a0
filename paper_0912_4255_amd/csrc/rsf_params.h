// Plain-old-data parameter blocks passed by value from the host launcher to
// the kernels of librsfstat.
#pragma once

#include <stdint.h>

#ifndef __HIP__
#include <hip/hip_runtime_api.h>
#endif
#include <hip/hip_vector_types.h>

namespace rsf {

constexpr int kMaxStages = 12;
constexpr int kMaxTaps = 32;
constexpr int kMaxDet = 4;
constexpr int kPassBCols = 8;       // columns of a second-pass block (two 4-column spill groups)
constexpr int kTwSplitBits = 12;    // inter-pass twiddle W_N^m = hi[m >> 12] * lo[m & 4095]
constexpr int kFftThreads = 512;    // threads of a first-pass workgroup
constexpr int kPassBThreads = 768;  // threads of a second-pass workgroup (3 waves per SIMD)
// complex pairs held per thread in a first-pass stage: 21 lets radix 3 and 7
// stages run 7 and 3 butterflies per thread (lengths with a factor 7 up to
// 10752); radices 2, 4, 5, 6, 8 ... 16 hold the same number as at 20
constexpr int kFftEPT = 21;
constexpr int kFftMaxLen = 10240;   // longest first-pass transform (10240 x 16 B = 160 KiB of LDS)

// Butterflies of radix R one thread holds in a stage: never more than EPT
// elements, so a stage of radix R covers at most fft_radix_cap(R) butterflies
// of a workgroup of NT threads.
constexpr int fft_bfly_per_thread(int R, int EPT) { return (EPT / R) > 0 ? (EPT / R) : 1; }
constexpr int fft_radix_cap(int R, int NT, int EPT) { return fft_bfly_per_thread(R, EPT) * NT; }

// Second pass: persistent workgroups, one per CU, transforming 8-column
// spill blocks in one LDS buffer filled by DMA loads; the stage capacity
// is kPassBEPT elements per thread (8 LB <= 512 x 21; 21 lets radix-7 stages
// hold 3 butterflies per thread).
constexpr int kPassBEPT = 21;
constexpr int kTwLoBits = 5;        // LDS twiddle table W_L^m = lo[m & 31] * hi[m >> 5]

struct FftStages {
    int len;
    int n_stages;
    int radix[kMaxStages];
};

struct EphDev {
    double au_c, re_c, inv_p_orb, inv_p_sid, ceps, seps, lambda0, theta0;
};

struct DetDev {
    double lon, clat, slat;
    double clon, slon;          // cos/sin of the longitude
    double cgu, sgu, cgv, sgv;  // cos/sin of the arm azimuths gamma +- pi/4
    double w;                   // 1 / sigma^2
};

// Interpolation kernel description.
struct InterpDev {
    int kernel;   // 0 Lanczos, 1 Dirichlet
    int taps;     // W (even)
    int n;        // series length (Dirichlet period)
    int n_odd;    // Dirichlet: sin instead of tan in the denominator
};

// Resampling kernel (one detector, a batch of sky positions).
struct ResampleArgs {
    int64_t n;
    double dt, t_start, f_het;
    EphDev eph;
    DetDev det;
    InterpDev ip;
    const float2* x;
    const int64_t* gaps;
    int n_gaps;
    const double* sky;        // [n_sky][sky_stride]: alpha, delta (, a_p, P_b, t_asc with a binary orbit)
    int sky_stride;           // 2, or 5 with a binary orbit
    int binary;
    // tile geometry: k = LB * n_a + n_b, 0 <= n_b < LB, 0 <= n_a < P
    int LB;
    int64_t P;
    int layout;               // 0: natural (API outputs), 1: FFT layout (internal)
    // natural-layout outputs, each with a per-sky stride of n (mask: n_words)
    float2* out_z;
    uint32_t* out_zh;         // half2 storage of z (if not null)
    float* out_a;
    float* out_b;
    double* out_tm;
    uint32_t* out_mask;
    int64_t n_words;
    // FFT-layout outputs: main = {z.re, z.im, a, b} (F32) or {z as half2, a, b, tm} (F16)
    float4* rs_main;
    float* rs_tm;
    int64_t rs_sky_stride;    // elements between skies
    int f16;
    // antenna-sum partials [n_sky][n_blocks][3]
    double* partials;
    int n_blocks;
    unsigned int* flags;
};

// Reduction of antenna-sum partials into F-statistic coefficients.
struct ReduceArgs {
    const double* partials;   // [n_det][n_sky][n_blocks][3]
    int n_blocks;
    int n_det;
    int n_sky;
    double w[kMaxDet];        // 1 / sigma_X^2
    double* abc_det[kMaxDet]; // per detector [n_sky][3] unweighted (each may be null)
    double* abc_w;            // [n_sky][3] weighted (may be null)
    float* coef;              // [n_sky][4] = 2B/D, 2A/D, -4C/D, degenerate flag
    unsigned int* flags;
};

// First FFT pass over the templates of one launch: n_sky_l sky positions
// (resampled series at rs_* + sky * rs_sky_stride) times nf_l spindowns
// (fdot[0..nf_l)).  Each workgroup transforms one input row n_b for up to fb
// spindowns of one sky, which share the row's inputs.  Template t = s nf_l + f.
struct PassAArgs {
    int64_t n, n_fft;
    double dt;
    int LA, LB;
    int64_t P;
    int n_det;
    double w[kMaxDet];
    const float4* rs_main[kMaxDet];
    const float* rs_tm[kMaxDet];
    int64_t rs_sky_stride;
    int f16;
    const double* fdot;       // [nf_l][spin_order]: f^(1) .. f^(spin_order) per template
    int spin_order;           // 1..3 (eq. eq4pt1)
    int nf_l;
    int n_sky_l;
    int fb;
    FftStages st;
    const float2* tws_lo;     // stage twiddles W_LA^m = tws_lo[m % 32] * tws_hi[m / 32]
    const float2* tws_hi;
    const float2* tw_lo;      // inter-pass twiddle W_N^m = tw_hi[m >> 12] * tw_lo[m & 4095]
    const float2* tw_hi;
    float4* spill;            // [n_sky_l * nf_l][2 * ceil(LA/8)][LB][4]: 4-column groups
    int64_t spill_tmpl_stride;
};

// Second FFT pass and F-statistic for the launch's n_sky_l * nf_l templates;
// template t = s nf_l + f goes to output row (sky0 + s) * n_fdot + f0 + f, or
// to row t of a scratch map (map_rows = 1).
struct PassBArgs {
    int64_t n_fft;
    int LA, LB;
    int n_groups;             // ceil(LA / 8)
    FftStages st;
    const float2* tw_lo;      // W_LB^m for m < 32
    const float2* tw_hi;      // W_LB^{32 m} for m < ceil(LB / 32)
    const float4* spill;
    int64_t spill_tmpl_stride;
    const float* coef;        // per sky of the launch {2B/D, 2A/D, -4C/D, flag}
    int n_sky_l;
    int64_t s_lo, n_out;
    float* twoF;
    int map_rows;
    int64_t sky0, n_fdot, f0;
    int nf_l;
    int n_tmpl;
};

// Top-k over a scratch map of 2F rows (template t = s nf_l + f of a launch):
// order by 2F descending, ties by the lower key (sky, fdot, bin) packed as
// ((sky * n_fdot) + fdot) * n_out + bin.
constexpr int kTopkMax = 64;
struct TopkItem {
    float v;
    int pad;
    unsigned long long key;
};

struct TopkScanArgs {
    const float* map;
    int64_t n_vals;           // rows * n_out
    int64_t n_out;
    int64_t sky0, n_fdot, f0;
    int nf_l;
    int k;
    TopkItem* cand;           // [gridDim.x][k]
};

struct TopkMergeArgs {
    const TopkItem* cand;     // n_cand items
    int64_t n_cand;
    const TopkItem* run_in;   // k items (may be null: start empty)
    TopkItem* run_out;        // k items (one-block grid)
    TopkItem* out_blocks;     // [gridDim.x][k] items (grids of several blocks)
    int k;
    int64_t n_fdot, n_out;
    void* entries;            // rsf_topk_entry[k] written if not null
};

// Continuous-parameter 2F and its gradient (one detector set, a batch of
// candidates theta = (f, fdot, alpha, delta)).
constexpr int kPointSums = 32;      // FP64 partial sums per (block, candidate)
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
    const double* theta;      // [n_cand][4]
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
    int grad;
    const float* g_twoF;      // [n_cand] (grad)
    float* twoF;              // [n_cand] (may be null)
    double* g_theta;          // [n_cand][4] (grad)
    unsigned int* flags;
};


// Semi-coherent sum: template t = s nf_l + f of a launch adds its 2F at the
// bin nearest f_lo + j df_c + fdot (t_seg - t_ref) to S[row][j].
struct SemicoArgs {
    const float* map;         // [n_tmpl][n_out] rows of the launch
    int64_t n_out, s_lo;
    double f_het, df;         // segment grid: bin s at f_het + s df
    double t_seg, t_ref;
    double f_lo, df_c;        // common grid
    int64_t n_c;
    const double* fdot;       // the call's spindowns
    int64_t sky0, n_fdot, f0;
    int nf_l, n_tmpl;
    float* S;                 // [n_sky * n_fdot][n_c], accumulated
};

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
    const float2* Y;      // the DFT tables of SftDftArgs
    int K;
    int64_t k_lo;
    int dk;
    float taper;          // Tukey fraction over the band
    const SftChunkDev* chunks;
    int n_chunks;
    float2* y;
};

// One chunk transform length n = LA LB of the SFT front end.  Its chunks are
// ids[id0 .. id0 + nc); in the single rows launch its workgroups are
// rows_blk0 + i LB + n_b (row n_b of its i-th chunk), in the single columns
// launch cols_blk0 + i n_groups + g (8-column group g of its i-th chunk).
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

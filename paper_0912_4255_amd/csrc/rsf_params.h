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
constexpr int kPassBCols = 8;       // columns of a second-pass block (one 8-column spill group)
constexpr int kTwSplitBits = 12;    // inter-pass twiddle W_N^m = hi[m >> 12] * lo[m & 4095]
constexpr int kFftThreads = 512;    // threads of a first-pass workgroup
constexpr int kPassBThreads = 768;  // threads of a second-pass workgroup (3 waves per SIMD)
// complex pairs held per thread in a first-pass stage: 21 lets radix 3 and 7
// stages run 7 and 3 butterflies per thread (lengths with a factor 7 up to
// 10752); radices 2, 4, 5, 6, 8 ... 16 hold the same number as at 20
constexpr int kFftEPT = 21;
constexpr int kFftMaxLen = 10240;   // longest first-pass transform (10240 x 16 B = 160 KiB of LDS)
constexpr size_t kLdsPerGroupMax = 163840;  // LDS one workgroup can hold (160 KiB)
// First-pass rows too long for two workgroups per CU (over half the LDS) run
// one workgroup of 8 waves per CU, 2 waves per SIMD, which leaves up to 256
// VGPRs per lane: their stages hold up to kFftEPTWide complex pairs per
// thread, so that radices 9 to 16 stay usable up to 10240 points (fewer
// stages; 9720 = 10 x 12 x 9 x 9 instead of 10 x 4 x 3^5).
constexpr int kFftEPTWide = 32;

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
    // the timing chain (inversion, beam patterns) exact at lanes 0, 32, 63 of each run
    // of 64 outputs and quadratic between them (no orbit, 63 dt w_sid <= 4e-3)
    int fast_chain;
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
    double* out_u;            // T^k / dt
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
    float4* spill;            // [n_sky_l * nf_l][ceil(LA/8)][LB][8]: 8-column groups
    int64_t spill_tmpl_stride;
    int nt_spill;             // spill larger than the last-level cache: non-temporal stores
    int ept;                  // stage capacity st was planned for: kFftEPT or kFftEPTWide
};

// Candidate gate of a top-k search (device memory, one per call): thr holds
// the bits of a float t such that at least k values of the call are known to
// be >= t (so a value below t is never among the k best; -inf at the start).
// Candidates go to kGateParts partitions of part_cap slots each, one per
// producer workgroup (index mod kGateParts), so that no counter is shared
// across the chip; count[p kGateStride] is partition p's fill since the last
// merge (counters 128 bytes apart).
constexpr int kGateParts = 256;
constexpr int kGateStride = 32;
struct TopkItem;
struct TopkGate {
    unsigned thr;
    unsigned pad_[kGateStride - 1];
    unsigned count[kGateParts * kGateStride];
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
    int nt_spill;             // the spill was written non-temporally: read it the same way
    const float* coef;        // per sky of the launch {2B/D, 2A/D, -4C/D, flag}
    int n_sky_l;
    int64_t s_lo, n_out;
    float* twoF;
    int map_rows;
    int64_t sky0, n_fdot, f0;
    int nf_l;
    int n_tmpl;
    int wave;                 // one column per wave when LB = 64 E, E = 4, 8, 12 (else the LDS-stage kernel)
    // top-k selection inside the one-column-per-wave kernel (topk != 0): no
    // 2F map is written; each block appends its candidates through the gate
    int topk, k;
    TopkGate* gate;
    TopkItem* cand;           // partition p = blockIdx.x at [p part_cap, (p + 1) part_cap)
    int64_t part_cap;
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

// Top-k gate: a producer unit with at most kGateFast values at or above the
// threshold appends them all, else its k best; so a unit appends at most
// kGateItemsPerUnit candidates.
constexpr int kGateFast = 32;
constexpr int kGateItemsPerUnit = kGateFast > kTopkMax ? kGateFast : kTopkMax;

struct TopkScanArgs {
    const float* map;
    int64_t n_vals;           // rows * n_out
    int64_t n_out;
    int64_t sky0, n_fdot, f0;
    int nf_l;
    int k;
    TopkItem* cand;           // partition p = blockIdx.x mod n_part at [p part_cap, (p + 1) part_cap)
    int64_t part_cap;
    int n_part;
    TopkGate* gate;
};

struct TopkMergeArgs {
    const TopkItem* cand;     // n_cand items (n_gate: partitions of part_cap items, filled per gate->count)
    int64_t n_cand;
    TopkGate* gate;           // the one-block level sets gate->thr from its k-th result and clears the counts
    int n_gate;
    int64_t part_cap;
    const TopkItem* run_in;   // k items (may be null: start empty)
    TopkItem* run_out;        // k items (one-block grid)
    TopkItem* out_blocks;     // [gridDim.x][k] items (grids of several blocks)
    int k;
    int64_t n_fdot, n_out;
    void* entries;            // rsf_topk_entry[k] written if not null
};

}  // namespace rsf

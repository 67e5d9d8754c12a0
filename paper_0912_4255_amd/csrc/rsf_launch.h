// Host-side launchers of the librsfstat kernels (defined in the .hip files).
#pragma once

#include <hip/hip_runtime_api.h>

#include "rsf_front_params.h"
#include "rsf_params.h"
#include "rsf_point_params.h"
#include "rsf_semico_params.h"

namespace rsf {

hipError_t launch_resample(const ResampleArgs& a, int n_sky, hipStream_t s);
int resample_blocks(int LB, int64_t P);
hipError_t launch_antenna_reduce(const ReduceArgs& r, hipStream_t s);

// row_fn: a run-time compiled RowPlan kernel of a.st per non-temporal flag
// (row_plan_kernels), used when no compiled-in plan serves the launch.
hipError_t launch_fft_pass_a(const PassAArgs& a, hipStream_t s, void* const* row_fn = nullptr);
bool fft_pass_a_fixed(const FftStages& st, int64_t P);  // a compiled-in row plan serves this launch
int row_plan_tab_entries(const FftStages& st);           // base-twiddle entries of RowPlan<st.radix...>
// The first-pass kernels RowPlan<plan.radix...> for spindown order `order`
// (fn[0]: cached spill stores, fn[1]: non-temporal) compiled at run time and
// loaded on the current device; false (fn null) when that is not available.
bool row_plan_kernels(int order, const FftStages& plan, void* fn[2]);
size_t fft_pass_a_lds(int LA);  // general stages
size_t fft_pass_a_plan_lds(const FftStages& st, int64_t P);  // the kernel a launch of plan st with P rows takes
hipError_t launch_fft_pass_b(const PassBArgs& b, int n_cu, hipStream_t s);
size_t fft_pass_b_lds(int LB, int n_sky_l, bool topk);
// E when the second pass runs one column of 64 E points per wave (E = 16 only
// when it feeds the top-k gate), else 0
int fft_pass_b_wave_e(int LB, bool topk);
hipError_t fft_set_lds_limits(size_t bytes);
int fft_pass_max_elems();

int64_t topk_scan_chunks(int64_t n_vals);  // candidate groups (k each) of a scan
hipError_t launch_topk_scan(const TopkScanArgs& a, hipStream_t s);
int topk_scan_parts(int64_t n_vals, int64_t* part_cap);  // gate partitions of a scan and their capacity
int fft_pass_b_grid(const PassBArgs& b, int n_cu);       // workgroups of a second-pass launch
hipError_t launch_topk_merge(const TopkMergeArgs& a, hipStream_t s);
int topk_merge_per_block();
hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t s);
hipError_t launch_semico(const SemicoArgs& a, hipStream_t s);
// spindowns [n][order] moved by D seconds along their Taylor series
hipError_t launch_spin_translate(const double* in, double* out, int64_t n, int order, double D, hipStream_t s);
size_t hetdec_lds(int L, int D);
hipError_t launch_hetdec(const HetdecArgs& a, int n_cu, hipStream_t s);  // n_cu: persistent grid of the D = 64 form
hipError_t hetdec_set_lds_limit(size_t bytes);

hipError_t launch_sft_norm(const SftNormArgs& a, int n_sft, hipStream_t s);
int64_t sft_dft_blocks(int64_t entries);  // DFT workgroups of a chunk of K M' entries
size_t sft_dft_lds(int Mp);
hipError_t launch_sft_dft(const SftDftArgs& a, int64_t blocks, size_t lds, hipStream_t s);
int64_t sft_merge_blocks(int n);  // merge workgroups of a chunk of n bins
hipError_t launch_sft_merge(const SftMergeArgs& a, int64_t blocks, hipStream_t s);
int64_t sft_fused_blocks(int n);         // fused DFT and merge workgroups of a chunk of n bins
size_t sft_fused_lds(int M, int Mp, int dk);  // their LDS for a chunk of M SFTs on a grid of M', dk terms per side
hipError_t launch_sft_dftmerge(const SftMergeArgs& a, int64_t blocks, size_t lds, hipStream_t s);
size_t sft_rows_lds(int LA, int R);  // R rows of LA points per workgroup
size_t sft_cols_lds(int LB, int C);  // C columns of LB points per workgroup
hipError_t launch_sft_rows(const SftRowsArgs& a, int64_t blocks, size_t lds, int R, hipStream_t s);  // R in {1, 2, 4, 8}
hipError_t launch_sft_cols(const SftColsArgs& b, int64_t blocks, size_t lds, int C, hipStream_t s);  // C in {8, 16, 32}
hipError_t sft_set_lds_limits(size_t bytes);

int point_blocks(int64_t P);
hipError_t launch_point(const PointArgs& a, bool grad, hipStream_t s);
hipError_t launch_point_reduce(const PointReduceArgs& r, hipStream_t s);

}  // namespace rsf

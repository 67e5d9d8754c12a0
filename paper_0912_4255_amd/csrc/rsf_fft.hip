// Zero-padded FFTs of F_a and F_b and the F-statistic (paper Sec. III.A.2,
// steps 6-7; eqs. eq19, eq20, eq6) as a two-pass four-step transform.
//
// N_fft = LA * LB.  With input index n = LB n_a + n_b and output index
// k = k_a + LA k_b:
//   X[k_a + LA k_b] = sum_{n_b} W_LB^{n_b k_b} W_N^{n_b k_a}
//                     sum_{n_a} x[LB n_a + n_b] W_LA^{n_a k_a}.
// Pass A: one workgroup per row n_b.  It forms the integrands
//   y^a = sum_X w_X a z~ exp(-i Phi_s),  y^b likewise  (eq. eq4pt1, FP64 phase)
// from the resampled series (stored transposed, so the row is contiguous),
// transforms the row in LDS (both spectra in one float4 per element), applies
// W_N^{n_b k_a} and spills in groups of 8 consecutive k_a (128-B rows).
// Pass B: persistent workgroups over blocks of 8 consecutive k_a (one spill
// group, one contiguous run).  Each block is transformed
// over n_b, one column per wave in registers when LB = 64 E (E = 4, 8, 12),
// otherwise as 8 columns through LDS Stockham stages, and every bin reduced
// to 2F = cA |f_a|^2 + cB |f_b|^2 + cC Re(f_a f_b^*), written in ascending
// frequency over the reported band.
#include <algorithm>

#include "rsf_device.h"
#include "rsf_launch.h"
#include "rsf_pass_a.h"
#include "rsf_spill.h"
#include "rsf_topk_gate.h"

namespace rsf {

namespace {
constexpr int kNT = kFftThreads;
constexpr int kNTB = kPassBThreads;
constexpr int kEPT = kFftEPT;
}  // namespace

// Second pass, persistent.  Workgroup g handles the spill blocks g, g +
// grid, ... (block = template * n_groups + group of 8 columns k_a): the
// block's 8-column spill group comes into one LDS buffer by DMA loads (global
// -> LDS, no registers), kept as one contiguous [LB][8] group; the block is
// transformed over n_b as 8 columns.  In the last stage every thread reads
// its inputs, the workgroup synchronises, the DMA of the next block is
// issued into the same buffer, and the last butterflies, the 2F reduction
// (eq. eq6 with the noise-weighted A', B', C') and the stores run while it
// is in flight.  Eight consecutive lanes hold the eight columns of one row,
// so each store covers 32 contiguous bytes of the output.

template <bool NT>
__device__ __forceinline__ void passb_dma(const PassBArgs& B, int unit, float4* dst) {
    const int t = unit / B.n_groups;
    const int c = unit - t * B.n_groups;
    const int blk = B.LB * kPassBCols;  // the block's spill group, one contiguous run
    const float4* base = B.spill + (int64_t)t * B.spill_tmpl_stride + (int64_t)c * blk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int e0 = wave * 64; e0 < blk; e0 += kNTB) {
        const int e = e0 + lane;
        if (e < blk) {
            // the spill is read once: non-temporal (cache policy nt) when it
            // was written so, else from the cache
            __builtin_amdgcn_global_load_lds((const void*)(base + e), (__attribute__((address_space(3))) void*)(dst + e0),
                                             16, 0, NT ? 2 : 0);
        }
    }
}

// 2F of the last stage's outputs: row k_b = j + r LB/R of column b of the
// block, bin k = 8c + b + LA k_b, reordered to the ascending band.
struct TwoFSink {
    float* out;
    int LA, LR, ka0, nf, s_lo, n_out;
    float cA, cB, cC;
    template <int R>
    __device__ __forceinline__ void put(int, int j, int b, cp (&v)[R]) {
        const int ka = ka0 + b;
        if (ka >= LA) return;
        const int hnf = (nf + 1) >> 1;  // k < hnf: non-negative signed bin
        const int kst = LA * LR;
        int k = ka + LA * j;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int o = ((k < hnf) ? k : k - nf) - s_lo;
            if ((unsigned)o < (unsigned)n_out) {
                const cp u = v[r];
                out[(unsigned)o] =
                    cA * (u.x * u.x + u.y * u.y) + cB * (u.z * u.z + u.w * u.w) + cC * (u.x * u.z + u.y * u.w);
            }
            k += kst;
        }
    }
};

template <bool NT>
struct PassBMid {
    const PassBArgs* B;
    int next;
    float4* buf;
    __device__ __forceinline__ void operator()() const {
        __syncthreads();  // every thread holds its last-stage inputs: the buffer is free
        if (next >= 0) passb_dma<NT>(*B, next, buf);
    }
};

template <bool NT>
__global__ __launch_bounds__(kNTB) void rsf_fft_pass_b_k(PassBArgs B) {
    extern __shared__ float4 lds[];
    const int blk = B.LB * kPassBCols;
    const int buf_elems = ((blk + 63) / 64) * 64;
    float2* twl = reinterpret_cast<float2*>(lds + buf_elems);
    const int n_hi = (B.LB + 31) >> kTwLoBits;
    float* cfl = reinterpret_cast<float*>(twl + 32 + n_hi);
    const int tid = threadIdx.x;
    for (int i = tid; i < 32 + n_hi; i += kNTB) twl[i] = (i < 32) ? B.tw_lo[i] : B.tw_hi[i - 32];
    for (int i = tid; i < 4 * B.n_sky_l; i += kNTB) cfl[i] = B.coef[i];
    const TwLds tw{twl, twl + 32};
    const Grouped8 lay{B.LB * kGroupCols};
    const int n_units = B.n_tmpl * B.n_groups;
    const int r_last = B.st.n_stages ? B.st.radix[B.st.n_stages - 1] : 1;

    int unit = blockIdx.x;
    if (unit < n_units) passb_dma<NT>(B, unit, lds);
    while (unit < n_units) {
        // this thread's DMA loads (and last block's stores) are complete;
        // after the barrier, everyone's
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int nunit = unit + (int)gridDim.x;
        const int t = unit / B.n_groups;
        const int c = unit - t * B.n_groups;
        const int s_l = t / B.nf_l;
        const int f = t - s_l * B.nf_l;
        const int64_t out_row = B.map_rows ? (int64_t)t : (B.sky0 + s_l) * B.n_fdot + B.f0 + f;
        TwoFSink sink{B.twoF + out_row * B.n_out, B.LA, B.LB / r_last, c * kPassBCols, (int)B.n_fft, (int)B.s_lo,
                      (int)B.n_out, cfl[4 * s_l], cfl[4 * s_l + 1], cfl[4 * s_l + 2]};
        const PassBMid<NT> mid{&B, nunit < n_units ? nunit : -1, lds};
        lds_fft_into<kNTB, kPassBEPT, kPassBCols, true>(lds, B.st, tw, lay, sink, mid);
        unit = nunit;
    }
}

// ---------------------------------------------------------------------------
// Second pass, one column per wave (columns of LB = 64 E points, E = 4, 8,
// 12).  Persistent workgroups of 8 waves take the same 8-column blocks as
// rsf_fft_pass_b_k; wave b transforms column b of the block in its own
// registers:
//   n = l + 64 m (lane l < 64, m < E), k = k1 + E k2:
//   X[k1 + E k2] = sum_l W_64^{l k2} W_LB^{l k1} sum_m x[l + 64 m] W_E^{m k1}.
// The radix-E DFT over m runs in each lane's registers; the 64-point DFT over
// the lanes is three radix-4 steps (l = 16 l1 + 4 a1 + a0 against
// k2 = k2a + 4 b0 + 16 b1), each after a 4 x 4 exchange of value blocks
// among four lanes: the lanes at stride 16 (the wave's four rows) by row
// swaps in registers, the lanes at stride 4 and 1 through a 4 KB LDS region
// of the wave, so no workgroup barrier is needed inside the transform.
// Every twiddle a lane applies (W_LB^{l k1}, W_64^{l0 k2a}, W_16^{a0 b0})
// is fixed for the kernel and computed once.
// The block arrives by DMA (HBM -> LDS, 1 KB of contiguous spill per wave
// instruction, stored column-major per 1 KB so that a column is read back
// without bank conflicts); the next block's DMA runs while the current one
// is transformed.  2F goes through an LDS stage so that each output row of
// eight bins is written as 32 contiguous bytes.  Stores and loads share one
// counter on this hardware, and once stores are outstanding a wait for a
// load waits for every outstanding operation, so the stores of a block are
// issued just before the DMA of the block after next, and each block's
// single wait covers operations issued a whole transform earlier.
// ---------------------------------------------------------------------------
constexpr int kWaveColsThreads = 64 * kPassBCols;

// DMA of block `unit` (one spill group of 8 columns x LB rows, one
// contiguous run) into dst: chunk i of 64 float4 (8 rows x 8 columns) goes to
// dst + 64 i with row r, column c at slot 8 (c ^ (i & 1)) + r: column-major,
// and odd chunks with their column pairs swapped, so that the two 8-lane
// halves of a 16-lane LDS cycle of a column read fall in different banks.
template <bool NT>
__device__ __forceinline__ void wave_dma(const PassBArgs& B, int unit, float4* dst, int wave, int lane) {
    const int t = unit / B.n_groups;
    const int g = unit - t * B.n_groups;
    const float4* base = B.spill + (int64_t)t * B.spill_tmpl_stride + (int64_t)g * B.LB * kPassBCols;
    const int n_chunks = B.LB * kPassBCols / 64;
    for (int i = wave; i < n_chunks; i += kPassBCols) {
        // lane 8 c' + r takes row r, column c' ^ (i & 1) of the chunk (float4 8 r + c)
        const int src = 8 * (lane & 7) + ((lane >> 3) ^ (i & 1));
        __builtin_amdgcn_global_load_lds((const void*)(base + 64 * i + src),
                                         (__attribute__((address_space(3))) void*)(dst + 64 * i), 16, 0, NT ? 2 : 0);
    }
}

// Column b of the block in LDS, rows l + 64 m of lane l (row l + 64 m is in
// chunk (l >> 3) + 8 m, whose parity is that of l >> 3).
template <int E>
__device__ __forceinline__ void wave_col_read(const float4* blk, int b, int lane, cp (&v)[E]) {
    const float4* col = blk + 64 * (lane >> 3) + 8 * (b ^ ((lane >> 3) & 1)) + (lane & 7);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = col[512 * m];
}

// Exchange among the lanes {src0 + i s : i < 4} as a 4 x 4 transpose of
// value blocks (K = 2: stride 4, K = 3: stride 1): the lane at position c of
// its group receives, for each value group e < E/4, the register c Q + e of
// the lane at position i as its register i Q + e.  One value group at a
// time through the wave's region of 4 x 64 slots; slot (row c', lane l) at
// c' * 64 + (l ^ X(c')), X = 4 c' (K = 2) or c' (K = 3), so that the 16
// lanes an LDS cycle serves read 16 different bank groups.  HALF: slots of
// one complex value (float2, a 2 KB region), the two spectra in turn.
// 16-byte LDS accesses as single vector loads and stores (not four dword
// accesses merged later), so that each keeps the alias information of the
// LDS array it addresses
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ cp lds_read4(const cp* p) {
    const f4v t = *reinterpret_cast<const f4v*>(p);
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ void lds_write4(cp* p, cp v) {
    *reinterpret_cast<f4v*>(p) = f4v{v.x, v.y, v.z, v.w};
}

template <int E, int K, bool HALF = false>
__device__ __forceinline__ void wave_exchange(cp* __restrict__ x, int lane, int c, int src0, int s, cp (&v)[E]) {
    constexpr int Q = E / 4;
    const int xr = K == 2 ? 4 * c : c;
    auto sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        if constexpr (HALF) {
            float2* xh = reinterpret_cast<float2*>(x);
            const float2* row = xh + c * 64;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const cp u = v[cc * Q + e];
                    xh[cc * 64 + (lane ^ (K == 2 ? 4 * cc : cc))] = h ? make_float2(u.z, u.w) : make_float2(u.x, u.y);
                }
                sync();
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float2 u = row[(src0 + i * s) ^ xr];
                    if (h) {
                        v[i * Q + e].z = u.x;
                        v[i * Q + e].w = u.y;
                    } else {
                        v[i * Q + e].x = u.x;
                        v[i * Q + e].y = u.y;
                    }
                }
                sync();
            }
        } else {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) lds_write4(x + cc * 64 + (lane ^ (K == 2 ? 4 * cc : cc)), v[cc * Q + e]);
            sync();
            const cp* row = x + c * 64;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i * Q + e] = lds_read4(row + ((src0 + i * s) ^ xr));
            sync();
        }
    }
}

// The exchange among the lanes at stride 16 (the four 16-lane rows of the
// wave) as a register transpose: row p receives from row i its registers
// [p Q, p Q + Q) as registers [i Q, i Q + Q).  For each dword of a value
// group the 4 x 4 (register block, row) transpose is two steps of row
// swaps: v_permlane32_swap exchanges the upper 32 lanes of one register with
// the lower 32 of another (blocks 0/2 and 1/3), then v_permlane16_swap the
// odd rows of one with the even rows of another (blocks 0/1 and 2/3).
__device__ __forceinline__ void row_transpose4(float& x0, float& x1, float& x2, float& x3) {
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0), __float_as_uint(x2), false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x1), __float_as_uint(x3), false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
    const auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
    x0 = __uint_as_float(c[0]);
    x1 = __uint_as_float(c[1]);
    x2 = __uint_as_float(d[0]);
    x3 = __uint_as_float(d[1]);
}

template <int E>
__device__ __forceinline__ void wave_exchange_rows(cp (&v)[E]) {
    constexpr int Q = E / 4;
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        row_transpose4(v[e].x, v[Q + e].x, v[2 * Q + e].x, v[3 * Q + e].x);
        row_transpose4(v[e].y, v[Q + e].y, v[2 * Q + e].y, v[3 * Q + e].y);
        row_transpose4(v[e].z, v[Q + e].z, v[2 * Q + e].z, v[3 * Q + e].z);
        row_transpose4(v[e].w, v[Q + e].w, v[2 * Q + e].w, v[3 * Q + e].w);
    }
}

// Radix-4 DFT over the exchanged index i for each of the Q value groups.
template <int E>
__device__ __forceinline__ void wave_dft4(cp (&v)[E]) {
    constexpr int Q = E / 4;
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        cp t[4] = {v[e], v[Q + e], v[2 * Q + e], v[3 * Q + e]};
        Dft<4>::run(t);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i * Q + e] = t[i];
    }
}

// The lane's fixed twiddles.
template <int E>
struct WaveTw {
    float2 w1[E];  // W_LB^{l k1}, k1 < E (w1[0] unused)
    float2 wa[4];  // W_64^{l0 k2a}
    float2 wb[4];  // W_16^{a0 b0}
};

// The column transform of one lane: registers (b1, e) come out holding bin
// k_b = Q p + e + E (q + 4 r + 16 b1), lane = 16 p + 4 q + r.
template <int E, bool HALF = false>
__device__ __forceinline__ void wave_transform(const WaveTw<E>& tw, cp* x, int lane, cp (&v)[E]) {
    constexpr int Q = E / 4;
    const int p = lane >> 4, q = (lane >> 2) & 3, r = lane & 3;
    Dft<E>::run(v);                                     // over m -> k1
#pragma unroll
    for (int k = 1; k < E; ++k) v[k] = cp_rot(v[k], tw.w1[k]);
    wave_exchange_rows<E>(v);                           // k1 block p gathers its four l1 values
    wave_dft4<E>(v);                                    // over l1 -> k2a
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < Q; ++e) v[k * Q + e] = cp_rot(v[k * Q + e], tw.wa[k]);
    wave_exchange<E, 2, HALF>(x, lane, q, 16 * p + r, 4, v);  // lane q takes k2a = q
    wave_dft4<E>(v);                                    // over a1 -> b0
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < Q; ++e) v[k * Q + e] = cp_rot(v[k * Q + e], tw.wb[k]);
    wave_exchange<E, 3, HALF>(x, lane, r, 16 * p + 4 * q, 1, v);  // lane r takes b0 = r
    wave_dft4<E>(v);                                    // over a0 -> b1
}

// The 2F rows of block `unit` from the stage ([k_b][8] floats, columns
// XOR-swizzled by bits 3..5 of k_b against bank conflicts): rows of eight
// bins, 32 contiguous bytes each; every stage value is read before any
// store is issued.
template <int E>
__device__ __forceinline__ void wave_output(const PassBArgs& B, int unit, const float* st, int tid, int hnf, int nf) {
    const int t = unit / B.n_groups;
    const int g = unit - t * B.n_groups;
    const int s_l = t / B.nf_l;
    const int f = t - s_l * B.nf_l;
    const int64_t out_row = B.map_rows ? (int64_t)t : (B.sky0 + s_l) * B.n_fdot + B.f0 + f;
    float* out = B.twoF + out_row * B.n_out;
    const int col = tid & 7;
    const int kac = g * kPassBCols + col;
    float v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int kb = (tid >> 3) + 64 * j;
        v[j] = st[kb * kPassBCols + (col ^ ((kb >> 3) & 7))];
    }
    if (kac < B.LA) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int kb = (tid >> 3) + 64 * j;
            const int k = kac + B.LA * kb;
            const int o = ((k < hnf) ? k : k - nf) - (int)B.s_lo;
            if ((unsigned)o < (unsigned)B.n_out) out[(unsigned)o] = v[j];
        }
    }
}

// LDS of the in-kernel top-k.
struct WaveTopkLds {
    int cnt[kPassBCols];
    float sv[kPassBCols];
    unsigned so[kPassBCols];
};

// Top-k gate of a block's 2F values, E per thread: v[j] at band offset o[j]
// (key row_key + o[j]), bit j of mask set when v[j] lies in the band and
// passes the gate's threshold.  With at most kGateFast values of the block
// passing, every wave appends its own; with more, the block selects its k
// best (k rounds of a block-wide argmax), appends them and raises the
// threshold to the k-th.  Called by every thread of the block.
template <int E>
__device__ __forceinline__ void block_gate(const PassBArgs& B, unsigned long long row_key, const float (&v)[E],
                                           const int (&o)[E], unsigned mask, int tid, WaveTopkLds* tl) {
    const int lane = tid & 63, wave = tid >> 6;
    int wsum;
    const int pre = wave_prefix(__popc(mask), lane, wsum);
    if (lane == 0) tl->cnt[wave] = wsum;
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int i = 0; i < kPassBCols; ++i) total += tl->cnt[i];
    if (total == 0) return;
    // this workgroup's partition of the candidate buffer
    TopkItem* pc = B.cand + (int64_t)blockIdx.x * B.part_cap;
    if (total <= kGateFast) {
        if (wsum > 0) {
            unsigned slot = gate_reserve(B.gate, (int)blockIdx.x, wsum, lane) + (unsigned)pre;
#pragma unroll
            for (int j = 0; j < E; ++j)
                if ((mask >> j) & 1u) {
                    if ((int64_t)slot < B.part_cap) {
                        TopkItem it;
                        it.v = v[j];
                        it.pad = 0;
                        it.key = row_key + (unsigned long long)o[j];
                        pc[slot] = it;
                    }
                    ++slot;
                }
        }
        return;
    }
    unsigned first_slot = 0u;
    if (tid == 0) first_slot = atomicAdd(&B.gate->count[blockIdx.x * kGateStride], (unsigned)B.k);
    // every value of the block is in one template row: the order of the keys
    // is that of the band offsets
    float pv = INFINITY;
    unsigned po = 0u;
    for (int r = 0; r < B.k; ++r) {
        float bv = -INFINITY;
        unsigned bo = ~0u;
#pragma unroll
        for (int j = 0; j < E; ++j)
            if ((mask >> j) & 1u) {
                const unsigned oj = (unsigned)o[j];
                if ((r == 0 || topk_better(pv, po, v[j], oj)) && topk_better(v[j], oj, bv, bo)) {
                    bv = v[j];
                    bo = oj;
                }
            }
        block_best<kWaveColsThreads>(bv, bo, tl->sv, tl->so);
        if (tid == 0 && (int64_t)(first_slot + r) < B.part_cap) {
            TopkItem it = topk_empty();
            if (bv != -INFINITY) {
                it.v = bv;
                it.key = row_key + (unsigned long long)bo;
            }
            pc[first_slot + r] = it;
        }
        pv = bv;
        po = bo;
    }
    if (tid == 0) gate_raise(B.gate, pv);  // -inf (no raise) when fewer than k values passed
}

// Key of the first bin of block `unit`'s template row.
__device__ __forceinline__ unsigned long long wave_row_key(const PassBArgs& B, int unit) {
    const int t = unit / B.n_groups;
    const int s_l = t / B.nf_l;
    const int f = t - s_l * B.nf_l;
    return (unsigned long long)((B.sky0 + s_l) * B.n_fdot + B.f0 + f) * (unsigned long long)B.n_out;
}

// The same 2F values as wave_output, from the stage, through the gate.
template <int E>
__device__ __forceinline__ void wave_topk(const PassBArgs& B, int unit, const float* st, int tid, int hnf, int nf,
                                          WaveTopkLds* tl) {
    const int t = unit / B.n_groups;
    const int g = unit - t * B.n_groups;
    const int col = tid & 7;
    const int kac = g * kPassBCols + col;
    const float thr = gate_threshold(B.gate);
    float v[E];
    int o[E];
    unsigned mask = 0u;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int kb = (tid >> 3) + 64 * j;
        v[j] = st[kb * kPassBCols + (col ^ ((kb >> 3) & 7))];
        const int k = kac + B.LA * kb;
        o[j] = ((k < hnf) ? k : k - nf) - (int)B.s_lo;
        if (kac < B.LA && (unsigned)o[j] < (unsigned)B.n_out && gate_pass(v[j], thr)) mask |= 1u << j;
    }
    block_gate<E>(B, wave_row_key(B, unit), v, o, mask, tid, tl);
}

// The 2F values straight from the column transform's registers, through
// the gate: lane 16 p + 4 q + r of wave w holds bin k_b = Q p + e + E (q +
// 4 r + 16 b1) of column k_a = 8 g + w in tf[b1 Q + e]; live: k_a < LA.
template <int E>
__device__ __forceinline__ void wave_topk_regs(const PassBArgs& B, int unit, const float (&tf)[E], bool live, int tid,
                                               int hnf, int nf, WaveTopkLds* tl) {
    constexpr int Q = E / 4;
    const int lane = tid & 63, wave = tid >> 6;
    const int p = lane >> 4, q = (lane >> 2) & 3, r = lane & 3;
    const int t = unit / B.n_groups;
    const int ka = (unit - t * B.n_groups) * kPassBCols + wave;
    const float thr = gate_threshold(B.gate);
    int o[E];
    unsigned mask = 0u;
#pragma unroll
    for (int b1 = 0; b1 < 4; ++b1)
#pragma unroll
        for (int e = 0; e < Q; ++e) {
            const int j = b1 * Q + e;
            const int kb = Q * p + e + E * (q + 4 * r + 16 * b1);
            const int k = ka + B.LA * kb;
            o[j] = ((k < hnf) ? k : k - nf) - (int)B.s_lo;
            if (live && (unsigned)o[j] < (unsigned)B.n_out && gate_pass(tf[j], thr)) mask |= 1u << j;
        }
    block_gate<E>(B, wave_row_key(B, unit), tf, o, mask, tid, tl);
}

// 2F of one transformed column value (eq. eq6 with the noise-weighted A', B', C').
__device__ __forceinline__ float two_f(const cp& u, float cA, float cB, float cC) {
    return cA * (u.x * u.x + u.y * u.y) + cB * (u.z * u.z + u.w * u.w) + cC * (u.x * u.z + u.y * u.w);
}

// TOPK: the block's 2F values go through the top-k gate (wave_topk), not to
// memory.  E = 16 (1024-point columns, top-k only): the 128 KB block leaves
// no room for the 2F stage, so the gate reads the transform's registers
// (wave_topk_regs), and the lane exchanges go through 2 KB per wave, one
// spectrum at a time.
template <int E, bool NT, bool TOPK>
__global__ __launch_bounds__(kWaveColsThreads) void rsf_fft_pass_b_wave_k(PassBArgs B) {
    constexpr int Q = E / 4;
    constexpr int LBW = 64 * E;
    constexpr bool kDirect = E == 16;
    static_assert(!kDirect || TOPK, "1024-point columns feed the top-k gate only");
    // The block, the exchange slots, the 2F stage and the gate's state are
    // LDS arrays of their own: the compiler then knows that the transform's
    // LDS accesses cannot touch the block the next DMA is filling, and does
    // not wait for that DMA before them.  Only the coefficients (read before
    // the DMA is issued) are in the dynamic LDS.
    __shared__ float4 blk[kPassBCols * LBW];                        // the block, 8 columns x LB
    __shared__ cp xch[kPassBCols * (kDirect ? 2 : 4) * 64];         // 8 waves x 4 x 64 slots
    __shared__ float st[kDirect ? 1 : LBW * kPassBCols];            // 2F stage [LB][8]
    __shared__ WaveTopkLds tkl_s;
    extern __shared__ float4 lds[];
    float* cfl = reinterpret_cast<float*>(lds);                     // 4 per sky of the launch
    WaveTopkLds* tkl = &tkl_s;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int p = lane >> 4, q = (lane >> 2) & 3, r = lane & 3;
    for (int i = tid; i < 4 * B.n_sky_l; i += kWaveColsThreads) cfl[i] = B.coef[i];
    // the lane's fixed twiddles from W_LB^m = hi[m >> 5] lo[m & 31]
    WaveTw<E> tw;
    auto w_lb = [&](int m) { return c_mul(B.tw_hi[m >> kTwLoBits], B.tw_lo[m & 31]); };
#pragma unroll
    for (int k = 1; k < E; ++k) tw.w1[k] = w_lb(lane * k);
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        tw.wa[k] = w_lb(E * (lane & 15) * k);
        tw.wb[k] = w_lb(4 * E * (lane & 3) * k);
    }
    cp* x = xch + wave * (kDirect ? 2 : 4) * 64;
    const int hnf = (int)((B.n_fft + 1) >> 1);
    const int nf = (int)B.n_fft;
    const int n_units = B.n_tmpl * B.n_groups;
    const int G = (int)gridDim.x;
    int unit = blockIdx.x;
    if (unit < n_units) wave_dma<NT>(B, unit, blk, wave, lane);
    if constexpr (kDirect) {
        for (; unit < n_units; unit += G) {
            // this block's DMA (and the previous block's candidate stores) are
            // complete in every wave; every wave has left the previous gate
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const int t = unit / B.n_groups;
            const bool live = (unit - t * B.n_groups) * kPassBCols + wave < B.LA;
            cp v[E];
            if (live) wave_col_read<E>(blk, wave, lane, v);
            const int s_l = t / B.nf_l;
            const float cA = cfl[4 * s_l], cB = cfl[4 * s_l + 1], cC = cfl[4 * s_l + 2];
            __syncthreads();  // the block buffer is free
            if (unit + G < n_units) wave_dma<NT>(B, unit + G, blk, wave, lane);
            float tf[E];
            if (live) {
                wave_transform<E, true>(tw, x, lane, v);
#pragma unroll
                for (int j = 0; j < E; ++j) tf[j] = two_f(v[j], cA, cB, cC);
            }
            wave_topk_regs<E>(B, unit, tf, live, tid, hnf, nf, tkl);
        }
        return;
    }
    int prev = -1;
    for (; unit < n_units; unit += G) {
        // this block's DMA (and the previous block's stores) are complete in
        // every wave; the previous block's stage is complete
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int t = unit / B.n_groups;
        const int ka = (unit - t * B.n_groups) * kPassBCols + wave;
        const bool live = ka < B.LA;
        cp v[E];
        if (live) wave_col_read<E>(blk, wave, lane, v);
        const int s_l = t / B.nf_l;
        const float cA = cfl[4 * s_l], cB = cfl[4 * s_l + 1], cC = cfl[4 * s_l + 2];
        if (prev >= 0) {
            if constexpr (TOPK)
                wave_topk<E>(B, prev, st, tid, hnf, nf, tkl);
            else
                wave_output<E>(B, prev, st, tid, hnf, nf);
        }
        __syncthreads();  // the block buffer and the stage are free
        if (unit + G < n_units) wave_dma<NT>(B, unit + G, blk, wave, lane);
        if (live) {
            wave_transform<E>(tw, x, lane, v);
#pragma unroll
            for (int b1 = 0; b1 < 4; ++b1)
#pragma unroll
                for (int e = 0; e < Q; ++e) {
                    const int kb = Q * p + e + E * (q + 4 * r + 16 * b1);
                    st[kb * kPassBCols + (wave ^ ((kb >> 3) & 7))] = two_f(v[b1 * Q + e], cA, cB, cC);
                }
        }
        prev = unit;
    }
    if (prev >= 0) {
        __syncthreads();
        if constexpr (TOPK)
            wave_topk<E>(B, prev, st, tid, hnf, nf, tkl);
        else
            wave_output<E>(B, prev, st, tid, hnf, nf);
    }
}

int fft_pass_max_elems() { return kFftMaxLen < kNT * kEPT ? kFftMaxLen : kNT * kEPT; }

// The first-pass row plans compiled in, with their kernels
// [spindown order - 1][non-temporal spill].
struct FixedRow {
    int n_stages;
    int radix[kMaxStages];
    int tab;  // base-twiddle table entries
    const void* fn[3][2];
};
#define RSF_ROW_FN(ORD, ...)                                                 \
    {(const void*)rsf_fft_pass_a_k<ORD, false, RowPlan<__VA_ARGS__>>,        \
     (const void*)rsf_fft_pass_a_k<ORD, true, RowPlan<__VA_ARGS__>>}
#define RSF_ROW(...)                                                                               \
    {RowPlan<__VA_ARGS__>::kStages, {__VA_ARGS__}, RowPlan<__VA_ARGS__>::tab_entries(),            \
     {RSF_ROW_FN(1, __VA_ARGS__), RSF_ROW_FN(2, __VA_ARGS__), RSF_ROW_FN(3, __VA_ARGS__)}}
const FixedRow kFixedRows[] = {
    RSF_ROW(10, 10, 10, 9),  // 9000: the rows of the 10-day and 30-day workloads
#ifdef RSF_EXTRA_ROW_PLANS
    RSF_EXTRA_ROW_PLANS
#endif
};
#undef RSF_ROW
#undef RSF_ROW_FN
constexpr int kNumFixedRows = (int)(sizeof(kFixedRows) / sizeof(kFixedRows[0]));

// The general-stage kernels [stage capacity: kFftEPT, kFftEPTWide][spindown order - 1][non-temporal spill].
const void* const kGeneralRows[2][3][2] = {
    {{(const void*)rsf_fft_pass_a_k<1, false, GeneralStages<kFftEPT>>, (const void*)rsf_fft_pass_a_k<1, true, GeneralStages<kFftEPT>>},
     {(const void*)rsf_fft_pass_a_k<2, false, GeneralStages<kFftEPT>>, (const void*)rsf_fft_pass_a_k<2, true, GeneralStages<kFftEPT>>},
     {(const void*)rsf_fft_pass_a_k<3, false, GeneralStages<kFftEPT>>, (const void*)rsf_fft_pass_a_k<3, true, GeneralStages<kFftEPT>>}},
    {{(const void*)rsf_fft_pass_a_k<1, false, GeneralStages<kFftEPTWide>>, (const void*)rsf_fft_pass_a_k<1, true, GeneralStages<kFftEPTWide>>},
     {(const void*)rsf_fft_pass_a_k<2, false, GeneralStages<kFftEPTWide>>, (const void*)rsf_fft_pass_a_k<2, true, GeneralStages<kFftEPTWide>>},
     {(const void*)rsf_fft_pass_a_k<3, false, GeneralStages<kFftEPTWide>>, (const void*)rsf_fft_pass_a_k<3, true, GeneralStages<kFftEPTWide>>}}};

// Bytes of LDS of a first-pass row of length LA on the general stages: the
// row and the two-level stage table.
size_t fft_pass_a_lds(int LA) { return (size_t)LA * sizeof(float4) + (32 + (LA + 31) / 32) * sizeof(float2); }

namespace {
// The compiled-in plan of a first-pass launch (-1: the general stages): the
// planned radices, a pruned first stage (P <= LA/2) and the tables in LDS.
int fixed_row_index(const FftStages& st, int64_t P) {
    if (2 * P > st.len || st.n_stages < 2) return -1;
    for (int i = 0; i < kNumFixedRows; ++i) {
        const FixedRow& f = kFixedRows[i];
        if (f.n_stages != st.n_stages) continue;
        bool same = true;
        for (int j = 0; j < f.n_stages; ++j) same = same && f.radix[j] == st.radix[j];
        if (same && fft_pass_a_lds(st.len) + (size_t)f.tab * sizeof(float2) <= kLdsPerGroupMax) return i;
    }
    return -1;
}
}  // namespace

bool fft_pass_a_fixed(const FftStages& st, int64_t P) { return fixed_row_index(st, P) >= 0; }

int row_plan_tab_entries(const FftStages& st) {
    int ns = st.n_stages ? st.radix[0] : 1, t = 0;
    for (int i = 1; i + 1 < st.n_stages; ++i) {
        t += ns;
        ns *= st.radix[i];
    }
    return t;
}

size_t fft_pass_a_plan_lds(const FftStages& st, int64_t P) {
    const int i = fixed_row_index(st, P);
    return fft_pass_a_lds(st.len) + (i >= 0 ? (size_t)kFixedRows[i].tab * sizeof(float2) : 0);
}

hipError_t launch_fft_pass_a(const PassAArgs& a, hipStream_t s, void* const* row_fn) {
    if (a.spin_order < 1 || a.spin_order > 3 || a.st.len != a.LA) return hipErrorInvalidValue;
    const int fi = fixed_row_index(a.st, a.P);
    const size_t lds = fft_pass_a_plan_lds(a.st, a.P);
    const unsigned gy = (unsigned)(a.n_sky_l * ((a.nf_l + a.fb - 1) / a.fb));
    const dim3 grid((unsigned)a.LB, gy);
    const int nt = a.nt_spill ? 1 : 0;
    void* args[] = {const_cast<PassAArgs*>(&a)};
    // a run-time compiled RowPlan (it prunes the first stage, like the compiled-in ones)
    const size_t lds_row = fft_pass_a_lds(a.LA) + (size_t)row_plan_tab_entries(a.st) * sizeof(float2);
    if (fi < 0 && row_fn && row_fn[nt] && 2 * a.P <= a.LA && a.st.n_stages > 1 && lds_row <= kLdsPerGroupMax)
        return hipModuleLaunchKernel((hipFunction_t)row_fn[nt], grid.x, grid.y, 1, kNT, 1, 1, (unsigned)lds_row, s,
                                     args, nullptr);
    const void* fn;
    if (fi >= 0)
        fn = kFixedRows[fi].fn[a.spin_order - 1][nt];
    else if (a.ept == kFftEPT || a.ept == kFftEPTWide)
        fn = kGeneralRows[a.ept == kFftEPTWide ? 1 : 0][a.spin_order - 1][nt];
    else
        return hipErrorInvalidValue;
    return hipLaunchKernel(fn, grid, dim3(kNT), args, lds, s);
}

// Columns of 64 E points, E = 4, 8, 12, and E = 16 when the pass feeds the
// top-k gate: the one-column-per-wave second pass.
int fft_pass_b_wave_e(int LB, bool topk) {
    const int E = LB / 64;
    return (LB % 64 == 0 && (E == 4 || E == 8 || E == 12 || (topk && E == 16))) ? E : 0;
}

size_t fft_pass_b_lds(int LB, int n_sky_l, bool topk) {
    const int E = fft_pass_b_wave_e(LB, topk);
    if (E == 16)
        return (size_t)kPassBCols * LB * sizeof(float4) + (size_t)kPassBCols * 2 * 64 * sizeof(float4) +
               (size_t)4 * std::max(n_sky_l, 64) * sizeof(float) + sizeof(WaveTopkLds);
    if (E)
        return (size_t)kPassBCols * LB * sizeof(float4) + (size_t)kPassBCols * 4 * 64 * sizeof(float4) +
               (size_t)LB * kPassBCols * sizeof(float) + (size_t)4 * std::max(n_sky_l, 64) * sizeof(float) +
               sizeof(WaveTopkLds);
    const size_t buf = (size_t)((LB * kPassBCols + 63) / 64) * 64;
    return buf * sizeof(float4) + (32 + (LB + 31) / 32) * sizeof(float2) + (size_t)4 * n_sky_l * sizeof(float);
}

// Persistent grid of the second pass: one workgroup per CU, and with the
// in-kernel top-k at most one per gate partition.
int fft_pass_b_grid(const PassBArgs& b, int n_cu) {
    const int n_items = b.n_tmpl * b.n_groups;
    return std::max(1, std::min({n_items, n_cu, b.topk ? kGateParts : n_cu}));
}

hipError_t launch_fft_pass_b(const PassBArgs& b, int n_cu, hipStream_t s) {
    const size_t lds = fft_pass_b_lds(b.LB, b.n_sky_l, b.topk != 0);
    // the wave kernels' block, exchange slots, stage and gate state are static
    const size_t lds_wave = (size_t)4 * std::max(b.n_sky_l, 64) * sizeof(float);
    const unsigned grid = (unsigned)fft_pass_b_grid(b, n_cu);
#define RSF_PASS_B_WAVE1(EE, NTT, TK) \
    hipLaunchKernelGGL((rsf_fft_pass_b_wave_k<EE, NTT, TK>), dim3(grid), dim3(kWaveColsThreads), lds_wave, s, b)
#define RSF_PASS_B_WAVE(EE)                  \
    case EE:                                 \
        if (b.nt_spill) {                    \
            if (b.topk)                      \
                RSF_PASS_B_WAVE1(EE, true, true);  \
            else                             \
                RSF_PASS_B_WAVE1(EE, true, false); \
        } else {                             \
            if (b.topk)                      \
                RSF_PASS_B_WAVE1(EE, false, true); \
            else                             \
                RSF_PASS_B_WAVE1(EE, false, false); \
        }                                    \
        return hipGetLastError();
    switch (b.wave ? fft_pass_b_wave_e(b.LB, b.topk) : 0) {
        RSF_PASS_B_WAVE(4)
        RSF_PASS_B_WAVE(8)
        RSF_PASS_B_WAVE(12)
        case 16:
            if (b.nt_spill)
                RSF_PASS_B_WAVE1(16, true, true);
            else
                RSF_PASS_B_WAVE1(16, false, true);
            return hipGetLastError();
        default: break;
    }
#undef RSF_PASS_B_WAVE
#undef RSF_PASS_B_WAVE1
    if (b.nt_spill)
        hipLaunchKernelGGL(rsf_fft_pass_b_k<true>, dim3(grid), dim3(kNTB), lds, s, b);
    else
        hipLaunchKernelGGL(rsf_fft_pass_b_k<false>, dim3(grid), dim3(kNTB), lds, s, b);
    return hipGetLastError();
}

hipError_t fft_set_lds_limits(size_t bytes) {
    // the limit only ever grows: a smaller request from another plan must not
    // undo a larger one
    static size_t granted = 0;
    if (bytes <= granted) return hipSuccess;
    // (the wave kernels of the second pass hold their LDS statically and
    // take 1 KB of dynamic LDS at most)
    const void* fns[] = {(const void*)rsf_fft_pass_b_k<false>, (const void*)rsf_fft_pass_b_k<true>};
    hipError_t out = hipSuccess;
    auto set = [&](const void* f) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (out == hipSuccess) out = e;
    };
    for (const void* f : fns) set(f);
    for (const auto& c : kGeneralRows)
        for (const auto& o : c)
            for (const void* f : o) set(f);
    for (const FixedRow& r : kFixedRows)
        for (const auto& o : r.fn)
            for (const void* f : o) set(f);
    if (out == hipSuccess) granted = bytes;
    return out;
}

}  // namespace rsf

// SFT front end (paper Sec. III.B): running-median normalisation of the
// SFT bands (eq. dimlessSFTs1), and per contiguous chunk the long-baseline
// transform by the truncated Dirichlet merge (eqs. dft3, e9, e91 with the
// large-N kernel of eq. e75), relabelled so that f_h is DC, windowed over
// the band and inverse transformed ("Downsampling and low-pass filtering"),
// then moved to the common heterodyne reference (eq. hetStartCorr), tapered
// at the chunk edges and written into the series ("Gaps in the data").
//
// The inverse transform is a forward four-step transform of the conjugated
// band (n = LA LB, input m = LB n_a + n_b, output j = k_a + LA k_b) on the
// LDS Stockham stages of the F-statistic passes: a rows pass that spills like
// the first F-statistic pass, and a columns pass that conjugates and writes
// the series.  The second member of each complex pair is unused.  Every
// launch covers all chunks (merge) or all chunks of one transform length
// (rows, columns), read from a device table of chunks.
#include "rsf_device.h"
#include "rsf_launch.h"
#include "rsf_spill.h"

namespace rsf {

namespace {
constexpr int kNormThreads = 256;
constexpr int kNormSort = 1024;  // >= kNormThreads + kSftMaxWindow - 1, a power of two
constexpr int kNT = kFftThreads;
constexpr int kNTB = kPassBThreads;
}  // namespace

// One workgroup per 256 bins of one SFT.  The powers |X|^2 of the bins that
// any of its windows touch (the tile and its halo, windows clamped inside the
// band) are sorted once in LDS with their positions; the median of bin k's
// window is then the (w/2 + 1)-th smallest sorted value whose position lies in
// the window, found by a pass over the sorted list that stops there.  The
// mean power is the median / ln 2 (|X|^2 of Gaussian noise is exponential),
// and X^ = X sqrt(ln 2 / median); a zero median gives zero.
__global__ __launch_bounds__(kNormThreads) void rsf_sft_norm_k(SftNormArgs a) {
    __shared__ float key[kNormSort];
    __shared__ int pos[kNormSort];
    const int alpha = blockIdx.y;
    const int h = a.w / 2;
    const int k0 = blockIdx.x * kNormThreads;
    const int k1 = min(k0 + kNormThreads, a.K) - 1;
    const int base = min(max(k0 - h, 0), a.K - a.w);
    const int end = min(max(k1 - h, 0), a.K - a.w) + a.w;
    const int count = end - base;
    int S = 1;
    while (S < count) S <<= 1;
    const float2* row = a.in + (int64_t)alpha * a.K;
    for (int i = threadIdx.x; i < S; i += kNormThreads) {
        float v = __builtin_inff();
        if (i < count) {
            const float2 x = row[base + i];
            v = x.x * x.x + x.y * x.y;
        }
        key[i] = v;
        pos[i] = i;
    }
    __syncthreads();
    // bitonic sort, ascending by (key, pos)
    for (int size = 2; size <= S; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < S; i += kNormThreads) {
                const int l = i ^ stride;
                if (l > i) {
                    const bool up = (i & size) == 0;
                    const float ki = key[i], kl = key[l];
                    const int pi = pos[i], pl = pos[l];
                    const bool gt = (ki > kl) || (ki == kl && pi > pl);
                    if (gt == up) {
                        key[i] = kl;
                        key[l] = ki;
                        pos[i] = pl;
                        pos[l] = pi;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int k = k0 + threadIdx.x;
    if (k < a.K) {
        const int lo = min(max(k - h, 0), a.K - a.w) - base;
        const int hi = lo + a.w;
        int cnt = 0;
        float med = 0.f;
        for (int i = 0; i < count && cnt <= h; ++i) {
            const int p = pos[i];
            if (p >= lo && p < hi) {
                ++cnt;
                med = key[i];
            }
        }
        const float2 x = row[k];
        const float g = med > 0.f ? sqrtf(0.69314718055994531f / med) : 0.f;
        a.out[(int64_t)alpha * a.K + k] = make_float2(x.x * g, x.y * g);
    }
}

// Merge: one workgroup per 256 consecutive relabelled bins u = q + n/2 of
// one chunk (all chunks in one launch; the chunk comes from the workgroup
// index).  The bins' long-baseline indices b = b0 - n/2 + u are contiguous,
// so their k* span a short range; the SFT bins they need,
// [k*_lo - dk, k*_hi + dk] of every SFT of the chunk, are staged in LDS in
// tiles of SFTs and read from there by all the workgroup's bins.  For bin b,
// k* = floor(b / M'), r = b - k* M'; the kernel of eq. e75 at
// y = 2 pi (r/M' - d) for k = k* + d has sin y = sin(2 pi r/M') and
// 1 - cos y = 2 sin^2(pi r/M') for every d, so P_d = (sin y - i (1 - cos y)) / y_d
// (1 at y = 0; 0 for d != 0 when r = 0); the phase e^{-2 pi i b alpha / M'}
// is e^{-2 pi i r alpha / M'}, read from the table of the M' roots.  Terms
// outside the stored band are absent.  The bin, windowed, scaled and
// conjugated, goes to y[y_off + m] with m = q mod n (natural order).
namespace {
constexpr int kMergeThreads = 256;
constexpr int kMergeStage = 32768;  // bytes of staged SFT bins per tile
}  // namespace

__global__ __launch_bounds__(kMergeThreads) void rsf_sft_merge_k(SftMergeArgs a) {
    extern __shared__ float2 sm[];
    // chunk of this workgroup: the last one whose first workgroup is <= ours
    int lo = 0, hi = a.n_chunks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.chunks[mid].blk0 <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const SftChunkDev c = a.chunks[lo];
    const int n = c.n;
    const int u0 = (int)((int64_t)blockIdx.x - c.blk0) * kMergeThreads;
    const int nb = min(kMergeThreads, n - u0);
    float2* roots = sm;                                        // M' entries
    float2* st = sm + ((c.Mp + 1) & ~1);                       // staged bins
    for (int i = threadIdx.x; i < c.Mp; i += kMergeThreads) {
        float s, co;
        sincospif(2.0f * (float)i / (float)c.Mp, &s, &co);
        roots[i] = make_float2(co, -s);
    }
    const int64_t bfirst = c.b0 - n / 2 + u0;
    const int64_t ks_lo = bfirst / c.Mp;
    const int64_t ks_hi = (bfirst + nb - 1) / c.Mp;
    const int64_t kl = max(ks_lo - a.dk, a.k_lo);
    const int64_t kh = min(ks_hi + a.dk, a.k_lo + a.K - 1);
    const int W = (int)max((int64_t)0, kh - kl + 1);           // staged bins per SFT
    const int TA = W > 0 ? max(1, min(c.M, kMergeStage / (int)sizeof(float2) / W)) : c.M;

    const int u = u0 + (int)threadIdx.x;
    const bool act = (int)threadIdx.x < nb;
    const int64_t b = bfirst + threadIdx.x;
    const int64_t ks = b / c.Mp;
    const int r = (int)(b - ks * c.Mp);
    float sy, cy, sh, ch;
    sincospif(2.0f * (float)r / (float)c.Mp, &sy, &cy);
    sincospif((float)r / (float)c.Mp, &sh, &ch);
    const float omc = 2.0f * sh * sh;  // 1 - cos y
    const float fr = (float)r / (float)c.Mp;
    const int d_lo = (int)max((int64_t)-a.dk, kl - ks);
    const int d_hi = (int)min((int64_t)a.dk, kh - ks);
    const int kb = (int)(ks - kl);                             // k* in the staged window
    float2 P[kSftMaxTerms];
#pragma unroll
    for (int t = 0; t < kSftMaxTerms; ++t) {
        const int d = t - a.dk;
        P[t] = make_float2(0.f, 0.f);
        if (d >= d_lo && d <= d_hi) {
            if (r == 0) {
                P[t].x = d == 0 ? 1.f : 0.f;
            } else {
                const float inv = 1.0f / (6.28318530717958648f * (fr - (float)d));
                P[t] = make_float2(sy * inv, -omc * inv);
            }
        }
    }
    float2 acc = make_float2(0.f, 0.f);
    int idx = 0;  // r alpha mod M'
    for (int t0 = 0; t0 < c.M; t0 += TA) {
        const int ta = min(TA, c.M - t0);
        __syncthreads();  // previous tile consumed (and the roots written)
        for (int i = threadIdx.x; i < ta * W; i += kMergeThreads) {
            const int al = i / W, k = i - al * W;
            st[i] = a.xh[(int64_t)(c.a0 + t0 + al) * a.K + (kl - a.k_lo) + k];
        }
        __syncthreads();
        if (act) {
            for (int al = 0; al < ta; ++al) {
                const float2* row = st + al * W + kb;
                float2 in = make_float2(0.f, 0.f);
#pragma unroll
                for (int t = 0; t < kSftMaxTerms; ++t) {
                    const int d = t - a.dk;
                    if (d >= d_lo && d <= d_hi) {
                        const float2 x = row[d];
                        in.x += x.x * P[t].x - x.y * P[t].y;
                        in.y += x.x * P[t].y + x.y * P[t].x;
                    }
                }
                const float2 e = roots[idx];
                acc.x += in.x * e.x - in.y * e.y;
                acc.y += in.x * e.y + in.y * e.x;
                idx += r;
                if (idx >= c.Mp) idx -= c.Mp;
            }
        }
    }
    if (!act) return;
    // Tukey window over the ascending band, x = (u + 1/2) / n
    float wgt = 1.0f;
    if (a.taper > 0.f) {
        const float x = ((float)u + 0.5f) / (float)n;
        const float e = 0.5f * a.taper;
        if (x < e) wgt = 0.5f * (1.0f - cospif(x / e));
        else if (x > 1.0f - e) wgt = 0.5f * (1.0f - cospif((1.0f - x) / e));
    }
    const float g = wgt * c.scale;
    const int q = u - n / 2;
    const int m = q < 0 ? q + n : q;
    a.y[c.y_off + m] = make_float2(acc.x * g, -acc.y * g);
}

// Rows pass: workgroup (n_b, i) gathers row n_b of chunk ids[i]'s band bins
// (elements m = LB n_a + n_b), transforms it over n_a and spills it with the
// inter-pass twiddle W_n^{n_b k_a}.
__global__ __launch_bounds__(kNT) void rsf_sft_rows_k(SftRowsArgs A) {
    extern __shared__ float4 lds[];
    float2* twl = reinterpret_cast<float2*>(lds + A.LA);
    const int n_hi = (A.LA + 31) >> kTwLoBits;
    for (int i = threadIdx.x; i < 32 + n_hi; i += kNT) twl[i] = (i < 32) ? A.tws_lo[i] : A.tws_hi[i - 32];
    const TwLds tws{twl, twl + 32};
    const SftChunkDev& c = A.chunks[A.ids[blockIdx.y]];
    const int n_b = blockIdx.x;
    const int tid = threadIdx.x;
    const float2* src = A.y + c.y_off + n_b;
    for (int n_a = tid; n_a < A.LA; n_a += kNT) {
        const float2 v = src[(int64_t)A.LB * n_a];
        lds[n_a] = make_float4(v.x, v.y, 0.f, 0.f);
    }
    const int64_t mb = ((int64_t)n_b * tid) % A.n;
    const int64_t ms = ((int64_t)n_b * kNT) % A.n;
    const int msk = (1 << kTwSplitBits) - 1;
    const float2 w_base = c_mul(A.tw_hi[mb >> kTwSplitBits], A.tw_lo[mb & msk]);
    const float2 w_step = c_mul(A.tw_hi[ms >> kTwSplitBits], A.tw_lo[ms & msk]);
    const int r_last = A.st.n_stages ? A.st.radix[A.st.n_stages - 1] : 1;
    const int lr = A.LA / r_last;
    const int64_t ml = ((int64_t)n_b * lr) % A.n;
    const float2 w_lr = c_mul(A.tw_hi[ml >> kTwSplitBits], A.tw_lo[ml & msk]);
    __syncthreads();
    SpillSink sink{reinterpret_cast<char*>(A.spill + c.spill_off), A.LB, n_b, lr, w_base, w_step, w_lr};
    lds_fft_into<kNT, kFftEPT, 1, false>(lds, A.st, tws, Interleaved<1>{}, sink, NoMid{});
}

// Output j = k_a + LA k_b of the chunk's transform: x[j0 + j] for j < n_keep.
struct SeriesSink {
    float2* x;
    int64_t j0, n_keep, n_out;
    int LA, LR, ka0, n_edge;
    float2 corr;
    template <int R>
    __device__ __forceinline__ void put(int, int j, int b, cp (&v)[R]) {
        const int ka = ka0 + b;
        if (ka >= LA) return;
        const int e = (int)min((int64_t)n_edge, n_keep / 2);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t jj = (int64_t)ka + (int64_t)LA * (j + r * LR);
            const int64_t o = j0 + jj;
            if (jj < n_keep && o >= 0 && o < n_out) {
                // conjugate (inverse transform), then the chunk's phase correction
                const float re = v[r].x, im = -v[r].y;
                float g = 1.0f;
                if (jj < e) g = 0.5f * (1.0f - cospif(((float)jj + 0.5f) / (float)e));
                else if (jj >= n_keep - e) g = 0.5f * (1.0f - cospif(((float)(n_keep - 1 - jj) + 0.5f) / (float)e));
                x[o] = make_float2(g * (re * corr.x - im * corr.y), g * (re * corr.y + im * corr.x));
            }
        }
    }
};

// Columns pass: workgroup (g, i) transforms the 8 columns of group pair g of
// chunk ids[i] (both 4-column spill groups) over n_b and writes the series.
__global__ __launch_bounds__(kNTB) void rsf_sft_cols_k(SftColsArgs B) {
    extern __shared__ float4 lds[];
    const int blk = B.LB * kPassBCols;
    const int buf_elems = ((blk + 63) / 64) * 64;
    float2* twl = reinterpret_cast<float2*>(lds + buf_elems);
    const int n_hi = (B.LB + 31) >> kTwLoBits;
    const int tid = threadIdx.x;
    for (int i = tid; i < 32 + n_hi; i += kNTB) twl[i] = (i < 32) ? B.tw_lo[i] : B.tw_hi[i - 32];
    const TwLds tw{twl, twl + 32};
    const SftChunkDev& ch = B.chunks[B.ids[blockIdx.y]];
    const int c = blockIdx.x;
    const float4* src = B.spill + ch.spill_off + (int64_t)c * blk;
    for (int e = tid; e < blk; e += kNTB) lds[e] = src[e];
    __syncthreads();
    const int r_last = B.st.n_stages ? B.st.radix[B.st.n_stages - 1] : 1;
    SeriesSink sink{B.x, ch.j0, ch.n_keep, B.n_out, B.LA, B.LB / r_last, c * kPassBCols, B.n_edge, ch.corr};
    lds_fft_into<kNTB, kPassBEPT, kPassBCols, false>(lds, B.st, tw, Grouped4{B.LB * kGroupCols}, sink, NoMid{});
}

hipError_t launch_sft_norm(const SftNormArgs& a, int n_sft, hipStream_t s) {
    const unsigned gx = (unsigned)((a.K + kNormThreads - 1) / kNormThreads);
    hipLaunchKernelGGL(rsf_sft_norm_k, dim3(gx, (unsigned)n_sft), dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

int64_t sft_merge_blocks(int n) { return (n + kMergeThreads - 1) / kMergeThreads; }

size_t sft_merge_lds(int Mp, int M, int dk) {
    (void)M;
    (void)dk;
    return (size_t)((Mp + 1) & ~1) * sizeof(float2) + kMergeStage;
}

hipError_t launch_sft_merge(const SftMergeArgs& a, int64_t blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(rsf_sft_merge_k, dim3((unsigned)blocks), dim3(kMergeThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_sft_rows(const SftRowsArgs& a, int n_chunks, hipStream_t s) {
    hipLaunchKernelGGL(rsf_sft_rows_k, dim3((unsigned)a.LB, (unsigned)n_chunks), dim3(kNT), fft_pass_a_lds(a.LA), s,
                       a);
    return hipGetLastError();
}

hipError_t launch_sft_cols(const SftColsArgs& b, int n_chunks, hipStream_t s) {
    hipLaunchKernelGGL(rsf_sft_cols_k, dim3((unsigned)b.n_groups, (unsigned)n_chunks), dim3(kNTB),
                       fft_pass_b_lds(b.LB, 0), s, b);
    return hipGetLastError();
}

hipError_t sft_set_lds_limits(size_t bytes) {
    static size_t granted = 0;  // only grows
    if (bytes <= granted) return hipSuccess;
    const void* fns[] = {(const void*)rsf_sft_merge_k, (const void*)rsf_sft_rows_k, (const void*)rsf_sft_cols_k};
    hipError_t out = hipSuccess;
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (out == hipSuccess) out = e;
    }
    if (out == hipSuccess) granted = bytes;
    return out;
}

}  // namespace rsf

// SFT front end (paper Sec. III.B): running-median normalisation of the
// SFT bands (eq. dimlessSFTs1), and per contiguous chunk the long-baseline
// transform by the truncated Dirichlet merge (eqs. dft3, e9, e91 with the
// large-N kernel of eq. e75; its double sum over SFTs and terms is taken as
// a DFT over the SFTs per stored bin, then the terms), relabelled so that
// f_h is DC, windowed over
// the band and inverse transformed ("Downsampling and low-pass filtering"),
// then moved to the common heterodyne reference (eq. hetStartCorr), tapered
// at the chunk edges and written into the series ("Gaps in the data").
//
// The inverse transform is a forward four-step transform of the conjugated
// band (n = LA LB, input m = LB n_a + n_b, output j = k_a + LA k_b) on the
// LDS Stockham stages of the F-statistic passes: a rows pass that spills like
// the first F-statistic pass, and a columns pass that conjugates and writes
// the series.  The second member of each complex pair is unused.  Every
// launch covers all chunks, read from device tables of the chunks and of the
// transform lengths.
#include "rsf_device.h"
#include "rsf_launch.h"
#include "rsf_spill.h"

namespace rsf {

namespace {
constexpr int kNormThreads = 256;
constexpr int kNormSort = 1024;  // >= kNormThreads + kSftMaxWindow - 1, a power of two
constexpr int kNT = kFftThreads;
constexpr int kNTB = kPassBThreads;
constexpr int kSftLoads = 8;     // global loads in flight per thread where a kernel stages its input in LDS
}  // namespace

// Running median for windows longer than kNormRegMax bins (the register
// version, rsf_sft_norm_reg_k, takes the shorter ones).  One workgroup per
// 256 bins of one SFT.  The powers |X|^2 of the bins that any of its windows
// touch (the tile and its halo, windows clamped inside the
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

// Running median for windows of at most kNormRegMax bins: each thread slides
// one window over kNormRun consecutive bins.  The window is a sorted array of
// kNormRegMax + 1 slots: the w values, (kNormRegMax - w) / 2 copies of -inf
// below and as many of +inf above, and one more +inf, so that the median is
// always slot kNormRegMax / 2 (a constant index).  The first window is sorted
// in registers by a sorting network, and only the kNormBand slots centred on
// the median are kept.  A step of the window removes the outgoing value y
// (slot i becomes s[i] if s[i] < y, else s[i+1]) and inserts the incoming x
// (slot i becomes max(s[i-1], min(x, s[i])), i descending: the median of
// s[i-1], x and s[i], one v_med3_f32, since the band stays sorted), with +inf
// above the band and -inf below it.  Both maps are monotone in the slots they read,
// so a slot that held a lower (upper) bound of its true value still does, and
// an exact slot stays exact while its neighbours are: each step turns at most
// the band's outermost exact slot on either side into a bound.  The band holds
// kNormRun - 1 slots on either side of the median, one per step of a run, so
// the median slot is exact throughout.  The powers of the workgroup's bins are
// staged in LDS, and the gains go back through LDS so that the scaled bins are
// written in order.
namespace {
constexpr int kNormRegMax = 127;              // odd; slots kNormRegMax + 1 = 128 = 2^7
constexpr int kNormRun = 15;                  // bins per thread (odd: conflict-free LDS strides)
constexpr int kNormTile = kNormThreads * kNormRun;
constexpr int kNormBandHalf = kNormRun - 1;   // steps of one run
constexpr int kNormBand = 2 * kNormBandHalf + 1;

__device__ __forceinline__ void cmp_swap(float& lo, float& hi) {
    const float a = fminf(lo, hi), b = fmaxf(lo, hi);
    lo = a;
    hi = b;
}

// ascending sort of N = 2^LOG2N values in registers by Batcher's odd-even
// merge sort: at merge level p = 2^LP (runs of p sorted values merged into
// runs of 2p) and distance k = 2^LK = p, p/2, .., 1, slot a is compared with
// a + k when both lie in one run of 2p and (a - k mod p) mod 2k < k.  One
// instance per (p, k), so every bound is a compile-time constant and the
// network unrolls to min/max pairs on fixed registers (1471 comparators for
// N = 128, against 1792 for a bitonic network; those that feed no kept slot
// are removed by the compiler).
template <int LOG2N, int LP, int LK>
__device__ __forceinline__ void oe_merge_sort(float (&v)[1 << LOG2N]) {
    constexpr int N = 1 << LOG2N, p = 1 << LP, k = 1 << LK, r = k % p;
#pragma unroll
    for (int a = 0; a + k < N; ++a)
        if (a >= r && (a - r) % (2 * k) < k && a / (2 * p) == (a + k) / (2 * p)) cmp_swap(v[a], v[a + k]);
    if constexpr (LK > 0)
        oe_merge_sort<LOG2N, LP, LK - 1>(v);
    else if constexpr (LP + 1 < LOG2N)
        oe_merge_sort<LOG2N, LP + 1, LP + 1>(v);
}

template <int LOG2N>
__device__ __forceinline__ void sort_regs(float (&v)[1 << LOG2N]) {
    oe_merge_sort<LOG2N, 0, 0>(v);
}
}  // namespace

__global__ __launch_bounds__(kNormThreads) __attribute__((amdgpu_waves_per_eu(2)))
void rsf_sft_norm_reg_k(SftNormArgs a) {
    constexpr int S = kNormRegMax + 1;
    __shared__ float pw[kNormTile + kNormRegMax - 1];
    __shared__ float gain[kNormTile];
    const int alpha = blockIdx.y;
    const int w = a.w, h = a.w / 2;
    const int k0 = blockIdx.x * kNormTile;
    const int kend = min(k0 + kNormTile, a.K);
    auto lo_of = [&](int k) { return min(max(k - h, 0), a.K - w); };  // first bin of k's window
    const int base = lo_of(k0);
    const int top = lo_of(kend - 1) + w;
    const float2* row = a.in + (int64_t)alpha * a.K;
    for (int i = threadIdx.x; i < top - base; i += kNormThreads) {
        const float2 x = row[base + i];
        pw[i] = x.x * x.x + x.y * x.y;
    }
    __syncthreads();
    const int kt = k0 + (int)threadIdx.x * kNormRun;
    if (kt < kend) {
        const int pad = (kNormRegMax - w) / 2;
        int lo = lo_of(kt);
        float v[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int j = i - pad;
            v[i] = (j < 0) ? -__builtin_inff() : ((j < w) ? pw[lo - base + j] : __builtin_inff());
        }
        sort_regs<7>(v);
        float b[kNormBand];
#pragma unroll
        for (int i = 0; i < kNormBand; ++i) b[i] = v[kNormRegMax / 2 - kNormBandHalf + i];
#pragma unroll 1
        for (int k = kt; k < min(kt + kNormRun, kend); ++k) {
            const int lk = lo_of(k);
            if (lk != lo) {  // lk = lo + 1
                const float y = pw[lo - base];
                const float x = pw[lo + w - base];
#pragma unroll
                for (int i = 0; i + 1 < kNormBand; ++i) b[i] = (b[i] < y) ? b[i] : b[i + 1];
                b[kNormBand - 1] = (b[kNormBand - 1] < y) ? b[kNormBand - 1] : __builtin_inff();
#pragma unroll
                for (int i = kNormBand - 1; i > 0; --i) b[i] = __builtin_amdgcn_fmed3f(b[i - 1], x, b[i]);
                b[0] = fminf(x, b[0]);
                lo = lk;
            }
            const float med = b[kNormBandHalf];
            gain[k - k0] = med > 0.f ? sqrtf(0.69314718055994531f / med) : 0.f;
        }
    }
    __syncthreads();
    for (int k = k0 + (int)threadIdx.x; k < kend; k += kNormThreads) {
        const float2 x = row[k];
        const float g = gain[k - k0];
        a.out[(int64_t)alpha * a.K + k] = make_float2(x.x * g, x.y * g);
    }
}

// DFT over each chunk's SFTs: one thread per (k, r) of a chunk, consecutive
// r on consecutive threads (they share X^_{alpha, k}); workgroups of one
// chunk are contiguous from dft_blk0.  The phases W_{M'}^{r alpha} come from
// a table of the M' roots in LDS, indexed by r alpha mod M'.
namespace {
constexpr int kDftThreads = 256;
constexpr int kMergeThreads = 256;

// the chunk whose first workgroup (member BLK0) is the last one not after w
template <int64_t SftChunkDev::*BLK0>
__device__ __forceinline__ int sft_chunk_of(const SftChunkDev* chunks, int n_chunks, int64_t w) {
    int lo = 0, hi = n_chunks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunks[mid].*BLK0 <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
}  // namespace

__global__ __launch_bounds__(kDftThreads) void rsf_sft_dft_k(SftDftArgs a) {
    extern __shared__ float2 roots[];
    const SftChunkDev c = a.chunks[sft_chunk_of<&SftChunkDev::dft_blk0>(a.chunks, a.n_chunks, blockIdx.x)];
    for (int i = threadIdx.x; i < c.Mp; i += kDftThreads) {
        float s, co;
        sincospif(2.0f * (float)i / (float)c.Mp, &s, &co);
        roots[i] = make_float2(co, -s);
    }
    __syncthreads();
    const int64_t e = ((int64_t)blockIdx.x - c.dft_blk0) * kDftThreads + threadIdx.x;
    if (e >= (int64_t)a.K * c.Mp) return;
    const int k = (int)(e / c.Mp);
    const int r = (int)(e - (int64_t)k * c.Mp);
    const float2* x = a.xh + (int64_t)c.a0 * a.K + k;
    float2 acc = make_float2(0.f, 0.f);
    int idx = 0;  // r alpha mod M'
    for (int al = 0; al < c.M; ++al) {
        const float2 v = x[(int64_t)al * a.K];
        const float2 w = roots[idx];
        acc.x += v.x * w.x - v.y * w.y;
        acc.y += v.x * w.y + v.y * w.x;
        idx += r;
        if (idx >= c.Mp) idx -= c.Mp;
    }
    a.Y[c.dft_off + e] = acc;
}

// Merge: one thread per relabelled bin u = q + n/2 of a chunk (all chunks in
// one launch; the chunk comes from the workgroup index).  For bin
// b = b0 - n/2 + u: k* = floor(b / M'), r = b - k* M'; the kernel of eq. e75
// at y = 2 pi (r/M' - d) for k = k* + d has sin y = sin(2 pi r/M') and
// 1 - cos y = 2 sin^2(pi r/M') for every d, so
// P_d = (sin y - i (1 - cos y)) / y_d (1 at y = 0; 0 for d != 0 when r = 0).
// The bin is sum_d P_d Y[k* + d][r], the sum over the chunk's SFTs of
// X^_{alpha, k*+d} e^{-2 pi i b alpha / M'} (e^{-2 pi i b alpha / M'} =
// W_{M'}^{r alpha}) taken once per (k, r) in the DFT tables.  Terms outside the
// stored band are absent.  The bin, windowed, scaled and conjugated, goes to
// y[y_off + m] with m = q mod n (natural order).
__global__ __launch_bounds__(kMergeThreads) void rsf_sft_merge_k(SftMergeArgs a) {
    const SftChunkDev c = a.chunks[sft_chunk_of<&SftChunkDev::blk0>(a.chunks, a.n_chunks, blockIdx.x)];
    const int n = c.n;
    const int u = (int)((int64_t)blockIdx.x - c.blk0) * kMergeThreads + (int)threadIdx.x;
    if (u >= n) return;
    const int64_t b = c.b0 - n / 2 + u;
    const int64_t ks = b / c.Mp;
    const int r = (int)(b - ks * c.Mp);
    float sy, cy, sh, ch;
    sincospif(2.0f * (float)r / (float)c.Mp, &sy, &cy);
    sincospif((float)r / (float)c.Mp, &sh, &ch);
    const float omc = 2.0f * sh * sh;  // 1 - cos y
    const float fr = (float)r / (float)c.Mp;
    const int d_lo = (int)max((int64_t)-a.dk, a.k_lo - ks);
    const int d_hi = (int)min((int64_t)a.dk, a.k_lo + a.K - 1 - ks);
    const float2* Yr = a.Y + c.dft_off + r;  // Y[k - k_lo][r]
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < kSftMaxTerms; ++t) {
        const int d = t - a.dk;
        if (d >= d_lo && d <= d_hi) {
            float2 P;
            if (r == 0) {
                P = make_float2(d == 0 ? 1.f : 0.f, 0.f);
            } else {
                const float inv = 1.0f / (6.28318530717958648f * (fr - (float)d));
                P = make_float2(sy * inv, -omc * inv);
            }
            const float2 v = Yr[(ks + d - a.k_lo) * c.Mp];
            acc.x += v.x * P.x - v.y * P.y;
            acc.y += v.x * P.y + v.y * P.x;
        }
    }
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

// The DFT over the SFTs and the merge in one pass, without the tables in
// HBM: workgroup g of a chunk takes its band bins u in [1024 g, 1024 g +
// 1024).  The stored bins k those bins reach (k* of the first and last bin,
// +- dk) come into LDS for every SFT of the chunk in one coalesced load (each
// thread with up to kSftLoads loads in flight); the rows Y[k][.] are formed
// there and merged as in rsf_sft_merge_k.  The phases W^{r alpha} are
// running products of W^r, the terms' sines come from the hardware sine
// (argument in revolutions) and their reciprocals from v_rcp_f32 (each within
// a few 1e-7 relative).  The merge runs 2 DK + 1 terms without branches (a
// term outside [-dk, dk] or the stored band reads a row in range and weighs
// it by zero), so that its LDS reads are issued together.  Chosen when every
// chunk fits the LDS (sft_fused_lds).
namespace {
constexpr int kFuseBins = 1024;

// q = x / d and x mod d for 0 <= x < 2^21, 0 < d: the float quotient
// x * (1/d) is within one of the exact one, and one correction each way
// makes it exact
__device__ __forceinline__ int div_small(int x, int d, float inv_d, int* rem) {
    int q = (int)((float)x * inv_d);
    int r = x - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
    *rem = r;
    return q;
}
}  // namespace

template <int DK>
__global__ __launch_bounds__(kMergeThreads) void rsf_sft_dftmerge_k(SftMergeArgs a) {
    extern __shared__ float2 sh[];
    const SftChunkDev c = a.chunks[sft_chunk_of<&SftChunkDev::fblk0>(a.chunks, a.n_chunks, blockIdx.x)];
    const int n = c.n, Mp = c.Mp, M = c.M;
    const int u0 = (int)((int64_t)blockIdx.x - c.fblk0) * kFuseBins;
    const int u1 = min(u0 + kFuseBins, n);
    const int64_t bb = c.b0 - n / 2 + u0;  // band bin of u0 (b = k* M' + r >= 0)
    const int64_t ks_first = bb / Mp;
    const int r_first = (int)(bb - ks_first * Mp);
    const int64_t ks_last = (bb + (u1 - 1 - u0)) / Mp;
    const int64_t k_min = max(ks_first - a.dk, a.k_lo);
    const int64_t k_max = min(ks_last + a.dk, a.k_lo + a.K - 1);
    const int rows = k_max >= k_min ? (int)(k_max - k_min + 1) : 0;
    const float inv_mp = 1.0f / (float)Mp;
    float2* roots = sh;                // M'
    float2* Xt = roots + Mp;           // [M][rows]: X^_{a0 + alpha, k_min + kr}
    float2* Yt = Xt + M * rows;        // [rows][M']
    for (int i = threadIdx.x; i < Mp; i += kMergeThreads) {
        float s, co;
        sincospif(2.0f * (float)i / (float)Mp, &s, &co);
        roots[i] = make_float2(co, -s);
    }
    const float2* xk = a.xh + (int64_t)c.a0 * a.K + (k_min - a.k_lo);
    const int n_x = M * rows;
    const float inv_rows = 1.0f / (float)max(rows, 1);
    for (int i0 = 0; i0 < n_x; i0 += kMergeThreads * kSftLoads) {
        float2 v[kSftLoads];
#pragma unroll
        for (int j = 0; j < kSftLoads; ++j) {
            const int i = i0 + j * kMergeThreads + (int)threadIdx.x;
            if (i < n_x) {
                int kr;
                const int al = div_small(i, rows, inv_rows, &kr);
                v[j] = xk[(int64_t)al * a.K + kr];
            }
        }
#pragma unroll
        for (int j = 0; j < kSftLoads; ++j) {
            const int i = i0 + j * kMergeThreads + (int)threadIdx.x;
            if (i < n_x) Xt[i] = v[j];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * Mp; e += kMergeThreads) {
        int r;
        const int kr = div_small(e, Mp, inv_mp, &r);
        // W_{M'}^{r alpha} by repeated products of W_{M'}^r (M <= M' factors,
        // a few ulp each): the threads of one k read the same X^ (one LDS
        // broadcast) and no table
        const float2 step = roots[r];
        float2 w = make_float2(1.f, 0.f);
        float2 acc = make_float2(0.f, 0.f);
        for (int al = 0; al < M; ++al) {
            const float2 v = Xt[al * rows + kr];
            acc.x += v.x * w.x - v.y * w.y;
            acc.y += v.x * w.y + v.y * w.x;
            w = make_float2(w.x * step.x - w.y * step.y, w.x * step.y + w.y * step.x);
        }
        Yt[e] = acc;
    }
    __syncthreads();
    if (rows == 0) {
        for (int u = u0 + (int)threadIdx.x; u < u1; u += kMergeThreads) {
            const int q = u - n / 2;
            a.y[c.y_off + (q < 0 ? q + n : q)] = make_float2(0.f, 0.f);
        }
        return;
    }
    for (int u = u0 + (int)threadIdx.x; u < u1; u += kMergeThreads) {
        int r;
        const int64_t ks = ks_first + div_small(r_first + (u - u0), Mp, inv_mp, &r);
        const float fr = (float)r * inv_mp;                // r / M' in [0, 1)
        const float sy = __builtin_amdgcn_sinf(fr);        // sin(2 pi r / M')
        const float sh2 = __builtin_amdgcn_sinf(0.5f * fr);  // sin(pi r / M')
        const float omc = 2.0f * sh2 * sh2;                // 1 - cos y
        const int d_lo = (int)max((int64_t)-a.dk, a.k_lo - ks);
        const int d_hi = (int)min((int64_t)a.dk, a.k_lo + a.K - 1 - ks);
        const int kr0 = (int)(ks - k_min);                 // row of d = 0
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t <= 2 * DK; ++t) {
            const int d = t - DK;
            const float2 v = Yt[min(max(kr0 + d, 0), rows - 1) * Mp + r];
            const float inv = __builtin_amdgcn_rcpf(6.28318530717958648f * (fr - (float)d));
            float px = r == 0 ? (d == 0 ? 1.f : 0.f) : sy * inv;
            float py = r == 0 ? 0.f : -omc * inv;
            const bool on = d >= d_lo && d <= d_hi;
            px = on ? px : 0.f;
            py = on ? py : 0.f;
            acc.x += v.x * px - v.y * py;
            acc.y += v.x * py + v.y * px;
        }
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
}

// The length whose first workgroup (at member BLK0) is the last one not
// after workgroup w.
template <int64_t SftLenDev::*BLK0>
__device__ __forceinline__ int sft_len_of(const SftLenDev* lens, int n_lens, int64_t w) {
    int lo = 0, hi = n_lens - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lens[mid].*BLK0 <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Spill writer of the rows pass, as the first F-statistic pass's: output
// k_a = j + r LA/R_last of row n_b, times W_n^{n_b k_a}, goes to the spill in
// 8-column groups; the twiddle of butterfly j = j0 + q s is
// W^{n_b j0} (W^{n_b s})^q and steps by W^{n_b LA/R_last} along r.  A row past
// the transform (ok false, in a workgroup's last group of rows) writes nothing.
struct SftSpillSink {
    char* out;
    int LB, n_b, LR;
    float2 wq, w_step, w_lr;
    bool ok;
    template <int R>
    __device__ __forceinline__ void put(int, int j, int, cp (&v)[R]) {
        if (!ok) return;
        float2 w = wq;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = (uint32_t)(j + r * LR);
            const uint32_t off = (((k >> 3) * (uint32_t)LB + (uint32_t)n_b) * kGroupCols + (k & 7u)) * 16u;
            *reinterpret_cast<float4*>(out + off) = cp_rot(v[r], w);
            if (r + 1 < R) w = c_mul(w, w_lr);
        }
        wq = c_mul(wq, w_step);
    }
};

// Rows pass: workgroup w gathers RB consecutive rows n_b of its chunk pair's
// band bins (elements m = LB n_a + n_b, the RB rows adjacent in memory; the
// first chunk's in the low complex half of each float4, the second's in the
// high half), transforms them over n_a as RB interleaved columns and spills
// them with the inter-pass twiddle W_n^{n_b k_a} into the first chunk's
// spill.  Thread tid always holds row tid mod RB (kNT is a multiple of RB), so
// its twiddle recurrences run for one n_b.
template <int RB>
__global__ __launch_bounds__(kNT) void rsf_sft_rows_k(SftRowsArgs A) {
    extern __shared__ float4 lds[];
    const SftLenDev& L = A.lens[sft_len_of<&SftLenDev::rows_blk0>(A.lens, A.n_lens, blockIdx.x)];
    const int LA = L.LA, LB = L.LB;
    const int64_t n = L.n;
    const int ng = (LB + RB - 1) / RB;  // row groups per chunk
    const int64_t local = (int64_t)blockIdx.x - L.rows_blk0;
    const int i = (int)(local / ng);
    const int nb0 = (int)(local - (int64_t)i * ng) * RB;
    const FftStages st = L.st1;
    float2* twl = reinterpret_cast<float2*>(lds + LA * RB);
    const int n_hi = (LA + 31) >> kTwLoBits;
    for (int e = threadIdx.x; e < 32 + n_hi; e += kNT) twl[e] = (e < 32) ? L.t1[e] : L.t1_hi[e - 32];
    const TwLds tws{twl, twl + 32};
    const SftChunkDev& c = A.chunks[A.ids[L.id0 + 2 * i]];
    const bool pair = 2 * i + 1 < L.nc;
    const float2* src = A.y + c.y_off;
    const float2* src2 = A.y + (pair ? A.chunks[A.ids[L.id0 + 2 * i + 1]].y_off : c.y_off);
    const int tid = threadIdx.x;
    // kSftLoads elements per thread in flight, then into LDS
    for (int e0 = 0; e0 < LA * RB; e0 += kNT * kSftLoads) {
        float4 v[kSftLoads];
#pragma unroll
        for (int j = 0; j < kSftLoads; ++j) {
            const int e = e0 + j * kNT + tid;
            const int n_a = e / RB, b = e - n_a * RB;
            const bool in = e < LA * RB && nb0 + b < LB;
            const int64_t m = (int64_t)LB * n_a + nb0 + b;
            const float2 x1 = in ? src[m] : make_float2(0.f, 0.f);
            const float2 x2 = in && pair ? src2[m] : make_float2(0.f, 0.f);
            v[j] = make_float4(x1.x, x1.y, x2.x, x2.y);
        }
#pragma unroll
        for (int j = 0; j < kSftLoads; ++j) {
            const int e = e0 + j * kNT + tid;
            if (e < LA * RB) lds[e] = v[j];
        }
    }
    const int n_b = nb0 + tid % RB;
    const int64_t mb = ((int64_t)n_b * (tid / RB)) % n;
    const int64_t ms = ((int64_t)n_b * (kNT / RB)) % n;
    const int msk = (1 << kTwSplitBits) - 1;
    const float2 w_base = c_mul(L.tw_hi[mb >> kTwSplitBits], L.tw_lo[mb & msk]);
    const float2 w_step = c_mul(L.tw_hi[ms >> kTwSplitBits], L.tw_lo[ms & msk]);
    const int r_last = st.n_stages ? st.radix[st.n_stages - 1] : 1;
    const int lr = LA / r_last;
    const int64_t ml = ((int64_t)n_b * lr) % n;
    const float2 w_lr = c_mul(L.tw_hi[ml >> kTwSplitBits], L.tw_lo[ml & msk]);
    __syncthreads();
    SftSpillSink sink{reinterpret_cast<char*>(A.spill + c.spill_off), LB, n_b, lr, w_base, w_step, w_lr, n_b < LB};
    lds_fft_into<kNT, kFftEPT, RB, false>(lds, st, tws, Interleaved<RB>{}, sink, NoMid{});
}

// One chunk's output: transform value (re, im) at j = k_a + LA k_b goes to
// x[j0 + j] for j < n_keep, conjugated, tapered at the edges and phase
// corrected.
struct SeriesOut {
    int64_t j0, n_keep;
    float2 corr;
    __device__ __forceinline__ void put(float2* x, int64_t n_out, int n_edge, int64_t jj, float re, float im) const {
        const int64_t o = j0 + jj;
        if (jj >= n_keep || o < 0 || o >= n_out) return;
        const int e = (int)min((int64_t)n_edge, n_keep / 2);
        // conjugate (inverse transform), then the chunk's phase correction
        im = -im;
        float g = 1.0f;
        if (jj < e) g = 0.5f * (1.0f - cospif(((float)jj + 0.5f) / (float)e));
        else if (jj >= n_keep - e) g = 0.5f * (1.0f - cospif(((float)(n_keep - 1 - jj) + 0.5f) / (float)e));
        x[o] = make_float2(g * (re * corr.x - im * corr.y), g * (re * corr.y + im * corr.x));
    }
};

// Output j = k_a + LA k_b of a chunk pair's transforms: the low halves to the
// first chunk's series, the high halves to the second's (when there is one).
struct SeriesSink {
    float2* x;
    int64_t n_out;
    int LA, LR, ka0, n_edge;
    SeriesOut c1, c2;
    bool pair;
    template <int R>
    __device__ __forceinline__ void put(int, int j, int b, cp (&v)[R]) {
        const int ka = ka0 + b;
        if (ka >= LA) return;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t jj = (int64_t)ka + (int64_t)LA * (j + r * LR);
            c1.put(x, n_out, n_edge, jj, v[r].x, v[r].y);
            if (pair) c2.put(x, n_out, n_edge, jj, v[r].z, v[r].w);
        }
    }
};

// Columns pass: workgroup w transforms the CB columns g CB .. g CB + CB - 1 of
// its chunk pair (CB / 8 consecutive 8-column spill groups of the first
// chunk's spill, one contiguous run) over n_b and writes both series.
// Columns at or past LA (padding of the last group) are transformed but not
// written.
template <int CB>
__global__ __launch_bounds__(kNTB) void rsf_sft_cols_k(SftColsArgs B) {
    extern __shared__ float4 lds[];
    const SftLenDev& L = B.lens[sft_len_of<&SftLenDev::cols_blk0>(B.lens, B.n_lens, blockIdx.x)];
    const int LA = L.LA, LB = L.LB;
    const int64_t local = (int64_t)blockIdx.x - L.cols_blk0;
    const int i = (int)(local / L.n_groups);
    const int c = (int)(local - (int64_t)i * L.n_groups);
    const FftStages st = L.st2;
    const int blk = LB * CB;
    const int buf_elems = ((blk + 63) / 64) * 64;
    float2* twl = reinterpret_cast<float2*>(lds + buf_elems);
    const int n_hi = (LB + 31) >> kTwLoBits;
    const int tid = threadIdx.x;
    for (int e = tid; e < 32 + n_hi; e += kNTB) twl[e] = (e < 32) ? L.t2[e] : L.t2_hi[e - 32];
    const TwLds tw{twl, twl + 32};
    const SftChunkDev& ch = B.chunks[B.ids[L.id0 + 2 * i]];
    const bool pair = 2 * i + 1 < L.nc;
    const SftChunkDev& ch2 = B.chunks[B.ids[L.id0 + (pair ? 2 * i + 1 : 2 * i)]];
    const float4* src = B.spill + ch.spill_off + (int64_t)c * blk;
    for (int e0 = 0; e0 < blk; e0 += kNTB * kSftLoads) {
        float4 v[kSftLoads];
#pragma unroll
        for (int j = 0; j < kSftLoads; ++j) {
            const int e = e0 + j * kNTB + tid;
            v[j] = e < blk ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < kSftLoads; ++j) {
            const int e = e0 + j * kNTB + tid;
            if (e < blk) lds[e] = v[j];
        }
    }
    __syncthreads();
    const int r_last = st.n_stages ? st.radix[st.n_stages - 1] : 1;
    SeriesSink sink{B.x, B.n_out, LA, LB / r_last, c * CB, B.n_edge, SeriesOut{ch.j0, ch.n_keep, ch.corr},
                    SeriesOut{ch2.j0, ch2.n_keep, ch2.corr}, pair};
    lds_fft_into<kNTB, kPassBEPT, CB, false>(lds, st, tw, Grouped8{LB * kGroupCols}, sink, NoMid{});
}

hipError_t launch_sft_norm(const SftNormArgs& a, int n_sft, hipStream_t s) {
    if (a.w <= kNormRegMax) {
        const unsigned gx = (unsigned)((a.K + kNormTile - 1) / kNormTile);
        hipLaunchKernelGGL(rsf_sft_norm_reg_k, dim3(gx, (unsigned)n_sft), dim3(kNormThreads), 0, s, a);
    } else {
        const unsigned gx = (unsigned)((a.K + kNormThreads - 1) / kNormThreads);
        hipLaunchKernelGGL(rsf_sft_norm_k, dim3(gx, (unsigned)n_sft), dim3(kNormThreads), 0, s, a);
    }
    return hipGetLastError();
}

int64_t sft_dft_blocks(int64_t entries) { return (entries + kDftThreads - 1) / kDftThreads; }

size_t sft_dft_lds(int Mp) { return (size_t)Mp * sizeof(float2); }

hipError_t launch_sft_dft(const SftDftArgs& a, int64_t blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(rsf_sft_dft_k, dim3((unsigned)blocks), dim3(kDftThreads), lds, s, a);
    return hipGetLastError();
}

int64_t sft_merge_blocks(int n) { return (n + kMergeThreads - 1) / kMergeThreads; }

int64_t sft_fused_blocks(int n) { return (n + kFuseBins - 1) / kFuseBins; }

// the roots, and the SFT bins and DFT rows of the most stored bins a
// workgroup's bins reach: ceil(1024 / M') + 1 + 2 dk
size_t sft_fused_lds(int M, int Mp, int dk) {
    const size_t rows = (size_t)((kFuseBins + Mp - 1) / Mp + 1 + 2 * dk);
    return sizeof(float2) * ((size_t)Mp + rows * (size_t)(M + Mp));
}

hipError_t launch_sft_dftmerge(const SftMergeArgs& a, int64_t blocks, size_t lds, hipStream_t s) {
    static_assert(2 * 16 + 1 == kSftMaxTerms, "the wide merge instance covers every dk");
    if (a.dk <= 8)
        hipLaunchKernelGGL(rsf_sft_dftmerge_k<8>, dim3((unsigned)blocks), dim3(kMergeThreads), lds, s, a);
    else
        hipLaunchKernelGGL(rsf_sft_dftmerge_k<16>, dim3((unsigned)blocks), dim3(kMergeThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_sft_merge(const SftMergeArgs& a, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(rsf_sft_merge_k, dim3((unsigned)blocks), dim3(kMergeThreads), 0, s, a);
    return hipGetLastError();
}

size_t sft_rows_lds(int LA, int R) {
    return (size_t)LA * R * sizeof(float4) + (32 + (LA + 31) / 32) * sizeof(float2);
}

size_t sft_cols_lds(int LB, int C) {
    return (size_t)((LB * C + 63) / 64) * 64 * sizeof(float4) + (32 + (LB + 31) / 32) * sizeof(float2);
}

hipError_t launch_sft_rows(const SftRowsArgs& a, int64_t blocks, size_t lds, int R, hipStream_t s) {
    const dim3 g((unsigned)blocks), b(kNT);
    switch (R) {
        case 1: hipLaunchKernelGGL(rsf_sft_rows_k<1>, g, b, lds, s, a); break;
        case 2: hipLaunchKernelGGL(rsf_sft_rows_k<2>, g, b, lds, s, a); break;
        case 4: hipLaunchKernelGGL(rsf_sft_rows_k<4>, g, b, lds, s, a); break;
        case 8: hipLaunchKernelGGL(rsf_sft_rows_k<8>, g, b, lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sft_cols(const SftColsArgs& k, int64_t blocks, size_t lds, int C, hipStream_t s) {
    const dim3 g((unsigned)blocks), b(kNTB);
    switch (C) {
        case 8: hipLaunchKernelGGL(rsf_sft_cols_k<8>, g, b, lds, s, k); break;
        case 16: hipLaunchKernelGGL(rsf_sft_cols_k<16>, g, b, lds, s, k); break;
        case 32: hipLaunchKernelGGL(rsf_sft_cols_k<32>, g, b, lds, s, k); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t sft_set_lds_limits(size_t bytes) {
    static size_t granted = 0;  // only grows
    if (bytes <= granted) return hipSuccess;
    const void* fns[] = {(const void*)rsf_sft_dft_k,      (const void*)rsf_sft_rows_k<1>,  (const void*)rsf_sft_rows_k<2>,
                         (const void*)rsf_sft_rows_k<4>,  (const void*)rsf_sft_rows_k<8>,  (const void*)rsf_sft_cols_k<8>,
                         (const void*)rsf_sft_cols_k<16>, (const void*)rsf_sft_cols_k<32>};
    hipError_t out = hipSuccess;
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (out == hipSuccess) out = e;
    }
    if (out == hipSuccess) granted = bytes;
    return out;
}

}  // namespace rsf

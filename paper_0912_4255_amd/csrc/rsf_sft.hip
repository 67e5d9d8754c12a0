// SFT front end (paper Sec. III.B): running-median normalisation of the
// SFT bands (eq. dimlessSFTs1) and the long-baseline transform of each
// contiguous chunk by the truncated Dirichlet merge (eqs. dft3, e9, e91 with
// the large-N kernel of eq. e75), relabelled so that f_h is DC and windowed
// over the band.  The inverse transform and the stitching run in the FFT
// kernels (rsf_fft.hip).
#include "rsf_device.h"
#include "rsf_launch.h"

namespace rsf {

namespace {
constexpr int kNormThreads = 256;
constexpr int kNormSort = 1024;  // >= kNormThreads + kSftMaxWindow - 1, a power of two
constexpr int kMergeThreads = 256;
}  // namespace

// One workgroup per 256 bins of one SFT.  The powers |X|^2 of the bins that
// any of its windows touch (the tile and its halo, windows clamped inside the
// band) are sorted once in LDS with their positions; the median of bin k's
// window is then the (w/2 + 1)-th smallest sorted value whose position lies in
// the window, found by one pass over the sorted list.  The mean power is the
// median / ln 2 (|X|^2 of Gaussian noise is exponential), and
// X^ = X sqrt(ln 2 / median); a zero median gives zero.
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
        for (int i = 0; i < count; ++i) {
            const int p = pos[i];
            const bool in = (p >= lo) && (p < hi);
            cnt += in ? 1 : 0;
            if (in && cnt == h + 1) med = key[i];
        }
        const float2 x = row[k];
        const float g = med > 0.f ? sqrtf(0.69314718055994531f / med) : 0.f;
        a.out[(int64_t)alpha * a.K + k] = make_float2(x.x * g, x.y * g);
    }
}

// One thread per bin m of the chunk's transform (natural order: relabelled
// bin q = m for m < n/2, m - n above).  Long-baseline bin b = b0 + q,
// k* = floor(b / M'), r = b - k* M'; the kernel of eq. e75 at y = 2 pi (r/M' - d)
// for k = k* + d has sin y = sin(2 pi r/M') and 1 - cos y = 2 sin^2(pi r/M')
// for every d, so P_d = (sin y - i (1 - cos y)) / y_d (1 at y = 0; 0 for
// d != 0 when r = 0).  The phase e^{-2 pi i b alpha / M'} = e^{-2 pi i r alpha / M'}
// comes from a table of the M' roots in LDS.  Terms outside the stored band
// are absent.
__global__ __launch_bounds__(kMergeThreads) void rsf_sft_merge_k(SftMergeArgs a) {
    extern __shared__ float2 roots[];  // e^{-2 pi i m / M'}, m < M'
    for (int i = threadIdx.x; i < a.Mp; i += kMergeThreads) {
        float s, c;
        sincospif(2.0f * (float)i / (float)a.Mp, &s, &c);
        roots[i] = make_float2(c, -s);
    }
    __syncthreads();
    const int m = blockIdx.x * kMergeThreads + threadIdx.x;
    if (m >= a.n) return;
    const int q = (m < a.n / 2) ? m : m - a.n;
    const int64_t b = a.b0 + q;
    const int64_t ks = b / a.Mp;
    const int r = (int)(b - ks * a.Mp);
    float sy, cy, sh, ch;
    sincospif(2.0f * (float)r / (float)a.Mp, &sy, &cy);
    sincospif((float)r / (float)a.Mp, &sh, &ch);
    const float omc = 2.0f * sh * sh;  // 1 - cos y
    const float fr = (float)r / (float)a.Mp;
    float2 P[kSftMaxTerms];
    int kk[kSftMaxTerms];
    const int nt = 2 * a.dk + 1;
#pragma unroll
    for (int t = 0; t < kSftMaxTerms; ++t) {
        P[t] = make_float2(0.f, 0.f);
        kk[t] = -1;
        if (t < nt) {
            const int d = t - a.dk;
            const int64_t k = ks + d - a.k_lo;
            if (k >= 0 && k < a.K) {
                kk[t] = (int)k;
                if (r == 0) {
                    P[t] = make_float2(d == 0 ? 1.f : 0.f, 0.f);
                } else {
                    const float inv = 1.0f / (6.28318530717958648f * (fr - (float)d));
                    P[t] = make_float2(sy * inv, -omc * inv);
                }
            }
        }
    }
    float2 acc = make_float2(0.f, 0.f);
    int idx = 0;  // r alpha mod M'
    for (int al = 0; al < a.M; ++al) {
        const float2* row = a.xh + (int64_t)(a.a0 + al) * a.K;
        float2 in = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < kSftMaxTerms; ++t) {
            if (kk[t] >= 0) {
                const float2 x = row[kk[t]];
                in.x += x.x * P[t].x - x.y * P[t].y;
                in.y += x.x * P[t].y + x.y * P[t].x;
            }
        }
        const float2 e = roots[idx];
        acc.x += in.x * e.x - in.y * e.y;
        acc.y += in.x * e.y + in.y * e.x;
        idx += r;
        if (idx >= a.Mp) idx -= a.Mp;
    }
    // Tukey window over the ascending band, x = (q + n/2 + 1/2) / n
    float wgt = 1.0f;
    if (a.taper > 0.f) {
        const float x = ((float)(q + a.n / 2) + 0.5f) / (float)a.n;
        const float e = 0.5f * a.taper;
        if (x < e) wgt = 0.5f * (1.0f - cospif(x / e));
        else if (x > 1.0f - e) wgt = 0.5f * (1.0f - cospif((1.0f - x) / e));
    }
    const float g = wgt * a.scale;
    const int m1 = m / a.L2, m2 = m - (m / a.L2) * a.L2;
    a.y[(int64_t)m2 * a.L1 + m1] = make_float2(acc.x * g, -acc.y * g);
}

hipError_t launch_sft_norm(const SftNormArgs& a, int n_sft, hipStream_t s) {
    const unsigned gx = (unsigned)((a.K + kNormThreads - 1) / kNormThreads);
    hipLaunchKernelGGL(rsf_sft_norm_k, dim3(gx, (unsigned)n_sft), dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sft_merge(const SftMergeArgs& a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.n + kMergeThreads - 1) / kMergeThreads);
    hipLaunchKernelGGL(rsf_sft_merge_k, dim3(gx), dim3(kMergeThreads), (size_t)a.Mp * sizeof(float2), s, a);
    return hipGetLastError();
}

}  // namespace rsf

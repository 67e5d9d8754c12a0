// C ABI of librsfstat: plans, argument validation, workspace layout and the
// launch sequences of the resampling F-statistic (declared in rsfstat.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rsfstat.h"
#include "rsf_launch.h"
#include "rsf_params.h"

using namespace rsf;

// Device scratch of rsf_fstat_backward_static (the entry for callers that
// cannot allocate): one array per GPU the library runs on, held until the
// process ends.  In host code `scratch` is only a stand-in for the symbol;
// its device address on each GPU comes from hipGetSymbolAddress, resolved
// once per device (scratch_setup) when the first plan is created there.
static constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(RSF_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define RSF_HIP(call, what)                          \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;  // MI355X Infinity Cache

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// With `device` current: resolve (once) and return its scratch address.
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        else
            g_scratch_ptr[device] = ptr;
    }
    return g_scratch_err[device];
}
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool is_7smooth(int64_t n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

int64_t next_7smooth(int64_t n) {
    int64_t m = std::max<int64_t>(1, n);
    while (!is_7smooth(m)) ++m;
    return m;
}

// Radix sequence for a length-len transform over a batch of B interleaved
// columns: fewest stages with radices whose butterfly count len*B/R fits the
// per-stage register capacity of the FFT kernels, ties broken by the largest
// smallest radix.
bool radix_plan(int len, int B, int NT, int EPT, FftStages* st) {
    static const int all_radices[] = {16, 15, 14, 12, 10, 9, 8, 7, 6, 5, 4, 3, 2};
    std::vector<int> radices;
    if ((int64_t)len * B > (int64_t)NT * EPT) return false;
    for (int r : all_radices)
        if ((int64_t)len * B / r <= fft_radix_cap(r, NT, EPT)) radices.push_back(r);
    st->len = len;
    st->n_stages = 0;
    if (len == 1) return true;
    // dp over divisors: best[m] = (stages, -minradix) for a length m
    std::vector<int> stages(len + 1, 1 << 20), minr(len + 1, 0), choice(len + 1, 0);
    stages[1] = 0;
    minr[1] = 1 << 20;
    for (int m = 2; m <= len; ++m) {
        if (len % m) continue;
        for (int r : radices) {
            if (m % r) continue;
            const int rest = m / r;
            if (stages[rest] >= (1 << 20)) continue;
            const int s = stages[rest] + 1;
            const int mr = std::min(minr[rest], r);
            if (s < stages[m] || (s == stages[m] && mr > minr[m])) {
                stages[m] = s;
                minr[m] = mr;
                choice[m] = r;
            }
        }
    }
    if (stages[len] >= (1 << 20) || stages[len] > kMaxStages) return false;
    int m = len;
    std::vector<int> seq;
    while (m > 1) {
        seq.push_back(choice[m]);
        m /= choice[m];
    }
    // larger radices first
    std::sort(seq.begin(), seq.end(), [](int a, int b) { return a > b; });
    st->n_stages = (int)seq.size();
    for (size_t i = 0; i < seq.size(); ++i) st->radix[i] = seq[i];
    return true;
}

// Stage capacity (complex pairs per thread) of a first-pass row of length
// la: kFftEPTWide when its LDS leaves room for one workgroup per CU only
// and the wider stages need fewer of them, else kFftEPT.
int pass_a_ept(int la) {
    if (fft_pass_a_lds(la) <= kLdsPerGroupMax / 2) return kFftEPT;
    FftStages narrow, wide;
    if (!radix_plan(la, 1, kFftThreads, kFftEPTWide, &wide)) return kFftEPT;
    if (!radix_plan(la, 1, kFftThreads, kFftEPT, &narrow)) return kFftEPTWide;
    return wide.n_stages < narrow.n_stages ? kFftEPTWide : kFftEPT;
}

// Factorisation n_fft = LA * LB for the two FFT passes on a device with
// lds_max bytes of LDS per workgroup: fewest total stages, LA a multiple of
// 8, then the most balanced LDS footprints.  fft_l1 > 0 forces LA.
// wave: prefer a second pass of one column per wave (the F-statistic's; the
// SFT front end's columns pass is the LDS-stage kind for every length).
bool choose_factors(int64_t n_fft, int lds_max, int fft_l1, int* out_la, int* out_lb, bool wave = true) {
    const int max_elems = fft_pass_max_elems();
    const int64_t la_max = std::min<int64_t>(max_elems, lds_max / (int)sizeof(float4));
    const int64_t lb_max = std::min<int64_t>(max_elems / kPassBCols, lds_max / (kPassBCols * (int)sizeof(float4)));
    int best_la = -1, best_lb = -1;
    double best_score = 1e300;
    for (int64_t lb = 1; lb <= lb_max; ++lb) {
        if (n_fft % lb) continue;
        const int64_t la = n_fft / lb;
        if (la > la_max || fft_pass_a_lds((int)la) > (size_t)lds_max) continue;
        if (fft_l1 > 0 && la != fft_l1) continue;
        FftStages sa, sb;
        if (!radix_plan((int)la, 1, kFftThreads, pass_a_ept((int)la), &sa) ||
            !radix_plan((int)lb, kPassBCols, kPassBThreads, kPassBEPT, &sb) ||
            fft_pass_b_lds((int)lb, 64, false) > (size_t)lds_max)
            continue;
        const double lds_a = (double)la * 16, lds_b = (double)lb * 128;
        // a second pass of one column per wave first: LB = 256, 512, 768
        // (the longest such), then LB = 1024 (one column per wave for the
        // top-k only); then the fewest stages, L1 a multiple of 8 and the
        // most balanced LDS footprints
        const int we = wave && fft_pass_b_lds((int)lb, 64, true) <= (size_t)lds_max ? fft_pass_b_wave_e((int)lb, true) : 0;
        const double wave_bonus = we == 0 ? 0.0 : we == 16 ? -5e11 : -1e12 - 1e9 * (double)lb;
        const double score = wave_bonus + (sa.n_stages + sb.n_stages) * 1e9 + ((la % 8) ? 1e8 : 0.0) +
                             std::max(lds_a, lds_b);
        if (score < best_score) {
            best_score = score;
            best_la = (int)la;
            best_lb = (int)lb;
        }
    }
    if (best_la < 0) return false;
    *out_la = best_la;
    *out_lb = best_lb;
    return true;
}

}  // namespace

namespace {
// Launch timing with hipEvents (instrumentation only).
struct Profiler {
    bool on = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    static constexpr int kKinds = 15;
    const char* names[kKinds] = {"rsf_resample_k", "rsf_antenna_reduce_k", "rsf_fft_pass_a_k", "rsf_fft_pass_b_k",
                                 "rsf_point_k",    "rsf_point_reduce_k",   "rsf_topk_k",       "rsf_sft_norm_k",
                                 "rsf_sft_merge_k", "rsf_sft_rows_k",      "rsf_sft_cols_k",   "rsf_semico_k",
                                 "rsf_hetdec_k",   "rsf_sft_dft_k",        "rsf_sft_dftmerge_k"};
    int64_t launches[kKinds] = {};
    double ms[kKinds] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~Profiler() {
        for (auto& r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
enum {
    K_RESAMPLE = 0, K_REDUCE = 1, K_PASS_A = 2, K_PASS_B = 3, K_POINT = 4, K_POINT_REDUCE = 5, K_TOPK = 6,
    K_SFT_NORM = 7, K_SFT_MERGE = 8, K_SFT_ROWS = 9, K_SFT_COLS = 10, K_SEMICO = 11, K_HETDEC = 12, K_SFT_DFT = 13,
    K_SFT_DFTMERGE = 14
};
}  // namespace

struct rsf_plan {
    rsf_plan_desc d;
    Profiler* prof;
    int device;
    int64_t n, n_fft, s_lo, n_out;
    double df;
    int LA, LB;          // first-pass length (over n_a), second-pass length (over n_b)
    int64_t P;           // rows of the transposed series: ceil(n / LB)
    int n_groups;        // ceil(LA / 8)
    int n_cu;            // compute units (persistent second-pass grid)
    int spin_order;      // spindown derivatives per template (eq. eq4pt1), 1..3
    int binary;          // sky rows carry a circular binary orbit (a_p, P_b, t_asc)
    int fb_override;     // spindowns sharing a row in the first pass (0 = automatic)
    int g_override;      // templates per FFT launch (0 = automatic)
    FftStages stA, stB;
    void* rowA_fn[2];    // run-time compiled RowPlan kernels of stA for spin_order (or null)
    float2* twA;
    float2* twA_hi;
    float2* twB;
    float2* twB_hi;
    float2* tw_lo;
    float2* tw_hi;
    EphDev eph;
    DetDev det[RSF_MAX_DET];
    InterpDev ip;
};

namespace {

struct WsLayout {
    size_t flags, rs_main[RSF_MAX_DET], rs_tm[RSF_MAX_DET], partials, coef, abc_w, spill, map, gate, cand, run, mtmp[2],
        spins, total;
    int64_t cap;      // top-k candidate capacity per FFT launch
    int n_blocks;
    int64_t G;        // templates per FFT launch
    int64_t S;        // sky positions per resampling chunk
    int64_t rs_stride;
};

// Templates per FFT launch: 1 (plain) or 64 (batched; the autotuned choice
// for every standard shape on MI355X).
int64_t batch_templates(const rsf_plan* p, int mode) {
    if (mode == RSF_MODE_PLAIN) return 1;
    if (p->g_override > 0) return p->g_override;
    return 64;
}

// Spindowns sharing one read of a resampled row in the first FFT pass.
int first_pass_share(const rsf_plan* p, int mode) {
    if (mode == RSF_MODE_PLAIN) return 1;
    return p->fb_override > 0 ? p->fb_override : 16;
}

int64_t batch_skies(int64_t n_sky, int64_t n_fdot, int64_t G, int mode) {
    if (mode == RSF_MODE_PLAIN) return 1;
    const int64_t per = std::max<int64_t>(1, (4 * G) / std::max<int64_t>(1, n_fdot));
    return std::max<int64_t>(1, std::min<int64_t>({n_sky, per, 64}));
}

// Merge cand (n_cand items) and run_in (k items, may be null) into the k
// best, written to run_out (and entries): levels of one-block-per-4096-items
// reductions through tmp[0], tmp[1] until one block remains.
hipError_t topk_merge_levels(const rsf_plan* p, hipStream_t s, const TopkItem* cand, int64_t n_cand,
                             const TopkItem* run_in, TopkItem* run_out, int k, int64_t n_fdot, void* entries,
                             TopkItem* const tmp[2], TopkGate* gate = nullptr, int64_t part_cap = 0);

// The first pass of a large transform (2^19 points or more, RSF_RTC=all: any)
// whose row plan is not compiled in runs a RowPlan kernel compiled at run
// time for its radices, when that is available (it prunes the first stage,
// so the rows must end below LA/2); else the general stages.
void prepare_row_kernels(rsf_plan* p) {
    p->rowA_fn[0] = p->rowA_fn[1] = nullptr;
    if (2 * p->P > p->LA || p->stA.n_stages < 2 || fft_pass_a_fixed(p->stA, p->P)) return;
    if (fft_pass_a_lds(p->LA) + (size_t)row_plan_tab_entries(p->stA) * sizeof(float2) > kLdsPerGroupMax) return;
    const char* env = getenv("RSF_RTC");
    if (p->n_fft < (int64_t(1) << 19) && !(env && strcmp(env, "all") == 0)) return;
    void* fn[2];
    if (row_plan_kernels(p->spin_order, p->stA, fn)) {
        p->rowA_fn[0] = fn[0];
        p->rowA_fn[1] = fn[1];
    }
}

// The second pass selects the top-k itself (no 2F map) when it runs one
// column per wave.
bool fused_topk(const rsf_plan* p) {
    return fft_pass_b_wave_e(p->LB, true) != 0 && fft_pass_b_lds(p->LB, 64, true) <= kLdsPerGroupMax;
}

// map: room for a launch's 2F map (the semi-coherent sum, or a top-k whose
// second pass cannot select in place); topk: the candidate gate, buffer and
// merge levels.
// spins: room for the call's spindowns moved to the segment start (the
// semi-coherent sum at spin order > 1)
WsLayout fstat_layout(const rsf_plan* p, int64_t n_sky, int64_t n_fdot, int mode, bool map, bool topk,
                      bool spins = false) {
    WsLayout L{};
    size_t off = 0;
    L.flags = off;
    off = align_up(off + 64);
    L.G = batch_templates(p, mode);
    L.S = batch_skies(n_sky, n_fdot, L.G, mode);
    L.rs_stride = (int64_t)p->LB * p->P;
    const size_t elems = (size_t)L.rs_stride * (size_t)L.S;
    for (int X = 0; X < p->d.n_det; ++X) {
        L.rs_main[X] = off;
        off = align_up(off + elems * sizeof(float4));
        if (p->d.storage == RSF_STORE_F32) {
            L.rs_tm[X] = off;
            off = align_up(off + elems * sizeof(float));
        }
    }
    L.n_blocks = resample_blocks(p->LB, p->P);
    L.partials = off;
    off = align_up(off + (size_t)p->d.n_det * L.S * L.n_blocks * 3 * sizeof(double));
    L.coef = off;
    off = align_up(off + (size_t)L.S * 4 * sizeof(float));
    L.abc_w = off;
    off = align_up(off + (size_t)L.S * 3 * sizeof(double));
    L.spill = off;
    off = align_up(off + (size_t)L.G * p->n_groups * p->LB * kPassBCols * sizeof(float4));
    if (map) {
        L.map = off;
        off = align_up(off + (size_t)L.G * p->n_out * sizeof(float));
    }
    if (topk) {
        // every producer unit of a launch (second-pass block, or scan wave
        // over the map) appends at most kGateItemsPerUnit candidates to its
        // workgroup's partition; partitions are sized for the workgroup with
        // the most units, so the total is below (units + units per workgroup
        // x partitions) items
        const int64_t units = map ? topk_scan_chunks(L.G * p->n_out) + 4 : L.G * p->n_groups;
        L.cap = (units + (int64_t)(map ? 4 : 1) * kGateParts) * kGateItemsPerUnit;
        L.gate = off;
        off = align_up(off + sizeof(TopkGate));
        L.cand = off;
        off = align_up(off + (size_t)L.cap * sizeof(TopkItem));
        L.run = off;
        off = align_up(off + 2 * kTopkMax * sizeof(TopkItem));
        // outputs of the first merge level (and of any further level)
        const int64_t n1 = L.cap + kTopkMax;
        const int64_t b1 = (n1 + topk_merge_per_block() - 1) / topk_merge_per_block();
        for (int i = 0; i < 2; ++i) {
            L.mtmp[i] = off;
            off = align_up(off + (size_t)b1 * kTopkMax * sizeof(TopkItem));
        }
    }
    if (spins) {
        L.spins = off;
        off = align_up(off + (size_t)n_fdot * p->spin_order * sizeof(double));
    }
    L.total = off;
    return L;
}

struct ResLayout {
    size_t flags, partials, coef, total;
    int n_blocks;
};

ResLayout resample_layout(const rsf_plan* p, int64_t n_sky) {
    ResLayout L{};
    size_t off = 0;
    L.flags = off;
    off = align_up(off + 64);
    const int64_t P = (p->n + 63) / 64;
    L.n_blocks = resample_blocks(64, P);
    L.partials = off;
    off = align_up(off + (size_t)p->d.n_det * n_sky * L.n_blocks * 3 * sizeof(double));
    L.coef = off;
    off = align_up(off + (size_t)n_sky * 4 * sizeof(float));
    L.total = off;
    return L;
}

struct PointLayout {
    size_t flags, partials, total;
    int n_blocks;
};

PointLayout point_layout(const rsf_plan* p, int64_t n_cand) {
    PointLayout L{};
    size_t off = 0;
    L.flags = off;
    off = align_up(off + 64);
    L.n_blocks = point_blocks((p->n + 63) / 64);
    L.partials = off;
    off = align_up(off + (size_t)n_cand * L.n_blocks * kPointSums * sizeof(double));
    L.total = off;
    return L;
}

bool is_fin(double x) { return std::isfinite(x); }

ResampleArgs base_resample_args(const rsf_plan* p, const rsf_segment* seg, int X) {
    ResampleArgs a{};
    a.n = p->n;
    a.dt = p->d.dt;
    a.t_start = p->d.t_start;
    a.f_het = p->d.f_het;
    a.eph = p->eph;
    a.det = p->det[X];
    a.ip = p->ip;
    a.x = (const float2*)seg->x[X];
    a.gaps = seg->gaps[X];
    a.n_gaps = seg->n_gaps[X];
    // the same criterion as the point kernel's interpolated chain
    a.fast_chain = (!p->binary && 63.0 * p->d.dt * 2.0 * M_PI * std::fabs(p->eph.inv_p_sid) <= 4e-3) ? 1 : 0;
    return a;
}

int check_segment(const rsf_plan* p, const rsf_segment* seg) {
    if (!seg) return fail(RSF_EINVAL, "segment is NULL");
    for (int X = 0; X < p->d.n_det; ++X) {
        if (!seg->x[X]) return fail(RSF_EINVAL, "segment x[%d] is NULL", X);
        if (seg->n_gaps[X] < 0) return fail(RSF_EINVAL, "segment n_gaps[%d] < 0", X);
        if (seg->n_gaps[X] > 0 && !seg->gaps[X]) return fail(RSF_EINVAL, "segment gaps[%d] is NULL", X);
    }
    return RSF_OK;
}

// Launch through fn(); with profiling on, bracket it with events on s.
template <typename Fn>
hipError_t timed_pr(Profiler* pr, int kind, hipStream_t s, Fn fn) {
    if (!pr || !pr->on) return fn();
    hipEvent_t a = pr->get(), b = pr->get();
    if (a) (void)hipEventRecord(a, s);
    hipError_t e = fn();
    if (b) (void)hipEventRecord(b, s);
    if (a && b) pr->pending.push_back({kind, a, b});
    return e;
}

template <typename Fn>
hipError_t timed(const rsf_plan* p, int kind, hipStream_t s, Fn fn) {
    return timed_pr(p->prof, kind, s, fn);
}

}  // namespace

extern "C" {

const char* rsf_last_error(void) { return g_last_error.c_str(); }

int rsf_version(void) { return 1; }

int rsf_plan_create(rsf_plan** out, const rsf_plan_desc* d) {
    if (!out) return fail(RSF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(RSF_EINVAL, "descriptor is NULL");
    if (d->n_det < 1 || d->n_det > RSF_MAX_DET) return fail(RSF_EINVAL, "n_det must be in 1..%d", RSF_MAX_DET);
    if (d->n < 2 || d->n > (int64_t)1 << 30) return fail(RSF_EINVAL, "n must be in 2..2^30");
    if (!is_fin(d->dt) || d->dt <= 0) return fail(RSF_EINVAL, "dt must be positive and finite");
    if (!is_fin(d->t_start) || !is_fin(d->f_het) || !is_fin(d->f_lo) || !is_fin(d->f_hi))
        return fail(RSF_EINVAL, "non-finite t_start/f_het/band");
    if (d->kernel != RSF_KERNEL_LANCZOS && d->kernel != RSF_KERNEL_DIRICHLET)
        return fail(RSF_EINVAL, "unknown kernel");
    if (d->taps < 2 || d->taps > RSF_MAX_TAPS || (d->taps & 1))
        return fail(RSF_EUNSUPPORTED, "taps must be even and in 2..%d", RSF_MAX_TAPS);
    if (d->storage != RSF_STORE_F32 && d->storage != RSF_STORE_F16) return fail(RSF_EINVAL, "unknown storage");
    if (d->fft_l1 < 0) return fail(RSF_EINVAL, "fft_l1 must be 0 (automatic) or positive");
    if (d->nfft_policy != RSF_NFFT_TWICE && d->nfft_policy != RSF_NFFT_SMOOTH7 &&
        d->nfft_policy != RSF_NFFT_SMOOTH7_256)
        return fail(RSF_EINVAL, "unknown FFT length policy");
    const rsf_ephemeris& E = d->eph;
    if (!is_fin(E.au_c) || !is_fin(E.re_c) || !is_fin(E.eps) || !is_fin(E.lambda0) || !is_fin(E.theta0) ||
        !(E.p_orb > 0) || !(E.p_sid > 0) || !is_fin(E.p_orb) || !is_fin(E.p_sid))
        return fail(RSF_EINVAL, "invalid ephemeris");
    for (int X = 0; X < d->n_det; ++X) {
        const rsf_detector& D = d->det[X];
        if (!is_fin(D.lat) || !is_fin(D.lon) || !is_fin(D.gamma) || !(D.sigma2 > 0) || !is_fin(D.sigma2))
            return fail(RSF_EINVAL, "invalid detector %d", X);
    }

    rsf_plan* p = new rsf_plan();
    p->d = *d;
    p->prof = new Profiler();
    p->spin_order = 1;
    p->binary = 0;
    p->n = d->n;
    // even, so that a band reaching f_het +- 1/(2 dt) has its edges on bins
    if (d->nfft_policy == RSF_NFFT_TWICE)
        p->n_fft = 2 * d->n;
    else if (d->nfft_policy == RSF_NFFT_SMOOTH7)
        p->n_fft = 2 * next_7smooth(d->n);
    else
        p->n_fft = 256 * next_7smooth((2 * d->n + 255) / 256);
    if (!is_7smooth(p->n_fft)) {
        delete p;
        return fail(RSF_EUNSUPPORTED, "FFT length %lld has a prime factor above 7", (long long)(2 * d->n));
    }
    p->df = 1.0 / ((double)p->n_fft * d->dt);
    p->s_lo = (int64_t)llround((d->f_lo - d->f_het) / p->df);
    p->n_out = (int64_t)llround((d->f_hi - d->f_lo) / p->df);
    if (p->n_out < 1 || p->s_lo < -(p->n_fft / 2) || p->s_lo + p->n_out - 1 > (p->n_fft + 1) / 2 - 1) {
        delete p;
        return fail(RSF_EINVAL, "band [%g, %g) is empty or outside the data band", d->f_lo, d->f_hi);
    }

    // device limits
    RSF_HIP(hipGetDevice(&p->device), "hipGetDevice");
    // the static scratch of this device; a failure only disables
    // rsf_fstat_backward_static, which reports it
    (void)scratch_setup(p->device);
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess ||
        lds_max <= 0)
        lds_max = 65536;
    int best_la = -1, best_lb = -1;
    if (!choose_factors(p->n_fft, lds_max, d->fft_l1, &best_la, &best_lb)) {
        delete p;
        return fail(RSF_EUNSUPPORTED, "no two-pass factorisation of n_fft = %lld (L1 = %d) fits the LDS (%d bytes)",
                    (long long)p->n_fft, (int)d->fft_l1, lds_max);
    }
    p->LA = best_la;
    p->LB = best_lb;
    radix_plan(p->LA, 1, kFftThreads, pass_a_ept(p->LA), &p->stA);
    radix_plan(p->LB, kPassBCols, kPassBThreads, kPassBEPT, &p->stB);
    p->P = (p->n + p->LB - 1) / p->LB;
    p->n_groups = (p->LA + kPassBCols - 1) / kPassBCols;
    if (p->P > p->LA) {
        delete p;
        return fail(RSF_EUNSUPPORTED, "internal: rows exceed first-pass length");
    }
    const size_t lds_need = std::max({fft_pass_a_plan_lds(p->stA, p->P), fft_pass_b_lds(p->LB, 64, false),
                                      fused_topk(p) ? fft_pass_b_lds(p->LB, 64, true) : (size_t)0});
    if (hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
        p->n_cu <= 0)
        p->n_cu = 256;
    if (lds_need > 65536) (void)fft_set_lds_limits(lds_need);
    prepare_row_kernels(p);

    // twiddle tables, built in FP64 and stored as FP32
    auto table = [](int64_t len, int64_t count, int64_t step) {
        std::vector<float2> t((size_t)count);
        for (int64_t m = 0; m < count; ++m) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L *
                                  (long double)((m * step) % len) / (long double)len;
            t[(size_t)m] = make_float2((float)std::cos((double)a), (float)std::sin((double)a));
        }
        return t;
    };
    std::vector<float2> ta = table(p->LA, 32, 1), tah = table(p->LA, (p->LA + 31) / 32, 32);
    // second-pass stage twiddles as two levels: W_LB^m = lo[m % 32] * hi[m / 32]
    std::vector<float2> tb = table(p->LB, 32, 1), tbh = table(p->LB, (p->LB + 31) / 32, 32);
    const int64_t nlo = 1 << kTwSplitBits;
    std::vector<float2> tlo = table(p->n_fft, nlo, 1);
    const int64_t nhi = p->n_fft / nlo + 1;
    std::vector<float2> thi = table(p->n_fft, nhi, nlo);
    auto upload = [&](float2** dst, const std::vector<float2>& src) -> int {
        RSF_HIP(hipMalloc((void**)dst, src.size() * sizeof(float2)), "hipMalloc(table)");
        RSF_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(float2), hipMemcpyHostToDevice), "hipMemcpy(table)");
        return RSF_OK;
    };
    int rc;
    if ((rc = upload(&p->twA, ta)) || (rc = upload(&p->twA_hi, tah)) || (rc = upload(&p->twB, tb)) || (rc = upload(&p->twB_hi, tbh)) ||
        (rc = upload(&p->tw_lo, tlo)) || (rc = upload(&p->tw_hi, thi))) {
        rsf_plan_destroy(p);
        return rc;
    }

    // constants of the timing model and the kernel
    p->eph.au_c = E.au_c;
    p->eph.re_c = E.re_c;
    p->eph.inv_p_orb = 1.0 / E.p_orb;
    p->eph.inv_p_sid = 1.0 / E.p_sid;
    p->eph.ceps = std::cos(E.eps);
    p->eph.seps = std::sin(E.eps);
    p->eph.lambda0 = E.lambda0;
    p->eph.theta0 = E.theta0;
    for (int X = 0; X < d->n_det; ++X) {
        const rsf_detector& D = d->det[X];
        DetDev& o = p->det[X];
        o.lon = D.lon;
        o.clon = std::cos(D.lon);
        o.slon = std::sin(D.lon);
        o.clat = std::cos(D.lat);
        o.slat = std::sin(D.lat);
        o.cgu = std::cos(D.gamma + M_PI / 4);
        o.sgu = std::sin(D.gamma + M_PI / 4);
        o.cgv = std::cos(D.gamma - M_PI / 4);
        o.sgv = std::sin(D.gamma - M_PI / 4);
        o.w = 1.0 / D.sigma2;
    }
    p->ip.kernel = d->kernel;
    p->ip.taps = d->taps;
    p->ip.n = (int)d->n;
    p->ip.n_odd = (int)(d->n & 1);
    *out = p;
    return RSF_OK;
}

int rsf_plan_destroy(rsf_plan* p) {
    if (!p) return RSF_OK;
    (void)hipFree(p->twA);
    (void)hipFree(p->twA_hi);
    (void)hipFree(p->twB);
    (void)hipFree(p->twB_hi);
    (void)hipFree(p->tw_lo);
    (void)hipFree(p->tw_hi);
    delete p->prof;
    delete p;
    return RSF_OK;
}

int rsf_plan_set_binary(rsf_plan* p, int on) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    p->binary = on ? 1 : 0;
    return RSF_OK;
}

int rsf_plan_set_spin_order(rsf_plan* p, int order) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    if (order < 1 || order > 3) return fail(RSF_EINVAL, "spin order must be 1, 2 or 3");
    if (p->spin_order != order) {
        p->spin_order = order;
        prepare_row_kernels(p);
    }
    return RSF_OK;
}

int rsf_plan_set_batching(rsf_plan* p, int fb, int templates) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    if (fb < 0 || fb > 16 || templates < 0 || templates > 256)
        return fail(RSF_EINVAL, "fb must be in 0..16 and templates in 0..256");
    p->fb_override = fb;
    p->g_override = templates;
    return RSF_OK;
}

int rsf_fft_factor(int64_t n_fft, int lds_bytes, int fft_l1, int32_t* l1, int32_t* l2) {
    if (n_fft < 1 || lds_bytes < 1 || fft_l1 < 0) return fail(RSF_EINVAL, "n_fft, lds_bytes must be positive");
    if (!is_7smooth(n_fft)) return fail(RSF_EUNSUPPORTED, "FFT length %lld has a prime factor above 7", (long long)n_fft);
    int la = 0, lb = 0;
    if (!choose_factors(n_fft, lds_bytes, fft_l1, &la, &lb))
        return fail(RSF_EUNSUPPORTED, "no two-pass factorisation of n_fft = %lld fits %d bytes of LDS", (long long)n_fft,
                    lds_bytes);
    if (l1) *l1 = la;
    if (l2) *l2 = lb;
    return RSF_OK;
}

int rsf_plan_batching(const rsf_plan* p, int64_t n_sky, int64_t n_fdot, int mode, int32_t* fb,
                      int32_t* templates, int32_t* skies) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    if (n_sky < 1 || n_fdot < 1) return fail(RSF_EINVAL, "n_sky and n_fdot must be positive");
    if (mode != RSF_MODE_PLAIN && mode != RSF_MODE_BATCHED) return fail(RSF_EINVAL, "unknown mode");
    const int64_t G = batch_templates(p, mode);
    if (fb) *fb = first_pass_share(p, mode);
    if (templates) *templates = (int32_t)G;
    if (skies) *skies = (int32_t)batch_skies(n_sky, n_fdot, G, mode);
    return RSF_OK;
}

int rsf_plan_query(const rsf_plan* p, int64_t* n_fft, int64_t* bin_lo, int64_t* n_out, int32_t* l1,
                   int32_t* l2, double* df) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    if (n_fft) *n_fft = p->n_fft;
    if (bin_lo) *bin_lo = p->s_lo;
    if (n_out) *n_out = p->n_out;
    if (l1) *l1 = p->LA;
    if (l2) *l2 = p->LB;
    if (df) *df = p->df;
    return RSF_OK;
}

int rsf_plan_first_pass(const rsf_plan* p, int32_t* kind) {
    if (!p || !kind) return fail(RSF_EINVAL, "plan or kind is NULL");
    *kind = fft_pass_a_fixed(p->stA, p->P) ? RSF_ROWS_FIXED
            : p->rowA_fn[0]                ? RSF_ROWS_RUNTIME
            : pass_a_ept(p->LA) == kFftEPTWide ? RSF_ROWS_GENERAL_WIDE
                                           : RSF_ROWS_GENERAL;
    return RSF_OK;
}

int rsf_workspace_size(const rsf_plan* p, int entry, int64_t n_sky, int64_t n_fdot, int mode, size_t* bytes) {
    if (!p || !bytes) return fail(RSF_EINVAL, "plan or bytes is NULL");
    if (n_sky < 1 || n_fdot < 1) return fail(RSF_EINVAL, "n_sky and n_fdot must be positive");
    switch (entry) {
        case RSF_ENTRY_RESAMPLE:
            *bytes = resample_layout(p, n_sky).total;
            return RSF_OK;
        case RSF_ENTRY_FSTAT:
            if (mode != RSF_MODE_PLAIN && mode != RSF_MODE_BATCHED) return fail(RSF_EINVAL, "unknown mode");
            *bytes = fstat_layout(p, n_sky, n_fdot, mode, false, false).total;
            return RSF_OK;
        case RSF_ENTRY_TOPK:
            *bytes = fstat_layout(p, n_sky, n_fdot, RSF_MODE_BATCHED, !fused_topk(p), true).total;
            return RSF_OK;
        case RSF_ENTRY_SEMICOHERENT:
            *bytes = fstat_layout(p, n_sky, n_fdot, RSF_MODE_BATCHED, true, false, p->spin_order > 1).total;
            return RSF_OK;
        case RSF_ENTRY_POINT:
        case RSF_ENTRY_BACKWARD:
            *bytes = point_layout(p, n_fdot).total;
            return RSF_OK;
        default:
            return fail(RSF_EINVAL, "unknown entry %d", entry);
    }
}

int rsf_resample(const rsf_plan* p, const rsf_segment* seg, const double* sky, int64_t n_sky,
                 const rsf_resampled* out, void* ws, size_t ws_bytes, void* stream) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    int rc = check_segment(p, seg);
    if (rc) return rc;
    if (!sky || !out || n_sky < 1 || n_sky > 65535) return fail(RSF_EINVAL, "sky/out NULL or n_sky outside 1..65535");
    if (!ws) return fail(RSF_EINVAL, "workspace is NULL");
    const ResLayout L = resample_layout(p, n_sky);
    if (ws_bytes < L.total) return fail(RSF_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    unsigned int* flags = (unsigned int*)(w + L.flags);
    RSF_HIP(launch_fill_u32(flags, 16, 0u, s), "flags clear");
    const int64_t P = (p->n + 63) / 64;
    for (int X = 0; X < p->d.n_det; ++X) {
        ResampleArgs a = base_resample_args(p, seg, X);
        a.sky = sky;
        a.sky_stride = p->binary ? 5 : 2;
        a.binary = p->binary;
        a.LB = 64;
        a.P = P;
        a.layout = 0;
        if (p->d.storage == RSF_STORE_F16) {
            a.f16 = 1;
            a.out_zh = (uint32_t*)out[X].z;
        } else {
            a.out_z = (float2*)out[X].z;
        }
        a.out_a = out[X].a;
        a.out_b = out[X].b;
        a.out_tm = out[X].tm;
        a.out_u = out[X].u;
        a.out_mask = out[X].mask;
        a.n_words = (p->n + 31) / 32;
        a.partials = (double*)(w + L.partials) + (size_t)X * n_sky * L.n_blocks * 3;
        a.n_blocks = L.n_blocks;
        a.flags = flags;
        RSF_HIP(timed(p, K_RESAMPLE, s, [&] { return launch_resample(a, (int)n_sky, s); }), "resample launch");
    }
    ReduceArgs r{};
    r.partials = (const double*)(w + L.partials);
    r.n_blocks = L.n_blocks;
    r.n_det = p->d.n_det;
    r.n_sky = (int)n_sky;
    for (int X = 0; X < p->d.n_det; ++X) {
        r.w[X] = p->det[X].w;
        r.abc_det[X] = out[X].abc;
    }
    r.coef = (float*)(w + L.coef);
    r.flags = flags;
    RSF_HIP(timed(p, K_REDUCE, s, [&] { return launch_antenna_reduce(r, s); }), "antenna reduce launch");
    return RSF_OK;
}

namespace {
// The full path over n_sky x n_fdot templates; writes the 2F map (twoF) or,
// when topk is not null, only the k best entries.
// Semi-coherent consumer of the per-launch maps (see rsf_fstat_semicoherent).
struct SemicoOut {
    double t_ref, f_lo, df_c;
    int64_t n_c;
    float* S;
};

int run_fstat(const rsf_plan* p, const rsf_segment* seg, const double* sky, int64_t n_sky, const double* fdot,
              int64_t n_fdot, int mode, float* twoF, int k, rsf_topk_entry* topk, void* ws, size_t ws_bytes,
              void* stream, const SemicoOut* semico = nullptr) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    int rc = check_segment(p, seg);
    if (rc) return rc;
    const bool want_topk = topk != nullptr;
    const bool in_pass = want_topk && semico == nullptr && fused_topk(p);  // top-k inside the second pass
    const bool want_map = semico != nullptr || (want_topk && !in_pass);
    if (!sky || !fdot || (!twoF && !want_map && !want_topk)) return fail(RSF_EINVAL, "sky, fdot or output is NULL");
    if (n_sky < 1 || n_fdot < 1) return fail(RSF_EINVAL, "n_sky and n_fdot must be positive");
    if (mode != RSF_MODE_PLAIN && mode != RSF_MODE_BATCHED) return fail(RSF_EINVAL, "unknown mode");
    if (want_topk && (k < 1 || k > kTopkMax)) return fail(RSF_EINVAL, "k must be in 1..%d", kTopkMax);
    if (!ws) return fail(RSF_EINVAL, "workspace is NULL");
    const bool translate = semico != nullptr && p->spin_order > 1;
    const WsLayout L = fstat_layout(p, n_sky, n_fdot, mode, want_map, want_topk, translate);
    if (ws_bytes < L.total) return fail(RSF_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    unsigned int* flags = (unsigned int*)(w + L.flags);
    RSF_HIP(launch_fill_u32(flags, 16, 0u, s), "flags clear");
    // the segment demodulates with the templates' spindowns moved from t_ref
    // to its start; the semi-coherent track reads the originals
    const double* fdot_demod = fdot;
    if (translate) {
        double* moved = (double*)(w + L.spins);
        RSF_HIP(launch_spin_translate(fdot, moved, n_fdot, p->spin_order, p->d.t_start - semico->t_ref, s),
                "spindown translation launch");
        fdot_demod = moved;
    }
    const int fb = first_pass_share(p, mode);
    float4* spill = (float4*)(w + L.spill);
    const int64_t spill_stride = (int64_t)p->n_groups * p->LB * kPassBCols;
    const bool f16 = p->d.storage == RSF_STORE_F16;
    TopkItem* run[2] = {nullptr, nullptr};
    int cur = 0;
    bool have_run = false;
    TopkGate* gate = nullptr;
    if (want_topk) {
        run[0] = (TopkItem*)(w + L.run);
        run[1] = run[0] + kTopkMax;
        // threshold -inf, no candidates
        gate = (TopkGate*)(w + L.gate);
        RSF_HIP(launch_fill_u32(&gate->thr, 1, 0xff800000u, s), "top-k gate threshold");
        RSF_HIP(launch_fill_u32(gate->count, kGateParts * kGateStride, 0u, s), "top-k gate counts");
    }

    for (int64_t c0 = 0; c0 < n_sky; c0 += L.S) {
        const int sc = (int)std::min<int64_t>(L.S, n_sky - c0);
        // steps 1-5 for the chunk's skies: the resampled series, A', B', C'
        auto resample_chunk = [&]() -> int {
            for (int X = 0; X < p->d.n_det; ++X) {
                ResampleArgs a = base_resample_args(p, seg, X);
                a.sky = sky + (p->binary ? 5 : 2) * c0;
                a.sky_stride = p->binary ? 5 : 2;
                a.binary = p->binary;
                a.LB = p->LB;
                a.P = p->P;
                a.layout = 1;
                a.f16 = f16;
                a.rs_main = (float4*)(w + L.rs_main[X]);
                a.rs_tm = f16 ? nullptr : (float*)(w + L.rs_tm[X]);
                a.rs_sky_stride = L.rs_stride;
                a.partials = (double*)(w + L.partials) + (size_t)X * sc * L.n_blocks * 3;
                a.n_blocks = L.n_blocks;
                a.flags = flags;
                RSF_HIP(timed(p, K_RESAMPLE, s, [&] { return launch_resample(a, sc, s); }), "resample launch");
            }
            ReduceArgs r{};
            r.partials = (const double*)(w + L.partials);
            r.n_blocks = L.n_blocks;
            r.n_det = p->d.n_det;
            r.n_sky = sc;
            for (int X = 0; X < p->d.n_det; ++X) r.w[X] = p->det[X].w;
            r.abc_w = (double*)(w + L.abc_w);
            r.coef = (float*)(w + L.coef);
            r.flags = flags;
            RSF_HIP(timed(p, K_REDUCE, s, [&] { return launch_antenna_reduce(r, s); }), "antenna reduce launch");
            return RSF_OK;
        };
        // the plain path is the paper's chain per template: it resamples again
        // before every template's FFTs (the batched path once per sky chunk)
        const bool per_template = mode == RSF_MODE_PLAIN;
        if (!per_template && (rc = resample_chunk()) != RSF_OK) return rc;

        // launches: (first sky of the chunk, skies, first spindown, spindowns)
        struct Launch {
            int s, ns;
            int64_t f0;
            int nf;
        };
        std::vector<Launch> launches;
        if (n_fdot >= L.G) {
            for (int sk = 0; sk < sc; ++sk)
                for (int64_t f0 = 0; f0 < n_fdot; f0 += L.G)
                    launches.push_back({sk, 1, f0, (int)std::min<int64_t>(L.G, n_fdot - f0)});
        } else {
            const int per = (int)(L.G / n_fdot);
            for (int sk = 0; sk < sc; sk += per) launches.push_back({sk, std::min(per, sc - sk), 0, (int)n_fdot});
        }
        for (const Launch& q : launches) {
            if (per_template && (rc = resample_chunk()) != RSF_OK) return rc;
            PassAArgs A{};
            A.n = p->n;
            A.n_fft = p->n_fft;
            A.dt = p->d.dt;
            A.LA = p->LA;
            A.LB = p->LB;
            A.P = p->P;
            A.n_det = p->d.n_det;
            for (int X = 0; X < p->d.n_det; ++X) {
                A.w[X] = p->det[X].w;
                A.rs_main[X] = (const float4*)(w + L.rs_main[X]) + (int64_t)q.s * L.rs_stride;
                A.rs_tm[X] = f16 ? nullptr : (const float*)(w + L.rs_tm[X]) + (int64_t)q.s * L.rs_stride;
            }
            A.rs_sky_stride = L.rs_stride;
            A.f16 = f16;
            A.fdot = fdot_demod + q.f0 * p->spin_order;
            A.spin_order = p->spin_order;
            A.nf_l = q.nf;
            A.n_sky_l = q.ns;
            A.fb = fb;
            A.st = p->stA;
            A.ept = pass_a_ept(p->LA);
            A.tws_lo = p->twA;
            A.tws_hi = p->twA_hi;
            A.tw_lo = p->tw_lo;
            A.tw_hi = p->tw_hi;
            A.spill = spill;
            A.spill_tmpl_stride = spill_stride;
            // a spill larger than the last-level cache goes out (and comes back) non-temporally
            A.nt_spill = (size_t)q.ns * q.nf * (size_t)spill_stride * sizeof(float4) > kLastLevelCacheBytes ? 1 : 0;
            RSF_HIP(timed(p, K_PASS_A, s, [&] { return launch_fft_pass_a(A, s, p->rowA_fn); }), "pass A launch");

            PassBArgs B{};
            B.n_fft = p->n_fft;
            B.LA = p->LA;
            B.LB = p->LB;
            B.n_groups = p->n_groups;
            B.st = p->stB;
            B.tw_lo = p->twB;
            B.tw_hi = p->twB_hi;
            B.spill = spill;
            B.spill_tmpl_stride = spill_stride;
            B.nt_spill = A.nt_spill;
            B.coef = (const float*)(w + L.coef) + 4 * q.s;
            B.n_sky_l = q.ns;
            B.s_lo = p->s_lo;
            B.n_out = p->n_out;
            B.map_rows = want_map ? 1 : 0;
            B.twoF = want_map ? (float*)(w + L.map) : twoF;
            B.sky0 = c0 + q.s;
            B.n_fdot = n_fdot;
            B.f0 = q.f0;
            B.nf_l = q.nf;
            B.n_tmpl = q.ns * q.nf;
            B.wave = fft_pass_b_wave_e(p->LB, in_pass) != 0 ? 1 : 0;
            int64_t n_cand = 0, part_cap = 0;  // this launch's gate partitions x capacity, capacity
            if (in_pass) {
                B.topk = 1;
                B.k = k;
                B.gate = gate;
                B.cand = (TopkItem*)(w + L.cand);
                const int parts = fft_pass_b_grid(B, p->n_cu);
                const int64_t n_units = (int64_t)B.n_tmpl * B.n_groups;
                B.part_cap = (n_units + parts - 1) / parts * kGateItemsPerUnit;
                part_cap = B.part_cap;
                n_cand = parts * part_cap;
            }
            RSF_HIP(timed(p, K_PASS_B, s, [&] { return launch_fft_pass_b(B, p->n_cu, s); }), "pass B launch");

            if (semico) {
                SemicoArgs sa{};
                sa.map = (const float*)(w + L.map);
                sa.n_out = p->n_out;
                sa.s_lo = p->s_lo;
                sa.f_het = p->d.f_het;
                sa.df = p->df;
                sa.t_seg = p->d.t_start;
                sa.t_ref = semico->t_ref;
                sa.f_lo = semico->f_lo;
                sa.df_c = semico->df_c;
                sa.n_c = semico->n_c;
                sa.fdot = fdot;
                sa.order = p->spin_order;
                sa.sky0 = B.sky0;
                sa.n_fdot = n_fdot;
                sa.f0 = q.f0;
                sa.nf_l = q.nf;
                sa.n_tmpl = B.n_tmpl;
                sa.S = semico->S;
                RSF_HIP(timed(p, K_SEMICO, s, [&] { return launch_semico(sa, s); }), "semi-coherent launch");
            }
            if (want_topk) {
                if (!in_pass) {
                    TopkScanArgs ta{};
                    ta.map = (const float*)(w + L.map);
                    ta.n_vals = (int64_t)B.n_tmpl * p->n_out;
                    ta.n_out = p->n_out;
                    ta.sky0 = B.sky0;
                    ta.n_fdot = n_fdot;
                    ta.f0 = q.f0;
                    ta.nf_l = q.nf;
                    ta.k = k;
                    ta.cand = (TopkItem*)(w + L.cand);
                    ta.n_part = topk_scan_parts(ta.n_vals, &ta.part_cap);
                    ta.gate = gate;
                    part_cap = ta.part_cap;
                    n_cand = ta.n_part * part_cap;
                    RSF_HIP(timed(p, K_TOPK, s, [&] { return launch_topk_scan(ta, s); }), "topk scan launch");
                }
                if (n_cand > L.cap) return fail(RSF_EHIP, "internal: top-k candidates exceed the workspace");
                // this launch's candidates into the running k best; the gate's
                // threshold becomes their k-th
                TopkItem* const tmp[2] = {(TopkItem*)(w + L.mtmp[0]), (TopkItem*)(w + L.mtmp[1])};
                RSF_HIP(topk_merge_levels(p, s, (const TopkItem*)(w + L.cand), n_cand,
                                          have_run ? run[cur] : nullptr, run[cur ^ 1], k, n_fdot, nullptr, tmp, gate,
                                          part_cap),
                        "topk merge launch");
                cur ^= 1;
                have_run = true;
            }
        }
    }
    if (want_topk) {
        TopkItem* const tmp[2] = {(TopkItem*)(w + L.mtmp[0]), (TopkItem*)(w + L.mtmp[1])};
        RSF_HIP(topk_merge_levels(p, s, run[cur], 0, run[cur], run[cur ^ 1], k, n_fdot, topk, tmp),
                "topk final merge launch");
    }
    return RSF_OK;
}

hipError_t topk_merge_levels(const rsf_plan* p, hipStream_t s, const TopkItem* cand, int64_t n_cand,
                             const TopkItem* run_in, TopkItem* run_out, int k, int64_t n_fdot, void* entries,
                             TopkItem* const tmp[2], TopkGate* gate, int64_t part_cap) {
    const int64_t per = topk_merge_per_block();
    int b = 0;
    bool first = true;
    for (;;) {
        TopkMergeArgs ma{};
        ma.cand = cand;
        ma.n_cand = n_cand;
        // the first level reads the gate's candidates; the last one updates the gate
        ma.gate = gate;
        ma.n_gate = (gate && first) ? 1 : 0;
        ma.part_cap = part_cap;
        first = false;
        ma.run_in = run_in;
        ma.k = k;
        ma.n_fdot = n_fdot;
        ma.n_out = p->n_out;
        const int64_t total = n_cand + (run_in ? k : 0);
        const int64_t blocks = (total + per - 1) / per;
        if (blocks <= 1) {
            ma.run_out = run_out;
            ma.entries = entries;
            return timed(p, K_TOPK, s, [&] { return launch_topk_merge(ma, s); });
        }
        ma.out_blocks = tmp[b];
        const hipError_t e = timed(p, K_TOPK, s, [&] { return launch_topk_merge(ma, s); });
        if (e != hipSuccess) return e;
        cand = tmp[b];
        n_cand = blocks * k;
        run_in = nullptr;
        b ^= 1;
    }
}
}  // namespace

int rsf_fstat(const rsf_plan* p, const rsf_segment* seg, const double* sky, int64_t n_sky, const double* fdot,
              int64_t n_fdot, int mode, float* twoF, void* ws, size_t ws_bytes, void* stream) {
    if (!twoF) return fail(RSF_EINVAL, "twoF is NULL");
    return run_fstat(p, seg, sky, n_sky, fdot, n_fdot, mode, twoF, 0, nullptr, ws, ws_bytes, stream);
}

int rsf_fstat_semicoherent(const rsf_plan* p, const rsf_segment* seg, const double* sky, int64_t n_sky,
                           const double* fdot, int64_t n_fdot, double t_ref, double f_lo, double df_c, int64_t n_c,
                           float* S, void* ws, size_t ws_bytes, void* stream) {
    if (!S) return fail(RSF_EINVAL, "S is NULL");
    if (!is_fin(t_ref) || !is_fin(f_lo) || !is_fin(df_c) || df_c <= 0)
        return fail(RSF_EINVAL, "t_ref, f_lo and df_c must be finite and df_c positive");
    if (n_c < 1 || n_c > INT32_MAX * 256LL) return fail(RSF_EINVAL, "n_c out of range");
    const SemicoOut so{t_ref, f_lo, df_c, n_c, S};
    return run_fstat(p, seg, sky, n_sky, fdot, n_fdot, RSF_MODE_BATCHED, nullptr, 0, nullptr, ws, ws_bytes, stream,
                     &so);
}

int rsf_fstat_topk(const rsf_plan* p, const rsf_segment* seg, const double* sky, int64_t n_sky, const double* fdot,
                   int64_t n_fdot, int k, rsf_topk_entry* topk, void* ws, size_t ws_bytes, void* stream) {
    if (!topk) return fail(RSF_EINVAL, "topk is NULL");
    return run_fstat(p, seg, sky, n_sky, fdot, n_fdot, RSF_MODE_BATCHED, nullptr, k, topk, ws, ws_bytes, stream);
}

}  // extern "C"

namespace {
// Plans of a multi-segment call: non-null, one detector set, spindown order
// and orbit setting for all of them.
int check_plans(const rsf_plan* const* plans, int64_t n_seg) {
    if (!plans) return fail(RSF_EINVAL, "plans is NULL");
    if (n_seg < 1) return fail(RSF_EINVAL, "n_seg must be positive");
    for (int64_t i = 0; i < n_seg; ++i) {
        if (!plans[i]) return fail(RSF_EINVAL, "plans[%lld] is NULL", (long long)i);
        if (plans[i]->d.n_det != plans[0]->d.n_det || plans[i]->spin_order != plans[0]->spin_order ||
            plans[i]->binary != plans[0]->binary)
            return fail(RSF_EINVAL, "plans[%lld] differs from plans[0] in detectors, spindown order or orbit setting",
                        (long long)i);
    }
    return RSF_OK;
}

size_t segments_ws(const rsf_plan* const* plans, int64_t n_seg, int64_t n_sky, int64_t n_fdot) {
    size_t m = 0;
    for (int64_t i = 0; i < n_seg; ++i)
        m = std::max(m, fstat_layout(plans[i], n_sky, n_fdot, RSF_MODE_BATCHED, !fused_topk(plans[i]), true).total);
    return m;
}

// Segment after segment on one stream, sharing the workspace; segment i's
// top-k goes to topk[i k .. i k + k).
int run_segments(const rsf_plan* const* plans, const rsf_segment* segs, int64_t n_seg, const double* sky,
                 int64_t n_sky, const double* fdot, int64_t n_fdot, int k, rsf_topk_entry* topk, void* ws,
                 size_t ws_bytes, void* stream) {
    int rc = check_plans(plans, n_seg);
    if (rc) return rc;
    if (!segs) return fail(RSF_EINVAL, "segs is NULL");
    if (!topk) return fail(RSF_EINVAL, "topk is NULL");
    if (n_sky < 1 || n_fdot < 1) return fail(RSF_EINVAL, "n_sky and n_fdot must be positive");
    const size_t need = segments_ws(plans, n_seg, n_sky, n_fdot);
    if (ws_bytes < need) return fail(RSF_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    for (int64_t i = 0; i < n_seg; ++i) {
        rc = run_fstat(plans[i], &segs[i], sky, n_sky, fdot, n_fdot, RSF_MODE_BATCHED, nullptr, k, topk + i * k, ws,
                       ws_bytes, stream);
        if (rc) return rc;
    }
    return RSF_OK;
}
}  // namespace

extern "C" {

int rsf_segments_workspace_size(const rsf_plan* const* plans, int64_t n_seg, int64_t n_sky, int64_t n_fdot,
                                size_t* bytes) {
    int rc = check_plans(plans, n_seg);
    if (rc) return rc;
    if (!bytes) return fail(RSF_EINVAL, "bytes is NULL");
    if (n_sky < 1 || n_fdot < 1) return fail(RSF_EINVAL, "n_sky and n_fdot must be positive");
    *bytes = segments_ws(plans, n_seg, n_sky, n_fdot);
    return RSF_OK;
}

int rsf_fstat_topk_segments(const rsf_plan* const* plans, const rsf_segment* segs, int64_t n_seg, const double* sky,
                            int64_t n_sky, const double* fdot, int64_t n_fdot, int k, rsf_topk_entry* topk, void* ws,
                            size_t ws_bytes, void* stream) {
    return run_segments(plans, segs, n_seg, sky, n_sky, fdot, n_fdot, k, topk, ws, ws_bytes, stream);
}

namespace {
int point_common(const rsf_plan* p, const rsf_segment* seg, const double* theta, int64_t n, const float* g_twoF,
                 float* twoF, double* g_theta, void* ws, size_t ws_bytes, void* stream, bool grad,
                 bool instrument = true) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    int rc = check_segment(p, seg);
    if (rc) return rc;
    if (!theta) return fail(RSF_EINVAL, "theta is NULL");
    if (n < 1 || n > 65535) return fail(RSF_EINVAL, "number of candidates must be in 1..65535");
    if (grad && (!g_twoF || !g_theta)) return fail(RSF_EINVAL, "g_twoF or g_theta is NULL");
    if (!grad && !twoF) return fail(RSF_EINVAL, "twoF is NULL");
    if (!ws) return fail(RSF_EINVAL, "workspace is NULL");
    {
        // the point kernel turns the run's orbital and sidereal angles by
        // w |delta| with |delta| <= 63 dt + max|t_m| (+ a_p <= 100 s for a
        // binary source); its series needs <= 0.3
        const double span = 63.0 * p->d.dt + p->eph.au_c + p->eph.re_c + (p->binary ? 100.0 : 0.0);
        const double w_max = 2.0 * M_PI * std::max(std::fabs(p->eph.inv_p_sid), std::fabs(p->eph.inv_p_orb));
        if (!(w_max * span <= 0.3))
            return fail(RSF_EINVAL, "point search needs (63 dt + max|t_m| + 100 s if binary) w_sid <= 0.3 (dt up to about 55 s)");
    }
    const PointLayout L = point_layout(p, n);
    if (ws_bytes < L.total) return fail(RSF_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    unsigned int* flags = (unsigned int*)(w + L.flags);
    RSF_HIP(launch_fill_u32(flags, 16, 0u, s), "flags clear");
    PointArgs a{};
    a.n = p->n;
    a.dt = p->d.dt;
    a.t_start = p->d.t_start;
    a.f_het = p->d.f_het;
    a.eph = p->eph;
    a.n_det = p->d.n_det;
    for (int X = 0; X < p->d.n_det; ++X) {
        a.det[X] = p->det[X];
        a.x[X] = (const float2*)seg->x[X];
        a.gaps[X] = seg->gaps[X];
        a.n_gaps[X] = seg->n_gaps[X];
    }
    a.ip = p->ip;
    a.theta = theta;
    a.order = p->spin_order;
    a.binary = p->binary ? 1 : 0;
    // runs of 64 samples short against a sidereal day: the chain is
    // interpolated along each run (remainder below 2e-11 s in t_m)
    a.fast = (!p->binary && p->d.n_det == 1 && 63.0 * p->d.dt * 2.0 * M_PI * std::fabs(p->eph.inv_p_sid) <= 4e-3) ? 1 : 0;
    a.n_cand = (int)n;
    a.P = (p->n + 63) / 64;
    a.n_blocks = L.n_blocks;
    a.partials = (double*)(w + L.partials);
    a.flags = flags;
    // the static-scratch entry records no instrumentation events
    const rsf_plan* tp = instrument ? p : nullptr;
    auto run = [&](int kind, auto fn) { return tp ? timed(tp, kind, s, fn) : fn(); };
    RSF_HIP(run(K_POINT, [&] { return launch_point(a, grad, s); }), "point launch");
    PointReduceArgs r{};
    r.partials = a.partials;
    r.n_blocks = L.n_blocks;
    r.n_cand = (int)n;
    r.order = p->spin_order;
    r.binary = p->binary ? 1 : 0;
    r.grad = grad ? 1 : 0;
    r.g_twoF = g_twoF;
    r.twoF = twoF;
    r.g_theta = g_theta;
    r.flags = flags;
    RSF_HIP(run(K_POINT_REDUCE, [&] { return launch_point_reduce(r, s); }), "point reduce launch");
    return RSF_OK;
}
}  // namespace

int rsf_fstat_point(const rsf_plan* p, const rsf_segment* seg, const double* theta, int64_t n, float* twoF, void* ws,
                    size_t ws_bytes, void* stream) {
    return point_common(p, seg, theta, n, nullptr, twoF, nullptr, ws, ws_bytes, stream, false);
}

int rsf_fstat_backward(const rsf_plan* p, const rsf_segment* seg, const double* theta, int64_t n,
                       const float* g_twoF, float* twoF, double* g_theta, void* ws, size_t ws_bytes,
                       void* stream) {
    return point_common(p, seg, theta, n, g_twoF, twoF, g_theta, ws, ws_bytes, stream, true);
}

int rsf_fstat_backward_static(const rsf_plan* p, const rsf_segment* seg, const double* theta, int64_t n,
                              const float* g_twoF, float* twoF, double* g_theta, void* stream) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    if (n < 1 || n > 65535) return fail(RSF_EINVAL, "number of candidates must be in 1..65535");
    const hipError_t e = scratch_setup(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    const size_t need = point_layout(p, n).total;
    if (need > kStaticScratchBytes) {
        const size_t per = point_layout(p, 2).total - point_layout(p, 1).total;
        return fail(RSF_EWORKSPACE,
                    "%lld candidates need %zu bytes of device scratch, above the static %zu bytes (at most %lld "
                    "candidates at this plan's length)",
                    (long long)n, need, kStaticScratchBytes,
                    (long long)((kStaticScratchBytes - point_layout(p, 1).total) / per + 1));
    }
    return point_common(p, seg, theta, n, g_twoF, twoF, g_theta, g_scratch_ptr[p->device], kStaticScratchBytes,
                        stream, true, false);
}

}  // extern "C"

struct rsf_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {
template <typename Fn>
int capture_graph_plans(rsf_graph** out, const rsf_plan* const* plans, int64_t n_plans, Fn body) {
    if (!out) return fail(RSF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || n_plans < 1) return fail(RSF_EINVAL, "plan is NULL");
    for (int64_t i = 0; i < n_plans; ++i)
        if (!plans[i]) return fail(RSF_EINVAL, "plan is NULL");
    hipStream_t cs = nullptr;
    RSF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    // no instrumentation events inside a graph
    std::vector<char> prof_on((size_t)n_plans);
    for (int64_t i = 0; i < n_plans; ++i) {
        prof_on[i] = plans[i]->prof->on;
        plans[i]->prof->on = false;
    }
    auto restore = [&] {
        for (int64_t i = 0; i < n_plans; ++i) plans[i]->prof->on = prof_on[i] != 0;
    };
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        restore();
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    const int rc = body(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    restore();
    (void)hipStreamDestroy(cs);
    if (rc != RSF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = new rsf_graph{g, x};
    return RSF_OK;
}

template <typename Fn>
int capture_graph(rsf_graph** out, const rsf_plan* p, Fn body) {
    return capture_graph_plans(out, &p, 1, body);
}
}  // namespace

extern "C" {

int rsf_graph_create_fstat(rsf_graph** out, const rsf_plan* p, const rsf_segment* seg, const double* sky,
                           int64_t n_sky, const double* fdot, int64_t n_fdot, float* twoF, void* ws,
                           size_t ws_bytes) {
    if (!twoF) return fail(RSF_EINVAL, "twoF is NULL");
    return capture_graph(out, p, [&](hipStream_t cs) {
        return run_fstat(p, seg, sky, n_sky, fdot, n_fdot, RSF_MODE_BATCHED, twoF, 0, nullptr, ws, ws_bytes, cs);
    });
}

int rsf_graph_create_topk(rsf_graph** out, const rsf_plan* p, const rsf_segment* seg, const double* sky,
                          int64_t n_sky, const double* fdot, int64_t n_fdot, int k, rsf_topk_entry* topk,
                          void* ws, size_t ws_bytes) {
    if (!topk) return fail(RSF_EINVAL, "topk is NULL");
    return capture_graph(out, p, [&](hipStream_t cs) {
        return run_fstat(p, seg, sky, n_sky, fdot, n_fdot, RSF_MODE_BATCHED, nullptr, k, topk, ws, ws_bytes, cs);
    });
}

int rsf_graph_create_topk_segments(rsf_graph** out, const rsf_plan* const* plans, const rsf_segment* segs,
                                   int64_t n_seg, const double* sky, int64_t n_sky, const double* fdot, int64_t n_fdot,
                                   int k, rsf_topk_entry* topk, void* ws, size_t ws_bytes) {
    int rc = check_plans(plans, n_seg);
    if (rc) return rc;
    return capture_graph_plans(out, plans, n_seg, [&](hipStream_t cs) {
        return run_segments(plans, segs, n_seg, sky, n_sky, fdot, n_fdot, k, topk, ws, ws_bytes, cs);
    });
}

int rsf_graph_launch(rsf_graph* g, void* stream) {
    if (!g) return fail(RSF_EINVAL, "graph is NULL");
    RSF_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
    return RSF_OK;
}

int rsf_graph_destroy(rsf_graph* g) {
    if (!g) return RSF_OK;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return RSF_OK;
}

int rsf_profile_enable(rsf_plan* p, int on) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    p->prof->on = on != 0;
    return RSF_OK;
}

}  // extern "C"

namespace {
int profile_read(Profiler* pr, rsf_kernel_time* out, int max_kinds, int* n_kinds) {
    for (auto& r : pr->pending) {
        RSF_HIP(hipEventSynchronize(r.b), "hipEventSynchronize");
        float ms = 0.f;
        RSF_HIP(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
        pr->ms[r.kind] += ms;
        pr->launches[r.kind] += 1;
        pr->pool.push_back(r.a);
        pr->pool.push_back(r.b);
    }
    pr->pending.clear();
    int n = 0;
    for (int k = 0; k < Profiler::kKinds; ++k) {
        if (!pr->launches[k]) continue;
        if (out && n < max_kinds) {
            std::snprintf(out[n].name, sizeof(out[n].name), "%s", pr->names[k]);
            out[n].launches = pr->launches[k];
            out[n].total_ms = pr->ms[k];
        }
        ++n;
        pr->launches[k] = 0;
        pr->ms[k] = 0;
    }
    *n_kinds = n;
    return RSF_OK;
}
}  // namespace

extern "C" {

int rsf_profile_read(rsf_plan* p, rsf_kernel_time* out, int max_kinds, int* n_kinds) {
    if (!p || !n_kinds) return fail(RSF_EINVAL, "plan or n_kinds is NULL");
    return profile_read(p->prof, out, max_kinds, n_kinds);
}

int rsf_get_flags(const rsf_plan* p, void* ws, uint32_t* flags, void* stream) {
    if (!p || !ws || !flags) return fail(RSF_EINVAL, "plan, ws or flags is NULL");
    hipStream_t s = (hipStream_t)stream;
    RSF_HIP(hipMemcpyAsync(flags, ws, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "hipMemcpyAsync(flags)");
    RSF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    RSF_HIP(launch_fill_u32((unsigned int*)ws, 1, 0u, s), "flags clear");
    return RSF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// SFT front end (paper Sec. III.B)
// ---------------------------------------------------------------------------
namespace {

// W_len^{m step} for m < count, built in FP64 (long double angle), as FP32.
std::vector<float2> root_table(int64_t len, int64_t count, int64_t step) {
    std::vector<float2> t((size_t)count);
    for (int64_t m = 0; m < count; ++m) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)((m * step) % len) /
                              (long double)len;
        t[(size_t)m] = make_float2((float)std::cos((double)a), (float)std::sin((double)a));
    }
    return t;
}

int64_t next_7smooth_i(int64_t n) {
    int64_t m = std::max<int64_t>(1, n);
    while (!is_7smooth(m)) ++m;
    return m;
}

// Transform plan and tables of one chunk length n = B T_sft M'.
struct SftXform {
    int64_t n;
    int L1, L2, n_groups;
    FftStages st1, st2;
    float2 *t1, *t1_hi, *t2, *t2_hi, *tw_lo, *tw_hi;
};

struct SftChunk {
    int a0, M, Mp, xf;   // first SFT, count, 7-smooth grid, transform index
    int64_t j0, n_keep;  // output offset and kept samples
    float2 corr;         // exp(-2 pi i f_h (t_c - t_s))
};

}  // namespace

struct rsf_sft_plan {
    rsf_sft_desc d;
    Profiler* prof;
    int64_t band_bins, f_het_bins;
    std::vector<SftXform> xf;
    std::vector<SftChunk> chunks;
    std::vector<std::vector<int>> group;  // chunk ids per transform length (index of xf)
    std::vector<int64_t> gaps;            // [n][2]
    int64_t y_total;                      // band bins of all chunks
    size_t spill_total;                   // float4 elements of all spills
    int64_t merge_blocks, dft_blocks;     // workgroups of the merge and DFT launches
    int64_t fused_blocks;                 // workgroups of the fused DFT and merge launch
    size_t fused_lds;                     // its LDS; 0: the DFT tables go through HBM instead
    int64_t dft_total;                    // elements of all chunks' DFT tables
    size_t dft_lds, lds_max;
    SftChunkDev* chunks_dev;              // device table
    int* ids_dev;                         // chunk ids, grouped by length
    std::vector<int64_t> ids_off;         // first id of each group in ids_dev
    SftLenDev* lens_dev;                  // device table of the transform lengths
    int rows_R, cols_C;                   // rows per rows workgroup, columns per columns workgroup
    int64_t rows_blocks, cols_blocks;     // workgroups of the single rows / columns launches
    size_t rows_lds, cols_lds;
};

namespace {

// Workspace: normalised bins | band bins y | spill.  The DFT tables live in
// the spill's space: the merge has consumed them before the rows pass
// writes the spill (stream order).
struct SftWs {
    size_t xh, y, spill, dft, total;
};

SftWs sft_ws(const rsf_sft_plan* p) {
    SftWs L{};
    size_t off = 0;
    L.xh = off;
    if (p->d.median_window > 0) off = align_up(off + (size_t)p->d.n_sft * p->d.n_bins * sizeof(float2));
    L.y = off;
    off = align_up(off + (size_t)p->y_total * sizeof(float2));
    L.spill = off;
    L.dft = off;
    off = align_up(off + std::max(p->spill_total * sizeof(float4), (size_t)p->dft_total * sizeof(float2)));
    L.total = off;
    return L;
}

void sft_free(rsf_sft_plan* p) {
    (void)hipFree(p->chunks_dev);
    (void)hipFree(p->ids_dev);
    (void)hipFree(p->lens_dev);
    for (auto& x : p->xf) {
        (void)hipFree(x.t1);
        (void)hipFree(x.t1_hi);
        (void)hipFree(x.t2);
        (void)hipFree(x.t2_hi);
        (void)hipFree(x.tw_lo);
        (void)hipFree(x.tw_hi);
    }
    delete p->prof;
    delete p;
}

bool near_int(double x, double tol = 1e-6) { return std::fabs(x - std::nearbyint(x)) <= tol * std::max(1.0, std::fabs(x)); }

}  // namespace

extern "C" {

int rsf_sft_plan_create(rsf_sft_plan** out, const rsf_sft_desc* d, const double* t_sft) {
    if (!out || !d || !t_sft) return fail(RSF_EINVAL, "out, desc or t_sft is NULL");
    *out = nullptr;
    if (d->n_sft < 1 || d->sft_len < 1 || d->n_bins < 1 || d->n_out < 1 || d->k_lo < 0)
        return fail(RSF_EINVAL, "n_sft, sft_len, n_bins and n_out must be positive and k_lo >= 0");
    if (d->n_sft > INT32_MAX || d->n_bins > INT32_MAX || d->n_out > INT32_MAX / 2)
        return fail(RSF_EINVAL, "sizes beyond the 32-bit indexing of the kernels");
    if (!is_fin(d->dt_raw) || d->dt_raw <= 0 || !is_fin(d->band) || d->band <= 0 || !is_fin(d->f_het) ||
        !is_fin(d->t_start) || !is_fin(d->band_taper) || d->band_taper < 0 || d->band_taper > 1 ||
        !is_fin(d->edge_taper_s) || d->edge_taper_s < 0)
        return fail(RSF_EINVAL, "non-finite or out-of-range dt_raw, band, f_het, t_start or tapers");
    const double T = (double)d->sft_len * d->dt_raw;
    const double bb = d->band * T, fb = d->f_het * T;
    if (!near_int(bb) || (int64_t)std::nearbyint(bb) % 2 != 0 || !near_int(fb))
        return fail(RSF_EINVAL, "B T_sft must be an even integer and f_het T_sft an integer");
    if (d->f_het < 0.5 * d->band) return fail(RSF_EINVAL, "f_het must be at least B/2");
    if (d->dk < 0 || 2 * d->dk + 1 > kSftMaxTerms) return fail(RSF_EINVAL, "dk must be in 0..16");
    if (d->median_window != 0 &&
        (d->median_window < 1 || d->median_window % 2 == 0 || d->median_window > kSftMaxWindow ||
         d->median_window > d->n_bins))
        return fail(RSF_EINVAL, "median_window must be 0 or odd, <= 511 and <= n_bins");
    for (int64_t a = 0; a < d->n_sft; ++a) {
        if (!is_fin(t_sft[a]) || (a > 0 && !(t_sft[a] > t_sft[a - 1])))
            return fail(RSF_EINVAL, "t_sft must be finite and increasing");
        if (!near_int((t_sft[a] - d->t_start) * d->band)) return fail(RSF_EINVAL, "(t_sft - t_start) B must be integers");
    }

    auto* p = new rsf_sft_plan();
    p->d = *d;
    p->prof = new Profiler();
    p->band_bins = (int64_t)std::nearbyint(bb);
    p->f_het_bins = (int64_t)std::nearbyint(fb);
    p->y_total = 0;
    p->spill_total = 0;
    p->merge_blocks = 0;
    p->dft_blocks = 0;
    p->fused_blocks = 0;
    p->fused_lds = 0;
    p->dft_total = 0;
    p->dft_lds = 0;
    p->lds_max = 0;
    p->chunks_dev = nullptr;
    p->ids_dev = nullptr;
    p->lens_dev = nullptr;
    p->rows_R = 1;
    p->cols_C = kPassBCols;
    p->rows_blocks = p->cols_blocks = 0;
    p->rows_lds = p->cols_lds = 0;
    int dev = 0, lds_dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lds_dev, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds_dev <= 0)
        lds_dev = 65536;
    const int lds_cap = std::max(lds_dev, 163840);

    // chunks: start times exactly T_sft apart
    int64_t a0 = 0;
    for (int64_t a = 1; a <= d->n_sft; ++a) {
        if (a < d->n_sft && t_sft[a] - t_sft[a - 1] == T) continue;
        SftChunk c{};
        c.a0 = (int)a0;
        c.M = (int)(a - a0);
        c.Mp = (int)next_7smooth_i(c.M);
        const int64_t n = p->band_bins * c.Mp;
        if (c.Mp > kSftMaxGrid || n > INT32_MAX / 2) {
            sft_free(p);
            return fail(RSF_EUNSUPPORTED, "chunk transform of %lld points is too long", (long long)n);
        }
        int xi = -1;
        for (size_t i = 0; i < p->xf.size(); ++i)
            if (p->xf[i].n == n) xi = (int)i;
        if (xi < 0) {
            SftXform x{};
            x.n = n;
            if (!choose_factors(n, lds_cap, 0, &x.L1, &x.L2, false)) {
                sft_free(p);
                return fail(RSF_EUNSUPPORTED, "chunk transform of %lld points has no factorisation", (long long)n);
            }
            radix_plan(x.L1, 1, kFftThreads, kFftEPT, &x.st1);
            radix_plan(x.L2, kPassBCols, kPassBThreads, kPassBEPT, &x.st2);
            x.n_groups = (x.L1 + kPassBCols - 1) / kPassBCols;
            auto upload = [&](float2** dst, const std::vector<float2>& src) -> int {
                RSF_HIP(hipMalloc((void**)dst, src.size() * sizeof(float2)), "hipMalloc(table)");
                RSF_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(float2), hipMemcpyHostToDevice),
                        "hipMemcpy(table)");
                return RSF_OK;
            };
            const int64_t nlo = 1 << kTwSplitBits;
            int rc;
            p->xf.push_back(x);  // owned from here: freed with the plan
            SftXform& xr = p->xf.back();
            if ((rc = upload(&xr.t1, root_table(xr.L1, 32, 1))) ||
                (rc = upload(&xr.t1_hi, root_table(xr.L1, (xr.L1 + 31) / 32, 32))) ||
                (rc = upload(&xr.t2, root_table(xr.L2, 32, 1))) ||
                (rc = upload(&xr.t2_hi, root_table(xr.L2, (xr.L2 + 31) / 32, 32))) ||
                (rc = upload(&xr.tw_lo, root_table(n, nlo, 1))) ||
                (rc = upload(&xr.tw_hi, root_table(n, n / nlo + 1, nlo)))) {
                sft_free(p);
                return rc;
            }
            xi = (int)p->xf.size() - 1;
            p->group.emplace_back();
            p->lds_max = std::max({p->lds_max, fft_pass_a_lds(xr.L1), fft_pass_b_lds(xr.L2, 0, false)});
        }
        c.xf = xi;
        p->group[(size_t)xi].push_back((int)p->chunks.size());
        p->dft_lds = std::max(p->dft_lds, sft_dft_lds(c.Mp));
        const double tc = t_sft[a0] - d->t_start;
        c.j0 = (int64_t)std::nearbyint(tc * d->band);
        c.n_keep = p->band_bins * c.M;
        // f_h (t_c - t_s) reduced to cycles in FP64 before the angle is formed
        const double cyc = d->f_het * tc;
        const double fr = cyc - std::floor(cyc);
        c.corr = make_float2((float)std::cos(2.0 * M_PI * fr), (float)(-std::sin(2.0 * M_PI * fr)));
        p->chunks.push_back(c);
        a0 = a;
    }
    // rows and columns per workgroup: the most that every transform length of
    // the plan fits (stage capacity and LDS), so that the many short rows and
    // columns of these transforms come several to a workgroup
    {
        auto rows_fit = [&](int R) {
            for (const auto& x : p->xf) {
                FftStages st;
                if (!radix_plan(x.L1, R, kFftThreads, kFftEPT, &st) || sft_rows_lds(x.L1, R) > (size_t)lds_cap)
                    return false;
            }
            return true;
        };
        auto cols_fit = [&](int C) {
            for (const auto& x : p->xf) {
                FftStages st;
                if (!radix_plan(x.L2, C, kPassBThreads, kPassBEPT, &st) || sft_cols_lds(x.L2, C) > (size_t)lds_cap)
                    return false;
            }
            return true;
        };
        int R = 8, C = 32;
        while (R > 1 && !rows_fit(R)) R /= 2;
        while (C > kPassBCols && !cols_fit(C)) C /= 2;
        p->rows_R = R;
        p->cols_C = C;
        p->lds_max = 0;
        for (auto& x : p->xf) {
            radix_plan(x.L1, R, kFftThreads, kFftEPT, &x.st1);
            radix_plan(x.L2, C, kPassBThreads, kPassBEPT, &x.st2);
            x.n_groups = (x.L1 + C - 1) / C;
            p->lds_max = std::max({p->lds_max, sft_rows_lds(x.L1, R), sft_cols_lds(x.L2, C)});
        }
    }
    // gaps: output samples outside every chunk
    std::vector<std::pair<int64_t, int64_t>> cov;
    for (const auto& c : p->chunks) {
        const int64_t lo = std::max<int64_t>(c.j0, 0), hi = std::min<int64_t>(c.j0 + c.n_keep, d->n_out);
        if (lo < hi) cov.push_back({lo, hi});
    }
    std::sort(cov.begin(), cov.end());
    int64_t j = 0;
    for (const auto& r : cov) {
        if (r.first > j) {
            p->gaps.push_back(j);
            p->gaps.push_back(r.first);
        }
        j = std::max(j, r.second);
    }
    if (j < d->n_out) {
        p->gaps.push_back(j);
        p->gaps.push_back(d->n_out);
    }
    // device table of chunks: band bins, spills and merge workgroups laid end to end
    std::vector<SftChunkDev> tab(p->chunks.size());
    for (size_t i = 0; i < p->chunks.size(); ++i) {
        const SftChunk& c = p->chunks[i];
        const SftXform& x = p->xf[(size_t)c.xf];
        SftChunkDev& t = tab[i];
        t.a0 = c.a0;
        t.M = c.M;
        t.Mp = c.Mp;
        t.n = (int)x.n;
        t.b0 = p->f_het_bins * c.Mp;
        t.y_off = p->y_total;
        t.spill_off = (int64_t)p->spill_total;
        t.j0 = c.j0;
        t.n_keep = c.n_keep;
        t.blk0 = p->merge_blocks;
        t.dft_off = p->dft_total;
        t.dft_blk0 = p->dft_blocks;
        t.fblk0 = p->fused_blocks;
        t.scale = (float)(1.0 / std::sqrt((double)x.n * (double)c.M));
        t.corr = c.corr;
        p->y_total += x.n;
        p->spill_total += (size_t)x.n_groups * p->cols_C * x.L2;
        p->merge_blocks += sft_merge_blocks((int)x.n);
        p->dft_total += (int64_t)d->n_bins * c.Mp;
        p->dft_blocks += sft_dft_blocks((int64_t)d->n_bins * c.Mp);
        p->fused_blocks += sft_fused_blocks((int)x.n);
        p->fused_lds = std::max(p->fused_lds, sft_fused_lds(c.M, c.Mp, d->dk));
    }
    std::vector<int> ids;
    for (const auto& g : p->group) {
        p->ids_off.push_back((int64_t)ids.size());
        ids.insert(ids.end(), g.begin(), g.end());
    }
    // table of the transform lengths: the workgroups of the single rows and
    // columns launches, length after length
    std::vector<SftLenDev> lens(p->xf.size());
    for (size_t g = 0; g < p->xf.size(); ++g) {
        const SftXform& x = p->xf[g];
        SftLenDev& l = lens[g];
        l.n = x.n;
        l.LA = x.L1;
        l.LB = x.L2;
        l.n_groups = x.n_groups;
        l.nc = (int)p->group[g].size();
        l.id0 = (int)p->ids_off[g];
        l.rows_blk0 = p->rows_blocks;
        l.cols_blk0 = p->cols_blocks;
        l.st1 = x.st1;
        l.st2 = x.st2;
        l.t1 = x.t1;
        l.t1_hi = x.t1_hi;
        l.t2 = x.t2;
        l.t2_hi = x.t2_hi;
        l.tw_lo = x.tw_lo;
        l.tw_hi = x.tw_hi;
        // chunks of one length go through both passes in pairs
        p->rows_blocks += (int64_t)((x.L2 + p->rows_R - 1) / p->rows_R) * ((l.nc + 1) / 2);
        p->cols_blocks += (int64_t)x.n_groups * ((l.nc + 1) / 2);
        p->rows_lds = std::max(p->rows_lds, sft_rows_lds(x.L1, p->rows_R));
        p->cols_lds = std::max(p->cols_lds, sft_cols_lds(x.L2, p->cols_C));
    }
    if (hipMalloc((void**)&p->chunks_dev, tab.size() * sizeof(SftChunkDev)) != hipSuccess ||
        hipMemcpy(p->chunks_dev, tab.data(), tab.size() * sizeof(SftChunkDev), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc((void**)&p->ids_dev, ids.size() * sizeof(int)) != hipSuccess ||
        hipMemcpy(p->ids_dev, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc((void**)&p->lens_dev, lens.size() * sizeof(SftLenDev)) != hipSuccess ||
        hipMemcpy(p->lens_dev, lens.data(), lens.size() * sizeof(SftLenDev), hipMemcpyHostToDevice) != hipSuccess) {
        sft_free(p);
        return fail(RSF_EHIP, "chunk table upload failed");
    }
    const size_t lds_need = std::max(p->lds_max, p->dft_lds);
    if (lds_need > 65536 && sft_set_lds_limits(lds_need) != hipSuccess) {
        sft_free(p);
        return fail(RSF_EUNSUPPORTED, "chunk transforms need %zu bytes of LDS", lds_need);
    }
    *out = p;
    return RSF_OK;
}

int rsf_sft_plan_destroy(rsf_sft_plan* p) {
    if (p) sft_free(p);
    return RSF_OK;
}

int rsf_sft_plan_query(const rsf_sft_plan* p, int64_t* n_chunks, int64_t* gaps, int64_t max_gaps, int64_t* n_gaps) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    if (n_chunks) *n_chunks = (int64_t)p->chunks.size();
    const int64_t ng = (int64_t)p->gaps.size() / 2;
    if (n_gaps) *n_gaps = ng;
    if (gaps)
        for (int64_t i = 0; i < std::min(ng, max_gaps); ++i) {
            gaps[2 * i] = p->gaps[(size_t)(2 * i)];
            gaps[2 * i + 1] = p->gaps[(size_t)(2 * i + 1)];
        }
    return RSF_OK;
}

int rsf_sft_workspace_size(const rsf_sft_plan* p, size_t* bytes) {
    if (!p || !bytes) return fail(RSF_EINVAL, "plan or bytes is NULL");
    *bytes = sft_ws(p).total;
    return RSF_OK;
}

int rsf_sft_heterodyne(const rsf_sft_plan* p, const float* sft, float* x_h, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !sft || !x_h || !ws) return fail(RSF_EINVAL, "plan, sft, x_h or ws is NULL");
    const SftWs L = sft_ws(p);
    if (ws_bytes < L.total) return fail(RSF_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    const rsf_sft_desc& d = p->d;
    char* w = (char*)ws;
    RSF_HIP(launch_fill_u32((unsigned int*)x_h, (int)(2 * d.n_out), 0u, s), "x_h clear");
    const float2* xh = reinterpret_cast<const float2*>(sft);
    if (d.median_window > 0) {
        SftNormArgs a{};
        a.in = xh;
        a.out = reinterpret_cast<float2*>(w + L.xh);
        a.K = (int)d.n_bins;
        a.w = d.median_window;
        RSF_HIP(timed_pr(p->prof, K_SFT_NORM, s, [&] { return launch_sft_norm(a, (int)d.n_sft, s); }),
                "sft normalisation launch");
        xh = a.out;
    }
    float2* y = reinterpret_cast<float2*>(w + L.y);
    float4* spill = reinterpret_cast<float4*>(w + L.spill);
    float2* Y = reinterpret_cast<float2*>(w + L.dft);
    SftMergeArgs m{};
    m.xh = xh;
    m.Y = Y;
    m.K = (int)d.n_bins;
    m.k_lo = d.k_lo;
    m.dk = d.dk;
    m.taper = (float)d.band_taper;
    m.chunks = p->chunks_dev;
    m.n_chunks = (int)p->chunks.size();
    m.y = y;
    const char* fused_env = getenv("RSF_SFT_FUSED");
    if (p->fused_lds > 0 && p->fused_lds <= 65536 && !(fused_env && fused_env[0] == '0')) {
        // the DFT rows each workgroup's bins reach are formed in its LDS
        RSF_HIP(timed_pr(p->prof, K_SFT_DFTMERGE, s,
                         [&] { return launch_sft_dftmerge(m, p->fused_blocks, p->fused_lds, s); }),
                "sft dft and merge launch");
    } else {
        SftDftArgs f{};
        f.xh = xh;
        f.K = (int)d.n_bins;
        f.chunks = p->chunks_dev;
        f.n_chunks = (int)p->chunks.size();
        f.Y = Y;
        RSF_HIP(timed_pr(p->prof, K_SFT_DFT, s, [&] { return launch_sft_dft(f, p->dft_blocks, p->dft_lds, s); }),
                "sft dft launch");
        RSF_HIP(timed_pr(p->prof, K_SFT_MERGE, s, [&] { return launch_sft_merge(m, p->merge_blocks, s); }),
                "sft merge launch");
    }
    SftRowsArgs r{};
    r.lens = p->lens_dev;
    r.n_lens = (int)p->xf.size();
    r.chunks = p->chunks_dev;
    r.ids = p->ids_dev;
    r.y = y;
    r.spill = spill;
    RSF_HIP(timed_pr(p->prof, K_SFT_ROWS, s, [&] { return launch_sft_rows(r, p->rows_blocks, p->rows_lds, p->rows_R, s); }),
            "sft rows launch");
    SftColsArgs k{};
    k.lens = p->lens_dev;
    k.n_lens = (int)p->xf.size();
    k.chunks = p->chunks_dev;
    k.ids = p->ids_dev;
    k.spill = spill;
    k.x = reinterpret_cast<float2*>(x_h);
    k.n_out = d.n_out;
    k.n_edge = (int)std::nearbyint(d.edge_taper_s * d.band);
    RSF_HIP(timed_pr(p->prof, K_SFT_COLS, s, [&] { return launch_sft_cols(k, p->cols_blocks, p->cols_lds, p->cols_C, s); }),
            "sft cols launch");
    return RSF_OK;
}

int rsf_sft_profile_enable(rsf_sft_plan* p, int on) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    p->prof->on = on != 0;
    return RSF_OK;
}

int rsf_sft_profile_read(rsf_sft_plan* p, rsf_kernel_time* out, int max_kinds, int* n_kinds) {
    if (!p || !n_kinds) return fail(RSF_EINVAL, "plan or n_kinds is NULL");
    return profile_read(p->prof, out, max_kinds, n_kinds);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Time-domain front end (paper Sec. III.A.1)
// ---------------------------------------------------------------------------
struct rsf_hetdec_plan {
    rsf_hetdec_desc d;
    Profiler* prof;
    int L, c;
    int n_cu;   // compute units (persistent grid of the matrix-core form)
    float2* g;  // device taps
};

extern "C" {

int rsf_hetdec_plan_create(rsf_hetdec_plan** out, const rsf_hetdec_desc* d) {
    if (!out || !d) return fail(RSF_EINVAL, "out or desc is NULL");
    *out = nullptr;
    if (d->n_raw < 1 || d->n_out < 1 || d->D < 1 || d->K < 0)
        return fail(RSF_EINVAL, "n_raw, n_out and D must be positive and K >= 0");
    if (!is_fin(d->dt_raw) || d->dt_raw <= 0 || !is_fin(d->f_het) || !is_fin(d->beta) || d->beta < 0)
        return fail(RSF_EINVAL, "dt_raw must be positive and f_het, beta finite (beta >= 0)");
    const int64_t L = 2LL * d->K * d->D + 1;
    if (L > (1 << 20) || d->n_out > (int64_t)INT32_MAX * 64) return fail(RSF_EINVAL, "filter or output too long");
    const size_t lds = hetdec_lds((int)L, d->D);
    if (lds > 163840) return fail(RSF_EUNSUPPORTED, "taps and raw tile need %zu bytes of LDS (> 160 KiB)", lds);
    // Kaiser-windowed sinc, cutoff 1/(2D) cycles per raw sample, unit DC gain
    const int64_t c = (int64_t)d->K * d->D;
    std::vector<double> h((size_t)L);
    double sum = 0.0;
    const double i0b = std::cyl_bessel_i(0.0, d->beta);
    for (int64_t i = 0; i < L; ++i) {
        const double n = (double)(i - c);
        const double x = n / (double)d->D;
        const double sinc = (i == c) ? 1.0 : std::sin(M_PI * x) / (M_PI * x);
        const double r = c > 0 ? n / (double)c : 0.0;
        const double w = c > 0 ? std::cyl_bessel_i(0.0, d->beta * std::sqrt(std::max(0.0, 1.0 - r * r))) / i0b : 1.0;
        h[(size_t)i] = sinc / (double)d->D * w;
        sum += h[(size_t)i];
    }
    // heterodyne folded into the taps: exp(-2 pi i f_h (c - i) dt), angle reduced in cycles
    std::vector<float2> g((size_t)L);
    for (int64_t i = 0; i < L; ++i) {
        const double cyc = d->f_het * ((double)(c - i) * d->dt_raw);
        const double fr = cyc - std::nearbyint(cyc);
        const double v = h[(size_t)i] / sum;
        g[(size_t)i] = make_float2((float)(v * std::cos(2.0 * M_PI * fr)), (float)(-v * std::sin(2.0 * M_PI * fr)));
    }
    auto* p = new rsf_hetdec_plan();
    p->d = *d;
    p->prof = new Profiler();
    p->L = (int)L;
    p->c = (int)c;
    p->g = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || p->n_cu <= 0)
        p->n_cu = 256;
    if (hipMalloc((void**)&p->g, g.size() * sizeof(float2)) != hipSuccess ||
        hipMemcpy(p->g, g.data(), g.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p->g);
        delete p->prof;
        delete p;
        return fail(RSF_EHIP, "tap upload failed");
    }
    if (lds > 65536 && hetdec_set_lds_limit(lds) != hipSuccess) {
        (void)hipFree(p->g);
        delete p->prof;
        delete p;
        return fail(RSF_EUNSUPPORTED, "cannot grant %zu bytes of LDS", lds);
    }
    *out = p;
    return RSF_OK;
}

int rsf_hetdec_plan_destroy(rsf_hetdec_plan* p) {
    if (p) {
        (void)hipFree(p->g);
        delete p->prof;
        delete p;
    }
    return RSF_OK;
}

int rsf_hetdec(const rsf_hetdec_plan* p, const float* x, float* x_h, void* stream) {
    if (!p || !x || !x_h) return fail(RSF_EINVAL, "plan, x or x_h is NULL");
    hipStream_t s = (hipStream_t)stream;
    HetdecArgs a{};
    a.x = x;
    a.n_raw = p->d.n_raw;
    a.g = p->g;
    a.L = p->L;
    a.c = p->c;
    a.D = p->d.D;
    a.cyc_per_out = p->d.f_het * ((double)p->d.D * p->d.dt_raw);
    a.out = reinterpret_cast<float2*>(x_h);
    a.n_out = p->d.n_out;
    RSF_HIP(timed_pr(p->prof, K_HETDEC, s, [&] { return launch_hetdec(a, p->n_cu, s); }), "hetdec launch");
    return RSF_OK;
}

int rsf_hetdec_profile_enable(rsf_hetdec_plan* p, int on) {
    if (!p) return fail(RSF_EINVAL, "plan is NULL");
    p->prof->on = on != 0;
    return RSF_OK;
}

int rsf_hetdec_profile_read(rsf_hetdec_plan* p, rsf_kernel_time* out, int max_kinds, int* n_kinds) {
    if (!p || !n_kinds) return fail(RSF_EINVAL, "plan or n_kinds is NULL");
    return profile_read(p->prof, out, max_kinds, n_kinds);
}

}  // extern "C"


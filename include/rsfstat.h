/*
 * rsfstat.h -- C ABI of librsfstat: barycentric resampling and the FFT
 * F-statistic on AMD gfx950 (MI355X).
 *
 * Method: Patel, Siemens, Dupuis & Betzwieser, "Implementation of barycentric
 * resampling for continuous wave searches in gravitational wave data"
 * (arXiv:0912.4255), Sec. III.A.2 (the seven-step resampling procedure) and
 * Sec. II (the F-statistic, eqs. eq6, eq9, eq10).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Time t is measured from the segment start; the segment starts t_start
 *   seconds after the ephemeris epoch.  Samples are x_h[j] at t_j = j dt.
 * - x_h is the heterodyned, downsampled complex series x(t) exp(-2 pi i f_het t)
 *   (heterodyne sign of the worked example in Sec. III.A.1), complex64
 *   interleaved (re, im), zero-filled inside gaps (Sec. III.B, "Gaps in the
 *   data").
 * - The SSB grid is t_b^k = k dt, k = 0..n-1.  T^k is the detector time with
 *   T^k + t_m(T^k) = t_b^k (eq. eq21), t_m = n0 . r_d / c (eq. eq4pt2).
 * - Spindown phase Phi_s = 2 pi fdot (T^2/2 + t_m T) (eq. eq4pt1, s = 1),
 *   applied as exp(-i Phi_s); orders 2 and 3 through rsf_plan_set_spin_order.
 * - Output bin s (signed) is the frequency f_het + s / (n_fft dt); bands are
 *   reported in ascending s.
 * - 2F = 2 (B'|f_a|^2 + A'|f_b|^2 - 2 C' Re(f_a f_b^*)) / D' with
 *   noise-weighted sums (weights 1/sigma_X^2) over detectors (eq. eq6).
 *
 * Memory and streams
 * ------------------
 * Every array argument is caller-owned DEVICE memory unless marked "host".
 * The library allocates device memory only in rsf_plan_create (constant
 * tables); every other call uses the caller's workspace `ws` of at least the
 * size reported by rsf_workspace_size.  `stream` is a hipStream_t passed as
 * void* (NULL = the default stream); all work is enqueued asynchronously on
 * it and no call synchronises the device.
 *
 * Errors
 * ------
 * Every call returns RSF_OK (0) or a negative rsf_status; the message of the
 * last failure on the calling thread is available from rsf_last_error().
 * Nothing aborts or throws across this interface.  A template whose Gram
 * determinant D' is not positive (e.g. an all-gap segment) yields NaN outputs
 * and sets RSF_FLAG_DEGENERATE in the flags word readable with rsf_get_flags.
 * A run of 64 consecutive resampled times whose interpolation windows span
 * more detector samples than a wave stages (only for time compressions far
 * beyond any physical Doppler factor) yields NaN samples there and sets
 * RSF_FLAG_WINDOW.  A binary orbit outside the admitted range (see
 * rsf_plan_set_binary) makes the kernels that read it set RSF_FLAG_ORBIT and
 * give NaN: every resampled sample of that sky row, hence every 2F of its
 * templates (which top-k selection then skips), or that candidate's 2F and
 * gradient in rsf_fstat_point / rsf_fstat_backward.
 */
#ifndef RSFSTAT_H
#define RSFSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSF_MAX_DET 4
#define RSF_MAX_TAPS 32

typedef enum rsf_status {
    RSF_OK = 0,
    RSF_EINVAL = -1,        /* null pointer, non-positive size, non-finite parameter, band outside data */
    RSF_EUNSUPPORTED = -2,  /* FFT length not 7-smooth or not decomposable; taps odd or > 32 */
    RSF_EWORKSPACE = -3,    /* workspace smaller than rsf_workspace_size */
    RSF_EHIP = -4           /* HIP runtime or launch error (message kept) */
} rsf_status;

enum { RSF_KERNEL_LANCZOS = 0, RSF_KERNEL_DIRICHLET = 1 };
enum { RSF_NFFT_TWICE = 0, RSF_NFFT_SMOOTH7 = 1, RSF_NFFT_SMOOTH7_256 = 2 };
enum { RSF_STORE_F32 = 0, RSF_STORE_F16 = 1 };
enum { RSF_MODE_PLAIN = 0, RSF_MODE_BATCHED = 1 };
enum {
    RSF_ENTRY_RESAMPLE = 0, RSF_ENTRY_FSTAT = 1, RSF_ENTRY_POINT = 2, RSF_ENTRY_BACKWARD = 3, RSF_ENTRY_TOPK = 4,
    RSF_ENTRY_SEMICOHERENT = 5
};
enum { RSF_FLAG_DEGENERATE = 1, RSF_FLAG_WINDOW = 2, RSF_FLAG_ORBIT = 4 };

/* Interferometer site: latitude, longitude (rad, east positive), azimuth of
 * the arm bisector counter-clockwise from local East (rad; arms at +-45 deg),
 * and the noise variance sigma^2 = E|n|^2 per complex sample. */
typedef struct rsf_detector {
    double lat, lon, gamma, sigma2;
} rsf_detector;

/* Analytic ephemeris: circular orbit of radius au_c light-seconds in the
 * ecliptic (obliquity eps) with period p_orb, spherical Earth of radius re_c
 * light-seconds rotating with sidereal period p_sid; lambda0 and theta0 are
 * the orbital longitude and Greenwich sidereal angle at the epoch. */
typedef struct rsf_ephemeris {
    double au_c, re_c, p_orb, p_sid, eps, lambda0, theta0;
} rsf_ephemeris;

typedef struct rsf_plan_desc {
    int32_t n_det;                   /* 1..RSF_MAX_DET */
    int32_t nfft_policy;             /* RSF_NFFT_TWICE: 2n; RSF_NFFT_SMOOTH7: smallest even 2^a3^b5^c7^d >= 2n;
                                        RSF_NFFT_SMOOTH7_256: smallest 256 2^a3^b5^c7^d >= 2n (a length the
                                        one-column-per-wave second pass can take, LB = 256, 512 or 768) */
    int32_t kernel;                  /* RSF_KERNEL_LANCZOS or RSF_KERNEL_DIRICHLET */
    int32_t taps;                    /* even, 2..RSF_MAX_TAPS */
    int32_t storage;                 /* RSF_STORE_F32 or RSF_STORE_F16 (resampled series kept as half2) */
    int32_t fft_l1;                  /* first-pass FFT length L1 (a divisor of n_fft), 0 = automatic */
    int64_t n;                       /* samples per detector */
    double dt;                       /* sampling interval, s */
    double t_start;                  /* segment start after the ephemeris epoch, s */
    double f_het;                    /* heterodyne frequency, Hz */
    double f_lo, f_hi;               /* reported band [f_lo, f_hi), Hz, inside f_het +- 1/(2 dt) */
    rsf_ephemeris eph;
    rsf_detector det[RSF_MAX_DET];
} rsf_plan_desc;

/* One data segment: per detector a device pointer to complex64[n] and a
 * device int64[n_gaps][2] list of half-open, sorted, disjoint gap ranges in
 * samples (may be NULL when n_gaps is 0). */
typedef struct rsf_segment {
    const void* x[RSF_MAX_DET];
    const int64_t* gaps[RSF_MAX_DET];
    int32_t n_gaps[RSF_MAX_DET];
} rsf_segment;

/* Outputs of rsf_resample for one detector, each [n_sky][...] row-major:
 * z: complex64[n] resampled series z~(t_b^k) (eq. eq19's z(t_b^k));
 * a, b: float32[n] beam patterns at T^k; tm: float64[n] t_m,k = t_b^k - T^k;
 * mask: uint32[ceil(n/32)] bit k = nearest-sample mask m~_k;
 * abc: float64[3] unweighted A' = sum m~ a^2, B' = sum m~ b^2, C' = sum m~ a b;
 * u: float64[n] u_k = T^k / dt, the detector-grid position the series is
 *    interpolated at (eq. eq21's inversion divided by the sampling interval).
 * Any pointer may be NULL to skip that output. */
typedef struct rsf_resampled {
    void* z;
    float* a;
    float* b;
    double* tm;
    uint32_t* mask;
    double* abc;
    double* u;
} rsf_resampled;

typedef struct rsf_topk_entry {
    float twoF;
    int32_t sky;
    int32_t fdot;
    int32_t bin;     /* index into the ascending band, 0..n_out-1 */
} rsf_topk_entry;

typedef struct rsf_plan rsf_plan;

/* Create a plan: validates the descriptor, chooses the FFT factorisation
 * n_fft = L1 * L2 and uploads constant tables (the only device allocation
 * the library makes).  *out is NULL on failure. */
int rsf_plan_create(rsf_plan** out, const rsf_plan_desc* desc);
int rsf_plan_destroy(rsf_plan* plan);

/* Spindown order of the plan's templates (eq. eq4pt1 with s = order, 1..3;
 * default 1).  With order s, every `fdot` argument of rsf_fstat,
 * rsf_fstat_topk and the graph builders is double [n_fdot][s]: row i holds
 * (f^(1), ..., f^(s)) of template i, and
 * Phi_s = 2 pi sum_j f^(j) (T^{j+1}/(j+1)! + t_m T^j/j!), and every `theta`
 * of rsf_fstat_point / rsf_fstat_backward is double [n][3 + s]:
 * (f, f^(1), ..., f^(s), alpha, delta).  The semi-coherent sum takes its
 * templates' spindowns at t_ref and moves them to each segment's start
 * (see rsf_fstat_semicoherent). */
int rsf_plan_set_spin_order(rsf_plan* plan, int order);

/* Sources in circular binary orbits (on != 0; default off).  Every `sky`
 * argument becomes double [n_sky][5]: (alpha, delta, a_p, P_b, t_asc) with
 * the projected semi-major axis a_p in light-seconds (0 <= a_p <= 100), the
 * period P_b in seconds (finite, > 0, 2 pi a_p / P_b <= 1e-2) and the time of
 * the ascending node t_asc (finite) on the clock of t_start; rows outside
 * this range give NaN and RSF_FLAG_ORBIT.  A wavefront emitted at tau_e reaches the
 * SSB at tau_e + R(tau_e), R = a_p sin(2 pi (tau_e - t_asc) / P_b).  The
 * resampled grid is then regular in emission time: T^k solves
 * T + t_m(T) = k dt + R(t_start + k dt), and the heterodyne correction and
 * the spindown phase use the total delay d = t_m - R(tau_e) in place of t_m.
 * Every `theta` of rsf_fstat_point / rsf_fstat_backward then ends with the
 * candidate's orbit, double [n][6 + s]: (f, f^(1), ..., f^(s), alpha, delta,
 * a_p, P_b, t_asc), with a_p <= 100 light-s, and the gradient includes
 * d2F/d(a_p, P_b, t_asc). */
int rsf_plan_set_binary(rsf_plan* plan, int on);
/* Batching knobs of RSF_MODE_BATCHED (0 = keep the automatic value):
 * fb = spindowns sharing one read of the resampled series in the first FFT
 * pass (1..16); templates = templates per FFT launch (1..256). */
int rsf_plan_set_batching(rsf_plan* plan, int fb, int templates);

/* Host only (no device needed): the factorisation n_fft = L1 * L2 that
 * rsf_plan_create would choose on a device with lds_bytes of LDS per
 * workgroup (fft_l1 > 0 forces L1), for checking FFT lengths in advance.
 * RSF_EUNSUPPORTED when n_fft is not 7-smooth or no factorisation fits. */
int rsf_fft_factor(int64_t n_fft, int lds_bytes, int fft_l1, int32_t* l1, int32_t* l2);

/* Effective batching of rsf_fstat / rsf_fstat_topk for n_sky x n_fdot
 * templates in `mode`: spindowns sharing a first-pass row (*fb), templates
 * per FFT launch (*templates) and sky positions resampled per launch
 * (*skies).  Host outputs, any may be NULL. */
int rsf_plan_batching(const rsf_plan* plan, int64_t n_sky, int64_t n_fdot, int mode, int32_t* fb,
                      int32_t* templates, int32_t* skies);

/* Host outputs (any may be NULL): FFT length, first signed bin and number of
 * bins of the reported band, FFT factors (L1 = first-pass length over the
 * slow input index, L2 = second-pass length), frequency spacing df. */
int rsf_plan_query(const rsf_plan* plan, int64_t* n_fft, int64_t* bin_lo, int64_t* n_out,
                   int32_t* l1, int32_t* l2, double* df);

/* First-pass kernel kinds (rsf_plan_first_pass).  The first FFT pass
 * (Sec. III.A.2, step 6: rows of length L1 in LDS) runs either the planned
 * radix stages of a general kernel or a kernel whose radix sequence is fixed
 * at compile time (constant stage sizes, per-stage twiddle tables): one
 * compiled into the library, or one compiled at plan creation with hipRTC
 * from the library's own headers (found beside the library, checked against
 * the hash recorded when it was built; cached on disk under
 * $RSF_KERNEL_CACHE, else $XDG_CACHE_HOME/rsfstat or ~/.cache/rsfstat).
 * Run-time kernels are made for transforms of 2^19 points or more
 * (RSF_RTC=all: any size; RSF_RTC=0: never) whose rows end below L1/2 (the
 * pruned first stage); when that is not possible the general kernel runs
 * (RSF_RTC_VERBOSE=1 prints the compiler's log of a failed compile).  A
 * cached code object that does not load is compiled again.
 * Every kind computes the same transform to FP32 rounding. */
enum { RSF_ROWS_GENERAL = 0, RSF_ROWS_GENERAL_WIDE = 1, RSF_ROWS_FIXED = 2, RSF_ROWS_RUNTIME = 3 };

/* Host output: the kind of first-pass kernel the plan's transforms run on
 * (RSF_ROWS_GENERAL: planned stages, up to 21 complex pairs per thread;
 * RSF_ROWS_GENERAL_WIDE: up to 32, for rows that run one workgroup per CU;
 * RSF_ROWS_FIXED, RSF_ROWS_RUNTIME: see above). */
int rsf_plan_first_pass(const rsf_plan* plan, int32_t* kind);

/* Workspace bytes for an entry point (RSF_ENTRY_*) with the given numbers of
 * sky positions, spindowns (or candidates for POINT/BACKWARD) and mode. */
int rsf_workspace_size(const rsf_plan* plan, int entry, int64_t n_sky, int64_t n_fdot, int mode,
                       size_t* bytes);

/* Steps 1-5 of Sec. III.A.2 for every sky position and detector:
 * heterodyne correction on the detector grid (z = x_h exp(-2 pi i f_het t_m),
 * eqs. absorb/Fa3), inversion of eq. eq21, interpolation of z at T^k, beam
 * patterns a, b at T^k and the masked antenna sums (eqs. eq9/eq10).
 * sky: device float64[n_sky][2] = (alpha, delta) in rad (equatorial).
 * out: host array of n_det rsf_resampled descriptors. */
int rsf_resample(const rsf_plan* plan, const rsf_segment* seg, const double* sky, int64_t n_sky,
                 const rsf_resampled* out, void* ws, size_t ws_bytes, void* stream);

/* The full path (Sec. III.A.2 steps 1-7) for n_sky x n_fdot templates:
 * 2F over the reported band for every (sky, fdot).
 * fdot: device float64[n_fdot] (Hz/s).  twoF: device float32
 * [n_sky * n_fdot][n_out], row = sky * n_fdot + fdot, ascending frequency.
 * mode RSF_MODE_PLAIN is the paper's chain per template: it resamples the
 * series and launches the two FFT passes once per template;
 * RSF_MODE_BATCHED resamples several sky positions per launch, shares each
 * resampled series between all spindowns of its sky and 16 of them in the
 * first FFT pass, and runs 64 templates per launch (defaults; see
 * rsf_plan_set_batching).  Both modes give identical results. */
int rsf_fstat(const rsf_plan* plan, const rsf_segment* seg, const double* sky, int64_t n_sky,
              const double* fdot, int64_t n_fdot, int mode, float* twoF,
              void* ws, size_t ws_bytes, void* stream);

/* As rsf_fstat (batched) but returning only the k largest 2F values over all
 * templates and bins of the band, descending, ties broken by the lower
 * (sky, fdot, bin); NaN values never enter; missing entries (fewer than k
 * finite values) have twoF = -inf and indices -1.  Workspace: entry
 * RSF_ENTRY_TOPK.  topk: device rsf_topk_entry[k], 1 <= k <= 64. */
int rsf_fstat_topk(const rsf_plan* plan, const rsf_segment* seg, const double* sky, int64_t n_sky,
                   const double* fdot, int64_t n_fdot, int k, rsf_topk_entry* topk,
                   void* ws, size_t ws_bytes, void* stream);

/* Several data segments of uneven length in one call: the template loop of
 * Sec. IV.A (over the sky positions and spindowns, the same templates for
 * every segment) run over n_seg segments, each reduced to its own k best.
 * plans: HOST array of n_seg plan pointers, plans[i] describing segment i
 * (its n, dt, t_start, f_het, band, interpolation kernel and taps, FFT
 * factorisation and batching knobs, so each segment may carry its own tuned
 * settings); every plan must have the same n_det, spindown order and orbit
 * setting, else RSF_EINVAL.  segs: HOST array of n_seg segment descriptors
 * (device series and gap lists, as for rsf_fstat).  sky, fdot: as for
 * rsf_fstat_topk, shared by all segments; each segment's spindowns refer to
 * its own start (phase reference t = 0 at its t_start).  topk: device
 * rsf_topk_entry [n_seg][k], 1 <= k <= 64: row i holds segment i's k largest
 * 2F over its templates and the bins of its band (bin = index into segment
 * i's ascending band), ordered and tie-broken as rsf_fstat_topk.  The
 * segments run one after another on `stream` without any host
 * synchronisation, sharing one workspace of at least
 * rsf_segments_workspace_size bytes (the largest any segment needs). */
int rsf_segments_workspace_size(const rsf_plan* const* plans, int64_t n_seg, int64_t n_sky, int64_t n_fdot,
                                size_t* bytes);
int rsf_fstat_topk_segments(const rsf_plan* const* plans, const rsf_segment* segs, int64_t n_seg, const double* sky,
                            int64_t n_sky, const double* fdot, int64_t n_fdot, int k, rsf_topk_entry* topk, void* ws,
                            size_t ws_bytes, void* stream);

/* Semi-coherent ("stack-slide") sum over segments, the hierarchical scheme
 * named in the paper's introduction, as a plain sum of per-segment 2F along
 * each template's frequency track.  Template (sky, f0, fdot) has f0 at the
 * reference time t_ref (seconds, the clock of t_start); this segment, whose
 * phase reference is its start t_start, sees f = f0 + fdot (t_start - t_ref)
 * (at spin order s: f = f0 + sum_k f^(k) D^k / k!, D = t_start - t_ref, the
 * terms formed and added in order of k in FP64 without fused multiply-adds,
 * and the segment demodulates with f^(j)(t_start) = sum_{k >= j} f^(k)
 * D^(k-j) / (k-j)!, computed into the workspace)
 * and adds its 2F at the nearest bin floor((f - f_het) / df + 1/2) (FP64),
 * nothing when that bin is outside its reported band.  Common grid
 * f0_j = f_lo + j df_c, j < n_c.  S: float [n_sky * n_fdot][n_c] (device,
 * row sky * n_fdot + fdot), ACCUMULATED (+=): zero it before the first
 * segment and call once per segment on one stream.  Workspace:
 * rsf_workspace_size(plan, RSF_ENTRY_SEMICOHERENT, n_sky, n_fdot, ...). */
int rsf_fstat_semicoherent(const rsf_plan* plan, const rsf_segment* seg, const double* sky, int64_t n_sky,
                           const double* fdot, int64_t n_fdot, double t_ref, double f_lo, double df_c, int64_t n_c,
                           float* S, void* ws, size_t ws_bytes, void* stream);

/* 2F at continuous parameters: theta device float64[n][3 + s] = (f Hz,
 * f^(1) Hz/s, ..., f^(s) Hz/s^s, alpha, delta rad) at the plan's spindown
 * order s (1 by default: (f, fdot, alpha, delta)), followed by the orbit
 * (a_p, P_b, t_asc) when the plan's sources are binary;
 * f_a(f) = sum_k y^a_k exp(-2 pi i (f - f_het) k dt) on the
 * resampled series of each candidate's own sky (equal to FFT bin s when
 * f = f_het + s df).  twoF: device float32[n]. */
int rsf_fstat_point(const rsf_plan* plan, const rsf_segment* seg, const double* theta, int64_t n,
                    float* twoF, void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of rsf_fstat_point: g_theta[i][:] = g_twoF[i] *
 * d2F/d(f, f^(1), ..., f^(s), alpha, delta[, a_p, P_b, t_asc]) at theta[i], through the
 * F-statistic, the Fourier sum, the spindown phase (including its
 * dependence on the sky through T and t_m), the interpolation, the heterodyne
 * correction, the beam patterns and the timing inversion (dT/dtheta =
 * -(dt_m/dtheta)/(1 + dt_m/dt)).  The resampled series is recomputed, never
 * stored.  g_twoF: device float32[n]; twoF: device float32[n] or NULL;
 * g_theta: device float64, the shape of theta. */
int rsf_fstat_backward(const rsf_plan* plan, const rsf_segment* seg, const double* theta, int64_t n,
                       const float* g_twoF, float* twoF, double* g_theta,
                       void* ws, size_t ws_bytes, void* stream);

/* rsf_fstat_backward for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the scratch (per-candidate partial sums and the
 * flags word) in a static device array of the library, 64 MiB per GPU, held
 * from the first plan created on that GPU until the process ends.  No
 * workspace argument; nothing is allocated and no instrumentation event is
 * recorded.  The caller passes theta, g_twoF, twoF (may be NULL) and g_theta
 * as for rsf_fstat_backward.  Returns RSF_EWORKSPACE (message: the largest n
 * that fits) when n candidates need more scratch than the array holds (about
 * 110 KB per candidate at n = 1,728,000 samples, i.e. up to about 600
 * candidates), RSF_EHIP if the array's device address could not be
 * resolved.  All calls on one GPU share the array: calls that overlap in
 * time on one GPU (several streams or threads) race and must be serialised
 * by the caller.  Flags are cleared at the start of each call. */
int rsf_fstat_backward_static(const rsf_plan* plan, const rsf_segment* seg, const double* theta, int64_t n,
                              const float* g_twoF, float* twoF, double* g_theta, void* stream);

/* A batched search captured once into a HIP graph and replayed with one
 * launch (the template loop of Sec. IV.A as a single launchable unit).
 * rsf_graph_create_fstat / _topk record exactly the work of rsf_fstat
 * (mode RSF_MODE_BATCHED) / rsf_fstat_topk with the given, fixed pointers,
 * on a private stream; nothing runs until rsf_graph_launch, which enqueues
 * the whole graph on `stream`.  Every pointer argument must stay valid and
 * unchanged while the graph exists; replays overwrite twoF / topk and the
 * workspace.  Returns RSF_EHIP if capture or instantiation fails. */
typedef struct rsf_graph rsf_graph;

int rsf_graph_create_fstat(rsf_graph** out, const rsf_plan* plan, const rsf_segment* seg, const double* sky,
                           int64_t n_sky, const double* fdot, int64_t n_fdot, float* twoF, void* ws,
                           size_t ws_bytes);
int rsf_graph_create_topk(rsf_graph** out, const rsf_plan* plan, const rsf_segment* seg, const double* sky,
                          int64_t n_sky, const double* fdot, int64_t n_fdot, int k, rsf_topk_entry* topk,
                          void* ws, size_t ws_bytes);
/* rsf_fstat_topk_segments over all n_seg segments captured into one graph
 * (plans and segs are read at capture; the device buffers they and the other
 * arguments point to must stay valid while the graph exists). */
int rsf_graph_create_topk_segments(rsf_graph** out, const rsf_plan* const* plans, const rsf_segment* segs,
                                   int64_t n_seg, const double* sky, int64_t n_sky, const double* fdot, int64_t n_fdot,
                                   int k, rsf_topk_entry* topk, void* ws, size_t ws_bytes);
int rsf_graph_launch(rsf_graph* graph, void* stream);
int rsf_graph_destroy(rsf_graph* graph);

/* Instrumentation (not part of the method): when enabled, every kernel the
 * plan launches is bracketed by hipEvents recorded on the launch stream.
 * rsf_profile_read synchronises on those events, writes up to max_kinds
 * records {kernel name, launches, summed milliseconds} (host memory), sets
 * *n_kinds and clears the counters. */
typedef struct rsf_kernel_time {
    char name[32];
    int64_t launches;
    double total_ms;
} rsf_kernel_time;

int rsf_profile_enable(rsf_plan* plan, int on);
int rsf_profile_read(rsf_plan* plan, rsf_kernel_time* out, int max_kinds, int* n_kinds);

/* Copy the device flags word (RSF_FLAG_*) of the workspace to *flags (host)
 * and clear it; synchronises `stream`. */
int rsf_get_flags(const rsf_plan* plan, void* ws, uint32_t* flags, void* stream);

/* ---------------------------------------------------------------------------
 * SFT front end (paper Sec. III.B): from short Fourier transforms to the
 * heterodyned, downsampled series x_h that the entry points above take.
 *
 * Input: SFTs X_{alpha,k} = sum_j x_{alpha,j} exp(-2 pi i j k / N) (eq. e25) of
 * consecutive stretches of N = sft_len raw samples (T_sft = N dt_raw), of
 * which bins k_lo .. k_lo + n_bins - 1 (frequency k / T_sft) are kept, as
 * complex64 [n_sft][n_bins]; SFT alpha starts at t_sft[alpha] (host, seconds,
 * increasing, on the clock of t_start).
 * Steps (the summary closing Sec. III.B):
 *   1. normalisation X^ = X / sqrt(S) (eq. dimlessSFTs1), S = running median
 *      of |X|^2 over median_window bins (window clamped inside the stored
 *      band) divided by ln 2; median_window = 0 skips it (S = 1);
 *   2. chunks: SFTs whose start times differ by exactly T_sft;
 *   3. per chunk of M SFTs, the long-baseline transform on the grid of
 *      M' = the smallest 7-smooth number >= M (zero SFTs appended; M' = M
 *      when M is 7-smooth): X_b = sum_alpha e^{-2 pi i b alpha / M'}
 *      sum_{|k - k*| <= dk} X^_{alpha,k} P_{b,k}, k* = floor(b / M'), with the
 *      large-N kernel P = sin(y)/y - i (1 - cos y)/y, y = 2 pi (b/M' - k)
 *      (eqs. e9, e91, e75); terms outside the stored band are absent;
 *   4. the band of B T_sft M' bins centred on bin f_h T_sft M' is relabelled
 *      (f_h -> DC), multiplied by a Tukey window (cosine taper over a
 *      fraction band_taper of the band) and inverse transformed; scale
 *      1 / sqrt(B T_sft M' M), so normalised white noise has unit power;
 *   5. the first B T_sft M samples are the chunk at t_c + j / B; they are
 *      multiplied by exp(-2 pi i f_h (t_c - t_start)) (eq. hetStartCorr with
 *      this interface's heterodyne sign), tapered over edge_taper_s seconds
 *      at each chunk edge (Tukey) and written to x_h[(t_c - t_start) B + j];
 *      samples outside every chunk are zero (gaps).
 * Requirements: f_het T_sft an integer, B T_sft an even integer, f_het >=
 * B/2, (t_sft - t_start) B integers, odd median_window <= min(n_bins, 511),
 * dk <= 16, and every chunk's transform length decomposable (up to about
 * 10^7 points); otherwise RSF_EINVAL / RSF_EUNSUPPORTED from
 * rsf_sft_plan_create.
 * ------------------------------------------------------------------------- */
typedef struct rsf_sft_desc {
    int64_t n_sft;          /* number of SFTs */
    int64_t sft_len;        /* raw samples per SFT, N */
    double dt_raw;          /* raw sampling interval, s */
    int64_t k_lo;           /* first stored bin */
    int64_t n_bins;         /* stored bins per SFT */
    double t_start;         /* start of the output series, s */
    double f_het;           /* heterodyne frequency, Hz */
    double band;            /* output band B, Hz (output dt = 1/B) */
    int64_t n_out;          /* output samples */
    int32_t dk;             /* Dirichlet terms on each side of k* */
    int32_t median_window;  /* running-median bins (odd), 0 = no normalisation */
    double band_taper;      /* Tukey fraction of the band window, 0..1 */
    double edge_taper_s;    /* taper at each chunk edge, s */
} rsf_sft_desc;

typedef struct rsf_sft_plan rsf_sft_plan;

/* Chunking, per-chunk transform plans and their twiddle tables (device
 * memory owned by the plan).  t_sft: host [n_sft]. */
int rsf_sft_plan_create(rsf_sft_plan** out, const rsf_sft_desc* desc, const double* t_sft);
int rsf_sft_plan_destroy(rsf_sft_plan* plan);
/* Number of chunks and the gaps of the output series as half-open sample
 * ranges (host [max_gaps][2]; *n_gaps is the full count even when larger
 * than max_gaps).  Pure host query. */
int rsf_sft_plan_query(const rsf_sft_plan* plan, int64_t* n_chunks, int64_t* gaps, int64_t max_gaps,
                       int64_t* n_gaps);
int rsf_sft_workspace_size(const rsf_sft_plan* plan, size_t* bytes);
/* sft: complex64 [n_sft][n_bins] (device, read only); x_h: complex64 [n_out]
 * (device, overwritten, gaps zero).  Asynchronous on `stream`.  The DFT over
 * a chunk's SFTs and the Dirichlet merge run as one kernel with the DFT rows
 * in LDS when every chunk fits 64 KiB of it (chunks up to several hundred
 * SFTs), else as two with the DFT tables in the workspace; RSF_SFT_FUSED=0
 * forces the second form. */
int rsf_sft_heterodyne(const rsf_sft_plan* plan, const float* sft, float* x_h, void* ws, size_t ws_bytes,
                       void* stream);
/* Kernel timing of the plan's launches, as rsf_profile_enable/read. */
int rsf_sft_profile_enable(rsf_sft_plan* plan, int on);
int rsf_sft_profile_read(rsf_sft_plan* plan, rsf_kernel_time* out, int max_kinds, int* n_kinds);

/* ---------------------------------------------------------------------------
 * Time-domain front end (paper Sec. III.A.1, eqs. eq14-eq16): from a real
 * high-rate series x[m] (float32, m < n_raw, sample m at m dt_raw from the
 * series start) to the heterodyned, downsampled series
 *   x_h[j] = sum_i h[i] x[j D + c - i] exp(-2 pi i f_het (j D + c - i) dt_raw),
 * j < n_out, with output sample j at j D dt_raw (band B = 1 / (D dt_raw)).
 * h: L = 2 K D + 1 taps centred on c = K D, a sinc with cutoff B/2 (the new
 * Nyquist frequency) times a Kaiser window of parameter beta, normalised to
 * unit gain at DC.  Raw samples outside [0, n_raw) count as zero.  The taps
 * (heterodyne folded in, FP64 then FP32) live in the plan.  Requirements:
 * D >= 1, K >= 0, beta >= 0, the taps and a tile of raw samples fitting in
 * LDS (about (63 D + 3 L) * 4 bytes <= 160 KiB). */
typedef struct rsf_hetdec_desc {
    int64_t n_raw;    /* raw samples */
    double dt_raw;    /* raw sampling interval, s */
    double f_het;     /* heterodyne frequency, Hz */
    int32_t D;        /* downsampling factor */
    int32_t K;        /* filter half-length in output samples */
    double beta;      /* Kaiser window parameter */
    int64_t n_out;    /* output samples */
} rsf_hetdec_desc;

typedef struct rsf_hetdec_plan rsf_hetdec_plan;

int rsf_hetdec_plan_create(rsf_hetdec_plan** out, const rsf_hetdec_desc* desc);
int rsf_hetdec_plan_destroy(rsf_hetdec_plan* plan);
/* x: float32 [n_raw] (device); x_h: complex64 [n_out] (device, overwritten).
 * No workspace.  Asynchronous on `stream`. */
int rsf_hetdec(const rsf_hetdec_plan* plan, const float* x, float* x_h, void* stream);
int rsf_hetdec_profile_enable(rsf_hetdec_plan* plan, int on);
int rsf_hetdec_profile_read(rsf_hetdec_plan* plan, rsf_kernel_time* out, int max_kinds, int* n_kinds);

/* Message of the last failed call on this thread ("" if none). */
const char* rsf_last_error(void);

/* ABI version, currently 1. */
int rsf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RSFSTAT_H */

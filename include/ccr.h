/*
 * ccr.h -- C ABI of the MI355X (gfx950) resampled cross-correlation library.
 *
 * The library computes the resampled cross-correlation statistic rho of
 * Meadors, Krishnan, Papa, Whelan and Zhang, "Resampling to accelerate
 * cross-correlation searches for continuous gravitational waves from binary
 * systems" (Phys. Rev. D 97, 044017), eq. final-formatted-rho, for every
 * orbital template (a_p, T_asc, P) of a band and every decimated output
 * frequency bin at once:
 *
 *   1. time base      per source sample tau_r = t0 + r dt: the detector time
 *                     t_r with tau(t_r) = tau_r, where t_SSB = t + r(t).n
 *                     (eq. t-ssb-equation) and tau = t_SSB - a_p sin(Omega
 *                     (t_SSB - T_asc)) (eq. tau-equation, circular orbit);
 *                     the delay Delta_r = t_r - tau_r;
 *   2. resampling     windowed-sinc interpolation of the heterodyned series
 *                     at t_r (eq. shannon-interp-formula, D taps each side,
 *                     Hamming window of length 2D+1) and the heterodyne
 *                     correction exp(+2 pi i f_h Delta_r)
 *                     (eq. resampled-time-series-q-eq);
 *   3. spectra        zero-padded FFT of each T_short segment, decimated bins
 *                     kbar = k_lo + floor(nu_R i), phase referenced to the
 *                     series origin (Phi_in, Sec. III.B.4-5);
 *   4. pair sum       rho_i = sqrt(2) Re sum_{pairs} W_KL conj(F_K) F_L / N with
 *                     W_KL = hat a_K hat a_L + hat b_K hat b_L (eq.
 *                     geometric-filter) over the pair set of Sec. III.B.1 and
 *                     the normalisation N of App. A.
 *
 * Conventions
 *   - Times are seconds after the context epoch (time 0); angles in radians.
 *   - Complex samples are interleaved float32 (re, im).
 *   - Every ccr_set_* call copies its inputs: caller buffers may be freed on
 *     return.  Outputs are caller-allocated.
 *   - Every call returns a status; on failure nothing is written to caller
 *     outputs and ccr_last_error() holds a message.  No C++ exception crosses
 *     this boundary.
 *   - One context is not thread-safe; separate contexts are independent.
 *   - Device work is queued on the given HIP stream (or the context's own
 *     stream when NULL); outputs are complete after ccr_sync().
 *   - FP64 results are bitwise reproducible for a given input and plan.
 */
#ifndef CCR_H
#define CCR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CCR_ABI_VERSION 4
#define CCR_MAX_DET 8
#define CCR_PAIRS_CROSS 1 /* pairs across detectors, |K - L| <= R        */
#define CCR_PAIRS_SAME 2  /* pairs within a detector, 0 < L - K <= R     */
#define CCR_PAIRS_ALL 4   /* every ordered pair of segments of every detector, auto-correlations
                             included, any lag: rho = sqrt2 (|F_a|^2 + |F_b|^2) / N, the
                             F-statistic limit (App. A.1-A.2); not combined with the two above */
#define CCR_WEIGHT_AVE 0  /* pair weight Gamma^ave (eq. geometric-filter)                     */
#define CCR_WEIGHT_CIRC 1 /* pair weight Gamma^circ = hat a_K hat b_L - hat b_K hat a_L (Sec.
                             II.B), on the imaginary part of conj(F_K) F_L              */

typedef struct ccr_ctx ccr_ctx;

typedef enum {
    CCR_OK = 0,
    CCR_EINVAL = -1,  /* bad argument: null pointer, NaN/Inf, inconsistent sizes or lattices */
    CCR_ENOMEM = -2,  /* host or device allocation failed */
    CCR_EDEVICE = -3, /* HIP runtime error */
    CCR_ESTATE = -4,  /* call order: data, weights or templates missing */
    CCR_ERANGE = -5,  /* a plan quantity outside what the kernels support */
    CCR_EUNSUP = -6   /* option not supported */
} ccr_status;

typedef enum {
    CCR_PREC_FP64 = 0,  /* time base, interpolation, FFT and pair sum in FP64 */
    CCR_PREC_SPLIT = 1  /* FP64 time base and phases; FP32 interpolation, FFT and pair products.
                           Pair products of one pass of a pair-sum kernel (the segments of one
                           step, a few at a time) are summed in FP32, the passes in FP64 */
} ccr_precision;

/* Source direction and the analytic Earth model of the detector position r(t):
 * circular orbit of radius au_s light-seconds in the ecliptic plane (ecliptic
 * longitude orbit_phase0 + 2 pi t / year_s), ecliptic tilted by `obliquity`;
 * rotation of a spherical Earth of radius re_s light-seconds with sidereal
 * angle gmst0 + 2 pi t / sidereal_day_s (Sec. II.A.2, eq. t-ssb-equation,
 * Roemer term only). */
typedef struct {
    double ra, dec;
    double au_s, re_s;
    double obliquity;
    double year_s, sidereal_day_s;
    double orbit_phase0, gmst0;
} ccr_sky;

/* Detector site on the spherical Earth (radians). */
typedef struct {
    double lat, lon;
} ccr_site;

/* One analysis band.
 *   f_min, f_band  output band [f_min, f_min + f_band] (Hz); f_h = f_min + f_band / 2
 *   t_short        segment length T_short (s)
 *   max_lag        R, T_max = R T_short (eq. lag-time-constraint)
 *   dirichlet_D    D interpolation taps on each side (typ. 8)
 *   window         0: Hamming indexed by tap, w_n = 0.54 - 0.46 cos(2 pi (n + D) / 2D);
 *                  1: Hamming at the continuous offset d, w = 0.54 + 0.46 cos(pi d / (D + 1))
 *   n_fft_override 0: N_FFT from eq. n-fft-final; otherwise N_FFT (a multiple of the power of
 *                  two holding N_K)
 *   mu_f           frequency mismatch (delta lambda_f = sqrt(6 mu_f / pi) / T_coh)
 *   pairs          CCR_PAIRS_CROSS | CCR_PAIRS_SAME, or CCR_PAIRS_ALL (max_lag then only sets
 *                  T_coh, hence the frequency resolution)
 *   a_p_max, orbit_period  size the Doppler wings of the load bandwidth (App. B,
 *                  eq. delta-f-load with eqs. f-drift-eq, delta-f-obs, v/c = 1e-4)
 *   weight         CCR_WEIGHT_AVE or CCR_WEIGHT_CIRC.  Gamma^circ:
 *                  rho = sqrt2 sum_P (hat b_K hat a_L - hat a_K hat b_L) Im(conj(F_K) F_L) / N with
 *                  N^2 = sum_P A_K B_L + B_K A_L - 2 C_K C_L (positive mean for cos iota > 0). */
typedef struct {
    double f_min, f_band, t_short;
    int32_t max_lag, dirichlet_D, window, n_fft_override;
    double mu_f;
    int32_t pairs;
    double a_p_max, orbit_period;
    int32_t weight;
} ccr_band;

/* Plan of a band.  Fields after n_k / dt are valid once every detector has data. */
typedef struct {
    int64_t n_k;          /* samples per segment; the series must be sampled at dt = t_short / n_k */
    int64_t n_seg;        /* M segments (floor(n / n_k)) */
    int64_t n_fft;        /* N_FFT */
    int64_t n_f;          /* decimated output bins per template */
    int64_t k_lo;         /* first FFT bin (signed) */
    int64_t n_pairs;      /* |P| */
    int64_t n_det;        /* detectors with data */
    int64_t n_templates;  /* templates set */
    int64_t n_active;     /* (detector, segment) entries that take part in a pair and are computed */
    double dt, f_het, df_load, t_coh, dlambda_f, t_fft, nu_r;
    double norm;          /* N of App. A (0 when no pair carries weight) */
    /* Split-precision resampling in Farrow form (Sec. III.A interpolation, eq.
     * shannon-interp-formula, evaluated as one
     * polynomial in the offset per sample): polynomial degree of the tap weights, 0 when the
     * band has no Farrow table (the fit's error bound is too large, or no device memory for
     * it: the direct 2D + 1-tap form runs instead); farrow_err = max over offsets of
     * sum_n |fitted - exact tap weight| (relative to the input amplitude). */
    int64_t farrow_degree;
    double farrow_err;
    /* The segment FFT as the kernels take it: N_FFT = P n_s, P transforms of n_s points per
     * (template, detector, segment), one per residue class of the output bins (n_s the power of
     * two holding N_K, at least 256 where N_FFT allows). */
    int64_t n_s, P;
} ccr_band_info;

int ccr_abi_version(void);

/* Create a context on HIP device `hip_device`.  `sky` is copied.  hip_device = -1 creates a
 * host-only context: bands, data, weights, templates and band plans work, every call that
 * needs a device returns CCR_EDEVICE. */
ccr_status ccr_create(ccr_ctx **out, int hip_device, const ccr_sky *sky);
/* Free every host and device resource of the context (waits for queued work). */
void ccr_destroy(ccr_ctx *ctx);
/* Message of the last failing call on this context ("" if none).  Valid until the next call. */
const char *ccr_last_error(const ccr_ctx *ctx);

/* Set an option (value >= 0).  Names:
 *   "template_batch"  templates per work item (one band's share of a launch), 0 = as many as
 *                     the workspace budget holds;
 *   "workspace_mb"    device workspace budget in MiB (resampled series, spectra, partials),
 *                     at least 64; 0 (the default) = 3/4 of the device memory that is free,
 *                     plus what the context's workspace already holds, at the context's first
 *                     compute call (fixed from then on; fewer, larger launch rounds);
 *   "k_chunk"         segments per pair-sum chunk, 0 = min(M, 256) or the tuned value;
 *   "fused"           1: fused resample + FFT + pair kernel where a band fits it, 0: staged;
 *   "items_per_launch" work items per launch, 0 = as many as the workspace holds (1 with
 *                     template_batch 1: one template per launch sequence, no batching);
 *   "timing"          1: time every kernel launch with HIP events (see ccr_kernel_time);
 *   "graph"           1: capture each distinct compute call (bands, precision, device
 *                     outputs) as a HIP graph on first use and replay it afterwards; a change
 *                     of data, templates, weights, workspace or launch options re-captures;
 *                     applies to device outputs only;
 *   "round_templates" at most this many templates in one launch round (0, the default: as
 *                     many as the workspace budget holds);
 *   "spectra_kernel"  1: run the 256- to 1024-point spectra + pair-sum kernel on every band
 *                     it takes, also where the 256-point one applies; 0 (default): the
 *                     256-point kernel first;
 *   "autotune"        1: on the first call for a given band list and precision, time the
 *                     first launch round of each candidate launch shape and keep the fastest
 *                     per template: the spectra kernel (where a band can take either) and
 *                     k_chunk = 32 ... 1024 on a round of at most 64 templates a band, then
 *                     the templates per launch round (the workspace budget's batch, its half
 *                     and quarter) where timing those rounds stays below about 12 s (an
 *                     explicit "k_chunk" disables tuning);
 *   "farrow"          1 (default): split-precision resampling in Farrow form where the band
 *                     has the table (see ccr_band_info.farrow_degree), 0: the direct
 *                     2D + 1-tap form.  FP64 always uses the direct form;
 *   "farrow_stage"    1 (default): the Farrow kernel stages each chunk's table entries in
 *                     LDS; 0: every sample reads them from global memory (the path a chunk
 *                     takes when its range is too wide for LDS; slower, for testing).
 * All bands of a compute call run in shared launches: one launch per stage covers the work
 * items of many bands (grouped by kernel variant, packed to the workspace budget).
 * Returns CCR_EUNSUP for an unknown name. */
ccr_status ccr_set_option(ccr_ctx *ctx, const char *name, int64_t value);

/* Read an option set with ccr_set_option, or "tuned_k_chunk" / "tuned_template_batch" /
 * "tuned_round_templates" / "tuned_spectra_kernel": the launch shape the autotuner chose last
 * (0, or -1 for the kernel, before any tuning), or "resample_templates": the
 * templates one resampling workgroup handles from one staged input window (a constant of the
 * build), "farrow_templates" / "farrow_degree": the same for the Farrow-form kernel and its
 * polynomial degree.  CCR_EUNSUP for an unknown name. */
ccr_status ccr_get_option(ccr_ctx *ctx, const char *name, int64_t *value);

/* Add a band; returns its id and the part of the plan known before data (n_k, dt, f_het,
 * df_load).  Bands are independent. */
ccr_status ccr_add_band(ccr_ctx *ctx, const ccr_band *band, int *band_id, ccr_band_info *info);

/* Heterodyned, downsampled complex series of detector `det` (0 <= det < CCR_MAX_DET) for a
 * band (Sec. III, App. B): x[2q], x[2q+1] = Re, Im of x'(t0 + q dt), q < n.
 * dt must equal t_short / n_k of the band and satisfy n_k >= t_short df_load (else
 * CCR_ERANGE); t0 and dt must be the same for every detector of the band; f_het must equal
 * f_min + f_band / 2; n >= n_k.  `valid` (n bytes, NULL = all valid) marks gaps: invalid
 * samples are read as zero.  NaN/Inf samples give CCR_EINVAL. */
ccr_status ccr_set_data(ccr_ctx *ctx, int band_id, int det, const ccr_site *site, double t0,
                        double dt, int64_t n, double f_het, const float *x, const uint8_t *valid);

/* Per-segment weights of detector `det` (n_seg = floor(n / n_k) entries each): antenna
 * functions a_K, b_K at the segment mid-time and the noise variance E|x'|^2 of the
 * segment (> 0).  hat a = a / sigma (Sec. II.B, eq. geometric-filter). */
ccr_status ccr_set_weights(ccr_ctx *ctx, int band_id, int det, int64_t n_seg, const double *a,
                           const double *b, const double *noise_var);

/* Per-sample antenna functions of detector `det` (Sec. III.B.3, eq. norm-a-eq): a[r], b[r] =
 * a(tau_r), b(tau_r) on the source lattice tau_r = t0 + r dt, r < n; n must be at least the
 * band's n_seg * n_k (checked when the band is prepared; CCR_EINVAL).  Once every detector of
 * the band has them, the resampled series is weighted sample by sample before the FFT, giving
 * two spectra per segment, F^a_K = FFT(hat a_r y_r) and F^b_K = FFT(hat b_r y_r) (hat a_r =
 * a_r / sigma_K), and rho = sqrt2 Re sum_P [conj(F^a_K) F^a_L + conj(F^b_K) F^b_L] / N with
 * N^2 = sum_P A_K A_L + 2 C_K C_L + B_K B_L, A_K the segment mean of m_r hat a_r^2 (m_r the gap
 * mask), B_K, C_K likewise (Gamma^circ: sqrt2 sum_P Im[conj(F^b_K) F^a_L - conj(F^a_K) F^b_L] / N).
 * The per-segment a_K, b_K of ccr_set_weights are then not used (their noise_var is).  Copied;
 * n = 0 (or null arrays) removes them.  NaN/Inf give CCR_EINVAL. */
ccr_status ccr_set_antenna(ccr_ctx *ctx, int band_id, int det, int64_t n, const double *a, const double *b);

/* Orbital templates of a band (the Doppler parameters lambda of Sec. II.A.2, circular orbit,
 * eq. tau-equation): n >= 1 triples (a_p [s], T_asc [s after epoch], P [s]).  a_p >= 0, P > 0,
 * all finite; otherwise (or n < 1, or a null array) CCR_EINVAL and the band keeps its previous
 * templates.  Replaces the band's template list (copied). */
ccr_status ccr_set_templates(ccr_ctx *ctx, int band_id, int64_t n, const double *a_p,
                             const double *t_asc, const double *period);


/* Eccentric orbital templates (Sec. II.A.2, eqs. solve-for-E and Kepler-equation): the binary
 * delay is R/c = a_p [sin omega (cos E - e) + cos omega sqrt(1 - e^2) sin E] with
 * E - e sin E = Omega (t_SSB - T_p), Omega = 2 pi / P, the anomaly taken at the SSB time of the
 * detector sample as the circular orbit takes its phase; with e = 0 this is the circular orbit
 * with T_asc = T_p - omega / Omega.  Arrays of n: a_p (s, >= 0), t_p (periapse time, s after
 * the epoch), omega (argument of periapse, rad), e (0 <= e <= 0.95, else CCR_EINVAL), period
 * (s, > 0).  Replaces the band's templates (as ccr_set_templates).  When the band is prepared
 * a template whose Kepler solve or time-base interpolation the library cannot bound over a
 * segment (e too large for the segment length) gives CCR_ERANGE. */
ccr_status ccr_set_templates_ecc(ccr_ctx *ctx, int band_id, int64_t n, const double *a_p, const double *t_p,
                                 const double *omega, const double *e, const double *period);

/* Full plan of a band (Sec. III.B.1-2: M, T_coh, delta lambda_f, N_FFT by eq. n-fft-final,
 * nu_R; App. B eq. delta-f-load; the normalisation N of App. A); bin_freqs (n_f doubles, may be
 * NULL) receives the output frequencies f_het + kbar_i / T_FFT, kbar_i = k_lo + floor(nu_R i)
 * (Sec. III.B.2, bin-centred frequencies).  CCR_ESTATE before every detector has data. */
ccr_status ccr_get_band_info(ccr_ctx *ctx, int band_id, ccr_band_info *info, double *bin_freqs);

/* rho of eq. final-formatted-rho (Sec. III.B.6) for every template and bin of each listed band:
 * steps 1-4 above on the device, in the precision `prec`.  rho_out[b] points to
 * n_templates * n_f values (row-major, template-major) of double (out_fp64 = 1) or float,
 * in device memory (out_on_device = 1, must stay valid until ccr_sync) or host memory
 * (written before the call returns).  hip_stream: a hipStream_t, or NULL for the context's
 * own stream.  The calls of one context share its workspace: queue them on one stream (or
 * synchronise between streams); calls that overlap on different streams race. */
ccr_status ccr_compute_rho(ccr_ctx *ctx, ccr_precision prec, int n_bands, const int *band_ids,
                           void *const *rho_out, int out_on_device, int out_fp64, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ccr_compute_rho with device outputs whose workspace
 * (band and work-item tables, time-base coefficients, resampled series, spectra, chunk
 * partials) lives in a fixed device array of 256 MiB per device instead of the context's
 * workspace.  The call makes no hipMalloc, hipFree or other allocating call; it queues a table
 * copy and the kernels on hip_stream (NULL: the context's stream) and returns.
 *   - Every band must be prepared beforehand (set-up that allocates): after its data, weights
 *     and templates are set, call ccr_get_band_info (or ccr_compute_rho) once; otherwise
 *     CCR_ESTATE.
 *   - rho_out[b]: device memory, n_templates * n_f values (double if out_fp64, else float), valid
 *     until the work completes.  Templates are processed in as many launch rounds as the fixed
 *     array requires; a band whose single-template workspace exceeds it (e.g. 240 days at
 *     T_short 1440 s in FP64) gives CCR_ERANGE, as do band and work-item tables over 1 MiB.
 *   - Options "template_batch" and "k_chunk" apply; "graph", "autotune" and "timing" do not.
 *   - The array is shared by every call on the device and keeps the last call's contents; no
 *     part of it needs to start at zero.  Calls that overlap on one device (different
 *     contexts or streams) race: order them on one stream or synchronise between them.
 * Results equal ccr_compute_rho's for the same options. */
ccr_status ccr_compute_rho_noalloc(ccr_ctx *ctx, ccr_precision prec, int n_bands, const int *band_ids,
                                   void *const *rho_out, int out_fp64, void *hip_stream);

/* The heterodyned, downsampled series of one detector from its short Fourier transforms (App. B,
 * downsampling and heterodyning), computed on the context's device: the input of ccr_set_data.
 *   n_sft, t_sft, t0   SFT K covers [t0 + K t_sft, t0 + (K + 1) t_sft) (seconds after the epoch)
 *   n_bins, k_first    bins held per SFT, frequencies k / t_sft for k = k_first .. k_first + n_bins - 1
 *   z                  n_sft x n_bins complex bins (interleaved float32, host), the transform
 *                      z_k = dt sum_j x_j exp(-2 pi i j k / N) of the SFT's N samples x_j
 *   sft_valid          n_sft flags (host) or NULL: a missing SFT (0) gives zeros
 *   f_het              heterodyne frequency (the band's f_min + f_band / 2)
 *   n_out              N' samples per SFT (1 .. 4096; at least t_sft x the band's load bandwidth)
 *   x_out, valid_out   n_sft x n_out complex (interleaved float32, host) and 0/1 bytes (or NULL)
 * Output sample j of SFT K, at t = t0 + K t_sft + j t_sft / N', is
 *   exp(-2 pi i f_het t_K) sum_{k} z_{K,k} exp(2 pi i (k - f_het t_sft) j / N') / t_sft,
 * the sum over the N' bins k_h - h .. k_h - h + N' - 1 around the nearest bin k_h to f_het
 * (h = floor(N'/2)), t_K = t0 + K t_sft: the band's inverse transform (eq. freq-shifted-eq),
 * stitched across SFTs by the phase of eq. long-time-series-het-corrected and heterodyned by
 * f_het itself (the remainder of f_het off the bin grid is applied, not dropped).  With
 * t_sft = the band's T_short and N' its N_K, the series has the band's lattice (dt = T_short /
 * N_K).  CCR_ERANGE when the SFTs do not hold the N' bins; CCR_EINVAL for NaN/Inf. */
ccr_status ccr_sft_series(ccr_ctx *ctx, int64_t n_sft, double t_sft, double t0, int64_t n_bins, int64_t k_first,
                          const float *z, const uint8_t *sft_valid, double f_het, int64_t n_out, float *x_out,
                          uint8_t *valid_out);

/* Wait for all work queued by this context. */
ccr_status ccr_sync(ccr_ctx *ctx);

/* Device time of the kernels ccr_compute_rho launched while option "timing" was 1, summed
 * since the last ccr_reset_kernel_times (HIP events recorded on the launch stream around each
 * launch).  kernel: 0 resampling, 1 segment spectra, 2 pair sum, 3 final scaling,
 * 4 fused resampling + spectra + pair sum, 5 FP64 time base (per-segment interpolating polynomial),
 * 6 spectra + pair sum in one kernel (split precision, 256-point segments), 7 the same for
 * 1024-point segments, 8 the SFT front end (ccr_sft_series).
 * Waits for the recorded launches to finish. */
ccr_status ccr_kernel_time(ccr_ctx *ctx, int kernel, double *ms, int64_t *launches);
ccr_status ccr_reset_kernel_times(ccr_ctx *ctx);

/* Stage outputs of one template, for kernel-level checks.  Host buffers.
 * ccr_resample_series: y of detector det, n_seg * n_k complex values (double pairs for
 *   CCR_PREC_FP64, float pairs for CCR_PREC_SPLIT) -- step 2 including the gap mask.
 *   Segments that no pair uses are returned as zeros.
 * ccr_segment_spectra: F[det][K][i], n_det * n_seg * n_f complex values, normalised by
 *   1 / (sigma_XK sqrt(n_k)) -- step 3.  Segments that no pair uses are zeros. */
ccr_status ccr_resample_series(ccr_ctx *ctx, ccr_precision prec, int band_id,
                               int64_t template_index, int det, void *y_out);
ccr_status ccr_segment_spectra(ccr_ctx *ctx, ccr_precision prec, int band_id,
                               int64_t template_index, void *f_out);
/* ccr_time_base: step 1 for every source sample r of segments [k0, k0 + n_seg_out) of
 *   detector det (active segments only; others are left untouched), as the resampler uses it:
 *   eta_out[r - k0 n_k] = eta_r (s) with the delay Delta_r = t_r - tau_r = eta_r - anchor_out[K - k0],
 *   anchor_out (n_seg_out doubles, may be NULL) = the segment's anchor offset D_a (s), and
 *   psi_out[r - k0 n_k] (may be NULL) = frac(f_het Delta_r) (cycles), the heterodyne phase.
 *   Host buffers of n_seg_out * n_k doubles (anchor_out: n_seg_out). */
ccr_status ccr_time_base(ccr_ctx *ctx, int band_id, int64_t template_index, int det, int64_t k0,
                         int64_t n_seg_out, double *eta_out, double *anchor_out, double *psi_out);

#ifdef __cplusplus
}
#endif
#endif /* CCR_H */

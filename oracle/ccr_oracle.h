/*
 * Oracle for the resampled cross-correlation statistic rho (test infrastructure).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code with the HIP library.
 *
 * A plain, slow, obviously-correct CPU implementation: long double for the
 * time base and every phase, double for interpolation, the DFT (a direct sum,
 * no FFT) and the pair sum (explicit pair loops).  Each function names the
 * passage of the paper it follows.  Times are seconds after a common epoch.
 */
#ifndef CCR_ORACLE_H
#define CCR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CCO_MAX_DET 8
#define CCO_PAIRS_CROSS 1
#define CCO_PAIRS_SAME 2
#define CCO_PAIRS_ALL 4   /* every ordered pair of segments of every detector, auto-correlations
                             included, any lag (App. A.1-A.2: the F-statistic limit) */

enum { CCO_OK = 0, CCO_EINVAL = -1, CCO_ENOMEM = -2, CCO_ERANGE = -5 };

typedef struct {
    double ra, dec;                 /* source direction (rad) */
    double au_s, re_s;              /* orbit radius, Earth radius (light-seconds) */
    double obliquity;               /* rad */
    double year_s, sidereal_day_s;  /* orbital and rotation periods (s) */
    double orbit_phase0, gmst0;     /* ecliptic longitude and sidereal angle at the epoch (rad) */
} cco_sky;

typedef struct {
    double f_min, f_band, t_short;
    int max_lag;          /* R: T_max = R * T_short */
    int dirichlet_D;      /* D taps each side */
    int window;           /* 0: Hamming indexed by tap; 1: Hamming at the continuous offset */
    int n_fft_override;   /* 0: eq. n-fft-final; else N_FFT (multiple of the pow2 >= N_K) */
    double mu_f;          /* frequency mismatch */
    int pairs;            /* CCO_PAIRS_CROSS | CCO_PAIRS_SAME, or CCO_PAIRS_ALL */
    double a_p_max;       /* largest a_p (sizes the Doppler wings) */
    double orbit_period;  /* P used for the wing width */
    int weight;           /* 0: Gamma^ave (eq. geometric-filter); 1: Gamma^circ (Sec. II.B) */
} cco_band;

typedef struct {
    int64_t n_k, n_seg, n_fft, n_f, k_lo;
    double dt, f_het, df_load, t_coh, dlambda_f, t_fft, nu_r;
} cco_plan;

typedef struct {
    cco_sky sky;
    cco_band band;
    int n_det;
    double lat[CCO_MAX_DET], lon[CCO_MAX_DET];
    double t0, dt;                          /* common sample lattice t_q = t0 + q dt */
    int64_t n;                              /* samples per detector */
    double f_het;
    const float *x[CCO_MAX_DET];            /* interleaved complex, n each */
    const uint8_t *valid[CCO_MAX_DET];      /* n each, or NULL = all valid */
    const double *a[CCO_MAX_DET], *b[CCO_MAX_DET], *noise_var[CCO_MAX_DET];  /* n_seg each */
    /* per-sample antenna functions a(tau_r), b(tau_r) on the source lattice (n_seg * n_k each,
       Sec. III.B.3 eq. norm-a-eq), or NULL: per-segment a, b above */
    const double *ar[CCO_MAX_DET], *br[CCO_MAX_DET];
    /* 0: templates (a_p, T_asc, P), circular orbit; 1: templates (a_p, T_p, omega, e, P),
       eccentric orbit (Sec. II.A.2 eqs. solve-for-E, Kepler-equation) */
    int ecc;
} cco_problem;

int cco_plan_band(const cco_problem *p, cco_plan *out);
/* frequency index kbar of output bin i (may be negative) */
int64_t cco_bin_index(const cco_plan *pl, int64_t i);

/* Earth Roemer delay r(t).n for detector det at time t. */
double cco_earth_delay(const cco_problem *p, int det, double t);
/* Forward map: tau(t) - t for one template (eqs. t-ssb-equation, tau-equation); a template
   is 3 doubles (a_p, T_asc, P) or, with ecc, 5 (a_p, T_p, omega, e, P). */
double cco_forward_offset(const cco_problem *p, int det, const double *tmpl, double t);
/* Eccentric anomaly E of mean anomaly M: E - e sin E = M (eq. solve-for-E). */
double cco_kepler(double M, double e);
/* Delay Delta_r = t_r - tau_r of source sample r (inverse map, long double Newton).
   Writes Delta as hi + lo doubles. */
int cco_delay(const cco_problem *p, int det, const double *tmpl, int64_t r, double *hi, double *lo);

/* Resampled series of one detector for one template: y (2 * n_seg * n_k doubles,
   interleaved), optional jstar / offset / mask per sample (may be NULL). */
int cco_resample(const cco_problem *p, int det, const double *tmpl, double *y,
                 int64_t *jstar, double *offset, uint8_t *mask);
/* Segment valid fractions phi[det][K] (n_det * n_seg). */
int cco_valid_fraction(const cco_problem *p, double *phi);
/* Per-segment spectra F[det][K][i] (2 * n_det * n_seg * n_bins doubles), tier 0 = resampled
   (method steps), tier 1 = direct detector-frame demodulation with no interpolation.
   bins: indices into 0..n_f-1, or NULL for all. */
int cco_spectra(const cco_problem *p, const double *tmpl, int tier, const int64_t *bins,
                int64_t n_bins, double *F);
/* Normalisation sqrt(sum_P A A + 2 C C + B B). */
double cco_norm(const cco_problem *p);
/* Number of pairs in P. */
int64_t cco_pair_count(const cco_problem *p);
/* rho[t][i] for n_tmpl templates (rows of 3 or, with ecc, 5), OpenMP over templates. */
int cco_rho(const cco_problem *p, const double *tmpl, int64_t n_tmpl, int tier,
            const int64_t *bins, int64_t n_bins, double *rho);
int cco_num_threads(void);
/* Heterodyned, downsampled series from SFT bins (App. B): z holds n_sft x n_bins complex bins
   (interleaved doubles) starting at bin k_first (frequency k_first / t_sft); SFT K starts at
   t0 + K t_sft; output x (2 * n_sft * n_out doubles) at t0 + K t_sft + j t_sft / n_out.  ERANGE when
   the n_out bins around f_het are not all held. */
int cco_sft_series(int64_t n_sft, double t_sft, double t0, int64_t n_bins, int64_t k_first, const double *z,
                   const uint8_t *sft_valid, double f_het, int64_t n_out, double *x);

#ifdef __cplusplus
}
#endif
#endif

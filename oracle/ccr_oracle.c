/*
 * Oracle for the resampled cross-correlation statistic rho.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.
 *
 * Steps follow the paper in its own order (Meadors et al., "Resampling to
 * accelerate cross-correlation searches for continuous gravitational waves
 * from binary systems"):
 *   plan      Sec. III.B.2 (eqs. n-fft-final, delta lambda_f), App. B (eq. delta-f-load)
 *   time base Sec. II.A.2 (eqs. t-ssb-equation, tau-equation; circular R/c, or the eccentric
 *             orbit of eqs. solve-for-E and Kepler-equation), Sec. III.A.2
 *   interp    Sec. III.A.1 (eq. shannon-interp-formula), Sec. III.A.2 (eqs. delta-q-eq,
 *             q-prime-eq, resampled-time-series-q-eq)
 *   spectra   Sec. III.B.5 (zero-padded DFT of each T_short segment) with Phi_in of Sec. III.B.4
 *   pairs     Sec. III.B.1 (pair selection {L|K}); all pairs with auto-correlations, App. A.1-A.2
 *   weights   eq. geometric-filter (Gamma^ave) or Gamma^circ (Sec. II.B); per-segment a_K, b_K
 *             or per-sample a_r, b_r (Sec. III.B.3, eq. norm-a-eq)
 *   rho       Sec. III.B.6 (eq. final-formatted-rho) with App. A normalisation
 *
 * Precision: long double (x87, 64-bit mantissa) for the time base and all
 * phases, double for interpolation, the direct DFT and the pair sum.  Nothing
 * is blocked, fused or reordered beyond the definitions.
 *
 * Parity status per function is listed in the pin tests; every function here
 * is pinned by at least one closed form, special case or printed value.
 */
#include "ccr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const long double PI_L = 3.141592653589793238462643383279502884L;

int cco_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ plan */

/* Band plan.
 *  - load bandwidth, App. B eq. delta-f-load, T_sft read as T_short; drift width from
 *    eqs. f-drift-eq and delta-f-obs taken at the top of the band with v/c = 1e-4;
 *  - the series must be sampled at dt = T_short / N_K with N_K >= T_short * df_load;
 *  - T_coh = 2 T_max + T_short (eq. lag-time-constraint), T_max = R T_short;
 *  - delta lambda_f = sqrt(6 mu_f / pi) / T_coh (Sec. III.B.2);
 *  - N_FFT0 = (df_load / delta lambda_f) ceil(delta lambda_f T_coh), N_FFT the next power
 *    of two (eq. n-fft-final), never below the power of two holding N_K;
 *  - nu_R = delta lambda_f dt N_FFT; N_f = floor(f_band / delta lambda_f);
 *  - output bins sit on the FFT grid: kbar(i) = k_lo + floor(nu_R i) with
 *    k_lo = ceil(-(f_band / 2) T_FFT), frequency f_het + kbar / T_FFT.
 */
int cco_plan_band(const cco_problem *p, cco_plan *o) {
    const cco_band *b = &p->band;
    if (!(b->t_short > 0.0) || !(b->f_band > 0.0) || b->dirichlet_D < 1 || b->max_lag < 0 ||
        !(p->dt > 0.0) || !(b->mu_f > 0.0) || !(b->orbit_period > 0.0) || b->a_p_max < 0.0 ||
        p->n_det < 1 || p->n_det > CCO_MAX_DET || (b->pairs & 7) == 0 || ((b->pairs & 4) && (b->pairs & 3)) ||
        b->weight < 0 || b->weight > 1)
        return CCO_EINVAL;
    const double pi = 3.14159265358979323846;
    double f_top = b->f_min + b->f_band;
    double omega = 2.0 * pi / b->orbit_period;
    double drift = 2.0 * (f_top * 1e-4 + b->a_p_max * omega * f_top);
    double dfl = (1.0 + 4.0 / (2.0 * b->dirichlet_D + 1.0)) * (b->f_band + drift + 16.0 / b->t_short);
    double ratio = b->t_short / p->dt;
    int64_t nk = (int64_t)llround(ratio);
    if (nk < 1 || fabs(ratio - (double)nk) > 1e-9 * ratio) return CCO_EINVAL;
    if ((double)nk < b->t_short * dfl * (1.0 - 1e-12)) return CCO_ERANGE;
    double fh = b->f_min + 0.5 * b->f_band;
    if (fabs(p->f_het - fh) > 1e-9 * fabs(fh) + 1e-12) return CCO_EINVAL;
    int64_t n_seg = p->n / nk;
    if (n_seg < 1) return CCO_EINVAL;
    double t_coh = (2.0 * b->max_lag + 1.0) * b->t_short;
    double dlf = sqrt(6.0 * b->mu_f / pi) / t_coh;
    double nfft0 = (dfl / dlf) * ceil(dlf * t_coh);
    int64_t ns = 1;
    while (ns < nk) ns *= 2;
    int64_t nfft = 1;
    if (b->n_fft_override > 0) {
        nfft = b->n_fft_override;
        if (nfft % ns != 0) return CCO_EINVAL;
    } else {
        while ((double)nfft < nfft0) nfft *= 2;
        if (nfft < ns) nfft = ns;
    }
    double t_fft = p->dt * (double)nfft;
    double nu_r = dlf * t_fft;
    int64_t n_f = (int64_t)floor(b->f_band / dlf);
    if (n_f < 1) return CCO_ERANGE;
    int64_t k_lo = (int64_t)ceil(-0.5 * b->f_band * t_fft);
    o->n_k = nk;
    o->n_seg = n_seg;
    o->n_fft = nfft;
    o->n_f = n_f;
    o->k_lo = k_lo;
    o->dt = p->dt;
    o->f_het = fh;
    o->df_load = dfl;
    o->t_coh = t_coh;
    o->dlambda_f = dlf;
    o->t_fft = t_fft;
    o->nu_r = nu_r;
    return CCO_OK;
}

int64_t cco_bin_index(const cco_plan *pl, int64_t i) {
    return pl->k_lo + (int64_t)floor(pl->nu_r * (double)i);
}

static int validate(const cco_problem *p, cco_plan *pl) {
    int st = cco_plan_band(p, pl);
    if (st != CCO_OK) return st;
    for (int X = 0; X < p->n_det; ++X) {
        if (!p->x[X] || !p->a[X] || !p->b[X] || !p->noise_var[X]) return CCO_EINVAL;
        for (int64_t K = 0; K < pl->n_seg; ++K)
            if (!(p->noise_var[X][K] > 0.0)) return CCO_EINVAL;
    }
    return CCO_OK;
}

/* ------------------------------------------------------------- time base */

/* Detector position r(t) and velocity, light-seconds, equatorial frame:
 * circular Earth orbit in the ecliptic (tilted by the obliquity about x) plus
 * rotation of a site on a spherical Earth.  e(t) = r(t).n enters
 * t_SSB = t + r.n (eq. t-ssb-equation). */
static void earth_delay_l(const cco_problem *p, int det, long double t, long double *e, long double *ed) {
    const cco_sky *s = &p->sky;
    long double n[3] = {cosl(s->ra) * cosl(s->dec), sinl(s->ra) * cosl(s->dec), sinl(s->dec)};
    long double wo = 2.0L * PI_L / s->year_s;
    long double lam = s->orbit_phase0 + wo * t;
    long double ce = cosl(s->obliquity), se = sinl(s->obliquity);
    long double cl = cosl(lam), sl = sinl(lam);
    long double ro[3] = {s->au_s * cl, s->au_s * sl * ce, s->au_s * sl * se};
    long double vo[3] = {-s->au_s * wo * sl, s->au_s * wo * cl * ce, s->au_s * wo * cl * se};
    long double wd = 2.0L * PI_L / s->sidereal_day_s;
    long double g = s->gmst0 + wd * t + p->lon[det];
    long double cla = cosl(p->lat[det]), sla = sinl(p->lat[det]);
    long double rr[3] = {s->re_s * cla * cosl(g), s->re_s * cla * sinl(g), s->re_s * sla};
    long double vr[3] = {-s->re_s * wd * cla * sinl(g), s->re_s * wd * cla * cosl(g), 0.0L};
    *e = n[0] * (ro[0] + rr[0]) + n[1] * (ro[1] + rr[1]) + n[2] * (ro[2] + rr[2]);
    if (ed) *ed = n[0] * (vo[0] + vr[0]) + n[1] * (vo[1] + vr[1]) + n[2] * (vo[2] + vr[2]);
}

double cco_earth_delay(const cco_problem *p, int det, double t) {
    long double e;
    earth_delay_l(p, det, t, &e, NULL);
    return (double)e;
}

/* Binary orbit of a template.  Circular (Sec. II.A.2, the circular-case R/c):
 *   R/c = a_p sin(Omega (t_SSB - T_asc)),  template (a_p, T_asc, P);
 * eccentric (eqs. solve-for-E, Kepler-equation), the anomaly taken at t_SSB as the circular
 * case takes its phase (tau ~ t, Sec. II.A.2):
 *   Omega (t_SSB - T_p) = E - e sin E,
 *   R/c = a_p [sin(omega) (cos E - e) + cos(omega) sqrt(1 - e^2) sin E],  template
 *   (a_p, T_p, omega, e, P).  With e = 0 this is the circular orbit with T_asc = T_p - omega/Omega. */
typedef struct {
    int ecc;
    long double ap, tref, om, w, e;  /* tref: T_asc (circular) or T_p; om = 2 pi / P; w = omega */
} orbit;

static orbit orbit_of(const cco_problem *p, const double *t) {
    orbit o;
    o.ecc = p->ecc;
    o.ap = t[0];
    o.tref = t[1];
    if (p->ecc) {
        o.w = t[2];
        o.e = t[3];
        o.om = 2.0L * PI_L / t[4];
    } else {
        o.w = 0.0L;
        o.e = 0.0L;
        o.om = 2.0L * PI_L / t[2];
    }
    return o;
}

/* Kepler's equation E - e sin E = M by Newton's method in long double from E = M + e sin M,
 * iterated until the step is below 1e-19 rad and then once more (0 <= e < 1). */
static long double kepler_l(long double M, long double e) {
    long double E = M + e * sinl(M);
    int extra = 0;
    for (int it = 0; it < 100; ++it) {
        long double step = (E - e * sinl(E) - M) / (1.0L - e * cosl(E));
        E -= step;
        if (fabsl(step) < 1e-19L && ++extra >= 1) break;
    }
    return E;
}

double cco_kepler(double M, double e) { return (double)kepler_l(M, e); }

/* Binary Roemer delay R/c at SSB time ts and its derivative d(R/c)/d ts. */
static void binary_delay_l(const orbit *o, long double ts, long double *R, long double *Rd) {
    if (!o->ecc) {
        long double th = o->om * (ts - o->tref);
        *R = o->ap * sinl(th);
        if (Rd) *Rd = o->ap * o->om * cosl(th);
        return;
    }
    long double M = o->om * (ts - o->tref);
    M -= 2.0L * PI_L * floorl(M / (2.0L * PI_L));
    long double E = kepler_l(M, o->e);
    long double sE = sinl(E), cE = cosl(E), sw = sinl(o->w), cw = cosl(o->w);
    long double q = sqrtl(1.0L - o->e * o->e);
    *R = o->ap * (sw * (cE - o->e) + cw * q * sE);
    if (Rd) *Rd = o->ap * (-sw * sE + cw * q * cE) * o->om / (1.0L - o->e * cE);
}

/* Forward map tau(t) - t = r.n - R(t_SSB)/c, t_SSB = t + r.n (eqs. t-ssb-equation,
 * tau-equation). */
static long double forward_offset_l(const cco_problem *p, int det, const orbit *o, long double t) {
    long double e, R;
    earth_delay_l(p, det, t, &e, NULL);
    binary_delay_l(o, t + e, &R, NULL);
    return e - R;
}

double cco_forward_offset(const cco_problem *p, int det, const double *tmpl, double t) {
    const orbit o = orbit_of(p, tmpl);
    return (double)forward_offset_l(p, det, &o, t);
}

/* Inverse map (Sec. III.A.2, t(tau) as the functional inverse of tau(t)): the
 * delay Delta = t - tau of source time tau solves
 *   G(Delta) = Delta + e(tau + Delta) - R(tau + Delta + e(tau + Delta))/c = 0
 * by Newton iteration in long double, started from guess, iterated until the
 * step is below 1e-15 s and then twice more. */
static long double solve_delay(const cco_problem *p, int det, const orbit *o, long double tau, long double guess) {
    long double D = guess;
    int extra = 0;
    for (int it = 0; it < 100; ++it) {
        long double t = tau + D, e, ed, R, Rd;
        earth_delay_l(p, det, t, &e, &ed);
        binary_delay_l(o, t + e, &R, &Rd);
        long double G = D + e - R;
        long double Gp = 1.0L + ed - Rd * (1.0L + ed);
        long double step = G / Gp;
        D -= step;
        if (fabsl(step) < 1e-15L) {
            if (++extra >= 2) break;
        }
    }
    return D;
}

static long double crude_guess(const cco_problem *p, int det, const orbit *o, long double tau) {
    long double e, R;
    earth_delay_l(p, det, tau, &e, NULL);
    binary_delay_l(o, tau, &R, NULL);
    return -e + R;
}

int cco_delay(const cco_problem *p, int det, const double *tmpl, int64_t r, double *hi, double *lo) {
    if (det < 0 || det >= p->n_det) return CCO_EINVAL;
    const orbit o = orbit_of(p, tmpl);
    long double tau = (long double)p->t0 + (long double)r * (long double)p->dt;
    long double g = crude_guess(p, det, &o, tau);
    long double D = solve_delay(p, det, &o, tau, g);
    *hi = (double)D;
    *lo = (double)(D - (long double)*hi);
    return CCO_OK;
}

/* Gap mask (reading of Sec. III.B: gaps are zero-padded and get zero weight):
 * m_r = valid(j*_r) with j*_r taken on the Earth-only map (a_p = 0), so the mask
 * and the normalisation do not depend on the template. */
static void earth_only_mask_segment(const cco_problem *p, const cco_plan *pl, int det, int64_t K, uint8_t *m) {
    long double guess = 0.0L;
    orbit none;
    none.ecc = 0;
    none.ap = none.tref = none.w = none.e = 0.0L;
    none.om = 2.0L * PI_L;
    for (int64_t r = K * pl->n_k; r < (K + 1) * pl->n_k; ++r) {
        long double tau = (long double)p->t0 + (long double)r * (long double)p->dt;
        if (r == K * pl->n_k) guess = crude_guess(p, det, &none, tau);
        long double D = solve_delay(p, det, &none, tau, guess);
        guess = D;
        int64_t j = r + (int64_t)floorl(D / (long double)p->dt + 0.5L);
        uint8_t v = 0;
        if (j >= 0 && j < p->n) v = p->valid[det] ? (p->valid[det][j] ? 1 : 0) : 1;
        m[r] = v;
    }
}

static void earth_only_mask(const cco_problem *p, const cco_plan *pl, int det, uint8_t *m) {
    for (int64_t K = 0; K < pl->n_seg; ++K) earth_only_mask_segment(p, pl, det, K, m);
}

int cco_valid_fraction(const cco_problem *p, double *phi) {
    cco_plan pl;
    int st = cco_plan_band(p, &pl);
    if (st) return st;
    int64_t nr = pl.n_seg * pl.n_k;
    for (int X = 0; X < p->n_det; ++X) {
        uint8_t *m = (uint8_t *)malloc((size_t)nr);
        if (!m) return CCO_ENOMEM;
        earth_only_mask(p, &pl, X, m);
        for (int64_t K = 0; K < pl.n_seg; ++K) {
            int64_t c = 0;
            for (int64_t s = 0; s < pl.n_k; ++s) c += m[K * pl.n_k + s];
            phi[X * pl.n_seg + K] = (double)c / (double)pl.n_k;
        }
        free(m);
    }
    return CCO_OK;
}

/* --------------------------------------------------------- interpolation */

/* Window of the Shannon formula (Sec. III.A.1): Hamming of length 2D+1.
 * window 0: indexed by tap n = j - j* in [-D, D], w = 0.54 - 0.46 cos(2 pi (n + D) / (2D));
 * window 1: evaluated at the continuous offset d, w = 0.54 + 0.46 cos(pi d / (D + 1)). */
static long double window_w(int D, int win, int n, long double d) {
    if (win == 0) return 0.54L - 0.46L * cosl(2.0L * PI_L * (long double)(n + D) / (2.0L * D));
    return 0.54L + 0.46L * cosl(PI_L * d / (D + 1.0L));
}

/* sinc(d) = sin(pi d) / (pi d), sinc(0) = 1. */
static long double sinc_l(long double d) {
    if (d == 0.0L) return 1.0L;
    return sinl(PI_L * d) / (PI_L * d);
}

/* Resampled series of detector det for one template (eqs. delta-q-eq, q-prime-eq,
 * resampled-time-series-q-eq):
 *   tau_r = t0 + r dt on the source lattice (same spacing and origin as the input);
 *   Delta_r = t(tau_r) - tau_r;  j* = round-half-up((t_r - t0) / dt) = r + floor(Delta_r/dt + 1/2);
 *   delta_j = (t_r - t_j) / dt;  xhat = sum_{j=j*-D}^{j*+D} w sinc(delta_j) x'_j  (taps outside
 *   the data or in gaps read zero);
 *   y_r = m_r exp(+2 pi i f_h Delta_r) xhat  (heterodyne correction exp(-i 2 pi f_h Dt*),
 *   Dt* = tau - t(tau)). */
/* Resampled samples r of segment K (r in [K N_K, (K+1) N_K)), written to ys[2 s], ys[2 s + 1]
 * with s = r - K N_K (jstar and offset, if given, are indexed by r):
 * delay by the Newton solve (started from crude_guess at the segment's first sample, then
 * from the previous sample's delay), windowed sinc over the valid input samples, heterodyne
 * correction, gap mask. */
static void resample_segment(const cco_problem *p, const cco_plan *pl, int det, const double *tmpl,
                             const uint8_t *mask, int64_t K, double *ys, int64_t *jstar, double *offset) {
    int D = p->band.dirichlet_D, win = p->band.window;
    const orbit o = orbit_of(p, tmpl);
    const float *x = p->x[det];
    const uint8_t *val = p->valid[det];
    long double guess = 0.0L;
    for (int64_t r = K * pl->n_k; r < (K + 1) * pl->n_k; ++r) {
        long double tau = (long double)p->t0 + (long double)r * (long double)p->dt;
        if (r == K * pl->n_k) guess = crude_guess(p, det, &o, tau);
        long double Dl = solve_delay(p, det, &o, tau, guess);
        guess = Dl;
        long double q = Dl / (long double)p->dt;
        int64_t k = (int64_t)floorl(q + 0.5L);
        int64_t js = r + k;
        long double dc = q - (long double)k;
        double re = 0.0, im = 0.0;
        for (int n = -D; n <= D; ++n) {
            int64_t j = js + n;
            if (j < 0 || j >= p->n) continue;
            if (val && !val[j]) continue;
            long double d = dc - (long double)n;
            double w = (double)(window_w(D, win, n, d) * sinc_l(d));
            re += w * (double)x[2 * j];
            im += w * (double)x[2 * j + 1];
        }
        long double psi = (long double)p->f_het * Dl;
        psi -= floorl(psi);
        double c = (double)cosl(2.0L * PI_L * psi), s = (double)sinl(2.0L * PI_L * psi);
        double m = mask[r] ? 1.0 : 0.0;
        ys[2 * (r - K * pl->n_k)] = m * (c * re - s * im);
        ys[2 * (r - K * pl->n_k) + 1] = m * (s * re + c * im);
        if (jstar) jstar[r] = js;
        if (offset) offset[r] = (double)dc;
    }
}

static int resample_det(const cco_problem *p, const cco_plan *pl, int det, const double *tmpl,
                        const uint8_t *mask, double *y, int64_t *jstar, double *offset) {
    for (int64_t K = 0; K < pl->n_seg; ++K)
        resample_segment(p, pl, det, tmpl, mask, K, y + 2 * K * pl->n_k, jstar, offset);
    return CCO_OK;
}

int cco_resample(const cco_problem *p, int det, const double *tmpl, double *y,
                 int64_t *jstar, double *offset, uint8_t *mask_out) {
    cco_plan pl;
    int st = validate(p, &pl);
    if (st) return st;
    if (det < 0 || det >= p->n_det) return CCO_EINVAL;
    int64_t nr = pl.n_seg * pl.n_k;
    uint8_t *m = (uint8_t *)malloc((size_t)nr);
    if (!m) return CCO_ENOMEM;
    earth_only_mask(p, &pl, det, m);
    st = resample_det(p, &pl, det, tmpl, m, y, jstar, offset);
    if (mask_out) memcpy(mask_out, m, (size_t)nr);
    free(m);
    return st;
}

/* ---------------------------------------------------------------- spectra */

static double *twiddles(int64_t nfft) {
    double *tw = (double *)malloc(sizeof(double) * 2 * (size_t)nfft);
    if (!tw) return NULL;
    for (int64_t j = 0; j < nfft; ++j) {
        long double a = -2.0L * PI_L * (long double)j / (long double)nfft;
        tw[2 * j] = (double)cosl(a);
        tw[2 * j + 1] = (double)sinl(a);
    }
    return tw;
}

static int64_t bin_mod(const cco_plan *pl, int64_t i) {
    int64_t k = cco_bin_index(pl, i) % pl->n_fft;
    return k < 0 ? k + pl->n_fft : k;
}

/* Tier R spectra (Sec. III.B.4-5): zero-padded DFT of segment K starting at
 * r_B = K N_K, referenced to the series origin (Phi_in folded into the kernel):
 *   F_XK(i) = (sigma_XK sqrt(N_K))^-1 sum_{s<N_K} y_{r_B+s} exp(-2 pi i kbar_i (r_B + s) / N_FFT),
 * the phase index (kbar (r_B + s)) mod N_FFT kept as an exact integer. */
/* Direct DFT of segment K from its resampled samples ys[2 s], s < N_K, decimated bins, Phi_in
 * through the exact integer phase index (kbar (r_B + s) mod N_FFT), 1 / (sigma sqrt N_K). */
static void spectra_segment(const cco_problem *p, const cco_plan *pl, int det, int64_t K, const double *ys,
                            const double *tw, const int64_t *bins, int64_t nb, double *F) {
    int64_t nk = pl->n_k, nfft = pl->n_fft;
    double scale = 1.0 / (sqrt(p->noise_var[det][K]) * sqrt((double)nk));
    int64_t rb = K * nk;
    for (int64_t ii = 0; ii < nb; ++ii) {
        int64_t kb = bin_mod(pl, bins ? bins[ii] : ii);
        int64_t idx = (kb * rb) % nfft;
        double re = 0.0, im = 0.0;
        for (int64_t s = 0; s < nk; ++s) {
            const double *yy = ys + 2 * s;
            double c = tw[2 * idx], sn = tw[2 * idx + 1];
            re += yy[0] * c - yy[1] * sn;
            im += yy[0] * sn + yy[1] * c;
            idx += kb;
            if (idx >= nfft) idx -= nfft;
        }
        double *o = F + 2 * ((det * pl->n_seg + K) * nb + ii);
        o[0] = re * scale;
        o[1] = im * scale;
    }
}

static void spectra_from_series(const cco_problem *p, const cco_plan *pl, int det, const double *y,
                                const double *tw, const int64_t *bins, int64_t nb, double *F) {
    for (int64_t K = 0; K < pl->n_seg; ++K) spectra_segment(p, pl, det, K, y + 2 * K * pl->n_k, tw, bins, nb, F);
}

/* Tier D spectra (App. A, eq. from-here-resamp; Sec. III.B.6 frame invariance):
 * no interpolation; each raw detector sample j is demodulated with the exact
 * phase model and assigned to the segment holding its source time:
 *   F^D_XK(i) = (sigma sqrt(N_K))^-1 sum_{j: tau(t_j) in K} valid_j x'_j
 *               exp(-2 pi i [nu_i (tau(t_j) - t0) - f_h Delta_j]),  nu_i = kbar_i / T_FFT. */
static void spectra_direct(const cco_problem *p, const cco_plan *pl, int det, const double *tmpl,
                           const int64_t *bins, int64_t nb, double *F) {
    int64_t nk = pl->n_k, nfft = pl->n_fft;
    const orbit o = orbit_of(p, tmpl);
    memset(F + 2 * det * pl->n_seg * nb, 0, sizeof(double) * 2 * (size_t)(pl->n_seg * nb));
    for (int64_t j = 0; j < p->n; ++j) {
        if (p->valid[det] && !p->valid[det][j]) continue;
        long double t = (long double)p->t0 + (long double)j * (long double)p->dt;
        long double off = forward_offset_l(p, det, &o, t);                          /* tau - t */
        long double u = (long double)j + off / (long double)p->dt;                /* (tau - t0)/dt */
        int64_t K = (int64_t)floorl(u / (long double)nk);
        if (K < 0 || K >= pl->n_seg) continue;
        double scale = 1.0 / (sqrt(p->noise_var[det][K]) * sqrt((double)nk));
        double xr = p->x[det][2 * j], xi = p->x[det][2 * j + 1];
        for (int64_t ii = 0; ii < nb; ++ii) {
            int64_t kb = bin_mod(pl, bins ? bins[ii] : ii);
            int64_t kfull = cco_bin_index(pl, bins ? bins[ii] : ii);
            /* cycles = kbar j / N_FFT + kbar off / (N_FFT dt) + f_h off, with Delta_j = -off */
            long double cyc = (long double)((kb * (j % nfft)) % nfft) / (long double)nfft +
                              (long double)kfull * off / ((long double)nfft * (long double)p->dt) +
                              (long double)p->f_het * off;
            cyc -= floorl(cyc);
            double c = (double)cosl(2.0L * PI_L * cyc), s = -(double)sinl(2.0L * PI_L * cyc);
            double *o = F + 2 * ((det * pl->n_seg + K) * nb + ii);
            o[0] += scale * (xr * c - xi * s);
            o[1] += scale * (xr * s + xi * c);
        }
    }
}

int cco_spectra(const cco_problem *p, const double *tmpl, int tier, const int64_t *bins,
                int64_t n_bins, double *F) {
    cco_plan pl;
    int st = validate(p, &pl);
    if (st) return st;
    int64_t nb = bins ? n_bins : pl.n_f;
    for (int64_t ii = 0; ii < nb; ++ii)
        if (bins && (bins[ii] < 0 || bins[ii] >= pl.n_f)) return CCO_EINVAL;
    int64_t nr = pl.n_seg * pl.n_k;
    double *tw = twiddles(pl.n_fft);
    double *y = (double *)malloc(sizeof(double) * 2 * (size_t)nr);
    uint8_t *m = (uint8_t *)malloc((size_t)nr);
    if (!tw || !y || !m) {
        free(tw); free(y); free(m);
        return CCO_ENOMEM;
    }
    for (int X = 0; X < p->n_det; ++X) {
        if (tier == 0) {
            earth_only_mask(p, &pl, X, m);
            resample_det(p, &pl, X, tmpl, m, y, NULL, NULL);
            spectra_from_series(p, &pl, X, y, tw, bins, nb, F);
        } else {
            spectra_direct(p, &pl, X, tmpl, bins, nb, F);
        }
    }
    free(tw); free(y); free(m);
    return CCO_OK;
}

/* ------------------------------------------------------------------ pairs */

/* Pair set P (Sec. III.B.1): cross-detector pairs X < Y with |K - L| <= R, and
 * same-detector pairs with K < L <= K + R (no auto-correlation); each unordered
 * pair once.  CCO_PAIRS_ALL: every ordered pair (X K, Y L), auto-correlations included and
 * any lag (App. A.1: all pairs P, the sum expanding into |F_a|^2 + |F_b|^2). */
static int pair_in_set(int pairs, int R, int X, int64_t K, int Y, int64_t L) {
    if (pairs & CCO_PAIRS_ALL) return 1;
    if ((pairs & CCO_PAIRS_CROSS) && X < Y && llabs(K - L) <= R) return 1;
    if ((pairs & CCO_PAIRS_SAME) && X == Y && L > K && L <= K + R) return 1;
    return 0;
}

/* Range of partner segments L of segment K that the pair loops visit. */
static int64_t lag_lo(const cco_problem *p, int64_t K) {
    return (p->band.pairs & CCO_PAIRS_ALL) ? 0 : K - p->band.max_lag;
}
static int64_t lag_hi(const cco_problem *p, const cco_plan *pl, int64_t K) {
    return (p->band.pairs & CCO_PAIRS_ALL) ? pl->n_seg - 1 : K + p->band.max_lag;
}

int64_t cco_pair_count(const cco_problem *p) {
    cco_plan pl;
    if (cco_plan_band(p, &pl)) return -1;
    int R = p->band.max_lag;
    int64_t c = 0;
    for (int X = 0; X < p->n_det; ++X)
        for (int64_t K = 0; K < pl.n_seg; ++K)
            for (int Y = 0; Y < p->n_det; ++Y)
                for (int64_t L = lag_lo(p, K); L <= lag_hi(p, &pl, K); ++L)
                    if (L >= 0 && L < pl.n_seg && pair_in_set(p->band.pairs, R, X, K, Y, L)) ++c;
    return c;
}

/* Normalisation (Sec. III.B.6 and App. A): N^2 = sum_P A_XK A_YL + 2 C_XK C_YL + B_XK B_YL
 * with hat a = a / sigma, A = hat a^2 phi, B = hat b^2 phi, C = hat a hat b phi, where phi is
 * the valid fraction of the segment (gaps carry zero weight).  This gives Var rho = 1 for
 * unit-variance segment spectra. */
static double norm_from_phi(const cco_problem *p, const cco_plan *pl, const double *phi) {
    int R = p->band.max_lag;
    long double acc = 0.0L;
    for (int X = 0; X < p->n_det; ++X)
        for (int64_t K = 0; K < pl->n_seg; ++K)
            for (int Y = 0; Y < p->n_det; ++Y)
                for (int64_t L = lag_lo(p, K); L <= lag_hi(p, pl, K); ++L) {
                    if (L < 0 || L >= pl->n_seg || !pair_in_set(p->band.pairs, R, X, K, Y, L)) continue;
                    double sK = sqrt(p->noise_var[X][K]), sL = sqrt(p->noise_var[Y][L]);
                    double aK = p->a[X][K] / sK, bK = p->b[X][K] / sK;
                    double aL = p->a[Y][L] / sL, bL = p->b[Y][L] / sL;
                    double fK = phi[X * pl->n_seg + K], fL = phi[Y * pl->n_seg + L];
                    double AK = aK * aK * fK, BK = bK * bK * fK, CK = aK * bK * fK;
                    double AL = aL * aL * fL, BL = bL * bL * fL, CL = aL * bL * fL;
                    acc += (long double)AK * AL + 2.0L * CK * CL + (long double)BK * BL;
                }
    return (double)sqrtl(acc);
}

/* ------------------------------------------------- weighted spectra streams */

/* Per-sample antenna weighting (Sec. III.B.3, eq. norm-a-eq): the resampled series is
 * multiplied by hat a_r = a(tau_r) / sigma_XK and by hat b_r before the DFT, giving two
 * spectra per segment,
 *   F^a_XK(i) = (sigma_XK sqrt(N_K))^-1 sum_s hat a_{r_B+s} y_{r_B+s} exp(-2 pi i kbar (r_B+s)/N_FFT),
 * and F^b likewise.  With per-segment weights the streams are F^a = hat a_K F, F^b = hat b_K F.
 * The pair sum and its normalisation then take one form for both (App. A.1,
 * eq. well-formatted-rho, and its Gamma^circ counterpart):
 *   Gamma^ave:  rho = sqrt2 Re sum_P [conj(F^a_K) F^a_L + conj(F^b_K) F^b_L] / N,
 *               N^2 = sum_P A_K A_L + 2 C_K C_L + B_K B_L;
 *   Gamma^circ: rho = sqrt2 sum_P Im[conj(F^b_K) F^a_L - conj(F^a_K) F^b_L] / N,
 *               N^2 = sum_P A_K B_L + B_K A_L - 2 C_K C_L,
 * with A_K = E|F^a_K|^2 = mean over the segment of m_r hat a_r^2, B_K, C_K = mean of
 * m_r hat a_r hat b_r likewise (per-segment: hat a^2 phi, ...), so that Var rho = 1 in Gaussian
 * noise.  The Gamma^circ term pairs (hat b_K hat a_L - hat a_K hat b_L) with the imaginary part
 * of conj(F_K) F_L, whose mean for a circularly polarised signal (cos iota = 1) is
 * proportional to that weight: the sign makes its expectation positive for cos iota > 0 with the
 * signal convention x' = (F+ A+ - i Fx Ax) exp(i Phi) / 2. */
static int per_sample(const cco_problem *p) {
    for (int X = 0; X < p->n_det; ++X)
        if (!p->ar[X] || !p->br[X]) return 0;
    return 1;
}

/* A_XK, B_XK, C_XK (3 * n_det * n_seg doubles) from the gap masks. */
static void stream_moments(const cco_problem *p, const cco_plan *pl, const uint8_t *masks, double *abc) {
    int64_t nr = pl->n_seg * pl->n_k;
    for (int X = 0; X < p->n_det; ++X)
        for (int64_t K = 0; K < pl->n_seg; ++K) {
            double sig = sqrt(p->noise_var[X][K]);
            double A = 0.0, B = 0.0, C = 0.0;
            for (int64_t s = 0; s < pl->n_k; ++s) {
                int64_t r = K * pl->n_k + s;
                if (!masks[X * nr + r]) continue;
                double ar = per_sample(p) ? p->ar[X][r] / sig : p->a[X][K] / sig;
                double br = per_sample(p) ? p->br[X][r] / sig : p->b[X][K] / sig;
                A += ar * ar;
                B += br * br;
                C += ar * br;
            }
            double *o = abc + 3 * (X * pl->n_seg + K);
            o[0] = A / (double)pl->n_k;
            o[1] = B / (double)pl->n_k;
            o[2] = C / (double)pl->n_k;
        }
}

static double stream_norm(const cco_problem *p, const cco_plan *pl, const double *abc) {
    int R = p->band.max_lag;
    long double acc = 0.0L;
    for (int X = 0; X < p->n_det; ++X)
        for (int64_t K = 0; K < pl->n_seg; ++K)
            for (int Y = 0; Y < p->n_det; ++Y)
                for (int64_t L = lag_lo(p, K); L <= lag_hi(p, pl, K); ++L) {
                    if (L < 0 || L >= pl->n_seg || !pair_in_set(p->band.pairs, R, X, K, Y, L)) continue;
                    const double *k = abc + 3 * (X * pl->n_seg + K), *l = abc + 3 * (Y * pl->n_seg + L);
                    if (p->band.weight == 0)
                        acc += (long double)k[0] * l[0] + 2.0L * k[2] * l[2] + (long double)k[1] * l[1];
                    else
                        acc += (long double)k[0] * l[1] + (long double)k[1] * l[0] - 2.0L * k[2] * l[2];
                }
    return (double)sqrtl(acc);
}

/* Streams of segment K from its resampled samples: Fa, Fb (2 * nb doubles each). */
static void streams_segment(const cco_problem *p, const cco_plan *pl, int det, int64_t K, const double *ys,
                            const double *tw, const int64_t *bins, int64_t nb, double *Fa, double *Fb) {
    int64_t nk = pl->n_k, nfft = pl->n_fft, rb = K * nk;
    double sig = sqrt(p->noise_var[det][K]);
    double scale = 1.0 / (sig * sqrt((double)nk));
    int ps = per_sample(p);
    for (int64_t ii = 0; ii < nb; ++ii) {
        int64_t kb = bin_mod(pl, bins ? bins[ii] : ii);
        int64_t idx = (kb * rb) % nfft;
        double ra = 0.0, ia = 0.0, rbb = 0.0, ib = 0.0;
        for (int64_t s = 0; s < nk; ++s) {
            const double *yy = ys + 2 * s;
            double wa = ps ? p->ar[det][rb + s] / sig : p->a[det][K] / sig;
            double wb = ps ? p->br[det][rb + s] / sig : p->b[det][K] / sig;
            double c = tw[2 * idx], sn = tw[2 * idx + 1];
            double tr = yy[0] * c - yy[1] * sn, ti = yy[0] * sn + yy[1] * c;
            ra += wa * tr;
            ia += wa * ti;
            rbb += wb * tr;
            ib += wb * ti;
            idx += kb;
            if (idx >= nfft) idx -= nfft;
        }
        double *oa = Fa + 2 * ((det * pl->n_seg + K) * nb + ii), *ob = Fb + 2 * ((det * pl->n_seg + K) * nb + ii);
        oa[0] = ra * scale;
        oa[1] = ia * scale;
        ob[0] = rbb * scale;
        ob[1] = ib * scale;
    }
}

static void rho_from_streams(const cco_problem *p, const cco_plan *pl, const double *Fa, const double *Fb,
                             int64_t nb, double N, double *rho) {
    int R = p->band.max_lag;
    for (int64_t ii = 0; ii < nb; ++ii) {
        double acc = 0.0;
        for (int X = 0; X < p->n_det; ++X)
            for (int64_t K = 0; K < pl->n_seg; ++K)
                for (int Y = 0; Y < p->n_det; ++Y)
                    for (int64_t L = lag_lo(p, K); L <= lag_hi(p, pl, K); ++L) {
                        if (L < 0 || L >= pl->n_seg || !pair_in_set(p->band.pairs, R, X, K, Y, L)) continue;
                        const double *ak = Fa + 2 * ((X * pl->n_seg + K) * nb + ii);
                        const double *bk = Fb + 2 * ((X * pl->n_seg + K) * nb + ii);
                        const double *al = Fa + 2 * ((Y * pl->n_seg + L) * nb + ii);
                        const double *bl = Fb + 2 * ((Y * pl->n_seg + L) * nb + ii);
                        if (p->band.weight == 0)  /* Re conj(a_K) a_L + Re conj(b_K) b_L */
                            acc += ak[0] * al[0] + ak[1] * al[1] + bk[0] * bl[0] + bk[1] * bl[1];
                        else                      /* Im conj(b_K) a_L - Im conj(a_K) b_L */
                            acc += (bk[0] * al[1] - bk[1] * al[0]) - (ak[0] * bl[1] - ak[1] * bl[0]);
                    }
        rho[ii] = (N > 0.0) ? sqrt(2.0) * acc / N : 0.0;
    }
}

static double stream_norm_of(const cco_problem *p, const cco_plan *pl) {
    int64_t nr = pl->n_seg * pl->n_k;
    uint8_t *masks = (uint8_t *)malloc((size_t)(p->n_det * nr));
    double *abc = (double *)malloc(sizeof(double) * 3 * (size_t)(p->n_det * pl->n_seg));
    if (!masks || !abc) {
        free(masks); free(abc);
        return -1.0;
    }
    for (int X = 0; X < p->n_det; ++X) earth_only_mask(p, pl, X, masks + X * nr);
    stream_moments(p, pl, masks, abc);
    double N = stream_norm(p, pl, abc);
    free(masks); free(abc);
    return N;
}

double cco_norm(const cco_problem *p) {
    cco_plan pl;
    if (validate(p, &pl)) return -1.0;
    if (per_sample(p) || p->band.weight != 0) return stream_norm_of(p, &pl);
    double *phi = (double *)malloc(sizeof(double) * (size_t)(p->n_det * pl.n_seg));
    if (!phi) return -1.0;
    cco_valid_fraction(p, phi);
    double N = norm_from_phi(p, &pl, phi);
    free(phi);
    return N;
}

/* rho_i = sqrt(2) Re sum_P (hat a_XK hat a_YL + hat b_XK hat b_YL) conj(F_XK(i)) F_YL(i) / N
 * (eq. final-formatted-rho with the geometric weight of eq. geometric-filter; the 1/10 and
 * the 2/S factors cancel against the normalisation).  rho = 0 when N = 0. */
static void rho_from_spectra(const cco_problem *p, const cco_plan *pl, const double *F, int64_t nb,
                             double N, double *rho) {
    int R = p->band.max_lag;
    for (int64_t ii = 0; ii < nb; ++ii) {
        double acc = 0.0;
        for (int X = 0; X < p->n_det; ++X)
            for (int64_t K = 0; K < pl->n_seg; ++K)
                for (int Y = 0; Y < p->n_det; ++Y)
                    for (int64_t L = lag_lo(p, K); L <= lag_hi(p, pl, K); ++L) {
                        if (L < 0 || L >= pl->n_seg || !pair_in_set(p->band.pairs, R, X, K, Y, L)) continue;
                        double sK = sqrt(p->noise_var[X][K]), sL = sqrt(p->noise_var[Y][L]);
                        double W = (p->a[X][K] / sK) * (p->a[Y][L] / sL) + (p->b[X][K] / sK) * (p->b[Y][L] / sL);
                        const double *fk = F + 2 * ((X * pl->n_seg + K) * nb + ii);
                        const double *fl = F + 2 * ((Y * pl->n_seg + L) * nb + ii);
                        acc += W * (fk[0] * fl[0] + fk[1] * fl[1]);
                    }
        rho[ii] = (N > 0.0) ? sqrt(2.0) * acc / N : 0.0;
    }
}

/* rho through the weighted streams (per-sample antenna functions or the Gamma^circ weight),
 * tier R only. */
static int rho_streams(const cco_problem *p, const cco_plan *pl, const double *tmpl, int64_t n_tmpl,
                       const int64_t *bins, int64_t nb, double *rho) {
    int64_t nr = pl->n_seg * pl->n_k;
    int Q = p->n_det;
    int stride = p->ecc ? 5 : 3;
    uint8_t *masks = (uint8_t *)malloc((size_t)(Q * nr));
    double *abc = (double *)malloc(sizeof(double) * 3 * (size_t)(Q * pl->n_seg));
    double *tw = twiddles(pl->n_fft);
    size_t fsz = (size_t)(Q * pl->n_seg * nb) * 2;
    double *Fa = (double *)malloc(sizeof(double) * fsz), *Fb = (double *)malloc(sizeof(double) * fsz);
    int nth = cco_num_threads();
    double *y = (double *)malloc(sizeof(double) * 2 * (size_t)pl->n_k * (size_t)nth);
    if (!masks || !abc || !tw || !Fa || !Fb || !y) {
        free(masks); free(abc); free(tw); free(Fa); free(Fb); free(y);
        return CCO_ENOMEM;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t w = 0; w < Q * pl->n_seg; ++w)
        earth_only_mask_segment(p, pl, (int)(w / pl->n_seg), w % pl->n_seg, masks + (w / pl->n_seg) * nr);
    stream_moments(p, pl, masks, abc);
    double N = stream_norm(p, pl, abc);
    for (int64_t t = 0; t < n_tmpl; ++t) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t w = 0; w < Q * pl->n_seg; ++w) {
            int X = (int)(w / pl->n_seg);
            int64_t K = w % pl->n_seg;
#ifdef _OPENMP
            double *yt = y + 2 * (size_t)pl->n_k * (size_t)omp_get_thread_num();
#else
            double *yt = y;
#endif
            resample_segment(p, pl, X, tmpl + stride * t, masks + X * nr, K, yt, NULL, NULL);
            streams_segment(p, pl, X, K, yt, tw, bins, nb, Fa, Fb);
        }
        rho_from_streams(p, pl, Fa, Fb, nb, N, rho + t * nb);
    }
    free(masks); free(abc); free(tw); free(Fa); free(Fb); free(y);
    return CCO_OK;
}

int cco_rho(const cco_problem *p, const double *tmpl, int64_t n_tmpl, int tier,
            const int64_t *bins, int64_t n_bins, double *rho) {
    cco_plan pl;
    int st = validate(p, &pl);
    if (st) return st;
    int64_t nb = bins ? n_bins : pl.n_f;
    for (int64_t ii = 0; ii < nb; ++ii)
        if (bins && (bins[ii] < 0 || bins[ii] >= pl.n_f)) return CCO_EINVAL;
    if (per_sample(p) || p->band.weight != 0) {
        if (tier != 0) return CCO_EINVAL;
        return rho_streams(p, &pl, tmpl, n_tmpl, bins, nb, rho);
    }
    int64_t nr = pl.n_seg * pl.n_k;
    int Q = p->n_det;
    const int stride = p->ecc ? 5 : 3;
    uint8_t *masks = (uint8_t *)malloc((size_t)(Q * nr));
    double *phi = (double *)malloc(sizeof(double) * (size_t)(Q * pl.n_seg));
    double *tw = twiddles(pl.n_fft);
    if (!masks || !phi || !tw) {
        free(masks); free(phi); free(tw);
        return CCO_ENOMEM;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t w = 0; w < Q * pl.n_seg; ++w)
        earth_only_mask_segment(p, &pl, (int)(w / pl.n_seg), w % pl.n_seg, masks + (w / pl.n_seg) * nr);
    for (int X = 0; X < Q; ++X)
        for (int64_t K = 0; K < pl.n_seg; ++K) {
            int64_t c = 0;
            for (int64_t s = 0; s < pl.n_k; ++s) c += masks[X * nr + K * pl.n_k + s];
            phi[X * pl.n_seg + K] = (double)c / (double)pl.n_k;
        }
    double N = norm_from_phi(p, &pl, phi);
    int fail = 0;
    /* templates in groups; within a group every (template, detector, segment) is an independent
     * work item (tier R) or every (template, detector) (tier D); the pair sum per template */
    int64_t G = cco_num_threads();
    if (G < 1) G = 1;
    size_t fsz = (size_t)(Q * pl.n_seg * nb) * 2;
    double *F = (double *)malloc(sizeof(double) * fsz * (size_t)G);
    int nth = cco_num_threads();
    double *y = (tier == 0) ? (double *)malloc(sizeof(double) * 2 * (size_t)pl.n_k * (size_t)nth) : NULL;
    if (!F || (tier == 0 && !y)) {
        free(F); free(y); free(masks); free(phi); free(tw);
        return CCO_ENOMEM;
    }
    for (int64_t g = 0; g < n_tmpl; g += G) {
        int64_t gn = (n_tmpl - g < G) ? n_tmpl - g : G;
        if (tier == 0) {
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t w = 0; w < gn * Q * pl.n_seg; ++w) {
                int64_t tl = w / (Q * pl.n_seg);
                int X = (int)((w / pl.n_seg) % Q);
                int64_t K = w % pl.n_seg;
#ifdef _OPENMP
                double *yt = y + 2 * (size_t)pl.n_k * (size_t)omp_get_thread_num();
#else
                double *yt = y;
#endif
                resample_segment(p, &pl, X, tmpl + stride * (g + tl), masks + X * nr, K, yt, NULL, NULL);
                spectra_segment(p, &pl, X, K, yt, tw, bins, nb, F + fsz * (size_t)tl);
            }
        } else {
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t w = 0; w < gn * Q; ++w)
                spectra_direct(p, &pl, (int)(w % Q), tmpl + stride * (g + w / Q), bins, nb, F + fsz * (size_t)(w / Q));
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t tl = 0; tl < gn; ++tl) rho_from_spectra(p, &pl, F + fsz * (size_t)tl, nb, N, rho + (g + tl) * nb);
    }
    free(F);
    free(y);
    free(masks); free(phi); free(tw);
    return fail ? CCO_ENOMEM : CCO_OK;
}

/* ------------------------------------------------- SFT front end */

/* Heterodyned, downsampled series from short Fourier transforms (App. B, Downsampling and
 * heterodyning).  SFT K holds bins z_{K,k}, k = k_first .. k_first + n_bins - 1 (frequency
 * k / T_sft), of the data starting at t0 + K T_sft; its inverse transform is
 * x_K(t0 + K T_sft + j dt) = sum_k z_{K,k} exp(2 pi i j k dt / T_sft) / T_sft (eq. inverse-fft-eq).
 * Steps in the appendix's order:
 *   - heterodyne bin k_h, the nearest bin to f_h, with bar f_h = k_h / T_sft and remainder
 *     f_r = f_h - bar f_h;
 *   - the band of N' = n_out bins k_h - h .. k_h - h + N' - 1 (h = floor(N'/2); the appendix's
 *     k_a .. k_b with k_b - k_a = N'), re-indexed m = l + h with l = k - k_h;
 *   - per SFT, x_{K,s}(j') = e^{-2 pi i j' h / N'} sum_m e^{2 pi i j' m / N'} z_{K,(m + k_h - h)} / T_sft
 *     at the downsampled samples j' = 0 .. N' - 1 (dt' = T_sft / N'); the leading factor is the
 *     appendix's (-1)^{-j'} for even N', written for any N';
 *   - the phase that stitches the SFTs: x^h(t) = e^{-2 pi i f_h (t_K - T_sft/2)} x_{K,s}(j') with
 *     t_K - T_sft/2 = t0 + K T_sft (eq. long-time-series-het-corrected);
 *   - and, where the appendix sets bar f_h ~ f_h (eq. heterodyne-shift-approx), the remainder
 *     kept exactly: a factor e^{-2 pi i f_r j' dt'}, so that the series is heterodyned by f_h
 *     itself (the resampler's correction e^{2 pi i f_h Delta} assumes that).
 * Missing SFTs (sft_valid[K] == 0) give zeros.  x: 2 * n_sft * n_out doubles (interleaved). */
int cco_sft_series(int64_t n_sft, double t_sft, double t0, int64_t n_bins, int64_t k_first, const double *z,
                   const uint8_t *sft_valid, double f_het, int64_t n_out, double *x) {
    if (n_sft < 1 || n_bins < 1 || n_out < 1 || !(t_sft > 0) || !z || !x) return CCO_EINVAL;
    long double ts = t_sft, fh = f_het;
    int64_t kh = (int64_t)llroundl(fh * ts);
    long double fr = fh - (long double)kh / ts;
    int64_t h = n_out / 2;
    if (kh - h < k_first || kh - h + n_out > k_first + n_bins) return CCO_ERANGE;
    long double dtp = ts / (long double)n_out;
#pragma omp parallel for schedule(static)
    for (int64_t K = 0; K < n_sft; ++K) {
        double *xo = x + 2 * K * n_out;
        if (sft_valid && !sft_valid[K]) {
            for (int64_t j = 0; j < 2 * n_out; ++j) xo[j] = 0.0;
            continue;
        }
        /* stitching phase of this SFT, cycles */
        long double tk = (long double)t0 + (long double)K * ts;
        long double ph = fh * tk;
        ph -= floorl(ph);
        long double cs = cosl(-2.0L * PI_L * ph), sn = sinl(-2.0L * PI_L * ph);
        const double *zk = z + 2 * (K * n_bins + (kh - h - k_first));
        for (int64_t j = 0; j < n_out; ++j) {
            long double re = 0.0L, im = 0.0L;
            for (int64_t m = 0; m < n_out; ++m) {
                long double a = 2.0L * PI_L * (long double)((j * m) % n_out) / (long double)n_out;
                long double c = cosl(a), s = sinl(a);
                re += (long double)zk[2 * m] * c - (long double)zk[2 * m + 1] * s;
                im += (long double)zk[2 * m] * s + (long double)zk[2 * m + 1] * c;
            }
            /* x_{K,s}: shift factor and 1 / T_sft */
            long double as = -2.0L * PI_L * (long double)((j * h) % n_out) / (long double)n_out;
            long double xr = (re * cosl(as) - im * sinl(as)) / ts;
            long double xi = (re * sinl(as) + im * cosl(as)) / ts;
            /* remainder f_r and stitching phase */
            long double ar = -2.0L * PI_L * fr * (long double)j * dtp;
            long double c2 = cosl(ar) * cs - sinl(ar) * sn, s2 = cosl(ar) * sn + sinl(ar) * cs;
            xo[2 * j] = (double)(xr * c2 - xi * s2);
            xo[2 * j + 1] = (double)(xr * s2 + xi * c2);
        }
    }
    return CCO_OK;
}

// Host side of the C ABI (include/ccr.h): argument validation, the band planner,
// template-independent set-up tables (Earth anchors, gap masks, weights, normalisation,
// work lists), device memory and kernel sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "ccr.h"
#include "ccr_internal.h"

using namespace ccr;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kRawStride = 5;
constexpr long double kPiL = 3.141592653589793238462643383279502884L;

// ------------------------------------------------------------------ device buffers

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        release();
        if (n == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = n;
        return hipSuccess;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct DetData {
    bool has_data = false, has_weights = false;
    ccr_site site{};
    double t0 = 0, dt = 0, f_het = 0;
    int64_t n = 0;
    std::vector<float> x;        // interleaved, zero where invalid
    std::vector<uint8_t> valid;  // empty = all valid
    std::vector<double> a, b, nv;
    std::vector<double> ar, br;  // per-sample antenna functions on the source lattice, or empty
};

struct Plan {
    int64_t n_k = 0, n_seg = 0, n_fft = 0, n_f = 0, k_lo = 0, n_s = 0, P = 0, n_pairs = 0;
    double dt = 0, f_het = 0, df_load = 0, t_coh = 0, dlf = 0, t_fft = 0, nu_r = 0, norm = 0;
};

struct Band {
    ccr_band p{};
    double df_load = 0;
    int64_t n_k_min = 0;
    DetData det[CCR_MAX_DET];
    std::vector<double> tmpl;  // kTmplStride per template
    std::vector<double> tmpl_raw;  // kRawStride per template: a_p, T_asc or T_p, P, e, omega
    bool ecc = false;               // eccentric templates (set by ccr_set_templates_ecc)
    int64_t n_tmpl = 0;
    bool prepared = false;
    Plan plan;
    int Q = 0;
    // device tables
    DevBuf d_x, d_mask, d_anchor, d_earth, d_win64, d_win32, d_cheb_x, d_mono, d_tw64, d_tw32, d_bin_m, d_bin_p,
        d_bin_kb, d_bin_pos, d_segw, d_segwf, d_active, d_work, d_seg_work, d_tmpl, d_lagph, d_seg_any, d_col_bin, d_bin_col, d_zero256,
        d_class_start, d_farrow, d_farrow_A, d_cls_m0, d_pw, d_pwf;
    bool per_sample = false;  // every detector has per-sample antenna functions (two spectra streams)
    int wide_jmax = 0, wide_ncol = 0;  // 1024-point spectra + pair-sum kernel (see BandDev)
    int64_t far_len = 0;  // plane length of the Farrow table, 0 when the band has none
    double far_err = 0;   // bound of the fitted tap weights' error, sum over taps
    int bins_unique = 0;
    int n_work = 0;
    int newton_steps = 3, cheb_split = kCheb;
    bool short_series = false;  // node solve with the x^7 / x^8 small-angle series
    int n_seg_any = 0;
    std::vector<double> freqs;
    std::vector<uint8_t> active;
};

}  // namespace

struct ccr_ctx {
    int device = 0;
    ccr_sky sky{};
    std::vector<std::unique_ptr<Band>> bands;
    std::string err;
    hipStream_t stream = nullptr;
    int64_t opt_template_batch = 0;
    int64_t opt_workspace_mb = 0;   // 0: automatic (see auto_budget)
    size_t auto_budget = 0;         // automatic workspace budget, fixed at the first compute call
    int64_t opt_k_chunk = 0;
    int64_t opt_spectra_kernel = 0;  // 1: the 256- to 1024-point spectra + pair-sum kernel wherever it applies
    int64_t opt_round_templates = 0;  // at most this many templates in one launch round (0: no limit)
    int64_t opt_fused = 0;
    int64_t opt_timing = 0;
    DevBuf ws_arena;                // workspace of the batched path: one arena, laid out per launch round
    DevBuf ws_part, ws_out, ws_coef;  // fused path: chunk partials, time-base coefficients; host outputs
    int64_t opt_graph = 0, opt_autotune = 0, opt_items_per_launch = 0;
    int64_t opt_farrow = 1;  // split-precision resampling in Farrow form where a band has the table
    int64_t opt_farrow_stage = 1;  // Farrow kernel: stage the table in LDS (0: global reads, for tests)
    // bumped whenever device memory a captured launch sequence refers to may have moved
    uint64_t gen = 1;
    // device copies of the band and work-item tables of the last eager call, their pinned
    // staging buffer and the event after which the staging buffer may be rewritten
    DevBuf d_tables;
    void *h_tables = nullptr;
    size_t h_tables_bytes = 0;
    hipEvent_t tables_copied = nullptr;
    struct GraphEntry;
    std::vector<std::unique_ptr<GraphEntry>> graphs;
    struct Tuned {
        std::vector<int> band_ids;
        int prec;
        int64_t k_chunk, template_batch, round_templates;
        int spectra;
    };
    std::vector<Tuned> tuned;
    int64_t last_tuned_k_chunk = 0, last_tuned_template_batch = 0, last_tuned_spectra = -1, last_tuned_round_templates = 0;
    struct Timed {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
    double kt_ms[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int64_t kt_n[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // no-allocation entry point: host staging of its band and work-item tables (fixed size,
    // allocated with the context) and the event after which the staging may be rewritten
    std::vector<char> na_host;
    hipEvent_t na_copied = nullptr;
};

// A compute call captured as a HIP graph: replayed while the call's arguments and the
// context's device memory are unchanged (`gen`).
struct ccr_ctx::GraphEntry {
    std::vector<int> band_ids;
    std::vector<void *> outs;
    int prec = 0, out_fp64 = 0;
    uint64_t gen = 0;
    void *tables = nullptr;  // device copy of the band and work-item tables
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphEntry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (tables) (void)hipFree(tables);
    }
};

namespace {

ccr_status fail(ccr_ctx *c, ccr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIP_OK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, e_ == hipErrorOutOfMemory ? CCR_ENOMEM : CCR_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                       \
    } while (0)

bool finite_all(const double *v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

template <typename F> void parallel_for(int64_t n, F &&f) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 16));
    if (n < 4 * nt) nt = 1;
    if (nt == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int64_t i = t; i < n; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

// ------------------------------------------------------------------ planner

// Load bandwidth of App. B (eq. delta-f-load) with T_sft read as T_short, the Doppler wings of
// eqs. f-drift-eq and delta-f-obs at the top of the band, v/c = 1e-4.
double load_bandwidth(const ccr_band &b) {
    double f_top = b.f_min + b.f_band;
    double omega = 2.0 * kPi / b.orbit_period;
    double drift = 2.0 * (f_top * 1e-4 + b.a_p_max * omega * f_top);
    return (1.0 + 4.0 / (2.0 * b.dirichlet_D + 1.0)) * (b.f_band + drift + 16.0 / b.t_short);
}

// Plan of Sec. III.B.2: T_coh = (2R+1) T_short, delta lambda_f = sqrt(6 mu_f / pi) / T_coh,
// N_FFT0 = (df_load / dlf) ceil(dlf T_coh), N_FFT the next power of two (at least the power of
// two n_s holding N_K), nu_R = dlf T_FFT, N_f = floor(f_band / dlf), output bins on the FFT grid
// kbar_i = k_lo + floor(nu_R i), k_lo = ceil(-f_band T_FFT / 2).
ccr_status make_plan(ccr_ctx *c, const Band &B, Plan &pl) {
    const ccr_band &b = B.p;
    pl.n_k = B.det[0].dt > 0 ? llround(b.t_short / B.det[0].dt) : 0;
    pl.dt = B.det[0].dt;
    pl.n_seg = B.det[0].n / pl.n_k;
    pl.f_het = b.f_min + 0.5 * b.f_band;
    pl.df_load = B.df_load;
    pl.t_coh = (2.0 * b.max_lag + 1.0) * b.t_short;
    pl.dlf = std::sqrt(6.0 * b.mu_f / kPi) / pl.t_coh;
    double nfft0 = (pl.df_load / pl.dlf) * std::ceil(pl.dlf * pl.t_coh);
    int64_t ns = 1;
    while (ns < pl.n_k) ns *= 2;
    int64_t nfft = 1;
    if (b.n_fft_override > 0) {
        nfft = b.n_fft_override;
        if (nfft % ns != 0)
            return fail(c, CCR_EINVAL, "n_fft_override %lld is not a multiple of %lld", (long long)nfft,
                        (long long)ns);
    } else {
        while ((double)nfft < nfft0) nfft *= 2;
        if (nfft < ns) nfft = ns;
    }
    // segments of at most 128 samples are transformed as 256 points (zero-padded; P halves) where
    // N_FFT allows: the same P n_s points per segment, on the kernels built for 256 to 1024 points
    if (ns < 256 && nfft >= 256 && nfft % 256 == 0) ns = 256;
    pl.n_s = ns;
    pl.n_fft = nfft;
    pl.P = nfft / ns;
    pl.t_fft = pl.dt * (double)nfft;
    pl.nu_r = pl.dlf * pl.t_fft;
    pl.n_f = (int64_t)std::floor(b.f_band / pl.dlf);
    pl.k_lo = (int64_t)std::ceil(-0.5 * b.f_band * pl.t_fft);
    if (pl.n_f < 1) return fail(c, CCR_ERANGE, "band holds no output bin");
    if (ns > 2048) return fail(c, CCR_ERANGE, "segment of %lld samples exceeds the 2048-point LDS FFT", (long long)pl.n_k);
    if (nfft > (1 << 22)) return fail(c, CCR_ERANGE, "N_FFT %lld too large", (long long)nfft);
    if (pl.n_seg < 1) return fail(c, CCR_EINVAL, "fewer samples than one segment");
    if (pl.n_seg * (int64_t)CCR_MAX_DET >= (1ll << 31) || pl.n_seg * pl.n_k >= (1ll << 40))
        return fail(c, CCR_ERANGE, "too many segments");
    return CCR_OK;
}

int64_t bin_index(const Plan &pl, int64_t i) { return pl.k_lo + (int64_t)std::floor(pl.nu_r * (double)i); }

// ------------------------------------------------------------------ Earth model

// r(t).n = C + A_o cos(theta_o) + A_d cos(theta_d):
//   orbit:    au [n_x cos(lam) + (n_y cos eps + n_z sin eps) sin(lam)] = A_o cos(lam - lam_n)
//   rotation: re [cos(lat) cos(dec) cos(g + lon - ra) + sin(lat) sin(dec)]
struct EarthModel {
    long double A_o, lam_n, w_o, ph_o, A_d, w_d, ph_d, C;
    long double theta_o(long double t) const { return ph_o + w_o * t - lam_n; }
    long double theta_d(long double t) const { return ph_d + w_d * t; }
    long double e(long double t) const { return C + A_o * cosl(theta_o(t)) + A_d * cosl(theta_d(t)); }
    long double ed(long double t) const {
        return -A_o * w_o * sinl(theta_o(t)) - A_d * w_d * sinl(theta_d(t));
    }
};

EarthModel earth_model(const ccr_sky &s, const ccr_site &site) {
    EarthModel m;
    long double nx = cosl(s.ra) * cosl(s.dec), ny = sinl(s.ra) * cosl(s.dec), nz = sinl(s.dec);
    long double q = ny * cosl(s.obliquity) + nz * sinl(s.obliquity);
    m.A_o = s.au_s * sqrtl(nx * nx + q * q);
    m.lam_n = atan2l(q, nx);
    m.w_o = 2.0L * kPiL / s.year_s;
    m.ph_o = s.orbit_phase0;
    m.A_d = s.re_s * cosl(site.lat) * cosl(s.dec);
    m.w_d = 2.0L * kPiL / s.sidereal_day_s;
    m.ph_d = s.gmst0 + site.lon - s.ra;
    m.C = s.re_s * sinl(site.lat) * sinl(s.dec);
    return m;
}

// Detector time t with t + r(t).n = tau (Earth-only inverse), long double Newton.
long double earth_inverse(const EarthModel &m, long double tau) {
    long double t = tau - m.e(tau);
    for (int it = 0; it < 8; ++it) {
        long double g = t + m.e(t) - tau;
        long double step = g / (1.0L + m.ed(t));
        t -= step;
        if (fabsl(step) < 1e-16L) break;
    }
    return t;
}

// Host copy of the anchored Earth-only delay (a_p = 0) used for the gap mask: eta solves
// eta + de(u + eta) = 0 where de(x) = r(t_a + x).n - r(t_a).n.
void sincos_small_h(double x, double &s, double &cm1) {
    const double x2 = x * x;
    s = x * (1.0 - x2 * (1.0 / 6.0) * (1.0 - x2 * (1.0 / 20.0) * (1.0 - x2 * (1.0 / 42.0) *
             (1.0 - x2 * (1.0 / 72.0) * (1.0 - x2 * (1.0 / 110.0))))));
    cm1 = -x2 * 0.5 * (1.0 - x2 * (1.0 / 12.0) * (1.0 - x2 * (1.0 / 30.0) * (1.0 - x2 * (1.0 / 56.0) *
             (1.0 - x2 * (1.0 / 90.0) * (1.0 - x2 * (1.0 / 132.0))))));
}

double earth_only_eta(const EarthConst &ec, const Anchor &an, double u) {
    double eta = 0.0;
    for (int it = 0; it < 3; ++it) {
        const double x = u + eta;
        double so, co, sd, cd;
        sincos_small_h(ec.w_o * x, so, co);
        sincos_small_h(ec.w_d * x, sd, cd);
        const double de = ec.A_o * (an.c_o * co - an.s_o * so) + ec.A_d * (an.c_d * cd - an.s_d * sd) + an.rho_a;
        const double dep = -ec.A_o * ec.w_o * (an.c_o * so + std::fma(an.s_o, co, an.s_o)) -
                           ec.A_d * ec.w_d * (an.c_d * sd + std::fma(an.s_d, cd, an.s_d));
        eta -= (eta + de) / (1.0 + dep);
    }
    return eta;
}

// ------------------------------------------------------------------ band preparation

template <typename T>
ccr_status upload(ccr_ctx *c, DevBuf &d, const std::vector<T> &h) {
    HIP_OK(c, d.ensure(std::max<size_t>(sizeof(T), h.size() * sizeof(T))));
    if (!h.empty()) HIP_OK(c, hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return CCR_OK;
}

ccr_status check_ready(ccr_ctx *c, Band &B) {
    int Q = 0;
    for (int X = 0; X < CCR_MAX_DET; ++X)
        if (B.det[X].has_data) Q = X + 1;
    if (Q == 0) return fail(c, CCR_ESTATE, "no detector data set");
    for (int X = 0; X < Q; ++X) {
        if (!B.det[X].has_data) return fail(c, CCR_ESTATE, "detector %d has no data", X);
        if (!B.det[X].has_weights) return fail(c, CCR_ESTATE, "detector %d has no weights", X);
        if (B.det[X].n != B.det[0].n)
            return fail(c, CCR_EINVAL, "detectors hold different sample counts");
    }
    B.Q = Q;
    return CCR_OK;
}

// Farrow form of the resampler's tap weights (split precision): c_n(dc) = w sinc(dc - n) on
// dc in [-1/2, 1/2] is fitted as [n == 0] + sum_{k=1..kFarDeg} A[k - 1][n + D] dc^k by least
// squares on 64 Chebyshev points (modified Gram-Schmidt, twice, in long double), with the
// constant term exact so that an on-grid sample stays the input sample.  Returns the largest
// sum_n |fit - c_n| over a grid of 4001 offsets (infinity if the window's centre weight is not 1).
double farrow_fit(int D, int window, const std::vector<double> &w64, std::vector<double> &A) {
    constexpr int NP = 64, NK = kFarDeg;
    const int NT = 2 * D + 1;
    auto tap = [&](long double dc, int n) -> long double {
        const long double d = dc - (long double)n;
        const long double sc = d == 0.0L ? 1.0L : sinl(kPiL * d) / (kPiL * d);
        const long double w =
            window == 0 ? (long double)w64[n + D] : 0.54L + 0.46L * cosl(kPiL * d / (long double)(D + 1));
        return w * sc;
    };
    const long double w0 = window == 0 ? (long double)w64[D] : 1.0L;
    if (fabsl(w0 - 1.0L) > 1e-15L) return INFINITY;
    long double x[NP], Qm[NK][NP], Rm[NK][NK] = {};
    for (int i = 0; i < NP; ++i) x[i] = 0.5L * cosl(kPiL * ((long double)i + 0.5L) / NP);
    for (int k = 0; k < NK; ++k) {
        for (int i = 0; i < NP; ++i) Qm[k][i] = powl(x[i], k + 1);
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < k; ++q) {
                long double d = 0.0L;
                for (int i = 0; i < NP; ++i) d += Qm[q][i] * Qm[k][i];
                Rm[q][k] += d;
                for (int i = 0; i < NP; ++i) Qm[k][i] -= d * Qm[q][i];
            }
        long double nn = 0.0L;
        for (int i = 0; i < NP; ++i) nn += Qm[k][i] * Qm[k][i];
        nn = sqrtl(nn);
        Rm[k][k] = nn;
        for (int i = 0; i < NP; ++i) Qm[k][i] /= nn;
    }
    A.assign((size_t)NK * NT, 0.0);
    std::vector<long double> Al((size_t)NK * NT);
    for (int n = -D; n <= D; ++n) {
        long double b[NP], qb[NK], a[NK];
        for (int i = 0; i < NP; ++i) b[i] = tap(x[i], n) - (n == 0 ? 1.0L : 0.0L);
        for (int k = 0; k < NK; ++k) {
            qb[k] = 0.0L;
            for (int i = 0; i < NP; ++i) qb[k] += Qm[k][i] * b[i];
        }
        for (int k = NK - 1; k >= 0; --k) {
            long double v = qb[k];
            for (int q = k + 1; q < NK; ++q) v -= Rm[k][q] * a[q];
            a[k] = v / Rm[k][k];
        }
        for (int k = 0; k < NK; ++k) {
            Al[(size_t)k * NT + n + D] = a[k];
            A[(size_t)k * NT + n + D] = (double)a[k];
        }
    }
    long double worst = 0.0L;
    for (int g = 0; g <= 4000; ++g) {
        const long double dc = -0.5L + (long double)g / 4000.0L;
        long double e = 0.0L;
        for (int n = -D; n <= D; ++n) {
            long double v = 0.0L;
            for (int k = NK - 1; k >= 0; --k) v = (v + (long double)A[(size_t)k * NT + n + D]) * dc;
            e += fabsl(v + (n == 0 ? 1.0L : 0.0L) - tap(dc, n));
        }
        worst = std::max(worst, e);
    }
    return (double)worst;
}

// Largest fit error accepted for the Farrow form (sum over the taps, relative to the input
// amplitude): below the split path's FP32 rounding of the tap sum.
constexpr double kFarTol = 4e-7;

ccr_status prepare(ccr_ctx *c, Band &B) {
    if (B.prepared) return CCR_OK;
    ccr_status st = check_ready(c, B);
    if (st) return st;
    // the band's device tables are about to be replaced: finish work that may read them
    if (c->device >= 0) HIP_OK(c, hipDeviceSynchronize());
    c->gen++;
    Plan pl;
    st = make_plan(c, B, pl);
    if (st) return st;
    const int Q = B.Q;
    const int64_t M = pl.n_seg, nk = pl.n_k, nr = M * nk;
    for (int X = 0; X < Q; ++X)
        if ((int64_t)B.det[X].a.size() != M)
            return fail(c, CCR_EINVAL, "detector %d weights hold %zu segments, plan has %lld", X,
                        B.det[X].a.size(), (long long)M);
    int n_ps = 0;
    for (int X = 0; X < Q; ++X) {
        if (B.det[X].ar.empty()) continue;
        ++n_ps;
        if ((int64_t)B.det[X].ar.size() < nr)
            return fail(c, CCR_EINVAL, "detector %d antenna functions hold %zu samples, the segments need %lld", X,
                        B.det[X].ar.size(), (long long)nr);
    }
    if (n_ps != 0 && n_ps != Q)
        return fail(c, CCR_EINVAL, "per-sample antenna functions set for %d of %d detectors", n_ps, Q);
    const bool per_sample = n_ps == Q;
    const double dt = pl.dt, t0 = B.det[0].t0;
    // Earth constants and per-segment anchors
    std::vector<EarthConst> earth(Q);
    std::vector<Anchor> anchors((size_t)Q * M);
    std::vector<EarthModel> em(Q);
    for (int X = 0; X < Q; ++X) {
        em[X] = earth_model(c->sky, B.det[X].site);
        earth[X] = EarthConst{(double)em[X].A_o, (double)em[X].w_o, (double)em[X].A_d, (double)em[X].w_d};
    }
    parallel_for((int64_t)Q * M, [&](int64_t e) {
        const int X = (int)(e / M);
        const int64_t K = e % M;
        const EarthModel &m = em[X];
        long double tau_a = (long double)t0 + ((long double)(K * nk) + 0.5L * (long double)nk) * (long double)dt;
        // t_a and tau_a are representable long doubles, so D_a = tau_a - t_a is exact; the
        // rounding of t_a leaves the residual rho_a = r(t_a).n - D_a, kept explicitly.
        long double ta = earth_inverse(m, tau_a);
        long double Da = tau_a - ta;
        long double rho = m.e(ta) - Da;
        long double psi = -(long double)pl.f_het * Da;
        psi -= floorl(psi);
        long double tho = m.theta_o(ta), thd = m.theta_d(ta);
        anchors[e] = Anchor{(double)cosl(tho), (double)sinl(tho), (double)cosl(thd), (double)sinl(thd),
                            (double)Da, (double)rho, (double)psi};
    });
    // gap mask of source samples (Earth-only centre tap) and valid fractions
    std::vector<uint8_t> mask((size_t)Q * nr);
    std::vector<double> phi((size_t)Q * M);
    const int64_t n = B.det[0].n;
    parallel_for((int64_t)Q * M, [&](int64_t e) {
        const int X = (int)(e / M);
        const int64_t K = e % M;
        const Anchor &an = anchors[e];
        const std::vector<uint8_t> &val = B.det[X].valid;
        int64_t cnt = 0;
        for (int64_t s = 0; s < nk; ++s) {
            const int64_t r = K * nk + s;
            const double u = ((double)s - 0.5 * (double)nk) * dt;
            const double eta = earth_only_eta(earth[X], an, u);
            const double q = (eta - an.D_a) / dt;
            const int64_t j = r + (int64_t)std::floor(q + 0.5);
            uint8_t m = 0;
            if (j >= 0 && j < n) m = val.empty() ? 1 : (val[j] ? 1 : 0);
            mask[(size_t)X * nr + r] = m;
            cnt += m;
        }
        phi[e] = (double)cnt / (double)nk;
    });
    // weights, pair set, normalisation, activity
    std::vector<SegWeight> segw((size_t)Q * M);
    for (int X = 0; X < Q; ++X)
        for (int64_t K = 0; K < M; ++K) {
            const double sg = std::sqrt(B.det[X].nv[K]);
            segw[X * M + K] = SegWeight{B.det[X].a[K] / sg, B.det[X].b[K] / sg, 1.0 / (sg * std::sqrt((double)nk))};
        }
    // stream moments A_XK = E|F^a_XK|^2, B_XK, C_XK (Sec. III.B.3 eq. norm-a-eq with App. A): the
    // segment mean of m_r hat a_r^2, m_r hat b_r^2, m_r hat a_r hat b_r (m the gap mask, hat a =
    // a / sigma_XK); with per-segment weights hat a_XK^2 phi_XK, ...
    std::vector<double> mom((size_t)3 * Q * M);
    parallel_for((int64_t)Q * M, [&](int64_t e) {
        const int X = (int)(e / M);
        const int64_t K = e % M;
        const SegWeight &w = segw[e];
        double A = w.ahat * w.ahat * phi[e], Bm = w.bhat * w.bhat * phi[e], C = w.ahat * w.bhat * phi[e];
        if (per_sample) {
            const double isg = 1.0 / std::sqrt(B.det[X].nv[K]);
            A = Bm = C = 0.0;
            for (int64_t s = 0; s < nk; ++s) {
                const int64_t r = K * nk + s;
                if (!mask[(size_t)X * nr + r]) continue;
                const double ar = B.det[X].ar[r] * isg, br = B.det[X].br[r] * isg;
                A += ar * ar;
                Bm += br * br;
                C += ar * br;
            }
            A /= (double)nk;
            Bm /= (double)nk;
            C /= (double)nk;
        }
        mom[3 * e] = A;
        mom[3 * e + 1] = Bm;
        mom[3 * e + 2] = C;
    });
    // pair set, normalisation N^2 = sum_P A_K A_L + 2 C_K C_L + B_K B_L (Gamma^ave) or
    // sum_P A_K B_L + B_K A_L - 2 C_K C_L (Gamma^circ), and the segments that take part
    const int R = B.p.max_lag;
    const bool cross = B.p.pairs & CCR_PAIRS_CROSS, same = B.p.pairs & CCR_PAIRS_SAME;
    const bool allp = B.p.pairs == CCR_PAIRS_ALL, circ = B.p.weight == CCR_WEIGHT_CIRC;
    std::vector<uint8_t> active((size_t)Q * M, 0);
    long double nacc = 0.0L;
    int64_t npairs = 0;
    auto pair_norm = [&](size_t k, size_t l) -> long double {
        const double *a = &mom[3 * k], *b = &mom[3 * l];
        return circ ? (long double)a[0] * b[1] + (long double)a[1] * b[0] - 2.0L * a[2] * b[2]
                    : (long double)a[0] * b[0] + 2.0L * a[2] * b[2] + (long double)a[1] * b[1];
    };
    if (allp) {
        // every ordered pair: the double sum factorises into sums over segments
        long double sa = 0.0L, sb = 0.0L, sc = 0.0L;
        for (int64_t e = 0; e < (int64_t)Q * M; ++e) {
            sa += mom[3 * e];
            sb += mom[3 * e + 1];
            sc += mom[3 * e + 2];
            active[e] = phi[e] > 0.0 ? 1 : 0;
        }
        nacc = circ ? 2.0L * sa * sb - 2.0L * sc * sc : sa * sa + 2.0L * sc * sc + sb * sb;
        npairs = (int64_t)Q * M * Q * M;
    } else {
        for (int X = 0; X < Q; ++X)
            for (int64_t K = 0; K < M; ++K)
                for (int Y = 0; Y < Q; ++Y)
                    for (int64_t L = std::max<int64_t>(0, K - R); L <= std::min<int64_t>(M - 1, K + R); ++L) {
                        bool in = (cross && X < Y) || (same && X == Y && L > K);
                        if (!in) continue;
                        ++npairs;
                        const double fk = phi[X * M + K], fl = phi[Y * M + L];
                        if (fk > 0.0 && fl > 0.0) {
                            active[X * M + K] = 1;
                            active[Y * M + L] = 1;
                        }
                        nacc += pair_norm((size_t)(X * M + K), (size_t)(Y * M + L));
                    }
    }
    pl.norm = nacc > 0.0L ? (double)sqrtl(nacc) : 0.0;
    pl.n_pairs = npairs;
    std::vector<int> work, seg_work((size_t)Q * M, -1);
    for (int X = 0; X < Q; ++X)
        for (int64_t K = 0; K < M; ++K)
            if (active[X * M + K]) {
                seg_work[X * M + K] = (int)work.size();
                work.push_back((int)(X * M + K));
            }
    // bins and twiddles
    std::vector<int> bm(pl.n_f), bp(pl.n_f), bkb(pl.n_f);
    B.freqs.resize(pl.n_f);
    for (int64_t i = 0; i < pl.n_f; ++i) {
        int64_t kb = bin_index(pl, i);
        B.freqs[i] = pl.f_het + (double)kb / pl.t_fft;
        int64_t km = kb % pl.n_fft;
        if (km < 0) km += pl.n_fft;
        bkb[i] = (int)km;
        bp[i] = (int)(km % pl.P);
        bm[i] = (int)(km / pl.P);
    }
    std::vector<int> bpos(pl.n_fft, -1);
    int unique = 1;
    for (int64_t i = 0; i < pl.n_f; ++i) {
        if (bpos[bkb[i]] >= 0) unique = 0;
        bpos[bkb[i]] = (int)i;
    }
    std::vector<double2> tw64(pl.n_fft);
    std::vector<float2> tw32(pl.n_fft);
    for (int64_t j = 0; j < pl.n_fft; ++j) {
        long double a = -2.0L * kPiL * (long double)j / (long double)pl.n_fft;
        tw64[j] = make_double2((double)cosl(a), (double)sinl(a));
        tw32[j] = make_float2((float)cosl(a), (float)sinl(a));
    }
    // ring columns of the spectra + pair-sum kernel: bins ordered by (residue class, index in
    // the class), so the 16 lanes of an FFT group, which hold consecutive outputs of one class,
    // write consecutive columns
    std::vector<int> col_bin(pl.n_f), bin_col(pl.n_f);
    for (int64_t i = 0; i < pl.n_f; ++i) col_bin[i] = (int)i;
    std::stable_sort(col_bin.begin(), col_bin.end(),
                     [&](int a, int b) { return bp[a] != bp[b] ? bp[a] < bp[b] : bm[a] < bm[b]; });
    for (int64_t cc = 0; cc < pl.n_f; ++cc) bin_col[col_bin[cc]] = (int)cc;
    // the same order groups the bins by residue class: class p is [class_start[p], class_start[p + 1])
    std::vector<int> class_start((size_t)pl.P + 1, 0);
    for (int64_t cc = 0; cc < pl.n_f; ++cc) ++class_start[(size_t)bp[col_bin[cc]] + 1];
    for (int64_t q = 0; q < pl.P; ++q) class_start[(size_t)q + 1] += class_start[(size_t)q];
    // 1024-point kernel: the bins of class p, at FFT outputs m (ascending in column order), span
    // a circular range of the n_s outputs; m0 = the output after the range's largest gap, so the
    // class occupies m0 .. m0 + span - 1 (mod n_s)
    std::vector<int> cls_m0((size_t)pl.P, 0);
    int wide_jmax = 0, wide_ncol = 0;
    for (int64_t q = 0; q < pl.P; ++q) {
        const int a = class_start[(size_t)q], b = class_start[(size_t)q + 1];
        wide_ncol = std::max(wide_ncol, b - a);
        if (b == a) continue;
        int best_gap = -1, m0 = bm[col_bin[a]];
        for (int cc = a; cc < b; ++cc) {
            const int m = bm[col_bin[cc]];
            const int prev = bm[col_bin[cc == a ? b - 1 : cc - 1]];
            const int gap = (int)((m - prev + pl.n_s) % pl.n_s);
            if (gap > best_gap) {
                best_gap = gap;
                m0 = m;
            }
        }
        int span = 0;
        for (int cc = a; cc < b; ++cc) span = std::max(span, (int)((bm[col_bin[cc]] - m0 + pl.n_s) % pl.n_s) + 1);
        cls_m0[(size_t)q] = m0;
        wide_jmax = std::max(wide_jmax, (span + 63) / 64);
    }
    // lag phases of the pair sum (spectra taken without Phi_in), in ring-column order
    const int64_t Rl = B.p.max_lag;
    std::vector<float2> lagph((size_t)(Rl + 1) * pl.n_f);
    for (int64_t dl = 0; dl <= Rl; ++dl)
        for (int64_t cc = 0; cc < pl.n_f; ++cc) {
            const int64_t i = col_bin[cc];
            const int64_t e = (int64_t)(((__int128)bkb[i] * dl * pl.n_k) % pl.n_fft);
            const long double a = 2.0L * kPiL * (long double)e / (long double)pl.n_fft;
            lagph[(size_t)(dl * pl.n_f + cc)] = make_float2((float)cosl(a), (float)sinl(a));
        }
    const int D = B.p.dirichlet_D;
    std::vector<double> w64(2 * D + 1);
    std::vector<float> w32(2 * D + 1);
    for (int nn = -D; nn <= D; ++nn) {
        long double w = 0.54L - 0.46L * cosl(2.0L * kPiL * (long double)(nn + D) / (2.0L * D));
        w64[nn + D] = (double)w;
        w32[nn + D] = (float)w;
    }
    B.n_work = (int)work.size();
    B.active = std::move(active);
    B.plan = pl;
    B.far_len = 0;
    std::vector<double> farA;
    B.far_err = farrow_fit(D, B.p.window, w64, farA);
    if (c->device < 0) {  // host-only context: planning and validation without device tables
        B.prepared = true;
        return CCR_OK;
    }
    // Chebyshev nodes x_j of an N-node rule (N = kCheb ... kChebSplitLow) and the maps from
    // node values to the monomial coefficients of the interpolant: Chebyshev coefficients
    // c_k = (2 / N) sum_j eta_j T_k(x_j) (c_0 halved), then the monomial coefficients of each
    // T_k (T_{k+1} = 2 x T_k - T_{k-1}); long double, rows and columns beyond N zero
    std::vector<double> cx(kChebNodesAll), mono(kChebRules * kCheb * kCheb, 0.0);
    {
        long double Tm[kCheb][kCheb] = {};  // Tm[k][m]: coefficient of x^m in T_k
        Tm[0][0] = 1.0L;
        Tm[1][1] = 1.0L;
        for (int k = 1; k + 1 < kCheb; ++k)
            for (int m = 0; m < kCheb; ++m)
                Tm[k + 1][m] = (m > 0 ? 2.0L * Tm[k][m - 1] : 0.0L) - Tm[k - 1][m];
        for (int N : {kCheb, kChebSplit, kChebSplitMin, kChebSplitLow}) {
            const int v = cheb_rule(N);
            for (int j = 0; j < N; ++j) cx[cheb_x_off(N) + j] = (double)cosl(kPiL * ((long double)j + 0.5L) / N);
            for (int m = 0; m < N; ++m)
                for (int j = 0; j < N; ++j) {
                    long double a = 0.0L;
                    for (int k = 0; k < N; ++k) {
                        const long double ck = (k == 0 ? 1.0L : 2.0L) / N *
                                               cosl(kPiL * (long double)k * ((long double)j + 0.5L) / N);
                        a += Tm[k][m] * ck;
                    }
                    mono[((size_t)v * kCheb + m) * kCheb + j] = (double)a;
                }
        }
    }
    // device upload
    std::vector<float2> xs((size_t)Q * n);
    for (int X = 0; X < Q; ++X)
        std::memcpy(&xs[(size_t)X * n], B.det[X].x.data(), sizeof(float2) * (size_t)n);
    if ((st = upload(c, B.d_x, xs))) return st;
    if ((st = upload(c, B.d_mask, mask))) return st;
    if ((st = upload(c, B.d_anchor, anchors))) return st;
    if ((st = upload(c, B.d_earth, earth))) return st;
    if ((st = upload(c, B.d_win64, w64))) return st;
    if ((st = upload(c, B.d_win32, w32))) return st;
    if ((st = upload(c, B.d_cheb_x, cx))) return st;
    if ((st = upload(c, B.d_mono, mono))) return st;
    if ((st = upload(c, B.d_tw64, tw64))) return st;
    if ((st = upload(c, B.d_tw32, tw32))) return st;
    if ((st = upload(c, B.d_lagph, lagph))) return st;
    if ((st = upload(c, B.d_col_bin, col_bin))) return st;
    if ((st = upload(c, B.d_bin_col, bin_col))) return st;
    if ((st = upload(c, B.d_class_start, class_start))) return st;
    if ((st = upload(c, B.d_cls_m0, cls_m0))) return st;
    B.wide_jmax = wide_jmax;
    B.wide_ncol = wide_ncol;
    if ((st = upload(c, B.d_zero256, std::vector<float2>(256, make_float2(0.f, 0.f))))) return st;
    {
        std::vector<int> any;
        for (int64_t K = 0; K < M; ++K) {
            bool a = false;
            for (int X = 0; X < Q; ++X) a = a || B.active[(size_t)X * M + K];
            if (a) any.push_back((int)K);
        }
        B.n_seg_any = (int)any.size();
        if ((st = upload(c, B.d_seg_any, any))) return st;
    }
    if ((st = upload(c, B.d_bin_m, bm))) return st;
    if ((st = upload(c, B.d_bin_p, bp))) return st;
    if ((st = upload(c, B.d_bin_kb, bkb))) return st;
    if ((st = upload(c, B.d_bin_pos, bpos))) return st;
    B.bins_unique = unique;
    if ((st = upload(c, B.d_segw, segw))) return st;
    {
        // the split path's pair weights: hat a scale and hat b scale rounded to FP32, zero for
        // a segment that takes part in no pair (no spectrum)
        std::vector<float2> segwf(segw.size());
        for (size_t e = 0; e < segw.size(); ++e)
            segwf[e] = seg_work[e] < 0 ? make_float2(0.f, 0.f)
                                       : make_float2((float)(segw[e].ahat * segw[e].scale),
                                                     (float)(segw[e].bhat * segw[e].scale));
        if ((st = upload(c, B.d_segwf, segwf))) return st;
    }
    // per-sample stream weights (a_r, b_r) / (sigma_XK^2 sqrt(N_K)): hat a_r times the spectra's
    // 1 / (sigma sqrt N_K)
    B.per_sample = per_sample;
    if (per_sample) {
        std::vector<double2> pw((size_t)Q * nr);
        parallel_for((int64_t)Q * M, [&](int64_t e) {
            const int X = (int)(e / M);
            const int64_t K = e % M;
            const double f = 1.0 / (B.det[X].nv[K] * std::sqrt((double)nk));
            for (int64_t s = 0; s < nk; ++s) {
                const int64_t r = K * nk + s;
                pw[(size_t)X * nr + r] = make_double2(B.det[X].ar[r] * f, B.det[X].br[r] * f);
            }
        });
        if ((st = upload(c, B.d_pw, pw))) return st;
        // FP32 copy for the split path's two-stream resampling
        std::vector<float2> pwf(pw.size());
        for (size_t i = 0; i < pw.size(); ++i) pwf[i] = make_float2((float)pw[i].x, (float)pw[i].y);
        if ((st = upload(c, B.d_pwf, pwf))) return st;
    } else {
        B.d_pw.release();
        B.d_pwf.release();
    }
    if ((st = upload(c, B.d_active, B.active))) return st;
    if ((st = upload(c, B.d_work, work))) return st;
    if ((st = upload(c, B.d_seg_work, seg_work))) return st;
    // Farrow table of the split-precision resampler (kept out when the fit is not accurate
    // enough or the table does not fit in device memory)
    {
        const int64_t L = (n + 2 * D + 255) / 256 * 256;
        if (B.far_err <= kFarTol) {
            if ((st = upload(c, B.d_farrow_A, farA))) return st;
            if (B.d_farrow.ensure((size_t)Q * (kFarDeg + 1) * L * sizeof(float2)) == hipSuccess) {
                HIP_OK(c, launch_farrow_table(B.d_x.as<float2>(), n, Q, D, B.d_farrow_A.as<double>(), L,
                                              B.d_farrow.as<float2>(), nullptr));
                HIP_OK(c, hipStreamSynchronize(nullptr));
                B.far_len = L;
            } else {
                (void)hipGetLastError();
            }
        }
    }
    B.prepared = true;
    return CCR_OK;
}

// Amplitudes of the harmonics of an eccentric orbit's delay R/c (eqs. solve-for-E,
// Kepler-equation) in the mean anomaly: with cos E = -e/2 + sum_k (2/k) J'_k(ke) cos kM and
// sin E = sum_k (2/(ke)) J_k(ke) sin kM, harmonic k of
// a_p [sin w (cos E - e) + cos w sqrt(1 - e^2) sin E] has amplitude
// a_p sqrt((sin w (2/k) J'_k(ke))^2 + (cos w sqrt(1 - e^2) (2/(ke)) J_k(ke))^2).  Harmonics are
// listed until they fall below 1e-24 a_p (at most 4000).
std::vector<double> orbit_harmonics(double ap, double e, double w) {
    std::vector<double> A;
    if (e == 0.0) {
        A.push_back(ap);
        return A;
    }
    const double sw = std::sin(w), cw = std::cos(w), q = std::sqrt(1.0 - e * e);
    for (int k = 1; k <= 4000; ++k) {
        const double x = k * e;
        const double jk = std::cyl_bessel_j((double)k, x);
        const double jd = 0.5 * (std::cyl_bessel_j((double)(k - 1), x) - std::cyl_bessel_j((double)(k + 1), x));
        const double a = sw * 2.0 / k * jd, b = cw * q * 2.0 / x * jk;
        const double amp = ap * std::sqrt(a * a + b * b);
        A.push_back(amp);
        if (k > 4 && amp < 1e-24 * ap) break;
    }
    return A;
}

// Bound on the Chebyshev coefficients from degree n on of A sin(omega u + phi) over [-h, h]:
// 2 A sum_{m >= n} z^m / m!, z = omega h / 2 (the coefficients are 2 A J_m(omega h)).
double cheb_tail(double A, double omega, double h, int n) {
    const double z = 0.5 * omega * h;
    if (z > 40.0) return HUGE_VAL;
    double term = 2.0 * A, sum = 0.0;
    for (int m = 1; m < n; ++m) term *= z / m;
    for (int m = n; m < n + 400; ++m) {
        if (m > 0) term *= z / m;
        sum += term;
        if (m > z && term < 1e-40 * (sum + 1e-300)) break;
    }
    return sum;
}

ccr_status prepare_templates(ccr_ctx *c, Band &B) {
    const Plan &pl = B.plan;
    if (c->device >= 0) HIP_OK(c, hipDeviceSynchronize());
    c->gen++;
    const int64_t T = B.n_tmpl;
    const long double t0 = B.det[0].t0, dt = pl.dt;
    const long double tseg = (long double)pl.n_k * dt;
    const long double tau_a0 = t0 + 0.5L * tseg;
    auto raw = [&](int64_t t, int k) { return B.tmpl_raw[(size_t)t * kRawStride + k]; };
    // Series validity of the in-kernel small-angle expansions (|angle| <= 0.3); for an eccentric
    // orbit the same bound keeps the mean-anomaly offsets of the Kepler solve small.
    const double ld = 0.5 * (double)tseg + 1.0;
    for (int64_t t = 0; t < T; ++t) {
        const double ap = raw(t, 0), P = raw(t, 2), e = raw(t, 3);
        const double apm = ap * (1.0 + e);  // largest |R/c|
        const double Om = 2.0 * kPi / P;
        if (Om * (ld + 2.0 * apm + 2.0) > 0.3)
            return fail(c, CCR_ERANGE, "template %lld: orbit too short for the segment length", (long long)t);
        // the kernels hold the sample shift of a delay (Earth + binary) in 32 bits
        if ((c->sky.au_s + c->sky.re_s + apm + 1.0) / (double)dt > (double)(1 << 30))
            return fail(c, CCR_ERANGE, "template %lld: delay too long for the sampling interval", (long long)t);
        if (B.ecc && e > 0.0) {
            // six Newton steps of the anchor-relative Kepler solve: from d0 = dM / (1 - e cos E_a)
            // the error is at most Kc d0^2, Kc = e / (2 (1 - e)) bounding f'' / (2 f'), and each
            // step maps err -> Kc err^2
            const double d0 = Om * (ld + 2.0 * apm + 2.0) / (1.0 - e);
            const double Kc = e / (2.0 * (1.0 - e));
            double err = Kc * d0 * d0;
            for (int it = 0; it < 6; ++it) err = Kc * err * err;
            if (!(err < 1e-17))
                return fail(c, CCR_ERANGE, "template %lld: Kepler solve does not converge over a segment (e = %.3g)",
                            (long long)t, e);
        }
    }
    {
        EarthModel m = earth_model(c->sky, B.det[0].site);
        if ((double)m.w_d * (ld + 4.0) > 0.3) return fail(c, CCR_ERANGE, "segment too long for the time base");
    }
    // Newton steps of the node solve and Chebyshev terms of the split path, from bounds over the
    // templates and detectors.  Newton: the binary-only start is off by at most
    // e0 = de + a_p Omega_1 (a_p (1 + e) + de) (de: Earth-delay change over the segment; Omega_1 =
    // Omega / (1 - e) bounds the rate of R/c / a_p), and each step maps e -> K e^2 with
    // K = G''/(2 G'), G'' bounded with a_p Omega^2 / (1 - e)^3; two steps suffice when
    // K^3 e0^4 < 1e-20 s.
    // Chebyshev: the series of A sin(omega u + phi) on [-h, h] has coefficients 2A J_k(omega h)
    // <= 2A (omega h / 2)^k / k!, summed over the Earth terms and the orbit's harmonics (one for
    // a circular orbit).  The FP64 path's 10 nodes must leave twice the tail from k = 10 below
    // 1e-12 cycles of the top frequency and 1e-12 samples (else the template is rejected); the
    // split path interpolates at 5, 6 or else 7 nodes (error at most twice the tail from k = 5,
    // 6 or 7) when twice the tail stays below 1e-8 cycles and 1e-8 samples: under the FP32
    // rounding of the phase and the offset the split path applies afterwards (up to 3e-8 cycles
    // and 3e-8 samples).
    {
        double Aw = 0.0, Aw2 = 0.0;
        std::vector<std::pair<double, double>> comps;  // (amplitude, angular rate) of the Earth terms
        for (int X = 0; X < B.Q; ++X) {
            const EarthModel m = earth_model(c->sky, B.det[X].site);
            Aw = std::max(Aw, (double)(m.A_o * m.w_o + m.A_d * m.w_d));
            Aw2 = std::max(Aw2, (double)(m.A_o * m.w_o * m.w_o + m.A_d * m.w_d * m.w_d));
            comps.push_back({(double)m.A_o, (double)m.w_o});
            comps.push_back({(double)m.A_d, (double)m.w_d});
        }
        const double h = 0.5 * (double)tseg;
        const double f_top = B.p.f_min + B.p.f_band;
        double worst_e2 = 0.0, worst_tail = 0.0, worst_tail6 = 0.0, worst_tail5 = 0.0;
        std::vector<std::pair<std::pair<double, double>, std::vector<double>>> harm;  // (e, omega) -> harmonics / a_p
        for (int64_t t = 0; t < T; ++t) {
            const double ap = raw(t, 0), Om = 2.0 * kPi / raw(t, 2), e = raw(t, 3);
            const double Om1 = Om / (1.0 - e), Om2 = Om * Om / ((1.0 - e) * (1.0 - e) * (1.0 - e));
            const double X = h + ap * (1.0 + e) + 1.0;
            const double de = 1.01 * Aw * X + 1e-9;
            const double e0 = de + ap * Om1 * (ap * (1.0 + e) + de);
            const double K = (1.1 * ap * Om2 + 1.1 * Aw2) / (2.0 * (1.0 - ap * Om1) * (1.0 - Aw));
            const double e1 = K * e0 * e0, e2 = K * e1 * e1;
            worst_e2 = std::max(worst_e2, e2);
            std::vector<std::pair<double, double>> all = comps;
            if (B.ecc) {
                const std::pair<double, double> key{e, raw(t, 4)};
                size_t hi = 0;
                while (hi < harm.size() && harm[hi].first != key) ++hi;
                if (hi == harm.size()) {
                    if (harm.size() >= 64) harm.erase(harm.begin());
                    harm.push_back({key, orbit_harmonics(1.0, e, key.second)});
                    hi = harm.size() - 1;
                }
                const std::vector<double> &hk = harm[hi].second;
                for (size_t k = 0; k < hk.size(); ++k) all.push_back({ap * hk[k], (double)(k + 1) * Om});
            } else {
                all.push_back({ap, Om});
            }
            double tail = 0.0, tail6 = 0.0, tail5 = 0.0, tail10 = 0.0;
            for (const auto &cw : all) {
                const double hh = 1.01 * h;
                tail += cheb_tail(cw.first, cw.second, hh, kChebSplit);
                tail6 += cheb_tail(cw.first, cw.second, hh, kChebSplitMin);
                tail5 += cheb_tail(cw.first, cw.second, hh, kChebSplitLow);
                tail10 += cheb_tail(cw.first, cw.second, hh, kCheb);
            }
            if (!(2.0 * tail10 * f_top < 1e-12 && 2.0 * tail10 / (double)dt < 1e-12))
                return fail(c, CCR_ERANGE,
                            "template %lld: the time base's interpolation error bound (%.3g s) is too large for the "
                            "segment length (orbit too eccentric or too short)",
                            (long long)t, 2.0 * tail10);
            worst_tail = std::max(worst_tail, tail);
            worst_tail6 = std::max(worst_tail6, tail6);
            worst_tail5 = std::max(worst_tail5, tail5);
        }
        // short small-angle series (through x^7 / x^8) in the node solve when the dropped terms,
        // amplitude x |angle|^9 / 9! summed over the binary and Earth terms, stay below 1e-16 s
        // for every template (angles bounded as in the validity check above); an eccentric
        // orbit's delay is evaluated with full-range sin / cos, so only the Earth terms count
        double worst_series = 0.0;
        {
            double earth = 0.0;
            for (const auto &cw : comps) earth += cw.first * std::pow(cw.second * (ld + 4.0), 9) / 362880.0;
            worst_series = earth;
            for (int64_t t = 0; t < T && !B.ecc; ++t) {
                const double ap = raw(t, 0), Om = 2.0 * kPi / raw(t, 2);
                worst_series = std::max(worst_series, ap * std::pow(Om * (ld + 2.0 * ap + 2.0), 9) / 362880.0 + earth);
            }
        }
        B.short_series = worst_series < 1e-16;
        B.newton_steps = worst_e2 < 1e-20 ? 2 : 3;
        auto fits = [&](double tl) { return 2.0 * tl * f_top < 1e-8 && 2.0 * tl / (double)dt < 1e-8; };
        B.cheb_split = fits(worst_tail5)   ? kChebSplitLow
                       : fits(worst_tail6) ? kChebSplitMin
                                           : (fits(worst_tail) ? kChebSplit : kCheb);
    }
    B.tmpl.assign((size_t)T * kTmplStride, 0.0);
    for (int64_t t = 0; t < T; ++t) {
        const long double ap = raw(t, 0), tref = raw(t, 1), P = raw(t, 2);
        long double c0 = (tau_a0 - tref) / P;
        c0 -= floorl(c0);
        long double c1 = tseg / P;
        double *o = &B.tmpl[(size_t)t * kTmplStride];
        o[0] = (double)ap;
        o[1] = (double)(2.0L * kPiL / P);
        o[2] = (double)c0;
        o[3] = (double)(c0 - (long double)o[2]);
        o[4] = (double)c1;
        o[5] = (double)(c1 - (long double)o[4]);
        const long double e = raw(t, 3), w = raw(t, 4);
        o[6] = (double)e;
        o[7] = (double)sinl(w);
        o[8] = (double)cosl(w);
        o[9] = (double)sqrtl(1.0L - e * e);
    }
    if (c->device < 0) return CCR_OK;
    return upload(c, B.d_tmpl, B.tmpl);
}

BandDev band_dev(const Band &B) {
    const Plan &pl = B.plan;
    BandDev d;
    d.Q = B.Q;
    d.n = B.det[0].n;
    d.n_k = (int)pl.n_k;
    d.n_seg = (int)pl.n_seg;
    d.n_fft = (int)pl.n_fft;
    d.n_s = (int)pl.n_s;
    d.P = (int)pl.P;
    d.nfft_mask = (pl.n_fft & (pl.n_fft - 1)) == 0 ? (int)(pl.n_fft - 1) : 0;
    d.n_f = (int)pl.n_f;
    d.D = B.p.dirichlet_D;
    d.window = B.p.window;
    d.R = B.p.max_lag;
    d.pairs = B.p.pairs;
    d.dt = pl.dt;
    d.inv_dt = 1.0 / pl.dt;
    d.f_het = pl.f_het;
    d.x = B.d_x.as<float2>();
    d.mask = B.d_mask.as<uint8_t>();
    d.anchors = B.d_anchor.as<Anchor>();
    d.earth = B.d_earth.as<EarthConst>();
    d.win64 = B.d_win64.as<double>();
    d.win32 = B.d_win32.as<float>();
    d.cheb_x = B.d_cheb_x.as<double>();
    d.mono = B.d_mono.as<double>();
    d.tw64 = B.d_tw64.as<double2>();
    d.tw32 = B.d_tw32.as<float2>();
    d.bin_m = B.d_bin_m.as<int>();
    d.bin_p = B.d_bin_p.as<int>();
    d.bin_kb = B.d_bin_kb.as<int>();
    d.bin_pos = B.d_bin_pos.as<int>();
    d.bins_unique = B.bins_unique;
    d.segw = B.d_segw.as<SegWeight>();
    d.segwf = B.d_segwf.as<float2>();
    d.active = B.d_active.as<uint8_t>();
    d.work = B.d_work.as<int>();
    d.seg_work = B.d_seg_work.as<int>();
    d.n_work = B.n_work;
    d.tmpl = B.d_tmpl.as<double>();
    d.lagph = B.d_lagph.as<float2>();
    d.col_bin = B.d_col_bin.as<int>();
    d.bin_col = B.d_bin_col.as<int>();
    d.class_start = B.d_class_start.as<int>();
    d.zero256 = B.d_zero256.as<float2>();
    d.seg_any = B.d_seg_any.as<int>();
    d.n_seg_any = B.n_seg_any;
    d.newton_steps = B.newton_steps;
    d.ecc = B.ecc ? 1 : 0;
    d.cheb_split = B.cheb_split;
    d.farrow = B.far_len > 0 ? B.d_farrow.as<float2>() : nullptr;
    d.far_len = B.far_len;
    d.far_stage = 1;
    d.cls_m0 = B.d_cls_m0.as<int>();
    d.wide_jmax = B.wide_jmax;
    d.wide_ncol = B.wide_ncol;
    d.weight = B.p.weight;
    d.allp = B.p.pairs == CCR_PAIRS_ALL ? 1 : 0;
    d.pw = B.per_sample ? B.d_pw.as<double2>() : nullptr;
    d.pwf = B.per_sample ? B.d_pwf.as<float2>() : nullptr;
    d.ps2 = 0;
    return d;
}

Band *get_band(ccr_ctx *c, int id) {
    if (id < 0 || id >= (int)c->bands.size()) return nullptr;
    return c->bands[id].get();
}

ccr_status ensure_ready(ccr_ctx *c, Band &B) {
    if (B.n_tmpl == 0 || B.tmpl_raw.empty()) return fail(c, CCR_ESTATE, "no templates set");
    bool was = B.prepared;
    ccr_status st = prepare(c, B);
    if (st) return st;
    if (!was || B.tmpl.empty()) {
        st = prepare_templates(c, B);
        if (st) return st;
    }
    return CCR_OK;
}

// Optional per-kernel device timing: events around a launch on its own stream.
struct LaunchTimer {
    ccr_ctx *c;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    LaunchTimer(ccr_ctx *c_, int k, hipStream_t s_, bool on = true) : c(c_), kind(k), s(s_) {
        if (!c->opt_timing || !on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    ~LaunchTimer() {
        if (!a) return;
        (void)hipEventRecord(b, s);
        c->timed.push_back({kind, a, b});
    }
};

void collect_times(ccr_ctx *c) {
    for (auto &t : c->timed) {
        float ms = 0.0f;
        if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            c->kt_ms[t.kind] += ms;
            c->kt_n[t.kind] += 1;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    c->timed.clear();
}


constexpr size_t kMaxLds = 65536;
// host staging (and scratch region) of the no-allocation entry point's tables
constexpr size_t kNoAllocTableBytes = (size_t)1 << 20;

ccr_status grow(ccr_ctx *c, DevBuf &b, size_t bytes);

// Fused path: one launch per template batch computes partial rho per (template, segment chunk)
// with every intermediate in LDS, then the chunk partials are summed in order.
ccr_status compute_fused(ccr_ctx *c, Band &B, const BandDev &bd, bool fp64, int S, void *rho_out,
                         int out_on_device, int out_fp64, hipStream_t s) {
    const Plan &pl = B.plan;
    int64_t kc = c->opt_k_chunk > 0 ? c->opt_k_chunk : std::min<int64_t>(pl.n_seg, 256);
    kc = std::max<int64_t>(kc, (pl.n_seg + 65534) / 65535);
    const int nch = (int)((pl.n_seg + kc - 1) / kc);
    int64_t tb = c->opt_template_batch;
    if (tb <= 0) {
        const int64_t per = (int64_t)nch * pl.n_f * 8 + (int64_t)std::max(B.n_work, 1) * kCheb * 8;
        tb = std::max<int64_t>(1, ((int64_t)2 << 30) / per);
    }
    tb = std::max<int64_t>(1, std::min<int64_t>({tb, (int64_t)65535, B.n_tmpl}));
    // workspace growth through grow(): finishes queued work and invalidates captured graphs
    ccr_status st = grow(c, c->ws_part, (size_t)tb * nch * pl.n_f * sizeof(double));
    if (!st) st = grow(c, c->ws_coef, (size_t)tb * std::max(B.n_work, 1) * kCheb * sizeof(double));
    if (st) return st;
    const size_t osz = out_fp64 ? sizeof(double) : sizeof(float);
    const size_t out_bytes = (size_t)B.n_tmpl * pl.n_f * osz;
    void *dst = rho_out;
    if (!out_on_device) {
        if ((st = grow(c, c->ws_out, out_bytes))) return st;
        dst = c->ws_out.p;
    }
    const double factor = pl.norm > 0.0 ? std::sqrt(2.0) / pl.norm : 0.0;
    for (int64_t t = 0; t < B.n_tmpl; t += tb) {
        const int nb = (int)std::min<int64_t>(tb, B.n_tmpl - t);
        const double *dtm = B.d_tmpl.as<double>() + (size_t)t * kTmplStride;
        {
            LaunchTimer lt(c, 5, s);
            HIP_OK(c, launch_timebase(bd, dtm, nb, c->ws_coef.as<double>(), s));
        }
        {
            LaunchTimer lt(c, 4, s);
            HIP_OK(c, launch_fused(bd, c->ws_coef.as<double>(), nb, fp64, c->ws_part.as<double>(), (int)kc, nch, S, s));
        }
        {
            LaunchTimer lt(c, 3, s);
            HIP_OK(c, launch_finish(bd, nb, c->ws_part.as<double>(), nch, factor,
                                    static_cast<char *>(dst) + (size_t)t * pl.n_f * osz, out_fp64 != 0, s));
        }
    }
    if (!out_on_device) {
        HIP_OK(c, hipMemcpyAsync(rho_out, dst, out_bytes, hipMemcpyDeviceToHost, s));
        HIP_OK(c, hipStreamSynchronize(s));
    }
    return CCR_OK;
}


// ------------------------------------------------------------------ batched execution
//
// One ccr_compute_rho call becomes a list of work items (runs of consecutive templates of one
// band), grouped by kernel variant and packed into rounds that fit the workspace.  Each round
// is one launch per stage (time base, resampling, spectra [+ pair sum], [pair sum,] finish)
// covering every item of the round, whatever band it belongs to.

// Kernel variant shared by the items of one round.
struct Variant {
    bool sp = false;     // spectra + pair sum in one kernel
    bool reg16 = false;  // otherwise: 256-point register FFT (else the LDS Stockham FFT on n_s points)
    bool z4 = false;     // spectra + pair sum: N_K <= 192 (4 of the 16 FFT input rows are zero)
    bool ss = false;     // time base with the short small-angle series
    bool far = false;    // split-precision resampling in Farrow form
    bool wide = false;   // spectra + pair sum in one kernel, 1024-point segments
    bool wallp = false;  // wide: every ordered pair (stream-sum partials)
    bool wps = false;    // wide: two spectra streams per segment (per-sample antenna functions)
    int wns = 0;         // wide: segment FFT length (256, 512 or 1024)
    int DT = 0, window = 0, n_s = 0, nr = 0, n_cheb = kCheb;
    int wcols = 0, wqm = 0, wts = 0, wwv = 0;  // wide: bins of a class per lane, detector count,
                                               // segments a step, wavefronts a workgroup
    bool operator==(const Variant &o) const {
        return sp == o.sp && reg16 == o.reg16 && z4 == o.z4 && ss == o.ss && far == o.far && wide == o.wide &&
               DT == o.DT && window == o.window && n_s == o.n_s && nr == o.nr && n_cheb == o.n_cheb &&
               wcols == o.wcols && wqm == o.wqm && wts == o.wts && wwv == o.wwv && wallp == o.wallp && wns == o.wns && wps == o.wps;
    }
};

// Workspace of one launch round, laid out in the arena: time-base coefficients, resampled series
// (with a tail pad of 256 complex FP64 samples: the spectra kernels read whole 256-sample rows
// of the last segment), segment spectra (general path), chunk partials; 256-byte aligned.
constexpr size_t kArenaAlign = 256;
constexpr size_t kYTailPad = 256 * sizeof(double2);
inline size_t arena_al(size_t v) { return (v + kArenaAlign - 1) & ~(kArenaAlign - 1); }
inline size_t arena_bytes_of(size_t coef, size_t y, size_t F, size_t part) {
    return arena_al(coef) + arena_al(y + kYTailPad) + arena_al(F) + arena_al(part);
}

struct Round {
    int i0 = 0, n = 0;  // items [i0, i0 + n) of the call's item table
    int64_t n_tmpl = 0;  // templates of those items
    Variant v;
    size_t lds = 0;     // dynamic LDS of the spectra + pair-sum kernel
    int64_t blocks[kStages] = {0, 0, 0, 0, 0};
    size_t y_bytes = 0, F_bytes = 0, part_bytes = 0, coef_bytes = 0;
    size_t arena() const { return arena_bytes_of(coef_bytes, y_bytes, F_bytes, part_bytes); }
};

struct CallPlan {
    std::vector<BandDev> bands;  // by position in the call
    std::vector<WorkItem> items;
    std::vector<Round> rounds;
    size_t arena_bytes = 0;       // largest round's workspace (rounds run in turn and share the arena)
    std::vector<size_t> out_off;  // host outputs: byte offset of each band's rho in ws_out
    size_t out_bytes = 0;
};

// Launch shape parameters (0 = default): templates per item and segments per pair-sum chunk.
struct BatchParams {
    int64_t template_batch = 0, k_chunk = 0;
    int64_t round_templates = 0;  // at most this many templates in one launch round (0: no limit)
    int64_t max_templates = 0;    // tuning: only the first this many templates of each band (0: all)
    bool no_streams = false;      // per-sample antenna functions stay on the general path
    int spectra = 0;  // 1: the wide spectra + pair-sum kernel wherever it applies, 0: the 256-point one first
};

Variant variant_of(const BandDev &bd, bool fp64, bool short_series, bool farrow, bool prefer_wide,
                   bool streams = true) {
    Variant v;
    v.ss = short_series;
    v.far = farrow && !fp64 && bd.farrow != nullptr;
    // the spectra + pair-sum kernels take the Gamma^ave weight over lagged pairs with per-segment
    // weights; the other forms run on the general path
    // the 256-point spectra + pair-sum kernel takes the Gamma^ave weight over lagged pairs with
    // per-segment weights, the 1024-point one either weight and every ordered pair as well; the
    // other forms (per-sample antenna functions: two spectra streams) run on the general path
    const bool plain = bd.weight == CCR_WEIGHT_AVE && !bd.allp && bd.pw == nullptr;
    // per-sample antenna functions: the wide kernel's two streams, written by the Farrow resampler
    BandDev bw = bd;
    bw.ps2 = bd.pw != nullptr ? 1 : 0;
    const bool wide_ok = (bd.pw == nullptr || (streams && v.far && bd.pwf != nullptr)) && spectra_wide_ok(bw, fp64, kMaxLds);
    v.sp = plain && spectra_pairs_ok(bd, fp64, kMaxLds) && !(prefer_wide && wide_ok);
    v.wide = !v.sp && wide_ok;
    v.wallp = v.wide && bd.allp;
    v.wps = v.wide && bd.pw != nullptr;
    v.DT = bd.D == 8 ? 8 : 0;
    v.window = bd.window;
    v.n_cheb = fp64 ? kCheb : bd.cheb_split;
    if (v.wide) {
        v.wns = bd.n_s;
        v.wcols = spectra_wide_cols(bd);
        v.wqm = bd.Q;
        v.wts = spectra_wide_segs(bw);
        v.wwv = spectra_wide_waves(bw);
    } else if (v.sp) {
        v.nr = spectra_pairs_rounds(bd);
        v.z4 = bd.n_k <= 192;
    } else {
        v.reg16 = !fp64 && bd.n_s == 256 && bd.bins_unique && bd.pw == nullptr;
        if (!v.reg16) v.n_s = bd.n_s;
    }
    return v;
}

constexpr int64_t kMaxBlocks = ((int64_t)1 << 31) - 1;

// Largest grid of a stage's kernel: at most 2^31 - 1 workgroups and 2^32 - 1 work-items.
int64_t stage_max_blocks(const Variant &v, int st) {
    int threads = 64;
    if (st == kStTimebase) threads = tb_entries(v.n_cheb) * v.n_cheb;
    else if (st == kStResample) threads = v.far ? 256 : 64;
    else if (st == kStSpectra) threads = v.sp ? 64 : (v.wide ? 64 * v.wwv : (v.reg16 ? 128 : spectra_threads(v.n_s)));
    else if (st == kStPairs) threads = kPairsThreads;
    else if (st == kStFinish) threads = kFinishThreads;
    return std::min<int64_t>(kMaxBlocks, (((int64_t)1 << 32) - 1) / threads);
}

// Grow a workspace buffer; device work that may still use the old allocation is finished
// first, and captured launch sequences that refer to it are invalidated.
ccr_status grow(ccr_ctx *c, DevBuf &b, size_t bytes) {
    if (bytes <= b.bytes && b.p) return CCR_OK;
    HIP_OK(c, hipDeviceSynchronize());
    HIP_OK(c, b.ensure(bytes));
    c->gen++;
    return CCR_OK;
}

// budget_override > 0: pack rounds to that many workspace bytes instead of the context's budget.
ccr_status build_plan(ccr_ctx *c, bool fp64, int n_bands, const int *band_ids, void *const *rho_out,
                      int out_on_device, int out_fp64, const BatchParams &bp, CallPlan &cp, size_t budget_override = 0) {
    const size_t cs = fp64 ? 16 : 8;
    const size_t osz = out_fp64 ? sizeof(double) : sizeof(float);
    if (budget_override == 0 && c->opt_workspace_mb == 0 && c->auto_budget == 0) {
        // 3/4 of the free device memory plus the workspace the context already holds
        size_t fr = 0, tot = 0;
        HIP_OK(c, hipMemGetInfo(&fr, &tot));
        const size_t held = c->ws_arena.bytes + c->ws_part.bytes + c->ws_coef.bytes;
        c->auto_budget = std::max<size_t>((fr + held) / 4 * 3, (size_t)64 << 20);
    }
    const size_t budget = budget_override > 0          ? budget_override
                          : c->opt_workspace_mb > 0 ? (size_t)c->opt_workspace_mb << 20
                                                    : c->auto_budget;
    cp = CallPlan();
    cp.out_off.assign((size_t)n_bands, 0);
    for (int bi = 0; bi < n_bands; ++bi) {
        const Band &B = *get_band(c, band_ids[bi]);
        cp.out_off[bi] = cp.out_bytes;
        cp.out_bytes += ((size_t)B.n_tmpl * B.plan.n_f * osz + 255) & ~(size_t)255;
    }
    if (!out_on_device) {
        ccr_status st = grow(c, c->ws_out, cp.out_bytes);
        if (st) return st;
    }
    struct Pending {
        WorkItem it;
        Variant v;
        size_t y, F, part, coef, lds;
        int64_t blk[kStages];
    };
    std::vector<Pending> pend;
    std::vector<Variant> variants;
    for (int bi = 0; bi < n_bands; ++bi) {
        const Band &B = *get_band(c, band_ids[bi]);
        const Plan &pl = B.plan;
        BandDev bd = band_dev(B);
        bd.far_stage = (int)c->opt_farrow_stage;
        cp.bands.push_back(bd);
        const Variant v = variant_of(bd, fp64, B.short_series, c->opt_farrow != 0, bp.spectra != 0, !bp.no_streams);
        if (v.wps) cp.bands.back().ps2 = 1;
        const int res_t = v.far ? kFarTemplates : kResTemplates;  // templates per resampler workgroup
        if (std::find(variants.begin(), variants.end(), v) == variants.end()) variants.push_back(v);
        int64_t kc = bp.k_chunk > 0 ? bp.k_chunk : std::min<int64_t>(pl.n_seg, 256);
        kc = std::max<int64_t>(1, std::min<int64_t>(kc, pl.n_seg));
        const int nch = (int)((pl.n_seg + kc - 1) / kc);
        const size_t y1 = (size_t)B.Q * pl.n_seg * pl.n_k * cs * (v.wps ? 2 : 1);
        // two spectra streams per segment with per-sample weights; four partials per bin (the
        // stream sums) for every ordered pair
        const size_t F1 = (v.sp || v.wide) ? 0 : (size_t)B.Q * pl.n_seg * pl.n_f * cs * (bd.pw ? 2 : 1);
        const size_t part1 = (size_t)nch * pl.n_f * sizeof(double) * (bd.allp ? 4 : 1);
        const size_t coef1 = (size_t)std::max(B.n_work, 1) * kCheb * sizeof(double);
        WorkItem proto;
        std::memset(&proto, 0, sizeof proto);
        proto.band = bi;
        proto.k_chunk = (int)kc;
        proto.n_chunks = nch;
        proto.factor = pl.norm > 0.0 ? std::sqrt(2.0) / pl.norm : 0.0;
        proto.out_fp64 = out_fp64 ? 1 : 0;
        proto.gx[kStTimebase] = (B.n_work + tb_entries(v.n_cheb) - 1) / tb_entries(v.n_cheb);
        proto.gx[kStResample] = B.n_work;
        proto.gx[kStSpectra] = v.wide ? nch * (int)pl.P
                               : v.sp ? nch
                                      : (v.reg16 ? (B.n_work + kSpec16Groups - 1) / kSpec16Groups : B.n_work);
        proto.gx[kStPairs] = (v.sp || v.wide) ? 0 : (int)((pl.n_f + kPairsThreads - 1) / kPairsThreads);
        proto.gx[kStFinish] = (int)((pl.n_f + kFinishThreads - 1) / kFinishThreads);
        const int64_t per_t[kStages] = {proto.gx[0], proto.gx[1], proto.gx[2], (int64_t)proto.gx[3] * nch, proto.gx[4]};
        int64_t tb = bp.template_batch > 0 ? bp.template_batch : c->opt_template_batch;
        if (tb <= 0) tb = (int64_t)std::max<size_t>(1, budget / std::max<size_t>(y1 + F1 + part1 + coef1, 1));
        for (int st = 0; st < kStages; ++st) {
            const int64_t mb = stage_max_blocks(v, st) / std::max<int64_t>(per_t[st], 1);
            tb = std::min<int64_t>(tb, st == kStResample ? mb * res_t : mb);
        }
        tb = std::max<int64_t>(1, std::min<int64_t>(tb, B.n_tmpl));
        char *dst = out_on_device ? static_cast<char *>(rho_out[bi]) : c->ws_out.as<char>() + cp.out_off[bi];
        const int64_t n_t = bp.max_templates > 0 ? std::min<int64_t>(B.n_tmpl, bp.max_templates) : B.n_tmpl;
        for (int64_t t = 0; t < n_t; t += tb) {
            Pending q;
            q.it = proto;
            const int nb = (int)std::min<int64_t>(tb, n_t - t);
            q.it.n_tmpl = nb;
            q.it.tmpl_off = t;
            q.it.out = dst + (size_t)t * pl.n_f * osz;
            q.v = v;
            q.y = y1 * nb;
            q.F = F1 * nb;
            q.part = part1 * nb;
            q.coef = coef1 * nb;
            q.lds = v.sp ? spectra_pairs_lds(cp.bands.back()) : (v.wide ? spectra_wide_lds(cp.bands.back()) : 0);
            for (int st = 0; st < kStages; ++st) q.blk[st] = per_t[st] * nb;
            q.blk[kStResample] = per_t[kStResample] * ((nb + res_t - 1) / res_t);
            pend.push_back(q);
        }
    }
    // rounds: items of one variant in call order, packed while the workspace and the grid allow
    for (const Variant &v : variants) {
        Round r;
        auto close = [&]() {
            if (r.n == 0) return;
            cp.rounds.push_back(r);
            cp.arena_bytes = std::max(cp.arena_bytes, r.arena());
        };
        r.v = v;
        r.i0 = (int)cp.items.size();
        for (const Pending &q : pend) {
            if (!(q.v == v)) continue;
            bool full = arena_bytes_of(r.coef_bytes + q.coef, r.y_bytes + q.y, r.F_bytes + q.F, r.part_bytes + q.part) > budget;
            for (int st = 0; st < kStages; ++st) full = full || r.blocks[st] + q.blk[st] > stage_max_blocks(v, st);
            if (c->opt_items_per_launch > 0 && r.n >= c->opt_items_per_launch) full = true;
            if (bp.round_templates > 0 && r.n_tmpl + q.it.n_tmpl > bp.round_templates) full = true;
            if (r.n > 0 && full) {
                close();
                r = Round();
                r.v = v;
                r.i0 = (int)cp.items.size();
            }
            WorkItem it = q.it;
            it.coef_off = (int64_t)(r.coef_bytes / sizeof(double));
            it.y_off = (int64_t)(r.y_bytes / cs);
            it.F_off = (int64_t)(r.F_bytes / cs);
            it.part_off = (int64_t)(r.part_bytes / sizeof(double));
            for (int st = 0; st < kStages; ++st) {
                it.first[st] = (int)r.blocks[st];
                r.blocks[st] += q.blk[st];
            }
            r.y_bytes += q.y;
            r.F_bytes += q.F;
            r.part_bytes += q.part;
            r.coef_bytes += q.coef;
            r.lds = std::max(r.lds, q.lds);
            r.n_tmpl += q.it.n_tmpl;
            r.n++;
            cp.items.push_back(it);
        }
        close();
    }
    return CCR_OK;
}

// The arena holds the largest round of the plan (each round fits the budget on its own); the
// fused path's buffers are released when the arena has to grow, so the two never add up.
ccr_status ensure_workspace(ccr_ctx *c, const CallPlan &cp) {
    if (cp.arena_bytes > c->ws_arena.bytes && (c->ws_part.p || c->ws_coef.p)) {
        HIP_OK(c, hipDeviceSynchronize());
        c->ws_part.release();
        c->ws_coef.release();
        c->gen++;
    }
    if (cp.arena_bytes > c->ws_arena.bytes && c->ws_arena.p) {
        // free the old arena before allocating the larger one
        HIP_OK(c, hipDeviceSynchronize());
        c->ws_arena.release();
        c->gen++;
    }
    return grow(c, c->ws_arena, std::max<size_t>(cp.arena_bytes, kArenaAlign));
}

// Bytes of the device table (band descriptors, then work items, 256-byte aligned).
size_t tables_bytes(const CallPlan &cp, size_t *items_off) {
    *items_off = (cp.bands.size() * sizeof(BandDev) + 255) & ~(size_t)255;
    return *items_off + cp.items.size() * sizeof(WorkItem);
}

void fill_tables(const CallPlan &cp, void *dst, size_t items_off) {
    std::memcpy(dst, cp.bands.data(), cp.bands.size() * sizeof(BandDev));
    std::memcpy(static_cast<char *>(dst) + items_off, cp.items.data(), cp.items.size() * sizeof(WorkItem));
}

// Device workspace of a launch sequence: time-base coefficients, resampled series, segment
// spectra (general path) and chunk partials.
struct Workspace {
    double *coef = nullptr;
    void *y = nullptr, *F = nullptr;
    double *part = nullptr;
};

// A round's buffers in the arena (layout of arena_bytes_of).
Workspace round_workspace(void *arena, const Round &r) {
    char *a = static_cast<char *>(arena);
    Workspace w;
    w.coef = reinterpret_cast<double *>(a);
    a += arena_al(r.coef_bytes);
    w.y = a;
    a += arena_al(r.y_bytes + kYTailPad);
    w.F = a;
    a += arena_al(r.F_bytes);
    w.part = reinterpret_cast<double *>(a);
    return w;
}

// Queue the rounds [r0, r1) of a plan on `s` (tables already on the device; each round's
// workspace at the start of `arena`).
ccr_status run_rounds(ccr_ctx *c, const CallPlan &cp, size_t r0, size_t r1, bool fp64, const void *d_tables,
                      size_t items_off, hipStream_t s, bool timing, void *arena) {
    const BandDev *db = static_cast<const BandDev *>(d_tables);
    const WorkItem *ditems = reinterpret_cast<const WorkItem *>(static_cast<const char *>(d_tables) + items_off);
    for (size_t ri = r0; ri < r1; ++ri) {
        const Round &r = cp.rounds[ri];
        const Workspace ws = round_workspace(arena, r);
        double *coef = ws.coef, *part = ws.part;
        const WorkItem *di = ditems + r.i0;
        {
            LaunchTimer lt(c, 5, s, timing);
            HIP_OK(c, launch_timebase_m(db, di, r.n, (int)r.blocks[kStTimebase], r.v.n_cheb, r.v.ss, coef, s));
        }
        {
            LaunchTimer lt(c, 0, s, timing);
            HIP_OK(c, launch_resample_m(db, di, r.n, (int)r.blocks[kStResample], fp64, r.v.DT, r.v.window,
                                        r.v.n_cheb, r.v.far, coef, ws.y, s));
        }
        if (r.v.sp) {
            LaunchTimer lt(c, 6, s, timing);
            HIP_OK(c, launch_spectra_pairs_m(db, di, r.n, (int)r.blocks[kStSpectra], r.v.nr, r.v.z4, r.lds, ws.y, part, s));
        } else if (r.v.wide) {
            LaunchTimer lt(c, 7, s, timing);
            HIP_OK(c, launch_spectra_wide_m(db, di, r.n, (int)r.blocks[kStSpectra], r.v.wns, r.v.wcols, r.v.wqm, r.v.wts, r.v.wwv,
                                            r.v.wallp, r.v.wps, r.lds, ws.y, part, s));
        } else {
            {
                LaunchTimer lt(c, 1, s, timing);
                HIP_OK(c, launch_spectra_m(db, di, r.n, (int)r.blocks[kStSpectra], fp64, r.v.reg16,
                                           spectra_threads(r.v.n_s), r.v.n_s, ws.y, ws.F, s));
            }
            {
                LaunchTimer lt(c, 2, s, timing);
                HIP_OK(c, launch_pairs_m(db, di, r.n, (int)r.blocks[kStPairs], fp64, ws.F, part, s));
            }
        }
        {
            LaunchTimer lt(c, 3, s, timing);
            HIP_OK(c, launch_finish_m(db, di, r.n, (int)r.blocks[kStFinish], part, s));
        }
    }
    return CCR_OK;
}

// Eager upload of a plan's tables through the pinned staging buffer (stream ordered).
ccr_status upload_tables(ccr_ctx *c, const CallPlan &cp, hipStream_t s, size_t *items_off) {
    const size_t bytes = tables_bytes(cp, items_off);
    if (c->tables_copied) HIP_OK(c, hipEventSynchronize(c->tables_copied));
    else HIP_OK(c, hipEventCreateWithFlags(&c->tables_copied, hipEventDisableTiming));
    if (c->h_tables_bytes < bytes) {
        if (c->h_tables) HIP_OK(c, hipHostFree(c->h_tables));
        c->h_tables = nullptr;
        c->h_tables_bytes = 0;
        HIP_OK(c, hipHostMalloc(&c->h_tables, bytes));
        c->h_tables_bytes = bytes;
    }
    fill_tables(cp, c->h_tables, *items_off);
    ccr_status st = grow(c, c->d_tables, bytes);
    if (st) return st;
    HIP_OK(c, hipMemcpyAsync(c->d_tables.p, c->h_tables, bytes, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipEventRecord(c->tables_copied, s));
    return CCR_OK;
}


// Launch shapes for a call: the tuned ones when autotuning is on.  Tuning on first use for a
// band list and precision times the call for each candidate and keeps the fastest per template:
//   1. the spectra kernel (where a band can take both the 256-point and the wide spectra +
//      pair-sum kernel) and k_chunk = 32 ... 1024, on the first (at most) 64 templates of
//      every band, in rounds of at most 64 templates;
//   2. the templates per launch round: the workspace budget's batch (the largest) and its half
//      and quarter, when the whole call is cheap enough to time (the estimate from step 1 for
//      all candidates below about 12 s).
ccr_status choose_params(ccr_ctx *c, ccr_precision prec, int n_bands, const int *band_ids, void *const *rho_out,
                         int out_on_device, int out_fp64, hipStream_t s, BatchParams &bp) {
    bp = BatchParams();
    bp.k_chunk = c->opt_k_chunk;
    bp.template_batch = c->opt_template_batch;
    bp.round_templates = c->opt_round_templates;
    bp.spectra = (int)c->opt_spectra_kernel;
    if (!c->opt_autotune || c->opt_k_chunk > 0) return CCR_OK;
    const std::vector<int> ids(band_ids, band_ids + n_bands);
    for (const auto &t : c->tuned)
        if (t.band_ids == ids && t.prec == (int)prec) {
            bp.k_chunk = t.k_chunk;
            bp.template_batch = t.template_batch;
            bp.round_templates = t.round_templates;
            bp.spectra = t.spectra;
            return CCR_OK;
        }
    int64_t max_seg = 1;
    bool both = false;  // some band can take either spectra kernel
    const bool fp64 = prec == CCR_PREC_FP64;
    for (int bi = 0; bi < n_bands; ++bi) {
        const Band &B = *get_band(c, band_ids[bi]);
        max_seg = std::max<int64_t>(max_seg, B.plan.n_seg);
        const BandDev bd = band_dev(B);
        const Variant v0 = variant_of(bd, fp64, B.short_series, c->opt_farrow != 0, false);
        const Variant v1 = variant_of(bd, fp64, B.short_series, c->opt_farrow != 0, true);
        both = both || !(v0 == v1);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(c, hipEventCreate(&e0));
    HIP_OK(c, hipEventCreate(&e1));
    // per-template time of a candidate over every round of its plan (one untimed pass, then a
    // timed one), so that calls over several bands compare like with like; n_round: templates
    auto trial = [&](const BatchParams &cand, float &per, int64_t &n_round) -> ccr_status {
        CallPlan cp;
        size_t items_off = 0;
        ccr_status st;
        if ((st = build_plan(c, fp64, n_bands, band_ids, rho_out, out_on_device, out_fp64, cand, cp))) return st;
        if ((st = ensure_workspace(c, cp))) return st;
        if ((st = upload_tables(c, cp, s, &items_off))) return st;
        // an untimed pass first, unless the plan has enough rounds to warm up within the timed one
        const int first = cp.rounds.size() >= 4 ? 1 : 0;
        for (int rep = first; rep < 2; ++rep) {
            if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) return fail(c, CCR_EDEVICE, "event record failed");
            if ((st = run_rounds(c, cp, 0, cp.rounds.size(), fp64, c->d_tables.p, items_off, s, false,
                                 c->ws_arena.p)))
                return st;
        }
        HIP_OK(c, hipEventRecord(e1, s));
        HIP_OK(c, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_OK(c, hipEventElapsedTime(&ms, e0, e1));
        n_round = 0;
        for (const WorkItem &it : cp.items) n_round += it.n_tmpl;
        per = ms / (float)std::max<int64_t>(n_round, 1);
        return CCR_OK;
    };
    ccr_status st = CCR_OK;
    // the workspace budget's template batch: templates of the first item of an untuned plan
    int64_t t_auto = 1;
    {
        CallPlan cp;
        if ((st = build_plan(c, fp64, n_bands, band_ids, rho_out, out_on_device, out_fp64, bp, cp))) goto done;
        if (!cp.items.empty()) t_auto = cp.items[0].n_tmpl;
    }
    {
        const int64_t t_tune = bp.template_batch > 0 ? bp.template_batch : std::min<int64_t>(t_auto, 64);
        float best = -1.0f, best_round_ms = 0.0f;
        BatchParams bestp = bp;
        for (int sk = both ? 0 : bp.spectra; sk <= (both ? 1 : bp.spectra); ++sk)
            for (int64_t kc = 32; kc <= 1024; kc *= 2) {
                if (kc > 2 * max_seg && kc > 32) break;
                BatchParams cand = bp;
                cand.k_chunk = kc;
                cand.spectra = sk;
                cand.template_batch = t_tune;
                cand.round_templates = t_tune;
                cand.max_templates = t_tune;
                float per = 0.0f;
                int64_t nr = 0;
                if ((st = trial(cand, per, nr))) goto done;
                if (best < 0.0f || per < best) {
                    best = per;
                    bestp = cand;
                    best_round_ms = per * (float)nr;
                }
            }
        if (bp.template_batch <= 0 && t_auto > t_tune) {
            // larger batches, if timing them stays cheap (the round time scales with the batch)
            const float est_ms = best_round_ms * (float)t_auto / (float)t_tune;
            if (est_ms * 2.0f * 1.75f < 12000.0f) {
                for (int64_t tb = t_auto; tb > t_tune; tb /= 2) {
                    BatchParams cand = bestp;
                    cand.template_batch = tb;
                    cand.round_templates = tb < t_auto ? tb : 0;
                    cand.max_templates = 0;
                    float per = 0.0f;
                    int64_t nr = 0;
                    if ((st = trial(cand, per, nr))) goto done;
                    if (per < best) {
                        best = per;
                        bestp = cand;
                    }
                    if (tb <= t_auto / 4) break;
                }
            } else {
                bestp.template_batch = t_auto;  // too costly to time: the largest batch
                bestp.round_templates = 0;
            }
        } else if (bp.template_batch <= 0) {
            bestp.template_batch = t_auto;
            bestp.round_templates = 0;
        } else {
            bestp.template_batch = bp.template_batch;  // the caller's batch and round limit
            bestp.round_templates = bp.round_templates;
        }
        bestp.max_templates = 0;  // the call itself covers every template
        bp = bestp;
    }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    c->tuned.push_back({ids, (int)prec, bp.k_chunk, bp.template_batch, bp.round_templates, bp.spectra});
    c->last_tuned_k_chunk = bp.k_chunk;
    c->last_tuned_template_batch = bp.template_batch;
    c->last_tuned_spectra = bp.spectra;
    c->last_tuned_round_templates = bp.round_templates;
    return CCR_OK;
}

ccr_status compute_batched(ccr_ctx *c, ccr_precision prec, int n_bands, const int *band_ids, void *const *rho_out,
                           int out_on_device, int out_fp64, hipStream_t s) {
    const bool fp64 = prec == CCR_PREC_FP64;
    ccr_status st;
    BatchParams bp;
    if ((st = choose_params(c, prec, n_bands, band_ids, rho_out, out_on_device, out_fp64, s, bp))) return st;
    const bool graph = c->opt_graph && out_on_device;
    if (graph) {
        const std::vector<int> ids(band_ids, band_ids + n_bands);
        const std::vector<void *> outs(rho_out, rho_out + n_bands);
        for (auto &g : c->graphs)
            if (g->band_ids == ids && g->outs == outs && g->prec == (int)prec && g->out_fp64 == out_fp64 &&
                g->gen == c->gen) {
                HIP_OK(c, hipGraphLaunch(g->exec, s));
                return CCR_OK;
            }
    }
    CallPlan cp;
    if ((st = build_plan(c, fp64, n_bands, band_ids, rho_out, out_on_device, out_fp64, bp, cp))) return st;
    if ((st = ensure_workspace(c, cp))) return st;
    if (graph) {
        // capture on the context's own stream (the caller's may be the null stream), replay on `s`
        auto g = std::make_unique<ccr_ctx::GraphEntry>();
        g->band_ids.assign(band_ids, band_ids + n_bands);
        g->outs.assign(rho_out, rho_out + n_bands);
        g->prec = (int)prec;
        g->out_fp64 = out_fp64;
        size_t items_off = 0;
        const size_t bytes = tables_bytes(cp, &items_off);
        std::vector<char> host(bytes);
        fill_tables(cp, host.data(), items_off);
        HIP_OK(c, hipMalloc(&g->tables, bytes));
        HIP_OK(c, hipMemcpy(g->tables, host.data(), bytes, hipMemcpyHostToDevice));
        HIP_OK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        st = run_rounds(c, cp, 0, cp.rounds.size(), fp64, g->tables, items_off, c->stream, false, c->ws_arena.p);
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(c->stream, &gr);
        if (st) {
            if (gr) (void)hipGraphDestroy(gr);
            return st;
        }
        if (ec != hipSuccess) return fail(c, CCR_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        g->graph = gr;
        HIP_OK(c, hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        g->gen = c->gen;
        HIP_OK(c, hipGraphLaunch(g->exec, s));
        // keep a handful of graphs; the oldest go first
        if (c->graphs.size() >= 16) {
            HIP_OK(c, hipDeviceSynchronize());
            c->graphs.erase(c->graphs.begin());
        }
        c->graphs.push_back(std::move(g));
        return CCR_OK;
    }
    size_t items_off = 0;
    if ((st = upload_tables(c, cp, s, &items_off))) return st;
    if ((st = run_rounds(c, cp, 0, cp.rounds.size(), fp64, c->d_tables.p, items_off, s, true, c->ws_arena.p)))
        return st;
    if (!out_on_device) {
        for (int bi = 0; bi < n_bands; ++bi) {
            const Band &B = *get_band(c, band_ids[bi]);
            const size_t bytes = (size_t)B.n_tmpl * B.plan.n_f * (out_fp64 ? sizeof(double) : sizeof(float));
            HIP_OK(c, hipMemcpyAsync(rho_out[bi], c->ws_out.as<char>() + cp.out_off[bi], bytes, hipMemcpyDeviceToHost, s));
        }
        HIP_OK(c, hipStreamSynchronize(s));
    }
    return CCR_OK;
}

}  // namespace

// ====================================================================== ABI

// Time base and resampled series of one template as the split-precision compute path makes
// them: the band's node rule and small-angle series (cheb_split, short_series) and the
// Farrow-form resampler where the band has its table, through the batched launchers on a plan
// of one-template rounds.  The series, [Q][n_seg n_k] complex64, is left in the workspace
// arena (*y_dev) until the next compute call.
static ccr_status split_series_of(ccr_ctx *c, int band_id, int64_t template_index, hipStream_t s, const void **y_dev) {
    BatchParams bp;
    bp.template_batch = 1;
    bp.round_templates = 1;
    bp.k_chunk = get_band(c, band_id)->plan.n_seg;  // one chunk: no partial sums to hold
    bp.no_streams = true;                            // the series itself, not its weighted streams
    CallPlan cp;
    void *none = nullptr;
    ccr_status st = build_plan(c, false, 1, &band_id, &none, 1, 0, bp, cp);
    if (st) return st;
    if ((size_t)template_index >= cp.rounds.size()) return fail(c, CCR_EINVAL, "template index out of range");
    if ((st = ensure_workspace(c, cp))) return st;
    size_t items_off = 0;
    if ((st = upload_tables(c, cp, s, &items_off))) return st;
    const Round &r = cp.rounds[(size_t)template_index];
    const Workspace ws = round_workspace(c->ws_arena.p, r);
    const BandDev *db = static_cast<const BandDev *>(c->d_tables.p);
    const WorkItem *di = reinterpret_cast<const WorkItem *>(static_cast<const char *>(c->d_tables.p) + items_off) + r.i0;
    // segments without a spectrum are not resampled: zero first, as the stage output shows them
    HIP_OK(c, launch_zero(ws.y, r.y_bytes, s));
    HIP_OK(c, launch_timebase_m(db, di, r.n, (int)r.blocks[kStTimebase], r.v.n_cheb, r.v.ss, ws.coef, s));
    HIP_OK(c, launch_resample_m(db, di, r.n, (int)r.blocks[kStResample], false, r.v.DT, r.v.window, r.v.n_cheb,
                                r.v.far, ws.coef, ws.y, s));
    *y_dev = ws.y;
    return CCR_OK;
}

extern "C" {

int ccr_abi_version(void) { return CCR_ABI_VERSION; }

ccr_status ccr_create(ccr_ctx **out, int hip_device, const ccr_sky *sky) {
    if (!out || !sky) return CCR_EINVAL;
    *out = nullptr;
    const double *sv = &sky->ra;
    if (!finite_all(sv, sizeof(ccr_sky) / sizeof(double))) return CCR_EINVAL;
    if (!(sky->year_s > 0) || !(sky->sidereal_day_s > 0) || sky->au_s < 0 || sky->re_s < 0) return CCR_EINVAL;
    if (hip_device == -1) {  // host-only context
        ccr_ctx *h = new (std::nothrow) ccr_ctx();
        if (!h) return CCR_ENOMEM;
        h->device = -1;
        h->sky = *sky;
        *out = h;
        return CCR_OK;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return CCR_EDEVICE;
    if (hip_device < 0 || hip_device >= ndev) return CCR_EINVAL;
    if (hipSetDevice(hip_device) != hipSuccess) return CCR_EDEVICE;
    ccr_ctx *c = new (std::nothrow) ccr_ctx();
    if (!c) return CCR_ENOMEM;
    c->device = hip_device;
    c->sky = *sky;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return CCR_EDEVICE;
    }
    // set-up of the no-allocation entry point: the device address of the fixed scratch on this
    // device (looked up once per device), its host staging and event
    if (scratch_init(hip_device) != hipSuccess || hipEventCreateWithFlags(&c->na_copied, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(c->stream);
        delete c;
        return CCR_EDEVICE;
    }
    try {
        c->na_host.assign(kNoAllocTableBytes, 0);
    } catch (const std::bad_alloc &) {
        (void)hipEventDestroy(c->na_copied);
        (void)hipStreamDestroy(c->stream);
        delete c;
        return CCR_ENOMEM;
    }
    *out = c;
    return CCR_OK;
}

void ccr_destroy(ccr_ctx *c) {
    if (!c) return;
    if (c->device < 0) {
        delete c;
        return;
    }
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    collect_times(c);
    c->bands.clear();
    c->ws_arena.release();
    c->ws_part.release();
    c->ws_out.release();
    c->ws_coef.release();
    c->graphs.clear();
    c->d_tables.release();
    if (c->h_tables) (void)hipHostFree(c->h_tables);
    if (c->tables_copied) (void)hipEventDestroy(c->tables_copied);
    if (c->na_copied) (void)hipEventDestroy(c->na_copied);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *ccr_last_error(const ccr_ctx *c) { return c ? c->err.c_str() : "null context"; }

ccr_status ccr_set_option(ccr_ctx *c, const char *name, int64_t value) {
    if (!c || !name) return CCR_EINVAL;
    c->err.clear();
    std::string k(name);
    if (value < 0) return fail(c, CCR_EINVAL, "negative option value");
    if (k == "template_batch") c->opt_template_batch = value;
    else if (k == "workspace_mb") c->opt_workspace_mb = value == 0 ? 0 : std::max<int64_t>(value, 64);
    else if (k == "k_chunk") c->opt_k_chunk = value;
    else if (k == "spectra_kernel") c->opt_spectra_kernel = value ? 1 : 0;
    else if (k == "round_templates") c->opt_round_templates = value;
    else if (k == "fused") c->opt_fused = value;
    else if (k == "timing") c->opt_timing = value;
    else if (k == "graph") c->opt_graph = value;
    else if (k == "autotune") c->opt_autotune = value;
    else if (k == "items_per_launch") c->opt_items_per_launch = value;
    else if (k == "farrow") c->opt_farrow = value ? 1 : 0;
    else if (k == "farrow_stage") c->opt_farrow_stage = value ? 1 : 0;
    else return fail(c, CCR_EUNSUP, "unknown option '%s'", name);
    if (k == "template_batch" || k == "workspace_mb" || k == "k_chunk" || k == "items_per_launch" || k == "farrow" ||
        k == "farrow_stage" || k == "fused" || k == "spectra_kernel" || k == "round_templates")
        c->gen++;
    return CCR_OK;
}

ccr_status ccr_get_option(ccr_ctx *c, const char *name, int64_t *value) {
    if (!c || !name || !value) return CCR_EINVAL;
    c->err.clear();
    std::string k(name);
    if (k == "template_batch") *value = c->opt_template_batch;
    else if (k == "workspace_mb") *value = c->opt_workspace_mb;
    else if (k == "k_chunk") *value = c->opt_k_chunk;
    else if (k == "fused") *value = c->opt_fused;
    else if (k == "timing") *value = c->opt_timing;
    else if (k == "graph") *value = c->opt_graph;
    else if (k == "autotune") *value = c->opt_autotune;
    else if (k == "items_per_launch") *value = c->opt_items_per_launch;
    else if (k == "tuned_k_chunk") *value = c->last_tuned_k_chunk;
    else if (k == "tuned_template_batch") *value = c->last_tuned_template_batch;
    else if (k == "tuned_spectra_kernel") *value = c->last_tuned_spectra;
    else if (k == "spectra_kernel") *value = c->opt_spectra_kernel;
    else if (k == "round_templates") *value = c->opt_round_templates;
    else if (k == "tuned_round_templates") *value = c->last_tuned_round_templates;
    else if (k == "resample_templates") *value = kResTemplates;
    else if (k == "farrow") *value = c->opt_farrow;
    else if (k == "farrow_stage") *value = c->opt_farrow_stage;
    else if (k == "farrow_templates") *value = kFarTemplates;
    else if (k == "farrow_degree") *value = kFarDeg;
    else return fail(c, CCR_EUNSUP, "unknown option '%s'", name);
    return CCR_OK;
}

ccr_status ccr_add_band(ccr_ctx *c, const ccr_band *band, int *band_id, ccr_band_info *info) {
    if (!c || !band || !band_id) return c ? fail(c, CCR_EINVAL, "null argument") : CCR_EINVAL;
    c->err.clear();
    const ccr_band &b = *band;
    const double dv[] = {b.f_min, b.f_band, b.t_short, b.mu_f, b.a_p_max, b.orbit_period};
    if (!finite_all(dv, 6)) return fail(c, CCR_EINVAL, "non-finite band field");
    if (!(b.f_band > 0) || !(b.t_short > 0) || !(b.mu_f > 0) || !(b.orbit_period > 0) || b.a_p_max < 0 ||
        b.f_min < 0)
        return fail(c, CCR_EINVAL, "band fields out of range");
    if (b.dirichlet_D < 1 || b.dirichlet_D > 64) return fail(c, CCR_ERANGE, "dirichlet_D must be 1..64");
    if (b.max_lag < 0 || b.max_lag > 1024) return fail(c, CCR_ERANGE, "max_lag must be 0..1024");
    if (b.window != 0 && b.window != 1) return fail(c, CCR_EINVAL, "window must be 0 or 1");
    if (b.pairs != CCR_PAIRS_ALL && ((b.pairs & 3) == 0 || (b.pairs & ~3)))
        return fail(c, CCR_EINVAL, "pairs must be a nonzero mask of CROSS|SAME, or ALL");
    if (b.weight != CCR_WEIGHT_AVE && b.weight != CCR_WEIGHT_CIRC) return fail(c, CCR_EINVAL, "weight must be AVE or CIRC");
    if (b.n_fft_override < 0) return fail(c, CCR_EINVAL, "negative n_fft_override");
    try {
        auto B = std::make_unique<Band>();
        B->p = b;
        B->df_load = load_bandwidth(b);
        B->n_k_min = (int64_t)std::ceil(b.t_short * B->df_load);
        if (info) {
            std::memset(info, 0, sizeof *info);
            info->n_k = B->n_k_min;
            info->dt = b.t_short / (double)B->n_k_min;
            info->f_het = b.f_min + 0.5 * b.f_band;
            info->df_load = B->df_load;
        }
        c->bands.push_back(std::move(B));
        *band_id = (int)c->bands.size() - 1;
    } catch (const std::bad_alloc &) {
        return fail(c, CCR_ENOMEM, "out of host memory");
    }
    return CCR_OK;
}

ccr_status ccr_set_data(ccr_ctx *c, int band_id, int det, const ccr_site *site, double t0, double dt,
                        int64_t n, double f_het, const float *x, const uint8_t *valid) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_id);
    if (det < 0 || det >= CCR_MAX_DET) return fail(c, CCR_EINVAL, "detector index %d out of range", det);
    if (!site || !x) return fail(c, CCR_EINVAL, "null site or data");
    if (!std::isfinite(site->lat) || !std::isfinite(site->lon) || !std::isfinite(t0) || !std::isfinite(dt) ||
        !std::isfinite(f_het))
        return fail(c, CCR_EINVAL, "non-finite scalar argument");
    if (!(dt > 0)) return fail(c, CCR_EINVAL, "dt must be positive");
    const double ratio = B->p.t_short / dt;
    const int64_t nk = llround(ratio);
    if (nk < 1 || std::fabs(ratio - (double)nk) > 1e-9 * ratio)
        return fail(c, CCR_EINVAL, "t_short / dt = %.12g is not an integer", ratio);
    if ((double)nk < B->p.t_short * B->df_load * (1.0 - 1e-12))
        return fail(c, CCR_ERANGE, "dt undersamples the load band (%lld < %.6g samples per segment)",
                    (long long)nk, B->p.t_short * B->df_load);
    const double fh = B->p.f_min + 0.5 * B->p.f_band;
    if (std::fabs(f_het - fh) > 1e-9 * std::fabs(fh) + 1e-12)
        return fail(c, CCR_EINVAL, "f_het %.12g differs from f_min + f_band / 2 = %.12g", f_het, fh);
    if (n < nk) return fail(c, CCR_EINVAL, "fewer than one segment of samples");
    if (n > (int64_t)1 << 34) return fail(c, CCR_ERANGE, "series too long");
    for (int X = 0; X < CCR_MAX_DET; ++X) {
        if (X == det || !B->det[X].has_data) continue;
        if (B->det[X].t0 != t0 || B->det[X].dt != dt)
            return fail(c, CCR_EINVAL, "t0/dt differ from detector %d", X);
    }
    for (int64_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(x[i])) return fail(c, CCR_EINVAL, "non-finite sample at %lld", (long long)(i / 2));
    try {
        DetData &d = B->det[det];
        d.x.assign(x, x + 2 * n);
        if (valid) {
            d.valid.assign(valid, valid + n);
            for (int64_t i = 0; i < n; ++i)
                if (!valid[i]) d.x[2 * i] = d.x[2 * i + 1] = 0.0f;
        } else {
            d.valid.clear();
        }
        d.site = *site;
        d.t0 = t0;
        d.dt = dt;
        d.n = n;
        d.f_het = f_het;
        d.has_data = true;
    } catch (const std::bad_alloc &) {
        return fail(c, CCR_ENOMEM, "out of host memory");
    }
    B->prepared = false;
    B->tmpl.clear();
    return CCR_OK;
}

ccr_status ccr_set_weights(ccr_ctx *c, int band_id, int det, int64_t n_seg, const double *a, const double *b,
                           const double *noise_var) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_id);
    if (det < 0 || det >= CCR_MAX_DET) return fail(c, CCR_EINVAL, "detector index %d out of range", det);
    if (!a || !b || !noise_var || n_seg < 1) return fail(c, CCR_EINVAL, "null or empty weights");
    if (!finite_all(a, n_seg) || !finite_all(b, n_seg) || !finite_all(noise_var, n_seg))
        return fail(c, CCR_EINVAL, "non-finite weight");
    for (int64_t k = 0; k < n_seg; ++k)
        if (!(noise_var[k] > 0)) return fail(c, CCR_EINVAL, "noise variance of segment %lld not positive", (long long)k);
    try {
        DetData &d = B->det[det];
        d.a.assign(a, a + n_seg);
        d.b.assign(b, b + n_seg);
        d.nv.assign(noise_var, noise_var + n_seg);
        d.has_weights = true;
    } catch (const std::bad_alloc &) {
        return fail(c, CCR_ENOMEM, "out of host memory");
    }
    B->prepared = false;
    B->tmpl.clear();
    return CCR_OK;
}

ccr_status ccr_set_antenna(ccr_ctx *c, int band_id, int det, int64_t n, const double *a, const double *b) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_id);
    if (det < 0 || det >= CCR_MAX_DET) return fail(c, CCR_EINVAL, "detector index %d out of range", det);
    if (n < 0) return fail(c, CCR_EINVAL, "negative sample count");
    try {
        DetData &d = B->det[det];
        if (n == 0 || !a || !b) {
            d.ar.clear();
            d.br.clear();
        } else {
            if (n > (int64_t)1 << 34) return fail(c, CCR_ERANGE, "series too long");
            if (!finite_all(a, n) || !finite_all(b, n)) return fail(c, CCR_EINVAL, "non-finite antenna function");
            d.ar.assign(a, a + n);
            d.br.assign(b, b + n);
        }
    } catch (const std::bad_alloc &) {
        return fail(c, CCR_ENOMEM, "out of host memory");
    }
    B->prepared = false;
    B->tmpl.clear();
    return CCR_OK;
}

ccr_status ccr_set_templates(ccr_ctx *c, int band_id, int64_t n, const double *a_p, const double *t_asc,
                             const double *period) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_id);
    if (n < 1 || !a_p || !t_asc || !period) return fail(c, CCR_EINVAL, "null or empty template arrays");
    if (!finite_all(a_p, n) || !finite_all(t_asc, n) || !finite_all(period, n))
        return fail(c, CCR_EINVAL, "non-finite template parameter");
    for (int64_t i = 0; i < n; ++i)
        if (a_p[i] < 0 || !(period[i] > 0)) return fail(c, CCR_EINVAL, "template %lld: a_p < 0 or P <= 0", (long long)i);
    try {
        B->tmpl_raw.assign((size_t)n * kRawStride, 0.0);
        for (int64_t i = 0; i < n; ++i) {
            B->tmpl_raw[kRawStride * i] = a_p[i];
            B->tmpl_raw[kRawStride * i + 1] = t_asc[i];
            B->tmpl_raw[kRawStride * i + 2] = period[i];
        }
        B->n_tmpl = n;
        B->ecc = false;
        B->tmpl.clear();
    } catch (const std::bad_alloc &) {
        return fail(c, CCR_ENOMEM, "out of host memory");
    }
    return CCR_OK;
}

ccr_status ccr_set_templates_ecc(ccr_ctx *c, int band_id, int64_t n, const double *a_p, const double *t_p,
                                 const double *omega, const double *e, const double *period) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_id);
    if (n < 1 || !a_p || !t_p || !omega || !e || !period) return fail(c, CCR_EINVAL, "null or empty template arrays");
    if (!finite_all(a_p, n) || !finite_all(t_p, n) || !finite_all(omega, n) || !finite_all(e, n) ||
        !finite_all(period, n))
        return fail(c, CCR_EINVAL, "non-finite template parameter");
    for (int64_t i = 0; i < n; ++i) {
        if (a_p[i] < 0 || !(period[i] > 0)) return fail(c, CCR_EINVAL, "template %lld: a_p < 0 or P <= 0", (long long)i);
        if (e[i] < 0 || e[i] > 0.95) return fail(c, CCR_EINVAL, "template %lld: e outside [0, 0.95]", (long long)i);
    }
    try {
        B->tmpl_raw.assign((size_t)n * kRawStride, 0.0);
        for (int64_t i = 0; i < n; ++i) {
            double *r = &B->tmpl_raw[kRawStride * i];
            r[0] = a_p[i];
            r[1] = t_p[i];
            r[2] = period[i];
            r[3] = e[i];
            r[4] = omega[i];
        }
        B->n_tmpl = n;
        B->ecc = true;
        B->tmpl.clear();
    } catch (const std::bad_alloc &) {
        return fail(c, CCR_ENOMEM, "out of host memory");
    }
    return CCR_OK;
}

ccr_status ccr_get_band_info(ccr_ctx *c, int band_id, ccr_band_info *info, double *bin_freqs) {
    if (!c || !info) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_id);
    if (c->device >= 0) HIP_OK(c, hipSetDevice(c->device));
    // with templates set, the band is prepared completely (device tables and template table;
    // a host-only context checks the templates without building device tables)
    ccr_status st = B->n_tmpl > 0 ? ensure_ready(c, *B) : prepare(c, *B);
    if (st) return st;
    const Plan &pl = B->plan;
    std::memset(info, 0, sizeof *info);
    info->n_k = pl.n_k;
    info->n_seg = pl.n_seg;
    info->n_fft = pl.n_fft;
    info->n_f = pl.n_f;
    info->k_lo = pl.k_lo;
    info->n_pairs = pl.n_pairs;
    info->n_det = B->Q;
    info->n_templates = B->n_tmpl;
    info->n_active = B->n_work;
    info->dt = pl.dt;
    info->f_het = pl.f_het;
    info->df_load = pl.df_load;
    info->t_coh = pl.t_coh;
    info->dlambda_f = pl.dlf;
    info->t_fft = pl.t_fft;
    info->nu_r = pl.nu_r;
    info->norm = pl.norm;
    info->farrow_degree = B->far_len > 0 ? kFarDeg : 0;
    info->farrow_err = B->far_err;
    info->n_s = B->plan.n_s;
    info->P = B->plan.P;
    if (bin_freqs) std::memcpy(bin_freqs, B->freqs.data(), sizeof(double) * (size_t)pl.n_f);
    return CCR_OK;
}

ccr_status ccr_compute_rho(ccr_ctx *c, ccr_precision prec, int n_bands, const int *band_ids, void *const *rho_out,
                           int out_on_device, int out_fp64, void *hip_stream) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    if (n_bands < 1 || !band_ids || !rho_out) return fail(c, CCR_EINVAL, "no bands or outputs");
    if (prec != CCR_PREC_FP64 && prec != CCR_PREC_SPLIT) return fail(c, CCR_EINVAL, "bad precision");
    if (c->device < 0) return fail(c, CCR_EDEVICE, "host-only context");
    HIP_OK(c, hipSetDevice(c->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    const bool fp64 = prec == CCR_PREC_FP64;
    ccr_status st;
    for (int bi = 0; bi < n_bands; ++bi) {
        Band *B = get_band(c, band_ids[bi]);
        if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_ids[bi]);
        if (!rho_out[bi]) return fail(c, CCR_EINVAL, "null output for band %d", band_ids[bi]);
        if ((st = ensure_ready(c, *B))) return st;
    }
    if (c->opt_fused) {
        // optional fused kernel, per band (bands it cannot hold use the batched path below)
        std::vector<int> rest;
        std::vector<void *> rest_out;
        for (int bi = 0; bi < n_bands; ++bi) {
            Band &B = *get_band(c, band_ids[bi]);
            const BandDev bd = band_dev(B);
            const bool plain = bd.weight == CCR_WEIGHT_AVE && !bd.allp && bd.pw == nullptr;
            const int S = plain ? fused_steps(bd, fp64, kMaxLds) : 0;
            if (S > 0) {
                if ((st = compute_fused(c, B, bd, fp64, S, rho_out[bi], out_on_device, out_fp64, s))) return st;
            } else {
                rest.push_back(band_ids[bi]);
                rest_out.push_back(rho_out[bi]);
            }
        }
        if (rest.empty()) return CCR_OK;
        return compute_batched(c, prec, (int)rest.size(), rest.data(), rest_out.data(), out_on_device, out_fp64, s);
    }
    return compute_batched(c, prec, n_bands, band_ids, rho_out, out_on_device, out_fp64, s);
}

ccr_status ccr_compute_rho_noalloc(ccr_ctx *c, ccr_precision prec, int n_bands, const int *band_ids,
                                   void *const *rho_out, int out_fp64, void *hip_stream) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    if (n_bands < 1 || !band_ids || !rho_out) return fail(c, CCR_EINVAL, "no bands or outputs");
    if (prec != CCR_PREC_FP64 && prec != CCR_PREC_SPLIT) return fail(c, CCR_EINVAL, "bad precision");
    if (c->device < 0) return fail(c, CCR_EDEVICE, "host-only context");
    HIP_OK(c, hipSetDevice(c->device));
    void *scr = scratch_device_ptr(c->device);
    if (!scr) return fail(c, CCR_EDEVICE, "no scratch address on device %d", c->device);
    for (int bi = 0; bi < n_bands; ++bi) {
        Band *B = get_band(c, band_ids[bi]);
        if (!B) return fail(c, CCR_EINVAL, "bad band id %d", band_ids[bi]);
        if (!rho_out[bi]) return fail(c, CCR_EINVAL, "null output for band %d", band_ids[bi]);
        // preparing a band allocates its device tables: that is set-up, done by
        // ccr_get_band_info (or ccr_compute_rho) after data, weights and templates are set
        if (!B->prepared || B->n_tmpl == 0 || B->tmpl.empty())
            return fail(c, CCR_ESTATE, "band %d is not prepared: call ccr_get_band_info after setting its data, "
                                       "weights and templates", band_ids[bi]);
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
    const bool fp64 = prec == CCR_PREC_FP64;
    // the scratch holds the band and work-item tables, then the workspace of the largest round
    const size_t tables_cap = arena_al(kNoAllocTableBytes);
    const size_t budget = kScratchBytes - tables_cap;
    BatchParams bp;
    bp.k_chunk = c->opt_k_chunk;
    bp.template_batch = c->opt_template_batch;
    bp.round_templates = c->opt_round_templates;
    bp.spectra = (int)c->opt_spectra_kernel;
    CallPlan cp;
    ccr_status st = build_plan(c, fp64, n_bands, band_ids, rho_out, 1, out_fp64, bp, cp, budget);
    if (st) return st;
    if (cp.arena_bytes > budget)
        return fail(c, CCR_ERANGE, "one template's workspace (%zu MiB) exceeds the fixed scratch of %zu MiB",
                    cp.arena_bytes >> 20, budget >> 20);
    size_t items_off = 0;
    const size_t tbytes = tables_bytes(cp, &items_off);
    if (tbytes > kNoAllocTableBytes)
        return fail(c, CCR_ERANGE, "band and work-item tables (%zu bytes) exceed the fixed %zu", tbytes,
                    (size_t)kNoAllocTableBytes);
    char *base = static_cast<char *>(scr);
    // the previous call's table copy has finished reading the staging before it is rewritten
    HIP_OK(c, hipEventSynchronize(c->na_copied));
    fill_tables(cp, c->na_host.data(), items_off);
    HIP_OK(c, hipMemcpyAsync(base, c->na_host.data(), tbytes, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipEventRecord(c->na_copied, s));
    return run_rounds(c, cp, 0, cp.rounds.size(), fp64, base, items_off, s, false, base + tables_cap);
}

ccr_status ccr_kernel_time(ccr_ctx *c, int kernel, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return CCR_EINVAL;
    if (kernel < 0 || kernel > 8) return fail(c, CCR_EINVAL, "kernel id %d out of range", kernel);
    collect_times(c);
    *ms = c->kt_ms[kernel];
    *launches = c->kt_n[kernel];
    return CCR_OK;
}

ccr_status ccr_reset_kernel_times(ccr_ctx *c) {
    if (!c) return CCR_EINVAL;
    collect_times(c);
    for (int k = 0; k < 9; ++k) {
        c->kt_ms[k] = 0.0;
        c->kt_n[k] = 0;
    }
    return CCR_OK;
}

ccr_status ccr_sync(ccr_ctx *c) {
    if (!c) return CCR_EINVAL;
    if (c->device < 0) return CCR_OK;
    HIP_OK(c, hipSetDevice(c->device));
    HIP_OK(c, hipDeviceSynchronize());
    return CCR_OK;
}

ccr_status ccr_sft_series(ccr_ctx *c, int64_t n_sft, double t_sft, double t0, int64_t n_bins, int64_t k_first,
                          const float *z, const uint8_t *sft_valid, double f_het, int64_t n_out, float *x_out,
                          uint8_t *valid_out) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    if (!z || !x_out) return fail(c, CCR_EINVAL, "null input or output");
    if (n_sft < 1 || n_bins < 1 || n_out < 1) return fail(c, CCR_EINVAL, "empty SFT set");
    if (!std::isfinite(t_sft) || !std::isfinite(t0) || !std::isfinite(f_het) || !(t_sft > 0) || !(f_het > 0))
        return fail(c, CCR_EINVAL, "t_sft, t0 or f_het not finite and positive");
    if (n_out > kSftMaxOut) return fail(c, CCR_ERANGE, "n_out %lld above %d", (long long)n_out, kSftMaxOut);
    if (n_sft > (int64_t)1 << 31 || n_sft * n_out > (int64_t)1 << 34)
        return fail(c, CCR_ERANGE, "too many SFTs for one call");
    if (c->device < 0) return fail(c, CCR_EDEVICE, "host-only context");
    // heterodyne bin, the band of n_out bins around it and the remainder of f_h off the bin grid
    const long double ts = t_sft, fh = f_het;
    const int64_t kh = (int64_t)llroundl(fh * ts);
    const long double nu = fh * ts - (long double)kh;
    const int64_t h = n_out / 2;
    const int64_t off = kh - h - k_first;
    if (off < 0 || off + n_out > n_bins)
        return fail(c, CCR_ERANGE, "the SFTs hold bins %lld..%lld, the band needs %lld..%lld", (long long)k_first,
                    (long long)(k_first + n_bins - 1), (long long)(kh - h), (long long)(kh - h + n_out - 1));
    for (int64_t i = 0; i < 2 * n_sft * n_bins; ++i)
        if (!std::isfinite(z[i])) return fail(c, CCR_EINVAL, "non-finite SFT bin at %lld", (long long)(i / 2));
    HIP_OK(c, hipSetDevice(c->device));
    std::vector<double2> roots((size_t)n_out), ej((size_t)n_out), sk((size_t)n_sft);
    for (int64_t m = 0; m < n_out; ++m) {
        const long double a = 2.0L * kPiL * (long double)m / (long double)n_out;
        roots[(size_t)m] = make_double2((double)cosl(a), (double)sinl(a));
        const long double b = -2.0L * kPiL * nu * (long double)m / (long double)n_out;
        ej[(size_t)m] = make_double2((double)(cosl(b) / ts), (double)(sinl(b) / ts));
    }
    for (int64_t K = 0; K < n_sft; ++K) {
        long double ph = fh * ((long double)t0 + (long double)K * ts);
        ph -= floorl(ph);
        const long double a = -2.0L * kPiL * ph;
        sk[(size_t)K] = make_double2((double)cosl(a), (double)sinl(a));
    }
    DevBuf dz, dx, dr, de, ds, dv;
    const size_t zb = (size_t)n_sft * n_bins * sizeof(float2), xb = (size_t)n_sft * n_out * sizeof(float2);
    HIP_OK(c, dz.ensure(zb));
    HIP_OK(c, dx.ensure(xb));
    ccr_status st;
    if ((st = upload(c, dr, roots)) || (st = upload(c, de, ej)) || (st = upload(c, ds, sk))) return st;
    if (sft_valid) {
        if ((st = upload(c, dv, std::vector<uint8_t>(sft_valid, sft_valid + n_sft)))) return st;
    }
    hipStream_t s = c->stream;
    HIP_OK(c, hipMemcpyAsync(dz.p, z, zb, hipMemcpyHostToDevice, s));
    {
        LaunchTimer lt(c, 8, s);
        HIP_OK(c, launch_sft_series(dz.as<float2>(), n_sft, n_bins, off, (int)n_out, (int)h, dr.as<double2>(),
                                    de.as<double2>(), ds.as<double2>(), sft_valid ? dv.as<uint8_t>() : nullptr,
                                    dx.as<float2>(), s));
    }
    HIP_OK(c, hipMemcpyAsync(x_out, dx.p, xb, hipMemcpyDeviceToHost, s));
    HIP_OK(c, hipStreamSynchronize(s));
    if (valid_out)
        for (int64_t K = 0; K < n_sft; ++K)
            std::memset(valid_out + K * n_out, sft_valid ? (sft_valid[K] ? 1 : 0) : 1, (size_t)n_out);
    return CCR_OK;
}

ccr_status ccr_resample_series(ccr_ctx *c, ccr_precision prec, int band_id, int64_t template_index, int det,
                               void *y_out) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B || !y_out) return fail(c, CCR_EINVAL, "bad band id or null output");
    if (prec != CCR_PREC_FP64 && prec != CCR_PREC_SPLIT) return fail(c, CCR_EINVAL, "bad precision");
    if (c->device < 0) return fail(c, CCR_EDEVICE, "host-only context");
    HIP_OK(c, hipSetDevice(c->device));
    ccr_status st = ensure_ready(c, *B);
    if (st) return st;
    if (template_index < 0 || template_index >= B->n_tmpl) return fail(c, CCR_EINVAL, "template index out of range");
    if (det < 0 || det >= B->Q) return fail(c, CCR_EINVAL, "detector index out of range");
    const bool fp64 = prec == CCR_PREC_FP64;
    const Plan &pl = B->plan;
    const size_t cs = fp64 ? 16 : 8;
    const size_t bytes = (size_t)B->Q * pl.n_seg * pl.n_k * cs;
    const size_t per = (size_t)pl.n_seg * pl.n_k * cs;
    hipStream_t s = c->stream;
    if (!fp64) {
        const void *yd = nullptr;
        if ((st = split_series_of(c, band_id, template_index, s, &yd))) return st;
        HIP_OK(c, hipMemcpyAsync(y_out, static_cast<const char *>(yd) + det * per, per, hipMemcpyDeviceToHost, s));
        HIP_OK(c, hipStreamSynchronize(s));
        return CCR_OK;
    }
    DevBuf y, cf;
    HIP_OK(c, y.ensure(bytes));
    HIP_OK(c, cf.ensure((size_t)std::max(B->n_work, 1) * kCheb * sizeof(double)));
    HIP_OK(c, launch_zero(y.p, bytes, s));
    BandDev bd = band_dev(*B);
    if (!c->opt_farrow) bd.farrow = nullptr;
    bd.far_stage = (int)c->opt_farrow_stage;
    HIP_OK(c, launch_timebase(bd, B->d_tmpl.as<double>() + (size_t)template_index * kTmplStride, 1, cf.as<double>(), s));
    HIP_OK(c, launch_resample(bd, cf.as<double>(), 1, fp64, y.p, s));
    HIP_OK(c, hipMemcpyAsync(y_out, y.as<char>() + det * per, per, hipMemcpyDeviceToHost, s));
    HIP_OK(c, hipStreamSynchronize(s));
    return CCR_OK;
}

ccr_status ccr_time_base(ccr_ctx *c, int band_id, int64_t template_index, int det, int64_t k0, int64_t n_seg_out,
                         double *eta_out, double *anchor_out, double *psi_out) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B || !eta_out) return fail(c, CCR_EINVAL, "bad band id or null output");
    if (c->device < 0) return fail(c, CCR_EDEVICE, "host-only context");
    HIP_OK(c, hipSetDevice(c->device));
    ccr_status st = ensure_ready(c, *B);
    if (st) return st;
    if (template_index < 0 || template_index >= B->n_tmpl) return fail(c, CCR_EINVAL, "template index out of range");
    if (det < 0 || det >= B->Q) return fail(c, CCR_EINVAL, "detector index out of range");
    const Plan &pl = B->plan;
    if (k0 < 0 || n_seg_out < 1 || k0 + n_seg_out > pl.n_seg) return fail(c, CCR_EINVAL, "segment range out of range");
    const size_t ns = (size_t)n_seg_out * pl.n_k;
    DevBuf cf, de, dp;
    HIP_OK(c, cf.ensure((size_t)std::max(B->n_work, 1) * kCheb * sizeof(double)));
    HIP_OK(c, de.ensure(ns * sizeof(double)));
    HIP_OK(c, dp.ensure(ns * sizeof(double)));
    hipStream_t s = c->stream;
    HIP_OK(c, hipMemcpyAsync(de.p, eta_out, ns * sizeof(double), hipMemcpyHostToDevice, s));
    if (psi_out) HIP_OK(c, hipMemcpyAsync(dp.p, psi_out, ns * sizeof(double), hipMemcpyHostToDevice, s));
    const BandDev bd = band_dev(*B);
    HIP_OK(c, launch_timebase(bd, B->d_tmpl.as<double>() + (size_t)template_index * kTmplStride, 1, cf.as<double>(), s));
    HIP_OK(c, launch_time_samples(bd, cf.as<double>(), det, (int)k0, (int)n_seg_out, de.as<double>(), dp.as<double>(), s));
    HIP_OK(c, hipMemcpyAsync(eta_out, de.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    if (psi_out) HIP_OK(c, hipMemcpyAsync(psi_out, dp.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(c, hipStreamSynchronize(s));
    if (anchor_out) {
        // the anchors as the device holds them
        std::vector<Anchor> an((size_t)n_seg_out);
        HIP_OK(c, hipMemcpy(an.data(), B->d_anchor.as<Anchor>() + (size_t)det * pl.n_seg + k0,
                            an.size() * sizeof(Anchor), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < n_seg_out; ++k) anchor_out[k] = an[(size_t)k].D_a;
    }
    return CCR_OK;
}

ccr_status ccr_segment_spectra(ccr_ctx *c, ccr_precision prec, int band_id, int64_t template_index, void *f_out) {
    if (!c) return CCR_EINVAL;
    c->err.clear();
    Band *B = get_band(c, band_id);
    if (!B || !f_out) return fail(c, CCR_EINVAL, "bad band id or null output");
    if (prec != CCR_PREC_FP64 && prec != CCR_PREC_SPLIT) return fail(c, CCR_EINVAL, "bad precision");
    if (c->device < 0) return fail(c, CCR_EDEVICE, "host-only context");
    HIP_OK(c, hipSetDevice(c->device));
    ccr_status st = ensure_ready(c, *B);
    if (st) return st;
    if (template_index < 0 || template_index >= B->n_tmpl) return fail(c, CCR_EINVAL, "template index out of range");
    const bool fp64 = prec == CCR_PREC_FP64;
    const Plan &pl = B->plan;
    const size_t cs = fp64 ? 16 : 8;
    DevBuf y, F, cf;
    HIP_OK(c, cf.ensure((size_t)std::max(B->n_work, 1) * kCheb * sizeof(double)));
    const size_t ybytes = (size_t)B->Q * pl.n_seg * pl.n_k * cs, fbytes = (size_t)B->Q * pl.n_seg * pl.n_f * cs;
    HIP_OK(c, F.ensure(fbytes));
    hipStream_t s = c->stream;
    HIP_OK(c, launch_zero(F.p, fbytes, s));
    BandDev bd = band_dev(*B);
    if (!c->opt_farrow) bd.farrow = nullptr;
    bd.far_stage = (int)c->opt_farrow_stage;
    const void *ysrc = nullptr;
    if (fp64) {
        HIP_OK(c, y.ensure(ybytes));
        HIP_OK(c, launch_zero(y.p, ybytes, s));
        HIP_OK(c, launch_timebase(bd, B->d_tmpl.as<double>() + (size_t)template_index * kTmplStride, 1, cf.as<double>(), s));
        HIP_OK(c, launch_resample(bd, cf.as<double>(), 1, fp64, y.p, s));
        ysrc = y.p;
    } else if ((st = split_series_of(c, band_id, template_index, s, &ysrc))) {
        return st;
    }
    bd.pw = nullptr;  // the unweighted spectra F
    HIP_OK(c, launch_spectra(bd, 1, fp64, ysrc, F.p, s));
    HIP_OK(c, hipMemcpyAsync(f_out, F.p, fbytes, hipMemcpyDeviceToHost, s));
    HIP_OK(c, hipStreamSynchronize(s));
    return CCR_OK;
}

}  // extern "C"

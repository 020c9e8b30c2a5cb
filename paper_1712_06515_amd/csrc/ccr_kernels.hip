// gfx950 kernels of the resampled cross-correlation hot path (staged form).
//
//   k_resample  FP64 time base + windowed-sinc resampling + heterodyne correction,
//               one workgroup per (template, detector, segment), one thread per sample.
//   k_spectra   zero-padded, input-pruned FFT of each segment in LDS (Stockham radix 4/2,
//               N_FFT = P * n_s, one n_s-point FFT per residue class of the output bins),
//               Phi_in phase reference and normalisation, decimated bins only.
//   k_pairs     weighted pair sum over the lag window, one thread per (template, bin,
//               segment chunk), fixed summation order.
//   k_finish    sum of chunk partials and the sqrt(2) / N factor.
#include <hip/hip_runtime.h>

#include <mutex>

#include <climits>

#include "ccr_internal.h"

namespace ccr {
namespace {

// Two 32-bit lanes: the data operand of the 64-bit buffer store builtin.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ complex helpers
template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };
template <typename T> using c2 = typename C2<T>::type;

template <typename T> __device__ __forceinline__ c2<T> mk(T re, T im) { c2<T> v; v.x = re; v.y = im; return v; }
template <typename T> __device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ c2<T> cscale(c2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by -i
template <typename T> __device__ __forceinline__ c2<T> cmul_mi(c2<T> a) { return mk<T>(a.y, -a.x); }

template <typename T> __device__ __forceinline__ const c2<T> *twiddles(const BandDev &B);
template <> __device__ __forceinline__ const float2 *twiddles<float>(const BandDev &B) { return B.tw32; }
template <> __device__ __forceinline__ const double2 *twiddles<double>(const BandDev &B) { return B.tw64; }

// Orders the LDS accesses of one wavefront around this point (compiler ordering only: the
// hardware executes a wavefront's LDS operations in issue order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ time base (FP64)

// sin(x) and cos(x) - 1 by their Taylor series: through x^11 / x^12 (|x| <= 0.3 keeps the
// truncation below 3e-17 relative), or with SHORT through x^7 / x^8, which a band uses when the
// host's bound on the dropped terms, amplitude x |x|^9 / 9! over its templates, is below 1e-16 s.
template <bool SHORT>
__device__ __forceinline__ void sincos_small(double x, double &s, double &cm1) {
    const double x2 = x * x;
    if constexpr (SHORT) {
        s = x * (1.0 - x2 * (1.0 / 6.0) * (1.0 - x2 * (1.0 / 20.0) * (1.0 - x2 * (1.0 / 42.0))));
        cm1 = -x2 * 0.5 * (1.0 - x2 * (1.0 / 12.0) * (1.0 - x2 * (1.0 / 30.0) * (1.0 - x2 * (1.0 / 56.0))));
    } else {
        s = x * (1.0 - x2 * (1.0 / 6.0) * (1.0 - x2 * (1.0 / 20.0) * (1.0 - x2 * (1.0 / 42.0) *
                 (1.0 - x2 * (1.0 / 72.0) * (1.0 - x2 * (1.0 / 110.0))))));
        cm1 = -x2 * 0.5 * (1.0 - x2 * (1.0 / 12.0) * (1.0 - x2 * (1.0 / 30.0) * (1.0 - x2 * (1.0 / 56.0) *
                 (1.0 - x2 * (1.0 / 90.0) * (1.0 - x2 * (1.0 / 132.0))))));
    }
}

// Binary orbital phase (cycles in [0,1)) of segment K's mid-time: frac(c0 + K c1), both in
// double-double, then (sin, cos) of 2 pi times it.
__device__ __forceinline__ void binary_anchor(const double *tp, int K, double &sb, double &cb) {
    // The product error eA must be added once: contraction of A - floor(A) into an FMA would
    // fold it in a second time (an error of up to half an ulp of K c1, growing with K).
#pragma clang fp contract(off)
    const double kd = (double)K;
    const double A = kd * tp[4];
    const double eA = fma(kd, tp[4], -A);
    const double fA = A - floor(A);
    double ph = fA + (eA + (kd * tp[5] + (tp[2] + tp[3])));
    ph -= floor(ph);
    sincospi(2.0 * ph, &sb, &cb);
}

// Delay of source sample u seconds after the segment anchor (see Anchor).  With the detector
// time t = t_a + u + eta, the source-time equation tau(t) = tau_a + u becomes
//   G(eta) = eta + rho_a + de(u + eta) - a_p sin(theta_b + Omega (u + eta + rho_a + de)) = 0,
// de(x) = r(t_a + x).n - r(t_a).n, theta_b the binary phase at tau_a; Delta = eta - D_a.
// Three Newton steps from eta_0 = a_p sin(theta_b + Omega u) (quadratic convergence from an
// initial error below 0.1 s leaves < 1e-25 s).
template <bool SHORT>
__device__ __forceinline__ double node_eta(double u, double a_p, double Om, double sb, double cb,
                                           const EarthConst &ec, const Anchor &an, int steps) {
    double s, cm;
    sincos_small<SHORT>(Om * u, s, cm);
    double eta = a_p * (fma(sb, cm, sb) + cb * s);
    // Newton from the binary-only value; `steps` (2 or 3) comes from the host's convergence bound
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        if (it >= steps) break;
        const double x = u + eta;
        double so, co, sd, cd;
        sincos_small<SHORT>(ec.w_o * x, so, co);
        sincos_small<SHORT>(ec.w_d * x, sd, cd);
        const double de = ec.A_o * (an.c_o * co - an.s_o * so) + ec.A_d * (an.c_d * cd - an.s_d * sd) + an.rho_a;
        const double dep = -ec.A_o * ec.w_o * (an.c_o * so + fma(an.s_o, co, an.s_o)) -
                           ec.A_d * ec.w_d * (an.c_d * sd + fma(an.s_d, cd, an.s_d));
        double sbn, cbn;
        sincos_small<SHORT>(Om * (x + de), sbn, cbn);
        const double sinb = fma(sb, cbn, sb) + cb * sbn;
        const double cosb = fma(cb, cbn, cb) - sb * sbn;
        const double G = eta + de - a_p * sinb;
        const double Gp = (1.0 + dep) * (1.0 - a_p * Om * cosb);
        eta -= G / Gp;
    }
    return eta;
}

// ---- eccentric orbits (Sec. II.A.2, eqs. solve-for-E and Kepler-equation): the binary delay is
// R/c = a_p [sin w (cos E - e) + cos w sqrt(1 - e^2) sin E] with E - e sin E = M, the mean
// anomaly M = Omega (t_SSB - T_p).

// E at segment K's anchor: the mean anomaly M_a = 2 pi frac(c0 + K c1) (as binary_anchor), then
// Newton's method on Kepler's equation from E = M + e sin M until the step is below 1e-15 rad
// (at most 50 steps; the host admits e <= 0.95).  Returns (sin E_a, cos E_a).
__device__ __forceinline__ void kepler_anchor(const double *tp, int K, double &sE, double &cE) {
#pragma clang fp contract(off)
    const double kd = (double)K;
    const double A = kd * tp[4];
    const double eA = fma(kd, tp[4], -A);
    const double fA = A - floor(A);
    double ph = fA + (eA + (kd * tp[5] + (tp[2] + tp[3])));
    ph -= floor(ph);
    const double e = tp[6];
    double sM, cM;
    sincospi(2.0 * ph, &sM, &cM);
    const double M = 2.0 * M_PI * ph;
    double E = M + e * sM;
    for (int it = 0; it < 50; ++it) {
        double s, c;
        sincos(E, &s, &c);
        const double step = (E - e * s - M) / (1.0 - e * c);
        E -= step;
        if (fabs(step) < 1e-15) break;
    }
    sincos(E, &sE, &cE);
}

// sin E, cos E at mean anomaly M_a + dM from (sin, cos) of E_a: E = E_a + d solves
// d - e [sin E_a (cos d - 1) + cos E_a sin d] = dM; six Newton steps from d = dM / (1 - e cos E_a)
// (the host bounds |dM| and e so that they converge to rounding).  (cos d - 1, sin d) from the
// half angle, so both stay accurate for small d.
__device__ __forceinline__ void kepler_offset(double dM, double e, double sEa, double cEa, double &sE, double &cE) {
    double d = dM / (1.0 - e * cEa);
    double sd = 0.0, cm = 0.0;
#pragma unroll
    for (int it = 0; it < 7; ++it) {
        double sh, ch;
        sincos(0.5 * d, &sh, &ch);
        sd = 2.0 * sh * ch;
        cm = -2.0 * sh * sh;
        if (it == 6) break;
        const double f = d - e * (sEa * cm + cEa * sd) - dM;
        const double fp = 1.0 - e * (cEa * (1.0 + cm) - sEa * sd);
        d -= f / fp;
    }
    sE = fma(sEa, cm, sEa) + cEa * sd;
    cE = fma(cEa, cm, cEa) - sEa * sd;
}

// Binary delay R/c and d(R/c)/dt_SSB at (sin E, cos E).
__device__ __forceinline__ void ecc_delay(const double *tp, double sE, double cE, double &R, double &Rd) {
    const double ap = tp[0], Om = tp[1], e = tp[6], sw = tp[7], cw = tp[8], q = tp[9];
    R = ap * (sw * (cE - e) + cw * q * sE);
    Rd = ap * Om * (cw * q * cE - sw * sE) / (1.0 - e * cE);
}

// node_eta for an eccentric orbit: the same equation with the Kepler delay,
//   G(eta) = eta + rho_a + de(u + eta) - R(M_a + Omega (u + eta + rho_a + de))/c = 0,
// Newton from the binary-only value R(M_a + Omega u).
template <bool SHORT>
__device__ __forceinline__ double node_eta_ecc(double u, const double *tp, double sEa, double cEa,
                                               const EarthConst &ec, const Anchor &an, int steps) {
    const double Om = tp[1], e = tp[6];
    double sE, cE, R, Rd;
    kepler_offset(Om * u, e, sEa, cEa, sE, cE);
    ecc_delay(tp, sE, cE, R, Rd);
    double eta = R;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        if (it >= steps) break;
        const double x = u + eta;
        double so, co, sd, cd;
        sincos_small<SHORT>(ec.w_o * x, so, co);
        sincos_small<SHORT>(ec.w_d * x, sd, cd);
        const double de = ec.A_o * (an.c_o * co - an.s_o * so) + ec.A_d * (an.c_d * cd - an.s_d * sd) + an.rho_a;
        const double dep = -ec.A_o * ec.w_o * (an.c_o * so + fma(an.s_o, co, an.s_o)) -
                           ec.A_d * ec.w_d * (an.c_d * sd + fma(an.s_d, cd, an.s_d));
        kepler_offset(Om * (x + de), e, sEa, cEa, sE, cE);
        ecc_delay(tp, sE, cE, R, Rd);
        const double G = eta + de - R;
        const double Gp = (1.0 + dep) * (1.0 - Rd);
        eta -= G / Gp;
    }
    return eta;
}

// eta(u) over a segment, u in [-h, h] with h = N_K dt / 2: the degree kCheb - 1 polynomial
// through the values at the Chebyshev nodes u_j = h cos(pi (j + 1/2) / kCheb), stored by its
// monomial coefficients in x = u / h: eta = sum_m p_m x^m.  eta is an entire function whose k-th
// Chebyshev coefficient is bounded by a_p (Omega h / 2)^k / k!, so degree 9 keeps the
// truncation below 1e-16 s for segments up to ~6000 s.  The host's table maps node values to
// p_m (row m of `V`); it is applied to differences from the first node, which are small, so
// the large entries of the monomial transform do not amplify the rounding of eta itself.
// Thread k of an entry computes p_k from its NN node values (table rows and columns < NN).
template <int NN>
__device__ __forceinline__ double mono_coef(const double *eta, const double *V, int k) {
    const double e0 = eta[0];
    double c = 0.0;
#pragma unroll
    for (int j = 1; j < NN; ++j) c = fma(eta[j] - e0, V[k * kCheb + j], c);
    return k == 0 ? e0 + c : c;
}

// Per sample: eta by Horner at x = u / h, then the interpolation centre j* = r +
// round-half-up(Delta / dt), the offset delta_c = Delta / dt - round(.) in [-1/2, 1/2) and the
// heterodyne phase frac(f_h Delta) = frac(psi_a + f_h eta), cycles.
// NC must be at least the number of nonzero coefficients the time base wrote.
template <int NC = kCheb>
__device__ __forceinline__ double eta_at(const double *coef, double x) {
    double eta = coef[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) eta = fma(eta, x, coef[k]);
    return eta;
}

template <int NC = kCheb>
__device__ __forceinline__ void sample_time(const double *coef, double x, const Anchor &an, double inv_dt,
                                            double f_het, int64_t r, int64_t &jstar, double &dc, double &psi) {
    const double eta = eta_at<NC>(coef, x);
    const double q = (eta - an.D_a) * inv_dt;
    const double k = floor(q + 0.5);
    jstar = r + (int64_t)(int)k;  // |delay| / dt < 2^30 (the host bounds dt and the delay)
    dc = q - k;
    const double ps = fma(f_het, eta, an.psi_a);
    psi = ps - floor(ps);
}

// Time base kernel: one thread per (template, active segment entry, Chebyshev node).  Writes the
// monomial coefficients of eta(u) for every (template, entry): coef[tb][entry][k], k < NN.
// NN = kCheb nodes (degree 9) for the FP64 path; NN = kChebSplit or kChebSplitMin nodes
// (degree 6 or 5) on the split path when the host's bound covers the interpolation error (at
// most twice the dropped Chebyshev tail).  tb_entries(NN) entries x NN nodes per workgroup
// (whole wavefronts); node values meet in LDS for the coefficient transform.
template <int NN, bool SHORT>
__device__ __forceinline__ void timebase_body(const BandDev &B, const double *tmpl, double *coef, int bx, int tb) {
    static_assert(NN == kCheb || NN == kChebSplit || NN == kChebSplitMin || NN == kChebSplitLow, "node rule");
    constexpr int E = tb_entries(NN);
    __shared__ double sh_eta[E * NN];
    __shared__ double2 sh_bin[E];
    const double *tp = tmpl + (size_t)kTmplStride * tb;
    // the binary phase (eccentric: E) at each entry's anchor, once per entry (threads 0 .. E - 1)
    if (threadIdx.x < E) {
        const int w0 = bx * E + (int)threadIdx.x;
        if (w0 < B.n_work) {
            double sb, cb;
            if (B.ecc)
                kepler_anchor(tp, B.work[w0] % B.n_seg, sb, cb);
            else
                binary_anchor(tp, B.work[w0] % B.n_seg, sb, cb);
            sh_bin[threadIdx.x] = make_double2(sb, cb);
        }
    }
    __syncthreads();
    const int le = threadIdx.x / NN;              // entry within the workgroup
    const int j = threadIdx.x - le * NN;          // node (and later coefficient) index
    const int w = bx * E + le;                    // entry in the work list
    const bool on = w < B.n_work;
    if (on) {
        const int entry = B.work[w];
        const int det = entry / B.n_seg;
        const double2 bn = sh_bin[le];
        const double sb = bn.x, cb = bn.y;
        const double h = 0.5 * (double)B.n_k * B.dt;
        const double *xn = B.cheb_x + cheb_x_off(NN);
        sh_eta[threadIdx.x] = B.ecc ? node_eta_ecc<SHORT>(h * xn[j], tp, sb, cb, B.earth[det], B.anchors[entry],
                                                          B.newton_steps)
                                    : node_eta<SHORT>(h * xn[j], tp[0], tp[1], sb, cb, B.earth[det],
                                                      B.anchors[entry], B.newton_steps);
    }
    __syncthreads();
    const double *V = B.mono + cheb_rule(NN) * kCheb * kCheb;
    if (on) coef[((size_t)tb * B.n_work + w) * kCheb + j] = mono_coef<NN>(sh_eta + le * NN, V, j);
}

__global__ void __launch_bounds__(tb_entries(kCheb) * kCheb) k_timebase(BandDev B, const double *tmpl, double *coef) {
    timebase_body<kCheb, false>(B, tmpl, coef, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------ resampling

template <typename T> __device__ __forceinline__ const T *win_table(const BandDev &B);
template <> __device__ __forceinline__ const float *win_table<float>(const BandDev &B) { return B.win32; }
template <> __device__ __forceinline__ const double *win_table<double>(const BandDev &B) { return B.win64; }

template <typename T> __device__ __forceinline__ T recip(T v);
// v_rcp_f32 (1 ulp) for the split path; IEEE division for FP64.
template <> __device__ __forceinline__ float recip<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ __forceinline__ double recip<double>(double v) { return 1.0 / v; }

// sin(pi v) and (cos, sin)(2 pi v): OCML sinpi / sincospi in FP64; in FP32 the hardware
// v_sin_f32 / v_cos_f32, which take their argument in revolutions (|v| <= 1 here).
template <typename T> __device__ __forceinline__ T sin_pi(T v);
template <> __device__ __forceinline__ double sin_pi<double>(double v) { return sinpi(v); }
template <> __device__ __forceinline__ float sin_pi<float>(float v) { return __builtin_amdgcn_sinf(0.5f * v); }
template <typename T> __device__ __forceinline__ void sincos_rev(double v, T &s, T &c);
template <> __device__ __forceinline__ void sincos_rev<double>(double v, double &s, double &c) {
    sincospi(2.0 * v, &s, &c);
}
template <> __device__ __forceinline__ void sincos_rev<float>(double v, float &s, float &c) {
    const float f = (float)v;
    s = __builtin_amdgcn_sinf(f);
    c = __builtin_amdgcn_cosf(f);
}
// cos(pi v) for the continuous window
template <typename T> __device__ __forceinline__ T cos_pi(T v);
template <> __device__ __forceinline__ double cos_pi<double>(double v) { return cospi(v); }
template <> __device__ __forceinline__ float cos_pi<float>(float v) { return __builtin_amdgcn_cosf(0.5f * v); }

// Weight of tap n for centre offset dc: w sinc(dc - n) with sin(pi (dc - n)) = (-1)^n sin(pi dc),
// s = sin(pi dc) / pi.  WIN 0: Hamming indexed by tap (table); WIN 1: Hamming at the offset.
template <typename T, int WIN>
__device__ __forceinline__ T tap_weight(const T *wt, int D, T inv_d1, T dc, T s, int n) {
    const T d = dc - (T)n;
    T tap;
    if (n == 0) {
        tap = (dc == (T)0) ? (T)1 : s * recip<T>(dc);
    } else {
        tap = ((n & 1) ? -s : s) * recip<T>(d);
    }
    const T w = (WIN == 0) ? wt[n + D] : (T)0.54 + (T)0.46 * cos_pi<T>(d * inv_d1);
    return w * tap;
}

// sum_{n=-D}^{D} w sinc(delta_c - n) x'_{j*+n}; taps outside [0, n) read zero.  DT > 0 fixes D
// at compile time (unrolled taps).  The bounds checks are taken only near the data edges.
// Fast form for the tap-indexed window (WIN 0) with every tap inside the data: the common
// factor sin(pi dc) / pi leaves the sum, y = s sum_n (-1)^n w_n x'_{j*+n} / (dc - n), and an
// on-grid sample (dc = 0) is x'_{j*} exactly (w_0 = 1).
// `cw[n + D]` = (-1)^n w_n, loaded once per workgroup.
template <typename T, int DT>
__device__ __forceinline__ c2<T> interpolate_w0_inside(const T *cw, const float2 *xc, T dc) {
    if (dc == (T)0) {
        const float2 x0 = xc[0];
        return mk<T>((T)x0.x, (T)x0.y);
    }
    const T s = sin_pi<T>(dc) * (T)0.318309886183790671537767526745;
    T re = 0, im = 0;
#pragma unroll
    for (int n = -DT; n <= DT; ++n) {
        const T q = cw[n + DT] * recip<T>(dc - (T)n);
        const float2 xv = xc[n];
        re = fma(q, (T)xv.x, re);
        im = fma(q, (T)xv.y, im);
    }
    return mk<T>(re * s, im * s);
}

// FP32 form: taps n and -n share one reciprocal, 1/(dc - n) = (dc + n) r and 1/(dc + n) =
// (dc - n) r with r = 1/(dc^2 - n^2) (|dc^2 - n^2| >= 3/4), and the window is symmetric
// (cw[D + n] = cw[D - n]).
template <>
__device__ __forceinline__ float2 interpolate_w0_inside<float, 8>(const float *cw, const float2 *xc, float dc) {
    if (dc == 0.f) return xc[0];
    const float s = sin_pi<float>(dc) * 0.318309886183790671537767526745f;
    const float q0 = cw[8] * recip<float>(dc);
    const float2 x0 = xc[0];
    float re = q0 * x0.x, im = q0 * x0.y;
#pragma unroll
    for (int n = 1; n <= 8; ++n) {
        const float r = recip<float>(fmaf(dc, dc, -(float)(n * n)));
        const float cr = cw[8 + n] * r;
        const float t = cr * dc;
        const float qp = fmaf(cr, (float)n, t);   // weight of x'_{j* + n}
        const float qm = fmaf(-cr, (float)n, t);  // weight of x'_{j* - n}
        const float2 xp = xc[n], xm = xc[-n];
        re = fmaf(qp, xp.x, re);
        im = fmaf(qp, xp.y, im);
        re = fmaf(qm, xm.x, re);
        im = fmaf(qm, xm.y, im);
    }
    return make_float2(re * s, im * s);
}

// Signed tap coefficients (-1)^n w_n of the tap-indexed window for interpolate_w0_inside.
template <typename T, int DT>
__device__ __forceinline__ void load_signed_window(const BandDev &B, T *cw) {
    const T *wt = win_table<T>(B);
#pragma unroll
    for (int n = -DT; n <= DT; ++n) cw[n + DT] = (n & 1) ? -wt[n + DT] : wt[n + DT];
}

// `cw` (signed window, see load_signed_window) is read only when WIN == 0 and DT > 0.
template <typename T, int DT, int WIN>
__device__ __forceinline__ c2<T> interpolate(const BandDev &B, const float2 *xd, int64_t jstar, double dcd,
                                             const T *cw) {
    const T dc = (T)dcd;
    const int D = DT > 0 ? DT : B.D;
    if constexpr (WIN == 0 && DT > 0) {
        if (jstar - D >= 0 && jstar + D < B.n) return interpolate_w0_inside<T, DT>(cw, xd + jstar, dc);
    }
    const T s = sin_pi<T>(dc) * (T)0.318309886183790671537767526745;
    const T *wt = win_table<T>(B);
    const T inv_d1 = (T)1 / (T)(D + 1);
    T re = 0, im = 0;
    if (jstar - D >= 0 && jstar + D < B.n) {
        const float2 *xc = xd + jstar;
        if constexpr (DT > 0) {
#pragma unroll
            for (int n = -DT; n <= DT; ++n) {
                const T wv = tap_weight<T, WIN>(wt, D, inv_d1, dc, s, n);
                const float2 xv = xc[n];
                re = fma(wv, (T)xv.x, re);
                im = fma(wv, (T)xv.y, im);
            }
        } else {
            for (int n = -D; n <= D; ++n) {
                const T wv = tap_weight<T, WIN>(wt, D, inv_d1, dc, s, n);
                const float2 xv = xc[n];
                re = fma(wv, (T)xv.x, re);
                im = fma(wv, (T)xv.y, im);
            }
        }
    } else {
        for (int n = -D; n <= D; ++n) {
            const int64_t j = jstar + n;
            if (j < 0 || j >= B.n) continue;
            const T wv = tap_weight<T, WIN>(wt, D, inv_d1, dc, s, n);
            const float2 xv = xd[j];
            re = fma(wv, (T)xv.x, re);
            im = fma(wv, (T)xv.y, im);
        }
    }
    return mk<T>(re, im);
}

// The same tap sum over an LDS window w[] holding x'_{j* - off + m}; the caller guarantees
// off - D >= 0 and off + D < W.
template <typename T, int DT, int WIN>
__device__ __forceinline__ c2<T> interpolate_window(const BandDev &B, const float2 *w, int off, double dcd) {
    const T dc = (T)dcd;
    const T s = sin_pi<T>(dc) * (T)0.318309886183790671537767526745;
    const T *wt = win_table<T>(B);
    const int D = DT > 0 ? DT : B.D;
    const T inv_d1 = (T)1 / (T)(D + 1);
    T re = 0, im = 0;
    if constexpr (DT > 0) {
#pragma unroll
        for (int n = -DT; n <= DT; ++n) {
            const T wv = tap_weight<T, WIN>(wt, D, inv_d1, dc, s, n);
            const float2 xv = w[off + n];
            re = fma(wv, (T)xv.x, re);
            im = fma(wv, (T)xv.y, im);
        }
    } else {
        for (int n = -D; n <= D; ++n) {
            const T wv = tap_weight<T, WIN>(wt, D, inv_d1, dc, s, n);
            const float2 xv = w[off + n];
            re = fma(wv, (T)xv.x, re);
            im = fma(wv, (T)xv.y, im);
        }
    }
    return mk<T>(re, im);
}

// Tap sum with every tap inside a zero-padded window (no bounds checks): the w0 form for the
// tap-indexed window, else the general taps.
template <typename T, int DT, int WIN>
__device__ __forceinline__ c2<T> interpolate_inside(const BandDev &B, const float2 *xc, double dcd, const T *cw) {
    const T dc = (T)dcd;
    if constexpr (WIN == 0 && DT > 0) {
        return interpolate_w0_inside<T, DT>(cw, xc, dc);
    } else {
        const int D = DT > 0 ? DT : B.D;
        const T s = sin_pi<T>(dc) * (T)0.318309886183790671537767526745;
        const T *wt = win_table<T>(B);
        const T inv_d1 = (T)1 / (T)(D + 1);
        T re = 0, im = 0;
        for (int n = -D; n <= D; ++n) {
            const T wv = tap_weight<T, WIN>(wt, D, inv_d1, dc, s, n);
            const float2 xv = xc[n];
            re = fma(wv, (T)xv.x, re);
            im = fma(wv, (T)xv.y, im);
        }
        return mk<T>(re, im);
    }
}

// Input window of one 64-sample pass of the resampler: j* is nondecreasing in the sample index
// (t(tau) is increasing), so the pass needs x'[j*_first - D, j*_last + D], at most 64 + 2D + 1
// samples plus the drift; kResWin holds that with room to spare.
constexpr int kResWin = 128;
static_assert(kResWin == 128, "the interior window fill loads 2 x 64 entries");

// Resampler: one 64-lane workgroup (one wavefront) per (active segment, templates [t0, t1)),
// looping over the segment's samples 64 at a time for each template; the segment's anchor and
// window coefficients are loaded once, each template's time-base coefficients are uniform
// (scalar loads).  Each pass stages its input window in LDS (two coalesced loads per lane,
// zero outside the data) and every lane reads its 2D + 1 taps from there.
template <typename T, int DT, int WIN, int NC = kCheb>
__device__ __forceinline__ void resample_body(const BandDev &B, const double *coef, c2<T> *y, int w, int t0,
                                              int t1) {
    __shared__ float2 win[kResWin];
    const int entry = B.work[w];
    const int det = entry / B.n_seg;
    const int K = entry - det * B.n_seg;
    const int64_t nr = (int64_t)B.n_seg * B.n_k;
    const uint8_t *mk_ = B.mask + (size_t)det * nr + (size_t)K * B.n_k;
    const float2 *xd = B.x + (size_t)det * B.n;
    const Anchor an = B.anchors[entry];
    const double inv_nk = 1.0 / (double)B.n_k;
    const int64_t r0 = (int64_t)K * B.n_k;
    const int D = DT > 0 ? DT : B.D;
    const int lane = threadIdx.x;
    T cw[2 * (DT > 0 ? DT : 0) + 1];
    if constexpr (WIN == 0 && DT > 0) load_signed_window<T, DT>(B, cw);
    for (int tb = t0; tb < t1; ++tb) {
    c2<T> *yo = y + ((size_t)tb * B.Q + det) * nr + (size_t)K * B.n_k;
    const double *cf = coef + ((size_t)tb * B.n_work + w) * kCheb;
    double cl[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) cl[k] = cf[k];
    for (int s0 = 0; s0 < B.n_k; s0 += 64) {
        const int s = s0 + lane;
        const bool in = s < B.n_k;
        const bool m = in && mk_[s];
        int64_t jstar = r0 + s;
        double dc = 0.0, psi = 0.0;
        if (in) sample_time<NC>(cl, (double)(2 * s - B.n_k) * inv_nk, an, B.inv_dt, B.f_het, r0 + s, jstar, dc, psi);
        // window bounds from the pass's first and last samples (shifts relative to r0 fit 32 bits)
        const int last = min(63, B.n_k - 1 - s0);
        const int jrel = (int)(jstar - r0);
        const int lo_rel = __builtin_amdgcn_readlane(jrel, 0) - D;
        const int span = __builtin_amdgcn_readlane(jrel, last) + D - lo_rel + 1;
        c2<T> acc = mk<T>((T)0, (T)0);
        if (span <= kResWin) {
            const int64_t j_lo = r0 + lo_rel;
            wave_sync();  // the previous pass's reads of the window are done (one wavefront)
            if (j_lo >= 0 && j_lo + kResWin <= B.n) {
                // interior (uniform branch): the whole LDS window, no bounds checks
                const float2 *xw = xd + j_lo;
                win[lane] = xw[lane];
                win[lane + 64] = xw[lane + 64];
            } else {
                for (int k = lane; k < span; k += 64) {
                    const int64_t j = j_lo + k;
                    win[k] = (j >= 0 && j < B.n) ? xd[j] : make_float2(0.f, 0.f);
                }
            }
            wave_sync();
            if (m) acc = interpolate_inside<T, DT, WIN>(B, win + (int)(jstar - j_lo), dc, cw);
        } else if (m) {
            acc = interpolate<T, DT, WIN>(B, xd, jstar, dc, cw);
        }
        if (in) {
            T c, sn;
            sincos_rev<T>(psi, sn, c);
            yo[s] = m ? mk<T>(c * acc.x - sn * acc.y, sn * acc.x + c * acc.y) : mk<T>((T)0, (T)0);
        }
    }
    }
}

template <typename T, int DT, int WIN>
__global__ void __launch_bounds__(64) k_resample(BandDev B, const double *coef, c2<T> *y) {
    resample_body<T, DT, WIN>(B, coef, y, blockIdx.x, blockIdx.y, blockIdx.y + 1);
}

// ------------------------------------------------------------------ Farrow-form resampling
// Split precision.  The weight of tap n as a function of the offset, c_n(dc) = w sinc(dc - n)
// on dc in [-1/2, 1/2], is replaced by a polynomial [n == 0] + sum_{k=1..kFarDeg} A_kn dc^k
// (least-squares fit by the host, which bounds sum_n |error| and keeps the direct kernel for a
// window whose bound is too large); then the interpolated value is a polynomial in dc,
// sum_n c_n(dc) x'_{j*+n} = sum_k F_k(j*) dc^k with F_k(j) = sum_n A_kn x'_{j+n} and F_0 = x'
// (the Farrow structure of fractional-delay filters).  F depends on the input series only, so it
// is tabulated once per band and detector; per sample the resampler evaluates one complex
// polynomial of degree kFarDeg instead of 2D + 1 reciprocals and products.  An on-grid sample
// (dc = 0) is x'_{j*} exactly, as in the direct form.

// F_k(j) for every detector and j + D in [0, far_len): FP64 sums, stored complex64.
__global__ void __launch_bounds__(256) k_farrow_table(const float2 *__restrict__ x, int64_t n, int D,
                                                      const double *__restrict__ A, int64_t far_len,
                                                      float2 *__restrict__ tab) {
    const int64_t jj = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (jj >= far_len) return;
    const int det = blockIdx.y;
    const float2 *xd = x + (size_t)det * n;
    float2 *td = tab + (size_t)det * (kFarDeg + 1) * far_len;
    const int64_t j = jj - D;
    double re[kFarDeg], im[kFarDeg];
#pragma unroll
    for (int k = 0; k < kFarDeg; ++k) re[k] = im[k] = 0.0;
    for (int m = -D; m <= D; ++m) {
        const int64_t jm = j + m;
        if (jm < 0 || jm >= n) continue;
        const float2 xv = xd[jm];
        const double *a = A + (m + D);
#pragma unroll
        for (int k = 0; k < kFarDeg; ++k) {
            re[k] = fma(a[k * (2 * D + 1)], (double)xv.x, re[k]);
            im[k] = fma(a[k * (2 * D + 1)], (double)xv.y, im[k]);
        }
    }
    td[jj] = (j >= 0 && j < n) ? xd[j] : make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < kFarDeg; ++k) td[(size_t)(k + 1) * far_len + jj] = make_float2((float)re[k], (float)im[k]);
}

// A wave-uniform double computed by the vector unit, moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
    const uint64_t b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b), hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// sum_k F_k dc^k by Horner from the kFarDeg + 1 coefficients of one entry, stored
// consecutively in LDS (16-byte aligned: five 128-bit reads).
__device__ __forceinline__ float2 farrow_eval_lds(const float2 *p, float dc) {
    float2 f[kFarDeg + 1];
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int k = 0; k < (kFarDeg + 1) / 2; ++k) {
        const float4 v = q[k];
        f[2 * k] = make_float2(v.x, v.y);
        f[2 * k + 1] = make_float2(v.z, v.w);
    }
    if constexpr ((kFarDeg + 1) % 2 == 1) f[kFarDeg] = p[kFarDeg];
    float re = f[kFarDeg].x, im = f[kFarDeg].y;
#pragma unroll
    for (int k = kFarDeg - 1; k >= 0; --k) {
        re = fmaf(re, dc, f[k].x);
        im = fmaf(im, dc, f[k].y);
    }
    return make_float2(re, im);
}

// Per sample, as sample_time: j* - r - the offset's integer part (jr), the offset dc and the
// heterodyne phase in cycles (v_fract_f64), the last two rounded to FP32.  `coef` holds the
// time base with D_a taken out of its constant term (its polynomial is the delay
// Delta = eta - D_a), and psi_b = frac(psi_a + f_h D_a), so psi = frac(psi_b + f_h Delta).
template <int NC>
__device__ __forceinline__ void sample_time_far(const double *coef, double x, double inv_dt, double f_het,
                                                double psi_b, int &jr, float &dc, float &psi) {
    const double delta = eta_at<NC>(coef, x);
    const double q = delta * inv_dt;
    const double k = floor(q + 0.5);
    jr = (int)k;
    dc = (float)(q - k);
    psi = (float)__builtin_amdgcn_fract(fma(f_het, delta, psi_b));
}

// The same from the table in global memory (the rare unstaged case), as a plain loop so that
// the planes' addresses are not kept in registers across the sample loop.
__device__ __forceinline__ float2 farrow_eval_global(const float2 *p, int64_t stride, float dc) {
    float re = 0.f, im = 0.f;
#pragma unroll 1
    for (int k = kFarDeg; k >= 0; --k) {
        const float2 f = p[k * stride];
        re = fmaf(re, dc, f.x);
        im = fmaf(im, dc, f.y);
    }
    return make_float2(re, im);
}

// One 256-thread workgroup per (active segment entry, templates [t0, t1)), t1 - t0 <=
// kFarTemplates; wavefront v takes templates t0 + v kFarPerWave + i.  Per chunk of kFarChunk
// samples the workgroup finds the range of j* over its templates (j* is nondecreasing in the
// sample index, so the chunk's first and last samples bound it), stages that range of every
// table plane in LDS with coalesced loads (entry-major there: an entry's kFarDeg + 1 = 9
// coefficients occupy 80 bytes, read by a lane with four 128-bit and one 64-bit LDS reads;
// the 20-dword stride between lanes keeps 16 lanes on distinct banks).  A range wider than
// kFarCap (not met for physical delays) reads the table in global memory instead.  The gap
// mask and the in-chunk test of each pass are wave-wide bit masks (ballots), applied as
// execution masks.
template <int NC>
__device__ __forceinline__ void resample_far_body(const BandDev &B, const double *coef, float2 *y, int w, int t0,
                                                  int t1) {
    constexpr int kE = kFarDeg + 1;          // coefficients of an entry
    constexpr int kES = (kE + 1) / 2 * 2;   // LDS stride of an entry (16-byte aligned)
    __shared__ __align__(16) float2 sf[kES * kFarCap];
    __shared__ int s_lo[kFarWaves], s_hi[kFarWaves];
    const int entry = B.work[w];
    const int det = entry / B.n_seg;
    const int K = entry - det * B.n_seg;
    const int64_t nr = (int64_t)B.n_seg * B.n_k;
    const uint8_t *mk_ = B.mask + (size_t)det * nr + (size_t)K * B.n_k;
    const float2 *tab = B.farrow + (size_t)det * (kFarDeg + 1) * B.far_len;
    const Anchor an = B.anchors[entry];
    const double psi_b = __builtin_amdgcn_fract(fma(B.f_het, an.D_a, an.psi_a));
    const double inv_nk = 1.0 / (double)B.n_k;
    const int64_t r0 = (int64_t)K * B.n_k;
    // wave-uniform (readfirstlane), so that a template's time-base coefficients are scalar
    // loads: a vector load's wait would also wait for the previous pass's stores
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int tw0 = t0 + wave * kFarPerWave;
    for (int c0 = 0; c0 < B.n_k; c0 += kFarChunk) {
        const int c1 = min(B.n_k, c0 + kFarChunk);
        {
            // lanes i < kFarPerWave: j* - r0 at sample c0 of template tw0 + i; lanes 32 + i: at c1 - 1
            const int i = lane & 31, tb = tw0 + i;
            int jr = 0;
            if (i < kFarPerWave && tb < t1) {
                const double *cf = coef + ((size_t)tb * B.n_work + w) * kCheb;
                double cl[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) cl[k] = cf[k];
                cl[0] -= an.D_a;
                const int s = lane < 32 ? c0 : c1 - 1;
                float dc, psi;
                sample_time_far<NC>(cl, (double)(2 * s - B.n_k) * inv_nk, B.inv_dt, B.f_het, psi_b, jr, dc, psi);
                jr += s;
            }
            int lo = INT_MAX, hi = INT_MIN;
#pragma unroll
            for (int q = 0; q < kFarPerWave; ++q) {
                if (tw0 + q < t1) {
                    lo = min(lo, __builtin_amdgcn_readlane(jr, q));
                    hi = max(hi, __builtin_amdgcn_readlane(jr, 32 + q));
                }
            }
            if (lane == 0) {
                s_lo[wave] = lo;
                s_hi[wave] = hi;
            }
        }
        __syncthreads();
        int jlo = s_lo[0], jhi = s_hi[0];  // wavefront 0 holds template t0 < t1
#pragma unroll
        for (int q = 1; q < kFarWaves; ++q) {
            jlo = min(jlo, s_lo[q]);
            jhi = max(jhi, s_hi[q]);
        }
        const int span = jhi - jlo + 1;
        const bool staged = B.far_stage && span <= kFarCap;
        if (staged) {
            const int64_t jb = r0 + jlo + B.D;  // table index of j* = r0 + jlo
            for (int i = threadIdx.x; i < span; i += 256) {
                const int64_t jj = jb + i;
                const bool ok = jj >= 0 && jj < B.far_len;
                float2 f[kE];
#pragma unroll
                for (int k = 0; k < kE; ++k) f[k] = ok ? tab[(size_t)k * B.far_len + jj] : make_float2(0.f, 0.f);
                float4 *d = reinterpret_cast<float4 *>(sf + i * kES);
#pragma unroll
                for (int k = 0; k < kE / 2; ++k) d[k] = make_float4(f[2 * k].x, f[2 * k].y, f[2 * k + 1].x, f[2 * k + 1].y);
                if constexpr (kE % 2 == 1) sf[i * kES + kE - 1] = f[kE - 1];
            }
        }
        // per pass p (sample c0 + 64 p + lane), shared by the templates: the samples inside the
        // chunk (ballot in_b[p]), those of them outside gaps (m_b[p]), the time-base abscissa
        // x and the sample's offset from the staged range
        constexpr int kPasses = kFarChunk / 64;
        static_assert(kFarChunk % 64 == 0, "whole passes");
        uint64_t in_b[kPasses], m_b[kPasses];
        double xs[kPasses];
        int sj[kPasses];
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            const int s = c0 + 64 * p + lane;
            xs[p] = (double)(2 * s - B.n_k) * inv_nk;
            sj[p] = s - jlo;
            const bool in = s < c1;
            in_b[p] = __builtin_amdgcn_ballot_w64(in);
            m_b[p] = __builtin_amdgcn_ballot_w64(in && mk_[s]);
        }
        __syncthreads();
        // STAGED (uniform per chunk): j* lies in the staged range (j* is nondecreasing over the
        // chunk and the range spans its first and last samples), so every lane reads LDS at a
        // clamped index; lanes outside the range, if a wave has any (a uniform test), take the
        // global-memory form instead.  Otherwise every sample reads the table in global memory.
        auto walk = [&](auto staged_c) {
            constexpr bool STAGED = decltype(staged_c)::value;
            for (int i = 0; i < kFarPerWave; ++i) {
                const int tb = tw0 + i;
                if (tb >= t1) break;
                // the series, or with per-sample weights its two streams y a_r and y b_r
                const int ns2 = B.ps2 ? 2 : 1;
                float2 *yo = y + ((size_t)tb * B.Q + det) * ns2 * nr + r0;
                const double *cf = coef + ((size_t)tb * B.n_work + w) * kCheb;
                double cl[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) cl[k] = cf[k];
                cl[0] = uniform_f64(cl[0] - an.D_a);  // once per template, kept in scalar registers
                // buffer stores: a uniform resource per stream and the sample's byte offset (no
                // 64-bit address arithmetic per pass); the range is the segment's n_k samples
                const __amdgpu_buffer_rsrc_t yb0 = __builtin_amdgcn_make_buffer_rsrc(yo, (short)0, B.n_k * 8, 0x00020000);
                const __amdgpu_buffer_rsrc_t yb1 = __builtin_amdgcn_make_buffer_rsrc(yo + nr, (short)0, B.n_k * 8, 0x00020000);
                auto put = [](const __amdgpu_buffer_rsrc_t &rs, unsigned idx, float2 v) {
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, (int)(idx * 8u), 0, 0);
                };
#pragma unroll
                for (int p = 0; p < kPasses; ++p) {
                    if (c0 + 64 * p >= c1) break;
                    const unsigned so = (unsigned)(c0 + 64 * p + lane);  // sample index (32-bit offset from yo)
                    // samples in gaps: zero (their own execution mask)
                    if (__builtin_amdgcn_inverse_ballot_w64(in_b[p] & ~m_b[p])) {
                        put(yb0, so, make_float2(0.f, 0.f));
                        if (B.ps2) put(yb1, so, make_float2(0.f, 0.f));
                    }
                    if (__builtin_amdgcn_inverse_ballot_w64(m_b[p])) {
                        int jr;
                        float dc, psi;
                        sample_time_far<NC>(cl, xs[p], B.inv_dt, B.f_het, psi_b, jr, dc, psi);
                        jr += sj[p];  // j* - r0 - jlo
                        float2 a;
                        bool far = true;
                        if constexpr (STAGED) {
                            const bool in_range = (unsigned)jr < (unsigned)span;
                            a = farrow_eval_lds(sf + __umul24(min((unsigned)jr, (unsigned)span - 1u), kES), dc);
                            far = __builtin_amdgcn_ballot_w64(!in_range) != 0 && !in_range;
                        }
                        if (far) {
                            const int64_t jj = r0 + jlo + jr + B.D;
                            a = (jj >= 0 && jj < B.far_len) ? farrow_eval_global(tab + jj, B.far_len, dc)
                                                             : make_float2(0.f, 0.f);
                        }
                        const float c = __builtin_amdgcn_cosf(psi), sn = __builtin_amdgcn_sinf(psi);
                        const float2 yv = make_float2(c * a.x - sn * a.y, sn * a.x + c * a.y);
                        if (B.ps2) {
                            const float2 wr = B.pwf[(size_t)det * nr + r0 + so];
                            put(yb0, so, make_float2(yv.x * wr.x, yv.y * wr.x));
                            put(yb1, so, make_float2(yv.x * wr.y, yv.y * wr.y));
                        } else {
                            put(yb0, so, yv);
                        }
                    }
                }
            }
        };
        if (staged) walk(std::integral_constant<bool, true>());
        else walk(std::integral_constant<bool, false>());
        __syncthreads();  // the next chunk restages sf
    }
}

__global__ void __launch_bounds__(256) k_resample_far(BandDev B, const double *coef, float2 *y, int n_tmpl) {
    const int t0 = blockIdx.y * kFarTemplates;
    resample_far_body<kCheb>(B, coef, y, blockIdx.x, t0, min(n_tmpl, t0 + kFarTemplates));
}

// Time base samples of one detector's segments [k0, k0 + n) for one template (stage output).
__global__ void __launch_bounds__(64) k_time_samples(BandDev B, const double *coef, int det, int k0, int n,
                                                     double *eta, double *psi) {
    const int K = k0 + (int)blockIdx.x;
    if ((int)blockIdx.x >= n) return;
    const int w = B.seg_work[det * B.n_seg + K];
    if (w < 0) return;
    const Anchor an = B.anchors[det * B.n_seg + K];
    const double *cf = coef + (size_t)w * kCheb;
    const double inv_nk = 1.0 / (double)B.n_k;
    for (int s = threadIdx.x; s < B.n_k; s += 64) {
        const double x = (double)(2 * s - B.n_k) * inv_nk;
        int64_t jstar;
        double dc, ps;
        sample_time(cf, x, an, B.inv_dt, B.f_het, (int64_t)K * B.n_k + s, jstar, dc, ps);
        const size_t o = (size_t)blockIdx.x * B.n_k + s;
        eta[o] = eta_at(cf, x);
        psi[o] = ps;
    }
}

// v mod N_FFT for 0 <= v (a mask when N_FFT is a power of two).
__device__ __forceinline__ int mod_fft(const BandDev &B, int64_t v) {
    return B.nfft_mask ? (int)(v & B.nfft_mask) : (int)(v % B.n_fft);
}

// ------------------------------------------------------------------ FFT in LDS

// Self-sorting Stockham passes (radix 4, a final radix 2 when log2 n is odd) over n points
// held in LDS; twiddles exp(-2 pi i k r / (Ns R)) read from the N_FFT-entry table.
// Threads g0, g0 + gs, ... of the block work on this transform; every thread of the block
// must call it the same number of times (it holds block-wide barriers); `active` = false lets
// a thread group skip the arithmetic while keeping the barriers.
template <typename T>
__device__ c2<T> *stockham(c2<T> *a, c2<T> *b, int n, const c2<T> *tw, int n_fft, int g0, int gs,
                           bool active = true) {
    for (int Ns = 1; Ns < n;) {
        const int R = (Ns * 4 <= n) ? 4 : 2;
        const int stride = n / R;
        const int twstep = n_fft / (Ns * R);
        for (int j = g0; active && j < stride; j += gs) {
            const int k = j & (Ns - 1);
            const int idxD = (j - k) * R + k;
            if (R == 4) {
                c2<T> v0 = a[j], v1 = a[j + stride], v2 = a[j + 2 * stride], v3 = a[j + 3 * stride];
                if (k) {
                    v1 = cmul<T>(v1, tw[k * twstep]);
                    v2 = cmul<T>(v2, tw[2 * k * twstep]);
                    v3 = cmul<T>(v3, tw[3 * k * twstep]);
                }
                const c2<T> a0 = cadd<T>(v0, v2), a1 = csub<T>(v0, v2);
                const c2<T> a2 = cadd<T>(v1, v3), a3 = cmul_mi<T>(csub<T>(v1, v3));
                b[idxD] = cadd<T>(a0, a2);
                b[idxD + Ns] = cadd<T>(a1, a3);
                b[idxD + 2 * Ns] = csub<T>(a0, a2);
                b[idxD + 3 * Ns] = csub<T>(a1, a3);
            } else {
                c2<T> v0 = a[j], v1 = a[j + stride];
                if (k) v1 = cmul<T>(v1, tw[k * twstep]);
                b[idxD] = cadd<T>(v0, v1);
                b[idxD + Ns] = csub<T>(v0, v1);
            }
        }
        __syncthreads();
        c2<T> *t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// Spectrum of one (template, detector, segment): for each residue class p of the output
// bins, twiddle the zero-padded segment by exp(-2 pi i p s / N_FFT), n_s-point FFT, pick
// bins kbar = m P + p, apply Phi_in = exp(-2 pi i kbar r_B / N_FFT) and 1 / (sigma sqrt N_K).
// ------------------------------------------------------------------ register FFT (256 points)


// 4-point forward DFT in place: (a0, a1, a2, a3) -> sum_n a_n exp(-2 pi i n k / 4).
template <typename T>
__device__ __forceinline__ void dft4(c2<T> &a0, c2<T> &a1, c2<T> &a2, c2<T> &a3) {
    const c2<T> t0 = cadd<T>(a0, a2), t1 = csub<T>(a0, a2);
    const c2<T> t2 = cadd<T>(a1, a3), t3 = cmul_mi<T>(csub<T>(a1, a3));
    a0 = cadd<T>(t0, t2);
    a2 = csub<T>(t0, t2);
    a1 = cadd<T>(t1, t3);
    a3 = csub<T>(t1, t3);
}

// 4-point DFT whose last input is zero.
template <typename T>
__device__ __forceinline__ void dft4_z(c2<T> &a0, c2<T> &a1, c2<T> &a2, c2<T> &a3) {
    const c2<T> t0 = cadd<T>(a0, a2), t1 = csub<T>(a0, a2);
    const c2<T> t3 = cmul_mi<T>(a1);
    a0 = cadd<T>(t0, a1);
    a2 = csub<T>(t0, a1);
    a3 = csub<T>(t1, t3);
    a1 = cadd<T>(t1, t3);
}

// 16-point forward DFT in registers, n = 4a + b, k = c + 4d: 4-point DFTs over a, twiddles
// W16^(b c), 4-point DFTs over b.  On return A[k] is held in v[4 (k % 4) + k / 4].  Z4: the
// inputs v[12..15] are zero (their values are not read).
template <typename T, bool Z4 = false>
__device__ __forceinline__ void dft16(c2<T> *v) {
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, h = (T)0.70710678118654752440;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if constexpr (Z4) dft4_z<T>(v[b], v[4 + b], v[8 + b], v[12 + b]);
        else dft4<T>(v[b], v[4 + b], v[8 + b], v[12 + b]);
    }
    // v[4c + b] *= W16^(b c)
    v[5] = cmul<T>(v[5], mk<T>(c1, -s1));    // b1 c1: W^1
    v[6] = cmul<T>(v[6], mk<T>(h, -h));      // b2 c1: W^2
    v[7] = cmul<T>(v[7], mk<T>(s1, -c1));    // b3 c1: W^3
    v[9] = cmul<T>(v[9], mk<T>(h, -h));      // b1 c2: W^2
    v[10] = cmul_mi<T>(v[10]);               // b2 c2: W^4 = -i
    v[11] = cmul<T>(v[11], mk<T>(-h, -h));   // b3 c2: W^6
    v[13] = cmul<T>(v[13], mk<T>(s1, -c1));  // b1 c3: W^3
    v[14] = cmul<T>(v[14], mk<T>(-h, -h));   // b2 c3: W^6
    v[15] = cmul<T>(v[15], mk<T>(-c1, s1));  // b3 c3: W^9
#pragma unroll
    for (int c = 0; c < 4; ++c) dft4<T>(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
}

// 256-point FFT held by 16 lanes (lane t = threadIdx.x % 16 of the group), n = 16 n1 + n2,
// k = k1 + 16 k2: lane t holds x[16 n1 + t] in v[n1]; 16-point DFTs over n1, twiddles
// W256^(t k1) from the N_FFT-entry table (stride N_FFT / 256), transpose through `sc`
// (16 x 17 padded), 16-point DFTs over n2.  On return lane t holds X[t + 16 k2] in
// v[4 (k2 % 4) + k2 / 4].  A group never straddles a wavefront and `sc` is private to the
// group, so the transpose needs wave-level ordering only (LDS operations of one wavefront
// execute in issue order); every lane of the wave calls it.
// `pre` (applied when `has_pre`) multiplies every stage-1 output of the lane: the per-lane part
// of a residue-class input twiddle, folded into the W256 twiddles.
// Stage 1 of the 256-point FFT below: 16-point DFTs over n1, then the twiddles (and `pre`).
template <typename T, bool Z4 = false>
__device__ __forceinline__ void fft256_stage1(c2<T> *v, int t, const c2<T> *tw, int tw_stride, bool has_pre,
                                              c2<T> pre) {
    dft16<T, Z4>(v);
    // pre * W256^(t k1) by recurrence from W256^t (FP32 rounding grows to ~1e-6 by k1 = 15)
    const c2<T> w1 = tw[t * tw_stride];
    c2<T> wk = has_pre ? cmul<T>(pre, w1) : w1;
    if (has_pre) v[0] = cmul<T>(v[0], pre);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) {
        const int pos = 4 * (k1 & 3) + (k1 >> 2);
        v[pos] = cmul<T>(v[pos], wk);
        wk = cmul<T>(wk, w1);
    }
}

template <typename T>
__device__ __forceinline__ void fft256_lanes(c2<T> *v, int t, c2<T> *sc, const c2<T> *tw, int tw_stride,
                                             bool on, bool has_pre = false, c2<T> pre = c2<T>{}) {
    if (on) {
        fft256_stage1<T>(v, t, tw, tw_stride, has_pre, pre);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) sc[k1 * 17 + t] = v[4 * (k1 & 3) + (k1 >> 2)];
    }
    wave_sync();
    if (on) {
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) v[n2] = sc[t * 17 + n2];
        dft16<T>(v);
    }
    wave_sync();
}

// The same FFT with half the scratch: the transpose moves the real parts, then the imaginary
// parts, through a 16 x 17 float array.  A lane has written all its real parts before it
// overwrites them with the transposed ones, so no extra registers are needed.
template <bool Z4>
__device__ __forceinline__ void fft256_lanes_half(float2 *v, int t, float *sc, const float2 *tw, int tw_stride,
                                                  bool on, bool has_pre, float2 pre) {
    if (on) {
        fft256_stage1<float, Z4>(v, t, tw, tw_stride, has_pre, pre);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) sc[k1 * 17 + t] = v[4 * (k1 & 3) + (k1 >> 2)].x;
    }
    wave_sync();
    if (on) {
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) v[n2].x = sc[t * 17 + n2];
    }
    wave_sync();  // every lane's reads of the real parts precede the writes below
    if (on) {
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) sc[k1 * 17 + t] = v[4 * (k1 & 3) + (k1 >> 2)].y;
    }
    wave_sync();
    if (on) {
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) v[n2].y = sc[t * 17 + n2];
        dft16<float>(v);
    }
    wave_sync();
}


// Spectra of 256-point segments (n_s = 256, distinct output bins): one 16-lane group per
// (template, detector, segment), 8 groups per 128-thread workgroup.  For each residue class p:
// twiddle the zero-padded segment by exp(-2 pi i p s / N_FFT), FFT in registers, and write the
// decimated bins kbar = m P + p with Phi_in and 1 / (sigma sqrt N_K).
template <typename T>
__device__ __forceinline__ void spectra16_body(const BandDev &B, const c2<T> *y, c2<T> *F, int bx, int tb) {
    __shared__ c2<T> sc_all[8 * 16 * 17];
    const int grp = threadIdx.x >> 4, t = threadIdx.x & 15;
    const int w = bx * 8 + grp;
    const bool on = w < B.n_work;
    const int entry = on ? B.work[w] : 0;
    const int det = entry / B.n_seg;
    const int K = entry - det * B.n_seg;
    const int64_t nr = (int64_t)B.n_seg * B.n_k;
    const c2<T> *ys = y + ((size_t)tb * B.Q + det) * nr + (size_t)K * B.n_k;
    const c2<T> *tw = twiddles<T>(B);
    const int rb_mod = mod_fft(B, (int64_t)K * B.n_k);
    const T scale = on ? (T)B.segw[entry].scale : (T)0;
    c2<T> *Fo = F + (((size_t)tb * B.Q + det) * B.n_seg + K) * B.n_f;
    c2<T> *sc = sc_all + grp * 16 * 17;
    for (int p = 0; p < B.P; ++p) {
        c2<T> v[16];
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
            const int sidx = 16 * n1 + t;
            c2<T> x = (on && sidx < B.n_k) ? ys[sidx] : mk<T>((T)0, (T)0);
            v[n1] = p ? cmul<T>(x, tw[p * sidx]) : x;
        }
        fft256_lanes<T>(v, t, sc, tw, B.n_fft >> 8, on);
        if (on) {
#pragma unroll
            for (int k2 = 0; k2 < 16; ++k2) {
                const int kb = (t + 16 * k2) * B.P + p;
                const int i = B.bin_pos[kb];
                if (i < 0) continue;
                const int ph = mod_fft(B, (int64_t)kb * rb_mod);
                Fo[i] = cscale<T>(cmul<T>(v[4 * (k2 & 3) + (k2 >> 2)], tw[ph]), scale);
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3)))
k_spectra16(BandDev B, const c2<T> *y, c2<T> *F) {
    spectra16_body<T>(B, y, F, blockIdx.x, blockIdx.y);
}

// Spectra + pair sum for 256-point segments (split precision, distinct bins): one wavefront =
// one template x one chunk of segments [K0, K1) (plus R halo segments before K0).  Each step
// transforms the next S = 4 / Q segments that take part in some pair (a compacted list; wholly
// idle segments are skipped) of every detector, one 16-lane group per
// (segment, detector), into an LDS ring of R + S decimated spectra, then accumulates each
// bin's pair sum for the step's segments in the same order as k_pairs.  The segment spectra
// never leave LDS and the workgroup is a single wavefront, so no step needs a block barrier;
// one partial per (template, chunk, bin) is written.
constexpr int kSpairMaxRounds = 8;  // bins per lane: n_f <= 64 * kSpairMaxRounds (NR: 3 or 8)

struct SpairLayout {
    int S, slots, cand;
    size_t off_ring, off_list, off_meta, off_flag, off_slotk, off_pos, off_dec, total;
};

// cand = candidate pairs per step: S segments x Q detectors x ring slots x Q.
__host__ __device__ inline SpairLayout spair_layout(int Q, int n_f, int R, int n_fft) {
    SpairLayout L;
    L.S = 4 / Q < 1 ? 1 : 4 / Q;
    L.slots = R + L.S;
    L.cand = L.S * Q * L.slots * Q;
    size_t o = 4 * 16 * 17 * sizeof(float);  // transpose scratch of the 4 groups (one component at a time)
    L.off_ring = o;
    o += (size_t)L.slots * Q * (n_f + 1) * sizeof(float2);
    o = (o + 15) & ~(size_t)15;
    L.off_list = o;
    o += (size_t)(L.cand + 1) * 16;  // count, then (ring offset 1, ring offset 2, weight, pad)
    L.off_meta = o;
    o += (size_t)L.slots * Q * 16;   // (hat a, hat b) of the spectrum in each ring slot
    L.off_flag = o;
    o += (size_t)L.slots * Q;
    o = (o + 15) & ~(size_t)15;
    L.off_slotk = o;                  // segment held by each ring slot, -1 if none
    o += (size_t)L.slots * sizeof(int);
    o = (o + 15) & ~(size_t)15;
    L.off_pos = o;                    // ring column of FFT output (p, k2, t), n_f if unused
    o += (size_t)n_fft * sizeof(int16_t);
    o = (o + 15) & ~(size_t)15;
    L.off_dec = o;                    // decoded pair candidates (cand_decode)
    o += (size_t)L.cand * sizeof(unsigned);
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// Pair candidate cd of a step = (s2, Xc, j, Y) in mixed radix (S, Q, slots, Q), packed one
// byte each (Y lowest); Q <= 4 and slots < 256.
__device__ __forceinline__ unsigned cand_decode(int cd, int Q, int slots) {
    const int Y = cd % Q, j = (cd / Q) % slots, Xc = (cd / (Q * slots)) % Q, s2 = cd / (Q * slots * Q);
    return (unsigned)Y | ((unsigned)j << 8) | ((unsigned)Xc << 16) | ((unsigned)s2 << 24);
}

template <int NR, bool Z4>
__device__ __forceinline__ void spectra_pairs_body(const BandDev &B, const float2 *y, double *part, int k_chunk,
                                                   int n_chunks, int c, int tb) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int Q = B.Q, n_f = B.n_f, n_k = B.n_k, P = B.P;
    const SpairLayout Ly = spair_layout(Q, n_f, B.R, B.n_fft);
    float2 *ring = reinterpret_cast<float2 *>(smem + Ly.off_ring);
    int4 *lst = reinterpret_cast<int4 *>(smem + Ly.off_list);
    double2 *meta = reinterpret_cast<double2 *>(smem + Ly.off_meta);
    uint8_t *flag = smem + Ly.off_flag;
    int *slotk = reinterpret_cast<int *>(smem + Ly.off_slotk);
    int16_t *opos = reinterpret_cast<int16_t *>(smem + Ly.off_pos);
    unsigned *ldec = reinterpret_cast<unsigned *>(smem + Ly.off_dec);
    const int lane = threadIdx.x;
    const int grp = lane >> 4, t = lane & 15;
    const int K0 = c * k_chunk;
    const int K1 = min(B.n_seg, K0 + k_chunk);
    const int Kh = max(0, K0 - B.R);
    const int S = Ly.S, slots = Ly.slots;
    const int64_t nr = (int64_t)B.n_seg * n_k;
    const float2 *tw = B.tw32;
    const bool cross = (B.pairs & 1) != 0, same = (B.pairs & 2) != 0;
    float *sc = reinterpret_cast<float *>(smem) + grp * 16 * 17;
    const int sd = grp / Q, X = grp - sd * Q;  // this group's (segment in step, detector)
    const bool used = sd < S;                  // Q = 3: the fourth group idles
    const int n_f1 = n_f + 1;                  // ring rows hold a dummy entry for unused outputs
    const float2 *ybase = y + ((size_t)tb * Q + (used ? X : 0)) * nr;

    // FFT output (p, k2, lane t) holds kbar = (t + 16 k2) P + p; its ring column
    for (int e = lane; e < B.n_fft; e += 64) {
        const int tt = e & 15, k2 = (e >> 4) & 15, pp = e >> 8;
        const int i = B.bin_pos[(tt + 16 * k2) * P + pp];
        opos[e] = (int16_t)(i >= 0 ? B.bin_col[i] : n_f);
    }
    for (int e = lane; e < slots * Q; e += 64) flag[e] = 0;
    for (int e = lane; e < slots; e += 64) slotk[e] = -1;
    for (int e = lane; e < Ly.cand; e += 64) ldec[e] = cand_decode(e, Q, slots);
    // the steps visit only segments where some detector takes part in a pair: the band's sorted
    // list seg_any, entries [lo, hi) for the chunk with its halo [Kh, K1)
    auto lower = [&](int key) {
        int a = 0, b = B.n_seg_any;
        while (a < b) {
            const int m = (a + b) >> 1;
            if (B.seg_any[m] < key) a = m + 1;
            else b = m;
        }
        return a;
    };
    const int lo = lower(Kh), hi = lower(K1);
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    const int rounds = (n_f + 63) >> 6;

    int slot_b = 0;  // ring slot of the step's first entry
    // this group's samples for the next step, loaded while the current step's pairs are summed
    float2 yv[16];
    // unconditional loads (no branches); a group without a segment reads the band's 256 zero
    // samples.  N_K > 128, so rows 16 n1 + t < 128 are always data; of the next 4 rows (the
    // last 4 of the 12 nonzero ones when Z4) a lane keeps the samples below N_K: samples past
    // N_K belong to the next segment or, after the last one, to the workspace's tail pad
    auto load_y = [&](int e) {
        const bool in = used && e < hi;
        const float2 *ysn = (in ? ybase + (size_t)B.seg_any[e] * n_k : B.zero256) + t;
        constexpr int kFull = Z4 ? 8 : 12, kRows = Z4 ? 12 : 16;
#pragma unroll
        for (int n1 = 0; n1 < kFull; ++n1) yv[n1] = ysn[16 * n1];
#pragma unroll
        for (int n1 = kFull; n1 < kRows; ++n1) {
            const float2 v = ysn[16 * n1];
            const bool keep = 16 * n1 + t < n_k;
            yv[n1] = make_float2(keep ? v.x : 0.f, keep ? v.y : 0.f);
        }
    };
    load_y(lo + sd);
    wave_sync();
    for (int eb = lo; eb < hi; eb += S) {
        const int ns = min(S, hi - eb);
        const bool mine = used && sd < ns;
        const int K = mine ? B.seg_any[eb + sd] : 0;
        const bool on = mine && B.seg_work[X * B.n_seg + K] >= 0;
        int myslot = slot_b + sd;
        if (myslot >= slots) myslot -= slots;
        if (mine && t == 0) {
            // weights with the spectrum normalisation 1 / (sigma sqrt N_K) folded in
            const SegWeight sw = B.segw[X * B.n_seg + K];
            flag[myslot * Q + X] = on ? 1 : 0;
            meta[myslot * Q + X] = make_double2(sw.ahat * sw.scale, sw.bhat * sw.scale);
            if (X == 0) slotk[myslot] = K;
        }
        float2 *Fo = ring + ((size_t)myslot * Q + X) * n_f1;
        for (int p = 0; p < P; ++p) {
            // residue class p: x_p[16 n1 + t] = y[16 n1 + t] W^(16 p n1) W^(p t), W = exp(-2 pi i / N);
            // W^(16 p n1) is uniform over lanes (16 p n1 < 256 P = N needs no reduction), W^(p t)
            // folds into the stage-1 twiddles
            float2 v[16];
            const int tstride = 16 * p;
#pragma unroll
            for (int n1 = 0; n1 < (Z4 ? 12 : 16); ++n1) v[n1] = p ? cmul<float>(yv[n1], tw[tstride * n1]) : yv[n1];
            fft256_lanes_half<Z4>(v, t, sc, tw, B.n_fft >> 8, on, p != 0, tw[p * t]);
            if (on) {
                // the spectrum without Phi_in and normalisation: both enter the pair sum (the
                // normalisation through the weights, Phi_in as the lag phase of each pair)
                const int16_t *op = opos + p * 256 + t;
#pragma unroll
                for (int k2 = 0; k2 < 16; ++k2) Fo[op[16 * k2]] = v[4 * (k2 & 3) + (k2 >> 2)];
            }
        }
        load_y(eb + sd + S);
        wave_sync();
        // pair list of the step, compacted with a ballot: step entry s2 (segment Kc, detector
        // Xc) with the spectrum of ring slot j (segment Kj, detector Y), dl = Kc - Kj: lags
        // 0 < dl <= R for any detector the pair kinds allow, dl = 0 (the entry itself) for
        // Y > Xc across detectors; both spectra present, Kc inside the chunk
        int ne = 0;
        for (int c0 = 0; c0 < Ly.cand; c0 += 64) {
            const int cd = c0 + lane;
            bool valid = false;
            int o1 = 0, o2 = 0, dl_c = 0;
            float W = 0.f;
            if (cd < Ly.cand) {
                // candidate index -> (s2, Xc, j, Y), decoded once per workgroup into LDS
                const unsigned dec = ldec[cd];
                const int Y = (int)(dec & 255u), j = (int)((dec >> 8) & 255u);
                const int Xc = (int)((dec >> 16) & 255u), s2 = (int)(dec >> 24);
                if (s2 < ns) {
                    int slot = slot_b + s2;
                    if (slot >= slots) slot -= slots;
                    const int Kc = slotk[slot], Kj = slotk[j];
                    const int dl = Kc - Kj;
                    const bool inc = (Kj >= 0 && Kc >= K0) &&
                                     ((dl > 0 && dl <= B.R) ? ((Y != Xc) ? cross : same)
                                                            : (dl == 0 && j == slot && cross && Y > Xc));
                    if (inc && flag[slot * Q + Xc] && flag[j * Q + Y]) {
                        valid = true;
                        const double2 wk = meta[slot * Q + Xc], wl = meta[j * Q + Y];
                        W = (float)(wk.x * wl.x + wk.y * wl.y);
                        o1 = (slot * Q + Xc) * n_f1;
                        o2 = (j * Q + Y) * n_f1;
                        dl_c = dl;
                    }
                }
            }
            const uint64_t m = __ballot(valid);
            if (valid) lst[ne + __popcll(m & ((1ull << lane) - 1ull))] = make_int4(o1, o2, __float_as_int(W), dl_c);
            ne += __popcll(m);
        }
        wave_sync();
        float st[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) st[r] = 0.f;
        for (int e = 0; e < ne; ++e) {
            const int4 en = lst[e];
            const float W = __int_as_float(en.z);
            if (en.w == 0) {
                // same-time pair: the Phi_in factors cancel
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int i = 64 * r + lane;
                    if (r < rounds && i < n_f) {
                        const float2 f1 = ring[en.x + i], f2 = ring[en.y + i];
                        st[r] = fma(W, f1.x * f2.x + f1.y * f2.y, st[r]);
                    }
                }
            } else {
                // lag dl = K - L: Re(exp(2 pi i kbar dl n_k / N) conj(F~_K) F~_L)
                const float2 *E = B.lagph + (size_t)en.w * n_f;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int i = 64 * r + lane;
                    if (r < rounds && i < n_f) {
                        const float2 f1 = ring[en.x + i], f2 = ring[en.y + i], ph = E[i];
                        const float a = f1.x * f2.x + f1.y * f2.y, b = f1.x * f2.y - f1.y * f2.x;
                        st[r] = fma(W, ph.x * a - ph.y * b, st[r]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] += (double)st[r];
        wave_sync();
        slot_b += S;
        if (slot_b >= slots) slot_b -= slots;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int i = 64 * r + lane;
        if (r < rounds && i < n_f) part[((size_t)tb * n_chunks + c) * n_f + B.col_bin[i]] = acc[r];
    }
}


// ------------------------------------------------------------------ spectra + pair sum, 1024-point segments

// Load of a table entry that is the same for every lane (uniform index into memory the kernel
// does not write), through the constant address space: a scalar load, whose wait does not wait
// for the wavefront's outstanding vector loads.
template <typename T> __device__ __forceinline__ T ld_uniform(const T *p, int i) {
    i = __builtin_amdgcn_readfirstlane(i);
    return ((const __attribute__((address_space(4))) T *)p)[i];
}
__device__ __forceinline__ float2 ld_uniform_f2(const float2 *p, int i) {
    const unsigned long long v = ld_uniform(reinterpret_cast<const unsigned long long *>(p), i);
    return make_float2(__uint_as_float((unsigned)v), __uint_as_float((unsigned)(v >> 32)));
}

// 1024-point forward FFT held by one wavefront: on entry lane l holds x[l + 64 r] in v[r]
// (r < 16), on return X[l + 64 J] in v[J].  Three self-sorting (Stockham) passes of radix 16,
// 16 and 4 run in registers; between passes the values go through `fx` (1024 complex, index i
// stored at i + i / 16 so that the strided accesses of a pass spread over the LDS banks).
// w2[r - 1] = W256^(r (l % 16)) (r = 1..15) and w3[q][r - 1] = W1024^(r (l + 64 q)) (q < 4,
// r = 1..3) are the pass twiddles of this lane, W_n = exp(-2 pi i / n).  Single wavefront:
// the hardware runs its LDS operations in issue order, wave_sync() keeps the compiler's order.
__device__ __forceinline__ void fft1024_wave(float2 *v, float2 *fx, const float2 *w2, const float2 (*w3)[3],
                                             int lane) {
    // pass 1 (radix 16 over r, no twiddles): output k of butterfly j = l goes to 16 l + k
    dft16<float>(v);
#pragma unroll
    for (int k = 0; k < 16; ++k) fx[17 * lane + k] = v[4 * (k & 3) + (k >> 2)];
    wave_sync();
    // pass 2 (sub-transforms of 16): butterfly j = l reads a[l + 64 r], twiddles W256^(r k) with
    // k = l % 16, writes output k2 to 256 (l / 16) + k + 16 k2
    const int g = lane >> 4, k = lane & 15;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = fx[lane + g + 68 * r];
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul<float>(v[r], w2[r - 1]);
    dft16<float>(v);
    wave_sync();
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) fx[272 * g + k + 17 * k2] = v[4 * (k2 & 3) + (k2 >> 2)];
    wave_sync();
    // pass 3 (sub-transforms of 256): butterflies j = l + 64 q read a[j + 256 r], twiddles
    // W1024^(r j), write output r to j + 256 r = l + 64 (q + 4 r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float2 u0 = fx[lane + g + 68 * q], u1 = fx[lane + g + 68 * q + 272], u2 = fx[lane + g + 68 * q + 544],
               u3 = fx[lane + g + 68 * q + 816];
        u1 = cmul<float>(u1, w3[q][0]);
        u2 = cmul<float>(u2, w3[q][1]);
        u3 = cmul<float>(u3, w3[q][2]);
        dft4<float>(u0, u1, u2, u3);
        v[q] = u0;
        v[q + 4] = u1;
        v[q + 8] = u2;
        v[q + 12] = u3;
    }
    wave_sync();
}

// 8-point forward DFT in place, natural order: 4-point DFTs of the even and odd inputs, then
// X[k] = E[k] + W8^k O[k], X[k + 4] = E[k] - W8^k O[k].
template <typename T>
__device__ __forceinline__ void dft8(c2<T> *v) {
    const T h = (T)0.70710678118654752440;
    c2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T>(e0, e1, e2, e3);
    dft4<T>(o0, o1, o2, o3);
    o1 = cmul<T>(o1, mk<T>(h, -h));
    o2 = cmul_mi<T>(o2);
    o3 = cmul<T>(o3, mk<T>(-h, -h));
    v[0] = cadd<T>(e0, o0);
    v[4] = csub<T>(e0, o0);
    v[1] = cadd<T>(e1, o1);
    v[5] = csub<T>(e1, o1);
    v[2] = cadd<T>(e2, o2);
    v[6] = csub<T>(e2, o2);
    v[3] = cadd<T>(e3, o3);
    v[7] = csub<T>(e3, o3);
}

// Pass twiddles of the one-wavefront FFTs (this lane's), W_n = exp(-2 pi i / n), from the
// N-entry table `tw` of W_N (N = N_FFT, a power of two, at least the FFT length):
//   1024 points (radix 16, 16, 4): w2[r - 1] = W256^(r (l % 16)), w3[q][r - 1] = W1024^(r (l + 64 q));
//   512 points (radix 8, 8, 8):    a[r - 1] = W64^(r (l % 8)), b[r - 1] = W512^(r l);
//   256 points (radix 4, 4, 4, 4): a[r - 1] = W16^(r (l % 4)), b[r - 1] = W64^(r (l % 16)),
//                                  c[r - 1] = W256^(r l).
template <int NS> struct WaveTw;
template <> struct WaveTw<1024> {
    float2 w2[15], w3[4][3];
    __device__ __forceinline__ void load(const float2 *tw, int N, int mask, int lane) {
#pragma unroll
        for (int r = 1; r < 16; ++r) w2[r - 1] = tw[(r * (lane & 15) * (N >> 8)) & mask];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 1; r < 4; ++r) w3[q][r - 1] = tw[(r * (lane + 64 * q) * (N >> 10)) & mask];
    }
};
template <> struct WaveTw<512> {
    float2 a[7], b[7];
    __device__ __forceinline__ void load(const float2 *tw, int N, int mask, int lane) {
#pragma unroll
        for (int r = 1; r < 8; ++r) {
            a[r - 1] = tw[(r * (lane & 7) * (N >> 6)) & mask];
            b[r - 1] = tw[(r * lane * (N >> 9)) & mask];
        }
    }
};
template <> struct WaveTw<256> {
    float2 a[3], b[3], c[3];
    __device__ __forceinline__ void load(const float2 *tw, int N, int mask, int lane) {
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            a[r - 1] = tw[(r * (lane & 3) * (N >> 4)) & mask];
            b[r - 1] = tw[(r * (lane & 15) * (N >> 6)) & mask];
            c[r - 1] = tw[(r * lane * (N >> 8)) & mask];
        }
    }
};

// NS-point forward FFT held by one wavefront (V = NS / 64 values a lane): on entry lane l holds
// x[l + 64 r] in v[r], on return X[l + 64 J] in v[J].  Self-sorting (Stockham) passes; a pass
// of radix V with stride Ns has butterfly j = l read a[l + 64 r], twiddle input r by
// W_(V Ns)^(r (l % Ns)) and write output r to (l / Ns) V Ns + l % Ns + r Ns; the last pass
// (Ns = 64) writes X[l + 64 r] straight to v[r].  Between passes the values go through `fx`,
// index i stored at i + i / V (the padding spreads the strided accesses over the LDS banks).
// 1024 points use fft1024_wave (radix 16, 16, 4).  Single wavefront: wave_sync() orders the
// LDS accesses for the compiler, the hardware runs them in issue order.
template <int NS>
__device__ __forceinline__ void fft_wave(float2 *v, float2 *fx, const WaveTw<NS> &t, int lane);

template <>
__device__ __forceinline__ void fft_wave<1024>(float2 *v, float2 *fx, const WaveTw<1024> &t, int lane) {
    fft1024_wave(v, fx, t.w2, t.w3, lane);
}

template <>
__device__ __forceinline__ void fft_wave<512>(float2 *v, float2 *fx, const WaveTw<512> &t, int lane) {
    const int g = lane >> 3, k = lane & 7;
    // pass 1 (Ns = 1): output r of butterfly l to 8 l + r
    dft8<float>(v);
#pragma unroll
    for (int r = 0; r < 8; ++r) fx[9 * lane + r] = v[r];
    wave_sync();
    // pass 2 (Ns = 8): output r to 64 (l / 8) + l % 8 + 8 r
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = fx[lane + g + 72 * r];
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul<float>(v[r], t.a[r - 1]);
    dft8<float>(v);
    wave_sync();
#pragma unroll
    for (int r = 0; r < 8; ++r) fx[72 * g + k + 9 * r] = v[r];
    wave_sync();
    // pass 3 (Ns = 64)
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = fx[lane + g + 72 * r];
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul<float>(v[r], t.b[r - 1]);
    dft8<float>(v);
    wave_sync();
}

template <>
__device__ __forceinline__ void fft_wave<256>(float2 *v, float2 *fx, const WaveTw<256> &t, int lane) {
    const int g4 = lane >> 2, k4 = lane & 3, g16 = lane >> 4, k16 = lane & 15;
    // pass 1 (Ns = 1): output r of butterfly l to 4 l + r
    dft4<float>(v[0], v[1], v[2], v[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) fx[5 * lane + r] = v[r];
    wave_sync();
    // pass 2 (Ns = 4): output r to 16 (l / 4) + l % 4 + 4 r
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = fx[lane + g4 + 80 * r];
#pragma unroll
    for (int r = 1; r < 4; ++r) v[r] = cmul<float>(v[r], t.a[r - 1]);
    dft4<float>(v[0], v[1], v[2], v[3]);
    wave_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) fx[20 * g4 + k4 + 5 * r] = v[r];
    wave_sync();
    // pass 3 (Ns = 16): output r to 64 (l / 16) + l % 16 + 16 r
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = fx[lane + g4 + 80 * r];
#pragma unroll
    for (int r = 1; r < 4; ++r) v[r] = cmul<float>(v[r], t.b[r - 1]);
    dft4<float>(v[0], v[1], v[2], v[3]);
    wave_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) fx[80 * g16 + k16 + (k16 >> 2) + 20 * r] = v[r];
    wave_sync();
    // pass 4 (Ns = 64)
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = fx[lane + g4 + 80 * r];
#pragma unroll
    for (int r = 1; r < 4; ++r) v[r] = cmul<float>(v[r], t.c[r - 1]);
    dft4<float>(v[0], v[1], v[2], v[3]);
    wave_sync();
}

// Pair term of segment K for one bin of the spectra + pair-sum kernel: sum over detectors X of
// the products of F_XK's two streams with its partners', the window sums G_Y (the two streams of
// the last R segments: Ga, Gb) of the detectors the pair set joins to X (CROSS: Y != X; SAME:
// Y = X) and, across detectors, the same-time partners Y > X (summed from the last detector
// down).  The streams of X are hat a_X F_X and hat b_X F_X (per-segment weights wa, wb), or with
// per-sample antenna functions (PS) the two transforms fa_X, fb_X themselves.  Gamma^ave:
// Re[conj(a_X) H^a] + Re[conj(b_X) H^b]; Gamma^circ (CIRC): Im[conj(b_X) H^a] - Im[conj(a_X) H^b].
// Every unordered pair enters once.
template <int Q, int U, bool CROSS, bool SAME, bool CIRC, bool PS>
__device__ __forceinline__ float wide_pair_term(const float2 (&fa)[Q], const float2 (&fb)[Q], const float (&wa)[Q],
                                                const float (&wb)[Q], const float2 (&Ga)[Q][U],
                                                const float2 (&Gb)[Q][U], int u) {
    float st = 0.f;
    float2 ta = make_float2(0.f, 0.f), tb = make_float2(0.f, 0.f);  // sum over Y > X of the streams
    // both pair kinds: every detector's window sum joins every X (summed once)
    float2 sa = Ga[0][u], sb = Gb[0][u];
    if constexpr (CROSS && SAME) {
#pragma unroll
        for (int Y = 1; Y < Q; ++Y) {
            sa.x += Ga[Y][u].x; sa.y += Ga[Y][u].y;
            sb.x += Gb[Y][u].x; sb.y += Gb[Y][u].y;
        }
    }
#pragma unroll
    for (int X = Q - 1; X >= 0; --X) {
        float2 ha = make_float2(0.f, 0.f), hb = make_float2(0.f, 0.f);
        if constexpr (CROSS && SAME) {
            ha = sa;
            hb = sb;
        } else {
            bool first = true;
#pragma unroll
            for (int Y = 0; Y < Q; ++Y) {
                if ((Y != X && CROSS) || (Y == X && SAME)) {
                    if (first) {
                        ha = Ga[Y][u];
                        hb = Gb[Y][u];
                    } else {
                        ha.x += Ga[Y][u].x; ha.y += Ga[Y][u].y;
                        hb.x += Gb[Y][u].x; hb.y += Gb[Y][u].y;
                    }
                    first = false;
                }
            }
        }
        if (CROSS && X < Q - 1) {
            ha.x += ta.x; ha.y += ta.y;
            hb.x += tb.x; hb.y += tb.y;
        }
        const float2 a = fa[X], b = PS ? fb[X] : fa[X];
        if constexpr (CIRC) {
            if constexpr (PS) {
                st += (b.x * ha.y - b.y * ha.x) - (a.x * hb.y - a.y * hb.x);
            } else {
                st = fmaf(wb[X], a.x * ha.y - a.y * ha.x, st);
                st = fmaf(-wa[X], a.x * hb.y - a.y * hb.x, st);
            }
        } else {
            if constexpr (PS) {
                st += (a.x * ha.x + a.y * ha.y) + (b.x * hb.x + b.y * hb.y);
            } else {
                st = fmaf(wa[X], a.x * ha.x + a.y * ha.y, st);
                st = fmaf(wb[X], a.x * hb.x + a.y * hb.y, st);
            }
        }
        if constexpr (CROSS) {
            if constexpr (PS) {
                ta.x += a.x; ta.y += a.y;
                tb.x += b.x; tb.y += b.y;
            } else {
                ta.x = fmaf(wa[X], a.x, ta.x); ta.y = fmaf(wa[X], a.y, ta.y);
                tb.x = fmaf(wb[X], a.x, tb.x); tb.y = fmaf(wb[X], a.y, tb.y);
            }
        }
    }
    return st;
}

// Workgroup of the spectra + pair-sum kernel for 256- to 1024-point segments: W wavefronts share
// one spectrum ring; wavefront w transforms the detectors X = w, w + W, ... and sums the pairs
// of the bins (ring columns) w 64 + l + 64 W u.  W = spw_waves(Q) (one wavefront a detector up
// to 3 detectors, two for 4), or one for 256- and 512-point segments whose classes one wavefront
// covers (its short transforms then run back to back, and its barriers cost nothing: 15 %
// faster on the 64-band workload).
__host__ __device__ constexpr int spw_waves(int q) { return q == 4 ? 2 : q; }

// LDS of the spectra + pair-sum kernel for ns-point segments (bytes), with a ring of R + ts
// spectra (the window's R segments and a step's ts new ones).
struct SpwLayout {
    int slots, ncol1;
    size_t off_fx, off_ring, off_pos, total;
};

__host__ __device__ inline SpwLayout spw_layout(int Q, int R, int ncol, int jmax, int ns, int streams, int ts, int w) {
    SpwLayout L;
    L.slots = R + ts;
    L.ncol1 = ncol + 1;  // the last column of a ring row takes FFT outputs that are not output bins
    size_t o = 0;
    L.off_fx = o;  // one FFT exchange buffer per wavefront (ns values, padded)
    o += (size_t)w * (ns + 64) * sizeof(float2);
    L.off_ring = o;
    o += (size_t)L.slots * Q * streams * L.ncol1 * sizeof(float2);
    L.off_pos = o;
    o += (size_t)jmax * 64 * sizeof(int16_t);
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// Segments per step of that kernel (transformed together, then their pair sums in order: one
// pair of barriers a step).  Two for 1024-point segments when the ring's extra slot costs no
// workgroup a CU (LDS of 160 KB a CU; at most 8 / W workgroups of W wavefronts at the kernel's
// ~232 registers) and keeps within 64 KB: 2 % faster on the 240-day workload.  One otherwise,
// and for shorter segments, where two to eight measured 1-10 % slower on the 64-band workload.
__host__ __device__ inline int spw_segs(int Q, int R, int ncol, int jmax, int ns, int streams, int w) {
    if (ns != 1024) return 1;
    const size_t l1 = spw_layout(Q, R, ncol, jmax, ns, streams, 1, w).total;
    const size_t l2 = spw_layout(Q, R, ncol, jmax, ns, streams, 2, w).total;
    const size_t cu = 160 * 1024, wmax = 8 / w;
    const size_t w1 = cu / l1 < wmax ? cu / l1 : wmax, w2 = cu / l2 < wmax ? cu / l2 : wmax;
    return l2 <= 65536 && w2 >= w1 ? 2 : 1;
}

// Spectra + pair sum for NS-point segments, NS = 256, 512 or 1024 (split precision, N_FFT a power
// of two, distinct bins): one workgroup of W wavefronts per (template, residue class p of
// the output bins, chunk [K0, K1) of segments plus R halo segments before it).
//   Spectra: for each segment K that some detector takes part in (the compacted list
//   seg_any) and each detector with data there, the zero-padded segment is multiplied by
//   W_N^(q s), q = p + P m0 (class p, its bins rotated so that the class's output indices
//   m0 .. m0 + span - 1 land on FFT outputs 0 .. span - 1), transformed by fft_wave<NS>, and its
//   class-p bins are written to a ring of R + TS spectra in LDS (TS = spw_segs(...) segments a
//   step).  Each wavefront loads the input of its next transform while it computes the current
//   one.
//   Pair sum: each spectrum is rotated by Phi_in = exp(-2 pi i (kbar r_B mod N) / N) (the phase
//   reference after eq. phi-out-eq, absolute, so a pair's lag phase is the product of its two
//   rotations), then the pairs whose later member is segment K enter: against the window sums
//   G^a_Y, G^b_Y = sum over the last R segments L of hat a_YL F_YL, hat b_YL F_YL (cross pairs:
//   Y != X; same-detector pairs: Y = X) and, across detectors, the same-time partners Y > X.
//   Each unordered pair of the pair set therefore enters once.  The window sums are kept in
//   registers: a spectrum is added after its own step and subtracted when its segment falls R
//   segments behind the next one.  Pair products of a segment are summed in FP32, segments in
//   FP64; one partial per (template, chunk, bin).  Two barriers a step: after the transforms of
//   its TS segments (the ring holds their spectra) and after their pair sums, taken segment by
//   segment (the step's ring slots are free again).
//   Gamma^circ (B.weight): the pair term is (hat b_K hat a_L - hat a_K hat b_L) Im[conj(F_K) F_L],
//   from the same window sums.  ALLP (every ordered pair, autos included): no windows; the
//   partials are the chunk's stream sums G^a = sum hat a_XK F_XK and G^b (4 doubles a bin), which
//   the finishing kernel combines.
// U: bins of a class per lane (class size <= 64 W U); Q: the band's detector count; W: wavefronts.
template <int NS, int U, int Q, bool ALLP, bool PS, int TS, int W>
__device__ __forceinline__ void spectra_wide_body(const BandDev &B, const float2 *__restrict__ y, double *part,
                                                  int k_chunk, int n_chunks, int c, int p, int tb) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int V = NS / 64;  // FFT values a lane
    constexpr int S = PS ? 2 : 1;      // spectra streams per (detector, segment)
    const int n_k = B.n_k, R = B.R, N = B.n_fft, mask = B.nfft_mask;
    const SpwLayout Ly = spw_layout(Q, R, B.wide_ncol, B.wide_jmax, NS, S, TS, W);
    // the wavefront index, uniform within the wavefront (readfirstlane makes that known to the
    // compiler, so that per-wavefront addresses and buffer descriptors stay in scalar registers)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    float2 *fx = reinterpret_cast<float2 *>(smem + Ly.off_fx) + wv * (NS + 64);
    float2 *ring = reinterpret_cast<float2 *>(smem + Ly.off_ring);
    int16_t *opos = reinterpret_cast<int16_t *>(smem + Ly.off_pos);
    const int slots = Ly.slots, ncol1 = Ly.ncol1, jmax = B.wide_jmax;
    const bool cross = (B.pairs & 1) != 0, same = (B.pairs & 2) != 0, circ = B.weight != 0;
    const float2 *tw = B.tw32;
    const int cs = B.class_start[p], n_p = B.class_start[p + 1] - cs;
    const int m0 = B.cls_m0[p];

    // FFT output m' = l + 64 J (J < jmax) of the rotated class: its ring column, or the spare one
    for (int e = threadIdx.x; e < jmax * 64; e += 64 * W) opos[e] = (int16_t)(ncol1 - 1);
    for (int e = threadIdx.x; e < slots * Q * S * ncol1; e += 64 * W) ring[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int col = threadIdx.x; col < n_p; col += 64 * W) {
        const int mm = (B.bin_m[B.col_bin[cs + col]] - m0) & (NS - 1);
        opos[mm] = (int16_t)col;
    }
    __syncthreads();
    // ring column of this lane's FFT outputs l + 64 J (J < jmax), two 16-bit columns a register
    unsigned cpos[(V + 1) / 2];
#pragma unroll
    for (int h = 0; h < (V + 1) / 2; ++h) {
        const int J0 = 2 * h, J1 = 2 * h + 1;
        const unsigned c0 = J0 < jmax ? (unsigned)(uint16_t)opos[lane + 64 * J0] : (unsigned)(ncol1 - 1);
        const unsigned c1 = J1 < jmax ? (unsigned)(uint16_t)opos[lane + 64 * J1] : (unsigned)(ncol1 - 1);
        cpos[h] = c0 | (c1 << 16);
    }
    // this lane's bins: kbar mod N (for Phi_in) and bin index
    int kbc[U], binc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int col = wv * 64 + lane + 64 * W * u;
        binc[u] = col < n_p ? B.col_bin[cs + col] : -1;
        kbc[u] = col < n_p ? B.bin_kb[binc[u]] : 0;
    }
    // pass twiddles and the class's input twiddles W_N^(q s), s = l + 64 r (N is a power of two)
    WaveTw<NS> wtw;
    wtw.load(tw, N, mask, lane);
    float2 win[V];
    const int qrot = (p + B.P * m0) & mask;
#pragma unroll
    for (int r = 0; r < V; ++r) win[r] = tw[(int)(((unsigned)qrot * (unsigned)(lane + 64 * r)) & (unsigned)mask)];

    const int K0 = c * k_chunk;
    const int K1 = min(B.n_seg, K0 + k_chunk);
    const int Kh = ALLP ? K0 : max(0, K0 - R);  // every ordered pair: no halo
    auto lower = [&](int key) {
        int a = 0, b = B.n_seg_any;
        while (a < b) {
            const int m = (a + b) >> 1;
            if (B.seg_any[m] < key) a = m + 1;
            else b = m;
        }
        return a;
    };
    const int lo = lower(Kh), hi = lower(K1);
    const int64_t nr = (int64_t)B.n_seg * n_k;
    const float2 *ybase = y + (size_t)tb * Q * S * nr;
    // this wavefront's transforms of a step: units j = S i + s, detector X = wv + W i (i < NJ;
    // W divides Q, so X < Q), stream s (the series of stream s of detector X: X S + s); each
    // unit's input is loaded while the previous unit is transformed.  Buffer loads with the
    // segment's n_k samples as the buffer range read zero past it (no branches, no zero padding
    // in memory).
    constexpr int NJ = Q / W;
    constexpr int NU = NJ * S;
    float2 nxt[V];
    auto load = [&](int e, int j) {
        const int X = wv + W * (j / S);
        const float2 *ys = ybase + (size_t)(X * S + j % S) * nr + (size_t)ld_uniform(B.seg_any, e) * n_k;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)ys, (short)0, n_k * 8, 0x00020000);
#pragma unroll
        for (int r = 0; r < V; ++r)
            nxt[r] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (lane + 64 * r) * 8, 0, 0));
    };
    if (lo < hi) load(lo, 0);

    float2 Ga[Q][U], Gb[Q][U];
    double acc[U];
    double2 sa[ALLP ? U : 1], sb[ALLP ? U : 1];  // all pairs: the chunk's stream sums
#pragma unroll
    for (int u = 0; u < U; ++u) {
        acc[u] = 0.0;
        if constexpr (ALLP) sa[u] = sb[u] = make_double2(0.0, 0.0);
#pragma unroll
        for (int X = 0; X < Q; ++X) Ga[X][u] = Gb[X][u] = make_float2(0.f, 0.f);
    }
    int head = 0, tail = 0, tail_e = lo;
    const int mode = (cross ? 1 : 0) | (same ? 2 : 0) | (circ ? 4 : 0);
    // steps of up to TS consecutive entries of the segment list: their transforms, one barrier,
    // their pair sums in segment order, one barrier
    for (int e0 = lo; e0 < hi; e0 += TS) {
        const int nts = TS == 1 ? 1 : min(TS, hi - e0);  // uniform
        // this wavefront's transforms of the step's segments; segment e0 + t goes to ring slot
        // head + t (mod slots)
#pragma unroll 1
        for (int t = 0; t < nts; ++t) {
            const int e = e0 + t;
            const int K = ld_uniform(B.seg_any, e);
            const int slot = head + t >= slots ? head + t - slots : head + t;
#pragma unroll
            for (int j = 0; j < NU; ++j) {
                const int X = wv + W * (j / S);
                float2 v[V];
#pragma unroll
                for (int r = 0; r < V; ++r) v[r] = cmul<float>(nxt[r], win[r]);
                // the next unit's input (unconditional: the last segment's last unit reloads its own)
                if (j + 1 < NU) load(e, j + 1);
                else load(min(e + 1, hi - 1), 0);
                float2 *row = ring + (((size_t)slot * Q + X) * S + j % S) * ncol1;
                if (ld_uniform(B.seg_work, X * B.n_seg + K) < 0) {
                    // no data of detector X in K: with per-sample streams the ring row is zeroed
                    // (they carry no weight of their own), else its weights are zero
                    if constexpr (PS) {
#pragma unroll
                        for (int J = 0; J < V; ++J)
                            if (J < jmax) row[(cpos[J >> 1] >> (16 * (J & 1))) & 0xffffu] = make_float2(0.f, 0.f);
                    }
                    continue;
                }
                fft_wave<NS>(v, fx, wtw, lane);
#pragma unroll
                for (int J = 0; J < V; ++J)
                    if (J < jmax) row[(cpos[J >> 1] >> (16 * (J & 1))) & 0xffffu] = v[J];
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int t = 0; t < nts; ++t) {
            const int e = e0 + t;
            const int K = ld_uniform(B.seg_any, e);
            // pair weights of this segment's spectra, zero where detector X has no data in it
            float wa[Q], wb[Q];
#pragma unroll
            for (int X = 0; X < Q; ++X) {
                const float2 w2 = ld_uniform_f2(B.segwf, X * B.n_seg + K);
                wa[X] = w2.x;
                wb[X] = w2.y;
            }
            // Phi_in and the pairs whose later member is segment K
            const unsigned rB = (unsigned)(((int64_t)K * n_k) & mask);
            const bool count_it = K >= K0;
            const float invN = 1.0f / (float)N;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int col = wv * 64 + lane + 64 * W * u;
                if (wv * 64 + 64 * W * u >= n_p) break;  // uniform: no lane of this wavefront has a bin here
                float2 *slot = ring + (size_t)head * Q * S * ncol1 + (col < n_p ? col : ncol1 - 1);
                float2 f[Q], g[Q];  // the segment's spectra (stream a; g: stream b with per-sample streams)
#pragma unroll
                for (int X = 0; X < Q; ++X) {
                    f[X] = slot[X * S * ncol1];
                    if constexpr (PS) g[X] = slot[(X * S + 1) * ncol1];
                }
                const float ph = -(float)(((unsigned)kbc[u] * rB) & (unsigned)mask) * invN;  // revolutions
                const float cph = __builtin_amdgcn_cosf(ph), sph = __builtin_amdgcn_sinf(ph);
#pragma unroll
                for (int X = 0; X < Q; ++X) {
                    f[X] = make_float2(f[X].x * cph - f[X].y * sph, f[X].x * sph + f[X].y * cph);
                    if (col < n_p) slot[X * S * ncol1] = f[X];
                    if constexpr (PS) {
                        g[X] = make_float2(g[X].x * cph - g[X].y * sph, g[X].x * sph + g[X].y * cph);
                        if (col < n_p) slot[(X * S + 1) * ncol1] = g[X];
                    }
                }
                if constexpr (ALLP) {
                    // this segment's share of G^a and G^b: FP32 over the detectors, FP64 over segments
                    float2 ta = make_float2(0.f, 0.f), tb2 = make_float2(0.f, 0.f);
#pragma unroll
                    for (int X = 0; X < Q; ++X) {
                        if constexpr (PS) {
                            ta.x += f[X].x; ta.y += f[X].y;
                            tb2.x += g[X].x; tb2.y += g[X].y;
                        } else {
                            ta.x = fmaf(wa[X], f[X].x, ta.x); ta.y = fmaf(wa[X], f[X].y, ta.y);
                            tb2.x = fmaf(wb[X], f[X].x, tb2.x); tb2.y = fmaf(wb[X], f[X].y, tb2.y);
                        }
                    }
                    sa[u].x += (double)ta.x; sa[u].y += (double)ta.y;
                    sb[u].x += (double)tb2.x; sb[u].y += (double)tb2.y;
                    continue;
                }
                if (count_it) {
                    float st;
                    switch (mode) {  // uniform
                        case 1: st = wide_pair_term<Q, U, true, false, false, PS>(f, g, wa, wb, Ga, Gb, u); break;
                        case 2: st = wide_pair_term<Q, U, false, true, false, PS>(f, g, wa, wb, Ga, Gb, u); break;
                        case 3: st = wide_pair_term<Q, U, true, true, false, PS>(f, g, wa, wb, Ga, Gb, u); break;
                        case 5: st = wide_pair_term<Q, U, true, false, true, PS>(f, g, wa, wb, Ga, Gb, u); break;
                        case 6: st = wide_pair_term<Q, U, false, true, true, PS>(f, g, wa, wb, Ga, Gb, u); break;
                        case 7: st = wide_pair_term<Q, U, true, true, true, PS>(f, g, wa, wb, Ga, Gb, u); break;
                        default: st = 0.f;
                    }
                    acc[u] += (double)st;
                }
#pragma unroll
                for (int X = 0; X < Q; ++X) {
                    if constexpr (PS) {
                        Ga[X][u].x += f[X].x; Ga[X][u].y += f[X].y;
                        Gb[X][u].x += g[X].x; Gb[X][u].y += g[X].y;
                    } else {
                        Ga[X][u].x = fmaf(wa[X], f[X].x, Ga[X][u].x); Ga[X][u].y = fmaf(wa[X], f[X].y, Ga[X][u].y);
                        Gb[X][u].x = fmaf(wb[X], f[X].x, Gb[X][u].x); Gb[X][u].y = fmaf(wb[X], f[X].y, Gb[X][u].y);
                    }
                }
            }
            head = head + 1 == slots ? 0 : head + 1;
            // spectra whose segment is more than R behind the next segment's leave the window
            // sums: the ring holds the entries tail_e .. e; their segments and weights come from
            // the (uniform) segment list and weight table.  A lane reads back only its own columns,
            // which it rotated itself, so no barrier is needed within the step.
            if (!ALLP && e + 1 < hi) {
                const int Kn = ld_uniform(B.seg_any, e + 1);
                while (tail_e <= e) {
                    const int Kt = ld_uniform(B.seg_any, tail_e);
                    if (Kt >= Kn - R) break;
                    float wta[Q], wtb[Q];
#pragma unroll
                    for (int X = 0; X < Q; ++X) {
                        const float2 w2 = ld_uniform_f2(B.segwf, X * B.n_seg + Kt);
                        wta[X] = w2.x;
                        wtb[X] = w2.y;
                    }
                    const float2 *rowt = ring + (size_t)tail * Q * S * ncol1;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (wv * 64 + 64 * W * u >= n_p) break;
                        const int col = wv * 64 + lane + 64 * W * u;
                        const float2 *gp = rowt + (col < n_p ? col : ncol1 - 1);
#pragma unroll
                        for (int X = 0; X < Q; ++X) {
                            const float2 ga = gp[X * S * ncol1];
                            if constexpr (PS) {
                                const float2 gb = gp[(X * S + 1) * ncol1];
                                Ga[X][u].x -= ga.x; Ga[X][u].y -= ga.y;
                                Gb[X][u].x -= gb.x; Gb[X][u].y -= gb.y;
                            } else {
                                Ga[X][u].x = fmaf(-wta[X], ga.x, Ga[X][u].x); Ga[X][u].y = fmaf(-wta[X], ga.y, Ga[X][u].y);
                                Gb[X][u].x = fmaf(-wtb[X], ga.x, Gb[X][u].x); Gb[X][u].y = fmaf(-wtb[X], ga.y, Gb[X][u].y);
                            }
                        }
                    }
                    tail = tail + 1 == slots ? 0 : tail + 1;
                    ++tail_e;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (binc[u] < 0) continue;
        if constexpr (ALLP) {
            double *o = part + (((size_t)tb * n_chunks + c) * B.n_f + binc[u]) * 4;
            o[0] = sa[u].x;
            o[1] = sa[u].y;
            o[2] = sb[u].x;
            o[3] = sb[u].y;
        } else {
            part[((size_t)tb * n_chunks + c) * B.n_f + binc[u]] = acc[u];
        }
    }
}

// The fused kernel keeps the activity bits of a step (S segments x Q detectors) in 64 bits.
__host__ __device__ inline bool Q_ok(const BandDev &B) { return B.Q >= 1 && B.Q * 4 <= 64; }

// PER: samples per thread, n_s / blockDim.x (at most 4 below n_s = 2048, else 8).
// With per-sample antenna weights (B.pw) the segment gives two spectra, of hat a_r y_r and of
// hat b_r y_r (the table's weights carry 1 / (sigma sqrt N_K)); the second is written `plane`
// entries after the first.
template <typename T, int PER>
__device__ __forceinline__ void spectra_body(const BandDev &B, const c2<T> *y, c2<T> *F, int w, int tb,
                                             size_t plane) {
    extern __shared__ __align__(16) unsigned char smem[];
    c2<T> *buf0 = reinterpret_cast<c2<T> *>(smem);
    c2<T> *buf1 = buf0 + B.n_s;
    const int entry = B.work[w];
    const int det = entry / B.n_seg;
    const int K = entry - det * B.n_seg;
    const int64_t nr = (int64_t)B.n_seg * B.n_k;
    const c2<T> *ys = y + ((size_t)tb * B.Q + det) * nr + (size_t)K * B.n_k;
    const c2<T> *tw = twiddles<T>(B);
    const int rb_mod = mod_fft(B, (int64_t)K * B.n_k);
    const bool two = B.pw != nullptr;
    const T scale = two ? (T)1 : (T)B.segw[entry].scale;
    const double2 *pws = two ? B.pw + (size_t)det * nr + (size_t)K * B.n_k : nullptr;
    // The FFT's stage twiddles are all n_s-th roots of unity: a copy of those n_s entries of
    // the N_FFT-entry table in LDS (when it fits beside the two work buffers) replaces the
    // strided gathers from global memory.
    const bool ltw = 3 * (size_t)B.n_s * sizeof(c2<T>) <= 65536;
    c2<T> *twl = buf1 + B.n_s;
    if (ltw) {
        const int st = B.n_fft / B.n_s;
        for (int j = threadIdx.x; j < B.n_s; j += blockDim.x) twl[j] = tw[j * st];
    }
    // input twiddles W^(p s) (W = exp(-2 pi i / N_FFT)) of this thread's samples
    // s = threadIdx.x + r blockDim.x, advanced from class to class by W^s and refreshed from the
    // table every 8 classes (bounding the product's rounding growth)
    constexpr int kPer = PER;
    c2<T> ts[kPer], ws[kPer], yv[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int s = threadIdx.x + r * blockDim.x;
        ws[r] = s < B.n_s ? tw[s] : mk<T>((T)1, (T)0);
    }
    for (int st = 0; st < (two ? 2 : 1); ++st) {
        c2<T> *Fo = F + (size_t)st * plane + (((size_t)tb * B.Q + det) * B.n_seg + K) * B.n_f;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int s = threadIdx.x + r * blockDim.x;
            ts[r] = mk<T>((T)1, (T)0);
            yv[r] = mk<T>((T)0, (T)0);
            if (s < B.n_k) {
                yv[r] = ys[s];
                if (two) {
                    const double2 wv = pws[s];
                    yv[r] = cscale<T>(yv[r], (T)(st ? wv.y : wv.x));
                }
            }
        }
        for (int p = 0; p < B.P; ++p) {
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int s = threadIdx.x + r * blockDim.x;
                if (s < B.n_s) {
                    if (p > 0) ts[r] = (p & 7) == 0 ? tw[mod_fft(B, (int64_t)p * s)] : cmul<T>(ts[r], ws[r]);
                    buf0[s] = p ? cmul<T>(yv[r], ts[r]) : yv[r];
                }
            }
            __syncthreads();
            const c2<T> *res = ltw ? stockham<T>(buf0, buf1, B.n_s, twl, B.n_s, threadIdx.x, blockDim.x)
                                   : stockham<T>(buf0, buf1, B.n_s, tw, B.n_fft, threadIdx.x, blockDim.x);
            // the output bins of class p only
            for (int c = B.class_start[p] + (int)threadIdx.x; c < B.class_start[p + 1]; c += blockDim.x) {
                const int i = B.col_bin[c];
                const int ph = mod_fft(B, (int64_t)B.bin_kb[i] * rb_mod);
                Fo[i] = cscale<T>(cmul<T>(res[B.bin_m[i]], tw[ph]), scale);
            }
            __syncthreads();
        }
    }
}

template <typename T, int PER>
__global__ void __launch_bounds__(256) k_spectra(BandDev B, const c2<T> *y, c2<T> *F, size_t plane) {
    spectra_body<T, PER>(B, y, F, blockIdx.x, blockIdx.y, plane);
}

// ------------------------------------------------------------------ pair sum

// Pair sums in stream form: segment (X, K) contributes the two streams F^a_XK and F^b_XK at
// bin i -- hat a_XK F_XK and hat b_XK F_XK with per-segment weights, or the two spectra of the
// weighted series (B.pw, stored `plane` entries apart).  A pair (K, L) adds
//   Gamma^ave:  Re[conj(F^a_K) F^a_L + conj(F^b_K) F^b_L]
//   Gamma^circ: Im[conj(F^b_K) F^a_L - conj(F^a_K) F^b_L]
// (with per-segment weights (hat a_K hat a_L + hat b_K hat b_L) Re[conj(F_K) F_L] and
// (hat b_K hat a_L - hat a_K hat b_L) Im[conj(F_K) F_L]); both are symmetric in K and L.
template <typename T> struct Streams {
    const c2<T> *F;  // this template's spectra
    size_t plane;    // offset of the b-stream, two-stream form only
    bool two;
    __device__ __forceinline__ void at(const BandDev &B, int el, int i, c2<T> &fa, c2<T> &fb) const {
        const c2<T> g = F[(size_t)el * B.n_f + i];
        if (two) {
            fa = g;
            fb = F[plane + (size_t)el * B.n_f + i];
        } else {
            const T a = (T)B.segw[el].ahat, b = (T)B.segw[el].bhat;
            fa = cscale<T>(g, a);
            fb = cscale<T>(g, b);
        }
    }
};

// Partial rho of one (template, bin, chunk of segments): for each segment K and detector X,
// segment (X, K) against the sum of its partners (Y, L) that precede it -- L in [K - R, K - 1]
// (other detectors if cross pairs, the same detector if same pairs) and L = K with Y > X (cross
// pairs) -- so each unordered pair of the set enters once.  The partner sums over
// L in [K - R, K - 1] are kept per detector as sliding windows of the two streams (add segment
// K - 1, drop K - R - 1), so each spectrum is read twice instead of (R + 1) Q times; inactive
// segments (whose spectra are not computed) never enter.
template <typename T>
__device__ __forceinline__ void pairs_body(const BandDev &B, const c2<T> *F, double *part, int k_chunk, int n_chunks,
                                           int bx, int c, int tb, size_t plane) {
    const int i = bx * blockDim.x + threadIdx.x;
    if (i >= B.n_f) return;
    const bool cross = (B.pairs & 1) != 0, same = (B.pairs & 2) != 0;
    const bool circ = B.weight != 0, two = B.pw != nullptr;
    const Streams<T> S{F + (size_t)tb * B.Q * B.n_seg * B.n_f, plane, two};
    const int Q = B.Q, R = B.R;
    const int K0 = c * k_chunk;
    const int K1 = min(B.n_seg, K0 + k_chunk);
    if (B.allp) {
        // every ordered pair, autos included: the pair sum is a function of the stream sums
        // G^a = sum_XK F^a_XK and G^b (combined by the finishing kernel); this chunk's share
        double ga_x = 0.0, ga_y = 0.0, gb_x = 0.0, gb_y = 0.0;
        for (int K = K0; K < K1; ++K)
            for (int X = 0; X < Q; ++X) {
                const int ek = X * B.n_seg + K;
                if (!B.active[ek]) continue;
                c2<T> fa, fb;
                S.at(B, ek, i, fa, fb);
                ga_x += (double)fa.x;
                ga_y += (double)fa.y;
                gb_x += (double)fb.x;
                gb_y += (double)fb.y;
            }
        double *o = part + (((size_t)tb * n_chunks + c) * B.n_f + i) * 4;
        o[0] = ga_x;
        o[1] = ga_y;
        o[2] = gb_x;
        o[3] = gb_y;
        return;
    }
    // wa[Y], wb[Y]: sum over L in [K - R, K - 1] of F^a_YL and F^b_YL
    c2<T> wa[CCR_MAX_DET_K], wb[CCR_MAX_DET_K];
#pragma unroll
    for (int Y = 0; Y < CCR_MAX_DET_K; ++Y) wa[Y] = wb[Y] = mk<T>((T)0, (T)0);
    auto add = [&](int Y, int L, T sign) {
        const int el = Y * B.n_seg + L;
        if (!B.active[el]) return;
        if (two) {
            c2<T> fa, fb;
            S.at(B, el, i, fa, fb);
            wa[Y] = mk<T>(fma(sign, fa.x, wa[Y].x), fma(sign, fa.y, wa[Y].y));
            wb[Y] = mk<T>(fma(sign, fb.x, wb[Y].x), fma(sign, fb.y, wb[Y].y));
        } else {
            const c2<T> g = S.F[(size_t)el * B.n_f + i];
            const T a = sign * (T)B.segw[el].ahat, b = sign * (T)B.segw[el].bhat;
            wa[Y] = mk<T>(fma(a, g.x, wa[Y].x), fma(a, g.y, wa[Y].y));
            wb[Y] = mk<T>(fma(b, g.x, wb[Y].x), fma(b, g.y, wb[Y].y));
        }
    };
    for (int L = max(0, K0 - R); L < K0; ++L)
#pragma unroll
        for (int Y = 0; Y < CCR_MAX_DET_K; ++Y)
            if (Y < Q) add(Y, L, (T)1);
    double acc = 0.0;
    for (int K = K0; K < K1; ++K) {
        if (R > 0 && K > K0) {
            // slide: segment K - 1 enters, K - 1 - R leaves
#pragma unroll
            for (int Y = 0; Y < CCR_MAX_DET_K; ++Y) {
                if (Y >= Q) continue;
                add(Y, K - 1, (T)1);
                if (K - 1 - R >= 0) add(Y, K - 1 - R, (T)-1);
            }
        }
        for (int X = 0; X < Q; ++X) {
            const int ek = X * B.n_seg + K;
            if (!B.active[ek]) continue;
            c2<T> ga = mk<T>((T)0, (T)0), gb = mk<T>((T)0, (T)0);
#pragma unroll
            for (int Y = 0; Y < CCR_MAX_DET_K; ++Y) {
                if (Y >= Q) continue;
                if (R > 0 && ((Y != X) ? cross : same)) {
                    ga = mk<T>(ga.x + wa[Y].x, ga.y + wa[Y].y);
                    gb = mk<T>(gb.x + wb[Y].x, gb.y + wb[Y].y);
                }
                const int el = Y * B.n_seg + K;
                if (cross && Y > X && B.active[el]) {
                    if (two) {
                        c2<T> fa, fb;
                        S.at(B, el, i, fa, fb);
                        ga = cadd<T>(ga, fa);
                        gb = cadd<T>(gb, fb);
                    } else {
                        const c2<T> g = S.F[(size_t)el * B.n_f + i];
                        const T wa_ = (T)B.segw[el].ahat, wb_ = (T)B.segw[el].bhat;
                        ga = mk<T>(fma(wa_, g.x, ga.x), fma(wa_, g.y, ga.y));
                        gb = mk<T>(fma(wb_, g.x, gb.x), fma(wb_, g.y, gb.y));
                    }
                }
            }
            if (two) {
                c2<T> fa, fb;
                S.at(B, ek, i, fa, fb);
                if (circ)
                    acc += (double)((fb.x * ga.y - fb.y * ga.x) - (fa.x * gb.y - fa.y * gb.x));
                else
                    acc += (double)(fa.x * ga.x + fa.y * ga.y + fb.x * gb.x + fb.y * gb.y);
            } else {
                const c2<T> f = S.F[(size_t)ek * B.n_f + i];
                const T aK = (T)B.segw[ek].ahat, bK = (T)B.segw[ek].bhat;
                if (circ) {
                    // Im[conj(F_K) (hat b_K G^a - hat a_K G^b)]
                    const T hx = bK * ga.x - aK * gb.x, hy = bK * ga.y - aK * gb.y;
                    acc += (double)(f.x * hy - f.y * hx);
                } else {
                    const T hx = aK * ga.x + bK * gb.x, hy = aK * ga.y + bK * gb.y;
                    acc += (double)(f.x * hx + f.y * hy);
                }
            }
        }
    }
    part[((size_t)tb * n_chunks + c) * B.n_f + i] = acc;
}


// ------------------------------------------------------------------ fused path

// Threads per FFT group: n_s / 4 (one radix-4 butterfly each), at most the whole block.
__host__ __device__ inline int fused_group(int n_s) {
    const int q = n_s / 4;
    return q < 1 ? 1 : (q > 256 ? 256 : q);
}

// Input window per (segment, detector) staged in LDS: the taps of every sample of a segment
// lie within n_k + 2D + 2 * margin samples around the segment's centre offset; taps outside
// (never for the workloads here) are read from global memory.
__host__ __device__ inline int fused_margin(int n_k, double dt) {
    return 3 + (int)(4e-4 * 0.5 * (double)n_k);
}

// LDS layout of the fused kernel: per-bin accumulators acc[n_f] (double), per (step segment,
// detector) time-base coefficients and anchor terms, window starts, input windows
// xwin[S][Q][W] (float2), resampled segments ybuf[S][Q][n_s], FFT work buffers [G][2][n_s],
// ring of decimated spectra [R+S][Q][n_f] and its activity flags.
struct FusedLayout {
    int G, S, W, slots;
    size_t off_acc, off_coef, off_ws, off_x, off_y, off_work, off_ring, off_flag, total;
};

__host__ __device__ inline FusedLayout fused_layout(int Q, int n_s, int n_k, int n_f, int R, int D, double dt,
                                                    size_t cs, int S) {
    FusedLayout L;
    L.G = 256 / fused_group(n_s);
    L.S = S;
    L.W = n_k + 2 * D + 2 * fused_margin(n_k, dt) + 1;
    L.slots = R + S;
    size_t o = 0;
    L.off_acc = o;
    o += (size_t)n_f * 8;
    L.off_coef = o;
    o += (size_t)S * Q * (kCheb + 2) * 8;
    L.off_ws = o;
    o += (size_t)S * Q * 8;
    L.off_x = o;
    o += (size_t)S * Q * L.W * 8;
    o = (o + 15) & ~(size_t)15;
    L.off_y = o;
    o += (size_t)S * Q * n_s * cs;
    L.off_work = o;
    o += (size_t)L.G * 2 * n_s * cs;
    L.off_ring = o;
    o += (size_t)L.slots * Q * n_f * cs;
    L.off_flag = o;
    o += (size_t)L.slots * Q;
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// One workgroup = one template x one chunk of segments [K0, K1), processed S segments per step
// (plus the R segments before K0 as a halo): stage the coefficients, anchors and input windows
// of the step's (segment, detector) pairs in LDS with one batch of loads, resample them, FFT
// them (Q P S transforms, G at a time), keep the decimated spectra in a ring of R + S segments,
// and accumulate each bin's pair sum for the chunk's segments in the same order as k_pairs.
// Writes one partial per (template, chunk, bin).
template <typename T, int DT>
__global__ void __launch_bounds__(256) k_fused(BandDev B, const double *coef, const int *seg_work,
                                              double *part, int k_chunk, int n_chunks, int S) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int Q = B.Q, n_s = B.n_s, n_k = B.n_k, n_f = B.n_f;
    const FusedLayout Ly = fused_layout(Q, n_s, n_k, n_f, B.R, B.D, B.dt, sizeof(c2<T>), S);
    double *acc = reinterpret_cast<double *>(smem + Ly.off_acc);
    double *scoef = reinterpret_cast<double *>(smem + Ly.off_coef);   // [S*Q][kCheb + 2]
    int64_t *wstart = reinterpret_cast<int64_t *>(smem + Ly.off_ws);  // [S*Q]
    float2 *xwin = reinterpret_cast<float2 *>(smem + Ly.off_x);       // [S*Q][W]
    c2<T> *ybuf = reinterpret_cast<c2<T> *>(smem + Ly.off_y);
    c2<T> *work = reinterpret_cast<c2<T> *>(smem + Ly.off_work);
    c2<T> *ring = reinterpret_cast<c2<T> *>(smem + Ly.off_ring);
    uint8_t *flag = smem + Ly.off_flag;

    const int c = blockIdx.x;
    const int tb = blockIdx.y;
    const int K0 = c * k_chunk;
    const int K1 = min(B.n_seg, K0 + k_chunk);
    const int Kh = max(0, K0 - B.R);
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int W = Ly.W, slots = Ly.slots;
    const int64_t nr = (int64_t)B.n_seg * n_k;
    const c2<T> *tw = twiddles<T>(B);
    const bool cross = (B.pairs & 1) != 0, same = (B.pairs & 2) != 0;
    const int per = fused_group(n_s);
    const double inv_nk = 1.0 / (double)n_k;  // same expression as k_resample
    const int margin = fused_margin(n_k, B.dt);
    const int D = DT > 0 ? DT : B.D;

    for (int i = tid; i < n_f; i += nth) acc[i] = 0.0;
    for (int i = tid; i < slots * Q; i += nth) flag[i] = 0;
    for (int i = tid; i < S * Q * n_s; i += nth) ybuf[i] = mk<T>((T)0, (T)0);
    __syncthreads();

    for (int Kb = Kh; Kb < K1; Kb += S) {
        const int ns = min(S, K1 - Kb);  // segments in this step
        // activity bits of the step: bit (sd * Q + X)
        uint64_t act = 0;
        for (int sd = 0; sd < ns; ++sd)
            for (int X = 0; X < Q; ++X)
                if (B.active[X * B.n_seg + Kb + sd]) act |= 1ull << (sd * Q + X);
        // phase A: coefficients, anchor terms, window starts
        if (tid < ns * Q) {
            const int sd = tid / Q, X = tid - sd * Q;
            const int K = Kb + sd;
            double *sc = scoef + (size_t)tid * (kCheb + 2);
            const int ws = seg_work[X * B.n_seg + K];
            int64_t start = 0;
            if (ws >= 0) {
                const double *cf = coef + ((size_t)tb * B.n_work + ws) * kCheb;
                double cl[kCheb];
#pragma unroll
                for (int k = 0; k < kCheb; ++k) {
                    cl[k] = cf[k];
                    sc[k] = cl[k];
                }
                const Anchor &an = B.anchors[X * B.n_seg + K];
                sc[kCheb] = an.D_a;
                sc[kCheb + 1] = an.psi_a;
                // eta at the segment centre: sum_k c_k T_k(0), T_k(0) = cos(k pi / 2)
                double em = cl[0];
#pragma unroll
                for (int k = 2; k < kCheb; k += 2) em += (k & 2) ? -cl[k] : cl[k];
                const int64_t kc = (int64_t)floor((em - an.D_a) * B.inv_dt + 0.5);
                start = (int64_t)K * n_k + kc - D - margin;
            }
            wstart[tid] = start;
            flag[((Kb + sd) % slots) * Q + X] = (ws >= 0) ? 1 : 0;
        }
        __syncthreads();
        // phase B: input windows (out-of-range samples read zero)
        for (int idx = tid; idx < ns * Q * W; idx += nth) {
            const int e = idx / W;
            if (!((act >> e) & 1ull)) continue;
            const int X = e % Q;
            const int64_t j = wstart[e] + (idx - e * W);
            xwin[idx] = (j >= 0 && j < B.n) ? B.x[(size_t)X * B.n + j] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        // phase C: resample into ybuf (the zero padding beyond n_k was written at the start)
        for (int idx = tid; idx < ns * Q * n_k; idx += nth) {
            const int e = idx / n_k;
            const int s = idx - e * n_k;
            if (!((act >> e) & 1ull)) continue;
            const int sd = e / Q, X = e - sd * Q;
            const int K = Kb + sd;
            const int64_t r = (int64_t)K * n_k + s;
            c2<T> v = mk<T>((T)0, (T)0);
            if (B.mask[(size_t)X * nr + r]) {
                const double *sc = scoef + (size_t)e * (kCheb + 2);
                Anchor an;
                an.D_a = sc[kCheb];
                an.psi_a = sc[kCheb + 1];
                int64_t jstar;
                double dc, psi;
                sample_time(sc, (double)(2 * s - n_k) * inv_nk, an, B.inv_dt, B.f_het, r, jstar, dc, psi);
                const int64_t off = jstar - wstart[e];
                c2<T> accv;
                if (off - D >= 0 && off + D < W) {
                    accv = B.window == 0 ? interpolate_window<T, DT, 0>(B, xwin + (size_t)e * W, (int)off, dc)
                                         : interpolate_window<T, DT, 1>(B, xwin + (size_t)e * W, (int)off, dc);
                } else {
                    T cw[2 * (DT > 0 ? DT : 0) + 1];
                    if constexpr (DT > 0) {
                        if (B.window == 0) load_signed_window<T, DT>(B, cw);
                    }
                    accv = B.window == 0 ? interpolate<T, DT, 0>(B, B.x + (size_t)X * B.n, jstar, dc, cw)
                                         : interpolate<T, DT, 1>(B, B.x + (size_t)X * B.n, jstar, dc, cw);
                }
                T cs_, sn_;
                sincos_rev<T>(psi, sn_, cs_);
                v = mk<T>(cs_ * accv.x - sn_ * accv.y, sn_ * accv.x + cs_ * accv.y);
            }
            ybuf[e * n_s + s] = v;
        }
        __syncthreads();
        // phase D: FFT jobs (segment, detector, residue), G at a time
        const int jobs = ns * Q * B.P;
        const int grp = tid / per, g0 = tid - grp * per;
        for (int jb = 0; jb < jobs; jb += Ly.G) {
            const int job = jb + grp;
            const int e = job / B.P;
            const bool on = grp < Ly.G && job < jobs && ((act >> e) & 1ull);
            const int p = on ? job - e * B.P : 0;
            const int sd = on ? e / Q : 0, X = on ? e - sd * Q : 0;
            const int K = Kb + sd;
            c2<T> *w0 = work + (size_t)(grp < Ly.G ? grp : 0) * 2 * n_s;
            c2<T> *w1 = w0 + n_s;
            if (on) {
                for (int s2 = g0; s2 < n_s; s2 += per) {
                    c2<T> v = ybuf[e * n_s + s2];
                    if (p && s2 < n_k) v = cmul<T>(v, tw[p * s2]);
                    w0[s2] = v;
                }
            }
            __syncthreads();
            const c2<T> *res = stockham<T>(w0, w1, n_s, tw, B.n_fft, g0, per, on);
            if (on) {
                const int rb_mod = mod_fft(B, (int64_t)K * n_k);
                const T scale = (T)B.segw[X * B.n_seg + K].scale;
                c2<T> *Fo = ring + ((size_t)(K % slots) * Q + X) * n_f;
                for (int c = B.class_start[p] + g0; c < B.class_start[p + 1]; c += per) {
                    const int i = B.col_bin[c];
                    const int ph = mod_fft(B, (int64_t)B.bin_kb[i] * rb_mod);
                    Fo[i] = cscale<T>(cmul<T>(res[B.bin_m[i]], tw[ph]), scale);
                }
            }
            __syncthreads();
        }
        // phase E: pair sums of the step's segments that belong to the chunk, in order
        for (int i = tid; i < n_f; i += nth) {
            double a = acc[i];
            for (int sd = 0; sd < ns; ++sd) {
                const int K = Kb + sd;
                if (K < K0) continue;
                const int slot = K % slots;
                for (int X = 0; X < Q; ++X) {
                    if (!flag[slot * Q + X]) continue;
                    c2<T> ga = mk<T>((T)0, (T)0), gb = mk<T>((T)0, (T)0);
                    for (int L = max(0, K - B.R); L <= K; ++L) {
                        const int sl = L % slots;
                        for (int Y = 0; Y < Q; ++Y) {
                            const bool inc = (L < K) ? ((Y != X) ? cross : same) : (cross && Y > X);
                            if (!inc || !flag[sl * Q + Y]) continue;
                            const c2<T> g = ring[((size_t)sl * Q + Y) * n_f + i];
                            const SegWeight &w = B.segw[Y * B.n_seg + L];
                            const T wa = (T)w.ahat, wb = (T)w.bhat;
                            ga.x += wa * g.x; ga.y += wa * g.y;
                            gb.x += wb * g.x; gb.y += wb * g.y;
                        }
                    }
                    const c2<T> f = ring[((size_t)slot * Q + X) * n_f + i];
                    const SegWeight &wk = B.segw[X * B.n_seg + K];
                    const T aK = (T)wk.ahat, bK = (T)wk.bhat;
                    const T hx = aK * ga.x + bK * gb.x, hy = aK * ga.y + bK * gb.y;
                    a += (double)(f.x * hx + f.y * hy);
                }
            }
            acc[i] = a;
        }
        __syncthreads();
    }
    for (int i = tid; i < n_f; i += nth) part[((size_t)tb * n_chunks + c) * n_f + i] = acc[i];
}

// allp = 0: rho = factor x the sum of the chunk partials.  allp = 1 (every ordered pair): the
// partials are chunk sums of the streams (G^a, G^b, 4 doubles); rho = factor x
// (|G^a|^2 + |G^b|^2) for Gamma^ave, factor x 2 Im[conj(G^b) G^a] for Gamma^circ.
__device__ __forceinline__ void finish_body(int n_f, int n_tmpl, const double *part, int n_chunks, double factor,
                                            void *out, int out_fp64, int bx, int t, int allp = 0, int circ = 0) {
    const int i = bx * blockDim.x + threadIdx.x;
    if (i >= n_f || t >= n_tmpl) return;
    double s = 0.0;
    if (allp) {
        double g[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < n_chunks; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) g[j] += part[(((size_t)t * n_chunks + c) * n_f + i) * 4 + j];
        s = circ ? 2.0 * (g[2] * g[1] - g[3] * g[0]) : g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3];
    } else {
        for (int c = 0; c < n_chunks; ++c) s += part[((size_t)t * n_chunks + c) * n_f + i];
    }
    s *= factor;
    if (out_fp64)
        static_cast<double *>(out)[(size_t)t * n_f + i] = s;
    else
        static_cast<float *>(out)[(size_t)t * n_f + i] = (float)s;
}

__global__ void k_finish(int n_f, int n_tmpl, const double *part, int n_chunks, double factor,
                         void *out, int out_fp64) {
    finish_body(n_f, n_tmpl, part, n_chunks, factor, out, out_fp64, blockIdx.x, blockIdx.y);
}

__global__ void k_zero(uint32_t *p, size_t n_words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n_words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ------------------------------------------------------------------ batched launches

// Pointers loaded from a device table are generic, and loads through generic pointers are
// slower than global loads (and hold more registers).  as_global() re-derives such a pointer
// from `base`, a kernel argument in global memory, as base + (p - base): the same 64-bit
// address, now known to the compiler to be global memory.
typedef __attribute__((address_space(1))) char gchar;
template <typename T> __device__ __forceinline__ T *as_global(T *p, const gchar *base) {
    const gchar *q = base + ((const char *)p - (const char *)base);
    return (T *)q;
}

// A copy of a band descriptor from the device band table with every pointer re-derived as a
// global-memory pointer.
__device__ __forceinline__ BandDev global_view(const BandDev &b, const void *base_) {
    const gchar *base = (const gchar *)base_;
    BandDev g = b;
    g.x = as_global(b.x, base);
    g.mask = as_global(b.mask, base);
    g.anchors = as_global(b.anchors, base);
    g.earth = as_global(b.earth, base);
    g.win64 = as_global(b.win64, base);
    g.win32 = as_global(b.win32, base);
    g.cheb_x = as_global(b.cheb_x, base);
    g.mono = as_global(b.mono, base);
    g.tw64 = as_global(b.tw64, base);
    g.tw32 = as_global(b.tw32, base);
    g.bin_m = as_global(b.bin_m, base);
    g.bin_p = as_global(b.bin_p, base);
    g.bin_kb = as_global(b.bin_kb, base);
    g.bin_pos = as_global(b.bin_pos, base);
    g.segw = as_global(b.segw, base);
    g.active = as_global(b.active, base);
    g.work = as_global(b.work, base);
    g.seg_work = as_global(b.seg_work, base);
    g.tmpl = as_global(b.tmpl, base);
    g.lagph = as_global(b.lagph, base);
    g.seg_any = as_global(b.seg_any, base);
    g.col_bin = as_global(b.col_bin, base);
    g.class_start = as_global(b.class_start, base);
    g.zero256 = as_global(b.zero256, base);
    g.bin_col = as_global(b.bin_col, base);
    g.farrow = as_global(b.farrow, base);
    g.cls_m0 = as_global(b.cls_m0, base);
    if (b.pw) g.pw = as_global(b.pw, base);
    return g;
}

// The item owning block b of a stage: the last item whose first block is <= b.
__device__ __forceinline__ int find_item(const WorkItem *__restrict__ items, int n_items, int stage, int b) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first[stage] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NN, bool SHORT>
__global__ void __launch_bounds__(tb_entries(NN) * NN)
k_timebase_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
             double *__restrict__ coef) {
    const WorkItem &it = items[find_item(items, n_items, kStTimebase, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStTimebase], gx = it.gx[kStTimebase];
    timebase_body<NN, SHORT>(B, B.tmpl + (size_t)it.tmpl_off * kTmplStride, coef + it.coef_off, l % gx, l / gx);
}

template <typename T, int DT, int WIN, int NC>
__global__ void __launch_bounds__(64)
k_resample_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
             const double *__restrict__ coef, c2<T> *__restrict__ y) {
    const WorkItem &it = items[find_item(items, n_items, kStResample, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    // consecutive workgroups take the template tiles of one segment entry, so that they run
    // together and read the segment's input (and mask) through L2 instead of once per tile
    const int l = blockIdx.x - it.first[kStResample];
    const int tiles = (it.n_tmpl + kResTemplates - 1) / kResTemplates;
    const int t0 = (l % tiles) * kResTemplates;
    resample_body<T, DT, WIN, NC>(B, coef + it.coef_off, y + it.y_off, l / tiles, t0,
                                  min(it.n_tmpl, t0 + kResTemplates));
}

template <int NC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_resample_far_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
                 const double *__restrict__ coef, float2 *__restrict__ y) {
    const WorkItem &it = items[find_item(items, n_items, kStResample, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    // A segment's template tiles are consecutive virtual indices v, and consecutive v run on
    // one XCD: the dispatcher hands workgroups to the 8 XCDs in turn (block b on XCD b mod 8),
    // so the item's blocks l with equal l mod 8 (one XCD) take the contiguous range of v
    // starting at (l mod 8) full / 8, in order; the table slice of a segment is then fetched
    // into that XCD's L2 once for all its tiles.  Blocks past the last multiple of 8 keep v = l.
    const int l = blockIdx.x - it.first[kStResample];
    const int tiles = (it.n_tmpl + kFarTemplates - 1) / kFarTemplates;
    const int full = (B.n_work * tiles) & ~7;  // the item's blocks: n_work segment entries x tiles
    const int v = l < full ? (l & 7) * (full >> 3) + (l >> 3) : l;
    const int t0 = (v % tiles) * kFarTemplates;
    resample_far_body<NC>(B, coef + it.coef_off, y + it.y_off, v / tiles, t0, min(it.n_tmpl, t0 + kFarTemplates));
}

template <int NR, bool Z4>
__global__ void __launch_bounds__(64)
k_spectra_pairs_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
                  const float2 *__restrict__ y, double *__restrict__ part) {
    const WorkItem &it = items[find_item(items, n_items, kStSpectra, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStSpectra], gx = it.gx[kStSpectra];
    spectra_pairs_body<NR, Z4>(B, y + it.y_off, part + it.part_off, it.k_chunk, it.n_chunks, l % gx, l / gx);
}

// Blocks of an item: n_tmpl x n_chunks groups of P workgroups (one per residue class).  The
// dispatcher hands workgroups to the 8 XCDs in turn, so block l runs on XCD l mod 8: the P class
// workgroups of one (template, chunk) group are given indices with equal l mod 8, which puts
// them on one XCD, where they read the group's resampled series through that XCD's L2.
template <int NS, int U, int Q, bool ALLP, bool PS, int TS, int W>
__global__ void __launch_bounds__(64 * W)
k_spectra_wide_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
                 const float2 *__restrict__ y, double *__restrict__ part) {
    const WorkItem &it = items[find_item(items, n_items, kStSpectra, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStSpectra];
    const int P = B.P, G = it.n_tmpl * it.n_chunks;
    const int full = (G >> 3) * 8 * P;
    int g, p;
    if (l < full) {
        const int r = l >> 3;
        p = r % P;
        g = (r / P) * 8 + (l & 7);
    } else {
        g = (G >> 3) * 8 + (l - full) / P;
        p = (l - full) % P;
    }
    spectra_wide_body<NS, U, Q, ALLP, PS, TS, W>(B, y + it.y_off, part + it.part_off, it.k_chunk, it.n_chunks, g % it.n_chunks, p,
                                   g / it.n_chunks);
}

template <typename T>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3)))
k_spectra16_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
              const c2<T> *__restrict__ y, c2<T> *__restrict__ F) {
    const WorkItem &it = items[find_item(items, n_items, kStSpectra, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStSpectra], gx = it.gx[kStSpectra];
    spectra16_body<T>(B, y + it.y_off, F + it.F_off, l % gx, l / gx);
}

template <typename T, int PER>
__global__ void __launch_bounds__(256)
k_spectra_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
            const c2<T> *__restrict__ y, c2<T> *__restrict__ F) {
    const WorkItem &it = items[find_item(items, n_items, kStSpectra, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStSpectra], gx = it.gx[kStSpectra];
    const size_t plane = (size_t)it.n_tmpl * B.Q * B.n_seg * B.n_f;
    spectra_body<T, PER>(B, y + it.y_off, F + it.F_off, l % gx, l / gx, plane);
}

template <typename T>
__global__ void __launch_bounds__(kPairsThreads)
k_pairs_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
          const c2<T> *__restrict__ F, double *__restrict__ part) {
    const WorkItem &it = items[find_item(items, n_items, kStPairs, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStPairs], gx = it.gx[kStPairs];
    const int bx = l % gx, rest = l / gx;
    const size_t plane = (size_t)it.n_tmpl * B.Q * B.n_seg * B.n_f;
    pairs_body<T>(B, F + it.F_off, part + it.part_off, it.k_chunk, it.n_chunks, bx, rest % it.n_chunks,
                  rest / it.n_chunks, plane);
}

__global__ void __launch_bounds__(kFinishThreads)
k_finish_m(const BandDev *__restrict__ bands, const WorkItem *__restrict__ items, int n_items,
           const double *__restrict__ part) {
    const WorkItem &it = items[find_item(items, n_items, kStFinish, blockIdx.x)];
    const BandDev B = global_view(bands[it.band], bands);
    const int l = blockIdx.x - it.first[kStFinish], gx = it.gx[kStFinish];
    finish_body(B.n_f, it.n_tmpl, part + it.part_off, it.n_chunks, it.factor, as_global(it.out, (const gchar *)part),
                it.out_fp64, l % gx, l / gx, B.allp, B.weight);
}

}  // namespace

hipError_t launch_timebase(const BandDev &B, const double *d_tmpl, int n_tmpl, double *coef,
                           hipStream_t stream) {
    if (B.n_work == 0 || n_tmpl == 0) return hipSuccess;
    constexpr int E = tb_entries(kCheb);
    dim3 grid((B.n_work + E - 1) / E, n_tmpl), block(E * kCheb);
    hipLaunchKernelGGL(k_timebase, grid, block, 0, stream, B, d_tmpl, coef);
    return hipGetLastError();
}

template <typename T, int DT>
static void launch_resample_t(const BandDev &B, const double *coef, int n_tmpl, void *y, hipStream_t stream) {
    dim3 grid((unsigned)B.n_work, n_tmpl), block(64);
    if (B.window == 0)
        hipLaunchKernelGGL((k_resample<T, DT, 0>), grid, block, 0, stream, B, coef, (c2<T> *)y);
    else
        hipLaunchKernelGGL((k_resample<T, DT, 1>), grid, block, 0, stream, B, coef, (c2<T> *)y);
}

hipError_t launch_resample(const BandDev &B, const double *coef, int n_tmpl, bool fp64, void *y,
                           hipStream_t stream) {
    if (B.n_work == 0 || n_tmpl == 0) return hipSuccess;
    if (!fp64 && B.farrow) {
        dim3 grid((unsigned)B.n_work, (n_tmpl + kFarTemplates - 1) / kFarTemplates);
        hipLaunchKernelGGL(k_resample_far, grid, dim3(256), 0, stream, B, coef, (float2 *)y, n_tmpl);
    } else if (fp64) {
        if (B.D == 8) launch_resample_t<double, 8>(B, coef, n_tmpl, y, stream);
        else launch_resample_t<double, 0>(B, coef, n_tmpl, y, stream);
    } else {
        if (B.D == 8) launch_resample_t<float, 8>(B, coef, n_tmpl, y, stream);
        else launch_resample_t<float, 0>(B, coef, n_tmpl, y, stream);
    }
    return hipGetLastError();
}

hipError_t launch_farrow_table(const float2 *x, int64_t n, int Q, int D, const double *A, int64_t far_len,
                               float2 *tab, hipStream_t stream) {
    if (Q == 0 || far_len == 0) return hipSuccess;
    dim3 grid((unsigned)((far_len + 255) / 256), Q);
    hipLaunchKernelGGL(k_farrow_table, grid, dim3(256), 0, stream, x, n, D, A, far_len, tab);
    return hipGetLastError();
}

hipError_t launch_spectra(const BandDev &B, int n_tmpl, bool fp64, const void *y, void *F,
                          hipStream_t stream) {
    if (B.n_work == 0 || n_tmpl == 0) return hipSuccess;
    if (!fp64 && B.n_s == 256 && B.bins_unique && !B.pw) {
        dim3 grid((B.n_work + 7) / 8, n_tmpl), block(128);
        hipLaunchKernelGGL(k_spectra16<float>, grid, block, 0, stream, B, (const float2 *)y, (float2 *)F);
        return hipGetLastError();
    }
    dim3 grid(B.n_work, n_tmpl), block(spectra_threads(B.n_s));
    const size_t plane = (size_t)n_tmpl * B.Q * B.n_seg * B.n_f;
    const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
    const size_t lds = (3 * (size_t)B.n_s * cs <= 65536 ? 3 : 2) * (size_t)B.n_s * cs;  // + stage twiddles
    const bool p8 = B.n_s > 4 * spectra_threads(B.n_s);
    if (fp64 && p8)
        hipLaunchKernelGGL((k_spectra<double, 8>), grid, block, lds, stream, B, (const double2 *)y, (double2 *)F, plane);
    else if (fp64)
        hipLaunchKernelGGL((k_spectra<double, 4>), grid, block, lds, stream, B, (const double2 *)y, (double2 *)F, plane);
    else if (p8)
        hipLaunchKernelGGL((k_spectra<float, 8>), grid, block, lds, stream, B, (const float2 *)y, (float2 *)F, plane);
    else
        hipLaunchKernelGGL((k_spectra<float, 4>), grid, block, lds, stream, B, (const float2 *)y, (float2 *)F, plane);
    return hipGetLastError();
}

bool spectra_pairs_ok(const BandDev &B, bool fp64, size_t limit) {
    const SpairLayout L = spair_layout(B.Q, B.n_f, B.R, B.n_fft);
    return !fp64 && B.n_s == 256 && B.n_k > 128 && B.bins_unique && B.Q <= 4 && B.n_f <= 64 * kSpairMaxRounds &&
           L.slots < 256 && L.total <= limit;
}



// Segments per step: the largest of 4, 2, 1 whose LDS footprint fits in `limit` bytes
// (0 if even one segment per step does not fit).
int fused_steps(const BandDev &B, bool fp64, size_t limit) {
    const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
    for (int S = 4; S >= 1; S /= 2)
        if (Q_ok(B) && fused_layout(B.Q, B.n_s, B.n_k, B.n_f, B.R, B.D, B.dt, cs, S).total <= limit) return S;
    return 0;
}

size_t fused_lds_bytes(const BandDev &B, bool fp64, int S) {
    return fused_layout(B.Q, B.n_s, B.n_k, B.n_f, B.R, B.D, B.dt, fp64 ? sizeof(double2) : sizeof(float2), S).total;
}

hipError_t launch_fused(const BandDev &B, const double *coef, int n_tmpl, bool fp64, double *part,
                        int k_chunk, int n_chunks, int S, hipStream_t stream) {
    if (n_tmpl == 0) return hipSuccess;
    if (S < 1 || !Q_ok(B)) return hipErrorInvalidValue;
    dim3 grid(n_chunks, n_tmpl), block(256);
    const size_t lds = fused_lds_bytes(B, fp64, S);
    if (fp64) {
        if (B.D == 8)
            hipLaunchKernelGGL((k_fused<double, 8>), grid, block, lds, stream, B, coef, B.seg_work, part, k_chunk, n_chunks, S);
        else
            hipLaunchKernelGGL((k_fused<double, 0>), grid, block, lds, stream, B, coef, B.seg_work, part, k_chunk, n_chunks, S);
    } else {
        if (B.D == 8)
            hipLaunchKernelGGL((k_fused<float, 8>), grid, block, lds, stream, B, coef, B.seg_work, part, k_chunk, n_chunks, S);
        else
            hipLaunchKernelGGL((k_fused<float, 0>), grid, block, lds, stream, B, coef, B.seg_work, part, k_chunk, n_chunks, S);
    }
    return hipGetLastError();
}

hipError_t launch_finish(const BandDev &B, int n_tmpl, const double *part, int n_chunks,
                         double factor, void *out, bool out_fp64, hipStream_t stream) {
    if (n_tmpl == 0) return hipSuccess;
    dim3 grid((B.n_f + 255) / 256, n_tmpl), block(256);
    hipLaunchKernelGGL(k_finish, grid, block, 0, stream, B.n_f, n_tmpl, part, n_chunks, factor, out,
                       out_fp64 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_time_samples(const BandDev &B, const double *coef, int det, int k0, int n, double *eta,
                               double *psi, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_time_samples, dim3(n), dim3(64), 0, stream, B, coef, det, k0, n, eta, psi);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    const unsigned blocks = (unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, stream, (uint32_t *)p, words);
    return hipGetLastError();
}


// ------------------------------------------------------------------ batched launchers

size_t spectra_pairs_lds(const BandDev &B) { return spair_layout(B.Q, B.n_f, B.R, B.n_fft).total; }

// Bin columns of a class per lane: 1, 2 or 4, and 8 with one detector (one wavefront a
// workgroup, so that a class of up to 512 bins still fits).
static int spw_max_cols(int q) { return q == 1 ? 8 : 4; }

int spectra_wide_waves(const BandDev &B) {
    return B.n_s <= 512 && B.wide_ncol <= spw_max_cols(B.Q) * 64 ? 1 : spw_waves(B.Q);
}

int spectra_wide_segs(const BandDev &B) {
    return spw_segs(B.Q, B.R, B.wide_ncol, B.wide_jmax, B.n_s, B.ps2 ? 2 : 1, spectra_wide_waves(B));
}

size_t spectra_wide_lds(const BandDev &B) {
    return spw_layout(B.Q, B.R, B.wide_ncol, B.wide_jmax, B.n_s, B.ps2 ? 2 : 1, spectra_wide_segs(B),
                      spectra_wide_waves(B))
        .total;
}

int spectra_wide_cols(const BandDev &B) {
    const int per = 64 * spectra_wide_waves(B);  // bin columns a workgroup covers per U
    return B.wide_ncol <= per ? 1 : (B.wide_ncol <= 2 * per ? 2 : (B.wide_ncol <= 4 * per ? 4 : 8));
}

bool spectra_wide_ok(const BandDev &B, bool fp64, size_t limit) {
    return !fp64 && (B.n_s == 1024 || B.n_s == 512 || B.n_s == 256) && B.nfft_mask != 0 && B.bins_unique &&
           B.Q >= 1 && B.Q <= 4 && B.wide_ncol <= spw_max_cols(B.Q) * 64 * spw_waves(B.Q) && B.wide_jmax >= 1 &&
           B.wide_jmax <= B.n_s / 64 &&
           B.cls_m0 != nullptr && spectra_wide_lds(B) <= limit;
}

int spectra_pairs_rounds(const BandDev &B) { return B.n_f <= 64 * 3 ? 3 : kSpairMaxRounds; }

int spectra_threads(int n_s) { return n_s / 4 >= 256 ? 256 : (n_s / 4 < 64 ? 64 : n_s / 4); }

template <int NN>
static void launch_timebase_m_t(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool short_series,
                                double *coef, hipStream_t stream) {
    if (short_series)
        hipLaunchKernelGGL((k_timebase_m<NN, true>), dim3(blocks), dim3(tb_entries(NN) * NN), 0, stream, bands, items,
                           n_items, coef);
    else
        hipLaunchKernelGGL((k_timebase_m<NN, false>), dim3(blocks), dim3(tb_entries(NN) * NN), 0, stream, bands, items,
                           n_items, coef);
}

hipError_t launch_timebase_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int n_cheb,
                             bool short_series, double *coef, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    if (n_cheb == kCheb) launch_timebase_m_t<kCheb>(bands, items, n_items, blocks, short_series, coef, stream);
    else if (n_cheb == kChebSplit) launch_timebase_m_t<kChebSplit>(bands, items, n_items, blocks, short_series, coef, stream);
    else if (n_cheb == kChebSplitMin)
        launch_timebase_m_t<kChebSplitMin>(bands, items, n_items, blocks, short_series, coef, stream);
    else launch_timebase_m_t<kChebSplitLow>(bands, items, n_items, blocks, short_series, coef, stream);
    return hipGetLastError();
}

template <typename T, int DT, int NC>
static void launch_resample_m_t(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int window,
                                const double *coef, void *y, hipStream_t stream) {
    if (window == 0)
        hipLaunchKernelGGL((k_resample_m<T, DT, 0, NC>), dim3(blocks), dim3(64), 0, stream, bands, items, n_items,
                           coef, (c2<T> *)y);
    else
        hipLaunchKernelGGL((k_resample_m<T, DT, 1, NC>), dim3(blocks), dim3(64), 0, stream, bands, items, n_items,
                           coef, (c2<T> *)y);
}

hipError_t launch_resample_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool fp64, int D,
                             int window, int n_cheb, bool farrow, const double *coef, void *y, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    if (farrow && !fp64) {
        if (n_cheb == kChebSplitLow)
            hipLaunchKernelGGL(k_resample_far_m<kChebSplitLow>, dim3(blocks), dim3(256), 0, stream, bands, items,
                               n_items, coef, (float2 *)y);
        else if (n_cheb == kChebSplitMin)
            hipLaunchKernelGGL(k_resample_far_m<kChebSplitMin>, dim3(blocks), dim3(256), 0, stream, bands, items,
                               n_items, coef, (float2 *)y);
        else if (n_cheb == kChebSplit)
            hipLaunchKernelGGL(k_resample_far_m<kChebSplit>, dim3(blocks), dim3(256), 0, stream, bands, items,
                               n_items, coef, (float2 *)y);
        else
            hipLaunchKernelGGL(k_resample_far_m<kCheb>, dim3(blocks), dim3(256), 0, stream, bands, items, n_items,
                               coef, (float2 *)y);
    } else if (fp64) {
        if (D == 8) launch_resample_m_t<double, 8, kCheb>(bands, items, n_items, blocks, window, coef, y, stream);
        else launch_resample_m_t<double, 0, kCheb>(bands, items, n_items, blocks, window, coef, y, stream);
    } else if (n_cheb == kChebSplit) {
        if (D == 8) launch_resample_m_t<float, 8, kChebSplit>(bands, items, n_items, blocks, window, coef, y, stream);
        else launch_resample_m_t<float, 0, kChebSplit>(bands, items, n_items, blocks, window, coef, y, stream);
    } else if (n_cheb == kChebSplitMin) {
        if (D == 8)
            launch_resample_m_t<float, 8, kChebSplitMin>(bands, items, n_items, blocks, window, coef, y, stream);
        else launch_resample_m_t<float, 0, kChebSplitMin>(bands, items, n_items, blocks, window, coef, y, stream);
    } else if (n_cheb == kChebSplitLow) {
        if (D == 8)
            launch_resample_m_t<float, 8, kChebSplitLow>(bands, items, n_items, blocks, window, coef, y, stream);
        else launch_resample_m_t<float, 0, kChebSplitLow>(bands, items, n_items, blocks, window, coef, y, stream);
    } else {
        if (D == 8) launch_resample_m_t<float, 8, kCheb>(bands, items, n_items, blocks, window, coef, y, stream);
        else launch_resample_m_t<float, 0, kCheb>(bands, items, n_items, blocks, window, coef, y, stream);
    }
    return hipGetLastError();
}

template <int NR>
static void launch_spectra_pairs_m_t(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool z4,
                                     size_t lds, const void *y, double *part, hipStream_t stream) {
    if (z4)
        hipLaunchKernelGGL((k_spectra_pairs_m<NR, true>), dim3(blocks), dim3(64), lds, stream, bands, items, n_items,
                           (const float2 *)y, part);
    else
        hipLaunchKernelGGL((k_spectra_pairs_m<NR, false>), dim3(blocks), dim3(64), lds, stream, bands, items,
                           n_items, (const float2 *)y, part);
}

hipError_t launch_spectra_pairs_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int rounds,
                                  bool z4, size_t lds, const void *y, double *part, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    if (rounds == 3) launch_spectra_pairs_m_t<3>(bands, items, n_items, blocks, z4, lds, y, part, stream);
    else launch_spectra_pairs_m_t<kSpairMaxRounds>(bands, items, n_items, blocks, z4, lds, y, part, stream);
    return hipGetLastError();
}

template <int NS, bool ALLP, bool PS, int TS, bool ONE>
static void launch_spectra_wide_u(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int cols,
                                  int q, size_t lds, const void *y, double *part, hipStream_t stream) {
#define CCR_WIDE(U_, Q_)                                                                                              \
    hipLaunchKernelGGL((k_spectra_wide_m<NS, U_, Q_, ALLP, PS, TS, ONE ? 1 : spw_waves(Q_)>),                       \
                       dim3(blocks), dim3(64 * (ONE ? 1 : spw_waves(Q_))), lds, stream, bands, items, n_items,       \
                       (const float2 *)y, part)
#define CCR_WIDE_Q(U_)          \
    do {                        \
        if (q == 1) CCR_WIDE(U_, 1); \
        else if (q == 2) CCR_WIDE(U_, 2); \
        else if (q == 3) CCR_WIDE(U_, 3); \
        else CCR_WIDE(U_, 4);   \
    } while (0)
    if (cols <= 1) CCR_WIDE_Q(1);
    else if (cols <= 2) CCR_WIDE_Q(2);
    else if (cols <= 4) CCR_WIDE_Q(4);
    else if (q == 1) CCR_WIDE(8, 1);  // spectra_wide_ok admits 8 columns a lane for one detector only
#undef CCR_WIDE_Q
#undef CCR_WIDE
}

template <int NS, int TS, bool ONE>
static void launch_spectra_wide_f(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int cols,
                                  int q, bool allp, bool ps, size_t lds, const void *y, double *part,
                                  hipStream_t stream) {
    if (allp && ps) launch_spectra_wide_u<NS, true, true, TS, ONE>(bands, items, n_items, blocks, cols, q, lds, y, part, stream);
    else if (allp) launch_spectra_wide_u<NS, true, false, TS, ONE>(bands, items, n_items, blocks, cols, q, lds, y, part, stream);
    else if (ps) launch_spectra_wide_u<NS, false, true, TS, ONE>(bands, items, n_items, blocks, cols, q, lds, y, part, stream);
    else launch_spectra_wide_u<NS, false, false, TS, ONE>(bands, items, n_items, blocks, cols, q, lds, y, part, stream);
}

hipError_t launch_spectra_wide_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int ns,
                                 int cols, int q, int ts, int waves, bool allp, bool ps, size_t lds, const void *y,
                                 double *part, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    const bool one = waves == 1 && q > 1;  // one detector has one wavefront either way
    if (ns == 1024 && ts == 2 && !one) launch_spectra_wide_f<1024, 2, false>(bands, items, n_items, blocks, cols, q, allp, ps, lds, y, part, stream);
    else if (ns == 1024 && ts == 1 && !one) launch_spectra_wide_f<1024, 1, false>(bands, items, n_items, blocks, cols, q, allp, ps, lds, y, part, stream);
    else if (ns == 512 && ts == 1 && !one) launch_spectra_wide_f<512, 1, false>(bands, items, n_items, blocks, cols, q, allp, ps, lds, y, part, stream);
    else if (ns == 256 && ts == 1 && !one) launch_spectra_wide_f<256, 1, false>(bands, items, n_items, blocks, cols, q, allp, ps, lds, y, part, stream);
    else if (ns == 256 && ts == 1 && one) launch_spectra_wide_f<256, 1, true>(bands, items, n_items, blocks, cols, q, allp, ps, lds, y, part, stream);
    else if (ns == 512 && ts == 1 && one) launch_spectra_wide_f<512, 1, true>(bands, items, n_items, blocks, cols, q, allp, ps, lds, y, part, stream);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_spectra_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool fp64,
                            bool reg16, int threads, int n_s, const void *y, void *F, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    if (reg16 && !fp64) {
        hipLaunchKernelGGL(k_spectra16_m<float>, dim3(blocks), dim3(16 * kSpec16Groups), 0, stream, bands, items,
                           n_items, (const float2 *)y, (float2 *)F);
        return hipGetLastError();
    }
    const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
    const size_t lds = (3 * (size_t)n_s * cs <= 65536 ? 3 : 2) * (size_t)n_s * cs;  // + stage twiddles
    const bool p8 = n_s > 4 * threads;
    if (fp64 && p8)
        hipLaunchKernelGGL((k_spectra_m<double, 8>), dim3(blocks), dim3(threads), lds, stream, bands, items, n_items,
                           (const double2 *)y, (double2 *)F);
    else if (fp64)
        hipLaunchKernelGGL((k_spectra_m<double, 4>), dim3(blocks), dim3(threads), lds, stream, bands, items, n_items,
                           (const double2 *)y, (double2 *)F);
    else if (p8)
        hipLaunchKernelGGL((k_spectra_m<float, 8>), dim3(blocks), dim3(threads), lds, stream, bands, items, n_items,
                           (const float2 *)y, (float2 *)F);
    else
        hipLaunchKernelGGL((k_spectra_m<float, 4>), dim3(blocks), dim3(threads), lds, stream, bands, items, n_items,
                           (const float2 *)y, (float2 *)F);
    return hipGetLastError();
}

hipError_t launch_pairs_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool fp64,
                          const void *F, double *part, hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_pairs_m<double>, dim3(blocks), dim3(kPairsThreads), 0, stream, bands, items, n_items,
                           (const double2 *)F, part);
    else
        hipLaunchKernelGGL(k_pairs_m<float>, dim3(blocks), dim3(kPairsThreads), 0, stream, bands, items, n_items,
                           (const float2 *)F, part);
    return hipGetLastError();
}

hipError_t launch_finish_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, const double *part,
                           hipStream_t stream) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish_m, dim3(blocks), dim3(kFinishThreads), 0, stream, bands, items, n_items, part);
    return hipGetLastError();
}

// ------------------------------------------------------------------ SFT front end
// Heterodyned, downsampled series from SFT bins (App. B): for SFT K and output sample j
// (dt' = T_sft / N'),
//   x(K, j) = S_K E_j sum_{l=-h}^{N'-1-h} z_{K, k_h + l} exp(2 pi i l j / N'),
// the inverse transform of the N' bins around the heterodyne bin k_h (h = floor(N'/2)), with
// E_j = exp(-2 pi i nu_r j / N') / T_sft the remainder nu_r = f_h T_sft - k_h of the heterodyne
// frequency off the bin grid, and S_K = exp(-2 pi i f_h t_K) the phase that makes consecutive
// SFTs continue one another (t_K the SFT's start).  One 256-thread workgroup per SFT: the SFT's
// bins (FP32 as given) and, for N' <= kSftTwLds, the N' roots of unity (FP64) sit in LDS; each
// thread sums outputs j, j + 256, ... in FP64 with the root index (l j) mod N' stepped exactly in
// integers.  Output complex64.
namespace {
constexpr int kSftThreads = 256;
constexpr int kSftTwLds = 2048;

__global__ void __launch_bounds__(kSftThreads)
k_sft_series(const float2 *__restrict__ z, int64_t n_bins, int64_t off, int n_out, int h,
             const double2 *__restrict__ roots, const double2 *__restrict__ ej, const double2 *__restrict__ sk,
             const uint8_t *__restrict__ present, float2 *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *tw = reinterpret_cast<double2 *>(smem);
    const bool lds_tw = n_out <= kSftTwLds;
    float2 *zb = reinterpret_cast<float2 *>(smem + (lds_tw ? (size_t)n_out * sizeof(double2) : 0));
    const int K = blockIdx.x;
    float2 *xo = x + (size_t)K * n_out;
    if (present && !present[K]) {
        for (int j = threadIdx.x; j < n_out; j += kSftThreads) xo[j] = make_float2(0.f, 0.f);
        return;
    }
    const float2 *zk = z + (size_t)K * n_bins + off;
    for (int m = threadIdx.x; m < n_out; m += kSftThreads) {
        zb[m] = zk[m];
        if (lds_tw) tw[m] = roots[m];
    }
    __syncthreads();
    const double2 *T = lds_tw ? tw : roots;
    const double2 s = sk[K];
    for (int j = threadIdx.x; j < n_out; j += kSftThreads) {
        // index of l = -h: (-h j) mod N'
        int idx = (int)((int64_t)(n_out - h) * j % n_out);
        double re = 0.0, im = 0.0;
        for (int m = 0; m < n_out; ++m) {
            const float2 v = zb[m];
            const double2 w = T[idx];
            re = fma((double)v.x, w.x, fma(-(double)v.y, w.y, re));
            im = fma((double)v.x, w.y, fma((double)v.y, w.x, im));
            idx += j;
            if (idx >= n_out) idx -= n_out;
        }
        const double2 e = ej[j];
        const double er = re * e.x - im * e.y, ei = re * e.y + im * e.x;
        xo[j] = make_float2((float)(er * s.x - ei * s.y), (float)(er * s.y + ei * s.x));
    }
}

}  // namespace

hipError_t launch_sft_series(const float2 *z, int64_t n_sft, int64_t n_bins, int64_t off, int n_out, int h,
                             const double2 *roots, const double2 *ej, const double2 *sk, const uint8_t *present,
                             float2 *x, hipStream_t stream) {
    if (n_sft == 0) return hipSuccess;
    if (n_out < 1 || n_out > kSftMaxOut) return hipErrorInvalidValue;
    const size_t lds = (size_t)n_out * sizeof(float2) + (n_out <= kSftTwLds ? (size_t)n_out * sizeof(double2) : 0);
    hipLaunchKernelGGL(k_sft_series, dim3((unsigned)n_sft), dim3(kSftThreads), lds, stream, z, n_bins, off, n_out, h,
                       roots, ej, sk, present, x);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fixed scratch

// Workspace of ccr_compute_rho_noalloc: a file-scope device array, so that the entry point
// allocates nothing.  Each device the library runs on holds its own copy (kScratchBytes) until
// the process ends.  In host code `scratch` is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
    if (device < 0 || device >= kScratchMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = ptr;
    if (cur != device) (void)hipSetDevice(cur);
    return e;
}

void *scratch_device_ptr(int device) {
    if (device < 0 || device >= kScratchMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace ccr

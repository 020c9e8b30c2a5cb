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

#include "ccr_internal.h"

namespace ccr {
namespace {

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

// ------------------------------------------------------------------ time base (FP64)

// sin(x) and cos(x) - 1 by their Taylor series through x^11 / x^12; |x| <= 0.3 keeps the
// truncation below 3e-17 relative.
__device__ __forceinline__ void sincos_small(double x, double &s, double &cm1) {
    const double x2 = x * x;
    s = x * (1.0 - x2 * (1.0 / 6.0) * (1.0 - x2 * (1.0 / 20.0) * (1.0 - x2 * (1.0 / 42.0) *
             (1.0 - x2 * (1.0 / 72.0) * (1.0 - x2 * (1.0 / 110.0))))));
    cm1 = -x2 * 0.5 * (1.0 - x2 * (1.0 / 12.0) * (1.0 - x2 * (1.0 / 30.0) * (1.0 - x2 * (1.0 / 56.0) *
             (1.0 - x2 * (1.0 / 90.0) * (1.0 - x2 * (1.0 / 132.0))))));
}

// Binary orbital phase (cycles in [0,1)) of segment K's mid-time: frac(c0 + K c1), both in
// double-double, then (sin, cos) of 2 pi times it.
__device__ __forceinline__ void binary_anchor(const double *tp, int K, double &sb, double &cb) {
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
// Two Newton steps from eta_0 = a_p sin(theta_b + Omega u).
// Outputs the interpolation centre j* = r + round-half-up(Delta / dt), the offset
// delta_c = Delta / dt - round(.) in [-1/2, 1/2) and the heterodyne phase frac(f_h Delta).
__device__ __forceinline__ void time_base(double u, double a_p, double Om, double sb, double cb,
                                          const EarthConst &ec, const Anchor &an, double dt,
                                          double f_het, int64_t r, int64_t &jstar, double &dc,
                                          double &psi) {
    double s, cm;
    sincos_small(Om * u, s, cm);
    double eta = a_p * (fma(sb, cm, sb) + cb * s);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double x = u + eta;
        double so, co, sd, cd;
        sincos_small(ec.w_o * x, so, co);
        sincos_small(ec.w_d * x, sd, cd);
        const double de = ec.A_o * (an.c_o * co - an.s_o * so) + ec.A_d * (an.c_d * cd - an.s_d * sd) + an.rho_a;
        const double dep = -ec.A_o * ec.w_o * (an.c_o * so + fma(an.s_o, co, an.s_o)) -
                           ec.A_d * ec.w_d * (an.c_d * sd + fma(an.s_d, cd, an.s_d));
        double sbn, cbn;
        sincos_small(Om * (x + de), sbn, cbn);
        const double sinb = fma(sb, cbn, sb) + cb * sbn;
        const double cosb = fma(cb, cbn, cb) - sb * sbn;
        const double G = eta + de - a_p * sinb;
        const double Gp = (1.0 + dep) * (1.0 - a_p * Om * cosb);
        eta -= G / Gp;
    }
    const double q = (eta - an.D_a) / dt;
    const double k = floor(q + 0.5);
    jstar = r + (int64_t)k;
    dc = q - k;
    double ps = an.psi_a + f_het * eta;
    psi = ps - floor(ps);
}

// ------------------------------------------------------------------ resampling

template <typename T> __device__ __forceinline__ T sinpi_t(T v);
template <> __device__ __forceinline__ float sinpi_t<float>(float v) { return sinpif(v); }
template <> __device__ __forceinline__ double sinpi_t<double>(double v) { return sinpi(v); }
template <typename T> __device__ __forceinline__ T cospi_t(T v);
template <> __device__ __forceinline__ float cospi_t<float>(float v) { return cospif(v); }
template <> __device__ __forceinline__ double cospi_t<double>(double v) { return cospi(v); }
template <typename T> __device__ __forceinline__ const T *win_table(const BandDev &B);
template <> __device__ __forceinline__ const float *win_table<float>(const BandDev &B) { return B.win32; }
template <> __device__ __forceinline__ const double *win_table<double>(const BandDev &B) { return B.win64; }

// sum_{n=-D}^{D} w sinc(delta_c - n) x'_{j*+n}, with sin(pi (dc - n)) = (-1)^n sin(pi dc);
// taps outside [0, n) read zero.
template <typename T>
__device__ __forceinline__ c2<T> interpolate(const BandDev &B, const float2 *xd, int64_t jstar,
                                             double dcd) {
    const T dc = (T)dcd;
    const T s = sinpi_t<T>(dc) * (T)0.318309886183790671537767526745;  // sin(pi dc) / pi
    const T *wt = win_table<T>(B);
    const int D = B.D;
    T re = 0, im = 0;
    for (int n = -D; n <= D; ++n) {
        const int64_t j = jstar + n;
        if (j < 0 || j >= B.n) continue;
        const T d = dc - (T)n;
        T tap;
        if (d == (T)0) {
            tap = (T)1;
        } else {
            tap = ((n & 1) ? -s : s) / d;
        }
        const T w = (B.window == 0) ? wt[n + D] : (T)0.54 + (T)0.46 * cospi_t<T>(d / (T)(D + 1));
        const float2 xv = xd[j];
        re += (w * tap) * (T)xv.x;
        im += (w * tap) * (T)xv.y;
    }
    return mk<T>(re, im);
}

template <typename T>
__global__ void __launch_bounds__(256) k_resample(BandDev B, const double *tmpl, c2<T> *y) {
    const int entry = B.work[blockIdx.x];
    const int det = entry / B.n_seg;
    const int K = entry - det * B.n_seg;
    const int tb = blockIdx.y;
    const double *tp = tmpl + (size_t)kTmplStride * tb;
    __shared__ double sh_sc[2];
    if (threadIdx.x == 0) {
        double sb, cb;
        binary_anchor(tp, K, sb, cb);
        sh_sc[0] = sb;
        sh_sc[1] = cb;
    }
    __syncthreads();
    const double sb = sh_sc[0], cb = sh_sc[1];
    const double a_p = tp[0], Om = tp[1];
    const Anchor an = B.anchors[entry];
    const EarthConst ec = B.earth[det];
    const int64_t nr = (int64_t)B.n_seg * B.n_k;
    const float2 *xd = B.x + (size_t)det * B.n;
    const uint8_t *mk_ = B.mask + (size_t)det * nr;
    c2<T> *yo = y + ((size_t)tb * B.Q + det) * nr;
    const double half = 0.5 * (double)B.n_k;
    for (int s = threadIdx.x; s < B.n_k; s += blockDim.x) {
        const int64_t r = (int64_t)K * B.n_k + s;
        if (!mk_[r]) {
            yo[r] = mk<T>((T)0, (T)0);
            continue;
        }
        const double u = ((double)s - half) * B.dt;
        int64_t jstar;
        double dc, psi;
        time_base(u, a_p, Om, sb, cb, ec, an, B.dt, B.f_het, r, jstar, dc, psi);
        const c2<T> acc = interpolate<T>(B, xd, jstar, dc);
        T c, sn;
        if constexpr (sizeof(T) == 8) {
            sincospi(2.0 * psi, &sn, &c);
        } else {
            sincospif(2.0f * (float)psi, &sn, &c);
        }
        yo[r] = mk<T>(c * acc.x - sn * acc.y, sn * acc.x + c * acc.y);
    }
}

// ------------------------------------------------------------------ FFT in LDS

// Self-sorting Stockham passes (radix 4, a final radix 2 when log2 n is odd) over n points
// held in LDS; twiddles exp(-2 pi i k r / (Ns R)) read from the N_FFT-entry table.
template <typename T>
__device__ c2<T> *stockham(c2<T> *a, c2<T> *b, int n, const c2<T> *tw, int n_fft) {
    for (int Ns = 1; Ns < n;) {
        const int R = (Ns * 4 <= n) ? 4 : 2;
        const int stride = n / R;
        const int twstep = n_fft / (Ns * R);
        for (int j = threadIdx.x; j < stride; j += blockDim.x) {
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
template <typename T>
__global__ void __launch_bounds__(256) k_spectra(BandDev B, const c2<T> *y, c2<T> *F) {
    extern __shared__ __align__(16) unsigned char smem[];
    c2<T> *buf0 = reinterpret_cast<c2<T> *>(smem);
    c2<T> *buf1 = buf0 + B.n_s;
    const int entry = B.work[blockIdx.x];
    const int det = entry / B.n_seg;
    const int K = entry - det * B.n_seg;
    const int tb = blockIdx.y;
    const int64_t nr = (int64_t)B.n_seg * B.n_k;
    const c2<T> *ys = y + ((size_t)tb * B.Q + det) * nr + (size_t)K * B.n_k;
    const c2<T> *tw = twiddles<T>(B);
    const int rb_mod = (int)(((int64_t)K * B.n_k) % B.n_fft);
    const T scale = (T)B.segw[entry].scale;
    c2<T> *Fo = F + (((size_t)tb * B.Q + det) * B.n_seg + K) * B.n_f;
    for (int p = 0; p < B.P; ++p) {
        for (int s = threadIdx.x; s < B.n_s; s += blockDim.x) {
            c2<T> v = mk<T>((T)0, (T)0);
            if (s < B.n_k) {
                v = ys[s];
                if (p) v = cmul<T>(v, tw[p * s]);
            }
            buf0[s] = v;
        }
        __syncthreads();
        const c2<T> *res = stockham<T>(buf0, buf1, B.n_s, tw, B.n_fft);
        for (int i = threadIdx.x; i < B.n_f; i += blockDim.x) {
            if (B.bin_p[i] != p) continue;
            const int ph = (int)(((int64_t)B.bin_kb[i] * rb_mod) % B.n_fft);
            Fo[i] = cscale<T>(cmul<T>(res[B.bin_m[i]], tw[ph]), scale);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ pair sum

// Partial rho of one (template, bin, chunk of segments): for each segment K and detector X,
// conj(F_XK) times the weighted sum of its partners (Y, L) that precede it -- L in
// [K - R, K - 1] (other detectors if cross pairs, the same detector if same pairs) and
// L = K with Y > X (cross pairs) -- so each unordered pair of the set enters once.
template <typename T>
__global__ void __launch_bounds__(256) k_pairs(BandDev B, const c2<T> *F, double *part, int k_chunk,
                                               int n_chunks) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    const int tb = blockIdx.z;
    if (i >= B.n_f) return;
    const bool cross = (B.pairs & 1) != 0, same = (B.pairs & 2) != 0;
    const c2<T> *Ft = F + (size_t)tb * B.Q * B.n_seg * B.n_f;
    const int K0 = c * k_chunk;
    const int K1 = min(B.n_seg, K0 + k_chunk);
    double acc = 0.0;
    for (int K = K0; K < K1; ++K) {
        for (int X = 0; X < B.Q; ++X) {
            const int ek = X * B.n_seg + K;
            if (!B.active[ek]) continue;
            c2<T> ga = mk<T>((T)0, (T)0), gb = mk<T>((T)0, (T)0);
            for (int L = max(0, K - B.R); L <= K; ++L) {
                for (int Y = 0; Y < B.Q; ++Y) {
                    const bool inc = (L < K) ? ((Y != X) ? cross : same) : (cross && Y > X);
                    const int el = Y * B.n_seg + L;
                    if (!inc || !B.active[el]) continue;
                    const c2<T> g = Ft[(size_t)el * B.n_f + i];
                    const T wa = (T)B.segw[el].ahat, wb = (T)B.segw[el].bhat;
                    ga.x += wa * g.x; ga.y += wa * g.y;
                    gb.x += wb * g.x; gb.y += wb * g.y;
                }
            }
            const c2<T> f = Ft[(size_t)ek * B.n_f + i];
            const T aK = (T)B.segw[ek].ahat, bK = (T)B.segw[ek].bhat;
            const T hx = aK * ga.x + bK * gb.x, hy = aK * ga.y + bK * gb.y;
            acc += (double)(f.x * hx + f.y * hy);
        }
    }
    part[((size_t)tb * n_chunks + c) * B.n_f + i] = acc;
}

__global__ void k_finish(int n_f, int n_tmpl, const double *part, int n_chunks, double factor,
                         void *out, int out_fp64) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (i >= n_f || t >= n_tmpl) return;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += part[((size_t)t * n_chunks + c) * n_f + i];
    s *= factor;
    if (out_fp64)
        static_cast<double *>(out)[(size_t)t * n_f + i] = s;
    else
        static_cast<float *>(out)[(size_t)t * n_f + i] = (float)s;
}

__global__ void k_zero(uint32_t *p, size_t n_words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n_words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

hipError_t launch_resample(const BandDev &B, const double *d_tmpl, int n_tmpl, bool fp64, void *y,
                           hipStream_t stream) {
    if (B.n_work == 0 || n_tmpl == 0) return hipSuccess;
    dim3 grid(B.n_work, n_tmpl), block(256);
    if (fp64)
        hipLaunchKernelGGL(k_resample<double>, grid, block, 0, stream, B, d_tmpl, (double2 *)y);
    else
        hipLaunchKernelGGL(k_resample<float>, grid, block, 0, stream, B, d_tmpl, (float2 *)y);
    return hipGetLastError();
}

hipError_t launch_spectra(const BandDev &B, int n_tmpl, bool fp64, const void *y, void *F,
                          hipStream_t stream) {
    if (B.n_work == 0 || n_tmpl == 0) return hipSuccess;
    const int threads = B.n_s / 4 >= 256 ? 256 : (B.n_s / 4 < 64 ? 64 : B.n_s / 4);
    dim3 grid(B.n_work, n_tmpl), block(threads);
    const size_t lds = 2 * (size_t)B.n_s * (fp64 ? sizeof(double2) : sizeof(float2));
    if (fp64)
        hipLaunchKernelGGL(k_spectra<double>, grid, block, lds, stream, B, (const double2 *)y, (double2 *)F);
    else
        hipLaunchKernelGGL(k_spectra<float>, grid, block, lds, stream, B, (const float2 *)y, (float2 *)F);
    return hipGetLastError();
}

hipError_t launch_pairsum(const BandDev &B, int n_tmpl, bool fp64, const void *F, double *part,
                          int k_chunk, int n_chunks, hipStream_t stream) {
    if (n_tmpl == 0) return hipSuccess;
    dim3 grid((B.n_f + 127) / 128, n_chunks, n_tmpl), block(128);
    if (fp64)
        hipLaunchKernelGGL(k_pairs<double>, grid, block, 0, stream, B, (const double2 *)F, part, k_chunk, n_chunks);
    else
        hipLaunchKernelGGL(k_pairs<float>, grid, block, 0, stream, B, (const float2 *)F, part, k_chunk, n_chunks);
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

hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    const unsigned blocks = (unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, stream, (uint32_t *)p, words);
    return hipGetLastError();
}

}  // namespace ccr

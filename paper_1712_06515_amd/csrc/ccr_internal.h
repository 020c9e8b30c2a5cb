// Internal types shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ccr {

// Earth Roemer delay of one detector in closed form:
//   r(t).n = C + A_o cos(theta_o(t)) + A_d cos(theta_d(t)),
//   theta_o advancing at w_o (orbit), theta_d at w_d (sidereal rotation).
struct EarthConst {
    double A_o, w_o, A_d, w_d;
};

// Per (detector, segment) anchor, template independent.  t_a is a detector time close to
// the Earth-only arrival of the segment mid-time tau_a (t_a + r(t_a).n ~ tau_a):
//   c_o, s_o, c_d, s_d  cos/sin of theta_o(t_a), theta_d(t_a)
//   D_a                 tau_a - t_a, exact difference of the two representable times
//   rho_a               r(t_a).n - D_a, the residual left because t_a is itself rounded
//   psi_a               frac(-f_het D_a), cycles
struct Anchor {
    double c_o, s_o, c_d, s_d, D_a, rho_a, psi_a;
};

// Per (detector, segment) weights: hat a = a / sigma, hat b = b / sigma,
// scale = 1 / (sigma sqrt(N_K)) for the segment spectra.
struct SegWeight {
    double ahat, bhat, scale;
};

// Per template, ten doubles: a_p, Omega = 2 pi / P, and the binary orbital phase (cycles)
// of segment K's mid-time as c0 + K c1 in double-double: c0h, c0l, c1h, c1l -- for a circular
// orbit measured from T_asc, for an eccentric one the mean anomaly measured from T_p -- then
// (eccentric orbits) e, sin omega, cos omega, sqrt(1 - e^2).
constexpr int kTmplStride = 10;

// Chebyshev nodes per segment for the time base; the split path may use kChebSplit,
// kChebSplitMin or kChebSplitLow nodes (degree 6, 5 or 4) when the host's bound on the
// Chebyshev tail allows; detector limit.
constexpr int kCheb = 10;
constexpr int kChebSplit = 7;
constexpr int kChebSplitMin = 6;
constexpr int kChebSplitLow = 5;
constexpr int kChebRules = 4;
// node rules: index of the table of an NN-node rule, and offset of its nodes in cheb_x
constexpr int cheb_rule(int nn) { return nn == kCheb ? 0 : (nn == kChebSplit ? 1 : (nn == kChebSplitMin ? 2 : 3)); }
constexpr int cheb_x_off(int nn) {
    return nn == kCheb ? 0
                       : (nn == kChebSplit ? kCheb : (nn == kChebSplitMin ? kCheb + kChebSplit : kCheb + kChebSplit + kChebSplitMin));
}
constexpr int kChebNodesAll = kCheb + kChebSplit + kChebSplitMin + kChebSplitLow;
#define CCR_MAX_DET_K 8

// Everything a kernel needs about a band (device pointers + scalars).
struct BandDev {
    int Q;              // detectors
    int64_t n;          // samples per detector
    int n_k, n_seg;     // samples per segment, segments
    int n_fft, n_s, P;  // N_FFT = P * n_s, n_s = 2^ceil(log2 n_k)
    int nfft_mask;      // N_FFT - 1 when N_FFT is a power of two, else 0
    int n_f;            // output bins
    int D, window;      // taps each side, window kind
    int R, pairs;       // max lag, pair kinds
    double dt, inv_dt, f_het;
    const float2 *x;          // [Q][n] complex64, zero where invalid
    const uint8_t *mask;      // [Q][n_seg * n_k] gap mask of source samples
    const Anchor *anchors;    // [Q][n_seg]
    const EarthConst *earth;  // [Q]
    const double *win64;      // [2D+1] tap window (window == 0)
    const float *win32;
    const double *cheb_x;     // nodes cos(pi (j + 1/2) / N) for N = kCheb, kChebSplit, kChebSplitMin, kChebSplitLow
    const double *mono;       // [kChebRules][kCheb][kCheb] node values -> monomial coefficients of the
                              // interpolant through the N Chebyshev nodes (rule cheb_rule(N))
    const double2 *tw64;      // [n_fft] exp(-2 pi i j / n_fft)
    const float2 *tw32;
    const int *bin_m;         // [n_f] FFT output index within residue class
    const int *bin_p;         // [n_f] residue class kbar mod P
    const int *bin_kb;        // [n_f] kbar mod n_fft
    const int *bin_pos;       // [n_fft] output bin i of FFT index kbar mod n_fft, -1 if none
    int bins_unique;          // 1 when every output bin has its own FFT index
    const SegWeight *segw;    // [Q][n_seg]
    const float2 *segwf;      // [Q][n_seg] (hat a scale, hat b scale) rounded to FP32
    const uint8_t *active;    // [Q][n_seg] 1 when the segment takes part in a pair
    const int *work;          // [n_work] det * n_seg + K of active segments
    const int *seg_work;      // [Q][n_seg] position of (det, K) in `work`, -1 if inactive
    int n_work;
    const double *tmpl;       // [n_templates][kTmplStride] template table
    // lag phases of the pair sum, lagph[dl n_f + c] = exp(+2 pi i kbar dl n_k / N_FFT) for the
    // bin of ring column c, dl <= R: F*_XK F_YL = lagph(K - L) conj(F~_XK) F~_YL for spectra F~
    // taken without Phi_in
    const float2 *lagph;
    const int *col_bin;       // [n_f] spectra + pair-sum ring: bin of column c (bins ordered by
    const int *bin_col;       // [n_f] residue class, then index in the class); column of bin i
    const int *class_start;   // [P + 1] the bins of residue class p are col_bin[class_start[p] ..
                              // class_start[p + 1])
    const float2 *zero256;    // [256] zero samples (input of FFT groups without a segment)
    const int *seg_any;       // [n_seg_any] ascending segments K where some detector is active
    int n_seg_any;
    int newton_steps;         // Newton steps of the time-base node solve (2 or 3)
    int ecc;                  // templates are eccentric orbits (Kepler solve in the time base)
    int cheb_split;           // time-base nodes of the split path (kChebSplitLow ... kChebSplit, or kCheb)
    // Farrow table of the split-precision resampler, [Q][kFarDeg + 1][far_len] complex64:
    // plane k at index j + D holds F_k(j) = sum_n A_kn x'_{j+n} (F_0 = x'), zero beyond
    // j + D >= n + 2D; null when the band has none
    const float2 *farrow;
    int64_t far_len;
    int far_stage;  // 1: stage the table in LDS (else every sample reads it from global memory)
    // 1024-point spectra + pair-sum kernel: per residue class p the first FFT output index m0 of
    // its bins in circular order (the class's bins occupy m0 .. m0 + span - 1 mod n_s); the
    // widest span in units of 64 outputs, and the largest class (bins)
    const int *cls_m0;
    int wide_jmax, wide_ncol;
    // pair weight (0 Gamma^ave, 1 Gamma^circ) and pair set (allp: every ordered pair, autos
    // included: the partials are the chunk sums of the two streams, 4 values a bin)
    int weight, allp;
    // per-sample antenna weights [Q][n_seg * n_k]: (a_r, b_r) / (sigma_K^2 sqrt(N_K)), or null
    // (per-segment weights: the two streams are hat a_K F and hat b_K F)
    const double2 *pw;
    // the same weights in FP32, [Q][n_seg * n_k] (a_r, b_r) / (sigma_K^2 sqrt(N_K)), or null
    const float2 *pwf;
    // split path with per-sample weights on the wide spectra + pair-sum kernel: the resampler
    // writes two series per detector, y a_r and y b_r (stream s of detector X at X 2 + s), that
    // kernel transforms both
    int ps2;
};

// One work item of a batched launch: a run of consecutive templates of one band.  A batched
// launch covers a list of items of several bands; each stage's grid is the concatenation of
// the items' grids (item i owns blocks [first[stage], next item's first[stage])).
enum Stage { kStTimebase = 0, kStResample = 1, kStSpectra = 2, kStPairs = 3, kStFinish = 4, kStages = 5 };
struct WorkItem {
    int band;               // index into the launch's BandDev table
    int n_tmpl;             // templates in the item
    int k_chunk, n_chunks;  // segment chunks of the pair sums
    int64_t tmpl_off;       // first template of the item (row of the band's template table)
    int64_t coef_off;       // doubles into the time-base coefficient workspace
    int64_t y_off;          // complex samples into the resampled-series workspace
    int64_t F_off;          // complex values into the segment-spectra workspace
    int64_t part_off;       // doubles into the chunk-partial workspace
    void *out;              // rho of the item's first template: n_tmpl x n_f, f32 or f64
    double factor;          // sqrt(2) / N
    int out_fp64;
    int first[kStages];     // first block of the item in each stage's grid
    int gx[kStages];        // blocks per template along the stage's first dimension
};

// Block geometry shared by the host planner and the kernels.
// time base: work entries per workgroup for NN nodes (x NN threads: whole wavefronts)
constexpr int tb_entries(int nn) { return nn == kCheb ? 32 : 64; }
constexpr int kSpec16Groups = 8;     // 256-point register FFT: segments per 128-thread workgroup
constexpr int kPairsThreads = 128;   // pair sum: bins per workgroup
constexpr int kFinishThreads = 256;  // finish: bins per workgroup
constexpr int kResTemplates = 4;     // resampling: templates per workgroup
// Farrow-form resampling (split precision): tap weights as polynomials of degree kFarDeg in the
// offset; a 256-thread workgroup (kFarWaves wavefronts, kFarPerWave templates each) stages the
// table planes of chunks of kFarChunk samples of one segment in LDS (kFarCap entries a plane)
constexpr int kFarDeg = 8;
constexpr int kFarWaves = 4;
constexpr int kFarPerWave = 16;
constexpr int kFarTemplates = kFarWaves * kFarPerWave;
constexpr int kFarChunk = 192;
constexpr int kFarCap = 224;

// Launchers (ccr_kernels.hip).  All queue work on `stream` and return the launch status.
// Monomial coefficients of the time base (interpolant through Chebyshev nodes), coef[n_tmpl][n_work][kCheb].
hipError_t launch_timebase(const BandDev &B, const double *d_tmpl, int n_tmpl, double *coef,
                           hipStream_t stream);
hipError_t launch_resample(const BandDev &B, const double *coef, int n_tmpl, bool fp64, void *y,
                           hipStream_t stream);
hipError_t launch_spectra(const BandDev &B, int n_tmpl, bool fp64, const void *y, void *F,
                          hipStream_t stream);
// Fused resample + FFT + pair sum, one workgroup per (template, chunk of k_chunk segments),
// S segments per step; fused_steps() picks S for an LDS budget (0: does not fit).
int fused_steps(const BandDev &B, bool fp64, size_t limit);
size_t fused_lds_bytes(const BandDev &B, bool fp64, int S);
hipError_t launch_fused(const BandDev &B, const double *coef, int n_tmpl, bool fp64, double *part,
                        int k_chunk, int n_chunks, int S, hipStream_t stream);
// Split-precision spectra + pair sum in one kernel (256-point segments, distinct bins, at most
// 4 detectors and 512 bins): whether a band qualifies for it.
bool spectra_pairs_ok(const BandDev &B, bool fp64, size_t limit);
hipError_t launch_finish(const BandDev &B, int n_tmpl, const double *part, int n_chunks,
                         double factor, void *out, bool out_fp64, hipStream_t stream);

// Batched launches: `blocks` = total blocks of the stage over the items; bands and items are
// device tables.  Every item of one launch shares the kernel variant chosen by the arguments.
size_t spectra_pairs_lds(const BandDev &B);
int spectra_pairs_rounds(const BandDev &B);  // bins per lane of the spectra+pairs kernel (3 or 8)
int spectra_threads(int n_s);               // threads of the LDS Stockham FFT workgroup
// short_series: the node solve's small-angle series end at x^7 / x^8 (a band's host bound).
hipError_t launch_timebase_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int n_cheb,
                             bool short_series, double *coef,
                             hipStream_t stream);
// farrow: the split-precision Farrow-form kernel (bands with a table; kFarTemplates templates a
// workgroup); else one wavefront per kResTemplates templates.
hipError_t launch_resample_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool fp64, int D,
                             int window, int n_cheb, bool farrow, const double *coef, void *y, hipStream_t stream);
// The Farrow table of a band (BandDev::farrow) from its input series x [Q][n] and the fitted
// coefficients A [kFarDeg][2D + 1] (row k - 1 for the power dc^k).
hipError_t launch_farrow_table(const float2 *x, int64_t n, int Q, int D, const double *A, int64_t far_len,
                               float2 *tab, hipStream_t stream);
// Split-precision spectra + pair sum for 256- to 1024-point segments (N_FFT a power of two,
// distinct bins, at most 4 detectors, classes of at most 64 W U bins, LDS within `limit`); its
// LDS bytes, the bins of a class per lane it is instantiated for (1, 2, 4 or 8), the segments
// it transforms a step (1 or 2) and its wavefronts a workgroup.
bool spectra_wide_ok(const BandDev &B, bool fp64, size_t limit);
size_t spectra_wide_lds(const BandDev &B);
int spectra_wide_cols(const BandDev &B);
int spectra_wide_segs(const BandDev &B);
int spectra_wide_waves(const BandDev &B);
// cols, ts, waves: spectra_wide_cols, spectra_wide_segs and spectra_wide_waves of the round's
// bands; q: their detector count (1-4, the same for all).
hipError_t launch_spectra_wide_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int ns,
                                 int cols, int q, int ts, int waves, bool allp, bool ps, size_t lds, const void *y,
                                 double *part, hipStream_t stream);
// z4: N_K <= 192, so the last 4 of the 16 input rows of each 256-point FFT are zero padding.
hipError_t launch_spectra_pairs_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, int rounds,
                                  bool z4, size_t lds, const void *y, double *part, hipStream_t stream);
// reg16: the 256-point register FFT (split precision, distinct bins); else the LDS Stockham FFT
// with `threads` threads and 2 n_s complex values of LDS.
hipError_t launch_spectra_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool fp64,
                            bool reg16, int threads, int n_s, const void *y, void *F, hipStream_t stream);
hipError_t launch_pairs_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, bool fp64,
                          const void *F, double *part, hipStream_t stream);
hipError_t launch_finish_m(const BandDev *bands, const WorkItem *items, int n_items, int blocks, const double *part,
                           hipStream_t stream);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream);
// SFT front end: the heterodyned series of n_sft SFTs (complex64 bins, n_bins per SFT; the band of
// n_out bins starts `off` bins in), roots[m] = exp(2 pi i m / n_out), ej[j] (remainder phase and
// 1 / T_sft), sk[K] (stitching phase), present[K] (null: all); x: n_sft x n_out complex64.
constexpr int kSftMaxOut = 4096;
hipError_t launch_sft_series(const float2 *z, int64_t n_sft, int64_t n_bins, int64_t off, int n_out, int h,
                             const double2 *roots, const double2 *ej, const double2 *sk, const uint8_t *present,
                             float2 *x, hipStream_t stream);

// Fixed device scratch of the no-allocation entry point (a file-scope device array of
// kScratchBytes per device).  scratch_init(device) looks up the array's device address on
// `device` once (hipGetSymbolAddress with that device current) and keeps it; scratch_device_ptr
// returns it (null before scratch_init succeeded).
constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kScratchMaxDevices = 64;
hipError_t scratch_init(int device);
void *scratch_device_ptr(int device);
// eta and the heterodyne phase of every sample of active segments [k0, k0 + n) of one detector
// (one template, coefficients from launch_timebase): eta[(K - k0) n_k + s], psi likewise.
hipError_t launch_time_samples(const BandDev &B, const double *coef, int det, int k0, int n, double *eta,
                               double *psi, hipStream_t stream);

}  // namespace ccr

"""Parity of the HIP path (through the C ABI) with the oracle, element by element.

Error measure for rho: max over (template, bin) of |rho_gpu - rho_oracle| / max(|rho_oracle|, 1)
(rho is in units of its noise standard deviation, so the floor is one sigma).  Bars: 1e-10 for
the FP64 path, 1e-4 for the split path.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from conftest import small_config

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


@pytest.fixture(scope="module")
def ccr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06515_amd import ccr as mod
    mod.load_library()
    return mod


def rho_err(a, ref):
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 1.0)))


def run_both(ccr, ds, templates, **opts):
    with ccr.Context(ds.sky, device=0) as ctx:
        for k, v in opts.items():
            ctx.set_option(k, v)
        bid = ctx.load(ds, templates=templates)
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
    return r64, r32


SMALL_CASES = {
    "lag0_cross": dict(max_lag=0, pairs=1, n_seg=14),
    "lag2_gaps_both": dict(max_lag=2, gap_fraction=0.25, n_seg=24, pairs=3),
    "three_det_lag3": dict(q=3, max_lag=3, n_seg=20, gap_fraction=0.1),
    "same_only_window1": dict(max_lag=1, pairs=2, window=1, n_seg=12),
    "fft_multiple_3": dict(n_fft_override=3 * 128, max_lag=1, n_seg=10),
    "D4_high_mu": dict(dirichlet_D=4, mu_f=0.4, n_seg=9, max_lag=1),
}


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("case", sorted(SMALL_CASES))
def test_rho_small_cases(ccr, case, fused):
    kw = SMALL_CASES[case]
    cfg = small_config(**kw, injections=[dict(f0=50.21, a_p=1.25, t_asc_off=0.0, period=68023.7, h0=0.35,
                                              cosi=0.5, psi=0.3, phi0=1.0)])
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    tm = ds.templates
    ref = oracle.Oracle(ds).rho(tm)
    r64, r32 = run_both(ccr, ds, tm, fused=fused, k_chunk=5)
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"{case} fused={fused}: fp64 {e64:.2e} split {e32:.2e} max|rho| {np.abs(ref).max():.2f}")
    assert e64 < TOL64
    assert e32 < TOL32


@pytest.mark.parametrize("case", sorted(SMALL_CASES))
def test_rho_small_cases_direct_taps(ccr, case):
    # the split path with the direct 2D + 1-tap resampler instead of the Farrow form
    kw = SMALL_CASES[case]
    cfg = small_config(**kw, injections=[dict(f0=50.21, a_p=1.25, t_asc_off=0.0, period=68023.7, h0=0.35,
                                              cosi=0.5, psi=0.3, phi0=1.0)])
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    tm = ds.templates
    ref = oracle.Oracle(ds).rho(tm)
    _, r32 = run_both(ccr, ds, tm, farrow=0, k_chunk=5)
    e32 = rho_err(r32, ref)
    print(f"{case} direct taps: split {e32:.2e}")
    assert e32 < TOL32


@pytest.mark.parametrize("farrow", [1, 0])
@pytest.mark.parametrize("window", [0, 1])
def test_resampled_series_parity(ccr, farrow, window):
    # farrow 1: split precision in Farrow form (the default), 0: the direct tap sum
    cfg = small_config(n_seg=12, gap_fraction=0.2, max_lag=1, window=window)
    ds = synth.make_dataset(cfg)
    o = oracle.Oracle(ds)
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("farrow", farrow)
        bid = ctx.load(ds)
        assert ctx.band_info(bid)["farrow_degree"] == ctx.get_option("farrow_degree")
        for t in (0, 3, 5):
            for X in range(2):
                y_ref, js, off, m = o.resample(X, ds.templates[t])
                y64 = ctx.resample_series(bid, t, X, prec=ccr.PREC_FP64)
                y32 = ctx.resample_series(bid, t, X, prec=ccr.PREC_SPLIT)
                scale = np.abs(y_ref).max()
                print(f"resampled series farrow={farrow} window={window} t={t} X={X}: fp64 {np.abs(y64 - y_ref).max() / scale:.2e}, "
                      f"split {np.abs(y32 - y_ref).max() / scale:.2e} of the peak")
                assert np.abs(y64 - y_ref).max() < 1e-12 * scale
                assert np.abs(y32 - y_ref).max() < 2e-6 * scale
                assert np.all((y64 == 0) >= (m == 0))


def test_split_without_farrow_table(ccr):
    # D = 24: the degree-8 fit's bound (5.2e-7) exceeds the library's 4e-7, so the band gets no
    # Farrow table and the split path resamples with the direct tap sum
    cfg = small_config(n_seg=8, dirichlet_D=24, max_lag=1)
    ds = synth.make_dataset(cfg)
    ref = oracle.Oracle(ds).rho(ds.templates)
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"D=24 (no Farrow table, bound {info['farrow_err']:.2e}): fp64 {e64:.2e} split {e32:.2e}")
    assert info["farrow_degree"] == 0 and info["farrow_err"] > 4e-7
    assert e64 < TOL64
    assert e32 < TOL32


def test_farrow_unstaged_path_identical(ccr):
    # the Farrow kernel's global-memory path (taken by a chunk whose j* range does not fit in
    # LDS) evaluates the same polynomial from the same table: bitwise the staged result
    cfg = small_config(n_seg=10, gap_fraction=0.2, max_lag=1)
    ds = synth.make_dataset(cfg)
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        y1 = [ctx.resample_series(bid, t, 1, prec=ccr.PREC_SPLIT) for t in (0, 4)]
        r1 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        ctx.set_option("farrow_stage", 0)
        y0 = [ctx.resample_series(bid, t, 1, prec=ccr.PREC_SPLIT) for t in (0, 4)]
        r0 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
    for a, b in zip(y1, y0):
        assert np.array_equal(a, b)
    assert np.array_equal(r1, r0)


def test_segment_spectra_parity(ccr):
    cfg = small_config(n_seg=10, max_lag=2, q=3, gap_fraction=0.1)
    ds = synth.make_dataset(cfg)
    o = oracle.Oracle(ds)
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        for t in (1, 4):
            F_ref = o.spectra(ds.templates[t])
            F64 = ctx.segment_spectra(bid, t, prec=ccr.PREC_FP64)
            F32 = ctx.segment_spectra(bid, t, prec=ccr.PREC_SPLIT)
            scale = np.abs(F_ref).max()
            used = np.abs(F64).max(axis=2) > 0
            assert np.abs(F64 - F_ref)[used].max() < 1e-11 * scale
            assert np.abs(F32 - F_ref)[used].max() < 1e-5 * scale


def test_segment_spectra_256_point(ccr):
    """Segment spectra through the 16-lane register FFT (256-point segments, split precision)
    and the LDS Stockham FFT (FP64) against the oracle's direct DFT."""
    ds = synth.make_dataset(synth.config("tiny", t_obs=30 * 360.0))
    o = oracle.Oracle(ds)
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        assert ctx.band_info(bid)["n_k"] > 128
        for t in (0, 9):
            F_ref = o.spectra(ds.templates[t])
            F64 = ctx.segment_spectra(bid, t, prec=ccr.PREC_FP64)
            F32 = ctx.segment_spectra(bid, t, prec=ccr.PREC_SPLIT)
            scale = np.abs(F_ref).max()
            assert np.abs(F64 - F_ref).max() < 1e-11 * scale
            assert np.abs(F32 - F_ref).max() < 1e-5 * scale


LAGGED_256 = {
    # (detectors, max lag, pair kinds): segments per step S = 4 / Q of the 256-point kernel
    "q1_lag3_same": (1, 3, 2),
    "q2_lag4_both": (2, 4, 3),
    "q2_lag2_cross": (2, 2, 1),
    "q3_lag3_both": (3, 3, 3),
    "q4_lag2_both": (4, 2, 3),
}


@pytest.mark.parametrize("case", sorted(LAGGED_256))
def test_spectra_pairs_256_lagged(ccr, case):
    """The 256-point spectra + pair-sum kernel with lagged pairs (Sec. III.B.1): N_K = 162
    (400 s at 0.405 Hz), lags 2-4, 1-4 detectors, so 1, 2 or 4 segments per step, pairs within a
    step and across the ring wrap, a short last step (23 segments), gaps; lag phases of eq.
    final-formatted-rho for |K - L| up to 4.  FP64 (general path) and split against the oracle."""
    q, R, pairs = LAGGED_256[case]
    cfg = small_config(q=q, n_seg=23, t_short=400.0, f_min=400.0, f_band=0.06, max_lag=R, pairs=pairs,
                       a_p_max=2.0, gap_fraction=0.2,
                       templates=dict(a_p=(1.0, 2.0, 2), t_asc=(-200.0, 200.0, 2), period=[68023.70]),
                       injections=[dict(f0=400.031, a_p=1.3, t_asc_off=0.0, period=68023.7, h0=0.3,
                                        cosi=0.7, psi=0.4, phi0=2.0)])
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    ref = oracle.Oracle(ds).rho(ds.templates)
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        assert 128 < info["n_k"] <= 256
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        ctx.kernel_times(reset=True)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        kt = ctx.kernel_times(reset=True)
    assert kt["spectra_pairs"][1] > 0, kt  # the split call ran the 256-point kernel
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"256-point lagged {case}: fp64 {e64:.2e} split {e32:.2e} max|rho| {np.abs(ref).max():.2f}")
    assert e64 < TOL64 and e32 < TOL32


WIDE_1024 = {
    # (detectors, max lag, pair kinds, chunk length): N_K = 731 (2000 s at 0.366 Hz), n_s = 1024
    "q1_lag3_same": (1, 3, 2, 7),
    "q2_lag4_both": (2, 4, 3, 7),
    "q2_lag0_cross": (2, 0, 1, 256),
    "q3_lag2_both": (3, 2, 3, 5),
    "q4_lag1_both": (4, 1, 3, 256),
}


@pytest.mark.parametrize("case", sorted(WIDE_1024))
def test_spectra_wide_1024(ccr, case):
    """The 1024-point spectra + pair-sum kernel (segment spectra of one residue class in
    registers and an LDS ring, window sums of the last R segments, Phi_in as an absolute
    rotation): 1-4 detectors, lags 0-4, 30 % gaps (runs of empty segments longer than R),
    chunks of 5-7 segments with their halo, classes of 86-155 bins.  FP64 (general path) and
    split against the oracle (Sec. III.B.1 pairs, eq. final-formatted-rho)."""
    q, R, pairs, kc = WIDE_1024[case]
    cfg = small_config(q=q, n_seg=30, t_short=2000.0, f_min=400.0, f_band=0.06, max_lag=R, pairs=pairs,
                       a_p_max=2.0, gap_fraction=0.3,
                       templates=dict(a_p=(1.0, 2.0, 2), t_asc=(-200.0, 200.0, 2), period=[68023.70]),
                       injections=[dict(f0=400.029, a_p=1.3, t_asc_off=0.0, period=68023.7, h0=0.2,
                                        cosi=0.7, psi=0.4, phi0=2.0)])
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    ref = oracle.Oracle(ds).rho(ds.templates)
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        ctx.set_option("k_chunk", kc)
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        assert 512 < info["n_k"] <= 1024
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        ctx.kernel_times(reset=True)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        kt = ctx.kernel_times(reset=True)
        ctx.set_option("template_batch", 1)
        r32b = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
    assert kt["spectra_wide"][1] > 0, kt  # the split call ran the 1024-point kernel
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"1024-point {case}: fp64 {e64:.2e} split {e32:.2e} max|rho| {np.abs(ref).max():.2f}")
    assert e64 < TOL64 and e32 < TOL32
    assert np.array_equal(r32, r32b)  # one template per launch: same kernel arithmetic


WEIGHTED = {
    # (pair set, weight, per-sample antenna functions, detectors, max lag, gap fraction, shape)
    "circ_lag2_both": (3, 1, False, 2, 2, 0.25, "small"),
    "circ_q3_cross": (1, 1, False, 3, 1, 0.1, "small"),
    "all_ave": (4, 0, False, 2, 1, 0.2, "small"),
    "all_circ_q3": (4, 1, False, 3, 1, 0.1, "small"),
    "ps_ave_lag2": (3, 0, True, 2, 2, 0.2, "small"),
    "ps_circ_cross": (1, 1, True, 2, 1, 0.1, "small"),
    "ps_all_ave": (4, 0, True, 2, 1, 0.2, "small"),
    "ps_all_circ_q3": (4, 1, True, 3, 0, 0.0, "small"),
    "circ_256_lag3": (3, 1, False, 2, 3, 0.2, "256"),
    "ps_ave_256_lag2": (3, 0, True, 2, 2, 0.2, "256"),
    "circ_1024_lag2": (3, 1, False, 2, 2, 0.3, "1024"),
    "circ_1024_q3_both": (3, 1, False, 3, 2, 0.3, "1024"),
    "all_1024_lag1": (4, 0, False, 2, 1, 0.3, "1024"),
    "all_circ_1024_q3": (4, 1, False, 3, 2, 0.3, "1024"),
    "ps_all_1024": (4, 0, True, 2, 1, 0.3, "1024"),
    "ps_circ_1024_q3": (3, 1, True, 3, 2, 0.3, "1024"),
    "ps_ave_1024_lag3": (3, 0, True, 2, 3, 0.2, "1024"),
    "ps_same_1024_q1": (2, 0, True, 1, 3, 0.2, "1024"),
    "ps_all_circ_256_q3": (4, 1, True, 3, 1, 0.2, "256"),
    "ps_cross_256_q4": (1, 0, True, 4, 1, 0.2, "256"),
}


def weighted_dataset(pairs, weight, per_sample, q, R, gaps, shape):
    inj = dict(a_p=1.3, t_asc_off=0.0, period=68023.7, h0=0.3, cosi=0.8, psi=0.4, phi0=2.0)
    if shape == "small":
        cfg = small_config(q=q, n_seg=18, max_lag=R, pairs=pairs, gap_fraction=gaps,
                           injections=[dict(inj, f0=50.21, a_p=1.25)])
    else:
        t_short, n_seg = (400.0, 23) if shape == "256" else (2000.0, 30)
        cfg = small_config(q=q, n_seg=n_seg, t_short=t_short, f_min=400.0, f_band=0.06, max_lag=R, pairs=pairs,
                           a_p_max=2.0, gap_fraction=gaps,
                           templates=dict(a_p=(1.0, 2.0, 2), t_asc=(-200.0, 200.0, 2), period=[68023.70]),
                           injections=[dict(inj, f0=400.031)])
    cfg["band"]["weight"] = weight
    return synth.make_dataset(cfg, sigma_wander=0.2, per_sample_antenna=per_sample)


@pytest.mark.parametrize("case", sorted(WEIGHTED))
def test_weighted_pair_sums(ccr, case):
    """The Gamma^circ weight (Sec. II.B), every ordered pair with auto-correlations (App.
    A.1-A.2) and per-sample antenna functions (Sec. III.B.3, eq. norm-a-eq: two spectra streams
    per segment), alone and combined, on 128-, 256- and 1024-point segments with gaps, against
    the oracle's stream form; FP64 and split, chunks of 5 segments with their halo, the fused
    option set.  The split path runs the spectra + pair-sum kernel of 256- to 1024-point segments
    for both weights, all pairs and per-sample antenna functions (the resampler writes the two
    weighted series, the kernel transforms both; 1-4 detectors), the general kernels otherwise."""
    pairs, weight, per_sample, q, R, gaps, shape = WEIGHTED[case]
    ds = weighted_dataset(pairs, weight, per_sample, q, R, gaps, shape)
    o = oracle.Oracle(ds)
    ref = o.rho(ds.templates)
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        ctx.set_option("k_chunk", 5)
        ctx.set_option("fused", 1)
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        assert abs(info["norm"] / o.norm() - 1.0) < 1e-12
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        ctx.kernel_times(reset=True)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        kt = ctx.kernel_times(reset=True)
        ctx.set_option("template_batch", 1)
        r64b = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        r32b = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
    ns = info["n_s"]
    wide = ns in (256, 512, 1024)  # per-sample antenna functions there too (two streams)
    assert kt["spectra_pairs"][1] == 0, kt
    assert (kt["spectra_wide"][1] > 0) == wide and (kt["pairs"][1] > 0) != wide, kt
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"weighted {case}: fp64 {e64:.2e} split {e32:.2e} max|rho| {np.abs(ref).max():.2f}")
    assert e64 < TOL64 and e32 < TOL32
    assert np.array_equal(r64, r64b)  # one template per launch: same arithmetic
    assert np.array_equal(r32, r32b)


def test_weighted_forms_reduce(ccr):
    """Per-sample antenna functions that are constant over each segment give the per-segment
    result (one spectrum stream scaled, against two weighted streams), for Gamma^ave and
    Gamma^circ; the FP64 results agree to rounding."""
    for weight in (0, 1):
        ds = weighted_dataset(3, weight, False, 2, 2, 0.2, "small")
        with ccr.Context(ds.sky, device=0) as ctx:
            bid = ctx.load(ds)
            r_seg = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
            n_k = ctx.band_info(bid)["n_k"]
            for X in range(2):
                ctx.set_antenna(bid, X, np.repeat(ds.a[X], n_k), np.repeat(ds.b[X], n_k))
            r_ps = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        err = np.max(np.abs(r_ps - r_seg)) / max(1.0, np.abs(r_seg).max())
        print(f"constant per-sample weights, weight {weight}: {err:.2e}")
        assert err < 1e-12


WIDE_SMALLER = {
    # (detectors, max lag, pair kinds, chunk length, T_short, f_band, weight): 512-point segments
    # (N_K 257-512) and 256-point segments that the 256-point kernel does not take (more than 512
    # bins, or the Gamma^circ weight)
    "n512_q2_lag2_both": (2, 2, 3, 7, 1000.0, 0.06, 0),
    "n512_q3_lag1_cross": (3, 1, 1, 256, 1000.0, 0.06, 0),
    "n512_q1_lag3_same": (1, 3, 2, 5, 1000.0, 0.06, 0),
    "n512_q4_lag1_circ": (4, 1, 3, 6, 1000.0, 0.06, 1),
    "n256_q2_lag2_many_bins": (2, 2, 3, 7, 400.0, 0.2, 0),
    "n256_q3_lag1_circ": (3, 1, 3, 5, 400.0, 0.06, 1),
}


@pytest.mark.parametrize("case", sorted(WIDE_SMALLER))
def test_spectra_wide_512_256(ccr, case):
    """The spectra + pair-sum kernel on 512-point segments (radix 8, 8, 8 in one wavefront) and on
    256-point segments (radix 4, 4, 4, 4) where the 256-point kernel does not apply: 1-4
    detectors, lags 1-3, 30 % gaps, chunks with their halo, both weights, against the oracle
    (Sec. III.B.1 pairs, eq. final-formatted-rho, Sec. II.B Gamma^circ)."""
    q, R, pairs, kc, ts, fb, weight = WIDE_SMALLER[case]
    cfg = small_config(q=q, n_seg=26, t_short=ts, f_min=400.0, f_band=fb, max_lag=R, pairs=pairs,
                       a_p_max=2.0, gap_fraction=0.3,
                       templates=dict(a_p=(1.0, 2.0, 2), t_asc=(-200.0, 200.0, 2), period=[68023.70]),
                       injections=[dict(f0=400.0 + 0.45 * fb, a_p=1.3, t_asc_off=0.0, period=68023.7, h0=0.3,
                                        cosi=0.7, psi=0.4, phi0=2.0)])
    cfg["band"]["weight"] = weight
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    ref = oracle.Oracle(ds).rho(ds.templates)
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        ctx.set_option("k_chunk", kc)
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        ns = info["n_s"]
        assert ns == (512 if case.startswith("n512") else 256), info
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        ctx.kernel_times(reset=True)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        kt = ctx.kernel_times(reset=True)
    assert kt["spectra_wide"][1] > 0 and kt["spectra_pairs"][1] == 0, kt
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"{ns}-point {case}: n_f {info['n_f']} fp64 {e64:.2e} split {e32:.2e} max|rho| {np.abs(ref).max():.2f}")
    assert e64 < TOL64 and e32 < TOL32


WIDE_ONE_DET = {
    # (T_short, f_band, max lag, pair set, weight, per-sample antenna functions): one detector,
    # 1024-point segments, classes of 371-429 bins (more than the 256 that four bin columns a
    # lane of one wavefront cover: eight columns a lane)
    "same_ave_429": (1000.0, 0.3, 2, 2, 0, False),
    "same_circ_371": (1440.0, 0.3, 1, 2, 1, False),
    "all_ave_429": (600.0, 0.5, 2, 4, 0, False),
    "same_ps_429": (1000.0, 0.3, 2, 2, 0, True),
}


@pytest.mark.parametrize("case", sorted(WIDE_ONE_DET))
def test_spectra_wide_one_detector_wide_classes(ccr, case):
    """The spectra + pair-sum kernel with one detector and more than 256 bins in a residue class
    (up to 8 bin columns a lane): same-detector pairs at lags 1-2, both weights, every ordered pair
    with autos, per-sample antenna functions; 30 % gaps, chunks with their halo; FP64 (general
    path) and split against the oracle (Sec. III.B.1 pairs, eq. final-formatted-rho)."""
    ts, fb, R, pairs, weight, per_sample = WIDE_ONE_DET[case]
    cfg = small_config(q=1, n_seg=26, t_short=ts, f_min=400.0, f_band=fb, max_lag=R, pairs=pairs,
                       a_p_max=2.0, gap_fraction=0.3,
                       templates=dict(a_p=(1.0, 2.0, 2), t_asc=(-200.0, 200.0, 2), period=[68023.70]),
                       injections=[dict(f0=400.0 + 0.45 * fb, a_p=1.3, t_asc_off=0.0, period=68023.7, h0=0.3,
                                        cosi=0.7, psi=0.4, phi0=2.0)])
    cfg["band"]["weight"] = weight
    ds = synth.make_dataset(cfg, sigma_wander=0.2, per_sample_antenna=per_sample)
    ref = oracle.Oracle(ds).rho(ds.templates)
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        ctx.set_option("k_chunk", 7)
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        assert info["n_s"] == 1024 and info["n_f"] / info["P"] > 256, info
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        ctx.kernel_times(reset=True)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        kt = ctx.kernel_times(reset=True)
    assert kt["spectra_wide"][1] > 0, kt
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"one detector {case}: n_f {info['n_f']} P {info['P']} fp64 {e64:.2e} split {e32:.2e} "
          f"max|rho| {np.abs(ref).max():.2f}")
    assert e64 < TOL64 and e32 < TOL32


def test_tiny_workload_full(ccr):
    """2 detectors, 2 days, T_short 360 s, 0.25 Hz at 100 Hz, 64 templates, same-time pairs."""
    ds = synth.make_dataset(synth.config("tiny"))
    ref = oracle.Oracle(ds).rho(ds.templates)
    r64, r32 = run_both(ccr, ds, ds.templates)
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"tiny: fp64 {e64:.2e} split {e32:.2e} peak {ref.max():.2f}")
    assert e64 < TOL64 and e32 < TOL32
    assert np.unravel_index(r32.argmax(), r32.shape) == np.unravel_index(ref.argmax(), ref.shape)


def test_batching_and_determinism(ccr):
    """One template per launch and many per launch give bitwise-identical FP64 rho; repeated
    runs are bitwise reproducible."""
    ds = synth.make_dataset(small_config(n_seg=16, max_lag=2, gap_fraction=0.2))
    a, _ = run_both(ccr, ds, ds.templates, template_batch=1)
    b, _ = run_both(ccr, ds, ds.templates, template_batch=0)
    c, _ = run_both(ccr, ds, ds.templates, template_batch=4, k_chunk=3)
    assert np.array_equal(a, b)
    assert np.max(np.abs(a - c)) < 1e-12 * max(1.0, np.abs(a).max())
    d, _ = run_both(ccr, ds, ds.templates)
    assert np.array_equal(b, d)


def test_fused_matches_staged(ccr):
    """The fused kernel (spectra kept in an LDS ring, halo of R segments recomputed at chunk
    starts) reproduces the staged kernels' FP64 rho for any chunking."""
    ds = synth.make_dataset(small_config(q=3, n_seg=30, max_lag=3, gap_fraction=0.2, pairs=3))
    staged, s32 = run_both(ccr, ds, ds.templates, fused=0, k_chunk=256)
    for kc in (1, 4, 7, 256):
        f64, f32 = run_both(ccr, ds, ds.templates, fused=1, k_chunk=kc)
        assert np.max(np.abs(f64 - staged)) < 1e-13 * max(1.0, np.abs(staged).max()), kc
        assert np.max(np.abs(f32 - s32)) < 1e-5 * max(1.0, np.abs(s32).max()), kc


def test_device_output_and_stream(ccr):
    import torch
    ds = synth.make_dataset(small_config(n_seg=8))
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        host = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        info = ctx.band_info(bid)
        out = torch.full((info["n_templates"], info["n_f"]), float("nan"), dtype=torch.float32, device="cuda")
        s = torch.cuda.Stream()
        ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False, outputs=[out.data_ptr()], stream=s.cuda_stream)
        ctx.sync()
        assert np.array_equal(out.cpu().numpy(), host)


def test_edge_cases(ccr):
    # one detector entirely in a gap: no pair carries weight, rho == 0 everywhere
    cfg = small_config(n_seg=6, max_lag=1, pairs=1)
    ds = synth.make_dataset(cfg)
    ds.valid[1][:] = 0
    ds.x[1][:] = 0
    r64, r32 = run_both(ccr, ds, ds.templates)
    assert np.all(r64 == 0) and np.all(r32 == 0)
    # a single segment, a single template, ragged data tail (n not a multiple of N_K)
    cfg = small_config(n_seg=1, max_lag=0, pairs=1)
    ds = synth.make_dataset(cfg)
    ds.x = np.concatenate([ds.x, ds.x[:, :37]], axis=1)
    ds.valid = np.concatenate([ds.valid, ds.valid[:, :37]], axis=1)
    ref = oracle.Oracle(ds).rho(ds.templates[:1])
    r64, r32 = run_both(ccr, ds, ds.templates[:1])
    assert rho_err(r64, ref) < TOL64 and rho_err(r32, ref) < TOL32


@pytest.fixture(scope="module")
def band_workload():
    return synth.make_dataset(synth.config("band"))


def golden(name):
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    index = json.load(open(os.path.join(here, "oracle_values.json")))
    return index[name], np.load(os.path.join(here, f"oracle_{name}.npy"))


def nearest_template(templates, inj):
    d = ((templates[:, 0] - inj["a_p"]) ** 2 + ((templates[:, 1] - inj["t_asc"]) / 1000.0) ** 2
         + ((templates[:, 2] - inj["period"]) / 0.04) ** 2)
    return int(np.argmin(d))


def test_band_workload_sampled(ccr, band_workload):
    """Full-size realistic band (120 days, 30 % gaps, 4096 templates, lag 0) in the benchmark's
    launch configuration: the templates nearest each of the 10 injections plus 8 random ones,
    every bin, against the oracle (values stored by tests/golden/make_oracle_values.py); the
    error at each injection's peak (nearest template, bin nearest f0) is reported."""
    ds = band_workload
    meta, ref = golden("band")
    pick = meta["templates"]
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        _, freqs = ctx.band_info(bid, freqs=True)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
    e64, e32 = rho_err(r64[pick], ref), rho_err(r32[pick], ref)
    print(f"band: fp64 {e64:.2e} split {e32:.2e} over {len(pick)} templates, peak {ref.max():.2f}")
    for i, inj in enumerate(ds.injections):
        t = pick.index(nearest_template(ds.templates, inj))
        k = int(np.argmin(np.abs(freqs - inj["f0"])))
        print(f"  injection {i}: f0 {inj['f0']:.5f} rho_oracle {ref[t, k]:7.3f}  |d rho|/rho fp64 "
              f"{abs(r64[pick[t], k] - ref[t, k]) / abs(ref[t, k]):.2e} split "
              f"{abs(r32[pick[t], k] - ref[t, k]) / abs(ref[t, k]):.2e}")
    assert e64 < TOL64 and e32 < TOL32
    # properties at full size: finite everywhere, noise-dominated bins near unit variance
    assert np.all(np.isfinite(r32)) and np.all(np.isfinite(r64))
    assert 0.8 < np.median(np.abs(r64)) / 0.6745 < 1.25


def test_workspace_rounds(ccr, band_workload):
    """The workspace budget only changes how templates are packed into launch rounds: 40
    templates of the band in one round (default budget) and in 40 (64 MiB, less than one
    template's FP64 series) give bitwise-equal FP64 rho and split rho within rounding."""
    ds = band_workload
    tm = ds.templates[:40]
    a64, a32 = run_both(ccr, ds, tm)
    b64, b32 = run_both(ccr, ds, tm, workspace_mb=64)
    assert np.array_equal(a64, b64)
    assert np.max(np.abs(a32 - b32)) <= 1e-6 * max(1.0, np.abs(a32).max())


@pytest.fixture(scope="module")
def large_workload():
    return synth.make_dataset(synth.config("large"))


@pytest.mark.parametrize("which", ["band", "large"])
def test_resampled_series_compute_path_time_base(ccr, which, band_workload, large_workload):
    """The split stage output is made by the compute path's own time base and resampler: the
    band's Chebyshev node rule and small-angle series (5 nodes and the short series on the
    120-day band, 6 nodes on the 240-day one, chosen by the host's error bounds) and the Farrow
    form; element by element over the full series of detector 0 against the oracle's
    long-double Newton solve and direct sinc sum (Sec. III.A.1-2), 2e-6 of the peak, for a
    template near an injection, over the first 3000 (120 days) or 400 (240 days) segments, on
    the segments the compute path resamples (those that take part in a pair).""" 
    import copy
    full = band_workload if which == "band" else large_workload
    inj = full.injections[0]
    t = int(np.argmin((full.templates[:, 0] - inj["a_p"]) ** 2 + ((full.templates[:, 1] - inj["t_asc"]) / 1000.0) ** 2))
    # the first segments of the workload (same band, lattice, gaps and templates; the time base
    # of a sample depends only on its time), so that the oracle's per-sample solve stays short
    m_sub = 3000 if which == "band" else 400
    ds = copy.copy(full)
    nsamp = m_sub * full.n_k
    ds.x, ds.valid = full.x[:, :nsamp], full.valid[:, :nsamp]
    ds.a, ds.b, ds.noise_var = full.a[:, :m_sub], full.b[:, :m_sub], full.noise_var[:, :m_sub]
    ds.n, ds.n_seg = nsamp, m_sub
    o = oracle.Oracle(ds)
    y_ref, js, off, m0 = o.resample(0, ds.templates[t])
    m1 = o.resample(1, ds.templates[t])[3]
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds, templates=ds.templates[t:t + 1])
        y32 = ctx.resample_series(bid, 0, 0, prec=ccr.PREC_SPLIT)
    # the compute path resamples only segments that take part in a pair (Sec. III.B.1 with the
    # band's lag and pair kinds): segment K of detector 0 has data and a partner with data
    M, nk, R, pairs = ds.n_seg, ds.n_k, ds.band["max_lag"], ds.band.get("pairs", 3)
    a0 = m0[:M * nk].reshape(M, nk).any(axis=1)
    a1 = m1[:M * nk].reshape(M, nk).any(axis=1)
    near = lambda a, same: np.array([a[max(0, K - R):K + R + 1].sum() - (a[K] if same else 0) > 0 for K in range(M)])
    active = a0 & (((pairs & 1) != 0) & near(a1, False) | ((pairs & 2) != 0) & near(a0, True))
    act = np.repeat(active, nk)
    scale = np.abs(y_ref).max()
    err = np.abs(y32[:M * nk][act] - y_ref[:M * nk][act]).max() / scale
    print(f"{which}: split resampled series over {act.sum()} samples of {active.sum()} active segments "
          f"(of {M}), template {t}: {err:.2e} of the peak")
    assert err < 2e-6
    assert not np.any(y32[:M * nk][~act])


def test_large_workload_sampled(ccr, large_workload):
    """Largest workload (2 detectors, 240 days, T_short 1440 s, lags up to 4 segments, 0.25 Hz
    at 400 Hz: N_K = 870, N_FFT = 32768 = 32 x 1024, 7413 bins, 2.4e5 pairs) in the benchmark's
    launch configuration (the first 1002 templates of the grid, graph capture, autotuned launch
    shapes), with the sampled templates appended: 8 random templates of the first 1002 and the
    templates nearest 8 injections whose frequency falls in the slice, over a contiguous
    1024-bin slice, against stored oracle values."""
    ds = large_workload
    meta, ref = golden("large")
    pick = meta["templates"]
    lo, hi = meta["bins"]
    tm = np.vstack([ds.templates[:meta["first_templates"]], ds.templates[pick]])
    rows = np.arange(meta["first_templates"], len(tm))
    print("large: data ready", flush=True)
    import torch
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds, templates=tm)
        info, freqs = ctx.band_info(bid, freqs=True)
        assert (info["n_k"], info["n_fft"], info["n_f"]) == (870, 32768, 7413)
        ctx.set_option("graph", 1)
        ctx.set_option("autotune", 1)
        out = torch.empty((len(tm), info["n_f"]), dtype=torch.float32, device="cuda")
        for _ in range(2):  # capture, then replay
            ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False, outputs=[out.data_ptr()])
            ctx.sync()
            r32 = out.cpu().numpy()
        ctx.set_option("graph", 0)
        ctx.set_option("autotune", 0)
        ctx.set_templates(bid, ds.templates[pick])
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
    print("large: device rho done", flush=True)
    e64, e32 = rho_err(r64[:, lo:hi], ref), rho_err(r32[rows, lo:hi], ref)
    print(f"large: fp64 {e64:.2e} split {e32:.2e} over {len(pick)} templates x {hi - lo} bins, "
          f"max|rho| {np.abs(ref).max():.2f}")
    for inj in ds.injections:
        t = nearest_template(ds.templates, inj)
        k = int(np.argmin(np.abs(freqs - inj["f0"])))
        if t in pick and lo <= k < hi:
            j = pick.index(t)
            print(f"  injection f0 {inj['f0']:.5f}: rho_oracle {ref[j, k - lo]:7.3f} |d rho|/rho fp64 "
                  f"{abs(r64[j, k] - ref[j, k - lo]) / abs(ref[j, k - lo]):.2e} split "
                  f"{abs(r32[rows[j], k] - ref[j, k - lo]) / abs(ref[j, k - lo]):.2e}")
    assert e64 < TOL64 and e32 < TOL32
    # every bin of every template at full size: finite; the split path within its bar of the
    # FP64 path on the sampled templates (100 injections fill the band, so noise-only
    # statistics do not apply here)
    assert np.all(np.isfinite(r32)) and np.all(np.isfinite(r64))
    assert rho_err(r32[rows], r64) < TOL32


def test_time_base_parity(ccr, large_workload):
    """Step 1 alone at the largest span (240 days, 400 Hz): the FP64 delay eta - D_a and the
    heterodyne phase frac(f_het Delta) of samples spread over the whole observation against the
    oracle's long-double Newton solve of the full time map.  The delay of sample r is returned
    as a small eta and the anchor offset D_a (|D_a| <= 500 s, stored in FP64: half an ulp is
    2.8e-14 s); the phase is carried without that rounding.  Bars from the FP64 arithmetic:
    |eta| <= a_p + A_o w_o T_short / 2 ~ 2.1 s, so evaluating the degree-9 interpolant rounds to
    ~10 eps |eta| ~ 2.3e-15 s, i.e. 1e-12 cycles at 400 Hz; the delay adds the D_a rounding."""
    worst_d, worst_p = _time_base_errors(ccr, large_workload, [7, 50000, 100199])
    print(f"time base: delay {worst_d:.2e} s, phase {worst_p:.2e} cycles")
    assert worst_d < 5e-14
    assert worst_p < 2e-12


def test_time_base_parity_band(ccr, band_workload):
    """The same check on the realistic band (120 days, 30 % gaps, T_short 600 s, 200 Hz), at the
    corners of its template grid."""
    worst_d, worst_p = _time_base_errors(ccr, band_workload, [0, 63, 4032, 4095])
    print(f"time base (band): delay {worst_d:.2e} s, phase {worst_p:.2e} cycles")
    assert worst_d < 5e-14
    assert worst_p < 2e-12


def _time_base_errors(ccr, ds, picks):
    o = oracle.Oracle(ds)
    LD = np.longdouble
    n_k, M = ds.n_k, ds.n_seg
    tm = ds.templates[picks]
    worst_d = worst_p = 0.0
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds, templates=tm)
        for t in range(len(tm)):
            for X in range(ds.n_det):
                for K in (0, 1, M // 3, M // 2, M - 2, M - 1):
                    eta, anc, psi = ctx.time_base(bid, t, X, k0=K, n_seg=1)
                    for s in (0, 1, n_k // 2, n_k - 1):
                        hi, lo = o.delay(X, tm[t], K * n_k + s)
                        dref = LD(hi) + LD(lo)
                        worst_d = max(worst_d, abs(float(LD(eta[0, s]) - LD(anc[0]) - dref)))
                        pref = LD(ds.f_het) * dref
                        dp = float(LD(psi[0, s]) - (pref - np.floor(pref)))
                        worst_p = max(worst_p, abs(dp - round(dp)))
    return worst_d, worst_p


@pytest.fixture(scope="module")
def multiband_small():
    """Eight bands of the batching workload (3 detectors with uneven coverage, gaps fixed in
    time, T_short 1400 s at 50 Hz down to 247 s at 395 Hz, N_K 150-400, lag 1) over 10 days."""
    return synth.make_multiband(synth.config("multiband"), bands=[0, 9, 18, 27, 36, 45, 54, 63],
                                t_obs=10 * 86400.0)


def test_multiband_one_call(ccr, multiband_small):
    """All bands in one compute call (shared launches across bands, mixed kernel variants):
    FP64 rho bitwise equal to one call per band, and both precisions against the oracle."""
    dss = multiband_small
    pick = [0, 531]
    with ccr.Context(dss[0].sky, device=0) as ctx:
        ids = [ctx.load(ds, templates=ds.templates[pick]) for ds in dss]
        nks = sorted({ctx.band_info(b)["n_k"] for b in ids})
        assert nks[0] <= 256 < nks[-1]  # both the 256-point and the general FFT path
        r64 = ctx.compute_rho(ids, prec=ccr.PREC_FP64)
        r32 = ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False)
        singles = [ctx.compute_rho(b, prec=ccr.PREC_FP64) for b in ids]
    for a, b in zip(r64, singles):
        assert np.array_equal(a, b)
    worst64 = worst32 = 0.0
    for ds, a, b in zip(dss, r64, r32):
        ref = oracle.Oracle(ds).rho(ds.templates[pick])
        worst64, worst32 = max(worst64, rho_err(a, ref)), max(worst32, rho_err(b, ref))
    print(f"multiband: fp64 {worst64:.2e} split {worst32:.2e} over {len(dss)} bands")
    assert worst64 < TOL64 and worst32 < TOL32


def test_multiband_full_size_one_call(ccr):
    """The batching form at its configured size: 8 bands of the multi-band workload (0.05-0.2 Hz
    between 50 and 395 Hz, T_short 1400-247 s, 3 detectors with uneven coverage and gaps, lag 1)
    over the full 120 days with 1024 templates each, all in one compute call with graph capture
    and autotuned launch shapes; 2 templates per band (the nearest to the band's injection where
    it has one) against stored oracle values, every bin."""
    import torch
    meta, ref = golden("multiband")
    dss = synth.make_multiband(synth.config("multiband"), bands=meta["bands"])
    print("multiband full: data ready", flush=True)
    with ccr.Context(dss[0].sky, device=0) as ctx:
        ids = [ctx.load(ds) for ds in dss]
        infos = [ctx.band_info(b) for b in ids]
        assert all(i["n_templates"] == 1024 for i in infos)
        assert [i["n_f"] for i in infos] == meta["n_f"]
        ctx.set_option("graph", 1)
        ctx.set_option("autotune", 1)
        outs = [torch.empty((1024, i["n_f"]), dtype=torch.float32, device="cuda") for i in infos]
        for _ in range(2):
            ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False, outputs=[o.data_ptr() for o in outs])
            ctx.sync()
        r32 = [o.cpu().numpy() for o in outs]
        ctx.set_option("graph", 0)
        ctx.set_option("autotune", 0)
        for b, p in zip(ids, meta["templates"]):
            ctx.set_templates(b, dss[ids.index(b)].templates[p])
        r64 = ctx.compute_rho(ids, prec=ccr.PREC_FP64)
    worst64 = worst32 = 0.0
    for i, (p, n_f) in enumerate(zip(meta["templates"], meta["n_f"])):
        e64, e32 = rho_err(r64[i], ref[i, :, :n_f]), rho_err(r32[i][p], ref[i, :, :n_f])
        print(f"  band {meta['bands'][i]} (n_k {infos[i]['n_k']}, n_f {n_f}): fp64 {e64:.2e} split {e32:.2e}")
        worst64, worst32 = max(worst64, e64), max(worst32, e32)
        assert np.all(np.isfinite(r32[i]))
    print(f"multiband full size: fp64 {worst64:.2e} split {worst32:.2e}")
    assert worst64 < TOL64 and worst32 < TOL32


def test_graph_capture_replays(ccr, multiband_small):
    """With option graph = 1 a compute call is captured once and replayed: every replay, with
    eager work and synchronisations between them, equals the eager result bitwise; a fused call
    that grows the workspace, and new templates, make the next call re-capture."""
    import torch
    dss = multiband_small[:3]
    with ccr.Context(dss[0].sky, device=0) as ctx:
        ids = [ctx.load(ds, templates=ds.templates[:6]) for ds in dss]
        eager = ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False)
        outs = [torch.empty(e.shape, dtype=torch.float32, device="cuda") for e in eager]
        ctx.set_option("graph", 1)
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False, outputs=[o.data_ptr() for o in outs])
            ctx.sync()
            for o, e in zip(outs, eager):
                assert np.array_equal(o.cpu().numpy(), e), rep
            ctx.compute_rho(ids[0], prec=ccr.PREC_FP64)  # eager work between replays
        # a fused call that needs a larger workspace moves it: the next call re-captures instead
        # of replaying launches that hold the old buffers
        ctx.set_option("fused", 1)
        ctx.set_option("timing", 1)
        big = ctx.load(dss[0], templates=dss[0].templates[:48])
        ctx.kernel_times(reset=True)
        ctx.compute_rho(big, prec=ccr.PREC_SPLIT, out_fp64=False)
        assert ctx.kernel_times(reset=True)["fused"][1] > 0  # the fused kernel ran
        ctx.set_option("timing", 0)
        ctx.set_option("fused", 0)
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False, outputs=[o.data_ptr() for o in outs])
        ctx.sync()
        for o, e in zip(outs, eager):
            assert np.array_equal(o.cpu().numpy(), e)
        ctx.set_templates(ids[1], dss[1].templates[10:16])
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False, outputs=[o.data_ptr() for o in outs])
        ctx.sync()
        ctx.set_option("graph", 0)
        fresh = ctx.compute_rho(ids, prec=ccr.PREC_SPLIT, out_fp64=False)
        for o, e in zip(outs, fresh):
            assert np.array_equal(o.cpu().numpy(), e)
        assert not np.array_equal(fresh[1], eager[1])


def test_autotune_picks_chunk(ccr):
    """Option autotune = 1 times the candidate pair-sum chunk lengths on the first call, keeps
    the fastest, and gives the untuned rho up to summation order."""
    ds = synth.make_dataset(small_config(n_seg=64, max_lag=1, gap_fraction=0.1))
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        base = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        ctx.set_option("autotune", 1)
        tuned = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        kc = ctx.get_option("tuned_k_chunk")
        assert kc in (32, 64, 128)
        assert ctx.get_option("tuned_template_batch") > 0
        assert ctx.get_option("tuned_spectra_kernel") in (0, 1)
        assert np.max(np.abs(tuned - base)) < 1e-12 * max(1.0, np.abs(base).max())
        again = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
        assert np.array_equal(again, tuned)
        assert ctx.get_option("tuned_k_chunk") == kc


def test_spectra_kernel_choice_and_tuning(ccr):
    """A band of 256-point segments that both spectra + pair-sum kernels take (Gamma^ave, lagged
    pairs of both kinds, 20 % gaps): option spectra_kernel selects the 256-point kernel (0) or
    the 256- to 1024-point one (1), both match the oracle (Sec. III.B.1 pairs, eq.
    final-formatted-rho), and the autotuner, timing both kernels, the chunk lengths and the
    template batches, keeps one shape and gives the same rho to FP32 rounding."""
    cfg = small_config(q=2, n_seg=40, t_short=400.0, f_min=400.0, f_band=0.06, max_lag=2, pairs=3,
                       a_p_max=2.0, gap_fraction=0.2,
                       templates=dict(a_p=(1.0, 2.0, 3), t_asc=(-200.0, 200.0, 3), period=[68023.70]),
                       injections=[dict(f0=400.03, a_p=1.5, t_asc_off=0.0, period=68023.7, h0=0.3,
                                        cosi=0.7, psi=0.4, phi0=2.0)])
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    ref = oracle.Oracle(ds).rho(ds.templates)
    out = {}
    with ccr.Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        assert 128 < info["n_k"] <= 256, info
        for sk in (0, 1):
            ctx.set_option("spectra_kernel", sk)
            ctx.kernel_times(reset=True)
            out[sk] = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
            kt = ctx.kernel_times(reset=True)
            assert (kt["spectra_pairs"][1] > 0) == (sk == 0) and (kt["spectra_wide"][1] > 0) == (sk == 1), kt
        ctx.set_option("spectra_kernel", 0)
        ctx.set_option("autotune", 1)
        tuned = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        sk = ctx.get_option("tuned_spectra_kernel")
        tb = ctx.get_option("tuned_template_batch")
        kc = ctx.get_option("tuned_k_chunk")
    e0, e1, et = rho_err(out[0], ref), rho_err(out[1], ref), rho_err(tuned, ref)
    print(f"256-point kernel {e0:.2e}, wide kernel {e1:.2e}, tuned (kernel {sk}, k_chunk {kc}, batch {tb}) {et:.2e}")
    assert e0 < TOL32 and e1 < TOL32 and et < TOL32
    assert sk in (0, 1) and tb > 0 and kc >= 32
    assert rho_err(tuned, out[sk]) < 1e-5


# ------------------------------------------------------- eccentric orbits

def _ecc_grid(t_p0):
    # eccentricities 0 ... 0.5, two arguments of periapse, two periapse times
    rows = []
    for e in (0.0, 0.1, 0.3, 0.5):
        for w in (0.8, 2.5):
            for dtp in (0.0, 900.0):
                rows.append([1.6, t_p0 + dtp, w, e, 68023.7])
    return np.array(rows)


def _ecc_dataset(q=2, R=1, pairs=3, gaps=0.2, n_seg=24, t_short=240.0):
    cfg = small_config(q=q, n_seg=n_seg, t_short=t_short, max_lag=R, pairs=pairs, gap_fraction=gaps,
                       f_min=100.0, f_band=0.3, a_p_max=2.0)
    cfg["injections"] = [dict(f0=100.13, a_p=1.6, t_asc_off=0.0, period=68023.7, h0=1.0, cosi=0.6, psi=0.2,
                              phi0=0.3, ecc=0.3, w=0.8, t_p_off=300.0)]
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    ds.templates = _ecc_grid(cfg["t_asc0"] + 300.0)
    ds.ecc = True
    return ds


ECC_CASES = {
    # (detectors, max lag, pair kinds, gap fraction, segments, T_short)
    "q2_lag1_both": (2, 1, 3, 0.2, 24, 240.0),
    "q3_lag2_cross": (3, 2, 1, 0.1, 18, 240.0),
    "q2_lag0_wide": (2, 0, 1, 0.2, 14, 600.0),
}


@pytest.mark.parametrize("case", sorted(ECC_CASES))
def test_eccentric_templates(ccr, case):
    """Eccentric orbital templates (Sec. II.A.2, eqs. solve-for-E and Kepler-equation; e up to
    0.5, two arguments of periapse, two periapse times) with an eccentric injection: the
    library's anchor-relative Kepler solve in the time base against the oracle's long-double
    solve of the full map, rho element by element, FP64 and split."""
    q, R, pairs, gaps, n_seg, ts = ECC_CASES[case]
    ds = _ecc_dataset(q, R, pairs, gaps, n_seg, ts)
    ref = oracle.Oracle(ds).rho(ds.templates)
    r64, r32 = run_both(ccr, ds, ds.templates, k_chunk=5)
    e64, e32 = rho_err(r64, ref), rho_err(r32, ref)
    print(f"eccentric {case}: fp64 {e64:.2e} split {e32:.2e} max|rho| {np.abs(ref).max():.2f} at template "
          f"{np.unravel_index(ref.argmax(), ref.shape)[0]}")
    assert e64 < TOL64 and e32 < TOL32


def test_eccentric_time_base(ccr):
    """The eccentric time base alone (e = 0.3 and 0.5): delay and heterodyne phase of samples of
    first, middle and last segments against the oracle's long-double Newton solve (bars as for
    the circular time base)."""
    ds = _ecc_dataset(n_seg=30, t_short=600.0, gaps=0.0)  # every segment computed
    ds.templates = ds.templates[[4, 5, 12, 15]]
    worst_d, worst_p = _time_base_errors(ccr, ds, [0, 1, 2, 3])
    print(f"eccentric time base: delay {worst_d:.2e} s, phase {worst_p:.2e} cycles")
    assert worst_d < 5e-14
    assert worst_p < 2e-12


def test_eccentric_zero_e_matches_circular(ccr):
    """e = 0 through the eccentric path equals the circular template with T_asc = T_p - omega /
    Omega (eq. Kepler-equation at e = 0) to rounding."""
    ds = _ecc_dataset(n_seg=16)
    P, w, tp = 68023.7, 0.8, ds.templates[0, 1]
    tm_e = np.array([[1.6, tp, w, 0.0, P], [1.2, tp + 500.0, 2.0, 0.0, P]])
    tm_c = np.array([[1.6, tp - w * P / (2 * math.pi), P], [1.2, tp + 500.0 - 2.0 * P / (2 * math.pi), P]])
    re64, re32 = run_both(ccr, ds, tm_e)
    rc64, rc32 = run_both(ccr, ds, tm_c)
    scale = max(1.0, np.abs(rc64).max())
    print(f"e = 0 vs circular: fp64 {np.abs(re64 - rc64).max() / scale:.2e} split {np.abs(re32 - rc32).max() / scale:.2e}")
    assert np.abs(re64 - rc64).max() < 1e-11 * scale
    assert np.abs(re32 - rc32).max() < 2e-5 * scale


# ------------------------------------------------------- SFT front end (App. B)

SFT_CASES = {
    # (N' samples per SFT, SFTs, f_het, SFT length)
    "n64_on_grid": (64, 16, 200.0, 240.0),
    "n63_odd": (63, 16, 200.013, 240.0),
    "n153_band1": (153, 12, 100.0, 360.0),
    "n179_prime": (179, 12, 199.9871, 600.0),
    "n870_large": (870, 6, 400.0, 1440.0),
    "n2048_lds_table": (2048, 4, 300.0021, 1800.0),
    "n3001_global_table": (3001, 3, 250.0003, 1800.0),
}


@pytest.mark.parametrize("case", sorted(SFT_CASES))
def test_sft_series_parity(ccr, case):
    """The SFT front end (App. B: band selection around k_h, inverse transform of the band, the
    remainder of f_h off the bin grid, the stitching phase across SFTs) against the oracle's
    long-double steps, element by element: white noise, two tones (one on a bin centre), a
    missing SFT; even, odd and prime N', twiddles from LDS and from global memory.  Bar: 2e-6 of
    the largest |x| (complex64 output of an FP64 sum)."""
    n_out, n_sft, f_het, t_sft = SFT_CASES[case]
    kh = int(round(f_het * t_sft))
    k_first = kh - n_out // 2 - 11
    n_bins = n_out + 23
    lines = [(f_het + 3.0 / t_sft, 2.0, 0.3), (f_het - 0.2 * n_out / t_sft + 0.37 / t_sft, 1.0, 1.1)]
    z, valid = synth.make_sfts(n_sft, t_sft, 1.0 / 4096.0, k_first, n_bins, t0=1234.0 * t_sft, lines=lines,
                               sigma=0.3, seed=n_out)
    valid[1] = 0
    z[1] = 0
    ref = oracle.sft_series(z, t_sft, 1234.0 * t_sft, k_first, f_het, n_out, sft_valid=valid)
    with ccr.Context(synth.default_sky(), device=0) as ctx:
        x, v = ctx.sft_series(z, t_sft, 1234.0 * t_sft, k_first, f_het, n_out, sft_valid=valid)
    err = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"SFT front end {case}: {err:.2e} of the peak")
    assert err < 2e-6
    assert np.array_equal(v, np.repeat(valid, n_out))
    assert np.all(x[n_out:2 * n_out] == 0)


def test_sft_series_errors(ccr):
    """Bins not held, too many output samples and NaN bins are rejected before any launch."""
    z, _ = synth.make_sfts(2, 240.0, 1.0 / 1024.0, 47900, 200, sigma=1.0)
    with ccr.Context(synth.default_sky(), device=0) as ctx:
        with pytest.raises(ccr.CcrError) as e:
            ctx.sft_series(z, 240.0, 0.0, 47900, 200.0, 256)
        assert e.value.status == ccr.ERANGE
        with pytest.raises(ccr.CcrError) as e:
            ctx.sft_series(z, 240.0, 0.0, 47900, 200.0, 5000)
        assert e.value.status == ccr.ERANGE
        zb = z.copy()
        zb[1, 3] = np.nan
        with pytest.raises(ccr.CcrError) as e:
            ctx.sft_series(zb, 240.0, 0.0, 47900, 200.0, 64)
        assert e.value.status == ccr.EINVAL


def test_sft_front_end_feeds_rho(ccr):
    """SFTs -> heterodyned series on the GPU -> rho on the GPU, against SFTs -> the oracle's series
    -> the oracle's rho: a bin-centred tone in noise, 2 detectors with their own SFTs (one SFT
    missing), T_sft = T_short and N' = N_K so the series falls on the band's lattice.  The two
    series differ by the complex64 rounding of the front end's output, so rho agrees to 1e-5."""
    cfg = small_config(n_seg=16, t_short=240.0, f_min=100.0, f_band=0.2, max_lag=1, gap_fraction=0.0)
    ds = synth.make_dataset(cfg, signal=False)
    n_k, t_sft = ds.n_k, cfg["band"]["t_short"]
    kh = int(round(ds.f_het * t_sft))
    k_first = kh - n_k // 2 - 4
    valid_sft = np.ones(ds.n_seg, dtype=np.uint8)
    valid_sft[5] = 0
    ref_ds = synth.make_dataset(cfg, signal=False)
    with ccr.Context(ds.sky, device=0) as ctx:
        for X in range(2):
            z, _ = synth.make_sfts(ds.n_seg, t_sft, 1.0 / 2048.0, k_first, n_k + 8, t0=ds.t0,
                                   lines=[((kh + 9) / t_sft, 2.0, 0.3 + X)], sigma=0.02, seed=10 + X)
            z[5] = 0
            x, v = ctx.sft_series(z, t_sft, ds.t0, k_first, ds.f_het, n_k, sft_valid=valid_sft)
            ds.x[X], ds.valid[X] = x, v
            xr = oracle.sft_series(z, t_sft, ds.t0, k_first, ds.f_het, n_k, sft_valid=valid_sft)
            ref_ds.x[X], ref_ds.valid[X] = xr.astype(np.complex64), np.repeat(valid_sft, n_k)
        bid = ctx.load(ds)
        r = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
    ref = oracle.Oracle(ref_ds).rho(ref_ds.templates)
    err = rho_err(r, ref)
    print(f"SFT -> series -> rho: {err:.2e}, max rho {ref.max():.2f}")
    assert err < 1e-5 and ref.max() > 5

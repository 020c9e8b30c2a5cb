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


def test_resampled_series_parity(ccr):
    cfg = small_config(n_seg=12, gap_fraction=0.2, max_lag=1)
    ds = synth.make_dataset(cfg)
    o = oracle.Oracle(ds)
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        for t in (0, 3, 5):
            for X in range(2):
                y_ref, js, off, m = o.resample(X, ds.templates[t])
                y64 = ctx.resample_series(bid, t, X, prec=ccr.PREC_FP64)
                y32 = ctx.resample_series(bid, t, X, prec=ccr.PREC_SPLIT)
                scale = np.abs(y_ref).max()
                assert np.abs(y64 - y_ref).max() < 1e-12 * scale
                assert np.abs(y32 - y_ref).max() < 2e-6 * scale
                assert np.all((y64 == 0) >= (m == 0))


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


def test_band_workload_sampled(ccr, band_workload):
    """Full-size realistic band (120 days, 30 % gaps, 4096 templates) in the benchmark's launch
    configuration; the oracle evaluates the templates nearest each injection plus random ones."""
    ds = band_workload
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        r32 = ctx.compute_rho(bid, prec=ccr.PREC_SPLIT, out_fp64=False)
        r64 = ctx.compute_rho(bid, prec=ccr.PREC_FP64)
    rng = np.random.default_rng(11)
    pick = set(rng.choice(len(ds.templates), 6, replace=False).tolist())
    for inj in ds.injections[:4]:
        d = (ds.templates[:, 0] - inj["a_p"]) ** 2 + ((ds.templates[:, 1] - inj["t_asc"]) / 1000.0) ** 2
        pick.add(int(np.argmin(d)))
    pick = sorted(pick)
    ref = oracle.Oracle(ds).rho(ds.templates[pick])
    e64, e32 = rho_err(r64[pick], ref), rho_err(r32[pick], ref)
    print(f"band: fp64 {e64:.2e} split {e32:.2e} over {len(pick)} templates, peak {ref.max():.2f}")
    assert e64 < TOL64 and e32 < TOL32
    # properties at full size: finite everywhere, noise-dominated bins near unit variance
    assert np.all(np.isfinite(r32)) and np.all(np.isfinite(r64))
    assert 0.8 < np.median(np.abs(r64)) / 0.6745 < 1.25

"""Host-side checks of the C ABI that need no GPU: the library loads, exports every symbol
include/ccr.h declares, validates arguments, and (in a host-only context, device -1) plans
bands exactly like the oracle."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import synth
from conftest import small_config
from paper_1712_06515_amd import ccr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ccr.LIB_PATH):
        from paper_1712_06515_amd import build
        build.build()
    return ccr.load_library()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ccr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ccr_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ccr.SIGNATURES), set(names) ^ set(ccr.SIGNATURES)
    assert lib.ccr_abi_version() == 4


def test_struct_layouts_match_header(lib):
    # sizes implied by the header field lists
    assert ctypes.sizeof(ccr.Sky) == 9 * 8
    assert ctypes.sizeof(ccr.Site) == 16
    assert ctypes.sizeof(ccr.Band) == 3 * 8 + 4 * 4 + 8 + 8 + 8 + 8 + 8  # int32 pairs, weight padded to 8
    assert ccr.Band.weight.offset == 72
    assert ctypes.sizeof(ccr.BandInfo) == 12 * 8 + 9 * 8  # 12 int64 (n_s, P last), 9 double


def test_null_and_bad_arguments(lib):
    assert lib.ccr_create(None, 0, None) == ccr.EINVAL
    h = ctypes.c_void_p()
    bad = ccr.Sky(0, 0, 499.0, 0.02, 0.4, -1.0, 86164.0, 0, 0)
    assert lib.ccr_create(ctypes.byref(h), -1, ctypes.byref(bad)) == ccr.EINVAL
    nan = ccr.Sky(float("nan"), 0, 499.0, 0.02, 0.4, 3e7, 86164.0, 0, 0)
    assert lib.ccr_create(ctypes.byref(h), -1, ctypes.byref(nan)) == ccr.EINVAL
    assert lib.ccr_set_option(None, b"fused", 1) == ccr.EINVAL
    assert lib.ccr_sync(None) == ccr.EINVAL
    assert lib.ccr_last_error(None) == b"null context"


def _host_ctx(ds):
    ctx = ccr.Context(ds.sky, device=-1)
    return ctx


def test_host_only_context_rejects_device_work(lib):
    ds = synth.make_dataset(small_config(n_seg=4), signal=False)
    ctx = _host_ctx(ds)
    bid = ctx.load(ds)
    with pytest.raises(ccr.CcrError) as e:
        ctx.compute_rho(bid)
    assert e.value.status == ccr.EDEVICE


def test_options_round_trip(lib):
    """Option values as documented in include/ccr.h: the workspace budget defaults to 0
    (automatic), explicit budgets are at least 64 MiB; read-only launch constants; unknown
    names and negative values are rejected."""
    ds = synth.make_dataset(small_config(n_seg=4), signal=False)
    ctx = _host_ctx(ds)
    assert ctx.get_option("workspace_mb") == 0
    ctx.set_option("workspace_mb", 10)
    assert ctx.get_option("workspace_mb") == 64
    ctx.set_option("workspace_mb", 4096)
    assert ctx.get_option("workspace_mb") == 4096
    ctx.set_option("workspace_mb", 0)
    assert ctx.get_option("workspace_mb") == 0
    assert ctx.get_option("resample_templates") == 4
    assert ctx.get_option("farrow") == 1
    ctx.set_option("farrow", 0)
    assert ctx.get_option("farrow") == 0
    assert ctx.get_option("farrow_templates") % 4 == 0  # whole wavefronts of a 4-wavefront workgroup
    assert ctx.get_option("farrow_degree") in (8, 9)
    assert ctx.get_option("farrow_stage") == 1
    assert ctx.get_option("tuned_k_chunk") == 0
    with pytest.raises(ccr.CcrError) as e:
        ctx.get_option("no_such_option")
    assert e.value.status == ccr.EUNSUP
    with pytest.raises(ccr.CcrError) as e:
        ctx.set_option("k_chunk", -1)
    assert e.value.status == ccr.EINVAL


def test_validation_errors(lib):
    ds = synth.make_dataset(small_config(n_seg=4), signal=False)
    ctx = _host_ctx(ds)
    bid, info = ctx.add_band(ds.band)
    assert info["n_k"] == ds.n_k and abs(info["dt"] - ds.dt) < 1e-15
    site = ds.sites[0]

    def err(fn, *a, **k):
        with pytest.raises(ccr.CcrError) as e:
            fn(*a, **k)
        return e.value.status

    # call order: no data yet
    assert err(ctx.band_info, bid) == ccr.ESTATE
    # dt that is not T_short / integer
    assert err(ctx.set_data, bid, 0, site, 0.0, ds.dt * 1.01, ds.x[0], ds.f_het) == ccr.EINVAL
    # dt that undersamples the load band
    assert err(ctx.set_data, bid, 0, site, 0.0, ds.band["t_short"] / (ds.n_k - 5), ds.x[0], ds.f_het) == ccr.ERANGE
    # wrong heterodyne frequency
    assert err(ctx.set_data, bid, 0, site, 0.0, ds.dt, ds.x[0], ds.f_het + 0.01) == ccr.EINVAL
    # NaN sample
    xb = ds.x[0].copy()
    xb[7] = np.nan
    assert err(ctx.set_data, bid, 0, site, 0.0, ds.dt, xb, ds.f_het) == ccr.EINVAL
    # bad detector index, too short
    assert err(ctx.set_data, bid, 9, site, 0.0, ds.dt, ds.x[0], ds.f_het) == ccr.EINVAL
    assert err(ctx.set_data, bid, 0, site, 0.0, ds.dt, ds.x[0][: ds.n_k - 1], ds.f_het) == ccr.EINVAL
    ctx.set_data(bid, 0, site, 0.0, ds.dt, ds.x[0], ds.f_het)
    # mismatched lattice origin for a second detector
    assert err(ctx.set_data, bid, 1, ds.sites[1], 1.0, ds.dt, ds.x[1], ds.f_het) == ccr.EINVAL
    # weights: non-positive noise, NaN
    nv = ds.noise_var[0].copy()
    nv[2] = 0.0
    assert err(ctx.set_weights, bid, 0, ds.a[0], ds.b[0], nv) == ccr.EINVAL
    aa = ds.a[0].copy()
    aa[1] = np.inf
    assert err(ctx.set_weights, bid, 0, aa, ds.b[0], ds.noise_var[0]) == ccr.EINVAL
    # weights of the wrong length are caught when the band is planned
    ctx.set_weights(bid, 0, ds.a[0][:-1], ds.b[0][:-1], ds.noise_var[0][:-1])
    assert err(ctx.band_info, bid) == ccr.EINVAL
    # templates
    assert err(ctx.set_templates, bid, np.array([[1.0, 0.0, -5.0]])) == ccr.EINVAL
    assert err(ctx.set_templates, bid, np.array([[-1.0, 0.0, 68023.7]])) == ccr.EINVAL
    assert err(ctx.set_templates, bid, np.zeros((0, 3))) == ccr.EINVAL  # no templates
    assert err(ctx.set_templates, bid, np.zeros((0, 5))) == ccr.EINVAL
    # options
    assert err(ctx.set_option, "no_such_option", 1) == ccr.EUNSUP
    # band fields
    b2 = dict(ds.band, pairs=0)
    assert err(ctx.add_band, b2) == ccr.EINVAL
    b3 = dict(ds.band, dirichlet_D=0)
    assert err(ctx.add_band, b3) == ccr.ERANGE
    b4 = dict(ds.band, n_fft_override=3 * 128 + 1)
    bid4, _ = ctx.add_band(b4)
    for X in range(2):
        ctx.set_data(bid4, X, ds.sites[X], 0.0, ds.dt, ds.x[X], ds.f_het)
        ctx.set_weights(bid4, X, ds.a[X], ds.b[X], ds.noise_var[X])
    assert err(ctx.band_info, bid4) == ccr.EINVAL
    # pair set ALL is not combined with CROSS / SAME; weight is AVE or CIRC
    assert err(ctx.add_band, dict(ds.band, pairs=ccr.PAIRS_ALL | ccr.PAIRS_CROSS)) == ccr.EINVAL
    assert err(ctx.add_band, dict(ds.band, pairs=8)) == ccr.EINVAL
    assert err(ctx.add_band, dict(ds.band, weight=2)) == ccr.EINVAL


def test_antenna_validation(lib):
    ds = synth.make_dataset(small_config(n_seg=4), signal=False, per_sample_antenna=True)
    ctx = _host_ctx(ds)
    bid = ctx.load(ds)
    ctx.band_info(bid)

    def err(fn, *a, **k):
        with pytest.raises(ccr.CcrError) as e:
            fn(*a, **k)
        return e.value.status

    bad = ds.ar[0].copy()
    bad[3] = np.nan
    assert err(ctx.set_antenna, bid, 0, bad, ds.br[0]) == ccr.EINVAL
    assert err(ctx.set_antenna, bid, 9, ds.ar[0], ds.br[0]) == ccr.EINVAL
    # too short for the band's segments: caught when the band is planned
    ctx.set_antenna(bid, 0, ds.ar[0][:-1], ds.br[0][:-1])
    assert err(ctx.band_info, bid) == ccr.EINVAL
    # set for one detector only
    ctx.set_antenna(bid, 0, None, None)
    assert err(ctx.band_info, bid) == ccr.EINVAL
    ctx.set_antenna(bid, 1, None, None)
    ctx.band_info(bid)  # per-segment weights again


@pytest.mark.parametrize("kw", [
    dict(),
    dict(max_lag=2, gap_fraction=0.25, n_seg=24),
    dict(max_lag=3, pairs=1, q=3, n_seg=20, gap_fraction=0.1),
    dict(max_lag=1, pairs=2, n_seg=12, mu_f=0.3),
    dict(n_fft_override=3 * 128, max_lag=1),
    dict(max_lag=2, gap_fraction=0.25, n_seg=24, weight=1),
    dict(max_lag=1, pairs=4, n_seg=12, gap_fraction=0.2),
    dict(max_lag=1, pairs=4, q=3, n_seg=10, weight=1),
    dict(max_lag=2, n_seg=14, gap_fraction=0.2, per_sample=True),
    dict(max_lag=1, pairs=1, n_seg=10, per_sample=True, weight=1),
    dict(max_lag=1, pairs=4, n_seg=10, per_sample=True, gap_fraction=0.1),
])
def test_plan_and_normalisation_match_oracle(lib, kw):
    """Band plan integers are bit-identical to the oracle's; the normalisation (weights, gap
    mask fractions, pair set, Gamma^ave or Gamma^circ, per-segment or per-sample antenna
    functions) agrees to rounding."""
    kw = dict(kw)
    weight, per_sample = kw.pop("weight", 0), kw.pop("per_sample", False)
    cfg = small_config(**kw)
    cfg["band"]["weight"] = weight
    ds = synth.make_dataset(cfg, sigma_wander=0.2, per_sample_antenna=per_sample)
    ctx = _host_ctx(ds)
    bid = ctx.load(ds)
    info, freqs = ctx.band_info(bid, freqs=True)
    o = oracle.Oracle(ds)
    pl = o.plan()
    for k in ("n_k", "n_seg", "n_fft", "n_f", "k_lo"):
        assert info[k] == getattr(pl, k), k
    for k in ("dt", "f_het", "df_load", "t_coh", "t_fft", "nu_r"):
        assert info[k] == getattr(pl, k), k
    assert info["dlambda_f"] == pl.dlambda_f
    assert info["n_pairs"] == o.pair_count()
    np.testing.assert_array_equal(freqs, o.frequencies())
    assert abs(info["norm"] / o.norm() - 1.0) < 1e-12


def test_plan_of_named_workloads(lib):
    """The library's recommended sampling matches the generator's App. B sizing for every named
    workload (three independent implementations of the load bandwidth)."""
    ctx = ccr.Context(synth.default_sky(), device=-1)
    for name in ("tiny", "band", "large"):
        band = synth.config(name)["band"]
        _, info = ctx.add_band(band)
        assert info["n_k"] == synth.samples_per_segment(band)
        assert abs(info["df_load"] - synth.load_bandwidth(band["f_min"], band["f_band"], band["t_short"],
                                                          band["a_p_max"])) < 1e-12


@pytest.mark.parametrize("window", [0, 1])
@pytest.mark.parametrize("D", [4, 8, 16])
def test_farrow_fit_error(lib, D, window):
    """The host's Farrow fit of the tap weights (polynomial in the offset of the library's
    degree, constant term exact): its reported bound, max over offsets of
    sum_n |fit - w sinc(dc - n)|, is below the 4e-7 the library accepts, for the Hamming window
    indexed by tap (0) and at the offset (1).  The
    bound is checked against an independent fit (numpy least squares on the same basis) that
    must reach the same error to within a factor 2, so neither a loose nor a wrong bound passes."""
    import numpy as np
    ds = synth.make_dataset(small_config(n_seg=4, dirichlet_D=D, window=window), signal=False)
    ctx = _host_ctx(ds)
    info = ctx.band_info(ctx.load(ds))
    assert info["farrow_degree"] == 0  # host-only context: no device table
    err = info["farrow_err"]
    deg = ctx.get_option("farrow_degree")
    n = np.arange(-D, D + 1)

    def taps(dc):
        d = dc[:, None] - n[None, :]
        w = (0.54 - 0.46 * np.cos(np.pi * (n + D) / D)) if window == 0 else 0.54 + 0.46 * np.cos(np.pi * d / (D + 1))
        return w * np.sinc(d)

    xs = 0.5 * np.cos(np.pi * (np.arange(64) + 0.5) / 64)
    V = np.vander(xs, deg, increasing=True) * xs[:, None]
    c0 = (n == 0).astype(float)
    A = np.linalg.lstsq(V, taps(xs) - c0[None, :], rcond=None)[0]
    xt = np.linspace(-0.5, 0.5, 4001)
    ref = np.abs(c0[None, :] + xt[:, None] * (np.vander(xt, deg, increasing=True) @ A) - taps(xt)).sum(1).max()
    assert err < 4e-7
    assert 0.5 * ref < err < 2.0 * ref


def test_farrow_fit_rejected_for_long_windows(lib):
    """Windows of 2D + 1 = 49 taps: the degree-8 fit's bound exceeds the 4e-7 the library
    accepts, so such a band keeps the direct tap sum on the split path."""
    ds = synth.make_dataset(small_config(n_seg=4, dirichlet_D=24), signal=False)
    ctx = _host_ctx(ds)
    info = ctx.band_info(ctx.load(ds))
    if ctx.get_option("farrow_degree") == 8:
        assert info["farrow_err"] > 4e-7
    assert info["farrow_degree"] == 0


def test_eccentric_template_validation(lib):
    """Eccentric templates (a_p, T_p, omega, e, P): e outside [0, 0.95] or a non-finite value is
    rejected when set; an orbit whose time-base interpolation over a segment the library cannot
    bound (e = 0.9 with 1800 s segments) is rejected when the band is prepared, while moderate
    eccentricities pass."""
    ds = synth.make_dataset(small_config(n_seg=4, t_short=1800.0), signal=False)
    ctx = _host_ctx(ds)
    bid = ctx.load(ds)

    def err(fn, *a, **k):
        with pytest.raises(ccr.CcrError) as e:
            fn(*a, **k)
        return e.value.status

    P = 68023.7
    assert err(ctx.set_templates, bid, np.array([[1.0, 0.0, 0.3, 0.96, P]])) == ccr.EINVAL
    assert err(ctx.set_templates, bid, np.array([[1.0, 0.0, 0.3, -0.1, P]])) == ccr.EINVAL
    assert err(ctx.set_templates, bid, np.array([[1.0, np.nan, 0.3, 0.1, P]])) == ccr.EINVAL
    with pytest.raises(ValueError):
        ctx.set_templates(bid, np.zeros((2, 4)))
    ctx.set_templates(bid, np.array([[1.5, 100.0, 0.3, 0.3, P], [1.0, 0.0, 2.0, 0.0, P]]))
    assert ctx.band_info(bid)["n_templates"] == 2
    ctx.set_templates(bid, np.array([[1.5, 100.0, 0.3, 0.9, P]]))
    assert err(ctx.band_info, bid) == ccr.ERANGE
    ctx.set_templates(bid, np.array([[1.5, 100.0, P]]))
    assert ctx.band_info(bid)["n_templates"] == 1

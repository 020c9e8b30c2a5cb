"""The timing model of eq. resampTimingModelEq (Sec. IV.B): its terms from a band plan, and the fit
of its three constants (host code, no GPU)."""

import math

import numpy as np
import pytest

import oracle
import synth
from conftest import small_config
from paper_1712_06515_amd import ccr, timing_model as tmod


def test_terms_from_plan():
    """The three terms for a 3-detector band against the formula written out from the oracle's own
    plan: N_orb N_det M [N_f triang, 2 N_K D / 8, N_FFT 5 log2 N_FFT triang], triang(3) = 3."""
    ds = synth.make_dataset(small_config(q=3, n_seg=12, max_lag=1, dirichlet_D=4), signal=False)
    ctx = ccr.Context(ds.sky, device=-1)
    info = ctx.band_info(ctx.load(ds))
    pl = oracle.Oracle(ds).plan()
    f = tmod.features(info, 10, 4)
    lead = 10 * 3 * pl.n_seg
    assert tmod.triang(3) == 3.0 and tmod.triang(1) == 2.0
    assert f[0] == lead * pl.n_f * 3.0
    assert f[1] == lead * 2.0 * pl.n_k * 0.5
    assert f[2] == pytest.approx(lead * pl.n_fft * 5 * math.log2(pl.n_fft) * 3.0, rel=1e-15)


def test_fit_recovers_known_constants():
    """Run times made from known constants (the paper's low-N_FFT Table II values) with 2 % noise
    over the sweep's plans: the fit returns the constants within their reported uncertainty (3
    sigma) and 10 %, and the relative rms residual near the noise level; a kernel path with too
    few rows is left unfitted."""
    rng = np.random.default_rng(3)
    tau = np.array([1.01e-7, 1.62e-7, 5.27e-10])
    rows = []
    for c in tmod.sweep_configs():
        n_k = int(rng.integers(100, 1000))
        ns = 1 << (n_k - 1).bit_length()
        info = dict(n_det=c["q"], n_seg=int(c["t_obs"] / c["t_short"]), n_f=int(rng.integers(50, 3000)), n_k=n_k,
                    n_fft=ns * int(rng.choice([1, 2, 4, 8, 16])))
        x = tmod.features(info, 256, c["D"])
        rows.append(dict(features=list(x), seconds=float(x @ tau) * (1 + 0.02 * rng.standard_normal()),
                         path="general" if len(rows) % 8 else "wide"))
    m = tmod.fit(rows)
    assert m["fused256"] is None and m["wide"] is not None
    low = m["general"]
    for i, n in enumerate(tmod.NAMES):
        assert abs(low["tau"][n] - tau[i]) < max(3 * low["sigma"][n], 1e-12)
        assert abs(low["tau"][n] / tau[i] - 1) < 0.1
    assert 0.01 < low["rel_rms"] < 0.03
    info = dict(n_det=2, n_seg=100, n_f=300, n_k=200, n_fft=1024)
    assert tmod.predict(m, info, 5, 8, "general") == pytest.approx(float(tmod.features(info, 5, 8) @
                                                               np.array([low["tau"][n] for n in tmod.NAMES])))

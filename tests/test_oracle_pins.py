"""Pins of the oracle against what the paper and mathematics fix (CPU only).

Each test names the passage it pins.  None re-calls the oracle's own formula
to check itself: the references are printed values (tests/golden), closed
forms, special cases with known answers, an independently written forward
model (synth) and numpy transforms.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth.generate import Dataset
from conftest import small_config

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
NO_EARTH = dict(au_s=0.0, re_s=0.0)


def _pole_site():
    return dict(lat=math.pi / 2, lon=0.0, xaz=0.0, yaz=math.pi / 2)


# ----------------------------------------------------------------- planner

def test_plan_mu_f_statements():
    """Sec. III.B.2: mu_f = 0.1 needs T_FFT >= 2.3 T_coh; delta lambda_f T_coh < 1 up to mu_f ~ 0.52."""
    g = GOLD["fft_duration_mu_0p1"]
    ds = synth.make_dataset(small_config(mu_f=g["mu_f"]), signal=False)
    pl = oracle.Oracle(ds).plan()
    ratio = 1.0 / (pl.dlambda_f * pl.t_coh)
    assert round(ratio, 1) == g["t_fft_over_t_coh"]
    assert pl.t_fft >= ratio * pl.t_coh * (1 - 1e-12)
    lim = GOLD["coarse_mismatch_limit"]["mu_f"]
    for mu, below in ((lim - 0.005, True), (lim + 0.01, False)):
        p2 = oracle.Oracle(synth.make_dataset(small_config(mu_f=mu), signal=False)).plan()
        assert (p2.dlambda_f * p2.t_coh < 1.0) == below


@pytest.mark.parametrize("name", ["tiny", "band", "large"])
def test_plan_invariants(name):
    """eq. n-fft-final and the bin selection: N_FFT is a power of two >= N_FFT0 and < 2 N_FFT0,
    T_FFT >= T_coh, decimated bins are distinct, increasing, within one bin of the band edges."""
    cfg = synth.config(name)
    band = cfg["band"]
    nk = synth.samples_per_segment(band)
    dt = band["t_short"] / nk
    ds = Dataset(sky=synth.default_sky(), band=band, sites=[synth.SITES["H"], synth.SITES["L"]],
                 dt=dt, t0=0.0, n=nk * 4, n_k=nk, n_seg=4, f_het=band["f_min"] + band["f_band"] / 2,
                 x=np.zeros((2, nk * 4), np.complex64), valid=np.ones((2, nk * 4), np.uint8),
                 a=np.ones((2, 4)), b=np.ones((2, 4)), noise_var=np.ones((2, 4)),
                 templates=np.zeros((1, 3)))
    o = oracle.Oracle(ds)
    pl = o.plan()
    assert pl.n_k == nk and 1.0 / dt >= pl.df_load
    n0 = (pl.df_load / pl.dlambda_f) * math.ceil(pl.dlambda_f * pl.t_coh)
    assert pl.n_fft & (pl.n_fft - 1) == 0 and n0 <= pl.n_fft < 2 * n0
    assert pl.t_fft >= pl.t_coh
    kb = o.bins()
    assert np.all(np.diff(kb) >= 1)
    f = o.frequencies()
    assert f[0] >= band["f_min"] - 1e-9 and f[0] - band["f_min"] < 1.0 / pl.t_fft
    assert f[-1] <= band["f_min"] + band["f_band"] + 1.0 / pl.t_fft


@pytest.mark.parametrize("name", ["tiny", "band", "large"])
def test_plan_matches_hand_derived_values(name):
    """App. B eq. delta-f-load (with eqs. f-drift-eq, delta-f-obs) and Sec. III.B.2 eq.
    n-fft-final worked by hand (tests/golden/paper_values.json, derivation written out there):
    a dropped (1 + 4/(2D+1)) factor, 16/T_sft term or Doppler wing moves df_load, N_K, N_FFT or N_f."""
    g = GOLD["plan_derived"][name]
    cfg = synth.config(name)
    band = cfg["band"]
    nk = synth.samples_per_segment(band)
    dt = band["t_short"] / nk
    ds = Dataset(sky=synth.default_sky(), band=band, sites=[synth.SITES["H"], synth.SITES["L"]],
                 dt=dt, t0=0.0, n=nk * 4, n_k=nk, n_seg=4, f_het=band["f_min"] + band["f_band"] / 2,
                 x=np.zeros((2, nk * 4), np.complex64), valid=np.ones((2, nk * 4), np.uint8),
                 a=np.ones((2, 4)), b=np.ones((2, 4)), noise_var=np.ones((2, 4)),
                 templates=np.zeros((1, 3)))
    pl = oracle.Oracle(ds).plan()
    assert abs(pl.df_load - g["df_load"]) < 5e-5
    assert (pl.n_k, pl.n_fft, pl.n_f) == (g["n_k"], g["n_fft"], g["n_f"])


def test_pair_counts_and_asymptotic_total():
    """Sec. III.B.1: 2R+1 cross partners and R same-detector partners per interior K; the total
    approaches N_det^2 T_max T_obs / T_short^2 (Sec. III.B) for large R."""
    for R in (0, 1, 4):
        cfg = small_config(q=2, n_seg=40, max_lag=R)
        o = oracle.Oracle(synth.make_dataset(cfg, signal=False))
        M = 40
        cross = sum(min(M - 1, K + R) - max(0, K - R) + 1 for K in range(M))
        same = 2 * sum(min(M - 1, K + R) - K for K in range(M))
        assert o.pair_count() == cross + same
        interior_cross, interior_same = 2 * R + 1, R
        assert cross == M * interior_cross - R * (R + 1)
        assert same == 2 * (M * interior_same - R * (R + 1) // 2)
    cfg = small_config(q=2, n_seg=400, max_lag=20, pairs=3)
    o = oracle.Oracle(synth.make_dataset(cfg, signal=False))
    approx = 2 ** 2 * (20 * 120.0) * (400 * 120.0) / 120.0 ** 2
    assert abs(o.pair_count() / approx - 1.0) < 0.05


# --------------------------------------------------------------- time base

def test_inverse_time_map_round_trip_against_independent_forward_model():
    """t(tau) is the functional inverse of tau(t) (Sec. III.A.2); forward map from eqs.
    t-ssb-equation / tau-equation written independently in numpy (synth.forward_delay)."""
    cfg = synth.config("band")
    ds = synth.make_dataset(small_config(n_seg=4, t_short=600.0), signal=False)
    o = oracle.Oracle(ds)
    rng = np.random.default_rng(3)
    for det in range(2):
        for _ in range(6):
            tm = np.array([rng.uniform(1.0, 2.0), rng.uniform(0, 7e4), cfg["templates"]["period"][0]])
            r = int(rng.integers(0, ds.n_k * ds.n_seg))
            hi, lo = o.delay(det, tm, r)
            tau = ds.t0 + r * ds.dt
            t = tau + hi + lo
            off_np = synth.forward_delay(np.array([t]), ds.sites[det], ds.sky, *tm)[0]
            assert abs(t + off_np - tau) < 2e-9
            assert abs(o.forward_offset(det, tm, t)[0] + hi + lo) < 1e-12


def test_earth_orbit_amplitude_is_ecliptic_latitude():
    """Circular orbit of 1 AU: max over a year of r.n equals AU cos(beta), with the ecliptic
    latitude sin(beta) = sin(dec) cos(eps) - cos(dec) sin(eps) sin(ra)."""
    ds = synth.make_dataset(small_config(n_seg=2), signal=False, sky=dict(re_s=0.0))
    o = oracle.Oracle(ds)
    s = ds.sky
    t = np.linspace(0.0, s["year_s"], 20001)
    e = o.earth_delay(0, t)
    sb = math.sin(s["dec"]) * math.cos(s["obliquity"]) - math.cos(s["dec"]) * math.sin(s["obliquity"]) * math.sin(s["ra"])
    assert abs(e.max() - s["au_s"] * math.sqrt(1 - sb * sb)) < 1e-4
    assert abs(e.min() + s["au_s"] * math.sqrt(1 - sb * sb)) < 1e-4


def test_earth_rotation_closed_form():
    """Rotation only: r.n = R_E [cos(lat) cos(dec) cos(gmst + lon - ra) + sin(lat) sin(dec)]."""
    ds = synth.make_dataset(small_config(n_seg=2), signal=False, sky=dict(au_s=0.0))
    o = oracle.Oracle(ds)
    s, st = ds.sky, ds.sites[1]
    t = np.linspace(0, 2e5, 97)
    g = s["gmst0"] + 2 * math.pi * t / s["sidereal_day_s"] + st["lon"] - s["ra"]
    ref = s["re_s"] * (math.cos(st["lat"]) * math.cos(s["dec"]) * np.cos(g) + math.sin(st["lat"]) * math.sin(s["dec"]))
    assert np.abs(o.earth_delay(1, t) - ref).max() < 1e-15


def test_pure_binary_delay_fixed_point():
    """No Earth motion: t_SSB = t, so Delta = a_p sin(Omega (tau + Delta - T_asc)) (tau-equation)."""
    ds = synth.make_dataset(small_config(n_seg=4), signal=False, sky=NO_EARTH)
    o = oracle.Oracle(ds)
    tm = np.array([1.7, 1234.0, 68023.7])
    om = 2 * math.pi / tm[2]
    for r in (0, 57, 301):
        hi, lo = o.delay(0, tm, r)
        tau = ds.t0 + r * ds.dt
        d = 0.0
        for _ in range(60):
            d = tm[0] * math.sin(om * (tau + d - tm[1]))
        assert abs((hi + lo) - d) < 1e-14


# ----------------------------------------------------------- interpolation

def test_zero_delay_resampling_is_identity():
    """Sec. III.B.6: with zero Roemer delay no resampling is needed; on-grid sinc returns the sample."""
    ds = synth.make_dataset(small_config(n_seg=6, gap_fraction=0.0), sky=NO_EARTH)
    o = oracle.Oracle(ds)
    y, js, off, m = o.resample(0, np.array([0.0, 0.0, 68023.7]))
    nr = ds.n_seg * ds.n_k
    assert np.all(js == np.arange(nr)) and np.all(off == 0.0) and np.all(m == 1)
    assert np.abs(y - ds.x[0, :nr]).max() < 1e-15 * np.abs(ds.x[0]).max() + 1e-300


def _pole_dataset(delay_samples, D=8, window=0, n_seg=6, tone=None):
    """Detector at the pole, source at the pole, no orbit: constant Earth delay r.n = R_E."""
    cfg = small_config(n_seg=n_seg, dirichlet_D=D, window=window)
    ds = synth.make_dataset(cfg, signal=False)
    sky = dict(ds.sky, dec=math.pi / 2, au_s=0.0, re_s=delay_samples * ds.dt)
    ds.sky = sky
    ds.sites = [_pole_site(), _pole_site()]
    if tone is not None:
        j = np.arange(ds.n)
        ds.x = np.stack([np.exp(2j * np.pi * tone * j)] * 2).astype(np.complex64)
    return ds


def test_integer_delay_is_exact_shift():
    """An integer-sample delay makes every tap land on the grid: y_r = exp(2 pi i f_h Delta) x_{r-m}."""
    ds = _pole_dataset(3)
    o = oracle.Oracle(ds)
    y, js, off, m = o.resample(0, np.array([0.0, 0.0, 68023.7]))
    nr = ds.n_seg * ds.n_k
    r = np.arange(nr)
    assert np.all(js == r - 3) and np.all(np.abs(off) < 1e-12)
    assert np.all(m[:3] == 0) and np.all(m[3:] == 1)
    delta = -3 * ds.dt
    ref = np.exp(2j * np.pi * ds.f_het * delta) * ds.x[0, :nr - 3].astype(np.complex128)
    assert np.abs(y[3:] - ref).max() < 1e-12


@pytest.mark.parametrize("window", [0, 1])
def test_sinc_interpolation_converges_with_D(window):
    """Sec. III.A.1: the windowed Shannon formula converges as D grows, for band-limited input."""
    errs = []
    for D in (4, 8, 16, 32):
        ds = _pole_dataset(2.37, D=D, window=window, n_seg=10, tone=0.19)
        o = oracle.Oracle(ds)
        y, js, off, m = o.resample(0, np.array([0.0, 0.0, 68023.7]))
        delta = -2.37 * ds.dt
        r = np.arange(len(y))
        exact = np.exp(2j * np.pi * 0.19 * (r + delta / ds.dt)) * np.exp(2j * np.pi * ds.f_het * delta)
        sel = slice(200, len(y) - 200)
        errs.append(np.abs(y[sel] - exact[sel]).max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    # D = 8 budget at this offset (0.37 samples) and tone (0.19 cycles/sample), as measured:
    # 4.29e-3 (window indexed by tap) and 2.45e-3 (window at the offset).  Two-sided, so that a
    # Hann window (5.6e-3 / 1.9e-4) or a Hamming indexed over 2D + 1 (2.2e-2) fails.
    lo, hi = (3.9e-3, 4.7e-3) if window == 0 else (2.2e-3, 2.7e-3)
    assert lo < errs[1] < hi, errs[1]


@pytest.mark.parametrize("window", [0, 1])
def test_tap_weights_are_hamming_times_sinc(window):
    """Sec. III.A.1 (eq. shannon-interp-formula, Hamming window of length 2D + 1): the resampled
    impulse response is w sinc(d) tap by tap, checked against numpy's Hamming window and sinc.
    Window 0 is indexed by tap n, w_n = np.hamming(2D + 1)[n + D]; window 1 is evaluated at the
    continuous offset d = delta_c - n, w(d) = 0.54 + 0.46 cos(pi d / (D + 1)), which at the
    half-integer offsets used here is np.hamming(4D + 5)[2d + 2D + 2]."""
    D = 8
    delay = 2.37 if window == 0 else 2.5
    ds = _pole_dataset(delay, D=D, window=window, n_seg=6)
    j0 = ds.n // 2
    ds.x = np.zeros_like(ds.x)
    ds.x[:, j0] = 1.0
    o = oracle.Oracle(ds)
    y, js, off, m = o.resample(0, np.array([0.0, 0.0, 68023.7]))
    phase = np.exp(2j * np.pi * ds.f_het * (-ds.sky["re_s"]))
    hit = np.nonzero(np.abs(js - j0) <= D)[0]
    assert len(hit) == 2 * D + 1
    for r in hit:
        n = j0 - js[r]
        d = off[r] - n
        if window == 0:
            w = np.hamming(2 * D + 1)[n + D]
        else:
            assert abs(abs(off[r]) - 0.5) < 1e-9
            w = np.hamming(4 * D + 5)[int(round(2 * d)) + 2 * D + 2]
        assert abs(y[r] / phase - w * np.sinc(d)) < 1e-9, (r, n, d)


# ------------------------------------------------------------- DFT, phases

def _tone_dataset(kappa_bins, n_seg=5, sigma=1.3, t_short=120.0):
    cfg = small_config(n_seg=n_seg, t_short=t_short, sigma=[sigma, sigma])
    ds = synth.make_dataset(cfg, signal=False, sky=NO_EARTH)
    pl = oracle.Oracle(ds).plan()
    kb = oracle.Oracle(ds).bins()
    i0 = len(kb) // 3
    j = np.arange(ds.n)
    ds.x = np.stack([np.exp(2j * np.pi * (kb[i0] + kappa_bins) * j / pl.n_fft)] * 2).astype(np.complex128).astype(np.complex64)
    return ds, pl, i0, kb


@pytest.mark.parametrize("kappa", [0.0, 0.25, -0.4, 0.5])
def test_segment_dft_is_geometric_series(kappa):
    """Zero-padded DFT of a tone at bin offset kappa (Sec. III.B.5): per segment
    sum_s exp(2 pi i kappa (r_B + s)/N_FFT) = exp(2 pi i kappa r_B/N) e^{i pi kappa (N_K-1)/N} sin(pi kappa N_K/N)/sin(pi kappa/N)."""
    ds, pl, i0, kb = _tone_dataset(kappa)
    o = oracle.Oracle(ds)
    F = o.spectra(np.array([0.0, 0.0, 68023.7]), bins=[i0])
    N, nk = pl.n_fft, pl.n_k
    for K in range(ds.n_seg):
        rb = K * nk
        if kappa == 0.0:
            geo = nk
        else:
            geo = np.exp(1j * np.pi * kappa * (nk - 1) / N) * math.sin(math.pi * kappa * nk / N) / math.sin(math.pi * kappa / N)
        # input tone phase kappa r_B/N (the kbar part cancels exactly against Phi_in)
        ref = np.exp(2j * np.pi * kappa * rb / N) * geo / (1.3 * math.sqrt(nk))
        assert abs(F[0, K, 0] - ref) < 1e-6 * abs(nk / (1.3 * math.sqrt(nk)))


def test_span_dft_equals_sum_of_phased_segments():
    """Sec. III.B.4-5: one DFT over an L-span equals the sum of per-segment DFTs once Phi_in is
    applied (linearity); reference DFT computed by numpy from the resampled series."""
    ds = synth.make_dataset(small_config(n_seg=8, sigma=[1.0, 1.0]))
    o = oracle.Oracle(ds)
    tm = ds.templates[1]
    pl = o.plan()
    y, _, _, _ = o.resample(1, tm)
    bins = np.array([3, 17, 40])
    F = o.spectra(tm, bins=bins)
    kb = o.bins()[bins] % pl.n_fft
    L0 = 2
    lo, hi = L0 * pl.n_k, (L0 + 3) * pl.n_k
    r = np.arange(lo, hi)
    for ii, k in enumerate(kb):
        span = np.sum(y[lo:hi] * np.exp(-2j * np.pi * ((k * r) % pl.n_fft) / pl.n_fft))
        segs = F[1, L0:L0 + 3, ii].sum() * math.sqrt(pl.n_k)
        assert abs(span - segs) < 1e-11 * max(1.0, abs(span))


def test_zero_delay_tiers_agree():
    """Sec. III.B.6: with zero Roemer delay the resampled rho exactly equals the detector-frame rho."""
    ds = synth.make_dataset(small_config(n_seg=10, gap_fraction=0.2, max_lag=2), sky=NO_EARTH)
    o = oracle.Oracle(ds)
    tm = np.array([[0.0, 0.0, 68023.7]])
    assert np.abs(o.spectra(tm[0], 0) - o.spectra(tm[0], 1)).max() < 1e-12
    assert np.abs(o.rho(tm, 0) - o.rho(tm, 1)).max() < 1e-12


# --------------------------------------------------------- normalisation

def test_unit_variance_in_noise_zero_delay():
    """Normalisation N (eq. norm-cc; App. A) gives E rho = 0, Var rho = 1 in Gaussian noise:
    zero delay, gaps, uneven noise, R = 2, same- and cross-detector pairs.  Bins 5 apart and
    independent seeds; 5-sigma bounds."""
    vals = []
    for seed in range(300):
        cfg = small_config(n_seg=12, max_lag=2, gap_fraction=0.15, seed=100 + seed, sigma=[1.0, 1.7])
        ds = synth.make_dataset(cfg, signal=False, sky=NO_EARTH, sigma_wander=0.3)
        o = oracle.Oracle(ds)
        r = o.rho(np.array([[0.0, 0.0, 68023.7]]), bins=np.arange(2, o.plan().n_f, 9))
        vals.append(r[0])
    v = np.concatenate(vals)
    n = len(v)
    assert abs(v.mean()) < 5.0 / math.sqrt(n)
    assert abs(v.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)


# ------------------------------------------------------ signal amplitude

def _w2(ds, R, pairs=3, phi=None):
    Q, M = ds.a.shape
    s = 0.0
    for X in range(Q):
        for K in range(M):
            for Y in range(Q):
                for L in range(max(0, K - R), min(M, K + R + 1)):
                    if not (((pairs & 1) and X < Y) or ((pairs & 2) and X == Y and L > K)):
                        continue
                    sK, sL = math.sqrt(ds.noise_var[X, K]), math.sqrt(ds.noise_var[Y, L])
                    W = ds.a[X, K] / sK * ds.a[Y, L] / sL + ds.b[X, K] / sK * ds.b[Y, L] / sL
                    f = 1.0 if phi is None else phi[X, K] * phi[Y, L]
                    s += W * W * f
    return s


def test_matched_signal_closed_form_amplitude():
    """Noiseless, circularly polarised (cos iota = 1), on-bin, antennas constant per segment,
    zero delay: E rho = (sqrt 2 / 4) N_K h0^2 sqrt(sum_P W^2 phi phi) (signal model of
    Sec. II.A.1 through eq. final-formatted-rho)."""
    cfg = small_config(n_seg=20, max_lag=2, pairs=3, sigma=[1.0, 1.4])
    ds0 = synth.make_dataset(cfg, signal=False, sky=NO_EARTH)
    o0 = oracle.Oracle(ds0)
    pl = o0.plan()
    i0 = 31
    f0 = ds0.f_het + o0.bins()[i0] / pl.t_fft
    cfg["injections"] = [dict(f0=f0, a_p=0.0, t_asc_off=0.0, period=68023.7, h0=0.3, cosi=1.0, psi=0.7, phi0=1.1)]
    ds = synth.make_dataset(cfg, noise=False, sky=NO_EARTH, antenna_piecewise=True, sigma_wander=0.2)
    o = oracle.Oracle(ds)
    r = o.rho(np.array([[0.0, 0.0, 68023.7]]))[0]
    pred = math.sqrt(2) / 4 * pl.n_k * 0.3 ** 2 * math.sqrt(_w2(ds, 2))
    assert abs(r[i0] / pred - 1.0) < 1e-6
    assert r.argmax() == i0


def _edge_phi(ds):
    """Valid fraction per segment: source samples whose Earth-only arrival lies outside the data
    carry no weight; the Earth-only inverse t + r.n = tau is solved here by fixed point."""
    nr = ds.n_seg * ds.n_k
    tau = ds.t0 + np.arange(nr) * ds.dt
    phi = np.zeros((ds.n_det, ds.n_seg))
    for X in range(ds.n_det):
        t = tau.copy()
        for _ in range(8):
            t = tau - synth.earth_roemer(t, ds.sites[X], ds.sky)
        j = np.arange(nr) + np.floor((t - tau) / ds.dt + 0.5).astype(np.int64)
        inside = ((j >= 0) & (j < ds.n)).astype(float)
        phi[X] = inside.reshape(ds.n_seg, ds.n_k).mean(axis=1)
    return phi


def test_matched_signal_with_delays_and_peak_location():
    """With Earth and binary Roemer delays the matched template still recovers the closed-form
    amplitude within the interpolation budget (Sec. III.A.1) and peaks at the injected bin and
    orbit (Sec. III.A.2: the signal is concentrated at a single frequency after resampling)."""
    cfg = small_config(n_seg=90, t_short=240.0, max_lag=1, pairs=1, sigma=[1.0, 1.0],
                       f_min=100.0, f_band=0.3, a_p_max=2.0)
    ds0 = synth.make_dataset(cfg, signal=False)
    o0 = oracle.Oracle(ds0)
    pl = o0.plan()
    i0 = 40
    f0 = ds0.f_het + o0.bins()[i0] / pl.t_fft
    inj = dict(f0=f0, a_p=1.6, t_asc_off=0.0, period=68023.7, h0=0.3, cosi=1.0, psi=0.2, phi0=0.3)
    cfg["injections"] = [inj]
    ds = synth.make_dataset(cfg, noise=False, antenna_piecewise=True)
    o = oracle.Oracle(ds)
    t_asc = cfg["t_asc0"]
    good = np.array([[1.6, t_asc, 68023.7]])
    off = np.array([[1.6, t_asc + 900.0, 68023.7], [1.1, t_asc, 68023.7]])
    r = o.rho(np.vstack([good, off]))
    phi = _edge_phi(ds)
    assert phi.min() < 1.0          # the data edges do cut the first or last segments
    pred = math.sqrt(2) / 4 * pl.n_k * 0.3 ** 2 * math.sqrt(_w2(ds, 1, pairs=1, phi=phi))
    assert r[0].argmax() == i0
    assert abs(r[0, i0] / pred - 1.0) < 0.03
    assert r[0, i0] > 1.5 * r[1, i0] and r[0, i0] > 1.5 * r[2, i0]
    assert r[0, i0] > r[1].max() and r[0, i0] > r[2].max()
    # Tier D (no interpolation) sees the same peak; the gap between tiers is the method error.
    rd = o.rho(good, tier=1)[0]
    assert rd.argmax() == i0 and abs(rd[i0] / pred - 1.0) < 0.03


# ----------------------------------------------------- zero-padding power

def test_recovered_power_printed_values():
    """Sec. III.B.2: averaging rho over a uniform sub-bin offset with R = 1 (T_coh = 3 T_short)
    recovers 0.861 / 0.963 / 0.983 of the on-bin power at T_FFT = 1 / 2 / 3 T_coh."""
    g = GOLD["xi2_resampled"]
    nodes, weights = np.polynomial.legendre.leggauss(16)
    kap = 0.25 * (nodes + 1.0)      # [0, 1/2]
    wts = 0.25 * weights
    for c, printed in zip(g["t_fft_over_t_coh"], g["value"]):
        nk, M = 64, 96
        cfg = small_config(n_seg=M, t_short=100.0, f_band=0.2, max_lag=1, pairs=1, sigma=[1.0, 1.0],
                           n_fft_override=3 * c * nk)
        cfg["n_k"] = nk
        base = synth.make_dataset(cfg, signal=False, noise=False, sky=dict(au_s=0.0, re_s=0.0, sidereal_day_s=1e18))
        ob = oracle.Oracle(base)
        pl = ob.plan()
        assert pl.n_fft == 3 * c * nk
        i0 = pl.n_f // 2
        kb = ob.bins()[i0]
        vals = []
        for k in np.concatenate([[0.0], kap]):
            f0 = base.f_het + (kb + k) / pl.t_fft
            cfg["injections"] = [dict(f0=f0, a_p=0.0, t_asc_off=0.0, period=68023.7, h0=1.0, cosi=1.0, psi=0.0, phi0=0.0)]
            ds = synth.make_dataset(cfg, noise=False, sky=dict(au_s=0.0, re_s=0.0, sidereal_day_s=1e18))
            vals.append(oracle.Oracle(ds).rho(np.array([[0.0, 0.0, 68023.7]]), bins=[i0])[0, 0])
        ratio = np.array(vals[1:]) / vals[0]
        avg = 2.0 * np.sum(wts * ratio)
        assert abs(avg - printed) < 1.5e-3, (c, avg, printed)


def test_demod_two_bin_value_quadrature():
    """Sec. III.B.2: 2 int_0^1 sinc^2 = 0.903 (m = 2 Dirichlet bins) -- checks the printed
    quadrature convention used for the resampled values."""
    from scipy.integrate import quad
    v = 2 * quad(lambda k: np.sinc(k) ** 2, 0, GOLD["xi2_demod_m2"]["m"] / 2)[0]
    assert round(v, 3) == GOLD["xi2_demod_m2"]["value"]


# --------------------------------------------- all pairs (the F-statistic limit)

def _circ_weights(ds, M):
    """a_K = cos(theta_K), b_K = sin(theta_K), theta_K = 2 pi K / M (M a multiple of 4): the sums
    of a^2 and b^2 over segments are equal and the sum of a b vanishes (A = B, C = 0)."""
    th = 2.0 * math.pi * np.arange(M) / M
    for X in range(ds.n_det):
        ds.a[X] = np.cos(th + 0.3 * X)
        ds.b[X] = np.sin(th + 0.3 * X)


def test_all_pairs_noise_is_chi2_4():
    """App. A.2: with every pair, auto-correlations included, rho = sqrt2 (|F_a|^2 + |F_b|^2) /
    sqrt(A^2 + 2 C^2 + B^2); in Gaussian noise with A = B and C = 0, 2 rho is the F-statistic's
    chi-squared variable with 4 degrees of freedom (mean 4, variance 8), checked over 300 seeds
    with a Kolmogorov-Smirnov test against scipy's distribution."""
    from scipy import stats
    vals = []
    for seed in range(300):
        cfg = small_config(n_seg=12, max_lag=1, pairs=4, seed=500 + seed, sigma=[1.0, 1.0])
        ds = synth.make_dataset(cfg, signal=False, sky=NO_EARTH)
        _circ_weights(ds, 12)
        o = oracle.Oracle(ds)
        r = o.rho(np.array([[0.0, 0.0, 68023.7]]), bins=np.arange(2, o.plan().n_f, 11))
        vals.append(2.0 * r[0])
    v = np.concatenate(vals)
    n = len(v)
    assert abs(v.mean() - 4.0) < 5.0 * math.sqrt(8.0 / n)
    assert abs(v.var() - 8.0) < 5.0 * math.sqrt(np.var((v - 4.0) ** 2) / n)
    assert stats.kstest(v, stats.chi2(4).cdf).pvalue > 1e-3


def _matched_zero_delay(cfg, cosi, psi=0.7, per_sample=False, piecewise=True, i0=31):
    ds0 = synth.make_dataset(cfg, signal=False, sky=NO_EARTH)
    o0 = oracle.Oracle(ds0)
    pl = o0.plan()
    f0 = ds0.f_het + o0.bins()[i0] / pl.t_fft
    cfg = dict(cfg, injections=[dict(f0=f0, a_p=0.0, t_asc_off=0.0, period=68023.7, h0=0.3, cosi=cosi, psi=psi,
                                     phi0=1.1)])
    ds = synth.make_dataset(cfg, noise=False, sky=NO_EARTH, antenna_piecewise=piecewise, sigma_wander=0.2,
                            per_sample_antenna=per_sample)
    return ds, pl, i0


def test_all_pairs_matched_signal_closed_form():
    """All pairs, noiseless circularly polarised matched signal, zero delay, antennas constant
    per segment: F_K = sqrt(N_K) h0 (a_K - i b_K) e^{i theta} / (2 sigma_K), so |F_a|^2 + |F_b|^2 =
    N_K h0^2 [(sum A)^2 + 2 (sum C)^2 + (sum B)^2] / 4 and rho = (sqrt2/4) N_K h0^2
    sqrt((sum A)^2 + 2 (sum C)^2 + (sum B)^2) with A = hat a^2, B = hat b^2, C = hat a hat b."""
    cfg = small_config(n_seg=16, max_lag=1, pairs=4, sigma=[1.0, 1.4])
    ds, pl, i0 = _matched_zero_delay(cfg, cosi=1.0)
    r = oracle.Oracle(ds).rho(np.array([[0.0, 0.0, 68023.7]]))[0]
    sig = np.sqrt(ds.noise_var)
    A = np.sum((ds.a / sig) ** 2)
    B = np.sum((ds.b / sig) ** 2)
    C = np.sum(ds.a * ds.b / sig ** 2)
    pred = math.sqrt(2) / 4 * pl.n_k * 0.3 ** 2 * math.sqrt(A * A + 2 * C * C + B * B)
    assert abs(r[i0] / pred - 1.0) < 1e-6
    assert r.argmax() == i0


# ------------------------------------------------------------ Gamma^circ

def _circ_w2(ds, R, pairs=3):
    Q, M = ds.a.shape
    s = 0.0
    for X in range(Q):
        for K in range(M):
            for Y in range(Q):
                for L in range(max(0, K - R), min(M, K + R + 1)):
                    if not (((pairs & 1) and X < Y) or ((pairs & 2) and X == Y and L > K)):
                        continue
                    sK, sL = math.sqrt(ds.noise_var[X, K]), math.sqrt(ds.noise_var[Y, L])
                    G = ds.a[X, K] / sK * ds.b[Y, L] / sL - ds.b[X, K] / sK * ds.a[Y, L] / sL
                    s += G * G
    return s


@pytest.mark.parametrize("cosi", [1.0, -1.0, 0.0])
def test_circ_weight_matched_signal_closed_form(cosi):
    """Sec. II.B Gamma^circ = hat a_K hat b_L - hat b_K hat a_L: for a matched circularly polarised
    signal (zero delay, antennas constant per segment) conj(F_K) F_L = N_K h0^2 [(hat a_K hat a_L +
    hat b_K hat b_L) + i (hat b_K hat a_L - hat a_K hat b_L)] / 4, so rho_circ = +-(sqrt2/4) N_K h0^2
    sqrt(sum_P Gamma^circ^2) for cos iota = +-1, and 0 for a linearly polarised one."""
    cfg = small_config(n_seg=16, max_lag=2, pairs=3, sigma=[1.0, 1.4])
    cfg["band"]["weight"] = 1
    ds, pl, i0 = _matched_zero_delay(cfg, cosi=cosi)
    ds.band = dict(ds.band, weight=1)
    r = oracle.Oracle(ds).rho(np.array([[0.0, 0.0, 68023.7]]))[0]
    pred = math.sqrt(2) / 4 * pl.n_k * 0.3 ** 2 * math.sqrt(_circ_w2(ds, 2))
    if cosi == 0.0:
        assert abs(r[i0]) < 1e-9 * pred
    else:
        assert abs(r[i0] / (cosi * pred) - 1.0) < 1e-6


@pytest.mark.parametrize("mode", ["circ", "per_sample"])
def test_weighted_streams_unit_variance_in_noise(mode):
    """Normalisation of the weighted streams (Gamma^circ: N^2 = sum_P A_K B_L + B_K A_L - 2 C_K C_L;
    per-sample antenna functions: A_K the segment mean of m_r hat a_r^2, ...): E rho = 0 and
    Var rho = 1 in Gaussian noise with gaps, uneven noise, R = 2, both pair kinds."""
    vals = []
    for seed in range(200):
        cfg = small_config(n_seg=12, max_lag=2, gap_fraction=0.15, seed=900 + seed, sigma=[1.0, 1.7])
        if mode == "circ":
            cfg["band"]["weight"] = 1
        ds = synth.make_dataset(cfg, signal=False, sky=NO_EARTH, sigma_wander=0.3,
                                per_sample_antenna=(mode == "per_sample"))
        if mode == "per_sample":  # a fast-varying weighting, so that per-sample weights matter
            r_idx = np.arange(ds.ar.shape[1])
            ds.ar = ds.ar * (1.0 + 0.5 * np.cos(2 * np.pi * r_idx / 97.0))
            ds.br = ds.br * (1.0 + 0.5 * np.sin(2 * np.pi * r_idx / 61.0))
        o = oracle.Oracle(ds)
        r = o.rho(np.array([[0.0, 0.0, 68023.7]]), bins=np.arange(2, o.plan().n_f, 9))
        vals.append(r[0])
    v = np.concatenate(vals)
    n = len(v)
    assert abs(v.mean()) < 5.0 / math.sqrt(n)
    assert abs(v.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)


# ---------------------------------------------- per-sample antenna weighting

def test_per_sample_antenna_constant_per_segment_reduces():
    """Sec. III.B.3: per-sample a_r, b_r that are constant over each segment give the per-segment
    statistic (F^a = hat a_K F, F^b = hat b_K F) to rounding."""
    cfg = small_config(n_seg=10, max_lag=2, gap_fraction=0.2,
                       injections=[dict(f0=50.21, a_p=1.25, t_asc_off=0.0, period=68023.7, h0=0.35, cosi=0.5,
                                        psi=0.3, phi0=1.0)])
    ds = synth.make_dataset(cfg, sigma_wander=0.2)
    ref = oracle.Oracle(ds).rho(ds.templates[:3])
    ds.ar = np.repeat(ds.a, ds.n_k, axis=1)
    ds.br = np.repeat(ds.b, ds.n_k, axis=1)
    got = oracle.Oracle(ds).rho(ds.templates[:3])
    assert np.max(np.abs(got - ref)) < 1e-11 * max(1.0, np.abs(ref).max())


def test_per_sample_antenna_matched_signal_closed_form():
    """Per-sample weighting with the true a(t), b(t) (eq. norm-a-eq) for a matched circularly
    polarised signal with continuously varying antenna response, zero delay:
    F^a_K = sqrt(N_K) h0 (A_K - i C_K) e^{i theta} / 2, F^b_K = sqrt(N_K) h0 (C_K - i B_K) e^{i theta} / 2
    with segment means A_K = <hat a^2>, B_K = <hat b^2>, C_K = <hat a hat b> (computed here from the
    antenna model), so rho = (sqrt2/4) N_K h0^2 sqrt(sum_P A_K A_L + 2 C_K C_L + B_K B_L)."""
    cfg = small_config(n_seg=16, max_lag=2, pairs=3, sigma=[1.0, 1.4], t_short=2400.0)
    ds, pl, i0 = _matched_zero_delay(cfg, cosi=1.0, per_sample=True, piecewise=False, i0=20)
    r = oracle.Oracle(ds).rho(np.array([[0.0, 0.0, 68023.7]]))[0]
    Q, M, nk = ds.n_det, ds.n_seg, ds.n_k
    sig = np.sqrt(ds.noise_var)[:, :, None]
    ar = ds.ar.reshape(Q, M, nk) / sig
    br = ds.br.reshape(Q, M, nk) / sig
    A, B, C = (ar * ar).mean(axis=2), (br * br).mean(axis=2), (ar * br).mean(axis=2)
    s = 0.0
    for X in range(Q):
        for K in range(M):
            for Y in range(Q):
                for L in range(max(0, K - 2), min(M, K + 3)):
                    if (X < Y) or (X == Y and L > K):
                        s += A[X, K] * A[Y, L] + 2 * C[X, K] * C[Y, L] + B[X, K] * B[Y, L]
    pred = math.sqrt(2) / 4 * pl.n_k * 0.3 ** 2 * math.sqrt(s)
    assert abs(r[i0] / pred - 1.0) < 1e-6
    # per-segment weights (antenna at the mid-time) recover less of this signal
    ds_seg = synth.make_dataset(cfg, noise=False, sky=NO_EARTH, sigma_wander=0.2)
    ds_seg.x = ds.x
    r_seg = oracle.Oracle(ds_seg).rho(np.array([[0.0, 0.0, 68023.7]]))[0]
    assert r_seg[i0] < r[i0]


# ------------------------------------------------------- eccentric orbits

def test_kepler_against_bracketing_root_finder():
    """eq. solve-for-E: the oracle's E solves E - e sin E = M, compared with scipy's brentq on a
    grid of mean anomalies and eccentricities."""
    from scipy.optimize import brentq
    for e in (0.0, 0.05, 0.3, 0.7, 0.95):
        for M in np.linspace(0.0, 2 * math.pi, 37):
            ref = brentq(lambda E: E - e * math.sin(E) - M, M - 1.0 - e, M + 1.0 + e, xtol=1e-15, rtol=1e-15)
            assert abs(oracle.kepler(M, e) - ref) < 1e-13


def _ecc_dataset(**kw):
    ds = synth.make_dataset(small_config(n_seg=6, t_short=600.0, **kw), signal=False)
    ds.ecc = True
    return ds


def test_eccentric_zero_e_is_circular():
    """eq. Kepler-equation with e = 0: R/c = a_p sin(Omega (t - T_p) + omega), the circular orbit
    with T_asc = T_p - omega / Omega; delays of both template forms agree."""
    ds = _ecc_dataset()
    oe = oracle.Oracle(ds)
    ds.ecc = False
    oc = oracle.Oracle(ds)
    P, w, tp = 68023.7, 1.1, 7000.0
    for r in (0, 517, 2 * ds.n_k + 3, ds.n_seg * ds.n_k - 1):
        for X in range(2):
            he, le = oe.delay(X, np.array([1.4, tp, w, 0.0, P]), r)
            hc, lc = oc.delay(X, np.array([1.4, tp - w * P / (2 * math.pi), P]), r)
            assert abs((he - hc) + (le - lc)) < 1e-12


def test_eccentric_inverse_map_round_trip_against_independent_forward_model():
    """The inverse map t(tau) with an eccentric binary (e = 0.3 and 0.6) against an independent
    numpy forward model (synth.forward_delay_ecc, its own vectorised Kepler solve)."""
    ds = _ecc_dataset()
    o = oracle.Oracle(ds)
    rng = np.random.default_rng(8)
    for e in (0.3, 0.6):
        for det in range(2):
            for _ in range(5):
                tm = np.array([rng.uniform(1.0, 2.0), rng.uniform(0, 7e4), rng.uniform(0, 2 * math.pi), e, 68023.7])
                r = int(rng.integers(0, ds.n_k * ds.n_seg))
                hi, lo = o.delay(det, tm, r)
                tau = ds.t0 + r * ds.dt
                t = tau + hi + lo
                off = synth.forward_delay_ecc(np.array([t]), ds.sites[det], ds.sky, tm[0], tm[1], tm[2], tm[3],
                                              tm[4])[0]
                assert abs(t + off - tau) < 2e-9
                assert abs(o.forward_offset(det, tm, t)[0] + hi + lo) < 1e-12


def test_eccentric_matched_template_recovers_injection():
    """An eccentric (e = 0.4) injection is recovered by its own eccentric template at the injected
    bin within the interpolation budget of the closed-form amplitude, while the circular template
    with the same a_p and ascending node loses most of it (Sec. II.A.2: resampling handles
    elliptical orbits)."""
    cfg = small_config(n_seg=60, t_short=240.0, max_lag=1, pairs=1, sigma=[1.0, 1.0], f_min=100.0, f_band=0.3,
                       a_p_max=2.0)
    ds0 = synth.make_dataset(cfg, signal=False)
    o0 = oracle.Oracle(ds0)
    pl = o0.plan()
    i0 = 40
    f0 = ds0.f_het + o0.bins()[i0] / pl.t_fft
    w, e, tpo, ap = 0.8, 0.4, 300.0, 1.6
    cfg["injections"] = [dict(f0=f0, a_p=ap, t_asc_off=0.0, period=68023.7, h0=0.3, cosi=1.0, psi=0.2, phi0=0.3,
                              ecc=e, w=w, t_p_off=tpo)]
    ds = synth.make_dataset(cfg, noise=False, antenna_piecewise=True)
    ds.ecc = True
    tp = cfg["t_asc0"] + tpo
    r = oracle.Oracle(ds).rho(np.array([[ap, tp, w, e, 68023.7], [ap, tp - w * 68023.7 / (2 * math.pi), 0.0, 0.0,
                                                                    68023.7]]))
    pred = math.sqrt(2) / 4 * pl.n_k * 0.3 ** 2 * math.sqrt(_w2(ds, 1, pairs=1, phi=_edge_phi(ds)))
    assert r[0].argmax() == i0
    assert abs(r[0, i0] / pred - 1.0) < 0.03
    assert r[1].max() < 0.5 * r[0, i0]


# ------------------------------------------------------- SFT front end (App. B)

def _tone_series(f0, amp, ph, f_het, t):
    return 0.5 * amp * np.exp(1j * (2 * np.pi * np.mod((f0 - f_het) * t, 1.0) + ph))


@pytest.mark.parametrize("n_out,f_het", [(64, 200.0), (63, 200.013), (153, 199.9871), (179, 200.0049)])
def test_sft_front_end_bin_centred_tone(n_out, f_het):
    """App. B: a real sinusoid on a bin centre inside the band becomes exactly the heterodyned
    complex tone (A/2) exp(i (2 pi (f0 - f_h) t + phi)) at every downsampled sample of every SFT.
    This fixes the inverse transform and its index shift (even and odd N'), the stitching phase
    exp(-2 pi i f_h (t_K - T_sft/2)) across SFTs and the remainder f_r = f_h - k_h / T_sft (f_h off
    the bin grid)."""
    t_sft, dt, t0 = 240.0, 1.0 / 1024.0, 7200.0
    k0 = int(round(200.0 * t_sft)) + 5
    f0 = k0 / t_sft
    kh = int(round(f_het * t_sft))
    k_first = kh - n_out // 2 - 7
    z, valid = synth.make_sfts(9, t_sft, dt, k_first, n_out + 14, t0=t0, lines=[(f0, 1.3, 0.4)])
    x = oracle.sft_series(z, t_sft, t0, k_first, f_het, n_out)
    t = t0 + np.arange(9 * n_out) * (t_sft / n_out)
    ref = _tone_series(f0, 1.3, 0.4, f_het, t)
    assert np.abs(x - ref).max() < 1e-11


def test_sft_front_end_off_bin_tone_and_gaps():
    """An off-bin tone (frequency between bins, mid-band) is reproduced to the band's truncation
    of its Dirichlet leakage, which shrinks as the band widens; a missing SFT gives zeros there
    and leaves its neighbours unchanged; bins not held give ERANGE."""
    t_sft, dt, t0, f_het = 240.0, 1.0 / 1024.0, 0.0, 100.0
    f0 = 100.0 + 0.37 / t_sft
    errs = []
    for n_out in (64, 256, 1024):
        kh = int(round(f_het * t_sft))
        k_first = kh - n_out // 2
        z, _ = synth.make_sfts(3, t_sft, dt, k_first, n_out, t0=t0, lines=[(f0, 1.0, 0.0)])
        x = oracle.sft_series(z, t_sft, t0, k_first, f_het, n_out)
        t = t0 + np.arange(3 * n_out) * (t_sft / n_out)
        # away from the SFT edges (the truncated leakage is largest at the edges)
        inner = np.concatenate([np.arange(K * n_out + n_out // 4, K * n_out + 3 * n_out // 4) for K in range(3)])
        errs.append(np.abs(x - _tone_series(f0, 1.0, 0.0, f_het, t))[inner].max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.02
    z, valid = synth.make_sfts(5, t_sft, dt, 24000 - 40, 80, lines=[(100.1, 1.0, 0.0)], sigma=0.5, seed=3)
    v = np.array([1, 1, 0, 1, 1], dtype=np.uint8)
    x_all = oracle.sft_series(z, t_sft, 0.0, 24000 - 40, f_het, 64)
    x_gap = oracle.sft_series(z, t_sft, 0.0, 24000 - 40, f_het, 64, sft_valid=v)
    assert np.all(x_gap[128:192] == 0)
    assert np.array_equal(x_gap[:128], x_all[:128]) and np.array_equal(x_gap[192:], x_all[192:])
    with pytest.raises(RuntimeError):
        oracle.sft_series(z, t_sft, 0.0, 24000 - 40, f_het, 96)

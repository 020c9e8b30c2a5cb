"""Seeded synthetic datasets: heterodyned complex series, gaps, weights, templates."""

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from .model import (SITES, antenna_ab, default_sky, earth_roemer, forward_delay, forward_delay_ecc,
                    samples_per_segment)


@dataclass
class Dataset:
    sky: dict
    band: dict
    sites: list
    dt: float
    t0: float
    n: int
    n_k: int
    n_seg: int
    f_het: float
    x: np.ndarray          # (Q, n) complex64, zero where invalid
    valid: np.ndarray      # (Q, n) uint8
    a: np.ndarray          # (Q, M) float64, a(t) at segment mid-times
    b: np.ndarray          # (Q, M)
    noise_var: np.ndarray  # (Q, M) noise variance E|x'|^2 per sample
    templates: np.ndarray  # (T, 3) columns a_p, T_asc, P; eccentric: (T, 5) a_p, T_p, omega, e, P
    injections: list = field(default_factory=list)
    name: str = ""
    ar: np.ndarray = None  # (Q, M N_K) a(tau_r) on the source lattice (per-sample weighting), or None
    br: np.ndarray = None
    ecc: bool = False      # templates are eccentric orbits

    @property
    def n_det(self):
        return self.x.shape[0]


def template_grid(spec, t_asc0):
    """Cartesian grid a_p x T_asc x P (a_p fastest), T_asc offsets relative to t_asc0."""
    ap = np.linspace(*spec["a_p"]) if isinstance(spec["a_p"], tuple) else np.asarray(spec["a_p"], float)
    ta = t_asc0 + (np.linspace(*spec["t_asc"]) if isinstance(spec["t_asc"], tuple)
                   else np.asarray(spec["t_asc"], float))
    per = np.asarray(spec["period"], dtype=np.float64)
    P, T, A = np.meshgrid(per, ta, ap, indexing="ij")
    return np.stack([A.ravel(), T.ravel(), P.ravel()], axis=1).astype(np.float64)


def _gap_mask(rng, n, dt, fraction, mean_len_s=6 * 3600.0):
    """Mask of valid samples: exponential-length gaps at uniform random starts
    until the requested fraction of the span is masked."""
    valid = np.ones(n, dtype=np.uint8)
    if fraction <= 0.0:
        return valid
    target = int(fraction * n)
    masked = 0
    while masked < target:
        start = int(rng.integers(0, n))
        length = max(1, int(rng.exponential(mean_len_s) / dt))
        seg = valid[start:start + length]
        masked += int(seg.sum())
        seg[:] = 0
    return valid


def _gap_intervals(rng, t_span, fraction, mean_len_s=6 * 3600.0):
    """Gaps as time intervals [start, end) over [0, t_span): exponential lengths at uniform
    random starts until the requested fraction of the span is covered (union)."""
    if fraction <= 0.0:
        return []
    grid = np.zeros(int(t_span) + 1, dtype=np.uint8)  # one-second bookkeeping of the covered time
    out = []
    target = fraction * t_span
    covered = 0.0
    while covered < target:
        a = float(rng.uniform(0.0, t_span))
        b = min(t_span, a + float(rng.exponential(mean_len_s)))
        out.append((a, b))
        seg = grid[int(a):int(b) + 1]
        covered += float(len(seg) - int(seg.sum()))
        seg[:] = 1
    return out


def _random_injections(rng, count, band, tspec, t_asc0, period):
    f_lo = band["f_min"] + 0.1 * band["f_band"]
    f_hi = band["f_min"] + 0.9 * band["f_band"]
    ap_lo, ap_hi = tspec["a_p"][0], tspec["a_p"][1]
    ta_lo, ta_hi = tspec["t_asc"][0], tspec["t_asc"][1]
    out = []
    for _ in range(count):
        out.append(dict(
            f0=float(rng.uniform(f_lo, f_hi)),
            a_p=float(rng.uniform(ap_lo, ap_hi)),
            t_asc_off=float(rng.uniform(ta_lo, ta_hi)),
            period=float(period),
            h0=float(rng.uniform(0.04, 0.07)),
            cosi=float(rng.uniform(-1.0, 1.0)),
            psi=float(rng.uniform(0.0, math.pi)),
            phi0=float(rng.uniform(0.0, 2.0 * math.pi)),
        ))
    return out


def make_dataset(cfg, seed=None, signal=True, noise=True, sky=None, antenna_piecewise=False,
                 sigma_wander=0.0, chunk=1 << 20, workers=None, per_sample_antenna=False):
    """Build a dataset from a workload dict (see ``configs.CONFIGS``).

    ``sky`` overrides Earth-model/sky fields (e.g. ``au_s=0`` to switch off the
    orbital delay).  ``antenna_piecewise`` injects signals whose a, b are held
    at the mid-segment values over each segment (closed-form tests).
    ``sigma_wander`` makes the noise level vary slowly from segment to segment.
    ``workers`` threads synthesise the injected signals chunk by chunk (default: CPU count,
    at most 16); the result does not depend on it.  ``per_sample_antenna`` also stores a(tau_r),
    b(tau_r) on the source lattice (ds.ar, ds.br).  An injection with keys ``ecc``, ``w`` and
    ``t_p_off`` follows an eccentric orbit (periapse time t_asc0 + t_p_off).
    """
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    seed = cfg["seed"] if seed is None else seed
    band = dict(cfg["band"])
    skyd = default_sky(**(sky or {}))
    sites = [dict(SITES[d]) if isinstance(d, str) else dict(d) for d in cfg["detectors"]]
    q = len(sites)
    n_k = int(cfg["n_k"]) if cfg.get("n_k") else samples_per_segment(band)
    t_short = band["t_short"]
    dt = t_short / n_k
    n_seg = int(round(cfg["t_obs"] / t_short))
    n = n_seg * n_k
    t0 = float(cfg.get("t0", 0.0))
    f_het = band["f_min"] + 0.5 * band["f_band"]

    t_mid = t0 + (np.arange(n_seg) + 0.5) * t_short
    a = np.zeros((q, n_seg))
    b = np.zeros((q, n_seg))
    noise_var = np.zeros((q, n_seg))
    x = np.zeros((q, n), dtype=np.complex64)
    valid = np.zeros((q, n), dtype=np.uint8)

    t_asc0 = cfg["t_asc0"]
    inj_spec = cfg.get("injections") or []
    if isinstance(inj_spec, str):
        count = int(inj_spec.replace("random", ""))
        inj_spec = _random_injections(np.random.Generator(np.random.PCG64(seed + 77)), count, band,
                                      cfg["templates"], t_asc0, cfg["templates"]["period"][len(cfg["templates"]["period"]) // 2])
    injections = [dict(i, t_asc=t_asc0 + i["t_asc_off"]) for i in inj_spec] if signal else []

    for X in range(q):
        s = sites[X]
        rng = np.random.Generator(np.random.PCG64(seed * 1000 + 10 * X + 1))
        aa, bb = antenna_ab(t_mid, s, skyd)
        a[X], b[X] = aa, bb
        sig0 = cfg["sigma"][X]
        if sigma_wander > 0.0:
            kk = np.arange(n_seg)
            sig_k = sig0 * (1.0 + sigma_wander * np.sin(2.0 * math.pi * kk / max(n_seg, 2) * 3.0 + X))
        else:
            sig_k = np.full(n_seg, sig0)
        noise_var[X] = sig_k ** 2

        v = np.ones(n, dtype=np.uint8)
        cov = cfg.get("coverage")
        if cov is not None:
            start_f, len_f = cov[X]
            lo = int(start_f * n)
            hi = min(n, lo + int(len_f * n))
            v[:lo] = 0
            v[hi:] = 0
        if cfg.get("gap_fraction", 0.0) > 0.0:
            if cfg.get("gap_seed") is not None:
                # gaps fixed in time (the same for every band of a multi-band workload)
                grng = np.random.Generator(np.random.PCG64(cfg["gap_seed"] * 1000 + 10 * X + 7))
                for a_, b_ in _gap_intervals(grng, n_seg * t_short, cfg["gap_fraction"]):
                    v[int(math.ceil(a_ / dt)):int(math.ceil(b_ / dt))] = 0  # samples with a <= j dt < b
            else:
                v &= _gap_mask(rng, n, dt, cfg["gap_fraction"])
        valid[X] = v

        xs_all = np.zeros(n, dtype=np.complex128)
        if noise:
            # one sequential stream of normal draws per detector, chunk after chunk
            for lo in range(0, n, chunk):
                hi = min(n, lo + chunk)
                m = hi - lo
                sk = np.repeat(np.sqrt(noise_var[X]), n_k)[lo:hi]
                z = rng.standard_normal(2 * m).reshape(m, 2)
                xs_all[lo:hi] += (z[:, 0] + 1j * z[:, 1]) * (sk / math.sqrt(2.0))

        def add_signals(lo, s=s, aa=aa, bb=bb, xs_all=xs_all):
            hi = min(n, lo + chunk)
            xs = xs_all[lo:hi]
            tj = t0 + np.arange(lo, hi, dtype=np.float64) * dt
            if not antenna_piecewise:
                at, bt = antenna_ab(tj, s, skyd)
            ej = earth_roemer(tj, s, skyd)
            for inj in injections:
                if "ecc" in inj:
                    d = forward_delay_ecc(tj, s, skyd, inj["a_p"], t_asc0 + inj["t_p_off"], inj["w"], inj["ecc"],
                                          inj["period"], e=ej)
                else:
                    d = forward_delay(tj, s, skyd, inj["a_p"], inj["t_asc"], inj["period"], e=ej)
                if antenna_piecewise:
                    # hold a, b at the value of the source-frame segment the sample lands in
                    kidx = np.clip(np.floor((tj + d - t0) / t_short).astype(np.int64), 0, n_seg - 1)
                    at, bt = aa[kidx], bb[kidx]
                c2, s2 = math.cos(2 * inj["psi"]), math.sin(2 * inj["psi"])
                fp = at * c2 + bt * s2
                fx = bt * c2 - at * s2
                ci = inj["cosi"]
                ap_ = inj["h0"] * 0.5 * (1.0 + ci * ci)
                ax_ = inj["h0"] * ci
                # Phi - 2 pi f_h t = phi0 + 2 pi [(f0 - f_h) t + f0 (tau - t)]
                cyc = (inj["f0"] - f_het) * tj + inj["f0"] * d
                cyc = cyc - np.floor(cyc)
                ph = inj["phi0"] + 2.0 * math.pi * cyc
                xs += 0.5 * (fp * ap_ - 1j * fx * ax_) * np.exp(1j * ph)

        if injections:
            # chunks are independent (no random draws): numpy releases the GIL in the array work
            with ThreadPoolExecutor(max_workers=max(1, min(workers, (n + chunk - 1) // chunk))) as ex:
                list(ex.map(add_signals, range(0, n, chunk)))
        xs_all *= v
        x[X] = xs_all.astype(np.complex64)

    templates = template_grid(cfg["templates"], t_asc0)
    ar = br = None
    if per_sample_antenna:
        tau = t0 + np.arange(n_seg * n_k) * dt
        ab = [antenna_ab(tau, s_, skyd) for s_ in sites]
        ar = np.stack([v[0] for v in ab])
        br = np.stack([v[1] for v in ab])
    return Dataset(sky=skyd, band=band, sites=sites, dt=dt, t0=t0, n=n, n_k=n_k, n_seg=n_seg,
                   f_het=f_het, x=x, valid=valid, a=a, b=b, noise_var=noise_var,
                   templates=templates, injections=injections, name=cfg.get("name", ""), ar=ar, br=br)


def multiband_bands(spec):
    """Band list of a multi-band workload: f_min linear over [f_lo, f_hi), f_band cycling
    through the given widths, T_short log-interpolated from t_short_lo (at f_lo) to
    t_short_hi (at f_hi) and rounded to whole seconds."""
    out = []
    cnt = spec["count"]
    for i in range(cnt):
        f_min = spec["f_lo"] + (spec["f_hi"] - spec["f_lo"]) * i / cnt
        frac = (f_min - spec["f_lo"]) / (spec["f_hi"] - spec["f_lo"])
        t_short = float(round(math.exp(math.log(spec["t_short_lo"]) +
                                       (math.log(spec["t_short_hi"]) - math.log(spec["t_short_lo"])) * frac)))
        out.append(dict(f_min=f_min, f_band=spec["f_band"][i % len(spec["f_band"])], t_short=t_short,
                        max_lag=spec["max_lag"], dirichlet_D=8, window=0, mu_f=0.1, n_fft_override=0,
                        pairs=spec.get("pairs", 3), a_p_max=spec["a_p_max"]))
    return out


def make_multiband(cfg, bands=None, workers=None, **over):
    """Datasets of a multi-band workload (one per band, same detectors, coverage and gap
    times; independent noise per band; one random injection in every `inject_every`-th
    band).  ``bands`` selects band indices; ``over`` overrides top-level fields."""
    cfg = dict(cfg, **over)
    blist = multiband_bands(cfg["bands"])
    idx = range(len(blist)) if bands is None else bands
    out = []
    for i in idx:
        c = dict(cfg)
        c["band"] = blist[i]
        c["seed"] = cfg["seed"] * 100 + i
        c["gap_seed"] = cfg["seed"]
        every = cfg.get("inject_every", 0)
        c["injections"] = "random1" if every and i % every == 0 else []
        ds = make_dataset(c, workers=workers)
        ds.name = f"{cfg.get('name', 'multiband')}[{i}]"
        out.append(ds)
    return out

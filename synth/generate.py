"""Seeded synthetic datasets: heterodyned complex series, gaps, weights, templates."""

import math
from dataclasses import dataclass, field

import numpy as np

from .model import SITES, antenna_ab, default_sky, earth_roemer, forward_delay, samples_per_segment


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
    templates: np.ndarray  # (T, 3) columns a_p, T_asc, P
    injections: list = field(default_factory=list)
    name: str = ""

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
                 sigma_wander=0.0, chunk=1 << 20):
    """Build a dataset from a workload dict (see ``configs.CONFIGS``).

    ``sky`` overrides Earth-model/sky fields (e.g. ``au_s=0`` to switch off the
    orbital delay).  ``antenna_piecewise`` injects signals whose a, b are held
    at the mid-segment values over each segment (closed-form tests).
    ``sigma_wander`` makes the noise level vary slowly from segment to segment.
    """
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
            v &= _gap_mask(rng, n, dt, cfg["gap_fraction"])
        valid[X] = v

        for lo in range(0, n, chunk):
            hi = min(n, lo + chunk)
            m = hi - lo
            xs = np.zeros(m, dtype=np.complex128)
            if noise:
                sk = np.repeat(np.sqrt(noise_var[X]), n_k)[lo:hi]
                z = rng.standard_normal(2 * m).reshape(m, 2)
                xs += (z[:, 0] + 1j * z[:, 1]) * (sk / math.sqrt(2.0))
            if injections:
                tj = t0 + np.arange(lo, hi, dtype=np.float64) * dt
                if not antenna_piecewise:
                    at, bt = antenna_ab(tj, s, skyd)
                ej = earth_roemer(tj, s, skyd)
                for inj in injections:
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
            xs *= v[lo:hi]
            x[X, lo:hi] = xs.astype(np.complex64)

    templates = template_grid(cfg["templates"], t_asc0)
    return Dataset(sky=skyd, band=band, sites=sites, dt=dt, t0=t0, n=n, n_k=n_k, n_seg=n_seg,
                   f_het=f_het, x=x, valid=valid, a=a, b=b, noise_var=noise_var,
                   templates=templates, injections=injections, name=cfg.get("name", ""))

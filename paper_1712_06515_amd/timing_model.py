"""Resampling timing model of the paper's three-term form (Sec. IV.B, eq. resampTimingModelEq),
with its constants fitted to run times measured on this GPU over a sweep of band configurations.

The paper models the run time of a band as

    T = N_orb N_det (T_obs / T_max) [ tau_CC  N_f triang(N_det)
                                    + tau_bary 2 Delta f_load T_max (D / 8)
                                    + tau_FFT  N_FFT 5 log2(N_FFT) triang(N_det) ],
    triang(N) = 1 + (N + 1) / 2,

one constant for the per-bin work (pair sums, copies, phase shifts), one for the barycentring
and interpolation of each source sample, one for the FFT.  Here the quantities come from the
library's band plan: T_obs / T_max is the number of segments per detector M (the paper takes
T_max = T_short, the segment length, which is what the plan's segments are), 2 Delta f_load T_max
is 2 N_K (N_K = ceil(T_short Delta f_load) complex samples per segment), N_FFT the plan's FFT
length and N_f its output bins; N_orb is the number of orbital templates of the call.  The fit is
a nonnegative least-squares fit of the relative residuals, done separately below and above the
N_FFT threshold (2^18) that the paper's table splits at when both sides have measurements.

This module measures and fits; it computes nothing of the statistic itself.  `python -m
paper_1712_06515_amd.timing_model --out FILE` runs the sweep on the GPU and writes the
measurements and the fitted constants.
"""

import argparse
import json
import math
import time

import numpy as np

NFFT_SPLIT = 1 << 18
NAMES = ("tau_CCbin", "tau_bary", "tau_FFT")


def triang(n):
    return 1.0 + (n + 1.0) / 2.0


def features(info, n_orb, dirichlet_D):
    """The three terms of eq. resampTimingModelEq without their constants, from a band plan
    (`ccr_get_band_info` fields n_det, n_seg, n_f, n_k, n_fft)."""
    q, m = float(info["n_det"]), float(info["n_seg"])
    lead = float(n_orb) * q * m
    nfft = float(info["n_fft"])
    return np.array([
        lead * float(info["n_f"]) * triang(q),
        lead * 2.0 * float(info["n_k"]) * (dirichlet_D / 8.0),
        lead * nfft * 5.0 * math.log2(nfft) * triang(q),
    ])


def _fit_one(X, t):
    """Nonnegative least squares of the relative residuals (pred - t) / t; constants, their 1-sigma
    uncertainties from the residual variance, and the rms relative residual."""
    from scipy.optimize import nnls
    A = X / t[:, None]
    b = np.ones_like(t)
    scale = np.maximum(A.max(axis=0), 1e-300)
    tau_s, _ = nnls(A / scale, b)
    tau = tau_s / scale
    res = A @ tau - b
    dof = max(1, len(t) - X.shape[1])
    s2 = float(res @ res) / dof
    cov = np.linalg.pinv(A.T @ A) * s2
    return {
        "tau": {n: float(v) for n, v in zip(NAMES, tau)},
        "sigma": {n: float(math.sqrt(max(cov[i, i], 0.0))) for i, n in enumerate(NAMES)},
        "rel_rms": float(math.sqrt(np.mean(res ** 2))),
        "rel_max": float(np.max(np.abs(res))),
        "n": int(len(t)),
    }


def fit(rows):
    """rows: dicts with 'features' (3 numbers), 'seconds' and 'n_fft'.  Returns {'low': fit,
    'high': fit or None} split at N_FFT = 2^18 (a side with fewer than 4 rows takes the other's
    fit)."""
    X = np.array([r["features"] for r in rows], dtype=float)
    t = np.array([r["seconds"] for r in rows], dtype=float)
    nf = np.array([r["n_fft"] for r in rows])
    lo, hi = nf < NFFT_SPLIT, nf >= NFFT_SPLIT
    out = {"low": None, "high": None}
    if lo.sum() >= 4:
        out["low"] = _fit_one(X[lo], t[lo])
    if hi.sum() >= 4:
        out["high"] = _fit_one(X[hi], t[hi])
    if out["low"] is None and out["high"] is None:
        out["low"] = _fit_one(X, t)
    return out


def predict(model, info, n_orb, dirichlet_D):
    """Predicted seconds for one band of `n_orb` templates."""
    side = model["high"] if info["n_fft"] >= NFFT_SPLIT and model.get("high") else (model["low"] or model["high"])
    tau = np.array([side["tau"][n] for n in NAMES])
    return float(features(info, n_orb, dirichlet_D) @ tau)


def sweep_configs():
    """Band configurations of the sweep: the parameters the paper varies (f_band, T_obs, T_max
    through the lag R, N_det, f_min, a_p, mu_f, D) one at a time around a base case, plus the
    segment length, then seeded random combinations."""
    day = 86400.0
    base = dict(q=2, t_obs=4 * day, t_short=600.0, f_min=200.0, f_band=0.1, R=0, a_p=1.5, mu_f=0.1, D=8)
    vary = dict(f_band=[0.05, 0.2, 0.4], t_obs=[2 * day, 8 * day, 16 * day], R=[1, 2, 4], q=[1, 3],
                f_min=[50.0, 400.0, 800.0], a_p=[0.5, 3.0], mu_f=[0.05, 0.3], D=[4, 16],
                t_short=[240.0, 1800.0])
    cfgs = [dict(base)]
    for k, vals in vary.items():
        for v in vals:
            c = dict(base)
            c[k] = v
            cfgs.append(c)
    rng = np.random.default_rng(1029)
    for _ in range(20):
        cfgs.append(dict(q=int(rng.integers(1, 4)), t_obs=float(rng.choice([2, 4, 8]) * day),
                         t_short=float(rng.choice([240.0, 600.0, 1440.0])), f_min=float(rng.choice([50.0, 200.0, 600.0])),
                         f_band=float(rng.choice([0.05, 0.1, 0.25])), R=int(rng.integers(0, 4)),
                         a_p=float(rng.choice([1.0, 2.0])), mu_f=float(rng.choice([0.1, 0.2])),
                         D=int(rng.choice([4, 8, 12]))))
    return cfgs


def _workload(c):
    dets = ["H", "L", "V"][:c["q"]]
    lag = max(c["R"], 1) if c["q"] == 1 else c["R"]  # one detector: pairs within it need a lag
    return dict(
        detectors=dets, t_obs=c["t_obs"], gap_fraction=0.0, coverage=None, sigma=[1.0 + 0.1 * i for i in range(c["q"])],
        band=dict(f_min=c["f_min"], f_band=c["f_band"], t_short=c["t_short"], max_lag=lag, dirichlet_D=c["D"],
                  window=0, mu_f=c["mu_f"], n_fft_override=0, pairs=3 if c["q"] > 1 else 2, a_p_max=c["a_p"]),
        templates=dict(a_p=(0.9 * c["a_p"], c["a_p"], 16), t_asc=(-500.0, 500.0, 16), period=[68023.7]),
        t_asc0=c["t_obs"] / 2, injections=[], seed=77,
    )


def run_sweep(n_orb=256, repeats=3, prec=1, progress=print):
    """Measure every sweep configuration on device 0 (split precision by default): the minimum
    over `repeats` of the wall time of one ccr_compute_rho call on device outputs, synchronised,
    after one untimed call.  Same-time pairs within a detector are used when N_det = 1."""
    import torch
    import synth
    from . import ccr
    rows = []
    for i, c in enumerate(sweep_configs()):
        ds = synth.make_dataset(_workload(c), signal=False)
        tm = ds.templates[:n_orb]
        with ccr.Context(ds.sky, device=0) as ctx:
            ctx.set_option("graph", 1)
            bid = ctx.load(ds, templates=tm)
            info = ctx.band_info(bid)
            out = torch.empty((len(tm), info["n_f"]), dtype=torch.float32, device="cuda")
            ctx.compute_rho(bid, prec=prec, out_fp64=False, outputs=[out.data_ptr()])
            ctx.sync()
            best = float("inf")
            for _ in range(repeats):
                t0 = time.perf_counter()
                ctx.compute_rho(bid, prec=prec, out_fp64=False, outputs=[out.data_ptr()])
                ctx.sync()
                best = min(best, time.perf_counter() - t0)
        row = dict(config=c, n_orb=len(tm), n_fft=int(info["n_fft"]), n_f=int(info["n_f"]), n_k=int(info["n_k"]),
                   n_seg=int(info["n_seg"]), seconds=best,
                   features=[float(v) for v in features(info, len(tm), c["D"])])
        rows.append(row)
        progress(f"[{i + 1}] {json.dumps(c)} n_fft={row['n_fft']} n_f={row['n_f']} n_k={row['n_k']} "
                 f"M={row['n_seg']}: {best * 1e3:.2f} ms")
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="text file for the measurements and the fit")
    ap.add_argument("--templates", type=int, default=256)
    ap.add_argument("--fp64", action="store_true", help="time the plain FP64 path instead of the split one")
    a = ap.parse_args()
    rows = run_sweep(n_orb=a.templates, prec=0 if a.fp64 else 1, progress=lambda s: print(s, flush=True))
    model = fit(rows)
    with open(a.out, "w") as f:
        f.write("# GPU timing model, eq. resampTimingModelEq form (Sec. IV.B): measured seconds per call and\n")
        f.write("# the fitted constants; one JSON object per line after the header\n")
        f.write(json.dumps({"fit": model, "precision": "fp64" if a.fp64 else "split", "templates": a.templates}) + "\n")
        for r in rows:
            f.write(json.dumps(r) + "\n")
    print(json.dumps(model, indent=1))


if __name__ == "__main__":
    main()

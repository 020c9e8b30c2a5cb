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
a nonnegative least-squares fit of the relative residuals.  The paper fits its constants
separately below and above N_FFT = 2^18, where its CPU FFT slows down; on this GPU the cost per
unit changes with the kernel that computes the segment spectra and pair sums (one fused kernel
for 256-point segments, one for 256- to 1024-point segments, the general staged kernels otherwise), so
the constants are fitted per kernel path (a path with fewer than 4 measurements takes the fit
over all of them).

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


PATHS = ("fused256", "wide", "general")


def fit(rows):
    """rows: dicts with 'features' (3 numbers), 'seconds' and 'path'.  Returns {'all': fit,
    path: fit or None for each kernel path}."""
    X = np.array([r["features"] for r in rows], dtype=float)
    t = np.array([r["seconds"] for r in rows], dtype=float)
    paths = np.array([r.get("path", "general") for r in rows])
    out = {"all": _fit_one(X, t)}
    for p in PATHS:
        sel = paths == p
        out[p] = _fit_one(X[sel], t[sel]) if sel.sum() >= 4 else None
    return out


def predict(model, info, n_orb, dirichlet_D, path="general"):
    """Predicted seconds for one band of `n_orb` templates on the given kernel path."""
    side = model.get(path) or model["all"]
    tau = np.array([side["tau"][n] for n in NAMES])
    return float(features(info, n_orb, dirichlet_D) @ tau)


def sweep_configs():
    """Band configurations of the sweep: the parameters the paper varies (f_band, T_obs, T_max
    through the lag R, N_det, f_min, a_p, mu_f, D) one at a time around a base case, plus the
    segment length, then seeded random combinations."""
    day = 86400.0
    base = dict(q=2, t_obs=16 * day, t_short=600.0, f_min=200.0, f_band=0.1, R=0, a_p=1.5, mu_f=0.1, D=8)
    vary = dict(f_band=[0.05, 0.2, 0.4], t_obs=[4 * day, 8 * day, 32 * day], R=[1, 2, 4], q=[1, 3],
                f_min=[50.0, 400.0, 800.0], a_p=[0.5, 3.0], mu_f=[0.05, 0.3], D=[4, 16],
                t_short=[240.0, 1800.0])
    cfgs = [dict(base)]
    for k, vals in vary.items():
        for v in vals:
            c = dict(base)
            c[k] = v
            cfgs.append(c)
    # 1024-point segments (N_K in 513 .. 1024): long segments over wider bands
    for ts, fb, R, q in ((1440.0, 0.25, 0, 2), (1440.0, 0.25, 2, 2), (1440.0, 0.25, 4, 2), (1440.0, 0.2, 1, 3),
                         (1800.0, 0.2, 0, 2), (1440.0, 0.3, 1, 1), (1200.0, 0.3, 2, 2), (1800.0, 0.25, 3, 3)):
        cfgs.append(dict(base, t_short=ts, f_band=fb, R=R, q=q, f_min=400.0, a_p=2.0))
    rng = np.random.default_rng(1029)
    for _ in range(20):
        cfgs.append(dict(q=int(rng.integers(1, 4)), t_obs=float(rng.choice([8, 16, 32]) * day),
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
        templates=dict(a_p=(0.9 * c["a_p"], c["a_p"], 32), t_asc=(-500.0, 500.0, 64), period=[68023.7]),
        t_asc0=c["t_obs"] / 2, injections=[], seed=77,
    )


def run_sweep(n_orb=2048, repeats=3, prec=1, progress=print):
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
            # which kernels computed the spectra and pair sums (one timed, untimed-for-the-fit call)
            ctx.set_option("graph", 0)
            ctx.set_option("timing", 1)
            ctx.compute_rho(bid, prec=prec, out_fp64=False, outputs=[out.data_ptr()])
            kt = ctx.kernel_times(reset=True)
            path = ("fused256" if kt["spectra_pairs"][1] else "wide" if kt["spectra_wide"][1] else "general")
        row = dict(config=c, n_orb=len(tm), n_fft=int(info["n_fft"]), n_f=int(info["n_f"]), n_k=int(info["n_k"]),
                   n_seg=int(info["n_seg"]), seconds=best, path=path,
                   features=[float(v) for v in features(info, len(tm), c["D"])])
        rows.append(row)
        progress(f"[{i + 1}] {json.dumps(c)} n_fft={row['n_fft']} n_f={row['n_f']} n_k={row['n_k']} "
                 f"M={row['n_seg']} {path}: {best * 1e3:.2f} ms")
    return rows


def load_fit(path):
    """The fitted constants from a summary written by main() (None if absent)."""
    try:
        for line in open(path):
            if line.startswith("fit = "):
                return json.loads(line[len("fit = "):])
    except OSError:
        return None
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="text summary: the fitted constants and one line per configuration")
    ap.add_argument("--templates", type=int, default=2048)
    ap.add_argument("--fp64", action="store_true", help="time the plain FP64 path instead of the split one")
    a = ap.parse_args()
    rows = run_sweep(n_orb=a.templates, prec=0 if a.fp64 else 1, progress=lambda s: print(s, flush=True))
    model = fit(rows)
    with open(a.out, "w") as f:
        f.write("# GPU timing model of the form of eq. resampTimingModelEq (Sec. IV.B), fitted per kernel path\n")
        f.write(f"# command: python -m paper_1712_06515_amd.timing_model --out {a.out}"
                f"{' --fp64' if a.fp64 else ''} --templates {a.templates}\n")
        f.write(f"# precision {'fp64' if a.fp64 else 'split'}, {a.templates} orbital templates per call, wall time of one\n"
                "# synchronised ccr_compute_rho call (minimum of 3, graph replay), no gaps, synthetic noise\n")
        for p in ("all",) + PATHS:
            v = model[p]
            if v:
                f.write(f"# {p:9s} n={v['n']:2d} " + " ".join(f"{n}={v['tau'][n]:.3e}+-{v['sigma'][n]:.1e}" for n in NAMES)
                        + f" rel_rms={v['rel_rms']:.3f} rel_max={v['rel_max']:.3f}\n")
        f.write("fit = " + json.dumps(model) + "\n")
        f.write("# q  R  T_short f_min f_band a_p  mu_f D  | N_K N_FFT  N_f     M path      | measured_ms predicted_ms\n")
        for r in rows:
            c = r["config"]
            pr = predict(model, dict(n_det=c["q"], n_seg=r["n_seg"], n_f=r["n_f"], n_k=r["n_k"], n_fft=r["n_fft"]),
                         r["n_orb"], c["D"], r["path"])
            f.write(f"  {c['q']}  {c['R']}  {c['t_short']:6.0f} {c['f_min']:5.0f} {c['f_band']:5.2f} {c['a_p']:4.1f} "
                    f"{c['mu_f']:4.2f} {c['D']:2d} | {r['n_k']:4d} {r['n_fft']:5d} {r['n_f']:5d} {r['n_seg']:5d} "
                    f"{r['path']:9s} | {r['seconds'] * 1e3:10.2f} {pr * 1e3:10.2f}\n")
    print(json.dumps(model, indent=1))


if __name__ == "__main__":
    main()

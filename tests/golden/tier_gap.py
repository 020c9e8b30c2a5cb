"""Tier R against Tier D per workload: the method's own error (interpolation, boundary and
Jacobian effects of resampling), reported beside the parity results, never asserted tightly.

Tier R is the resampled statistic the library reproduces (App. A eq. well-formatted-rho with the
resampled series of Sec. III.A); Tier D demodulates the raw detector-frame samples with the
exact phase model and no interpolation (App. A eq. from-here-resamp, the definition resampling
approximates).  Both come from the oracle alone (``oracle/``); the HIP library is not loaded.

    python tests/golden/tier_gap.py        # writes tests/golden/tier_gap.json

Subsets (Tier D sums every raw sample for every bin, so the long workloads are cut to their
first segments and, for the 240-day band, to a slice of bins):
  tiny       16 templates (the injection's nearest first) x every bin, the whole 2 days;
  band       the nearest template of each of the 10 injections x every bin, first 1440 segments;
  large      the nearest template of each injection in the bin slice, first 240 segments, 512 bins.
Per workload: max over (template, bin) of |rho_R - rho_D| / max(|rho_D|, 1), and at each
injection's peak (nearest template, bin nearest f0) the relative gap |rho_R - rho_D| / |rho_D|.
"""

import copy
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "tier_gap.json")


def nearest(templates, inj):
    d = ((templates[:, 0] - inj["a_p"]) ** 2 + ((templates[:, 1] - inj["t_asc"]) / 1000.0) ** 2
         + ((templates[:, 2] - inj["period"]) / 0.04) ** 2)
    return int(np.argmin(d))


def first_segments(ds, m):
    sub = copy.copy(ds)
    nsamp = m * ds.n_k
    sub.x, sub.valid = ds.x[:, :nsamp], ds.valid[:, :nsamp]
    sub.a, sub.b, sub.noise_var = ds.a[:, :m], ds.b[:, :m], ds.noise_var[:, :m]
    sub.n, sub.n_seg = nsamp, m
    return sub


def gap(ds, picks, injs, bins=None):
    o = oracle.Oracle(ds)
    tm = ds.templates[picks]
    t0 = time.time()
    R = o.rho(tm, tier=0, bins=bins)
    D = o.rho(tm, tier=1, bins=bins)
    freqs = o.frequencies() if bins is None else o.frequencies()[bins]
    peaks = []
    for j, inj in enumerate(injs):
        i = int(np.argmin(np.abs(freqs - inj["f0"])))
        peaks.append(dict(f0=inj["f0"], rho_D=float(D[j, i]), rho_R=float(R[j, i]),
                          rel_gap=float(abs(R[j, i] - D[j, i]) / max(abs(D[j, i]), 1e-300))))
    return dict(templates=len(picks), bins=int(R.shape[1]), segments=int(ds.n_seg),
                max_gap=float(np.max(np.abs(R - D) / np.maximum(np.abs(D), 1.0))),
                max_abs_rho_D=float(np.abs(D).max()), peaks=peaks, seconds=round(time.time() - t0, 1))


def main():
    out = {}
    ds = synth.make_dataset(synth.config("tiny"))
    inj = ds.injections
    picks = [nearest(ds.templates, inj[0])] + [t for t in range(0, len(ds.templates), 4) if t != nearest(ds.templates, inj[0])][:15]
    out["tiny"] = gap(ds, picks, inj)
    print("tiny", out["tiny"]["max_gap"], flush=True)

    ds = synth.make_dataset(synth.config("band"))
    sub = first_segments(ds, 1440)
    picks = [nearest(ds.templates, i) for i in ds.injections]
    out["band"] = gap(sub, picks, ds.injections)
    print("band", out["band"]["max_gap"], flush=True)

    ds = synth.make_dataset(synth.config("large"))
    sub = first_segments(ds, 240)
    freqs = oracle.Oracle(sub).frequencies()
    lo, hi = 3000, 3512
    inside = [i for i in ds.injections if freqs[lo] <= i["f0"] <= freqs[hi - 1]][:4]
    picks = [nearest(ds.templates, i) for i in inside]
    out["large"] = gap(sub, picks, inside, bins=np.arange(lo, hi))
    print("large", out["large"]["max_gap"], flush=True)
    json.dump(out, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()

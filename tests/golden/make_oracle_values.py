"""Write the oracle's rho for the sampled templates and bins of the three full-size workloads.

The oracle (``oracle/``) is slow by design: at full size (120 and 240 days) the sampled
templates take it minutes on a few host cores, so the GPU parity tests read its values from
here instead of recomputing them.  Nothing but ``synth`` (seeded inputs) and ``oracle`` is
called; the HIP library is not loaded.  Re-run after any change to ``synth`` or to the oracle:

    python tests/golden/make_oracle_values.py            # all three
    python tests/golden/make_oracle_values.py band       # one of band / large / multiband

Sampling (the parity protocol of the workloads):
  band       the template nearest each of the 10 injections + 8 seeded random templates, every bin;
  large      8 seeded random templates of the first 1002 + the templates nearest 8 injections whose
             frequency falls in a contiguous 1024-bin slice, over that slice;
  multiband  8 bands at full size (120 days, 1024 templates each), 2 templates per band (the
             nearest to the band's injection where it has one, else random), every bin.
"""

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

INDEX = os.path.join(HERE, "oracle_values.json")
MB_BANDS = [0, 9, 18, 27, 36, 45, 54, 63]
LARGE_FIRST = 1002
LARGE_SLICE = (3000, 4024)


def nearest(templates, inj, period_scale=0.04):
    d = ((templates[:, 0] - inj["a_p"]) ** 2 + ((templates[:, 1] - inj["t_asc"]) / 1000.0) ** 2
         + ((templates[:, 2] - inj["period"]) / period_scale) ** 2)
    return int(np.argmin(d))


def picks_band(ds):
    rng = np.random.default_rng(11)
    pick = [nearest(ds.templates, inj) for inj in ds.injections]
    for t in rng.choice(len(ds.templates), 8, replace=False).tolist():
        if t not in pick:
            pick.append(int(t))
    return pick, None


def picks_large(ds, freqs):
    lo, hi = LARGE_SLICE
    rng = np.random.default_rng(17)
    pick = [int(t) for t in rng.choice(LARGE_FIRST, 8, replace=False)]
    inside = [inj for inj in ds.injections if freqs[lo] <= inj["f0"] <= freqs[hi - 1]]
    for inj in inside[:8]:
        t = nearest(ds.templates, inj)
        if t not in pick:
            pick.append(t)
    return pick, list(range(lo, hi))


def picks_multiband(dss):
    rng = np.random.default_rng(23)
    out = []
    for ds in dss:
        pick = [nearest(ds.templates, ds.injections[0])] if ds.injections else []
        while len(pick) < 2:
            t = int(rng.integers(len(ds.templates)))
            if t not in pick:
                pick.append(t)
        out.append(pick)
    return out


def main(which):
    index = json.load(open(INDEX)) if os.path.exists(INDEX) else {}
    index["_about"] = ("rho of the oracle (Tier R, oracle/ccr_oracle.c) at sampled templates and bins of the "
                       "full-size workloads; written by tests/golden/make_oracle_values.py, which calls only "
                       "synth and oracle")
    if "band" in which:
        t0 = time.time()
        ds = synth.make_dataset(synth.config("band"))
        pick, _ = picks_band(ds)
        rho = oracle.Oracle(ds).rho(ds.templates[pick])
        np.save(os.path.join(HERE, "oracle_band.npy"), rho)
        index["band"] = dict(templates=pick, bins="all", shape=list(rho.shape),
                             injections_nearest=len(ds.injections), seconds=round(time.time() - t0, 1))
        print(f"band: {rho.shape} in {time.time() - t0:.0f} s", flush=True)
    if "large" in which:
        t0 = time.time()
        ds = synth.make_dataset(synth.config("large"))
        o = oracle.Oracle(ds)
        pick, bins = picks_large(ds, o.frequencies())
        rho = o.rho(ds.templates[pick], bins=bins)
        np.save(os.path.join(HERE, "oracle_large.npy"), rho)
        index["large"] = dict(templates=pick, bins=[bins[0], bins[-1] + 1], shape=list(rho.shape),
                              first_templates=LARGE_FIRST, seconds=round(time.time() - t0, 1))
        print(f"large: {rho.shape} in {time.time() - t0:.0f} s", flush=True)
    if "multiband" in which:
        t0 = time.time()
        dss = synth.make_multiband(synth.config("multiband"), bands=MB_BANDS)
        picks = picks_multiband(dss)
        rhos = [oracle.Oracle(ds).rho(ds.templates[p]) for ds, p in zip(dss, picks)]
        width = max(r.shape[1] for r in rhos)
        arr = np.full((len(dss), 2, width), np.nan)
        for i, r in enumerate(rhos):
            arr[i, :, :r.shape[1]] = r
        np.save(os.path.join(HERE, "oracle_multiband.npy"), arr)
        index["multiband"] = dict(bands=MB_BANDS, templates=picks, n_f=[int(r.shape[1]) for r in rhos],
                                  seconds=round(time.time() - t0, 1))
        print(f"multiband: {arr.shape} in {time.time() - t0:.0f} s", flush=True)
    json.dump(index, open(INDEX, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["band", "large", "multiband"])

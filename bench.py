"""Throughput of the resampled cross-correlation hot path on one MI355X.

One step = one ccr_compute_rho over every orbital template of the step and every output bin
(time base, resampling, segment FFTs, pair sums, normalisation), inputs resident in HBM, output
on device, split precision (FP64 time base and phases; FP32 interpolation, FFT and pair
products), the call captured as a HIP graph and its launch shapes autotuned on first use.

Workload "large" (default): 2 detectors, 240 days, no gaps, T_short = 1440 s, lags up to
4 segments, 0.25 Hz band at 400 Hz (N_K 870, N_FFT 32768, 7413 bins), Gaussian noise + 100
injections; its grid has 100 200 templates (200 a_p x 167 T_asc x 3 P), of which a step takes
the first 1002 (one GPU's share of a 100-GPU template split; the rate is per rho evaluation).
The plain FP64 path (one template per launch sequence, no graph) is timed beside it, and the
realistic 120-day band and the 64-band batching workload are timed as extra lines.

Prints one JSON line.  Also: --profile-steps N runs N untimed steps only (for rocprofv3),
--copy-calibration runs a 1 GiB device copy (for scaling HBM counters).
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ρ evaluations (templates×freq bins)/s, FP32-batched vs plain FP64 at ≤1e-4 rel err"
HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak (published).  It counts packed FP32 (two lanes of arithmetic per
# instruction); the library is compiled without packed FP32, so its kernels can reach at most half.
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "large": "2 detectors, 240 d, no gaps, T_short 1440 s, lags up to 4, 0.25 Hz at 400 Hz (7413 bins), "
             "noise + 100 injections; grid of 100200 templates (200 a_p x 167 T_asc x 3 P), first {n} per step",
    "band": "2 detectors, 120 d, 30% gaps, T_short 600 s, 0.1 Hz at 200 Hz, 4096 templates "
            "(64 a_p x 64 T_asc), lag 0 cross-detector pairs, noise + 10 injections",
    "tiny": "2 detectors, 2 d, T_short 360 s, 0.25 Hz at 100 Hz, 64 templates, same-time pairs",
    "multiband": "3 detectors (100/120/80 d of 120 d, 15% gaps), 64 bands of 0.05-0.2 Hz between 50 and "
                 "400 Hz, T_short 1400-240 s, lag 1, 1024 templates per band, one call",
}


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank lines removed (a comment edit does
    not change the kernels the counters were taken on)."""
    h = hashlib.sha256()
    for f in ("ccr_kernels.hip", "ccr_internal.h"):
        text = open(os.path.join(ROOT, "paper_1712_06515_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for line in text.splitlines():
            line = line.split("//", 1)[0].rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def read_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        m = re.match(r"^(\w+)\s*=\s*(\S+)", line)
        if m:
            kv[m.group(1)] = m.group(2)
    if kv.get("kernel_source_sha") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(ds, n_templates, seg_fraction):
    """The oracle timed on the host's cores over a bounded sample of the workload: as many
    templates as the oracle has threads (one template per thread, drawn from the step's
    templates), every bin, over the first `seg_fraction` of the segments (same band, detectors,
    sampling, gaps and weights).  The oracle's cost is linear in the number of segments, so the
    rate is scaled to full-length templates: value = templates x bins / (wall x M / M_sample)."""
    import copy

    import numpy as np
    import oracle
    nthreads = oracle.num_threads()
    m_sub = max(1, int(ds.n_seg * seg_fraction))
    sub = copy.copy(ds)
    nsamp = m_sub * ds.n_k
    sub.x, sub.valid = ds.x[:, :nsamp], ds.valid[:, :nsamp]
    sub.a, sub.b, sub.noise_var = ds.a[:, :m_sub], ds.b[:, :m_sub], ds.noise_var[:, :m_sub]
    sub.n, sub.n_seg = nsamp, m_sub
    o = oracle.Oracle(sub)
    n_f = o.plan().n_f
    rng = np.random.default_rng(5)
    n = min(n_templates, max(1, nthreads))
    idx = rng.choice(n_templates, size=n, replace=False)
    t0 = time.perf_counter()
    o.rho(ds.templates[idx])
    dt = time.perf_counter() - t0
    scale = ds.n_seg / m_sub
    return {"value": n * n_f / (dt * scale), "unit": "rho-evals/s", "cores": int(n), "kind": "oracle",
            "sample": f"{n} random templates of the step x all {n_f} bins over the first {m_sub} of {ds.n_seg} "
                      f"segments ({dt:.1f} s wall on {n} threads), rate scaled by {scale:.1f} to full-length templates"}


def roofline(name, avg_ms, tb, info, workload, streams=1):
    """Roofline entry of one kernel: `tb` templates per launch, `avg_ms` mean launch time;
    `streams` spectra per segment (2 with per-sample antenna functions)."""
    import numpy as np
    n_active = info["n_active"]
    ns, P = int(info["n_s"]), int(info["P"])
    if name == "resample" and info.get("farrow_used"):
        # Farrow form: one complex64 sample written per resampled sample, plus the band's
        # table (kFarDeg + 1 complex64 planes per input sample and detector) read once
        planes = info["farrow_degree"] + 1
        table = info["n_det"] * planes * 8.0 * info["n_seg"] * info["n_k"]
        byts = n_active * info["n_k"] * tb * 8.0 + table
        ach = byts / (avg_ms * 1e-3) / 1e9
        return {"kernel": "k_resample_far_m", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": read_traffic("resample", workload),
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": byts,
                "per_unit": f"8 B written per resampled sample + the Farrow table ({planes} x 8 B per input "
                            f"sample and detector) read once per launch"}
    if name == "resample":
        # one complex sample written per resampled sample; the input sample is read once per
        # tile of T_b templates
        T_b = info["resample_templates"]
        byts = n_active * info["n_k"] * tb * (8.0 + 8.0 / T_b)
        ach = byts / (avg_ms * 1e-3) / 1e9
        return {"kernel": "k_resample_m", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": read_traffic("resample", workload),
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": byts,
                "per_unit": f"{8.0 + 8.0 / T_b:g} B per resampled sample (8 B written, 8 B input "
                            f"per tile of {T_b} templates)"}
    flops = streams * n_active * tb * P * (5.0 * ns * np.log2(ns) + 6.0 * ns)
    per_unit = f"P (5 n_s log2 n_s + 6 n_s) FP32 flop per (template, detector, segment), n_s={ns}, P={P}"
    if streams != 1:
        per_unit += f", x{streams} spectra per segment"
    if name in ("spectra_pairs", "fused"):
        # the direct pair sum runs in the same kernel: 8 flop per (template, pair, bin) over the
        # pairs whose two spectra are present
        flops += 8.0 * info["n_pairs_present"] * info["n_f"] * tb
        per_unit += " + 8 flop per (template, pair with both spectra present, bin)"
    if name == "spectra_wide":
        per_unit += " (segment FFTs only: the pair sums, done as window sums, are not counted)"
    ach = flops / (avg_ms * 1e-3) / 1e12
    kern = {"spectra": "k_spectra16_m" if ns == 256 else "k_spectra_m", "spectra_pairs": "k_spectra_pairs_m",
            "fused": "k_fused", "spectra_wide": "k_spectra_wide_m"}[name]
    return {"kernel": kern, "bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP32_PEAK_TFLOPS, "traffic": read_traffic(name, workload),
            "avg_launch_ms": avg_ms, "algorithmic_flops_per_launch": flops, "per_unit": per_unit}


def pairs_present(ds, R, pairs):
    """Pairs of the pair set (Sec. III.B.1) whose two segment spectra exist, approximately: both
    segments hold valid input samples of their detector (the library marks a segment active from
    its source samples mapped through the Earth delay, which can differ at gap edges by a
    segment).  Exact for workloads without gaps."""
    import numpy as np
    Q, M = ds.n_det, ds.n_seg
    act = ds.valid[:, :M * ds.n_k].reshape(Q, M, ds.n_k).any(axis=2)
    n = 0
    for X in range(Q):
        for Y in range(Q):
            for dl in range(-R, R + 1):
                if not (((pairs & 1) and X < Y) or ((pairs & 2) and X == Y and dl > 0)):
                    continue
                a = act[X, max(0, -dl):M - max(0, dl)]
                b = act[Y, max(0, dl):M - max(0, -dl)]
                n += int(np.sum(a & b))
    return n


def golden_error(ds, rho, n_templates):
    """max |rho - rho_oracle| / max(|rho_oracle|, 1) of the timed output against the oracle's
    stored values (tests/golden, written by a script that calls only the oracle) for the sampled
    templates that lie in the step."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    if not os.path.exists(path):
        return None
    meta = json.load(open(path)).get("large")
    if meta is None:
        return None
    ref = np.load(os.path.join(ROOT, "tests", "golden", "oracle_large.npy"))
    lo, hi = meta["bins"]
    rows = [(j, t) for j, t in enumerate(meta["templates"]) if t < n_templates]
    if not rows:
        return None
    err = max(float(np.max(np.abs(rho[t, lo:hi] - ref[j]) / np.maximum(np.abs(ref[j]), 1.0))) for j, t in rows)
    return {"max_rel_err": err, "templates": len(rows), "bins": hi - lo,
            "against": "oracle (tests/golden/oracle_large.npy)"}


def time_steps(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["large", "band", "tiny", "multiband"],
                    help="multiband: the 64-band batching workload, with --profile-steps only (its timed line "
                         "is part of the default run)")
    ap.add_argument("--templates", type=int, default=1002,
                    help="templates per step (first N of the grid; 0: all)")
    ap.add_argument("--fp64-templates", type=int, default=32, help="templates timed on the plain FP64 path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra workload lines")
    ap.add_argument("--profile-steps", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--form-templates", type=int, default=256,
                    help="templates per step of the weighting / pair-set / orbit / front-end lines")
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--k-chunk", type=int, default=0,
                    help="segments per chunk of the spectra kernels (0: the library's choice, or the autotuner's); "
                         "for --profile-steps, the value the autotuner picked in the timed run")
    ap.add_argument("--template-batch", type=int, default=0,
                    help="templates per work item (0: the library's choice, or the autotuner's)")
    ap.add_argument("--round-templates", type=int, default=0,
                    help="templates per launch round at most (0: as many as the workspace holds)")
    ap.add_argument("--spectra-kernel", type=int, default=0,
                    help="1: the 256-1024-point spectra + pair-sum kernel wherever it applies")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU. Templates (and bands) are independent, so N GPUs would each "
              "take 1/N of the template list with the band data replicated, and exchange nothing but an "
              "optional final gather of candidates; that path is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return

    import synth
    from paper_1712_06515_amd import Context, PREC_FP64, PREC_SPLIT

    if args.workload == "multiband":
        if not args.profile_steps:
            print("--workload multiband runs with --profile-steps only", file=sys.stderr)
            sys.exit(2)
        dss = synth.make_multiband(synth.config("multiband"))
        ctx = Context(dss[0].sky, device=0)
        ids = [ctx.load(d) for d in dss]
        infos = [ctx.band_info(b) for b in ids]
        outs = [torch.empty((i["n_templates"], i["n_f"]), dtype=torch.float32, device="cuda") for i in infos]
        for opt in ("k_chunk", "template_batch", "round_templates", "spectra_kernel"):
            v = getattr(args, opt)
            if v:
                ctx.set_option(opt, v)
        log(f"multiband data: {len(ids)} bands")
        for i in range(args.profile_steps):
            ctx.compute_rho(ids, prec=PREC_SPLIT, out_fp64=False, outputs=[x.data_ptr() for x in outs])
            torch.cuda.synchronize()
            log(f"profile step {i} done")
        return

    t_gen = time.perf_counter()
    cfg = synth.config(args.workload)
    ds = synth.make_dataset(cfg)
    n_grid = len(ds.templates)
    if args.templates and args.templates < n_grid:
        ds.templates = ds.templates[:args.templates]
    log(f"dataset {args.workload}: {ds.n_det} det x {ds.n} samples, {len(ds.templates)} of {n_grid} templates "
        f"({time.perf_counter() - t_gen:.1f} s)")
    ctx = Context(ds.sky, device=0)
    bid = ctx.load(ds)
    info = ctx.band_info(bid)
    info["resample_templates"] = ctx.get_option("resample_templates")
    info["farrow_used"] = bool(ctx.get_option("farrow")) and info["farrow_degree"] > 0
    info["n_pairs_present"] = pairs_present(ds, cfg["band"]["max_lag"], cfg["band"].get("pairs", 3))
    n_t, n_f = info["n_templates"], info["n_f"]
    out = torch.empty((n_t, n_f), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        ctx.compute_rho(bid, prec=PREC_SPLIT, out_fp64=False, outputs=[out.data_ptr()], stream=stream.cuda_stream)

    for opt in ("k_chunk", "template_batch", "round_templates", "spectra_kernel"):
        if getattr(args, opt):
            ctx.set_option(opt, getattr(args, opt))
    if args.profile_steps:
        for i in range(args.profile_steps):
            step()
            torch.cuda.synchronize()
            log(f"profile step {i} done")
        return

    # the timed path: graph capture + autotuned launch shapes (tuning and capture happen in the
    # warm-up); at least one warm-up step so that neither is timed
    ctx.set_option("autotune", args.autotune)
    ctx.set_option("graph", args.graph)
    sec = time_steps(step, args.steps, max(1, args.warmup))
    ms_per_step = 1e3 * sec
    value = n_t * n_f / sec
    log(f"split path {ms_per_step:.2f} ms/step ({value:.3e} rho/s)")
    rho = out.cpu().numpy()
    err = golden_error(ds, rho, n_t) if args.workload == "large" else None
    tuned = {"k_chunk": ctx.get_option("tuned_k_chunk"), "template_batch": ctx.get_option("tuned_template_batch"),
             "round_templates": ctx.get_option("tuned_round_templates"),
             "spectra_kernel": ctx.get_option("tuned_spectra_kernel")}

    # per-kernel device time (HIP events on the launch stream), separate eager pass with the
    # same launches (graph replays are not timed per kernel)
    ctx.set_option("graph", 0)
    ctx.set_option("timing", 1)
    ctx.kernel_times(reset=True)
    k_steps = min(args.steps, 3)
    for _ in range(k_steps):
        step()
    kt = ctx.kernel_times(reset=True)
    ctx.set_option("timing", 0)

    # plain FP64 path: one template per launch sequence, no graph, on a bounded subset
    nsub = min(args.fp64_templates, n_t)
    ctx2 = Context(ds.sky, device=0)
    ctx2.set_option("template_batch", 1)
    ctx2.set_option("items_per_launch", 1)
    bid2 = ctx2.load(ds, templates=ds.templates[:nsub])
    out2 = torch.empty((nsub, n_f), dtype=torch.float64, device="cuda")

    def step64():
        ctx2.compute_rho(bid2, prec=PREC_FP64, out_fp64=True, outputs=[out2.data_ptr()], stream=stream.cuda_stream)

    s64 = time_steps(step64, 3, 1)
    value64 = nsub * n_f / s64
    log(f"fp64 plain {1e3 * s64:.1f} ms for {nsub} templates ({value64:.3e} rho/s)")
    ctx2.close()

    rooflines = {}
    for kname, (ms_tot, nl) in kt.items():
        if nl == 0 or kname not in ("resample", "spectra", "spectra_pairs", "fused", "spectra_wide"):
            continue
        rooflines[kname] = roofline(kname, ms_tot / nl, n_t / max(1, nl // k_steps), info, args.workload)
    name = max((k for k in rooflines), key=lambda k: kt[k][0])
    roof = rooflines.pop(name)
    workload = WORKLOADS[args.workload].format(n=n_t)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "rho-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 time base and phases)",
        "data": "synthetic (seeded noise, injections, gaps; analytic Earth model)",
        "config": {"workload": f"{args.workload}: {workload}", "templates": n_t, "bins": n_f,
                   "n_k": info["n_k"], "n_seg": info["n_seg"], "n_fft": info["n_fft"], "max_lag": cfg["band"]["max_lag"],
                   "graph": args.graph, "autotune": args.autotune, "tuned": tuned},
        "rho_error": err,
        "fp64_plain": {"value": value64, "unit": "rho-evals/s", "templates_timed": nsub,
                       "speedup_split_batched_over_fp64_plain": value / value64},
        "kernels_ms_per_step": {k: v[0] / k_steps for k, v in kt.items() if v[1]},
        "roofline": roof,
        "roofline_other_kernels": rooflines,
    }
    ctx.close()

    if not args.no_extra and args.workload == "large":
        result["forms"] = form_lines(args, ds, info)
        result["extra"] = extra_lines(args)
    if not args.no_cpu_baseline:
        frac = {"large": 1.0 / 24.0, "band": 0.25, "tiny": 1.0}[args.workload]
        result["cpu_baseline"] = cpu_baseline(ds, n_t, frac)
    print(json.dumps(result))


def form_lines(args, ds, info0):
    """The same 240-day band with the other forms of the statistic, each timed on the split path
    (graph capture, no autotuning) over the first --form-templates templates: the Gamma^circ
    weight (Sec. II.B), every ordered pair with auto-correlations (App. A.1-A.2), per-sample
    antenna functions (Sec. III.B.3, two spectra streams), eccentric orbits (e = 0.1, Sec. II.A.2);
    and the SFT front end (App. B) for the band's 2 x 14400 SFTs of 1440 s.  rho-evals/s, with the
    roofline of the form's dominant kernel."""
    import copy

    import numpy as np
    import torch
    import synth
    from paper_1712_06515_amd import Context, PREC_SPLIT
    n = min(args.form_templates, len(ds.templates))
    out = {}

    def run(name, dsf, tm, streams=1):
        t0 = time.perf_counter()
        with Context(dsf.sky, device=0) as ctx:
            bid = ctx.load(dsf, templates=tm)
            inf = ctx.band_info(bid)
            inf["resample_templates"] = ctx.get_option("resample_templates")
            inf["farrow_used"] = bool(ctx.get_option("farrow")) and inf["farrow_degree"] > 0
            inf["n_pairs_present"] = info0["n_pairs_present"]
            o = torch.empty((len(tm), inf["n_f"]), dtype=torch.float32, device="cuda")

            def step():
                ctx.compute_rho(bid, prec=PREC_SPLIT, out_fp64=False, outputs=[o.data_ptr()])

            ctx.set_option("graph", 1)
            sec = time_steps(step, 3, 1)
            ctx.set_option("graph", 0)
            ctx.set_option("timing", 1)
            ctx.kernel_times(reset=True)
            step()
            kt = ctx.kernel_times(reset=True)
        dom = max((k for k in kt if kt[k][1]), key=lambda k: kt[k][0])
        line = {"value": len(tm) * inf["n_f"] / sec, "unit": "rho-evals/s", "ms_per_step": 1e3 * sec,
                "templates": len(tm), "kernels_ms_per_step": {k: v[0] for k, v in kt.items() if v[1]},
                "dominant_kernel": dom}
        if dom in ("resample", "spectra", "spectra_pairs", "fused", "spectra_wide"):
            line["roofline"] = roofline(dom, kt[dom][0] / kt[dom][1], len(tm) / kt[dom][1], inf, "large_" + name,
                                        streams=streams)
        out[name] = line
        log(f"form {name}: {line['ms_per_step']:.1f} ms/step, dominant {dom} ({time.perf_counter() - t0:.0f} s)")

    tm = ds.templates[:n]
    d = copy.copy(ds)
    d.band = dict(ds.band, weight=1)
    run("gamma_circ", d, tm)
    d = copy.copy(ds)
    d.band = dict(ds.band, pairs=4)
    run("all_pairs_with_autos", d, tm)
    d = copy.copy(ds)
    tau = ds.t0 + np.arange(ds.n_seg * ds.n_k) * ds.dt
    ab = [synth.antenna_ab(tau, s_, ds.sky) for s_ in ds.sites]
    d.ar = np.stack([v[0] for v in ab])
    d.br = np.stack([v[1] for v in ab])
    del ab, tau
    run("per_sample_antenna", d, tm, streams=2)
    d.ar = d.br = None
    d = copy.copy(ds)
    d.ecc = True
    tme = np.stack([tm[:, 0], tm[:, 1], np.full(n, 0.7), np.full(n, 0.1), tm[:, 2]], axis=1)
    run("eccentric_e0.1", d, tme)

    # SFT front end: one detector's SFTs at a time (the call takes host bins and returns host samples)
    t_sft, n_out = ds.band["t_short"], ds.n_k
    kh = int(round(ds.f_het * t_sft))
    k_first = kh - n_out // 2 - 16
    z, valid = synth.make_sfts(ds.n_seg, t_sft, 1.0 / 4096.0, k_first, n_out + 32, t0=ds.t0,
                               lines=[(ds.f_het + 0.01, 1.0, 0.2)], sigma=1.0, seed=9)
    with Context(ds.sky, device=0) as ctx:
        ctx.set_option("timing", 1)
        walls = []
        for _ in range(3):
            ctx.kernel_times(reset=True)
            t0 = time.perf_counter()
            for X in range(ds.n_det):
                ctx.sft_series(z, t_sft, ds.t0, k_first, ds.f_het, n_out, sft_valid=valid)
            walls.append(time.perf_counter() - t0)
            kt = ctx.kernel_times(reset=True)
    wall = min(walls)
    k_ms = kt["sft_series"][0] / kt["sft_series"][1]
    flops = ds.n_seg * float(n_out) ** 2 * 8.0
    samples = ds.n_det * ds.n_seg * n_out
    out["sft_front_end"] = {
        "value": samples / wall, "unit": "series-samples/s (host bins in, host samples out)",
        "ms_per_band": 1e3 * wall, "sfts": ds.n_det * ds.n_seg, "n_out": n_out,
        "kernel_ms_per_detector": k_ms,
        "roofline": {"kernel": "k_sft_series", "bound": "alu", "achieved": flops / (k_ms * 1e-3) / 1e12,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": flops / (k_ms * 1e-3) / 1e12 / 78.6, "traffic": None,
                     "avg_launch_ms": k_ms, "algorithmic_flops_per_launch": flops,
                     "per_unit": "8 FP64 flop per (SFT, output sample, band bin): the direct inverse transform"}}
    log(f"form sft_front_end: {1e3 * wall:.1f} ms for {ds.n_det} detectors, kernel {k_ms:.2f} ms per detector")
    return out


def extra_lines(args):
    """The realistic band (120 days, 4096 templates, split) and the batching workload (64 bands
    x 1024 templates in one call), both with graph capture and autotuning: rho-evals/s."""
    import torch
    import synth
    from paper_1712_06515_amd import Context, PREC_SPLIT
    out = {}
    t0 = time.perf_counter()
    ds = synth.make_dataset(synth.config("band"))
    with Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds)
        info = ctx.band_info(bid)
        o = torch.empty((info["n_templates"], info["n_f"]), dtype=torch.float32, device="cuda")
        ctx.set_option("autotune", 1)
        ctx.set_option("graph", 1)
        sec = time_steps(lambda: ctx.compute_rho(bid, prec=PREC_SPLIT, out_fp64=False, outputs=[o.data_ptr()]),
                         10, 2)
        out["band"] = {"workload": WORKLOADS["band"], "value": info["n_templates"] * info["n_f"] / sec,
                       "unit": "rho-evals/s", "ms_per_step": 1e3 * sec,
                       "tuned": {"k_chunk": ctx.get_option("tuned_k_chunk"),
                                 "template_batch": ctx.get_option("tuned_template_batch"),
                                 "round_templates": ctx.get_option("tuned_round_templates"),
                                 "spectra_kernel": ctx.get_option("tuned_spectra_kernel")}}
    log(f"extra band: {out['band']['ms_per_step']:.1f} ms/step ({time.perf_counter() - t0:.0f} s)")
    t0 = time.perf_counter()
    dss = synth.make_multiband(synth.config("multiband"))
    log(f"multiband data ({time.perf_counter() - t0:.0f} s)")
    with Context(dss[0].sky, device=0) as ctx:
        ids = [ctx.load(d) for d in dss]
        infos = [ctx.band_info(b) for b in ids]
        outs = [torch.empty((i["n_templates"], i["n_f"]), dtype=torch.float32, device="cuda") for i in infos]
        ctx.set_option("autotune", 1)
        ctx.set_option("graph", 1)
        sec = time_steps(lambda: ctx.compute_rho(ids, prec=PREC_SPLIT, out_fp64=False,
                                                 outputs=[x.data_ptr() for x in outs]), 3, 1)
        n_eval = sum(i["n_templates"] * i["n_f"] for i in infos)
        out["multiband"] = {"workload": WORKLOADS["multiband"], "value": n_eval / sec, "unit": "rho-evals/s",
                            "ms_per_step": 1e3 * sec, "bands": len(ids), "rho_evals_per_step": n_eval,
                            "tuned": {"k_chunk": ctx.get_option("tuned_k_chunk"),
                                      "template_batch": ctx.get_option("tuned_template_batch"),
                                      "round_templates": ctx.get_option("tuned_round_templates"),
                                      "spectra_kernel": ctx.get_option("tuned_spectra_kernel")}}
    log(f"extra multiband: {out['multiband']['ms_per_step']:.1f} ms/step")
    return out


if __name__ == "__main__":
    main()

"""Throughput of the resampled cross-correlation hot path on one MI355X.

One step = one ccr_compute_rho over every orbital template and output bin of the workload
(time base, resampling, segment FFTs, pair sum), inputs resident in HBM, output on device.

Workload "band" (default): 2 detectors, 120 days with 30 % seeded gaps, T_short = 600 s,
0.1 Hz band at 200 Hz, 4096 orbital templates (64 a_p in [1, 2] lt-s x 64 T_asc over
+-1000 s), lag-0 cross-detector pairs, Gaussian noise + 10 injections.  The value is
rho evaluations (templates x bins) per second of the split-precision path (FP64 time base and
phases, FP32 interpolation / FFT / pair products); the plain FP64 path (one template per
launch sequence) is timed beside it on a bounded template subset.

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
# MI355X FP32 vector peak.  A probe of plain (non-packed) v_fma_f32 throughput on the chip retires
# a wave64 instruction every ~2 cycles per SIMD, i.e. 256 CU x 4 SIMD x 32 lanes x 2 flop x 2.4 GHz
# = 157.3 TFLOP/s, the published figure, without packed FP32.
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "band": "2 detectors, 120 d, 30% gaps, T_short 600 s, 0.1 Hz at 200 Hz, 4096 templates "
            "(64 a_p x 64 T_asc), lag 0 cross-detector pairs, noise + 10 injections",
    "tiny": "2 detectors, 2 d, T_short 360 s, 0.25 Hz at 100 Hz, 64 templates, same-time pairs",
    "large": "2 detectors, 240 d, T_short 1440 s, lag 4, 0.25 Hz at 400 Hz, 100200 templates",
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


def cpu_baseline(ds, seg_fraction=0.25):
    """The oracle timed on the host's cores over a bounded sample of the workload: as many
    templates as the oracle has threads (one template per thread), each over the first
    `seg_fraction` of the segments (same band, detectors, sampling, gaps and weights).  The
    oracle's cost is linear in the number of segments, so the rate is scaled to full-length
    templates: value = templates x bins / (wall x M / M_sample)."""
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
    n = min(len(ds.templates), max(1, nthreads))
    idx = rng.choice(len(ds.templates), size=n, replace=False)
    t0 = time.perf_counter()
    o.rho(ds.templates[idx])
    dt = time.perf_counter() - t0
    scale = ds.n_seg / m_sub
    return {"value": n * n_f / (dt * scale), "unit": "rho-evals/s", "cores": int(n), "kind": "oracle",
            "sample": f"{n} random templates x all {n_f} bins over the first {m_sub} of {ds.n_seg} segments "
                      f"({dt:.1f} s wall on {n} threads), rate scaled by {scale:.2f} to full-length templates"}


def roofline(name, avg_ms, tb, info, workload):
    """Roofline entry of one kernel: `tb` templates per launch, `avg_ms` mean launch time."""
    import numpy as np
    n_active = info["n_active"]
    ns = 1 << (int(info["n_k"]) - 1).bit_length()
    P = info["n_fft"] // ns
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
        # one complex64 sample written per resampled sample; the input sample is read once per
        # tile of T_b templates (the templates one workgroup resamples from one staged input
        # window)
        T_b = info["resample_templates"]
        byts = n_active * info["n_k"] * tb * (8.0 + 8.0 / T_b)
        ach = byts / (avg_ms * 1e-3) / 1e9
        return {"kernel": "k_resample_m", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": read_traffic("resample", workload),
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": byts,
                "per_unit": f"{8.0 + 8.0 / T_b:g} B per resampled sample (8 B written, 8 B input "
                            f"per tile of {T_b} templates)"}
    flops = n_active * tb * P * (5.0 * ns * np.log2(ns) + 6.0 * ns)
    per_unit = f"P (5 n_s log2 n_s + 6 n_s) FP32 flop per (template, detector, segment), n_s={ns}, P={P}"
    if name in ("spectra_pairs", "fused"):
        # the pair sum runs in the same kernel: 8 flop per (template, pair, bin)
        flops += 8.0 * info["n_pairs"] * info["n_f"] * tb
        per_unit += " + 8 flop per (template, pair, bin)"
    ach = flops / (avg_ms * 1e-3) / 1e12
    kern = {"spectra": "k_spectra16_m" if ns == 256 else "k_spectra_m", "spectra_pairs": "k_spectra_pairs_m",
            "fused": "k_fused"}[name]
    return {"kernel": kern, "bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP32_PEAK_TFLOPS, "traffic": read_traffic(name, workload),
            "avg_launch_ms": avg_ms, "algorithmic_flops_per_launch": flops, "per_unit": per_unit}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="band", choices=sorted(WORKLOADS))
    ap.add_argument("--fp64-templates", type=int, default=256,
                    help="templates timed on the plain FP64 path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--fused", type=int, default=0, help="1: fused kernel, 0: staged kernels (default)")
    ap.add_argument("--workspace-mb", type=int, default=0, help="workspace budget (0: the library default)")
    ap.add_argument("--farrow", type=int, default=None,
                    help="split-precision resampler: 1 Farrow form (library default), 0 direct tap sum")
    ap.add_argument("--max-templates", type=int, default=0,
                    help="time only the first N templates of the workload (0: all; the rate is per rho evaluation)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (orbital templates are "
              "independent, so they would shard across GPUs with no exchange but a final gather)",
              file=sys.stderr)
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

    t_gen = time.perf_counter()
    ds = synth.make_dataset(synth.config(args.workload))
    if args.max_templates and args.max_templates < len(ds.templates):
        ds.templates = ds.templates[:args.max_templates]
    print(f"[bench] dataset {args.workload}: {ds.n_det} det x {ds.n} samples, {len(ds.templates)} templates "
          f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    ctx = Context(ds.sky, device=0)
    ctx.set_option("fused", args.fused)
    if args.workspace_mb:
        ctx.set_option("workspace_mb", args.workspace_mb)
    bid = ctx.load(ds)
    info = ctx.band_info(bid)
    if args.farrow is not None:
        ctx.set_option("farrow", args.farrow)
    info["resample_templates"] = ctx.get_option("resample_templates")
    info["farrow_used"] = bool(ctx.get_option("farrow")) and info["farrow_degree"] > 0
    n_t, n_f = info["n_templates"], info["n_f"]
    out = torch.empty((n_t, n_f), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(prec=PREC_SPLIT, band=bid, o=out):
        ctx.compute_rho(band, prec=prec, out_fp64=False, outputs=[o.data_ptr()], stream=stream.cuda_stream)

    if args.profile_steps:
        for i in range(args.profile_steps):
            step()
            torch.cuda.synchronize()
            print(f"[bench] profile step {i} done", file=sys.stderr, flush=True)
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = n_t * n_f / (wall / args.steps)
    print(f"[bench] split path {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    # per-kernel device time (events on the launch stream), separate pass
    ctx.set_option("timing", 1)
    ctx.kernel_times(reset=True)
    for _ in range(args.steps):
        step()
    kt = ctx.kernel_times(reset=True)
    ctx.set_option("timing", 0)

    # plain FP64 path: one template per launch sequence, on a bounded subset
    nsub = min(args.fp64_templates, n_t)
    ctx2 = Context(ds.sky, device=0)
    ctx2.set_option("template_batch", 1)
    ctx2.set_option("items_per_launch", 1)
    ctx2.set_option("fused", 0)
    bid2 = ctx2.load(ds, templates=ds.templates[:nsub])
    out2 = torch.empty((nsub, n_f), dtype=torch.float64, device="cuda")

    def step64():
        ctx2.compute_rho(bid2, prec=PREC_FP64, out_fp64=True, outputs=[out2.data_ptr()], stream=stream.cuda_stream)

    step64()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step64()
    torch.cuda.synchronize()
    w64 = time.perf_counter() - t0
    value64 = nsub * n_f / w64
    print(f"[bench] fp64 plain {1e3 * w64:.1f} ms for {nsub} templates", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (device time per launch from HIP events on the launch
    # stream; algorithmic work per launch = per-unit figure x units per launch); the other
    # hot kernel's roofline is reported beside it
    rooflines = {}
    for kname, (ms_tot, nl) in kt.items():
        if nl == 0 or kname not in ("resample", "spectra", "spectra_pairs", "fused"):
            continue
        rooflines[kname] = roofline(kname, ms_tot / nl, n_t / max(1, nl // args.steps), info, args.workload)
    name = max((k for k in rooflines), key=lambda k: kt[k][0])
    roof = rooflines.pop(name)
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
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "templates": n_t, "bins": n_f,
                   "n_k": info["n_k"], "n_seg": info["n_seg"], "n_fft": info["n_fft"]},
        "fp64_plain": {"value": value64, "unit": "rho-evals/s", "templates_timed": nsub,
                       "speedup_split_batched_over_fp64_plain": value / value64},
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "roofline": roof,
        "roofline_other_kernels": rooflines,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(ds)
    print(json.dumps(result))


if __name__ == "__main__":
    main()

"""The no-allocation entry point (ccr_compute_rho_noalloc) against ccr_compute_rho.

Both run the same kernels; the no-allocation call keeps its tables and workspace in the
library's fixed device array and packs templates into as many launch rounds as that array
needs.  FP64 rho is bitwise reproducible for any template batching, so the two calls must
agree bitwise in FP64; split precision within 1e-6 of max(|rho|, 1).  Two calls in a row, the
second on a smaller input, and a workload whose templates need several rounds of the array.
"""

import numpy as np
import pytest

import synth
from conftest import small_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ccr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06515_amd import ccr as mod
    mod.load_library()
    return mod


def _both(ccr, ctx, bid, prec, out_fp64):
    import torch
    info = ctx.band_info(bid)
    dt = torch.float64 if out_fp64 else torch.float32
    ref = ctx.compute_rho(bid, prec=prec, out_fp64=out_fp64)
    out = torch.full((info["n_templates"], info["n_f"]), float("nan"), dtype=dt, device="cuda")
    torch.cuda.synchronize()
    ctx.compute_rho_noalloc(bid, [out.data_ptr()], prec=prec, out_fp64=out_fp64)
    ctx.sync()
    return out.cpu().numpy(), ref


def _check(got, ref, prec, ccr):
    assert np.all(np.isfinite(got))
    if prec == ccr.PREC_FP64:
        assert np.array_equal(got, ref)
    else:
        assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)) <= 1e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_two_calls_second_smaller(ccr, prec):
    big = synth.make_dataset(small_config(q=3, n_seg=24, max_lag=2, gap_fraction=0.2,
                                          injections=[dict(f0=50.21, a_p=1.25, t_asc_off=0.0, period=68023.7,
                                                           h0=0.35, cosi=0.5, psi=0.3, phi0=1.0)]),
                             sigma_wander=0.2)
    small = synth.make_dataset(small_config(q=2, n_seg=9, max_lag=1, gap_fraction=0.1, seed=19))
    out_fp64 = prec == ccr.PREC_FP64
    with ccr.Context(big.sky, device=0) as ctx:
        b1 = ctx.load(big)
        b2 = ctx.load(small, templates=small.templates[:3])
        for bid, name in ((b1, "first"), (b2, "second, smaller")):
            print(f"no-alloc {name} call, precision {prec}", flush=True)
            got, ref = _both(ccr, ctx, bid, prec, out_fp64)
            _check(got, ref, prec, ccr)
        # both bands in one call
        import torch
        outs = [torch.full((ctx.band_info(b)["n_templates"], ctx.band_info(b)["n_f"]), float("nan"),
                           dtype=torch.float64 if out_fp64 else torch.float32, device="cuda") for b in (b1, b2)]
        ctx.compute_rho_noalloc([b1, b2], [o.data_ptr() for o in outs], prec=prec, out_fp64=out_fp64)
        ctx.sync()
        refs = ctx.compute_rho([b1, b2], prec=prec, out_fp64=out_fp64)
        for o, r in zip(outs, refs):
            _check(o.cpu().numpy(), r, prec, ccr)


def test_noalloc_several_rounds(ccr):
    """40 templates of the 120-day band: ~50 MB of resampled series per template in split
    precision and ~100 MB in FP64, so the fixed array holds a few templates per round."""
    ds = synth.make_dataset(synth.config("band"))
    with ccr.Context(ds.sky, device=0) as ctx:
        bid = ctx.load(ds, templates=ds.templates[:40])
        for prec in (ccr.PREC_FP64, ccr.PREC_SPLIT):
            print(f"no-alloc band workload, precision {prec}", flush=True)
            got, ref = _both(ccr, ctx, bid, prec, prec == ccr.PREC_FP64)
            _check(got, ref, prec, ccr)


def test_noalloc_rejects_unprepared_band(ccr):
    import torch
    ds = synth.make_dataset(small_config(n_seg=6))
    with ccr.Context(ds.sky, device=0) as ctx:
        bid, _ = ctx.add_band(ds.band)
        for X in range(ds.x.shape[0]):
            ctx.set_data(bid, X, ds.sites[X], ds.t0, ds.dt, ds.x[X], ds.f_het, ds.valid[X])
            ctx.set_weights(bid, X, ds.a[X], ds.b[X], ds.noise_var[X])
        ctx.set_templates(bid, ds.templates)
        out = torch.zeros((len(ds.templates), 4096), dtype=torch.float64, device="cuda")
        with pytest.raises(ccr.CcrError) as e:
            ctx.compute_rho_noalloc(bid, [out.data_ptr()])
        assert e.value.status == ccr.ESTATE
        ctx.band_info(bid)  # prepares the band
        info = ctx.band_info(bid)
        out = torch.zeros((info["n_templates"], info["n_f"]), dtype=torch.float64, device="cuda")
        ctx.compute_rho_noalloc(bid, [out.data_ptr()])
        ctx.sync()
        assert np.array_equal(out.cpu().numpy(), ctx.compute_rho(bid, prec=ccr.PREC_FP64))

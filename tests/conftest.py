import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def small_config(q=2, n_seg=16, t_short=120.0, f_min=50.0, f_band=0.4, max_lag=1, pairs=3,
                 gap_fraction=0.0, window=0, dirichlet_D=8, n_fft_override=0, mu_f=0.1,
                 a_p_max=1.5, seed=7, injections=None, sigma=None, t_asc0=5000.0,
                 templates=None, coverage=None):
    """A small workload for oracle and parity tests (several FFT tiles, ragged tails)."""
    dets = ["H", "L", "V"][:q] if q <= 3 else ["H", "L", "V"] + ["H"] * (q - 3)
    return dict(
        detectors=dets,
        t_obs=n_seg * t_short,
        gap_fraction=gap_fraction,
        coverage=coverage,
        sigma=sigma or [1.0 + 0.2 * X for X in range(q)],
        band=dict(f_min=f_min, f_band=f_band, t_short=t_short, max_lag=max_lag, dirichlet_D=dirichlet_D,
                  window=window, mu_f=mu_f, n_fft_override=n_fft_override, pairs=pairs, a_p_max=a_p_max),
        templates=templates or dict(a_p=(1.0, 1.5, 3), t_asc=(-200.0, 200.0, 2), period=[68023.70]),
        t_asc0=t_asc0,
        injections=injections or [],
        seed=seed,
    )


@pytest.fixture
def small_cfg():
    return small_config

"""Workload definitions.

Shapes follow the five workloads the method is measured on; physical values
follow Table I (Sco X-1 position, orbital period, a_p range).  Quantities the
workload descriptions leave open are fixed here:

* mismatch mu_f = 0.1 (Sec. III.B.2 worked value), Dirichlet D = 8 (Sec. III.A.1);
* "same-time pairs only" / "pairs within lag 0" mean max lag R = 0;
* a_p_max (sizes the Doppler wings of the load band) is the top of the a_p grid;
* T_asc grids are centred on ``t_asc0`` (seconds after the epoch) and P = 68023.70 s.
"""

P0 = 68023.70
DAY = 86400.0

CONFIGS = {
    # Plain method, tiny: 2 detectors, 2 days, no gaps, T_short 360 s, 0.25 Hz band at 100 Hz,
    # one circular-orbit injection, 8 x 8 templates, same-time pairs only.
    "tiny": dict(
        detectors=["H", "L"],
        t_obs=2 * DAY,
        gap_fraction=0.0,
        coverage=None,
        sigma=[1.0, 1.25],
        band=dict(f_min=99.875, f_band=0.25, t_short=360.0, max_lag=0, dirichlet_D=8,
                  window=0, mu_f=0.1, n_fft_override=0, pairs=3, a_p_max=1.5),
        templates=dict(a_p=(1.40, 1.50, 8), t_asc=(-300.0, 300.0, 8), period=[P0]),
        t_asc0=86400.0 + 1234.5,
        injections=[dict(f0=100.05, a_p=1.45, t_asc_off=37.0, period=P0, h0=0.165,
                         cosi=1.0, psi=0.0, phi0=0.4)],
        seed=1001,
    ),
    # Plain method, realistic band: 120 days, 30 % gaps, T_short 600 s, 0.1 Hz at 200 Hz,
    # 64 x 64 templates, lag 0 cross-detector pairs, 10 injections.
    "band": dict(
        detectors=["H", "L"],
        t_obs=120 * DAY,
        gap_fraction=0.30,
        coverage=None,
        sigma=[1.0, 1.15],
        band=dict(f_min=199.95, f_band=0.1, t_short=600.0, max_lag=0, dirichlet_D=8,
                  window=0, mu_f=0.1, n_fft_override=0, pairs=3, a_p_max=2.0),
        templates=dict(a_p=(1.0, 2.0, 64), t_asc=(-1000.0, 1000.0, 64), period=[P0]),
        t_asc0=60 * DAY + 777.0,
        injections="random10",
        seed=2002,
    ),
    # Batching form: 3 detectors with uneven coverage (100 / 120 / 80 days of a 120-day span,
    # independent gap times), 64 bands between 50 and 400 Hz of 0.05-0.2 Hz, T_short from 1400 s
    # (50 Hz) to 240 s (400 Hz), lag 1, 32 x 32 templates per band, an injection in every
    # fourth band.  Built by make_multiband (one dataset per band).
    "multiband": dict(
        detectors=["H", "L", "V"],
        t_obs=120 * DAY,
        gap_fraction=0.15,
        coverage=[(0.0, 100.0 / 120.0), (0.0, 1.0), (20.0 / 120.0, 80.0 / 120.0)],
        sigma=[1.0, 1.1, 1.3],
        bands=dict(count=64, f_lo=50.0, f_hi=400.0, f_band=[0.05, 0.10, 0.15, 0.20],
                   t_short_lo=1400.0, t_short_hi=240.0, max_lag=1, pairs=3, a_p_max=2.0),
        templates=dict(a_p=(1.0, 2.0, 32), t_asc=(-1000.0, 1000.0, 32), period=[P0]),
        t_asc0=60 * DAY + 555.0,
        inject_every=4,
        seed=4004,
        name="multiband",
    ),
    # Largest: 240 days, T_short 1440 s, lag 4, 0.25 Hz at 400 Hz, 200 x 167 x 3 templates.
    "large": dict(
        detectors=["H", "L"],
        t_obs=240 * DAY,
        gap_fraction=0.0,
        coverage=None,
        sigma=[1.0, 1.1],
        band=dict(f_min=399.875, f_band=0.25, t_short=1440.0, max_lag=4, dirichlet_D=8,
                  window=0, mu_f=0.1, n_fft_override=0, pairs=3, a_p_max=2.0),
        templates=dict(a_p=(1.0, 2.0, 200), t_asc=(-1000.0, 1000.0, 167),
                       period=[P0 - 0.04, P0, P0 + 0.04]),
        t_asc0=120 * DAY + 321.0,
        injections="random100",
        seed=5005,
    ),
}


def config(name, **over):
    """A copy of a named workload with top-level or band fields overridden."""
    import copy
    c = copy.deepcopy(CONFIGS[name])
    band_over = over.pop("band", None)
    c.update(over)
    if band_over:
        c["band"].update(band_over)
    return c

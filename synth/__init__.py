"""Seeded synthetic inputs for the resampled cross-correlation hot path.

This module is shared by the tests, the benchmark and the oracle's tests.  It
holds no step of the rho computation itself (no inverse time map, no
interpolation, no DFT, no pair sum).  What it does:

* forward signal synthesis: a circular-orbit continuous wave seen at a ground
  detector, built from the signal model of Sec. II.A (strain with beam-pattern
  functions F+, Fx and amplitudes A+, Ax; phase from the forward time map
  t -> t_SSB -> tau of eqs. t-ssb-equation and tau-equation, circular case),
  heterodyned by f_h as the complex series the method starts from (Sec. III,
  App. B);
* circular complex Gaussian noise, exponential-length data gaps and uneven
  detector coverage (Sec. III.B: gaps are zero-filled);
* per-segment antenna values a_K, b_K (mid-segment) and noise variances;
* orbital template grids;
* short Fourier transforms of sampled real sinusoids plus white noise, in closed form (the input
  of the SFT front end, App. B).

The sample interval of the heterodyned series comes from the load bandwidth of
App. B (eq. delta-f-load), rounded so that T_short holds an integer number of
samples.  Every array is produced from numpy PCG64 generators seeded from the
configuration.
"""

from .model import (  # noqa: F401
    SPEED_OF_LIGHT, default_sky, site, SITES, earth_roemer, forward_delay, forward_delay_ecc, kepler_E,
    antenna_ab, load_bandwidth, samples_per_segment,
)
from .configs import CONFIGS, config  # noqa: F401
from .generate import Dataset, make_dataset, make_multiband, multiband_bands, template_grid  # noqa: F401
from .sft import make_sfts  # noqa: F401

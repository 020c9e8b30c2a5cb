"""Seeded synthetic short Fourier transforms (SFTs): the bins a data file of SFTs would hold for a
band, computed in closed form for real sinusoids sampled at a high rate, plus white noise.

SFT K covers the samples t0 + K T_sft + j dt, j < N = T_sft / dt, and holds
z_{K,k} = dt sum_j x_j exp(-2 pi i j k / N) for k = k_first .. k_first + n_bins - 1.  For
x = A cos(2 pi f0 t + phi) each of the two exponentials is a geometric series in j, summed exactly
here; white noise of variance sigma^2 per sample gives independent complex Gaussian bins of
variance N dt^2 sigma^2.  This module holds no arithmetic of the method: it makes inputs.
"""

import numpy as np


def _geom(alpha, n):
    """sum_{j<n} exp(2 pi i alpha j) for an array of alpha (n at integer alpha)."""
    a = np.asarray(alpha, dtype=np.float64)
    frac = a - np.round(a)
    out = np.empty(a.shape, dtype=np.complex128)
    on = np.abs(frac) < 1e-15
    out[on] = n
    f = frac[~on]
    num = 1.0 - np.exp(2j * np.pi * f * n)
    den = 1.0 - np.exp(2j * np.pi * f)
    out[~on] = num / den
    return out


def make_sfts(n_sft, t_sft, dt, k_first, n_bins, t0=0.0, lines=(), sigma=0.0, seed=0, valid_fraction=1.0):
    """SFT bins (n_sft x n_bins complex128) and a per-SFT valid flag (uint8).

    lines: (f0, amplitude, phase) of real sinusoids A cos(2 pi f0 t + phi), t in seconds after the
    epoch; sigma: white-noise standard deviation per time sample; SFTs are dropped (flag 0, bins
    zero) at random with probability 1 - valid_fraction."""
    n = int(round(t_sft / dt))
    if abs(n * dt - t_sft) > 1e-9 * t_sft:
        raise ValueError("t_sft must be a whole number of samples")
    rng = np.random.default_rng(seed)
    k = k_first + np.arange(n_bins)
    z = np.zeros((n_sft, n_bins), dtype=np.complex128)
    tk = (np.longdouble(t0) + np.arange(n_sft, dtype=np.longdouble) * np.longdouble(t_sft))
    for f0, amp, ph in lines:
        cyc = np.longdouble(f0) * tk
        cyc = np.asarray(cyc - np.floor(cyc), dtype=np.float64)  # f0 t_K mod 1
        theta = 2.0 * np.pi * cyc + ph
        gp = _geom(f0 * dt - k / n, n)
        gm = _geom(-f0 * dt - k / n, n)
        z += 0.5 * amp * dt * (np.exp(1j * theta)[:, None] * gp[None, :] + np.exp(-1j * theta)[:, None] * gm[None, :])
    if sigma > 0:
        s = sigma * dt * np.sqrt(n / 2.0)
        z += s * (rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape))
    valid = (rng.random(n_sft) < valid_fraction).astype(np.uint8)
    z[valid == 0] = 0.0
    return z, valid

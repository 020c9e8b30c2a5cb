"""Forward physical model used to synthesise detector data (numpy, float64).

Conventions (all times in seconds relative to a common epoch, angles in
radians):

* source direction n(alpha, delta) = (cos a cos d, sin a cos d, sin d)
  (Sec. II.A.2);
* Earth: circular orbit of radius ``au_s`` light-seconds in the ecliptic,
  ecliptic longitude ``orbit_phase0 + 2 pi t / year_s``, ecliptic tilted by
  ``obliquity`` about the equatorial x axis; rotation with sidereal angle
  ``gmst0 + 2 pi t / sidereal_day_s``; detectors on a sphere of radius ``re_s``
  light-seconds;
* SSB arrival time t_SSB = t + r(t).n  (eq. t-ssb-equation, Roemer term only);
* binary Roemer delay, circular orbit: tau = t_SSB - a_p sin(Omega (t_SSB -
  T_asc)), Omega = 2 pi / P  (eq. tau-equation with the circular R/c; the
  orbital phase is taken at t_SSB because T_asc is an SSB time).
"""

import math

import numpy as np

SPEED_OF_LIGHT = 299792458.0


def default_sky(**over):
    """Sco X-1 position (Table I) and the analytic Earth model parameters."""
    ra = (16.0 + 19.0 / 60.0 + 55.067 / 3600.0) * 15.0 * math.pi / 180.0
    dec = -(15.0 + 38.0 / 60.0 + 25.02 / 3600.0) * math.pi / 180.0
    sky = dict(
        ra=ra,
        dec=dec,
        au_s=499.004784,
        re_s=6.371e6 / SPEED_OF_LIGHT,
        obliquity=23.4393 * math.pi / 180.0,
        year_s=365.25636 * 86400.0,
        sidereal_day_s=86164.0905,
        orbit_phase0=0.7,
        gmst0=1.3,
    )
    sky.update(over)
    return sky


def site(lat_deg, lon_deg, xarm_az_deg, yarm_az_deg):
    """A detector site: geodetic-free spherical latitude/longitude and the
    azimuths (clockwise from North) of its two arms."""
    d = math.pi / 180.0
    return dict(lat=lat_deg * d, lon=lon_deg * d,
                xaz=xarm_az_deg * d, yaz=yarm_az_deg * d)


# Approximate sites; any fixed values serve, they are part of each config.
SITES = {
    "H": site(46.455, -119.408, 324.0, 234.0),
    "L": site(30.563, -90.774, 252.3, 162.3),
    "V": site(43.631, 10.504, 70.6, 340.6),
}


def _source_unit(sky):
    a, d = sky["ra"], sky["dec"]
    return np.array([math.cos(a) * math.cos(d), math.sin(a) * math.cos(d), math.sin(d)])


def _earth_position(t, s, sky):
    """Detector position r(t) in light-seconds, equatorial SSB frame, shape (3, n)."""
    t = np.asarray(t, dtype=np.float64)
    lam = sky["orbit_phase0"] + 2.0 * math.pi * t / sky["year_s"]
    eps = sky["obliquity"]
    au = sky["au_s"]
    xo = au * np.cos(lam)
    yo = au * np.sin(lam) * math.cos(eps)
    zo = au * np.sin(lam) * math.sin(eps)
    g = sky["gmst0"] + 2.0 * math.pi * t / sky["sidereal_day_s"] + s["lon"]
    re = sky["re_s"]
    cl = math.cos(s["lat"])
    xr = re * cl * np.cos(g)
    yr = re * cl * np.sin(g)
    zr = re * math.sin(s["lat"]) * np.ones_like(t)
    return np.stack([xo + xr, yo + yr, zo + zr])


def earth_roemer(t, s, sky):
    """r(t).n / c in seconds (the Earth part of t_SSB - t)."""
    n = _source_unit(sky)
    r = _earth_position(t, s, sky)
    return n[0] * r[0] + n[1] * r[1] + n[2] * r[2]


def forward_delay(t, s, sky, a_p, t_asc, period, e=None):
    """tau(t) - t for detector time t (forward map, explicit, no solve).  ``e`` may pass in
    earth_roemer(t, s, sky) when it is already at hand (several injections on one lattice)."""
    if e is None:
        e = earth_roemer(t, s, sky)
    t_ssb_minus_t = e
    omega = 2.0 * math.pi / period
    # Omega (t_SSB - T_asc) evaluated as Omega (t - T_asc) + Omega e; t is at
    # most a few 1e7 s so the angle keeps ~1e-12 rad, ample for synthesis.
    ang = omega * (np.asarray(t, dtype=np.float64) - t_asc) + omega * e
    return t_ssb_minus_t - a_p * np.sin(ang)


def kepler_E(M, ecc, iters=40):
    """Eccentric anomaly for mean anomaly M (array) and eccentricity ecc: E - ecc sin E = M,
    Newton iterations from E = M + ecc sin M (vectorised, float64)."""
    M = np.asarray(M, dtype=np.float64)
    E = M + ecc * np.sin(M)
    for _ in range(iters):
        E = E - (E - ecc * np.sin(E) - M) / (1.0 - ecc * np.cos(E))
    return E


def forward_delay_ecc(t, s, sky, a_p, t_p, omega_p, ecc, period, e=None):
    """tau(t) - t for an eccentric binary orbit (forward map, explicit): t_SSB = t + r.n,
    mean anomaly Omega (t_SSB - T_p) = E - ecc sin E, R/c = a_p [sin w (cos E - ecc) +
    cos w sqrt(1 - ecc^2) sin E] (eqs. solve-for-E, Kepler-equation), tau = t_SSB - R/c."""
    if e is None:
        e = earth_roemer(t, s, sky)
    omega = 2.0 * math.pi / period
    M = omega * (np.asarray(t, dtype=np.float64) - t_p) + omega * e
    M = np.mod(M, 2.0 * math.pi)
    E = kepler_E(M, ecc)
    R = a_p * (math.sin(omega_p) * (np.cos(E) - ecc) + math.cos(omega_p) * math.sqrt(1.0 - ecc * ecc) * np.sin(E))
    return e - R


def antenna_ab(t, s, sky):
    """Beam-pattern functions a(t) = F+(psi=0), b(t) = Fx(psi=0).

    Built from the detector tensor d = (u u^T - v v^T)/2 of unit arm vectors
    and the polarisation tensors e+ = p p^T - q q^T, ex = p q^T + q p^T of an
    orthonormal pair (p, q) transverse to the source direction, so that
    F+ = a cos 2psi + b sin 2psi and Fx = b cos 2psi - a sin 2psi.
    """
    t = np.asarray(t, dtype=np.float64)
    lat, lon = s["lat"], s["lon"]
    up = np.array([math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])
    east = np.array([-math.sin(lon), math.cos(lon), 0.0])
    north = np.cross(up, east)
    u0 = math.cos(s["xaz"]) * north + math.sin(s["xaz"]) * east
    v0 = math.cos(s["yaz"]) * north + math.sin(s["yaz"]) * east
    g = sky["gmst0"] + 2.0 * math.pi * t / sky["sidereal_day_s"]
    cg, sg = np.cos(g), np.sin(g)

    def rot(w):
        return np.stack([cg * w[0] - sg * w[1], sg * w[0] + cg * w[1], np.full_like(t, w[2])])

    u, v = rot(u0), rot(v0)
    a_, d_ = sky["ra"], sky["dec"]
    p = np.array([-math.sin(a_), math.cos(a_), 0.0])
    q = np.array([-math.cos(a_) * math.sin(d_), -math.sin(a_) * math.sin(d_), math.cos(d_)])
    up_ = p[0] * u[0] + p[1] * u[1] + p[2] * u[2]
    uq_ = q[0] * u[0] + q[1] * u[1] + q[2] * u[2]
    vp_ = p[0] * v[0] + p[1] * v[1] + p[2] * v[2]
    vq_ = q[0] * v[0] + q[1] * v[1] + q[2] * v[2]
    # d:e+ = 1/2[(u.p)^2 - (u.q)^2 - (v.p)^2 + (v.q)^2]; d:ex = (u.p)(u.q) - (v.p)(v.q)
    a = 0.5 * (up_ ** 2 - uq_ ** 2 - vp_ ** 2 + vq_ ** 2)
    b = up_ * uq_ - vp_ * vq_
    return a, b


def load_bandwidth(f_min, f_band, t_short, a_p_max, dirichlet_D=8, v_over_c=1e-4,
                   period=68023.70):
    """Load bandwidth of App. B, eq. delta-f-load, with T_sft read as T_short and
    the drift width of eqs. f-drift-eq / delta-f-obs taken at the top of the band:
    df_drift = 2 (f_top v/c + a_p_max Omega f_top)."""
    f_top = f_min + f_band
    drift = 2.0 * (f_top * v_over_c + a_p_max * (2.0 * math.pi / period) * f_top)
    return (1.0 + 4.0 / (2.0 * dirichlet_D + 1.0)) * (f_band + drift + 16.0 / t_short)


def samples_per_segment(band):
    """N_K = ceil(T_short * df_load); the series is sampled at dt = T_short / N_K."""
    dfl = load_bandwidth(band["f_min"], band["f_band"], band["t_short"], band["a_p_max"],
                         band.get("dirichlet_D", 8))
    return int(math.ceil(band["t_short"] * dfl))

"""Python access to the C oracle (test infrastructure).

THIS IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  The product library never
loads it and shares no code with it.

``build()`` compiles ``ccr_oracle.c`` with gcc (OpenMP, IEEE double/long double,
no fast-math) into ``oracle/libccr_oracle.so``.
"""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ccr_oracle.c")
LIB = os.path.join(HERE, "libccr_oracle.so")
MAX_DET = 8

_lib = None


def build(extra_flags=(), out=LIB, quiet=True):
    """Compile the oracle; returns the path of the shared object."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-Wall", "-Wno-unknown-pragmas", *extra_flags, SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(out + ".tmp", out)
    return out


class Sky(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("ra", "dec", "au_s", "re_s", "obliquity", "year_s", "sidereal_day_s",
                 "orbit_phase0", "gmst0")]


class Band(ctypes.Structure):
    _fields_ = [("f_min", ctypes.c_double), ("f_band", ctypes.c_double), ("t_short", ctypes.c_double),
                ("max_lag", ctypes.c_int), ("dirichlet_D", ctypes.c_int), ("window", ctypes.c_int),
                ("n_fft_override", ctypes.c_int), ("mu_f", ctypes.c_double), ("pairs", ctypes.c_int),
                ("a_p_max", ctypes.c_double), ("orbit_period", ctypes.c_double), ("weight", ctypes.c_int)]


class Plan(ctypes.Structure):
    _fields_ = [("n_k", ctypes.c_int64), ("n_seg", ctypes.c_int64), ("n_fft", ctypes.c_int64),
                ("n_f", ctypes.c_int64), ("k_lo", ctypes.c_int64),
                ("dt", ctypes.c_double), ("f_het", ctypes.c_double), ("df_load", ctypes.c_double),
                ("t_coh", ctypes.c_double), ("dlambda_f", ctypes.c_double), ("t_fft", ctypes.c_double),
                ("nu_r", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class Problem(ctypes.Structure):
    _fields_ = [("sky", Sky), ("band", Band), ("n_det", ctypes.c_int),
                ("lat", ctypes.c_double * MAX_DET), ("lon", ctypes.c_double * MAX_DET),
                ("t0", ctypes.c_double), ("dt", ctypes.c_double), ("n", ctypes.c_int64),
                ("f_het", ctypes.c_double),
                ("x", ctypes.c_void_p * MAX_DET), ("valid", ctypes.c_void_p * MAX_DET),
                ("a", ctypes.c_void_p * MAX_DET), ("b", ctypes.c_void_p * MAX_DET),
                ("noise_var", ctypes.c_void_p * MAX_DET),
                ("ar", ctypes.c_void_p * MAX_DET), ("br", ctypes.c_void_p * MAX_DET),
                ("ecc", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.cco_plan_band.argtypes = [P, ctypes.POINTER(Plan)]
        L.cco_bin_index.argtypes = [ctypes.POINTER(Plan), ctypes.c_int64]
        L.cco_bin_index.restype = ctypes.c_int64
        L.cco_earth_delay.argtypes = [P, ctypes.c_int, ctypes.c_double]
        L.cco_earth_delay.restype = ctypes.c_double
        L.cco_forward_offset.argtypes = [P, ctypes.c_int, dp, ctypes.c_double]
        L.cco_forward_offset.restype = ctypes.c_double
        L.cco_delay.argtypes = [P, ctypes.c_int, dp, ctypes.c_int64, dp, dp]
        L.cco_resample.argtypes = [P, ctypes.c_int, dp, dp, i64p, dp, ctypes.c_void_p]
        L.cco_valid_fraction.argtypes = [P, dp]
        L.cco_spectra.argtypes = [P, dp, ctypes.c_int, i64p, ctypes.c_int64, dp]
        L.cco_norm.argtypes = [P]
        L.cco_norm.restype = ctypes.c_double
        L.cco_pair_count.argtypes = [P]
        L.cco_pair_count.restype = ctypes.c_int64
        L.cco_rho.argtypes = [P, dp, ctypes.c_int64, ctypes.c_int, i64p, ctypes.c_int64, dp]
        L.cco_num_threads.restype = ctypes.c_int
        L.cco_kepler.argtypes = [ctypes.c_double, ctypes.c_double]
        L.cco_kepler.restype = ctypes.c_double
        L.cco_sft_series.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                     dp, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64p(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


class Oracle:
    """Wraps one problem (data, weights, band) for repeated oracle calls.

    ``ds`` is a ``synth.Dataset``-like object with fields sky, band, sites, dt,
    t0, n, f_het, x, valid, a, b, noise_var, and optionally ar, br (per-sample antenna
    functions on the source lattice, [n_det][n_seg * n_k]) and ecc (templates of 5 values:
    a_p, T_p, omega, e, P).  Arrays are kept alive here."""

    def __init__(self, ds):
        self._keep = []
        p = Problem()
        s = ds.sky
        p.sky = Sky(s["ra"], s["dec"], s["au_s"], s["re_s"], s["obliquity"], s["year_s"],
                    s["sidereal_day_s"], s["orbit_phase0"], s["gmst0"])
        b = ds.band
        p.band = Band(b["f_min"], b["f_band"], b["t_short"], int(b["max_lag"]), int(b.get("dirichlet_D", 8)),
                      int(b.get("window", 0)), int(b.get("n_fft_override", 0)), float(b.get("mu_f", 0.1)),
                      int(b.get("pairs", 3)), float(b.get("a_p_max", 0.0)),
                      float(b.get("orbit_period", 68023.70)), int(b.get("weight", 0)))
        q = ds.x.shape[0]
        p.n_det = q
        for X in range(q):
            p.lat[X] = ds.sites[X]["lat"]
            p.lon[X] = ds.sites[X]["lon"]
            xf = np.ascontiguousarray(ds.x[X]).view(np.float32)
            vv = np.ascontiguousarray(ds.valid[X], dtype=np.uint8) if ds.valid is not None else None
            aa = np.ascontiguousarray(ds.a[X], dtype=np.float64)
            bb = np.ascontiguousarray(ds.b[X], dtype=np.float64)
            nv = np.ascontiguousarray(ds.noise_var[X], dtype=np.float64)
            self._keep += [xf, vv, aa, bb, nv]
            p.x[X] = xf.ctypes.data
            p.valid[X] = vv.ctypes.data if vv is not None else None
            p.a[X] = aa.ctypes.data
            p.b[X] = bb.ctypes.data
            p.noise_var[X] = nv.ctypes.data
            ar = getattr(ds, "ar", None)
            br = getattr(ds, "br", None)
            if ar is not None and br is not None:
                arr = np.ascontiguousarray(ar[X], dtype=np.float64)
                brr = np.ascontiguousarray(br[X], dtype=np.float64)
                self._keep += [arr, brr]
                p.ar[X] = arr.ctypes.data
                p.br[X] = brr.ctypes.data
        p.ecc = 1 if getattr(ds, "ecc", False) else 0
        p.t0 = ds.t0
        p.dt = ds.dt
        p.n = ds.x.shape[1]
        p.f_het = ds.f_het
        self.p = p
        self.n_det = q

    @property
    def _pp(self):
        return ctypes.byref(self.p)

    def plan(self):
        pl = Plan()
        _check(lib().cco_plan_band(self._pp, ctypes.byref(pl)), "plan")
        return pl

    def bins(self):
        pl = self.plan()
        return np.array([lib().cco_bin_index(ctypes.byref(pl), i) for i in range(pl.n_f)], dtype=np.int64)

    def frequencies(self):
        pl = self.plan()
        return pl.f_het + self.bins() / pl.t_fft

    def earth_delay(self, det, t):
        return np.array([lib().cco_earth_delay(self._pp, det, float(tt)) for tt in np.atleast_1d(t)])

    def forward_offset(self, det, tmpl, t):
        tm = np.ascontiguousarray(tmpl, dtype=np.float64)
        return np.array([lib().cco_forward_offset(self._pp, det, _dp(tm), float(tt)) for tt in np.atleast_1d(t)])

    def delay(self, det, tmpl, r):
        tm = np.ascontiguousarray(tmpl, dtype=np.float64)
        hi, lo = ctypes.c_double(), ctypes.c_double()
        _check(lib().cco_delay(self._pp, det, _dp(tm), int(r), ctypes.byref(hi), ctypes.byref(lo)), "delay")
        return hi.value, lo.value

    def resample(self, det, tmpl):
        pl = self.plan()
        nr = pl.n_seg * pl.n_k
        y = np.zeros(2 * nr)
        js = np.zeros(nr, dtype=np.int64)
        off = np.zeros(nr)
        m = np.zeros(nr, dtype=np.uint8)
        tm = np.ascontiguousarray(tmpl, dtype=np.float64)
        _check(lib().cco_resample(self._pp, det, _dp(tm), _dp(y), _i64p(js), _dp(off), m.ctypes.data),
               "resample")
        return y.view(np.complex128), js, off, m

    def valid_fraction(self):
        pl = self.plan()
        phi = np.zeros((self.n_det, pl.n_seg))
        _check(lib().cco_valid_fraction(self._pp, _dp(phi)), "valid_fraction")
        return phi

    def spectra(self, tmpl, tier=0, bins=None):
        pl = self.plan()
        b = None if bins is None else np.ascontiguousarray(bins, dtype=np.int64)
        nb = pl.n_f if b is None else len(b)
        F = np.zeros(2 * self.n_det * pl.n_seg * nb)
        tm = np.ascontiguousarray(tmpl, dtype=np.float64)
        _check(lib().cco_spectra(self._pp, _dp(tm), int(tier), _i64p(b), nb, _dp(F)), "spectra")
        return F.view(np.complex128).reshape(self.n_det, pl.n_seg, nb)

    def norm(self):
        return lib().cco_norm(self._pp)

    def pair_count(self):
        return lib().cco_pair_count(self._pp)

    def rho(self, templates, tier=0, bins=None):
        pl = self.plan()
        tm = np.ascontiguousarray(np.atleast_2d(templates), dtype=np.float64)
        b = None if bins is None else np.ascontiguousarray(bins, dtype=np.int64)
        nb = pl.n_f if b is None else len(b)
        out = np.zeros((tm.shape[0], nb))
        _check(lib().cco_rho(self._pp, _dp(tm), tm.shape[0], int(tier), _i64p(b), nb, _dp(out)), "rho")
        return out


def num_threads():
    return lib().cco_num_threads()


def kepler(M, e):
    """Eccentric anomaly E with E - e sin E = M (the oracle's long-double Newton solve)."""
    return lib().cco_kepler(float(M), float(e))


def sft_series(z, t_sft, t0, k_first, f_het, n_out, sft_valid=None):
    """Heterodyned, downsampled series (n_sft * n_out complex128) from SFT bins z (n_sft x n_bins
    complex, first bin k_first) by the steps of App. B."""
    zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    n_sft, n_bins = zz.shape
    zv = zz.view(np.float64).reshape(-1)
    out = np.zeros(2 * n_sft * n_out)
    vv = None if sft_valid is None else np.ascontiguousarray(sft_valid, dtype=np.uint8)
    _check(lib().cco_sft_series(n_sft, float(t_sft), float(t0), n_bins, int(k_first), _dp(zv),
                                None if vv is None else vv.ctypes.data, float(f_het), int(n_out), _dp(out)),
           "sft_series")
    return out.view(np.complex128)

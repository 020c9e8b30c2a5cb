"""Python binding of the C ABI in include/ccr.h (argument marshalling only).

Every computation runs in libccr.so (host planner + gfx950 kernels).  There is no
fallback: if the library is not built, importing this module raises.
"""

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libccr.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ERANGE, EUNSUP = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_SPLIT = 0, 1
PAIRS_CROSS, PAIRS_SAME, PAIRS_ALL = 1, 2, 4
WEIGHT_AVE, WEIGHT_CIRC = 0, 1
MAX_DET = 8
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "ERANGE", -6: "EUNSUP"}


class CcrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Sky(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("ra", "dec", "au_s", "re_s", "obliquity", "year_s", "sidereal_day_s",
                 "orbit_phase0", "gmst0")]


class Site(ctypes.Structure):
    _fields_ = [("lat", ctypes.c_double), ("lon", ctypes.c_double)]


class Band(ctypes.Structure):
    _fields_ = [("f_min", ctypes.c_double), ("f_band", ctypes.c_double), ("t_short", ctypes.c_double),
                ("max_lag", ctypes.c_int32), ("dirichlet_D", ctypes.c_int32), ("window", ctypes.c_int32),
                ("n_fft_override", ctypes.c_int32), ("mu_f", ctypes.c_double), ("pairs", ctypes.c_int32),
                ("a_p_max", ctypes.c_double), ("orbit_period", ctypes.c_double), ("weight", ctypes.c_int32)]


class BandInfo(ctypes.Structure):
    _fields_ = [("n_k", ctypes.c_int64), ("n_seg", ctypes.c_int64), ("n_fft", ctypes.c_int64),
                ("n_f", ctypes.c_int64), ("k_lo", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_det", ctypes.c_int64), ("n_templates", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("dt", ctypes.c_double), ("f_het", ctypes.c_double), ("df_load", ctypes.c_double),
                ("t_coh", ctypes.c_double), ("dlambda_f", ctypes.c_double), ("t_fft", ctypes.c_double),
                ("nu_r", ctypes.c_double), ("norm", ctypes.c_double), ("farrow_degree", ctypes.c_int64),
                ("farrow_err", ctypes.c_double), ("n_s", ctypes.c_int64), ("P", ctypes.c_int64)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


# Exported symbols and their C signatures (must match include/ccr.h).
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "ccr_abi_version": ([], ctypes.c_int),
    "ccr_create": ([ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(Sky)], ctypes.c_int),
    "ccr_destroy": ([_vp], None),
    "ccr_last_error": ([_vp], ctypes.c_char_p),
    "ccr_set_option": ([_vp, ctypes.c_char_p, ctypes.c_int64], ctypes.c_int),
    "ccr_get_option": ([_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ccr_add_band": ([_vp, ctypes.POINTER(Band), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(BandInfo)], ctypes.c_int),
    "ccr_set_data": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Site), ctypes.c_double, ctypes.c_double,
                      ctypes.c_int64, ctypes.c_double, _vp, _vp], ctypes.c_int),
    "ccr_set_weights": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp], ctypes.c_int),
    "ccr_set_antenna": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, _dp], ctypes.c_int),
    "ccr_set_templates": ([_vp, ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp], ctypes.c_int),
    "ccr_set_templates_ecc": ([_vp, ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "ccr_get_band_info": ([_vp, ctypes.c_int, ctypes.POINTER(BandInfo), _dp], ctypes.c_int),
    "ccr_compute_rho": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp),
                         ctypes.c_int, ctypes.c_int, _vp], ctypes.c_int),
    "ccr_compute_rho_noalloc": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp),
                                 ctypes.c_int, _vp], ctypes.c_int),
    "ccr_sft_series": ([_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, _vp,
                        _vp, ctypes.c_double, ctypes.c_int64, _vp, _vp], ctypes.c_int),
    "ccr_sync": ([_vp], ctypes.c_int),
    "ccr_kernel_time": ([_vp, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ccr_reset_kernel_times": ([_vp], ctypes.c_int),
    "ccr_resample_series": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _vp], ctypes.c_int),
    "ccr_segment_spectra": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _vp], ctypes.c_int),
    "ccr_time_base": ([_vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _dp, _dp, _dp],
                      ctypes.c_int),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libccr.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or "
                          "python paper_1712_06515_amd/build.py")
    L = ctypes.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if path == LIB_PATH:
        _lib = L
    return L


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Context:
    """One ccr_ctx: bands, data, weights, templates, and rho."""

    def __init__(self, sky, device=0):
        self.L = load_library()
        s = Sky(*(float(sky[k]) for k in ("ra", "dec", "au_s", "re_s", "obliquity", "year_s",
                                           "sidereal_day_s", "orbit_phase0", "gmst0")))
        h = _vp()
        st = self.L.ccr_create(ctypes.byref(h), int(device), ctypes.byref(s))
        if st != OK:
            raise CcrError(st, "ccr_create failed")
        self.h = h
        self.n_templates = {}

    def close(self):
        if getattr(self, "h", None):
            self.L.ccr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != OK:
            raise CcrError(st, self.L.ccr_last_error(self.h).decode())

    def set_option(self, name, value):
        self._check(self.L.ccr_set_option(self.h, name.encode(), int(value)))

    def get_option(self, name):
        v = ctypes.c_int64()
        self._check(self.L.ccr_get_option(self.h, name.encode(), ctypes.byref(v)))
        return v.value

    def add_band(self, band):
        b = Band(float(band["f_min"]), float(band["f_band"]), float(band["t_short"]), int(band["max_lag"]),
                 int(band.get("dirichlet_D", 8)), int(band.get("window", 0)), int(band.get("n_fft_override", 0)),
                 float(band.get("mu_f", 0.1)), int(band.get("pairs", PAIRS_CROSS | PAIRS_SAME)),
                 float(band.get("a_p_max", 0.0)), float(band.get("orbit_period", 68023.70)),
                 int(band.get("weight", WEIGHT_AVE)))
        bid = ctypes.c_int()
        info = BandInfo()
        self._check(self.L.ccr_add_band(self.h, ctypes.byref(b), ctypes.byref(bid), ctypes.byref(info)))
        return bid.value, info.as_dict()

    def set_data(self, band_id, det, site, t0, dt, x, f_het, valid=None):
        xs = _arr(x, np.complex64)
        vs = None if valid is None else _arr(valid, np.uint8)
        st = Site(float(site["lat"]), float(site["lon"]))
        self._check(self.L.ccr_set_data(self.h, band_id, det, ctypes.byref(st), float(t0), float(dt),
                                        xs.shape[0], float(f_het), xs.ctypes.data,
                                        None if vs is None else vs.ctypes.data))

    def set_weights(self, band_id, det, a, b, noise_var):
        a_, b_, n_ = _arr(a, np.float64), _arr(b, np.float64), _arr(noise_var, np.float64)
        self._check(self.L.ccr_set_weights(self.h, band_id, det, a_.shape[0],
                                           a_.ctypes.data_as(_dp), b_.ctypes.data_as(_dp), n_.ctypes.data_as(_dp)))

    def set_antenna(self, band_id, det, a, b):
        """Per-sample antenna functions on the source lattice; a = None removes them."""
        if a is None:
            self._check(self.L.ccr_set_antenna(self.h, band_id, det, 0, None, None))
            return
        a_, b_ = _arr(a, np.float64), _arr(b, np.float64)
        if a_.shape != b_.shape or a_.ndim != 1:
            raise ValueError("a and b must be 1-d arrays of one length")
        self._check(self.L.ccr_set_antenna(self.h, band_id, det, a_.shape[0], a_.ctypes.data_as(_dp),
                                           b_.ctypes.data_as(_dp)))

    def set_templates(self, band_id, templates):
        """Rows (a_p, T_asc, P) of circular orbits or (a_p, T_p, omega, e, P) of eccentric ones."""
        t = _arr(np.atleast_2d(templates), np.float64)
        cols = [_arr(t[:, k], np.float64) for k in range(t.shape[1])]
        if t.shape[1] == 3:
            self._check(self.L.ccr_set_templates(self.h, band_id, t.shape[0], *(c.ctypes.data_as(_dp) for c in cols)))
        elif t.shape[1] == 5:
            self._check(self.L.ccr_set_templates_ecc(self.h, band_id, t.shape[0],
                                                     *(c.ctypes.data_as(_dp) for c in cols)))
        else:
            raise ValueError("templates need 3 (circular) or 5 (eccentric) columns")
        self.n_templates[band_id] = t.shape[0]

    def band_info(self, band_id, freqs=False):
        info = BandInfo()
        self._check(self.L.ccr_get_band_info(self.h, band_id, ctypes.byref(info), None))
        d = info.as_dict()
        if freqs:
            f = np.zeros(info.n_f)
            self._check(self.L.ccr_get_band_info(self.h, band_id, ctypes.byref(info), f.ctypes.data_as(_dp)))
            return d, f
        return d

    def compute_rho(self, band_ids, prec=PREC_FP64, out_fp64=True, outputs=None, stream=None):
        """rho per band.  With ``outputs`` (device pointers, e.g. torch tensors' data_ptr()) the
        results stay on the device and nothing is returned; otherwise host numpy arrays."""
        ids = [band_ids] if isinstance(band_ids, int) else list(band_ids)
        idarr = (ctypes.c_int * len(ids))(*ids)
        if outputs is None:
            arrs = []
            for b in ids:
                info = self.band_info(b)
                arrs.append(np.zeros((info["n_templates"], info["n_f"]), dtype=np.float64 if out_fp64 else np.float32))
            ptrs = (_vp * len(ids))(*[a.ctypes.data for a in arrs])
            self._check(self.L.ccr_compute_rho(self.h, int(prec), len(ids), idarr, ptrs, 0, int(bool(out_fp64)), None))
            return arrs[0] if isinstance(band_ids, int) else arrs
        ptrs = (_vp * len(ids))(*[int(p) for p in outputs])
        self._check(self.L.ccr_compute_rho(self.h, int(prec), len(ids), idarr, ptrs, 1, int(bool(out_fp64)),
                                           None if stream is None else _vp(int(stream))))
        return None

    def compute_rho_noalloc(self, band_ids, outputs, prec=PREC_FP64, out_fp64=True, stream=None):
        """ccr_compute_rho_noalloc: rho into device buffers `outputs` (addresses), workspace in the
        library's fixed device array; the bands must be prepared (band_info after loading)."""
        ids = [band_ids] if isinstance(band_ids, int) else list(band_ids)
        idarr = (ctypes.c_int * len(ids))(*ids)
        ptrs = (_vp * len(ids))(*[int(p) for p in outputs])
        self._check(self.L.ccr_compute_rho_noalloc(self.h, int(prec), len(ids), idarr, ptrs, int(bool(out_fp64)),
                                                   None if stream is None else _vp(int(stream))))

    def sync(self):
        self._check(self.L.ccr_sync(self.h))

    KERNELS = ("resample", "spectra", "pairs", "finish", "fused", "timebase", "spectra_pairs", "spectra_wide",
               "sft_series")

    def kernel_times(self, reset=False):
        """{kernel: (total_ms, launches)} recorded while option "timing" is 1."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            self._check(self.L.ccr_kernel_time(self.h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        if reset:
            self._check(self.L.ccr_reset_kernel_times(self.h))
        return out

    def resample_series(self, band_id, template_index, det, prec=PREC_FP64):
        info = self.band_info(band_id)
        n = info["n_seg"] * info["n_k"]
        out = np.zeros(n, dtype=np.complex128 if prec == PREC_FP64 else np.complex64)
        self._check(self.L.ccr_resample_series(self.h, int(prec), band_id, int(template_index), int(det),
                                               out.ctypes.data))
        return out

    def time_base(self, band_id, template_index, det, k0=0, n_seg=None):
        """(eta [n_seg, n_k], anchor D_a [n_seg], psi [n_seg, n_k]) of segments k0.. of one
        detector: the delay of sample r is eta - D_a (NaN rows: segments not computed)."""
        info = self.band_info(band_id)
        n = info["n_seg"] - k0 if n_seg is None else n_seg
        eta = np.full((n, info["n_k"]), np.nan)
        psi = np.full((n, info["n_k"]), np.nan)
        anc = np.zeros(n)
        self._check(self.L.ccr_time_base(self.h, band_id, int(template_index), int(det), int(k0), int(n),
                                         eta.ctypes.data_as(_dp), anc.ctypes.data_as(_dp), psi.ctypes.data_as(_dp)))
        return eta, anc, psi

    def sft_series(self, z, t_sft, t0, k_first, f_het, n_out, sft_valid=None):
        """ccr_sft_series: (x complex64 [n_sft * n_out], valid uint8 [n_sft * n_out]) from SFT bins z
        (n_sft x n_bins complex, first bin k_first)."""
        zz = _arr(np.atleast_2d(z), np.complex64)
        n_sft, n_bins = zz.shape
        vs = None if sft_valid is None else _arr(sft_valid, np.uint8)
        x = np.zeros(n_sft * int(n_out), dtype=np.complex64)
        v = np.zeros(n_sft * int(n_out), dtype=np.uint8)
        self._check(self.L.ccr_sft_series(self.h, n_sft, float(t_sft), float(t0), n_bins, int(k_first), zz.ctypes.data,
                                          None if vs is None else vs.ctypes.data, float(f_het), int(n_out),
                                          x.ctypes.data, v.ctypes.data))
        return x, v

    def segment_spectra(self, band_id, template_index, prec=PREC_FP64):
        info = self.band_info(band_id)
        out = np.zeros((info["n_det"], info["n_seg"], info["n_f"]),
                       dtype=np.complex128 if prec == PREC_FP64 else np.complex64)
        self._check(self.L.ccr_segment_spectra(self.h, int(prec), band_id, int(template_index), out.ctypes.data))
        return out

    def load(self, ds, templates=None):
        """Add a band and set data, weights and templates from a dataset-like object with
        fields sky, band, sites, t0, dt, f_het, x, valid, a, b, noise_var, templates."""
        bid, _ = self.add_band(ds.band)
        for X in range(ds.x.shape[0]):
            self.set_data(bid, X, ds.sites[X], ds.t0, ds.dt, ds.x[X], ds.f_het,
                          None if ds.valid is None else ds.valid[X])
            self.set_weights(bid, X, ds.a[X], ds.b[X], ds.noise_var[X])
            if getattr(ds, "ar", None) is not None:
                self.set_antenna(bid, X, ds.ar[X], ds.br[X])
        self.set_templates(bid, ds.templates if templates is None else templates)
        return bid

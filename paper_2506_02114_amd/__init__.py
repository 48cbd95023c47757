"""Python binding of libmlmap (MI355X microlensing magnification maps).

Argument marshalling only: every step of a map runs in the HIP library
(``libmlmap.so``, built in-tree by ``paper_2506_02114_amd._build``).  Arrays
may be numpy arrays (host) or torch tensors on a HIP device (device); the
binding passes their pointers and a flag saying which they are.  If the
library is not built, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlmap.so")

MLM_OK, MLM_EINVAL, MLM_EDEGENERATE, MLM_ERANGE, MLM_ENOMEM, MLM_EDEVICE, MLM_ENOTSUP = range(7)
SHEET_CIRCLE, SHEET_NONE, SHEET_RECT = 0, 1, 2
MASS_EQUAL, MASS_SALPETER, MASS_KROUPA = 0, 1, 2
MAP_IPM, MAP_IRS = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
REFINE_NONE, REFINE_PLAIN, REFINE_LEARNED = 0, 1, 2
REFINER_PARAMS = 5057
METHOD_FMM, METHOD_DIRECT = 0, 1

EXPORTED = [
    "mlm_abi_version", "mlm_status_str", "mlm_last_error", "mlm_lens_create", "mlm_lens_destroy", "mlm_map_batch",
    "mlm_lens_get_info", "mlm_map_request_init", "mlm_map_region", "mlm_map", "mlm_deflect",
    "mlm_fmm_export", "mlm_refiner_create", "mlm_refiner_destroy", "mlm_refiner_get_params",
    "mlm_refiner_set_params", "mlm_refiner_predict", "mlm_refiner_grads", "mlm_train_opts_init",
    "mlm_refiner_train", "mlm_cell_samples", "mlm_map_noalloc", "mlm_lens_stars", "mlm_field_params_init",
    "mlm_field_moments", "mlm_field_count", "mlm_field_sample", "mlm_field_cover", "mlm_lens_create_sampled",
    "mlm_philox4x32_10", "mlm_light_curve", "mlm_histogram",
]


class MLMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib().mlm_status_str(status).decode()}: {msg}")
        self.status = status


class LensParams(C.Structure):
    _fields_ = [("kappa_star", C.c_double), ("kappa_smooth", C.c_double), ("gamma", C.c_double),
                ("sheet", C.c_int32), ("reserved", C.c_int32), ("rect_aspect", C.c_double),
                ("psi3", C.c_double * 4)]


class LensInfo(C.Structure):
    _fields_ = [("n_stars", C.c_int64), ("mass_sum", C.c_double), ("mean_m", C.c_double),
                ("mean_m2", C.c_double), ("r_star", C.c_double), ("kappa", C.c_double),
                ("mu_macro", C.c_double), ("max_abs", C.c_double), ("extent1", C.c_double),
                ("extent2", C.c_double)]


class FieldParams(C.Structure):
    _fields_ = [("kappa_star", C.c_double), ("mass_fn", C.c_int32), ("shape", C.c_int32),
                ("m_equal", C.c_double), ("m_lo", C.c_double), ("m_hi", C.c_double), ("n_stars", C.c_int64),
                ("extent1", C.c_double), ("extent2", C.c_double), ("rect_aspect", C.c_double),
                ("seed", C.c_uint64)]


class MapRequest(C.Structure):
    _fields_ = [("y1c", C.c_double), ("y2c", C.c_double), ("hw1", C.c_double), ("hw2", C.c_double),
                ("n1", C.c_int32), ("n2", C.c_int32), ("rays_per_pixel", C.c_double),
                ("nray1", C.c_int32), ("nray2", C.c_int32), ("flux_fraction", C.c_double),
                ("dx1", C.c_double), ("dx2", C.c_double), ("order", C.c_int32), ("leaf_max", C.c_int32),
                ("max_level", C.c_int32), ("precision", C.c_int32), ("method", C.c_int32),
                ("device_out", C.c_int32), ("eps", C.c_double), ("row_begin", C.c_int64),
                ("row_end", C.c_int64), ("stream", C.c_void_p), ("w_out", C.c_void_p),
                ("timing", C.c_int32), ("refine", C.c_int32), ("refine_depth", C.c_int32),
                ("refine_window", C.c_int32), ("refine_tau", C.c_double), ("refine_threshold", C.c_double),
                ("refiner", C.c_void_p), ("mapping", C.c_int32), ("one_stream", C.c_int32),
                ("x1c", C.c_double), ("x2c", C.c_double), ("centre_set", C.c_int32), ("big_pixels", C.c_int32)]


class Region(C.Structure):
    _fields_ = [("lam1", C.c_double), ("lam2", C.c_double), ("mu_macro", C.c_double), ("border", C.c_double),
                ("X1", C.c_double), ("X2", C.c_double), ("dX1", C.c_double), ("dX2", C.c_double),
                ("pix1", C.c_double), ("pix2", C.c_double), ("d1", C.c_double), ("d2", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("L0", C.c_double), ("nr1", C.c_int64),
                ("nr2", C.c_int64), ("order", C.c_int32), ("reserved", C.c_int32)]


class MapStats(C.Structure):
    _fields_ = [("n_rays", C.c_int64), ("n_cells", C.c_int64), ("n_skipped", C.c_int64),
                ("n_nodes", C.c_int64), ("n_leaves", C.c_int64), ("n_levels", C.c_int32),
                ("order", C.c_int32), ("near_pairs", C.c_int64), ("n_tiles", C.c_int64),
                ("tri_area", C.c_double), ("t_tree_ms", C.c_double), ("t_fmm_ms", C.c_double),
                ("t_shoot_ms", C.c_double), ("t_ipm_ms", C.c_double), ("t_total_ms", C.c_double),
                ("n_shoot_launches", C.c_int32), ("n_ipm_launches", C.c_int32),
                ("n_big", C.c_int64), ("n_big_rows", C.c_int64), ("t_cells_ms", C.c_double),
                ("t_band_ms", C.c_double), ("n_band_rows", C.c_int64), ("n_band_pieces", C.c_int64),
                ("n_refine_candidates", C.c_int64), ("n_refined", C.c_int64), ("n_refine_tests", C.c_int64),
                ("n_refine_large", C.c_int64), ("t_refine_ms", C.c_double),
                ("n_small", C.c_int64), ("n_col_items", C.c_int64), ("n_col_pieces", C.c_int64),
                ("n_pieces", C.c_int64), ("leaf_max", C.c_int32), ("big_pixels", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("vertex_budget", C.c_int64), ("autotune", C.c_int32), ("reserved0", C.c_int32),
                ("reserved", C.c_int64 * 6)]


class BatchStats(C.Structure):
    _fields_ = [("n_maps", C.c_int64), ("n_chunks", C.c_int64), ("n_rays", C.c_int64), ("n_cells", C.c_int64),
                ("n_big", C.c_int64), ("t_prep_ms", C.c_double), ("t_shoot_ms", C.c_double),
                ("t_ipm_ms", C.c_double), ("t_total_ms", C.c_double), ("reserved", C.c_int64 * 4)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("pos_weight", C.c_float),
                ("seed", C.c_uint64), ("device_ptrs", C.c_int32), ("graph", C.c_int32), ("stream", C.c_void_p)]


class TreeInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_leaves", C.c_int64), ("n_levels", C.c_int32),
                ("order", C.c_int32), ("L0", C.c_double)]


def _asdict(s: C.Structure) -> dict:
    return {k: getattr(s, k) for k, _ in s._fields_ if k != "reserved"}


_L = None


def _lib():
    """Load libmlmap.so; raises if it has not been built (no fallback path)."""
    global _L
    if _L is not None:
        return _L
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_02114_amd._build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)
    L.mlm_abi_version.restype = i32
    L.mlm_status_str.argtypes = [C.c_int]
    L.mlm_status_str.restype = C.c_char_p
    L.mlm_last_error.restype = C.c_char_p
    L.mlm_lens_create.argtypes = [C.POINTER(LensParams), vp, vp, vp, i64, i32, C.POINTER(vp)]
    L.mlm_lens_create.restype = C.c_int
    L.mlm_lens_destroy.argtypes = [vp]
    L.mlm_lens_destroy.restype = None
    L.mlm_lens_get_info.argtypes = [vp, C.POINTER(LensInfo)]
    L.mlm_lens_get_info.restype = C.c_int
    L.mlm_map_request_init.argtypes = [C.POINTER(MapRequest)]
    L.mlm_map_request_init.restype = None
    L.mlm_map_region.argtypes = [vp, C.POINTER(MapRequest), C.POINTER(Region)]
    L.mlm_map_region.restype = C.c_int
    L.mlm_map.argtypes = [vp, C.POINTER(MapRequest), vp, C.POINTER(MapStats)]
    L.mlm_map.restype = C.c_int
    L.mlm_map_noalloc.argtypes = [vp, C.POINTER(MapRequest), vp, C.POINTER(MapStats)]
    L.mlm_map_noalloc.restype = C.c_int
    L.mlm_lens_stars.argtypes = [vp, vp, vp, vp, i64, C.POINTER(i64)]
    L.mlm_field_params_init.argtypes = [C.POINTER(FieldParams)]
    L.mlm_field_params_init.restype = None
    L.mlm_field_moments.argtypes = [C.POINTER(FieldParams), dp, dp]
    L.mlm_field_count.argtypes = [C.POINTER(FieldParams), C.POINTER(i64)]
    L.mlm_field_sample.argtypes = [C.POINTER(FieldParams), vp, vp, vp, i64, C.POINTER(i64), dp, dp]
    L.mlm_field_cover.argtypes = [C.POINTER(LensParams), C.POINTER(FieldParams), C.POINTER(MapRequest), C.c_double,
                                  dp, dp]
    L.mlm_lens_create_sampled.argtypes = [C.POINTER(LensParams), C.POINTER(FieldParams), C.POINTER(vp)]
    L.mlm_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    L.mlm_philox4x32_10.restype = None
    L.mlm_light_curve.argtypes = [C.POINTER(MapRequest), vp, C.c_double, C.c_double, C.c_double, C.c_double, i64,
                                  vp]
    L.mlm_histogram.argtypes = [C.POINTER(MapRequest), vp, C.c_double, C.c_double, i32, vp]
    for nm in ("mlm_lens_stars", "mlm_field_moments", "mlm_field_count", "mlm_field_sample", "mlm_field_cover",
               "mlm_lens_create_sampled", "mlm_light_curve", "mlm_histogram"):
        getattr(L, nm).restype = C.c_int
    L.mlm_deflect.argtypes = [vp, C.POINTER(MapRequest), vp, i64, vp]
    L.mlm_deflect.restype = C.c_int
    L.mlm_fmm_export.argtypes = [vp, C.POINTER(MapRequest), C.POINTER(TreeInfo), vp, vp, vp, vp, vp, vp, vp, vp, i64]
    L.mlm_fmm_export.restype = C.c_int
    L.mlm_map_batch.argtypes = [C.POINTER(vp), C.POINTER(MapRequest), i32, C.POINTER(vp), C.POINTER(MapStats),
                                C.POINTER(BatchOpts), C.POINTER(BatchStats)]
    L.mlm_map_batch.restype = C.c_int
    fp, u8p = C.POINTER(C.c_float), C.POINTER(C.c_uint8)
    L.mlm_refiner_create.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    L.mlm_refiner_destroy.argtypes = [vp]
    L.mlm_refiner_destroy.restype = None
    L.mlm_refiner_get_params.argtypes = [vp, vp]
    L.mlm_refiner_set_params.argtypes = [vp, vp]
    L.mlm_refiner_predict.argtypes = [vp, vp, i64, vp, i32, vp]
    L.mlm_refiner_grads.argtypes = [vp, vp, vp, i64, C.c_float, vp, C.POINTER(C.c_double), i32, vp]
    L.mlm_train_opts_init.argtypes = [C.POINTER(TrainOpts)]
    L.mlm_train_opts_init.restype = None
    L.mlm_refiner_train.argtypes = [vp, C.POINTER(TrainOpts), vp, vp, i64, vp]
    L.mlm_cell_samples.argtypes = [vp, C.POINTER(MapRequest), vp, i64, vp, vp, i32]
    for f in ("mlm_refiner_create", "mlm_refiner_get_params", "mlm_refiner_set_params", "mlm_refiner_predict",
              "mlm_refiner_grads", "mlm_refiner_train", "mlm_cell_samples"):
        getattr(L, f).restype = C.c_int
    _L = L
    return L


def load():
    return _lib()


def _check(st: int):
    if st != MLM_OK:
        raise MLMError(st, _lib().mlm_last_error().decode())


def _is_torch_cuda(a) -> bool:
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


REQUEST_KEYS = {k for k, _ in MapRequest._fields_} - {"stream", "w_out", "device_out", "refiner"}


def _sheet_code(sheet) -> int:
    if sheet is True or sheet == "circle":
        return SHEET_CIRCLE
    if sheet is False or sheet is None or sheet == "none":
        return SHEET_NONE
    if sheet == "rect":
        return SHEET_RECT
    raise ValueError(f"unknown sheet {sheet!r}")


_MASS = {"equal": MASS_EQUAL, "salpeter": MASS_SALPETER, "kroupa": MASS_KROUPA}


def field_params(kappa_star: float, mass_fn: str = "equal", n_stars: int = 0, seed: int = 0, shape: str = "circle",
                 m_lo: float = 0.1, m_hi: float = 1.0, m_equal: float = 1.0, extent=(0.0, 0.0),
                 rect_aspect: float = 0.0) -> FieldParams:
    """mlm_field_params of a star field the library draws."""
    f = FieldParams()
    _lib().mlm_field_params_init(C.byref(f))
    f.kappa_star, f.mass_fn, f.shape = kappa_star, _MASS[mass_fn], _sheet_code(shape)
    f.m_lo, f.m_hi, f.m_equal, f.n_stars, f.seed = m_lo, m_hi, m_equal, int(n_stars), int(seed)
    f.extent1, f.extent2, f.rect_aspect = float(extent[0]), float(extent[1]), rect_aspect
    return f


def field_moments(f: FieldParams):
    a, b = C.c_double(), C.c_double()
    _check(_lib().mlm_field_moments(C.byref(f), C.byref(a), C.byref(b)))
    return a.value, b.value


def field_count(f: FieldParams) -> int:
    n = C.c_int64()
    _check(_lib().mlm_field_count(C.byref(f), C.byref(n)))
    return n.value


def field_sample(f: FieldParams):
    """(x, y, m, extent1, extent2) of the field (host arrays)."""
    n = field_count(f)
    x, y, m = (np.empty(n) for _ in range(3))
    cnt, e1, e2 = C.c_int64(), C.c_double(), C.c_double()
    _check(_lib().mlm_field_sample(C.byref(f), x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                   m.ctypes.data_as(C.c_void_p), n, C.byref(cnt), C.byref(e1), C.byref(e2)))
    return x, y, m, e1.value, e2.value


def field_cover(kappa_star: float, kappa_smooth: float, gamma: float, f: FieldParams, margin: float = 1.1,
                **req):
    """Star-region extents (extent1, extent2) covering a request's shooting region."""
    p = LensParams(kappa_star, kappa_smooth, gamma, f.shape, 0, 0.0)
    r = make_request(**req)
    e1, e2 = C.c_double(), C.c_double()
    _check(_lib().mlm_field_cover(C.byref(p), C.byref(f), C.byref(r), margin, C.byref(e1), C.byref(e2)))
    return e1.value, e2.value


def _map_args(mu, req: dict):
    r = make_request(**req)
    if _is_torch_cuda(mu):
        import torch
        assert mu.dtype == torch.float64 and mu.is_contiguous() and mu.numel() == r.n1 * r.n2
        r.device_out = 1
        r.stream = _current_stream()
        return r, C.c_void_p(mu.data_ptr()), True
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    assert mu.size == r.n1 * r.n2
    return r, mu, False


def light_curve(mu, start, end, npts: int, **req):
    """mu along the straight track start -> end (source-plane points), npts
    samples (mlm_light_curve).  mu: the map (numpy, or a torch tensor on the
    GPU, which gives a torch result); req: the map's request fields."""
    r, m, dev = _map_args(mu, req)
    if dev:
        import torch
        out = torch.empty(npts, dtype=torch.float64, device=mu.device)
        _check(_lib().mlm_light_curve(C.byref(r), m, start[0], start[1], end[0], end[1], npts,
                                      C.c_void_p(out.data_ptr())))
        return out
    out = np.empty(npts)
    _check(_lib().mlm_light_curve(C.byref(r), m.ctypes.data_as(C.c_void_p), start[0], start[1], end[0], end[1],
                                  npts, out.ctypes.data_as(C.c_void_p)))
    return out


def histogram(mu, lo: float, hi: float, nbins: int, **req):
    """Counts of log10(mu) in nbins bins on [lo, hi), with the underflow
    (mu <= 0 included) first and the overflow last (mlm_histogram)."""
    r, m, dev = _map_args(mu, req)
    if dev:
        import torch
        out = torch.empty(nbins + 2, dtype=torch.int64, device=mu.device)
        _check(_lib().mlm_histogram(C.byref(r), m, lo, hi, nbins, C.c_void_p(out.data_ptr())))
        return out
    out = np.empty(nbins + 2, np.int64)
    _check(_lib().mlm_histogram(C.byref(r), m.ctypes.data_as(C.c_void_p), lo, hi, nbins,
                                out.ctypes.data_as(C.c_void_p)))
    return out


def philox4x32_10(counter, key):
    """The published Philox4x32-10 block the sampler draws from."""
    c = (C.c_uint32 * 4)(*counter)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    _lib().mlm_philox4x32_10(c, k, o)
    return tuple(o)


def make_request(**kw) -> MapRequest:
    r = MapRequest()
    _lib().mlm_map_request_init(C.byref(r))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[v]
        if k == "method" and isinstance(v, str):
            v = {"fmm": METHOD_FMM, "direct": METHOD_DIRECT}[v]
        if k == "mapping" and isinstance(v, str):
            v = {"ipm": MAP_IPM, "irs": MAP_IRS}[v]
        if k == "refine" and isinstance(v, str):
            v = {"none": REFINE_NONE, "plain": REFINE_PLAIN, "learned": REFINE_LEARNED}[v]
        if k == "refiner":
            r.refiner = v._h if v is not None else None
            continue
        if k == "rows":
            if v is not None:
                r.row_begin, r.row_end = int(v[0]), int(v[1])
            continue
        if k in ("x1c", "x2c"):
            if v is None:
                continue
            r.centre_set = 1
        if k not in REQUEST_KEYS:
            raise TypeError(f"unknown map request field {k!r}")
        setattr(r, k, v)
    return r


class Lens:
    """Macro model + star field resident on the GPU (see mlm_lens_create)."""

    def __init__(self, kappa_star: float, kappa_smooth: float, gamma: float, x, y, m, sheet=True,
                 rect_aspect: float = 0.0, psi3=None):
        """sheet: True / "circle" (disc sheet), "rect" (rectangular sheet of
        aspect c2 / c1 = rect_aspect), False / "none".  psi3: the macro
        potential's third derivatives (psi_111, psi_112, psi_122, psi_222),
        near a macro critical curve (None: second order only)."""
        L = _lib()
        self._h = C.c_void_p()
        p = LensParams(kappa_star, kappa_smooth, gamma, _sheet_code(sheet), 0, rect_aspect,
                       (C.c_double * 4)(*([0.0] * 4 if psi3 is None else [float(v) for v in psi3])))
        if x is None:   # a field the library draws: see Lens.sampled
            return
        if _is_torch_cuda(x):
            import torch
            x, y, m = (t.to(torch.float64).contiguous() for t in (x, y, m))
            n = x.numel()
            _check(L.mlm_lens_create(C.byref(p), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                     C.c_void_p(m.data_ptr()), n, 1, C.byref(self._h)))
        else:
            x, y, m = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, m))
            n = x.size
            _check(L.mlm_lens_create(C.byref(p), x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                     m.ctypes.data_as(C.c_void_p), n, 0, C.byref(self._h)))
        self.n = n

    @classmethod
    def sampled(cls, kappa_star: float, kappa_smooth: float, gamma: float, field: "FieldParams", sheet=True):
        """A lens whose stars the library draws (mlm_lens_create_sampled)."""
        self = cls(kappa_star, kappa_smooth, gamma, None, None, None, sheet=sheet)
        p = LensParams(kappa_star, kappa_smooth, gamma, _sheet_code(sheet), 0, 0.0)
        _check(_lib().mlm_lens_create_sampled(C.byref(p), C.byref(field), C.byref(self._h)))
        self.n = self.info()["n_stars"]
        return self

    def stars(self):
        """The lens's stars (x, y, m) as host arrays (mlm_lens_stars)."""
        n = C.c_int64()
        st = _lib().mlm_lens_stars(self._h, None, None, None, 0, C.byref(n))
        if st not in (MLM_OK, MLM_ERANGE):
            _check(st)
        x, y, m = (np.empty(n.value) for _ in range(3))
        _check(_lib().mlm_lens_stars(self._h, x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                     m.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        return x, y, m

    def close(self):
        if getattr(self, "_h", None):
            _lib().mlm_lens_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        I = LensInfo()
        _check(_lib().mlm_lens_get_info(self._h, C.byref(I)))
        return _asdict(I)

    def region(self, **req) -> dict:
        r = make_request(**req)
        R = Region()
        _check(_lib().mlm_map_region(self._h, C.byref(r), C.byref(R)))
        return _asdict(R)

    def map(self, out=None, w_out=None, stream=None, noalloc: bool = False, **req):
        """Magnification map, (n2, n1) row-major.  `out` may be a float64 torch
        tensor on the GPU (the map stays on the device) or None (host numpy).
        noalloc: through mlm_map_noalloc (scratch from the library's static
        device array, no device allocation)."""
        r = make_request(**req)
        device = out is not None and _is_torch_cuda(out)
        if out is None:
            out = np.empty((r.n2, r.n1), dtype=np.float64)
        if device:
            import torch
            assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == r.n1 * r.n2
            r.device_out = 1
            r.stream = stream if stream is not None else _current_stream()
            ptr = C.c_void_p(out.data_ptr())
            if w_out is not None:
                assert _is_torch_cuda(w_out) and w_out.dtype == torch.float64 and w_out.is_contiguous()
                r.w_out = C.c_void_p(w_out.data_ptr())
        else:
            assert out.dtype == np.float64 and out.flags.c_contiguous and out.size == r.n1 * r.n2
            ptr = out.ctypes.data_as(C.c_void_p)
            if w_out is not None:
                assert isinstance(w_out, np.ndarray) and w_out.dtype == np.float64 and w_out.flags.c_contiguous
                r.w_out = w_out.ctypes.data_as(C.c_void_p)
        s = MapStats()
        fn = _lib().mlm_map_noalloc if noalloc else _lib().mlm_map
        _check(fn(self._h, C.byref(r), ptr, C.byref(s)))
        return out, _asdict(s)

    def deflect(self, z, stream=None, **req):
        """Source positions w of image-plane points z ((n, 2) float64)."""
        r = make_request(**req)
        if _is_torch_cuda(z):
            import torch
            z = z.to(torch.float64).contiguous()
            w = torch.empty_like(z)
            r.device_out = 1
            r.stream = stream if stream is not None else _current_stream()
            _check(_lib().mlm_deflect(self._h, C.byref(r), C.c_void_p(z.data_ptr()), z.shape[0],
                                      C.c_void_p(w.data_ptr())))
            return w
        z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 2)
        w = np.empty_like(z)
        _check(_lib().mlm_deflect(self._h, C.byref(r), z.ctypes.data_as(C.c_void_p), z.shape[0],
                                  w.ctypes.data_as(C.c_void_p)))
        return w

    def cell_samples(self, cells, **req):
        """Features (n x 12, float32) and first-level refinement labels of
        ray-grid cells (n x 2 int64 of (a, b)) of a request."""
        r = make_request(**req)
        cells = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1, 2)
        n = cells.shape[0]
        feats = np.empty((n, 12), np.float32)
        labels = np.empty(n, np.uint8)
        _check(_lib().mlm_cell_samples(self._h, C.byref(r), cells.ctypes.data_as(C.c_void_p), n,
                                       feats.ctypes.data_as(C.c_void_p), labels.ctypes.data_as(C.c_void_p), 0))
        return feats, labels

    def fmm_export(self, **req) -> dict:
        r = make_request(**req)
        I = TreeInfo()
        st = _lib().mlm_fmm_export(self._h, C.byref(r), C.byref(I), None, None, None, None, None, None, None,
                                   None, 0)
        if st not in (MLM_OK, MLM_ERANGE):
            _check(st)
        n, P1 = I.n_nodes, I.order + 1
        level = np.empty(n, np.int32); ix = np.empty(n, np.int64); iy = np.empty(n, np.int64)
        leaf = np.empty(n, np.int32); ns = np.empty(n, np.int64); blk = np.empty(n, np.int64)
        mult = np.empty(2 * n * P1); loc = np.empty(2 * n * P1)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(_lib().mlm_fmm_export(self._h, C.byref(r), C.byref(I), ptr(level), ptr(ix), ptr(iy), ptr(leaf),
                                     ptr(ns), ptr(blk), ptr(mult), ptr(loc), n))
        return dict(info=_asdict(I), level=level, i=ix, j=iy, leaf=leaf, nstars=ns, block=blk,
                    mult=mult.view(np.complex128).reshape(n, P1), local=loc.view(np.complex128).reshape(n, P1))


def map_batch(lenses, requests, outs, stream=None, autotune: bool = False, vertex_budget: int = 0):
    """Maps of many lenses in one call (mlm_map_batch).  `requests` are dicts
    of map-request fields, `outs` float64 arrays of (n2, n1): all numpy (host)
    or all torch tensors on the GPU.  Returns (per-map stats, batch stats)."""
    n = len(lenses)
    if not (len(requests) == n == len(outs)) or n == 0:
        raise ValueError("lenses, requests and outs must have the same non-zero length")
    device = _is_torch_cuda(outs[0])
    reqs = (MapRequest * n)()
    ptrs = (C.c_void_p * n)()
    hs = (C.c_void_p * n)()
    for i, (lens, kw, out) in enumerate(zip(lenses, requests, outs)):
        r = make_request(**kw)
        if device:
            import torch
            assert _is_torch_cuda(out) and out.dtype == torch.float64 and out.is_contiguous()
            assert out.numel() == r.n1 * r.n2
            r.device_out = 1
            r.stream = stream if stream is not None else _current_stream()
            ptrs[i] = out.data_ptr()
        else:
            assert isinstance(out, np.ndarray) and out.dtype == np.float64 and out.flags.c_contiguous
            assert out.size == r.n1 * r.n2
            ptrs[i] = out.ctypes.data
        reqs[i] = r
        hs[i] = lens._h.value
    stats = (MapStats * n)()
    o = BatchOpts(int(vertex_budget), 1 if autotune else 0, 0)
    b = BatchStats()
    _check(_lib().mlm_map_batch(hs, reqs, n, ptrs, stats, C.byref(o), C.byref(b)))
    return [_asdict(s) for s in stats], _asdict(b)


class Refiner:
    """The refinement network (mlm_refiner_*): FP32 parameters on the host
    side as one array of REFINER_PARAMS floats (W1, b1, W2, b2, W3, b3)."""

    def __init__(self, params=None, seed: int = 0):
        self._h = C.c_void_p()
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if p is not None:
            assert p.size == REFINER_PARAMS
        _check(_lib().mlm_refiner_create(p.ctypes.data_as(C.c_void_p) if p is not None else None, seed,
                                         C.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None):
            _lib().mlm_refiner_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        p = np.empty(REFINER_PARAMS, np.float32)
        _check(_lib().mlm_refiner_get_params(self._h, p.ctypes.data_as(C.c_void_p)))
        return p

    @params.setter
    def params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == REFINER_PARAMS
        _check(_lib().mlm_refiner_set_params(self._h, p.ctypes.data_as(C.c_void_p)))

    def predict(self, feats) -> np.ndarray:
        f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 12)
        out = np.empty(f.shape[0], np.float32)
        _check(_lib().mlm_refiner_predict(self._h, f.ctypes.data_as(C.c_void_p), f.shape[0],
                                          out.ctypes.data_as(C.c_void_p), 0, None))
        return out

    def grads(self, feats, labels, pos_weight: float = 1.0):
        f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 12)
        y = np.ascontiguousarray(labels, dtype=np.uint8)
        g = np.empty(REFINER_PARAMS, np.float32)
        loss = C.c_double()
        _check(_lib().mlm_refiner_grads(self._h, f.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                        f.shape[0], pos_weight, g.ctypes.data_as(C.c_void_p), C.byref(loss), 0,
                                        None))
        return loss.value, g

    def train(self, feats, labels, epochs: int = 4, batch: int = 4096, lr: float = 1e-3, pos_weight: float = 1.0,
              seed: int = 0, graph: bool = True):
        f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 12)
        y = np.ascontiguousarray(labels, dtype=np.uint8)
        o = TrainOpts()
        _lib().mlm_train_opts_init(C.byref(o))
        o.epochs, o.batch, o.lr, o.pos_weight, o.seed = epochs, batch, lr, pos_weight, seed
        o.graph = 1 if graph else 0
        losses = np.empty(max(epochs, 1), np.float32)
        _check(_lib().mlm_refiner_train(self._h, C.byref(o), f.ctypes.data_as(C.c_void_p),
                                        y.ctypes.data_as(C.c_void_p), f.shape[0], losses.ctypes.data_as(C.c_void_p)))
        return losses[:epochs]


def params_to_dict(p) -> dict:
    """Split a flat parameter array into the named tensors (float64)."""
    p = np.asarray(p, dtype=np.float64)
    return dict(W1=p[0:768].reshape(12, 64), b1=p[768:832], W2=p[832:4928].reshape(64, 64), b2=p[4928:4992],
                W3=p[4992:5056], b3=p[5056:5057])

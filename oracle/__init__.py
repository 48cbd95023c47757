"""FP64 CPU oracle of the magnification-map hot path (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
built from ``oracle.c`` with gcc) and composes its steps in the order the
paper gives them:

  set-up of the shooting region and ray grid (sec. 2.3, appendix A)
  -> lens equation for every grid vertex, the star deflection either by direct
     summation (sec. 2.2) or by the FMM of appendix C
  -> IPM: apportion every mapped triangle among source pixels (sec. 3.2)
  -> magnification = deposited image area / pixel area.

Nothing here is shared with, or calls into, the HIP library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
          "-fcx-limited-range", "-pthread", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (generic x86-64, no host-specific ISA)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def use_native_build(directory: str) -> str:
    """Compile the same source with -O3 -march=native for the host it runs
    on, into `directory`, and load that build instead (the CPU baseline's
    timing build; the arithmetic is the same, contraction stays off)."""
    global _lib
    path = os.path.join(directory, "liboracle_native.so")
    flags = ["-O3", "-march=native"] + [f for f in CFLAGS if f != "-O2"]
    subprocess.run(["gcc", *flags, _SRC, "-o", path, "-lm"], check=True)
    _lib = None
    lib(path)
    return path


_lib = None
_dp = C.POINTER(C.c_double)
_lp = C.POINTER(C.c_long)
_ip = C.POINTER(C.c_int)


class Region(C.Structure):
    _fields_ = [
        ("y1c", C.c_double), ("y2c", C.c_double), ("hw1", C.c_double), ("hw2", C.c_double),
        ("n1", C.c_long), ("n2", C.c_long),
        ("rays_per_pixel", C.c_double),
        ("nray1", C.c_long), ("nray2", C.c_long),
        ("flux_fraction", C.c_double),
        ("dx1_set", C.c_double), ("dx2_set", C.c_double),
        ("x1c_set", C.c_double), ("x2c_set", C.c_double), ("centre_set", C.c_long),
        ("kappa", C.c_double), ("lam1", C.c_double), ("lam2", C.c_double), ("mu_macro", C.c_double),
        ("mean_m", C.c_double), ("mean_m2", C.c_double), ("border", C.c_double),
        ("X1", C.c_double), ("X2", C.c_double), ("dX1", C.c_double), ("dX2", C.c_double),
        ("pix1", C.c_double), ("pix2", C.c_double),
        ("nr1", C.c_long), ("nr2", C.c_long),
        ("d1", C.c_double), ("d2", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("L0", C.c_double),
    ]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib(path: Optional[str] = None):
    global _lib
    if _lib is None:
        if path is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        L = C.CDLL(path)
        L.orc_alpha_direct.argtypes = [C.c_long, _dp, _dp, _dp, C.c_long, _dp, _dp, _dp, _dp, C.c_int]
        L.orc_alpha_direct_reversed.argtypes = [C.c_long, _dp, _dp, _dp, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_lens_equation.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                        _dp, C.c_long, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_sheet_alpha.argtypes = [C.c_double, C.c_int, C.c_double, C.c_double, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_star_rect.argtypes = [C.c_long, _dp, C.c_double, C.c_double, _dp, _dp]
        L.orc_irs_rows.argtypes = [C.POINTER(Region), C.c_double, C.c_double, C.c_double, C.c_int, C.c_double,
                                   C.c_double, _dp, C.c_long, _dp, _dp, _dp, C.c_void_p, C.c_long, C.c_long, _lp,
                                   _dp, C.c_int]
        L.orc_irs_rows.restype = C.c_long
        L.orc_star_radius.argtypes = [C.c_long, _dp, C.c_double]
        L.orc_star_radius.restype = C.c_double
        L.orc_region_setup.argtypes = [C.POINTER(Region), C.c_double, C.c_double, C.c_double,
                                       C.c_long, _dp, _dp, _dp, C.c_int]
        L.orc_region_setup.restype = C.c_int
        L.orc_grid_points.argtypes = [C.POINTER(Region), C.c_long, C.c_long, _dp, _dp]
        L.orc_fmm_build.argtypes = [C.c_long, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_fmm_build.restype = C.c_void_p
        L.orc_fmm_free.argtypes = [C.c_void_p]
        L.orc_fmm_num_nodes.argtypes = [C.c_void_p]
        L.orc_fmm_num_nodes.restype = C.c_long
        L.orc_fmm_num_levels.argtypes = [C.c_void_p]
        L.orc_fmm_num_levels.restype = C.c_int
        L.orc_fmm_nodes.argtypes = [C.c_void_p, _ip, _lp, _lp, _ip, _lp, _lp]
        L.orc_fmm_coeffs.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_fmm_alpha.argtypes = [C.c_void_p, C.c_long, _dp, _dp, _dp, _dp, _lp, C.c_int]
        L.orc_fmm_eval_multipole.argtypes = [C.c_void_p, C.c_long, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_fmm_eval_local.argtypes = [C.c_void_p, C.c_long, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_fmm_sorted_stars.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_fmm_sorted_stars.restype = C.c_long
        for nm in ("orc_op_m2m", "orc_op_m2l", "orc_op_l2l"):
            getattr(L, nm).argtypes = [C.c_int, _dp, C.c_double, C.c_double, _dp]
        L.orc_tri_pixel_area.argtypes = [_dp, _dp, C.c_long, C.c_long]
        L.orc_tri_pixel_area.restype = C.c_double
        L.orc_ipm_rows.argtypes = [C.POINTER(Region), C.c_long, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_cell_features.argtypes = [_dp, _dp, _dp]
        L.orc_refine_cells.argtypes = [C.POINTER(Region), C.c_double, C.c_double, C.c_double, C.c_int, C.c_double,
                                       C.c_double, _dp,
                                       C.c_long, _dp, _dp, _dp, C.c_void_p, C.c_long, _lp, _lp, C.c_double,
                                       C.c_int, C.c_int, C.POINTER(C.c_ubyte), _dp, _lp]
        L.orc_normalise.argtypes = [C.POINTER(Region), _dp, _dp]
        L.orc_shoot_rows.argtypes = [C.POINTER(Region), C.c_double, C.c_double, C.c_double, C.c_int,
                                     C.c_double, C.c_double, _dp, C.c_long, _dp, _dp, _dp, C.c_void_p, C.c_long,
                                     C.c_long, _dp, _dp, C.c_int]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# lens
# --------------------------------------------------------------------------

@dataclass
class Lens:
    """Macro model + star field (sec. 2.2).  sheet=True (or "circle") adds the
    circular compensating sheet of radius R_* = sqrt(sum m / kappa_*) (sec.
    3.1); sheet="rect" the rectangular one of app. B over [-c1, c1] x
    [-c2, c2] with c2 = rect_aspect c1 and 4 c1 c2 = pi sum m / kappa_*."""
    kappa_star: float
    kappa_smooth: float
    gamma: float
    x: np.ndarray
    y: np.ndarray
    m: np.ndarray
    sheet: object = True
    rect_aspect: float = 0.0
    psi3: object = None     # (psi_111, psi_112, psi_122, psi_222): third-order macro terms (app. D)

    def __post_init__(self):
        self.x, self.y, self.m = _f64(self.x), _f64(self.y), _f64(self.m)
        self.psi3 = _f64(np.zeros(4) if self.psi3 is None else self.psi3)
        assert self.psi3.shape == (4,)
        self.r_star = lib().orc_star_radius(len(self.m), _d(self.m), self.kappa_star)
        if self.sheet is True or self.sheet == "circle":
            self.sheet_code, self.e1, self.e2 = (1 if self.n else 0), self.r_star, self.r_star
        elif self.sheet == "rect":
            c1, c2 = C.c_double(), C.c_double()
            lib().orc_star_rect(self.n, _d(self.m), self.kappa_star, self.rect_aspect, C.byref(c1), C.byref(c2))
            self.sheet_code, self.e1, self.e2 = (2 if self.n else 0), c1.value, c2.value
        elif self.sheet is False or self.sheet is None or self.sheet == "none":
            self.sheet_code, self.e1, self.e2 = 0, 0.0, 0.0
        else:
            raise ValueError(f"unknown sheet {self.sheet!r}")

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def alpha_direct(lens: Lens, zx, zy, nthreads: int = 0, reversed_order: bool = False):
    """Star deflection a_*(z) by direct summation (sec. 2.2)."""
    zx, zy = _f64(zx), _f64(zy)
    ax, ay = np.empty_like(zx), np.empty_like(zy)
    if reversed_order:
        lib().orc_alpha_direct_reversed(lens.n, _d(lens.x), _d(lens.y), _d(lens.m), zx.size,
                                        _d(zx), _d(zy), _d(ax), _d(ay))
    else:
        lib().orc_alpha_direct(lens.n, _d(lens.x), _d(lens.y), _d(lens.m), zx.size,
                               _d(zx), _d(zy), _d(ax), _d(ay), nthreads)
    return ax, ay


def lens_equation(lens: Lens, zx, zy, ax, ay):
    zx, zy, ax, ay = map(_f64, (zx, zy, ax, ay))
    wx, wy = np.empty_like(zx), np.empty_like(zy)
    lib().orc_lens_equation(lens.kappa_star, lens.kappa_smooth, lens.gamma, lens.sheet_code,
                            lens.e1, lens.e2, _d(lens.psi3), zx.size, _d(zx), _d(zy), _d(ax), _d(ay), _d(wx), _d(wy))
    return wx, wy


def sheet_alpha(kappa_star: float, sheet: str, e1: float, e2: float, zx, zy):
    """Deflection a_s of a compensating sheet alone: "circle" of radius e1
    (sec. 3.1) or "rect" with corner (e1, e2) (app. B)."""
    zx, zy = _f64(zx), _f64(zy)
    ax, ay = np.empty_like(zx), np.empty_like(zy)
    lib().orc_sheet_alpha(kappa_star, {"circle": 1, "rect": 2}[sheet], e1, e2, zx.size, _d(zx), _d(zy),
                          _d(ax), _d(ay))
    return ax, ay


def shoot_direct(lens: Lens, zx, zy, nthreads: int = 0):
    ax, ay = alpha_direct(lens, zx, zy, nthreads)
    return lens_equation(lens, zx, zy, ax, ay)


# --------------------------------------------------------------------------
# region
# --------------------------------------------------------------------------

class DegenerateMacro(ValueError):
    pass


def region(lens: Lens, y1c=0.0, y2c=0.0, hw1=5.0, hw2=5.0, n1=256, n2=256, rays_per_pixel=1.0,
           nray1=0, nray2=0, flux_fraction=0.01, dx1=0.0, dx2=0.0, x1c=None, x2c=None, **_ignored) -> Region:
    """Shooting region and ray grid; x1c/x2c give the image-plane centre
    explicitly (needed, with dx1/dx2, when the lens has third-order terms)."""
    centre = x1c is not None and x2c is not None
    R = Region(y1c=y1c, y2c=y2c, hw1=hw1, hw2=hw2, n1=n1, n2=n2, rays_per_pixel=rays_per_pixel,
               nray1=nray1, nray2=nray2, flux_fraction=flux_fraction, dx1_set=dx1, dx2_set=dx2,
               x1c_set=x1c if centre else 0.0, x2c_set=x2c if centre else 0.0, centre_set=1 if centre else 0)
    rc = lib().orc_region_setup(C.byref(R), lens.kappa_star, lens.kappa_smooth, lens.gamma,
                                lens.n, _d(lens.x), _d(lens.y), _d(lens.m), 1 if np.any(lens.psi3 != 0) else 0)
    if rc == 2:
        raise DegenerateMacro("|1-kappa+-gamma| vanishes: shooting region is unbounded")
    if rc != 0:
        raise ValueError("invalid map request")
    return R


def grid_points(R: Region, row_lo: int, row_hi: int):
    n = (row_hi - row_lo) * R.nr1
    zx, zy = np.empty(n), np.empty(n)
    lib().orc_grid_points(C.byref(R), row_lo, row_hi, _d(zx), _d(zy))
    return zx, zy


# --------------------------------------------------------------------------
# FMM (appendix C)
# --------------------------------------------------------------------------

MAX_LEVEL = 24


class FMM:
    """Tree + multipole/local coefficients of appendix C, built on the CPU."""

    def __init__(self, lens: Lens, L0: float, p: int, nmax: int = 32, lmax: int = MAX_LEVEL,
                 nthreads: int = 0):
        self.lens, self.L0, self.p, self.nmax, self.lmax = lens, L0, p, nmax, lmax
        self._h = lib().orc_fmm_build(lens.n, _d(lens.x), _d(lens.y), _d(lens.m), L0, p, nmax,
                                      lmax, nthreads)
        if not self._h:
            raise ValueError("oracle FMM build failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc_fmm_free(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def num_nodes(self) -> int:
        return lib().orc_fmm_num_nodes(self._h)

    @property
    def num_levels(self) -> int:
        return lib().orc_fmm_num_levels(self._h)

    def nodes(self):
        n = self.num_nodes
        level = np.empty(n, np.int32); i = np.empty(n, np.int64); j = np.empty(n, np.int64)
        leaf = np.empty(n, np.int32); ns = np.empty(n, np.int64); blk = np.empty(n, np.int64)
        lib().orc_fmm_nodes(self._h, level.ctypes.data_as(_ip), i.ctypes.data_as(_lp),
                            j.ctypes.data_as(_lp), leaf.ctypes.data_as(_ip),
                            ns.ctypes.data_as(_lp), blk.ctypes.data_as(_lp))
        return dict(level=level, i=i, j=j, leaf=leaf, nstars=ns, block=blk)

    def coeffs(self):
        n, P1 = self.num_nodes, self.p + 1
        a = np.empty(2 * n * P1); c = np.empty(2 * n * P1)
        lib().orc_fmm_coeffs(self._h, _d(a), _d(c))
        a = a.view(np.complex128).reshape(n, P1)
        c = c.view(np.complex128).reshape(n, P1)
        return a, c

    def alpha(self, zx, zy, nthreads: int = 0, want_leaf: bool = False):
        zx, zy = _f64(zx), _f64(zy)
        ax, ay = np.empty_like(zx), np.empty_like(zy)
        leaf = np.empty(zx.size, np.int64) if want_leaf else None
        lib().orc_fmm_alpha(self._h, zx.size, _d(zx), _d(zy), _d(ax), _d(ay),
                            leaf.ctypes.data_as(_lp) if want_leaf else None, nthreads)
        return (ax, ay, leaf) if want_leaf else (ax, ay)

    def eval_multipole(self, q: int, zx, zy):
        zx, zy = _f64(zx), _f64(zy)
        gx, gy = np.empty_like(zx), np.empty_like(zy)
        lib().orc_fmm_eval_multipole(self._h, q, zx.size, _d(zx), _d(zy), _d(gx), _d(gy))
        return gx + 1j * gy

    def eval_local(self, q: int, zx, zy):
        zx, zy = _f64(zx), _f64(zy)
        gx, gy = np.empty_like(zx), np.empty_like(zy)
        lib().orc_fmm_eval_local(self._h, q, zx.size, _d(zx), _d(zy), _d(gx), _d(gy))
        return gx + 1j * gy

    def sorted_stars(self):
        n = self.lens.n
        x, y, m = np.empty(n), np.empty(n), np.empty(n)
        lib().orc_fmm_sorted_stars(self._h, _d(x), _d(y), _d(m))
        return x, y, m


def _op(name: str, p: int, coeffs: np.ndarray, z0: complex) -> np.ndarray:
    ci = np.ascontiguousarray(np.asarray(coeffs, np.complex128)).view(np.float64).copy()
    out = np.empty(2 * (p + 1))
    getattr(lib(), name)(p, _d(ci), float(np.real(z0)), float(np.imag(z0)), _d(out))
    return out.view(np.complex128)


def op_m2m(p, a, z0):
    return _op("orc_op_m2m", p, a, z0)


def op_m2l(p, b, z0):
    return _op("orc_op_m2l", p, b, z0)


def op_l2l(p, c, z0):
    return _op("orc_op_l2l", p, c, z0)


def auto_order(mean_m: float, mean_m2: float, L: float, eps: float, pmax: int = 31) -> int:
    """Expansion order of appendix C.3: smallest integer p with
    p > log2( (<m^2>/<m>) / (L |eps|) ), capped at pmax."""
    import math
    if mean_m <= 0:
        return 1
    t = math.log2((mean_m2 / mean_m) / (L * eps))
    p = int(math.floor(t)) + 1
    return max(1, min(pmax, p))


# --------------------------------------------------------------------------
# IPM (sec. 3.2)
# --------------------------------------------------------------------------

def tri_pixel_area(tu, tv, i: int, j: int) -> float:
    tu, tv = _f64(tu), _f64(tv)
    return lib().orc_tri_pixel_area(_d(tu), _d(tv), i, j)


def shoot_rows(R: Region, lens: Lens, row_lo: int, row_hi: int, fmm: Optional[FMM] = None,
               nthreads: int = 0):
    """Source positions w of vertex rows [row_lo, row_hi)."""
    n = (row_hi - row_lo) * R.nr1
    wx, wy = np.empty(n), np.empty(n)
    lib().orc_shoot_rows(C.byref(R), lens.kappa_star, lens.kappa_smooth, lens.gamma,
                         lens.sheet_code, lens.e1, lens.e2, _d(lens.psi3), lens.n, _d(lens.x), _d(lens.y), _d(lens.m),
                         fmm.handle if fmm is not None else None, row_lo, row_hi, _d(wx), _d(wy),
                         nthreads)
    return wx, wy


def ipm_rows(R: Region, row_lo: int, row_hi: int, wx, wy, dep: np.ndarray, stats: np.ndarray):
    """Apportion the triangles of cell rows [row_lo, row_hi); wx, wy hold vertex
    rows row_lo .. row_hi inclusive."""
    wx, wy = _f64(wx), _f64(wy)
    assert wx.size == (row_hi - row_lo + 1) * R.nr1
    lib().orc_ipm_rows(C.byref(R), row_lo, row_hi, _d(wx), _d(wy), _d(dep), _d(stats))


@dataclass
class MapResult:
    mu: np.ndarray             # (n2, n1), row j = y2 ascending, column i = y1 ascending
    region: Region
    dep_total: float           # image area deposited inside the map
    a_out: float               # image area mapped outside the map
    a_skip: float              # image area of skipped (non-finite) triangles
    n_skip: int
    n_zero: int
    rows: tuple


def magnification_map(lens: Lens, spec: dict, method: str = "fmm", p: int = 0,
                      nmax: int = 32, lmax: int = MAX_LEVEL, rows=None, eps: float = 1e-7,
                      nthreads: int = 0, chunk_rows: int = 256) -> MapResult:
    """Whole map (or the cell rows `rows` = (lo, hi)) in FP64 on the CPU."""
    R = region(lens, **spec)
    row_lo, row_hi = rows if rows is not None else (0, R.nr2 - 1)
    fmm = None
    if method == "fmm":
        if p <= 0:
            p = spec.get("order", 0) or 0
        if p <= 0:
            # smallest node half-length the tree can have with these stars is not
            # known before building; use the root / 2^levels estimate after build
            fmm_probe = FMM(lens, R.L0, 1, nmax, lmax, nthreads)
            nl = fmm_probe.num_levels
            del fmm_probe
            p = auto_order(R.mean_m, R.mean_m2, R.L0 / 2 ** (nl - 1), eps)
        fmm = FMM(lens, R.L0, p, nmax, lmax, nthreads)
    elif method != "direct":
        raise ValueError(method)
    dep = np.zeros(R.n1 * R.n2)
    stats = np.zeros(5)
    b = row_lo
    while b < row_hi:
        e = min(row_hi, b + chunk_rows)
        wx, wy = shoot_rows(R, lens, b, e + 1, fmm, nthreads)
        ipm_rows(R, b, e, wx, wy, dep, stats)
        b = e
    mu = np.empty_like(dep)
    lib().orc_normalise(C.byref(R), _d(dep), _d(mu))
    return MapResult(mu.reshape(R.n2, R.n1), R, stats[0], stats[1], stats[2], int(stats[3]),
                     int(stats[4]), (row_lo, row_hi))


@dataclass
class IRSResult:
    counts: np.ndarray         # (n2, n1) rays per pixel
    mu: np.ndarray             # counts D1 D2 / (pix1 pix2)
    region: Region
    n_out: int                 # rays landing outside the map
    uv: Optional[np.ndarray]   # (rays, 2) landing points in pixel units, if asked for
    rows: tuple


def irs_map(lens: Lens, spec: dict, method: str = "direct", p: int = 0, rows=None, want_uv: bool = False,
            nthreads: int = 0, nmax: int = 32) -> IRSResult:
    """Inverse ray shooting (sec. 2.3, 4): one ray at the centre of every
    cell of the ray grid (or of the cell rows `rows`), counted in the pixel
    it lands in."""
    R = region(lens, **spec)
    row_lo, row_hi = rows if rows is not None else (0, R.nr2 - 1)
    fmm = None
    if method == "fmm":
        fmm = FMM(lens, R.L0, p if p > 0 else 20, nmax, MAX_LEVEL, nthreads)
    elif method != "direct":
        raise ValueError(method)
    counts = np.zeros(R.n1 * R.n2, np.int64)
    nrays = (row_hi - row_lo) * (R.nr1 - 1)
    uv = np.empty(2 * max(nrays, 1)) if want_uv else None
    out = lib().orc_irs_rows(C.byref(R), lens.kappa_star, lens.kappa_smooth, lens.gamma, lens.sheet_code,
                             lens.e1, lens.e2, _d(lens.psi3), lens.n, _d(lens.x), _d(lens.y), _d(lens.m),
                             fmm.handle if fmm is not None else None, row_lo, row_hi,
                             counts.ctypes.data_as(_lp), _d(uv) if want_uv else None, nthreads)
    mu = counts * (R.d1 * R.d2 / (R.pix1 * R.pix2))
    return IRSResult(counts.reshape(R.n2, R.n1), mu.reshape(R.n2, R.n1), R, int(out),
                     uv[:2 * nrays].reshape(-1, 2) if want_uv else None, (row_lo, row_hi))


# ---------------------------------------------------------------------------
# Cell refinement and its learned stand-in.  The paper apportions every cell
# as two triangles and does no subdivision (sec. 3.2); the refinement below is
# the plain test the learned variant is trained on and judged against:
#   refine a (sub)cell if its mapped ears disagree in orientation (a critical
#   curve crosses it) or if splitting it 2 x 2 changes its in-map deposits
#   by more than TAU times its image area (L1 over pixels); a refined cell is
#   replaced by its four children, tested again down to MAX_DEPTH levels;
#   cells whose triangles span more than WINDOW pixels are left alone.
# ---------------------------------------------------------------------------
REFINE_TAU = 1e-3
REFINE_MAX_DEPTH = 3
REFINE_WINDOW = 8


def cell_features(u4, v4) -> np.ndarray:
    """12 features of a mapped cell (corners in the order 00, 10, 11, 01)."""
    f = np.empty(12)
    lib().orc_cell_features(_d(_f64(u4)), _d(_f64(v4)), _d(f))
    return f


def refine_cells(R: Region, lens: Lens, cells_a, cells_b, fmm: Optional[FMM] = None, tau: float = REFINE_TAU,
                 max_depth: int = REFINE_MAX_DEPTH, window: int = REFINE_WINDOW):
    """Plain refinement of ray-grid cells (a, b): per-cell labels (1: the
    cell itself is refined), the magnification change of the map (refined
    minus plain, n2 x n1) and {tested, refined, too large} counts."""
    ca = np.ascontiguousarray(cells_a, dtype=np.int64)
    cb = np.ascontiguousarray(cells_b, dtype=np.int64)
    labels = np.zeros(ca.size, np.uint8)
    dep = np.zeros(R.n1 * R.n2)
    st = np.zeros(3, np.int64)
    lib().orc_refine_cells(C.byref(R), lens.kappa_star, lens.kappa_smooth, lens.gamma, lens.sheet_code,
                           lens.e1, lens.e2, _d(lens.psi3), lens.n, _d(lens.x), _d(lens.y), _d(lens.m),
                           fmm.handle if fmm is not None else None, ca.size, ca.ctypes.data_as(_lp),
                           cb.ctypes.data_as(_lp), tau, max_depth, window,
                           labels.ctypes.data_as(C.POINTER(C.c_ubyte)), _d(dep), st.ctypes.data_as(_lp))
    dmu = np.empty_like(dep)
    lib().orc_normalise(C.byref(R), _d(dep), _d(dmu))
    return labels, dmu.reshape(R.n2, R.n1), st


# The refinement network: 12 -> 64 -> 64 -> 1, ReLU between layers, a logit
# out; trained with the weighted binary cross-entropy
#   loss = mean_i [ w+ y_i softplus(-z_i) + (1 - y_i) softplus(z_i) ].
MLP_SIZES = (12, 64, 64, 1)


def mlp_init(seed: int = 0) -> dict:
    """He-normal weights, zero biases (a fixed, seeded start)."""
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, np.sqrt(2 / 12), (12, 64)), b1=np.zeros(64),
                W2=rng.normal(0, np.sqrt(2 / 64), (64, 64)), b2=np.zeros(64),
                W3=rng.normal(0, np.sqrt(2 / 64), 64), b3=np.zeros(1))


def mlp_forward(P: dict, X: np.ndarray):
    """Logits of samples X (n x 12), with the hidden activations."""
    A1 = X @ P["W1"] + P["b1"]
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ P["W2"] + P["b2"]
    H2 = np.maximum(A2, 0.0)
    z = H2 @ P["W3"] + P["b3"][0]
    return z, (X, A1, H1, A2, H2)


def _softplus(x):
    return np.logaddexp(0.0, x)


def mlp_loss_grad(P: dict, X: np.ndarray, y: np.ndarray, pos_weight: float = 1.0):
    """Loss and its gradient with respect to every parameter (FP64)."""
    z, (X, A1, H1, A2, H2) = mlp_forward(P, X)
    y = y.astype(np.float64)
    n = X.shape[0]
    loss = np.mean(pos_weight * y * _softplus(-z) + (1 - y) * _softplus(z))
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (pos_weight * y * (sig - 1.0) + (1 - y) * sig) / n
    G = {}
    G["W3"] = H2.T @ dz
    G["b3"] = np.array([dz.sum()])
    dA2 = np.outer(dz, P["W3"]) * (A2 > 0)
    G["W2"] = H1.T @ dA2
    G["b2"] = dA2.sum(axis=0)
    dA1 = (dA2 @ P["W2"].T) * (A1 > 0)
    G["W1"] = X.T @ dA1
    G["b1"] = dA1.sum(axis=0)
    return loss, G


# ---------------------------------------------------------------------------
# Products of a map (sec. 4.1, 5): light curves and magnification histograms
# ---------------------------------------------------------------------------

def light_curve(mu: np.ndarray, spec: dict, start, end, npts: int) -> np.ndarray:
    """mu of a point source at npts points evenly spaced from start to end
    (source-plane coordinates, both ends included), interpolated bilinearly
    between pixel centres: pixel (i, j) is centred at
    (y1c - hw1 + (i + 1/2) pix1, y2c - hw2 + (j + 1/2) pix2); within half a
    pixel of the map's edge the nearest row or column is repeated; NaN
    outside the map.  Plain loops over the points."""
    n2, n1 = mu.shape
    hw1, hw2 = spec["hw1"], spec["hw2"]
    y1c, y2c = spec.get("y1c", 0.0), spec.get("y2c", 0.0)
    pix1, pix2 = 2.0 * hw1 / n1, 2.0 * hw2 / n2
    out = np.empty(npts)
    for k in range(npts):
        f = k / (npts - 1) if npts > 1 else 0.0
        y1 = start[0] + f * (end[0] - start[0])
        y2 = start[1] + f * (end[1] - start[1])
        u = (y1 - (y1c - hw1)) / pix1
        v = (y2 - (y2c - hw2)) / pix2
        if not (0.0 <= u <= n1 and 0.0 <= v <= n2):
            out[k] = math.nan
            continue
        s = min(max(u - 0.5, 0.0), n1 - 1.0)
        t = min(max(v - 0.5, 0.0), n2 - 1.0)
        i0, j0 = min(int(math.floor(s)), n1 - 1), min(int(math.floor(t)), n2 - 1)
        i1, j1 = min(i0 + 1, n1 - 1), min(j0 + 1, n2 - 1)
        fs, ft = s - i0, t - j0
        out[k] = ((1 - ft) * ((1 - fs) * mu[j0, i0] + fs * mu[j0, i1])
                  + ft * ((1 - fs) * mu[j1, i0] + fs * mu[j1, i1]))
    return out


def histogram(mu: np.ndarray, lo: float, hi: float, nbins: int) -> np.ndarray:
    """Counts of log10(mu): [0] mu <= 0 or log10(mu) < lo, [1 + b] the bin
    [lo + b w, lo + (b + 1) w), w = (hi - lo) / nbins, [nbins + 1] at or above
    hi or NaN; a value's bin is floor((log10(mu) - lo) nbins / (hi - lo))."""
    out = np.zeros(nbins + 2, np.int64)
    scale = nbins / (hi - lo)
    for m in np.asarray(mu, np.float64).ravel():
        if math.isnan(m):
            out[nbins + 1] += 1
        elif m <= 0:
            out[0] += 1
        else:
            x = (math.log10(m) - lo) * scale
            out[0 if x < 0 else (nbins + 1 if x >= nbins else 1 + int(x))] += 1
    return out

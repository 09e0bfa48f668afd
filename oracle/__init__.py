"""FP64 CPU oracle for adaptive image ray-tracing (Parkin 2010).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use this package; the product path (the HIP library and its
binding) never imports it.  It shares no code with the HIP path; the two only
share the seeded input generators.

The arithmetic lives in air_oracle.c (built to liboracle.so by build.py);
this module marshals numpy arrays.  cnn.py holds the FP64 reference CNN.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

EXIST, TESTED, FLAGGED, BALANCE, REFINED = 1, 2, 4, 8, 16
MAXB = 1024


class _Grid(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bs", C.c_int32), ("max_level", C.c_int32), ("n_blocks", C.c_int32),
                ("blevel", C.c_void_p), ("bcoord", C.c_void_p), ("bchild", C.c_void_p)]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_bands", C.c_int32), ("rho", C.c_void_p), ("emis", C.c_void_p),
                ("kappa", C.c_void_p), ("temp", C.c_void_p), ("band", C.c_void_p)]


class _View(C.Structure):
    _fields_ = [("dir", C.c_double * 3), ("up", C.c_double * 3), ("center", C.c_double * 3),
                ("width", C.c_double)]


class _Ray(C.Structure):
    _fields_ = [("I", C.c_double * MAXB), ("N", C.c_double), ("rho_min", C.c_double), ("rho_max", C.c_double),
                ("lmax", C.c_int32), ("nvis", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        _lib.orc_trace.argtypes = [vp, vp, vp, vp, vp]
        _lib.orc_view_basis.argtypes = [vp, vp, vp, vp]
        _lib.orc_pixel_center.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp]
        _lib.orc_trace_pixels.argtypes = [vp, vp, vp, C.c_int, C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_render_fixed.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp, vp, vp, vp]
        _lib.orc_xi.argtypes = [vp, C.c_int, C.c_int]
        _lib.orc_xi.restype = C.c_double
        _lib.orc_air.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_double, C.c_double, vp, vp,
                                 vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_air.restype = C.c_int64
        _lib.orc_paint_leaves.argtypes = [C.c_int, C.c_int, vp, vp, vp]
        _lib.orc_superres.argtypes = [C.c_int, C.c_int, vp, vp, vp]
        _lib.orc_leaf_flux.argtypes = [C.c_int, C.c_int, C.c_double, vp, vp]
        _lib.orc_leaf_flux.restype = C.c_double
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_set_threads.restype = None
        _lib.orc_xi_sens.argtypes = [C.c_int64, vp, vp, vp, C.c_double, vp, vp]
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Keep:
    """Holds the ctypes structs and the arrays they point at."""

    def __init__(self, grid, field):
        self.arrs = []
        g = _Grid()
        g.kind = grid.kind
        g.n[:] = list(grid.n)
        g.lo[:] = list(grid.lo)
        g.hi[:] = list(grid.hi)
        g.bs = grid.bs
        g.max_level = grid.max_level
        g.n_blocks = grid.n_blocks
        if grid.kind == 1:
            for name in ("block_level", "block_coord", "block_child"):
                self.arrs.append(np.ascontiguousarray(getattr(grid, name), dtype=np.int32))
            g.blevel, g.bcoord, g.bchild = (a.ctypes.data for a in self.arrs[-3:])
        self.g = g
        f = _Field()
        f.kind = field.kind
        f.n_bands = field.n_bands
        for name in ("rho", "emis", "kappa", "temp"):
            a = getattr(field, name)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
                self.arrs.append(a)
                setattr(f, name, a.ctypes.data)
        if field.bands is not None:
            b = np.ascontiguousarray(field.bands, dtype=np.float64)
            self.arrs.append(b)
            f.band = b.ctypes.data
        self.f = f

    @property
    def gp(self):
        return C.addressof(self.g)

    @property
    def fp(self):
        return C.addressof(self.f)


def _view(v) -> _View:
    s = _View()
    s.dir[:] = list(v.dir)
    s.up[:] = list(v.up)
    s.center[:] = list(v.center)
    s.width = float(v.width)
    return s


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops."""
    lib().orc_set_threads(int(n))


def trace(grid, field, origin, direction) -> Dict:
    """Exact integral along one ray x(t) = origin + t*direction."""
    k = _Keep(grid, field)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    d = np.ascontiguousarray(direction, dtype=np.float64)
    r = _Ray()
    lib().orc_trace(k.gp, k.fp, o.ctypes.data, d.ctypes.data, C.addressof(r))
    nb = field.n_bands
    return dict(I=np.array(r.I[:nb]), N=r.N, lmax=r.lmax, nvis=r.nvis, rho_min=r.rho_min, rho_max=r.rho_max)


def view_basis(view):
    v = _view(view)
    d, eu, ev = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_view_basis(C.addressof(v), d.ctypes.data, eu.ctypes.data, ev.ctypes.data)
    return d, eu, ev


def pixel_center(view, N0, L, i, j):
    v = _view(view)
    c = np.zeros(3)
    lib().orc_pixel_center(C.addressof(v), N0, L, i, j, c.ctypes.data)
    return c


def trace_pixels(grid, field, view, N0, L, i, j) -> Dict:
    """Trace individual pixels (L[k], i[k], j[k])."""
    L = np.ascontiguousarray(L, dtype=np.int32)
    i = np.ascontiguousarray(i, dtype=np.int32)
    j = np.ascontiguousarray(j, dtype=np.int32)
    n = L.shape[0]
    nb = field.n_bands
    I = np.zeros((nb, n))
    N = np.zeros(n)
    lm = np.zeros(n, dtype=np.int32)
    nv = np.zeros(n, dtype=np.int32)
    rmin = np.zeros(n)
    rmax = np.zeros(n)
    k = _Keep(grid, field)
    v = _view(view)
    lib().orc_trace_pixels(k.gp, k.fp, C.addressof(v), N0, n, L.ctypes.data, i.ctypes.data, j.ctypes.data,
                           I.ctypes.data, N.ctypes.data, lm.ctypes.data, nv.ctypes.data, rmin.ctypes.data,
                           rmax.ctypes.data)
    return dict(I=I, N=N, lmax=lm, nvis=nv, rho_min=rmin, rho_max=rmax)


def render_fixed(grid, field, view, N0, L) -> Dict:
    """Fixed-resolution image at level L: arrays [R, R] indexed [j, i]."""
    R = N0 << L
    nb = field.n_bands
    I = np.zeros((nb, R, R))
    N = np.zeros((R, R))
    lm = np.zeros((R, R), dtype=np.int32)
    nv = np.zeros((R, R), dtype=np.int32)
    k = _Keep(grid, field)
    v = _view(view)
    lib().orc_render_fixed(k.gp, k.fp, C.addressof(v), N0, L, I.ctypes.data, N.ctypes.data, lm.ctypes.data,
                           nv.ctypes.data)
    return dict(I=I, N=N, lmax=lm, nvis=nv)


def xi(p, hx=True, hy=True) -> float:
    """Truncation-error estimate of a 3x3 stencil p[b+1][a+1] (a along u)."""
    a = np.ascontiguousarray(p, dtype=np.float64).reshape(9)
    return float(lib().orc_xi(a.ctypes.data, int(bool(hx)), int(bool(hy))))


@dataclasses.dataclass
class Tree:
    """Oracle AIR result: dense per-level arrays, row-major [j, i]."""

    N0: int
    Lmax: int
    nodes: int
    counts: np.ndarray
    state: List[np.ndarray]
    xiI: List[np.ndarray]
    xiN: List[np.ndarray]
    I: List[np.ndarray]  # [n_bands, R, R] per level
    N: List[np.ndarray]
    lmax: List[np.ndarray]
    nvis: List[np.ndarray]
    flat_state: np.ndarray
    flat_I: np.ndarray
    flat_N: np.ndarray

    def leaves(self, L):
        s = self.state[L]
        return (s & EXIST).astype(bool) & ~(s & REFINED).astype(bool)


def air(grid, field, view, N0, Lmax, xi_crit_I=0.5, xi_crit_N=2.0, band_w=None, force_flags=None,
        want_rho_range=False, values=None) -> Tree:
    """Plain AIR for one view (level-synchronous, 2:1 closure).

    force_flags (flat, one byte per position of the concatenated level
    rasters) replaces the criterion's decision at every tested node; then no
    ray is traced and the node values are those given in values = (I [total]
    or [n_bands, total], N [total]) (zeros if None): the criterion is still
    evaluated on them, with the tree as it stands when each level is tested,
    so xiI / xiN are the estimates of those values on the forced tree."""
    sizes = [(N0 << L) ** 2 for L in range(Lmax + 1)]
    total = int(sum(sizes))
    nb = field.n_bands if field is not None else 1
    state = np.zeros(total, dtype=np.uint8)
    xiI = np.zeros(total)
    xiN = np.zeros(total)
    I = np.zeros((nb, total))
    N = np.zeros(total)
    if values is not None:
        if force_flags is None:
            raise ValueError("values are only used with force_flags (no ray is traced then)")
        I[...] = np.asarray(values[0], dtype=np.float64).reshape(nb, total)
        N[...] = np.asarray(values[1], dtype=np.float64).reshape(total)
    lm = np.full(total, -1, dtype=np.int32)
    nv = np.zeros(total, dtype=np.int32)
    rmin = np.zeros(total) if want_rho_range else None
    rmax = np.zeros(total) if want_rho_range else None
    counts = np.zeros(Lmax + 1, dtype=np.int64)
    born = np.zeros(total, dtype=np.int8)
    w = None if band_w is None else np.ascontiguousarray(band_w, dtype=np.float64)
    ff = None if force_flags is None else np.ascontiguousarray(force_flags, dtype=np.uint8)
    v = _view(view)
    if grid is not None:
        k = _Keep(grid, field)
        gp, fp = k.gp, k.fp
    else:
        gp = fp = None
    n = lib().orc_air(gp, fp, C.addressof(v), N0, Lmax, float(xi_crit_I), float(xi_crit_N), _p(w), _p(ff),
                      state.ctypes.data, xiI.ctypes.data, xiN.ctypes.data, I.ctypes.data, N.ctypes.data,
                      lm.ctypes.data, nv.ctypes.data, _p(rmin), _p(rmax), counts.ctypes.data, born.ctypes.data)
    if n < 0:
        raise RuntimeError(f"oracle AIR failed: {n}")
    offs = np.concatenate([[0], np.cumsum(sizes)])

    def split(a):
        return [a[..., offs[L]:offs[L + 1]].reshape(a.shape[:-1] + (N0 << L, N0 << L)) for L in range(Lmax + 1)]

    t = Tree(N0, Lmax, int(n), counts, split(state), split(xiI), split(xiN), split(I), split(N), split(lm),
             split(nv), state, I, N)
    t.born = split(born)
    if want_rho_range:
        t.rmin = split(rmin)
        t.rmax = split(rmax)
    return t


def paint_leaves(tree: Tree, vals_flat: np.ndarray) -> np.ndarray:
    R = tree.N0 << tree.Lmax
    out = np.zeros((R, R))
    v = np.ascontiguousarray(vals_flat, dtype=np.float64)
    lib().orc_paint_leaves(tree.N0, tree.Lmax, tree.flat_state.ctypes.data, v.ctypes.data, out.ctypes.data)
    return out


def superres(tree: Tree, vals_flat: np.ndarray) -> np.ndarray:
    """The interpolated finest raster (section 2 step vi super-resolution,
    reading in air_oracle.c: orc_superres)."""
    R = tree.N0 << tree.Lmax
    out = np.zeros((R, R))
    v = np.ascontiguousarray(vals_flat, dtype=np.float64)
    lib().orc_superres(tree.N0, tree.Lmax, tree.flat_state.ctypes.data, v.ctypes.data, out.ctypes.data)
    return out


def leaf_flux(tree: Tree, width: float, vals_flat: np.ndarray) -> float:
    v = np.ascontiguousarray(vals_flat, dtype=np.float64)
    return float(lib().orc_leaf_flux(tree.N0, tree.Lmax, float(width), tree.flat_state.ctypes.data,
                                     v.ctypes.data))


def xi_sensitivity(stencils: np.ndarray, hx: np.ndarray, hy: np.ndarray, delta: float):
    """(xi, bound): xi of each 3x3 stencil and the first-order bound on its
    change when every input moves by relative delta."""
    p = np.ascontiguousarray(stencils, dtype=np.float64).reshape(-1, 9)
    n = p.shape[0]
    hx = np.ascontiguousarray(hx, dtype=np.int32)
    hy = np.ascontiguousarray(hy, dtype=np.int32)
    xi_ = np.zeros(n)
    out = np.zeros(n)
    lib().orc_xi_sens(n, p.ctypes.data, hx.ctypes.data, hy.ctypes.data, float(delta), xi_.ctypes.data,
                      out.ctypes.data)
    return xi_, out


def stencils(tree: Tree, L: int, which: str = "I", band_w=None):
    """3x3 level-L stencils of every tested node of the oracle tree (the
    covering level-(L-1) value where a level-L neighbour does not exist),
    with the image-edge flags.  Returns (positions (j, i), p[n, 9], hx, hy)."""
    R = tree.N0 << L
    st = tree.state[L]
    js, is_ = np.nonzero((st & TESTED) > 0)
    if which == "N":
        val = [tree.N[l] for l in range(tree.Lmax + 1)]
    else:
        nb = tree.I[0].shape[0]
        w = np.ones(nb) if band_w is None else np.asarray(band_w, dtype=float)[:nb]
        val = [np.tensordot(w, tree.I[l], axes=1) for l in range(tree.Lmax + 1)]
    p = np.zeros((len(js), 9))
    for b in (-1, 0, 1):
        for a in (-1, 0, 1):
            qj, qi = js + b, is_ + a
            ok = (qi >= 0) & (qj >= 0) & (qi < R) & (qj < R)
            qjc, qic = np.clip(qj, 0, R - 1), np.clip(qi, 0, R - 1)
            # existence when level L was tested: created before step L
            ex = ((st[qjc, qic] & EXIST) > 0) & (tree.born[L][qjc, qic] < L)
            v = np.where(ex, val[L][qjc, qic], val[L - 1][qjc // 2, qic // 2] if L > 0 else 0.0)
            p[:, (b + 1) * 3 + (a + 1)] = np.where(ok, v, 0.0)
    hx = ((is_ > 0) & (is_ < R - 1)).astype(np.int32)
    hy = ((js > 0) & (js < R - 1)).astype(np.int32)
    return (js, is_), p, hx, hy

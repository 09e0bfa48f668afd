"""Seeded synthetic inputs for AIR: simulation grids, fields and views.

This module holds input generation only -- no step of the rendering method
(no ray geometry, no integration, no refinement test).  Both the HIP path
and the FP64 oracle consume what it produces, so it must stay free of the
method's arithmetic.  It imports numpy only.

Field arrays are float32, shape (nz, ny, nx) C-ordered, so the flat index is
x + nx*(y + ny*z) ("x fastest").  Block-AMR data is block-major: block b
holds bs^3 cells starting at b*bs^3, x fastest inside the block.

Workloads (synthetic stand-ins; the paper's FLASH grid and MEKAL tables
are not available):
  * gaussian  -- uniform 64^3 unit box, rho = rho0 exp(-r^2/2 sigma^2) + 1e-3,
                 j = rho^2, kappa = 0.5 rho (the small FP64 case);
  * winds2    -- uniform n^3 unit box, two wind sources rho ~ 1/r^2 with a
                 seeded mass-loss ratio and phase, a shocked shell a few
                 cells thick on the ram-pressure balance surface (density x4,
                 T x10), j = rho^2 T^0.5, kappa = kappa0 rho T^-1.5;
  * winds3    -- three sources and their pairwise shells (the large case);
  * amr_winds -- block-AMR hierarchy over the winds2 field, ratio 2,
                 refined near the shell and the sources;
  * ring      -- the paper's section-3 ring test (Eq. 1) with a
                 PARAMESH-like block hierarchy.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

GRID_UNIFORM = 0
GRID_AMR = 1
FIELD_RHO_J_KAPPA = 0
FIELD_RHO_T = 1


@dataclasses.dataclass
class Grid:
    """Simulation grid.  Uniform: n = cells per axis.  AMR: n = base blocks
    per axis, bs = cells per block edge, levels 0..max_level, block tables
    (level, coord at its own level, first child or -1; 8 children stored
    consecutively with child offset cx + 2cy + 4cz)."""

    kind: int
    n: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bs: int = 1
    max_level: int = 0
    block_level: Optional[np.ndarray] = None
    block_coord: Optional[np.ndarray] = None
    block_child: Optional[np.ndarray] = None

    @property
    def n_blocks(self) -> int:
        return 0 if self.block_level is None else int(self.block_level.shape[0])

    @property
    def n_cells(self) -> int:
        if self.kind == GRID_UNIFORM:
            return int(np.prod(self.n))
        return self.n_blocks * self.bs ** 3


@dataclasses.dataclass
class Field:
    """Cell data.  kind 0: rho, emis, kappa (one band).  kind 1: rho, temp and
    bands [n_bands][3] = (kappa0, s, q) with kappa_b = kappa0 rho T^-s and
    j_b = rho^2 T^q.  kind 2 (spectral bins): rho, temp and bands
    [n_bins][5] = (kappa0, s, e0, q, E) with kappa_b = kappa0 rho T^-s and
    j_b = e0 rho^2 T^q exp(-E / T)."""

    kind: int
    rho: np.ndarray
    emis: Optional[np.ndarray] = None
    kappa: Optional[np.ndarray] = None
    temp: Optional[np.ndarray] = None
    bands: Optional[np.ndarray] = None

    @property
    def n_bands(self) -> int:
        return 1 if self.kind == FIELD_RHO_J_KAPPA else int(self.bands.shape[0])


@dataclasses.dataclass
class View:
    """Orthographic view: looking direction, up hint, image centre, width."""

    dir: tuple
    up: tuple
    center: tuple
    width: float


# ----------------------------------------------------------------- helpers
def _centres(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    h = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * h


def view_for(direction: Sequence[float], center=(0.5, 0.5, 0.5), width: float = math.sqrt(3.0)) -> View:
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    up = (0.0, 1.0, 0.0)
    if abs(float(d[1])) > 0.99:
        up = (0.0, 0.0, 1.0)
    return View(tuple(float(x) for x in d), up, tuple(center), float(width))


# ------------------------------------------------------------ the workloads
def gaussian(n: int = 64, rho0: float = 1.0, sigma: float = 0.1, background: float = 1e-3,
             kappa_scale: float = 0.5, thin: bool = False) -> (Grid, Field):
    """Centred Gaussian blob on a uniform n^3 unit box (cell-centre sampling)."""
    c = _centres(n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    rho = rho0 * np.exp(-r2 / (2.0 * sigma * sigma)) + background
    emis = rho * rho
    kappa = np.zeros_like(rho) if thin else kappa_scale * rho
    g = Grid(GRID_UNIFORM, (n, n, n))
    f = Field(FIELD_RHO_J_KAPPA, rho.astype(np.float32), emis.astype(np.float32), kappa.astype(np.float32))
    return g, f


def gaussian_view() -> View:
    """+z looking direction, up = +y, unit width image centred on the box."""
    return View((0.0, 0.0, 1.0), (0.0, 1.0, 0.0), (0.5, 0.5, 0.5), 1.0)


def _winds_params(seed: int):
    rng = np.random.default_rng(seed)
    eta = float(rng.uniform(0.1, 1.0))
    phi = float(rng.uniform(0.0, 2.0 * math.pi))
    return eta, phi


def winds_rho_t(points: np.ndarray, sources: np.ndarray, etas: np.ndarray, h: float,
                r0: float = 0.05, shell_cells: float = 1.5):
    """Density and temperature of overlapping 1/r^2 winds at points (..., 3).
    Wind k has density etas[k] (r0/r_k)^2 with r_k softened to >= 2h.  Where
    the two strongest winds balance (r_l = sqrt(eta_l/eta_k) r_k) within
    shell_cells cells the gas is shocked: density x4, T x10."""
    pts = np.asarray(points, dtype=np.float64)
    dk = []
    for s in sources:
        dv = pts - s
        r = np.sqrt(np.sum(dv * dv, axis=-1))
        dk.append((np.maximum(r, 2.0 * h), dv, r))
    dens = np.stack([etas[k] * (r0 / dk[k][0]) ** 2 for k in range(len(sources))], axis=0)
    rho = dens.max(axis=0)
    temp = np.ones_like(rho)
    if len(sources) >= 2:
        order = np.argsort(-dens, axis=0)
        k1, k2 = order[0], order[1]
        shell = np.zeros(rho.shape, dtype=bool)
        for a in range(len(sources)):
            for b in range(len(sources)):
                if a == b:
                    continue
                m = (k1 == a) & (k2 == b)
                if not np.any(m):
                    continue
                ra, dva, rra = dk[a]
                rb, dvb, rrb = dk[b]
                q = math.sqrt(etas[b] / etas[a])  # balance: r_b = q r_a
                gfun = rrb - q * rra
                with np.errstate(invalid="ignore", divide="ignore"):
                    grad = dvb / np.maximum(rrb, 1e-300)[..., None] - q * dva / np.maximum(rra, 1e-300)[..., None]
                gn = np.sqrt(np.sum(grad * grad, axis=-1))
                dist = np.abs(gfun) / np.maximum(gn, 1e-12)
                shell |= m & (dist <= shell_cells * h)
        rho = np.where(shell, 4.0 * rho, rho)
        temp = np.where(shell, 10.0, temp)
    return rho, temp


def winds2_sources(seed: int):
    eta, phi = _winds_params(seed)
    c = np.array([0.5, 0.5, 0.5])
    off = 0.2 * np.array([math.cos(phi), math.sin(phi), 0.0])
    return np.stack([c + off, c - off]), np.array([1.0, eta])


def winds2(seed: int = 0, n: int = 256, kappa0: float = 1.0, kind: int = FIELD_RHO_J_KAPPA,
           bands: Optional[np.ndarray] = None) -> (Grid, Field):
    """Colliding-winds-like field on a uniform n^3 unit box."""
    src, etas = winds2_sources(seed)
    return _winds_uniform(src, etas, n, kappa0, kind, bands)


def winds3_sources(seed: int):
    rng = np.random.default_rng(10_000 + seed)
    c = np.array([0.5, 0.5, 0.5])
    nrm = rng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    a = np.cross(nrm, [1.0, 0.0, 0.0])
    if np.linalg.norm(a) < 0.1:
        a = np.cross(nrm, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(nrm, a)
    ph = rng.uniform(0, 2 * math.pi)
    src = np.stack([c + 0.25 * (math.cos(ph + 2 * math.pi * k / 3) * a + math.sin(ph + 2 * math.pi * k / 3) * b)
                    for k in range(3)])
    etas = np.concatenate([[1.0], rng.uniform(0.1, 1.0, size=2)])
    return src, etas


def winds3(seed: int = 0, n: int = 512, kappa0: float = 1.0, kind: int = FIELD_RHO_T,
           bands: Optional[np.ndarray] = None) -> (Grid, Field):
    """Three wind sources with their pairwise shells on a uniform n^3 box."""
    src, etas = winds3_sources(seed)
    return _winds_uniform(src, etas, n, kappa0, kind, bands)


def _winds_uniform(src, etas, n, kappa0, kind, bands):
    h = 1.0 / n
    c = _centres(n)
    rho = np.empty((n, n, n), dtype=np.float32)
    temp = np.empty((n, n, n), dtype=np.float32)
    y, x = np.meshgrid(c, c, indexing="ij")
    for k in range(n):  # one z slab at a time keeps the temporaries small
        pts = np.stack([x, y, np.full_like(x, c[k])], axis=-1)
        r, t = winds_rho_t(pts, src, etas, h)
        rho[k] = r
        temp[k] = t
    g = Grid(GRID_UNIFORM, (n, n, n))
    if kind == FIELD_RHO_J_KAPPA:
        r64 = rho.astype(np.float64)
        t64 = temp.astype(np.float64)
        emis = (r64 * r64 * np.sqrt(t64)).astype(np.float32)
        kap = (kappa0 * r64 * t64 ** -1.5).astype(np.float32)
        return g, Field(FIELD_RHO_J_KAPPA, rho, emis, kap)
    if bands is None:
        bands = default_bands(8)
    return g, Field(FIELD_RHO_T, rho, temp=temp, bands=np.asarray(bands, dtype=np.float64))


def default_bands(n_bands: int = 8) -> np.ndarray:
    """(kappa0_b, s_b, q_b): kappa0 = 10^(-1 + 2b/7), s = 1 + b/7, q = 0.5."""
    b = np.arange(8, dtype=np.float64)
    tab = np.stack([10.0 ** (-1.0 + 2.0 * b / 7.0), 1.0 + b / 7.0, np.full(8, 0.5)], axis=1)
    if n_bands == 8:
        return tab
    if n_bands == 4:
        return tab[[0, 2, 5, 7]]
    return tab[:n_bands]


FIELD_SPECTRAL = 2


def spectral_bins(n_bins: int, e_lo: float = 0.1, e_hi: float = 20.0, band=(1.0, 10.0)):
    """A synthetic spectrum table standing in for the paper's MEKAL tables
    (missing): n_bins log-spaced bin energies E in [e_lo, e_hi] (the field's
    temperature units; the wind is at 1, the shocked shell at 10), opacity
    kappa0 = 0.5 / (1 + E)^2 with s = 1.5, emission e0 = 1, q = -0.5 (a
    thermal-bremsstrahlung-like shape), and broadband weights equal to the
    bin widths for E in `band` (the analogue of the 1-10 keV band), else 0.
    Returns (table [n_bins][5] float64, weights [n_bins] float32)."""
    edges = np.geomspace(e_lo, e_hi, n_bins + 1)
    E = np.sqrt(edges[:-1] * edges[1:])
    tab = np.stack([0.5 / (1.0 + E) ** 2, np.full(n_bins, 1.5), np.ones(n_bins), np.full(n_bins, -0.5), E], axis=1)
    w = np.where((E >= band[0]) & (E <= band[1]), np.diff(edges), 0.0).astype(np.float32)
    return tab, w


def winds2_views() -> List[View]:
    """The three views of the uniform-winds workload: +z, +x, (1,1,1)/sqrt3."""
    return [view_for((0, 0, 1)), view_for((1, 0, 0)), view_for((1, 1, 1))]


def isotropic_views(n: int, seed: int = 3, width: float = math.sqrt(3.0)) -> List[View]:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        v = rng.normal(size=3)
        out.append(view_for(v / np.linalg.norm(v), width=width))
    return out


# ----------------------------------------------------------------- block AMR
def amr_from_predicate(base_blocks: int, bs: int, max_level: int, refine_pred, lo=(0.0, 0.0, 0.0),
                       hi=(1.0, 1.0, 1.0)) -> Grid:
    """Build a block hierarchy: base_blocks^3 level-0 blocks of bs^3 cells;
    a block at level l < max_level is split into 8 when refine_pred(l, lo_b,
    size_b) is true.  Children of a block are stored consecutively."""
    levels, coords, child = [], [], []
    nb0 = base_blocks
    for bz in range(nb0):
        for by in range(nb0):
            for bx in range(nb0):
                levels.append(0)
                coords.append((bx, by, bz))
                child.append(-1)
    size0 = (hi[0] - lo[0]) / nb0
    q = list(range(len(levels)))
    head = 0
    while head < len(q):
        b = q[head]
        head += 1
        l = levels[b]
        if l >= max_level:
            continue
        sz = size0 / (1 << l)
        blo = tuple(lo[a] + coords[b][a] * sz for a in range(3))
        if not refine_pred(l, blo, sz):
            continue
        first = len(levels)
        child[b] = first
        for k in range(8):
            cx, cy, cz = k & 1, (k >> 1) & 1, (k >> 2) & 1
            levels.append(l + 1)
            coords.append((2 * coords[b][0] + cx, 2 * coords[b][1] + cy, 2 * coords[b][2] + cz))
            child.append(-1)
            q.append(first + k)
    return Grid(GRID_AMR, (nb0, nb0, nb0), tuple(lo), tuple(hi), bs, max_level,
                np.asarray(levels, dtype=np.int32), np.asarray(coords, dtype=np.int32).reshape(-1, 3),
                np.asarray(child, dtype=np.int32))


def amr_cell_centres(grid: Grid) -> np.ndarray:
    """(n_blocks*bs^3, 3) cell centres in the block-major data order."""
    bs = grid.bs
    size0 = (grid.hi[0] - grid.lo[0]) / grid.n[0]
    ar = (np.arange(bs) + 0.5) / bs
    cz, cy, cx = np.meshgrid(ar, ar, ar, indexing="ij")
    local = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    out = np.empty((grid.n_blocks * bs ** 3, 3))
    sz = size0 / (1 << grid.block_level.astype(np.int64))
    lo = np.asarray(grid.lo)
    for b in range(grid.n_blocks):
        out[b * bs ** 3:(b + 1) * bs ** 3] = lo + (grid.block_coord[b] + local) * sz[b]
    return out


def amr_winds(seed: int = 0, base_cells: int = 128, bs: int = 16, max_level: int = 2,
              frac=(0.10, 0.03), kind: int = FIELD_RHO_T, bands=None, kappa0: float = 1.0):
    """Block AMR over the two-wind field: a block whose centre lies within a
    distance of the shell surface or a source is refined; the distances are
    bisected so the level-1 and level-2 blocks cover about frac[0] and
    frac[1] of the volume."""
    src, etas = winds2_sources(seed)
    nb0 = base_cells // bs
    q = math.sqrt(etas[1] / etas[0])

    def surf_dist(p):
        p = np.asarray(p, dtype=np.float64)
        r1 = np.linalg.norm(p - src[0], axis=-1)
        r2 = np.linalg.norm(p - src[1], axis=-1)
        g = np.abs(r2 - q * r1)
        return np.minimum(np.minimum(g, r1), r2)

    def build(d1, d2):
        ds = (d1, d2, 0.0)

        def pred(l, blo, sz):
            cc = np.asarray(blo) + 0.5 * sz
            return surf_dist(cc) < ds[l]
        return amr_from_predicate(nb0, bs, max_level, pred)

    def vol_frac(grid, lev):
        sz = 1.0 / (grid.n[0] << lev)
        return float(np.sum(grid.block_level == lev)) * sz ** 3

    lo_d, hi_d = 0.0, 0.5
    for _ in range(20):  # level-1 coverage
        mid = 0.5 * (lo_d + hi_d)
        if vol_frac(build(mid, 0.0), 1) > frac[0]:
            hi_d = mid
        else:
            lo_d = mid
    d1 = 0.5 * (lo_d + hi_d)
    lo_d, hi_d = 0.0, d1
    for _ in range(20):
        mid = 0.5 * (lo_d + hi_d)
        if max_level < 2 or vol_frac(build(d1, mid), 2) > frac[1]:
            hi_d = mid
        else:
            lo_d = mid
    grid = build(d1, 0.5 * (lo_d + hi_d))
    pts = amr_cell_centres(grid)
    hfin = 1.0 / (base_cells << max_level)
    rho, temp = winds_rho_t(pts, src, etas, hfin * 2)
    rho = rho.astype(np.float32)
    temp = temp.astype(np.float32)
    if kind == FIELD_RHO_J_KAPPA:
        r64, t64 = rho.astype(np.float64), temp.astype(np.float64)
        return grid, Field(FIELD_RHO_J_KAPPA, rho, (r64 * r64 * np.sqrt(t64)).astype(np.float32),
                           (kappa0 * r64 * t64 ** -1.5).astype(np.float32))
    if bands is None:
        bands = default_bands(8)
    return grid, Field(FIELD_RHO_T, rho, temp=temp, bands=np.asarray(bands, dtype=np.float64))


def uniform_as_amr(grid: Grid, field: Field, bs: int) -> (Grid, Field):
    """Express a uniform grid as a single-level block hierarchy (same data)."""
    n = grid.n[0]
    assert grid.n == (n, n, n) and n % bs == 0
    nb0 = n // bs
    g = amr_from_predicate(nb0, bs, 0, lambda *a: False, grid.lo, grid.hi)

    def reblock(a):
        if a is None:
            return None
        a = a.reshape(nb0, bs, nb0, bs, nb0, bs)  # z, cz, y, cy, x, cx
        return np.ascontiguousarray(a.transpose(0, 2, 4, 1, 3, 5)).reshape(-1)

    f = Field(field.kind, reblock(field.rho), reblock(field.emis), reblock(field.kappa), reblock(field.temp),
              field.bands)
    return g, f


# ------------------------------------------------------------ the ring test
def ring(base_blocks: int = 4, bs: int = 8, max_level: int = 4, beta: float = 2.5e9, r_inner: float = 3.5e17,
         r_outer: float = 4e17, width: float = 1e17) -> (Grid, Field):
    """Section-3 ring (Eq. 1) in scaled units: length unit 1e17 cm, density
    unit 1e-26 g/cm^3 (cgs rho^2 underflows float32).  rho = beta / r_yz^2
    for r_i <= r_yz <= r_o and |x| < w/2, else 1e-25 g/cm^3; T = 1e8 K
    inside, 1e4 K outside; box +-5e17 cm.  beta is in g/cm, the radii and
    the width in cm (the defaults are the section's).  The block hierarchy
    is refined where a block straddles the ring surface.  Emission is rho^2
    inside the ring and 0 outside (1-10 keV emission of 1e4 K gas is
    negligible); no absorption.  Returned as a one-band rho/j/kappa field."""
    lu, du = 1e17, 1e-26
    L = 5e17 / lu
    w, ri, ro = width / lu, r_inner / lu, r_outer / lu
    beta_s = beta / (lu * lu) / du  # rho[du] = beta_s / r[lu]^2
    lo, hi = (-L, -L, -L), (L, L, L)

    def in_ring(p):
        p = np.asarray(p)
        ryz = np.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2)
        return (ryz >= ri) & (ryz <= ro) & (np.abs(p[..., 0]) < 0.5 * w)

    def pred(l, blo, sz):
        s = (np.arange(5) / 4.0) * sz
        zz, yy, xx = np.meshgrid(s, s, s, indexing="ij")
        pts = np.stack([blo[0] + xx, blo[1] + yy, blo[2] + zz], axis=-1)
        m = in_ring(pts)
        return bool(m.any() and not m.all())

    grid = amr_from_predicate(base_blocks, bs, max_level, pred, lo, hi)
    pts = amr_cell_centres(grid)
    m = in_ring(pts)
    ryz2 = pts[:, 1] ** 2 + pts[:, 2] ** 2
    rho = np.where(m, beta_s / np.maximum(ryz2, 1e-300), 1e-25 / du)
    emis = np.where(m, rho * rho, 0.0)
    f = Field(FIELD_RHO_J_KAPPA, rho.astype(np.float32), emis.astype(np.float32),
              np.zeros_like(rho, dtype=np.float32))
    return grid, f


def ring_view() -> View:
    """Face-on: looking along +x, up = +z, so (u, v) = (y, z) (Fig. 1 note)."""
    return View((1.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 0.0, 0.0), 10.0)


def ring_geometry(k: int) -> dict:
    """Ring k of a family for training and evaluating the depth proposal:
    k = 0 is the section-3 ring; k > 0 draws the inner radius (2.5-4.0e17
    cm), the radial thickness (0.3-1.0e17 cm, outer radius at most 4.6e17
    cm) and the width along the axis (0.5-1.5e17 cm) from default_rng(k).
    Keyword arguments of ring()."""
    if k == 0:
        return {}
    rng = np.random.default_rng(1000 + k)
    ri = rng.uniform(2.5e17, 4.0e17)
    ro = min(ri + rng.uniform(0.3e17, 1.0e17), 4.6e17)
    return dict(r_inner=float(ri), r_outer=float(ro), width=float(rng.uniform(0.5e17, 1.5e17)))


def ring_family_view(seed: int) -> View:
    """A seeded view of the ring family: the looking direction within 70
    degrees of face-on (+x), uniform in solid angle, a random roll of the
    up vector, image width 10 (the box face)."""
    rng = np.random.default_rng(seed)
    cos_max = math.cos(math.radians(70.0))
    ct = rng.uniform(cos_max, 1.0)
    st, ph = math.sqrt(max(0.0, 1.0 - ct * ct)), rng.uniform(0.0, 2.0 * math.pi)
    d = np.array([ct, st * math.cos(ph), st * math.sin(ph)])
    # roll: a random direction perpendicular to d
    a = rng.normal(size=3)
    up = a - np.dot(a, d) * d
    up = up / np.linalg.norm(up)
    return View(tuple(float(x) for x in d), tuple(float(x) for x in up), (0.0, 0.0, 0.0), 10.0)


# ------------------------------------------------- depth-proposal network
CNN_CHANNELS = (4, 32, 32, 32, 6)


def cnn_init(seed: int) -> np.ndarray:
    """Seeded He-normal initial parameters of the depth-proposal network,
    float32, laid out per layer as weights [cout][3][3][cin] then bias
    [cout] (biases zero)."""
    rng = np.random.default_rng(50_000 + seed)
    parts = []
    for l in range(4):
        cin, cout = CNN_CHANNELS[l], CNN_CHANNELS[l + 1]
        parts.append(rng.normal(size=cout * 9 * cin) * math.sqrt(2.0 / (9 * cin)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def winds_field_torch(src: np.ndarray, etas: np.ndarray, n: int, device, r0: float = 0.05,
                      shell_cells: float = 1.5, slab: int = 64):
    """winds_rho_t on the cell centres of the uniform n^3 unit box, evaluated
    with torch in float64 on `device` (a GPU makes the many-seed training
    sets cheap); returns float32 (rho, T) tensors [n, n, n], z slowest.  Same
    formulas and operation order as winds_rho_t; cells exactly on a shell's
    distance threshold or a density tie may round the other way."""
    import torch
    h = 1.0 / n
    c = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * h
    rho_out = torch.empty((n, n, n), dtype=torch.float32, device=device)
    t_out = torch.empty((n, n, n), dtype=torch.float32, device=device)
    y, x = torch.meshgrid(c, c, indexing="ij")
    S = torch.as_tensor(np.asarray(src, dtype=np.float64), device=device)
    K = len(src)
    for z0 in range(0, n, slab):
        z1 = min(n, z0 + slab)
        zz = c[z0:z1].view(-1, 1, 1).expand(-1, n, n)
        pts = torch.stack([x.expand(z1 - z0, n, n), y.expand(z1 - z0, n, n), zz], dim=-1)
        dk = []
        for k in range(K):
            dv = pts - S[k]
            r = torch.sqrt(torch.sum(dv * dv, dim=-1))
            dk.append((torch.clamp(r, min=2.0 * h), dv, r))
        dens = torch.stack([float(etas[k]) * (r0 / dk[k][0]) ** 2 for k in range(K)], dim=0)
        rho = dens.max(dim=0).values
        temp = torch.ones_like(rho)
        if K >= 2:
            order = torch.argsort(-dens, dim=0)
            k1, k2 = order[0], order[1]
            shell = torch.zeros(rho.shape, dtype=torch.bool, device=device)
            for a in range(K):
                for b in range(K):
                    if a == b:
                        continue
                    m = (k1 == a) & (k2 == b)
                    ra, dva, rra = dk[a]
                    rb, dvb, rrb = dk[b]
                    q = math.sqrt(etas[b] / etas[a])
                    gfun = rrb - q * rra
                    grad = dvb / torch.clamp(rrb, min=1e-300)[..., None] - q * dva / torch.clamp(rra, min=1e-300)[..., None]
                    gn = torch.sqrt(torch.sum(grad * grad, dim=-1))
                    dist = torch.abs(gfun) / torch.clamp(gn, min=1e-12)
                    shell |= m & (dist <= shell_cells * h)
            rho = torch.where(shell, 4.0 * rho, rho)
            temp = torch.where(shell, torch.full_like(temp, 10.0), temp)
        rho_out[z0:z1] = rho.to(torch.float32)
        t_out[z0:z1] = temp.to(torch.float32)
    return rho_out, t_out


def training_scene(seed: int):
    """One training sample of the depth proposal: the two-wind sources of
    `seed` (mass-loss ratio and phase) and a seeded isotropic view."""
    src, etas = winds2_sources(seed)
    rng = np.random.default_rng(20_000 + seed)
    d = rng.normal(size=3)
    return src, etas, view_for(d / np.linalg.norm(d))

"""Pins for the oracle's per-ray integral (section 2 step ii: one ray per
pixel integrating the column density and the formal radiative-transfer
solution) against closed forms and an independent brute force.

None of these re-types the oracle's method: the brute force finds cells by
intersecting every cell box with the ray (no plane merging, no midpoint
location) and composes the segments back to front; closed forms come from
the analytic solution of dI/ds = j - kappa I for constant coefficients."""
import math

import numpy as np
import pytest
from scipy.special import erf

from paper_1010_5534_amd import inputs


def _uniform(n, rho, j, kap, lo=(0, 0, 0), hi=(1, 1, 1)):
    g = inputs.Grid(inputs.GRID_UNIFORM, (n, n, n), tuple(map(float, lo)), tuple(map(float, hi)))
    shape = (n, n, n)
    f = inputs.Field(inputs.FIELD_RHO_J_KAPPA, np.full(shape, rho, np.float32), np.full(shape, j, np.float32),
                     np.full(shape, kap, np.float32))
    return g, f


def _chord_bisect(o, d, lo, hi):
    """Chord of a ray through an axis-aligned box by bracketing the inside
    interval numerically (independent of any slab formula)."""
    o, d = np.asarray(o, float), np.asarray(d, float)
    inside = lambda t: bool(np.all(o + t * d >= lo) and np.all(o + t * d <= hi))
    ts = np.linspace(-10, 10, 200001)
    pts = o[None, :] + ts[:, None] * d[None, :]
    m = np.all((pts >= lo) & (pts <= hi), axis=1)
    if not m.any():
        return 0.0
    k = np.nonzero(m)[0]

    def edge(a, b):  # a inside, b outside
        for _ in range(200):
            c = 0.5 * (a + b)
            if inside(c):
                a = c
            else:
                b = c
        return 0.5 * (a + b)

    t_in = edge(ts[k[0]], ts[k[0]] - (ts[1] - ts[0]))
    t_out = edge(ts[k[-1]], ts[k[-1]] + (ts[1] - ts[0]))
    return t_out - t_in


@pytest.mark.parametrize("o,d,chord", [
    ((0.3, 0.6, -2.0), (0, 0, 1), 1.0),
    ((0.5, 0.5, 0.5), (1, 1, 1), math.sqrt(3.0)),
    ((0.5, 0.5, 0.5), (1, -1, 0), math.sqrt(2.0)),
    ((0.25, -3.0, 0.7), (0, 1, 0), 1.0),
])
def test_uniform_box_closed_form(orc, o, d, chord):
    rho, j, kap = 0.75, 2.5, 1.25
    g, f = _uniform(8, rho, j, kap)
    r = orc.trace(g, f, o, d)
    dn = np.asarray(d, float) / np.linalg.norm(d)
    r2 = orc.trace(g, f, o, dn)
    # the direction is normalised before use: same answer either way
    assert r["N"] == pytest.approx(r2["N"], rel=1e-14)
    assert r["N"] == pytest.approx(rho * chord, rel=1e-13)
    assert r["I"][0] == pytest.approx(j / kap * (1 - math.exp(-kap * chord)), rel=1e-13)


def test_uniform_box_random_rays_bisection_chord(orc):
    rng = np.random.default_rng(1)
    rho, j, kap = 1.5, 0.5, 3.0
    lo, hi = np.array([-0.5, 0.0, 0.25]), np.array([0.5, 2.0, 1.25])
    g, f = _uniform(6, rho, j, kap, lo, hi)
    for _ in range(20):
        o = lo + rng.uniform(0, 1, 3) * (hi - lo)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        chord = _chord_bisect(o, d, lo, hi)
        r = orc.trace(g, f, o, d)
        assert r["N"] == pytest.approx(rho * chord, rel=1e-9)
        assert r["I"][0] == pytest.approx(j / kap * (1 - math.exp(-kap * chord)), rel=1e-9)


def test_miss_is_exact_zero(orc):
    g, f = _uniform(4, 1.0, 1.0, 1.0)
    for o, d in [((2, 2, 2), (0, 0, 1)), ((0.5, 0.5, 3), (1, 0, 0)), ((1.0, 0.5, 0.5), (0, 1, 0)),
                 ((0.5, 5.0, 0.5), (1, 1, 0))]:
        r = orc.trace(g, f, o, d)
        assert r["N"] == 0.0 and r["I"][0] == 0.0 and r["lmax"] == -1 and r["nvis"] == 0


def test_isothermal_slab(orc):
    """I = S (1 - exp(-kappa * dz/|d_z|)) for a source-function-S slab."""
    n = 16
    rho = np.zeros((n, n, n), np.float32)
    emis = np.zeros_like(rho)
    kap = np.zeros_like(rho)
    za, zb = 5, 11  # cells [5, 11): planes z = 5/16 .. 11/16
    rho[za:zb] = 2.0
    emis[za:zb] = 3.0
    kap[za:zb] = 1.75
    g = inputs.Grid(inputs.GRID_UNIFORM, (n, n, n))
    f = inputs.Field(inputs.FIELD_RHO_J_KAPPA, rho, emis, kap)
    rng = np.random.default_rng(7)
    for _ in range(25):
        d = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), 1.0])
        d /= np.linalg.norm(d)
        o = np.array([0.5, 0.5, 0.5]) + rng.uniform(-0.1, 0.1, 3)
        path = (zb - za) / n / abs(d[2])
        r = orc.trace(g, f, o, d)
        assert r["I"][0] == pytest.approx(3.0 / 1.75 * (1 - math.exp(-1.75 * path)), rel=1e-13)
        assert r["N"] == pytest.approx(2.0 * path, rel=1e-13)


def _gauss_line(s, b2, s0):
    """integral over z in [0,1] of exp(-(b^2 + (z-1/2)^2) / (2 s^2))"""
    return math.exp(-b2 / (2 * s * s)) * s * math.sqrt(2 * math.pi) * erf(0.5 / (s * math.sqrt(2)))


def test_gaussian_column_erf(orc):
    """Axis rays through cell-column centres of the 64^3 Gaussian: N and the
    optically thin I match the erf closed forms up to the midpoint rule."""
    n, sigma, bg = 64, 0.1, 1e-3
    g, f = inputs.gaussian(n=n, thin=True)
    for (ci, cj) in [(32, 32), (20, 40), (10, 50), (45, 31), (2, 60)]:
        x, y = (ci + 0.5) / n, (cj + 0.5) / n
        b2 = (x - 0.5) ** 2 + (y - 0.5) ** 2
        r = orc.trace(g, f, (x, y, -1.0), (0, 0, 1))
        N_exact = _gauss_line(sigma, b2, 0) + bg
        I_exact = (_gauss_line(sigma / math.sqrt(2), b2, 0) + 2 * bg * _gauss_line(sigma, b2, 0) + bg * bg)
        assert r["N"] == pytest.approx(N_exact, rel=1e-6)
        assert r["I"][0] == pytest.approx(I_exact, rel=1e-6)
        assert r["nvis"] == n and r["lmax"] == 0


# ----------------------------------------------------------- brute force
def brute_force(lo, h, n, rho, emis, kap, o, d):
    """Every cell box intersected with the ray, kept if it has length,
    ordered by entry, composed back to front:
    I <- I exp(-k ds) + (j/k)(1 - exp(-k ds))."""
    o = np.asarray(o, float)
    d = np.asarray(d, float)
    d = d / np.linalg.norm(d)
    segs = []
    for kz in range(n[2]):
        for ky in range(n[1]):
            for kx in range(n[0]):
                clo = lo + np.array([kx, ky, kz]) * h
                chi = clo + h
                tin, tout = -np.inf, np.inf
                ok = True
                for a in range(3):
                    if d[a] == 0:
                        if not (clo[a] <= o[a] < chi[a]):
                            ok = False
                        continue
                    t1, t2 = (clo[a] - o[a]) / d[a], (chi[a] - o[a]) / d[a]
                    tin, tout = max(tin, min(t1, t2)), min(tout, max(t1, t2))
                if ok and tout > tin:
                    segs.append((tin, tout, (kz, ky, kx)))
    segs.sort()
    I, N = 0.0, 0.0
    for tin, tout, c in reversed(segs):
        ds = tout - tin
        k, j = float(kap[c]), float(emis[c])
        N += float(rho[c]) * ds
        I = I * math.exp(-k * ds) + (j / k) * (-math.expm1(-k * ds)) if k > 0 else I + j * ds
    return I, N, len(segs)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_random_grids(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = tuple(int(x) for x in rng.integers(4, 10, 3))
    lo = rng.uniform(-1, 1, 3)
    hi = lo + rng.uniform(0.5, 2.0, 3)
    h = (hi - lo) / np.array(n)
    shape = (n[2], n[1], n[0])
    rho = rng.uniform(0.1, 2, shape).astype(np.float32)
    emis = rng.uniform(0.1, 2, shape).astype(np.float32)
    kap = rng.uniform(0.1, 3, shape).astype(np.float32)
    g = inputs.Grid(inputs.GRID_UNIFORM, n, tuple(lo), tuple(hi))
    f = inputs.Field(inputs.FIELD_RHO_J_KAPPA, rho, emis, kap)
    for k in range(12):
        o = lo + rng.uniform(0, 1, 3) * (hi - lo)
        d = rng.normal(size=3)
        if k % 4 == 0:
            d[rng.integers(3)] = 0.0  # parallel to one family of planes
        I, N, nseg = brute_force(lo, h, n, rho, emis, kap, o, d)
        r = orc.trace(g, f, o, d)
        assert r["N"] == pytest.approx(N, rel=1e-12, abs=1e-300)
        assert r["I"][0] == pytest.approx(I, rel=1e-12, abs=1e-300)
        assert r["nvis"] == nseg


def test_brute_force_rays_on_cell_faces(orc):
    """Rays lying in cell faces follow the half-open rule [lo, hi)."""
    n = (8, 8, 8)
    rng = np.random.default_rng(5)
    shape = n
    rho = rng.uniform(0.1, 2, shape).astype(np.float32)
    emis = rng.uniform(0.1, 2, shape).astype(np.float32)
    kap = rng.uniform(0.1, 3, shape).astype(np.float32)
    g = inputs.Grid(inputs.GRID_UNIFORM, n)
    f = inputs.Field(inputs.FIELD_RHO_J_KAPPA, rho, emis, kap)
    h = np.full(3, 1 / 8)
    for o, d in [((0.25, 0.5, -1), (0, 0, 1)), ((0.0, 0.125, -1), (0, 0, 1)), ((0.375, -1, 0.75), (0, 1, 0)),
                 ((-1, 0.5, 0.5), (1, 0, 0)), ((0.5, 0.5, -1), (1, 0, 1))]:
        I, N, nseg = brute_force(np.zeros(3), h, n, rho, emis, kap, o, d)
        r = orc.trace(g, f, o, d)
        assert r["N"] == pytest.approx(N, rel=1e-12)
        assert r["I"][0] == pytest.approx(I, rel=1e-12)


def test_power_law_bands_match_precomputed(orc):
    """A rho/T field with power-law bands equals, band by band, the rho/j/kappa
    field filled with kappa0 rho T^-s and rho^2 T^q."""
    rng = np.random.default_rng(3)
    n = 6
    rho = rng.uniform(0.2, 2, (n, n, n)).astype(np.float32)
    T = rng.uniform(0.5, 10, (n, n, n)).astype(np.float32)
    bands = inputs.default_bands(4)
    g = inputs.Grid(inputs.GRID_UNIFORM, (n, n, n))
    fb = inputs.Field(inputs.FIELD_RHO_T, rho, temp=T, bands=bands)
    o, d = (0.1, 0.2, -1.0), (0.3, 0.2, 1.0)
    r = orc.trace(g, fb, o, d)
    r64, t64 = rho.astype(float), T.astype(float)
    for b in range(4):
        k0, s, q = bands[b]
        I, N, _ = brute_force(np.zeros(3), np.full(3, 1 / n), (n, n, n), rho, r64 * r64 * t64 ** q,
                              k0 * r64 * t64 ** -s, o, d)
        assert r["I"][b] == pytest.approx(I, rel=1e-12)
        assert r["N"] == pytest.approx(N, rel=1e-12)


# ------------------------------------------------------------------- AMR
def test_uniform_as_amr_equals_uniform(orc):
    g, f = inputs.gaussian(n=32)
    ga, fa = inputs.uniform_as_amr(g, f, bs=8)
    rng = np.random.default_rng(11)
    for _ in range(10):
        o = rng.uniform(0, 1, 3)
        d = rng.normal(size=3)
        r1 = orc.trace(g, f, o, d)
        r2 = orc.trace(ga, fa, o, d)
        assert r2["N"] == pytest.approx(r1["N"], rel=1e-14)
        assert r2["I"][0] == pytest.approx(r1["I"][0], rel=1e-14)
        assert r2["nvis"] == r1["nvis"]


def _amr_brute(grid, field, o, d):
    """Brute force over the cells of every leaf block."""
    bs = grid.bs
    size0 = (np.asarray(grid.hi) - np.asarray(grid.lo)) / np.asarray(grid.n)
    lo = np.asarray(grid.lo)
    d = np.asarray(d, float) / np.linalg.norm(d)
    o = np.asarray(o, float)
    segs = []
    for b in range(grid.n_blocks):
        if grid.block_child[b] >= 0:
            continue
        l = grid.block_level[b]
        h = size0 / (1 << l) / bs
        blo = lo + grid.block_coord[b] * size0 / (1 << l)
        for cz in range(bs):
            for cy in range(bs):
                for cx in range(bs):
                    clo = blo + np.array([cx, cy, cz]) * h
                    chi = clo + h
                    tin, tout, ok = -np.inf, np.inf, True
                    for a in range(3):
                        if d[a] == 0:
                            ok &= clo[a] <= o[a] < chi[a]
                            continue
                        t1, t2 = (clo[a] - o[a]) / d[a], (chi[a] - o[a]) / d[a]
                        tin, tout = max(tin, min(t1, t2)), min(tout, max(t1, t2))
                    if ok and tout > tin:
                        segs.append((tin, tout, b * bs ** 3 + cx + bs * (cy + bs * cz), l))
    segs.sort()
    I, N = 0.0, 0.0
    for tin, tout, idx, l in reversed(segs):
        ds = tout - tin
        k, j = float(field.kappa[idx]), float(field.emis[idx])
        N += float(field.rho[idx]) * ds
        I = I * math.exp(-k * ds) + (j / k) * (-math.expm1(-k * ds))
    return I, N, len(segs), max([s[3] for s in segs], default=-1)


def test_amr_brute_force(orc):
    rng = np.random.default_rng(4)
    # refine blocks near a point, two levels
    c = np.array([0.4, 0.55, 0.5])
    grid = inputs.amr_from_predicate(2, 4, 2, lambda l, blo, sz: np.linalg.norm(np.asarray(blo) + sz / 2 - c) < 0.45 * (1 + l))
    nc = grid.n_cells
    f = inputs.Field(inputs.FIELD_RHO_J_KAPPA, rng.uniform(0.1, 2, nc).astype(np.float32),
                     rng.uniform(0.1, 2, nc).astype(np.float32), rng.uniform(0.5, 3, nc).astype(np.float32))
    assert grid.block_level.max() == 2
    for k in range(8):
        o = rng.uniform(0, 1, 3)
        d = rng.normal(size=3)
        if k == 0:
            d = np.array([0.0, 0.0, 1.0])
        I, N, nseg, lm = _amr_brute(grid, f, o, d)
        r = orc.trace(grid, f, o, d)
        assert r["N"] == pytest.approx(N, rel=1e-12)
        assert r["I"][0] == pytest.approx(I, rel=1e-12)
        assert r["nvis"] == nseg
        assert r["lmax"] == lm


def test_amr_refined_constant_children_equal_parent(orc):
    """Refining a block whose children repeat the parent cell values does not
    change the integral (the finer planes split constant segments)."""
    g, f = inputs.gaussian(n=16)
    ga, fa = inputs.uniform_as_amr(g, f, bs=4)
    # refine base block 5 and one of its children: data copied down
    grid = inputs.amr_from_predicate(4, 4, 2, lambda l, blo, sz: (l == 0 and np.allclose(blo, (0.25, 0.25, 0.25)))
                                     or (l == 1 and np.allclose(blo, (0.25, 0.25, 0.25))))
    pts = inputs.amr_cell_centres(grid)
    k = np.floor(pts * 16).astype(int)
    flat = k[:, 0] + 16 * (k[:, 1] + 16 * k[:, 2])
    ff = inputs.Field(0, f.rho.reshape(-1)[flat], f.emis.reshape(-1)[flat], f.kappa.reshape(-1)[flat])
    rng = np.random.default_rng(2)
    for _ in range(8):
        o = rng.uniform(0.2, 0.6, 3)
        d = rng.normal(size=3)
        r1 = orc.trace(g, f, o, d)
        r2 = orc.trace(grid, ff, o, d)
        assert r2["N"] == pytest.approx(r1["N"], rel=1e-13)
        assert r2["I"][0] == pytest.approx(r1["I"][0], rel=1e-13)


# -------------------------------------------------------------- geometry
def test_view_basis_conventions(orc):
    # section 3 face-on view along x: (u, v) = (y, z) (Fig. 1 caption)
    d, eu, ev = orc.view_basis(inputs.View((1, 0, 0), (0, 0, 1), (0, 0, 0), 1.0))
    assert np.allclose(d, [1, 0, 0]) and np.allclose(eu, [0, 1, 0]) and np.allclose(ev, [0, 0, 1])
    d, eu, ev = orc.view_basis(inputs.gaussian_view())
    assert np.allclose(eu, [1, 0, 0]) and np.allclose(ev, [0, 1, 0])
    # pixel centres of the 16^2 base image of the unit box: (2i+1)/32
    v = inputs.gaussian_view()
    assert np.array_equal(orc.pixel_center(v, 16, 0, 0, 0), [1 / 32, 1 / 32, 0.5])
    assert np.array_equal(orc.pixel_center(v, 16, 0, 5, 9), [11 / 32, 19 / 32, 0.5])
    assert np.array_equal(orc.pixel_center(v, 16, 4, 255, 0), [511 / 512, 1 / 512, 0.5])

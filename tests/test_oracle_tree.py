"""Pins for the oracle's refinement test (Eq. 2 / Eq. 3, section 3) and its
level-synchronous image tree (section 2 steps i-vi).

The criterion pins come from the paper and from mathematics: Eq. 2 is the
1-D case (a one-row image has no second direction), the estimate is bounded
(0 <= xi <= 1 once the noise filter is dropped), dimensionless (invariant
under p -> a p + c) and symmetric under the square's rotations and
reflections; strict extrema give 1 and linear data give 0.

The tree pins: xi_crit = 0 refines everything, xi_crit > 1 nothing; the
2:1 rule holds between every pair of adjacent leaves; node counts are
N0^2 + 4k (Table 1 counts every traced ray); leaves tile the image; the
closure equals an independent fixpoint balancer; the fully refined image
equals the fixed-resolution image; and the fixed image's flux equals the
sum over grid cells (Table 1 caption: the exact flux is summed from the
grid)."""
import itertools
import math

import numpy as np
import pytest

from paper_1010_5534_amd import inputs


def eq2(pm, p0, pp):
    """Eq. 2 as printed."""
    d = abs(pp - p0) + abs(p0 - pm)
    return 0.0 if d == 0 else abs(pp - 2 * p0 + pm) / d


def _stencil_1row(pm, p0, pp):
    s = np.zeros((3, 3))
    s[1] = [pm, p0, pp]
    return s


def test_xi_reduces_to_eq2_on_one_row(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        pm, p0, pp = rng.normal(size=3) * rng.uniform(0.01, 100)
        assert orc.xi(_stencil_1row(pm, p0, pp), True, False) == pytest.approx(eq2(pm, p0, pp), rel=1e-14, abs=1e-15)
        # the same data laid along v
        assert orc.xi(_stencil_1row(pm, p0, pp).T, False, True) == pytest.approx(eq2(pm, p0, pp), rel=1e-14, abs=1e-15)


def test_xi_hand_values(orc):
    assert orc.xi(_stencil_1row(0, 1, 0), True, False) == 1.0
    assert orc.xi(_stencil_1row(0, 1, 3), True, False) == pytest.approx(1 / 3)
    assert orc.xi(_stencil_1row(1, 2, 3), True, False) == 0.0
    spike = np.zeros((3, 3))
    spike[1, 1] = 1.0
    assert orc.xi(spike) == pytest.approx(1.0)
    corner = np.zeros((3, 3))
    corner[2, 2] = 1.0  # only the (+1, +1) neighbour differs
    assert orc.xi(corner) == pytest.approx(1.0)
    flat = np.full((3, 3), 7.0)
    assert orc.xi(flat) == 0.0  # 0/0 -> 0
    a, b = np.meshgrid([-1, 0, 1], [-1, 0, 1])
    assert orc.xi(3.0 * a - 2.0 * b + 5.0) == 0.0  # linear data


def test_xi_bounded_affine_invariant_symmetric(orc):
    rng = np.random.default_rng(1)
    for k in range(300):
        p = rng.normal(size=(3, 3))
        if k % 3 == 0:
            p = np.round(p)  # ties and zero differences
        x = orc.xi(p)
        assert 0.0 <= x <= 1.0 + 1e-12
        alpha, c = rng.uniform(-50, 50), rng.uniform(-1e3, 1e3)
        if abs(alpha) > 1e-3:
            assert orc.xi(alpha * p + c) == pytest.approx(x, rel=1e-9, abs=1e-9)
        for q in (np.rot90(p), np.rot90(p, 2), np.rot90(p, 3), p[::-1], p[:, ::-1], p.T):
            assert orc.xi(q) == pytest.approx(x, rel=1e-12, abs=1e-14)


def test_xi_edge_drops_direction_and_cross_terms(orc):
    # without the v direction the cross terms must not enter either
    p = np.array([[9.0, -4.0, 2.0], [0.0, 1.0, 3.0], [5.0, 8.0, -7.0]])
    assert orc.xi(p, True, False) == pytest.approx(eq2(0.0, 1.0, 3.0))
    assert orc.xi(p, False, True) == pytest.approx(eq2(-4.0, 1.0, 8.0))
    assert orc.xi(p, False, False) == 0.0


# ------------------------------------------------------------------ trees
def _leaf_levels(tree):
    """Finest raster holding each leaf's level."""
    R = tree.N0 << tree.Lmax
    out = np.full((R, R), -1, dtype=np.int64)
    for L in range(tree.Lmax + 1):
        lv = tree.leaves(L)
        sc = 1 << (tree.Lmax - L)
        out[np.kron(lv, np.ones((sc, sc), dtype=bool))] = L
    return out


def check_balanced(tree):
    lev = _leaf_levels(tree)
    assert (lev >= 0).all(), "leaves must tile the image"
    # adjacent (edge or corner) raster cells: leaf levels differ by <= 1
    for dj, di in [(0, 1), (1, 0), (1, 1), (1, -1)]:
        a = lev[max(0, -dj):lev.shape[0] - max(0, dj), max(0, -di):lev.shape[1] - max(0, di)]
        b = lev[max(0, dj):, max(0, di):][:a.shape[0], :a.shape[1]]
        assert np.abs(a - b).max() <= 1


def check_structure(tree, orc):
    refined = 0
    for L in range(tree.Lmax + 1):
        s = tree.state[L]
        ex = (s & orc.EXIST) > 0
        if L > 0:  # every node's parent exists and is refined, children come in fours
            par = tree.state[L - 1]
            assert np.array_equal(ex, np.kron((par & orc.REFINED) > 0, np.ones((2, 2), dtype=bool)))
        refined += int(((s & orc.REFINED) > 0).sum())
        assert tree.counts[L] == ex.sum()
    assert tree.nodes == tree.N0 ** 2 + 4 * refined
    assert tree.nodes == int(tree.counts.sum())


def test_full_and_empty_refinement(orc):
    g, f = inputs.gaussian(n=32)
    v = inputs.gaussian_view()
    t = orc.air(g, f, v, 8, 3, xi_crit_I=0.0)
    assert list(t.counts) == [(8 << L) ** 2 for L in range(4)]
    t = orc.air(g, f, v, 8, 3, xi_crit_I=1.01)
    assert list(t.counts) == [64, 0, 0, 0]


def test_constant_field_stays_coarse(orc):
    n = 16
    g = inputs.Grid(inputs.GRID_UNIFORM, (n, n, n))
    shape = (n, n, n)
    f = inputs.Field(0, np.ones(shape, np.float32), np.ones(shape, np.float32), np.ones(shape, np.float32))
    t = orc.air(g, f, inputs.gaussian_view(), 8, 3, xi_crit_I=0.5, xi_crit_N=0.5)
    assert t.nodes == 64


@pytest.mark.parametrize("xc", [0.2, 0.5, 0.8])
def test_gaussian_tree_invariants(orc, xc):
    g, f = inputs.gaussian()
    v = inputs.gaussian_view()
    t = orc.air(g, f, v, 16, 4, xi_crit_I=xc)
    check_structure(t, orc)
    check_balanced(t)
    # only tested nodes carry an xi; balance nodes never do
    for L in range(4):
        s = t.state[L]
        tested = (s & orc.TESTED) > 0
        assert np.all(np.isfinite(t.xiI[L][tested]))
        assert np.all(np.isnan(t.xiI[L][~tested]))
        assert not np.any((s & orc.BALANCE) & (s & orc.TESTED))
        fl = (s & orc.FLAGGED) > 0
        assert np.array_equal(fl, tested & (t.xiI[L] >= xc))
    # flagged nodes' children are tested nodes
    for L in range(4):
        fl = (t.state[L] & orc.FLAGGED) > 0
        ch = np.kron(fl, np.ones((2, 2), dtype=bool))
        assert np.all((t.state[L + 1][ch] & orc.TESTED) > 0)


def _fixpoint_tree(N0, Lmax, flags):
    """Independent structure builder: level by level, refine the flagged
    tested leaves, then refine any leaf adjacent (8-neighbourhood) to a leaf
    two or more levels deeper until no such pair is left."""
    ex = [np.zeros((N0 << L, N0 << L), bool) for L in range(Lmax + 1)]
    tested = [np.zeros_like(e) for e in ex]
    ex[0][:] = True
    tested[0][:] = True

    def refined(L):
        return ex[L + 1][::2, ::2] if L < Lmax else np.zeros_like(ex[L])

    def leaf_level_map():
        R = N0 << Lmax
        out = np.full((R, R), -1)
        for L in range(Lmax + 1):
            lv = ex[L] & ~refined(L)
            sc = 1 << (Lmax - L)
            out[np.kron(lv, np.ones((sc, sc), bool))] = L
        return out

    for L in range(Lmax):
        fl = tested[L] & flags[L]
        if not fl.any():
            break
        for j, i in zip(*np.nonzero(fl)):
            ex[L + 1][2 * j:2 * j + 2, 2 * i:2 * i + 2] = True
            tested[L + 1][2 * j:2 * j + 2, 2 * i:2 * i + 2] = True
        while True:
            lev = leaf_level_map()
            R = lev.shape[0]
            changed = False
            pad = np.pad(lev, 1, constant_values=-1)
            nmax = np.max([pad[1 + dj:1 + dj + R, 1 + di:1 + di + R] for dj in (-1, 0, 1) for di in (-1, 0, 1)],
                          axis=0)
            bad = nmax >= lev + 2
            if not bad.any():
                break
            leaves = [ex[Lb] & ~refined(Lb) for Lb in range(Lmax)]  # before any change
            for Lb in range(Lmax):
                sc = 1 << (Lmax - Lb)
                badL = bad.reshape(N0 << Lb, sc, N0 << Lb, sc).any(axis=(1, 3)) & leaves[Lb]
                for j, i in zip(*np.nonzero(badL)):
                    ex[Lb + 1][2 * j:2 * j + 2, 2 * i:2 * i + 2] = True
                    changed = True
            assert changed
    return ex, tested


@pytest.mark.parametrize("seed", range(6))
def test_closure_equals_fixpoint_balancer(orc, seed):
    rng = np.random.default_rng(seed)
    N0, Lmax = int(rng.integers(2, 6)), int(rng.integers(2, 5))
    p = [0.3, 0.15, 0.08, 0.05, 0.05][:Lmax + 1]
    flags = [rng.uniform(size=(N0 << L, N0 << L)) < p[L] for L in range(Lmax + 1)]
    flat = np.concatenate([f.reshape(-1) for f in flags]).astype(np.uint8)
    t = orc.air(None, None, inputs.gaussian_view(), N0, Lmax, force_flags=flat)
    ex, tested = _fixpoint_tree(N0, Lmax, flags)
    for L in range(Lmax + 1):
        assert np.array_equal((t.state[L] & orc.EXIST) > 0, ex[L]), f"level {L}"
        assert np.array_equal((t.state[L] & orc.TESTED) > 0, tested[L]), f"level {L}"
    check_structure(t, orc)
    check_balanced(t)


def test_hand_built_closure():
    """4x4 base, flag (1,1) at level 0 and then its child (2,2): the three
    base pixels (0,0), (1,0), (0,1) next to (2,2)'s parent must be refined."""
    import oracle
    N0, Lmax = 4, 2
    flags = [np.zeros((N0 << L, N0 << L), np.uint8) for L in range(3)]
    flags[0][1, 1] = 1
    flags[1][2, 2] = 1
    flat = np.concatenate([f.reshape(-1) for f in flags])
    t = oracle.air(None, None, inputs.gaussian_view(), N0, Lmax, force_flags=flat)
    assert list(t.counts) == [16, 16, 4]
    ref0 = (t.state[0] & oracle.REFINED) > 0
    assert set(zip(*np.nonzero(ref0))) == {(1, 1), (0, 0), (0, 1), (1, 0)}
    bal = (t.state[1] & oracle.BALANCE) > 0
    assert bal.sum() == 12
    assert t.nodes == 36


def test_full_refinement_equals_fixed_image(orc):
    g, f = inputs.gaussian(n=32)
    v = inputs.gaussian_view()
    t = orc.air(g, f, v, 8, 3, xi_crit_I=0.0)
    fx = orc.render_fixed(g, f, v, 8, 3)
    img = orc.paint_leaves(t, t.flat_I[0])
    assert np.array_equal(img, fx["I"][0])
    assert np.array_equal(orc.paint_leaves(t, t.flat_N), fx["N"])


def test_grid_sum_flux(orc):
    """Optically thin, axis view, image = box face, one pixel per cell
    column: the image flux equals the emissivity summed over the grid."""
    n = 32
    g, f = inputs.gaussian(n=n, thin=True)
    v = inputs.gaussian_view()
    exact = float(np.sum(f.emis.astype(np.float64))) / n ** 3
    fx = orc.render_fixed(g, f, v, 8, 2)  # 32^2 pixels
    assert float(np.sum(fx["I"][0])) / (32 * 32) == pytest.approx(exact, rel=1e-13)
    t = orc.air(g, f, v, 8, 2, xi_crit_I=0.0)
    assert orc.leaf_flux(t, 1.0, t.flat_I[0]) == pytest.approx(exact, rel=1e-13)
    # AIR with a real threshold: the flux error is small but not zero
    t = orc.air(g, f, v, 8, 2, xi_crit_I=0.5)
    err = abs(orc.leaf_flux(t, 1.0, t.flat_I[0]) - exact) / exact
    assert 0 < err < 0.05


# ------------------------------------------------ injection (coarser neighbours)
def _injection_case():
    """4x4 base, three levels below, forced flags: level 0 flags (1,1); level 1
    flags its child (3,2), whose 2:1 closure refines base pixels (1,0), (2,0)
    and (2,1) in the same step; level 2 flags (7,5), whose closure refines the
    level-1 nodes (4,2), (3,3) and (4,3) in the same step.  Every position of
    every level holds a distinct value (as if traced), so a stencil that reads
    the wrong node gives a different estimate."""
    import oracle
    N0, Lmax = 4, 3
    flags = [np.zeros((N0 << L, N0 << L), np.uint8) for L in range(Lmax + 1)]
    flags[0][1, 1] = 1     # [j, i]
    flags[1][2, 3] = 1     # (i, j) = (3, 2)
    flags[2][5, 7] = 1     # (i, j) = (7, 5)
    rng = np.random.default_rng(42)
    vals = [rng.permutation((N0 << L) ** 2).reshape(N0 << L, N0 << L).astype(np.float64) * 0.37 + 100 * L + 1
            for L in range(Lmax + 1)]
    colv = [v[::-1, ::-1].copy() * 1.7 + 3.0 for v in vals]
    flat = lambda a: np.concatenate([x.reshape(-1) for x in a])
    t = oracle.air(None, None, inputs.gaussian_view(), N0, Lmax, force_flags=flat(flags),
                   values=(flat(vals), flat(colv)))
    return t, vals, colv


# stencils written out by hand: for each tested node (L, i, j), the source of
# each offset (a, b) (a along i, b along j), row by row b = -1, 0, 1, as
# (level, i, j) of the node whose value the test must read.  A level-L
# neighbour counts only if it existed when level L was tested: here that is
# the four tested children of the level-(L-1) flag; every other position reads
# the covering level-(L-1) node, including positions the same step's closure
# creates afterwards.
HAND_STENCILS = {
    (1, 3, 3): [(1, 2, 2), (1, 3, 2), (0, 2, 1),
                (1, 2, 3), (1, 3, 3), (0, 2, 1),
                (0, 1, 2), (0, 1, 2), (0, 2, 2)],
    (1, 2, 2): [(0, 0, 0), (0, 1, 0), (0, 1, 0),
                (0, 0, 1), (1, 2, 2), (1, 3, 2),
                (0, 0, 1), (1, 2, 3), (1, 3, 3)],
    (1, 3, 2): [(0, 1, 0), (0, 1, 0), (0, 2, 0),
                (1, 2, 2), (1, 3, 2), (0, 2, 1),
                (1, 2, 3), (1, 3, 3), (0, 2, 1)],
    (2, 6, 4): [(1, 2, 1), (1, 3, 1), (1, 3, 1),
                (1, 2, 2), (2, 6, 4), (2, 7, 4),
                (1, 2, 2), (2, 6, 5), (2, 7, 5)],
    # (8, *) and (*, 6) read level-1 balance nodes created by step 1 (they
    # existed when level 2 was tested) and are themselves created at level 2
    # by the closure of (7, 5) in step 2 (too late to count)
    (2, 7, 5): [(2, 6, 4), (2, 7, 4), (1, 4, 2),
                (2, 6, 5), (2, 7, 5), (1, 4, 2),
                (1, 3, 3), (1, 3, 3), (1, 4, 3)],
}


def test_injection_hand_stencils(orc):
    """Eq. 3 at a node whose neighbours include coarser leaves takes the
    covering level-(L-1) node's value; nodes created by the same step's 2:1
    closure do not count (the test of a level sees the tree as it was before
    the level changed).  Checked on hand-written stencils of intensity and
    column at levels 1 and 2."""
    t, vals, colv = _injection_case()
    for (L, i, j), src in HAND_STENCILS.items():
        assert t.state[L][j, i] & orc.TESTED, (L, i, j)
        p = np.array([vals[l][jj, ii] for (l, ii, jj) in src]).reshape(3, 3)
        q = np.array([colv[l][jj, ii] for (l, ii, jj) in src]).reshape(3, 3)
        R = 4 << L
        hx, hy = 0 < i < R - 1, 0 < j < R - 1
        assert t.xiI[L][j, i] == orc.xi(p, hx, hy), (L, i, j)
        assert t.xiN[L][j, i] == orc.xi(q, hx, hy), (L, i, j)


def test_injection_case_creates_same_step_nodes(orc):
    """The positions the hand stencils read through the coarser level do get
    created, by the closure of the same step: so a test that counted them
    would read them."""
    t, _, _ = _injection_case()
    for (L, i, j) in [(1, 4, 2), (1, 4, 3), (1, 2, 1), (1, 3, 1), (2, 8, 4), (2, 8, 5), (2, 8, 6), (2, 6, 6),
                      (2, 7, 6)]:
        assert t.state[L][j, i] & orc.EXIST, (L, i, j)
        assert t.state[L][j, i] & orc.BALANCE, (L, i, j)
        assert t.born[L][j, i] == L, (L, i, j)
    # created one step later still (the closure of (7, 5) at level 2 needs the
    # level-1 neighbours of (3, 3))
    for (L, i, j) in [(1, 2, 4), (1, 3, 4), (1, 4, 4)]:
        assert t.state[L][j, i] & orc.EXIST and t.born[L][j, i] == 2, (L, i, j)
    for (L, i, j) in [(2, 5, 3), (2, 5, 4)]:
        assert not t.state[L][j, i] & orc.EXIST, (L, i, j)


def test_injection_detects_planted_mistakes(orc):
    """The hand stencils would catch the two plausible mistakes: a covering
    index rounded the other way and counting the same step's nodes."""
    t, vals, _ = _injection_case()
    L, i, j = 1, 3, 3
    src = HAND_STENCILS[(L, i, j)]
    wrong_cover = [(l, (ii + 1) >> 1, (jj + 1) >> 1) if l < L else (l, ii, jj)
                   for (l, ii, jj) in [(1, 2, 2), (1, 3, 2), (0, 4, 2), (1, 2, 3), (1, 3, 3), (0, 4, 3),
                                       (0, 2, 4), (0, 3, 4), (0, 4, 4)]]
    same_step = [(1, 2, 2), (1, 3, 2), (1, 4, 2), (1, 2, 3), (1, 3, 3), (1, 4, 3), (0, 1, 2), (0, 1, 2), (0, 2, 2)]
    good = orc.xi(np.array([vals[l][jj, ii] for (l, ii, jj) in src]).reshape(3, 3))
    for bad in (wrong_cover, same_step):
        p = np.array([vals[l][jj, ii] if jj < vals[l].shape[0] and ii < vals[l].shape[1] else 0.0
                      for (l, ii, jj) in bad]).reshape(3, 3)
        assert orc.xi(p) != good
    assert t.xiI[L][j, i] == good

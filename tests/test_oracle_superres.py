"""Pins of the oracle's super-resolution output (section 2 step vi: the
final image may be sharpened by interpolating across neighbouring pixels
whose levels differ; reading: bilinear interpolation of the leaf level's point
samples, a missing sample taken from the covering node one level up, edges
clamped).  Pinned by hand values on small forced trees, by the limits (a
fully refined tree gives the painted image; an unrefined tree with affine
values reproduces the affine function inside the image; constants stay
constant)."""
import numpy as np
import pytest

from paper_1010_5534_amd import inputs


def _forced(orc, N0, Lmax, flags, vals):
    flat = np.concatenate([f.reshape(-1) for f in flags]).astype(np.uint8)
    fv = np.concatenate([v.reshape(-1) for v in vals])
    t = orc.air(None, None, inputs.gaussian_view(), N0, Lmax, force_flags=flat, values=(fv, fv))
    return t, fv


def test_hand_values_one_level(orc):
    """2x2 base, (0,0) refined once: a, b, c, d at level 0 (row-major
    [j][i]), e, f, g, h its children; 4x4 raster."""
    a, b, c, d, e, f, g, h = 1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0
    flags = [np.array([[1, 0], [0, 0]]), np.zeros((4, 4))]
    vals = [np.array([[a, b], [c, d]]), np.zeros((4, 4))]
    vals[1][0, 0], vals[1][0, 1], vals[1][1, 0], vals[1][1, 1] = e, f, g, h
    t, fv = _forced(orc, 2, 1, flags, vals)
    out = orc.superres(t, fv)
    # level-1 leaves: the pixel's own sample (weights 1 and 0)
    assert out[0, 0] == e and out[0, 1] == f and out[1, 0] == g and out[1, 1] == h
    # level-0 leaf (1, 0), pixel (x, y) = (2, 0): u = 0.75, v = -0.25 (clamped row)
    assert out[0, 2] == pytest.approx(0.25 * a + 0.75 * b, rel=1e-15)
    # level-0 leaf (1, 1), pixel (2, 2): all four base samples
    assert out[2, 2] == pytest.approx(0.0625 * a + 0.1875 * b + 0.1875 * c + 0.5625 * d, rel=1e-15)
    # pixel (3, 3): beyond the last sample on both axes -> d
    assert out[3, 3] == d


def test_hand_values_injection(orc):
    """2x2 base, (0,0) refined, two refinement levels allowed: the level-1
    leaves' neighbours beyond their parent do not exist at level 1, so their
    samples come from the level-0 nodes covering them."""
    a, b, c, d, e, f, g, h = 1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0
    flags = [np.array([[1, 0], [0, 0]]), np.zeros((4, 4)), np.zeros((8, 8))]
    vals = [np.array([[a, b], [c, d]]), np.full((4, 4), 1e6), np.full((8, 8), 1e9)]
    vals[1][0, 0], vals[1][0, 1], vals[1][1, 0], vals[1][1, 1] = e, f, g, h
    t, fv = _forced(orc, 2, 2, flags, vals)
    out = orc.superres(t, fv)
    # level-1 leaf (1, 1), pixel (2, 2): u = v = 0.75 -> e, f, g, h
    assert out[2, 2] == pytest.approx(0.0625 * e + 0.1875 * f + 0.1875 * g + 0.5625 * h, rel=1e-15)
    # pixel (3, 3): u = v = 1.25 -> h, and the injected (2,1) -> b, (1,2) -> c, (2,2) -> d
    assert out[3, 3] == pytest.approx(0.5625 * h + 0.1875 * b + 0.1875 * c + 0.0625 * d, rel=1e-15)
    # level-0 leaf (1, 0), pixel (4, 0): u = 0.625, v = -0.375 (clamped) -> a, b
    assert out[0, 4] == pytest.approx(0.375 * a + 0.625 * b, rel=1e-15)


def test_full_refinement_equals_painting(orc):
    g, f = inputs.gaussian(n=32)
    t = orc.air(g, f, inputs.gaussian_view(), 8, 3, xi_crit_I=0.0)
    assert np.array_equal(orc.superres(t, t.flat_I[0]), orc.paint_leaves(t, t.flat_I[0]))


def test_affine_values_on_unrefined_tree(orc):
    """No refinement: the finest pixels inside the outermost sample centres
    get the affine function at their own position exactly."""
    N0, Lmax = 5, 3
    flags = [np.zeros((N0 << L, N0 << L)) for L in range(Lmax + 1)]
    jj, ii = np.mgrid[0:N0, 0:N0].astype(float)
    vals = [3.0 + 0.5 * ii - 1.25 * jj] + [np.zeros((N0 << L, N0 << L)) for L in range(1, Lmax + 1)]
    t, fv = _forced(orc, N0, Lmax, flags, vals)
    out = orc.superres(t, fv)
    s = 1 << Lmax
    x = (np.arange(N0 * s) + 0.5) / s - 0.5
    ref = 3.0 + 0.5 * x[None, :] - 1.25 * x[:, None]
    inside = (x >= 0) & (x <= N0 - 1)
    m = inside[:, None] & inside[None, :]
    assert np.allclose(out[m], ref[m], rtol=0, atol=1e-13)
    # outside, the nearest edge sample's coordinate
    xc = np.clip(x, 0, N0 - 1)
    assert np.allclose(out, 3.0 + 0.5 * xc[None, :] - 1.25 * xc[:, None], rtol=0, atol=1e-13)


def test_constant_stays_constant_on_mixed_tree(orc):
    rng = np.random.default_rng(4)
    N0, Lmax = 4, 3
    flags = [(rng.uniform(size=(N0 << L, N0 << L)) < 0.3).astype(np.uint8) for L in range(Lmax + 1)]
    vals = [np.full((N0 << L, N0 << L), 2.5) for L in range(Lmax + 1)]
    t, fv = _forced(orc, N0, Lmax, flags, vals)
    assert np.all(orc.superres(t, fv) == 2.5)

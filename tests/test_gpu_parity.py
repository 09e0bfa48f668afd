"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Values within 1e-5 relative per node; flags identical
except at nodes the oracle itself marks ambiguous (see parity.py); misses
exactly zero."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import parity
from paper_1010_5534_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1010_5534_amd import air
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = air.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def gauss():
    from paper_1010_5534_amd import air
    g, f = inputs.gaussian()
    return g, f, air.upload(g, f)


def test_fixed_levels_match_oracle(ctx, gauss):
    g, f, scene = gauss
    v = inputs.gaussian_view()
    for L in range(5):
        say(f"fixed gaussian64 N0=16 L={L}")
        img, flux, st = ctx.render_fixed(scene, [v], 16, L)
        ref = oracle.render_fixed(g, f, v, 16, L)
        gi = img[0].cpu().numpy().astype(np.float64)
        assert parity.rel_err(gi[0], ref["I"][0]).max() <= 1e-5
        assert parity.rel_err(gi[1], ref["N"]).max() <= 1e-5
        R = 16 << L
        exact_flux = float(np.sum(ref["I"][0])) / (R * R)
        assert flux[0][0] == pytest.approx(exact_flux, rel=1e-5)
        assert st["rays"] == R * R and st["hits"] == R * R


@pytest.mark.parametrize("direction", [(1, 1, 1), (1, 0, 0), (0.3, -0.8, 0.52), (0, 1, 0), (-1, -0.2, 0.1)])
def test_fixed_oblique_views(ctx, direction):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=1, n=48)
    scene = air.upload(g, f)
    v = inputs.view_for(direction)
    say(f"fixed winds2 n=48 dir={direction} N0=12 L=3")
    img, _, st = ctx.render_fixed(scene, [v], 12, 3)
    ref = oracle.render_fixed(g, f, v, 12, 3)
    gi = img[0].cpu().numpy().astype(np.float64)
    assert parity.rel_err(gi[0], ref["I"][0]).max() <= 1e-5
    assert parity.rel_err(gi[1], ref["N"]).max() <= 1e-5
    # misses are exact zeros on both sides
    assert np.array_equal(gi[0] == 0, ref["I"][0] == 0)


@pytest.mark.parametrize("case", ["edges", "corners"])
def test_rays_on_cell_faces_and_corners(ctx, case):
    """Exact ties of the geometry: with a 16^3 unit box and an 8x8 image of
    width 1 looking along +z, every pixel centre lies on a cell edge (x and y
    both on cell faces), so the half-open cell rule alone picks the cells; along
    (1, 1, 0)/sqrt2 with an image of width sqrt2, every ray meets its x and y
    faces at the same points (it passes through cell corners), so the walk
    takes ties at every other step.  Both against the oracle."""
    from paper_1010_5534_amd import air
    g, f = inputs.gaussian(n=16)
    scene = air.upload(g, f)
    if case == "edges":
        v = inputs.View((0.0, 0.0, 1.0), (0.0, 1.0, 0.0), (0.5, 0.5, 0.5), 1.0)
        N0, L = 8, 0
        u = (-0.5 + (np.arange(N0) + 0.5) / N0 + 0.5) * 16
        assert np.all(u == np.round(u)) and np.all(u.astype(int) % 2 == 1)
    else:
        r = 1.0 / math.sqrt(2.0)
        v = inputs.View((r, r, 0.0), (0.0, 0.0, 1.0), (0.5, 0.5, 0.5), math.sqrt(2.0))
        N0, L = 8, 1
    say(f"fixed gaussian16 {case} N0={N0} L={L}")
    img, flux, st = ctx.render_fixed(scene, [v], N0, L)
    ref = oracle.render_fixed(g, f, v, N0, L)
    gi = img[0].cpu().numpy().astype(np.float64)
    assert parity.rel_err(gi[0], ref["I"][0]).max() <= 1e-5
    assert parity.rel_err(gi[1], ref["N"]).max() <= 1e-5
    assert np.array_equal(gi[0] == 0, ref["I"][0] == 0)
    assert st["hits"] == int(np.count_nonzero(ref["lmax"] >= 0))


@pytest.mark.parametrize("xc", [0.2, 0.5, 0.8])
def test_air_tree_parity_gaussian(ctx, gauss, xc):
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    v = inputs.gaussian_view()
    say(f"air gaussian64 N0=16 Lmax=4 xi_crit={xc}")
    trees, img, flux, st = ctx.render(scene, [v], air.params(16, 4, xc))
    rep = parity.check(trees[0], g, f, v, 16, 4, xc, image=img[0], flux=flux[0], own=True,
                       label=f"gaussian64 N0=16 Lmax=4 xi_crit={xc}")
    say(parity.summary(rep))
    parity.assert_parity(rep)
    assert st["rays"] == trees[0].n_nodes


def test_full_refinement_equals_fixed_bitwise(ctx, gauss):
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    v = inputs.gaussian_view()
    trees, img, flux, st = ctx.render(scene, [v], air.params(16, 4, 0.0))
    assert trees[0].n_per_level[:5] == [(16 << L) ** 2 for L in range(5)]
    fimg, fflux, _ = ctx.render_fixed(scene, [v], 16, 4)
    assert torch.equal(img, fimg)


def test_no_refinement_above_one(ctx, gauss):
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    trees, img, flux, st = ctx.render(scene, [inputs.gaussian_view()], air.params(16, 4, 1.01))
    assert trees[0].n_nodes == 256 and st["rays"] == 256 and st["flagged"] == 0


def test_batched_views_equal_single_views_bitwise(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=2, n=64)
    scene = air.upload(g, f)
    views = inputs.winds2_views()
    prm = air.params(16, 3, 0.5)
    trees, img, flux, _ = ctx.render(scene, views, prm)
    for k, v in enumerate(views):
        t1, i1, f1, _ = ctx.render(scene, [v], prm)
        assert t1[0].n_nodes == trees[k].n_nodes
        for name in ("level", "ix", "iy", "parent", "first_child", "state", "I", "N", "visits"):
            assert torch.equal(getattr(t1[0], name), getattr(trees[k], name)), name
        assert torch.equal(i1[0], img[k])
        assert f1[0][0] == flux[k][0]


def test_run_twice_bitwise(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=3, n=64)
    scene = air.upload(g, f)
    prm = air.params(16, 4, 0.3)
    a = ctx.render(scene, inputs.winds2_views(), prm)
    b = ctx.render(scene, inputs.winds2_views(), prm)
    for ta, tb in zip(a[0], b[0]):
        assert ta.n_nodes == tb.n_nodes
        assert torch.equal(ta.I, tb.I) and torch.equal(ta.state, tb.state)
        # bit patterns, so the NaN of non-evaluated nodes compares equal
        assert torch.equal(ta.xi_I.view(torch.int32), tb.xi_I.view(torch.int32))
    assert torch.equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("seed,direction", [(0, (0, 0, 1)), (4, (1, 1, 1)), (5, (0.2, 0.9, -0.4))])
def test_air_tree_parity_winds(ctx, seed, direction):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=seed, n=64)
    scene = air.upload(g, f)
    v = inputs.view_for(direction)
    say(f"air winds2 n=64 seed={seed} dir={direction} N0=16 Lmax=4")
    trees, img, flux, st = ctx.render(scene, [v], air.params(16, 4, 0.5))
    rep = parity.check(trees[0], g, f, v, 16, 4, 0.5, image=img[0], flux=flux[0], own=True,
                       label=f"winds2 n=64 seed={seed} dir={direction}")
    say(parity.summary(rep))
    parity.assert_parity(rep)


# the workloads' band tables step s evenly with one q (the march's ladder
# form); an uneven table takes the per-band form
UNEVEN_BANDS = np.array([[0.3, 1.1, 0.5], [3.0, 1.7, 0.4], [1.2, 1.3, 0.65], [8.0, 0.9, 0.5]])


@pytest.mark.parametrize("bands", [inputs.default_bands(4), UNEVEN_BANDS], ids=["ladder", "uneven"])
def test_multiband_rho_t(ctx, bands):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=6, n=48, kind=inputs.FIELD_RHO_T, bands=bands)
    scene = air.upload(g, f)
    v = inputs.view_for((0.4, 0.5, 0.77))
    w = [1.0, 0.5, 2.0, 0.25]
    say("air winds2 rho/T 4 bands n=48 N0=12 Lmax=3")
    trees, img, flux, st = ctx.render(scene, [v], air.params(12, 3, 0.5, band_weight=w))
    rep = parity.check(trees[0], g, f, v, 12, 3, 0.5, band_w=w, image=img[0], flux=flux[0], own=True,
                       label="winds2 rho/T 4 bands")
    say(parity.summary(rep))
    parity.assert_parity(rep)
    fimg, fflux, _ = ctx.render_fixed(scene, [v], 12, 3)
    ref = oracle.render_fixed(g, f, v, 12, 3)
    for b in range(4):
        assert parity.rel_err(fimg[0, b].cpu().numpy(), ref["I"][b]).max() <= 1e-5


def test_column_refinement_variable(ctx, gauss):
    """N as a second refinement variable, OR-ed with I."""
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    v = inputs.gaussian_view()
    trees, img, flux, _ = ctx.render(scene, [v], air.params(16, 3, 1.01, 0.5))
    rep = parity.check(trees[0], g, f, v, 16, 3, 1.01, 0.5, image=img[0], flux=flux[0], own=True,
                       label="column variable")
    say(parity.summary(rep))
    parity.assert_parity(rep)
    assert trees[0].n_nodes > 256


# the raster is painted four pixels per thread when its side is a multiple
# of 4, else one: (4, 0) and (6, 1) take the first form with no or one level
# above the pixels, (7, 0) and (7, 1) the second
@pytest.mark.parametrize("N0,Lmax", [(1, 3), (13, 2), (7, 0), (2, 5), (4, 0), (6, 1), (7, 1)])
def test_ragged_and_degenerate_images(ctx, N0, Lmax):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=7, n=40)
    scene = air.upload(g, f)
    v = inputs.view_for((0.1, 0.2, 1.0), width=1.3)
    say(f"air winds2 n=40 N0={N0} Lmax={Lmax}")
    trees, img, flux, st = ctx.render(scene, [v], air.params(N0, Lmax, 0.3))
    rep = parity.check(trees[0], g, f, v, N0, Lmax, 0.3, image=img[0], flux=flux[0], own=True,
                       label=f"ragged N0={N0} Lmax={Lmax}")
    say(parity.summary(rep))
    parity.assert_parity(rep)


def test_view_missing_the_grid(ctx, gauss):
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    v = inputs.View((0, 0, 1), (0, 1, 0), (5.0, 5.0, 0.5), 1.0)
    trees, img, flux, st = ctx.render(scene, [v], air.params(8, 3, 0.0))
    assert st["hits"] == 0
    assert torch.count_nonzero(img).item() == 0 and flux[0][0] == 0.0


def test_offset_box_nonuniform_cells(ctx):
    from paper_1010_5534_amd import air
    rng = np.random.default_rng(9)
    n = (20, 33, 17)
    shape = (n[2], n[1], n[0])
    g = inputs.Grid(inputs.GRID_UNIFORM, n, (-0.7, 0.1, 2.0), (0.9, 1.3, 2.6))
    f = inputs.Field(0, rng.uniform(0.1, 2, shape).astype(np.float32),
                     rng.uniform(0.1, 2, shape).astype(np.float32), rng.uniform(0.1, 3, shape).astype(np.float32))
    scene = air.upload(g, f)
    v = inputs.View((0.3, -0.4, 0.8), (0, 0, 1), (0.1, 0.7, 2.3), 2.0)
    img, _, _ = ctx.render_fixed(scene, [v], 10, 3)
    ref = oracle.render_fixed(g, f, v, 10, 3)
    assert parity.rel_err(img[0, 0].cpu().numpy(), ref["I"][0]).max() <= 1e-5
    assert parity.rel_err(img[0, 1].cpu().numpy(), ref["N"]).max() <= 1e-5


def test_trace_pixels_matches_oracle(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=0, n=64)
    scene = air.upload(g, f)
    v = inputs.view_for((1, 1, 1))
    rng = np.random.default_rng(1)
    L = rng.integers(0, 6, 3000)
    R = 16 << L
    i = (rng.uniform(size=3000) * R).astype(np.int64)
    j = (rng.uniform(size=3000) * R).astype(np.int64)
    I, N, vis = ctx.trace_pixels(scene, v, 16, L, i, j)
    ref = oracle.trace_pixels(g, f, v, 16, L, i, j)
    assert parity.rel_err(I[0].cpu().numpy(), ref["I"][0]).max() <= 1e-5
    assert parity.rel_err(N.cpu().numpy(), ref["N"]).max() <= 1e-5


def test_argument_errors(ctx, gauss):
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    v = inputs.gaussian_view()
    bad = [
        (inputs.View((0, 0, 0), (0, 1, 0), (0.5, 0.5, 0.5), 1.0), air.params(8, 2)),
        (inputs.View((0, 1, 0), (0, 2, 0), (0.5, 0.5, 0.5), 1.0), air.params(8, 2)),
        (inputs.View((0, 0, 1), (0, 1, 0), (0.5, 0.5, 0.5), float("nan")), air.params(8, 2)),
        (v, air.params(0, 2)),
        (v, air.params(8, 12)),
        (v, air.params(4096, 10)),
        (v, air.params(8, 2, -0.1)),
    ]
    for view, prm in bad:
        with pytest.raises(air.AirError) as e:
            ctx.render(scene, [view], prm, want_tree=False, want_image=False, want_flux=False)
        assert e.value.code == air.AIR_EINVAL
    prm = air.params(8, 2)
    prm.flags = 4  # unknown bit
    with pytest.raises(air.AirError):
        ctx.render(scene, [v], prm, want_tree=False, want_image=False, want_flux=False)


def test_capacity_error_reports_needed_size(ctx, gauss):
    import ctypes as C
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    v = inputs.gaussian_view()
    prm = air.params(16, 4, 0.5)
    trees = (air.air_tree * 1)()
    s, keep = ctx._alloc_tree(100, 1)
    trees[0] = s
    vs = air._views([v])
    rc = air.lib().air_render(ctx._p, C.addressof(scene.grid), C.addressof(scene.field), C.addressof(vs), 1,
                              C.addressof(prm), C.addressof(trees), None, None, None,
                              torch.cuda.current_stream().cuda_stream)
    assert rc == air.AIR_ECAPACITY
    full, _, _, _ = ctx.render(scene, [v], prm)
    assert trees[0].n_nodes == full[0].n_nodes > 100


def _brick_order(a, n):
    """numpy reference of the packed layout: 2x2x2 bricks, x fastest."""
    nx, ny, nz = n
    bx, by, bz = (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2
    pad = np.zeros((2 * bz, 2 * by, 2 * bx) + a.shape[3:], a.dtype)
    pad[:nz, :ny, :nx] = a
    pad = pad.reshape(bz, 2, by, 2, bx, 2, *a.shape[3:])      # z, cz, y, cy, x, cx
    pad = pad.transpose(0, 2, 4, 1, 3, 5, *range(6, pad.ndim))  # brick z, y, x, then cz, cy, cx
    return pad.reshape(bz * by * bx * 8, *a.shape[3:])


def test_packed_layout_contents(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=8, n=6)
    f.rho = np.arange(216, dtype=np.float32).reshape(6, 6, 6)
    g = inputs.Grid(inputs.GRID_UNIFORM, (6, 5, 3))
    f = inputs.Field(0, np.arange(90, dtype=np.float32).reshape(3, 5, 6), 1000 + np.arange(90, dtype=np.float32).reshape(3, 5, 6),
                     2000 + np.arange(90, dtype=np.float32).reshape(3, 5, 6))
    sc = ctx.prepare(air.upload(g, f))
    got = sc.tensors[-1].cpu().numpy().view(np.float32).reshape(-1, 4)
    stacked = np.stack([f.rho, f.emis, f.kappa, np.zeros_like(f.rho)], axis=-1)
    ref = _brick_order(stacked, g.n)
    assert np.array_equal(got[:, :3], ref[:, :3])
    # fourth word: 1/kappa by the hardware reciprocal (within 1 ulp); padding cells 0
    real = ref[:, 2] != 0
    assert np.allclose(got[real, 3], 1.0 / ref[real, 2].astype(np.float64), rtol=2.5e-7, atol=0)
    assert np.all(got[~real, 3] == 0)


def test_prepacked_field_equals_per_call_packing(ctx):
    """A field packed once (air_field_pack) renders bit for bit like one the
    library packs on every call."""
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=8, n=50)  # even and odd brick counts
    views = inputs.winds2_views()
    prm = air.params(10, 4, 0.4)
    a = ctx.render(air.upload(g, f), views, prm)
    b = ctx.render(ctx.prepare(air.upload(g, f)), views, prm)
    for ta, tb in zip(a[0], b[0]):
        assert torch.equal(ta.I, tb.I) and torch.equal(ta.state, tb.state)
    assert torch.equal(a[1], b[1])
    g2, f2 = inputs.winds2(seed=8, n=33, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    s1, s2 = air.upload(g2, f2), ctx.prepare(air.upload(g2, f2))
    i1, _, _ = ctx.render_fixed(s1, views, 8, 2)
    i2, _, _ = ctx.render_fixed(s2, views, 8, 2)
    assert torch.equal(i1, i2)


def test_tree_links_consistent(ctx, gauss):
    from paper_1010_5534_amd import air
    g, f, scene = gauss
    trees, _, _, _ = ctx.render(scene, [inputs.gaussian_view()], air.params(16, 4, 0.5))
    t = trees[0]
    lv = t.level.cpu().numpy().astype(int)
    ix, iy = t.ix.cpu().numpy(), t.iy.cpu().numpy()
    par, fc = t.parent.cpu().numpy(), t.first_child.cpu().numpy()
    st = t.state.cpu().numpy()
    assert np.all(np.diff(lv) >= 0)  # canonical order: by level
    for k in np.nonzero(lv > 0)[0][:5000]:
        p = par[k]
        assert lv[p] == lv[k] - 1 and ix[p] == ix[k] // 2 and iy[p] == iy[k] // 2
    for k in np.nonzero(fc >= 0)[0][:5000]:
        c = fc[k]
        assert np.all(par[c:c + 4] == k)
        assert set(zip(ix[c:c + 4] - 2 * ix[k], iy[c:c + 4] - 2 * iy[k])) == {(0, 0), (1, 0), (0, 1), (1, 1)}
    assert np.array_equal(fc >= 0, (st & air.NODE_REFINED) > 0)


def test_packed_rho_t_copy_contents(ctx):
    """A one-band (rho, T) field on a uniform grid: the 16-byte records, then
    at the next multiple of 256 bytes the same bricks as (rho, T) pairs (the
    copy the sparse levels march)."""
    from paper_1010_5534_amd import air
    g = inputs.Grid(inputs.GRID_UNIFORM, (5, 5, 5))
    rho = np.arange(125, dtype=np.float32).reshape(5, 5, 5) + 1.0
    T = 1000 + np.arange(125, dtype=np.float32).reshape(5, 5, 5)
    f = inputs.Field(1, rho, temp=T, bands=np.array([[1.0, 1.5, 0.5]]))
    raw = ctx.prepare(air.upload(g, f)).tensors[-1].cpu().numpy().view(np.uint8)
    bricks = 3 * 3 * 3  # odd: the records end off a 256-byte boundary
    main = bricks * 8 * 16
    off = (main + 255) // 256 * 256
    assert off > main and raw.size == off + bricks * 8 * 8
    recs = raw[:main].view(np.float32).reshape(-1, 4)
    copy = raw[off:].view(np.float32).reshape(-1, 2)
    ref = _brick_order(np.stack([rho, T], axis=-1), g.n)
    assert np.array_equal(copy, ref)
    assert np.array_equal(recs[:, 0], ref[:, 0])

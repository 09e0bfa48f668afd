"""Run-twice determinism of every path with dynamic scheduling or atomics
(ticketed tiles, claimed refinements, work-list reservations, per-block
partial sums): each call repeated gives the same bits."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _bits(t):
    return t.contiguous().view(torch.int32) if t.dtype == torch.float32 else t


def _same_render(a, b):
    for x, y in zip(a[0], b[0]):
        assert x.n_nodes == y.n_nodes
        for name in ("level", "ix", "iy", "parent", "first_child", "state", "I", "N", "xi_I", "visits"):
            assert torch.equal(_bits(getattr(x, name)), _bits(getattr(y, name))), name
    if a[1] is not None:
        assert torch.equal(_bits(a[1]), _bits(b[1]))
    assert np.array_equal(a[2], b[2])


def test_block_amr_multiband_twice(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.amr_winds(seed=2, base_cells=64, bs=8, max_level=2, bands=inputs.default_bands(8))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(6, seed=9)
    prm = air.params(64, 3, 0.4)
    say("determinism: block AMR, 6 views x 8 bands, eager and batch")
    a = ctx.render(scene, views, prm, reuse=False)
    b = ctx.render(scene, views, prm, reuse=False)
    _same_render(a, b)
    _same_render(a, ctx.render_batch(scene, views, prm))
    _same_render(a, ctx.render_batch(scene, views, prm))


def test_large_level_ticketed_twice(ctx):
    """A launch with many tiles per block takes them from ticket counters in
    whatever order the blocks arrive; the values do not depend on it."""
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=6, n=128, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(4, seed=2)
    prm = air.params(64, 5, 0.3, band_weight=[1.0, 1.0])
    say("determinism: winds2 128^3, 4 views, 5 levels")
    a = ctx.render(scene, views, prm, want_image=False, reuse=False)
    b = ctx.render(scene, views, prm, want_image=False, reuse=False)
    assert a[3]["rays"] > 100000
    _same_render(a, b)


def test_fixed_and_spectra_twice(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=7, n=48, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(1))
    scene = air.upload(g, f)
    v = inputs.view_for((0.4, -0.3, 0.85))
    say("determinism: fixed image and spectra")
    i1, f1, _ = ctx.render_fixed(scene, [v], 16, 3)
    i2, f2, _ = ctx.render_fixed(scene, [v], 16, 3)
    assert torch.equal(_bits(i1), _bits(i2)) and np.array_equal(f1, f2)
    table, w = inputs.spectral_bins(96)
    s1 = ctx.render_spectra(scene, [v], air.params(12, 3, 0.5), table, w)
    s2 = ctx.render_spectra(scene, [v], air.params(12, 3, 0.5), table, w)
    n = s1[0][0].n_nodes
    assert n == s2[0][0].n_nodes
    assert torch.equal(_bits(s1[1][:, :n]), _bits(s2[1][:, :n]))
    assert np.array_equal(s1[3], s2[3])


def test_learned_and_training_twice(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=8, n=64, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(1))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.winds2_views()
    prm = air.params(16, 4, 0.4)
    net = air.Network(ctx, inputs.cnn_init(3))
    say("determinism: learned render with speculation, network gradient")
    a = ctx.render_learned(scene, views, prm, net, 1.0, 30.0, reuse=False)
    b = ctx.render_learned(scene, views, prm, net, 1.0, 30.0, reuse=False)
    _same_render(a, b)
    assert a[4]["spec_rays"] == b[4]["spec_rays"] and a[4]["wasted"] == b[4]["wasted"]
    rng = np.random.default_rng(4)
    x = torch.from_numpy(rng.normal(size=(6, 40, 36, 4)).astype(np.float32)).cuda()
    lab = torch.from_numpy(rng.integers(0, 6, size=(6, 40, 36)).astype(np.int32)).cuda()
    cw = np.ones(6, np.float32)
    l1, g1 = net.loss_grad(x, lab, cw, want_grad=True)
    l2, g2 = net.loss_grad(x, lab, cw, want_grad=True)
    assert l1 == l2 and torch.equal(_bits(g1), _bits(g2))
    net.close()

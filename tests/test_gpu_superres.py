"""The super-resolution output (section 2 step vi, air_params flag
AIR_FLAG_SUPERRES) through the C ABI: the interpolated raster against the
oracle's interpolation of its own values on the GPU's tree (1e-5 relative per
pixel), full refinement equal to the fixed image bit for bit, and the
batched and learned paths equal to the eager one bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


@pytest.mark.parametrize("case", ["gaussian", "winds 4 bands", "ring"])
def test_superres_matches_oracle(ctx, case):
    from paper_1010_5534_amd import air
    if case == "gaussian":
        g, f = inputs.gaussian()
        v, N0, L, xc, w = inputs.gaussian_view(), 16, 4, 0.5, None
    elif case == "winds 4 bands":
        g, f = inputs.winds2(seed=6, n=48, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(4))
        v, N0, L, xc, w = inputs.view_for((0.4, 0.5, 0.77)), 12, 3, 0.5, [1.0, 0.5, 2.0, 0.25]
    else:
        g, f = inputs.ring()
        v, N0, L, xc, w = inputs.ring_view(), 32, 4, 0.8, None
    scene = ctx.prepare(air.upload(g, f))
    say(f"super-resolution {case}")
    trees, img, flux, st = ctx.render(scene, [v], air.params(N0, L, xc, band_weight=w, superres=True))
    rep = parity.check(trees[0], g, f, v, N0, L, xc, band_w=w, image=img[0], flux=flux[0], superres=True,
                       label=f"superres {case}")
    say(parity.summary(rep))
    parity.assert_parity(rep)


def test_superres_full_refinement_equals_fixed(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.gaussian()
    scene = air.upload(g, f)
    v = inputs.gaussian_view()
    _, img, _, _ = ctx.render(scene, [v], air.params(16, 4, 0.0, superres=True))
    fimg, _, _ = ctx.render_fixed(scene, [v], 16, 4)
    assert torch.equal(img.view(torch.int32), fimg.view(torch.int32))


def test_superres_batch_and_learned_equal_eager(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=2, n=64, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.winds2_views()
    prm = air.params(16, 4, 0.4, superres=True)
    ref = ctx.render(scene, views, prm)
    painted = ctx.render(scene, views, air.params(16, 4, 0.4))
    assert not torch.equal(ref[1], painted[1])  # the flag changes the raster ...
    assert np.array_equal(ref[2], painted[2])   # ... not the flux
    b = ctx.render_batch(scene, views, prm)
    assert torch.equal(b[1].view(torch.int32), ref[1].view(torch.int32))
    net = air.Network(ctx, inputs.cnn_init(5))
    lo = ctx.render_learned(scene, views, prm, net, 1.0, 100.0)
    assert torch.equal(lo[1].view(torch.int32), ref[1].view(torch.int32))
    net.close()

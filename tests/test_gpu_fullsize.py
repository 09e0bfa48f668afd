"""Parity at the full benchmark size: 256^3 two-wind field (seed 0), the
float32 (rho, T) form with one band (j = rho^2 T^0.5, kappa = rho T^-1.5),
64x64 coarse image, 5 levels, xi_crit 0.5, the three views, traced in one
call on the packed field exactly as bench.py times it.  Every node of the
GPU trees is traced by the oracle and compared; the flags are compared with
Eq. 3 on those values; the three painted 2048^2 rasters (intensity and
column) and the fluxes are compared with the oracle's painting of its values
on the GPU's trees; the oracle's own trees are compared too.  The fixed
2048^2 images are compared on a seeded sample of pixels the oracle traces
one by one."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import parity
from paper_1010_5534_amd import inputs

pytestmark = pytest.mark.gpu

N0, LMAX, XC = 64, 5, 0.5
BAND = np.array([[1.0, 1.5, 0.5]])


@pytest.fixture(scope="module")
def setup():
    from paper_1010_5534_amd import air
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("full-size winds2 256^3 seed 0 (rho, T), N0=64, Lmax=5, 3 views", flush=True)
    g, f = inputs.winds2(0, 256, kind=inputs.FIELD_RHO_T, bands=BAND)
    ctx = air.Context(0)
    scene = ctx.prepare(air.upload(g, f))
    yield g, f, ctx, scene
    ctx.close()


def test_fullsize_air_trees(setup):
    from paper_1010_5534_amd import air
    g, f, ctx, scene = setup
    views = inputs.winds2_views()
    trees, img, flux, st = ctx.render(scene, views, air.params(N0, LMAX, XC))
    for k, v in enumerate(views):
        print(f"view {k}: oracle on the GPU tree, raster and flux", flush=True)
        rep = parity.check(trees[k], g, f, v, N0, LMAX, XC, image=img[k], flux=flux[k], own=True,
                           label=f"full size winds2 256^3 view {k}")
        print(parity.summary(rep), flush=True)
        parity.assert_parity(rep)


def test_fullsize_fixed_sampled(setup):
    g, f, ctx, scene = setup
    views = inputs.winds2_views()
    img, flux, st = ctx.render_fixed(scene, views, N0, LMAX)
    R = N0 << LMAX
    rng = np.random.default_rng(2024)
    for k, v in enumerate(views):
        i = rng.integers(0, R, 6000)
        j = rng.integers(0, R, 6000)
        ref = oracle.trace_pixels(g, f, v, N0, np.full(6000, LMAX), i, j)
        gi = img[k].cpu().numpy()
        assert parity.rel_err(gi[0][j, i], ref["I"][0]).max() <= 1e-5
        assert parity.rel_err(gi[1][j, i], ref["N"]).max() <= 1e-5

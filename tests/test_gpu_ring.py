"""The section-3 ring experiment (Eq. 1, Table 1) on the GPU through the C
ABI: the block-AMR ring (4^3 base blocks of 8^3 cells, 4 levels, 512^3
effective), 32^2 base image and 4 image levels at xi_crit 0.2, 0.5 and 0.8,
and the fixed 512^2 image, against the FP64 oracle (trees node by node,
rasters, fluxes) and against Table 1's exact flux, the emission summed over
the grid's leaf cells."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import parity
from paper_1010_5534_amd import inputs
from test_oracle_ring import LMAX, N0, W, grid_sum

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ring():
    from paper_1010_5534_amd import air
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("ring: 4^3 blocks of 8^3 cells, 4 levels")
    g, f = inputs.ring()
    ctx = air.Context(0)
    scene = ctx.prepare(air.upload(g, f))
    yield g, f, inputs.ring_view(), ctx, scene, grid_sum(g, f)
    ctx.close()


def test_ring_fixed_image(ring):
    g, f, v, ctx, scene, exact = ring
    say("ring fixed 512^2")
    img, flux, st = ctx.render_fixed(scene, [v], N0, LMAX)
    assert st["rays"] == 512 * 512
    rel = abs(flux[0][0] - exact) / exact
    say(f"fixed 512^2: flux {flux[0][0]:.9e}, grid sum {exact:.9e}, rel {rel:.2e}")
    assert rel <= 1e-5
    rng = np.random.default_rng(3)
    i, j = rng.integers(0, 512, 5000), rng.integers(0, 512, 5000)
    ref = oracle.trace_pixels(g, f, v, N0, np.full(5000, LMAX), i, j)
    gi = img[0].cpu().numpy()
    assert parity.rel_err(gi[0][j, i], ref["I"][0]).max() <= 1e-5
    assert parity.rel_err(gi[1][j, i], ref["N"]).max() <= 1e-5


@pytest.mark.parametrize("xc", [0.2, 0.5, 0.8])
def test_ring_air_parity(ring, xc):
    from paper_1010_5534_amd import air
    g, f, v, ctx, scene, exact = ring
    say(f"ring AIR xi_crit={xc}")
    trees, img, flux, st = ctx.render(scene, [v], air.params(N0, LMAX, xc))
    rep = parity.check(trees[0], g, f, v, N0, LMAX, xc, image=img[0], flux=flux[0], own=True,
                       label=f"ring xi_crit={xc}")
    say(parity.summary(rep))
    parity.assert_parity(rep)
    n = trees[0].n_nodes
    assert (n - N0 * N0) % 4 == 0
    say(f"Table 1 row: xi_crit {xc}: pixels {n} = 32^2 + 4 x {(n - N0 * N0) // 4}, "
        f"flux error {(exact - flux[0][0]) / exact:.3e}")

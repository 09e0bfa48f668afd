"""Coarse levels traced as split tiles (one wave job per tile and
sub-interval, partials folded in a second launch) give the same bits as the
tile form (S waves of one block folding in LDS): a context with the split
form switched off renders the same trees, images, fluxes and counters."""
import os
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
def ctxs():
    from paper_1010_5534_amd import air
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    on = air.Context(0)
    old = os.environ.get("AIR_SPLIT_TILES")
    os.environ["AIR_SPLIT_TILES"] = "0"
    try:
        off = air.Context(0)
    finally:
        if old is None:
            del os.environ["AIR_SPLIT_TILES"]
        else:
            os.environ["AIR_SPLIT_TILES"] = old
    yield on, off
    on.close()
    off.close()


def _same(a, b):
    for x, y in zip(a[0], b[0]):
        assert x.n_nodes == y.n_nodes
        for name in ("level", "ix", "iy", "parent", "first_child", "state", "I", "N", "visits"):
            assert torch.equal(getattr(x, name), getattr(y, name)), name
        assert torch.equal(x.xi_I.view(torch.int32), y.xi_I.view(torch.int32))
    assert torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
    assert np.array_equal(a[2], b[2])
    for k in ("rays", "hits", "visits", "leaves", "flagged", "balance"):
        assert a[3][k] == b[3][k], k


CASES = [
    ("winds2 one band (rho, j, kappa)", lambda: inputs.winds2(seed=1, n=64), 16, 4, 0.4),
    ("winds2 (rho, T) 2 bands", lambda: inputs.winds2(seed=2, n=48, kind=inputs.FIELD_RHO_T,
                                                      bands=inputs.default_bands(2)), 12, 3, 0.4),
    ("winds2 (rho, T) 4 bands", lambda: inputs.winds2(seed=3, n=48, kind=inputs.FIELD_RHO_T,
                                                      bands=inputs.default_bands(4)), 16, 3, 0.5),
    ("block AMR 8 bands", lambda: inputs.amr_winds(seed=3, base_cells=64, bs=8, max_level=2, frac=(0.10, 0.03),
                                                   bands=inputs.default_bands(8)), 16, 3, 0.5),
]


@pytest.mark.parametrize("name,make,n0,lmax,xc", CASES, ids=[c[0] for c in CASES])
def test_split_tiles_equal_tile_form(ctxs, name, make, n0, lmax, xc):
    from paper_1010_5534_amd import air
    on, off = ctxs
    g, f = make()
    views = inputs.isotropic_views(3, seed=7)
    prm = air.params(n0, lmax, xc)
    say(f"split vs tile form: {name}, N0={n0} Lmax={lmax}")
    a = on.render(on.prepare(air.upload(g, f)), views, prm)
    b = off.render(off.prepare(air.upload(g, f)), views, prm)
    say(a[3]["rays_per_level"][:lmax + 1])
    _same(a, b)

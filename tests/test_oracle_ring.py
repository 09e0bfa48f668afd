"""The section-3 experiment (Eq. 1 ring, Table 1) re-created with the
oracle: a face-on ring on a PARAMESH-like block hierarchy (4^3 base blocks
of 8^3 cells, 4 nested levels, 512^3 effective), a 32^2 base image with 4
image levels against the fixed 512^2 image.  Pinned by the Table 1 caption's
exact flux (the emission summed over the grid's leaf cells): the fixed image
through the cell-column centres of an optically thin grid gives it exactly;
AIR's pixel counts have Table 1's form 32^2 + 4k, and its flux error and
pixel count shrink as xi_crit falls."""
import json
import os

import numpy as np
import pytest

from paper_1010_5534_amd import inputs

N0, LMAX, W = 32, 4, 10.0
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_ring.json")


def grid_sum(g, f):
    """Table 1 caption: the exact flux, summed from the hydrodynamic grid:
    emission times volume over the leaf cells (a refined block's own cells
    are covered by its children)."""
    bs = g.bs
    leaf = np.repeat(np.asarray(g.block_child) < 0, bs ** 3)
    h = (g.hi[0] - g.lo[0]) / (g.n[0] * bs) / 2.0 ** np.repeat(np.asarray(g.block_level), bs ** 3)
    return float(np.sum(np.where(leaf, f.emis.astype(np.float64) * h ** 3, 0.0)))


@pytest.fixture(scope="module")
def ring():
    g, f = inputs.ring()
    return g, f, inputs.ring_view()


def test_ring_hierarchy_and_field(ring):
    g, f, v = ring
    assert g.n == (4, 4, 4) and g.bs == 8 and g.max_level == 4
    assert int(np.asarray(g.block_level).max()) == 4
    # emission only inside the ring (beta / r^2, about 2e-26 g/cm^3, below the
    # 1e-25 g/cm^3 background: 10 in the field's unit of 1e-26), no absorption
    assert np.all(f.kappa == 0) and np.all((f.emis > 0) == (f.rho < 10.0 * (1 - 1e-6)))


def test_fixed_image_flux_is_the_grid_sum(orc, ring):
    g, f, v = ring
    fx = orc.render_fixed(g, f, v, N0, LMAX)
    R = N0 << LMAX
    flux = float(np.sum(fx["I"][0])) * (W / R) ** 2
    assert flux == pytest.approx(grid_sum(g, f), rel=1e-12)
    # the ring fills about 1/8 of the image (section 3's rule of thumb)
    fill = float(np.mean(fx["I"][0] > 0))
    assert 0.08 < fill < 0.2


def test_air_table1_structure(orc, ring):
    g, f, v = ring
    exact = grid_sum(g, f)
    rows = []
    for xc in (0.2, 0.5, 0.8):
        t = orc.air(g, f, v, N0, LMAX, xc)
        err = (exact - orc.leaf_flux(t, W, t.flat_I[0])) / exact
        rows.append((xc, t.nodes, err))
        assert (t.nodes - N0 * N0) % 4 == 0
        assert t.nodes < (N0 << LMAX) ** 2 // 5
    print(rows)
    nodes = [r[1] for r in rows]
    errs = [abs(r[2]) for r in rows]
    assert nodes[0] > nodes[1] > nodes[2]
    assert errs[0] < errs[1] < errs[2] < 0.02


def test_table1_printed_values_fit_the_reading():
    """The printed Table 1 (golden fixture): the fixed image is (32 x 2^4)^2
    pixels and every AIR count is 32^2 + 4k -- a base image of 32^2 and four
    children per refinement, the reading the oracle and the library share
    -- and the counts fall as xi_crit rises."""
    t1 = json.load(open(GOLDEN))
    assert t1["fixed"]["pixels"] == (N0 << LMAX) ** 2
    counts = [r["pixels"] for r in t1["air"]]
    for n in counts:
        assert n > N0 * N0 and (n - N0 * N0) % 4 == 0
    assert counts[0] > counts[1] > counts[2]


def test_air_pixel_counts_near_table1(orc, ring):
    """Our synthetic ring (Eq. 1 on a PARAMESH-like hierarchy; MEKAL emission
    and the FLASH grid are not available) refines to within 25% of the
    pixel counts printed in Table 1 at each xi_crit (measured 0.82, 1.07 and
    0.88 of them).  A loose check of the whole refinement: the criterion
    compared in squares (xi^2 against xi_crit) fails it at xi_crit 0.5
    (1.33), compared as a square root at 0.2 (0.62)."""
    g, f, v = ring
    t1 = json.load(open(GOLDEN))
    for row in t1["air"]:
        t = orc.air(g, f, v, N0, LMAX, row["xi_crit"])
        assert abs(t.nodes / row["pixels"] - 1.0) < 0.25, (row["xi_crit"], t.nodes, row["pixels"])

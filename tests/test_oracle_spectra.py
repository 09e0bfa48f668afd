"""Pins of the oracle's spectral bins (field kind 2: kappa_b = k0 rho T^-s,
j_b = e0 rho^2 T^q exp(-E/T)), the reference of the many-bin spectra.

Closed forms of the constant-coefficient transfer equation per bin, the
reduction to the power-law bands when E = 0 and e0 = 1, and bins that do not
depend on their neighbours in the table (each bin of a 300-bin table equals
that bin traced alone)."""
import math

import numpy as np
import pytest

from paper_1010_5534_amd import inputs


def _uniform_rt(n, rho, T, table):
    g = inputs.Grid(inputs.GRID_UNIFORM, (n, n, n))
    shape = (n, n, n)
    f = inputs.Field(inputs.FIELD_SPECTRAL, np.full(shape, rho, np.float32), temp=np.full(shape, T, np.float32),
                     bands=np.asarray(table, np.float64))
    return g, f


def test_isothermal_box_per_bin(orc):
    """Uniform (rho, T): every bin is the slab solution S_b (1 - e^-tau_b)
    along the chord, S_b = j_b / kappa_b."""
    rho, T = 0.75, 3.0  # exact in float32
    table, _ = inputs.spectral_bins(40)
    g, f = _uniform_rt(6, rho, T, table)
    o, d = (0.5, 0.5, -1.0), (0.2, -0.1, 1.0)
    dn = np.asarray(d) / np.linalg.norm(d)
    # chord: enter at z = 0, leave at z = 1 (x stays in [0.7, 0.9], y in [0.3, 0.4])
    chord = 1.0 / dn[2]
    r = orc.trace(g, f, o, d)
    for b, (k0, s, e0, q, E) in enumerate(table):
        kap = k0 * rho * T ** -s
        j = e0 * rho * rho * T ** q * math.exp(-E / T)
        assert r["I"][b] == pytest.approx(j / kap * (1.0 - math.exp(-kap * chord)), rel=1e-12)
    assert r["N"] == pytest.approx(rho * chord, rel=1e-13)


def test_reduces_to_power_law_bands(orc):
    """E = 0 and e0 = 1 give the power-law bands of field kind 1 bit for bit."""
    g, f = inputs.winds2(seed=3, n=24, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(4))
    tab = np.stack([f.bands[:, 0], f.bands[:, 1], np.ones(4), f.bands[:, 2], np.zeros(4)], axis=1)
    fs = inputs.Field(inputs.FIELD_SPECTRAL, f.rho, temp=f.temp, bands=tab)
    v = inputs.view_for((0.3, 0.8, 0.5))
    a = orc.render_fixed(g, f, v, 6, 1)
    b = orc.render_fixed(g, fs, v, 6, 1)
    assert np.array_equal(a["I"], b["I"]) and np.array_equal(a["N"], b["N"])


def test_bins_independent_of_the_table(orc):
    """A 300-bin table traced at once equals each bin traced alone."""
    g, f = inputs.winds2(seed=1, n=20, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(1))
    table, _ = inputs.spectral_bins(300)
    fs = inputs.Field(inputs.FIELD_SPECTRAL, f.rho, temp=f.temp, bands=table)
    v = inputs.view_for((1, 1, 1))
    rng = np.random.default_rng(0)
    L = np.full(40, 2)
    i, j = rng.integers(0, 16, 40), rng.integers(0, 16, 40)
    allb = orc.trace_pixels(g, fs, v, 4, L, i, j)
    for b in (0, 1, 137, 299):
        one = inputs.Field(inputs.FIELD_SPECTRAL, f.rho, temp=f.temp, bands=table[b:b + 1])
        r = orc.trace_pixels(g, one, v, 4, L, i, j)
        assert np.array_equal(r["I"][0], allb["I"][b])


def test_broadband_weights():
    """The synthetic table's broadband weights are the bin widths inside the
    band and zero outside; the energies rise through the table."""
    table, w = inputs.spectral_bins(64)
    E = table[:, 4]
    assert np.all(np.diff(E) > 0)
    assert np.all((w > 0) == ((E >= 1.0) & (E <= 10.0)))

"""The tree-parity harness (tests/parity.py) on the CPU: a tree built by the
oracle itself, rounded to float32 as a GPU tree would be, passes; mistakes
planted in it (a flag decided against the criterion, with the tree that
follows from it; a value off by 3e-5; a wrong xi output; a missing balance
node) are each caught by the check meant for them."""
import numpy as np
import pytest

import oracle
import parity
from paper_1010_5534_amd import inputs

EVALUATED = 32


class _Arr:
    def __init__(self, a):
        self.a = np.asarray(a)

    def cpu(self):
        return self

    def numpy(self):
        return self.a


class _Tree:
    """Node list in the layout of a GPU tree (level, ix, iy, state, I [nb, n],
    N, xi_I, xi_N), values in float32."""

    def __init__(self, t, nb, vals_I=None, vals_N=None):
        lv, ix, iy, st, I, N, xI, xN = [], [], [], [], [], [], [], []
        for L in range(t.Lmax + 1):
            js, is_ = np.nonzero(t.state[L] & oracle.EXIST)
            s = t.state[L][js, is_].astype(np.uint8)
            ev = ((s & oracle.TESTED) > 0) & (L < t.Lmax) & ~np.isnan(t.xiI[L][js, is_])
            s = s | np.where(ev, EVALUATED, 0).astype(np.uint8)
            lv.append(np.full(js.size, L, np.int8))
            ix.append(is_.astype(np.int32))
            iy.append(js.astype(np.int32))
            st.append(s)
            src_I = t.I[L] if vals_I is None else vals_I[L]
            src_N = t.N[L] if vals_N is None else vals_N[L]
            I.append(src_I[:, js, is_].astype(np.float32))
            N.append(src_N[js, is_].astype(np.float32))
            xI.append(t.xiI[L][js, is_].astype(np.float32))
            xN.append(t.xiN[L][js, is_].astype(np.float32))
        self.level = _Arr(np.concatenate(lv))
        self.ix = _Arr(np.concatenate(ix))
        self.iy = _Arr(np.concatenate(iy))
        self.state = _Arr(np.concatenate(st))
        self.I = _Arr(np.concatenate(I, axis=1))
        self.N = _Arr(np.concatenate(N))
        self.xi_I = _Arr(np.concatenate(xI))
        self.xi_N = _Arr(np.concatenate(xN))
        self.n_nodes = int(self.level.a.size)


N0, LMAX, XC = 8, 3, 0.5


@pytest.fixture(scope="module")
def scene():
    g, f = inputs.gaussian(n=32)
    v = inputs.gaussian_view()
    t = oracle.air(g, f, v, N0, LMAX, XC)
    return g, f, v, t


def test_oracle_tree_as_gpu_tree_passes(scene):
    g, f, v, t = scene
    rep = parity.check(_Tree(t, 1), g, f, v, N0, LMAX, XC, own=True)
    parity.assert_parity(rep)
    assert rep["flips"] == 0 and rep["nodes_oracle_own"] == rep["nodes_gpu"] == t.nodes


def _flipped_tree(g, f, v, t):
    """The tree that follows from the oracle's flags with one flag planted
    against the criterion (a node far from the threshold), traced by the
    oracle: the structure is self-consistent, only the decision is wrong."""
    flags = [((s & oracle.FLAGGED) > 0).astype(np.uint8) for s in t.state]
    L = 1
    js, is_ = np.nonzero((t.state[L] & oracle.TESTED) > 0)
    far = np.abs(t.xiI[L][js, is_] - XC) > 0.2
    k = int(np.nonzero(far & (flags[L][js, is_] == 0))[0][0])
    flags[L][js[k], is_[k]] = 1
    flat = np.concatenate([a.reshape(-1) for a in flags])
    tf = oracle.air(None, None, v, N0, LMAX, force_flags=flat)
    vI, vN = [], []
    for Lv in range(LMAX + 1):
        jj, ii = np.nonzero(tf.state[Lv] & oracle.EXIST)
        r = oracle.trace_pixels(g, f, v, N0, np.full(jj.size, Lv), ii, jj)
        a = np.zeros((1,) + tf.state[Lv].shape)
        a[:, jj, ii] = r["I"]
        b = np.zeros(tf.state[Lv].shape)
        b[jj, ii] = r["N"]
        vI.append(a)
        vN.append(b)
    flatv = lambda x: np.concatenate([a.reshape(a.shape[:-2] + (-1,)) for a in x], axis=-1)
    tx = oracle.air(None, None, v, N0, LMAX, force_flags=flat, values=(flatv(vI), flatv(vN)))
    return tx, vI, vN, (L, int(is_[k]), int(js[k]))


def test_planted_flag_flip_is_set3(scene):
    g, f, v, t = scene
    tx, vI, vN, where = _flipped_tree(g, f, v, t)
    rep = parity.check(_Tree(tx, 1, vI, vN), g, f, v, N0, LMAX, XC)
    assert rep["structure_mismatch"] == 0 and rep["max_rel_I"] <= parity.REL_TOL
    got = [r[:3] for r in rep["set3"]]
    assert where in got
    # the rest are the planted node's own children, whose flags were planted
    # as 0 whatever the criterion says of them
    L, i, j = where
    assert all(r == where or (r[0] == L + 1 and r[1] >> 1 == i and r[2] >> 1 == j) for r in got), got
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)


def test_planted_value_error_is_caught(scene):
    g, f, v, t = scene
    vI = [a.copy() for a in t.I]
    jj, ii = np.nonzero(t.state[2] & oracle.EXIST)
    vI[2][0, jj[3], ii[3]] *= 1 + 3e-5
    rep = parity.check(_Tree(t, 1, vI, None), g, f, v, N0, LMAX, XC)
    assert 2e-5 < rep["max_rel_I"] < 4e-5
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)


def test_planted_xi_output_error_is_caught(scene):
    g, f, v, t = scene
    tr = _Tree(t, 1)
    x = tr.xi_I.a
    k = int(np.nonzero(~np.isnan(x) & (x > 0.05))[0][5])
    x[k] *= 1.001
    rep = parity.check(tr, g, f, v, N0, LMAX, XC)
    assert rep["xi_arith_fail"] == 1
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)


def test_planted_missing_balance_node_is_caught(scene):
    g, f, v, t = scene
    tr = _Tree(t, 1)
    st = tr.state.a
    k = int(np.nonzero((st & oracle.BALANCE) > 0)[0][0])
    keep = np.ones(st.size, bool)
    keep[k] = False
    for name in ("level", "ix", "iy", "state", "N", "xi_I", "xi_N"):
        setattr(tr, name, _Arr(getattr(tr, name).a[keep]))
    tr.I = _Arr(tr.I.a[:, keep])
    tr.n_nodes -= 1
    rep = parity.check(tr, g, f, v, N0, LMAX, XC)
    assert rep["structure_mismatch"] >= 1
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)


def test_raster_and_flux_checked_against_the_gpu_tree(scene):
    g, f, v, t = scene
    tr = _Tree(t, 1)
    img = np.stack([oracle.paint_leaves(t, t.flat_I[0]), oracle.paint_leaves(t, t.flat_N)]).astype(np.float32)
    flux = [oracle.leaf_flux(t, v.width, t.flat_I[0])]
    rep = parity.check(tr, g, f, v, N0, LMAX, XC, image=img, flux=flux)
    parity.assert_parity(rep)
    assert rep["max_rel_image"] <= 1e-7 and rep["rel_flux"] <= 1e-7
    img[0, 5, 7] *= 1.0001
    rep = parity.check(tr, g, f, v, N0, LMAX, XC, image=img, flux=[flux[0] * (1 + 2e-5)])
    assert rep["max_rel_image"] > 5e-5 and rep["rel_flux"] > 1.5e-5


def test_sampled_flags_on_oracle_tree(scene):
    g, f, v, t = scene
    rep = parity.sampled_flags(_Tree(t, 1), g, f, v, N0, LMAX, XC, frac=1.0)
    parity.assert_sampled(rep)
    assert rep["sampled"] == int(sum(np.sum(~np.isnan(t.xiI[L])) for L in range(LMAX)))
    assert rep["flips"] == 0


def test_sampled_flags_catch_planted_flip(scene):
    g, f, v, t = scene
    tx, vI, vN, where = _flipped_tree(g, f, v, t)
    rep = parity.sampled_flags(_Tree(tx, 1, vI, vN), g, f, v, N0, LMAX, XC, frac=1.0)
    assert where in [r[:3] for r in rep["set3"]]
    with pytest.raises(AssertionError):
        parity.assert_sampled(rep)


def test_sampled_flags_agree_with_forced_oracle_run(scene):
    """The sampled check assembles stencils itself; on every evaluated node
    its xi equals the oracle's own forced-run xi on the same values."""
    g, f, v, t = scene
    # the forced run on the tree's own float32 values: its xi, rounded to
    # float32, is what an exact float32 evaluation would output
    flags = np.concatenate([((s & oracle.FLAGGED) > 0).reshape(-1) for s in t.state]).astype(np.uint8)
    v32I = t.flat_I.astype(np.float32).astype(np.float64)
    v32N = t.flat_N.astype(np.float32).astype(np.float64)
    tx = oracle.air(None, None, v, N0, LMAX, force_flags=flags, values=(v32I, v32N))
    tr = _Tree(t, 1)
    tr.xi_I = _Tree(tx, 1).xi_I
    rep = parity.sampled_flags(tr, g, f, v, N0, LMAX, XC, frac=1.0)
    assert rep["xi_arith_fail"] == 0 and rep["max_xi_gpu_err"] <= 1e-7


def test_balance_check_whole_tree(scene):
    g, f, v, t = scene
    assert parity.balanced_everywhere(_Tree(t, 1)) == 0
    flags = [np.zeros((N0 << L, N0 << L), np.uint8) for L in range(LMAX + 1)]
    flags[0][3, 3] = 1
    flags[1][6, 6] = 1
    flags[2][12, 12] = 1
    # the oracle's closure keeps 2:1 ...
    flat = np.concatenate([a.reshape(-1) for a in flags])
    tf = oracle.air(None, None, v, N0, LMAX, force_flags=flat)
    assert parity.balanced_everywhere(_Tree(tf, 1)) == 0
    # ... a tree without it (children of flags only) does not
    st = [np.zeros_like(s) for s in tf.state]
    st[0][:] = oracle.EXIST | oracle.TESTED
    for L in range(LMAX):
        jj, ii = np.nonzero(flags[L] & ((st[L] & oracle.EXIST) > 0))
        st[L][jj, ii] |= oracle.FLAGGED | oracle.REFINED
        for b in range(2):
            for a in range(2):
                st[L + 1][2 * jj + b, 2 * ii + a] = oracle.EXIST | oracle.TESTED
    tf.state = st
    assert parity.balanced_everywhere(_Tree(tf, 1)) > 0

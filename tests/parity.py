"""Parity helpers: GPU pixel trees against the FP64 oracle's trees.

Values: every node present in both trees must agree to REL_TOL relative
(misses are exact zeros on both sides).

Flags: the GPU decides xi >= xi_crit on float32 values, the oracle on
float64 values, so a flag may legitimately differ where the oracle's xi lies
within max(1e-6 xi_crit, B) of the threshold, B being the oracle's own
first-order bound on the change of xi when each stencil input moves by the
value tolerance (oracle.xi_sensitivity).  Such nodes are "ambiguous".  A
differing flag at a non-ambiguous node is a bug.  A legitimate flip changes
the tree locally (children, 2:1 closure down the levels, later stencils):
all of it stays within two coarse pixels of the flip, so coarse pixels
within Chebyshev distance 2 of a flip's coarse pixel are excluded from the
exact structure comparison (values there are still compared on the nodes
both trees share)."""
import numpy as np

import oracle

REL_TOL = 1e-5
FLAG_BAND = 1e-6
BIT_MASK = 1 | 2 | 4 | 8 | 16  # exist, tested, flagged, balance, refined


def gpu_dense(tree, N0, Lmax, nb):
    """Node list (device) -> per-level dense arrays [R, R] indexed [j, i]."""
    n = tree.n_nodes
    lv = tree.level.cpu().numpy().astype(np.int64)
    ix = tree.ix.cpu().numpy().astype(np.int64)
    iy = tree.iy.cpu().numpy().astype(np.int64)
    st = tree.state.cpu().numpy()
    I = tree.I.cpu().numpy().astype(np.float64)
    N = tree.N.cpu().numpy().astype(np.float64)
    xI = tree.xi_I.cpu().numpy()
    xN = tree.xi_N.cpu().numpy()
    out = dict(state=[], I=[], N=[], xiI=[], xiN=[])
    for L in range(Lmax + 1):
        R = N0 << L
        m = lv == L
        s = np.zeros((R, R), np.uint8)
        s[iy[m], ix[m]] = st[m]
        vI = np.zeros((nb, R, R))
        vI[:, iy[m], ix[m]] = I[:, m]
        vN = np.zeros((R, R))
        vN[iy[m], ix[m]] = N[m]
        a = np.full((R, R), np.nan, np.float32)
        a[iy[m], ix[m]] = xI[m]
        b = np.full((R, R), np.nan, np.float32)
        b[iy[m], ix[m]] = xN[m]
        out["state"].append(s)
        out["I"].append(vI)
        out["N"].append(vN)
        out["xiI"].append(a)
        out["xiN"].append(b)
    assert n == sum(int(((s & 1) > 0).sum()) for s in out["state"])
    return out


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(den > 0, np.abs(a - b) / den, np.where(a == 0, 0.0, np.inf))
    return r


def compare(g, t, xc_I, xc_N=2.0, band_w=None, delta=REL_TOL):
    """Compare GPU dense tree g with oracle tree t.  Returns a report."""
    N0, Lmax = t.N0, t.Lmax
    rep = dict(nodes_gpu=int(sum(((s & 1) > 0).sum() for s in g["state"])), nodes_oracle=t.nodes, flips=0,
               ambiguous_flips=[], unexplained_flips=[], ambiguous_nodes=0, max_rel_I=0.0, max_rel_N=0.0,
               structure_mismatch=0, tainted_roots=0)
    flip_roots = set()
    for L in range(Lmax):
        ev_o = (t.state[L] & 2) > 0
        pos, p, hx, hy = oracle.stencils(t, L, "I", band_w)
        xo, sens = oracle.xi_sensitivity(p, hx, hy, delta)
        amb = np.zeros_like(ev_o)
        js, is_ = pos
        amb[js, is_] = np.abs(xo - xc_I) <= np.maximum(FLAG_BAND * xc_I, sens)
        if xc_N <= 1.0:
            posN, pN, hxN, hyN = oracle.stencils(t, L, "N")
            xoN, sensN = oracle.xi_sensitivity(pN, hxN, hyN, delta)
            amb[js, is_] |= np.abs(xoN - xc_N) <= np.maximum(FLAG_BAND * xc_N, sensN)
        rep["ambiguous_nodes"] += int(amb.sum())
        ev_g = (g["state"][L] & 32) > 0
        both = ev_o & ev_g
        fo = (t.state[L] & 4) > 0
        fg = (g["state"][L] & 4) > 0
        flips = both & (fo != fg)
        for j, i in zip(*np.nonzero(flips)):
            rec = (L, int(i), int(j), float(t.xiI[L][j, i]), float(g["xiI"][L][j, i]))
            rep["flips"] += 1
            if amb[j, i]:
                rep["ambiguous_flips"].append(rec)
                flip_roots.add((int(j) >> L, int(i) >> L))
            else:
                rep["unexplained_flips"].append(rec)
    # taint: coarse pixels within distance 2 of a legitimate flip
    taint0 = np.zeros((N0, N0), bool)
    for (rj, ri) in flip_roots:
        taint0[max(0, rj - 2):rj + 3, max(0, ri - 2):ri + 3] = True
    rep["tainted_roots"] = int(taint0.sum())
    nb = t.I[0].shape[0]
    for L in range(Lmax + 1):
        sc = 1 << L
        taint = np.kron(taint0, np.ones((sc, sc), bool))
        so = t.state[L] & BIT_MASK
        sg = g["state"][L] & BIT_MASK
        rep["structure_mismatch"] += int(((so != sg) & ~taint).sum())
        common = ((so & 1) > 0) & ((sg & 1) > 0)
        for b in range(nb):
            r = rel_err(g["I"][L][b][common], t.I[L][b][common])
            if r.size:
                rep["max_rel_I"] = max(rep["max_rel_I"], float(r.max()))
        r = rel_err(g["N"][L][common], t.N[L][common])
        if r.size:
            rep["max_rel_N"] = max(rep["max_rel_N"], float(r.max()))
    return rep


def assert_parity(rep, allow_taint=True):
    assert rep["max_rel_I"] <= REL_TOL, rep["max_rel_I"]
    assert rep["max_rel_N"] <= REL_TOL, rep["max_rel_N"]
    assert not rep["unexplained_flips"], rep["unexplained_flips"][:10]
    assert rep["structure_mismatch"] == 0, rep["structure_mismatch"]
    if not allow_taint:
        assert rep["flips"] == 0

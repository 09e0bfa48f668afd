"""Parity of a GPU pixel tree with the FP64 oracle, node by node on the GPU's
own tree, so one legitimate flag flip cannot cascade into mismatches.

1. Structure: the oracle re-runs the level loop with the GPU's flags forced
   (oracle.air(force_flags=...)): its 2:1 closure and children must give the
   GPU's tree bit for bit (exist, tested, flagged, balance, refined).
2. Values: the oracle traces every GPU node; intensity and column must agree
   to REL_TOL relative (misses are exact zeros on both sides).
3. Criterion: on the same forced tree the oracle evaluates Eq. 3 twice, once
   on its own FP64 values (xi_o) and once on the GPU's float32 values promoted
   to FP64 (xi_g64).  The GPU's float32 xi must match xi_g64 within the
   first-order float32 bound of its inputs (GPU arithmetic check).  A flag
   that differs from the oracle's decision (xi_o >= xi_crit) is
     set 1  allowed:     |xi_o - xi_crit| <= 1e-6 xi_crit;
     set 2  unresolvable in float32: the GPU's decision is the decision of
            Eq. 3 on the GPU's own values (xi_g64, within its float32 bound),
            i.e. the flip comes from the 1e-5-level value differences and not
            from the criterion or the tree logic.  Listed one by one as
            (L, i, j, xi_oracle, xi_gpu, margin, bound) with margin =
            |xi_o - xi_crit| and bound = |xi_g64 - xi_o|;
     set 3  anything else: a bug, must be empty.
4. Output: the GPU raster and flux against the oracle's painting and leaf
   flux of its own values on the GPU's tree (REL_TOL).
5. Optionally (own=True) the oracle's own plain run: with no flips the trees
   are identical; the node count difference is reported either way.
"""
import json
import os

import numpy as np

import oracle

REL_TOL = 1e-5
FLAG_BAND = 1e-6
BIT_MASK = 1 | 2 | 4 | 8 | 16  # exist, tested, flagged, balance, refined
EPS32 = 2.0 ** -24


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
    out = dict(state=[], I=[], N=[], xiI=[], xiN=[], nodes=(lv, ix, iy), node_I=I, node_N=N)
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


def _flat(levels):
    return np.concatenate([a.reshape(a.shape[:-2] + (-1,)) for a in levels], axis=-1)


def _weighted(I_levels, w):
    nb = I_levels[0].shape[0]
    w = np.ones(nb) if w is None else np.asarray(w, dtype=np.float64)[:nb]
    return [np.tensordot(w, a, axes=1) for a in I_levels]


def _forced(view, N0, Lmax, flags_flat, Iw_flat, N_flat):
    return oracle.air(None, None, view, N0, Lmax, 2.0, 2.0, force_flags=flags_flat, values=(Iw_flat, N_flat))


def _stencils_of(tree, L, which, positions):
    """3x3 stencils (as the forced oracle run assembled them) are not exposed;
    rebuild them from the forced tree for the float32 bound: a level-L
    neighbour that was tested exists at test time, otherwise the covering
    level-(L-1) node holds the value."""
    R = tree.N0 << L
    js, is_ = positions
    st = tree.state[L]
    val = tree.N if which == "N" else [a[0] for a in tree.I]
    p = np.zeros((len(js), 9))
    for b in (-1, 0, 1):
        for a in (-1, 0, 1):
            qj, qi = js + b, is_ + a
            ok = (qi >= 0) & (qj >= 0) & (qi < R) & (qj < R)
            qjc, qic = np.clip(qj, 0, R - 1), np.clip(qi, 0, R - 1)
            ex = ((st[qjc, qic] & oracle.EXIST) > 0) & (tree.born[L][qjc, qic] < L)
            v = np.where(ex, val[L][qjc, qic], val[L - 1][qjc // 2, qic // 2] if L > 0 else 0.0)
            p[:, (b + 1) * 3 + (a + 1)] = np.where(ok, v, 0.0)
    hx = ((is_ > 0) & (is_ < R - 1)).astype(np.int32)
    hy = ((js > 0) & (js < R - 1)).astype(np.int32)
    return p, hx, hy


def check(gtree, grid, field, view, N0, Lmax, xc_I, xc_N=2.0, band_w=None, image=None, flux=None, own=False,
          label="", superres=False, ref=None, own_band_w=None):
    """Compare one GPU tree (air.Tree of `view`) with the oracle.  image:
    the view's raster [nb + 1, R, R] (device or host), painted from the leaves
    or, with superres, interpolated (oracle.superres); flux: its [nb] fluxes.
    ref: the oracle's values at the GPU's nodes (I [nb, n], N [n], in the
    tree's node order) when they are computed elsewhere (spectra: the
    broadband of the oracle's bins); else the oracle traces them here.
    own_band_w: the band weights of the oracle's own run when they differ
    from band_w (with ref, the bins' broadband weights).
    Returns a report; assert_parity() applies the bar."""
    nb = field.n_bands if ref is None else np.asarray(ref["I"]).shape[0]
    g = gpu_dense(gtree, N0, Lmax, nb)
    rep = dict(label=label, nodes_gpu=int(gtree.n_nodes), structure_mismatch=0, max_rel_I=0.0, max_rel_N=0.0,
               flips=0, set1=[], set2=[], set3=[], xi_arith_fail=0, max_xi_gpu_err=0.0, ambiguous_band=0,
               max_rel_image=None, rel_flux=None, nodes_oracle_own=None)
    flags = _flat([(s & oracle.FLAGGED) > 0 for s in g["state"]]).astype(np.uint8)
    # 2. oracle values at every GPU node
    lv, ix, iy = g["nodes"]
    if ref is None:
        ref = oracle.trace_pixels(grid, field, view, N0, lv, ix, iy)
    rI = rel_err(g["node_I"], ref["I"])
    rN = rel_err(g["node_N"], ref["N"])
    rep["max_rel_I"] = float(rI.max()) if rI.size else 0.0
    rep["max_rel_N"] = float(rN.max()) if rN.size else 0.0
    # dense oracle values on the GPU's positions
    o_I, o_N = [], []
    for L in range(Lmax + 1):
        R = N0 << L
        m = lv == L
        a = np.zeros((nb, R, R))
        a[:, iy[m], ix[m]] = ref["I"][:, m]
        b = np.zeros((R, R))
        b[iy[m], ix[m]] = ref["N"][m]
        o_I.append(a)
        o_N.append(b)
    # 1. + 3. the forced runs: oracle values and GPU values on the GPU's tree
    t_o = _forced(view, N0, Lmax, flags, _flat(_weighted(o_I, band_w)), _flat(o_N))
    t_g = _forced(view, N0, Lmax, flags, _flat(_weighted(g["I"], band_w)), _flat(g["N"]))
    for L in range(Lmax + 1):
        rep["structure_mismatch"] += int(((t_o.state[L] & BIT_MASK) != (g["state"][L] & BIT_MASK)).sum())
    # float32 bound of the GPU's xi: each stencil input carries the rounding
    # of its band sum (nb terms) and of the estimate's own arithmetic
    delta = (nb + 8) * EPS32
    for L in range(Lmax):
        ev = (g["state"][L] & 32) > 0
        tested = (t_o.state[L] & oracle.TESTED) > 0
        if not np.array_equal(ev, tested):
            rep["structure_mismatch"] += int((ev != tested).sum())
        js, is_ = np.nonzero(ev & tested)
        if js.size == 0:
            continue
        fg = (g["state"][L][js, is_] & oracle.FLAGGED) > 0
        dec_o = np.zeros(js.size, bool)     # oracle decision on its own values
        dec_g64 = np.zeros(js.size, bool)   # Eq. 3 decision on the GPU's values
        in_band = np.zeros(js.size, bool)
        near = np.zeros(js.size, bool)
        margin = np.full(js.size, np.inf)
        bound = np.zeros(js.size)
        for which, xc in (("I", xc_I), ("N", xc_N)):
            if which == "N" and xc_N > 1.0:
                continue
            xo = (t_o.xiI if which == "I" else t_o.xiN)[L][js, is_]
            xg64 = (t_g.xiI if which == "I" else t_g.xiN)[L][js, is_]
            xg = (g["xiI"] if which == "I" else g["xiN"])[L][js, is_].astype(np.float64)
            p, hx, hy = _stencils_of(t_g, L, which, (js, is_))
            _, sens = oracle.xi_sensitivity(p, hx, hy, delta)
            tol = np.maximum(sens, 4 * EPS32)
            err = np.abs(xg - xg64)
            rep["max_xi_gpu_err"] = max(rep["max_xi_gpu_err"], float(np.nanmax(err)) if err.size else 0.0)
            rep["xi_arith_fail"] += int(np.sum(~(err <= tol)))
            dec_o |= xo >= xc
            dec_g64 |= xg64 >= xc
            band = np.abs(xo - xc) <= FLAG_BAND * xc
            rep["ambiguous_band"] += int(band.sum())
            in_band |= band
            near |= np.abs(xg64 - xc) <= tol
            margin = np.minimum(margin, np.abs(xo - xc))
            bound = np.maximum(bound, np.abs(xg64 - xo))
        explained = (dec_g64 == fg) | near
        flips = dec_o != fg
        for k in np.nonzero(flips)[0]:
            j, i = int(js[k]), int(is_[k])
            rec = (L, i, j, float(t_o.xiI[L][j, i]), float(g["xiI"][L][j, i]), float(margin[k]), float(bound[k]))
            rep["flips"] += 1
            if in_band[k]:
                rep["set1"].append(rec)
            elif explained[k]:
                rep["set2"].append(rec)
            else:
                rep["set3"].append(rec)
    # 4. raster and flux against the oracle's values painted on the GPU's tree
    if image is not None:
        img = image.cpu().numpy() if hasattr(image, "cpu") else np.asarray(image)
        worst = 0.0
        for b in range(nb + 1):
            vals = _flat([o_I[L][b] for L in range(Lmax + 1)]) if b < nb else _flat(o_N)
            ref_img = oracle.superres(t_o, vals) if superres else oracle.paint_leaves(t_o, vals)
            worst = max(worst, float(rel_err(img[b], ref_img).max()))
        rep["max_rel_image"] = worst
    if flux is not None:
        worst = 0.0
        for b in range(nb):
            ref_f = oracle.leaf_flux(t_o, view.width, _flat([o_I[L][b] for L in range(Lmax + 1)]))
            worst = max(worst, float(rel_err(np.asarray(flux)[b], ref_f)))
        rep["rel_flux"] = worst
    # 5. the oracle's own tree
    if own:
        t = oracle.air(grid, field, view, N0, Lmax, xc_I, xc_N, band_w=band_w if own_band_w is None else own_band_w)
        rep["nodes_oracle_own"] = t.nodes
        rep["own_structure_diff"] = int(sum(((t.state[L] & BIT_MASK) != (g["state"][L] & BIT_MASK)).sum()
                                            for L in range(Lmax + 1)))
    _record(rep)
    return rep


def summary(rep):
    """Report without the per-flip lists (their lengths instead), plus every
    flip outside the 1e-6 band, one per line."""
    s = {k: (len(v) if isinstance(v, list) else v) for k, v in rep.items()}
    lines = [str(s)]
    for name in ("set2", "set3"):
        for r in rep[name]:
            lines.append(f"  {name} flip L={r[0]} i={r[1]} j={r[2]} xi_oracle={r[3]:.9g} xi_gpu={r[4]:.9g} "
                         f"margin={r[5]:.3g} bound={r[6]:.3g}")
    return "\n".join(lines)


def _record(rep):
    """Append the report to parity_flips.jsonl in the folder that the
    AIR_PARITY_LOG environment variable names, when it is set, so listed
    flips can be collected after a run (the test output prints them too)."""
    d = os.environ.get("AIR_PARITY_LOG")
    if not d or not os.path.isdir(d):
        return
    rec = {k: v for k, v in rep.items()}
    with open(os.path.join(d, "parity_flips.jsonl"), "a") as fh:
        fh.write(json.dumps(rec) + "\n")


def assert_parity(rep):
    assert rep["structure_mismatch"] == 0, rep["structure_mismatch"]
    assert rep["max_rel_I"] <= REL_TOL, rep["max_rel_I"]
    assert rep["max_rel_N"] <= REL_TOL, rep["max_rel_N"]
    assert rep["xi_arith_fail"] == 0, (rep["xi_arith_fail"], rep["max_xi_gpu_err"])
    assert not rep["set3"], rep["set3"][:10]
    if rep["max_rel_image"] is not None:
        assert rep["max_rel_image"] <= REL_TOL, rep["max_rel_image"]
    if rep["rel_flux"] is not None:
        assert rep["rel_flux"] <= REL_TOL, rep["rel_flux"]
    if rep["nodes_oracle_own"] is not None and rep["flips"] == 0:
        assert rep["own_structure_diff"] == 0 and rep["nodes_oracle_own"] == rep["nodes_gpu"]


def _keys(L, i, j):
    return (np.asarray(L, np.int64) << 42) | (np.asarray(j, np.int64) << 21) | np.asarray(i, np.int64)


def sampled_flags(gtree, grid, field, view, N0, Lmax, xc_I, band_w=None, frac=0.01, seed=0, label=""):
    """Flag parity on a seeded sample of the evaluated nodes of a tree too
    large for the whole-tree check: for each sampled level-L node the oracle
    traces its 3x3 stencil as the test read it (a level-L neighbour if it was
    tested at level L, i.e. existed when level L was tested, otherwise the
    covering level-(L-1) node), evaluates Eq. 3, and the GPU's flag is
    classified into the three sets of check().  The stencil nodes' values are
    compared too."""
    nb = field.n_bands
    lv = gtree.level.cpu().numpy().astype(np.int64)
    ix = gtree.ix.cpu().numpy().astype(np.int64)
    iy = gtree.iy.cpu().numpy().astype(np.int64)
    st = gtree.state.cpu().numpy()
    I = gtree.I.cpu().numpy().astype(np.float64)
    N = gtree.N.cpu().numpy().astype(np.float64)
    xg_all = gtree.xi_I.cpu().numpy().astype(np.float64)
    w = np.ones(nb) if band_w is None else np.asarray(band_w, np.float64)[:nb]
    Iw = w @ I
    keys = _keys(lv, ix, iy)
    order = np.argsort(keys)
    skeys = keys[order]
    tested = np.sort(keys[(st & oracle.TESTED) > 0])
    ev = np.nonzero((st & 32) > 0)[0]
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(ev, size=max(1, int(len(ev) * frac)), replace=False))
    n = pick.size
    L, i0, j0 = lv[pick], ix[pick], iy[pick]
    R = N0 << L
    src = np.zeros((n, 9), np.int64)
    inside = np.zeros((n, 9), bool)
    for b in (-1, 0, 1):
        for a in (-1, 0, 1):
            k = (b + 1) * 3 + (a + 1)
            qi, qj = i0 + a, j0 + b
            ok = (qi >= 0) & (qj >= 0) & (qi < R) & (qj < R)
            qi, qj = np.clip(qi, 0, R - 1), np.clip(qj, 0, R - 1)
            kq = _keys(L, qi, qj)
            pos = np.searchsorted(tested, kq)
            was = (pos < tested.size) & (tested[np.minimum(pos, tested.size - 1)] == kq)
            # a tested node's own position is always level L; a neighbour that
            # was not tested then reads the covering node one level up
            ks = np.where(was, kq, _keys(np.maximum(L - 1, 0), qi >> 1, qj >> 1))
            src[:, k] = ks
            inside[:, k] = ok
    p = np.searchsorted(skeys, src.reshape(-1))
    found = (p < skeys.size) & (skeys[np.minimum(p, skeys.size - 1)] == src.reshape(-1))
    need = found | ~inside.reshape(-1)
    rep = dict(label=label, sampled=int(n), missing_source=int(np.sum(~need)), flips=0, set1=[], set2=[], set3=[],
               xi_arith_fail=0, max_xi_gpu_err=0.0, max_rel_I=0.0, max_rel_N=0.0)
    idx = order[np.minimum(p, skeys.size - 1)]
    # the oracle traces every distinct source node once
    uniq, inv = np.unique(src.reshape(-1), return_inverse=True)
    uL, uj, ui = uniq >> 42, (uniq >> 21) & ((1 << 21) - 1), uniq & ((1 << 21) - 1)
    ref = oracle.trace_pixels(grid, field, view, N0, uL, ui, uj)
    o_w = (w @ ref["I"])[inv]
    g_idx = idx
    rI = rel_err(I[:, g_idx][:, inside.reshape(-1)], ref["I"][:, inv][:, inside.reshape(-1)])
    rN = rel_err(N[g_idx][inside.reshape(-1)], ref["N"][inv][inside.reshape(-1)])
    rep["max_rel_I"] = float(rI.max()) if rI.size else 0.0
    rep["max_rel_N"] = float(rN.max()) if rN.size else 0.0
    po = np.where(inside.reshape(-1), o_w, 0.0).reshape(n, 9)
    pg = np.where(inside.reshape(-1), Iw[g_idx], 0.0).reshape(n, 9)
    hx = ((i0 > 0) & (i0 < R - 1)).astype(np.int32)
    hy = ((j0 > 0) & (j0 < R - 1)).astype(np.int32)
    xo, _ = oracle.xi_sensitivity(po, hx, hy, 0.0)
    xg64, sens = oracle.xi_sensitivity(pg, hx, hy, (nb + 8) * EPS32)
    tol = np.maximum(sens, 4 * EPS32)
    xg = xg_all[pick]
    err = np.abs(xg - xg64)
    rep["max_xi_gpu_err"] = float(err.max()) if err.size else 0.0
    rep["xi_arith_fail"] = int(np.sum(~(err <= tol)))
    fg = (st[pick] & oracle.FLAGGED) > 0
    fo = xo >= xc_I
    band = np.abs(xo - xc_I) <= FLAG_BAND * xc_I
    explained = ((xg64 >= xc_I) == fg) | (np.abs(xg64 - xc_I) <= tol)
    for k in np.nonzero(fo != fg)[0]:
        rec = (int(L[k]), int(i0[k]), int(j0[k]), float(xo[k]), float(xg[k]), float(abs(xo[k] - xc_I)),
               float(abs(xg64[k] - xo[k])))
        rep["flips"] += 1
        rep["set1" if band[k] else "set2" if explained[k] else "set3"].append(rec)
    _record(rep)
    return rep


def assert_sampled(rep):
    assert rep["missing_source"] == 0, rep["missing_source"]
    assert rep["max_rel_I"] <= REL_TOL and rep["max_rel_N"] <= REL_TOL, (rep["max_rel_I"], rep["max_rel_N"])
    assert rep["xi_arith_fail"] == 0, (rep["xi_arith_fail"], rep["max_xi_gpu_err"])
    assert not rep["set3"], rep["set3"][:10]


def balanced_everywhere(gtree):
    """2:1 rule on the whole tree: every leaf's 8 neighbour positions at its
    level (inside the image) exist, or their parent one level coarser exists.
    Returns the number of violations."""
    lv = gtree.level.cpu().numpy().astype(np.int64)
    ix = gtree.ix.cpu().numpy().astype(np.int64)
    iy = gtree.iy.cpu().numpy().astype(np.int64)
    st = gtree.state.cpu().numpy()
    keys = np.sort(_keys(lv, ix, iy))
    leaf = ((st & oracle.EXIST) > 0) & ((st & oracle.REFINED) == 0)
    L, i, j = lv[leaf], ix[leaf], iy[leaf]
    bad = 0
    N0 = int(np.sqrt(np.sum(lv == 0)))
    R = N0 << L
    for b in (-1, 0, 1):
        for a in (-1, 0, 1):
            if a == 0 and b == 0:
                continue
            qi, qj = i + a, j + b
            ok = (qi >= 0) & (qj >= 0) & (qi < R) & (qj < R) & (L > 0)
            kq = _keys(L, qi, qj)[ok]
            kp = _keys(L - 1, qi >> 1, qj >> 1)[ok]
            has = lambda k: (np.searchsorted(keys, k) < keys.size) & (keys[np.minimum(np.searchsorted(keys, k), keys.size - 1)] == k)
            bad += int(np.sum(~(has(kq) | has(kp))))
    return bad

"""GPU checks of the learned depth proposal through the C ABI: the network's
bf16 MFMA forward and backward against the FP64 reference (oracle/cnn.py)
on identical inputs, the Adam step, the coarse feature maps and depth
labels against the FP64 AIR oracle, and air_render_learned equal to
air_render bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import parity
from oracle import cnn as ocnn
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


def he_params(seed):
    return inputs.cnn_init(seed)


def _maps(seed, n, h, w):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, h, w, 4)).astype(np.float32)
    labels = rng.integers(0, 6, size=(n, h, w)).astype(np.int32)
    return x, labels


# ------------------------------------------------------------------ network
# Element-wise parity, layer by layer: every layer is fed the GPU's own
# bfloat16 input (read back with air_cnn_tensor), the FP64 reference computes
# the same layer on it, and each output element must lie within the float32
# accumulation bound 4 K 2^-24 sum|a b| of the exact value (K products per
# output), plus half a bfloat16 step where the kernel rounds its output.
EPS32 = 2.0 ** -24


def _f64(t):
    return t.float().cpu().numpy().astype(np.float64)


def _half_ulp_bf16(a):
    a = np.abs(a)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 8), 2.0 ** -133)


def _bad(got, exact, tol, name):
    """Elements outside the bound (there must be none)."""
    viol = ~(np.abs(got - exact) <= tol)
    k = int(viol.sum())
    if k:
        i = np.argmax(np.abs(got - exact) - tol)
        say(f"{name}: {k} of {got.size} outside; worst got {got.flat[i]!r} exact {exact.flat[i]!r} "
            f"tol {tol.flat[i]!r}")
    return k


def _forward_layers(net, theta, x, mean, scale, shape):
    """Checks of every forward layer; returns the GPU's tensors."""
    n, h, w = shape
    P = n * h * w
    T = {k: net.tensor(k, P) for k in ("x0", "a1", "a2", "a3", "z")}
    acts = [_f64(T["x0"]).reshape(n, h, w, 8), _f64(T["a1"]).reshape(n, h, w, 32),
            _f64(T["a2"]).reshape(n, h, w, 32), _f64(T["a3"]).reshape(n, h, w, 32)]
    z = T["z"].cpu().numpy().astype(np.float64).reshape(n, h, w, 8)
    bad = 0
    xs = (x.astype(np.float64) - mean) / scale
    # (x - mean) * (1 / scale) in float32: three roundings
    tol_x = 4 * EPS32 * (np.abs(x.astype(np.float64)) + np.abs(mean)) / scale
    bad += _bad(acts[0][..., :4], xs, _half_ulp_bf16(acts[0][..., :4]) + tol_x, "x0")
    assert np.all(acts[0][..., 4:] == 0)
    p = ocnn.unpack(theta.astype(np.float64))
    cin = [4, 32, 32, 32]
    for l in range(4):
        a_in = acts[l][..., :cin[l]]
        wl = ocnn.bf16(p[f"w{l}"])
        y = ocnn.conv3x3(a_in, wl, p[f"b{l}"])
        tol = 4 * (9 * cin[l] + 1) * EPS32 * ocnn.conv3x3(np.abs(a_in), np.abs(wl), np.abs(p[f"b{l}"]))
        if l < 3:
            out = acts[l + 1]
            bad += _bad(out, np.maximum(y, 0.0), _half_ulp_bf16(out) + tol, f"layer {l} output")
        else:
            bad += _bad(z[..., :6], y, tol, "logits")
    return T, acts, z, bad


@pytest.mark.parametrize("n,h,w", [(2, 64, 64), (3, 13, 21)])
def test_forward_layers_elementwise(ctx, n, h, w):
    from paper_1010_5534_amd import air
    theta = he_params(1)
    mean = np.array([0.1, -0.2, 0.3, 0.0], np.float32)
    scale = np.array([1.5, 0.5, 2.0, 1.0], np.float32)
    net = air.Network(ctx, theta, mean, scale)
    x, _ = _maps(2, n, h, w)
    say(f"cnn forward n={n} {h}x{w}, layer by layer")
    z = net.forward(torch.from_numpy(x).cuda())
    T, acts, zt, bad = _forward_layers(net, theta, x, mean.astype(np.float64), scale.astype(np.float64), (n, h, w))
    assert torch.equal(T["z"].reshape(z.shape), z)
    assert bad == 0
    net.close()


# (3, 13, 21): 819 pixels, a ragged last 64-pixel chunk of the weight
# gradient, rows of a width that is not a multiple of 4 (pixel quads cross
# rows) and map borders inside chunks; (1, 3, 5): a single partial chunk
@pytest.mark.parametrize("n,h,w", [(2, 64, 64), (3, 13, 21), (1, 3, 5)])
def test_backward_layers_elementwise(ctx, n, h, w):
    from paper_1010_5534_amd import air
    theta = he_params(3)
    net = air.Network(ctx, theta)
    P = n * h * w
    x, labels = _maps(4, n, h, w)
    cw = np.array([0.5, 1.0, 2.0, 1.5, 3.0, 4.0], np.float32)
    say(f"cnn loss and gradient n={n} {h}x{w}, layer by layer")
    loss, g = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(labels).cuda(), cw, want_grad=True)
    g = g.cpu().numpy().astype(np.float64)
    T, acts, z, bad = _forward_layers(net, theta, x, 0.0, 1.0, (n, h, w))
    # the loss and its logit gradient, from the GPU's logits
    lref, dz = ocnn.loss_and_logit_grad(z[..., :6], labels, cw.astype(np.float64))
    assert loss == pytest.approx(lref, rel=1e-5)
    DZ = _f64(net.tensor("dz", P)).reshape(n, h, w, 8)
    assert np.all(DZ[..., 6:] == 0)
    wpix = cw.astype(np.float64)[labels] / cw.astype(np.float64)[labels].sum()
    onehot = np.eye(6)[labels]
    tol_dz = 32 * EPS32 * (ocnn.softmax(z[..., :6]) + onehot) * wpix[..., None]
    bad += _bad(DZ[..., :6], dz, _half_ulp_bf16(DZ[..., :6]) + tol_dz, "logit gradient")
    # gradients at the inputs of layers 3..1, each from the GPU's own
    # gradient of the layer above, masked by the stored activation
    p = ocnn.unpack(theta.astype(np.float64))
    D = {4: DZ[..., :6]}
    cout = {3: 6, 2: 32, 1: 32}
    for l in (3, 2, 1):
        dy = D[l + 1]
        wl = ocnn.bf16(p[f"w{l}"])
        v = ocnn.conv3x3_input_grad(dy, wl) * (acts[l] > 0)
        tol = 4 * 9 * cout[l] * EPS32 * ocnn.conv3x3_input_grad(np.abs(dy), np.abs(wl))
        got = _f64(net.tensor(f"d{l}", P)).reshape(n, h, w, 32)
        bad += _bad(got, v, _half_ulp_bf16(got) + tol, f"gradient at a{l}")
        D[l] = got
    # weight and bias gradients of every layer from the GPU's (dy, input)
    cin = [4, 32, 32, 32]
    for l in range(4):
        dy = D[l + 1]
        xin = acts[l][..., :cin[l]]
        dw, db = ocnn.conv3x3_weight_grad(dy, xin)
        sw, sb = ocnn.conv3x3_weight_grad(np.abs(dy), np.abs(xin))
        K = n * h * w
        for name, exact, s_abs in ((f"w{l}", dw, sw), (f"b{l}", db, sb)):
            off, shape = [(o, sh) for nm, sh, o in ocnn.layout() if nm == name][0]
            got = g[off:off + int(np.prod(shape))].reshape(shape)
            bad += _bad(got, exact, 4 * K * EPS32 * s_abs + 1e-30, f"gradient {name}")
    assert bad == 0
    net.close()


def test_adam_step_matches_reference(ctx):
    from paper_1010_5534_amd import air
    theta = he_params(5)
    net = air.Network(ctx, theta)
    x, labels = _maps(6, 1, 32, 32)
    cw = np.ones(6, np.float32)
    m = np.zeros(ocnn.N_PARAMS)
    v = np.zeros(ocnn.N_PARAMS)
    th = theta.astype(np.float64)
    for t in (1, 2, 3):
        _, g = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(labels).cuda(), cw, want_loss=False,
                             want_grad=True)
        net.adam(lr=1e-3)
        th, m, v = ocnn.adam_step(th, g.cpu().numpy().astype(np.float64), m, v, t, lr=1e-3)
        got, _, _ = net.get()
        assert np.max(np.abs(got - th)) <= 1e-6, t
        th = got.astype(np.float64)  # continue from the device's float32 state


def test_training_lowers_the_loss(ctx):
    from paper_1010_5534_amd import air
    net = air.Network(ctx, he_params(7))
    rng = np.random.default_rng(8)
    x = rng.normal(size=(8, 32, 32, 4)).astype(np.float32)
    # a learnable rule: the class follows the first map's value
    labels = np.clip(np.floor((x[..., 0] + 1.5) * 2), 0, 5).astype(np.int32)
    xt, lt = torch.from_numpy(x).cuda(), torch.from_numpy(labels).cuda()
    cw = np.ones(6, np.float32)
    first, _ = net.loss_grad(xt, lt, cw)
    for _ in range(60):
        net.loss_grad(xt, lt, cw, want_loss=False)
        net.adam(lr=3e-3)
    last, _ = net.loss_grad(xt, lt, cw)
    say(f"loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first


# ------------------------------------------------------- features and labels
def test_features_match_oracle(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=3, n=64, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = air.upload(g, f)
    views = [inputs.view_for((0.3, 0.5, 0.8)), inputs.view_for((1, 0, 0), width=1.6)]
    w = [1.0, 0.5]
    feat = ctx.features(scene, views, 16, w).cpu().numpy().astype(np.float64)
    for k, v in enumerate(views):
        t = oracle.air(g, f, v, 16, 0, 2.0, band_w=w, want_rho_range=True)
        Iw = w[0] * t.I[0][0] + w[1] * t.I[0][1]
        hit = t.lmax[0] >= 0
        ref = ocnn.features(Iw, t.N[0], t.lmax[0], t.rmin[0], t.rmax[0], hit, np.zeros(4), np.ones(4))
        assert np.array_equal(feat[k][..., 2], ref[..., 2])           # level crossed: exact
        assert np.abs(feat[k][..., :2] - ref[..., :2]).max() <= 1e-5  # log10 of values within 1e-5 relative
        assert np.abs(feat[k][..., 3] - ref[..., 3]).max() <= 1e-5


def test_tree_depth_labels(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.gaussian()
    scene = air.upload(g, f)
    v = inputs.gaussian_view()
    trees, _, _, _ = ctx.render(scene, [v], air.params(16, 4, 0.5))
    d = ctx.tree_depth(trees[0], 16).cpu().numpy()
    # the label's definition on the same tree: deepest node per coarse pixel
    lv = trees[0].level.cpu().numpy().astype(np.int64)
    ix, iy = trees[0].ix.cpu().numpy(), trees[0].iy.cpu().numpy()
    ref = np.zeros((16, 16), np.int64)
    np.maximum.at(ref, (iy >> lv, ix >> lv), lv)
    assert np.array_equal(d, ref)
    # and the oracle's labels wherever the two trees agree on the coarse pixel
    rep = parity.check(trees[0], g, f, v, 16, 4, 0.5, own=True, label="depth labels")
    parity.assert_parity(rep)
    if rep["flips"] == 0:
        assert np.array_equal(d, ocnn.depth_labels(oracle.air(g, f, v, 16, 4, 0.5)))


# ----------------------------------------------------------- learned render
def _assert_same(a, b):
    ta, ia, fa = a[0], a[1], a[2]
    tb, ib, fb = b[0], b[1], b[2]
    for x, y in zip(ta, tb):
        assert x.n_nodes == y.n_nodes and x.n_per_level == y.n_per_level
        for name in ("level", "ix", "iy", "parent", "first_child", "state", "I", "N", "visits"):
            assert torch.equal(getattr(x, name), getattr(y, name)), name
        assert torch.equal(x.xi_I.view(torch.int32), y.xi_I.view(torch.int32))
    assert torch.equal(ia.view(torch.int32), ib.view(torch.int32))
    assert np.array_equal(fa, fb)


@pytest.mark.parametrize("c_ray,c_sweep", [(1.0, 0.0), (0.0, 1.0), (1.0, 300.0), (1.0, 30.0)])
def test_learned_equals_plain_bitwise(ctx, c_ray, c_sweep):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=4, n=64)
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.winds2_views()
    prm = air.params(16, 4, 0.4)
    net = air.Network(ctx, he_params(9), np.array([-3.0, -1.0, 0.0, 1.0], np.float32), np.full(4, 2.0, np.float32))
    plain = ctx.render(scene, views, prm)
    say(f"learned winds2 n=64 c_ray={c_ray} c_sweep={c_sweep}")
    learned = ctx.render_learned(scene, views, prm, net, c_ray, c_sweep)
    _assert_same(plain, learned)
    ls = learned[4]
    say(ls)
    nodes_above0 = sum(t.n_nodes - t.n_per_level[0] for t in plain[0])
    # every tree node above level 0 was speculative or missing
    assert ls["spec_rays"] - ls["wasted"] + ls["missing"] == nodes_above0
    assert sum(ls["depth_hist"]) == 3 * 16 * 16
    if c_sweep == 0.0:
        assert ls["spec_rays"] == 0 and ls["missing"] == nodes_above0
    if c_ray == 0.0:  # free rays: the full depth unless deeper classes have probability 0 in float32
        assert ls["depth_hist"][4] >= 0.9 * 3 * 16 * 16
    # the chosen depths follow the reference decision on the device's logits
    feat = ctx.features(scene, views, 16)
    z = net.forward(feat).cpu().numpy()[..., :6]
    d_ref, cost = ocnn.decide_depth(z, c_ray, c_sweep, max_depth=4)
    hist = np.bincount(d_ref.ravel(), minlength=6)
    srt = np.sort(cost[..., :5], axis=-1)
    near = int(np.sum(srt[..., 1] - srt[..., 0] <= 1e-5 * np.abs(srt[..., 0]) + 1e-12))
    assert np.abs(hist[:5] - np.asarray(ls["depth_hist"][:5])).sum() <= 2 * near
    net.close()


@pytest.mark.parametrize("n0,nviews", [(16, 3), (32, 8), (64, 16)])
def test_fused_inference_tile_sizes(ctx, n0, nviews):
    """The fused inference runs 4x4 tiles on the smallest launches (3 views
    of 16^2: 12 tiles of 8x8), 8x8 tiles on small ones (8 views of 32^2: 128)
    and 16x16 tiles on large ones (16 views of 64^2: 256 tiles of 16x16):
    the chosen depths follow the reference decision on the layer-by-layer
    logits."""
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=6, n=64)
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(nviews, seed=2)
    prm = air.params(n0, 2, 0.4)
    net = air.Network(ctx, he_params(4), np.array([-3.0, -1.0, 0.0, 1.0], np.float32), np.full(4, 2.0, np.float32))
    say(f"fused inference n0={n0} views={nviews}")
    plain = ctx.render(scene, views, prm)
    learned = ctx.render_learned(scene, views, prm, net, 1.0, 30.0)
    _assert_same(plain, learned)
    ls = learned[4]
    z = net.forward(ctx.features(scene, views, n0)).cpu().numpy()[..., :6]
    d_ref, cost = ocnn.decide_depth(z, 1.0, 30.0, max_depth=2)
    hist = np.bincount(d_ref.ravel(), minlength=6)
    srt = np.sort(cost[..., :3], axis=-1)
    near = int(np.sum(srt[..., 1] - srt[..., 0] <= 1e-5 * np.abs(srt[..., 0]) + 1e-12))
    assert sum(ls["depth_hist"]) == nviews * n0 * n0
    assert np.abs(hist[:3] - np.asarray(ls["depth_hist"][:3])).sum() <= 2 * near
    net.close()


def test_learned_equals_plain_amr_multiband(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.amr_winds(seed=1, base_cells=32, bs=4, max_level=2, frac=(0.2, 0.05),
                            bands=inputs.default_bands(3))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(4, seed=2)
    prm = air.params(12, 3, 0.5, band_weight=[1.0, 0.3, 0.1])
    net = air.Network(ctx, he_params(10))
    plain = ctx.render(scene, views, prm)
    learned = ctx.render_learned(scene, views, prm, net, 1.0, 50.0, max_depth=3)
    _assert_same(plain, learned)
    net.close()


def test_learned_render_matches_oracle(ctx):
    """The learned render is also a plain render to the oracle's bar."""
    from paper_1010_5534_amd import air
    g, f = inputs.gaussian()
    scene = air.upload(g, f)
    v = inputs.gaussian_view()
    net = air.Network(ctx, he_params(11))
    trees, img, flux, st, ls = ctx.render_learned(scene, [v], air.params(16, 4, 0.5), net, 1.0, 100.0)
    rep = parity.check(trees[0], g, f, v, 16, 4, 0.5, image=img[0], flux=flux[0], own=True,
                       label="learned render")
    parity.assert_parity(rep)
    net.close()


def test_learned_argument_errors(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.gaussian(16)
    scene = air.upload(g, f)
    net = air.Network(ctx)
    for c_ray, c_sweep, md in [(-1.0, 1.0, 3), (1.0, float("nan"), 3), (1.0, 1.0, -1)]:
        with pytest.raises(air.AirError) as e:
            ctx.render_learned(scene, [inputs.gaussian_view()], air.params(8, 2), net, c_ray, c_sweep, md)
        assert e.value.code == air.AIR_EINVAL
    with pytest.raises(air.AirError):
        net.set(np.full(air.CNN_PARAMS, np.nan, np.float32))
    with pytest.raises(air.AirError):
        net.set(np.zeros(air.CNN_PARAMS, np.float32), scale=np.zeros(4, np.float32))
    net.close()


# ----------------------------------------------- proposal baselines (config 4)
def test_proposal_baselines_equal_plain(ctx):
    """Speculation to a given depth (air_render_proposal): constant depths
    0, 1, 2 and the deepest possible, and the true depths of the plain tree,
    all give air_render's outputs bit for bit; the counters follow from the
    depths (with the true depths no tree node is left for the level loop)."""
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=6, n=64)
    scene = ctx.prepare(air.upload(g, f))
    views = [inputs.view_for((0.3, 0.5, 0.8)), inputs.view_for((0, 1, 0))]
    N0, Lm = 16, 4
    prm = air.params(N0, Lm, 0.5)
    plain = ctx.render(scene, views, prm)
    V = len(views)
    for d in (0, 1, 2, 7):
        depth = torch.full((V, N0, N0), d, dtype=torch.uint8, device="cuda")
        out = ctx.render_proposal(scene, views, prm, depth)
        _assert_same(plain, out)
        dd = min(d, Lm)
        assert out[4]["spec_rays"] == V * N0 * N0 * sum(4 ** l for l in range(1, dd + 1))
        assert out[4]["depth_hist"][dd] == V * N0 * N0
    true = torch.stack([ctx.tree_depth(t, N0) for t in plain[0]]).to(torch.uint8)
    out = ctx.render_proposal(scene, views, prm, true)
    _assert_same(plain, out)
    say(out[4])
    assert out[4]["missing"] == 0
    assert out[4]["spec_rays"] - out[4]["wasted"] == sum(t.n_nodes for t in plain[0]) - V * N0 * N0


def test_learned_ring_beats_plain(ctx):
    """The committed ring network (trained on ring geometries 1-8) on held-out
    renders of geometries 0, 9 and 10 (keys 41..46 of the training script's
    ring family): every output equals plain AIR's bit for bit, and the
    learned proposal takes less device time per image than plain AIR (its
    levels are latency-bound, so tracing the predicted subtrees in one
    launch saves more than the extra rays cost)."""
    import os
    from paper_1010_5534_amd import air
    wz = np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1010_5534_amd",
                              "weights", "ring_cnn.npz"))
    net = air.Network(ctx, wz["params"], wz["mean"], wz["scale"])
    c_ray, c_sweep = float(wz["c_ray"]), float(wz["c_sweep"])
    prm = air.params(32, 4, 0.2)
    scenes, tp, tl = {}, 0.0, 0.0

    def med(fn):
        fn()
        ms = sorted(fn()[3]["ms_total"] for _ in range(5))
        return ms[2]

    for s in range(41, 47):
        k = (0, 9, 10)[s % 3]
        if k not in scenes:
            g, f = inputs.ring(**inputs.ring_geometry(k))
            scenes[k] = ctx.prepare(air.upload(g, f))
        sc, view = scenes[k], inputs.ring_family_view(1000000 + s)
        ref = ctx.render(sc, [view], prm)
        out = ctx.render_learned(sc, [view], prm, net, c_ray, c_sweep, max_depth=4)
        t, r = out[0][0], ref[0][0]
        assert t.n_nodes == r.n_nodes and np.array_equal(out[2], ref[2])
        for name in ("level", "ix", "iy", "parent", "first_child", "state", "visits"):
            assert torch.equal(getattr(t, name), getattr(r, name)), name
        assert torch.equal(t.I.view(torch.int32), r.I.view(torch.int32))
        assert torch.equal(out[1].view(torch.int32), ref[1].view(torch.int32))
        p_ms = med(lambda: ctx.render(sc, [view], prm, reuse=True))
        l_ms = med(lambda: ctx.render_learned(sc, [view], prm, net, c_ray, c_sweep, max_depth=4, reuse=True))
        say(f"ring geometry {k} view {1000000 + s}: plain {p_ms:.3f} ms, learned {l_ms:.3f} ms "
            f"({r.n_nodes} rays; speculative {out[4]['spec_rays']}, wasted {out[4]['wasted']}, "
            f"missing {out[4]['missing']})")
        tp, tl = tp + p_ms, tl + l_ms
    say(f"ring family, 6 held-out renders: plain {tp / 6:.3f} ms, learned {tl / 6:.3f} ms per image "
        f"({tp / tl:.2f}x)")
    assert tl < 0.9 * tp
    net.close()

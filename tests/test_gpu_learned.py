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
@pytest.mark.parametrize("n,h,w", [(2, 64, 64), (3, 13, 21)])
def test_forward_matches_reference(ctx, n, h, w):
    from paper_1010_5534_amd import air
    theta = he_params(1)
    mean = np.array([0.1, -0.2, 0.3, 0.0], np.float32)
    scale = np.array([1.5, 0.5, 2.0, 1.0], np.float32)
    net = air.Network(ctx, theta, mean, scale)
    x, _ = _maps(2, n, h, w)
    say(f"cnn forward n={n} {h}x{w}")
    z = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()[..., :6].astype(np.float64)
    xs = (x.astype(np.float64) - mean) / scale
    zr, _ = ocnn.forward(theta.astype(np.float32).astype(np.float64), xs, rounding=True)
    # identical bf16 operands, float32 against float64 accumulation: the
    # logits agree to float32 rounding except downstream of the rare hidden
    # activation whose pre-activation lies within the accumulation error of a
    # bf16 rounding boundary; such a flip moves one input of the next layer
    # by one bf16 step (2^-8 relative) and shows as a small patch of
    # receptive-field size, a few 1e-3 of the logit scale
    scale = np.abs(zr) + np.abs(zr).mean()
    err = np.abs(z - zr)
    assert np.mean(err <= 1e-5 * scale) >= 0.95, np.mean(err <= 1e-5 * scale)
    assert np.all(err <= 2e-2 * scale), (err / scale).max()
    net.close()


def test_loss_and_gradient_match_reference(ctx):
    from paper_1010_5534_amd import air
    theta = he_params(3)
    net = air.Network(ctx, theta)
    x, labels = _maps(4, 2, 64, 64)
    cw = np.array([0.5, 1.0, 2.0, 1.5, 3.0, 4.0], np.float32)
    loss, g = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(labels).cuda(), cw, want_grad=True)
    g = g.cpu().numpy().astype(np.float64)
    lr_, gr = ocnn.loss_and_grads(theta.astype(np.float32).astype(np.float64), x.astype(np.float64), labels,
                                  cw.astype(np.float64), rounding=True)
    say(f"loss gpu {loss:.8f} ref {lr_:.8f}")
    assert loss == pytest.approx(lr_, rel=1e-4)
    for name, shape, off in ocnn.layout():
        k = int(np.prod(shape))
        a, b = g[off:off + k], gr[off:off + k]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        say(f"{name}: rel {rel:.2e} cos {cos:.8f}")
        assert rel <= 2e-2 and cos >= 0.9998, name


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
    t = oracle.air(g, f, v, 16, 4, 0.5)
    rep = parity.compare(parity.gpu_dense(trees[0], 16, 4, 1), t, 0.5)
    parity.assert_parity(rep)
    if rep["flips"] == 0:
        assert np.array_equal(d, ocnn.depth_labels(t))


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


@pytest.mark.parametrize("n0,nviews", [(16, 3), (64, 16)])
def test_fused_inference_tile_sizes(ctx, n0, nviews):
    """The fused inference runs 8x8 tiles on small maps (3 views of 16^2)
    and 16x16 tiles on large ones (16 views of 64^2: 256 tiles): the chosen
    depths follow the reference decision on the layer-by-layer logits."""
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
    t = oracle.air(g, f, v, 16, 4, 0.5)
    rep = parity.compare(parity.gpu_dense(trees[0], 16, 4, 1), t, 0.5)
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

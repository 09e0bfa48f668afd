"""Pins of the FP64 reference of the depth-proposal network (oracle/cnn.py):
library routines for the special cases, adjoint identities, central finite
differences, closed forms of the loss and of Adam's first steps, the
bfloat16 format's definition, and the decision rule's limits."""
import numpy as np
import pytest
import scipy.signal

from oracle import cnn


def rnd(seed, *shape, scale=1.0):
    return np.random.default_rng(seed).normal(size=shape) * scale


# ------------------------------------------------------------------ bfloat16
def test_bf16_definition():
    # 8 exponent bits, 7 stored mantissa bits: spacing 2^-7 in [1, 2)
    assert cnn.bf16(1.0) == 1.0
    assert cnn.bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    assert cnn.bf16(1.0 + 2 ** -8) == 1.0            # tie -> even mantissa (0)
    assert cnn.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (2)
    assert cnn.bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert cnn.bf16(-3.0) == -3.0
    assert cnn.bf16(2.0 ** 100) == 2.0 ** 100
    assert cnn.bf16(0.0) == 0.0
    x = np.random.default_rng(0).normal(size=10000)
    r = cnn.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 + 1e-300)  # half an ulp
    assert np.array_equal(cnn.bf16(r), r)  # idempotent


# -------------------------------------------------------------- convolution
def test_conv_matches_scipy_correlate():
    x = rnd(1, 2, 5, 7, 3)
    w = rnd(2, 4, 3, 3, 3)
    b = rnd(3, 4)
    y = cnn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(y[n, :, :, o], ref, rtol=1e-13, atol=1e-13)


def test_conv_delta_kernels_shift():
    x = rnd(4, 1, 6, 6, 2)
    w = np.zeros((2, 3, 3, 2))
    w[0, 1, 1, 0] = 1.0          # identity on channel 0
    w[1, 0, 2, 1] = 1.0          # output (i, j) reads x at (i - 1, j + 1), channel 1
    y = cnn.conv3x3(x, w, np.zeros(2))
    assert np.array_equal(y[..., 0], x[..., 0])
    ref = np.zeros((1, 6, 6))
    ref[:, 1:, :-1] = x[:, :-1, 1:, 1]
    assert np.array_equal(y[..., 1], ref)


def test_input_and_weight_grads_are_adjoints():
    x = rnd(5, 2, 6, 5, 3)
    w = rnd(6, 4, 3, 3, 3)
    dy = rnd(7, 2, 6, 5, 4)
    y = cnn.conv3x3(x, w, np.zeros(4))
    lhs = float(np.sum(y * dy))
    assert lhs == pytest.approx(float(np.sum(x * cnn.conv3x3_input_grad(dy, w))), rel=1e-12)
    dw, db = cnn.conv3x3_weight_grad(dy, x)
    assert lhs == pytest.approx(float(np.sum(w * dw)), rel=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


# -------------------------------------------------------------------- loss
def test_loss_closed_forms():
    z = np.zeros((1, 2, 2, 6))
    labels = np.array([[[0, 3], [5, 1]]])
    loss, g = cnn.loss_and_logit_grad(z, labels, np.ones(6))
    assert loss == pytest.approx(np.log(6.0), rel=1e-15)
    # gradient: (1/6 - onehot) / pixels
    assert g[0, 0, 1, 3] == pytest.approx((1 / 6 - 1) / 4)
    assert g[0, 0, 1, 0] == pytest.approx(1 / 24)
    # a confident correct prediction has almost no loss
    z2 = np.zeros((1, 1, 1, 6))
    z2[..., 2] = 40.0
    l2, _ = cnn.loss_and_logit_grad(z2, np.array([[[2]]]), np.ones(6))
    assert l2 < 1e-16
    # scaling all class weights changes nothing (weighted mean)
    zr = rnd(8, 2, 3, 3, 6)
    lab = np.random.default_rng(9).integers(0, 6, (2, 3, 3))
    cw = np.abs(rnd(10, 6)) + 0.1
    la, ga = cnn.loss_and_logit_grad(zr, lab, cw)
    lb, gb = cnn.loss_and_logit_grad(zr, lab, 7.0 * cw)
    assert la == pytest.approx(lb, rel=1e-14) and np.allclose(ga, gb, rtol=1e-13)
    # the logit gradient of each pixel sums to zero
    assert np.allclose(ga.sum(axis=-1), 0.0, atol=1e-15)


def _small_problem(seed):
    rng = np.random.default_rng(seed)
    theta = np.zeros(cnn.N_PARAMS)
    for name, shape, off in cnn.layout():
        n = int(np.prod(shape))
        fan = 9 * shape[3] if name.startswith("w") else 1
        theta[off:off + n] = rng.normal(size=n) * (np.sqrt(2.0 / fan) if name.startswith("w") else 0.1)
    x = rng.normal(size=(2, 5, 6, 4))
    labels = rng.integers(0, 6, size=(2, 5, 6))
    cw = np.array([1.0, 2.0, 0.5, 1.5, 3.0, 1.0])
    return theta, x, labels, cw


def test_gradient_matches_central_differences():
    theta, x, labels, cw = _small_problem(11)
    _, g = cnn.loss_and_grads(theta, x, labels, cw, rounding=False)
    rng = np.random.default_rng(12)
    # parameters of every layer, weights and biases
    picks = []
    for name, shape, off in cnn.layout():
        n = int(np.prod(shape))
        picks += list(off + rng.choice(n, size=min(n, 6), replace=False))
    h = 1e-6
    for k in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp, _ = cnn.loss_and_grads(tp, x, labels, cw, rounding=False)
        lm, _ = cnn.loss_and_grads(tm, x, labels, cw, rounding=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3), (k, fd, g[k])


def test_rounded_gradient_close_to_exact():
    """The bf16 rounding points perturb the gradient by a few bf16 ulps."""
    theta, x, labels, cw = _small_problem(13)
    _, g64 = cnn.loss_and_grads(theta, x, labels, cw, rounding=False)
    _, g16 = cnn.loss_and_grads(theta, x, labels, cw, rounding=True)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


# -------------------------------------------------------------------- Adam
def test_adam_first_steps_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    t1, m, v = cnn.adam_step(theta, g, m, v, 1, lr=0.01, eps=1e-8)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # with a constant gradient the second step is the same size
    t2, m, v = cnn.adam_step(t1, g, m, v, 2, lr=0.01, eps=1e-8)
    assert np.allclose(t2 - t1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# ---------------------------------------------------------------- decision
def test_decision_limits():
    z = rnd(14, 3, 4, 4, 6)
    d0, _ = cnn.decide_depth(z, c_ray=1.0, c_sweep=0.0)
    assert np.all(d0 == 0)  # sweeping is free: speculate nothing
    d5, _ = cnn.decide_depth(z, c_ray=0.0, c_sweep=1.0)
    assert np.all(d5 == 5)  # rays are free: speculate to the deepest class
    dcap, _ = cnn.decide_depth(z, c_ray=0.0, c_sweep=1.0, max_depth=2)
    assert np.all(dcap == 2)


def test_decision_hand_example():
    # probabilities 0.5, 0.25, 0.25 on depths 0, 1, 2
    p = np.array([0.5, 0.25, 0.25, 0.0, 0.0, 0.0]) + 1e-30
    z = np.log(p)[None]
    # costs: d=0: 0.5 c_s ; d=1: 4 c_r + 0.25 c_s ; d=2: 20 c_r
    d, cost = cnn.decide_depth(z, c_ray=1.0, c_sweep=100.0)
    assert np.allclose(cost[0, :3], [50.0, 29.0, 20.0], rtol=1e-6)
    assert d[0] == 2
    d, _ = cnn.decide_depth(z, c_ray=1.0, c_sweep=10.0)
    assert d[0] == 0  # 5 vs 6.5 vs 20
    d, _ = cnn.decide_depth(z, c_ray=1.0, c_sweep=30.0)
    assert d[0] == 1  # 15 vs 11.5 vs 20
    assert cnn.subtree_rays(0) == 0 and cnn.subtree_rays(3) == 4 + 16 + 64


# -------------------------------------------------------------- features
def test_features_values():
    I = np.array([1e-3, 0.0, 5.0])
    N = np.array([2.0, 0.0, 1e-10])
    lmax = np.array([0, -1, 2])
    rmin = np.array([0.5, 0.0, 1e-3])
    rmax = np.array([5.0, 0.0, 1e-3])
    hit = lmax >= 0
    f = cnn.features(I, N, lmax, rmin, rmax, hit, np.zeros(4), np.ones(4))
    assert np.allclose(f[0], [-3.0, np.log10(2.0), 0.0, 1.0])
    assert np.allclose(f[1], [-30.0, -30.0, -1.0, 0.0])
    assert np.allclose(f[2], [np.log10(5.0), -10.0, 2.0, 0.0], atol=1e-12)
    g = cnn.features(I, N, lmax, rmin, rmax, hit, np.ones(4), 2.0 * np.ones(4))
    assert np.allclose(g, (f - 1.0) / 2.0)


def test_depth_labels_from_oracle_trees(orc):
    from paper_1010_5534_amd import inputs
    g, f = inputs.gaussian(32)
    v = inputs.gaussian_view()
    full = orc.air(g, f, v, 8, 3, 0.0)
    assert np.all(cnn.depth_labels(full) == 3)
    none = orc.air(g, f, v, 8, 3, 1.01)
    assert np.all(cnn.depth_labels(none) == 0)
    t = orc.air(g, f, v, 8, 3, 0.5)
    d = cnn.depth_labels(t)
    # every coarse pixel's subtree holds at least one node at its depth
    for L in range(4):
        ex = (t.state[L] & 1) > 0
        jj, ii = np.nonzero(ex)
        assert np.all(d[jj >> L, ii >> L] >= L)


# ----------------------------------------------- rounding points, by hand
def _one_path_net():
    """A network on a 1x1 map whose only live path runs through channel 0 of
    every layer (centre tap), with values chosen so that each bfloat16
    rounding point changes the result: see the hand derivation in the
    tests below."""
    p = {name: np.zeros(shape) for name, shape, _ in cnn.layout()}
    p["w0"][0, 1, 1, 0] = 1 + 3 * 2 ** -9   # bf16 -> 1 + 2^-7
    p["b0"][0] = 2 ** -9
    p["w1"][0, 1, 1, 0] = 3.0
    p["b1"][0] = -2 ** -6
    p["w2"][0, 1, 1, 0] = 0.5
    p["b2"][0] = 2 ** -10
    for c in range(6):
        p["w3"][c, 1, 1, 0] = c * (1 + 2 ** -8)
        p["b3"][c] = 0.125 * c
    x = np.zeros((1, 1, 1, 4))
    x[0, 0, 0, 0] = 1 + 2 ** -9             # bf16 -> 1
    return cnn.pack(p), x


def test_forward_rounding_points_by_hand():
    """Input rounded: 1 + 2^-9 -> 1.  Layer 0: 1 * (1 + 2^-7) + 2^-9, stored
    as bf16 1 + 2^-7 (2^-9 is below half a step).  Layer 1: 3 (1 + 2^-7) -
    2^-6 = 3 + 2^-7, a tie between 3 and 3 + 2^-6, stored as 3 (even).
    Layer 2: 1.5 + 2^-10 -> 1.5.  Logits (not rounded): 1.5 bf16(c (1 +
    2^-8)) + c / 8, the weights rounding to 0, 1, 2 (tie), 3 + 2^-6, 4 (tie),
    5 + 2^-5."""
    theta, x = _one_path_net()
    z, acts = cnn.forward(theta, x, rounding=True)
    assert acts[0][0, 0, 0, 0] == 1.0
    assert acts[1][0, 0, 0, 0] == 1 + 2 ** -7
    assert acts[2][0, 0, 0, 0] == 3.0
    assert acts[3][0, 0, 0, 0] == 1.5
    w3 = [0.0, 1.0, 2.0, 3 + 2 ** -6, 4.0, 5 + 2 ** -5]
    assert list(z[0, 0, 0]) == [1.5 * w3[c] + 0.125 * c for c in range(6)]
    # without the rounding points every value is carried exactly
    z2, acts2 = cnn.forward(theta, x, rounding=False)
    y0 = (1 + 2 ** -9) * (1 + 3 * 2 ** -9) + 2 ** -9
    y1 = 3 * y0 - 2 ** -6
    y2 = 0.5 * y1 + 2 ** -10
    assert acts2[1][0, 0, 0, 0] == y0 and acts2[2][0, 0, 0, 0] == y1 and acts2[3][0, 0, 0, 0] == y2
    assert np.allclose(z2[0, 0, 0], [y2 * c * (1 + 2 ** -8) + 0.125 * c for c in range(6)], rtol=1e-15)


def test_backward_rounding_points_by_hand():
    """On the same path: the logit gradient is rounded to bf16 before the
    backward pass; the weight gradient of the last layer is that rounded
    gradient times its stored input 1.5; the gradient at that input is the
    sum over classes of rounded gradient times rounded weight, itself rounded
    (the input is > 0), and makes the layer-2 weight gradient with layer 2's
    stored input 3; and so on down to layer 0."""
    theta, x = _one_path_net()
    labels = np.array([[[2]]])
    cw = np.ones(6)
    z, _ = cnn.forward(theta, x, rounding=True)
    _, dz = cnn.loss_and_logit_grad(z, labels, cw)
    dzr = cnn.bf16(dz[0, 0, 0])
    assert not np.array_equal(dzr, dz[0, 0, 0])  # the rounding point matters here
    _, g = cnn.loss_and_grads(theta, x, labels, cw, rounding=True)
    gp = cnn.unpack(g)
    assert np.array_equal(gp["w3"][:, 1, 1, 0], dzr * 1.5)
    assert np.array_equal(gp["b3"], dzr)
    w3 = np.array([0.0, 1.0, 2.0, 3 + 2 ** -6, 4.0, 5 + 2 ** -5])
    da2 = cnn.bf16(np.sum(dzr * w3))
    assert gp["w2"][0, 1, 1, 0] == da2 * 3.0
    assert gp["b2"][0] == da2
    da1 = cnn.bf16(da2 * 0.5)
    assert gp["w1"][0, 1, 1, 0] == da1 * (1 + 2 ** -7)
    da0 = cnn.bf16(da1 * 3.0)
    assert gp["w0"][0, 1, 1, 0] == da0 * 1.0
    # every other weight and bias gradient is zero (a 1x1 map sees only the
    # centre tap; the other channels carry zeros)
    assert da0 != 0
    assert np.count_nonzero(gp["w3"]) == np.count_nonzero(dzr)
    for l in range(3):
        assert np.count_nonzero(gp[f"w{l}"]) == 1 and np.count_nonzero(gp[f"b{l}"]) == 1

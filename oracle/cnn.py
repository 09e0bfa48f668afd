"""FP64 reference of the learned depth proposal: features, network, loss,
gradients, optimiser step and the cost-aware depth decision.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU baseline, never by the library.  Plain numpy, float64, one
obvious loop per formula; matrix products over the channel axis are the only
library primitive used.

Network (the learned component beside plain AIR): four 3x3 convolutions with
zero 'same' padding, written as cross-correlation

    y[b, i, j, o] = bias[o] + sum_{ky, kx, c} x[b, i + ky - 1, j + kx - 1, c] w[o, ky, kx, c],

channels 4 -> 32 -> 32 -> 32 -> 6, ReLU after the first three; the six
outputs are the logits of the depth classes 0..5 of each coarse pixel.

Loss: class-weighted softmax cross-entropy, the weighted mean over pixels,

    loss = sum_p cw[t_p] (-log softmax(z_p)[t_p]) / sum_p cw[t_p].

Optimiser: Adam with bias correction (Kingma and Ba, 2015).

Rounding points (rounding=True) mirror the GPU kernels, which store weights,
activations and back-propagated gradients as bfloat16 and accumulate in
float32: the features and the weights are rounded to bfloat16 before use;
each hidden layer's output is rounded after the ReLU; the logits stay
unrounded; the logit gradient is rounded before the backward pass and each
back-propagated activation gradient after the ReLU mask.  Biases, weight
gradients and the optimiser state are float (here float64).  With
rounding=False every step is plain float64, which is what the
finite-difference pins check."""
import numpy as np

CHANNELS = (4, 32, 32, 32, 6)
N_CLASSES = 6
N_LAYERS = 4


def layout():
    """[(name, shape, offset)] of the flat parameter vector: for each layer
    the weights [cout][3][3][cin], then the bias [cout]."""
    out, off = [], 0
    for l in range(N_LAYERS):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        out.append((f"w{l}", (cout, 3, 3, cin), off))
        off += cout * 9 * cin
        out.append((f"b{l}", (cout,), off))
        off += cout
    return out


N_PARAMS = sum(int(np.prod(s)) for _, s, _ in layout())


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    return {name: theta[off:off + int(np.prod(shape))].reshape(shape) for name, shape, off in layout()}


def pack(parts):
    theta = np.zeros(N_PARAMS)
    for name, shape, off in layout():
        theta[off:off + int(np.prod(shape))] = np.asarray(parts[name], dtype=np.float64).reshape(-1)
    return theta


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), via float32, returned as
    float64.  bfloat16 keeps the top 16 bits of a float32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def conv3x3(x, w, b):
    """x [B, H, W, cin], w [cout, 3, 3, cin], b [cout] -> [B, H, W, cout]."""
    B, H, W, _ = x.shape
    xp = np.zeros((B, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.broadcast_to(b, (B, H, W, w.shape[0])).copy()
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
    return y


def conv3x3_input_grad(dy, w):
    """d loss / d x of conv3x3 given dy = d loss / d y: the transposed
    correlation  dx[i, j, c] = sum_{ky, kx, o} dy[i - ky + 1, j - kx + 1, o] w[o, ky, kx, c]."""
    B, H, W, _ = dy.shape
    dyp = np.zeros((B, H + 2, W + 2, dy.shape[3]))
    dyp[:, 1:H + 1, 1:W + 1] = dy
    dx = np.zeros((B, H, W, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            # position (i, j) of x meets output (i - ky + 1, j - kx + 1)
            dx += dyp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W, :] @ w[:, ky, kx, :]
    return dx


def conv3x3_weight_grad(dy, x):
    """d loss / d w [cout, 3, 3, cin] and d loss / d b [cout]."""
    B, H, W, cin = x.shape
    xp = np.zeros((B, H + 2, W + 2, cin))
    xp[:, 1:H + 1, 1:W + 1] = x
    cout = dy.shape[3]
    dw = np.zeros((cout, 3, 3, cin))
    d2 = dy.reshape(-1, cout)
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = d2.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, cin)
    return dw, d2.sum(axis=0)


def forward(theta, x, rounding=True):
    """Returns (logits [B, H, W, 6], activations [input, a0, a1, a2])."""
    r = bf16 if rounding else _id
    p = unpack(theta)
    a = r(x)
    acts = [a]
    for l in range(N_LAYERS):
        y = conv3x3(a, r(p[f"w{l}"]), p[f"b{l}"])
        if l == N_LAYERS - 1:
            return y, acts
        a = r(np.maximum(y, 0.0))
        acts.append(a)


def softmax(z):
    m = z.max(axis=-1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=-1, keepdims=True)


def loss_and_logit_grad(z, labels, class_w):
    """Weighted cross-entropy and its gradient with respect to the logits."""
    labels = np.asarray(labels, dtype=np.int64)
    cw = np.asarray(class_w, dtype=np.float64)
    w = cw[labels]
    W = w.sum()
    m = z.max(axis=-1, keepdims=True)
    lse = (m[..., 0] + np.log(np.exp(z - m).sum(axis=-1)))
    zt = np.take_along_axis(z, labels[..., None], axis=-1)[..., 0]
    loss = float((w * (lse - zt)).sum() / W)
    g = softmax(z)
    onehot = np.zeros_like(z)
    np.put_along_axis(onehot, labels[..., None], 1.0, axis=-1)
    return loss, (g - onehot) * (w / W)[..., None]


def loss_and_grads(theta, x, labels, class_w, rounding=True):
    """(loss, flat gradient) of one batch, backward through the rounding
    points listed in the module docstring."""
    r = bf16 if rounding else _id
    p = unpack(theta)
    z, acts = forward(theta, x, rounding)
    loss, dz = loss_and_logit_grad(z, labels, class_w)
    grads = {}
    dy = r(dz)
    for l in range(N_LAYERS - 1, -1, -1):
        dw, db = conv3x3_weight_grad(dy, acts[l])
        grads[f"w{l}"], grads[f"b{l}"] = dw, db
        if l == 0:
            break
        da = conv3x3_input_grad(dy, r(p[f"w{l}"]))
        dy = r(da * (acts[l] > 0))  # ReLU: the stored output is positive where it passed
    return loss, pack(grads)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------------ the features
def features(I, N, lmax, rmin, rmax, hit, mean, std):
    """Four standardised input maps of one view from its coarse trace:
    log10(I + 1e-30), log10(N + 1e-30), the finest grid level crossed (-1
    for a miss) and the log dynamic range of the density met by the ray,
    log10(rho_max / rho_min) (0 for a miss or a zero density)."""
    I = np.asarray(I, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    hit = np.asarray(hit, bool)
    rmin = np.asarray(rmin, dtype=np.float64)
    rmax = np.asarray(rmax, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        rng = np.where(hit & (rmin > 0), np.log10(rmax / np.where(rmin > 0, rmin, 1.0)), 0.0)
    raw = np.stack([np.log10(I + 1e-30), np.log10(N + 1e-30), np.asarray(lmax, dtype=np.float64), rng], axis=-1)
    return (raw - np.asarray(mean)) / np.asarray(std)


def depth_labels(tree):
    """Deepest level of the final tree inside each coarse pixel [N0, N0]."""
    N0 = tree.N0
    d = np.zeros((N0, N0), np.int64)
    for L in range(tree.Lmax + 1):
        jj, ii = np.nonzero(tree.state[L] & 1)
        np.maximum.at(d, (jj >> L, ii >> L), L)
    return d


def subtree_rays(d):
    """Rays below a coarse pixel traced speculatively to depth d (levels 1..d)."""
    return sum(4 ** l for l in range(1, int(d) + 1))


def decide_depth(z, c_ray, c_sweep, max_depth=5):
    """Cost-aware depth choice per pixel: argmin over d of
    c_ray * (rays of levels 1..d) + c_sweep * P(depth > d), P from the
    softmax of the logits; ties go to the shallower depth.  Evaluated in
    float32, as the kernel does, since it turns floats into an integer."""
    z = np.asarray(z, dtype=np.float32)
    m = z.max(axis=-1, keepdims=True)
    e = np.exp(z - m, dtype=np.float32)
    p = e / e.sum(axis=-1, keepdims=True, dtype=np.float32)
    best = np.zeros(z.shape[:-1], np.int64)
    best_cost = np.full(z.shape[:-1], np.inf, np.float32)
    cost_all = []
    for d in range(max_depth + 1):
        tail = p[..., d + 1:].sum(axis=-1, dtype=np.float32) if d + 1 < z.shape[-1] else np.zeros(z.shape[:-1], np.float32)
        cost = np.float32(c_ray) * np.float32(subtree_rays(d)) + np.float32(c_sweep) * tail
        cost_all.append(cost)
        better = cost < best_cost
        best = np.where(better, d, best)
        best_cost = np.where(better, cost, best_cost)
    return best, np.stack(cost_all, axis=-1)

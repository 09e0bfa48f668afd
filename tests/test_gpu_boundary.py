"""Entry points around the renders: network checkpoints that resume training
exactly (air_cnn_save / air_cnn_load), the batch's launch-shape cache kept
across contexts (air_tune_save / air_tune_load) and library-allocated trees
(air_tree_alloc / air_tree_free), each through the C ABI."""
import ctypes as C
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
def ctx():
    from paper_1010_5534_amd import air
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = air.Context(0)
    yield c
    c.close()


def _batch(seed, n=8, h=24, w=20):
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.normal(size=(n, h, w, 4)).astype(np.float32)).cuda()
    lab = torch.from_numpy(rng.integers(0, 6, size=(n, h, w)).astype(np.int32)).cuda()
    return x, lab


def _step(net, x, lab, cw):
    net.loss_grad(x, lab, cw, want_loss=False)
    net.adam(lr=1e-3)


def test_cnn_checkpoint_resumes_training_exactly(ctx, tmp_path):
    from paper_1010_5534_amd import air
    cw = np.array([1.0, 2.0, 0.5, 1.0, 3.0, 1.5], np.float32)
    a = air.Network(ctx, inputs.cnn_init(5), np.array([0.1, 0.2, -0.3, 0.0], np.float32),
                    np.array([1.0, 2.0, 0.5, 1.5], np.float32))
    x, lab = _batch(1)
    say("cnn checkpoint: 3 Adam steps, save, load into a second network")
    for _ in range(3):
        _step(a, x, lab, cw)
    path = str(tmp_path / "net.ckpt")
    a.save(path)
    b = air.Network(ctx)
    b.load(path)
    pa, ma, sa = a.get()
    pb, mb, sb = b.get()
    assert np.array_equal(pa, pb) and np.array_equal(ma, mb) and np.array_equal(sa, sb)
    # the optimiser state came along: one more step on each gives the same bits
    x2, lab2 = _batch(2)
    _step(a, x2, lab2, cw)
    _step(b, x2, lab2, cw)
    assert np.array_equal(a.get()[0], b.get()[0])
    assert torch.equal(a.forward(x2), b.forward(x2))
    # a fresh network with the same parameters but no optimiser state differs
    c = air.Network(ctx, pa, ma, sa)
    _step(c, x2, lab2, cw)
    assert not np.array_equal(c.get()[0], b.get()[0])
    a.close(), b.close(), c.close()


def test_cnn_load_rejects_bad_files(ctx, tmp_path):
    from paper_1010_5534_amd import air
    net = air.Network(ctx, inputs.cnn_init(6))
    before = net.get()[0]
    good = str(tmp_path / "good.ckpt")
    net.save(good)
    raw = open(good, "rb").read()
    cases = {"truncated": raw[:-4], "extra": raw + b"\0", "magic": b"X" + raw[1:], "empty": b""}
    # a non-finite parameter: the first parameter follows the 24-byte header
    # and the 8 standardisation floats
    bad = bytearray(raw)
    bad[24 + 32:24 + 36] = np.array([np.nan], np.float32).tobytes()
    cases["nan"] = bytes(bad)
    for name, blob in cases.items():
        p = tmp_path / f"{name}.ckpt"
        p.write_bytes(blob)
        with pytest.raises(air.AirError) as e:
            net.load(str(p))
        assert e.value.code == air.AIR_EINVAL, name
    with pytest.raises(air.AirError):
        net.load(str(tmp_path / "missing.ckpt"))
    assert np.array_equal(net.get()[0], before)  # nothing was taken
    net.close()


def _entries(path):
    lines = open(path).read().splitlines()
    return lines[0], sorted(lines[1:])


def test_tune_cache_roundtrip(ctx, tmp_path):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=3, n=64, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    prm = air.params(16, 3, 0.4, band_weight=[1.0, 0.5])
    views = inputs.winds2_views()
    say("tune cache: batch on one context, save, load on another")
    ref = ctx.render_batch(scene, views, prm)
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    head, ent = _entries(path)
    assert head.startswith("libair-tune 1 gfx950")
    assert len(ent) >= 1
    ctx2 = air.Context(0)
    ctx2.tune_load(path)
    out = ctx2.render_batch(scene, views, prm)
    assert np.array_equal(out[2], ref[2])
    assert torch.equal(out[1].view(torch.int32), ref[1].view(torch.int32))
    for x, y in zip(out[0], ref[0]):
        assert x.n_nodes == y.n_nodes and torch.equal(x.state, y.state) and torch.equal(x.I, y.I)
    path2 = str(tmp_path / "tune2.txt")
    ctx2.tune_save(path2)
    assert _entries(path2) == (head, ent)  # the loaded shapes were used, none tuned anew
    # rejected files leave the cache as it was
    arch, cus = head.split()[2], int(head.split()[3])
    bad = {"arch": f"libair-tune 1 gfx000 {cus}\n" + "\n".join(ent) + "\n",
           "cus": f"libair-tune 1 {arch} {cus + 1}\n" + "\n".join(ent) + "\n",
           "entry": head + "\n" + "1/64,64,64/0,0/3/16/3/2/plain 7 4\n",
           "header": "tune 1\n"}
    for name, text in bad.items():
        p = tmp_path / f"{name}.txt"
        p.write_text(text)
        with pytest.raises(air.AirError) as e:
            ctx2.tune_load(str(p))
        assert e.value.code == air.AIR_EINVAL, name
    ctx2.tune_save(path2)
    assert _entries(path2) == (head, ent)
    ctx2.close()


class _DevArray:
    """A device pointer seen by torch through the CUDA array interface."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = dict(shape=(n,), typestr=typestr, data=(ptr, False), version=2)


def test_library_allocated_tree(ctx):
    from paper_1010_5534_amd import air
    L = air.lib()
    g, f = inputs.winds2(seed=4, n=32, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    prm = air.params(16, 3, 0.3)
    views = inputs.winds2_views()[:1]
    ref = ctx.render(scene, views, prm)
    n = ref[0][0].n_nodes
    say(f"library-allocated tree: {n} nodes")
    trees = (air.air_tree * 1)()
    # too small: ECAPACITY with the size needed, then a tree that fits
    assert L.air_tree_alloc(ctx._p, scene.n_bands, n - 1, C.addressof(trees[0])) == air.AIR_OK
    assert trees[0].capacity == n - 1
    vs = air._views(views)
    st = air.air_stats()
    args = (C.addressof(scene.grid), C.addressof(scene.field), C.addressof(vs), 1, C.addressof(prm),
            C.addressof(trees), None, None, C.addressof(st), ctx._stream())
    assert L.air_render(ctx._p, *args) == air.AIR_ECAPACITY
    assert trees[0].n_nodes == n
    assert L.air_tree_free(ctx._p, C.addressof(trees[0])) == air.AIR_OK
    assert trees[0].capacity == 0 and not trees[0].level and not trees[0].I
    assert L.air_tree_alloc(ctx._p, scene.n_bands, n, C.addressof(trees[0])) == air.AIR_OK
    assert L.air_render(ctx._p, *args) == air.AIR_OK
    torch.cuda.synchronize()
    t = trees[0]
    assert t.n_nodes == n and t.n_leaves == ref[0][0].n_leaves
    want = ref[0][0]
    for name, ptr, ts, dt in (("level", t.level, "|i1", None), ("ix", t.ix, "<i4", None), ("iy", t.iy, "<i4", None),
                              ("parent", t.parent, "<i4", None), ("first_child", t.first_child, "<i4", None),
                              ("state", t.state, "|u1", None), ("N", t.N, "<f4", torch.int32),
                              ("visits", t.visits, "<i4", None)):
        got = torch.as_tensor(_DevArray(ptr, n, ts), device="cuda")
        exp = getattr(want, name)[:n]
        if dt is not None:
            got, exp = got.view(dt), exp.view(dt)
        assert torch.equal(got.cpu(), exp.cpu()), name
    # I is [n_bands][capacity]: band b starts at b * capacity
    got_i = torch.as_tensor(_DevArray(t.I, scene.n_bands * n, "<f4"), device="cuda")
    assert torch.equal(got_i.view(scene.n_bands, n).view(torch.int32).cpu(),
                       want.I.contiguous().view(torch.int32).cpu())
    assert L.air_tree_free(ctx._p, C.addressof(trees[0])) == air.AIR_OK
    # argument errors, checked before anything is allocated
    assert L.air_tree_alloc(ctx._p, 0, 10, C.addressof(trees[0])) == air.AIR_EINVAL
    assert L.air_tree_alloc(ctx._p, 1, 0, C.addressof(trees[0])) == air.AIR_EINVAL
    assert L.air_tree_alloc(ctx._p, 1, 1 << 31, C.addressof(trees[0])) == air.AIR_EINVAL
    assert L.air_tree_alloc(ctx._p, 1, 10, None) == air.AIR_EINVAL


def test_training_resume_matches_uninterrupted(ctx, tmp_path):
    """Three epochs in one go against two epochs, a checkpoint (network,
    optimiser and shuffling state), and the third epoch in a fresh network
    loaded from it: the same parameters bit for bit."""
    from paper_1010_5534_amd import air, train_depth
    rng = np.random.default_rng(21)
    ftr = torch.from_numpy(rng.normal(size=(40, 32, 32, 4)).astype(np.float32)).cuda()
    ltr = torch.from_numpy(rng.integers(0, 6, size=(40, 32, 32)).astype(np.int32)).cuda()
    cw = np.ones(6, np.float32)
    say("training: 3 epochs straight against 2 + checkpoint + 1")
    a = air.Network(ctx, inputs.cnn_init(7))
    train_depth.train_epochs(a, ftr, ltr, cw, 3, 8, 1e-3, np.random.default_rng(1234))
    b = air.Network(ctx, inputs.cnn_init(7))
    rb = np.random.default_rng(1234)
    saved = {}

    def keep(epoch, hist):
        b.save(str(tmp_path / "b.ckpt"))
        saved["rng"] = rb.bit_generator.state

    train_depth.train_epochs(b, ftr, ltr, cw, 2, 8, 1e-3, rb, on_epoch=keep)
    c = air.Network(ctx)
    c.load(str(tmp_path / "b.ckpt"))
    rc = np.random.default_rng(0)
    rc.bit_generator.state = saved["rng"]
    train_depth.train_epochs(c, ftr, ltr, cw, 3, 8, 1e-3, rc, first_epoch=2)
    pa, pc = a.get(), c.get()
    assert all(np.array_equal(x, y) for x, y in zip(pa, pc))
    a.close(), b.close(), c.close()

"""air_render_batch (captured, autotuned launch sequence) against air_render
bit for bit, and the batched block-AMR many-view many-band workload against
the FP64 oracle on sampled views."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import parity
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


def _same(a, b):
    for x, y in zip(a[0], b[0]):
        assert x.n_nodes == y.n_nodes
        for name in ("level", "ix", "iy", "parent", "first_child", "state", "I", "N", "visits"):
            assert torch.equal(getattr(x, name), getattr(y, name)), name
    assert torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
    assert np.array_equal(a[2], b[2])
    assert a[3]["rays"] == b[3]["rays"] and a[3]["visits"] == b[3]["visits"]


def test_batch_equals_render_and_replays(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=2, n=64, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    prm = air.params(16, 4, 0.4, band_weight=[1.0, 0.5])
    views = inputs.winds2_views()
    say("batch winds2 n=64 2 bands, 3 views")
    ref = ctx.render(scene, views, prm)
    b1 = ctx.render_batch(scene, views, prm)
    _same(ref, b1)
    b2 = ctx.render_batch(scene, views, prm)  # replay of the captured sequence
    _same(ref, b2)
    # new view contents, same shapes: the captured sequence reads them
    views2 = inputs.isotropic_views(3, seed=11)
    _same(ctx.render(scene, views2, prm), ctx.render_batch(scene, views2, prm))


def test_view_counts_changing_between_calls(ctx):
    """The result block lives in a pinned host buffer that k_finish writes
    directly; it grows (after the device drains) when a call has more views,
    and a captured sequence is keyed on its address.  Calls with 1, 4, 2 and
    6 views in turn, eager and captured, each equal to the views rendered one
    at a time, bit for bit (trees, flux, counts)."""
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=3, n=48, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    prm = air.params(12, 3, 0.4)
    pool = inputs.isotropic_views(6, seed=5)
    single = [ctx.render(scene, [v], prm, want_image=False) for v in pool]
    for n in (1, 4, 2, 6):
        for mode in ("eager", "batch"):
            say(f"view counts: {n} views, {mode}")
            fn = ctx.render if mode == "eager" else ctx.render_batch
            trees, _, flux, st = fn(scene, pool[:n], prm, want_image=False)
            for k in range(n):
                t1, f1, s1 = single[k][0][0], single[k][2], single[k][3]
                assert trees[k].n_nodes == t1.n_nodes
                for name in ("level", "ix", "iy", "state", "I", "N", "visits"):
                    assert torch.equal(getattr(trees[k], name), getattr(t1, name)), (n, mode, k, name)
                assert np.array_equal(flux[k], f1[0]), (n, mode, k)
            assert st["rays"] == sum(single[k][3]["rays"] for k in range(n))
            assert st["hits"] == sum(single[k][3]["hits"] for k in range(n))


def test_batch_amr_many_views_bands(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.amr_winds(seed=3, base_cells=64, bs=8, max_level=2, frac=(0.10, 0.03),
                            bands=inputs.default_bands(8))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(16, seed=3)
    prm = air.params(32, 3, 0.5)
    say("batch amr 64/8 L2, 16 views x 8 bands, N0=32 Lmax=3")
    ref = ctx.render(scene, views, prm)
    out = ctx.render_batch(scene, views, prm)
    _same(ref, out)
    for k in (0, 9):
        rep = parity.check(out[0][k], g, f, views[k], 32, 3, 0.5, image=out[1][k], flux=out[2][k], own=True,
                           label=f"batch amr 16 views x 8 bands, view {k}")
        say(parity.summary(rep))
        parity.assert_parity(rep)


def test_batch_config3_full_size_sampled(ctx):
    """Block AMR 128^3 base in 16^3 blocks, levels 0-2, 64 views x 8 bands,
    128x128 coarse, 3 levels: one batched call, two sampled views against
    the oracle."""
    from paper_1010_5534_amd import air
    g, f = inputs.amr_winds(seed=0, base_cells=128, bs=16, max_level=2, bands=inputs.default_bands(8))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(64, seed=3)
    prm = air.params(128, 3, 0.5)
    say(f"batch config3: {g.n_blocks} blocks, 64 views x 8 bands")
    out = ctx.render_batch(scene, views, prm, want_image=False)
    say(out[3]["rays"], out[3]["visits"])
    for k in (5, 40):
        rep = parity.check(out[0][k], g, f, views[k], 128, 3, 0.5, flux=out[2][k],
                           label=f"config3 64 views x 8 bands, view {k}")
        say(parity.summary(rep))
        parity.assert_parity(rep)


def test_graph_recaptured_after_context_buffers_grow(ctx):
    """A captured sequence holds the addresses of the context's workspace.
    Calls between two batched calls of one shape that grow that workspace
    (a fixed image with flux at a larger size grows the partial sums; an
    eager render of a larger tree grows the index maps) must not leave the
    second batched call replaying launches into freed memory: it equals
    air_render bit for bit."""
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=4, n=48, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    prm = air.params(12, 3, 0.4)
    views = inputs.isotropic_views(2, seed=21)
    say("graph buffers: batch, fixed with flux at 1024^2, batch")
    ref = ctx.render(scene, views, prm, reuse=False)
    _same(ref, ctx.render_batch(scene, views, prm))
    ctx.render_fixed(scene, views, 64, 4)  # flux partial sums for 1024^2 images
    _same(ref, ctx.render_batch(scene, views, prm))
    say("graph buffers: batch, eager render of a larger tree, batch")
    ctx.render(scene, views, air.params(32, 4, 0.3), want_image=False)
    _same(ref, ctx.render_batch(scene, views, prm))

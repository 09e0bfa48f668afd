"""The allocation-free fixed render (air_render_fixed_noalloc) against
air_render_fixed through the C ABI, bit for bit (images and fluxes), on two
calls in a row, the second with a smaller input; and its limits.  Collected
last (test_zz_*): it must pass alone and after every other test."""
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


def _compare(ctx, scene, views, n0, level):
    ref_img, ref_flux, _ = ctx.render_fixed(scene, views, n0, level)
    img, flux = ctx.render_fixed_noalloc(scene, views, n0, level)
    torch.cuda.synchronize()
    assert torch.equal(img.view(torch.int32), ref_img.view(torch.int32))
    assert np.array_equal(flux.cpu().numpy(), ref_flux)


def test_noalloc_equals_fixed_two_calls(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=5, n=64, kind=inputs.FIELD_RHO_T, bands=inputs.default_bands(4))
    scene = ctx.prepare(air.upload(g, f))
    say("no-alloc fixed: winds2 64^3 4 bands, 3 views, 16 x 2^4")
    _compare(ctx, scene, inputs.winds2_views(), 16, 4)
    say("no-alloc fixed: 2 views, 8 x 2^3 (smaller)")
    _compare(ctx, scene, inputs.isotropic_views(2, seed=9), 8, 3)


def test_noalloc_amr_after_pack(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.amr_winds(seed=2, base_cells=32, bs=4, max_level=2, frac=(0.2, 0.05),
                            bands=inputs.default_bands(2))
    scene = ctx.prepare(air.upload(g, f))
    say("no-alloc fixed: block AMR 32/4, 2 bands, 2 views")
    _compare(ctx, scene, inputs.isotropic_views(2, seed=4), 8, 3)


def test_noalloc_limits(ctx):
    from paper_1010_5534_amd import air
    g, f = inputs.winds2(seed=5, n=32)
    unpacked = air.upload(g, f)
    with pytest.raises(air.AirError) as e:
        ctx.render_fixed_noalloc(unpacked, inputs.winds2_views(), 8, 2)
    assert e.value.code == air.AIR_EINVAL
    scene = ctx.prepare(air.upload(g, f))
    with pytest.raises(air.AirError) as e:
        ctx.render_fixed_noalloc(scene, inputs.isotropic_views(17, seed=1), 4, 1)
    assert e.value.code == air.AIR_EINVAL
    # flux partial sums beyond the workspace: 16 views of 8192^2 pixels
    # (16384 chunks of 4096 each) need 16 x 16384 x 8 B = 2 MiB, more than
    # the workspace holds after its counters and view table; the host rejects
    # the call before any launch, so the image buffer is never touched
    with pytest.raises(air.AirError) as e:
        ctx.render_fixed_noalloc(scene, inputs.isotropic_views(16, seed=1), 128, 6, images=torch.empty(1, device="cuda"))
    assert e.value.code == air.AIR_EINVAL

"""The C-ABI library loads, exports every entry point include/air.h
declares, and its structs match the binding's layouts (CPU only: no compute
call is made)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "air.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:air_status|void|const char\*|int64_t)\s+(air_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    assert {"air_create", "air_destroy", "air_last_error", "air_render", "air_render_fixed"} <= set(names)


def test_library_exports_every_declared_symbol():
    from paper_1010_5534_amd import air
    lib = air.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(air.EXPORTS)


def test_struct_layouts_match_header():
    """sizeof/offsetof from a C compiler reading air.h == ctypes layouts."""
    from paper_1010_5534_amd import air
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "air.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(air_grid), sizeof(air_field), sizeof(air_view),
         sizeof(air_params), sizeof(air_tree), sizeof(air_stats));
  printf("%zu %zu %zu %zu %zu\n", offsetof(air_grid, block_level), offsetof(air_field, band),
         offsetof(air_tree, level), offsetof(air_tree, visits), offsetof(air_field, packed));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(x) for x in out]
    assert sizes[:6] == [C.sizeof(t) for t in (air.air_grid, air.air_field, air.air_view, air.air_params,
                                                 air.air_tree, air.air_stats)]
    assert sizes[6:] == [air.air_grid.block_level.offset, air.air_field.band.offset, air.air_tree.level.offset,
                         air.air_tree.visits.offset, air.air_field.packed.offset]


def test_stats_unpacking_reads_every_field():
    """The binding's stats dictionary reports every air_stats field with its
    value (distinct values in every field)."""
    from paper_1010_5534_amd import air
    s = air.air_stats()
    names = [n for n, _ in air.air_stats._fields_]
    for k, n in enumerate(names):
        if n == "rays_per_level":
            for i in range(air.MAX_LEVELS):
                s.rays_per_level[i] = 1000 + 7 * i
        elif n.startswith("ms_"):
            setattr(s, n, 0.5 + k)
        else:
            setattr(s, n, 3 + 11 * k)
    d = air.stats_dict(s)
    assert set(d) == set(names)
    for n in names:
        want = list(getattr(s, n)) if n == "rays_per_level" else getattr(s, n)
        assert d[n] == want, n


def test_packed_bytes_without_device():
    """air_field_packed_bytes needs no device: 2x2x2 bricks, 16 B or 8 B cells."""
    import ctypes as C
    from paper_1010_5534_amd import air
    g = air.air_grid()
    g.kind = 0
    g.n[:] = [5, 8, 3]
    g.hi[:] = [1.0, 1.0, 1.0]
    f = air.air_field()
    f.kind, f.n_bands, f.rho, f.emis, f.kappa = 0, 1, 16, 16, 16  # non-NULL, never dereferenced
    assert air.lib().air_field_packed_bytes(C.addressof(g), C.addressof(f)) == 3 * 4 * 2 * 8 * 16
    f.kind, f.temp, f.n_bands = 1, 16, 4
    assert air.lib().air_field_packed_bytes(C.addressof(g), C.addressof(f)) == 3 * 4 * 2 * 8 * 8
    # one band: (rho, j, kappa) evaluated once when packing, then the (rho, T)
    # copy at the next multiple of 256 bytes
    f.n_bands = 1
    assert air.lib().air_field_packed_bytes(C.addressof(g), C.addressof(f)) == 3 * 4 * 2 * 8 * 16 + 3 * 4 * 2 * 8 * 8
    g.n[:] = [5, 6, 5]  # 27 bricks: 3456 bytes of records, the copy at 3584
    assert air.lib().air_field_packed_bytes(C.addressof(g), C.addressof(f)) == 3584 + 27 * 8 * 8
    g.n[:] = [5, 8, 3]
    f.n_bands = 9
    assert air.lib().air_field_packed_bytes(C.addressof(g), C.addressof(f)) == air.AIR_EINVAL
    # block AMR: 2^3 base blocks of 4^3 cells and 8 children (16 blocks, 1024
    # cells of 16 B), then the leaf map of the 4^3 finest block lattice
    # (4 B each) at the next multiple of 256 bytes; no map for a lattice
    # above 2^26 positions
    a = air.air_grid()
    a.kind, a.bs, a.max_level, a.n_blocks = 1, 4, 1, 16
    a.n[:] = [2, 2, 2]
    a.hi[:] = [1.0, 1.0, 1.0]
    a.block_level, a.block_coord, a.block_child = 16, 16, 16  # non-NULL, never dereferenced
    f.n_bands = 1
    assert air.lib().air_field_packed_bytes(C.addressof(a), C.addressof(f)) == 1024 * 16 + 64 * 4
    f.n_bands = 2  # (rho, T): 8 B per cell
    assert air.lib().air_field_packed_bytes(C.addressof(a), C.addressof(f)) == 1024 * 8 + 64 * 4
    a.n_blocks, a.bs = 9, 2  # 9 * 8 * 8 = 576 bytes of records: the map at 768
    assert air.lib().air_field_packed_bytes(C.addressof(a), C.addressof(f)) == 768 + 64 * 4
    a.n_blocks, a.max_level, a.bs = 16, 8, 2  # (2 << 8)^3 = 2^27 lattice positions: no map
    assert air.lib().air_field_packed_bytes(C.addressof(a), C.addressof(f)) == 16 * 8 * 8


def test_null_context_is_rejected_without_device_work():
    from paper_1010_5534_amd import air
    lib = air.lib()
    assert lib.air_render(None, None, None, None, 1, None, None, None, None, None, None) == air.AIR_EINVAL
    assert lib.air_render_fixed(None, None, None, None, 1, 16, 0, None, None, None, None) == air.AIR_EINVAL
    assert lib.air_last_error(None) == b"context is NULL"
    lib.air_destroy(None)


def test_product_path_does_not_import_oracle():
    """The binding and the library sources never reference the oracle."""
    for rel in ("paper_1010_5534_amd/air.py", "paper_1010_5534_amd/__init__.py",
                "paper_1010_5534_amd/csrc/api.cpp", "paper_1010_5534_amd/csrc/march.hip",
                "paper_1010_5534_amd/csrc/tree.hip", "paper_1010_5534_amd/csrc/air_common.h",
                "paper_1010_5534_amd/csrc/learn.hip", "paper_1010_5534_amd/csrc/cnn.hip",
                "paper_1010_5534_amd/csrc/cnn.h", "paper_1010_5534_amd/csrc/noalloc.hip",
                "paper_1010_5534_amd/csrc/spectra.hip",
                "paper_1010_5534_amd/build.py"):
        txt = open(os.path.join(ROOT, rel)).read()
        assert "oracle" not in txt.lower(), rel


def test_binding_keeps_the_grown_tree_capacity(monkeypatch):
    """A call whose tree outgrows the capacity comes back AIR_ECAPACITY with
    the size it needs; the binding retries with that size once and starts
    the next call of the same shape from it, so a large tree is rendered
    once per call (host logic only: the library is a stand-in that checks
    the capacity it is handed)."""
    from paper_1010_5534_amd import air
    need = 5000
    seen = []

    class StandIn:
        def air_render(self, ctx, grid, field, views, n_views, prm, trees, images, flux, stats, stream):
            t = C.cast(trees, C.POINTER(air.air_tree))
            caps = [t[k].capacity for k in range(n_views)]
            seen.append(min(caps))
            for k in range(n_views):
                t[k].n_nodes = need
            return air.AIR_OK if min(caps) >= need else air.AIR_ECAPACITY

    monkeypatch.setattr(air, "lib", lambda: StandIn())
    ctx = object.__new__(air.Context)
    ctx.device, ctx._p, ctx._cache = 0, None, {}
    ctx._views_key, ctx._views_arr, ctx._cap_hint = None, None, {}
    ctx._stream = lambda: None

    def alloc(cap, nb):
        s = air.air_tree()
        s.capacity = cap
        return s, {}

    ctx._alloc_tree = alloc

    class Scene:
        n_bands = 1
        grid = C.c_int(0)
        field = C.c_int(0)

    from paper_1010_5534_amd import inputs
    views = [inputs.gaussian_view()]
    prm = air.params(16, 4, 0.5)
    for reuse in (False, True):
        seen.clear()
        for _ in range(3):
            trees, _, _, _ = ctx.render(Scene(), views, prm, want_image=False, want_flux=False, capacity=100,
                                        reuse=reuse)
            assert trees[0].n_nodes == need
        assert seen == ([100, need, need, need] if not reuse else [need, need, need]), seen

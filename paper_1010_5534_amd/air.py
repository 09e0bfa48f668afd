"""ctypes binding to libair.so (the HIP library).  Argument marshalling
only: every step of the rendering runs in the library's kernels; torch
provides device memory and the stream.  Names follow include/air.h."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libair.so")

AIR_OK, AIR_EINVAL, AIR_ENOMEM, AIR_EDEVICE, AIR_ECAPACITY, AIR_ENOTSUP = 0, -1, -2, -3, -4, -5
MAX_LEVELS, MAX_BANDS, MAX_VIEWS = 12, 8, 4096
GRID_UNIFORM, GRID_BLOCK_AMR = 0, 1
FIELD_RHO_J_KAPPA, FIELD_RHO_T = 0, 1
NODE_EXIST, NODE_TESTED, NODE_FLAGGED, NODE_BALANCE, NODE_REFINED, NODE_EVALUATED = 1, 2, 4, 8, 16, 32

EXPORTS = ("air_create", "air_destroy", "air_last_error", "air_render", "air_render_fixed", "air_trace_pixels",
           "air_field_packed_bytes", "air_field_pack", "air_cnn_create", "air_cnn_destroy", "air_cnn_set",
           "air_cnn_get", "air_features", "air_cnn_forward", "air_cnn_loss_grad", "air_cnn_adam", "air_tree_depth",
           "air_render_learned", "air_render_batch", "air_cnn_tensor", "air_render_fixed_noalloc",
           "air_render_spectra", "air_render_proposal", "air_cnn_save", "air_cnn_load", "air_tune_save",
           "air_tune_load", "air_tree_alloc", "air_tree_free")
CNN_FEATURES, CNN_CLASSES, CNN_PARAMS = 4, 6, 21414


class AirError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"AIR error {code}: {msg}")
        self.code = code


class air_grid(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bs", C.c_int32), ("max_level", C.c_int32), ("n_blocks", C.c_int32),
                ("block_level", C.c_void_p), ("block_coord", C.c_void_p), ("block_child", C.c_void_p)]


class air_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_bands", C.c_int32), ("rho", C.c_void_p), ("emis", C.c_void_p),
                ("kappa", C.c_void_p), ("temp", C.c_void_p), ("band", (C.c_double * 3) * MAX_BANDS),
                ("packed", C.c_void_p)]


class air_view(C.Structure):
    _fields_ = [("dir", C.c_double * 3), ("up", C.c_double * 3), ("center", C.c_double * 3), ("width", C.c_double)]


class air_params(C.Structure):
    _fields_ = [("coarse_n", C.c_int32), ("max_level", C.c_int32), ("xi_crit_I", C.c_float),
                ("xi_crit_N", C.c_float), ("band_weight", C.c_float * MAX_BANDS), ("flags", C.c_uint32)]


class air_tree(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("n_nodes", C.c_int64), ("n_per_level", C.c_int64 * MAX_LEVELS),
                ("n_leaves", C.c_int64), ("level", C.c_void_p), ("ix", C.c_void_p), ("iy", C.c_void_p),
                ("parent", C.c_void_p), ("first_child", C.c_void_p), ("state", C.c_void_p), ("I", C.c_void_p),
                ("N", C.c_void_p), ("xi_I", C.c_void_p), ("xi_N", C.c_void_p), ("visits", C.c_void_p)]


class air_stats(C.Structure):
    _fields_ = [("rays", C.c_int64), ("rays_per_level", C.c_int64 * MAX_LEVELS), ("hits", C.c_int64),
                ("visits", C.c_int64), ("leaves", C.c_int64), ("tested", C.c_int64), ("flagged", C.c_int64),
                ("balance", C.c_int64), ("depth", C.c_int32), ("march_launches", C.c_int32),
                ("ms_total", C.c_double), ("ms_march", C.c_double), ("ms_test", C.c_double)]


class air_spectrum(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("bins", C.c_void_p), ("weight", C.c_void_p)]


class air_learn_params(C.Structure):
    _fields_ = [("c_ray", C.c_float), ("c_sweep", C.c_float), ("max_depth", C.c_int32), ("flags", C.c_uint32)]


class air_learn_stats(C.Structure):
    _fields_ = [("spec_rays", C.c_int64), ("wasted", C.c_int64), ("missing", C.c_int64),
                ("depth_hist", C.c_int64 * MAX_LEVELS), ("ms_features", C.c_double), ("ms_spec", C.c_double)]


_lib = None


def lib():
    """Load libair.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python paper_1010_5534_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.air_create.argtypes = [C.POINTER(vp), C.c_int32]
        L.air_create.restype = C.c_int32
        L.air_destroy.argtypes = [vp]
        L.air_destroy.restype = None
        L.air_last_error.argtypes = [vp]
        L.air_last_error.restype = C.c_char_p
        L.air_render.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.air_render.restype = C.c_int32
        L.air_render_batch.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.air_render_batch.restype = C.c_int32
        L.air_render_fixed.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.air_render_fixed.restype = C.c_int32
        L.air_render_fixed_noalloc.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
        L.air_render_fixed_noalloc.restype = C.c_int32
        L.air_render_spectra.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.air_render_spectra.restype = C.c_int32
        L.air_render_proposal.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.air_render_proposal.restype = C.c_int32
        L.air_trace_pixels.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int64, vp, vp, vp, vp, vp, vp, vp]
        L.air_trace_pixels.restype = C.c_int32
        L.air_field_packed_bytes.argtypes = [vp, vp]
        L.air_field_packed_bytes.restype = C.c_int64
        L.air_field_pack.argtypes = [vp, vp, vp, vp, C.c_int64, vp]
        L.air_field_pack.restype = C.c_int32
        i32 = C.c_int32
        L.air_cnn_create.argtypes = [vp, C.POINTER(vp)]
        L.air_cnn_destroy.argtypes = [vp]
        L.air_cnn_destroy.restype = None
        L.air_cnn_set.argtypes = [vp, vp, vp, vp, vp]
        L.air_cnn_get.argtypes = [vp, vp, vp, vp, vp]
        L.air_features.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp]
        L.air_cnn_forward.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
        L.air_cnn_loss_grad.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.air_cnn_adam.argtypes = [vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.air_tree_depth.argtypes = [vp, vp, i32, vp, vp]
        L.air_cnn_tensor.argtypes = [vp, i32, vp, C.c_int64, vp]
        L.air_render_learned.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        cp = C.c_char_p
        L.air_cnn_save.argtypes = [vp, vp, cp]
        L.air_cnn_load.argtypes = [vp, vp, cp]
        L.air_tune_save.argtypes = [vp, cp]
        L.air_tune_load.argtypes = [vp, cp]
        L.air_tree_alloc.argtypes = [vp, i32, C.c_int64, vp]
        L.air_tree_free.argtypes = [vp, vp]
        for name in ("air_cnn_create", "air_cnn_set", "air_cnn_get", "air_features", "air_cnn_forward",
                     "air_cnn_loss_grad", "air_cnn_adam", "air_tree_depth", "air_render_learned", "air_cnn_tensor",
                     "air_cnn_save", "air_cnn_load", "air_tune_save", "air_tune_load", "air_tree_alloc",
                     "air_tree_free"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


@dataclasses.dataclass
class DeviceScene:
    """Grid and field resident in device memory (torch tensors)."""

    grid: air_grid
    field: air_field
    tensors: list
    n_bands: int


def upload(grid, field, device="cuda") -> DeviceScene:
    """Copy an inputs.Grid / inputs.Field to the GPU once."""
    torch = _torch()
    keep = []

    def dev(a, dtype):
        if a is None:
            return None
        t = torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(device=device, dtype=dtype)
        keep.append(t)
        return t.data_ptr()

    g = air_grid()
    g.kind = grid.kind
    g.n[:] = [int(x) for x in grid.n]
    g.lo[:] = [float(x) for x in grid.lo]
    g.hi[:] = [float(x) for x in grid.hi]
    g.bs = grid.bs
    g.max_level = grid.max_level
    g.n_blocks = grid.n_blocks
    if grid.kind == GRID_BLOCK_AMR:
        g.block_level = dev(grid.block_level, torch.int32)
        g.block_coord = dev(grid.block_coord, torch.int32)
        g.block_child = dev(grid.block_child, torch.int32)
    f = air_field()
    f.kind = field.kind
    f.n_bands = field.n_bands
    f.rho = dev(field.rho, torch.float32)
    f.emis = dev(field.emis, torch.float32)
    f.kappa = dev(field.kappa, torch.float32)
    f.temp = dev(field.temp, torch.float32)
    if field.bands is not None:
        for b in range(field.n_bands):
            for k in range(3):
                f.band[b][k] = float(field.bands[b][k])
    return DeviceScene(g, f, keep, field.n_bands)


def scene_from_tensors(n: int, rho, temp, bands) -> DeviceScene:
    """A uniform n^3 unit-box (rho, T) scene from float32 device tensors
    (z slowest, x fastest) and host band parameters [n_bands][3]."""
    torch = _torch()
    rho = rho.contiguous().to(torch.float32)
    temp = temp.contiguous().to(torch.float32)
    bands = np.asarray(bands, dtype=np.float64).reshape(-1, 3)
    g = air_grid()
    g.kind = GRID_UNIFORM
    g.n[:] = [n, n, n]
    g.lo[:] = [0.0, 0.0, 0.0]
    g.hi[:] = [1.0, 1.0, 1.0]
    f = air_field()
    f.kind = FIELD_RHO_T
    f.n_bands = len(bands)
    f.rho = rho.data_ptr()
    f.temp = temp.data_ptr()
    for b in range(len(bands)):
        for k in range(3):
            f.band[b][k] = float(bands[b][k])
    return DeviceScene(g, f, [rho, temp], len(bands))


def _views(views) -> C.Array:
    arr = (air_view * len(views))()
    for k, v in enumerate(views):
        arr[k].dir[:] = [float(x) for x in v.dir]
        arr[k].up[:] = [float(x) for x in v.up]
        arr[k].center[:] = [float(x) for x in v.center]
        arr[k].width = float(v.width)
    return arr


FLAG_TIMING = 1
FLAG_SUPERRES = 2


def params(coarse_n, max_level, xi_crit_I=0.5, xi_crit_N=2.0, band_weight=None, timing=False,
           superres=False) -> air_params:
    p = air_params()
    p.coarse_n = coarse_n
    p.max_level = max_level
    p.xi_crit_I = xi_crit_I
    p.xi_crit_N = xi_crit_N
    w = [1.0] * MAX_BANDS if band_weight is None else list(band_weight) + [0.0] * (MAX_BANDS - len(band_weight))
    p.band_weight[:] = [float(x) for x in w[:MAX_BANDS]]
    p.flags = (FLAG_TIMING if timing else 0) | (FLAG_SUPERRES if superres else 0)
    return p


def stats_dict(s: air_stats) -> dict:
    return dict(rays=s.rays, rays_per_level=list(s.rays_per_level), hits=s.hits, visits=s.visits, leaves=s.leaves,
                tested=s.tested, flagged=s.flagged, balance=s.balance, depth=s.depth,
                march_launches=s.march_launches, ms_total=s.ms_total, ms_march=s.ms_march, ms_test=s.ms_test)


class Tree:
    """Pixel quadtree of one view (device tensors, canonical order).  The
    node arrays (level, ix, iy, parent, first_child, state, I [bands, n],
    N, xi_I, xi_N, visits) are views of the output buffers, cut to n_nodes
    when first read."""

    ARRAYS = ("level", "ix", "iy", "parent", "first_child", "state", "I", "N", "xi_I", "xi_N", "visits")

    def __init__(self, n_nodes: int, n_per_level: list, n_leaves: int, buffers: dict):
        self.n_nodes = n_nodes
        self.n_per_level = n_per_level
        self.n_leaves = n_leaves
        self._buf = buffers

    def __getattr__(self, name):
        if name in Tree.ARRAYS:
            b = self.__dict__["_buf"][name]
            return b[:, :self.n_nodes] if name == "I" else b[:self.n_nodes]
        raise AttributeError(name)


class Context:
    """One air_ctx on one device."""

    def __init__(self, device: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the AIR library runs on the GPU only")
        self.device = device
        self._cache = {}
        self._views_key, self._views_arr = None, None
        self._cap_hint = {}
        self._p = C.c_void_p()
        rc = lib().air_create(C.byref(self._p), device)
        if rc != AIR_OK:
            raise AirError(rc, "air_create failed")

    def close(self):
        if self._p:
            lib().air_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != AIR_OK:
            raise AirError(rc, lib().air_last_error(self._p).decode())

    def _stream(self):
        return _torch().cuda.current_stream(self.device).cuda_stream

    def tune_save(self, path):
        """Write the batch's tuned launch shapes to a text file (air_tune_save)."""
        self._check(lib().air_tune_save(self._p, os.fsencode(path)))

    def tune_load(self, path):
        """Read launch shapes written by tune_save (air_tune_load)."""
        self._check(lib().air_tune_load(self._p, os.fsencode(path)))

    def prepare(self, scene: DeviceScene) -> DeviceScene:
        """Write the field's march layout once (air_field_pack) and attach it,
        so renders skip the per-call packing."""
        torch = _torch()
        nbytes = lib().air_field_packed_bytes(C.addressof(scene.grid), C.addressof(scene.field))
        if nbytes < 0:
            raise AirError(int(nbytes), "air_field_packed_bytes failed")
        buf = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(lib().air_field_pack(self._p, C.addressof(scene.grid), C.addressof(scene.field), buf.data_ptr(),
                                         int(nbytes), self._stream()))
        scene.tensors.append(buf)
        scene.field.packed = buf.data_ptr()
        return scene

    def _alloc_tree(self, cap, nb):
        torch = _torch()
        dev = f"cuda:{self.device}"
        t = dict(level=torch.empty(cap, dtype=torch.int8, device=dev),
                 ix=torch.empty(cap, dtype=torch.int32, device=dev),
                 iy=torch.empty(cap, dtype=torch.int32, device=dev),
                 parent=torch.empty(cap, dtype=torch.int32, device=dev),
                 first_child=torch.empty(cap, dtype=torch.int32, device=dev),
                 state=torch.empty(cap, dtype=torch.uint8, device=dev),
                 I=torch.empty((nb, cap), dtype=torch.float32, device=dev),
                 N=torch.empty(cap, dtype=torch.float32, device=dev),
                 xi_I=torch.empty(cap, dtype=torch.float32, device=dev),
                 xi_N=torch.empty(cap, dtype=torch.float32, device=dev),
                 visits=torch.empty(cap, dtype=torch.int32, device=dev))
        s = air_tree()
        s.capacity = cap
        for k, v in t.items():
            setattr(s, k, v.data_ptr())
        return s, t

    def render(self, scene: DeviceScene, views: Sequence, prm: air_params, want_tree=True, want_image=True,
               want_flux=True, capacity: Optional[int] = None, reuse: bool = False):
        """Plain AIR over the views.  Returns (trees, images, flux, stats).
        reuse=True hands back the same output tensors on every call with the
        same shapes (the next call overwrites them)."""
        return self._render(scene, views, prm, want_tree, want_image, want_flux, capacity, reuse, None, None)

    def render_batch(self, scene: DeviceScene, views: Sequence, prm: air_params, want_tree=True, want_image=True,
                     want_flux=True, capacity: Optional[int] = None, reuse: bool = True):
        """air_render_batch: the same outputs as render(), from a captured,
        autotuned launch sequence (reuse keeps the output buffers, so the
        captured sequence can be replayed)."""
        return self._render(scene, views, prm, want_tree, want_image, want_flux, capacity, reuse, "batch", None)

    def render_learned(self, scene: DeviceScene, views: Sequence, prm: air_params, net: "Network",
                       c_ray: float, c_sweep: float, max_depth: int = 5, want_tree=True, want_image=True,
                       want_flux=True, capacity: Optional[int] = None, reuse: bool = False):
        """AIR with the learned depth proposal (air_render_learned).  Returns
        (trees, images, flux, stats, learn_stats); outputs equal render()'s."""
        lp = air_learn_params()
        lp.c_ray, lp.c_sweep, lp.max_depth, lp.flags = c_ray, c_sweep, max_depth, 0
        ls = air_learn_stats()
        out = self._render(scene, views, prm, want_tree, want_image, want_flux, capacity, reuse, (net, lp), ls)
        return out + (dict(spec_rays=ls.spec_rays, wasted=ls.wasted, missing=ls.missing,
                           depth_hist=list(ls.depth_hist)[:6], ms_features=ls.ms_features, ms_spec=ls.ms_spec),)

    def render_proposal(self, scene: DeviceScene, views: Sequence, prm: air_params, depth, max_depth: int = 5,
                        want_tree=True, want_image=True, want_flux=True, capacity: Optional[int] = None,
                        reuse: bool = False):
        """air_render_proposal: speculation to the given depth per coarse
        pixel (device uint8 [V, N0, N0]) in place of the network's choice.
        Returns (trees, images, flux, stats, learn_stats); outputs equal
        render()'s."""
        depth = depth.contiguous()
        ls = air_learn_stats()
        out = self._render(scene, views, prm, want_tree, want_image, want_flux, capacity, reuse,
                           ("proposal", depth, max_depth), ls)
        return out + (dict(spec_rays=ls.spec_rays, wasted=ls.wasted, missing=ls.missing,
                           depth_hist=list(ls.depth_hist)[:6], ms_features=ls.ms_features, ms_spec=ls.ms_spec),)

    def _view_array(self, views) -> C.Array:
        # the last conversion is kept: repeated calls with the same view
        # values skip building the ctypes array
        key = tuple((tuple(v.dir), tuple(v.up), tuple(v.center), v.width) for v in views)
        if key != self._views_key:
            self._views_arr, self._views_key = _views(views), key
        return self._views_arr

    def _tree_array(self, V, nb, cap, reuse):
        trees = (air_tree * V)()
        tkey = ("tree", V, nb, cap)
        if reuse and tkey in self._cache:
            pairs = self._cache[tkey]
        else:
            pairs = [self._alloc_tree(cap, nb) for _ in range(V)]
            if reuse:
                self._cache[tkey] = pairs
        keep = []
        for k in range(V):
            s, t = pairs[k]
            trees[k] = s
            keep.append(t)
        return trees, keep

    def _render(self, scene, views, prm, want_tree, want_image, want_flux, capacity, reuse, learned, ls):
        V, nb = len(views), scene.n_bands
        vs = self._view_array(views)
        # with reuse, the output buffers and the argument structures of a call
        # shape are built once (flux is handed back as a copy)
        ckey = ("call", V, nb, prm.coarse_n, prm.max_level, capacity, want_tree, want_image, want_flux)
        bundle = self._cache.get(ckey) if reuse else None
        if bundle is None:
            torch = _torch()
            R = prm.coarse_n << prm.max_level
            bound = sum((prm.coarse_n << L) ** 2 for L in range(prm.max_level + 1))
            # start from the capacity this call shape needed last time, so a
            # large tree does not come back AIR_ECAPACITY (and get rendered
            # again) on every call
            cap = max(min(bound, capacity or (1 << 21)), self._cap_hint.get(ckey, 0))
            ikey = ("img", V, nb, R)
            if want_image and reuse and ikey in self._cache:
                images = self._cache[ikey]
            else:
                images = torch.empty((V, nb + 1, R, R), dtype=torch.float32, device=f"cuda:{self.device}") \
                    if want_image else None
                if want_image and reuse:
                    self._cache[ikey] = images
            flux = np.zeros((V, nb), dtype=np.float64) if want_flux else None
            trees, keep = self._tree_array(V, nb, cap, reuse) if want_tree else (None, [])
            bundle = [images, flux, air_stats(), trees, keep, cap]
            if reuse:
                self._cache[ckey] = bundle
        images, flux, st, trees, keep, cap = bundle
        C.memset(C.addressof(st), 0, C.sizeof(st))  # fields a call does not fill read as zero
        if want_flux:
            flux.fill(0.0)
        while True:
            targs = (C.addressof(trees) if want_tree else None, images.data_ptr() if want_image else None,
                     flux.ctypes.data if want_flux else None, C.addressof(st))
            if isinstance(learned, tuple) and learned[0] == "proposal":
                rc = lib().air_render_proposal(self._p, C.addressof(scene.grid), C.addressof(scene.field),
                                               C.addressof(vs), V, C.addressof(prm), learned[1].data_ptr(),
                                               learned[2], *targs, C.addressof(ls), self._stream())
            elif learned is None or learned == "batch":
                fn = lib().air_render if learned is None else lib().air_render_batch
                rc = fn(self._p, C.addressof(scene.grid), C.addressof(scene.field), C.addressof(vs),
                        V, C.addressof(prm), *targs, self._stream())
            else:
                rc = lib().air_render_learned(self._p, C.addressof(scene.grid), C.addressof(scene.field),
                                              C.addressof(vs), V, C.addressof(prm), learned[0]._p,
                                              C.addressof(learned[1]), *targs, C.addressof(ls), self._stream())
            if rc == AIR_ECAPACITY and want_tree:
                cap = max(trees[k].n_nodes for k in range(V))
                self._cap_hint[ckey] = cap
                trees, keep = self._tree_array(V, nb, cap, reuse)
                bundle[3:6] = [trees, keep, cap]
                continue
            self._check(rc)
            break
        out = []
        if want_tree:
            for k in range(V):
                n = trees[k].n_nodes
                t = keep[k]
                out.append(Tree(n, list(trees[k].n_per_level), trees[k].n_leaves, t))
        return out, images, (flux.copy() if reuse and want_flux else flux), stats_dict(st)

    def render_fixed(self, scene: DeviceScene, views: Sequence, coarse_n: int, level: int, want_image=True,
                     want_flux=True):
        torch = _torch()
        V, nb = len(views), scene.n_bands
        R = coarse_n << level
        vs = _views(views)
        images = torch.empty((V, nb + 1, R, R), dtype=torch.float32, device=f"cuda:{self.device}") \
            if (want_image or want_flux) else None
        flux = np.zeros((V, nb), dtype=np.float64) if want_flux else None
        st = air_stats()
        rc = lib().air_render_fixed(self._p, C.addressof(scene.grid), C.addressof(scene.field), C.addressof(vs), V,
                                    coarse_n, level, images.data_ptr() if images is not None else None,
                                    flux.ctypes.data if want_flux else None, C.addressof(st), self._stream())
        self._check(rc)
        return images, flux, stats_dict(st)

    def render_spectra(self, scene: DeviceScene, views: Sequence, prm: air_params, bins, weight,
                       want_spectra=True, want_image=True, want_flux=True, capacity: Optional[int] = None):
        """air_render_spectra: plain AIR on the broadband sum_b weight_b I_b
        of the bin table bins [n_bins][5] (k0, s, e0, q, E).  Returns (trees,
        spectra [V, capacity, n_bins] device or None, images [V, 2, R, R],
        flux [V, n_bins] host (the image spectra), stats)."""
        torch = _torch()
        bins = np.ascontiguousarray(bins, dtype=np.float64).reshape(-1, 5)
        w = np.ascontiguousarray(weight, dtype=np.float32).reshape(-1)
        B, V = bins.shape[0], len(views)
        spec = air_spectrum()
        spec.n_bins, spec.bins, spec.weight = B, bins.ctypes.data, w.ctypes.data
        R = prm.coarse_n << prm.max_level
        bound = sum((prm.coarse_n << L) ** 2 for L in range(prm.max_level + 1))
        cap = min(bound, capacity or (1 << 20))
        dev = f"cuda:{self.device}"
        vs = _views(views)
        while True:
            trees, keep = self._tree_array(V, 1, cap, False)
            spectra = torch.empty((V, cap, B), dtype=torch.float32, device=dev) if want_spectra else None
            images = torch.empty((V, 2, R, R), dtype=torch.float32, device=dev) if want_image else None
            flux = np.zeros((V, B), dtype=np.float64) if want_flux else None
            st = air_stats()
            rc = lib().air_render_spectra(self._p, C.addressof(scene.grid), C.addressof(scene.field),
                                          C.addressof(vs), V, C.addressof(prm), C.addressof(spec),
                                          C.addressof(trees), spectra.data_ptr() if want_spectra else None,
                                          images.data_ptr() if want_image else None,
                                          flux.ctypes.data if want_flux else None, C.addressof(st), self._stream())
            if rc == AIR_ECAPACITY:
                cap = max(trees[k].n_nodes for k in range(V))
                continue
            self._check(rc)
            break
        out = [Tree(trees[k].n_nodes, list(trees[k].n_per_level), trees[k].n_leaves, keep[k]) for k in range(V)]
        return out, spectra, images, flux, stats_dict(st)

    def render_fixed_noalloc(self, scene: DeviceScene, views: Sequence, coarse_n: int, level: int, images=None,
                             flux=None, want_flux=True):
        """air_render_fixed_noalloc: the fixed-resolution render with its
        workspace in the library's static device array (the scene must be
        prepared).  images / flux: device tensors [V, nb + 1, R, R] float32 /
        [V, nb] float64, allocated here when not given.  Returns (images,
        flux); nothing waits for the stream."""
        torch = _torch()
        V, nb = len(views), scene.n_bands
        R = coarse_n << level
        dev = f"cuda:{self.device}"
        if images is None:
            images = torch.empty((V, nb + 1, R, R), dtype=torch.float32, device=dev)
        if want_flux and flux is None:
            flux = torch.empty((V, nb), dtype=torch.float64, device=dev)
        vs = _views(views)
        rc = lib().air_render_fixed_noalloc(self._p, C.addressof(scene.grid), C.addressof(scene.field),
                                            C.addressof(vs), V, coarse_n, level, images.data_ptr(),
                                            flux.data_ptr() if want_flux else None, self._stream())
        self._check(rc)
        return images, (flux if want_flux else None)

    def trace_pixels(self, scene: DeviceScene, view, coarse_n: int, level, ix, iy):
        torch = _torch()
        dev = f"cuda:{self.device}"
        lv = torch.as_tensor(np.asarray(level, dtype=np.int32), device=dev)
        xi = torch.as_tensor(np.asarray(ix, dtype=np.int32), device=dev)
        yi = torch.as_tensor(np.asarray(iy, dtype=np.int32), device=dev)
        n = lv.numel()
        I = torch.empty((scene.n_bands, n), dtype=torch.float32, device=dev)
        N = torch.empty(n, dtype=torch.float32, device=dev)
        vis = torch.empty(n, dtype=torch.int32, device=dev)
        vs = _views([view])
        rc = lib().air_trace_pixels(self._p, C.addressof(scene.grid), C.addressof(scene.field), C.addressof(vs),
                                    coarse_n, n, lv.data_ptr(), xi.data_ptr(), yi.data_ptr(), I.data_ptr(),
                                    N.data_ptr(), vis.data_ptr(), self._stream())
        self._check(rc)
        return I, N, vis

    # ---------------------------------------------------- learned proposal
    def features(self, scene: DeviceScene, views: Sequence, coarse_n: int, band_weight=None):
        """Raw coarse feature maps [V, N0, N0, 4] (air_features)."""
        torch = _torch()
        V = len(views)
        w = np.ones(scene.n_bands, np.float32) if band_weight is None else np.asarray(band_weight, np.float32)
        out = torch.empty((V, coarse_n, coarse_n, CNN_FEATURES), dtype=torch.float32, device=f"cuda:{self.device}")
        vs = _views(views)
        self._check(lib().air_features(self._p, C.addressof(scene.grid), C.addressof(scene.field), C.addressof(vs),
                                       V, coarse_n, w.ctypes.data, out.data_ptr(), self._stream()))
        return out

    def tree_depth(self, tree: Tree, coarse_n: int):
        """Depth label per coarse pixel [N0, N0] int32 (air_tree_depth)."""
        torch = _torch()
        t = air_tree()
        t.capacity = tree.n_nodes
        t.n_nodes = tree.n_nodes
        t.level, t.ix, t.iy = tree.level.data_ptr(), tree.ix.data_ptr(), tree.iy.data_ptr()
        out = torch.empty((coarse_n, coarse_n), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(lib().air_tree_depth(self._p, C.addressof(t), coarse_n, out.data_ptr(), self._stream()))
        return out


class Network:
    """The depth-proposal network (air_cnn) of a context."""

    def __init__(self, ctx: Context, params=None, mean=None, scale=None):
        self.ctx = ctx
        self._p = C.c_void_p()
        ctx._check(lib().air_cnn_create(ctx._p, C.byref(self._p)))
        if params is not None:
            self.set(params, mean, scale)

    def close(self):
        if self._p:
            lib().air_cnn_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, params, mean=None, scale=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (CNN_PARAMS,)
        m = np.zeros(CNN_FEATURES, np.float32) if mean is None else np.ascontiguousarray(mean, np.float32)
        s = np.ones(CNN_FEATURES, np.float32) if scale is None else np.ascontiguousarray(scale, np.float32)
        self.ctx._check(lib().air_cnn_set(self.ctx._p, self._p, p.ctypes.data, m.ctypes.data, s.ctypes.data))

    def save(self, path):
        """Checkpoint: parameters, standardisation and optimiser state (air_cnn_save)."""
        self.ctx._check(lib().air_cnn_save(self.ctx._p, self._p, os.fsencode(path)))

    def load(self, path):
        """Restore a checkpoint written by save (air_cnn_load)."""
        self.ctx._check(lib().air_cnn_load(self.ctx._p, self._p, os.fsencode(path)))

    def get(self):
        p = np.zeros(CNN_PARAMS, np.float32)
        m = np.zeros(CNN_FEATURES, np.float32)
        s = np.zeros(CNN_FEATURES, np.float32)
        self.ctx._check(lib().air_cnn_get(self.ctx._p, self._p, p.ctypes.data, m.ctypes.data, s.ctypes.data))
        return p, m, s

    def forward(self, feat):
        """feat: float32 device [n, h, w, 4] -> logits [n, h, w, 8]."""
        torch = _torch()
        feat = feat.contiguous()
        n, h, w, _ = feat.shape
        z = torch.empty((n, h, w, 8), dtype=torch.float32, device=feat.device)
        self.ctx._check(lib().air_cnn_forward(self.ctx._p, self._p, feat.data_ptr(), n, h, w, z.data_ptr(),
                                              self.ctx._stream()))
        return z

    def loss_grad(self, feat, labels, class_weight, want_loss=True, want_grad=False):
        torch = _torch()
        feat = feat.contiguous()
        labels = labels.to(torch.int32).contiguous()
        n, h, w, _ = feat.shape
        cw = np.ascontiguousarray(class_weight, np.float32)
        loss = C.c_double(0.0)
        g = torch.empty(CNN_PARAMS, dtype=torch.float32, device=feat.device) if want_grad else None
        self.ctx._check(lib().air_cnn_loss_grad(self.ctx._p, self._p, feat.data_ptr(), labels.data_ptr(), n, h, w,
                                                cw.ctypes.data, C.byref(loss) if want_loss else None,
                                                g.data_ptr() if want_grad else None, self.ctx._stream()))
        return (loss.value if want_loss else None), g

    TENSORS = dict(x0=(0, 8), a1=(1, 32), a2=(2, 32), a3=(3, 32), z=(4, 8), dz=(5, 8), d3=(6, 32), d2=(7, 32),
                   d1=(8, 32))

    def tensor(self, name, pixels):
        """Intermediate of the last forward / loss_grad call (air_cnn_tensor):
        [pixels, channels], bfloat16 except the float32 logits."""
        torch = _torch()
        which, ch = Network.TENSORS[name]
        dt = torch.float32 if name == "z" else torch.bfloat16
        out = torch.empty((pixels, ch), dtype=dt, device=f"cuda:{self.ctx.device}")
        self.ctx._check(lib().air_cnn_tensor(self.ctx._p, which, out.data_ptr(), out.numel() * out.element_size(),
                                             self.ctx._stream()))
        return out

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx._check(lib().air_cnn_adam(self.ctx._p, self._p, lr, beta1, beta2, eps, self.ctx._stream()))

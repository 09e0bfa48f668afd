#!/usr/bin/env python3
"""Benchmark of adaptive image ray-tracing on one MI355X.

Workload (the uniform colliding-winds case): 256^3 float32 (rho, T) field
with two wind sources and a shocked shell (seed 0), one band j = rho^2
T^0.5, kappa = rho T^-1.5 (evaluated once per cell when the field is packed); 64x64 coarse image, 5 refinement levels (2048^2 effective),
xi_crit = 0.5, three views (+z, +x, (1,1,1)/sqrt3).  One step = plain AIR of
the three views in one call: march every level, refinement test, 2:1
closure, compaction, canonical quadtree, raster assembly and float64 flux.
Beside it: the fixed 2048^2 image of the same views.

Prints one JSON line.  `value` is plain-AIR rays/s over the whole job (all
tree nodes traced, inputs resident in HBM, host overhead included)."""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s & per-image time: learned AIR vs plain AIR vs fixed-res, 1 GPU"
HBM_PEAK_GBS = 8000.0
N0, LMAX, XI_CRIT, SEED, NGRID = 64, 5, 0.5, 0, 256
# algorithmic bytes of the march: per (ray, cell) visit the three float32
# values the one-band integration reads (rho, j, kappa: the packed record
# evaluates j and kappa from (rho, T) once per field); per ray its queue entry
# (8 B) and results (I, N, visits: 12 B, state byte)
BYTES_PER_VISIT = 12
BYTES_PER_RAY_QUEUE = 8 + 12 + 1
BYTES_PER_RAY_FIXED = 8  # I and N written to the raster


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_from_profile(kernel):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "march_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1010_5534_amd", "csrc", "march.hip"), "rb").read()
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get(kernel)


def cpu_baseline(g, f, views, min_seconds=10.0):
    """The FP64 oracle on the host cores: plain AIR of the same three views,
    repeated until about min_seconds have passed.  Also returns the first
    repetition's trees."""
    import oracle
    oracle.lib()
    t = time.perf_counter()
    nodes, reps, first = 0, 0, None
    while True:
        trees = [oracle.air(g, f, v, N0, LMAX, XI_CRIT) for v in views]
        nodes += sum(tr.nodes for tr in trees)
        first = first or trees
        reps += 1
        dt = time.perf_counter() - t
        if dt >= min_seconds:
            break
    cores = oracle.num_threads()
    # one thread: plain AIR of the first view, repeated for about 5 s
    oracle.set_threads(1)
    t1, n1, r1 = time.perf_counter(), 0, 0
    while True:
        n1 += oracle.air(g, f, views[0], N0, LMAX, XI_CRIT).nodes
        r1 += 1
        d1 = time.perf_counter() - t1
        if d1 >= min_seconds / 2:
            break
    oracle.set_threads(cores)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=nodes / dt, unit="rays/s", cores=cores, kind="oracle",
                sample=f"full plain AIR of the 3 views, {reps} times ({nodes} rays) in {dt:.1f} s, FP64, OpenMP",
                seconds=dt, value_1_thread=n1 / d1,
                sample_1_thread=f"plain AIR of view 0, {r1} times ({n1} rays) in {d1:.1f} s on 1 thread",
                cpu_model=model, host_cpus=len(os.sched_getaffinity(0))), first


def oracle_error(gpu_trees, orc_trees, np):
    """The timed plain-AIR trees (host copies) against the oracle's: node sets, and the
    largest relative difference of I and N over every node (misses are exact
    zeros on both sides)."""
    worst_i = worst_n = 0.0
    same = True
    for tg, to in zip(gpu_trees, orc_trees):
        lv, ix, iy = (tg[k].astype(np.int64) for k in ("level", "ix", "iy"))
        I, Nn = tg["I"].astype(np.float64), tg["N"].astype(np.float64)
        same = same and len(lv) == to.nodes
        for L in range(LMAX + 1):
            m = lv == L
            ex = (to.state[L][iy[m], ix[m]] & 1) > 0
            same = same and bool(ex.all()) and int(m.sum()) == int(((to.state[L] & 1) > 0).sum())
            for a, b in ((I[:, m], to.I[L][:, iy[m], ix[m]]), (Nn[m], to.N[L][iy[m], ix[m]])):
                den = np.abs(b)
                with np.errstate(invalid="ignore", divide="ignore"):
                    r = np.where(den > 0, np.abs(a - b) / den, np.where(a == 0, 0.0, np.inf))
                e = float(r[..., ex].max()) if ex.any() else 0.0
                if a.ndim == 2:
                    worst_i = max(worst_i, e)
                else:
                    worst_n = max(worst_n, e)
    return dict(trees_identical=same, max_rel_err_I=worst_i, max_rel_err_N=worst_n, tolerance=1e-5)


def device_median(fn, reps, torch):
    """Median device time (ms) of fn over reps calls, from each call's own
    air_stats.ms_total (HIP events on the call's stream), after one warm-up."""
    out = fn()
    ms = []
    for _ in range(reps):
        out = fn()
        # render calls return (trees, images, flux, stats[, learn stats]); render_fixed (images, flux, stats)
        ms.append((out[3] if len(out) >= 4 else out[-1])["ms_total"])
    torch.cuda.synchronize()
    ms.sort()
    return out, ms[len(ms) // 2]


def ring_experiment(ctx, air, inputs, np, torch, args):
    """Section 3's experiment re-created (Eq. 1 ring, Table 1): the face-on
    ring on a block hierarchy of 4^3 base blocks of 8^3 cells with 4 nested
    levels (512^3 effective), a 32^2 base image with 4 image levels at
    xi_crit 0.2, 0.5 and 0.8, against the fixed 512^2 image.  Error as in
    Table 1: (F_exact - F) / F_exact with F_exact the emission summed over the
    grid's leaf cells; time = median device time of one image."""
    log("ring experiment (Table 1)")
    g, f = inputs.ring()
    scene = ctx.prepare(air.upload(g, f))
    v = inputs.ring_view()
    n0, lm, width = 32, 4, float(v.width)
    bs = g.bs
    leaf = np.repeat(np.asarray(g.block_child) < 0, bs ** 3)
    h = (g.hi[0] - g.lo[0]) / (g.n[0] * bs) / 2.0 ** np.repeat(np.asarray(g.block_level), bs ** 3)
    exact = float(np.sum(np.where(leaf, f.emis.astype(np.float64) * h ** 3, 0.0)))
    reps = max(5, args.steps)
    out_f, ms_f = device_median(lambda: ctx.render_fixed(scene, [v], n0, lm), reps, torch)
    rows = [dict(calc="fixed", xi_crit=None, pixels=out_f[2]["rays"],
                 flux_err=(exact - float(out_f[1][0][0])) / exact, ms=ms_f, speedup=1.0)]
    for xc in (0.2, 0.5, 0.8):
        prm = air.params(n0, lm, xc)
        out, ms = device_median(lambda: ctx.render(scene, [v], prm, reuse=True), reps, torch)
        rows.append(dict(calc="AIR", xi_crit=xc, pixels=out[3]["rays"],
                         refined=(out[3]["rays"] - n0 * n0) // 4,
                         flux_err=(exact - float(out[2][0][0])) / exact, ms=ms, speedup=ms_f / ms))
    return dict(workload="Eq. 1 ring, block AMR 4^3 x 8^3 cells, 4 levels (512^3 effective), face-on view, "
                         "32^2 base image, 4 image levels (512^2 effective)",
                blocks=g.n_blocks, exact_flux=exact, rows=rows,
                paper_table1="fixed 262144 px; AIR 0.2: 40512 px, 2e-6; 0.5: 23384 px, 1e-4; 0.8: 22748 px, 1e-4 "
                             "(hardware not named; context only)")


def xi_sweep(ctx, air, scene, views, flux_fixed, np, torch, args):
    """The benchmark workload at xi_crit 0.2, 0.5 and 0.8: rays, device time
    per call and the flux error against the fixed 2048^2 image per view."""
    rows = []
    for xc in (0.2, 0.5, 0.8):
        prm = air.params(N0, LMAX, xc)
        out, ms = device_median(lambda: ctx.render(scene, views, prm, want_image=False, reuse=True),
                                max(3, args.steps // 2), torch)
        err = None if flux_fixed is None else [float((flux_fixed[k][0] - out[2][k][0]) / flux_fixed[k][0])
                                               for k in range(len(views))]
        rows.append(dict(xi_crit=xc, rays=out[3]["rays"], ms_device=ms, flux_rel_err_vs_fixed=err))
    return rows


def spectra_run(ctx, air, inputs, np, torch, g, f, views, args):
    """Per-pixel spectra: the benchmark's field and views with a 256-bin
    synthetic thermal spectrum (inputs.spectral_bins), refined on the 1-10
    band; trees, every node's spectrum, the broadband raster and the images'
    spectra in one call.  Time = median device time per call."""
    log("spectra: 256 bins")
    table, w = inputs.spectral_bins(256)
    scene = air.upload(g, f)
    prm = air.params(N0, LMAX, XI_CRIT)
    ms = []
    out = ctx.render_spectra(scene, views, prm, table, w)
    for _ in range(max(3, args.steps // 3)):
        out = ctx.render_spectra(scene, views, prm, table, w, capacity=out[0][0].n_nodes + 65536)
        ms.append(out[4]["ms_total"])
    torch.cuda.synchronize()
    ms.sort()
    t = ms[len(ms) // 2]
    st = out[4]
    return dict(workload=f"winds2 {NGRID}^3 (rho, T) seed {SEED}, 256 spectral bins, 3 views, {N0}^2 coarse, "
                         f"{LMAX} levels, refined on the 1-10 broadband",
                bins=256, rays=st["rays"], visits=st["visits"], ms_device=t, per_image_ms=t / len(views),
                bin_visits_per_s=256 * st["visits"] / (t * 1e-3), rays_per_s=st["rays"] / (t * 1e-3),
                spectra_bytes=int(st["rays"]) * 256 * 4)


def learned_eval(ctx, air, inputs, np, torch, args, seeds=range(2001, 2009)):
    """The learned proposal on held-out seeds (the network was trained on
    seeds 1..2000): per seed, the two-wind 256^3 field and seeded isotropic
    view of the training set, 64^2 coarse, 5 levels; median device time per
    image of plain AIR, the learned proposal (committed network and cost
    model), speculation to a constant depth 1 or 2, and speculation to the
    true depths (the deepest level of each coarse pixel in the plain tree: the
    best any depth proposal can do).  Every proposal's output is checked equal
    to plain AIR's."""
    log("learned proposal: held-out seeds")
    wpath = os.path.join(ROOT, "paper_1010_5534_amd", "weights", "depth_cnn.npz")
    wz = np.load(wpath)
    net = air.Network(ctx, wz["params"], wz["mean"], wz["scale"])
    c_ray, c_sweep = float(wz["c_ray"]), float(wz["c_sweep"])
    prm = air.params(N0, LMAX, XI_CRIT)
    reps = 5
    tot = dict(plain=0.0, learned=0.0, depth1=0.0, depth2=0.0, true_depth=0.0)
    rays = dict(plain=0, learned=0, depth1=0, depth2=0, true_depth=0)
    missing = dict(learned=0, depth1=0, depth2=0, true_depth=0)
    equal = True
    for seed in seeds:
        src, etas, view = inputs.training_scene(seed)
        rho, temp = inputs.winds_field_torch(src, etas, NGRID, "cuda")
        scene = ctx.prepare(air.scene_from_tensors(NGRID, rho, temp, [[1.0, 1.5, 0.5]]))
        runs = {"plain": lambda: ctx.render(scene, [view], prm, reuse=True),
                "learned": lambda: ctx.render_learned(scene, [view], prm, net, c_ray, c_sweep, reuse=True)}
        ref = ctx.render(scene, [view], prm, reuse=False)
        true = ctx.tree_depth(ref[0][0], N0).to(torch.uint8)[None]
        for name, d in (("depth1", torch.full_like(true, 1)), ("depth2", torch.full_like(true, 2)),
                        ("true_depth", true)):
            runs[name] = (lambda dd: (lambda: ctx.render_proposal(scene, [view], prm, dd, reuse=True)))(d)
        for name, fn in runs.items():
            out, ms = device_median(fn, reps, torch)
            tot[name] += ms
            st = out[3]
            rays[name] += st["rays"] + (out[4]["wasted"] if len(out) > 4 else 0)
            if len(out) > 4:
                missing[name] += out[4]["missing"]
            equal = equal and bool(torch.equal(out[1].view(torch.int32), ref[1].view(torch.int32))
                                   and np.array_equal(out[2], ref[2]))
        del scene, rho, temp
    n = len(seeds)
    net.close()
    return dict(workload=f"winds2 {NGRID}^3 seeds {seeds[0]}..{seeds[-1]} (held out), isotropic views, "
                         f"{N0}^2 coarse, {LMAX} levels, xi_crit {XI_CRIT}",
                per_image_ms={k: v / n for k, v in tot.items()},
                speedup_vs_plain={k: tot["plain"] / v for k, v in tot.items()},
                rays_traced=rays, missing=missing, outputs_equal_to_plain=equal, c_ray=c_ray, c_sweep=c_sweep)


def ring_learned(ctx, air, inputs, np, torch, args):
    """The learned proposal on the section-3 ring family (network trained on
    ring geometries 1..8; geometries 0 = the section's ring, 9 and 10 held
    out): 32x32 coarse, 4 levels, xi_crit 0.2, per held-out render the median
    device time of plain AIR, the learned proposal (committed ring network
    and cost model), speculation to the true depths and to a constant depth
    2.  Renders: the section's face-on view of ring 0, then held-out keys
    41..52 of the training script's ring family (geometry (0, 9, 10)[s mod
    3], view seed 1000000 + s), which were not used to pick the cost model.
    Every proposal's output is checked equal to plain AIR's."""
    log("learned proposal: ring family")
    wz = np.load(os.path.join(ROOT, "paper_1010_5534_amd", "weights", "ring_cnn.npz"))
    net = air.Network(ctx, wz["params"], wz["mean"], wz["scale"])
    c_ray, c_sweep = float(wz["c_ray"]), float(wz["c_sweep"])
    n0, lm, xc = 32, 4, 0.2
    prm = air.params(n0, lm, xc)
    scenes = {}

    def scene(k):
        if k not in scenes:
            g, f = inputs.ring(**inputs.ring_geometry(k))
            scenes[k] = ctx.prepare(air.upload(g, f))
        return scenes[k]

    renders = [(0, inputs.ring_view(), "ring 0 face-on")]
    renders += [((0, 9, 10)[s % 3], inputs.ring_family_view(1000000 + s), f"key {s}") for s in range(41, 53)]
    names = ("plain", "learned", "true_depth", "depth2")
    tot = {k: 0.0 for k in names}
    rays = {k: 0 for k in names}
    rows, equal = [], True
    for k, view, label in renders:
        sc = scene(k)
        ref = ctx.render(sc, [view], prm, reuse=False)
        depth = ctx.tree_depth(ref[0][0], n0).to(torch.uint8)[None]
        runs = {"plain": lambda: ctx.render(sc, [view], prm, reuse=True),
                "learned": lambda: ctx.render_learned(sc, [view], prm, net, c_ray, c_sweep, max_depth=lm, reuse=True),
                "true_depth": lambda: ctx.render_proposal(sc, [view], prm, depth, max_depth=lm, reuse=True),
                "depth2": lambda: ctx.render_proposal(sc, [view], prm, torch.full_like(depth, 2), max_depth=lm,
                                                      reuse=True)}
        row = dict(render=label, geometry=k, rays=ref[3]["rays"])
        for name in names:
            out, ms = device_median(runs[name], 5, torch)
            tot[name] += ms
            rays[name] += out[3]["rays"] + (out[4]["wasted"] if len(out) > 4 else 0)
            row[name + "_ms"] = ms
            equal = equal and bool(np.array_equal(out[2], ref[2])
                                   and torch.equal(out[1].view(torch.int32), ref[1].view(torch.int32))
                                   and out[0][0].n_nodes == ref[0][0].n_nodes
                                   and torch.equal(out[0][0].state, ref[0][0].state)
                                   and torch.equal(out[0][0].I.view(torch.int32), ref[0][0].I.view(torch.int32)))
        rows.append(row)
    net.close()
    n = len(renders)
    return dict(workload="section-3 ring family, 32x32 coarse, 4 levels, xi_crit 0.2; ring 0 face-on and 12 held-out "
                         "renders (geometries 0, 9, 10; network trained on geometries 1-8)",
                per_image_ms={k: v / n for k, v in tot.items()},
                speedup_vs_plain={k: tot["plain"] / v for k, v in tot.items()},
                rays_traced=rays, outputs_equal_to_plain=equal, c_ray=c_ray, c_sweep=c_sweep, renders=rows,
                network="paper_1010_5534_amd/weights/ring_cnn.npz")


def hbm_probe(torch):
    """Measured device-to-device copy bandwidth (read + write bytes per
    second) of a 1 GiB buffer, best of 5, beside the vendor's 8 TB/s."""
    src = torch.empty(256 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    gbs = 2 * src.numel() * 4 / (best * 1e-3) / 1e9
    del src, dst
    return gbs


def batched_amr(ctx, air, inputs, np, torch, args):
    """Block AMR (128^3 base in 16^3 blocks, levels 0-2 over about 10% and 3%
    of the volume), 64 isotropic views x 8 bands, 128x128 coarse, 3 levels,
    in one air_render_batch call."""
    log("batched AMR: 64 views x 8 bands")
    g, f = inputs.amr_winds(seed=0, base_cells=128, bs=16, max_level=2, bands=inputs.default_bands(8))
    scene = ctx.prepare(air.upload(g, f))
    views = inputs.isotropic_views(64, seed=3)
    prm = air.params(128, 3, 0.5)
    for _ in range(2):
        ctx.render_batch(scene, views, prm, want_image=False)
    torch.cuda.synchronize()
    steps = max(2, args.steps // 3)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.render_batch(scene, views, prm, want_image=False)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st = out[3]
    t1 = time.perf_counter()
    ref = ctx.render(scene, views, prm, want_image=False, reuse=True)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t1
    same = bool(np.array_equal(ref[2], out[2]) and ref[3]["rays"] == st["rays"])
    visits = st["visits"]
    return dict(workload="block AMR 128^3 base, 16^3 blocks, levels 0-2 (seed 0), (rho, T) 8 bands, 64 views, "
                         "128x128 coarse, 3 levels, xi_crit 0.5",
                blocks=g.n_blocks, cells=g.n_cells, rays=st["rays"], hits=st["hits"], visits=visits,
                ms_wall=wall * 1e3, per_image_ms=wall * 1e3 / len(views), rays_per_s=st["rays"] / wall,
                band_visits_per_s=8 * visits / wall, ms_wall_eager_render=wall_eager * 1e3,
                equal_to_render=same)


def large_scale(ctx, air, inputs, np, torch, args):
    """Uniform 512^3 (rho, T) field with three wind sources and their pairwise
    shells (seed 0), 4 bands, 16 isotropic views, 128x128 coarse, 6 levels
    (8192^2 effective): plain AIR of all views in one call, trees and flux
    (no raster), and the learned proposal beside it."""
    log("large scale: 512^3, 16 views x 4 bands, 6 levels")
    src, etas = inputs.winds3_sources(0)
    rho, temp = inputs.winds_field_torch(src, etas, 512, "cuda")
    scene = ctx.prepare(air.scene_from_tensors(512, rho, temp, inputs.default_bands(4)))
    views = inputs.isotropic_views(16, seed=5)
    prm = air.params(128, 6, 0.5, band_weight=[1.0, 1.0, 1.0, 1.0])
    out = ctx.render(scene, views, prm, want_image=False, reuse=True)
    torch.cuda.synchronize()
    steps = 3
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.render(scene, views, prm, want_image=False, reuse=True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st = out[3]
    res = dict(workload="winds3 512^3 (rho, T) seed 0, 4 bands, 16 views, 128x128 coarse, 6 levels (8192^2), "
                        "xi_crit 0.5", rays=st["rays"], hits=st["hits"], visits=st["visits"],
               rays_per_level=st["rays_per_level"][:7], ms_wall=wall * 1e3, per_image_ms=wall * 1e3 / 16,
               rays_per_s=st["rays"] / wall, band_visits_per_s=4 * st["visits"] / wall,
               fixed_rays_equivalent=16 * 8192 * 8192)
    wpath = os.path.join(ROOT, "paper_1010_5534_amd", "weights", "depth_cnn.npz")
    if os.path.exists(wpath):
        wz = np.load(wpath)
        net = air.Network(ctx, wz["params"], wz["mean"], wz["scale"])
        c_ray, c_sweep = float(wz["c_ray"]), float(wz["c_sweep"])
        lo = ctx.render_learned(scene, views, prm, net, c_ray, c_sweep, want_image=False, reuse=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lo = ctx.render_learned(scene, views, prm, net, c_ray, c_sweep, want_image=False, reuse=True)
        torch.cuda.synchronize()
        wl = (time.perf_counter() - t0) / steps
        res["learned"] = dict(ms_wall=wl * 1e3, speedup_vs_plain=wall / wl,
                              equal_to_plain=bool(np.array_equal(lo[2], out[2]) and lo[3]["rays"] == st["rays"]),
                              spec_rays=lo[4]["spec_rays"], wasted=lo[4]["wasted"], missing=lo[4]["missing"])
        net.close()
    del scene, rho, temp
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fixed", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
    ap.add_argument("--skip-amr", action="store_true")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--skip-ring", action="store_true")
    ap.add_argument("--skip-spectra", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, one 256 MiB device copy whose counters calibrate HBM bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the adaptive render of one scene runs on one device; "
              "sharding over several GPUs is not built here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1010_5534_amd import air, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("generating winds2 field", NGRID)
    g, f = inputs.winds2(SEED, NGRID, kind=inputs.FIELD_RHO_T, bands=np.array([[1.0, 1.5, 0.5]]))
    views = inputs.winds2_views()
    ctx = air.Context(0)
    scene = ctx.prepare(air.upload(g, f))
    prm = air.params(N0, LMAX, XI_CRIT)
    prm_timed = air.params(N0, LMAX, XI_CRIT, timing=True)
    torch.cuda.synchronize()

    def plain():
        return ctx.render(scene, views, prm, reuse=True)

    def fixed():
        return ctx.render_fixed(scene, views, N0, LMAX)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            out = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev_ms, march_ms, stats = 0.0, 0.0, None
        for _ in range(steps):
            out = fn()
            stats = out[3] if len(out) > 3 else out[-1]
            dev_ms += stats["ms_total"]
            march_ms += stats["ms_march"]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        return out, wall, dev_ms / steps, march_ms / steps, stats

    log("plain AIR")
    out_p, wall_p, dev_p, _, st_p = timed(plain, args.steps, args.warmup)
    trees, img_p, flux_p, _ = out_p
    trees_host = [{k: getattr(t, k).cpu().numpy() for k in ("level", "ix", "iy", "I", "N")} for t in trees]
    img_p = img_p.clone()
    rays_p = st_p["rays"]
    # per-launch march time: a separate pass with an event around every
    # launch (the events lengthen the call, so the throughput above has none)
    _, _, _, march_p, st_t = timed(lambda: ctx.render(scene, views, prm_timed, reuse=True), max(3, args.steps // 3), 1)
    res = dict(metric=METRIC, value=rays_p / wall_p, unit="rays/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=wall_p * 1e3, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=f"winds2 {NGRID}^3 (rho, T) seed {SEED}, {N0}x{N0} coarse, {LMAX} levels "
                                    f"({N0 << LMAX}^2 effective), xi_crit {XI_CRIT}, 3 views (+z, +x, diag)",
                           views=3, coarse=N0, levels=LMAX, grid=NGRID))
    per_level = st_p["rays_per_level"][:LMAX + 1]
    res["plain_air"] = dict(rays=rays_p, rays_per_level=per_level, hits=st_p["hits"], visits=st_p["visits"],
                            leaves=st_p["leaves"], flagged=st_p["flagged"], balance=st_p["balance"],
                            ms_wall=wall_p * 1e3, ms_device=dev_p, ms_march_timed_pass=march_p,
                            ms_test_timed_pass=st_t["ms_test"], per_image_ms=wall_p * 1e3 / len(views),
                            rays_per_s_device=rays_p / (dev_p * 1e-3))
    bytes_p = st_p["visits"] * BYTES_PER_VISIT + rays_p * BYTES_PER_RAY_QUEUE
    achieved = bytes_p / (march_p * 1e-3) / 1e9
    res["roofline"] = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=achieved / HBM_PEAK_GBS, traffic=traffic_from_profile("march_level"),
                           kernel="march of one level: k_march_queue, or k_march_parts + k_fold_parts on the "
                                  "split coarse levels", launches=st_t["march_launches"],
                           avg_launch_ms=march_p / st_t["march_launches"],
                           bytes_per_launch=bytes_p / st_t["march_launches"],
                           bytes_rule=f"{BYTES_PER_VISIT} B/visit + {BYTES_PER_RAY_QUEUE} B/ray")

    if not args.skip_fixed:
        log("fixed-resolution image")
        out_f, wall_f, dev_f, march_f, st_f = timed(fixed, max(2, args.steps // 2), 1)
        img_f, flux_f, _ = out_f
        rays_f = st_f["rays"]
        bytes_f = st_f["visits"] * BYTES_PER_VISIT + rays_f * BYTES_PER_RAY_FIXED
        res["fixed"] = dict(rays=rays_f, hits=st_f["hits"], visits=st_f["visits"], ms_wall=wall_f * 1e3,
                            ms_device=dev_f, ms_march=march_f, per_image_ms=wall_f * 1e3 / len(views),
                            rays_per_s=rays_f / wall_f,
                            march_roofline=dict(achieved=bytes_f / (march_f * 1e-3) / 1e9, unit="GB/s",
                                                frac=bytes_f / (march_f * 1e-3) / 1e9 / HBM_PEAK_GBS))
        # Table-1 style accuracy: AIR flux against the fixed image's flux
        res["air_vs_fixed"] = dict(speedup=wall_f / wall_p, ray_reduction=rays_f / rays_p,
                                   flux_rel_err=[float((flux_f[k][0] - flux_p[k][0]) / flux_f[k][0])
                                                 for k in range(len(views))])
        del out_f, img_f
    log("xi_crit sweep")
    res["xi_sweep"] = xi_sweep(ctx, air, scene, views, None if args.skip_fixed else flux_f, np, torch, args)

    # the same plain AIR through the captured, autotuned launch sequence
    log("plain AIR, captured batch")
    out_b, wall_b, dev_b, _, st_b = timed(lambda: ctx.render_batch(scene, views, prm), args.steps, args.warmup)
    same_b = bool(torch.equal(out_b[1].view(torch.int32), img_p.view(torch.int32)) and np.array_equal(out_b[2], flux_p))
    res["plain_air_batch"] = dict(ms_wall=wall_b * 1e3, ms_device=dev_b, per_image_ms=wall_b * 1e3 / len(views),
                                  rays_per_s=st_b["rays"] / wall_b, equal_to_plain=same_b)
    del out_b

    res["learned_air"] = None
    wpath = os.path.join(ROOT, "paper_1010_5534_amd", "weights", "depth_cnn.npz")
    if os.path.exists(wpath) and not args.skip_learned:
        log("learned AIR")
        wz = np.load(wpath)
        net = air.Network(ctx, wz["params"], wz["mean"], wz["scale"])
        c_ray, c_sweep = float(wz["c_ray"]), float(wz["c_sweep"])

        def learned():
            return ctx.render_learned(scene, views, prm, net, c_ray, c_sweep, reuse=True)

        out_l, wall_l, dev_l, _, st_l = timed(learned, args.steps, args.warmup)
        ls = out_l[4]
        same = bool(torch.equal(out_l[1].view(torch.int32), img_p.view(torch.int32))
                    and np.array_equal(out_l[2], flux_p) and st_l["rays"] == rays_p)
        tl = ctx.render_learned(scene, views, prm_timed, net, c_ray, c_sweep, reuse=True)
        res["learned_air"] = dict(rays=st_l["rays"], ms_wall=wall_l * 1e3, ms_device=dev_l,
                                  per_image_ms=wall_l * 1e3 / len(views), rays_per_s=st_l["rays"] / wall_l,
                                  speedup_vs_plain=wall_p / wall_l, equal_to_plain=same,
                                  spec_rays=ls["spec_rays"], wasted=ls["wasted"], missing=ls["missing"],
                                  depth_hist=ls["depth_hist"], c_ray=c_ray, c_sweep=c_sweep,
                                  ms_features_timed_pass=tl[4]["ms_features"], ms_spec_timed_pass=tl[4]["ms_spec"],
                                  network="paper_1010_5534_amd/weights/depth_cnn.npz (trained on seeds 1..2000; "
                                          "this workload's seed 0 is held out)")
        net.close()

    if not args.skip_ring:
        res["ring"] = ring_experiment(ctx, air, inputs, np, torch, args)
    if not args.skip_spectra:
        res["spectra"] = spectra_run(ctx, air, inputs, np, torch, g, f, views, args)
    if not args.skip_learned:
        res["learned_eval"] = learned_eval(ctx, air, inputs, np, torch, args)
        res["ring_learned"] = ring_learned(ctx, air, inputs, np, torch, args)
    if not args.skip_amr:
        res["batched_amr"] = batched_amr(ctx, air, inputs, np, torch, args)
    if not args.skip_large:
        res["large_scale"] = large_scale(ctx, air, inputs, np, torch, args)

    gbs = hbm_probe(torch)
    res["roofline"]["peak_measured_copy"] = gbs
    res["roofline"]["frac_of_measured_copy"] = achieved / gbs
    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        cb, orc_trees = cpu_baseline(g, f, views)
        res["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "value_1_thread",
                                                  "sample_1_thread", "cpu_model", "host_cpus")}
        res["plain_air"]["vs_oracle"] = oracle_error(trees_host, orc_trees, np)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

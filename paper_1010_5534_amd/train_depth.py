"""Train the depth-proposal network on the GPU with the library's own
kernels, on plain-AIR trees of many seeded renders of one workload family.

Families:
  winds2 -- for each seed, the two-wind field (mass-loss ratio and phase
            drawn from the seed) on a uniform 256^3 grid, one band (kappa0 1,
            T exponents -1.5 and 0.5), a seeded isotropic view, a 64x64
            coarse image with 5 refinement levels at xi_crit 0.5;
  ring   -- the section-3 ring test on its block hierarchy: ring geometries
            1..8 (inputs.ring_geometry) for training, geometries 0 (the
            section's own ring), 9 and 10 held out, each seen from seeded
            views within 70 degrees of face-on; a 32x32 coarse image with 4
            refinement levels at xi_crit 0.2 (the first row of Table 1).
Inputs are the four coarse maps of air_features; labels the deepest level of
each coarse pixel's plain-AIR tree (air_tree_depth).  Training:
class-weighted cross-entropy, Adam, the bf16 MFMA forward and backward
kernels of the library.  Evaluation on held-out renders: label accuracy,
and air_render_learned against air_render (speculative, wasted and missing
rays, device time per image), with the cost ratio of the depth choice
picked on part of the held-out set.

Writes <out>.npz (parameters, feature standardisation, cost model, class
weights) and <out>.json (training log and evaluation)."""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1010_5534_amd import air, inputs  # noqa: E402

GRID = 256
BANDS = [[1.0, 1.5, 0.5]]


def log(*a):
    print(*a, flush=True)


def scene_for(seed, device="cuda"):
    src, etas, view = inputs.training_scene(seed)
    rho, temp = inputs.winds_field_torch(src, etas, GRID, device)
    return air.scene_from_tensors(GRID, rho, temp, BANDS), view


class Winds2:
    """Two-wind fields, one per seed: training seeds 1..n_train, held-out
    seeds after them."""

    name, N0, LMAX, XC = "winds2", 64, 5, 0.5
    workload = f"two-wind {GRID}^3, one band, 64x64 coarse, 5 levels, xi_crit 0.5, isotropic seeded views"

    def __init__(self, n_train, n_val):
        self.train = list(range(1, n_train + 1))
        self.val = list(range(n_train + 1, n_train + n_val + 1))

    def scene(self, ctx, key):
        scene, view = scene_for(key)
        return ctx.prepare(scene), view

    def describe(self, keys):
        return [keys[0], keys[-1]]


class Ring:
    """Section-3 rings: key s of the training set is geometry 1 + (s-1) mod 8
    seen from view seed s; key s of the held-out set is geometry 0, 9 or 10
    (s mod 3) seen from view seed 1000000 + s.  Each geometry's hierarchy is
    built and uploaded once."""

    name, N0, LMAX, XC = "ring", 32, 4, 0.2
    workload = ("section-3 ring family on its block hierarchy (4^3 base blocks of 8^3 cells, 4 levels), "
                "32x32 coarse, 4 levels, xi_crit 0.2, views within 70 degrees of face-on")
    TRAIN_GEOMETRIES, VAL_GEOMETRIES = tuple(range(1, 9)), (0, 9, 10)

    def __init__(self, n_train, n_val):
        self.train = [(1 + (s - 1) % 8, s) for s in range(1, n_train + 1)]
        self.val = [(self.VAL_GEOMETRIES[s % 3], 1000000 + s) for s in range(1, n_val + 1)]
        self.scenes = {}

    def scene(self, ctx, key):
        k, seed = key
        if k not in self.scenes:
            g, f = inputs.ring(**inputs.ring_geometry(k))
            self.scenes[k] = ctx.prepare(air.upload(g, f))
        return self.scenes[k], inputs.ring_family_view(seed)

    def describe(self, keys):
        return dict(geometries=sorted({k for k, _ in keys}), view_seeds=[keys[0][1], keys[-1][1]])


FAMILIES = dict(winds2=Winds2, ring=Ring)


def build_dataset(ctx, fam, keys):
    import torch
    N0 = fam.N0
    prm = air.params(N0, fam.LMAX, fam.XC)
    feats = torch.empty((len(keys), N0, N0, 4), dtype=torch.float32, device="cuda")
    labels = torch.empty((len(keys), N0, N0), dtype=torch.int32, device="cuda")
    t0 = time.time()
    for k, key in enumerate(keys):
        scene, view = fam.scene(ctx, key)
        trees, _, _, _ = ctx.render(scene, [view], prm, want_image=False, want_flux=False, reuse=True)
        labels[k] = ctx.tree_depth(trees[0], N0)
        feats[k] = ctx.features(scene, [view], N0)[0]
        if (k + 1) % 100 == 0:
            torch.cuda.synchronize()
            log(f"  data {k + 1}/{len(keys)} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return feats, labels


def train_epochs(net, ftr, ltr, cw, epochs, batch, lr, rng, first_epoch=0, on_epoch=None, fva=None, lva=None):
    """Adam over shuffled batches, epochs first_epoch .. epochs-1.  rng (a
    numpy Generator) draws each epoch's permutation; on_epoch(epoch, hist)
    runs after every epoch (checkpointing).  Returns the loss history of
    these epochs."""
    import torch
    nb = len(ftr) // batch
    hist = []
    for ep in range(first_epoch, epochs):
        order = torch.as_tensor(rng.permutation(len(ftr)), device="cuda")
        for b in range(nb):
            idx = order[b * batch:(b + 1) * batch]
            net.loss_grad(ftr[idx].contiguous(), ltr[idx].contiguous(), cw, want_loss=False)
            net.adam(lr=lr)
        ltrain, _ = net.loss_grad(ftr[:256].contiguous(), ltr[:256].contiguous(), cw)
        rec = dict(epoch=ep + 1, train_loss=ltrain)
        if fva is not None:
            rec["val_loss"] = net.loss_grad(fva, lva, cw)[0]
        hist.append(rec)
        log(f"epoch {ep + 1}: train {ltrain:.4f}" + (f"  held-out {rec['val_loss']:.4f}" if fva is not None else ""))
        if on_epoch is not None:
            on_epoch(ep + 1, hist)
    return hist


def evaluate_labels(net, feats, labels):
    import torch
    z = net.forward(feats)[..., :6]
    pred = z.argmax(dim=-1).to(torch.int32)
    acc = float((pred == labels).float().mean())
    under = float((pred < labels).float().mean())
    conf = torch.zeros((6, 6), dtype=torch.int64)
    for a in range(6):
        for b in range(6):
            conf[a, b] = int(((labels == a) & (pred == b)).sum())
    return dict(accuracy=acc, under_predicted=under, confusion=conf.tolist())


def time_renders(ctx, net, fam, keys, c_ray, c_sweep, repeats=3):
    """Median device ms per image of plain and learned AIR, and the learned
    counters, over the held-out renders (outputs checked equal)."""
    import torch
    prm = air.params(fam.N0, fam.LMAX, fam.XC)
    plain_ms, learned_ms = [], []
    tot = dict(spec_rays=0, wasted=0, missing=0, rays=0)
    for key in keys:
        scene, view = fam.scene(ctx, key)
        tp, ip, fp, sp = ctx.render(scene, [view], prm, want_tree=False, reuse=True)
        tl, il, fl, sl, ls = ctx.render_learned(scene, [view], prm, net, c_ray, c_sweep, want_tree=False, reuse=True)
        assert np.array_equal(fp, fl), "learned flux differs from plain"
        a, b = [], []
        for _ in range(repeats):
            a.append(ctx.render(scene, [view], prm, want_tree=False, reuse=True)[3]["ms_total"])
            b.append(ctx.render_learned(scene, [view], prm, net, c_ray, c_sweep, want_tree=False,
                                        reuse=True)[3]["ms_total"])
        plain_ms.append(float(np.median(a)))
        learned_ms.append(float(np.median(b)))
        for k in ("spec_rays", "wasted", "missing"):
            tot[k] += ls[k]
        tot["rays"] += sp["rays"]
    torch.cuda.synchronize()
    return dict(plain_ms=float(np.mean(plain_ms)), learned_ms=float(np.mean(learned_ms)),
                speedup=float(np.mean(plain_ms) / np.mean(learned_ms)), **tot)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", choices=sorted(FAMILIES), default="winds2")
    ap.add_argument("--train", type=int, default=2000, help="training renders (seeds 1..N)")
    ap.add_argument("--val", type=int, default=200, help="held-out renders")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "depth_cnn"))
    ap.add_argument("--data-cache", default=None,
                    help=".npz of the training and held-out maps and labels: read if present, else written")
    ap.add_argument("--checkpoint", default=None,
                    help="path prefix: <prefix>.ckpt (network and optimiser) and <prefix>.json (epoch, "
                         "history, shuffling state) written after every epoch")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint if it exists")
    args = ap.parse_args()

    import torch
    assert torch.cuda.is_available(), "training runs on the GPU"
    ctx = air.Context(0)
    fam = FAMILIES[args.family](args.train, args.val)
    t0 = time.time()
    tag = np.array([args.family, str(args.train), str(args.val)])
    if args.data_cache and os.path.exists(args.data_cache):
        log(f"maps and labels from {args.data_cache}")
        z = np.load(args.data_cache)
        assert z["tag"].tolist() == tag.tolist(), "the cache holds another family or other renders"
        ftr, ltr, fva, lva = (torch.from_numpy(z[k]).cuda() for k in ("ftr", "ltr", "fva", "lva"))
    else:
        log(f"building {len(fam.train)} training and {len(fam.val)} held-out {fam.name} maps")
        ftr, ltr = build_dataset(ctx, fam, fam.train)
        fva, lva = build_dataset(ctx, fam, fam.val)
        if args.data_cache:
            np.savez(args.data_cache, ftr=ftr.cpu().numpy(), ltr=ltr.cpu().numpy(), fva=fva.cpu().numpy(),
                     lva=lva.cpu().numpy(), tag=tag)
    t_data = time.time() - t0
    # standardisation and class weights from the training set
    flat = ftr.reshape(-1, 4).double()
    mean = flat.mean(dim=0).float().cpu().numpy()
    scale = flat.std(dim=0).clamp(min=1e-3).float().cpu().numpy()
    freq = torch.bincount(ltr.reshape(-1).long(), minlength=6).double().cpu().numpy()
    freq = freq / freq.sum()
    cw = 1.0 / np.sqrt(np.maximum(freq, 1e-4))
    cw = (cw / np.sum(cw * freq)).astype(np.float32)
    log(f"label frequencies {np.round(freq, 4).tolist()}  class weights {np.round(cw, 3).tolist()}")

    net = air.Network(ctx, inputs.cnn_init(args.init_seed), mean, scale)
    rng = np.random.default_rng(1234)
    hist, first = [], 0
    if args.resume and args.checkpoint and os.path.exists(args.checkpoint + ".json"):
        meta = json.load(open(args.checkpoint + ".json"))
        net.load(args.checkpoint + ".ckpt")
        rng.bit_generator.state = meta["rng"]
        hist, first = meta["history"], meta["epoch"]
        log(f"resumed after epoch {first} from {args.checkpoint}")

    def save(epoch, h):
        if args.checkpoint:
            net.save(args.checkpoint + ".ckpt")
            with open(args.checkpoint + ".json", "w") as fh:
                json.dump(dict(epoch=epoch, history=hist + h, rng=rng.bit_generator.state), fh)

    t1 = time.time()
    hist = hist + train_epochs(net, ftr, ltr, cw, args.epochs, args.batch, args.lr, rng, first, save, fva, lva)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    ev = evaluate_labels(net, fva, lva)
    log(f"held-out accuracy {ev['accuracy']:.4f}, under-predicted {ev['under_predicted']:.4f}")

    # cost ratio of the depth choice: c_ray 1, c_sweep picked on the first 40
    # held-out renders, the rest kept for the final evaluation
    pick, rest_keys = fam.val[:40], fam.val[40:]
    sweep = []
    for cs in (0.0, 20.0, 60.0, 200.0, 600.0, 2000.0, 6000.0, 20000.0, 60000.0, 200000.0):
        r = time_renders(ctx, net, fam, pick, 1.0, cs, repeats=2)
        sweep.append(dict(c_sweep=cs, **r))
        log(f"c_sweep {cs}: plain {r['plain_ms']:.3f} ms learned {r['learned_ms']:.3f} ms "
            f"spec {r['spec_rays']} wasted {r['wasted']} missing {r['missing']}")
    best = min(sweep, key=lambda r: r["learned_ms"])
    c_sweep = best["c_sweep"]
    rest = time_renders(ctx, net, fam, rest_keys, 1.0, c_sweep)
    log(f"held-out ({len(rest_keys)} renders): plain {rest['plain_ms']:.3f} ms, learned "
        f"{rest['learned_ms']:.3f} ms per image, speedup {rest['speedup']:.3f}")
    params, m_, s_ = net.get()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out + ".npz", params=params, mean=m_, scale=s_, c_ray=np.float32(1.0),
             c_sweep=np.float32(c_sweep), class_weight=cw)
    summary = dict(family=fam.name, workload=fam.workload, train=fam.describe(fam.train),
                   held_out=fam.describe(fam.val), epochs=args.epochs, batch=args.batch, lr=args.lr,
                   label_freq=freq.tolist(), class_weight=cw.tolist(), seconds_data=t_data,
                   seconds_train=t_train, history=hist, held_out_labels=ev, cost_sweep=sweep, c_sweep=c_sweep,
                   held_out_render=rest)
    with open(args.out + ".json", "w") as fh:
        json.dump(summary, fh, indent=1)
    log(f"wrote {args.out}.npz and .json")


if __name__ == "__main__":
    main()

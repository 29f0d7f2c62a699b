"""Trains the learned proposal on the GPU with the library's own kernels.

Data: seeded 640x480 scenes (scene seeds 1000 onwards) with a source count drawn
from 4..16 per scene (--n-src), sources listed nearest first as at inference.
For each scene the plain method (random initialisation, 3 iterations with refinement)
produces the labels: at the pixel (4j + 2, 4i + 2) of every 4 x 4 cell its
depth, normal and final cost m; the confidence target is C(m) =
exp(-m^2 / (2 beta^2)) of Eq. 3, which also weights the depth and normal terms,
so cells the plain method did not resolve count little.  The network input is
the library's plane-sweep features of the same scene, and its depth head
corrects the sweep's winning inverse depth.  Training: Adam with a
cosine-decayed learning rate over shuffled mini-batches; forward, loss,
backward and the update all run in the library (amh_nn_*).

    python -m paper_1805_07920_amd.train_proposal --scenes 2000 --out paper_1805_07920_amd/weights/proposal.bin

Prints one line per 100 scenes and per epoch.  Needs a GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1805_07920_amd as amh  # noqa: E402
import scenegen  # noqa: E402

DEFAULT_OUT = os.path.join(HERE, "weights", "proposal.bin")


def log(*a):
    print(*a, flush=True)


def scene_views(ctx, sc):
    ctx.init_views([torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in sc.images], sc.cams)


def nearest_first(sc):
    """Source indices by angular distance from the reference camera: the sweep reads the first few."""
    ang = scenegen.source_angles(len(sc.srcs), sc.meta["arc_deg"])
    return [int(i) + 1 for i in np.argsort(np.abs(ang), kind="stable")]


def make_dataset(ctx, seeds, iters: int = 3, n_src=(8, 8)):
    """n_src: (lo, hi) -- each scene draws its source count uniformly from lo..hi (seeded by the scene)."""
    feats, qrefs, targets = [], [], []
    t0 = time.time()
    for k, seed in enumerate(seeds):
        n = int(np.random.default_rng(seed).integers(n_src[0], n_src[1] + 1))
        sc = scenegen.config_scene("640x480_n8", seed, device="cuda", n_src=n)
        srcs = nearest_first(sc)
        scene_views(ctx, sc)
        ctx.run_checkerboard(0, srcs, iters)
        H, W = sc.height, sc.width
        depth = torch.empty((H, W), device="cuda")
        normal = torch.empty((H, W, 3), device="cuda")
        cost = torch.empty((H, W), device="cuda")
        ctx.get_depth_normal_cost(depth, normal, cost)
        targets.append(ctx.nn_targets(depth, normal, cost))  # Eq. 3 on the device
        f, q = ctx.sweep_features()
        feats.append(f)
        qrefs.append(q)
        if (k + 1) % 100 == 0 or k + 1 == len(seeds):
            torch.cuda.synchronize()
            log(f"data: {k + 1}/{len(seeds)} scenes, {time.time() - t0:.1f} s")
    return torch.stack(feats), torch.stack(qrefs), torch.stack(targets)


def train(ctx, feats, qrefs, targets, epochs: int, batch: int, lr: float, seed: int):
    S = feats.shape[0]
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    history = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(S)).cuda()
        losses = []
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            x = feats.index_select(0, idx).contiguous()
            q = qrefs.index_select(0, idx).contiguous()
            t = targets.index_select(0, idx).contiguous()
            ctx.nn_forward(x, q)
            want = b % 20 == 0
            loss = ctx.nn_backward(t, want_loss=want)
            if want:
                losses.append(loss)
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * step / max(total, 1))))
            ctx.nn_adam_step(lr_t)
            step += 1
        torch.cuda.synchronize()
        history.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.4f}, {time.time() - t0:.1f} s")
    return history


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--scenes", type=int, default=2000)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--n-src", type=int, nargs=2, default=(4, 16), metavar=("LO", "HI"),
                    help="source count per training scene, drawn uniformly from LO..HI")
    ap.add_argument("--sweep-sources", type=int, default=0,
                    help="sources the plane sweep reads (amh_params.sweep_sources; 0: the library's 4)")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--report", default=None, help="JSON file for the loss history")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    torch.cuda.init()
    ctx = amh.Context(seed=args.init_seed, sweep_sources=args.sweep_sources)
    t0 = time.time()
    feats, qrefs, targets = make_dataset(ctx, range(args.seed0, args.seed0 + args.scenes), n_src=tuple(args.n_src))
    t_data = time.time() - t0
    ctx.nn_init(args.init_seed)
    t1 = time.time()
    hist = train(ctx, feats, qrefs, targets, args.epochs, args.batch, args.lr, args.init_seed)
    t_train = time.time() - t1
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    ctx.nn_save(args.out)
    rep = dict(scenes=args.scenes, seed0=args.seed0, n_src=list(args.n_src), sweep_sources=args.sweep_sources or 4,
               epochs=args.epochs, batch=args.batch,
               lr=args.lr,
               loss_per_epoch=hist, data_seconds=t_data, train_seconds=t_train, out=os.path.relpath(args.out, ROOT))
    log(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()

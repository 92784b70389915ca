"""Train the level-policy network on the GPU from measured per-level times.

    python -m paper_2008_05718_amd.train_policy [--out policy_weights.npy] [--report report.json]

Training graphs (seeds >= 100, disjoint from every benchmark input): R-MAT
scales 16-20 and 256^2 - 1024^2 damaged grids with and without shortcuts.
For each graph the batched engine runs 64-source batches in timing
mode (bc_collect_level_times): every forward level is executed with each of
the three variants from the same state, every path-count and backward step
with each of the three summation options, each timed on the device clock.
The samples (each with the three outputs of its own choice measured) train
the 5 -> 32 -> 32 -> 9 network with the library's own HIP kernels
(bc_mlp_train); the weights are written as float32[BC_MLP_PARAMS].
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2008_05718_amd import binding as b  # noqa: E402
from paper_2008_05718_amd import workloads as W  # noqa: E402


def he_init(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    H, I, O = 32, b.BC_MLP_IN, b.BC_MLP_OUT
    parts = [rng.normal(0, np.sqrt(2.0 / I), H * I), np.zeros(H), rng.normal(0, np.sqrt(2.0 / H), H * H),
             np.zeros(H), rng.normal(0, np.sqrt(1.0 / H), O * H), np.full(O, 6.0)]
    return np.concatenate(parts).astype(np.float32)


GROUPS = {"discover": 0, "path_counts": 3, "backward": 6}


def group_report(Y, pred):
    """Per choice group: samples, how often the argmin of the prediction is
    the measured best, and the summed time of the choices (and of each fixed
    choice) over the summed best time."""
    out = {}
    for name, k0 in GROUPS.items():
        rows = np.isfinite(Y[:, k0])
        if not rows.any():
            continue
        y = Y[rows, k0:k0 + 3]
        ch = np.argmin(pred[rows, k0:k0 + 3], axis=1)
        tb = np.exp2(y.min(axis=1)).sum()
        out[name] = {"samples": int(rows.sum()),
                     "argmin_accuracy": float((ch == np.argmin(y, axis=1)).mean()),
                     "time_of_choices_over_best": float(np.exp2(y[np.arange(len(y)), ch]).sum() / tb),
                     "time_of_fixed_choice_over_best": [float(np.exp2(y[:, v]).sum() / tb) for v in range(3)]}
    return out


def training_graphs(quick: bool):
    specs = []
    scales = [16, 17] if quick else [16, 17, 18, 19, 20]
    for i, sc in enumerate(scales):
        specs.append((f"rmat{sc}", lambda sc=sc, i=i: W.rmat(sc, 16, seed=100 + i), 256 if quick else 2048))
    grids = [256] if quick else [256, 512, 1024]
    for j, L in enumerate(grids):
        specs.append((f"grid{L}_sc", lambda L=L, j=j: W.grid(L, 0.10, 0.001, seed=110 + j), 64))
        specs.append((f"grid{L}", lambda L=L, j=j: W.grid(L, 0.10, 0.0, seed=120 + j), 64))
    return specs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "policy_weights.npy"))
    ap.add_argument("--report", default="")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--quick", action="store_true", help="small training set (smoke runs)")
    args = ap.parse_args()

    Xs, Ys, meta = [], [], []
    for name, make, nsrc in training_graphs(args.quick):
        t0 = time.time()
        g = make()
        srcs = W.choose_sources(g, nsrc, seed=7)
        with b.Graph(g) as G:
            X, Y = G.collect_level_times(srcs)
        Xs.append(X)
        Ys.append(Y)
        best = {}
        for gname, k0 in GROUPS.items():
            rows = np.isfinite(Y[:, k0])
            best[gname] = np.bincount(np.argmin(Y[rows, k0:k0 + 3], axis=1), minlength=3).tolist()
        meta.append({"graph": name, "n": g.n, "m": g.m, "sources": int(nsrc), "samples": int(len(X)),
                     "best_choice_counts": best, "seconds": round(time.time() - t0, 1)})
        print(f"[train] {name}: {len(X)} samples, best choice counts {best}", flush=True)
    # every graph weighs about the same in the loss: a deep grid yields
    # thousands of levels, a power-law graph a handful per batch
    top = max(len(x) for x in Xs)
    reps = [int(min(50, max(1, round(top / max(len(x), 1))))) for x in Xs]
    for m, r in zip(meta, reps):
        m["replicated"] = r
    X = np.concatenate([np.repeat(x, r, axis=0) for x, r in zip(Xs, reps)]).astype(np.float32)
    Yr = np.concatenate([np.repeat(y, r, axis=0) for y, r in zip(Ys, reps)]).astype(np.float32)
    M = np.isfinite(Yr).astype(np.uint8)  # each sample measured one choice group
    Y = np.nan_to_num(Yr)
    w0 = he_init(0)
    loss0, _ = b.bc_mlp_loss_grad(w0, X, Y, M)
    w, loss = b.bc_mlp_train(w0, X, Y, M, args.steps, args.lr)
    wp = b.bc_mlp_predict(w, np.concatenate(Xs).astype(np.float32))
    o = 0
    for m, y in zip(meta, Ys):
        m["choices"] = group_report(y, wp[o:o + len(y)])
        o += len(y)
    report = {"samples": int(len(X)), "loss_initial": loss0, "loss_final": loss, "steps": args.steps,
              "lr": args.lr, "choices": group_report(Yr, b.bc_mlp_predict(w, X)), "graphs": meta}
    print(json.dumps(report, indent=1), flush=True)
    np.save(args.out, w)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()

"""Trains the learned free-surface classifier on labels the exact criterion
produces on the solver's own snapshots.

Data: the 3D dam break (660,000 fluid at dx = 0.01; delta-SPH, shifting, TIC,
exact detection) up to t ~ 0.53 s (before the front hits the far wall), a
second, taller dam-break column (0.5 x 0.6 x 0.6 m in a 2.0 x 0.6 x 1.0 m
tank), a 3D sloshing tank, and strongly disordered fluid blocks (lattice
jitter 0.2-0.4 dx: candidates inside the fluid, mostly covered, supply the
interior class), evaluated on the GPU; at every snapshot the particles lambda_min alone cannot
decide (0.2 < lambda <= 0.75) are collected with their 16 features and the
scan-region label.  Split: seeded 80/20 over blocks of consecutive snapshots
(ten snapshots of one trajectory, or one disordered block, per group; 20% of
each source's groups), so that no validation candidate has a neighbour in
time in the training set.
Training: the library's FP32 HIP kernels (forward, backward, Adam),
weighted binary cross-entropy with class weights balancing the two labels.
The fallback margin tau is the smallest |logit| threshold whose confident
predictions misclassify at most `target` of the validation candidates; the
rest goes to the exact test.

Usage: python -m paper_2608_22269_amd.train_classifier [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_OUT = os.path.join(HERE, "data", "fs_classifier.npz")


def log(msg):
    print(f"[train {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def collect(case, nsteps, every, label):
    from paper_2608_22269_amd import Simulation
    from paper_2608_22269_amd.learn import candidate_samples
    import workloads as wl

    sim = Simulation(wl.with_params(case, features=True, fs_mode="exact"))
    X, Y, S = [], [], []
    for k in range(nsteps // every):
        sim.step(every)
        sim.eval_rates()
        f, y = candidate_samples(sim)
        X.append(f)
        Y.append(y)
        S.append(np.full(len(y), k, np.int64))
        st = sim.stats()
        log(f"{label}: t={st['t']:.3f} s, max|U|={st['umax']:.3f}, candidates {len(y)} ({y.mean():.3f} surface)")
    sim.close()
    return np.concatenate(X), np.concatenate(Y), np.concatenate(S)


def collect_disordered(seeds=(11, 12, 13, 14, 15, 16), sigmas=(0.2, 0.3, 0.4)):
    """Candidates of jittered 3D blocks with random velocity (one right-hand
    side each)."""
    from paper_2608_22269_amd import Simulation
    from paper_2608_22269_amd.learn import candidate_samples
    import workloads as wl

    X, Y, S = [], [], []
    for sd in seeds:
        for sg in sigmas:
            c = wl.box3d(0.01, (0.6, 0.4, 0.5), (0.6, 0.4, 0.3), delta_sph=True, pst=True, tic=True,
                         fs_project=True, cont_uncorr=True, features=True, fs_mode="exact")
            c = wl.random_velocity(wl.jitter(c, sg, sd), 0.1, sd + 100)
            c = wl.with_params(c, cell_size=c["params"]["h"])
            sim = Simulation(c)
            sim.eval_rates()
            f, y = candidate_samples(sim)
            sim.close()
            X.append(f)
            Y.append(y)
            S.append(np.full(len(y), len(S), np.int64))
            log(f"disordered block sigma={sg} seed={sd}: candidates {len(y)} ({y.mean():.3f} surface)")
    return np.concatenate(X), np.concatenate(Y), np.concatenate(S)


def initial_params(seed):
    """He-style uniform initialisation (layout W1 b1 W2 b2 W3 b3)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((16, 64), (64, 64), (64, 1)):
        lim = np.sqrt(6.0 / fan_in) * 0.5
        parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(Xtr, ytr, epochs=20, batch=4096, lr=2e-3, seed=0):
    import torch
    from paper_2608_22269_amd.learn import MLPTrainer

    mean = Xtr.mean(0).astype(np.float32)
    std = np.maximum(Xtr.std(0), 1e-6).astype(np.float32)
    pos = ytr.mean()
    w = np.where(ytr > 0.5, 0.5 / max(pos, 1e-6), 0.5 / max(1 - pos, 1e-6)).astype(np.float32)
    tr = MLPTrainer(initial_params(seed), mean, std, max_batch=batch)
    Xd = torch.as_tensor(Xtr, device="cuda")
    yd = torch.as_tensor(ytr, device="cuda")
    wd = torch.as_tensor(w, device="cuda")
    rng = np.random.default_rng(seed + 1)
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(len(ytr)).astype(np.int32), device="cuda")
        lr_ep = lr * (0.5 ** (ep // 10))
        hist.append(tr.train_epoch(Xd, yd, wd, perm, batch, lr_ep))
        log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return tr.params(), mean, std, hist


def choose_margin(logits, y, target):
    """Smallest tau with (errors among |logit| >= tau) / n <= target."""
    wrong = (logits > 0) != (y > 0.5)
    order = np.argsort(np.abs(logits))[::-1]  # most confident first
    a = np.abs(logits)[order]
    cum_wrong = np.cumsum(wrong[order])
    n = len(y)
    ok = np.nonzero(cum_wrong <= target * n)[0]
    if len(ok) == 0:
        return float("inf")
    k = ok[-1]  # keep the k+1 most confident predictions
    return float(a[k])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--dambreak-steps", type=int, default=8000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--target", type=float, default=1e-4,
                    help="misclassification allowed among the validation candidates (sets the margin)")
    args = ap.parse_args()
    import workloads as wl
    from paper_2608_22269_amd.learn import infer_bf16

    t0 = time.time()
    db = wl.dambreak3d(dx=0.01)
    db = wl.with_params(db, cell_size=db["params"]["h"])
    Xa, ya, sa = collect(db, args.dambreak_steps, args.every, "dambreak3d")
    tall = wl.dambreak3d(dx=0.01, tank=(2.0, 0.6, 1.0), column=(0.5, 0.6, 0.6))
    tall = wl.with_params(tall, cell_size=tall["params"]["h"])
    tall_steps = min(args.dambreak_steps, 6000)  # t ~ 0.34 s: the front reaches the far wall
    Xt, yt, st = collect(tall, tall_steps, args.every, "dambreak3d tall column")
    sl = wl.slosh3d(dx=0.004, amp=0.02)
    sl = wl.with_params(sl, cell_size=sl["params"]["h"])
    Xb, yb, sb = collect(sl, 4000, 250, "slosh3d")
    Xc, yc, sc = collect_disordered()
    X = np.concatenate([Xa, Xt, Xb, Xc]).astype(np.float32)
    y = np.concatenate([ya, yt, yb, yc]).astype(np.float32)
    names = ["dambreak3d", "dambreak3d_tall", "slosh3d", "disordered_blocks"]
    src = np.concatenate([np.full(len(v), k) for k, v in enumerate((ya, yt, yb, yc))])
    # groups: blocks of ten consecutive snapshots of a trajectory; each
    # disordered block on its own
    grp = np.concatenate([sa // 10, st // 10, sb // 10, sc]) + 1000 * src
    ugrp = np.unique(grp)
    rng = np.random.default_rng(0)
    # 20% of each source's groups (at least one), so every source is validated
    val_groups = []
    for k in range(len(names)):
        gk = ugrp[ugrp // 1000 == k]
        val_groups.extend(rng.permutation(gk)[: max(1, int(round(0.2 * len(gk))))].tolist())
    val_groups = np.array(val_groups)
    is_val = np.isin(grp, val_groups)
    tr_i, va_i = np.nonzero(~is_val)[0], np.nonzero(is_val)[0]
    ntr = len(tr_i)
    log(f"{len(y)} labelled candidates ({y.mean():.3f} surface) in {len(ugrp)} snapshot groups; "
        f"train {ntr}, validation {len(va_i)} ({len(val_groups)} groups)")
    params, mean, std, hist = train(X[tr_i], y[tr_i], epochs=args.epochs)
    lg = infer_bf16(params, mean, std, X[va_i]).cpu().numpy()
    yv = y[va_i]
    err_raw = float(((lg > 0) != (yv > 0.5)).mean())
    tau = choose_margin(lg, yv, args.target)
    conf = np.abs(lg) >= tau
    err_conf = float((((lg > 0) != (yv > 0.5)) & conf).sum() / len(yv))
    sv = src[va_i]
    per_source = {}
    for k, nm in enumerate(names):
        m = sv == k
        if m.any():
            wrong = ((lg[m] > 0) != (yv[m] > 0.5)) & conf[m]
            per_source[nm] = {"n_val": int(m.sum()), "misclassified": int(wrong.sum()),
                              "rate": float(wrong.mean()), "fallback_fraction": float(1.0 - conf[m].mean())}
    log(f"per source: {per_source}")
    log(f"validation: raw misclassification {err_raw:.4%}; tau {tau:.3f} keeps {conf.mean():.1%} of candidates "
        f"with {err_conf:.4%} errors; {1 - conf.mean():.1%} fall back to the exact test")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out, params=params, mean=mean, std=std, margin=np.float32(tau))
    report = {"n_samples": int(len(y)), "surface_fraction": float(y.mean()), "n_train": int(ntr),
              "n_val": int(len(va_i)), "split": "by blocks of ten consecutive snapshots (seeded 80/20 per source over "
                                                 f"{len(ugrp)} groups, {len(val_groups)} for validation)",
              "loss_history": hist, "val_misclassification_raw": err_raw,
              "margin": tau, "val_confident_fraction": float(conf.mean()),
              "val_misclassification_with_fallback": err_conf, "val_per_source": per_source,
              "seconds": time.time() - t0, "epochs": args.epochs,
              "target": args.target,
              "sources": {"dambreak3d": {"dx": 0.01, "steps": args.dambreak_steps, "every": args.every,
                                         "n": int(len(ya))},
                          "dambreak3d_tall": {"dx": 0.01, "tank": [2.0, 0.6, 1.0], "column": [0.5, 0.6, 0.6],
                                              "steps": tall_steps, "every": args.every, "n": int(len(yt))},
                          "slosh3d": {"dx": 0.004, "amp": 0.02, "steps": 4000, "every": 250, "n": int(len(yb))},
                          "disordered_blocks": {"dx": 0.01, "jitter": [0.2, 0.3, 0.4], "seeds": 6,
                                                "n": int(len(yc))}}}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps({k: v for k, v in report.items() if k != "loss_history"}))


if __name__ == "__main__":
    main()

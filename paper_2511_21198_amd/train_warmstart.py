"""Train the warm-start network on pairs the solver generates itself.

    python -m paper_2511_21198_amd.train_warmstart [--n 255] [--seeds 1-100]
        [--steps 200] [--crops 1] [--crop 48] [--iters 12000] [--out FILE]

Defaults: the configured scale, 20,000 pairs (100 seeds x 200 steps, one
crop each), validation on seeds 101-102.

Data: for each training seed, the learned-warm-start workload (3D
symmetric, orders drawn per seed, moving Gaussian bumps, M steps to T = 1)
is advanced with the float64 PCG solver (tol 1e-10, x0 = u^{m-1}); every step
gives a sample (u^{m-1}, u^{m-2}, F^{m-1/2}, F^{m-3/2}) -> u^m, turned into
network features and the scaled extrapolation-error target by
fsd_nn_features (the first step has no history), from which `--crops` random
boxes of `--crop`^3 voxels are cut (fsd_nn_crop) into slots of one shuffled
buffer, so that every mini-batch is a contiguous slice.  Training: Adam on
the interior mean squared error (margin 4), learning rate with a cosine
decay.  The parameters (float32, the layout of fsd_nn.h) are written as a
.npy file.
"""
from __future__ import annotations

import argparse
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

import workloads  # noqa: E402
from paper_2511_21198_amd import warmstart  # noqa: E402
from paper_2511_21198_amd.solver import Problem  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_3d_sym.npy")
LAYERS = [(ci, co) for ci, co, _ in warmstart.layers()]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source(w, n, m, dt, device):
    """F^{m-1/2}: the moving bumps at t_{m-1/2} (GPU-side input generation)."""
    b = w.bumps
    t = (m - 0.5) * dt
    return workloads.bumps_source_torch([n] * 3, b["c0"] + b["v"] * t, b["width"], device)


def generate(seeds, n, steps, crops, c, rng, device="cuda"):
    total = len(seeds) * steps * crops
    X = torch.empty((total, 5, c, c, c), dtype=torch.float32, device=device)
    T = torch.empty((total, c, c, c), dtype=torch.float32, device=device)
    slots = rng.permutation(total)
    full = warmstart.Net(n, n, n, device=device)
    k = 0
    for seed in seeds:
        w = workloads.config_learned(seed, n=n, M=steps)
        prob = Problem(3, [n] * 3, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="pcg",
                       tol=1e-10, x0="prev")
        eta = prob_eta(prob)
        dt = w.T / w.M
        u = torch.zeros((n, n, n), dtype=torch.float64, device=device)
        un = torch.empty_like(u)
        up = torch.empty_like(u)
        its = []
        Fp = None
        for m in range(1, steps + 1):
            F = source(w, n, m, dt, device)
            un, st = prob.cn_step(u, F, out=un)
            its.append(st["iters"])
            x, t, _ = full.features(u, F, dt, eta, unext=un, u_prev=up if m > 1 else None,
                                    F_prev=Fp)
            for _ in range(crops):
                z0, y0, x0 = (int(v) for v in rng.integers(0, n - c + 1, 3))
                sl = int(slots[k])
                warmstart.crop(x, (z0, y0, x0), (c, c, c), out=X[sl])
                warmstart.crop(t[None], (z0, y0, x0), (c, c, c), out=T[sl:sl + 1].view(1, c, c, c))
                k += 1
            up, u, un = u, un, up
            Fp = F
        log(f"seed {seed}: delta={np.round(w.delta, 3).tolist()} mean PCG iters {np.mean(its):.2f}")
    return X, T


def prob_eta(prob):
    return [prob.coefficients(i)[2] for i in range(3)]


def train(X, T, iters, batch, lr, margin, seed=0, log_every=200):
    n = X.shape[0]
    c = X.shape[-1]
    net = warmstart.Net(c, c, c, batch=batch, training=True, device=X.device)
    p = torch.from_numpy(workloads.nn_initial_params(seed, LAYERS)).to(X.device)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    g = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float64, device=X.device)
    nb = n // batch
    hist = []
    for it in range(1, iters + 1):
        k = (it - 1) % nb
        xb, tb = X[k * batch:(k + 1) * batch], T[k * batch:(k + 1) * batch]
        net.loss_grad(p, xb, tb, margin, grad=g, loss=loss)
        a = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * (it - 1) / iters)))
        warmstart.adam(p, g, m, v, it, a)
        if it % log_every == 0 or it == 1:
            hist.append((it, float(loss.cpu()[0])))
            log(f"iter {it}: loss {hist[-1][1]:.4e}")
    return p, hist


def evaluate(p, X, T, batch, margin):
    """Mean interior loss of the network and of plain linear extrapolation
    (y = 0) over the given crops."""
    c = X.shape[-1]
    net = warmstart.Net(c, c, c, batch=batch, training=True, device=X.device)
    g = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float64, device=X.device)
    ln, l0 = [], []
    sl = slice(margin, c - margin)
    for k in range(X.shape[0] // batch):
        net.loss_grad(p, X[k * batch:(k + 1) * batch], T[k * batch:(k + 1) * batch], margin,
                      grad=g, loss=loss)
        ln.append(float(loss.cpu()[0]))
        tb = T[k * batch:(k + 1) * batch][:, sl, sl, sl]
        l0.append(float((tb.double() ** 2).mean().cpu()))
    return float(np.mean(ln)), float(np.mean(l0))


def parse_seeds(s):
    if "-" in s:
        a, b = s.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in s.split(",")]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=255)
    ap.add_argument("--seeds", default="1-100")
    ap.add_argument("--val-seeds", default="101-102")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--crops", type=int, default=1)
    ap.add_argument("--crop", type=int, default=48)
    ap.add_argument("--iters", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--margin", type=int, default=4)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args(argv)
    rng = np.random.default_rng(2024)
    t0 = time.perf_counter()
    X, T = generate(parse_seeds(a.seeds), a.n, a.steps, a.crops, a.crop, rng)
    Xv, Tv = generate(parse_seeds(a.val_seeds), a.n, a.steps, 1, a.crop, rng)
    t1 = time.perf_counter()
    log(f"data: {X.shape[0]} training crops, {Xv.shape[0]} validation crops, {t1 - t0:.1f} s")
    p, hist = train(X, T, a.iters, a.batch, a.lr, a.margin)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lv, l0 = evaluate(p, Xv, Tv, a.batch, a.margin)
    log(f"training {t2 - t1:.1f} s; validation loss {lv:.4e} vs {l0:.4e} for extrapolation")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.save(a.out, p.cpu().numpy())
    print({"out": a.out, "train_crops": int(X.shape[0]), "val_loss": lv, "val_loss_extrap": l0,
           "data_s": round(t1 - t0, 1), "train_s": round(t2 - t1, 1), "hist": hist})


if __name__ == "__main__":
    main()

"""Data generation, training and evaluation of the learned coarse-grained
surrogate of spinodal decomposition (host orchestration only: the lattice
steps, coarse-graining, network passes, optimiser and S(k, t) measurement all
run in libfsc.so; PyTorch provides device memory).

Workload: D2Q9, E8 stencil, FP32-shifted populations, n0 = 1 at T_hat = 0.7
(deep quench into the unstable region), kBT = 1e-4, lattice side n (1024 by
default), coarse-grained by 8 x 8 block means; the surrogate maps the coarse
density at time t to the one at t + stride (256 by default).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import _lib as F

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "surrogate_model.npz")

QUENCH = dict(D=2, stencil=8, precision="fp32", T_hat=0.7, rho0=1.0, kBT=1e-4)


def run_quench(torch, seeds, n=1024, factor=8, stride=256, n_snap=80, seed_base=0):
    """Runs one replica per seed (one ensemble, one launch per step) and
    returns the coarse densities at t = 0, stride, ..., n_snap * stride as a
    device tensor [n_snap + 1][len(seeds)][n/factor][n/factor], plus the LBM
    wall time in seconds (steps only)."""
    plist = [F.make_params(nx=n, ny=n, seed=seed_base + s, replica=s, **QUENCH) for s in seeds]
    stream = torch.cuda.Stream()
    ens = F.Ensemble(plist, stream=stream)
    ens.init_uniform()
    m = n // factor
    out = torch.zeros((n_snap + 1, len(seeds), m, m), dtype=torch.float32, device="cuda")
    for r in range(len(seeds)):
        ens.coarsen(r, factor, out[0, r])
    t_lbm = 0.0
    for k in range(1, n_snap + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.run(stride, 0)
        torch.cuda.synchronize()
        t_lbm += time.perf_counter() - t0
        for r in range(len(seeds)):
            ens.coarsen(r, factor, out[k, r])
    torch.cuda.synchronize()
    for r in range(len(seeds)):
        st = ens.stats(r)
        if st["bad"]:
            raise RuntimeError(f"replica {r} diverged")
    ens.close()
    return out, t_lbm


def train(torch, snaps, t_first, layers=5, steps=3000, batch=32, lr=1e-3, seed=0, log=None):
    """Trains on consecutive snapshot pairs (snaps[k], snaps[k+1]) for k >= t_first."""
    K, R, m, _ = snaps.shape
    x = snaps[t_first:K - 1].reshape(-1, m, m)
    y = snaps[t_first + 1:K].reshape(-1, m, m)
    mean = 1.0
    in_scale = float((x - mean).std().item())
    out_scale = float((y - x).std().item())
    sur = F.Surrogate(layers, m, m, batch, seed=seed)
    sur.set_norm(mean, in_scale, out_scale)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    npairs = x.shape[0]
    losses = []
    xb = torch.empty((batch, m, m), dtype=torch.float32, device="cuda")
    yb = torch.empty_like(xb)
    for it in range(steps):
        idx = torch.randint(0, npairs, (batch,), device="cuda", generator=g)
        # random periodic shifts and the square's symmetries keep the physics
        sh = torch.randint(0, m, (2,), generator=None).tolist()
        xs = torch.roll(x[idx], shifts=sh, dims=(1, 2))
        ys = torch.roll(y[idx], shifts=sh, dims=(1, 2))
        if it % 2:
            xs, ys = xs.transpose(1, 2), ys.transpose(1, 2)
        xb.copy_(xs)
        yb.copy_(ys)
        rate = lr * 0.5 * (1 + math.cos(math.pi * it / steps))
        loss = sur.train_step(xb, yb, batch, max(rate, 1e-5), want_loss=(it % 50 == 0))
        if loss is not None:
            losses.append((it, loss))
            if log:
                log(f"step {it} loss {loss:.4e}")
    return sur, dict(mean=mean, in_scale=in_scale, out_scale=out_scale, losses=losses,
                     npairs=int(npairs))


def rollout(torch, sur, start, n_out, batch):
    """Applies the surrogate n_out times from `start` [batch][m][m]; returns
    [n_out + 1][batch][m][m] and the wall time of the passes."""
    m = start.shape[-1]
    traj = torch.zeros((n_out + 1, batch, m, m), dtype=torch.float32, device="cuda")
    traj[0].copy_(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_out):
        sur.forward(traj[k], traj[k + 1], batch)
    torch.cuda.synchronize()
    return traj, time.perf_counter() - t0


def sk_error(torch, a, b, m, kmax_shell):
    """Relative S(k) error sum_b |S_a - S_b| / sum_b S_b over shells 1..kmax
    of the ensemble means of two stacks of fields [batch][m][m]."""
    sa, La = F.field_sk(a.contiguous(), a.shape[0], m)
    sb, Lb = F.field_sk(b.contiguous(), b.shape[0], m)
    A = sa.mean(axis=0)[1:kmax_shell + 1]
    B = sb.mean(axis=0)[1:kmax_shell + 1]
    return float(np.abs(A - B).sum() / B.sum()), float(La.mean()), float(Lb.mean())


def evaluate(torch, sur, seeds, n=1024, factor=8, stride=256, t0_snap=8, n_out=24,
             seed_base=1000):
    """Held-out seeds: LBM reference trajectory vs surrogate rollout from the
    LBM state at snapshot t0_snap.  S(k, t) error over k <= pi/8 (lattice
    units) and L(t), per rollout time; speedup = LBM time / surrogate time
    for the same horizon on the same GPU."""
    snaps, t_lbm = run_quench(torch, seeds, n=n, factor=factor, stride=stride,
                              n_snap=t0_snap + n_out, seed_base=seed_base)
    m = n // factor
    traj, t_sur = rollout(torch, sur, snaps[t0_snap], n_out, len(seeds))
    # shells of the coarse grid: k = 2 pi b / n in lattice units; k <= pi/8 -> b <= n/16
    kmax = n // 16
    rows = []
    for k in range(1, n_out + 1):
        err, L_sur, L_lbm = sk_error(torch, traj[k], snaps[t0_snap + k], m, kmax)
        rows.append(dict(t=(t0_snap + k) * stride, sk_rel_err=err, L_surrogate=L_sur * factor,
                         L_lbm=L_lbm * factor))
    horizon_lbm = t_lbm * n_out / (t0_snap + n_out)  # LBM time for the same n_out strides
    return dict(rows=rows, max_sk_rel_err=max(r["sk_rel_err"] for r in rows),
                lbm_seconds=horizon_lbm, surrogate_seconds=t_sur,
                speedup=horizon_lbm / t_sur, seeds=list(seeds), n=n, stride=stride,
                t0=t0_snap * stride)


def save_model(sur, meta, path=MODEL_PATH):
    np.savez(path, params=sur.get_params(), layers=sur.layers, H=sur.H, W=sur.W,
             meta=json.dumps(meta))


def load_model(path=MODEL_PATH, max_batch=16):
    d = np.load(path, allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    sur = F.Surrogate(int(d["layers"]), int(d["H"]), int(d["W"]), max_batch)
    sur.set_params(d["params"])
    sur.set_norm(meta["mean"], meta["in_scale"], meta["out_scale"])
    return sur, meta


def main(argv=None):
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="train and evaluate the coarse-grained surrogate")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--train-seeds", type=int, default=32)
    ap.add_argument("--eval-seeds", type=int, default=8)
    ap.add_argument("--snaps", type=int, default=80)
    ap.add_argument("--t-first", type=int, default=4)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "surrogate_eval.json"))
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    snaps, t_lbm = run_quench(torch, range(a.train_seeds), n=a.n, n_snap=a.snaps)
    print(f"data: {a.train_seeds} seeds x {a.snaps} snapshots in {t_lbm:.1f} s of lattice time",
          flush=True)
    sur, meta = train(torch, snaps, a.t_first, steps=a.steps, log=lambda s: print(s, flush=True))
    del snaps
    ev = evaluate(torch, sur, range(a.eval_seeds), n=a.n)
    meta.update(dict(train_seeds=a.train_seeds, snaps=a.snaps, t_first=a.t_first, n=a.n,
                     eval=ev, wall_seconds=time.perf_counter() - t0))
    save_model(sur, meta)
    with open(a.out, "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps({k: ev[k] for k in ("max_sk_rel_err", "speedup", "lbm_seconds",
                                         "surrogate_seconds")}), flush=True)


if __name__ == "__main__":
    main()

"""Data generation, training and evaluation of the learned coarse-grained
surrogate of spinodal decomposition (host orchestration only: the lattice
steps, coarse-graining, network passes, optimiser and S(k, t) measurement all
run in libfsc.so; PyTorch provides device memory).

Workload: D2Q9, E8 stencil, FP32-shifted populations, n0 = 1 at T_hat = 0.7
(deep quench into the unstable region), kBT = 1e-4, lattice side n (1024 by
default), coarse-grained by 8 x 8 block means; the surrogate maps the coarse
densities at t - stride and t to the one at t + stride (stride 256 lattice
steps).  The plain lattice stays the reference: evaluation rolls the network
out from lattice states of held-out seeds and compares S(k, t) and L(t) with
the lattice's own, stride by stride.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import _lib as F

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "surrogate_model.npz")  # 9 layers, two input channels
# the network the workload names: 5 layers (1 -> 32 -> 32 -> 32 -> 32 -> 1)
MODEL_5X1_PATH = os.path.join(HERE, "surrogate_model_5layer_1ch.npz")

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
    ens.autotune()  # outside the timed strides
    m = n // factor
    out = torch.zeros((n_snap + 1, len(seeds), m, m), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()  # the lattice writes on its own stream
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


def _draw_batch(rng, K, R, t_first, batch, m, ahead):
    """Random batch indices (snapshot t, run r), a common periodic shift and
    the transpose flag: the lattice's symmetries augment the data."""
    t = rng.integers(t_first, K - ahead, size=batch)
    r = rng.integers(0, R, size=batch)
    shift = (int(rng.integers(0, m)), int(rng.integers(0, m)))
    return t, r, shift


def train(torch, snaps, t_first, layers=7, in_ch=2, steps=6000, batch=32, lr=1e-3, push=0.5,
          push_depth=1, seed=0, log=None):
    """Trains on snapshot pairs (k, k+1), k >= t_first, with the previous
    snapshot as second input channel (in_ch = 2).  After the first tenth of the
    steps, a fraction `push` of every batch starts from the network's own
    rollout of d = 1..push_depth strides (no gradient through it; the pushed
    rows are split evenly over d) and is trained against the snapshot d + 1
    strides ahead: the network learns to correct the errors its rollouts
    make.  Batches are gathered by the library (fsc_sur_gather) with random
    periodic shifts and, every other step, a transpose; the input and output
    scales come from the library's FP64 moments of the stack."""
    K, R, m, _ = snaps.shape
    mean = 1.0
    in_scale, out_scale = F.stack_scales(snaps[t_first:], 0, centre=mean)
    sur = F.Surrogate(layers, m, m, batch, seed=seed, in_ch=in_ch)
    sur.set_norm(mean, in_scale, out_scale)
    rng = np.random.default_rng(seed)
    bufs = [torch.empty((batch, m, m), dtype=torch.float32, device="cuda") for _ in range(4)]
    prev_b, cur_b, tgt_b, pred_b = bufs
    nxt_b = [torch.empty((batch, m, m), dtype=torch.float32, device="cuda")
             for _ in range(push_depth + 1)]
    losses = []
    n_push = int(round(push * batch))
    # rows [edges[d-1], edges[d]) of the batch are pushed d strides
    edges = [round(n_push * d / push_depth) for d in range(push_depth + 1)]
    for it in range(steps):
        t, r, shift = _draw_batch(rng, K, R, t_first, batch, m, push_depth + 1)
        tr = bool(it % 2)
        sur.gather(snaps, t, r, -1, shift, tr, prev_b)
        sur.gather(snaps, t, r, 0, shift, tr, cur_b)
        for d in range(push_depth + 1):
            sur.gather(snaps, t, r, d + 1, shift, tr, nxt_b[d])
        tgt_b.copy_(nxt_b[0])
        if n_push and it >= steps // 10:
            for d in range(1, push_depth + 1):
                a, b = edges[d - 1], edges[d]
                if b <= a:
                    continue
                for _ in range(d):  # roll rows a..b-1 out d strides
                    sur.forward(prev_b[a:b], cur_b[a:b], pred_b[a:b], b - a)
                    prev_b[a:b].copy_(cur_b[a:b])
                    cur_b[a:b].copy_(pred_b[a:b])
                tgt_b[a:b].copy_(nxt_b[d][a:b])
        rate = lr * 0.5 * (1 + math.cos(math.pi * it / steps))
        loss = sur.train_step(prev_b, cur_b, tgt_b, batch, max(rate, 1e-5),
                              want_loss=(it % 100 == 0))
        if loss is not None:
            losses.append((it, loss))
            if log:
                log(f"step {it} loss {loss:.4e}")
    return sur, dict(mean=mean, in_scale=in_scale, out_scale=out_scale, losses=losses,
                     layers=layers, in_ch=in_ch, steps=steps, batch=batch, lr=lr, push=push,
                     push_depth=push_depth,
                     pairs=int((K - 2 - t_first) * R))


def rollout(torch, sur, prev, start, n_out, batch, reps=3):
    """Applies the surrogate n_out times from (prev, start) [batch][m][m]
    (one captured graph of the n_out passes, fsc_sur_rollout); returns
    [n_out + 1][batch][m][m] and the wall time of the passes (the fastest of
    `reps` replays after a first one that captures the graph)."""
    m = start.shape[-1]
    traj = torch.zeros((n_out + 1, batch, m, m), dtype=torch.float32, device="cuda")
    traj[0].copy_(start)
    prev = prev.contiguous()
    sur.rollout(prev, traj, batch, n_out)  # capture
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sur.rollout(prev, traj, batch, n_out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return traj, best


def sk_error(torch, a, b, m, kmax_shell):
    """Relative S(k) error sum_b |S_a - S_b| / sum_b S_b over shells 1..kmax
    of the ensemble means of two stacks of fields [batch][m][m]."""
    sa, La = F.field_sk(a.contiguous(), a.shape[0], m)
    sb, Lb = F.field_sk(b.contiguous(), b.shape[0], m)
    A = sa.mean(axis=0)[1:kmax_shell + 1]
    B = sb.mean(axis=0)[1:kmax_shell + 1]
    return float(np.abs(A - B).sum() / B.sum()), float(La.mean()), float(Lb.mean())


def horizon(rows, tol=0.05, key="sk_rel_err"):
    """Strides before the S(k) error first exceeds tol."""
    for k, r in enumerate(rows):
        if r[key] > tol:
            return k
    return len(rows)


def evaluate(torch, sur, seeds, n=1024, factor=8, stride=256, t0_snaps=(4, 8, 16), n_out=24,
             seed_base=1000, snaps=None, t_lbm=None):
    """Held-out seeds: the lattice's trajectory against the surrogate's
    rollouts started from the lattice state at each snapshot in t0_snaps.
    Per rollout stride: relative S(k) error over k <= pi/8 (lattice units) and
    L(t) of both.  The persistence forecast (the start field held fixed) is
    the method without the surrogate's learned dynamics.  Speedup = lattice
    wall time / surrogate wall time for the same strides on the same GPU."""
    n_snap = max(t0_snaps) + n_out
    if snaps is None:
        snaps, t_lbm = run_quench(torch, seeds, n=n, factor=factor, stride=stride, n_snap=n_snap,
                                  seed_base=seed_base)
    m = n // factor
    kmax = n // 16  # coarse shells: k = 2 pi b / n; k <= pi/8 -> b <= n/16
    starts = []
    for t0 in t0_snaps:
        traj, t_sur = rollout(torch, sur, snaps[t0 - 1], snaps[t0], n_out, len(seeds))
        rows = []
        for k in range(1, n_out + 1):
            err, L_sur, L_lbm = sk_error(torch, traj[k], snaps[t0 + k], m, kmax)
            pers, _, _ = sk_error(torch, snaps[t0], snaps[t0 + k], m, kmax)
            rows.append(dict(t=(t0 + k) * stride, sk_rel_err=err, persistence_err=pers,
                             L_surrogate=L_sur * factor, L_lbm=L_lbm * factor))
        per = t_lbm / n_snap  # lattice seconds per stride
        lbm_s = per * n_out  # lattice time for the same n_out strides
        h = horizon(rows)
        # reaching t0 + h strides: the lattice alone, against the lattice to t0
        # (the warm-up the rollout starts from) plus h surrogate strides
        with_warm = (t0 + h) * per / (t0 * per + t_sur * h / n_out) if h else None
        starts.append(dict(t0=t0 * stride, rows=rows, horizon_5pct=h,
                           persistence_horizon_5pct=horizon(rows, key="persistence_err"),
                           lbm_seconds=lbm_s, surrogate_seconds=t_sur, speedup=lbm_s / t_sur,
                           speedup_with_warmup=with_warm, warmup_lattice_seconds=t0 * per))
    return dict(starts=starts, seeds=list(seeds), n=n, stride=stride, n_out=n_out)


def save_model(sur, meta, path=MODEL_PATH):
    np.savez(path, params=sur.get_params(), layers=sur.layers, in_ch=sur.in_ch, H=sur.H, W=sur.W,
             meta=json.dumps(meta))


def load_model(path=MODEL_PATH, max_batch=16):
    d = np.load(path, allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    sur = F.Surrogate(int(d["layers"]), int(d["H"]), int(d["W"]), max_batch, in_ch=int(d["in_ch"]))
    sur.set_params(d["params"])
    sur.set_norm(meta["mean"], meta["in_scale"], meta["out_scale"])
    return sur, meta


def summary(ev):
    """Headline numbers of an evaluation: the horizon (strides within 5% S(k)
    error) and speedup of each rollout start."""
    return [dict(t0=s["t0"], horizon_5pct=s["horizon_5pct"],
                 persistence_horizon_5pct=s["persistence_horizon_5pct"],
                 err_first=round(s["rows"][0]["sk_rel_err"], 4),
                 err_last=round(s["rows"][-1]["sk_rel_err"], 4),
                 speedup=round(s["speedup"], 1)) for s in ev["starts"]]


def main(argv=None):
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="train and evaluate the coarse-grained surrogate")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--train-seeds", type=int, default=200)
    ap.add_argument("--eval-seeds", type=int, default=16)
    ap.add_argument("--snaps", type=int, default=40)
    ap.add_argument("--t-first", type=int, default=4)
    ap.add_argument("--steps", type=int, default=12000)
    ap.add_argument("--models", nargs="+", default=["9:2", "5:1"],
                    help="networks to train, as layers:input_channels")
    ap.add_argument("--push-depth", type=int, default=2)
    ap.add_argument("--save", action="store_true",
                    help="store 9:2 as the package model and 5:1 as the five-layer model")
    ap.add_argument("--save-dir", default=None,
                    help="with --save: directory for the model files (default: the package)")
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "surrogate_eval.json"))
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    snaps, t_lbm = run_quench(torch, range(a.train_seeds), n=a.n, n_snap=a.snaps)
    print(f"data: {a.train_seeds} seeds x {a.snaps} snapshots, {t_lbm:.1f} s of lattice steps",
          flush=True)
    ev_snaps, ev_t = run_quench(torch, range(a.eval_seeds), n=a.n, n_snap=40, seed_base=1000)
    results = []
    for spec in a.models:
        layers, in_ch = (int(v) for v in spec.split(":"))
        t1 = time.perf_counter()
        sur, meta = train(torch, snaps, a.t_first, layers=layers, in_ch=in_ch, steps=a.steps,
                          push_depth=a.push_depth, log=lambda s: print(s, flush=True))
        meta["train_seconds"] = time.perf_counter() - t1
        ev = evaluate(torch, sur, range(a.eval_seeds), n=a.n, snaps=ev_snaps, t_lbm=ev_t)
        meta.update(dict(train_seeds=a.train_seeds, snaps=a.snaps, t_first=a.t_first, n=a.n,
                         eval=ev, summary=summary(ev)))
        print(json.dumps(dict(layers=layers, in_ch=in_ch, summary=meta["summary"])), flush=True)
        dest = {"9:2": MODEL_PATH, "5:1": MODEL_5X1_PATH}.get(spec)
        if a.save and dest:
            if a.save_dir:
                os.makedirs(a.save_dir, exist_ok=True)
                dest = os.path.join(a.save_dir, os.path.basename(dest))
            save_model(sur, meta, dest)
        results.append(meta)
        sur.close()
    with open(a.out, "w") as fh:
        json.dump(dict(models=results, wall_seconds=time.perf_counter() - t0), fh, indent=1)


if __name__ == "__main__":
    main()

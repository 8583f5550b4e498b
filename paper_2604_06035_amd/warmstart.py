"""Train and evaluate the learned warm start on the GPU.

Training fields: lognormal densities on a periodic n^3 grid whose spectral
slope ~ U[-3, -2] and variance ~ U[0.5, 2] are drawn from each seed's
generator (seeds 10000, 10001, ...).  Targets are the library's own FP64
multigrid solutions (relative residual 1e-12).  Each field is used for one
training step (forward, loss, backward, Adam) with a cosine learning-rate
schedule.  Evaluation on held-out seeds (20000, ...) compares the V-cycles and
wall time to relative residual 1e-10 of the plain solve from zero with the
warm-started solve (network + residual check + solve, automatic fallback to
zero when the guess is no better than zero).

    python -m paper_2604_06035_amd.warmstart train --n 256 --fields 2000 --out W.npy
    python -m paper_2604_06035_amd.warmstart eval --n 256 --seeds 200 --weights W.npy

The loss is the relative MSE to the multigrid target plus res_weight (default
10) times the mean squared residual of the guess; the committed weights
(weights/warmstart_c24_l5.npy) come from the train command above with these
defaults and seed 0.

Field generation runs in a pool of CPU worker processes created before the
GPU is touched; the workers only run NumPy.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_SEED0 = 10000
EVAL_SEED0 = 20000
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_c24_l5.npy")


def make_field(args):
    """(seed, n, f32) -> oct-major density of one seeded lognormal field."""
    seed, n, as_f32 = args
    from workloads import cnn_field_params, dense_to_oct, lognormal_density
    slope, var, rng = cnn_field_params(seed)
    rho = lognormal_density(n, slope=slope, var=var, rng=rng)
    o = dense_to_oct(rho)
    return o.astype(np.float32) if as_f32 else o


def _pool(workers: int):
    return mp.get_context("fork").Pool(workers)


def train(n: int, fields: int, out: str, lr0: float = 1e-3, lr1: float = 1e-5, res_weight: float = 10.0,
          seed: int = 0, workers: int = 16, log_every: int = 50, init: str | None = None) -> dict:
    pool = _pool(workers)           # before any GPU call
    import torch

    from . import abi
    dev = torch.device("cuda:0")
    L = abi.mg_build_level(n)
    net = abi.mgnn_create(24, 5, seed)
    if init:
        abi.mgnn_set_weights(net, np.load(init))
    losses = []
    t0 = time.perf_counter()
    try:
        rho = torch.empty((n // 2) ** 3 * 8, dtype=torch.float64, device=dev)
        phi = torch.zeros_like(rho)
        jobs = ((TRAIN_SEED0 + i, n, True) for i in range(fields))
        for i, r32 in enumerate(pool.imap(make_field, jobs, chunksize=1)):
            rho.copy_(torch.from_numpy(r32.reshape(-1)))
            phi.zero_()
            st, info = abi.mg_solve(L, rho, None, 1.0, None, phi, 1e-12, 80)
            if st != abi.MG_OK:
                raise RuntimeError(f"target solve failed for field {i}: {info}")
            lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * i / max(fields - 1, 1)))
            losses.append(abi.mgnn_train_step(net, n, rho, None, 1.0, phi, lr, res_weight))
            if (i + 1) % log_every == 0 or i + 1 == fields:
                print(f"train step {i + 1}/{fields} loss {np.mean(losses[-log_every:]):.5e} lr {lr:.2e} "
                      f"elapsed {time.perf_counter() - t0:.1f}s", flush=True)
        w = abi.mgnn_get_weights(net)
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        np.save(out, w)
    finally:
        abi.mgnn_destroy(net)
        abi.mg_destroy_level(L)
        pool.close()
    return {"fields": fields, "n": n, "first_loss": float(np.mean(losses[:log_every])),
            "last_loss": float(np.mean(losses[-log_every:])), "seconds": time.perf_counter() - t0,
            "res_weight": res_weight, "weights": out}


def evaluate(n: int, seeds: int, weights: str, workers: int = 16, tol: float = 1e-10) -> dict:
    pool = _pool(workers)
    import torch

    from . import abi
    dev = torch.device("cuda:0")
    L = abi.mg_build_level(n)
    net = abi.mgnn_create(24, 5, 0)
    abi.mgnn_set_weights(net, np.load(weights))
    rows = []
    try:
        rho = torch.empty((n // 2) ** 3 * 8, dtype=torch.float64, device=dev)
        phi = torch.zeros_like(rho)
        jobs = ((EVAL_SEED0 + i, n, False) for i in range(seeds))
        for i, r64 in enumerate(pool.imap(make_field, jobs, chunksize=1)):
            rho.copy_(torch.from_numpy(r64.reshape(-1)))
            if i == 0:   # warm up both paths once
                phi.zero_()
                abi.mg_solve(L, rho, None, 1.0, None, phi, tol, 80)
                abi.mgnn_solve_warm(net, L, rho, None, 1.0, phi, tol, 80)
            phi.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st0, i0 = abi.mg_solve(L, rho, None, 1.0, None, phi, tol, 80)
            torch.cuda.synchronize()
            ms0 = (time.perf_counter() - t) * 1e3
            t = time.perf_counter()
            st1, i1 = abi.mgnn_solve_warm(net, L, rho, None, 1.0, phi, tol, 80)
            torch.cuda.synchronize()
            ms1 = (time.perf_counter() - t) * 1e3
            if st0 != abi.MG_OK or st1 != abi.MG_OK:
                raise RuntimeError(f"seed {EVAL_SEED0 + i}: solve failed {i0} {i1}")
            rows.append((i0["cycles"], ms0, i1["cycles"], ms1, i1["used_fallback"], i1["relres0"], i1["relres"]))
            if (i + 1) % 25 == 0:
                print(f"eval {i + 1}/{seeds}", flush=True)
    finally:
        abi.mgnn_destroy(net)
        abi.mg_destroy_level(L)
        pool.close()
    a = np.array(rows, dtype=np.float64)

    def stats(col):
        return {"median": float(np.median(a[:, col])), "p10": float(np.percentile(a[:, col], 10)),
                "p90": float(np.percentile(a[:, col], 90))}

    saved = a[:, 0] - a[:, 2]
    return {"n": n, "seeds": seeds, "tol": tol, "weights": os.path.relpath(weights, ROOT),
            "zero_guess": {"cycles": stats(0), "ms": stats(1)},
            "warm_start": {"cycles": stats(2), "ms": stats(3), "relres0": stats(5),
                           "fallbacks": int(a[:, 4].sum()), "max_final_relres": float(a[:, 6].max())},
            # per seed: zero-guess cycles minus warm-started cycles
            "cycles_saved_median": float(np.median(saved)), "cycles_saved_mean": float(saved.mean()),
            "cycles_saved_counts": {str(int(k)): int((saved == k).sum()) for k in np.unique(saved)},
            "time_ratio_median": float(np.median(a[:, 3] / a[:, 1]))}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n", type=int, default=256)
    t.add_argument("--fields", type=int, default=2000)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--lr0", type=float, default=1e-3)
    t.add_argument("--lr1", type=float, default=1e-5)
    t.add_argument("--res-weight", type=float, default=10.0)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--workers", type=int, default=16)
    t.add_argument("--init", default=None)
    e = sub.add_parser("eval")
    e.add_argument("--n", type=int, default=256)
    e.add_argument("--seeds", type=int, default=200)
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--workers", type=int, default=16)
    args = ap.parse_args(argv)
    if args.cmd == "train":
        res = train(args.n, args.fields, args.out, args.lr0, args.lr1, args.res_weight, args.seed, args.workers,
                    init=args.init)
    else:
        res = evaluate(args.n, args.seeds, args.weights, args.workers)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

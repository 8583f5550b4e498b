#!/usr/bin/env python
"""Benchmark: multigrid Poisson solve to relative residual 1e-10 on one MI355X.

Workload (one "step" = one full solve from a zero guess, inputs resident in
HBM): periodic 512^3 grid (134M cells, the largest single-GPU configuration
and the size the smoother's bandwidth target is stated for), lognormal density
rho = exp(g - var/2) from a Gaussian random field with P(k) ~ k^-2.5 and
variance 1.5 (seed 2), 4 pi G = 1, FP64 multigrid V(2,2) cycles (red-black
Gauss-Seidel) down to 4^3, stopping at ||f - L phi||_2 / ||f||_2 <= 1e-10.
The same input is also solved with FP32 V-cycles inside the FP64
defect-correction loop ("mixed"), and the 256^3 field of the same generator
is solved as a variant.

Prints one JSON line.  ``value`` is Mcell/s of the plain FP64 solve.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

METRIC = "Poisson solve time to rel. residual 1e-10 (Mcell/s, % HBM) plain vs mixed/NN"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell: every kernel reads each input once and writes
# each output once.  The dominant kernel (one fused red+black sweep) reads phi
# and f and writes phi: 24 B/cell (f64).
# V(2,2) cycle, f64, per finest cell: finest level = 2 sweeps (48) + residual
# and restriction (17) + prolongation with the first post sweep (25) + 1 sweep
# (24) = 114; each coarser level m (zero guess: the first sweep reads only b)
# 106 / 8^m  ->  ~129 B/cell.
# Mixed: FP64 residual rounded to FP32 (20) + FP32 finest level (8 + 12 + 8.5 +
# 12.5, and the last sweep adds its result to phi in place: 24) + FP32 coarser
# levels 53 / 8^m  ->  ~93 B/cell.
# Forming the right-hand side once reads rho twice and writes f: 24 B/cell.
SWEEP_BYTES_F64 = 24.0
VCYCLE_BYTES_F64 = 129.1
VCYCLE_BYTES_MIXED = 92.6
RHS_BYTES = 24.0
FORCE_BYTES_F64 = 32.0      # g = -grad(phi): read phi (8 B), write three components (24 B) per cell
# HBM traffic of the dominant kernel per launch at 256^3, bytes: rocprofv3
# FETCH_SIZE (x 1.99951) + WRITE_SIZE (x 1.0), the factors being what the same
# counters read for a device copy of known size (profiles/ holds the runs).
# Valid for n = 256 only; set to None whenever the kernel changes.
TRAFFIC_256 = 428528566
# the same at 512^3 (FETCH_SIZE x 1.99992 for the 1074 MB calibration copy)
TRAFFIC_512 = 3456105130


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="cells per dimension (default 512)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=0,
                    help="oracle V-cycles timed for the CPU baseline (default: 1 at 512^3 and up, else 2)")
    ap.add_argument("--sweep-reps", type=int, default=20, help="smoother sweeps timed for the roofline")
    ap.add_argument("--no-small", action="store_true", help="skip the 256^3 plain-vs-mixed variant")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--no-amr", action="store_true", help="skip the refined-level (AMR) leg")
    ap.add_argument("--weights", default=None, help="warm-start weights (.npy); default: the package's trained set")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only a calibration copy of one field (n^3 f64) and the timed smoother sweeps "
                         "(for hardware-counter runs)")
    ap.add_argument("--hash-only", action="store_true",
                    help="only the incremental key-table leg (for kernel traces)")
    ap.add_argument("--amr-only", action="store_true",
                    help="only a calibration copy of a 128^3 f64 field and the refined-level leg "
                         "(for hardware-counter runs)")
    ap.add_argument("--nn-only", action="store_true",
                    help="only the warm-started 256^3 leg (for kernel traces of the network)")
    ap.add_argument("--force-only", action="store_true",
                    help="only a calibration copy of one field (n^3 f64) and the timed force launches "
                         "(for hardware-counter runs)")
    return ap.parse_args()


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_2604_06035_amd import abi
    from workloads import dense_to_oct, lognormal_density

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    cells = n ** 3
    h = 1.0 / n
    if args.roofline_only:
        return roofline_only(args, abi, torch, n)
    if args.force_only:
        return force_only(args, abi, torch, n)
    if args.hash_only:
        print(json.dumps(hash_leg(abi, torch)), flush=True)
        return 0
    if args.nn_only:
        print(json.dumps({"nn": nn_leg(args, abi, torch, dev, torch.cuda.current_stream())}), flush=True)
        return 0
    if args.amr_only:
        src = torch.randn(128 ** 3, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(json.dumps({"copy_bytes": 2 * 8 * 128 ** 3, "amr": amr_leg(args, abi, torch, dev)}), flush=True)
        return 0
    rho_h = lognormal_density(n, seed=args.seed)
    rho = torch.from_numpy(dense_to_oct(rho_h)).to(dev)
    stream = torch.cuda.current_stream()

    def run(precision: int, rho=rho, n=n, steps=args.steps, warmup=args.warmup):
        L = abi.mg_build_level(n, precision=precision, stream=stream)
        phi = torch.zeros_like(rho)
        infos = []
        try:
            for _ in range(warmup):
                phi.zero_()
                abi.mg_solve(L, rho, None, 1.0, None, phi, args.tol, 100)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                phi.zero_()
                st, info = abi.mg_solve(L, rho, None, 1.0, None, phi, args.tol, 100)
                if st != abi.MG_OK:
                    raise RuntimeError(f"solve did not converge: {info}")
                infos.append(info)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        finally:
            abi.mg_destroy_level(L)
        return t / steps * 1e3, infos, phi

    ms_plain, infos_plain, phi_plain = run(abi.MG_PREC_FP64)
    ms_mixed, infos_mixed, phi_mixed = run(abi.MG_PREC_MIXED)
    cyc_plain = infos_plain[-1]["cycles"]
    cyc_mixed = infos_mixed[-1]["cycles"]
    mcell = cells / (ms_plain * 1e-3) / 1e6
    alg_plain = cells * (RHS_BYTES + cyc_plain * VCYCLE_BYTES_F64)
    alg_mixed = cells * (RHS_BYTES + cyc_mixed * VCYCLE_BYTES_MIXED)

    # dominant kernel: the fused red-black sweep on the finest level (same
    # launch configuration as inside the solve), timed with HIP events on the
    # stream the library launches on
    sweep_ms = time_sweeps(abi, torch, n, h, stream, args.sweep_reps)
    sweep_gbs = SWEEP_BYTES_F64 * cells / (sweep_ms * 1e-3) / 1e9

    fft = fft_leg(args, abi, torch, rho, n, stream, phi_plain, ms_plain)
    force = force_leg(abi, torch, phi_plain, n, stream, args.sweep_reps)
    table = hash_leg(abi, torch)
    phi_plain_h, phi_mixed_h = phi_plain.cpu().numpy(), phi_mixed.cpu().numpy()
    del phi_plain, phi_mixed
    torch.cuda.empty_cache()
    small = None if (args.no_small or n == 256) else small_leg(args, abi, torch, run, dev)
    nn = None if args.no_nn else nn_leg(args, abi, torch, dev, stream)
    amr = None if args.no_amr else amr_leg(args, abi, torch, dev)

    out = {
        "metric": METRIC,
        "value": round(mcell, 2),
        "unit": "Mcell/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_plain, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"periodic {n}^3 lognormal GRF (P(k)~k^-2.5, var 1.5, seed {args.seed}); "
                        f"FP64 multigrid V(2,2), red-black GS, to relres {args.tol:g} from phi=0",
            "n": n, "cells": cells, "tol": args.tol, "nu_pre": 2, "nu_post": 2, "coarsest": 4,
        },
        "cycles": cyc_plain,
        "relres": infos_plain[-1]["relres"],
        "solve_ms_hip_event_median": round(statistics.median(i["ms"] for i in infos_plain), 4),
        "hbm_pct_algorithmic": round(100.0 * alg_plain / (ms_plain * 1e-3) / (HBM_PEAK_GBS * 1e9), 2),
        "variants": {
            "mixed": {
                "dtype": "f32 V-cycles in f64 defect correction",
                "ms_per_step": round(ms_mixed, 4),
                "mcell_s": round(cells / (ms_mixed * 1e-3) / 1e6, 2),
                "cycles": cyc_mixed,
                "relres": infos_mixed[-1]["relres"],
                "speedup_vs_plain": round(ms_plain / ms_mixed, 3),
                "hbm_pct_algorithmic": round(100.0 * alg_mixed / (ms_mixed * 1e-3) / (HBM_PEAK_GBS * 1e9), 2),
            },
            "nn": nn,
            "fft": fft,
        },
        "force": force,
        "hash_table": table,
        "periodic_256": small,
        "amr": amr,
        "roofline": {
            "kernel": "k_smooth_march<double,false,false>: one red+black Gauss-Seidel sweep (z-marching LDS ring), finest level",
            "bound": "hbm",
            "achieved": round(sweep_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(sweep_gbs / HBM_PEAK_GBS, 4),
            "traffic": {256: TRAFFIC_256, 512: TRAFFIC_512}.get(n),
            "launch_ms": round(sweep_ms, 5),
            "bytes_per_cell": SWEEP_BYTES_F64,
            "cells_per_launch": cells,
        },
        "cpu_baseline": None,
    }
    traffic = out["roofline"]["traffic"]
    if traffic:
        out["roofline"]["measured_GBs"] = round(traffic / (sweep_ms * 1e-3) / 1e9, 1)
        out["roofline"]["measured_frac"] = round(traffic / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    if not args.no_cpu_baseline:
        cpu_cycles = args.cpu_cycles or (1 if n >= 512 else 2)
        out["cpu_baseline"], out["oracle_check"] = cpu_baseline(
            rho_h, n, cpu_cycles, cyc_plain, {"plain": phi_plain_h, "mixed": phi_mixed_h})
    print(json.dumps(out), flush=True)
    return 0


def time_sweeps(abi, torch, n, h, stream, reps):
    """Average duration of one sweep launch: mg_op_smooth with an even sweep
    count runs that many launches back to back (ping-pong between the caller's
    buffer and the work buffer, ending in the caller's: no copy)."""
    reps = max(2, reps + (reps & 1))
    b = torch.randn(n ** 3, dtype=torch.float64, device="cuda")
    ph = torch.zeros_like(b)
    work = torch.empty_like(b)
    abi.mg_op_smooth(n, h, ph, b, 2, work, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    abi.mg_op_smooth(n, h, ph, b, reps, work, stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def roofline_only(args, abi, torch, n):
    """Calibration copy (reads and writes n^3 * 8 bytes once) followed by the
    launches of the dominant kernel, each a separate dispatch."""
    stream = torch.cuda.current_stream()
    src = torch.randn(n ** 3, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    ms = time_sweeps(abi, torch, n, 1.0 / n, stream, args.sweep_reps)
    print(json.dumps({"n": n, "copy_bytes": 2 * 8 * n ** 3, "sweeps": max(2, args.sweep_reps + (args.sweep_reps & 1)),
                      "launch_ms": round(ms, 5),
                      "alg_GBs": round(SWEEP_BYTES_F64 * n ** 3 / (ms * 1e-3) / 1e9, 1)}), flush=True)
    return 0


def force_only(args, abi, torch, n):
    """Calibration copy (reads and writes n^3 * 8 bytes once), then the force
    launches of force_leg (one warm-up + sweep_reps timed) on a random phi."""
    stream = torch.cuda.current_stream()
    src = torch.randn(n ** 3, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del dst
    res = force_leg(abi, torch, src, n, stream, args.sweep_reps)
    print(json.dumps({"n": n, "copy_bytes": 2 * 8 * n ** 3, "launches": 1 + max(2, args.sweep_reps), **res}),
          flush=True)
    return 0


def fft_leg(args, abi, torch, rho, n, stream, phi_mg, ms_plain):
    """The direct FFT solve of the same level (discrete Green's function):
    wall time per call with the input resident, its relative residual and its
    distance from the multigrid solution."""
    L = abi.mg_build_level(n, stream=stream)
    phi = torch.empty_like(rho)
    try:
        abi.mg_fft_solve(L, rho, None, 1.0, phi)   # warm-up (allocates the work space)
        torch.cuda.synchronize()
        steps = max(3, args.steps)
        t0 = time.perf_counter()
        for _ in range(steps):
            st, info = abi.mg_fft_solve(L, rho, None, 1.0, phi)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
    finally:
        abi.mg_destroy_level(L)
    diff = float((phi - phi_mg).abs().max() / phi_mg.abs().max())
    res = {"ms_per_step": round(ms, 4), "mcell_s": round(n ** 3 / (ms * 1e-3) / 1e6, 2),
           "relres": info["relres"], "solve_ms_hip_event": round(info["ms"], 4),
           "speedup_vs_plain": round(ms_plain / ms, 2), "maxdiff_vs_multigrid": diff,
           "method": "real-to-complex forward FFT, discrete Green's function, inverse FFT (own radix-4 HIP kernels, FP64)"}
    del phi
    torch.cuda.empty_cache()
    return res


def force_leg(abi, torch, phi, n, stream, reps):
    """g = -grad(phi) of the solved potential (the force step after the
    solve): average launch duration of mg_op_force over `reps` back-to-back
    launches (HIP events on the launch stream) against the HBM peak."""
    reps = max(2, reps)
    g = torch.empty((3,) + tuple(phi.shape), dtype=torch.float64, device="cuda")
    abi.mg_op_force(n, 1.0 / n, phi, g, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        abi.mg_op_force(n, 1.0 / n, phi, g, stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = FORCE_BYTES_F64 * n ** 3 / (ms * 1e-3) / 1e9
    del g
    torch.cuda.empty_cache()
    return {"kernel": "k_force: central differences, one thread per oct, component-major output",
            "launch_ms": round(ms, 5), "bytes_per_cell": FORCE_BYTES_F64, "achieved_GBs": round(gbs, 1),
            "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def hash_leg(abi, torch):
    """The incrementally maintained Morton-key table: 2^21 distinct octs of a
    1024^3-oct level (64-bit keys) and the same octs 2^30 deeper in each
    coordinate (128-bit keys): insert into a presized table and into a
    16-slot one that doubles as it fills, look every key up, build the
    6-neighbour rows, erase half and rebuild.  Host wall time per call with
    the keys resident (insert, erase and rebuild synchronise by contract)."""
    import numpy as np
    rng = np.random.default_rng(7)
    n = 1 << 21
    lin = rng.choice(1 << 30, size=n, replace=False)
    ijk = np.stack([lin & 1023, (lin >> 10) & 1023, lin >> 20], axis=1).astype(np.int64)
    vals = torch.arange(n, dtype=torch.int32, device="cuda")
    out = {"keys": n}

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps

    for W, shift, n_dim in ((1, 0, 1024), (2, 30, 1 << 40)):
        c = torch.from_numpy(ijk + (shift and (1 << shift) - 512)).cuda()
        if W == 1:
            keys = torch.empty(n, dtype=torch.int64, device="cuda")
            abi.mg_op_morton(c.to(torch.int32), keys)
        else:
            keys = torch.empty((n, 2), dtype=torch.int64, device="cuda")
            abi.mg_op_morton128(c, keys)
        torch.cuda.synchronize()
        rec = {}
        ins = []
        for _ in range(4):
            H = abi.mg_hash_create(W, int(n / 0.7) + 1, 0.7)
            torch.cuda.synchronize()
            t = time.perf_counter()
            abi.mg_hash_insert(H, keys, vals)
            ins.append((time.perf_counter() - t) * 1e3)
            abi.mg_hash_destroy(H)
        H = abi.mg_hash_create(W, int(n / 0.7) + 1, 0.7)
        try:
            abi.mg_hash_insert(H, keys, vals)
            rec["insert_presized_ms"] = round(statistics.median(ins[1:]), 3)
            rec["update_existing_ms"] = round(timed(lambda: abi.mg_hash_insert(H, keys, vals)), 3)
            got = torch.empty(n, dtype=torch.int32, device="cuda")
            rec["lookup_ms"] = round(timed(lambda: abi.mg_hash_lookup(H, keys, got)), 3)
            assert torch.equal(got, vals)
            nbr = torch.empty((n, 6), dtype=torch.int32, device="cuda")
            rec["neighbours_ms"] = round(timed(lambda: abi.mg_hash_neighbours(H, keys, n_dim, nbr)), 3)
            rec["capacity"] = abi.mg_hash_info(H)["capacity"]
        finally:
            abi.mg_hash_destroy(H)

        def grow_erase_rebuild():
            H2 = abi.mg_hash_create(W, 0, 0.7)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                abi.mg_hash_insert(H2, keys, vals)
                t1 = time.perf_counter()
                abi.mg_hash_erase(H2, keys[::2].contiguous())
                t2 = time.perf_counter()
                abi.mg_hash_rebuild(H2)
                t3 = time.perf_counter()
                return (t1 - t0) * 1e3, (t2 - t1) * 1e3, (t3 - t2) * 1e3, abi.mg_hash_info(H2)
            finally:
                abi.mg_hash_destroy(H2)
        grow_erase_rebuild()
        g = [grow_erase_rebuild() for _ in range(3)]
        rec["insert_from_16_slots_ms"] = round(statistics.median(x[0] for x in g), 3)
        rec["erase_half_ms"] = round(statistics.median(x[1] for x in g), 3)
        rec["rebuild_ms"] = round(statistics.median(x[2] for x in g), 3)
        rec["after_rebuild"] = g[-1][3]
        rec["lookup_mkeys_s"] = round(n / (rec["lookup_ms"] * 1e-3) / 1e6, 1)
        out["key64" if W == 1 else "key128"] = rec
    return out


def nn_leg(args, abi, torch, dev, stream):
    """Warm-started solves of the 256^3 field (the size the network was
    trained at): network + residual check + multigrid (fallback to zero when
    the guess is no better), and the forward pass alone for its matrix-core
    utilisation."""
    import numpy as np

    from paper_2604_06035_amd.warmstart import DEFAULT_WEIGHTS
    from workloads import dense_to_oct, lognormal_density
    path = args.weights or DEFAULT_WEIGHTS
    if not os.path.exists(path):
        return {"status": f"no trained weights at {os.path.relpath(path)}"}
    n = 256
    rho = torch.from_numpy(dense_to_oct(lognormal_density(n, seed=args.seed))).to(dev)
    net = abi.mgnn_create(24, 5, 0)
    L = abi.mg_build_level(n, stream=stream)
    try:
        abi.mgnn_set_weights(net, np.load(path))
        phi = torch.zeros_like(rho)
        for _ in range(args.warmup):
            abi.mgnn_solve_warm(net, L, rho, None, 1.0, phi, args.tol, 100)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st, info = abi.mgnn_solve_warm(net, L, rho, None, 1.0, phi, args.tol, 100)
            if st != abi.MG_OK:
                raise RuntimeError(f"warm-started solve did not converge: {info}")
            infos.append(info)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            abi.mgnn_forward(net, n, rho, None, 1.0, phi, stream)
        e1.record(stream)
        e1.synchronize()
        fwd_ms = e0.elapsed_time(e1) / reps
    finally:
        abi.mgnn_destroy(net)
        abi.mg_destroy_level(L)
    # useful flops per cell: 2 x (27*24 + 3*27*24*24 + 27*24) multiply-adds
    flops = 2.0 * (27 * 24 + 3 * 27 * 24 * 24 + 27 * 24) * n ** 3
    return {
        "ms_per_step": round(ms, 4), "cycles": infos[-1]["cycles"], "relres0": infos[-1]["relres0"],
        "relres": infos[-1]["relres"], "used_fallback": infos[-1].get("used_fallback"),
        "mcell_s": round(n ** 3 / (ms * 1e-3) / 1e6, 2),
        "forward_ms": round(fwd_ms, 4),
        "forward_tflops": round(flops / (fwd_ms * 1e-3) / 1e12, 2),
        "forward_mfma_util": round(flops / (fwd_ms * 1e-3) / 2.5e15, 4),
        "weights": os.path.relpath(path),
        "n": n,
    }


def amr_leg(args, abi, torch, dev):
    """Periodic 128^3 base + three refined levels around 64 Plummer clumps
    (seeded; built on the host, ~30 s): per level the build (GPU Morton keys,
    hash table, neighbour cache, father-cell hierarchy, ghost map) and the
    solve to the same tolerance from zero, FP64 and mixed, each level taking
    its Dirichlet ghosts from the level above's solution."""
    import numpy as np

    from workloads import build_amr_input, dense_to_oct
    t0 = time.perf_counter()
    amr = build_amr_input()
    t_input = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    out = {"input": "base 128^3 + 3 refined levels, 64 Plummer clumps (seeds 3/1003)",
           "host_input_s": round(t_input, 1), "levels": []}
    for precision, tag in ((abi.MG_PREC_FP64, "plain"), (abi.MG_PREC_MIXED, "mixed")):
        handles, rhos, phis = [], [], []
        try:
            parent = None
            for lv in amr.levels:
                if lv.level == 0:
                    rho = torch.from_numpy(dense_to_oct(lv.rho)).to(dev)
                    octs = None
                else:
                    rho = torch.from_numpy(np.ascontiguousarray(lv.rho.reshape(-1))).to(dev)
                    octs = torch.from_numpy(lv.oct_ijk).to(dev)
                def build():
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    if lv.level == 0:
                        h_ = abi.mg_build_level(amr.base_n, 0, precision=precision, stream=stream)
                    else:
                        h_ = abi.mg_build_level(amr.base_n, lv.level, lv.n_oct, octs, parent, precision=precision,
                                                stream=stream)
                    torch.cuda.synchronize()
                    return h_, (time.perf_counter() - t) * 1e3
                hd, build_first_ms = build()
                # warm builds of the same level (the first one also pays one-time set-up)
                build_warm = []
                for _ in range(3):
                    h_, b_ms = build()
                    abi.mg_destroy_level(h_)
                    build_warm.append(b_ms)
                handles.append(hd)
                rhos.append(rho)
                parent = hd
                phi = torch.zeros_like(rho)
                pp = phis[-1] if phis else None
                rm = None if lv.level == 0 else amr.rho_mean
                abi.mg_solve(hd, rho, rm, 1.0, pp, phi, args.tol, 100)      # warm-up
                ms = []
                for _ in range(3):
                    phi.zero_()
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    st, info = abi.mg_solve(hd, rho, rm, 1.0, pp, phi, args.tol, 100)
                    torch.cuda.synchronize()
                    ms.append((time.perf_counter() - t) * 1e3)
                    if st != abi.MG_OK:
                        raise RuntimeError(f"AMR level {lv.level} ({tag}) did not converge: {info}")
                phis.append(phi)
                cells = lv.n_oct * 8 if lv.level else amr.base_n ** 3
                g = torch.empty(3 * cells, dtype=torch.float64, device=dev)
                abi.mg_force(hd, pp, phi, g)                                  # warm-up
                t = time.perf_counter()
                for _ in range(5):
                    abi.mg_force(hd, pp, phi, g)
                force_ms = (time.perf_counter() - t) * 1e3 / 5
                del g
                rec = {"level": lv.level, "n_oct": int(lv.n_oct if lv.level else (amr.base_n // 2) ** 3),
                       "cells": int(cells), "cycles": info["cycles"], "relres": info["relres"],
                       "solve_ms": round(statistics.median(ms), 3),
                       "mcell_s": round(cells / (statistics.median(ms) * 1e-3) / 1e6, 1),
                       "force_ms": round(force_ms, 3)}
                rec["build_ms"] = round(statistics.median(build_warm), 2)
                rec["build_first_ms"] = round(build_first_ms, 2)
                if tag == "plain":
                    out["levels"].append({"plain": rec})
                else:
                    out["levels"][len(phis) - 1]["mixed"] = rec
            # the whole hierarchy in one call (the gravity step's solve), base
            # level by V-cycles or by the direct FFT solve
            for base_fft in (False, True):
                ms = []
                for _ in range(3):
                    for p_ in phis:
                        p_.zero_()
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    st, infos = abi.mg_solve_chain(handles, rhos, None, 1.0, phis, args.tol, 100, base_fft=base_fft)
                    torch.cuda.synchronize()
                    ms.append((time.perf_counter() - t) * 1e3)
                    if st != abi.MG_OK:
                        raise RuntimeError(f"AMR chain ({tag}, base_fft={base_fft}) did not converge: {infos}")
                out.setdefault("chain_ms", {})[f"{tag}{'_fft_base' if base_fft else ''}"] = \
                    round(statistics.median(ms), 3)
        finally:
            for hd in handles:
                abi.mg_destroy_level(hd)
    return out


def small_leg(args, abi, torch, run, dev):
    """256^3, same generator (seed 2): plain FP64 vs FP32-in-FP64 multigrid,
    the direct FFT solve and the smoother at this size (its working set of
    3 x 134 MB fits the 256 MB last-level cache, so its rates are not HBM
    rates)."""
    from workloads import dense_to_oct, lognormal_density
    n = 256
    rho = torch.from_numpy(dense_to_oct(lognormal_density(n, seed=args.seed))).to(dev)
    ms_p, inf_p, _ = run(abi.MG_PREC_FP64, rho=rho, n=n, steps=max(3, args.steps), warmup=1)
    ms_m, inf_m, _ = run(abi.MG_PREC_MIXED, rho=rho, n=n, steps=max(3, args.steps), warmup=1)
    cells = n ** 3
    L = abi.mg_build_level(n, stream=torch.cuda.current_stream())
    try:
        phi = torch.empty_like(rho)
        abi.mg_fft_solve(L, rho, None, 1.0, phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            _, inf_f = abi.mg_fft_solve(L, rho, None, 1.0, phi)
        torch.cuda.synchronize()
        ms_f = (time.perf_counter() - t0) / 3 * 1e3
    finally:
        abi.mg_destroy_level(L)
    del rho, phi
    torch.cuda.empty_cache()
    sweep_ms = time_sweeps(abi, torch, n, 1.0 / n, torch.cuda.current_stream(), args.sweep_reps)
    sweep_gbs = SWEEP_BYTES_F64 * cells / (sweep_ms * 1e-3) / 1e9
    res = {"n": n, "plain": {"ms": round(ms_p, 3), "mcell_s": round(cells / (ms_p * 1e-3) / 1e6, 1),
                             "cycles": inf_p[-1]["cycles"], "relres": inf_p[-1]["relres"],
                             "hbm_pct_algorithmic": round(100.0 * cells * (RHS_BYTES + inf_p[-1]["cycles"] *
                                                          VCYCLE_BYTES_F64) / (ms_p * 1e-3) / (HBM_PEAK_GBS * 1e9), 2)},
           "mixed": {"ms": round(ms_m, 3), "mcell_s": round(cells / (ms_m * 1e-3) / 1e6, 1),
                     "cycles": inf_m[-1]["cycles"], "relres": inf_m[-1]["relres"]},
           "speedup_mixed": round(ms_p / ms_m, 3),
           "fft": {"ms": round(ms_f, 3), "mcell_s": round(cells / (ms_f * 1e-3) / 1e6, 1), "relres": inf_f["relres"],
                   "speedup_vs_plain": round(ms_p / ms_f, 2)},
           "sweep": {"kernel": "k_smooth_march<double,false,false>", "launch_ms": round(sweep_ms, 5),
                     "achieved_GBs": round(sweep_gbs, 1), "frac": round(sweep_gbs / HBM_PEAK_GBS, 4),
                     "traffic": TRAFFIC_256}}
    if TRAFFIC_256:
        res["sweep"]["measured_GBs"] = round(TRAFFIC_256 / (sweep_ms * 1e-3) / 1e9, 1)
    torch.cuda.empty_cache()
    return res


def cpu_baseline(rho_h, n, n_cycles, gpu_cycles, gpu_phis):
    """The oracle (plain NumPy FP64 V-cycles, one host core) on the same input."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import poisson as P
    from workloads import oct_to_dense

    with threadpool_limits(1):
        h = 1.0 / n
        f = P.rhs(rho_h, 1.0)
        phi = np.zeros_like(f)
        t0 = time.perf_counter()
        for _ in range(n_cycles):
            P.vcycle(phi, f, h)
            phi = P.project_mean(phi)
        t = time.perf_counter() - t0
        per_cycle = t / n_cycles
        value = n ** 3 / (per_cycle * gpu_cycles) / 1e6
        ref = P.fft_solve(f, h)
        check = {}
        for k, v in gpu_phis.items():
            d = oct_to_dense(v, n)
            check[k] = {"relres_oracle": P.relres(d, f, h), "maxdiff_vs_fft": P.maxdiff(d, ref)}
    base = {
        "value": round(value, 4),
        "unit": "Mcell/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n_cycles} oracle V(2,2) cycles on the same {n}^3 input ({t:.1f} s, {per_cycle:.2f} s/cycle), "
                  f"extrapolated to the {gpu_cycles} cycles the solve needs",
        "host_cores_available": len(os.sched_getaffinity(0)),
        "cpu_model": _cpu_model(),
    }
    return base, check


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    sys.exit(main())

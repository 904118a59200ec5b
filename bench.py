#!/usr/bin/env python3
"""Throughput of the GRMHD Runge-Kutta step on one MI355X.

Workload (default): the synthetic star on a 256^3 grid split into 64
MeshBlocks of 64^3 cells (3 ghost layers), Gamma = 2 ideal gas, WENOZ + HLLE,
FOFC + DMP (M = 1.1), atmosphere rho_atm = 1.28e-13, T_atm = 1.28e-11,
f_thr = 0.1; one step = SSP-RK2 (two stages, ghost exchange after each) with
dt from the on-device CFL reduction (CFL 0.25).  Inputs are resident in HBM
before timing starts.

Metric: zone-updates/s = interior cells x RK2 steps / second.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


STAR_PARAMS = dict(gamma=2.0, rho_atm=1.28e-13, T_atm=1.28e-11, f_thr=0.1, M_max=100.0, recon=2,
                   riemann=1, fofc=1, dmp_M=1.1)


def cpu_baseline(st, n_per_side, nb, params_kw, target_s=12.0):
    """The FP64 oracle as it stands, on one block of the same workload (the
    block at the star's centre, ghosts frozen at the analytic data), RK2
    steps until ~target_s seconds of CPU work."""
    from paper_2409_10384_amd import inputs
    import oracle as O
    threads = os.cpu_count() or 1
    c = n_per_side // 2
    blk = inputs.star_block_numpy(st, c, c, c, n_per_side, nb)
    m = O.Mesh([blk], O.Params(**params_kw))
    dt = m.dt(0.25)
    steps, t0 = 0, time.perf_counter()
    while True:
        m.rk2_step(dt)
        steps += 1
        el = time.perf_counter() - t0
        if el > target_s or steps >= 50:
            break
    zu = blk.nx * blk.ny * blk.nz * steps / el
    return {"value": zu, "unit": "zone-updates/s", "cores": int(os.environ.get("OMP_NUM_THREADS", threads)),
            "kind": "oracle",
            "sample": f"one {blk.nx}^3 block of the star (frozen ghosts), {steps} RK2 steps, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--blocks-per-side", type=int, default=4)
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the stage shards by MeshBlocks; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_10384_amd import inputs, lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lib.load()
    t0 = time.perf_counter()
    log(f"building inputs: star, {args.blocks_per_side}^3 blocks of {args.block}^3")
    blocks, st = inputs.star_blocks(n_per_side=args.blocks_per_side, nb=args.block, device="cuda")
    log(f"inputs built in {time.perf_counter() - t0:.1f} s")
    params = lib.MethodParams(**STAR_PARAMS)
    mesh = lib.DeviceMesh(blocks, params, device="cuda")
    torch.cuda.synchronize()
    log(f"mesh resident in HBM ({time.perf_counter() - t0:.1f} s)")
    ncell = sum(b.nx * b.ny * b.nz for b in blocks)
    for s in range(args.warmup):
        mesh.rk2_step(cfl=0.25)
    torch.cuda.synchronize()
    log("warmup done")
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for s in range(args.steps):
        mesh.rk2_step(cfl=0.25)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = ncell * args.steps / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.2f} ms, {value:.3e} zone-updates/s")
    out = {
        "metric": "zone-updates/s per GPU (GRMHD SSP-RK2 step, plain C2P)",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"star {args.blocks_per_side * args.block}^3 as "
                               f"{args.blocks_per_side ** 3} MeshBlocks of {args.block}^3, Gamma=2, "
                               f"WENOZ+HLLE, FOFC+DMP, RK2 CFL 0.25",
                   "cells": ncell},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(st, args.blocks_per_side, args.block, STAR_PARAMS)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

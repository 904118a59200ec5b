#!/usr/bin/env python3
"""Throughput of the GRMHD Runge-Kutta step on one MI355X.

Workload: the synthetic star on a 256^3 grid split into 64 MeshBlocks of 64^3
cells (3 ghost layers), Gamma = 2 ideal gas, WENOZ + HLLE, FOFC + DMP
(M = 1.1), atmosphere rho_atm = 1.28e-13, T_atm = 1.28e-11, f_thr = 0.1.  One
step = SSP-RK2 (two stages, ghost exchange after each) with dt from the
on-device CFL reduction (CFL 0.25).  Inputs are resident in HBM before timing
starts.

Metric: zone-updates/s = interior cells x RK2 steps / second (plain C2P).
Also reported: C2P solves/s on 2^24 random states at root tolerance 1e-12
(plain bracket vs learned bracket, network trained in this run on the GPU),
the roofline of the dominant kernel (HIP events on the launch stream), the
whole-step roofline, and the FP64 oracle on the host as a CPU baseline.
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6          # MI355X FP64 vector peak
# ADM matter sources per interior cell: w (5), two faces per direction (6) and
# gamma_ij (6) read, E, S_i, S_ij (10) written
MATTER_BYTES_PER_CELL = (5 + 6 + 6 + 10) * 8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


STAR_PARAMS = dict(gamma=2.0, rho_atm=1.28e-13, T_atm=1.28e-11, f_thr=0.1, M_max=100.0, recon=2,
                   riemann=1, fofc=1, dmp_M=1.1)
C2P_PARAMS = dict(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30, f_thr=1.0, M_max=1e30, c2p_tol=1e-12)


# ---------------------------------------------------------------------------
# algorithmic bytes (minimum HBM traffic of each kernel if every value it
# needs were read once and every value it produces written once)
# ---------------------------------------------------------------------------
def kernel_bytes(family, blocks):
    tot = 0
    for b in blocks:
        n = (b.nx, b.ny, b.nz)
        g = b.ng
        cells_in = n[0] * n[1] * n[2]
        if family.startswith("flux_"):
            d = "xyz".index(family[-1])
            box, faces = 1, 1
            for a in range(3):
                box *= (n[a] + 2 * g) if a == d else (n[a] + 2)
                faces *= (n[a] + 1) if a == d else (n[a] + 2)
            # stencil inputs: rho, W v^i, P, 2 transverse B, 10 metric fields;
            # per face: normal field in, 7 flux components out
            tot += 8 * (17 * box + 8 * faces)
        elif family == "update":
            # the stage's update with the inversion in its tail: U^n 5,
            # U^(s) 5, w 5, B~ of the stage input 3, ADM 16, flux divergence
            # 15, B~ of the updated faces 3 in; U 5, w 5 out; flag in/out
            tot += 8 * 62 * cells_in + 4 * cells_in
        elif family == "fofc_flags":
            # U^n 5, U^(s) 5, B~ 3, metric 6, fluxes 15 in; flag out
            tot += 8 * 34 * cells_in + 2 * cells_in
        elif family == "stage_c2p":
            # U 5 in/out, B~ 3, metric 6 in, w 5 out, flag in/out
            tot += 8 * 24 * cells_in + 4 * cells_in
        elif family == "dt":
            tot += 8 * 18 * cells_in
        elif family == "bcc":
            m = (n[0] + 2 * g) * (n[1] + 2 * g) * (n[2] + 2 * g)
            tot += 8 * 12 * m
        else:
            return None
    return tot


def step_bytes(blocks):
    """whole RK2 step: per stage, 18 stencil-read fields over the padded block
    (w 5, B~ 3, alpha, beta 3, gamma 6) plus pointwise K 6 and U^n 5 (stage 2
    adds U^(s) 5 and B~^n 3), writes U 5, B~ 3, w 5"""
    tot = 0
    for b in blocks:
        m = (b.nx + 2 * b.ng) * (b.ny + 2 * b.ng) * (b.nz + 2 * b.ng)
        c = b.nx * b.ny * b.nz
        tot += 8 * (18 * m + 11 * c + 13 * c) + 8 * (18 * m + 19 * c + 13 * c)
    return tot


def source_hash():
    """hash of the step kernels' sources (as the counter summaries record it)"""
    from paper_2409_10384_amd import profiling
    return profiling.source_hash()


def pmc_fp64():
    """FP64 operations per launch by kernel family from the committed counter
    summary (None when the kernel sources changed since)"""
    path = os.path.join(ROOT, "profiles", "pmc_fp64.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash():
        return None
    return {k: v["flops_per_launch"] for k, v in d.get("kernels", {}).items()}


def pmc_step(name, key):
    """a per-step total (FP64 operations or counted HBM bytes of every kernel
    of the RK step) from a committed counter summary; None when the kernel
    sources changed since the counters were taken"""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash():
        return None
    return d.get(key)


def pmc_traffic(family, launches_per_step):
    """HBM bytes per launch of the kernel from the committed counter summary,
    null when the kernel sources changed since the counters were taken"""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(family)
    if not k:
        return None
    return k.get("bytes_per_launch")


# ---------------------------------------------------------------------------
def cpu_model():
    """the host CPU's model name (from /proc/cpuinfo, as lscpu shows it)"""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(st, n_per_side, nb, params_kw, target_s=12.0, single_s=6.0):
    """The FP64 oracle as it stands, on one block of the same workload (the
    block at the star's centre, ghosts frozen at the analytic data): RK2
    steps until ~target_s seconds of CPU work with OpenMP over k-slabs on the
    host's threads, then on one thread for ~single_s seconds."""
    from paper_2409_10384_amd import inputs
    import oracle as O
    c = n_per_side // 2
    blk = inputs.star_block_numpy(st, c, c, c, n_per_side, nb)

    def run(budget, max_steps):
        m = O.Mesh([copy_block(blk)], O.Params(**params_kw))
        dt = m.dt(0.25)
        steps, t0 = 0, time.perf_counter()
        while True:
            m.rk2_step(dt)
            steps += 1
            el = time.perf_counter() - t0
            if el > budget or steps >= max_steps:
                return steps, el

    threads = O.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    steps, el = run(target_s, 50)
    O.set_threads(1)
    s1, e1 = run(single_s, 20)
    O.set_threads(threads)
    n = blk.nx * blk.ny * blk.nz
    return {"value": n * steps / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": n * s1 / e1, "steps": s1, "s": e1},
            "sample": f"one {blk.nx}^3 block of the star (frozen ghosts), {steps} RK2 steps, "
                      f"{el:.1f} s, OpenMP over k-slabs on {threads} threads; single thread "
                      f"{s1} steps in {e1:.1f} s"}


def copy_block(b):
    import copy
    c = copy.copy(b)
    c.w = np.array(b.w)
    c.bf = [np.array(x) for x in b.bf]
    c.adm = np.array(b.adm)
    return c


def copy_bandwidth(torch, lib, n=1 << 27, reps=10):
    """HBM bandwidth a plain streaming copy reaches here: 1 GiB read and 1 GiB
    written per k_copy launch, HIP events over `reps` launches (GB/s of bytes
    read plus written)"""
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    lib.copy(a, b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lib.copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def star_section(args, torch, inputs, lib):
    t0 = time.perf_counter()
    log(f"building inputs: star, {args.blocks_per_side}^3 blocks of {args.block}^3")
    # --host-inputs: the initial data built with numpy and copied over (a
    # counter pass then sees a few copies instead of thousands of small
    # elementwise kernels)
    blocks, st = inputs.star_blocks(n_per_side=args.blocks_per_side, nb=args.block,
                                    device=None if args.host_inputs else "cuda")
    params = lib.MethodParams(**STAR_PARAMS)
    mesh = lib.DeviceMesh(blocks, params, device="cuda")
    torch.cuda.synchronize()
    log(f"mesh resident in HBM ({time.perf_counter() - t0:.1f} s)")
    ncell = sum(b.nx * b.ny * b.nz for b in blocks)
    tuned = None
    if args.threads:
        # fixed workgroup sizes (profiled runs: the autotuner's timings are not
        # meaningful under counter collection)
        from paper_2409_10384_amd import autotune
        tuned = {}
        for item in args.threads.split(","):
            fam, th = item.split("=")
            autotune.set_threads(fam, int(th))
            tuned[fam] = int(th)
        log(f"workgroup sizes set: {tuned}")
    elif not args.no_autotune:
        from paper_2409_10384_amd import autotune
        dt0 = float(mesh.compute_dt(0.25).item())
        tuned = {k: v["best"] for k, v in autotune.autotune(mesh, dt0, log=log).items()}
        tuned.pop("stage_c2p", None)     # fused into the update in the plain stage
    for _ in range(args.warmup):
        mesh.rk2_step(cfl=0.25)
    torch.cuda.synchronize()
    log("warmup done")
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    lib.timing(True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        mesh.rk2_step(cfl=0.25)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    fam = lib.timing_read()
    lib.timing(False)
    value = ncell * args.steps / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.2f} ms, {value:.3e} zone-updates/s")
    breakdown = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1]} for k, v in fam.items()}
    dom = max(fam.items(), key=lambda kv: kv[1][0])[0]
    dms = fam[dom][0] / fam[dom][1]
    nbytes = kernel_bytes(dom, blocks)
    roof = None
    if nbytes is not None:
        ach = nbytes / (dms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": lib.KERNEL_OF_FAMILY.get(dom, dom), "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": pmc_traffic(dom, None), "bytes_per_launch": nbytes,
                "avg_launch_ms": dms}
        copy = copy_bandwidth(torch, lib)
        roof["copy_GBps_measured"] = copy
        if roof["traffic"]:
            # the dominant kernel's counted bytes over its launch time, beside
            # what a plain copy reaches on this GPU
            roof["traffic_GBps"] = roof["traffic"] / (dms * 1e-3) / 1e9
    # FP64 rate of every stage kernel from the committed FP64 instruction
    # counters (operations per launch) and the launch times measured here
    fp64 = None
    ops = pmc_fp64()
    if ops:
        per = {}
        tot = 0.0
        for k, v in fam.items():
            if k in ops:
                per[k] = {"tflops": ops[k] / (v[0] / v[1] * 1e-3) / 1e12,
                          "frac": ops[k] / (v[0] / v[1] * 1e-3) / 1e12 / FP64_PEAK_TFS}
                tot += ops[k] * v[1]
        fp64 = {"peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "kernels": per,
                "counted_kernels_tflops": tot / (sum(v[0] for k, v in fam.items() if k in ops) * 1e-3) / 1e12}
    # the whole step (every kernel of both stages, the ghost fills and dt):
    # its algorithmic HBM bytes and its FP64 operations (counters of this
    # build) over the timed ms per step; the binding roofline is the one the
    # step's minimum time is set by
    sb = step_bytes(blocks)
    step_s = ms / args.steps * 1e-3
    traffic_step = pmc_step("pmc_traffic.json", "bytes_per_step")
    hbm = {"bound": "hbm", "algorithmic_bytes_per_step": sb, "achieved": sb / step_s / 1e9,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sb / step_s / 1e9 / HBM_PEAK_GBS,
           "traffic": traffic_step}
    flops = pmc_step("pmc_fp64.json", "flops_per_step")
    scope = "whole SSP-RK2 step: both stages, ghost fills and the dt reduction"
    if flops:
        t_fp, t_hbm = flops / (FP64_PEAK_TFS * 1e12), sb / (HBM_PEAK_GBS * 1e9)
        path = {"bound": "alu", "scope": scope, "achieved": flops / step_s / 1e12,
                "peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "frac": flops / step_s / 1e12 / FP64_PEAK_TFS,
                "traffic": traffic_step, "flops_per_step": flops, "flops_per_zone_update": flops / ncell,
                "binding": "fp64" if t_fp >= t_hbm else "hbm",
                "min_ms_per_step": max(t_fp, t_hbm) * 1e3, "hbm": hbm}
    else:
        # FP64 counters not taken on this build: the HBM roofline alone
        path = dict(hbm, scope=scope, note="FP64 counters of this build not committed")
    mass = float(mesh.mass().item())
    variants = None if args.no_variants else variant_section(args, torch, lib, mesh, params, ncell)
    if tuned:
        autotune.reset()
    return dict(value=value, ms=ms, ncell=ncell, roofline=roof, path=path, breakdown=breakdown,
                st=st, mass=mass, fp64=fp64, variants=variants, workgroup_sizes=tuned)


def variant_section(args, torch, lib, mesh, params, ncell, steps=3):
    """After the timed run, on the same resident star: the other
    reconstructions (flux kernel times and RK2 step rate), the SSP-RK3 step,
    and the ADM matter-source kernel with its HBM roofline"""
    import dataclasses
    out = {"steps": steps, "recon": {}}

    def run(fn, n):
        lib.timing(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        fam = lib.timing_read()
        lib.timing(False)
        return e0.elapsed_time(e1) / n, fam

    names = {0: "donor_cell", 1: "plm", 2: "wenoz", 3: "ppm4", 4: "ppmx"}
    for rc in (0, 1, 3, 4, 2):
        mesh.params = dataclasses.replace(params, recon=rc)
        mesh.rk2_step(cfl=0.25)
        ms, fam = run(lambda: mesh.rk2_step(cfl=0.25), steps)
        flux = {k: fam[k][0] / fam[k][1] for k in ("flux_x", "flux_y", "flux_z") if k in fam}
        out["recon"][names[rc]] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3),
                                   "flux_ms_per_launch": flux}
        log(f"variant {names[rc]}: {ms:.2f} ms per RK2 step, flux {flux}")
    mesh.params = params
    ms, _ = run(lambda: mesh.rk3_step(cfl=0.25), steps)
    out["rk3"] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3), "recon": "wenoz"}
    log(f"variant SSP-RK3: {ms:.2f} ms per step, {ncell / (ms * 1e-3):.3e} zone-updates/s")
    mesh.matter_sources(0)
    ms, fam = run(lambda: mesh.matter_sources(0), 10)
    mms = fam["matter"][0] / fam["matter"][1]
    nbytes = MATTER_BYTES_PER_CELL * ncell
    ach = nbytes / (mms * 1e-3) / 1e9
    out["matter_sources"] = {"ms_per_launch": mms, "bytes_per_launch": nbytes, "achieved": ach,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    log(f"matter sources: {mms:.3f} ms per launch, {ach:.0f} GB/s")
    return out


def refined_section(args, torch, inputs, lib):
    """~1500 independent blocks of 16^3/24^3/32^3 over 6 levels (frozen
    ghosts): RK2 steps launched block by block, batched (one launch per kernel
    and stage over the whole list), batched after the autotuner, and the
    batched step replayed from a captured HIP graph"""
    from paper_2409_10384_amd import autotune
    t0 = time.perf_counter()
    blocks, st = inputs.refined_star_blocks(nblocks=args.refined_blocks, device="cuda")
    mesh = lib.DeviceMesh(blocks, lib.MethodParams(**STAR_PARAMS), device="cuda")
    ncell = sum(b.nx * b.ny * b.nz for b in blocks)
    torch.cuda.synchronize()
    log(f"refined mesh: {len(blocks)} blocks, {ncell} cells ({time.perf_counter() - t0:.1f} s)")
    dt = float(mesh.compute_dt(0.25).item())
    K = args.refined_steps

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    res = {"blocks": len(blocks), "cells": ncell, "sizes": sorted({b.nx for b in blocks}),
           "levels": len({b.level for b in blocks}), "steps": K}
    ms = timed(lambda: mesh.rk2_step_per_block(dt=dt))
    res["per_block_launches"] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3)}
    log(f"refined per-block launches: {ms:.2f} ms/step")
    ms = timed(lambda: mesh.rk2_step(dt=dt))
    res["batched"] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3)}
    log(f"refined batched: {ms:.2f} ms/step")
    # the library's autotuner (grmhd_autotune) over the pencil length of
    # every stage kernel family
    tune = mesh.autotune(dt, reps=2)
    for fam, (best, ms_c) in tune.items():
        log(f"autotune {fam}: " + ", ".join(f"{k}:{v:.3f}" for k, v in ms_c.items()) + f" -> {best}")
    ms = timed(lambda: mesh.rk2_step(dt=dt))
    res["batched_autotuned"] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3),
                                "workgroup_sizes": {k: v[0] for k, v in tune.items()}}
    log(f"refined batched + autotuned: {ms:.2f} ms/step")
    # the whole step with device dt as one library call, and captured once
    # into the library's HIP graph and replayed
    ms = timed(lambda: mesh.rk2_step_lib(cfl=0.25))
    res["library_step_autotuned"] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3)}
    log(f"refined library step (device dt): {ms:.2f} ms/step")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = mesh.rk2_graph(side, cfl=0.25)
    try:
        def replay():
            g.launch(side)
        replay()
        side.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(side)
        for _ in range(K):
            g.launch(side)
        e1.record(side)
        side.synchronize()
        ms = e0.elapsed_time(e1) / K
    finally:
        g.close()
    res["graph_autotuned"] = {"ms_per_step": ms, "zone_updates_per_s": ncell / (ms * 1e-3)}
    log(f"refined library graph replay: {ms:.2f} ms/step")
    autotune.reset()
    return res


def _clone_blocks(blocks):
    import copy
    out = []
    for b in blocks:
        c = copy.copy(b)
        c.w = b.w.clone()
        c.bf = [x.clone() for x in b.bf]
        c.adm = b.adm.clone()
        out.append(c)
    return out


def _block_numpy(b):
    import copy
    c = copy.copy(b)
    c.w = b.w.cpu().numpy()
    c.bf = [x.cpu().numpy() for x in b.bf]
    c.adm = b.adm.cpu().numpy()
    return c


def c5_section(args, torch, inputs, lib, amr=True):
    """End-to-end: the star with a seeded 3-piece piecewise polytrope +
    Gamma_th = 1.75 thermal part, K RK2 steps with device dt, plain C2P (in
    the tail of the stage's update, its fastest form; the inversion
    statistics from a second run that inverts in a kernel of its own)
    against the learned bracket in the stage inversion (network trained on
    prim/cons pairs of the run's own states).  amr: the star on a leaf mesh
    of 32^3 blocks over 4 levels with the inter-level transfer (ghost fills
    across levels, flux and EMF correction); else the ~1500 independent
    blocks of 16^3, 24^3 and 32^3 over 6 levels with ghosts frozen at the
    analytic data."""
    pp, pK = inputs.pp_eos()
    st = inputs.calibrate_field(inputs.StarSetup(pp=pp, pp_K=pK))
    params_kw = {**STAR_PARAMS, **pp}
    params = lib.MethodParams(**params_kw)
    K = args.c5_steps
    if amr:
        blocks, leaf, st = inputs.star_leaf_blocks(st=st, device="cuda")
        make = lambda bl: lib.RefinedDeviceMesh(bl, params, leaf, device="cuda")
        # the oracle check: the same leaf structure with 8^3 blocks, whole mesh
        small_np, small_leaf, _ = inputs.star_leaf_blocks(st=st, nb=8)
        subset = list(range(len(small_np)))
        init_sub = small_np
        warm_mesh = lambda: lib.RefinedDeviceMesh([_copy_np(b) for b in small_np], params, small_leaf,
                                                  device="cuda")
        log(f"c5 (refined mesh, inter-level transfer): {len(blocks)} leaves of 32^3 on levels "
            f"{sorted(set(leaf.levels))}")
    else:
        blocks, st = inputs.refined_star_blocks(nblocks=args.refined_blocks, device="cuda", st=st)
        make = lambda bl: lib.DeviceMesh(bl, params, device="cuda")
        # seeded subset of 16 of the 16^3 blocks for the oracle check on the host
        rng = np.random.default_rng(inputs.SEED_BASE + 55)
        small = [i for i, b in enumerate(blocks) if b.nx == 16]
        subset = sorted(int(i) for i in rng.choice(small, size=min(16, len(small)), replace=False))
        init_sub = [_block_numpy(blocks[i]) for i in subset]
        warm_mesh = lambda: lib.DeviceMesh(_clone_blocks(blocks[:2]), params, device="cuda")
    ncell = sum(b.nx * b.ny * b.nz for b in blocks)
    log(f"c5: {len(blocks)} blocks, {ncell} cells, piecewise polytrope Gamma={pp['Gam'][:3]}")
    plain = make(blocks)
    learned = make(_clone_blocks(blocks))
    # the plain inversion's statistics come from a run of their own: with
    # them the stage inverts in a kernel of its own, without them (the timed
    # plain run) in the tail of the update
    counted = make(_clone_blocks(blocks))
    if amr:
        counted.ghost_fill(0)
        plain.ghost_fill(0)
        learned.ghost_fill(0)
    net = lib.LearnedC2P(seed=0)
    # warm every kernel of both paths once on a small mesh
    warm = warm_mesh()
    wu, wb, wg, ww = warm.c2p_pairs(0)
    net.fit(wu, wb, wg, params, ww, steps=2)
    warm.rk2_step(cfl=0.25)
    warm.rk2_step(cfl=0.25, mlp=net)
    del warm
    torch.cuda.synchronize()

    def run(mesh, mlp=None, stats=None, dts_in=None):
        # device dt every step; with dts_in the stages take that sequence
        # instead (same work, so that both runs see the same time steps)
        dts = torch.zeros(K, dtype=torch.float64, device="cuda")
        m0 = float(mesh.mass().item())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lib.timing(True)
        e0.record()
        for k in range(K):
            mesh.compute_dt(0.25)
            dk = mesh.dt_dev if dts_in is None else dts_in[k:k + 1]
            mesh.stage(1, dt_dev=dk, mlp=mlp, stats=stats)
            mesh.ghost_fill(1)
            mesh.stage(2, dt_dev=dk, mlp=mlp, stats=stats)
            mesh.ghost_fill(0)
            dts[k:k + 1].copy_(dk)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kt = {k: round(v[0] / K, 4) for k, v in lib.timing_read().items()}
        lib.timing(False)
        m1 = float(mesh.mass().item())
        return ms, (m1 - m0) / m0, dts, kt

    train_u = [plain.c2p_pairs(0, stride=2)]
    ms_p, drift_p, dts_p, kt_p = run(plain)
    log(f"c5 plain: {K} steps {ms_p:.1f} ms, {ncell * K / (ms_p * 1e-3):.3e} zone-updates/s, "
        f"mass drift {drift_p:.3e}")
    stats_p = torch.zeros(4, dtype=torch.int64, device="cuda")
    ms_c, _, _, kt_c = run(counted, stats=stats_p, dts_in=dts_p)
    pn_s, pn_ev = (int(x) for x in stats_p.cpu()[:2])
    del counted
    log(f"c5 plain with inversion statistics: {K} steps {ms_c:.1f} ms, "
        f"{ncell * K / (ms_c * 1e-3):.3e} zone-updates/s")
    train_u.append(plain.c2p_pairs(0, stride=2))
    u, bt, gam, w = (torch.cat([t[i] for t in train_u], dim=1).contiguous() for i in range(4))
    t0 = time.perf_counter()
    # states met during the run stray further from the training pairs than
    # the benchmark states do: widen the bracket to the 99.9% quantile of the
    # training residual, at least 0.05 in logit units
    losses = net.fit(u, bt, gam, params, w, steps=args.train_steps, log_every=max(1, args.train_steps // 4),
                     calibrate=0.999, width_min=0.05)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"c5 network trained on {u.shape[1]} pairs of the run's own states in {train_s:.1f} s, "
        f"losses {['%.3g' % x for x in losses]}, bracket width factor {net.width_k:.3g}")
    del u, bt, gam, w, train_u
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    ms_l, drift_l, _, kt_l = run(learned, mlp=net, stats=stats, dts_in=dts_p)
    n_s, n_ev, n_fb, n_fail = (int(x) for x in stats.cpu())
    log(f"c5 plain evals/solve {pn_ev / max(pn_s, 1):.2f}")
    log(f"c5 kernels plain (ms/step) {kt_p}")
    log(f"c5 kernels learned (ms/step) {kt_l}")
    log(f"c5 learned: {K} steps {ms_l:.1f} ms, {ncell * K / (ms_l * 1e-3):.3e} zone-updates/s, "
        f"mass drift {drift_l:.3e}, fallback {n_fb / max(n_s, 1):.4f}, evals/solve {n_ev / max(n_s, 1):.2f}")
    res = {"blocks": len(blocks), "cells": ncell, "steps": K, "eos": {k: pp[k] for k in ("Gam", "rho_b", "K0", "gamma_th")},
           "plain": {"ms": ms_p, "zone_updates_per_s": ncell * K / (ms_p * 1e-3), "mass_drift": drift_p,
                     "evals_per_solve": pn_ev / max(pn_s, 1), "kernel_ms_per_step": kt_p,
                     "with_statistics": {"ms": ms_c, "zone_updates_per_s": ncell * K / (ms_c * 1e-3),
                                         "kernel_ms_per_step": kt_c}},
           "learned": {"ms": ms_l, "zone_updates_per_s": ncell * K / (ms_l * 1e-3), "mass_drift": drift_l,
                       "fallback_rate": n_fb / max(n_s, 1), "evals_per_solve": n_ev / max(n_s, 1),
                       "failures": n_fail, "solves": n_s, "kernel_ms_per_step": kt_l},
           "learned_speedup": ms_p / ms_l, "train_s": train_s}
    if amr:
        res["mesh"] = {"leaves": len(blocks), "block": 32, "levels": sorted(set(leaf.levels)),
                       "leaves_per_level": {int(l): int(leaf.levels.count(l)) for l in set(leaf.levels)},
                       "domain": "[-48, 48]^3, outflow", "refined_within": [28.0, 14.0, 8.0]}
        res["note"] = ("ghosts filled across levels every stage (copy / restriction / prolongation), "
                       "flux and EMF correction at level boundaries; the drift is the floors' and the "
                       "outflow boundary's")
        # the oracle check's GPU leg: the 8^3-block mesh, a few steps from the
        # same initial data, plain and learned
        del plain, learned
        torch.cuda.synchronize()
        sub = {"subset": subset, "init": init_sub, "leaf": small_leaf, "params": params_kw}
        for kind, mlp in (("plain", None), ("learned", net)):
            gm = warm_mesh()
            gm.ghost_fill(0)
            dts = []
            for _ in range(args.c5_check_steps):
                gm.compute_dt(0.25)
                dts.append(float(gm.dt_dev.item()))
                gm.rk2_step(dt=dts[-1], mlp=mlp)
            torch.cuda.synchronize()
            sub["dts_" + kind] = np.array(dts)
            sub["gpu_" + kind] = [(gm.u0[i].cpu().numpy(), gm.w0[i].cpu().numpy(),
                                   [f.cpu().numpy() for f in gm.b0[i]]) for i in subset]
            del gm
        sub["dts"] = sub["dts_plain"]
        return res, sub
    res["note"] = "ghosts frozen at the analytic data, so mass also flows through block faces"
    # the oracle check runs on the host in the cpu leg, from these
    sub = {"subset": subset, "init": init_sub, "dts": dts_p.cpu().numpy(),
           "gpu_plain": [(plain.u0[i].cpu().numpy(), plain.w0[i].cpu().numpy(),
                          [f.cpu().numpy() for f in plain.b0[i]]) for i in subset],
           "gpu_learned": [(learned.u0[i].cpu().numpy(), learned.w0[i].cpu().numpy(),
                            [f.cpu().numpy() for f in learned.b0[i]]) for i in subset],
           "params": params_kw}
    del plain, learned
    torch.cuda.synchronize()
    return res, sub


def c5_oracle_check(sub):
    """The FP64 oracle (plain C2P) on the seeded 16-block subset with the GPU
    run's dt sequence; max deviation of the GPU's final state from it: the
    five conserved fields, the five primitives and the three face-field
    components, each over every interior cell (face) of the 16 blocks, in
    the pointwise metric (positive fields |d|/|x|; signed fields against
    max(|x|, 1e-3 max|x| of the block)), and D~ also relative to the
    block's largest D~ and over the star's cells alone."""
    import oracle as O
    from tests import parity as PM
    amr = "leaf" in sub
    out = {"blocks": sub["subset"] if not amr else f"all {len(sub['subset'])} leaves of the 8^3 mesh"}
    names_u = ("D", "S_x", "S_y", "S_z", "tau")
    names_w = ("rho", "u_x", "u_y", "u_z", "P")
    el = 0.0
    meshes = {}
    for kind in ("learned", "plain"):
        dts = sub.get("dts_" + kind, sub["dts"])
        key = tuple(float(x) for x in dts)
        if key not in meshes:
            if amr:
                m = O.RefinedMesh([_copy_np(b) for b in sub["init"]], O.Params(**sub["params"]), sub["leaf"])
                m.ghost_fill_state(0)
            else:
                m = O.Mesh([_copy_np(b) for b in sub["init"]], O.Params(**sub["params"]))
            t0 = time.perf_counter()
            for dt in dts:
                m.rk2_step(float(dt))
            el += time.perf_counter() - t0
            meshes[key] = m
        m = meshes[key]
        worst_all, worst_star = 0.0, 0.0
        fields = {}
        for j, (gu, gw, gb) in enumerate(sub["gpu_" + kind]):
            blk = sub["init"][j]
            ou, ow = m.interior(m.u0[j], j), m.interior(m.w0[j], j)
            gu_i, gw_i = m.interior(gu, j), m.interior(gw, j)
            scale = np.max(np.abs(ou[0]))
            worst_all = max(worst_all, float(np.max(np.abs(gu_i[0] - ou[0])) / scale))
            star = ow[0] > 1e-6 * 1.28e-3
            if star.any():
                worst_star = max(worst_star, float(np.max(np.abs(gu_i[0][star] - ou[0][star]) / ou[0][star])))
            errs = list(zip(names_u, PM.cons_errors(gu_i, ou))) + list(zip(names_w, PM.prim_errors(gw_i, ow)))
            g = blk.ng
            for d in range(3):
                sl = [slice(g, g + blk.nz), slice(g, g + blk.ny), slice(g, g + blk.nx)]
                sl[2 - d] = slice(g, g + (blk.nx, blk.ny, blk.nz)[d] + 1)
                errs.append(("B" + "xyz"[d], PM.rel_signed(gb[d][tuple(sl)], m.b0[j][d][tuple(sl)])))
            for name, e in errs:
                fields[name] = max(fields.get(name, 0.0), float(e))
        out[kind] = {"max_dev_D_over_block_max": worst_all, "max_rel_dev_D_star": worst_star,
                     "max_dev_by_field": fields, "max_dev_all_fields": max(fields.values())}
        log(f"c5 oracle check ({kind}): max |dD|/max D {worst_all:.2e}, star rel {worst_star:.2e}, "
            f"all fields {max(fields.values()):.2e} ({ {k: float('%.1e' % v) for k, v in fields.items()} })")
    out["oracle_s"] = el
    out["steps"] = len(sub["dts"])
    cells = sum(b.nx * b.ny * b.nz for b in sub["init"])
    out["oracle_zone_updates_per_s"] = cells * len(sub["dts"]) * len(meshes) / el
    log(f"c5 oracle: {len(sub['dts'])} steps of {len(sub['init'])} blocks in {el:.1f} s")
    return out


def _copy_np(b):
    import copy
    c = copy.copy(b)
    c.w = np.array(b.w)
    c.bf = [np.array(x) for x in b.bf]
    c.adm = np.array(b.adm)
    return c


def _eps_cold(rho, pp, K):
    """cold specific energy of the 3-piece polytrope (P and eps continuous at
    the dividing densities), for the exact labels of the hybrid states"""
    import torch
    G, rb = pp["Gam"], pp["rho_b"]
    a = [0.0]
    for i in (1, 2):
        pr = K[i - 1] * rb[i - 1] ** G[i - 1]
        a.append(a[-1] + pr / (rb[i - 1] * (G[i - 1] - 1.0)) - pr / (rb[i - 1] * (G[i] - 1.0)))
    e = [a[i] + K[i] * rho ** (G[i] - 1.0) / (G[i] - 1.0) for i in range(3)]
    return torch.where(rho < rb[0], e[0], torch.where(rho < rb[1], e[1], e[2]))


def c2p_section(args, torch, inputs, lib, eos="ideal"):
    """C2P solves/s on 2^k random states, plain vs learned bracket; eos
    'ideal' (Gamma = 5/3, the benchmark states) or 'hybrid' (the end-to-end
    piecewise polytrope, densities up to 10^-2.9 where it stays causal)"""
    n = 1 << args.c2p_log2
    kw = {}
    if eos == "ideal":
        p = lib.MethodParams(**C2P_PARAMS)
    else:
        pp, pK = inputs.pp_eos()
        p = lib.MethodParams(**{**C2P_PARAMS, **pp})
        kw = dict(pp=pp, pp_K=pK, log_rho=(-10.0, -2.9))
    log(f"c2p ({eos}): {n} states")
    s = inputs.c2p_states_torch(n, seed_offset=3, device="cuda", **kw)
    u0 = lib.prim2con(s["w"], s["bt"], s["gam"], p)
    if eos == "ideal":
        eps = s["w"][4] / ((C2P_PARAMS["gamma"] - 1.0) * s["w"][0])
    else:
        eps = _eps_cold(s["w"][0], pp, pK) + s["eps"]
    mu_exact = 1.0 / ((1.0 + eps + s["w"][4] / s["w"][0]) * s["W"])
    # train the guess network on separate states (own forward/backward kernels)
    t0 = time.perf_counter()
    tr = inputs.c2p_states_torch(1 << 18, seed_offset=300, device="cuda", **kw)
    ut = lib.prim2con(tr["w"], tr["bt"], tr["gam"], p)
    net = lib.LearnedC2P(seed=0)
    steps = args.train_steps
    losses = net.fit(ut, tr["bt"], tr["gam"], p, tr["w"], steps=steps, log_every=max(1, steps // 4))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"trained {steps} steps in {train_s:.1f} s, losses {['%.3g' % x for x in losses]}, "
        f"bracket width factor {net.width_k:.3g}")
    res = {}
    ws = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    for kind in ("plain", "learned", "learned_split"):
        times = []
        for rep in range(args.c2p_reps + 1):
            if rep == 1:
                lib.timing(True)
            u = u0.clone()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            if kind == "plain":
                out = lib.c2p_batch(u, s["bt"], s["gam"], p, want_mu=True, want_nev=True, stats=True)
            else:
                # learned: the fused kernel (network + root solve in one pass);
                # learned_split: bracket kernel, then the plain kernel reading it
                out = lib.c2p_batch_learned(u, s["bt"], s["gam"], p, net, want_mu=True, want_nev=True,
                                            stats=True, split=(kind == "learned_split"), workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            if rep > 0:
                times.append(e0.elapsed_time(e1))
        kt = lib.timing_read()
        lib.timing(False)
        ms = sorted(times)[len(times) // 2]
        err = ((out["mu"] - mu_exact).abs() / mu_exact).max().item()
        stt = out["stats"].cpu().tolist()
        res[kind] = {"solves_per_s": n / (ms * 1e-3), "ms": ms, "max_mu_rel_err": err,
                     "mean_master_evals": stt[1] / stt[0], "fallback_rate": stt[2] / stt[0],
                     "unrecovered_failures": int(stt[3]),
                     "kernel_ms": {k: v[0] / v[1] for k, v in kt.items() if v[1]}}
        log(f"c2p ({eos}) {kind}: {res[kind]['solves_per_s']:.3e} solves/s, err {err:.2e}, "
            f"evals {res[kind]['mean_master_evals']:.2f}, fallback {res[kind]['fallback_rate']:.4f}, "
            f"kernels {res[kind]['kernel_ms']}")
    res["eos"] = eos
    res["states"] = n
    res["train_steps"] = steps
    res["bracket_width_k"] = net.width_k
    res["train_s"] = train_s
    res["learned_speedup"] = res["learned"]["solves_per_s"] / res["plain"]["solves_per_s"]
    res["bytes_per_solve"] = 153
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the star workload is 20 RK2 steps (after the warm-up steps)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--blocks-per-side", type=int, default=4)
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--c2p-log2", type=int, default=24)
    ap.add_argument("--c2p-reps", type=int, default=3)
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--no-c2p", action="store_true")
    ap.add_argument("--c2p-only", action="store_true", help="only the C2P solves/s section")
    ap.add_argument("--no-refined", action="store_true")
    ap.add_argument("--refined-only", action="store_true", help="only the refined-mesh section")
    ap.add_argument("--refined-blocks", type=int, default=1500)
    ap.add_argument("--refined-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the end-to-end refined star section")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default workgroup size (256) for the star instead of autotuning it")
    ap.add_argument("--threads", default="",
                    help="fixed star workgroup sizes instead of autotuning, e.g. update=512,flux_x=64")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the reconstruction / RK3 / matter-source measurements on the star")
    ap.add_argument("--c5-only", action="store_true", help="only the end-to-end section (+ its oracle check)")
    ap.add_argument("--c5-steps", type=int, default=100)
    ap.add_argument("--c5-check-steps", type=int, default=2,
                    help="steps of the refined-mesh oracle check (whole 8^3-block mesh)")
    ap.add_argument("--c5-frozen", action="store_true",
                    help="also the end-to-end run on the independent block list with frozen ghosts")
    ap.add_argument("--host-inputs", action="store_true",
                    help="build the star's initial data on the host (counter passes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB plain copy first (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the stage would shard by MeshBlocks, with a halo exchange per stage)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_10384_amd import inputs, lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lib.load()
    if args.calibrate_copy:
        # one plain copy of known size, for scaling hardware traffic counters
        n = 1 << 27
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        lib.copy(a, b)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 8} bytes read, {n * 8} bytes written")
        del a, b
    if args.c2p_only:
        print(json.dumps({"c2p": c2p_section(args, torch, inputs, lib),
                          "c2p_hybrid_eos": c2p_section(args, torch, inputs, lib, eos="hybrid")}),
              flush=True)
        return
    if args.refined_only:
        print(json.dumps({"refined": refined_section(args, torch, inputs, lib)}), flush=True)
        return
    if args.c5_only:
        res, sub = c5_section(args, torch, inputs, lib, amr=not args.c5_frozen)
        if not args.no_cpu_baseline:
            res["oracle_check"] = c5_oracle_check(sub)
        print(json.dumps({"end_to_end": res}), flush=True)
        return
    star = star_section(args, torch, inputs, lib)
    out = {
        "metric": "zone-updates/s per GPU (GRMHD SSP-RK2 step, plain C2P)",
        "value": star["value"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": star["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"star {args.blocks_per_side * args.block}^3 as "
                               f"{args.blocks_per_side ** 3} MeshBlocks of {args.block}^3 (+3 ghosts), "
                               f"Gamma=2, WENOZ+HLLE, FOFC+DMP M=1.1, SSP-RK2 CFL 0.25",
                   "cells": star["ncell"], "workgroup_sizes": star["workgroup_sizes"]},
        "roofline": star["path"],
        "kernel_roofline": star["roofline"],
        "fp64_rate": star["fp64"],
        "kernel_breakdown": star["breakdown"],
        "variants": star["variants"],
    }
    if not args.no_refined:
        out["refined"] = refined_section(args, torch, inputs, lib)
    if not args.no_c2p:
        out["c2p"] = c2p_section(args, torch, inputs, lib)
        out["c2p_hybrid_eos"] = c2p_section(args, torch, inputs, lib, eos="hybrid")
    c5_sub = c5f_sub = None
    if not args.no_c5:
        out["end_to_end"], c5_sub = c5_section(args, torch, inputs, lib, amr=True)
        if args.c5_frozen:
            out["end_to_end_frozen"], c5f_sub = c5_section(args, torch, inputs, lib, amr=False)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(star["st"], args.blocks_per_side, args.block, STAR_PARAMS)
        if c5_sub is not None:
            out["end_to_end"]["oracle_check"] = c5_oracle_check(c5_sub)
        if c5f_sub is not None:
            out["end_to_end_frozen"]["oracle_check"] = c5_oracle_check(c5f_sub)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

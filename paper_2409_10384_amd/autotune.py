"""Workgroup-size autotuner for the stage kernels.

Every stage kernel walks a flattened list of 64-item waves (cells or faces,
x fastest), so its workgroup size is the length of the x-pencil a workgroup
covers: 64, 128, 256 or 512 consecutive items.  The tuner times each kernel
family of the stage at each size on the actual block list (HIP events inside
the library) and keeps the fastest; results apply to the running process.
"""
from __future__ import annotations

import json

from . import lib

# kernel families of one stage (grmhd_timing numbering)
TUNABLE = {"flux_x": 0, "flux_y": 1, "flux_z": 2, "fofc_flags": 3, "fofc_fix": 4, "ct": 5,
           "update": 6, "stage_c2p": 7}
SIZES = (64, 128, 256, 512)


def set_threads(family: str, threads: int):
    lib.check(lib.load().grmhd_set_threads(TUNABLE[family], threads), "grmhd_set_threads")


def time_stage(mesh: "lib.DeviceMesh", dt: float, reps: int = 2):
    """per-family ms of stage 1 (inputs are not modified by stage 1)"""
    import torch
    mesh.stage(1, dt=dt)             # warm
    torch.cuda.synchronize()
    lib.timing(True)
    for _ in range(reps):
        mesh.stage(1, dt=dt)
    torch.cuda.synchronize()
    t = lib.timing_read()
    lib.timing(False)
    return {k: v[0] / v[1] for k, v in t.items()}


def autotune(mesh: "lib.DeviceMesh", dt: float, families=None, sizes=SIZES, log=None):
    """choose the fastest workgroup size per family; returns
    {family: {"best": size, "ms": {size: ms}}}"""
    families = families or list(TUNABLE)
    result = {}
    for fam in families:
        ms = {}
        for th in sizes:
            set_threads(fam, th)
            ms[th] = time_stage(mesh, dt)[fam]
        best = min(ms, key=ms.get)
        set_threads(fam, best)
        result[fam] = {"best": best, "ms": ms}
        if log:
            log(f"autotune {fam}: " + ", ".join(f"{k}:{v:.3f}" for k, v in ms.items()) + f" -> {best}")
    return result


def reset():
    for fam in TUNABLE:
        set_threads(fam, 256)


def dumps(result) -> str:
    return json.dumps({k: v["best"] for k, v in result.items()})

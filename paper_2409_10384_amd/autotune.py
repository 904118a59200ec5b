"""Workgroup-size autotuner for the stage kernels.

Every stage kernel walks a flattened list of 64-item waves (cells or faces,
x fastest), so its workgroup size is the length of the x-pencil a workgroup
covers: 64, 128, 256 or 512 consecutive items (for the update, 512 selects
the 2-row x 4-plane brick tile where the blocks allow it).  The tuner lives
in the library (grmhd_autotune): it times each kernel family of the stage at
each size on the actual block list (HIP events inside the library) and keeps
the fastest; results apply to the running process.
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


def autotune(mesh: "lib.DeviceMesh", dt: float, reps: int = 2, log=None):
    """the library's autotuner (grmhd_autotune) on the mesh's first stage:
    the fastest workgroup size per family is kept for the process; returns
    {family: {"best": size, "ms": {size: ms}}}"""
    res = mesh.autotune(dt, reps=reps)
    out = {}
    for fam, (best, ms) in res.items():
        out[fam] = {"best": best, "ms": ms}
        if log:
            log(f"autotune {fam}: " + ", ".join(f"{k}:{v:.3f}" for k, v in ms.items()) + f" -> {best}")
    return out


def reset():
    for fam in TUNABLE:
        set_threads(fam, 256)


def dumps(result) -> str:
    return json.dumps({k: v["best"] for k, v in result.items()})

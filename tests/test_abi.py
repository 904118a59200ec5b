"""The C-ABI library loads on the CPU, exports every function that
include/grmhd.h declares, and its struct sizes match the Python binding.
No compute call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grmhd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*\b([a-z_][a-z_0-9]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("sizeof",)))


def test_header_declares_the_stage_entry_points():
    names = declared_functions()
    for n in ("grmhd_stage", "c2p_batch", "fofc_correct", "ct_update"):
        assert n in names
    assert len(names) >= 20, names


def test_library_exports_every_declared_symbol():
    from paper_2409_10384_amd import lib
    L = lib.load()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_binding():
    from paper_2409_10384_amd import lib
    L = lib.load()
    L.grmhd_struct_size.restype = ctypes.c_int32
    assert L.grmhd_struct_size(0) == ctypes.sizeof(lib.GrmhdParams)
    assert L.grmhd_struct_size(1) == ctypes.sizeof(lib.GrmhdBlock)
    assert L.grmhd_struct_size(2) == ctypes.sizeof(lib.C2PMlp)
    assert L.grmhd_struct_size(3) == ctypes.sizeof(lib.C2PStats)
    assert L.grmhd_struct_size(9) == -1


def test_host_side_argument_checks_reject_bad_input():
    """argument errors return GRMHD_EINVAL before anything is enqueued"""
    from paper_2409_10384_amd import lib
    L = lib.load()
    p = lib.MethodParams().c()
    assert L.grmhd_stage(None, None, 0, ctypes.byref(p), None, 0.0, 0.0, 1.0, 1.0, None) == -1
    bad = lib.MethodParams(recon=7).c()
    blk = (lib.GrmhdBlock * 1)()
    assert L.grmhd_stage(ctypes.cast(blk, ctypes.c_void_p), ctypes.c_void_p(1), 1, ctypes.byref(bad),
                         None, 0.0, 0.0, 1.0, 1.0, None) == -3
    assert L.grmhd_scratch_doubles(0, 4, 4, 3) == -1
    assert L.grmhd_flux_offset(8, 8, 8, 3, 3, 0) == -1
    # scratch layout: 21 face arrays + 6 cell arrays + 3 edge arrays + 2 bracket
    # arrays + the FOFC cell list ((n+2)^3 int32 after an 8-byte counter)
    n, g = 8, 3
    s = n + 2 * g
    expect = 7 * 3 * (s + 1) * s * s + 6 * s ** 3 + 3 * (s + 1) ** 3 + 2 * s ** 3 + \
        ((n + 2) ** 3 + 3) // 2
    assert L.grmhd_scratch_doubles(n, n, n, g) == expect


def _shape_items(nx, ny, nz, g, cls):
    n = (nx, ny, nz)
    s = tuple(v + 2 * g for v in n)
    if cls == 0:
        return s[0] * s[1] * s[2]
    if cls == 1:
        return nx * ny * nz
    if cls == 2:
        return (nx + 2) * (ny + 2) * (nz + 2)
    c = 1
    if 3 <= cls <= 5:
        for a in range(3):
            c *= n[a] + 1 if a == cls - 3 else n[a] + 2
    elif 6 <= cls <= 8:
        for a in range(3):
            c *= n[a] if a == cls - 6 else n[a] + 1
    elif 9 <= cls <= 11:
        for a in range(3):
            c *= n[a] + 1 if a == cls - 9 else n[a]
    else:
        d = cls - 12
        for a in range(3):
            c *= s[a] + (1 if a == d else 0)
    return c


def test_launch_layout_covers_every_item_once():
    """grmhd_blocks_prepare (host code of the library) + an emulation of the
    device-side wave -> (block, item) search, over a mixed block list"""
    import numpy as np
    from paper_2409_10384_amd import lib
    L = lib.load()
    rng = np.random.default_rng(0)
    sizes = [16, 24, 32, 5, 3]
    nb = 37
    arr = (lib.GrmhdBlock * nb)()
    dims = []
    for i in range(nb):
        n = [int(rng.choice(sizes)) for _ in range(3)]
        arr[i].nx, arr[i].ny, arr[i].nz, arr[i].ng = n[0], n[1], n[2], 3
        dims.append(n)
    assert L.grmhd_blocks_prepare(ctypes.cast(arr, ctypes.c_void_p), nb) == 0
    for cls in range(15):
        wave0 = [arr[i].wave0[cls] for i in range(nb)]
        assert arr[0].nblk == nb
        items = [_shape_items(*dims[i], 3, cls) for i in range(nb)]
        total_waves = wave0[-1] + (items[-1] + 63) // 64
        seen = [np.zeros(it, dtype=np.int32) for it in items]
        for threads in (64, 256, 512):
            for s in seen:
                s[:] = 0
            nwg = (total_waves * 64 + threads - 1) // threads
            for L_ in range(nwg):       # every workgroup, through the XCD renumbering
                x, i = L_ % 8, L_ // 8
                q, r = divmod(nwg, 8)
                lp = (x * (q + 1) if x < r else r * (q + 1) + (x - r) * q) + i
                for lane0 in range(0, threads, 64):
                    w = (lp * threads + lane0) >> 6
                    b = max(k for k in range(nb) if wave0[k] <= w)
                    if b == nb - 1 and w >= wave0[-1] + (items[-1] + 63) // 64:
                        continue
                    t0 = (w - wave0[b]) * 64
                    t = np.arange(t0, t0 + 64)
                    t = t[t < items[b]]
                    seen[b][t] += 1
            for s in seen:
                assert np.all(s == 1), cls



def test_bench_refuses_more_than_one_gpu():
    """the benchmark measures one GPU: --gpus above 1 exits with a message
    (before touching torch or the GPU)"""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr

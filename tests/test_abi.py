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


def test_empty_batches_are_valid_calls():
    """n = 0 returns GRMHD_OK before anything else is looked at (an empty
    tensor's pointers may be NULL); n < 0 is GRMHD_EINVAL.  Nothing is
    launched either way, so no GPU is needed"""
    from paper_2409_10384_amd import lib
    L = lib.load()
    p = lib.MethodParams().c()
    N = None
    assert L.c2p_batch(0, N, N, N, N, N, ctypes.byref(p), N, N, N, N, N) == 0
    assert L.prim2con(0, N, N, N, N, ctypes.byref(p), N) == 0
    assert L.grmhd_copy(N, N, 0, N) == 0
    assert L.c2p_batch(-1, N, N, N, N, N, ctypes.byref(p), N, N, N, N, N) == -1
    assert L.prim2con(-1, N, N, N, N, ctypes.byref(p), N) == -1
    assert L.grmhd_copy(N, N, -1, N) == -1
    # with n > 0 the missing arrays are refused
    assert L.c2p_batch(4, N, N, N, N, N, ctypes.byref(p), N, N, N, N, N) == -1
    assert L.grmhd_copy(N, N, 4, N) == -1


def test_pointwise_block_calls_reject_missing_arrays():
    """grmhd_mass, grmhd_dt and grmhd_prim2con_blocks check the arrays their
    kernels read before launching anything (no GPU is touched)"""
    from paper_2409_10384_amd import lib
    L = lib.load()
    p = lib.MethodParams().c()
    arr = (lib.GrmhdBlock * 1)()
    arr[0].nx = arr[0].ny = arr[0].nz = 4
    arr[0].ng = 3
    assert L.grmhd_blocks_prepare(ctypes.cast(arr, ctypes.c_void_p), 1) == 0
    h, d = ctypes.cast(arr, ctypes.c_void_p), ctypes.c_void_p(8)
    one = ctypes.c_void_p(16)
    # no us[0]
    assert L.grmhd_mass(h, d, 1, one, one, None) == -1
    # no w / bs / metric
    assert L.grmhd_dt(h, d, 1, ctypes.byref(p), 0.25, one, one, None) == -1
    for v in range(5):
        arr[0].w[v] = 64
    assert L.grmhd_dt(h, d, 1, ctypes.byref(p), 0.25, one, one, None) == -1
    for v in range(3):
        arr[0].bs[v] = 64
    assert L.grmhd_dt(h, d, 1, ctypes.byref(p), 0.25, one, one, None) == -1
    assert L.grmhd_prim2con_blocks(h, d, 1, ctypes.byref(p), None) == -1
    # NULL outputs
    arr[0].us[0] = 64
    assert L.grmhd_mass(h, d, 1, None, one, None) == -1
    assert L.grmhd_dt(h, d, 1, ctypes.byref(p), 0.25, None, one, None) == -1
    assert L.grmhd_dt(h, d, 1, ctypes.byref(p), 0.0, one, one, None) == -1
    # a stale layout (block 0 resized after prepare, so block 1's first waves
    # no longer follow) is refused, with every array present
    two = (lib.GrmhdBlock * 2)()
    for b in two:
        b.nx = b.ny = b.nz = 4
        b.ng = 3
        b.us[0] = 64
    assert L.grmhd_blocks_prepare(ctypes.cast(two, ctypes.c_void_p), 2) == 0
    two[0].nx = 5
    assert L.grmhd_mass(ctypes.cast(two, ctypes.c_void_p), d, 2, one, one, None) == -1


def _shape_items(nx, ny, nz, g, cls):
    n = (nx, ny, nz)
    s = tuple(v + 2 * g for v in n)
    if cls == 20:   # cell corners [g, g+n]^3 (CT)
        return (nx + 1) * (ny + 1) * (nz + 1)
    if cls == 15:   # ghost cells
        return s[0] * s[1] * s[2] - nx * ny * nz
    if cls == 16:   # first ghost shell
        return (nx + 2) * (ny + 2) * (nz + 2) - nx * ny * nz
    if 17 <= cls <= 19:   # ghost faces
        d = cls - 17
        pad = inner = 1
        for a in range(3):
            pad *= s[a] + (1 if a == d else 0)
            inner *= n[a] + (1 if a == d else 0)
        return pad - inner
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
    L.grmhd_launch_shapes.restype = ctypes.c_int32
    nshape = L.grmhd_launch_shapes()
    assert nshape == 21 and nshape <= len(arr[0].wave0)
    for cls in range(nshape):
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



def test_prepare_writes_only_the_layout_fields():
    """grmhd_blocks_prepare writes wave0, nblk and reserved of each
    descriptor and nothing else: every other byte of the table, the next
    descriptor's sizes included, is unchanged (a layout with more launch
    shapes than wave0 slots would spill into nblk and the next block)"""
    import numpy as np
    from paper_2409_10384_amd import lib
    L = lib.load()
    nb = 5
    arr = (lib.GrmhdBlock * nb)()
    rng = np.random.default_rng(3)
    for i in range(nb):
        arr[i].nx, arr[i].ny, arr[i].nz = (int(x) for x in rng.integers(1, 40, 3))
        arr[i].ng = 3
        arr[i].dx = (ctypes.c_double * 3)(0.1 * i, 0.2, 0.3)
        arr[i].flags = 1000 + i
        arr[i].scratch = 2000 + i
        arr[i].nbr = (ctypes.c_int32 * 27)(*[(i + k) % nb for k in range(27)])
        arr[i].bc = 1
        for s in range(len(arr[i].wave0)):
            arr[i].wave0[s] = -7
        arr[i].nblk = -7
        arr[i].reserved = -7
    before = bytearray(memoryview(arr).cast("B"))
    assert L.grmhd_blocks_prepare(ctypes.cast(arr, ctypes.c_void_p), nb) == 0
    after = bytearray(memoryview(arr).cast("B"))
    size = ctypes.sizeof(lib.GrmhdBlock)
    off_w = lib.GrmhdBlock.wave0.offset
    end_w = lib.GrmhdBlock.reserved.offset + 4
    for i in range(nb):
        b0, a0 = before[i * size:(i + 1) * size], after[i * size:(i + 1) * size]
        assert b0[:off_w] == a0[:off_w]
        assert b0[end_w:] == a0[end_w:]
        assert arr[i].nblk == nb and arr[i].reserved == 0
        L.grmhd_launch_shapes.restype = ctypes.c_int32
        ns = L.grmhd_launch_shapes()
        assert all(arr[i].wave0[s] == 0 for s in range(ns, len(arr[i].wave0)))
        assert arr[0].wave0[0] == 0


_RING_HARNESS = r"""
#include "blocks.hpp"
#include <cstdio>
#include <vector>
// every item of the ghost launch shapes lies in the padded range, is a
// ghost entry, and every ghost entry is reached exactly once
int main() {
  const int sizes[][3] = {{1, 1, 1}, {2, 5, 3}, {3, 3, 3}, {5, 6, 7}, {16, 16, 16}, {64, 4, 2}};
  int bad = 0;
  for (auto& n : sizes) {
    gk::Geo q;
    q.nx = n[0]; q.ny = n[1]; q.nz = n[2]; q.g = 3;
    q.sx = q.nx + 6; q.sy = q.ny + 6; q.sz = q.nz + 6;
    for (int cls = gk::S_GCELLS; cls <= gk::S_GZFACE; ++cls) {
      const gk::Ring r = gk::ghost_ring(q, cls);
      const int d = cls - gk::S_GXFACE;
      const bool face = cls >= gk::S_GXFACE;
      int e[3], lo[3], hi[3];   // box of the items; interior [lo, hi]
      for (int a = 0; a < 3; ++a) {
        const int f = face && a == d ? 1 : 0;
        const int na = a == 0 ? q.nx : a == 1 ? q.ny : q.nz;
        if (cls == gk::S_GSHELL) { e[a] = na + 2; lo[a] = 1; hi[a] = na; }
        else { e[a] = na + 6 + f; lo[a] = 3; hi[a] = 3 + na - 1 + f; }
      }
      std::vector<int> seen((size_t)e[0] * e[1] * e[2], 0);
      if (r.size() != gk::shape_items(q, cls)) ++bad;
      for (int64_t t = 0; t < r.size(); ++t) {
        int i, j, k;
        r.at(t, i, j, k);
        if (i < 0 || j < 0 || k < 0 || i >= e[0] || j >= e[1] || k >= e[2]) { ++bad; continue; }
        const bool in = i >= lo[0] && i <= hi[0] && j >= lo[1] && j <= hi[1] && k >= lo[2] && k <= hi[2];
        if (in) ++bad;
        seen[((size_t)k * e[1] + j) * e[0] + i] += 1;
      }
      for (int k = 0; k < e[2]; ++k)
        for (int j = 0; j < e[1]; ++j)
          for (int i = 0; i < e[0]; ++i) {
            const bool in = i >= lo[0] && i <= hi[0] && j >= lo[1] && j <= hi[1] && k >= lo[2] && k <= hi[2];
            if (seen[((size_t)k * e[1] + j) * e[0] + i] != (in ? 0 : 1)) ++bad;
          }
    }
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
"""


def test_ghost_launch_shapes_cover_each_ghost_once(tmp_path):
    """the ghost-only launch shapes (host build of the same header): each
    item is an in-range ghost cell or face, each ghost reached once"""
    import subprocess
    src = tmp_path / "ring.cpp"
    src.write_text(_RING_HARNESS)
    exe = tmp_path / "ring"
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2409_10384_amd", "csrc"),
                           str(src), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr


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

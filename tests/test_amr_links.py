"""The library's host-side links of a refined mesh (grmhd_amr_links): the
leaves named for each neighbour region of a block, and the meshes it
refuses (no GPU involved)."""
import ctypes as C

import pytest

from paper_2409_10384_amd import inputs, lib


def _links(m, nb=8, ng=3):
    return lib.amr_links(m.levels, [m.org(i) for i in range(len(m.leaves))], nb, ng, m.n0, m.periodic)


def _dir(ox, oy, oz):
    return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)


def test_links_of_a_two_level_mesh():
    m = inputs.leaf_mesh((2, 2, 2), 8, refine=lambda lv, b: lv == 0 and b == (0, 0, 0), max_level=1)
    L = _links(m)
    where = {lf: i for i, lf in enumerate(m.leaves)}
    # the coarse leaf at (1, 0, 0): its -x face region holds the 4 fine leaves
    # of the refined block's upper x half, its +x face region (across the
    # periodic boundary) the 4 of its lower x half; the self entry is itself
    c = where[(0, (1, 0, 0))]
    lk = L[c]
    assert lk.level == 0 and tuple(lk.org) == (8, 0, 0) and tuple(lk.N) == (16, 16, 16)
    assert lk.periodic == 7
    assert lk.rel[_dir(0, 0, 0)] == 0 and lk.src[_dir(0, 0, 0)][0] == c
    fine_x = sorted(x for x in lk.src[_dir(-1, 0, 0)] if x >= 0)
    assert lk.rel[_dir(-1, 0, 0)] == 1
    assert fine_x == sorted(where[(1, (1, j, k))] for j in (0, 1) for k in (0, 1))
    assert lk.rel[_dir(1, 0, 0)] == 1
    assert sorted(x for x in lk.src[_dir(1, 0, 0)] if x >= 0) == sorted(
        where[(1, (0, j, k))] for j in (0, 1) for k in (0, 1))
    assert lk.rel[_dir(0, 1, 0)] == 0 and lk.src[_dir(0, 1, 0)][0] == where[(0, (1, 1, 0))]
    # the coarse leaf at (1, 1, 0): its -x,-y edge region holds 2 fine leaves;
    # the one at (1, 1, 1): its -x,-y,-z corner region 1
    lk = L[where[(0, (1, 1, 0))]]
    e = [x for x in lk.src[_dir(-1, -1, 0)] if x >= 0]
    assert lk.rel[_dir(-1, -1, 0)] == 1 and sorted(e) == sorted(where[(1, (1, 1, k))] for k in (0, 1))
    lk = L[where[(0, (1, 1, 1))]]
    corner = [x for x in lk.src[_dir(-1, -1, -1)] if x >= 0]
    assert lk.rel[_dir(-1, -1, -1)] == 1 and corner == [where[(1, (1, 1, 1))]]
    # a fine leaf: its +x region is fine (same level), its -x region coarse
    f = where[(1, (1, 0, 0))]
    lf = L[f]
    assert lf.level == 1 and tuple(lf.N) == (32, 32, 32)
    assert lf.rel[_dir(1, 0, 0)] == -1 and lf.src[_dir(1, 0, 0)][0] == c
    assert lf.rel[_dir(-1, 0, 0)] == 0 and lf.src[_dir(-1, 0, 0)][0] == where[(1, (0, 0, 0))]


def test_outflow_regions_are_marked():
    m = inputs.leaf_mesh((2, 2, 2), 8, periodic=(0, 1, 1))
    L = _links(m)
    lo = L[0]     # the leaf at (0, 0, 0)
    assert lo.rel[_dir(-1, 0, 0)] == -9 and lo.rel[_dir(-1, 1, 1)] == -9
    assert lo.rel[_dir(0, -1, 0)] == 0


def _call(levels, orgs, nb=8, ng=3, n0=(16, 16, 16), periodic=(1, 1, 1)):
    n = len(levels)
    out = (lib.GrmhdAmrLink * n)()
    return lib.load().grmhd_amr_links(n, C.cast((C.c_int32 * n)(*levels), C.c_void_p),
                                      C.cast((C.c_int32 * (3 * n))(*[x for o in orgs for x in o]), C.c_void_p),
                                      nb, ng, C.cast((C.c_int32 * 3)(*n0), C.c_void_p),
                                      C.cast((C.c_int32 * 3)(*periodic), C.c_void_p), out)


def test_meshes_that_are_refused():
    m = inputs.leaf_mesh((2, 2, 2), 8)
    lv, og = m.levels, [m.org(i) for i in range(8)]
    assert _call(lv, og) == 0
    assert _call(lv, og, nb=7) != 0                      # odd block size
    assert _call(lv, og, nb=6) != 0                      # smaller than 2 ng + 2
    assert _call(lv[:7], og[:7]) != 0                    # a hole
    assert _call(lv + [0], og + [og[0]]) != 0            # overlapping leaves
    assert _call(lv, [(1, 0, 0)] + og[1:]) != 0          # off the block lattice
    # a level jump of two across a face: refine one leaf twice without balance
    fine = [(2, (x, y, z)) for x in range(4) for y in range(4) for z in range(4)]
    leaves = [(0, b) for (_, b) in m.leaves if b != (0, 0, 0)] + fine
    assert _call([l for l, _ in leaves], [tuple(8 * c for c in b) for _, b in leaves]) != 0

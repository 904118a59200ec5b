"""The oracle's inter-level transfer on refined meshes (block-based mesh
refinement, Sec. I; prolongation and restriction, Sec. V-A), pinned by what
the mathematics fixes:

* a mesh whose leaves are all on one level reproduces the single-level mesh
  with neighbour tables bit for bit (copies are the only transfer);
* linear data are reproduced exactly in every ghost cell and ghost face by
  copy, restriction and prolongation (each index, child offset and slope
  direction enters), and a parent at an extremum gives its children its own
  value (the minmod limiter);
* restriction of a prolongation is the identity: the 8 prolonged children
  average to their parent, the 4 prolonged faces on a parent face are that
  face, and a prolonged ghost cell has its parent's divergence;
* a two-level stage conserves every conserved total to round-off (flat
  metric), keeps div B~ at round-off in every cell of every leaf, and keeps
  each coarse face on a level boundary equal to the mean of the fine faces;
  with the flux (or the EMF) correction switched off these break;
* a uniform state stays uniform across levels."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2409_10384_amd import inputs

LOW = lambda lv, b: lv == 0 and b == (0, 0, 0)


def _two_level(nb=8, periodic=(1, 1, 1), refine=LOW, max_level=1, **kw):
    m = inputs.leaf_mesh((2, 2, 2), nb, refine=refine, max_level=max_level, periodic=periodic)
    return m, inputs.smooth_leaf_blocks(m, **kw)


def _nbr_tables(m, blocks):
    """neighbour tables of a mesh whose leaves are all on one level"""
    lv = m.leaves[0][0]
    nbk = [n << lv for n in m.nblocks0]
    where = {b: i for i, (_, b) in enumerate(m.leaves)}
    for i, (_, b) in enumerate(m.leaves):
        tab = []
        for oz in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    q = [b[0] + ox, b[1] + oy, b[2] + oz]
                    ok = True
                    for a in range(3):
                        if q[a] < 0 or q[a] >= nbk[a]:
                            if m.periodic[a]:
                                q[a] %= nbk[a]
                            else:
                                ok = False
                    tab.append(where[tuple(q)] if ok else -1)
        blocks[i].nbr = tab


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 1, 0)])
def test_one_level_leaf_mesh_is_the_neighbour_table_mesh(periodic):
    m = inputs.leaf_mesh((2, 2, 2), 8, periodic=periodic)
    blocks = inputs.smooth_leaf_blocks(m)
    _nbr_tables(m, blocks)
    p = O.Params(gamma=5.0 / 3.0, fofc=1, dmp_M=1.0)
    ref = O.Mesh(copy.deepcopy(blocks), p)
    amr = O.RefinedMesh(copy.deepcopy(blocks), p, m)
    ref.ghost_fill_state(0)
    amr.ghost_fill_state(0)
    for ib in range(len(blocks)):
        np.testing.assert_array_equal(ref.w0[ib], amr.w0[ib])
        for d in range(3):
            np.testing.assert_array_equal(ref.b0[ib][d], amr.b0[ib][d])
    dt = ref.dt(0.3)
    assert amr.dt(0.3) == dt
    for _ in range(2):
        ref.rk2_step(dt)
        amr.rk2_step(dt)
    assert any(np.any(f & O.F_DMP) for f in ref.flags)
    for ib in range(len(blocks)):
        np.testing.assert_array_equal(ref.u0[ib], amr.u0[ib])
        np.testing.assert_array_equal(ref.w0[ib], amr.w0[ib])
        for d in range(3):
            np.testing.assert_array_equal(ref.b0[ib][d], amr.b0[ib][d])


def _cell_xyz(b, ib, m, h0):
    lv = m.leaves[ib][0]
    h = h0 / 2 ** lv
    o = m.org(ib)
    c = [(o[a] - b.ng + np.arange(b.shape[2 - a]) + 0.5) * h for a in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return X, Y, Z


def _face_x(b, ib, m, h0, d):
    """coordinate along d of every face of direction d (broadcast shape)"""
    lv = m.leaves[ib][0]
    h = h0 / 2 ** lv
    o = m.org(ib)
    n = b.shape[2 - d] + 1
    x = (o[d] - b.ng + np.arange(n)) * h
    shp = [1, 1, 1]
    shp[2 - d] = n
    return x.reshape(shp)


def _ghost_mask(b):
    g = b.ng
    msk = np.ones(b.shape, dtype=bool)
    msk[g:g + b.nz, g:g + b.ny, g:g + b.nx] = False
    return msk


def _face_ghost_mask(b, d):
    g = b.ng
    shp = list(b.shape)
    shp[2 - d] += 1
    msk = np.ones(shp, dtype=bool)
    sl = [slice(g, g + b.nz), slice(g, g + b.ny), slice(g, g + b.nx)]
    sl[2 - d] = slice(g, g + [b.nx, b.ny, b.nz][d] + 1)
    msk[tuple(sl)] = False
    return msk


@pytest.mark.parametrize("max_level", [1, 2])
def test_ghost_fill_is_exact_for_linear_data(max_level):
    """outflow mesh of 4^3 level-0 blocks refined inside (so no parent's
    slope reaches the domain boundary, where outflow ghosts are constant);
    ghosts inside the domain are checked.  Every cell field a different
    linear function, each face field linear along its normal."""
    refine = lambda lv, b: b == (1, 1, 1) or (lv == 1 and b == (3, 3, 3))
    m = inputs.leaf_mesh((4, 4, 4), 8, refine=refine, max_level=max_level, periodic=(0, 0, 0))
    blocks = inputs.smooth_leaf_blocks(m)
    assert len(set(m.levels)) == max_level + 1
    om = O.RefinedMesh(blocks, O.Params(gamma=5.0 / 3.0), m)
    h0 = 1.0 / 32
    coef = np.random.default_rng(1).uniform(-1.0, 1.0, size=(10, 4))
    fc = np.random.default_rng(2).uniform(-1.0, 1.0, size=(3, 2))
    lin = lambda c, X, Y, Z: c[0] + c[1] * X + c[2] * Y + c[3] * Z
    for ib, b in enumerate(om.blocks):
        X, Y, Z = _cell_xyz(b, ib, m, h0)
        gm = _ghost_mask(b)
        for v in range(5):
            om.w0[ib][v] = np.where(gm, np.nan, lin(coef[v], X, Y, Z))
            om.u0[ib][v] = np.where(gm, np.nan, lin(coef[5 + v], X, Y, Z))
        for d in range(3):
            fm = _face_ghost_mask(b, d)
            om.b0[ib][d][...] = np.where(fm, np.nan, fc[d, 0] + fc[d, 1] * _face_x(b, ib, m, h0, d))
    om.ghost_fill_state(0)
    checked = 0
    for ib, b in enumerate(om.blocks):
        X, Y, Z = _cell_xyz(b, ib, m, h0)
        inside = (X > 0) & (X < 1) & (Y > 0) & (Y < 1) & (Z > 0) & (Z < 1)
        sel = _ghost_mask(b) & inside
        checked += int(sel.sum())
        for v in range(5):
            for got, c in ((om.w0[ib][v], coef[v]), (om.u0[ib][v], coef[5 + v])):
                ref = lin(c, X, Y, Z)
                np.testing.assert_allclose(got[sel], ref[sel], rtol=0, atol=1e-14)
        for d in range(3):
            xf = np.broadcast_to(_face_x(b, ib, m, h0, d), om.b0[ib][d].shape)
            # face positions: along d from xf, across d the cell centres
            shp = om.b0[ib][d].shape
            ins = (xf >= 0) & (xf <= 1)
            # across-d positions
            lv = m.leaves[ib][0]
            h = h0 / 2 ** lv
            o = m.org(ib)
            for a in range(3):
                if a == d:
                    continue
                n = shp[2 - a]
                xa = (o[a] - b.ng + np.arange(n) + 0.5) * h
                s = [1, 1, 1]
                s[2 - a] = n
                xa = xa.reshape(s)
                ins &= (xa > 0) & (xa < 1)
            selF = _face_ghost_mask(b, d) & ins
            ref = fc[d, 0] + fc[d, 1] * xf
            np.testing.assert_allclose(om.b0[ib][d][selF], ref[selF], rtol=0, atol=1e-14)
            assert np.all(np.isfinite(om.b0[ib][d][selF]))
    assert checked > 1000


def test_prolongation_limits_at_an_extremum_and_restriction_inverts_it():
    """|x - x0| with x0 on the centre of a coarse cell next to the fine
    block: that parent's limited slope is 0 and its 8 children take its
    value; everywhere the prolonged children of a parent average to it"""
    m, blocks = _two_level(periodic=(1, 1, 1))
    om = O.RefinedMesh(blocks, O.Params(gamma=5.0 / 3.0), m)
    h0 = 1.0 / 16
    x0 = 8.5 * h0                       # centre of coarse cell 8 (block (1, 0, 0))
    for ib, b in enumerate(om.blocks):
        X, Y, Z = _cell_xyz(b, ib, m, h0)
        gm = _ghost_mask(b)
        om.w0[ib][0] = np.where(gm, np.nan, np.abs(X - x0) + 0.3 * np.sin(2 * np.pi * Y))
        om.w0[ib][1] = np.where(gm, np.nan, np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z) + 2 * Y)
    om.ghost_fill_state(0)
    fine = [ib for ib in range(len(om.blocks)) if m.leaves[ib][0] == 1]
    coarse = {m.leaves[ib][1]: ib for ib in range(len(om.blocks)) if m.leaves[ib][0] == 0}
    c1 = om.blocks[coarse[(1, 0, 0)]]
    n_ext = n_par = 0
    for ib in fine:
        b = om.blocks[ib]
        o = m.org(ib)
        g = b.ng
        # fine global index of padded cell x: o + x - g; parent = that >> 1 (wrapped to 16)
        for v in (0, 1):
            a = om.w0[ib][v]
            for kz in range(0, b.shape[0] - 1, 1):
                for jy in range(0, b.shape[1] - 1):
                    for ix in range(0, b.shape[2] - 1):
                        G = [o[0] + ix - g, o[1] + jy - g, o[2] + kz - g]
                        if any(x % 2 for x in G):
                            continue
                        # the 2x2x2 children of one parent, all ghosts of block ib
                        sl = (slice(kz, kz + 2), slice(jy, jy + 2), slice(ix, ix + 2))
                        inner = ~_ghost_mask(b)[sl]
                        if inner.any():
                            continue
                        P = [((x >> 1) % 16) for x in G]
                        pb = (P[0] // 8, P[1] // 8, P[2] // 8)
                        if pb not in coarse:
                            continue
                        L = om.blocks[coarse[pb]]
                        po = m.org(coarse[pb])
                        pv = om.w0[coarse[pb]][v][P[2] - po[2] + L.ng, P[1] - po[1] + L.ng, P[0] - po[0] + L.ng]
                        ch = a[sl]
                        assert abs(ch.mean() - pv) <= 1e-15 * max(1.0, abs(pv)), (ib, G, v)
                        n_par += 1
                        if v == 0 and P[0] == 8:
                            # the extremum along x: every child's x-slope is 0
                            assert np.all(ch[:, :, 0] == ch[:, :, 1])
                            n_ext += 1
    assert n_par > 100 and n_ext > 4
    assert c1 is not None


def test_prolonged_faces_keep_the_parent_divergence():
    """div-free face data (discrete curl): every ghost cell of a fine block
    whose 6 faces were all prolonged from one parent has divergence 0, the
    faces on a parent face equal it"""
    m, blocks = _two_level(periodic=(1, 1, 1))
    om = O.RefinedMesh(blocks, O.Params(gamma=5.0 / 3.0), m)
    # zero the fine blocks' ghost faces, then fill them
    for ib, b in enumerate(om.blocks):
        if m.leaves[ib][0] == 1:
            for d in range(3):
                om.b0[ib][d][_face_ghost_mask(b, d)] = np.nan
    om.ghost_fill_state(0)
    worst, n = 0.0, 0
    for ib, b in enumerate(om.blocks):
        if m.leaves[ib][0] != 1:
            continue
        bx, by, bz = om.b0[ib]
        assert all(np.all(np.isfinite(f)) for f in (bx, by, bz))
        div = (bx[:, :, 1:] - bx[:, :, :-1]) + (by[:, 1:, :] - by[:, :-1, :]) + (bz[1:, :, :] - bz[:-1, :, :])
        scale = max(np.abs(bx).max(), np.abs(by).max(), np.abs(bz).max())
        g = b.ng
        o = m.org(ib)
        for kz in range(b.shape[0]):
            for jy in range(b.shape[1]):
                for ix in range(b.shape[2]):
                    G = [o[0] + ix - g, o[1] + jy - g, o[2] + kz - g]
                    # a face is prolonged when the cells on both of its sides lie
                    # in the coarse region (the fine leaves cover [0, 16)^3 of the
                    # 32^3 fine lattice): keep cells whose 6 neighbours and itself
                    # all do
                    fine_at = lambda q: all((x % 32) < 16 for x in q)
                    nbrs = [G] + [[G[0] + (a == 0) * s, G[1] + (a == 1) * s, G[2] + (a == 2) * s]
                                  for a in range(3) for s in (-1, 1)]
                    if any(fine_at(q) for q in nbrs):
                        continue
                    if not _ghost_mask(b)[kz, jy, ix]:
                        continue
                    worst = max(worst, abs(div[kz, jy, ix]) / scale)
                    n += 1
    assert n > 100
    assert worst < 1e-14, worst


def _divb(om, which=0):
    Bf = om._set(which)[2]
    worst = 0.0
    for ib, b in enumerate(om.blocks):
        g, n = b.ng, b.nx
        bx, by, bz = Bf[ib]
        s = slice(g, g + n)
        d = ((bx[s, s, g + 1:g + n + 1] - bx[s, s, s]) + (by[s, g + 1:g + n + 1, s] - by[s, s, s])
             + (bz[g + 1:g + n + 1, s, s] - bz[s, s, s]))
        worst = max(worst, float(np.abs(d).max()) / max(np.abs(bx).max(), np.abs(by).max(), np.abs(bz).max()))
    return worst


def _interface_mismatch(om, m):
    """max over coarse boundary faces next to fine leaves of |coarse face -
    mean of the 4 fine faces| / max |B|"""
    fine = {m.leaves[ib][1]: ib for ib in range(len(om.blocks)) if m.leaves[ib][0] == 1}
    worst, n = 0.0, 0
    for ib, (lv, bb) in enumerate(m.leaves):
        if lv != 0:
            continue
        b = om.blocks[ib]
        g, nb = b.ng, b.nx
        o = m.org(ib)
        for d in range(3):
            for side in (0, 1):
                G = o[d] - 1 if side == 0 else o[d] + nb
                G %= 16
                for q2 in range(nb):
                    for q1 in range(nb):
                        t1, t2 = (d + 1) % 3, (d + 2) % 3
                        I = [0, 0, 0]
                        I[d], I[t1], I[t2] = G, o[t1] + q1, o[t2] + q2
                        fb = tuple((2 * I[a]) // 8 for a in range(3))
                        if fb not in fine:
                            continue
                        if any(x >= 16 for x in I):
                            continue
                        L = om.blocks[fine[fb]]
                        lo = m.org(fine[fb])
                        x = [0, 0, 0]
                        x[d] = g + (nb if side else 0)
                        x[t1], x[t2] = g + q1, g + q2
                        cv = om.b0[ib][d][x[2], x[1], x[0]]
                        s = 0.0
                        for c in range(4):
                            J = [0, 0, 0]
                            J[d] = 2 * I[d] + (0 if side else 2)
                            J[t1] = 2 * I[t1] + (c & 1)
                            J[t2] = 2 * I[t2] + (c >> 1)
                            y = [J[a] - lo[a] + L.ng for a in range(3)]
                            s += om.b0[fine[fb]][d][y[2], y[1], y[0]]
                        worst = max(worst, abs(cv - 0.25 * s))
                        n += 1
    scale = max(max(np.abs(f).max() for f in om.b0[ib]) for ib in range(len(om.blocks)))
    return worst / scale, n


def _run_two_level(flux=1, emf=1, steps=2):
    m, blocks = _two_level(flat=True)
    om = O.RefinedMesh(blocks, O.Params(gamma=5.0 / 3.0, fofc=1, dmp_M=1.0), m)
    om.ghost_fill_state(0)
    t0 = om.totals(0)
    mis0, n = _interface_mismatch(om, m)
    O.lib().or_set_amr_corrections(flux, emf)
    try:
        for _ in range(steps):
            om.rk2_step(cfl=0.3)
    finally:
        O.lib().or_set_amr_corrections(1, 1)
    dtot = np.abs(om.totals(0) - t0) / np.abs(t0).max()
    mis, n = _interface_mismatch(om, m)
    return dtot, _divb(om), mis0, mis, n, om


def test_two_level_stage_conserves_and_keeps_div_b():
    dtot, divb, mis0, mis, n, om = _run_two_level()
    print("conservation", dtot, "div B", divb, "interface", mis0, mis, n)
    assert any(np.any(f & (O.F_DMP | O.F_FOFC)) for f in om.flags)
    assert n > 0
    assert np.all(dtot < 2e-15), dtot
    assert divb < 1e-14
    assert mis0 < 1e-15 and mis < 1e-14


def _shared_face_mismatch(om, m):
    """max |difference| between the two copies of every face that two leaves
    of the same level share (each leaf evolves its boundary faces itself)"""
    where = {lf: i for i, lf in enumerate(m.leaves)}
    worst = 0.0
    for i, (lv, b) in enumerate(m.leaves):
        nbk = [x << lv for x in m.nblocks0]
        blk = om.blocks[i]
        g, n = blk.ng, blk.nx
        for d in range(3):
            q = list(b)
            q[d] = (q[d] + 1) % nbk[d]
            j = where.get((lv, tuple(q)))
            if j is None:
                continue
            si = [slice(g, g + n)] * 3
            sj = [slice(g, g + n)] * 3
            si[2 - d], sj[2 - d] = g + n, g
            worst = max(worst, float(np.abs(om.b0[i][d][tuple(si)] - om.b0[j][d][tuple(sj)]).max()))
    return worst


def test_same_level_leaves_keep_their_shared_faces_identical():
    """the EMF correction also makes every same-level block around an edge
    next to a finer leaf use one EMF there; without it the copies drift"""
    _, _, _, _, _, om = _run_two_level()
    m = om.leafmesh
    # round-off only: the initial data of a face on a periodic boundary are
    # computed at coordinate 0 in one leaf and 1 in the other
    assert _shared_face_mismatch(om, m) < 2e-15
    _, _, _, _, _, om = _run_two_level(emf=0)
    assert _shared_face_mismatch(om, m) > 1e-9


def test_without_the_corrections_conservation_and_consistency_break():
    dtot, divb, _, mis, _, _ = _run_two_level(flux=0)
    assert dtot[0] > 1e-9, dtot
    dtot, divb, _, mis, _, _ = _run_two_level(emf=0)
    assert mis > 1e-9 and divb < 1e-14, (mis, divb)


def test_uniform_state_stays_uniform_across_levels():
    m, blocks = _two_level(flat=True, uniform=(1.0, (0.3, -0.2, 0.1), 0.5, (0.2, 0.1, -0.3)))
    om = O.RefinedMesh(blocks, O.Params(gamma=5.0 / 3.0), m)
    om.ghost_fill_state(0)
    for _ in range(2):
        om.rk2_step(cfl=0.3)
    for ib in range(len(om.blocks)):
        w = om.interior(om.w0[ib], ib)
        for v, ref in enumerate((1.0, 0.3, -0.2, 0.1, 0.5)):
            assert np.abs(w[v] - ref).max() < 1e-14, (ib, v)


def test_leaf_lookup_table_answers_as_the_search():
    """the per-level lookup table of the leaves gives the search's answer:
    ghost fills and a stage bit for bit the same with it and without it"""
    refine = lambda lv, b: b == (0, 0, 0)
    m = inputs.leaf_mesh((2, 2, 2), 8, refine=refine, max_level=2, periodic=(1, 0, 1))
    blocks = inputs.smooth_leaf_blocks(m)
    p = O.Params(gamma=5.0 / 3.0, fofc=1, dmp_M=1.0)
    runs = []
    for use in (1, 0):
        O.lib().or_set_leaf_index(use)
        try:
            om = O.RefinedMesh(copy.deepcopy(blocks), p, m)
            om.ghost_fill_state(0)
            om.rk2_step(cfl=0.3)
        finally:
            O.lib().or_set_leaf_index(1)
        runs.append(om)
    a, b = runs
    for ib in range(len(blocks)):
        np.testing.assert_array_equal(a.u0[ib], b.u0[ib])
        np.testing.assert_array_equal(a.w0[ib], b.w0[ib])
        for d in range(3):
            np.testing.assert_array_equal(a.b0[ib][d], b.b0[ib][d])

"""Per-stage parity of the HIP stage against the oracle on multi-block
meshes with floors, FOFC and the DMP active (test helper).

Each stage of a Runge-Kutta step is compared from a common input: the oracle
steps its mesh, and before every stage the device mesh takes the oracle's
state sets (ghosts included), runs the same stage, and its output is compared
with the oracle's over every interior cell and face of every block, block
edges included.

Decisions at a threshold.  The oracle is run on the same stage input twice
more with every threshold test of the method moved by a relative +-margin
(oracle.set_decision_margin).  Cells whose flags differ between those runs
and the plain one hold a decision within `margin` of its threshold; the
device may decide those either way, and only those.  Cells (and faces) whose
values move between the runs depend on such a decision and are left out of
the value gate.

The gate (reading of the parity metric for values formed by cancellation).
The conserved state U and the face field are sums, U = a0 U^n + a1 U^(s) +
b dt (G - div F) and B = a0 B^n + a1 B^(s) - b dt curl E; their rounding
error scales with the magnitudes of the terms summed, not with the result.
Where the terms cancel -- the momentum of a star near hydrostatic balance,
the face field under a nearly vanishing curl -- two correct evaluations that
round differently differ by far more than 1e-12 of the result (the oracle
built with fused multiply-adds differs from the plain oracle by up to 1.4e-10
there in the pointwise metric).  So U and the faces are gated at `tol`
relative to max(|x|, 1e-3 max|x| of the block, T), T the oracle's magnitude
of the summed terms of that value (oracle.Mesh.stage_sets(term_scales=True));
where nothing cancels T ~ |x| and this is the pointwise metric.  The
primitives are gated as the inversion of the device's own state: the
device's w against the oracle's inversion of the device's U and field, at
`tol` in the pointwise metric of tests/parity.py; where the inversion fired
a floor rule, the device's U against the oracle's Eq. 7 of the device's w
instead (compare_block).  The pointwise metric of the stage output against
the oracle's is reported beside the gates."""
import copy

import numpy as np

import oracle as O

MOVE_TOL = 1e-13      # a value "moves" between margin runs beyond this (same metric)


def _metric(got, ref, kind, scale=None):
    """elementwise error of got against ref: kind 'pos' (pointwise relative),
    'sgn' (against max(|x|, 1e-3 max|x|)) or 'tau' (pos where ref > 0, else
    sgn); with scale, against max(that denominator, scale)"""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    floor = 1e-3 * max(float(np.max(np.abs(ref))) if ref.size else 0.0, 1e-300)
    den_s = np.maximum(np.abs(ref), floor)
    den_p = np.maximum(np.abs(ref), 1e-300)
    den = den_s if kind == "sgn" else (den_p if kind == "pos" else np.where(ref > 0.0, den_p, den_s))
    if scale is not None:
        den = np.maximum(den, scale)
    return d / den


U_KINDS = ("pos", "sgn", "sgn", "sgn", "tau")
W_KINDS = ("pos", "sgn", "sgn", "sgn", "pos")


def _face_slices(b, d):
    g = b.ng
    n = (b.nx, b.ny, b.nz)
    sl = [slice(g, g + b.nz), slice(g, g + b.ny), slice(g, g + b.nx)]
    sl[2 - d] = slice(g, g + n[d] + 1)
    return tuple(sl)


def _face_mask(cells, d):
    """faces of direction d with a masked cell on either side (cells is an
    interior (nz, ny, nx) mask)"""
    ax = 2 - d
    pad = [(0, 0)] * 3
    pad[ax] = (1, 0)
    lo = np.pad(cells, pad)              # face f has cell f on its upper side
    pad[ax] = (0, 1)
    hi = np.pad(cells, pad)              # and cell f - 1 on its lower side
    return lo | hi


def _outputs(mesh, dst, ib):
    """(U, w, faces, flags) of state set dst, block ib, interiors only"""
    U, W, Bf = mesh._set(dst)
    b = mesh.blocks[ib]
    return (np.array(mesh.interior(U[ib], ib)), np.array(mesh.interior(W[ib], ib)),
            [np.array(Bf[ib][d][_face_slices(b, d)]) for d in range(3)],
            np.array(mesh.interior(mesh.flags[ib], ib)))


def _moved(a, ref, kinds):
    m = np.zeros(ref.shape[1:], bool)
    for c, kd in enumerate(kinds):
        m |= _metric(a[c], ref[c], kd) > MOVE_TOL
    return m


def _cell_bt(b, faces):
    """densitized cell-centred field of the interior from interior faces"""
    fx, fy, fz = faces
    return np.stack([0.5 * (fx[:, :, 1:] + fx[:, :, :-1]), 0.5 * (fy[:, 1:, :] + fy[:, :-1, :]),
                     0.5 * (fz[1:, :, :] + fz[:-1, :, :])])


def _inversion(om, ib, U, faces):
    """the oracle's inversion of (U, faces) on block ib's interior, and the
    cells where it fired a rule"""
    b = om.blocks[ib]
    gam = np.array(om.interior(om.adm[ib][4:10], ib)).reshape(6, -1)
    bt = _cell_bt(b, faces).reshape(3, -1)
    u = np.ascontiguousarray(U.reshape(5, -1))
    _, wr, fl, _, _ = O.c2p(u.copy(), bt, gam, om.params)
    refired = (fl.reshape(U.shape[1:]) & O.F_FLOORS) != 0
    return wr.reshape(U.shape), refired


def _prim2con(om, ib, w, faces):
    """the oracle's conserved state (Eq. 7) of (w, faces) on block ib's interior"""
    b = om.blocks[ib]
    gam = np.array(om.interior(om.adm[ib][4:10], ib)).reshape(6, -1)
    bt = _cell_bt(b, faces).reshape(3, -1)
    return O.prim2con(np.ascontiguousarray(w.reshape(5, -1)), bt, gam, om.params).reshape(w.shape)


def compare_block(om, ib, ref, dev, TU, TB, keep, fmask, note):
    """Gate one block's stage output dev = (U, w, faces, flags) against the
    oracle's ref, with the term magnitudes TU (5 cell arrays) and TB (3 face
    arrays) of the oracle's update and CT sums; keep: the cells to gate,
    fmask[d]: the faces to gate.  note(key, err) records each error.

    * cells whose inversion fired no rule: U against the oracle's U relative
      to max(pointwise denominator, T); w as the oracle's inversion of the
      device's own U and faces (pointwise metric);
    * cells whose inversion fired a rule (floors; the same decision on both
      sides, checked by the caller): U as the oracle's Eq. 7 of the device's
      own w (pointwise), and w against the oracle's w -- rho and P pointwise,
      W v^i relative to the momentum's term magnitude over D~ (u = S/(D h)
      with h >= 1), since the floors keep the inverted velocity;
    * faces relative to max(pointwise denominator, T).
    Returns the pointwise metric of U, w and faces against the oracle's."""
    Ur, Wr, Fr, fr = ref
    Ug, Wg, Fg, fg = dev
    fired = (fg & O.F_FLOORS) != 0
    wi, refired = _inversion(om, ib, Ug, Fg)
    free = keep & ~fired & ~refired
    floored = keep & (fired | refired)
    raw = {"U": 0.0, "w": 0.0, "faces": 0.0}
    mx = lambda e: float(e.max()) if e.size else 0.0
    uc = _prim2con(om, ib, Wg, Fg) if np.any(floored) else None
    TUvel = np.max(TU[1:4], axis=0) / np.maximum(np.abs(Ur[0]), 1e-300)
    for c, kd in enumerate(U_KINDS):
        e = mx(_metric(Ug[c], Ur[c], kd, scale=TU[c])[free])
        if uc is not None:
            e = max(e, mx(_metric(Ug[c], uc[c], kd)[floored]))
        note(f"U{c}", e)
        raw["U"] = max(raw["U"], mx(_metric(Ug[c], Ur[c], kd)[keep]))
    for c, kd in enumerate(W_KINDS):
        e = mx(_metric(Wg[c], wi[c], kd)[free])
        if c in (1, 2, 3):
            e = max(e, mx(_metric(Wg[c], Wr[c], kd, scale=TUvel)[floored]))
        else:
            e = max(e, mx(_metric(Wg[c], Wr[c], kd)[floored]))
        note(f"w{c}", e)
        raw["w"] = max(raw["w"], mx(_metric(Wg[c], Wr[c], kd)[keep]))
    for d in range(3):
        note(f"B{d}", mx(_metric(Fg[d], Fr[d], "sgn", scale=TB[d])[fmask[d]]))
        raw["faces"] = max(raw["faces"], mx(_metric(Fg[d], Fr[d], "sgn")[fmask[d]]))
    return raw


def stage_parity(gm, om, scheme, dt, tol=1e-12, margin=1e-9, say=print, upload=None,
                 download=None):
    """Step the oracle mesh om through `scheme` (O.Mesh.RK2 / RK3) with dt;
    before each stage copy the oracle's state sets into the device mesh gm
    (upload(gm, om)), run the stage there, read it back (download(gm, dst, ib)
    -> (U, w, faces, flags)) and compare.  Returns the per-stage summary."""
    nb = len(om.blocks)
    summary = []
    for k, (src, dst, (a0, a1, b)) in enumerate(scheme):
        # the oracle at the plain thresholds and moved by +-margin, same input
        alt = []
        for m in (margin, -margin):
            o2 = copy.deepcopy(om)
            O.set_decision_margin(m)
            try:
                o2.stage_sets(src, dst, dt, a0, a1, b)
            finally:
                O.set_decision_margin(0.0)
            alt.append(o2)
        upload(gm, om)
        gm.stage_sets(src, dst, (a0, a1, b), dt=dt)
        tu, tb = om.stage_sets(src, dst, dt, a0, a1, b, term_scales=True)
        worst = {"U": 0.0, "faces": 0.0, "w": 0.0}
        raw = {"U": 0.0, "w": 0.0, "faces": 0.0}
        where = {}
        fails = []
        n_near = n_moved = n_flag_diff = n_fired = 0
        ncell = 0
        for ib in range(nb):
            blk = om.blocks[ib]
            ref = _outputs(om, dst, ib)
            dev = download(gm, dst, ib)
            Ur, Wr, Fr, fr = ref
            fg = dev[3]
            TU = np.array(om.interior(tu[ib], ib))
            TB = [tb[ib][d][_face_slices(blk, d)] for d in range(3)]
            near = np.zeros(fr.shape, bool)
            moved = np.zeros(fr.shape, bool)
            fmoved = [np.zeros(f.shape, bool) for f in Fr]
            for o2 in alt:
                Ua, Wa, Fa, fa = _outputs(o2, dst, ib)
                near |= fa != fr
                moved |= _moved(Ua, Ur, U_KINDS) | _moved(Wa, Wr, W_KINDS)
                for d in range(3):
                    fmoved[d] |= _metric(Fa[d], Fr[d], "sgn") > MOVE_TOL
            diff = fg != fr
            # a decision may differ only where it lies within the margin
            if np.any(diff & ~near):
                fails.append(("decision", k, ib, int(np.sum(diff & ~near)),
                              [int(x) for x in np.unique((fg ^ fr)[diff & ~near])]))
            # a cell whose flags differ changes its faces and its neighbours
            # through them: those join the excluded set
            grow = diff.copy()
            for ax in range(3):
                grow = grow | np.roll(grow, 1, axis=ax) | np.roll(grow, -1, axis=ax)
            skip = moved | grow
            n_near += int(near.sum())
            n_moved += int(skip.sum())
            n_flag_diff += int(diff.sum())
            n_fired += int(np.sum((fg & O.F_FLOORS) != 0))
            ncell += fr.size

            def note(key, e, ib=ib):
                if e > where.get(key, (0.0,))[0]:
                    where[key] = (e, ib)
                grp = "faces" if key[0] == "B" else key[0]
                worst[grp] = max(worst[grp], e)
                if e >= tol:
                    fails.append(("value", k, ib, key, e))

            fmask = [~(_face_mask(skip, d) | fmoved[d]) for d in range(3)]
            r = compare_block(om, ib, ref, dev, TU, TB, ~skip, fmask, note)
            for key in raw:
                raw[key] = max(raw[key], r[key])
        say(f"  stage {k + 1}: gated U {worst['U']:.1e}, w {worst['w']:.1e}, faces "
            f"{worst['faces']:.1e}; pointwise metric against the oracle's output: U {raw['U']:.1e}, "
            f"w {raw['w']:.1e}, faces {raw['faces']:.1e}")
        say(f"    decisions within {margin:g} of a threshold in {n_near} of {ncell} cells, device "
            f"decided otherwise in {n_flag_diff}; cells left out of the value gate {n_moved}; "
            f"cells whose inversion fired a rule {n_fired}")
        say("    gated, per field (max, block): " +
            ", ".join(f"{key} {v[0]:.1e} ({v[1]})" for key, v in sorted(where.items())))
        assert not fails, fails[:8]
        summary.append(dict(worst=worst, raw=raw, near=n_near, flag_diff=n_flag_diff,
                            skipped=n_moved, cells=ncell, tu=tu, tb=tb))
        om.ghost_fill_state(dst)
    return summary

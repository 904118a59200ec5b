"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: 1e-12 per stage (values), flags bit-exact where no decision lies
at its threshold; 1e-9 after 100 steps of a smooth periodic run.
"""
import copy
import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2409_10384_amd import inputs
from tests import parity as PM

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10384_amd import lib
    lib.load()
    return lib


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_mp(G, p: O.Params):
    return G.MethodParams(**dataclasses.asdict(p))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------------------
# pointwise: prim2con and c2p_batch
# ---------------------------------------------------------------------------
def test_prim2con_parity(G):
    say("prim2con parity: c2p_states 65536")
    st = inputs.c2p_states(1 << 16, seed_offset=201)
    p = O.Params(gamma=5.0 / 3.0)
    ref = O.prim2con(st["w"], st["bt"], st["gam"], p)
    d = lambda a: torch.as_tensor(a).cuda()
    got = host(G.prim2con(d(st["w"]), d(st["bt"]), d(st["gam"]), to_mp(G, p)))
    errs = PM.cons_errors(got, ref)
    assert max(errs) < 1e-13, errs


def test_c2p_batch_parity_wide_ranges(G):
    say("c2p_batch parity: c2p_states 65536, tol 1e-12")
    st = inputs.c2p_states(1 << 16, seed_offset=202)
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30, M_max=1e30, c2p_tol=1e-12)
    u = O.prim2con(st["w"], st["bt"], st["gam"], p)
    _, wref, fref, nref, muref = O.c2p(u, st["bt"], st["gam"], p)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    out = G.c2p_batch(d(u), d(st["bt"]), d(st["gam"]), to_mp(G, p), want_mu=True, want_nev=True)
    w = host(out["w"])
    np.testing.assert_array_equal(host(out["flags"]).astype(np.uint16), fref)
    mu = host(out["mu"])
    assert np.max(np.abs(mu - muref) / muref) < 2e-12
    # exact label mu* = 1/(hW)
    eps = st["w"][4] / (2.0 / 3.0 * st["w"][0])
    mus = 1.0 / ((1 + eps + st["w"][4] / st["w"][0]) * st["W"])
    assert np.max(np.abs(mu - mus) / mus) < 1e-10
    # rho = D/W inherits the root tolerance amplified by dlnW/dlnmu ~ W^2 v^2
    drho = np.abs(w[0] - wref[0]) / wref[0]
    assert np.all(drho <= 4e-12 * st["W"] ** 2), np.max(drho / st["W"] ** 2)


def test_c2p_batch_parity_hybrid_eos(G):
    """piecewise polytrope + thermal part: same flags, mu to 2e-12, the
    primitives within the conditioning of the root.  Densities up to
    10^-2.9 (about the star's central density): above a few times that the
    seeded polytrope's sound speed exceeds 1 and the master function loses
    its single root."""
    say("c2p_batch parity, hybrid EOS: 32768 states")
    pp, K = inputs.pp_eos()
    st = inputs.c2p_states(1 << 15, seed_offset=204, pp=pp, pp_K=K, log_rho=(-10.0, -2.9))
    p = O.Params(rho_atm=1e-20, T_atm=1e-30, M_max=1e30, c2p_tol=1e-12, **pp)
    u = O.prim2con(st["w"], st["bt"], st["gam"], p)
    _, wref, fref, _, muref = O.c2p(u, st["bt"], st["gam"], p)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    out = G.c2p_batch(d(u), d(st["bt"]), d(st["gam"]), to_mp(G, p), want_mu=True)
    flags = host(out["flags"]).astype(np.uint16)
    w = host(out["w"])
    # Dense hot states whose thermal part is a tiny fraction of P recover
    # eps at the cold floor eps_cold(rho) up to rounding: whether the
    # temperature floor fires there is the sign of rounding noise, and both
    # answers are valid.  Only that bit may differ, and only where the side
    # without the floor recovered a temperature below 1e-6 of P/rho.
    diff = flags != fref
    say(f"  temperature-floor coin flips: {int(diff.sum())} of {flags.size}")
    assert np.all((flags[diff] ^ fref[diff]) == O.F_TFLOOR)
    unfloored = np.where(fref[diff] & O.F_TFLOOR, w[4][diff] / w[0][diff], wref[4][diff] / wref[0][diff])
    pc_rho = inputs.pp_cold_pressure(st["w"][0][diff], pp, K) / st["w"][0][diff]
    t_rel = (unfloored - pc_rho) / unfloored
    assert np.all(t_rel < 1e-6), np.max(t_rel)
    mu = host(out["mu"])
    assert np.max(np.abs(mu - muref) / muref) < 2e-12
    same = ~diff
    drho = np.abs(w[0] - wref[0]) / wref[0]
    assert np.all(drho[same] <= 4e-12 * st["W"][same] ** 2), np.max(drho / st["W"] ** 2)
    dP = np.abs(w[4] - wref[4]) / wref[4]
    say(f"  max rel dP {np.max(dP[same]):.2e}")


def test_c2p_batch_atmosphere_rules_parity(G):
    """random states straddling every floor threshold: flags identical and
    values within 1e-12 away from the thresholds"""
    say("c2p_batch atmosphere parity")
    st = inputs.c2p_states(1 << 14, seed_offset=203, log_rho=(-8.0, 0.0), log_eps=(-8.0, 0.0))
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-6, T_atm=1e-5, f_thr=3.0, M_max=20.0)
    u = O.prim2con(st["w"], st["bt"], st["gam"], p)
    rng = np.random.default_rng(5)
    bad = rng.random(u.shape[1]) < 0.01
    u[1][bad] = np.nan
    u2, wref, fref, _, _ = O.c2p(u, st["bt"], st["gam"], p)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    ud = d(u)
    out = G.c2p_batch(ud, d(st["bt"]), d(st["gam"]), to_mp(G, p))
    flags = host(out["flags"]).astype(np.uint16)
    same = flags == fref
    assert np.mean(same) > 0.999, np.mean(same)
    assert np.all(np.isfinite(host(out["w"])))
    for c in range(5):
        assert PM.rel_signed(host(out["w"])[c][same], wref[c][same]) < 1e-10
    assert np.any(fref & O.F_DFLOOR) and np.any(fref & O.F_TFLOOR) and np.any(fref & O.F_C2P_FAIL)


# ---------------------------------------------------------------------------
# one stage / one step on the smooth periodic block
# ---------------------------------------------------------------------------
def _meshes(G, blocks, p):
    om = O.Mesh(copy.deepcopy(blocks), p)
    gm = G.DeviceMesh(copy.deepcopy(blocks), to_mp(G, p))
    return om, gm


def _compare_state(om, gm, which, tol, label):
    worst = 0.0
    for ib in range(len(om.blocks)):
        if which == 1:
            pairs = [(gm.u1[ib], om.u1[ib], "U"), (gm.w1[ib], om.w1[ib], "w")]
            faces = list(zip(gm.b1[ib], om.b1[ib]))
        else:
            pairs = [(gm.u0[ib], om.u0[ib], "U"), (gm.w0[ib], om.w0[ib], "w")]
            faces = list(zip(gm.b0[ib], om.b0[ib]))
        for gt, ref, name in pairs:
            got = om.interior(host(gt), ib)
            r = om.interior(ref, ib)
            errs = PM.cons_errors(got, r) if name == "U" else PM.prim_errors(got, r)
            say(f"  {label} block {ib} {name} errs {['%.1e' % e for e in errs]}")
            assert max(errs) < tol, (label, name, errs)
            worst = max(worst, max(errs))
        b = om.blocks[ib]
        g = b.ng
        for d, (gf, rf) in enumerate(faces):
            got = host(gf)
            sl = [slice(g, g + b.nz), slice(g, g + b.ny), slice(g, g + b.nx)]
            sl[2 - d] = slice(g, g + [b.nx, b.ny, b.nz][d] + 1)
            e = PM.rel_signed(got[tuple(sl)], rf[tuple(sl)])
            assert e < tol, (label, "faces", d, e)
            worst = max(worst, e)
    return worst


def test_flux_parity_smooth_block(G):
    say("flux parity: smooth periodic block 32^3")
    blk = inputs.smooth_periodic_block(n=32)
    p = O.Params(gamma=5.0 / 3.0)
    om, gm = _meshes(G, [blk], p)
    F = O.alloc_fluxes(om)
    O.stage_steps(om, 1, 0.01, F, 1)
    gm.run_steps(1, 0.01, 1)
    b = blk
    g = b.ng
    for d in range(3):
        for c in range(7):
            got = host(gm.flux_view(0, d, c))
            ref = F[0][d][c]
            sl = [slice(g - 1, g + b.nz + 1), slice(g - 1, g + b.ny + 1), slice(g - 1, g + b.nx + 1)]
            sl[2 - d] = slice(g, g + [b.nx, b.ny, b.nz][d] + 1)
            # every component with the signed metric: a face flux that nearly
            # cancels is compared against 1e-3 of the component's largest value,
            # so 3e-12 there is ~3e-15 of that scale (the GPU divides through a
            # refined hardware reciprocal, the oracle with IEEE division)
            e = PM.rel_signed(got[tuple(sl)], ref[tuple(sl)])
            say(f"  flux d={d} c={c}: {e:.2e}")
            assert e < 3e-12, (d, c, e)


def test_stage_and_step_parity_smooth_block(G):
    say("stage parity: smooth periodic block 32^3, WENOZ+HLLE, 1 RK2 step")
    blk = inputs.smooth_periodic_block(n=32)
    p = O.Params(gamma=5.0 / 3.0)
    om, gm = _meshes(G, [blk], p)
    _compare_state(om, gm, 0, 1e-13, "init")
    dt = om.dt(0.25)
    gdt = host(gm.compute_dt(0.25))[0]
    assert abs(gdt - dt) / dt < 1e-13
    om.stage(1, dt)
    gm.stage(1, dt=dt)
    _compare_state(om, gm, 1, 1e-12, "stage1")
    om.ghost_fill_state(1)
    gm.ghost_fill(1)
    om.stage(2, dt)
    gm.stage(2, dt=dt)
    om.ghost_fill_state(0)
    gm.ghost_fill(0)
    _compare_state(om, gm, 0, 1e-12, "step")
    m_ref = om.mass()
    m_gpu = host(gm.mass())[0]
    assert abs(m_gpu - m_ref) / m_ref < 1e-14


def test_stage_parity_fofc_dmp_flags(G):
    say("stage parity: FOFC+DMP(M=1) on the smooth block 24^3")
    blk = inputs.smooth_periodic_block(n=24)
    p = O.Params(gamma=5.0 / 3.0, fofc=1, dmp_M=1.0, T_atm=0.085)
    om, gm = _meshes(G, [blk], p)
    dt = om.dt(0.25)
    om.stage(1, dt)
    gm.stage(1, dt=dt)
    fl_ref = om.flags[0]
    fl = host(gm.flags[0]).astype(np.uint16)
    g = 3
    inner = (slice(g, -g),) * 3
    assert np.any(fl_ref[inner] & O.F_DMP) and np.any(fl_ref[inner] & O.F_FOFC)
    np.testing.assert_array_equal(fl[inner], fl_ref[inner])
    _compare_state(om, gm, 1, 1e-12, "fofc stage1")


def test_hundred_steps_parity(G):
    say("100-step parity: smooth periodic block 16^3")
    blk = inputs.smooth_periodic_block(n=16)
    p = O.Params(gamma=5.0 / 3.0)
    om, gm = _meshes(G, [blk], p)
    worst = 0.0
    for s in range(100):
        dt = om.dt(0.25)
        om.rk2_step(dt)
        gm.rk2_step(dt=dt)
    worst = _compare_state(om, gm, 0, 1e-9, "100 steps")
    say(f"  worst after 100 steps {worst:.2e}")


def test_device_dt_drives_the_step(G):
    say("device dt: rk2_step with the on-device CFL dt")
    blk = inputs.smooth_periodic_block(n=16)
    p = O.Params(gamma=5.0 / 3.0)
    om, gm = _meshes(G, [blk], p)
    for _ in range(3):
        om.rk2_step(cfl=0.25)
        gm.rk2_step(cfl=0.25)
    _compare_state(om, gm, 0, 1e-12, "device dt")


# ---------------------------------------------------------------------------
# multi-block star: same-level exchange, outflow, atmosphere, FOFC+DMP
# ---------------------------------------------------------------------------
STAR_P = O.Params(gamma=2.0, rho_atm=1.28e-13, T_atm=1.28e-11, f_thr=0.1, M_max=100.0, fofc=1,
                  dmp_M=1.1)


def test_star_multiblock_parity(G):
    say("star parity: 2^3 blocks of 16^3, exchange + outflow, FOFC+DMP, 1 RK2 step")
    blocks, st = inputs.star_blocks(n_per_side=2, nb=16)
    _star_parity(G, blocks, STAR_P)


def test_star_multiblock_parity_hybrid_eos(G):
    say("star parity, piecewise polytrope + thermal part: 2^3 blocks of 16^3, 1 RK2 step")
    pp, K = inputs.pp_eos()
    st = inputs.calibrate_field(inputs.StarSetup(pp=pp, pp_K=K))
    blocks, st = inputs.star_blocks(n_per_side=2, nb=16, st=st)
    p = dataclasses.replace(STAR_P, **pp)
    _star_parity(G, blocks, p)


def _star_parity(G, blocks, params, scheme="RK2"):
    """one step of `scheme` (RK2 or RK3) on both sides with the oracle's dt"""
    om, gm = _meshes(G, blocks, params)
    dt = om.dt(0.25)
    for k, (src, dst, (a0, a1, b)) in enumerate(getattr(O.Mesh, scheme)):
        om.stage_sets(src, dst, dt, a0, a1, b)
        gm.stage_sets(src, dst, (a0, a1, b), dt=dt)
        torch.cuda.synchronize()
        if k == 0:
            s1_bad = 0
            for ib in range(len(blocks)):
                fr = om.interior(om.flags[ib], ib)
                fg = om.interior(host(gm.flags[ib]).astype(np.uint16), ib)
                s1_bad += int(np.sum(fr != fg))
            say(f"  stage 1 decision mismatches: {s1_bad}")
            assert s1_bad <= 0.001 * sum(b.nx * b.ny * b.nz for b in blocks)
        om.ghost_fill_state(dst)
        gm.ghost_fill(dst)
    torch.cuda.synchronize()
    nflag = 0
    for ib in range(len(blocks)):
        fr = om.interior(om.flags[ib], ib)
        fg = om.interior(host(gm.flags[ib]).astype(np.uint16), ib)
        nflag += int(np.sum(fr != 0))
        bad = fr != fg
        mism = np.mean(bad)
        kinds = np.unique(fr[bad] ^ fg[bad]) if bad.any() else []
        say(f"  block {ib}: flagged {int(np.sum(fr != 0))}, decision mismatches {int(bad.sum())}"
            f" (xor bits {list(kinds)})")
        assert mism < 0.01, mism
        # a cell's update depends on the decisions of its 27-cell neighbourhood
        # (FOFC faces, corner EMFs): gate only cells whose whole neighbourhood
        # decided alike, and keep off the block edge (neighbour-block flags)
        dil = bad.copy()
        for ax in range(3):
            dil = dil | np.roll(dil, 1, axis=ax) | np.roll(dil, -1, axis=ax)
        ok = ~dil
        ok[[0, -1], :, :] = False
        ok[:, [0, -1], :] = False
        ok[:, :, [0, -1]] = False
        energy = om.interior(om.u0[ib], ib)
        energy = float(np.max(energy[0] + energy[4]))
        for name, gt, ref in (("U", gm.u0[ib], om.u0[ib]), ("w", gm.w0[ib], om.w0[ib])):
            got = om.interior(host(gt), ib)
            r = om.interior(ref, ib)
            for c in range(5):
                e = PM.rel_signed(got[c][ok], r[c][ok]) if c in (1, 2, 3) else \
                    PM.rel_positive(got[c][ok], r[c][ok])
                say(f"    {name}[{c}] max rel err {e:.2e} over {int(ok.sum())} cells")
                if e >= 1e-10 and c in (1, 2, 3):
                    # Near hydrostatic balance the momentum after one step is the
                    # small difference of the pressure-gradient and gravity terms,
                    # and its rounding is that of those terms: judge it against the
                    # energy density (|S| <= E) for S~, against c = 1 for W v^i.
                    d = float(np.max(np.abs(got[c][ok] - r[c][ok])))
                    e = d / energy if name == "U" else d
                    say(f"      near balance: max |error| {d:.2e}, relative to the scale {e:.2e}")
                    assert e < 1e-14, (ib, name, c, e)
                    continue
                assert e < 1e-10, (ib, name, c, e)
    assert nflag > 0


def test_riemann_tube_parity_and_exact_solution(G):
    """the 1-D relativistic blast wave (B = 0, flat space, 200 cells, t = 0.4,
    about 320 steps) on the GPU: the oracle's dt sequence; the exact
    solution's L1 error of the oracle to 1e-6 of itself; pointwise density
    within 1e-8 of the oracle (three times the smooth run's 100 steps, through
    two shocks whose nonlinear reconstruction weights amplify rounding)"""
    from tests import exact_riemann as X
    from tests.test_oracle_riemann import PROBLEMS, _tube, GAM
    say("Riemann tube (blast wave), 200 cells, GPU vs oracle vs exact")
    L, R = PROBLEMS["blast"]
    N = 200
    blk = _tube(L, R, N)
    p = O.Params(gamma=GAM, rho_atm=1e-12, T_atm=1e-14, f_thr=1.0, recon=2, riemann=1)
    om, gm = _meshes(G, [blk], p)
    t, t_end = 0.0, 0.4
    while t < t_end - 1e-14:
        dt = min(om.dt(0.25), t_end - t)
        om.rk2_step(dt)
        gm.rk2_step(dt=dt)
        t += dt
    ro = om.interior(om.w0[0], 0)[0, 0, 0, :]
    rg = om.interior(host(gm.w0[0]), 0)[0, 0, 0, :]
    e = np.max(np.abs(rg - ro) / ro)
    xc = (np.arange(N) + 0.5) / N
    ex = X.sample(L, R, (xc - 0.5) / t_end)[0]
    l1o, l1g = np.mean(np.abs(ro - ex)), np.mean(np.abs(rg - ex))
    say(f"  max rel GPU-oracle {e:.2e}; L1 vs exact: oracle {l1o:.4e}, GPU {l1g:.4e}")
    assert e < 1e-8
    assert abs(l1g - l1o) <= 1e-6 * l1o

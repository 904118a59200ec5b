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
from tests import stage_parity as SP

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
    # W v^i: u = W mu chi (r + mu s B) inherits the same amplification plus one
    W = st["W"]
    un = np.sqrt(np.sum(wref[1:4] ** 2, axis=0))
    du = np.max(np.abs(w[1:4] - wref[1:4]), axis=0) / un
    say(f"  max |du| / (|u| (W^2 + 1)) {np.max(du / (W ** 2 + 1)):.2e}")
    assert np.all(du <= 4e-12 * (W ** 2 + 1))
    # the recovery itself (reading R17): at the device's own root the oracle's
    # recovery formula gives the device's rho and W v^i to 1e-12 and its P to
    # 1e-12 of the magnitude of the terms eps is summed from (eps is a small
    # difference of O(W h) terms for cold fast states, so its rounding scales
    # with those terms, not with eps; the oracle built with fused multiply-adds
    # differs from the plain one by 5e-16 of that scale)
    wat, teps = O.recover(u, st["bt"], st["gam"], mu, p, eps_terms=True)
    eps = wat[4] / ((p.gamma - 1.0) * wat[0])
    e_r = np.abs(w[0] - wat[0]) / wat[0]
    e_u = np.max(np.abs(w[1:4] - wat[1:4]), axis=0) / np.sqrt(np.sum(wat[1:4] ** 2, axis=0))
    e_p = np.abs(w[4] - wat[4]) / wat[4] / np.maximum(1.0, teps / eps)
    say(f"  recovery at the device's root: rho {e_r.max():.2e}, W v {e_u.max():.2e}, "
        f"P/(eps terms/eps) {e_p.max():.2e}; unscaled P {np.max(np.abs(w[4] - wat[4]) / wat[4]):.2e}")
    assert e_r.max() < 1e-12 and e_u.max() < 1e-12 and e_p.max() < 1e-12


@pytest.mark.parametrize("n", [1, 63, 65, 4097])
def test_c2p_batch_parity_ragged_lengths(G, n):
    """batches that end inside a wave: the same flags as the oracle and mu
    to 2e-12 in every state, the last one included"""
    say(f"c2p_batch parity: {n} states")
    st = inputs.c2p_states(n, seed_offset=400 + n)
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30, M_max=1e30, c2p_tol=1e-12)
    u = O.prim2con(st["w"], st["bt"], st["gam"], p)
    _, wref, fref, nref, muref = O.c2p(u, st["bt"], st["gam"], p)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    out = G.c2p_batch(d(u), d(st["bt"]), d(st["gam"]), to_mp(G, p), want_mu=True)
    np.testing.assert_array_equal(host(out["flags"]).astype(np.uint16), fref)
    mu = host(out["mu"])
    assert mu.shape == (n,) and np.max(np.abs(mu - muref) / muref) < 2e-12


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


@pytest.mark.parametrize("scale", [1.0, 1e120])
def test_flux_parity_smooth_block(G, scale):
    """scale multiplies rho and P (and B by its square root, so every
    velocity is unchanged): at 1e120 the WENOZ smoothness indicators reach
    ~1e240, where the product of three of them would overflow; the kernel
    takes one refined reciprocal per indicator and must stay exact there"""
    say(f"flux parity: smooth periodic block 32^3, rho and P scaled by {scale:g}")
    blk = inputs.smooth_periodic_block(n=32)
    if scale != 1.0:
        blk.w[0] *= scale
        blk.w[4] *= scale
        for f in blk.bf:
            f *= np.sqrt(scale)
    p = O.Params(gamma=5.0 / 3.0)
    om, gm = _meshes(G, [blk], p)
    F = O.alloc_fluxes(om)
    Fs = O.alloc_fluxes(om)
    O.stage_steps(om, 1, 0.01, F, 1, flux_scales=Fs)
    gm.run_steps(1, 0.01, 1)
    b = blk
    g = b.ng
    for d in range(3):
        for c in range(7):
            got = host(gm.flux_view(0, d, c))
            ref = F[0][d][c]
            sl = [slice(g - 1, g + b.nz + 1), slice(g - 1, g + b.ny + 1), slice(g - 1, g + b.nx + 1)]
            sl[2 - d] = slice(g, g + [b.nx, b.ny, b.nz][d] + 1)
            sl = tuple(sl)
            # a face flux is a sum of terms (both sides' fluxes and the
            # Riemann dissipation of the face jump) that may cancel: gated
            # against the magnitude of those terms (tests/stage_parity.py),
            # the signed pointwise metric reported beside it
            e = float(SP._metric(got[sl], ref[sl], "sgn", scale=Fs[0][d][c][sl]).max())
            r = PM.rel_signed(got[sl], ref[sl])
            say(f"  flux d={d} c={c}: {e:.2e} (pointwise {r:.2e})")
            assert e < 1e-12, (d, c, e)


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
    say("100-step parity: smooth periodic block 32^3")
    blk = inputs.smooth_periodic_block(n=32)
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


def _upload(gm, om):
    """the oracle's state sets (ghosts included) into the device mesh"""
    for k in range(3):
        if k == 2 and gm.u2 is None:
            continue
        for dev, ref in zip(gm._set(k), om._set(k)):
            for ib in range(len(om.blocks)):
                if isinstance(ref[ib], list):
                    for d in range(3):
                        dev[ib][d].copy_(torch.from_numpy(ref[ib][d]))
                else:
                    dev[ib].copy_(torch.from_numpy(ref[ib]))


def _download(gm, dst, ib):
    """interior U, w, faces and flags of the device's state set dst, block ib"""
    U, W, Bf = gm._set(dst)
    b = gm.blocks[ib]
    return (om_interior(b, host(U[ib])), om_interior(b, host(W[ib])),
            [host(Bf[ib][d])[SP._face_slices(b, d)] for d in range(3)],
            om_interior(b, host(gm.flags[ib]).astype(np.uint16)))


def om_interior(b, a):
    g = b.ng
    return a[..., g:g + b.nz, g:g + b.ny, g:g + b.nx]


def _star_parity(G, blocks, params, scheme="RK2", chained_tol=1e-11):
    """Every stage of one step of `scheme` (RK2 or RK3) from the oracle's
    stage input, gated at 1e-12 over every interior cell and face of every
    block (tests/stage_parity.py: only cells whose values depend on a decision
    within 1e-9 of its threshold are left out, and the device may decide
    otherwise only there); then the whole step chained on the device alone
    against the oracle's step, with the same gate (the oracle's term
    magnitudes of the last stage) at chained_tol."""
    om = O.Mesh(copy.deepcopy(blocks), params)
    gm = G.DeviceMesh(copy.deepcopy(blocks), to_mp(G, params))
    sch = getattr(O.Mesh, scheme)
    if scheme == "RK3":
        gm._ensure_set_c()
    dt = om.dt(0.25)
    summary = SP.stage_parity(gm, om, sch, dt, tol=1e-12, margin=1e-9, say=say, upload=_upload,
                              download=_download)
    del gm
    # the device on its own through the whole step
    gc = G.DeviceMesh(copy.deepcopy(blocks), to_mp(G, params))
    for src, dst, (a0, a1, b) in sch:
        gc.stage_sets(src, dst, (a0, a1, b), dt=dt)
        gc.ghost_fill(dst)
    torch.cuda.synchronize()
    tu, tb = summary[-1]["tu"], summary[-1]["tb"]
    worst = {}
    nflag = 0

    def note(key, e):
        worst[key] = max(worst.get(key, 0.0), e)

    raw = 0.0
    for ib, blk in enumerate(blocks):
        ref = SP._outputs(om, 0, ib)
        dev = _download(gc, 0, ib)
        nflag += int(np.sum(ref[3] != 0))
        if np.any(dev[3] != ref[3]):
            # a decision at its threshold went the other way somewhere in the
            # chained run: the chained comparison stops at the flags
            say(f"  chained step: block {ib} decisions differ in {int(np.sum(dev[3] != ref[3]))} cells")
            continue
        TU = np.array(om.interior(tu[ib], ib))
        TB = [tb[ib][d][SP._face_slices(blk, d)] for d in range(3)]
        keep = np.ones(ref[3].shape, bool)
        r = SP.compare_block(om, ib, ref, dev, TU, TB, keep, [np.ones(f.shape, bool) for f in ref[2]],
                             note)
        raw = max(raw, max(r.values()))
    w = max(worst.values())
    say(f"  chained step on the device: gated {w:.1e} (bar {chained_tol:g}), pointwise {raw:.1e}")
    assert w < chained_tol, worst
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

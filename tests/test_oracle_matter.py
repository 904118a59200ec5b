"""Pins of the oracle's ADM matter sources (the fluid's stress-energy tensor
of Eq. 2 with Eq. 5 and 8, projected on the slice for the spacetime coupling
of Sec. III-A) and of its lapse excision (Sec. IV)."""
import copy

import numpy as np

import oracle as O
from paper_2409_10384_amd import inputs
from tests import fourmetric as FM
from tests.test_oracle_pins import P_IDEAL, hybrid_params, rand_state


def test_matter_sources_vs_the_four_metric_projections():
    rng = np.random.default_rng(90)
    for _ in range(40):
        g6, alpha, beta, rho, u3, P, B3 = rand_state(rng)
        eps = P / ((5.0 / 3.0 - 1.0) * rho)
        st = FM.state(alpha, beta, g6, rho, u3, P, B3, eps)
        E, S, Sij = FM.adm_projections(st)
        w = np.array([[rho], [u3[0]], [u3[1]], [u3[2]], [P]])
        bt = (B3 * st["sqrtg3"]).reshape(3, 1)
        got = O.matter_sources(w, bt, g6.reshape(6, 1), P_IDEAL)[:, 0]
        ref = np.array([E, *S, *[Sij[i, j] for i, j in FM.SYM]])
        scale = np.max(np.abs(ref))
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13 * scale)


def _hybrid_states(params, n, seed):
    """random states of the piecewise polytrope: cold part plus a thermal part"""
    rng = np.random.default_rng(seed)
    gam = np.array([1.0, 0.0, 0.0, 1.0, 0.0, 1.0])[:, None] + \
        0.05 * rng.normal(size=(6, n)) * np.array([1, 0.3, 0.3, 1, 0.3, 1])[:, None]
    rho = 10 ** rng.uniform(-6.0, -3.2, n)
    eps = O.eos(4, rho, 0.0, 0.0, params) + 10 ** rng.uniform(-4.0, -1.0, n)
    P = O.eos(0, rho, eps, 0.0, params)
    w = np.vstack([rho, rng.uniform(-0.8, 0.8, (3, n)), P])
    return w, rng.normal(size=(3, n)) * 1e-3, gam


def test_energy_and_momentum_densities_are_the_conserved_variables():
    """E sqrt(gamma) = tau~ + D~ and S_i sqrt(gamma) = S~_i (Eq. 7), for both
    equations of state, over wide random states"""
    st = inputs.c2p_states(4096, seed_offset=91, log_rho=(-8.0, -3.0))
    cases = [(P_IDEAL, st["w"], st["bt"], st["gam"])]
    hp = hybrid_params()
    cases.append((hp, *_hybrid_states(hp, 4096, 92)))
    for params, w, bt, gam in cases:
        out = O.matter_sources(w, bt, gam, params)
        U = O.prim2con(w, bt, gam, params)
        sg = np.sqrt(np.array([np.linalg.det(FM.gam33(gam[:, x])) for x in range(gam.shape[1])]))
        np.testing.assert_allclose(out[0] * sg, U[4] + U[0], rtol=1e-12)
        scale = np.max(np.abs(U[1:4]), axis=0) + 1e-300
        assert np.max(np.abs(out[1:4] * sg - U[1:4]) / scale) < 1e-12


def test_fluid_at_rest_without_field():
    """v = 0, B = 0: E = rho (1 + eps), S_i = 0, S_ij = P gamma_ij"""
    rng = np.random.default_rng(93)
    g6 = np.array([1.1, 0.05, -0.02, 0.95, 0.01, 1.05])
    rho, P = 0.3, 0.02
    w = np.array([[rho], [0.0], [0.0], [0.0], [P]])
    out = O.matter_sources(w, np.zeros((3, 1)), g6.reshape(6, 1), P_IDEAL)[:, 0]
    eps = P / (2.0 / 3.0 * rho)
    np.testing.assert_allclose(out[0], rho * (1 + eps), rtol=1e-15)
    np.testing.assert_allclose(out[1:4], 0.0, atol=1e-18)
    np.testing.assert_allclose(out[4:], P * g6, rtol=1e-15)


def _dipped_block():
    """smooth periodic block whose lapse dips below 0.2 in a ball"""
    blk = inputs.smooth_periodic_block(n=12, seed_offset=40)
    g = blk.ng
    s = blk.nx + 2 * g
    x = (np.arange(s) - g + 0.5) / blk.nx
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r2 = ((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2).transpose(2, 1, 0)
    blk.adm[0] = blk.adm[0] * (1.0 - 0.95 * np.exp(-r2 / 0.05))
    return blk


def test_excision_replaces_exactly_the_low_lapse_cells():
    """one stage with and without excision at alpha < 0.2: excised cells hold
    the atmosphere and the conserved state of the atmosphere with the
    unchanged field; every other cell, and every face, is bit-identical"""
    blk = _dipped_block()
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-8, T_atm=1e-6)
    ma, mb = O.Mesh([copy.deepcopy(blk)], p), O.Mesh([copy.deepcopy(blk)], p)
    dt = ma.dt(0.2)
    ma.stage(1, dt)
    mb.stage(1, dt)
    mb.excise(1, 0.2)
    alpha = mb.interior(mb.adm[0][0], 0)
    low = alpha < 0.2
    assert 0 < low.sum() < low.size
    wa, wb = mb.interior(ma.w1[0], 0), mb.interior(mb.w1[0], 0)
    ua, ub = mb.interior(ma.u1[0], 0), mb.interior(mb.u1[0], 0)
    assert np.array_equal(wa[:, ~low], wb[:, ~low]) and np.array_equal(ua[:, ~low], ub[:, ~low])
    assert np.all(wb[0][low] == p.rho_atm) and np.all(wb[1:4][:, low] == 0.0)
    np.testing.assert_allclose(wb[4][low], p.rho_atm * p.T_atm, rtol=1e-15)
    fl = mb.interior(mb.flags[0], 0)
    assert np.all(fl[low] & O.F_EXCISED) and not np.any(fl[~low] & O.F_EXCISED)
    bt = O.cell_bt(mb.b1[0])[:, blk.ng:-blk.ng, blk.ng:-blk.ng, blk.ng:-blk.ng]
    gam = mb.interior(mb.adm[0][4:10], 0)
    ref = O.prim2con(wb[:, low], bt[:, low], gam[:, low], p)
    np.testing.assert_array_equal(ub[:, low], ref)
    for d in range(3):
        assert np.array_equal(ma.b1[0][d], mb.b1[0][d])

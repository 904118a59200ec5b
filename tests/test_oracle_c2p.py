"""Pins of the oracle's conservative-to-primitive inversion and atmosphere rules.

The root of the Kastaun master function is labelled exactly by the generating
primitives, mu* = 1/(h W); the round trip prim -> cons -> prim is a closed
form; Brent's root is checked against plain bisection to its rounding band; each
atmosphere rule of the paper's floor policy gets one forced case.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2409_10384_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

P_C4 = O.Params(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30, f_thr=1.0, M_max=1e30,
                c2p_tol=1e-12)


def exact_mu(st, gamma=5.0 / 3.0):
    w = st["w"]
    eps = w[4] / ((gamma - 1.0) * w[0])
    h = 1.0 + eps + w[4] / w[0]
    return 1.0 / (h * st["W"])


def test_master_function_vanishes_at_exact_label():
    st = inputs.c2p_states(2000, seed_offset=101)
    u = O.prim2con(st["w"], st["bt"], st["gam"], P_C4)
    mu = exact_mu(st)
    f, fa = O.master(u, st["bt"], st["gam"], mu, P_C4)
    # |f| at the exact root is rounding-level relative to mu
    assert np.max(np.abs(f) / mu) < 1e-9, np.max(np.abs(f) / mu)
    # the auxiliary bound: mu* <= mu_+  <=>  f_a(mu*) <= 0
    assert np.all(fa <= 1e-12)


def test_root_accuracy_on_wide_ranges():
    """mu relative error <= 1e-10 against the exact label over the wide C2P
    ranges (log rho in [-10,-2], log eps in [-6,1], W in [1,10], b^2/rho up to
    10), with the solver tolerance 1e-12; no failures, no floors."""
    st = inputs.c2p_states(20000, seed_offset=102)
    u = O.prim2con(st["w"], st["bt"], st["gam"], P_C4)
    u2, w, flags, nev, mu = O.c2p(u, st["bt"], st["gam"], P_C4)
    assert np.all(flags == 0), np.unique(flags)
    mus = exact_mu(st)
    err = np.abs(mu - mus) / mus
    assert np.max(err) < 1e-10, np.max(err)
    # well-conditioned recovered quantities
    np.testing.assert_allclose(w[0], st["w"][0], rtol=1e-9)
    assert np.mean(nev) < 60


def test_round_trip_smooth_block_ranges():
    """prim -> cons -> prim to 1e-12 on the smooth block's ranges (rho ~ 1,
    P ~ 0.1, |v| <= 0.3, weak field, metric within 5% of flat)."""
    b = inputs.smooth_periodic_block(n=16)
    p = O.Params(gamma=5.0 / 3.0)
    w = b.w.reshape(5, -1)
    bt = O.cell_bt(b.bf).reshape(3, -1)
    gam = b.adm[4:10].reshape(6, -1)
    u = O.prim2con(w, bt, gam, p)
    _, w2, flags, nev, mu = O.c2p(u, bt, gam, p)
    assert np.all(flags == 0)
    np.testing.assert_allclose(w2[0], w[0], rtol=1e-13)
    np.testing.assert_allclose(w2[4], w[4], rtol=1e-12)
    for c in (1, 2, 3):
        np.testing.assert_allclose(w2[c], w[c], rtol=1e-12, atol=1e-13 * np.max(np.abs(w[c])))


def test_fluid_at_rest_without_field_closed_form():
    """B = 0, v = 0: mu = 1/h, rho = D, eps = tau/D."""
    n = 5
    rho = np.array([1e-8, 1e-4, 0.1, 1.0, 3.0])
    P = np.array([1e-10, 1e-6, 0.02, 0.5, 40.0])
    w = np.stack([rho, np.zeros(n), np.zeros(n), np.zeros(n), P])
    gam = np.tile(np.array([[1.0], [0], [0], [1.0], [0], [1.0]]), (1, n))
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30)
    u = O.prim2con(w, np.zeros((3, n)), gam, p)
    _, w2, flags, _, mu = O.c2p(u, np.zeros((3, n)), gam, p)
    eps = P / (2.0 / 3.0 * rho)
    h = 1 + eps + P / rho
    np.testing.assert_allclose(mu, 1.0 / h, rtol=1e-14)
    np.testing.assert_allclose(w2[0], rho, rtol=1e-15)
    np.testing.assert_allclose(w2[4], P, rtol=1e-12)


def test_brent_root_matches_bisection_within_rounding_band():
    """f(mu) carries ~1e-16 rounding noise, so its sign flips a few times
    within ~20 ulp of the root; Brent and bisection must agree to that band."""
    st = inputs.c2p_states(40, seed_offset=103)
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30, M_max=1e30, c2p_tol=0.0)
    u = O.prim2con(st["w"], st["bt"], st["gam"], p)
    _, _, flags, _, mu = O.c2p(u, st["bt"], st["gam"], p)
    assert np.all(flags == 0)
    for x in range(u.shape[1]):
        sl = lambda a: a[:, x:x + 1]
        f = lambda m: O.master(sl(u), sl(st["bt"]), sl(st["gam"]), np.array([m]), p)[0][0]
        lo, hi = 0.0, 1.0
        if f(hi) < 0:       # bracket end from the auxiliary bound
            hi = mu[x] * 2.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid in (lo, hi):
                break
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        assert abs(mu[x] - lo) <= 64 * np.spacing(lo), (x, mu[x], lo)


def test_learned_bracket_gives_the_same_root_and_fallback_flags():
    st = inputs.c2p_states(500, seed_offset=104)
    u = O.prim2con(st["w"], st["bt"], st["gam"], P_C4)
    _, w0, f0, n0, mu0 = O.c2p(u, st["bt"], st["gam"], P_C4)
    good_lo, good_hi = mu0 * (1 - 1e-3), mu0 * (1 + 1e-3)
    _, w1, f1, n1, mu1 = O.c2p(u, st["bt"], st["gam"], P_C4, good_lo, good_hi)
    assert np.all(f1 == 0)
    assert np.max(np.abs(mu1 - mu0) / mu0) < 1e-11
    assert np.mean(n1) < np.mean(n0)
    # a bracket that misses the root falls back to the full bracket
    bad_lo, bad_hi = mu0 * 1.5, mu0 * 2.0
    _, w2, f2, _, mu2 = O.c2p(u, st["bt"], st["gam"], P_C4, bad_lo, bad_hi)
    assert np.all(f2 == O.F_BRACKET_FALLBACK)
    assert np.max(np.abs(mu2 - mu0) / mu0) < 1e-11


# ---------------------------------------------------------------------------
# atmosphere rules, one forced case each
# ---------------------------------------------------------------------------
P_ATM = O.Params(gamma=5.0 / 3.0, rho_atm=1e-6, T_atm=1e-4, f_thr=10.0, M_max=50.0)
FLAT = np.array([[1.0], [0], [0], [1.0], [0], [1.0]])


def one(rho, u3, P, B3, p=P_ATM, gam=FLAT):
    w = np.array([[rho], [u3[0]], [u3[1]], [u3[2]], [P]])
    sg = math.sqrt(np.linalg.det(np.array([[gam[0, 0], gam[1, 0], gam[2, 0]],
                                           [gam[1, 0], gam[3, 0], gam[4, 0]],
                                           [gam[2, 0], gam[4, 0], gam[5, 0]]])))
    bt = np.array(B3, dtype=float).reshape(3, 1) * sg
    return w, bt, O.prim2con(w, bt, gam, p)


def atm_P(p):
    return p.rho_atm * p.T_atm


def test_rule_density_floor_resets_to_atmosphere():
    w, bt, u = one(5e-6, [0.1, 0, 0], 1e-5, [0.01, 0, 0])   # D < f_thr rho_atm = 1e-5
    u2, w2, fl, _, _ = O.c2p(u, bt, FLAT, P_ATM)
    assert fl[0] == O.F_DFLOOR
    np.testing.assert_array_equal(w2[:, 0], [P_ATM.rho_atm, 0, 0, 0, atm_P(P_ATM)])
    # conserved rewritten from the atmosphere prims (B unchanged)
    _, _, uref = one(P_ATM.rho_atm, [0, 0, 0], atm_P(P_ATM), [0.01, 0, 0])
    np.testing.assert_allclose(u2[:, 0], uref[:, 0], rtol=1e-15, atol=1e-30)


def test_rule_tau_floor():
    w, bt, u = one(1.0, [0.0, 0, 0], 1e-3, [0.0, 0, 0])
    u[4] = 0.5 * 1e-4 * 1.0 * 1.5 * 0.5        # below tau_atm = D eps(D, T_atm)
    _, w2, fl, _, _ = O.c2p(u, bt, FLAT, P_ATM)
    assert fl[0] & O.F_TAUFLOOR
    assert abs(w2[4, 0] - 1.0 * P_ATM.T_atm) < 1e-15


def test_rule_magnetisation_cap():
    w, bt, u = one(1e-3, [0.0, 0, 0], 1e-5, [0.5, 0, 0])   # B^2/D = 250 > 50
    _, w2, fl, _, _ = O.c2p(u, bt, FLAT, P_ATM)
    assert fl[0] & O.F_MAGCAP
    assert abs(w2[0, 0] - 0.25 / 50.0) < 1e-15 * 0.005 * 10


def test_rule_temperature_floor_keeps_rho_and_velocity():
    w, bt, u = one(0.5, [0.2, -0.1, 0.05], 0.5 * 1e-4 * 0.5, [0.01, 0.02, 0.0])
    u2, w2, fl, _, _ = O.c2p(u, bt, FLAT, P_ATM)
    assert fl[0] == O.F_TFLOOR
    np.testing.assert_allclose(w2[0:4, 0], w[0:4, 0], rtol=1e-12)
    assert abs(w2[4, 0] - 0.5 * P_ATM.T_atm) < 1e-18
    _, _, uref = one(w2[0, 0], w2[1:4, 0], w2[4, 0], [0.01, 0.02, 0.0])
    np.testing.assert_allclose(u2[:, 0], uref[:, 0], rtol=1e-15)


def test_state_at_the_floor_values_does_not_need_the_floor():
    """a fluid at rest at exactly (rho, T_atm) inverts back within rounding of
    T_atm and does not count as needing the T or tau floor"""
    rng = np.random.default_rng(9)
    for rho in 10 ** rng.uniform(-5, 0, size=50):
        P = rho * P_ATM.T_atm
        w, bt, u = one(rho, [0.0, 0.0, 0.0], P, [0.0, 0.0, 0.0])
        _, w2, fl, _, _ = O.c2p(u, bt, FLAT, P_ATM)
        assert fl[0] == 0, (rho, fl[0])
        assert abs(w2[4, 0] - P) <= 1e-12 * P


def test_rule_primitive_density_floor_after_inversion():
    # D above f_thr rho_atm, but rho = D/W below it
    W = 3.0
    v = math.sqrt(1 - 1 / W ** 2)
    w, bt, u = one(5e-6, [W * v, 0, 0], 5e-6 * 2e-4, [0, 0, 0])
    assert u[0, 0] > P_ATM.f_thr * P_ATM.rho_atm
    _, w2, fl, _, _ = O.c2p(u, bt, FLAT, P_ATM)
    assert fl[0] & O.F_RHOFLOOR
    np.testing.assert_array_equal(w2[:, 0], [P_ATM.rho_atm, 0, 0, 0, atm_P(P_ATM)])


def test_failure_policies_nan_and_iteration_cap():
    w, bt, u = one(1.0, [0.3, 0, 0], 0.1, [0.1, 0, 0])
    bad = u.copy()
    bad[1, 0] = np.nan
    _, w2, fl, _, _ = O.c2p(bad, bt, FLAT, P_ATM)
    assert fl[0] & O.F_C2P_FAIL
    assert np.all(np.isfinite(w2))
    np.testing.assert_array_equal(w2[:, 0], [P_ATM.rho_atm, 0, 0, 0, atm_P(P_ATM)])
    import dataclasses
    p1 = dataclasses.replace(P_ATM, c2p_maxit=1)
    _, w3, fl3, _, _ = O.c2p(u, bt, FLAT, p1)
    assert fl3[0] & O.F_C2P_FAIL and fl3[0] & O.F_MAXIT
    assert np.all(np.isfinite(w3))

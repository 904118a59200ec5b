"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks one oracle function against something other than itself:
closed forms, an independent 4-metric tensor route, finite differences,
invariants or exact special cases.  A plausible mistake (dropped term, wrong
sign or index, transposed operand) fails at least one of these.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import fourmetric as FM

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rand_metric(rng, dev=0.15):
    A = rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(A)
    lam = rng.uniform(1 - dev, 1 + dev, size=3)
    G = Q @ np.diag(lam) @ Q.T
    return np.array([G[i, j] for i, j in FM.SYM])


def rand_state(rng, vmax=0.7, bmax=0.8):
    g6 = rand_metric(rng)
    alpha = rng.uniform(0.6, 1.3)
    beta = rng.uniform(-0.2, 0.2, size=3)
    rho = 10 ** rng.uniform(-2, 0)
    P = rho * 10 ** rng.uniform(-2, 0.5)
    u3 = rng.uniform(-vmax, vmax, size=3)
    B3 = rng.uniform(-bmax, bmax, size=3)
    return g6, alpha, beta, rho, u3, P, B3


P_IDEAL = O.Params(gamma=5.0 / 3.0)


def hybrid_params():
    return O.Params(eos=1, npieces=3, K0=100.0, Gam=(2.8, 2.2, 3.0, 2.0), rho_b=(6.4e-5, 3.84e-4, 0),
                    gamma_th=1.75, rho_atm=1e-12, T_atm=1e-14, f_thr=1.0)


# ---------------------------------------------------------------------------
# EOS (ideal gas; hybrid piecewise polytrope + thermal part)
# ---------------------------------------------------------------------------
def test_eos_ideal_closed_form():
    rho = np.array([1e-8, 0.3, 2.0])
    eps = np.array([1e-5, 0.7, 3.0])
    P = O.eos(0, rho, eps, 0.0, P_IDEAL)
    np.testing.assert_allclose(P, (5.0 / 3.0 - 1.0) * rho * eps, rtol=1e-15)
    np.testing.assert_allclose(O.eos(1, rho, P, 0.0, P_IDEAL), eps, rtol=1e-15)
    np.testing.assert_allclose(O.eos(2, rho, P, 0.0, P_IDEAL), P / rho, rtol=1e-15)
    h = 1 + eps + P / rho
    np.testing.assert_allclose(O.eos(3, rho, eps, P, P_IDEAL), (5.0 / 3.0) * P / (rho * h), rtol=1e-14)


def test_eos_hybrid_continuity_and_cs2_by_finite_differences():
    p = hybrid_params()
    for rb in p.rho_b[:2]:
        lo, hi = rb * (1 - 1e-12), rb * (1 + 1e-12)
        pc = O.eos(5, np.array([lo, hi]), 0.0, 0.0, p)
        ec = O.eos(4, np.array([lo, hi]), 0.0, 0.0, p)
        assert abs(pc[1] - pc[0]) / pc[0] < 1e-10
        assert abs(ec[1] - ec[0]) / ec[0] < 1e-10
    # first piece: P_cold = K0 rho^G0, eps_cold = K0 rho^(G0-1)/(G0-1)
    r = 1e-6
    assert abs(O.eos(5, np.array([r]), 0, 0, p)[0] - 100.0 * r ** 2.8) / (100.0 * r ** 2.8) < 1e-14
    # c_s^2 = (dP/drho|eps + P/rho^2 dP/deps|rho) / h, by central differences
    for rho in [1e-5, 1e-4, 1e-3]:
        eps = O.eos(4, np.array([rho]), 0, 0, p)[0] * 1.3 + 1e-3
        Pf = lambda r, e: O.eos(0, np.array([r]), np.array([e]), 0, p)[0]
        P = Pf(rho, eps)
        hr, he = rho * 1e-6, eps * 1e-6
        dPdr = (Pf(rho + hr, eps) - Pf(rho - hr, eps)) / (2 * hr)
        dPde = (Pf(rho, eps + he) - Pf(rho, eps - he)) / (2 * he)
        h = 1 + eps + P / rho
        ref = (dPdr + P / rho ** 2 * dPde) / h
        got = O.eos(3, np.array([rho]), np.array([eps]), np.array([P]), p)[0]
        assert abs(got - ref) / ref < 1e-7


# ---------------------------------------------------------------------------
# Eq. 7 prim -> cons against the 4-metric route (Eq. 2, 5, 8)
# ---------------------------------------------------------------------------
def test_prim2con_vs_stress_energy_tensor():
    rng = np.random.default_rng(11)
    for _ in range(40):
        g6, alpha, beta, rho, u3, P, B3 = rand_state(rng)
        eps = P / ((5.0 / 3.0 - 1.0) * rho)
        st = FM.state(alpha, beta, g6, rho, u3, P, B3, eps)
        ref = FM.conserved(st)
        sg = st["sqrtg3"]
        w = np.array([[rho], [u3[0]], [u3[1]], [u3[2]], [P]])
        bt = (B3 * sg).reshape(3, 1)
        got = O.prim2con(w, bt, g6.reshape(6, 1), P_IDEAL)[:, 0]
        scale = np.max(np.abs(ref))
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * scale)


def test_prim2con_fluid_at_rest():
    """v = 0: D = rho, S = 0, tau = rho eps + B^2/2 (all times sqrt(gamma))."""
    rng = np.random.default_rng(12)
    g6 = rand_metric(rng)
    G = FM.gam33(g6)
    sg = math.sqrt(np.linalg.det(G))
    rho, P = 0.37, 0.05
    B = np.array([0.2, -0.1, 0.3])
    w = np.array([[rho], [0.0], [0.0], [0.0], [P]])
    u = O.prim2con(w, (B * sg).reshape(3, 1), g6.reshape(6, 1), P_IDEAL)[:, 0]
    eps = P / (2.0 / 3.0 * rho)
    np.testing.assert_allclose(u[0], sg * rho, rtol=1e-15)
    np.testing.assert_allclose(u[1:4], 0.0, atol=1e-17)
    np.testing.assert_allclose(u[4], sg * (rho * eps + 0.5 * B @ G @ B), rtol=1e-14)


# ---------------------------------------------------------------------------
# Eq. 9 fluxes against sqrt(-g) T^j_mu and sqrt(-g) *F^{ij}; wave speeds
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [0, 1, 2])
def test_fluxes_vs_stress_energy_tensor(d):
    rng = np.random.default_rng(20 + d)
    for _ in range(30):
        g6, alpha, beta, rho, u3, P, B3 = rand_state(rng)
        eps = P / ((5.0 / 3.0 - 1.0) * rho)
        st = FM.state(alpha, beta, g6, rho, u3, P, B3, eps)
        Fh, FB = FM.fluxes(st, d)
        q = np.array([[rho], [u3[0]], [u3[1]], [u3[2]], [P]])
        U, F, lm, lp = O.face_physics(d, q, B3.reshape(3, 1), np.array([alpha]),
                                      beta.reshape(3, 1), g6.reshape(6, 1), P_IDEAL)
        scale = max(np.max(np.abs(Fh)), 1e-300)
        np.testing.assert_allclose(F[:5, 0], Fh, rtol=1e-12, atol=1e-13 * scale)
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        np.testing.assert_allclose(F[5:, 0], [FB[t1], FB[t2]], rtol=1e-12,
                                   atol=1e-13 * np.max(np.abs(FB)))
        np.testing.assert_allclose(U[:5, 0], FM.conserved(st), rtol=1e-12,
                                   atol=1e-13 * np.max(np.abs(FM.conserved(st))))


def test_wave_speeds_relativistic_velocity_addition():
    """Flat space, B = 0, v along x: lambda = (v +- c_s)/(1 +- v c_s)."""
    g6 = np.array([1.0, 0, 0, 1.0, 0, 1.0])
    for v in [-0.9, -0.3, 0.0, 0.5, 0.95]:
        W = 1 / math.sqrt(1 - v * v)
        rho, P = 1.0, 0.4
        q = np.array([[rho], [W * v], [0.0], [0.0], [P]])
        _, _, lm, lp = O.face_physics(0, q, np.zeros((3, 1)), np.array([1.0]), np.zeros((3, 1)),
                                      g6.reshape(6, 1), P_IDEAL)
        h = 1 + P / (2 / 3 * rho) + P / rho
        cs = math.sqrt(5 / 3 * P / (rho * h))
        assert abs(lp[0] - (v + cs) / (1 + v * cs)) < 1e-14
        assert abs(lm[0] - (v - cs) / (1 - v * cs)) < 1e-14


def test_wave_speeds_are_jacobian_eigenvalues_hydro():
    """B = 0 in a curved metric: the extreme eigenvalues of dF/dU (finite
    differences through the primitive variables) equal lambda_-, lambda_+."""
    rng = np.random.default_rng(31)
    for _ in range(5):
        g6, alpha, beta, rho, u3, P, _ = rand_state(rng)
        d = int(rng.integers(0, 3))
        w0 = np.array([rho, *u3, P])

        def UF(w):
            q = w.reshape(5, 1)
            U, F, lm, lp = O.face_physics(d, q, np.zeros((3, 1)), np.array([alpha]),
                                          beta.reshape(3, 1), g6.reshape(6, 1), P_IDEAL)
            return U[:5, 0], F[:5, 0], lm[0], lp[0]

        _, _, lm, lp = UF(w0)
        JU = np.zeros((5, 5))
        JF = np.zeros((5, 5))
        for c in range(5):
            hstep = 1e-6 * max(abs(w0[c]), 1e-3)
            wp, wm = w0.copy(), w0.copy()
            wp[c] += hstep
            wm[c] -= hstep
            Up, Fp, _, _ = UF(wp)
            Um, Fm, _, _ = UF(wm)
            JU[:, c] = (Up - Um) / (2 * hstep)
            JF[:, c] = (Fp - Fm) / (2 * hstep)
        ev = np.sort(np.linalg.eigvals(JF @ np.linalg.inv(JU)).real)
        assert abs(ev[0] - lm) < 1e-6 * (1 + abs(lm))
        assert abs(ev[-1] - lp) < 1e-6 * (1 + abs(lp))


def test_wave_speed_perpendicular_field_at_rest():
    """v = 0, B perpendicular to x, flat: lambda = +-sqrt(cs^2 + ca^2 - cs^2 ca^2)."""
    rho, P, By = 1.0, 0.1, 0.7
    q = np.array([[rho], [0.0], [0.0], [0.0], [P]])
    _, _, lm, lp = O.face_physics(0, q, np.array([[0.0], [By], [0.0]]), np.array([1.0]),
                                  np.zeros((3, 1)), np.array([[1.0], [0], [0], [1.0], [0], [1.0]]), P_IDEAL)
    h = 1 + P / (2 / 3 * rho) + P / rho
    cs2 = 5 / 3 * P / (rho * h)
    ca2 = By ** 2 / (rho * h + By ** 2)
    c = math.sqrt(cs2 + ca2 - cs2 * ca2)
    assert abs(lp[0] - c) < 2e-16 * 4 and abs(lm[0] + c) < 2e-16 * 4


# ---------------------------------------------------------------------------
# Riemann solvers
# ---------------------------------------------------------------------------
def _rand_faces(rng, n):
    UL, FL, UR, FR = (rng.normal(size=(7, n)) for _ in range(4))
    lmL, lmR = -rng.uniform(0.1, 1, n), -rng.uniform(0.1, 1, n)
    lpL, lpR = rng.uniform(0.1, 1, n), rng.uniform(0.1, 1, n)
    return UL, FL, lmL, lpL, UR, FR, lmR, lpR


@pytest.mark.parametrize("kind", [0, 1])
def test_riemann_consistency(kind):
    """F(U, U) = F(U)."""
    rng = np.random.default_rng(40)
    UL, FL, lmL, lpL, _, _, lmR, lpR = _rand_faces(rng, 50)
    F = O.riemann(kind, UL, FL, lmL, lpL, UL, FL, lmR, lpR)
    np.testing.assert_allclose(F, FL, rtol=1e-14, atol=1e-14)


def test_hlle_upwinding_and_formula():
    rng = np.random.default_rng(41)
    UL, FL, lmL, lpL, UR, FR, lmR, lpR = _rand_faces(rng, 50)
    # all waves move right: F = F_L
    F = O.riemann(1, UL, FL, np.abs(lmL), lpL, UR, FR, np.abs(lmR), lpR)
    np.testing.assert_allclose(F, FL, rtol=1e-14)
    # all waves move left: F = F_R
    F = O.riemann(1, UL, FL, lmL, -np.abs(lpL), UR, FR, lmR, -np.abs(lpR))
    np.testing.assert_allclose(F, FR, rtol=1e-14)
    # subsonic: the two-wave HLLE average
    F = O.riemann(1, UL, FL, lmL, lpL, UR, FR, lmR, lpR)
    ar = np.maximum(lpL, lpR)
    al = np.minimum(lmL, lmR)
    ref = (ar * FL - al * FR + ar * al * (UR - UL)) / (ar - al)
    np.testing.assert_allclose(F, ref, rtol=1e-13)
    # LLF: central flux with the largest speed
    F = O.riemann(0, UL, FL, lmL, lpL, UR, FR, lmR, lpR)
    a = np.max(np.abs(np.stack([lmL, lpL, lmR, lpR])), axis=0)
    np.testing.assert_allclose(F, 0.5 * (FL + FR) - 0.5 * a * (UR - UL), rtol=1e-13)


@pytest.mark.parametrize("kind", [0, 1])
def test_mass_flux_dead_band(kind):
    """A face mass flux that vanishes in exact arithmetic (equal densities at
    rest on both sides, differing only by rounding) comes out exactly zero, so
    the upwind CT averages instead of following the sign of the noise; a real
    mass flux a million times larger than the noise passes unchanged."""
    n = 6
    UL = np.zeros((7, n)); UR = np.zeros((7, n)); FL = np.zeros((7, n)); FR = np.zeros((7, n))
    D = np.array([1.28e-13, 1.0, 3.7e-7, 2.0, 5e-9, 1.0])
    UL[0] = D
    UR[0] = D * (1 + np.array([1, -1, 2, -3, 1, 4]) * 2.0 ** -52)
    lm = np.full(n, -0.3); lp = np.full(n, 0.5)
    F = O.riemann(kind, UL, FL, lm, lp, UR, FR, lm, lp)
    assert np.all(F[0] == 0.0)
    UR[0] = D * (1 + 1e-9)
    F = O.riemann(kind, UL, FL, lm, lp, UR, FR, lm, lp)
    if kind == 1:
        ref = (-0.3 * 0.5) * (UR[0] - UL[0]) / 0.8
    else:
        ref = -0.5 * 0.5 * (UR[0] - UL[0])
    np.testing.assert_allclose(F[0], ref, rtol=1e-6)


# ---------------------------------------------------------------------------
# WENOZ reconstruction
# ---------------------------------------------------------------------------
def test_wenoz_exact_for_quadratics_and_constants():
    """Every three-cell candidate is exact for cell averages of a quadratic, so
    the weighted value equals the point value at the interface."""
    rng = np.random.default_rng(50)
    for _ in range(20):
        a, b, c = rng.normal(size=3)
        hh = 0.1
        # cell averages of p(x) = a + b x + c x^2 over [x_i - h/2, x_i + h/2]
        xs = np.arange(-2, 3) * hh
        avg = a + b * xs + c * (xs ** 2 + hh ** 2 / 12)
        xf = 0.5 * hh
        exact = a + b * xf + c * xf ** 2
        got = O.wenoz(avg)[0]
        assert abs(got - exact) < 1e-13 * (1 + abs(exact))
    assert O.wenoz(np.full(5, 3.25))[0] == 3.25


def test_wenoz_fifth_order_on_smooth_data():
    errs = []
    for n in [20, 40, 80]:
        hh = 1.0 / n
        i = np.arange(n)
        x = (i + 0.5) * hh
        # cell averages of sin(2 pi x)
        avg = (np.cos(2 * np.pi * (x - hh / 2)) - np.cos(2 * np.pi * (x + hh / 2))) / (2 * np.pi * hh)
        st = np.stack([np.roll(avg, 2), np.roll(avg, 1), avg, np.roll(avg, -1), np.roll(avg, -2)], 1)
        got = O.wenoz(st)
        errs.append(np.max(np.abs(got - np.sin(2 * np.pi * (x + hh / 2)))))
    order = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(order) > 4.5, (errs, order)


def test_wenoz_selects_smooth_stencil_at_jump():
    got = O.wenoz(np.array([1.0, 1.0, 1.0, 0.0, 0.0]))[0]
    assert abs(got - 1.0) < 1e-10
    got = O.wenoz(np.array([0.0, 0.0, 1.0, 1.0, 1.0]))[0]
    assert abs(got - 1.0) < 1e-10


# ---------------------------------------------------------------------------
# Eq. 10 sources against the 4-metric forms
# ---------------------------------------------------------------------------
def _metric_derivs(rng):
    dal = rng.normal(size=3) * 0.1
    dbe = rng.normal(size=(3, 3)) * 0.1        # [i][j] = d_i beta^j
    dg = rng.normal(size=(3, 6)) * 0.1         # [i][jk] = d_i gamma_jk
    return dal, dbe, dg


def _dg4(alpha, beta, G, dal, dbe, dg, dt_alpha=0.0, dt_beta=None, dt_G=None):
    """d_mu g_{nu lam} (mu = 0 time, 1..3 space) from the ADM derivatives."""
    out = np.zeros((4, 4, 4))
    ders = []
    dt_beta = np.zeros(3) if dt_beta is None else dt_beta
    dt_G = np.zeros((3, 3)) if dt_G is None else dt_G
    ders.append((dt_alpha, dt_beta, dt_G))
    for i in range(3):
        ders.append((dal[i], dbe[i], FM.gam33(dg[i])))
    for mu, (da, db, dG) in enumerate(ders):
        beta_l = G @ beta
        d_beta_l = dG @ beta + G @ db
        out[mu, 0, 0] = -2 * alpha * da + d_beta_l @ beta + beta_l @ db
        out[mu, 0, 1:] = out[mu, 1:, 0] = d_beta_l
        out[mu, 1:, 1:] = dG
    return out


def test_momentum_source_vs_half_sqrtg_T_dg():
    """G^S_i = 1/2 sqrt(-g) T^{mu nu} d_i g_{mu nu} for any metric derivatives."""
    rng = np.random.default_rng(60)
    for _ in range(20):
        g6, alpha, beta, rho, u3, P, B3 = rand_state(rng)
        eps = P / (2 / 3 * rho)
        st = FM.state(alpha, beta, g6, rho, u3, P, B3, eps)
        dal, dbe, dg = _metric_derivs(rng)
        K6 = rng.normal(size=6) * 0.1
        U = FM.conserved(st)
        G = O.sources_point(np.array([rho, *u3, P]), B3 * st["sqrtg3"], U, g6, alpha, dal, dbe, dg,
                            K6, P_IDEAL)
        d4 = _dg4(alpha, beta, st["G"], dal, dbe, dg)
        ref = np.array([0.5 * st["sqrtg4"] * np.sum(st["T"] * d4[1 + i]) for i in range(3)])
        np.testing.assert_allclose(G[1:4], ref, rtol=1e-11, atol=1e-12 * np.max(np.abs(ref)))
        assert G[0] == 0.0


def test_energy_source_vs_four_metric_christoffel_form():
    """G^tau = sqrt(-g) (T^{mu 0} d_mu alpha - alpha T^{mu nu} Gamma^0_{mu nu}) with
    d_t gamma_ij = -2 alpha K_ij + D_i beta_j + D_j beta_i; arbitrary d_t alpha
    and d_t beta^i must drop out."""
    rng = np.random.default_rng(61)
    for _ in range(20):
        g6, alpha, beta, rho, u3, P, B3 = rand_state(rng)
        eps = P / (2 / 3 * rho)
        st = FM.state(alpha, beta, g6, rho, u3, P, B3, eps)
        G33 = st["G"]
        dal, dbe, dg = _metric_derivs(rng)
        K6 = rng.normal(size=6) * 0.1
        K = FM.gam33(K6)
        dG = np.array([FM.gam33(dg[i]) for i in range(3)])     # dG[a, b, c] = d_a g_bc
        Gi = np.linalg.inv(G33)
        # Gamma^k_ij = 1/2 g^kl (d_i g_lj + d_j g_li - d_l g_ij)
        bracket = np.transpose(dG, (1, 0, 2)) + np.transpose(dG, (1, 2, 0)) - dG
        chr3 = 0.5 * np.einsum("kl,lij->kij", Gi, bracket)
        beta_l = G33 @ beta
        d_beta_l = np.array([dG[i] @ beta + G33 @ dbe[i] for i in range(3)])   # [i][j] = d_i beta_j
        Dbeta = d_beta_l - np.einsum("kij,k->ij", chr3, beta_l)
        dtG = -2 * alpha * K + Dbeta + Dbeta.T
        dt_alpha = rng.normal()
        d4 = _dg4(alpha, beta, G33, dal, dbe, dg, dt_alpha=dt_alpha, dt_beta=rng.normal(size=3),
                  dt_G=dtG)
        g4i = st["gi"]
        # Gamma^0_{mu nu} = 1/2 g^{0 l} (d_mu g_{l nu} + d_nu g_{l mu} - d_l g_{mu nu})
        Gam0 = 0.5 * (np.einsum("l,mln->mn", g4i[0], d4) + np.einsum("l,nlm->mn", g4i[0], d4)
                      - np.einsum("l,lmn->mn", g4i[0], d4))
        T = st["T"]
        dalpha4 = np.array([dt_alpha, *dal])
        ref = st["sqrtg4"] * (T[:, 0] @ dalpha4 - alpha * np.sum(T * Gam0))
        U = FM.conserved(st)
        Gs = O.sources_point(np.array([rho, *u3, P]), B3 * st["sqrtg3"], U, g6, alpha, dal, dbe, dg,
                             K6, P_IDEAL)
        assert abs(Gs[4] - ref) < 1e-11 * (1 + abs(ref)), (Gs[4], ref)

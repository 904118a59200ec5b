"""Exact solution of the one-dimensional special-relativistic Riemann problem
of an ideal gas without magnetic field or tangential velocity (Marti &
Mueller 1994, J. Fluid Mech. 258, 317; also their Living Review, Sec. on the
exact solution).  Test infrastructure, written from the published relations:

* rarefactions follow the isentrope P / rho^Gamma = const with the Riemann
  invariant of the simple wave, which for an ideal gas gives
      v_b = ((1 + v_a) A - (1 - v_a)) / ((1 + v_a) A + (1 - v_a)),
      A = [((g - c_b)/(g + c_b)) ((g + c_a)/(g - c_a))]^(+-2/g),  g = sqrt(Gamma - 1)
  (+ for the wave moving left, - for the one moving right);
* shocks follow the Taub adiabat [h^2] = (h_b/rho_b + h_a/rho_a)[P] (a
  quadratic in h_b for an ideal gas), the mass flux j^2 = -[P]/[h/rho], the
  shock speed and the post-shock velocity of the same paper;
* the pressure of the two intermediate states solves v_L*(P) = v_R*(P).

The test suite checks the shock relations against the conservation laws
before using the solution.
"""
import numpy as np
from scipy.optimize import brentq


class State:
    def __init__(self, rho, p, v, gam):
        self.rho, self.p, self.v, self.gam = float(rho), float(p), float(v), float(gam)

    @property
    def h(self):
        return 1.0 + self.gam / (self.gam - 1.0) * self.p / self.rho

    @property
    def cs(self):
        return np.sqrt(self.gam * self.p / (self.rho * self.h))

    @property
    def W(self):
        return 1.0 / np.sqrt(1.0 - self.v ** 2)


def _cs(rho, p, gam):
    h = 1.0 + gam / (gam - 1.0) * p / rho
    return np.sqrt(gam * p / (rho * h))


def rarefaction(a: State, pb, side):
    """state behind a rarefaction of side 'L' (moving left) or 'R'"""
    gam = a.gam
    g = np.sqrt(gam - 1.0)
    rb = a.rho * (pb / a.p) ** (1.0 / gam)
    cb = _cs(rb, pb, gam)
    ratio = ((g - cb) / (g + cb)) * ((g + a.cs) / (g - a.cs))
    A = ratio ** ((2.0 if side == "L" else -2.0) / g)
    vb = ((1.0 + a.v) * A - (1.0 - a.v)) / ((1.0 + a.v) * A + (1.0 - a.v))
    return State(rb, pb, vb, gam)


def shock(a: State, pb, side):
    """state behind a shock of side 'L' or 'R', and the shock speed"""
    gam = a.gam
    ha = a.h
    dp = a.p - pb
    A2 = 1.0 + (gam - 1.0) * dp / (gam * pb)
    B2 = -(gam - 1.0) * dp / (gam * pb)
    C2 = ha * dp / a.rho - ha * ha
    hb = (-B2 + np.sqrt(B2 * B2 - 4.0 * A2 * C2)) / (2.0 * A2)
    rb = gam * pb / ((gam - 1.0) * (hb - 1.0))
    j2 = -(pb - a.p) / (hb / rb - ha / a.rho)
    j = np.sqrt(j2) * (1.0 if side == "R" else -1.0)
    rw2 = (a.rho * a.W) ** 2
    Vs = (rw2 * a.v + j * np.sqrt(j2 + rw2 * (1.0 - a.v ** 2))) / (rw2 + j2)
    Ws = 1.0 / np.sqrt(1.0 - Vs * Vs)
    vb = (ha * a.W * a.v + Ws * (pb - a.p) / j) / \
        (ha * a.W + (pb - a.p) * (Ws * a.v / j + 1.0 / (a.rho * a.W)))
    return State(rb, pb, vb, gam), Vs


def behind(a: State, pb, side):
    if pb > a.p:
        return shock(a, pb, side)[0]
    return rarefaction(a, pb, side)


def solve(L: State, R: State):
    """pressure and velocity of the intermediate states"""
    f = lambda p: behind(L, p, "L").v - behind(R, p, "R").v
    lo, hi = 1e-14 * min(L.p, R.p), 10.0 * max(L.p, R.p)
    while f(hi) > 0.0:
        hi *= 10.0
    ps = brentq(f, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
    return ps, behind(L, ps, "L").v


def sample(L: State, R: State, xi):
    """(rho, p, v) at the self-similar coordinates xi = (x - x0) / t"""
    ps, vs = solve(L, R)
    out = np.zeros((3, len(xi)))
    SL, SR = behind(L, ps, "L"), behind(R, ps, "R")
    for n, x in enumerate(np.asarray(xi, dtype=float)):
        if x < vs:      # left of the contact
            a, s = L, SL
            if ps > L.p:
                _, Vs = shock(L, ps, "L")
                st = L if x < Vs else s
            else:
                head = (L.v - L.cs) / (1.0 - L.v * L.cs)
                tail = (s.v - s.cs) / (1.0 - s.v * s.cs)
                if x < head:
                    st = L
                elif x > tail:
                    st = s
                else:
                    g = lambda p: (lambda q: (q.v - q.cs) / (1.0 - q.v * q.cs) - x)(rarefaction(L, p, "L"))
                    st = rarefaction(L, brentq(g, ps, L.p, rtol=1e-14), "L")
        else:
            a, s = R, SR
            if ps > R.p:
                _, Vs = shock(R, ps, "R")
                st = R if x > Vs else s
            else:
                head = (R.v + R.cs) / (1.0 + R.v * R.cs)
                tail = (s.v + s.cs) / (1.0 + s.v * s.cs)
                if x > head:
                    st = R
                elif x < tail:
                    st = s
                else:
                    g = lambda p: (lambda q: (q.v + q.cs) / (1.0 + q.v * q.cs) - x)(rarefaction(R, p, "R"))
                    st = rarefaction(R, brentq(g, ps, R.p, rtol=1e-14), "R")
        out[:, n] = st.rho, st.p, st.v
    return out

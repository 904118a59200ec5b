"""Independent 4-metric route to the Valencia quantities (test helper).

Builds g_{mu nu} from (alpha, beta^i, gamma_ij) (Eq. 5), the 4-velocity and
b^mu from (rho, W v^i, B^i) (Eq. 8 through u^mu and the projections), the
stress-energy tensor of Eq. 2 and the dual Faraday tensor of Eq. 3, and reads
conserved variables, fluxes and sources off them with full 4x4 tensor
algebra.  Shares nothing with the oracle.
"""
import numpy as np

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def gam33(g6):
    G = np.zeros((3, 3))
    for c, (i, j) in enumerate(SYM):
        G[i, j] = G[j, i] = g6[c]
    return G


def four_metric(alpha, beta, G):
    beta_l = G @ beta
    g = np.zeros((4, 4))
    g[0, 0] = -alpha ** 2 + beta @ beta_l
    g[0, 1:] = g[1:, 0] = beta_l
    g[1:, 1:] = G
    return g


def state(alpha, beta, g6, rho, u3, P, B3, eps):
    """u3 = W v^i (Eulerian), B3 = Eulerian B^i (un-densitized)."""
    G = gam33(g6)
    g = four_metric(alpha, beta, G)
    gi = np.linalg.inv(g)
    W = np.sqrt(1.0 + u3 @ G @ u3)
    v = u3 / W
    # u^mu = W n^mu + W v^i e_i: n^mu = (1/alpha, -beta/alpha)
    umu = np.zeros(4)
    umu[0] = W / alpha
    umu[1:] = W * (v - beta / alpha)
    n_up = np.array([1.0 / alpha, *(-beta / alpha)])
    # B^mu (Eulerian field vector) = (0, B^i); b^mu = (B^mu + (u.B) u^mu)/W ... projection
    Bmu = np.array([0.0, *B3])
    uB = umu @ g @ Bmu
    bmu = (Bmu + uB * umu) / W
    h = 1.0 + eps + P / rho
    b2 = bmu @ g @ bmu
    T = (rho * h + b2) * np.outer(umu, umu) + (P + 0.5 * b2) * gi - np.outer(bmu, bmu)
    sqrtg3 = np.sqrt(np.linalg.det(G))
    sqrtg4 = alpha * sqrtg3
    return dict(G=G, g=g, gi=gi, W=W, v=v, umu=umu, bmu=bmu, T=T, sqrtg3=sqrtg3,
                sqrtg4=sqrtg4, n_up=n_up, rho=rho, b2=b2)


def conserved(st):
    """D~ = sqrt(-g) rho u^0; S~_i = sqrt(-g) T^0_i; tau~ = sqrt(-g)(alpha T^00 - rho u^0)."""
    T, g, sg4 = st["T"], st["g"], st["sqrtg4"]
    alpha = 1.0 / st["n_up"][0]
    Tmixed = T @ g  # T^mu_nu
    D = sg4 * st["rho"] * st["umu"][0]
    S = sg4 * Tmixed[0, 1:]
    tau = sg4 * (alpha * T[0, 0] - st["rho"] * st["umu"][0])
    return np.array([D, *S, tau])


def fluxes(st, d):
    """direction d (0..2): F(D~) = sqrt(-g) rho u^j; F(S~_i) = sqrt(-g) T^j_i;
    F(tau~) = sqrt(-g)(alpha T^{0j} - rho u^j); F(B~^i) = sqrt(-g) (*F)^{ij}
    with *F^{mu nu} = b^mu u^nu - b^nu u^mu."""
    T, g, sg4 = st["T"], st["g"], st["sqrtg4"]
    alpha = 1.0 / st["n_up"][0]
    j = d + 1
    Tmixed = T @ g
    F = np.zeros(5)
    F[0] = sg4 * st["rho"] * st["umu"][j]
    F[1:4] = sg4 * Tmixed[j, 1:]
    F[4] = sg4 * (alpha * T[0, j] - st["rho"] * st["umu"][j])
    b, u = st["bmu"], st["umu"]
    dual = np.outer(b, u) - np.outer(u, b)
    FB = sg4 * dual[1:, j]   # flux of B~^i in direction j: sqrt(-g) *F^{ij}
    return F, FB


def adm_projections(st):
    """E = n_mu n_nu T^{mu nu}, S_i = -gamma_i^mu n^nu T_{mu nu} and
    S_ij = gamma_i^mu gamma_j^nu T_{mu nu}, by 4x4 algebra with n_mu = (-alpha, 0)."""
    g, T = st["g"], st["T"]
    alpha = 1.0 / st["n_up"][0]
    n_dn = np.array([-alpha, 0.0, 0.0, 0.0])
    n_up = st["n_up"]
    T_dn = g @ T @ g
    proj = np.eye(4) + np.outer(n_up, n_dn)          # gamma^mu_nu
    E = n_dn @ T @ n_dn
    S = -(proj.T @ T_dn @ n_up)[1:]
    Sij = (proj.T @ T_dn @ proj)[1:, 1:]
    return E, S, Sij

"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module builds initial data only: primitive fields (rho, W v^i, P), the
densitized face field B~ as the discrete curl of an edge vector potential, and
the ADM fields (alpha, beta^i, gamma_ij, K_ij) at cell centres.  It holds none
of the method's arithmetic (no prim->cons, no fluxes, no inversion): each side
computes the conserved state from these inputs with its own code.

Layout of one block (all float64, C order, index [k, j, i] with i fastest):
  cells   (sz, sy, sx)          sx = nx + 2 ng, ...
  x-faces (sz, sy, sx + 1)      face i = left face of cell i
  y-faces (sz, sy + 1, sx)
  z-faces (sz + 1, sy, sx)
  adm     (16, sz, sy, sx)      alpha, beta^x..z, g_xx g_xy g_xz g_yy g_yz g_zz,
                                K_xx K_xy K_xz K_yy K_yz K_zz

Workloads (seed = 2409_10384 + workload index):
  smooth_periodic_block  one periodic MeshBlock of sums of three random
                         sinusoids (rho = 1 + 0.1 s, P = 0.1 + 0.01 s, ...)
  star_blocks            a synthetic star rho = rho_c (1 - r^2/R^2) in a
                         conformally flat metric, poloidal field from
                         A_phi ~ max(P - 0.04 P_max, 0), tiled into blocks
  refined_star_blocks    the same star sampled on ~1500 blocks of 16^3, 24^3
                         and 32^3 cells spread over 6 refinement levels
                         (independent blocks with frozen ghosts)
  leaf_mesh              a refined mesh: leaves of a 2:1-balanced octree of
                         equal blocks (the structure only)
  smooth_leaf_blocks     smooth periodic data on such a mesh, the face field
                         the discrete curl of a vector potential whose
                         components do not depend on their own coordinate
                         (so coarse faces are the means of fine faces exactly)
  star_leaf_blocks       the star on a leaf mesh refined towards its centre
  c2p_states             random primitive states over wide ranges of density,
                         specific energy, Lorentz factor and magnetisation in
                         random SPD 3-metrics near flat
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2409_10384


def _sqrt(a):
    return a.sqrt() if hasattr(a, "sqrt") and not isinstance(a, np.ndarray) else np.sqrt(a)


def _maximum(a, b):
    if isinstance(a, np.ndarray):
        return np.maximum(a, b)
    import torch
    return torch.maximum(a, b)


def _maxs(a, s):
    """elementwise max(a, scalar) for numpy arrays or torch tensors"""
    if isinstance(a, np.ndarray) or np.isscalar(a):
        return np.maximum(a, s)
    return a.clamp(min=s)


def _where(c, a, b):
    if isinstance(c, np.ndarray) or np.isscalar(c):
        return np.where(c, a, b)
    import torch
    return torch.where(c, a, b)


def pp_cold_pressure(rho, pp, K):
    """cold pressure K_i rho^Gamma_i of the 3-piece polytrope of pp_eos"""
    G, rb = pp["Gam"], pp["rho_b"]
    return _where(rho < rb[0], K[0] * rho ** G[0],
                  _where(rho < rb[1], K[1] * rho ** G[1], K[2] * rho ** G[2]))


def pp_eos(seed_offset=5, rho_c=1.28e-3, K_ref=100.0, gamma_th=1.75):
    """Seeded 3-piece cold piecewise polytrope with a thermal part (the
    end-to-end star's gas): adiabatic indices Gamma_i ~ U[1.8, 3.2], dividing
    densities rho_c * {0.05, 0.3}, and K of the lowest piece chosen so that
    the cold pressure at rho_c is K_ref rho_c^2 with P continuous at the
    dividing densities.  Returns the EOS fields of the method parameters
    (eos, npieces, rho_b, K0, Gam, gamma_th) and the per-piece K."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    G = rng.uniform(1.8, 3.2, size=3)
    rb = (0.05 * rho_c, 0.3 * rho_c)
    K2 = K_ref * rho_c ** 2 / rho_c ** G[2]
    K1 = K2 * rb[1] ** G[2] / rb[1] ** G[1]
    K0 = K1 * rb[0] ** G[1] / rb[0] ** G[0]
    return dict(eos=1, npieces=3, rho_b=(rb[0], rb[1], 0.0), K0=float(K0),
                Gam=(float(G[0]), float(G[1]), float(G[2]), float(G[2])),
                gamma_th=gamma_th), (float(K0), float(K1), float(K2))

# neighbour table order: (ox+1) + 3 (oy+1) + 9 (oz+1)
def nbr_index(ox: int, oy: int, oz: int) -> int:
    return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)


@dataclasses.dataclass
class BlockInit:
    """Initial data of one MeshBlock (host numpy arrays)."""

    nx: int
    ny: int
    nz: int
    ng: int
    dx: tuple
    w: np.ndarray          # (5, sz, sy, sx): rho, W v^x, W v^y, W v^z, P
    bf: list               # 3 face arrays of densitized B~
    adm: np.ndarray        # (16, sz, sy, sx)
    nbr: list              # 27 neighbour block indices, -1 = none (outflow)
    bc: int                # 0 ghosts frozen, 1 ghosts filled from neighbours
    level: int = 0
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def shape(self):
        g = self.ng
        return (self.nz + 2 * g, self.ny + 2 * g, self.nx + 2 * g)

    @property
    def ncell_interior(self):
        return self.nx * self.ny * self.nz


def face_shape(sz, sy, sx, d):
    return [(sz, sy, sx + 1), (sz, sy + 1, sx), (sz + 1, sy, sx)][d]


# ---------------------------------------------------------------------------
# smooth periodic block (sums of three random sinusoids)
# ---------------------------------------------------------------------------
def _random_waves(rng, nwaves=3):
    ks = []
    while len(ks) < nwaves:
        k = rng.integers(-2, 3, size=3)
        if np.any(k != 0):
            ks.append(k)
    phis = rng.uniform(0.0, 2.0 * np.pi, size=nwaves)
    return np.array(ks, dtype=np.float64), phis


def _wave_sum(ks, phis, x, y, z):
    s = np.zeros(np.broadcast(x, y, z).shape)
    for k, ph in zip(ks, phis):
        s += np.sin(2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
    return s / len(phis)


def _wrap_pad_cells(a, g):
    return np.pad(a, [(g, g)] * 3, mode="wrap")


def _wrap_pad_face(a, g, d):
    """a: periodic lattice of faces along d (N per axis, lattice face 0 at the
    lower boundary).  Padded face index f in [0, N + 2g] maps to lattice face
    (f - g) mod N; the cell axes are padded as cells."""
    out = a
    for ax in range(3):
        n = a.shape[ax]
        cnt = n + 2 * g + (1 if ax == 2 - d else 0)
        idx = (np.arange(cnt) - g) % n
        out = np.take(out, idx, axis=ax)
    return out


def smooth_periodic_block(n=32, ng=3, seed_offset=0, amp_rho=0.1, amp_p=0.01, amp_v=0.3,
                          amp_a=0.05, amp_lapse=0.05, amp_shift=0.01, amp_g=0.05, amp_k=0.01,
                          const_metric=None, uniform=None, shape=None):
    """One periodic block on [0,1)^3 with n^3 cells and ng ghost layers.

    Every field draws its own three integer wave vectors k in [-2,2]^3 \\ 0
    and phases.  rho = 1 + amp_rho s, P = 0.1 + amp_p s, W v^i = amp_v s_i /
    sqrt(3), alpha = 1 + amp_lapse s, beta^i = amp_shift s, gamma_ij =
    delta_ij + amp_g s_ij, K_ij = amp_k s_ij; A_i = amp_a s_{A_i} on edges and
    B~ = discrete curl of A (so div B~ = 0 to round-off).

    const_metric: optional (alpha, beta[3], gamma6[6]) for a spatially
    constant metric with K_ij = 0 (free-stream tests).
    uniform: optional (rho, u3, P, Bt3) to replace the matter fields by a
    uniform state with a uniform densitized face field.
    shape: optional (nx, ny, nz) for a non-cubic periodic block (cell size
    1/n along every axis)."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    h = 1.0 / n
    nx, ny, nz = shape if shape is not None else (n, n, n)
    ic = [(np.arange(m) + 0.5) * h for m in (nx, ny, nz)]     # cell centres
    ifc = [np.arange(m) * h for m in (nx, ny, nz)]            # faces (lower)
    Z, Y, X = np.meshgrid(ic[2], ic[1], ic[0], indexing="ij")

    def field():
        ks, ph = _random_waves(rng)
        return _wave_sum(ks, ph, X, Y, Z)

    rho = 1.0 + amp_rho * field()
    P = 0.1 + amp_p * field()
    u = [amp_v * field() / math.sqrt(3.0) for _ in range(3)]
    alpha = 1.0 + amp_lapse * field()
    beta = [amp_shift * field() for _ in range(3)]
    gam = []
    for c in range(6):
        diag = c in (0, 3, 5)
        gam.append((1.0 if diag else 0.0) + amp_g * field())
    K = [amp_k * field() for _ in range(6)]
    if const_metric is not None:
        a0, b0, g0 = const_metric
        alpha = np.full_like(rho, a0)
        beta = [np.full_like(rho, b0[c]) for c in range(3)]
        gam = [np.full_like(rho, g0[c]) for c in range(6)]
        K = [np.zeros_like(rho) for _ in range(6)]
    # edge vector potential: A_x at (x_c, y_f, z_f), A_y at (x_f, y_c, z_f), A_z at (x_f, y_f, z_c)
    ksx, phx = _random_waves(rng)
    ksy, phy = _random_waves(rng)
    ksz, phz = _random_waves(rng)
    Zf, Yf, Xc = np.meshgrid(ifc[2], ifc[1], ic[0], indexing="ij")
    Ax = amp_a * _wave_sum(ksx, phx, Xc, Yf, Zf)
    Zf2, Yc2, Xf2 = np.meshgrid(ifc[2], ic[1], ifc[0], indexing="ij")
    Ay = amp_a * _wave_sum(ksy, phy, Xf2, Yc2, Zf2)
    Zc3, Yf3, Xf3 = np.meshgrid(ic[2], ifc[1], ifc[0], indexing="ij")
    Az = amp_a * _wave_sum(ksz, phz, Xf3, Yf3, Zc3)
    # discrete curl on the periodic lattice (arrays indexed [k, j, i])
    def sh(a, ax):  # value at index + 1 along axis ax (periodic)
        return np.roll(a, -1, axis=ax)
    Bx = (sh(Az, 1) - Az) / h - (sh(Ay, 0) - Ay) / h
    By = (sh(Ax, 0) - Ax) / h - (sh(Az, 2) - Az) / h
    Bz = (sh(Ay, 2) - Ay) / h - (sh(Ax, 1) - Ax) / h
    if uniform is not None:
        r0, u0, p0, b0 = uniform
        rho = np.full_like(rho, r0)
        P = np.full_like(rho, p0)
        u = [np.full_like(rho, u0[c]) for c in range(3)]
        Bx, By, Bz = (np.full_like(rho, b0[c]) for c in range(3))

    w = np.stack([_wrap_pad_cells(a, ng) for a in [rho, u[0], u[1], u[2], P]])
    adm = np.stack([_wrap_pad_cells(a, ng) for a in [alpha] + beta + gam + K])
    bf = [_wrap_pad_face(Bx, ng, 0), _wrap_pad_face(By, ng, 1), _wrap_pad_face(Bz, ng, 2)]
    nbr = [0] * 27
    return BlockInit(nx, ny, nz, ng, (h, h, h), np.ascontiguousarray(w),
                     [np.ascontiguousarray(b) for b in bf], np.ascontiguousarray(adm), nbr, 1)


# ---------------------------------------------------------------------------
# synthetic star (conformally flat metric, poloidal field)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class StarSetup:
    rho_c: float = 1.28e-3
    radius: float = 9.6           # 0.4 of the box [-12, 12]
    K: float = 100.0
    Gamma: float = 2.0
    mass: float = 1.4
    rho_atm: float = 1.28e-13
    T_atm: float = 1.28e-11
    beta_min: float = 100.0       # minimum plasma beta 2P/b^2
    box: float = 12.0
    pcut: float = 0.04
    A_b: float = 0.0              # set by calibrate_field
    pp: dict | None = None        # piecewise-polytrope gas (pp_eos); None: P = K rho^Gamma
    pp_K: tuple = ()
    center: tuple = (0.0, 0.0, 0.0)   # star centre (the origin: mirror-symmetric about cell faces)

    def rho(self, r):
        return _maxs(self.rho_c * (1.0 - (r / self.radius) ** 2), self.rho_atm)

    def press(self, r):
        rho = self.rho(r)
        if self.pp is None:
            return _maximum(self.K * rho ** self.Gamma, rho * self.T_atm)
        # cold star: P_cold(rho) plus the atmosphere temperature everywhere
        return pp_cold_pressure(rho, self.pp, self.pp_K) + rho * self.T_atm

    def p_max(self):
        if self.pp is None:
            return self.K * self.rho_c ** self.Gamma
        return float(self.press(np.array([0.0]))[0])

    def potential_scale(self, r):
        return _maxs(self.press(r) - self.pcut * self.p_max(), 0.0)

    def metric(self, x, y, z):
        r2 = x * x + y * y + z * z
        rt = _sqrt(r2 + (0.5 * self.radius) ** 2)
        q = self.mass / (2.0 * rt)
        psi = 1.0 + q
        alpha = (1.0 - q) / (1.0 + q)
        return alpha, psi ** 4


class _NumpyBackend:
    def arange(self, n):
        return np.arange(n, dtype=np.float64)

    def empty(self, shape):
        return np.empty(shape)

    def contiguous(self, a):
        return np.ascontiguousarray(a)


class _TorchBackend:
    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device

    def arange(self, n):
        return self.torch.arange(n, dtype=self.torch.float64, device=self.device)

    def empty(self, shape):
        return self.torch.empty(shape, dtype=self.torch.float64, device=self.device)

    def contiguous(self, a):
        return a.contiguous()


def _star_block_arrays(st: StarSetup, i0, j0, k0, n, ng, h, xmin, backend=None):
    """Padded arrays of a block whose first interior cell has global integer
    index (i0, j0, k0) on a lattice of spacing h starting at xmin.  backend:
    numpy (default) or torch tensors on a device (same formulas)."""
    be = backend or _NumpyBackend()
    s = n + 2 * ng
    gi = be.arange(s) - ng          # local padded -> global cell offset
    fa = be.arange(s + 1) - ng
    # 1-D coordinates, broadcast as [k, j, i]
    # coordinates relative to the star centre
    cx, cy, cz = st.center
    xc = (xmin + (i0 + gi + 0.5) * h - cx)[None, None, :]
    yc = (xmin + (j0 + gi + 0.5) * h - cy)[None, :, None]
    zc = (xmin + (k0 + gi + 0.5) * h - cz)[:, None, None]
    xf = (xmin + (i0 + fa) * h - cx)[None, None, :]
    yf = (xmin + (j0 + fa) * h - cy)[None, :, None]
    zf = (xmin + (k0 + fa) * h - cz)[:, None, None]
    R = _sqrt(xc * xc + yc * yc + zc * zc)
    rho = st.rho(R)
    P = st.press(R)
    alpha, g = st.metric(xc, yc, zc)
    adm = be.empty((16, s, s, s))
    adm[:] = 0.0
    adm[0] = alpha
    adm[4] = g
    adm[7] = g
    adm[9] = g
    w = be.empty((5, s, s, s))
    w[0] = rho
    w[1:4] = 0.0
    w[4] = P
    # A = A_b * max(P - pcut Pmax, 0) * (-y, x, 0) on edges; A_z = 0
    # A_x at (x_c, y_f, z_f): shape (s+1, s+1, s); A_y at (x_f, y_c, z_f): (s+1, s, s+1)
    Ax = -yf * st.A_b * st.potential_scale(_sqrt(xc * xc + yf * yf + zf * zf))
    Ay = xf * st.A_b * st.potential_scale(_sqrt(xf * xf + yc * yc + zf * zf))
    # B~x at (x_f, y_c, z_c) = dy Az - dz Ay = -(Ay[k+1] - Ay[k]) / h
    Bx = -(Ay[1:, :, :] - Ay[:-1, :, :]) / h                 # (s, s, s+1)
    # B~y at (x_c, y_f, z_c) = dz Ax - dx Az = (Ax[k+1] - Ax[k]) / h
    By = (Ax[1:, :, :] - Ax[:-1, :, :]) / h                  # (s, s+1, s)
    # B~z at (x_c, y_c, z_f) = dx Ay - dy Ax
    Bz = (Ay[:, :, 1:] - Ay[:, :, :-1]) / h - (Ax[:, 1:, :] - Ax[:, :-1, :]) / h  # (s+1, s, s)
    return w, [be.contiguous(Bx), be.contiguous(By), be.contiguous(Bz)], adm


def calibrate_field(st: StarSetup, n=64):
    """Fix A_b so that the minimum plasma beta 2P/b^2 over the magnetised
    region of an n^3 sampling of the box equals st.beta_min (v = 0, so
    b^2 = gamma_ij B^i B^j with B = B~/sqrt(gamma))."""
    st.A_b = 1.0
    h = 2.0 * st.box / n
    w, bf, adm = _star_block_arrays(st, 0, 0, 0, n, 0, h, -st.box)
    bx = 0.5 * (bf[0][:, :, 1:] + bf[0][:, :, :-1])
    by = 0.5 * (bf[1][:, 1:, :] + bf[1][:, :-1, :])
    bz = 0.5 * (bf[2][1:, :, :] + bf[2][:-1, :, :])
    g = adm[4]                        # psi^4 (conformally flat)
    sqrtg = g ** 1.5
    b2 = g * (bx * bx + by * by + bz * bz) / (sqrtg * sqrtg)
    P = w[4]
    mask = b2 > 0
    ratio = np.min(2.0 * P[mask] / b2[mask])
    st.A_b = math.sqrt(ratio / st.beta_min)
    return st


def star_blocks(n_per_side=4, nb=64, ng=3, st: StarSetup | None = None, device=None):
    """The star on a uniform grid of (n_per_side * nb)^3 cells over
    [-box, box]^3, split into n_per_side^3 blocks of nb^3; ghosts are filled
    by same-level copies between blocks with outflow at the domain edge.
    device: None for numpy arrays, else a torch device (arrays built there)."""
    st = st or calibrate_field(StarSetup())
    backend = _TorchBackend(device) if device is not None else None
    ntot = n_per_side * nb
    h = 2.0 * st.box / ntot
    blocks = []
    for kb in range(n_per_side):
        for jb in range(n_per_side):
            for ib in range(n_per_side):
                w, bf, adm = _star_block_arrays(st, ib * nb, jb * nb, kb * nb, nb, ng, h, -st.box,
                                                backend)
                nbr = []
                for oz in (-1, 0, 1):
                    for oy in (-1, 0, 1):
                        for ox in (-1, 0, 1):
                            a, b, c = ib + ox, jb + oy, kb + oz
                            if 0 <= a < n_per_side and 0 <= b < n_per_side and 0 <= c < n_per_side:
                                nbr.append(a + n_per_side * (b + n_per_side * c))
                            else:
                                nbr.append(-1)
                blocks.append(BlockInit(nb, nb, nb, ng, (h, h, h), w, bf, adm, nbr, 1, 0,
                                        (-st.box + ib * nb * h, -st.box + jb * nb * h,
                                         -st.box + kb * nb * h)))
    return blocks, st


def star_block_numpy(st: StarSetup, ib, jb, kb, n_per_side=4, nb=64, ng=3):
    """One block (ib, jb, kb) of star_blocks as numpy arrays, ghosts frozen at
    the analytic data (for CPU samples of the same workload)."""
    h = 2.0 * st.box / (n_per_side * nb)
    w, bf, adm = _star_block_arrays(st, ib * nb, jb * nb, kb * nb, nb, ng, h, -st.box)
    return BlockInit(nb, nb, nb, ng, (h, h, h), w, bf, adm, [-1] * 27, 0, 0,
                     (-st.box + ib * nb * h, -st.box + jb * nb * h, -st.box + kb * nb * h))


def refined_star_blocks(nblocks=1500, nlevels=6, sizes=(16, 24, 32), ng=3, seed_offset=2,
                        st: StarSetup | None = None, max_blocks=None, device=None):
    """Independent blocks of the star on nlevels nested levels (level l has
    spacing h0 / 2^l on the cube [-box/2^l, box/2^l]^3).  Block sizes and the
    number of blocks per level are drawn from a seeded multinomial; each block
    origin lies on its level lattice.  Ghosts are frozen at the analytic data."""
    st = st or calibrate_field(StarSetup())
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    weights = rng.dirichlet(np.ones(nlevels) * 2.0)
    per_level = rng.multinomial(nblocks, weights)
    blocks = []
    h0 = 2.0 * st.box / 64.0
    for lev in range(nlevels):
        h = h0 / 2 ** lev
        half = st.box / 2 ** lev
        ncell_level = int(round(2 * half / h))   # 64 cells per level cube side
        cnt = per_level[lev]
        nsz = rng.integers(0, len(sizes), size=cnt)
        for t in range(cnt):
            n = sizes[nsz[t]]
            # origin on the lattice, block inside the level cube
            i0, j0, k0 = (rng.integers(0, ncell_level - n + 1) for _ in range(3))
            w, bf, adm = _star_block_arrays(st, int(i0), int(j0), int(k0), n, ng, h, -half,
                                            _TorchBackend(device) if device is not None else None)
            blocks.append(BlockInit(n, n, n, ng, (h, h, h), w, bf, adm, [-1] * 27, 0, lev,
                                    (-half + i0 * h, -half + j0 * h, -half + k0 * h)))
            if max_blocks is not None and len(blocks) >= max_blocks:
                return blocks, st
    return blocks, st


# ---------------------------------------------------------------------------
# conservative-to-primitive test states
# ---------------------------------------------------------------------------
def c2p_states(n, seed_offset=3, gamma=5.0 / 3.0, log_rho=(-10.0, -2.0), log_eps=(-6.0, 1.0),
               W_range=(1.0, 10.0), log_bsq_rho=(-4.0, 1.0), metric_dev=0.1, pp=None, pp_K=None):
    """n primitive states with their densitized field and 3-metric.

    log10 rho ~ U[log_rho]; log10 eps ~ U[log_eps]; W ~ U[W_range];
    b^2/rho ~ log-U; the velocity direction is isotropic in the gamma norm;
    the field direction n is isotropic, |B| set from b^2 = B^2/W^2 + (B.v)^2;
    gamma = Q diag(lambda) Q^T with lambda ~ U[1-dev, 1+dev], Q a random
    rotation.  The ideal-gas pressure P = (gamma-1) rho eps specifies the
    state; with a piecewise polytrope (pp, pp_K from pp_eos) the drawn eps is
    the thermal part: P = P_cold(rho) + (gamma_th - 1) rho eps.  Returns dict
    with w (5,n), bt (3,n) densitized, gam (6,n)."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    rho = 10.0 ** rng.uniform(*log_rho, size=n)
    eps = 10.0 ** rng.uniform(*log_eps, size=n)
    W = rng.uniform(*W_range, size=n)
    bsq = rho * 10.0 ** rng.uniform(*log_bsq_rho, size=n)
    # random rotations from normalised quaternions
    qv = rng.normal(size=(n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    a, b, c, d = qv.T
    Q = np.stack([
        np.stack([a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)], -1),
        np.stack([2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)], -1),
        np.stack([2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d], -1),
    ], 1)
    lam = rng.uniform(1.0 - metric_dev, 1.0 + metric_dev, size=(n, 3))
    G = np.einsum("nij,nj,nkj->nik", Q, lam, Q)
    gam = np.stack([G[:, 0, 0], G[:, 0, 1], G[:, 0, 2], G[:, 1, 1], G[:, 1, 2], G[:, 2, 2]])
    def unit_gamma(vec):
        nrm = np.sqrt(np.einsum("ni,nij,nj->n", vec, G, vec))
        return vec / nrm[:, None]
    e = unit_gamma(rng.normal(size=(n, 3)))
    vmag = np.sqrt(1.0 - 1.0 / (W * W))
    v = e * vmag[:, None]
    nb = unit_gamma(rng.normal(size=(n, 3)))
    nv = np.einsum("ni,nij,nj->n", nb, G, v)
    Bmag = np.sqrt(bsq / (1.0 / (W * W) + nv * nv))
    B = nb * Bmag[:, None]
    sqrtg = np.sqrt(np.linalg.det(G))
    if pp is None:
        P = (gamma - 1.0) * rho * eps
    else:
        P = pp_cold_pressure(rho, pp, pp_K) + (pp["gamma_th"] - 1.0) * rho * eps
    w = np.stack([rho, W * v[:, 0], W * v[:, 1], W * v[:, 2], P])
    bt = (B * sqrtg[:, None]).T
    return {"w": np.ascontiguousarray(w), "bt": np.ascontiguousarray(bt),
            "gam": np.ascontiguousarray(gam), "eps": eps, "W": W, "bsq": bsq}


def c2p_states_torch(n, seed_offset=3, gamma=5.0 / 3.0, log_rho=(-10.0, -2.0), log_eps=(-6.0, 1.0),
                     W_range=(1.0, 10.0), log_bsq_rho=(-4.0, 1.0), metric_dev=0.1, device="cuda",
                     pp=None, pp_K=None):
    """c2p_states with the same distributions, drawn with torch on a device
    (for workloads too large to build on the host; different random stream).
    pp, pp_K: piecewise polytrope as in c2p_states (eps is the thermal part)."""
    import torch
    g = torch.Generator(device=device).manual_seed(SEED_BASE + seed_offset)
    f64 = dict(dtype=torch.float64, device=device)

    def U(lo, hi, *shape):
        return lo + (hi - lo) * torch.rand(*shape, generator=g, **f64)

    rho = 10.0 ** U(*log_rho, n)
    eps = 10.0 ** U(*log_eps, n)
    W = U(*W_range, n)
    bsq = rho * 10.0 ** U(*log_bsq_rho, n)
    qv = torch.randn(n, 4, generator=g, **f64)
    qv = qv / qv.norm(dim=1, keepdim=True)
    a, b, c, d = qv.unbind(1)
    Q = torch.stack([
        torch.stack([a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)], -1),
        torch.stack([2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)], -1),
        torch.stack([2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d], -1),
    ], 1)
    lam = U(1.0 - metric_dev, 1.0 + metric_dev, n, 3)
    G = (Q * lam[:, None, :]) @ Q.transpose(1, 2)
    gam = torch.stack([G[:, 0, 0], G[:, 0, 1], G[:, 0, 2], G[:, 1, 1], G[:, 1, 2], G[:, 2, 2]])

    def unit_gamma(vec):
        nrm = torch.sqrt(torch.einsum("ni,nij,nj->n", vec, G, vec))
        return vec / nrm[:, None]

    e = unit_gamma(torch.randn(n, 3, generator=g, **f64))
    v = e * torch.sqrt(1.0 - 1.0 / (W * W))[:, None]
    nb = unit_gamma(torch.randn(n, 3, generator=g, **f64))
    nv = torch.einsum("ni,nij,nj->n", nb, G, v)
    Bmag = torch.sqrt(bsq / (1.0 / (W * W) + nv * nv))
    B = nb * Bmag[:, None]
    sqrtg = torch.sqrt(torch.linalg.det(G))
    if pp is None:
        P = (gamma - 1.0) * rho * eps
    else:
        P = pp_cold_pressure(rho, pp, pp_K) + (pp["gamma_th"] - 1.0) * rho * eps
    w = torch.stack([rho, W * v[:, 0], W * v[:, 1], W * v[:, 2], P]).contiguous()
    bt = (B * sqrtg[:, None]).T.contiguous()
    return {"w": w, "bt": bt, "gam": gam.contiguous(), "W": W, "eps": eps}


# ---------------------------------------------------------------------------
# refined meshes: leaves of a 2:1-balanced octree of equal blocks
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class LeafMesh:
    """Leaves (level, (bi, bj, bk)) of an octree over nblocks0 level-0 blocks
    of nb^3 cells; leaf l covers global cells [b nb, (b+1) nb) of its level
    (cell size h0 / 2^level).  periodic: per axis, 1 periodic, 0 outflow."""
    nblocks0: tuple
    nb: int
    periodic: tuple
    leaves: list

    @property
    def n0(self):
        return tuple(int(x) * self.nb for x in self.nblocks0)

    def org(self, i):
        return tuple(int(x) * self.nb for x in self.leaves[i][1])

    @property
    def levels(self):
        return [lv for lv, _ in self.leaves]


def leaf_mesh(nblocks0=(2, 2, 2), nb=8, refine=None, max_level=1, periodic=(1, 1, 1)):
    """refine(level, (bi, bj, bk)) -> bool marks leaves to split (repeated up
    to max_level); then leaves are split until every two leaves that touch
    (across a face, an edge or a corner, periodic images included) differ by
    at most one level.  Leaves are listed by level, then z, y, x."""
    leaves = {(0, (i, j, k)) for k in range(nblocks0[2]) for j in range(nblocks0[1])
              for i in range(nblocks0[0])}
    for _ in range(max_level):
        split = [lf for lf in leaves if lf[0] < max_level and refine is not None and refine(*lf)]
        if not split:
            break
        for lv, b in split:
            leaves.remove((lv, b))
            for c in range(8):
                leaves.add((lv + 1, (2 * b[0] + (c & 1), 2 * b[1] + ((c >> 1) & 1), 2 * b[2] + (c >> 2))))

    def covering(lv, b):
        for L in range(lv, -1, -1):
            key = (L, tuple(x >> (lv - L) for x in b))
            if key in leaves:
                return key
        return None

    changed = True
    while changed:
        changed = False
        for lv, b in sorted(leaves, key=lambda t: -t[0]):
            if (lv, b) not in leaves or lv < 2:
                continue
            nbk = [n << lv for n in nblocks0]
            for oz in (-1, 0, 1):
                for oy in (-1, 0, 1):
                    for ox in (-1, 0, 1):
                        if ox == oy == oz == 0:
                            continue
                        q = [b[0] + ox, b[1] + oy, b[2] + oz]
                        ok = True
                        for a in range(3):
                            if q[a] < 0 or q[a] >= nbk[a]:
                                if periodic[a]:
                                    q[a] %= nbk[a]
                                else:
                                    ok = False
                        if not ok:
                            continue
                        cov = covering(lv, tuple(q))
                        if cov is not None and cov[0] < lv - 1:
                            leaves.remove(cov)
                            L, cb = cov
                            for c in range(8):
                                leaves.add((L + 1, (2 * cb[0] + (c & 1), 2 * cb[1] + ((c >> 1) & 1),
                                                    2 * cb[2] + (c >> 2))))
                            changed = True
    order = sorted(leaves, key=lambda t: (t[0], t[1][2], t[1][1], t[1][0]))
    return LeafMesh(tuple(nblocks0), nb, tuple(int(x) for x in periodic), order)


def _leaf_coords(mesh: LeafMesh, i, ng, h0):
    lv, b = mesh.leaves[i]
    h = h0 / 2 ** lv
    o = [b[a] * mesh.nb for a in range(3)]
    m = mesh.nb + 2 * ng
    cc = [(o[a] - ng + np.arange(m) + 0.5) * h for a in range(3)]      # cell centres
    fc = [(o[a] - ng + np.arange(m + 1)) * h for a in range(3)]        # faces / corners
    return h, cc, fc


def _waves_without(rng, axis, nwaves=3):
    """random integer wave vectors with no component along `axis`"""
    ks = []
    while len(ks) < nwaves:
        k = rng.integers(-2, 3, size=3)
        k[axis] = 0
        if np.any(k != 0):
            ks.append(k)
    return np.array(ks, dtype=np.float64), rng.uniform(0.0, 2.0 * np.pi, size=nwaves)


def smooth_leaf_blocks(mesh: LeafMesh, ng=3, seed_offset=7, amp_rho=0.1, amp_p=0.01, amp_v=0.3,
                       amp_a=0.05, flat=False, amp_lapse=0.05, amp_shift=0.01, amp_g=0.05,
                       amp_k=0.01, uniform=None):
    """Smooth periodic data on [0, 1)^3 sampled on every leaf of `mesh` (a
    cubic domain: h0 = 1 / (nblocks0[0] nb)), ghosts included.  The fields are
    those of smooth_periodic_block; the vector potential has A_x(y, z),
    A_y(z, x), A_z(x, y) sampled at cell corners, so each edge value is the
    exact line average and every face's B~ is the exact face average of the
    curl.  flat: Minkowski metric (no sources).  uniform: (rho, u3, P, Bt3)
    for a uniform state."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    waves = {}
    for name in ("rho", "P", "u0", "u1", "u2", "alpha", "b0", "b1", "b2") + tuple(f"g{c}" for c in range(6)) \
            + tuple(f"k{c}" for c in range(6)):
        waves[name] = _random_waves(rng)
    aw = [_waves_without(rng, a) for a in range(3)]
    h0 = 1.0 / (mesh.nblocks0[0] * mesh.nb)
    out = []
    for i in range(len(mesh.leaves)):
        lv, _ = mesh.leaves[i]
        h, cc, fc = _leaf_coords(mesh, i, ng, h0)
        Z, Y, X = np.meshgrid(cc[2], cc[1], cc[0], indexing="ij")
        f = lambda nm: _wave_sum(*waves[nm], X, Y, Z)
        rho = 1.0 + amp_rho * f("rho")
        P = 0.1 + amp_p * f("P")
        u = [amp_v * f(f"u{c}") / math.sqrt(3.0) for c in range(3)]
        if flat:
            alpha = np.ones_like(rho)
            beta = [np.zeros_like(rho) for _ in range(3)]
            gam = [np.full_like(rho, 1.0 if c in (0, 3, 5) else 0.0) for c in range(6)]
            K = [np.zeros_like(rho) for _ in range(6)]
        else:
            alpha = 1.0 + amp_lapse * f("alpha")
            beta = [amp_shift * f(f"b{c}") for c in range(3)]
            gam = [(1.0 if c in (0, 3, 5) else 0.0) + amp_g * f(f"g{c}") for c in range(6)]
            K = [amp_k * f(f"k{c}") for c in range(6)]
        # A at corners (z, y, x lattices of m + 1 points); A_x depends on (y, z) ...
        Zc, Yc, Xc = np.meshgrid(fc[2], fc[1], fc[0], indexing="ij")
        Ax = amp_a * _wave_sum(*aw[0], Xc, Yc, Zc)
        Ay = amp_a * _wave_sum(*aw[1], Xc, Yc, Zc)
        Az = amp_a * _wave_sum(*aw[2], Xc, Yc, Zc)
        # face averages of curl A from corner values (A_x constant along x, ...)
        Bx = ((Az[:-1, 1:, :] - Az[:-1, :-1, :]) - (Ay[1:, :-1, :] - Ay[:-1, :-1, :])) / h
        By = ((Ax[1:, :, :-1] - Ax[:-1, :, :-1]) - (Az[:-1, :, 1:] - Az[:-1, :, :-1])) / h
        Bz = ((Ay[:, :-1, 1:] - Ay[:, :-1, :-1]) - (Ax[:, 1:, :-1] - Ax[:, :-1, :-1])) / h
        if uniform is not None:
            r0, u0, p0, b0 = uniform
            rho = np.full_like(rho, r0)
            P = np.full_like(rho, p0)
            u = [np.full_like(rho, u0[c]) for c in range(3)]
            Bx, By, Bz = (np.full_like(a, b0[c]) for c, a in enumerate((Bx, By, Bz)))
        w = np.stack([rho, u[0], u[1], u[2], P])
        adm = np.stack([alpha] + beta + gam + K)
        org = mesh.org(i)
        out.append(BlockInit(mesh.nb, mesh.nb, mesh.nb, ng, (h, h, h), np.ascontiguousarray(w),
                             [np.ascontiguousarray(b) for b in (Bx, By, Bz)], np.ascontiguousarray(adm),
                             [-1] * 27, 1, lv, tuple(org[a] * h for a in range(3))))
    return out


def star_leaf_mesh(nblocks0=4, nb=32, half=48.0, radii=(28.0, 14.0, 8.0)):
    """A leaf mesh about the star at the origin on [-half, half]^3 (outflow
    boundaries): a level-0 leaf of level l < len(radii) is split while its
    box comes within radii[l] of the centre, then 2:1-balanced."""
    h0 = 2.0 * half / (nblocks0 * nb)

    def refine(lv, b):
        if lv >= len(radii):
            return False
        side = nb * h0 / 2 ** lv
        lo = [-half + b[a] * side for a in range(3)]
        d2 = sum(max(lo[a], 0.0, -(lo[a] + side)) ** 2 for a in range(3))
        return d2 < radii[lv] ** 2

    m = leaf_mesh((nblocks0,) * 3, nb, refine=refine, max_level=len(radii), periodic=(0, 0, 0))
    return m, h0


def star_leaf_blocks(st: StarSetup | None = None, nblocks0=4, nb=32, ng=3, half=48.0,
                     radii=(28.0, 14.0, 8.0), device=None):
    """The star (StarSetup) sampled on every leaf of star_leaf_mesh, ghosts
    included; returns (blocks, leaf mesh, star setup)."""
    st = st or calibrate_field(StarSetup())
    backend = _TorchBackend(device) if device is not None else None
    m, h0 = star_leaf_mesh(nblocks0, nb, half, radii)
    blocks = []
    for i, (lv, b) in enumerate(m.leaves):
        h = h0 / 2 ** lv
        o = m.org(i)
        w, bf, adm = _star_block_arrays(st, o[0], o[1], o[2], nb, ng, h, -half, backend)
        blocks.append(BlockInit(nb, nb, nb, ng, (h, h, h), w, bf, adm, [-1] * 27, 1, lv,
                                tuple(-half + o[a] * h for a in range(3))))
    return blocks, m, st

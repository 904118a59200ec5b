"""Python binding of the plain FP64 CPU oracle (``libgrmhd_oracle.so``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark are the only users.  The product path (the HIP
library and its binding) never imports this package.

The oracle is plain C built with ``-O2 -fno-fast-math -ffp-contract=off``
(see ``oracle/build.sh``); this module marshals numpy arrays into its structs.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgrmhd_oracle.so")
_lib = None

# flag bits (per-cell uint16)
F_C2P_FAIL, F_DFLOOR, F_TAUFLOOR, F_MAGCAP, F_TFLOOR, F_RHOFLOOR, F_FOFC, F_DMP, \
    F_BRACKET_FALLBACK, F_MAXIT, F_EXCISED = [1 << b for b in range(11)]
F_FLOORS = F_C2P_FAIL | F_DFLOOR | F_TAUFLOOR | F_MAGCAP | F_TFLOOR | F_RHOFLOOR | F_MAXIT
GF_W, GF_US, GF_BS, GF_FLAGS = 1, 2, 4, 8


def build(force=False):
    """Compile the oracle with gcc (no GPU involved)."""
    src = os.path.join(_HERE, "grmhd_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        subprocess.check_call(["bash", os.path.join(_HERE, "build.sh")], cwd=_HERE)
    return _LIB_PATH


class OrParams(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("rho_b", C.c_double * 3), ("K0", C.c_double),
        ("Gam", C.c_double * 4), ("gamma_th", C.c_double), ("rho_atm", C.c_double),
        ("T_atm", C.c_double), ("f_thr", C.c_double), ("M_max", C.c_double),
        ("dmp_M", C.c_double), ("c2p_tol", C.c_double),
        ("eos", C.c_int32), ("npieces", C.c_int32), ("recon", C.c_int32),
        ("riemann", C.c_int32), ("fofc", C.c_int32), ("c2p_maxit", C.c_int32),
    ]


PD = C.POINTER(C.c_double)


class OrBlock(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ng", C.c_int32),
        ("dx", C.c_double * 3),
        ("w", PD * 5), ("un", PD * 5), ("us", PD * 5), ("bn", PD * 3), ("bs", PD * 3),
        ("adm", PD * 16), ("uo", PD * 5), ("bo", PD * 3), ("wo", PD * 5),
        ("flags", C.POINTER(C.c_uint16)), ("nbr", C.c_int32 * 27), ("bc", C.c_int32),
    ]


class OrAmr(C.Structure):
    _fields_ = [
        ("n0", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
        ("level", C.POINTER(C.c_int32)), ("org", C.POINTER(C.c_int32)),
    ]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        for name, res in [("or_dt", C.c_double), ("or_mass", C.c_double)]:
            getattr(L, name).restype = res
        assert L.or_sizeof_params() == C.sizeof(OrParams), "or_params layout mismatch"
        assert L.or_sizeof_block() == C.sizeof(OrBlock), "or_block layout mismatch"
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's loops (n <= 0 leaves them); returns
    the number now in use"""
    return int(lib().or_set_threads(C.c_int(n)))


def set_decision_margin(m: float):
    """Move every threshold test of the method by the relative amount m
    (test instrument; 0 restores the method exactly).  Oracle runs at +m and
    -m differ exactly where a decision lies within m of its threshold."""
    lib().or_set_decision_margin(C.c_double(m))


@dataclasses.dataclass
class Params:
    """Method options: EOS, atmosphere (rho_atm, T_atm, f_thr, M_max),
    reconstruction (0 donor cell, 1 PLM, 2 WENOZ, 3 PPM4, 4 PPMX), Riemann
    solver (0 LLF, 1 HLLE),
    FOFC on/off, DMP factor M (<= 0 off), C2P tolerance and iteration cap."""

    gamma: float = 5.0 / 3.0
    eos: int = 0
    npieces: int = 1
    rho_b: tuple = (0.0, 0.0, 0.0)
    K0: float = 0.0
    Gam: tuple = (2.0, 2.0, 2.0, 2.0)
    gamma_th: float = 1.75
    rho_atm: float = 1e-10
    T_atm: float = 1e-12
    f_thr: float = 1.0
    M_max: float = 100.0
    recon: int = 2
    riemann: int = 1
    fofc: int = 0
    dmp_M: float = 0.0
    c2p_tol: float = 2.220446049250313e-16
    c2p_maxit: int = 300

    def c(self) -> OrParams:
        p = OrParams()
        p.gamma = self.gamma
        p.rho_b = (C.c_double * 3)(*self.rho_b)
        p.K0 = self.K0
        p.Gam = (C.c_double * 4)(*self.Gam)
        p.gamma_th = self.gamma_th
        p.rho_atm, p.T_atm, p.f_thr, p.M_max = self.rho_atm, self.T_atm, self.f_thr, self.M_max
        p.dmp_M, p.c2p_tol = self.dmp_M, self.c2p_tol
        p.eos, p.npieces, p.recon, p.riemann = self.eos, self.npieces, self.recon, self.riemann
        p.fofc, p.c2p_maxit = self.fofc, self.c2p_maxit
        return p


def _pd(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(PD)


def _ptrs(arrs, n=None):
    arrs = list(arrs)
    t = PD * len(arrs)
    return t(*[_pd(a) for a in arrs])


# ---------------------------------------------------------------------------
# pointwise entry points
# ---------------------------------------------------------------------------
def prim2con(w, bt, gam, params: Params):
    """Eq. 7 (densitized): w (5,n), bt (3,n) densitized field, gam (6,n)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    gam = np.ascontiguousarray(gam, dtype=np.float64)
    n = w.shape[1]
    u = np.zeros((5, n))
    lib().or_prim2con(C.c_int64(n), _ptrs(w), _ptrs(bt), _ptrs(gam), _ptrs(u), C.byref(params.c()))
    return u


def c2p(u, bt, gam, params: Params, blo=None, bhi=None):
    """C2P with atmosphere rules.  Returns (u_out, w, flags, nev, mu)."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    gam = np.ascontiguousarray(gam, dtype=np.float64)
    n = u.shape[1]
    w = np.zeros((5, n))
    flags = np.zeros(n, dtype=np.uint16)
    nev = np.zeros(n, dtype=np.int32)
    mu = np.zeros(n)
    lo = _pd(np.ascontiguousarray(blo, dtype=np.float64)) if blo is not None else None
    hi = _pd(np.ascontiguousarray(bhi, dtype=np.float64)) if bhi is not None else None
    if blo is not None:
        blo_a = np.ascontiguousarray(blo, dtype=np.float64)
        bhi_a = np.ascontiguousarray(bhi, dtype=np.float64)
        lo, hi = _pd(blo_a), _pd(bhi_a)
    lib().or_c2p(C.c_int64(n), _ptrs(u), _ptrs(bt), _ptrs(gam), _ptrs(w),
                 flags.ctypes.data_as(C.POINTER(C.c_uint16)), C.byref(params.c()), lo, hi,
                 nev.ctypes.data_as(C.POINTER(C.c_int32)), _pd(mu))
    return u, w, flags, nev, mu


def matter_sources(w, bt, gam, params: Params):
    """ADM matter sources (E, S_x, S_y, S_z, S_xx, S_xy, S_xz, S_yy, S_yz, S_zz)
    of n points: w (5, n), densitized cell-centred field bt (3, n), gamma_ij
    (6, n); returns (10, n), not densitized."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    gam = np.ascontiguousarray(gam, dtype=np.float64)
    n = w.shape[1]
    out = np.zeros((10, n))
    lib().or_matter_sources(C.c_int64(n), _ptrs(w), _ptrs(bt), _ptrs(gam), _ptrs(out),
                            C.byref(params.c()))
    return out


def recover(u, bt, gam, mu, params: Params, eps_terms=False):
    """the primitives (rho, W v^i, P) the inversion recovers at the root mu
    (the recovery step of c2p, without the floors); with eps_terms also the
    magnitude of the terms the specific internal energy is summed from, the
    scale of its rounding error"""
    u = np.ascontiguousarray(u, dtype=np.float64)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    gam = np.ascontiguousarray(gam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n = u.shape[1]
    w = np.zeros((5, n))
    te = np.zeros(n)
    lib().or_recover(C.c_int64(n), _ptrs(u), _ptrs(bt), _ptrs(gam), _pd(mu), _ptrs(w), _pd(te),
                     C.byref(params.c()))
    return (w, te) if eps_terms else w


def master(u, bt, gam, mu, params: Params):
    """Kastaun master function f(mu) and auxiliary f_a(mu) at given mu."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    bt = np.ascontiguousarray(bt, dtype=np.float64)
    gam = np.ascontiguousarray(gam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n = u.shape[1]
    f = np.zeros(n)
    fa = np.zeros(n)
    lib().or_master(C.c_int64(n), _ptrs(u), _ptrs(bt), _ptrs(gam), _pd(mu), _pd(f), _pd(fa),
                    C.byref(params.c()))
    return f, fa


def face_physics(d, q, B, alpha, beta, gam, params: Params):
    """Eq. 7-9 on one side of a d-face: returns U (7,n), F (7,n), lm, lp."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    gam = np.ascontiguousarray(gam, dtype=np.float64)
    n = q.shape[1]
    U = np.zeros((7, n))
    F = np.zeros((7, n))
    lm = np.zeros(n)
    lp = np.zeros(n)
    lib().or_face_physics(C.c_int64(n), C.c_int(d), _ptrs(q), _ptrs(B), _pd(alpha), _ptrs(beta),
                          _ptrs(gam), _ptrs(U), _ptrs(F), _pd(lm), _pd(lp), C.byref(params.c()))
    return U, F, lm, lp


def sources_point(w, bt, u, gam6, alpha, dal, dbe, dg, K6, params: Params):
    """Eq. 10 at one point; dbe[i][j] = d_i beta^j, dg[i][jk] = d_i gamma_jk."""
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
            for a in (w, bt, u, gam6, dal, dbe, dg, K6)]
    G = np.zeros(5)
    lib().or_sources_point(_pd(arrs[0]), _pd(arrs[1]), _pd(arrs[2]), _pd(arrs[3]),
                           C.c_double(alpha), _pd(arrs[4]), _pd(arrs[5]), _pd(arrs[6]),
                           _pd(arrs[7]), _pd(G), C.byref(params.c()))
    return G


def wenoz(q5):
    q5 = np.ascontiguousarray(q5, dtype=np.float64).reshape(-1, 5)
    out = np.zeros(q5.shape[0])
    lib().or_wenoz(C.c_int64(q5.shape[0]), _pd(q5), _pd(out))
    return out


def recon_edges(kind, q5):
    """lower and upper edge values of the middle cell of five-cell stencils
    q5 (n, 5) for reconstruction kind 0 DC, 1 PLM, 2 WENOZ, 3 PPM4, 4 PPMX"""
    q5 = np.ascontiguousarray(q5, dtype=np.float64).reshape(-1, 5)
    lo = np.zeros(q5.shape[0])
    hi = np.zeros(q5.shape[0])
    if lib().or_recon_edges(C.c_int(kind), C.c_int64(q5.shape[0]), _pd(q5), _pd(lo), _pd(hi)) != 0:
        raise ValueError(f"reconstruction kind {kind}")
    return lo, hi


def riemann(riemann_kind, UL, FL, lmL, lpL, UR, FR, lmR, lpR):
    arr = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    UL, FL, UR, FR = arr(UL), arr(FL), arr(UR), arr(FR)
    lmL, lpL, lmR, lpR = arr(lmL), arr(lpL), arr(lmR), arr(lpR)
    n = UL.shape[1]
    F = np.zeros((7, n))
    lib().or_riemann(C.c_int64(n), C.c_int(riemann_kind), _ptrs(UL), _ptrs(FL), _pd(lmL),
                     _pd(lpL), _ptrs(UR), _ptrs(FR), _pd(lmR), _pd(lpR), _ptrs(F))
    return F


def corner_emf(EA_b, EA_bm, EB_a, EB_am, mA_b, mA_bm, mB_a, mB_am, E00, E10, E01, E11):
    """upwind corner EMF of constrained transport at n points (arrays or
    scalars): face EMFs and mass fluxes of the two a-faces (at b and b-1) and
    the two b-faces (at a and a-1), cell-centre EMFs of cells (a, b),
    (a-1, b), (a, b-1), (a-1, b-1)"""
    args = [np.atleast_1d(np.asarray(x, dtype=np.float64)) for x in
            (EA_b, EA_bm, EB_a, EB_am, mA_b, mA_bm, mB_a, mB_am, E00, E10, E01, E11)]
    args = [np.ascontiguousarray(a) for a in np.broadcast_arrays(*args)]
    n = args[0].size
    out = np.zeros(n)
    lib().or_corner_emf(C.c_int64(n), _ptrs([a.ravel() for a in args]), _pd(out))
    return out


def eos(mode, rho, x, y, params: Params):
    arr = lambda a: np.ascontiguousarray(np.broadcast_to(a, np.shape(rho)), dtype=np.float64)
    rho_a, x_a, y_a = arr(rho), arr(x), arr(y)
    out = np.zeros(rho_a.shape)
    lib().or_eos(C.c_int64(rho_a.size), C.c_int(mode), _pd(rho_a), _pd(x_a), _pd(y_a), _pd(out),
                 C.byref(params.c()))
    return out


# ---------------------------------------------------------------------------
# mesh of blocks (host numpy state) and the stage driver
# ---------------------------------------------------------------------------
def cell_bt(bf):
    """densitized cell-centred field: average of the two faces per direction"""
    return np.stack([0.5 * (bf[0][:, :, 1:] + bf[0][:, :, :-1]),
                     0.5 * (bf[1][:, 1:, :] + bf[1][:, :-1, :]),
                     0.5 * (bf[2][1:, :, :] + bf[2][:-1, :, :])])


class Mesh:
    """Blocks with three state sets (A = U^n side, B and C = intermediates).
    SSP-RK2 in Shu-Osher form: U1 = U0 + dt L(U0); U2 = 1/2 U0 + 1/2 U1 +
    1/2 dt L(U1).  SSP-RK3 (Gottlieb, Ketcheson & Shu 2009, the three-stage
    third-order scheme): U1 = U0 + dt L(U0); U2 = 3/4 U0 + 1/4 U1 + 1/4 dt L(U1);
    U3 = 1/3 U0 + 2/3 U2 + 2/3 dt L(U2).  A stage with coefficients (a0, a1, b)
    computes a0 U^n + a1 U^(s) + b dt L(U^(s))."""

    RK2 = ((0, 1, (0.0, 1.0, 1.0)), (1, 0, (0.5, 0.5, 0.5)))
    RK3 = ((0, 1, (0.0, 1.0, 1.0)), (1, 2, (0.75, 0.25, 0.25)),
           (2, 0, (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)))

    def __init__(self, blocks, params: Params):
        self.params = params
        self.blocks = blocks
        self.u0, self.w0, self.b0, self.u1, self.w1, self.b1, self.flags = [], [], [], [], [], [], []
        self.u2, self.w2, self.b2 = [], [], []
        for b in blocks:
            shp = b.shape
            w = np.array(b.w, dtype=np.float64, order="C", copy=True)
            bf = [np.array(x, dtype=np.float64, order="C", copy=True) for x in b.bf]
            gam = b.adm[4:10].reshape(6, -1)
            u = prim2con(w.reshape(5, -1), cell_bt(bf).reshape(3, -1), gam, params).reshape((5,) + shp)
            self.u0.append(np.ascontiguousarray(u))
            self.w0.append(w)
            self.b0.append(bf)
            # sets B and C start as copies of set A, so that frozen ghosts
            # (bc == 0) hold the initial data in every set (stages write
            # interiors only)
            for U, W, Bf in ((self.u1, self.w1, self.b1), (self.u2, self.w2, self.b2)):
                U.append(np.ascontiguousarray(u).copy())
                W.append(w.copy())
                Bf.append([x.copy() for x in bf])
            self.flags.append(np.zeros(shp, dtype=np.uint16))
        self.adm = [np.ascontiguousarray(b.adm) for b in blocks]

    def _set(self, k):
        return ((self.u0, self.w0, self.b0), (self.u1, self.w1, self.b1), (self.u2, self.w2, self.b2))[k]

    def _desc(self, ib, w, un, us, bn, bs, uo, bo, wo):
        b = self.blocks[ib]
        d = OrBlock()
        d.nx, d.ny, d.nz, d.ng = b.nx, b.ny, b.nz, b.ng
        d.dx = (C.c_double * 3)(*b.dx)
        d.w = _ptrs(w)
        d.un = _ptrs(un)
        d.us = _ptrs(us)
        d.bn = _ptrs(bn)
        d.bs = _ptrs(bs)
        d.adm = _ptrs(self.adm[ib])
        d.uo = _ptrs(uo)
        d.bo = _ptrs(bo)
        d.wo = _ptrs(wo)
        d.flags = self.flags[ib].ctypes.data_as(C.POINTER(C.c_uint16))
        d.nbr = (C.c_int32 * 27)(*b.nbr)
        d.bc = b.bc
        return d

    def stage_descs(self, src, dst):
        """stage input w, U^(s), B^(s) from set src, U^n and B^n from set A;
        output U, B, w into set dst"""
        (us, ws, bs), (ua, _, ba), (uo, wo, bo) = self._set(src), self._set(0), self._set(dst)
        arr = (OrBlock * len(self.blocks))()
        for ib in range(len(self.blocks)):
            arr[ib] = self._desc(ib, ws[ib], ua[ib], us[ib], ba[ib], bs[ib], uo[ib], bo[ib], wo[ib])
        return arr

    def descs(self, stage):
        """RK2 stage 1: (w0, U0, U0, B0, B0) -> (U1, B1, w1);
        stage 2: (w1, U0, U1, B0, B1) -> (U0, B0, w0)."""
        return self.stage_descs(0, 1) if stage == 1 else self.stage_descs(1, 0)

    def ghost_fill_state(self, which):
        """fill ghosts of state set A (which=0), B (1) or C (2): w, U, faces"""
        U, W, Bf = self._set(which)
        arr = (OrBlock * len(self.blocks))()
        for ib in range(len(self.blocks)):
            arr[ib] = self._desc(ib, W[ib], U[ib], U[ib], Bf[ib], Bf[ib], U[ib], Bf[ib], W[ib])
        lib().or_ghost_fill(arr, len(self.blocks), GF_W | GF_US | GF_BS)

    def dt(self, cfl):
        arr = self.descs(1)
        return lib().or_dt(arr, len(self.blocks), C.byref(self.params.c()), C.c_double(cfl))

    def stage_sets(self, src, dst, dt, a0, a1, b, term_scales=False):
        """one stage; with term_scales, also returns per block the magnitudes
        of the terms each interior value of U (5 cell arrays) and of the faces
        (3 face arrays) is summed from (or_set_term_scales)"""
        arr = self.stage_descs(src, dst)
        nb = len(self.blocks)
        out = None
        if term_scales:
            tu = [np.zeros((5,) + blk.shape) for blk in self.blocks]
            tb = [[np.zeros(f.shape) for f in self.b0[ib]] for ib in range(nb)]
            pu, pb = (PD * (5 * nb))(), (PD * (3 * nb))()
            for ib in range(nb):
                for v in range(5):
                    pu[ib * 5 + v] = _pd(tu[ib][v])
                for d in range(3):
                    pb[ib * 3 + d] = _pd(tb[ib][d])
            lib().or_set_term_scales(pu, pb)
            out = (tu, tb)
        try:
            self._run_stage(arr, nb, dt, a0, a1, b)
        finally:
            if term_scales:
                lib().or_set_term_scales(None, None)
        return out

    def _run_stage(self, arr, nb, dt, a0, a1, b):
        lib().or_stage(arr, nb, C.byref(self.params.c()), C.c_double(dt), C.c_double(a0),
                       C.c_double(a1), C.c_double(b))

    def stage(self, stage, dt):
        src, dst, (a0, a1, b) = self.RK2[stage - 1]
        self.stage_sets(src, dst, dt, a0, a1, b)

    # lapse below which the stage output is excised (0: no excision)
    alpha_excise = 0.0

    def excise(self, which, alpha_min):
        """atmosphere in the interior cells of state set `which` where the lapse
        is below alpha_min (field unchanged; flagged F_EXCISED)"""
        arr = self.stage_descs(which, which)
        lib().or_excise(arr, len(self.blocks), C.byref(self.params.c()), C.c_double(alpha_min))

    def rk_step(self, scheme, dt):
        """one step of the Shu-Osher scheme `scheme` (RK2 or RK3), each stage's
        output excised (when alpha_excise > 0) and its ghosts filled before the
        next stage"""
        for src, dst, (a0, a1, b) in scheme:
            self.stage_sets(src, dst, dt, a0, a1, b)
            if self.alpha_excise > 0.0:
                self.excise(dst, self.alpha_excise)
            self.ghost_fill_state(dst)

    def rk3_step(self, dt=None, cfl=0.25):
        if dt is None:
            dt = self.dt(cfl)
        self.rk_step(self.RK3, dt)
        return dt

    def rk2_step(self, dt=None, cfl=0.25):
        if dt is None:
            dt = self.dt(cfl)
        self.rk_step(self.RK2, dt)
        return dt

    def mass(self):
        tot = 0.0
        for ib, b in enumerate(self.blocks):
            g = b.ng
            dv = b.dx[0] * b.dx[1] * b.dx[2]
            tot += float(np.sum(self.u0[ib][0, g:g + b.nz, g:g + b.ny, g:g + b.nx])) * dv
        return tot

    def interior(self, a, ib):
        b = self.blocks[ib]
        g = b.ng
        return a[..., g:g + b.nz, g:g + b.ny, g:g + b.nx]


class RefinedMesh(Mesh):
    """A Mesh whose blocks are the leaves of a refined mesh (LeafMesh from
    paper_2409_10384_amd.inputs, blocks in its leaf order): ghost fills across
    levels (or_ghost_fill_amr) and stages with the flux and EMF corrections
    at level boundaries (or_stage_amr)."""

    def __init__(self, blocks, params: Params, leafmesh):
        super().__init__(blocks, params)
        self.leafmesh = leafmesh

    def _amr(self):
        """the or_amr of the leaf mesh and the arrays it points into"""
        m = self.leafmesh
        nb = len(self.blocks)
        level = (C.c_int32 * nb)(*m.levels)
        org = (C.c_int32 * (3 * nb))(*[o for i in range(nb) for o in m.org(i)])
        amr = OrAmr()
        amr.n0 = (C.c_int32 * 3)(*m.n0)
        amr.periodic = (C.c_int32 * 3)(*m.periodic)
        amr.level = C.cast(level, C.POINTER(C.c_int32))
        amr.org = C.cast(org, C.POINTER(C.c_int32))
        return amr, (level, org)

    def ghost_fill_state(self, which):
        self.ghost_fill_mask(which, GF_W | GF_US | GF_BS)

    def ghost_fill_mask(self, which, mask):
        """ghost fill of the selected fields (GF_* bits) of state set `which`"""
        U, W, Bf = self._set(which)
        arr = (OrBlock * len(self.blocks))()
        for ib in range(len(self.blocks)):
            arr[ib] = self._desc(ib, W[ib], U[ib], U[ib], Bf[ib], Bf[ib], U[ib], Bf[ib], W[ib])
        amr, keep = self._amr()
        lib().or_ghost_fill_amr(arr, len(self.blocks), mask, C.byref(amr))

    def _run_stage(self, arr, nb, dt, a0, a1, b):
        amr, keep = self._amr()
        lib().or_stage_amr(arr, nb, C.byref(self.params.c()), C.c_double(dt), C.c_double(a0),
                           C.c_double(a1), C.c_double(b), C.byref(amr))

    def mass_total(self, which=0):
        """sum of D~ dV over every leaf's interior (each leaf with its own dV)"""
        U = self._set(which)[0]
        return sum(float(np.sum(self.interior(U[ib][0], ib))) * np.prod(b.dx)
                   for ib, b in enumerate(self.blocks))

    def totals(self, which=0):
        """sums of the five conserved fields over every leaf's interior (x dV)"""
        U = self._set(which)[0]
        return np.array([sum(float(np.sum(self.interior(U[ib][v], ib))) * np.prod(b.dx)
                             for ib, b in enumerate(self.blocks)) for v in range(5)])


def stage_steps(mesh: Mesh, stage, dt, fluxes, mode, flux_scales=None):
    """Run selected steps of one stage with caller-provided flux arrays
    fluxes[ib][d][c] (face arrays); see or_stage_steps for the mode bits.
    flux_scales (same layout as fluxes): filled with the magnitudes of the
    terms of every flux the steps compute (or_set_flux_term_scales)."""
    arr = mesh.descs(stage)
    a0, a1, b = (0.0, 1.0, 1.0) if stage == 1 else (0.5, 0.5, 0.5)
    nb = len(mesh.blocks)
    ptrs = (PD * (21 * nb))()
    sptrs = (PD * (21 * nb))() if flux_scales is not None else None
    for ib in range(nb):
        for d in range(3):
            for c in range(7):
                ptrs[ib * 21 + d * 7 + c] = _pd(fluxes[ib][d][c])
                if sptrs is not None:
                    sptrs[ib * 21 + d * 7 + c] = _pd(flux_scales[ib][d][c])
    if sptrs is not None:
        lib().or_set_flux_term_scales(sptrs)
    try:
        lib().or_stage_steps(arr, nb, C.byref(mesh.params.c()), C.c_double(dt), C.c_double(a0),
                             C.c_double(a1), C.c_double(b), ptrs, C.c_int(mode))
    finally:
        if sptrs is not None:
            lib().or_set_flux_term_scales(None)


def alloc_fluxes(mesh: Mesh):
    out = []
    for b in mesh.blocks:
        sz, sy, sx = b.shape
        shapes = [(sz, sy, sx + 1), (sz, sy + 1, sx), (sz + 1, sy, sx)]
        out.append([[np.zeros(shapes[d]) for _ in range(7)] for d in range(3)])
    return out

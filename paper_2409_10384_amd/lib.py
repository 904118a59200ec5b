"""Thin Python binding of libgrmhd.so: argument marshalling only.

Every step of the path runs in the HIP kernels of the library; torch supplies
device memory and streams.  There is no CPU fallback: importing the binding
without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrmhd.so")
_lib = None

# flag bits
F_C2P_FAIL, F_DFLOOR, F_TAUFLOOR, F_MAGCAP, F_TFLOOR, F_RHOFLOOR, F_FOFC, F_DMP, \
    F_BRACKET_FALLBACK, F_MAXIT, F_EXCISED = [1 << b for b in range(11)]
GF_W, GF_US, GF_BS, GF_FLAGS = 1, 2, 4, 8


class GrmhdError(RuntimeError):
    pass


class GrmhdParams(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("rho_b", C.c_double * 3), ("K0", C.c_double),
        ("Gam", C.c_double * 4), ("gamma_th", C.c_double), ("rho_atm", C.c_double),
        ("T_atm", C.c_double), ("f_thr", C.c_double), ("M_max", C.c_double),
        ("dmp_M", C.c_double), ("c2p_tol", C.c_double),
        ("eos", C.c_int32), ("npieces", C.c_int32), ("recon", C.c_int32),
        ("riemann", C.c_int32), ("fofc", C.c_int32), ("c2p_maxit", C.c_int32),
    ]


VP = C.c_void_p


class GrmhdBlock(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ng", C.c_int32),
        ("dx", C.c_double * 3),
        ("w", VP * 5), ("un", VP * 5), ("us", VP * 5), ("bn", VP * 3), ("bs", VP * 3),
        ("adm", VP * 16), ("uo", VP * 5), ("bo", VP * 3), ("wo", VP * 5),
        ("flags", VP), ("scratch", VP), ("nbr", C.c_int32 * 27), ("bc", C.c_int32),
        ("wave0", C.c_int32 * 24), ("nblk", C.c_int32), ("reserved", C.c_int32),
    ]


class Rk2Tables(C.Structure):
    """grmhd_rk2_tables: host and device tables of set A, set B, stage 1
    (A -> B) and stage 2 (B -> A)"""
    _fields_ = [(n, C.c_void_p) for n in ("a_h", "a_d", "b_h", "b_d", "ab_h", "ab_d", "ba_h", "ba_d")]


class GrmhdAmrLink(C.Structure):
    """grmhd_amr_link: a leaf's level, origin, domain size and the leaves
    covering each of its 27 neighbour regions"""
    _fields_ = [
        ("level", C.c_int32), ("org", C.c_int32 * 3), ("N", C.c_int32 * 3), ("periodic", C.c_int32),
        ("rel", C.c_int32 * 27), ("src", (C.c_int32 * 4) * 27),
    ]


class C2PStats(C.Structure):
    _fields_ = [("solves", C.c_uint64), ("evaluations", C.c_uint64), ("fallbacks", C.c_uint64),
                ("failures", C.c_uint64)]


def load():
    """Load the in-tree libgrmhd.so (built by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GrmhdError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    L.grmhd_scratch_doubles.restype = C.c_int64
    L.grmhd_scratch_doubles.argtypes = [C.c_int32] * 4
    L.grmhd_flux_offset.restype = C.c_int64
    L.grmhd_flux_offset.argtypes = [C.c_int32] * 6
    L.grmhd_version.restype = C.c_char_p
    L.grmhd_blocks_prepare.argtypes = [C.c_void_p, C.c_int32]
    blk = [C.c_void_p, C.c_void_p, C.c_int32]
    stage = blk + [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p]
    for name in ("grmhd_stage", "fofc_correct", "ct_update", "grmhd_update"):
        getattr(L, name).argtypes = stage
    L.grmhd_fluxes.argtypes = blk + [C.c_void_p, C.c_void_p]
    L.grmhd_stage_c2p.argtypes = blk + [C.c_void_p, C.c_void_p]
    L.grmhd_stage_cfl.argtypes = blk + [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_double, C.c_double, C.c_void_p]
    L.grmhd_stage_learned.argtypes = stage[:-1] + [C.c_void_p, C.c_void_p, C.c_void_p]
    L.grmhd_stage_c2p_learned.argtypes = blk + [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.grmhd_matter_sources.argtypes = blk + [C.c_void_p, C.c_void_p, C.c_void_p]
    L.grmhd_excise.argtypes = blk + [C.c_void_p, C.c_double, C.c_void_p]
    L.grmhd_prim2con_blocks.argtypes = blk + [C.c_void_p, C.c_void_p]
    L.grmhd_ghost_fill.argtypes = blk + [C.c_int32, C.c_void_p]
    L.grmhd_dt.argtypes = blk + [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
    L.grmhd_mass.argtypes = blk + [C.c_void_p, C.c_void_p, C.c_void_p]
    L.grmhd_mass_noalloc.argtypes = blk + [C.c_void_p, C.c_void_p]
    L.grmhd_mass_noalloc_max_blocks.restype = C.c_int32
    L.prim2con.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_void_p]
    L.c2p_batch.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    vp = C.c_void_p
    L.grmhd_rk2_step.argtypes = [vp, C.c_int32, vp, C.c_double, vp, vp, vp]
    L.grmhd_graph_build.argtypes = [vp, C.c_int32, vp, C.c_double, vp, vp, vp, C.POINTER(vp)]
    L.grmhd_graph_launch.argtypes = [vp, vp]
    L.grmhd_graph_destroy.argtypes = [vp]
    L.grmhd_autotune.argtypes = blk + [vp, C.c_double, C.c_int32, vp, vp, vp]
    L.grmhd_timing.argtypes = [C.c_int32]
    L.grmhd_set_threads.argtypes = [C.c_int32, C.c_int32]
    L.grmhd_timing_read.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.grmhd_copy.argtypes = [vp, vp, C.c_int64, vp]
    L.c2p_mlp_features.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.c2p_mlp_forward.argtypes = [vp, C.c_int64, vp, vp, vp]
    L.c2p_mlp_to_bf16.argtypes = [vp, vp, vp]
    L.c2p_mlp_calibrate_width.argtypes = [vp, C.c_int64, vp, vp, C.c_double, C.c_float, vp, vp]
    L.grmhd_c2p_pairs.argtypes = blk + [C.c_int32, vp, vp, vp, vp, vp, vp]
    L.c2p_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, C.c_float, C.c_int32, vp, vp,
                                     vp, vp, vp]
    L.grmhd_amr_links.argtypes = [C.c_int32, vp, vp, C.c_int32, C.c_int32, vp, vp, vp]
    L.grmhd_ghost_fill_amr.argtypes = blk + [vp, vp, C.c_int32, vp]
    L.grmhd_stage_amr.argtypes = blk + [vp, vp] + stage[3:-1] + [vp, vp, vp]
    _lib = L
    return L


def amr_links(levels, orgs, nb, ng, n0, periodic):
    """host array of grmhd_amr_link of a leaf mesh (grmhd_amr_links)"""
    n = len(levels)
    lv = (C.c_int32 * n)(*levels)
    og = (C.c_int32 * (3 * n))(*[int(x) for o in orgs for x in o])
    links = (GrmhdAmrLink * n)()
    check(load().grmhd_amr_links(n, C.cast(lv, C.c_void_p), C.cast(og, C.c_void_p), nb, ng,
                                 C.cast((C.c_int32 * 3)(*n0), C.c_void_p),
                                 C.cast((C.c_int32 * 3)(*periodic), C.c_void_p), links),
          "grmhd_amr_links")
    return links


def _nullctx():
    import contextlib
    return contextlib.nullcontext()


def check(rc, what):
    if rc != 0:
        raise GrmhdError(f"{what} failed with status {rc}")


def stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclasses.dataclass
class MethodParams:
    """Method options (same meaning as the fields of grmhd_params); recon: 0
    donor cell, 1 PLM, 2 WENOZ, 3 PPM4, 4 PPMX."""

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

    def c(self) -> GrmhdParams:
        p = GrmhdParams()
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if f.name == "rho_b":
                p.rho_b = (C.c_double * 3)(*v)
            elif f.name == "Gam":
                p.Gam = (C.c_double * 4)(*v)
            else:
                setattr(p, f.name, v)
        return p


def _ptr(t: torch.Tensor):
    return t.data_ptr()


def _ptr_array(ts):
    arr = (C.c_void_p * len(ts))(*[_ptr(t) for t in ts])
    return arr


# ---------------------------------------------------------------------------
# measurement helpers
# ---------------------------------------------------------------------------
FAMILIES = ["flux_x", "flux_y", "flux_z", "fofc_flags", "fofc_fix", "ct", "update", "stage_c2p",
            "ghost", "dt", "bcc", "c2p_batch", "c2p_learned", "mlp_train", "mlp_bracket",
            "stage_c2p_learned", "matter", "excise"]
KERNEL_OF_FAMILY = {"flux_x": "k_flux<0>", "flux_y": "k_flux<1>", "flux_z": "k_flux<2>",
                    "fofc_flags": "k_fofc_flags", "update": "k_update", "stage_c2p": "k_stage_c2p",
                    "dt": "k_dt", "bcc": "k_bcc", "c2p_batch": "k_c2p_batch",
                    "c2p_learned": "k_c2p_learned", "mlp_train": "k_mlp_train",
                    "mlp_bracket": "k_mlp_bracket", "stage_c2p_learned": "k_stage_c2p_learned"}


def timing(on: bool):
    check(load().grmhd_timing(1 if on else 0), "grmhd_timing")


def timing_read():
    """{family: (total ms, launches)} since timing was enabled"""
    L = load()
    out = {}
    for f, name in enumerate(FAMILIES):
        ms = C.c_double(0.0)
        cnt = C.c_int64(0)
        check(L.grmhd_timing_read(f, C.byref(ms), C.byref(cnt)), "grmhd_timing_read")
        if cnt.value:
            out[name] = (ms.value, cnt.value)
    return out


def copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    check(load().grmhd_copy(_ptr(src), _ptr(dst), src.numel(), stream_ptr(stream)), "grmhd_copy")


# ---------------------------------------------------------------------------
# pointwise entry points
# ---------------------------------------------------------------------------
def prim2con(w: torch.Tensor, bt: torch.Tensor, gam: torch.Tensor, params: MethodParams, stream=None):
    """Eq. 7 on device: w (5,n), bt (3,n), gam (6,n) float64 cuda -> u (5,n)."""
    L = load()
    n = w.shape[1]
    u = torch.empty((5, n), dtype=torch.float64, device=w.device)
    pw, pb, pg, pu = _ptr_array(list(w)), _ptr_array(list(bt)), _ptr_array(list(gam)), _ptr_array(list(u))
    check(L.prim2con(n, pw, pb, pg, pu, C.byref(params.c()), stream_ptr(stream)), "prim2con")
    return u


def c2p_batch(u: torch.Tensor, bt: torch.Tensor, gam: torch.Tensor, params: MethodParams,
              want_mu=False, want_nev=False, stats=False, stream=None):
    """C2P on device.  u (5,n) is rewritten in place where a floor fires.
    Returns dict(w, flags[, mu, nev, stats])."""
    L = load()
    n = u.shape[1]
    dev = u.device
    w = torch.empty((5, n), dtype=torch.float64, device=dev)
    flags = torch.empty(n, dtype=torch.int16, device=dev)
    mu = torch.empty(n, dtype=torch.float64, device=dev) if want_mu else None
    nev = torch.empty(n, dtype=torch.int32, device=dev) if want_nev else None
    st = torch.zeros(4, dtype=torch.int64, device=dev) if stats else None
    rc = L.c2p_batch(n, _ptr_array(list(u)), _ptr_array(list(bt)), _ptr_array(list(gam)),
                     _ptr_array(list(w)), _ptr(flags), C.byref(params.c()), None,
                     _ptr(st) if st is not None else None, _ptr(mu) if mu is not None else None,
                     _ptr(nev) if nev is not None else None, stream_ptr(stream))
    check(rc, "c2p_batch")
    out = {"w": w, "flags": flags}
    if mu is not None:
        out["mu"] = mu
    if nev is not None:
        out["nev"] = nev
    if st is not None:
        out["stats"] = st
    return out


# ---------------------------------------------------------------------------
# device mesh of blocks and the RK2 driver
# ---------------------------------------------------------------------------
def scratch_doubles(nx, ny, nz, ng):
    return load().grmhd_scratch_doubles(nx, ny, nz, ng)


def flux_offset(nx, ny, nz, ng, d, c):
    return load().grmhd_flux_offset(nx, ny, nz, ng, d, c)


class DeviceMesh:
    """Blocks resident in HBM with the state sets of the SSP Runge-Kutta
    schemes in Shu-Osher form (A: U^n side, B: first-stage output, C: second-
    stage output of RK3, allocated on first use), the per-block scratch, and
    the descriptor tables of the stages (host and device copies).

    A stage with coefficients (a0, a1, b) computes a0 U^n + a1 U^(s) + b dt
    L(U^(s)) reading U^(s) from one set and writing another:
      RK2: A -> B (0, 1, 1); B -> A (1/2, 1/2, 1/2)
      RK3: A -> B (0, 1, 1); B -> C (3/4, 1/4, 1/4); C -> A (1/3, 2/3, 2/3)
    (Gottlieb, Ketcheson & Shu 2009, the second- and third-order SSP schemes)."""

    RK2 = ((0, 1, (0.0, 1.0, 1.0)), (1, 0, (0.5, 0.5, 0.5)))
    RK3 = ((0, 1, (0.0, 1.0, 1.0)), (1, 2, (0.75, 0.25, 0.25)),
           (2, 0, (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)))

    def __init__(self, blocks, params: MethodParams, device="cuda", stream=None):
        L = load()
        self.params = params
        self.blocks = blocks
        self.device = torch.device(device)
        self.stream = stream
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.w0, self.u0, self.b0, self.w1, self.u1, self.b1 = [], [], [], [], [], []
        self.w2, self.u2, self.b2 = None, None, None
        self.adm, self.flags, self.scratch = [], [], []
        def up(a):
            if isinstance(a, torch.Tensor):
                return a.to(dev, dtype=torch.float64).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

        for b in blocks:
            shp = b.shape
            self.w0.append(up(b.w))
            self.b0.append([up(x) for x in b.bf])
            self.adm.append(up(b.adm))
            self.u0.append(torch.zeros((5,) + shp, **f64))
            self.w1.append(torch.zeros((5,) + shp, **f64))
            self.u1.append(torch.zeros((5,) + shp, **f64))
            self.b1.append([torch.zeros_like(x) for x in self.b0[-1]])
            self.flags.append(torch.zeros(shp, dtype=torch.int16, device=dev))
            self.scratch.append(torch.zeros(L.grmhd_scratch_doubles(b.nx, b.ny, b.nz, b.ng), **f64))
        self.tables = {}
        for key in ((0, 1), (1, 0), (0, 0), (1, 1)):
            self.tables[key] = self._make_table(key)
        # conserved state from the primitives (Eq. 7) on the device, all cells
        check(L.grmhd_prim2con_blocks(*self._args((0, 0)), C.byref(params.c()), self.sp()),
              "grmhd_prim2con_blocks")
        # set B starts as a copy of set A: frozen ghosts (bc == 0) then hold the
        # initial data in both sets (the stages write interiors only)
        with torch.cuda.stream(self.stream) if self.stream is not None else _nullctx():
            for ib in range(len(blocks)):
                self.u1[ib].copy_(self.u0[ib])
                self.w1[ib].copy_(self.w0[ib])
                for d in range(3):
                    self.b1[ib][d].copy_(self.b0[ib][d])
        self.red = torch.zeros(1, **f64)
        self.dt_dev = torch.zeros(1, **f64)
        self.mass_part = torch.zeros(len(blocks), **f64)
        self.mass_out = torch.zeros(1, **f64)

    def _desc(self, ib, w, un, us, bn, bs, uo, bo, wo):
        b = self.blocks[ib]
        d = GrmhdBlock()
        d.nx, d.ny, d.nz, d.ng = b.nx, b.ny, b.nz, b.ng
        d.dx = (C.c_double * 3)(*b.dx)
        d.w = _ptr_array(list(w))
        d.un = _ptr_array(list(un))
        d.us = _ptr_array(list(us))
        d.bn = _ptr_array(bn)
        d.bs = _ptr_array(bs)
        d.adm = _ptr_array(list(self.adm[ib]))
        d.uo = _ptr_array(list(uo))
        d.bo = _ptr_array(bo)
        d.wo = _ptr_array(list(wo))
        d.flags = _ptr(self.flags[ib])
        d.scratch = _ptr(self.scratch[ib])
        d.nbr = (C.c_int32 * 27)(*b.nbr)
        d.bc = b.bc
        return d

    def _set(self, k):
        """(U, w, faces) lists of state set k (0 A, 1 B, 2 C)"""
        if k == 2:
            self._ensure_set_c()
        return ((self.u0, self.w0, self.b0), (self.u1, self.w1, self.b1),
                (self.u2, self.w2, self.b2))[k]

    def _ensure_set_c(self):
        """set C (RK3 only) starts as a copy of set A: frozen ghosts then hold
        the initial data, as in the other sets"""
        if self.u2 is not None:
            return
        with torch.cuda.stream(self.stream) if self.stream is not None else _nullctx():
            self.u2 = [u.clone() for u in self.u0]
            self.w2 = [w.clone() for w in self.w0]
            self.b2 = [[x.clone() for x in bf] for bf in self.b0]

    def _make_table(self, key):
        """key (src, dst): a stage reading w, U^(s), B^(s) from set src and
        U^n, B^n from set A, writing U, B, w into set dst; (k, k) is the
        table of set k alone (ghost fills, dt, mass)"""
        src, dst = key
        n = len(self.blocks)
        arr = (GrmhdBlock * n)()
        (us, ws, bs), (ua, _, ba), (uo, wo, bo) = self._set(src), self._set(0), self._set(dst)
        if src == dst:
            ua, ba = us, bs
        for ib in range(n):
            arr[ib] = self._desc(ib, ws[ib], ua[ib], us[ib], ba[ib], bs[ib], uo[ib], bo[ib], wo[ib])
        check(load().grmhd_blocks_prepare(C.cast(arr, C.c_void_p), n), "grmhd_blocks_prepare")
        raw = bytes(memoryview(arr).cast("B"))
        dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        return arr, dev

    def _args(self, key):
        if key not in self.tables:
            self.tables[key] = self._make_table(key)
        arr, dev = self.tables[key]
        return C.cast(arr, C.c_void_p), C.c_void_p(dev.data_ptr()), len(self.blocks)

    def sp(self):
        return stream_ptr(self.stream)

    # --- steps --------------------------------------------------------------
    def stage(self, stage, dt=None, dt_dev=None, mlp=None, stats=None):
        """Stage 1 or 2 of SSP-RK2; mlp (a LearnedC2P) starts the final
        inversion from the learned bracket, stats (a 4-element int64 device
        tensor) accumulates its solves, evaluations, fallbacks and failures."""
        src, dst, coef = self.RK2[stage - 1]
        self.stage_sets(src, dst, coef, dt=dt, dt_dev=dt_dev, mlp=mlp, stats=stats)

    def stage_sets(self, src, dst, coef, dt=None, dt_dev=None, mlp=None, stats=None):
        """One stage with coefficients coef = (a0, a1, b) from set src into
        set dst (dt from dt_dev on the device when given)."""
        L = load()
        a0, a1, b = coef
        key = (src, dst)
        dptr = C.c_void_p(dt_dev.data_ptr()) if dt_dev is not None else None
        dval = float(dt) if dt is not None else 0.0
        if mlp is None and stats is None:
            rc = L.grmhd_stage(*self._args(key), C.byref(self.params.c()), dptr, dval, a0, a1, b,
                               self.sp())
        elif mlp is None:
            rc = L.grmhd_stage_learned(*self._args(key), C.byref(self.params.c()), dptr, dval, a0,
                                       a1, b, None, C.c_void_p(stats.data_ptr()), self.sp())
        else:
            self._mlp_keep = mlp.c()
            sptr = C.c_void_p(stats.data_ptr()) if stats is not None else None
            rc = L.grmhd_stage_learned(*self._args(key), C.byref(self.params.c()), dptr, dval, a0,
                                       a1, b, C.byref(self._mlp_keep), sptr, self.sp())
        check(rc, "grmhd_stage")

    def stage_cfl(self, src, dst, coef, cfl):
        """one stage whose dt is the CFL dt of its input, reduced in the
        stage's first kernel (grmhd_stage_cfl); dt left in self.dt_dev"""
        a0, a1, b = coef
        check(load().grmhd_stage_cfl(*self._args((src, dst)), C.byref(self.params.c()), float(cfl),
                                     C.c_void_p(self.red.data_ptr()), C.c_void_p(self.dt_dev.data_ptr()),
                                     a0, a1, b, self.sp()), "grmhd_stage_cfl")
        return self.dt_dev

    # the first stage of a device-dt step takes its dt from grmhd_stage_cfl
    # (plain inversion, one-level mesh); else from grmhd_dt before it
    fused_dt = True

    def ghost_fill(self, which, mask=GF_W | GF_US | GF_BS):
        """ghosts of state set which (0 A, 1 B, 2 C)"""
        check(load().grmhd_ghost_fill(*self._args((which, which)), mask, self.sp()),
              "grmhd_ghost_fill")

    def compute_dt(self, cfl):
        """dt on device (kept in self.dt_dev)."""
        rc = load().grmhd_dt(*self._args((0, 0)), C.byref(self.params.c()), cfl,
                             C.c_void_p(self.red.data_ptr()), C.c_void_p(self.dt_dev.data_ptr()),
                             self.sp())
        check(rc, "grmhd_dt")
        return self.dt_dev

    def rk_step(self, scheme, dt=None, cfl=0.25, mlp=None, stats=None):
        """One step of `scheme` (RK2 or RK3); dt from the device CFL reduction
        when dt is None; the ghosts of each stage's output are filled before
        the next stage; mlp/stats as for stage()."""
        fused = dt is None and self.fused_dt and mlp is None and stats is None
        if dt is None:
            if not fused:
                self.compute_dt(cfl)
            kw = dict(dt_dev=self.dt_dev)
        else:
            kw = dict(dt=dt)
        for k, (src, dst, coef) in enumerate(scheme):
            if fused and k == 0:
                self.stage_cfl(src, dst, coef, cfl)
            else:
                self.stage_sets(src, dst, coef, mlp=mlp, stats=stats, **kw)
            if self.alpha_excise > 0.0:
                self.excise(dst, self.alpha_excise)
            self.ghost_fill(dst)

    # lapse below which each stage's output is excised (0: no excision)
    alpha_excise = 0.0

    def excise(self, which, alpha_min):
        """atmosphere in the interior cells of state set `which` where the lapse
        is below alpha_min (field unchanged; flag bit F_EXCISED)"""
        check(load().grmhd_excise(*self._args((which, which)), C.byref(self.params.c()),
                                  float(alpha_min), self.sp()), "grmhd_excise")

    def matter_sources(self, which=0):
        """ADM matter sources (E, S_i, S_ij; not densitized) of state set
        `which` at the interior cells: per block a (10, sz, sy, sx) tensor whose
        ghost cells are zero"""
        if getattr(self, "_matter", None) is None:
            f64 = dict(dtype=torch.float64, device=self.device)
            self._matter = [torch.zeros((10,) + b.shape, **f64) for b in self.blocks]
            ptrs = [t[n].data_ptr() for t in self._matter for n in range(10)]
            self._matter_ptrs = torch.tensor(ptrs, dtype=torch.int64).to(self.device)
        check(load().grmhd_matter_sources(*self._args((which, which)), C.byref(self.params.c()),
                                          C.c_void_p(self._matter_ptrs.data_ptr()), self.sp()),
              "grmhd_matter_sources")
        return self._matter

    def rk2_step(self, dt=None, cfl=0.25, mlp=None, stats=None):
        self.rk_step(self.RK2, dt=dt, cfl=cfl, mlp=mlp, stats=stats)

    def rk3_step(self, dt=None, cfl=0.25, mlp=None, stats=None):
        self.rk_step(self.RK3, dt=dt, cfl=cfl, mlp=mlp, stats=stats)

    def rk2_step_per_block(self, dt=None, cfl=0.25):
        """The same RK2 step launched block by block (one-block tables): the
        unbatched baseline.  Only for blocks with frozen ghosts (bc == 0)."""
        L = load()
        if any(b.bc != 0 for b in self.blocks):
            raise GrmhdError("per-block launches need independent blocks (bc == 0)")
        if not hasattr(self, "_single"):
            self._single = []
            for ib in range(len(self.blocks)):
                t = {}
                for key, stage in (("s1", 1), ("s2", 2)):
                    arr = (GrmhdBlock * 1)()
                    if stage == 1:
                        arr[0] = self._desc(ib, self.w0[ib], self.u0[ib], self.u0[ib], self.b0[ib],
                                            self.b0[ib], self.u1[ib], self.b1[ib], self.w1[ib])
                    else:
                        arr[0] = self._desc(ib, self.w1[ib], self.u0[ib], self.u1[ib], self.b0[ib],
                                            self.b1[ib], self.u0[ib], self.b0[ib], self.w0[ib])
                    arr[0].nbr = (C.c_int32 * 27)(*([-1] * 27))
                    check(L.grmhd_blocks_prepare(C.cast(arr, C.c_void_p), 1), "grmhd_blocks_prepare")
                    raw = bytes(memoryview(arr).cast("B"))
                    t[key] = (arr, torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device))
                self._single.append(t)
        if dt is None:
            self.compute_dt(cfl)
            dptr, dval = C.c_void_p(self.dt_dev.data_ptr()), 0.0
        else:
            dptr, dval = None, float(dt)
        pc = C.byref(self.params.c())
        for stage, (a0, a1, b) in ((1, (0.0, 1.0, 1.0)), (2, (0.5, 0.5, 0.5))):
            key = "s1" if stage == 1 else "s2"
            for t in self._single:
                arr, dev = t[key]
                check(L.grmhd_stage(C.cast(arr, C.c_void_p), C.c_void_p(dev.data_ptr()), 1, pc, dptr,
                                    dval, a0, a1, b, self.sp()), "grmhd_stage")

    # --- the step as one library call, as a HIP graph, and the autotuner ----
    def _rk2_tables(self):
        t = Rk2Tables()
        for name, key in (("a", (0, 0)), ("b", (1, 1)), ("ab", (0, 1)), ("ba", (1, 0))):
            h, d, _ = self._args(key)
            setattr(t, name + "_h", h.value)
            setattr(t, name + "_d", d.value)
        self._t_keep = t
        return t

    def rk2_step_lib(self, cfl=0.25):
        """the whole SSP-RK2 step with the device dt as one library call
        (grmhd_rk2_step); dt lands in self.dt_dev"""
        t = self._rk2_tables()
        check(load().grmhd_rk2_step(C.byref(t), len(self.blocks), C.byref(self.params.c()), cfl,
                                    C.c_void_p(self.red.data_ptr()), C.c_void_p(self.dt_dev.data_ptr()),
                                    self.sp()), "grmhd_rk2_step")

    def rk2_graph(self, stream, cfl=0.25):
        """the SSP-RK2 step captured on `stream` (a torch.cuda.Stream) into a
        library HIP graph; returns a Rk2Graph (launch(stream), close())"""
        t = self._rk2_tables()
        self._graph_params = self.params.c()
        g = C.c_void_p()
        check(load().grmhd_graph_build(C.byref(t), len(self.blocks), C.byref(self._graph_params), cfl,
                                       C.c_void_p(self.red.data_ptr()),
                                       C.c_void_p(self.dt_dev.data_ptr()),
                                       C.c_void_p(stream.cuda_stream), C.byref(g)),
              "grmhd_graph_build")
        return Rk2Graph(g, self)

    def autotune(self, dt, reps=2):
        """the library's autotuner over the first stage (grmhd_autotune):
        {family: (best size, {size: ms})}"""
        th = (C.c_int32 * 8)()
        ms = (C.c_double * 32)()
        check(load().grmhd_autotune(*self._args((0, 1)), C.byref(self.params.c()), float(dt), reps,
                                    th, ms, self.sp()), "grmhd_autotune")
        names = ("flux_x", "flux_y", "flux_z", "fofc_flags", "fofc_fix", "ct", "update", "stage_c2p")
        return {n: (int(th[f]), {sz: float(ms[f * 4 + c]) for c, sz in enumerate((64, 128, 256, 512))})
                for f, n in enumerate(names)}

    def mass(self):
        check(load().grmhd_mass(*self._args((0, 0)), C.c_void_p(self.mass_part.data_ptr()),
                                C.c_void_p(self.mass_out.data_ptr()), self.sp()), "grmhd_mass")
        return self.mass_out

    def mass_noalloc(self, out):
        """grmhd_mass_noalloc into the device double `out` (the partial sums
        in the library's fixed device array)"""
        check(load().grmhd_mass_noalloc(*self._args((0, 0)), C.c_void_p(out.data_ptr()), self.sp()),
              "grmhd_mass_noalloc")
        return out

    # --- granular steps (for tests) ------------------------------------------
    def run_steps(self, stage, dt, mode):
        """mode bits: 1 fluxes, 2 FOFC, 4 CT, 8 update, 16 C2P (host dt)."""
        L = load()
        a0, a1, b = (0.0, 1.0, 1.0) if stage == 1 else (0.5, 0.5, 0.5)
        args = self._args((0, 1) if stage == 1 else (1, 0))
        pc = C.byref(self.params.c())
        if mode & 1:
            check(L.grmhd_fluxes(*args, pc, self.sp()), "grmhd_fluxes")
        if mode & 2:
            check(L.fofc_correct(*args, pc, None, dt, a0, a1, b, self.sp()), "fofc_correct")
        if mode & 4:
            check(L.ct_update(*args, pc, None, dt, a0, a1, b, self.sp()), "ct_update")
        if mode & 8:
            check(L.grmhd_update(*args, pc, None, dt, a0, a1, b, self.sp()), "grmhd_update")
        if mode & 16:
            check(L.grmhd_stage_c2p(*args, pc, self.sp()), "grmhd_stage_c2p")

    def flux_view(self, ib, d, c):
        """face array of flux component c in direction d from block ib's scratch"""
        b = self.blocks[ib]
        sz, sy, sx = b.shape
        shape = [(sz, sy, sx + 1), (sz, sy + 1, sx), (sz + 1, sy, sx)][d]
        off = flux_offset(b.nx, b.ny, b.nz, b.ng, d, c)
        n = shape[0] * shape[1] * shape[2]
        return self.scratch[ib][off:off + n].view(shape)

    def c2p_pairs(self, which=0, stride=1):
        """Conserved/primitive pairs of the interior cells of every block (the
        states this mesh holds), flattened: u (5, n), densitized cell-centred
        field bt (3, n), gamma_ij (6, n), w (5, n).  stride > 1 keeps every
        stride-th cell along x (to subsample).  Gathered by the library
        (grmhd_c2p_pairs)."""
        counts = [b.nz * b.ny * ((b.nx + stride - 1) // stride) for b in self.blocks]
        base = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
        n = int(sum(counts))
        f64 = dict(dtype=torch.float64, device=self.device)
        u, bt = torch.empty((5, n), **f64), torch.empty((3, n), **f64)
        gam, w = torch.empty((6, n), **f64), torch.empty((5, n), **f64)
        base_d = torch.as_tensor(base).to(self.device)
        check(load().grmhd_c2p_pairs(*self._args((which, which)), int(stride),
                                     C.c_void_p(base_d.data_ptr()), _ptr_array(list(u)),
                                     _ptr_array(list(bt)), _ptr_array(list(gam)), _ptr_array(list(w)),
                                     self.sp()), "grmhd_c2p_pairs")
        if self.stream is None:
            torch.cuda.current_stream(self.device).synchronize()
        else:
            self.stream.synchronize()
        return u, bt, gam, w

    def interior(self, t, ib):
        b = self.blocks[ib]
        g = b.ng
        return t[..., g:g + b.nz, g:g + b.ny, g:g + b.nx]


# ---------------------------------------------------------------------------
# learned guess and bracket for the inversion
# ---------------------------------------------------------------------------
NPARAM = 8834


class RefinedDeviceMesh(DeviceMesh):
    """A DeviceMesh whose blocks are the leaves of a refined mesh (a LeafMesh
    of paper_2409_10384_amd.inputs, blocks in its leaf order): ghost fills
    across levels (grmhd_ghost_fill_amr) and stages with the flux and EMF
    corrections at level boundaries (grmhd_stage_amr)."""

    fused_dt = False

    def __init__(self, blocks, params: MethodParams, leafmesh, device="cuda", stream=None):
        b0 = blocks[0]
        self.links = amr_links(leafmesh.levels, [leafmesh.org(i) for i in range(len(blocks))],
                               b0.nx, b0.ng, leafmesh.n0, leafmesh.periodic)
        self.leafmesh = leafmesh
        super().__init__(blocks, params, device=device, stream=stream)
        raw = bytes(memoryview(self.links).cast("B"))
        self.links_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)

    def _links(self):
        return C.cast(self.links, C.c_void_p), C.c_void_p(self.links_dev.data_ptr())

    def stage_sets(self, src, dst, coef, dt=None, dt_dev=None, mlp=None, stats=None):
        a0, a1, b = coef
        dptr = C.c_void_p(dt_dev.data_ptr()) if dt_dev is not None else None
        dval = float(dt) if dt is not None else 0.0
        mptr = None
        if mlp is not None:
            self._mlp_keep = mlp.c()
            mptr = C.byref(self._mlp_keep)
        sptr = C.c_void_p(stats.data_ptr()) if stats is not None else None
        check(load().grmhd_stage_amr(*self._args((src, dst)), *self._links(), C.byref(self.params.c()),
                                     dptr, dval, a0, a1, b, mptr, sptr, self.sp()), "grmhd_stage_amr")

    def ghost_fill(self, which, mask=GF_W | GF_US | GF_BS):
        check(load().grmhd_ghost_fill_amr(*self._args((which, which)), *self._links(), mask, self.sp()),
              "grmhd_ghost_fill_amr")


class Rk2Graph:
    """an instantiated library graph of one SSP-RK2 step (keeps its mesh,
    whose arrays and tables it replays, alive)"""

    def __init__(self, handle, mesh):
        self.handle, self.mesh = handle, mesh

    def launch(self, stream=None):
        s = C.c_void_p(stream.cuda_stream) if stream is not None else None
        check(load().grmhd_graph_launch(self.handle, s), "grmhd_graph_launch")

    def close(self):
        if self.handle:
            check(load().grmhd_graph_destroy(self.handle), "grmhd_graph_destroy")
            self.handle = None


class C2PMlp(C.Structure):
    _fields_ = [("w_bf16", C.c_void_p), ("w_f32", C.c_void_p), ("feat_mean", C.c_float * 5),
                ("feat_scale", C.c_float * 5), ("width_k", C.c_float), ("width_min", C.c_float),
                ("bracket_ws", C.c_void_p)]


class LearnedC2P:
    """Parameters (fp32 master + bf16 copy), Adam moments and feature
    standardisation of the guess network, resident on the device."""

    def __init__(self, device="cuda", seed=0, width_k=4.0, width_min=1e-3):
        g = torch.Generator(device="cpu").manual_seed(seed)
        theta = torch.zeros(NPARAM, dtype=torch.float32)
        # He-normal weights, zero biases; layout W1 b1 W2 b2 W3 b3 W4 b4
        offs = [(0, 64, 5), (384, 64, 64), (4544, 64, 64), (8704, 2, 64)]
        for off, o, i in offs:
            theta[off:off + o * i] = torch.randn(o * i, generator=g) * (2.0 / i) ** 0.5
        self.device = torch.device(device)
        self.theta = theta.to(self.device)
        self.theta_h = torch.zeros(NPARAM, dtype=torch.int16, device=self.device)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.mean = [0.0] * 5
        self.scale = [1.0] * 5
        self.width_k, self.width_min = width_k, width_min
        self.step = 0
        self.refresh_bf16()

    def refresh_bf16(self, stream=None):
        check(load().c2p_mlp_to_bf16(_ptr(self.theta), _ptr(self.theta_h), stream_ptr(stream)),
              "c2p_mlp_to_bf16")

    def c(self):
        s = C2PMlp()
        s.w_bf16 = _ptr(self.theta_h)
        s.w_f32 = _ptr(self.theta)
        s.feat_mean = (C.c_float * 5)(*self.mean)
        s.feat_scale = (C.c_float * 5)(*self.scale)
        s.width_k, s.width_min = self.width_k, self.width_min
        return s

    def features(self, u, bt, gam, params: MethodParams, w_true=None, standardise=True, stream=None):
        """features [5][n] (fp32) and targets [n] (when w_true is given)"""
        n = u.shape[1]
        feats = torch.empty((5, n), dtype=torch.float32, device=u.device)
        target = torch.empty(n, dtype=torch.float32, device=u.device) if w_true is not None else None
        mean = (C.c_float * 5)(*(self.mean if standardise else [0.0] * 5))
        scale = (C.c_float * 5)(*(self.scale if standardise else [1.0] * 5))
        rc = load().c2p_mlp_features(n, _ptr_array(list(u)), _ptr_array(list(bt)), _ptr_array(list(gam)),
                                     _ptr_array(list(w_true)) if w_true is not None else None,
                                     C.byref(params.c()), C.cast(mean, C.c_void_p),
                                     C.cast(scale, C.c_void_p), _ptr(feats),
                                     _ptr(target) if target is not None else None, stream_ptr(stream))
        check(rc, "c2p_mlp_features")
        return feats, target

    def fit_standardisation(self, raw_feats):
        """mean and 1/std of raw features (setup, not the hot path)"""
        self.mean = [float(x) for x in raw_feats.double().mean(dim=1).cpu()]
        sd = raw_feats.double().std(dim=1).cpu()
        self.scale = [float(1.0 / max(x, 1e-12)) for x in sd]

    def fit(self, u, bt, gam, params: MethodParams, w_true, steps=20000, batch=4096, lr=2e-3,
            seed=0, log_every=0, log=None, calibrate=0.99, width_min=1e-4):
        """Standardise on the raw features of (u, bt, gam), then train on the
        targets of w_true for `steps` Adam steps of `batch` samples with a
        cosine-decaying learning rate (the training kernels of this library),
        then (calibrate = q, not None) set the bracket width so that it holds
        the label of a fraction q of the training samples.  Returns the loss of
        every log_every-th step."""
        import math
        raw, _ = self.features(u, bt, gam, params, standardise=False)
        self.fit_standardisation(raw)
        feats, target = self.features(u, bt, gam, params, w_true=w_true)
        keep = torch.isfinite(target) & (target.abs() < 40.0)
        if not bool(keep.all()):
            feats, target = feats[:, keep].contiguous(), target[keep].contiguous()
        gen = torch.Generator(device=feats.device).manual_seed(seed)
        losses = []
        for it in range(steps):
            idx = torch.randint(0, feats.shape[1], (batch,), device=feats.device, generator=gen)
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps)) + 1e-5
            loss, _ = self.train_step(feats[:, idx].contiguous(), target[idx].contiguous(), lr=rate)
            if log_every and it % log_every == 0:
                losses.append(float(loss.item()))
                if log:
                    log(f"  train step {it}: loss {losses[-1]:.4g}")
        if calibrate is not None:
            self.calibrate_width(feats, target, q=calibrate, seed=seed, width_min=width_min)
        return losses

    def calibrate_width(self, feats, target, q=0.99, nmax=1 << 20, seed=0, width_min=1e-4):
        """Set the bracket half-width factor k so that the bracket logistic(y0
        -+ (k exp(y1) + width_min)) holds the training label for a fraction q
        of (up to nmax, drawn at random) training samples: the library's
        c2p_mlp_calibrate_width (k = the q-quantile of |y0 - t| / exp(y1))."""
        n = feats.shape[1]
        if n > nmax:
            gen = torch.Generator(device=feats.device).manual_seed(seed + 1)
            idx = torch.randint(0, n, (nmax,), device=feats.device, generator=gen)
            feats, target = feats[:, idx].contiguous(), target[idx].contiguous()
            n = nmax
        ws = torch.empty(3 * n, dtype=torch.float32, device=feats.device)
        m = self.c()
        check(load().c2p_mlp_calibrate_width(C.byref(m), n, _ptr(feats), _ptr(target), float(q),
                                             float(width_min), _ptr(ws), None),
              "c2p_mlp_calibrate_width")
        self.width_k = float(m.width_k)
        self.width_min = float(m.width_min)
        return self.width_k

    def forward(self, feats, stream=None):
        n = feats.shape[1]
        y = torch.empty((2, n), dtype=torch.float32, device=feats.device)
        mlp = self.c()
        check(load().c2p_mlp_forward(C.byref(mlp), n, _ptr(feats), _ptr(y), stream_ptr(stream)),
              "c2p_mlp_forward")
        return y

    def train_step(self, feats, target, lr=1e-3, apply=True, stream=None, want_grad=False):
        """one Adam step on a batch (feats [5][nb], target [nb], nb % 64 == 0)"""
        nb = feats.shape[1]
        nwg = nb // 64
        partial = torch.empty(nwg * NPARAM, dtype=torch.float32, device=feats.device)
        loss_part = torch.empty(nwg, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        grad = torch.empty(NPARAM, dtype=torch.float32, device=feats.device) if want_grad else None
        if apply:
            self.step += 1
        rc = load().c2p_mlp_train_step(_ptr(self.theta), _ptr(self.m), _ptr(self.v), _ptr(self.theta_h),
                                       _ptr(feats), _ptr(target), nb, float(lr),
                                       self.step if apply else 0, _ptr(partial), _ptr(loss_part),
                                       _ptr(loss), _ptr(grad) if grad is not None else None,
                                       stream_ptr(stream))
        check(rc, "c2p_mlp_train_step")
        return loss, grad


def c2p_batch_learned(u, bt, gam, params: MethodParams, net: LearnedC2P, want_mu=False,
                      want_nev=False, stats=False, stream=None, split=False, workspace=None):
    """c2p_batch with the learned bracket (same outputs as c2p_batch).
    Default: one fused kernel (network and root solve per wave).  split: the
    network runs as its own MFMA kernel writing the brackets into a workspace
    of 2n doubles, then the FP64 root kernel."""
    L = load()
    n = u.shape[1]
    dev = u.device
    w = torch.empty((5, n), dtype=torch.float64, device=dev)
    flags = torch.empty(n, dtype=torch.int16, device=dev)
    mu = torch.empty(n, dtype=torch.float64, device=dev) if want_mu else None
    nev = torch.empty(n, dtype=torch.int32, device=dev) if want_nev else None
    st = torch.zeros(4, dtype=torch.int64, device=dev) if stats else None
    mlp = net.c()
    if split:
        ws = workspace if workspace is not None else torch.empty(2 * n, dtype=torch.float64, device=dev)
        mlp.bracket_ws = _ptr(ws)
    rc = L.c2p_batch(n, _ptr_array(list(u)), _ptr_array(list(bt)), _ptr_array(list(gam)),
                     _ptr_array(list(w)), _ptr(flags), C.byref(params.c()), C.byref(mlp),
                     _ptr(st) if st is not None else None, _ptr(mu) if mu is not None else None,
                     _ptr(nev) if nev is not None else None, stream_ptr(stream))
    check(rc, "c2p_batch (learned)")
    out = {"w": w, "flags": flags}
    if mu is not None:
        out["mu"] = mu
    if nev is not None:
        out["nev"] = nev
    if st is not None:
        out["stats"] = st
    return out

"""Parity metric between the HIP path and the oracle (test helper).

Positive quantities (D~, tau~ where positive, rho, P): max pointwise |d|/|x|.
Signed quantities (S~_i, W v^i, B~): max |d| / max(|x|, 1e-3 max|x|).
"""
import numpy as np


def rel_positive(got, ref):
    ref = np.asarray(ref)
    got = np.asarray(got)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


def rel_signed(got, ref):
    ref = np.asarray(ref)
    got = np.asarray(got)
    floor = 1e-3 * max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), floor)))


def cons_errors(got, ref):
    """per-component errors of (D~, S~_x, S~_y, S~_z, tau~)"""
    return [rel_positive(got[0], ref[0])] + [rel_signed(got[c], ref[c]) for c in (1, 2, 3)] + \
        [rel_signed(got[4], ref[4])]


def prim_errors(got, ref):
    """per-component errors of (rho, W v^x, W v^y, W v^z, P)"""
    return [rel_positive(got[0], ref[0])] + [rel_signed(got[c], ref[c]) for c in (1, 2, 3)] + \
        [rel_positive(got[4], ref[4])]

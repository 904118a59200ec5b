"""The per-stage parity helper (tests/stage_parity.py) on the CPU, with the
oracle itself standing in for the device: it must find no difference, it must
catch a difference planted in one cell of the stand-in's output, and on the
star its decision-margin runs must find the atmosphere's near-threshold
trial floors without letting any value move."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2409_10384_amd import inputs
from tests import stage_parity as SP

STAR_P = O.Params(gamma=2.0, rho_atm=1.28e-13, T_atm=1.28e-11, f_thr=0.1, M_max=100.0, fofc=1,
                  dmp_M=1.1)


class Standin:
    """an oracle mesh behind the device-mesh calls the helper makes"""

    def __init__(self, om, plant=None):
        self.m = copy.deepcopy(om)
        self.plant = plant

    def stage_sets(self, src, dst, coef, dt=None):
        self.m.stage_sets(src, dst, dt, *coef)
        if self.plant is not None:
            ib, c, rel = self.plant
            U = self.m._set(dst)[0][ib]
            g = self.m.blocks[ib].ng
            U[c, g + 1, g + 2, g + 3] *= 1.0 + rel


def upload(gm, om):
    for k in range(3):
        for a, b in zip(gm.m._set(k), om._set(k)):
            for ib in range(len(om.blocks)):
                if isinstance(b[ib], list):
                    for d in range(3):
                        a[ib][d][...] = b[ib][d]
                else:
                    a[ib][...] = b[ib]


def download(gm, dst, ib):
    return SP._outputs(gm.m, dst, ib)


def _star():
    blocks, _ = inputs.star_blocks(n_per_side=2, nb=8)
    return O.Mesh(copy.deepcopy(blocks), STAR_P)


def test_helper_finds_no_difference_against_itself():
    om = _star()
    dt = om.dt(0.25)
    s = SP.stage_parity(Standin(om), om, O.Mesh.RK2, dt, upload=upload, download=download)
    for st in s:
        assert st["worst"]["faces"] == 0.0
        assert st["raw"] == {"U": 0.0, "w": 0.0, "faces": 0.0}
        # the oracle's own primitives against its re-inversion of its own
        # state: equal where no rule fired (the same function of the same
        # input); a floored cell's U against Eq. 7 of its w: equal up to the
        # rounding of that evaluation
        assert st["worst"]["w"] == 0.0 and st["worst"]["U"] < 1e-14
        assert st["flag_diff"] == 0
    # the atmosphere's trial states sit between (1 - 1e-10) and (1 - 1e-9) of
    # the tau floor: their FOFC decision is within the margin, their values
    # do not depend on it
    assert s[0]["near"] > 0
    assert s[0]["skipped"] == 0


def test_helper_catches_a_planted_difference():
    om = _star()
    dt = om.dt(0.25)
    with pytest.raises(AssertionError):
        SP.stage_parity(Standin(om, plant=(3, 0, 5e-12)), om, O.Mesh.RK2, dt, upload=upload,
                        download=download)


def test_term_scales_bound_the_values_and_expose_the_cancellation():
    """The magnitudes of the summed terms are at least the magnitude of the
    sum (triangle inequality), in every interior cell and face where no floor
    rebuilt the state; in the star at rest the density is not formed by
    cancellation (T within a few |D~|: the state and the Riemann flux's
    dissipation term of the face jumps) while the momentum is (T above 10 |S~| in a
    tenth of the star's cells, even on these coarse 8^3 blocks)."""
    om = _star()
    dt = om.dt(0.25)
    src, dst, (a0, a1, b) = O.Mesh.RK2[0]
    tu, tb = om.stage_sets(src, dst, dt, a0, a1, b, term_scales=True)
    ratio_D, ratio_S = [], []
    for ib, blk in enumerate(om.blocks):
        U = np.array(om.interior(om.u1[ib], ib))
        T = np.array(om.interior(tu[ib], ib))
        fl = np.array(om.interior(om.flags[ib], ib))
        free = (fl & O.F_FLOORS) == 0
        for c in range(5):
            assert np.all(T[c][free] >= np.abs(U[c][free]) * (1 - 1e-14)), (ib, c)
        star = free & (U[0] > 1e-6)
        if np.any(star):
            ratio_D.append(float(np.max(T[0][star] / U[0][star])))
            ratio_S.append(float(np.percentile(T[1][star] / np.maximum(np.abs(U[1][star]), 1e-300),
                                               90)))
        for d in range(3):
            f = om.b1[ib][d][SP._face_slices(blk, d)]
            t = tb[ib][d][SP._face_slices(blk, d)]
            assert np.all(t >= np.abs(f) * (1 - 1e-14)), (ib, d)
    assert max(ratio_D) < 4.0
    assert min(ratio_S) > 10.0

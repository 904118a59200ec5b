"""Balsara magnetized shock tubes (flat space, B along x plus transverse
components), the initial states of the paper's Table 1 (tests/golden/
balsara_table1.json): a tube of N x 1 x 1 cells on [0, 1], outflow in x,
periodic in y and z, discontinuity at x = 0.5 (test helper)."""
import json
import os

import numpy as np

import oracle as O
from paper_2409_10384_amd import inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = json.load(open(os.path.join(_HERE, "golden", "balsara_table1.json")))["tests"]


def tube(test, N, g=3):
    t = TABLE[str(test)]
    L, R = np.array(t["L"]), np.array(t["R"])
    sx, sy, sz = N + 2 * g, 1 + 2 * g, 1 + 2 * g
    x = (np.arange(sx) - g + 0.5) / N
    left = x < 0.5
    w = np.zeros((5, sz, sy, sx))
    st = np.where(left[None, :], L[:, None], R[:, None])          # (8, sx)
    rho, P, v = st[0], st[1], st[2:5]
    W = 1.0 / np.sqrt(1.0 - np.sum(v * v, axis=0))
    w[0] = rho[None, None, :]
    w[1] = (W * v[0])[None, None, :]
    w[2] = (W * v[1])[None, None, :]
    w[3] = (W * v[2])[None, None, :]
    w[4] = P[None, None, :]
    adm = np.zeros((16, sz, sy, sx))
    adm[0] = 1.0
    adm[4] = adm[7] = adm[9] = 1.0
    bx = np.full((sz, sy, sx + 1), L[5])                          # B^x is the same on both sides
    by = np.repeat(st[6][None, None, :], sy + 1, axis=1).repeat(sz, axis=0)
    bz = np.repeat(st[7][None, None, :], sy, axis=1).repeat(sz + 1, axis=0)
    nbr = []
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                nbr.append(-1 if ox != 0 else 0)
    h = 1.0 / N
    return inputs.BlockInit(N, 1, 1, g, (h, h, h), w, [bx, by, bz], adm, nbr, 1)


def params(test, recon=3, riemann=0):
    """the paper's tube method: PPM4 reconstruction, LLF, no FOFC; no
    magnetisation cap (the tubes never approach the atmosphere)"""
    return O.Params(gamma=TABLE[str(test)]["gamma"], rho_atm=1e-12, T_atm=1e-14, f_thr=1.0,
                    M_max=1e30, recon=recon, riemann=riemann, fofc=0)


def run_oracle(test, N, t_end, cfl=0.25, recon=3):
    m = O.Mesh([tube(test, N)], params(test, recon=recon))
    t, dts = 0.0, []
    while t < t_end - 1e-14:
        dt = min(m.dt(cfl), t_end - t)
        m.rk2_step(dt)
        dts.append(dt)
        t += dt
    return m, dts

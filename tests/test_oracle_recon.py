"""Pins of the oracle's reconstructions (Sec. III-B: donor cell, PLM with van
Leer's limiter, PPM4 = Colella & Woodward 1984, PPMX = Colella & Sekora 2008,
WENOZ = Borges et al. 2008) against exact polynomial data, mirror symmetry,
the limiters' defining properties and measured orders of accuracy."""
import math

import numpy as np
import pytest

import oracle as O

DC, PLM, WENOZ, PPM4, PPMX = 0, 1, 2, 3, 4
KINDS = (DC, PLM, WENOZ, PPM4, PPMX)


def cell_averages(F, x, h):
    """averages over [x - h/2, x + h/2] of the function whose antiderivative is F"""
    return (F(x + h / 2) - F(x - h / 2)) / h


def stencils(a):
    """periodic five-cell stencils around every cell of a"""
    return np.stack([np.roll(a, 2), np.roll(a, 1), a, np.roll(a, -1), np.roll(a, -2)], 1)


@pytest.mark.parametrize("kind", KINDS)
def test_constant_data_is_reproduced(kind):
    for c in (3.25, -1e-7, 1e5):
        lo, hi = O.recon_edges(kind, np.full((1, 5), c))
        assert abs(lo[0] - c) <= 4e-16 * abs(c) and abs(hi[0] - c) <= 4e-16 * abs(c)


@pytest.mark.parametrize("kind", (PLM, WENOZ, PPM4, PPMX))
def test_linear_data_is_exact(kind):
    """every limiter leaves a straight line alone: both edges are its point values"""
    rng = np.random.default_rng(70)
    for _ in range(50):
        c0, c1 = rng.normal(size=2)
        h = 10 ** rng.uniform(-3, 0)
        x = np.arange(-2, 3) * h
        lo, hi = O.recon_edges(kind, (c0 + c1 * x)[None])
        tol = 1e-13 * (abs(c0) + abs(c1) * h)
        assert abs(lo[0] - (c0 - c1 * h / 2)) < tol and abs(hi[0] - (c0 + c1 * h / 2)) < tol


@pytest.mark.parametrize("kind", (PPM4, PPMX))
def test_ppm_edges_exact_for_cubic_averages(kind):
    """The fourth-order interface value is exact for cell averages of a cubic;
    on monotone data with mild curvature no limiter acts, so both PPM edges
    are the cubic's point values."""
    rng = np.random.default_rng(71)
    for _ in range(50):
        c = rng.uniform(0.5, 1.0, size=4) * np.array([1.0, 1.0, 0.1, 0.02])
        P = lambda y: c[0] * y + c[1] * y ** 2 / 2 + c[2] * y ** 3 / 3 + c[3] * y ** 4 / 4
        p = lambda y: c[0] + c[1] * y + c[2] * y ** 2 + c[3] * y ** 3
        h = 0.05
        x0 = rng.uniform(0.0, 1.0)
        x = x0 + np.arange(-2, 3) * h
        lo, hi = O.recon_edges(kind, cell_averages(P, x, h)[None])
        assert abs(lo[0] - p(x0 - h / 2)) < 1e-13 and abs(hi[0] - p(x0 + h / 2)) < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_mirrored_stencil_swaps_the_edges(kind):
    """reversing the stencil must give the same two edges, swapped (an index or
    sign slip in any one-sided term breaks this)"""
    rng = np.random.default_rng(72)
    q = rng.normal(size=(4000, 5))
    q[:1000] = np.sort(q[:1000], axis=1)                 # monotone stencils too
    q[1000:1500, 3:] = q[1000:1500, 2:3] + 1.0           # one jump
    lo, hi = O.recon_edges(kind, q)
    lo_m, hi_m = O.recon_edges(kind, q[:, ::-1])
    np.testing.assert_array_equal(lo, hi_m)
    np.testing.assert_array_equal(hi, lo_m)


def test_plm_slope_is_the_harmonic_mean_and_total_variation_diminishing():
    rng = np.random.default_rng(73)
    q = rng.normal(size=(4000, 5))
    lo, hi = O.recon_edges(PLM, q)
    dl, dr = q[:, 2] - q[:, 1], q[:, 3] - q[:, 2]
    # the edges never leave the range of the cell and its neighbour on that side
    assert np.all((hi - q[:, 2]) * np.sign(dr) >= 0) and np.all(np.abs(hi - q[:, 2]) <= np.abs(dr) + 1e-15)
    assert np.all((q[:, 2] - lo) * np.sign(dl) >= 0) and np.all(np.abs(q[:, 2] - lo) <= np.abs(dl) + 1e-15)
    # harmonic mean where the differences agree in sign, flat elsewhere
    slope = hi - lo
    same = dl * dr > 0
    np.testing.assert_allclose(slope[same], (2 / (1 / dl + 1 / dr))[same], rtol=1e-12)
    assert np.all(slope[~same] == 0)


def _a6(lo, hi, a):
    return 6.0 * (a - 0.5 * (lo + hi))


def _monotone_parabola(lo, hi, a):
    """no interior extremum of the parabola with these edges and mean: |a6| <=
    |hi - lo|, up to the rounding of a6 (a few ulps of the values)"""
    slack = 32 * np.finfo(float).eps * np.maximum(np.abs(a), np.maximum(np.abs(lo), np.abs(hi)))
    return np.abs(_a6(lo, hi, a)) <= np.abs(hi - lo) + slack


def test_ppm4_flat_at_extrema_and_monotone_parabolas_elsewhere():
    rng = np.random.default_rng(74)
    q = rng.normal(size=(20000, 5))
    lo, hi = O.recon_edges(PPM4, q)
    a = q[:, 2]
    ext = (q[:, 3] - a) * (a - q[:, 1]) <= 0
    assert np.all(lo[ext] == a[ext]) and np.all(hi[ext] == a[ext])
    # elsewhere the parabola has no interior extremum and spans the cell value
    assert np.all(_monotone_parabola(lo, hi, a)[~ext])
    assert np.all(((hi - a) * (a - lo))[~ext] >= 0)
    # the interface values lie between the two cells they separate
    mono = np.all(np.diff(q, axis=1) > 0, axis=1)
    assert np.all(lo[mono] >= q[mono, 1] - 1e-15) and np.all(hi[mono] <= q[mono, 3] + 1e-15)


def test_ppmx_monotone_parabolas_where_the_data_are_monotone():
    rng = np.random.default_rng(75)
    q = np.sort(rng.normal(size=(20000, 5)), axis=1)
    q[::2] = q[::2, ::-1].copy()
    lo, hi = O.recon_edges(PPMX, q)
    a = q[:, 2]
    assert np.all(((hi - a) * (a - lo)) >= 0)
    assert np.all(_monotone_parabola(lo, hi, a))


@pytest.mark.parametrize("kind", (PLM, PPM4, PPMX))
def test_no_new_extrema_at_a_jump(kind):
    """a single discontinuity anywhere in the stencil: both edges stay inside
    the range of the cell and its two neighbours"""
    rng = np.random.default_rng(76)
    for pos in range(1, 5):
        q = np.repeat(rng.normal(size=(500, 1)), 5, axis=1)
        q[:, pos:] += rng.normal(size=(500, 1))
        lo, hi = O.recon_edges(kind, q)
        mn, mx = q[:, 1:4].min(1), q[:, 1:4].max(1)
        assert np.all(lo >= mn - 1e-14) and np.all(lo <= mx + 1e-14)
        assert np.all(hi >= mn - 1e-14) and np.all(hi <= mx + 1e-14)


def _edge_errors(kind, n):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    ph = 0.3
    a = cell_averages(lambda y: -np.cos(2 * np.pi * y + ph) / (2 * np.pi), x, h)
    lo, hi = O.recon_edges(kind, stencils(a))
    e = np.maximum(np.abs(lo - np.sin(2 * np.pi * (x - h / 2) + ph)),
                   np.abs(hi - np.sin(2 * np.pi * (x + h / 2) + ph)))
    return e.max(), e.mean()


@pytest.mark.parametrize("kind,max_order,l1_order", [
    (PLM, (1.9, 2.6), (1.9, 2.6)),
    (PPM4, (1.9, 2.6), (3.0, 4.0)),      # clipped to flat at the two extrema
    (PPMX, (3.8, 4.3), (3.8, 4.3)),      # keeps its accuracy there
    (WENOZ, (4.8, 5.2), (4.8, 5.2)),
])
def test_orders_of_accuracy_on_a_sine(kind, max_order, l1_order):
    """Edge errors on cell averages of a sine: second order for PLM; PPM4 is
    flattened at the two smooth extrema (second order in the maximum norm,
    higher in the mean); PPMX is fourth order everywhere; WENOZ fifth."""
    e = [_edge_errors(kind, n) for n in (64, 128, 256)]
    om = math.log2(e[1][0] / e[2][0])
    o1 = math.log2(e[1][1] / e[2][1])
    assert max_order[0] < om < max_order[1], (e, om)
    assert l1_order[0] < o1 < l1_order[1], (e, o1)


def test_ppmx_branch_jumps_at_an_exact_tie_and_ppm4_does_not():
    """A plateau of two exactly equal cells S between low values (a mirror-
    symmetric profile two cells wide, as at the rim of a star centred on a
    cell face).  PPMX's extremum test is the sign of (q[i+1] - q[i]) (q[i] -
    q[i-1]): at the tie the first plateau cell is an extremum and is kept flat;
    one ulp more in its right neighbour makes the data monotone, and the
    overshoot rule moves its lower edge to about 2/3 S.  PPM4's limited slopes
    are continuous there, so its edges move by rounding only."""
    low, S = 1.0e-13, 8.5e-6
    base = np.array([low, low, S, S, low])
    up = base.copy()
    up[3] = np.nextafter(S, 1.0)
    lo_tie = O.recon_edges(PPMX, base[None])[0][0]
    lo_up = O.recon_edges(PPMX, up[None])[0][0]
    assert lo_tie == S
    assert abs(lo_up - 2.0 / 3.0 * S) < 0.05 * S, lo_up
    lo4 = [O.recon_edges(PPM4, q[None])[0][0] for q in (base, up)]
    assert abs(lo4[0] - lo4[1]) <= 4 * np.spacing(S), lo4

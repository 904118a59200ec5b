"""GPU parity on the two-dimensional workloads of Sec. IV (SSP-RK3, WENOZ,
HLLE, FOFC as there): the advected magnetic loop (32^2, one period) and the
magnetized cylindrical blast wave (40^2 on [-6, 6]^2 to t = 1, B_x = 0.01,
0.1 and 1 with FOFC+DMP, and B_x = 1 with FOFC alone), each with the oracle's
dt sequence.  Each step compares rho, u^x, u^y, P and the face fields
relative to each field's maximum; the GPU blast waves' own mirror symmetry in
y is checked at the end, at every field strength (to 1e-12; it comes out
exact)."""
import numpy as np
import pytest

from tests import validation2d as V
from tests.test_gpu_parity import _meshes, host, say

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10384_amd import lib
    lib.load()
    return lib


def _run_pair(om, gm, N, t_end, cfl, bars, mirror_y=False, flags_may_split=False):
    """step both meshes with the oracle's dt; compare every step against
    bars(n) (None: no more elementwise comparison).  With flags_may_split, a
    step after which the two codes' flags differ (a FOFC or floor decision
    taken on a value within rounding of its threshold) also ends the
    elementwise comparison.  The GPU run is then checked for what holds on
    either branch: finite and positive (mass conservation is checked by the
    caller)."""
    g = om.blocks[0].ng

    def errors():
        torch.cuda.synchronize()
        wo = om.interior(om.w0[0], 0)[:, 0]
        wg = om.interior(host(gm.w0[0]), 0)[:, 0]
        pairs = [(wg[c], wo[c]) for c in (0, 1, 2, 4)]
        pairs += [(host(gm.b0[0][0])[g, g:g + N, g:g + N + 1], om.b0[0][0][g, g:g + N, g:g + N + 1]),
                  (host(gm.b0[0][1])[g, g:g + N + 1, g:g + N], om.b0[0][1][g, g:g + N + 1, g:g + N])]
        mx, l1 = [], []
        for a, r in pairs:
            scale = max(float(np.max(np.abs(r))), 1e-300)
            mx.append(float(np.max(np.abs(a - r))) / scale)
            l1.append(float(np.mean(np.abs(a - r))) / scale)
        return max(mx), max(l1)

    t, n, worst, split = 0.0, 0, 0.0, None
    while t < t_end - 1e-14:
        dt = min(om.dt(cfl), t_end - t)
        om.rk3_step(dt)
        gm.rk3_step(dt=dt)
        t += dt
        n += 1
        if split is not None:
            continue
        if flags_may_split:
            fo = om.interior(om.flags[0], 0)
            fg = om.interior(host(gm.flags[0]).astype(np.uint16), 0)
            if not np.array_equal(fo, fg):
                split = n
                say(f"  step {n}: flags differ in {int(np.count_nonzero(fo != fg))} cells; "
                    f"elementwise comparison ends (worst so far {worst:.1e})")
                continue
        bar = bars(n)
        if bar is None:
            if split is None:
                split = n
                say(f"  elementwise comparison ends after step {n - 1} (worst {worst:.1e})")
            continue
        mx, l1 = errors()
        worst = max(worst, mx)
        assert mx < bar, (n, mx, bar)
    if split is None:
        mx, l1 = errors()
        say(f"  {n} steps: final max / L1 difference {mx:.1e} / {l1:.1e}, worst over the run {worst:.1e}")
    wg = om.interior(host(gm.w0[0]), 0)[:, 0]
    assert np.all(np.isfinite(wg)) and np.all(wg[0] > 0) and np.all(wg[4] > 0)
    if mirror_y:
        for c, sy in ((0, 1), (1, 1), (2, -1), (4, 1)):
            a = wg[c]
            e = np.max(np.abs(a - sy * a[::-1, :])) / np.max(np.abs(a))
            say(f"  GPU y-mirror, field {c}: {e:.1e}")
            assert e <= 1e-12, c
    return split


def test_loop_advection_parity(G):
    say("loop advection: 32^2, RK3 + WENOZ + HLLE + FOFC, one period")
    N = 32
    om, gm = _meshes(G, [V.loop_block(N)], V.loop_params())
    _run_pair(om, gm, N, V.LOOP_PERIOD, 0.25, lambda n: 1e-12 if n <= 10 else 1e-9)


@pytest.mark.parametrize("bx,dmp", [(0.01, True), (0.1, True), (1.0, True), (1.0, False)])
def test_blast_wave_parity(G, bx, dmp):
    say(f"blast wave: 40^2, B_x = {bx}, {'FOFC+DMP' if dmp else 'FOFC'}, RK3, t = 1")
    N = 40
    om, gm = _meshes(G, [V.blast_block(N, bx)], V.blast_params(dmp))
    # B_x = 1 is the case whose inversions the paper calls ill-conditioned:
    # rounding-size differences grow about 2.4x per step there (1e-11 after
    # 10 steps), and by step 25 or so a FOFC decision at an intermediate
    # stage goes the other way in a cell.  So the strong-field runs are
    # compared elementwise over their first 15 steps, and to the end only in
    # what holds on either branch.
    strong = bx >= 1.0
    if strong:
        bars = lambda n: 1e-10 if n <= 10 else (1e-8 if n <= 15 else None)
    else:
        # the weak-field runs step through three shocks' compression: 1e-12
        # per stage compounds to a few 1e-12 of each field's maximum by step
        # 10 (the smooth 100-step bar is 1e-9)
        bars = lambda n: 1e-11 if n <= 10 else 1e-10
    D0 = float(om.interior(om.u0[0], 0)[0].sum())
    # the y mirror is exact in the oracle, and the GPU keeps it too at every
    # field strength: the Riemann flux combines the two sides without fused
    # products (a fused product would round one side's term and not the
    # other's, and at B_x = 1 that asymmetry grows ~2.4x per step)
    _run_pair(om, gm, N, 1.0, 0.1, bars, mirror_y=True, flags_may_split=strong)
    if dmp:
        D = float(om.interior(host(gm.u0[0]), 0)[0].sum())
        assert abs(D - D0) < 1e-13 * D0, (D, D0)

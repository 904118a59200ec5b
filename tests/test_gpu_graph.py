"""The whole SSP-RK2 step through the library: one call (grmhd_rk2_step),
its HIP-graph capture (grmhd_graph_build / grmhd_graph_launch) and the
library autotuner (grmhd_autotune), on the 2^3 x 16^3 star (same-level
exchange, outflow, atmosphere, FOFC+DMP) with the device dt.  The graph is
replayed several times with eager work and host synchronisations between the
replays; every replay is compared bit for bit with the same step launched
directly."""
import copy
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2409_10384_amd import inputs

pytestmark = [pytest.mark.gpu]

torch = pytest.importorskip("torch")

STAR_P = O.Params(gamma=2.0, rho_atm=1.28e-13, T_atm=1.28e-11, f_thr=0.1, M_max=100.0, fofc=1,
                  dmp_M=1.1)


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10384_amd import lib
    lib.load()
    return lib


def say(*a):
    print(*a, flush=True)


def _mesh(G, blocks):
    return G.DeviceMesh(copy.deepcopy(blocks), G.MethodParams(**dataclasses.asdict(STAR_P)))


def _state(m):
    torch.cuda.synchronize()
    return [torch.cat([m.u0[i].flatten(), m.w0[i].flatten()] + [f.flatten() for f in m.b0[i]]).cpu()
            for i in range(len(m.blocks))] + [m.dt_dev.cpu()]


def _equal(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_library_step_equals_the_binding_step(G):
    say("grmhd_rk2_step against the binding's stage-by-stage step: 2^3 x 16^3 star, 2 steps")
    blocks, _ = inputs.star_blocks(n_per_side=2, nb=16)
    a, b = _mesh(G, blocks), _mesh(G, blocks)
    for _ in range(2):
        a.rk2_step(cfl=0.25)
        b.rk2_step_lib(cfl=0.25)
    assert _equal(_state(a), _state(b))


def test_graph_replays_equal_direct_launches(G):
    say("graph replay against direct launches: 2^3 x 16^3 star, 4 replays")
    blocks, _ = inputs.star_blocks(n_per_side=2, nb=16)
    direct, graphed = _mesh(G, blocks), _mesh(G, blocks)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = graphed.rk2_graph(s, cfl=0.25)
    try:
        torch.cuda.synchronize()
        # capture launches nothing: the graphed mesh is still at its start
        assert _equal(_state(graphed)[:-1], _state(_mesh(G, blocks))[:-1])
        for k in range(4):
            direct.rk2_step_lib(cfl=0.25)
            g.launch(s)
            s.synchronize()
            # eager work between replays on the default stream
            junk = torch.ones(1 << 16, dtype=torch.float64, device="cuda").sum()
            torch.cuda.synchronize()
            assert _equal(_state(direct), _state(graphed)), k
            say(f"  replay {k + 1}: bitwise equal (dt {float(direct.dt_dev.item()):.6e})")
            del junk
    finally:
        g.close()


def test_library_autotuner(G):
    say("grmhd_autotune on the 2^3 x 16^3 star; the tuned step equals the default one")
    from paper_2409_10384_amd import autotune
    blocks, _ = inputs.star_blocks(n_per_side=2, nb=16)
    tuned, ref = _mesh(G, blocks), _mesh(G, blocks)
    dt = float(tuned.compute_dt(0.25).item())
    try:
        res = tuned.autotune(dt, reps=2)
        for fam, (best, ms) in res.items():
            say(f"  {fam}: " + ", ".join(f"{k}:{v:.3f}" for k, v in ms.items()) + f" -> {best}")
            assert best in (64, 128, 256, 512)
            if all(v == 0.0 for v in ms.values()):
                continue            # a family the stage does not launch on its own
            assert all(v > 0.0 for v in ms.values())
            assert ms[best] == min(ms.values())
        tuned.rk2_step(dt=dt)
    finally:
        autotune.reset()
    ref.rk2_step(dt=dt)
    assert _equal(_state(tuned)[:-1], _state(ref)[:-1])


def test_dt_reduced_in_the_stage_equals_grmhd_dt(G):
    """grmhd_stage_cfl: the CFL dt reduced inside the stage's field kernel is
    grmhd_dt's, bit for bit, and the step it drives equals the step driven by
    grmhd_dt followed by plain stages"""
    say("dt reduced in the first stage against grmhd_dt: 2^3 x 16^3 star, 2 steps")
    blocks, _ = inputs.star_blocks(n_per_side=2, nb=16)
    fused, plain = _mesh(G, blocks), _mesh(G, blocks)
    plain.fused_dt = False
    for k in range(2):
        ref = float(plain.compute_dt(0.25).item())
        fused.rk2_step(cfl=0.25)
        plain.rk2_step(cfl=0.25)
        got = float(fused.dt_dev.item())
        say(f"  step {k + 1}: dt {got!r} (grmhd_dt {ref!r})")
        assert got == ref
        assert _equal(_state(fused), _state(plain))

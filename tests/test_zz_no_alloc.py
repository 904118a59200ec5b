"""The allocation-free mass sum (grmhd_mass_noalloc) against grmhd_mass
through the C ABI: bit for bit, on two calls in a row, the second over a
smaller block table (the fixed device array keeps the first call's partial
sums, which the second must not read)."""
import copy

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


def _mesh(G, blocks):
    import dataclasses
    return G.DeviceMesh(copy.deepcopy(blocks), G.MethodParams(**dataclasses.asdict(STAR_P)))


def test_mass_noalloc_matches_mass(G):
    print("no-alloc mass: star as 27 blocks of 8^3, then as 8 blocks of 8^3", flush=True)
    blocks, _ = inputs.star_blocks(n_per_side=3, nb=8)
    big = _mesh(G, blocks)
    big.rk2_step(cfl=0.25)
    blocks_s, _ = inputs.star_blocks(n_per_side=2, nb=8)
    small = _mesh(G, blocks_s)
    small.rk2_step(cfl=0.25)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for mesh, n, bl in ((big, 27, blocks), (small, 8, blocks_s)):
        ref = float(mesh.mass().item())
        got = float(mesh.mass_noalloc(out).item())
        print(f"  {n} blocks: grmhd_mass {ref!r}, grmhd_mass_noalloc {got!r}", flush=True)
        assert got == ref
        # and against a host sum of the same interiors (another summation order)
        D = sum(float(np.sum(mesh.interior(mesh.u0[ib], ib)[0].cpu().numpy()))
                * float(np.prod(bl[ib].dx)) for ib in range(n))
        assert abs(got - D) <= 1e-13 * abs(D)
    assert G.load().grmhd_mass_noalloc_max_blocks() == 65536

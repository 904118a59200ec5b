"""GPU parity of the ADM matter sources and of the lapse excision against the
oracle, through the C ABI."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2409_10384_amd import inputs
from tests import parity as PM
from tests.test_gpu_parity import STAR_P, _compare_state, _meshes, host, say
from tests.test_oracle_matter import _dipped_block

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10384_amd import lib
    lib.load()
    return lib


def _oracle_matter(w, bf, adm, g, params):
    """oracle sources at the interior cells of one block's state (w, faces)"""
    sl = (slice(None), slice(g, -g), slice(g, -g), slice(g, -g))
    wi = w[sl]
    bt = O.cell_bt(bf)[sl].reshape(3, -1)
    gam = adm[4:10][sl].reshape(6, -1)
    return O.matter_sources(wi.reshape(5, -1), bt, gam, params).reshape((10,) + wi.shape[1:]), sl


@pytest.mark.parametrize("case", ["smooth", "star_hybrid"])
def test_matter_sources_parity(G, case):
    """E, S_i, S_ij at every interior cell, after one RK2 step (so the state
    and field are the evolved ones), against the oracle's pointwise sources
    of the GPU's own state (the kernel's arithmetic: 1e-12 on the scale of
    rel_signed, as the stress terms cancel in places) and of the oracle's
    state (the whole path, to the stage tolerance)"""
    if case == "smooth":
        say("matter sources: smooth periodic block 24^3")
        blocks = [inputs.smooth_periodic_block(n=24, seed_offset=50)]
        p = O.Params(gamma=5.0 / 3.0)
    else:
        say("matter sources: star 2^3 x 16^3, piecewise polytrope")
        pp, K = inputs.pp_eos()
        st = inputs.calibrate_field(inputs.StarSetup(pp=pp, pp_K=K))
        blocks, _ = inputs.star_blocks(n_per_side=2, nb=16, st=st)
        import dataclasses
        p = dataclasses.replace(STAR_P, **pp)
    om, gm = _meshes(G, blocks, p)
    dt = om.dt(0.25)
    om.rk2_step(dt)
    gm.rk2_step(dt=dt)
    got = gm.matter_sources(0)
    torch.cuda.synchronize()
    worst = 0.0
    for ib in range(len(blocks)):
        g = blocks[ib].ng
        own, sl = _oracle_matter(host(gm.w0[ib]), [host(x) for x in gm.b0[ib]], om.adm[ib], g, p)
        path, _ = _oracle_matter(om.w0[ib], om.b0[ib], om.adm[ib], g, p)
        gg = host(got[ib])[sl].reshape(own.shape)
        for n in range(10):
            e = PM.rel_signed(gg[n], own[n])
            worst = max(worst, e)
            assert e < 1e-12, (ib, n, e)
            assert PM.rel_signed(gg[n], path[n]) < 1e-11, (ib, n)
        # ghost cells stay untouched (zero)
        gh = host(got[ib]).copy()
        gh[sl] = 0.0
        assert not np.any(gh)
    say(f"  worst component error {worst:.2e}")


def test_excision_parity(G):
    """a lapse dip below 0.2: three RK3 steps with excision after every stage,
    against the oracle; the excised cells and their flags agree exactly"""
    say("excision: smooth block 12^3 with a lapse dip, 3 RK3 steps")
    blk = _dipped_block()
    p = O.Params(gamma=5.0 / 3.0, rho_atm=1e-8, T_atm=1e-6)
    om, gm = _meshes(G, [blk], p)
    om.alpha_excise = 0.2
    gm.alpha_excise = 0.2
    for _ in range(3):
        dt = om.dt(0.2)
        om.rk3_step(dt)
        gm.rk3_step(dt=dt)
    torch.cuda.synchronize()
    fl = om.interior(host(gm.flags[0]).astype(np.uint16), 0)
    fr = om.interior(om.flags[0], 0)
    assert np.any(fr & O.F_EXCISED)
    np.testing.assert_array_equal(fl & O.F_EXCISED, fr & O.F_EXCISED)
    _compare_state(om, gm, 0, 1e-11, "excised RK3")

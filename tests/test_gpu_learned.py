"""GPU tests of the learned C2P guess: MFMA forward and backward against the
FP64 oracle on the same bf16-rounded weights and inputs, training on the GPU,
and the trained network's gain over the plain bracketed solve at an equal
final error with no unrecovered failures."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from paper_2409_10384_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]
torch = pytest.importorskip("torch")

OFFS = [(0, 64, 5), (384, 64, 64), (4544, 64, 64), (8704, 2, 64)]
BOFFS = [320, 4480, 8640, 8832]


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10384_amd import lib
    lib.load()
    return lib


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16(x):
    a = np.asarray(x, dtype=np.float32).astype(np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(theta, round_w=True):
    ps = []
    for (off, o, i), bo in zip(OFFS, BOFFS):
        W = theta[off:off + o * i].reshape(o, i).astype(np.float64)
        ps.append([bf16(W) if round_w else W, theta[bo:bo + o].astype(np.float64)])
    return ps


def flat_grads(grads):
    out = np.zeros(8834)
    for (off, o, i), bo, (dW, db) in zip(OFFS, BOFFS, grads):
        out[off:off + o * i] = dW.ravel()
        out[bo:bo + o] = db
    return out


def cosine(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_mfma_forward_matches_oracle(G):
    say("learned: MFMA forward vs FP64 oracle on bf16-rounded operands")
    net = G.LearnedC2P(seed=3)
    # non-zero biases
    net.theta[320:384] = torch.linspace(-0.5, 0.5, 64, device=net.theta.device)
    net.theta[8832:8834] = torch.tensor([0.3, -0.2], device=net.theta.device)
    net.refresh_bf16()
    rng = np.random.default_rng(7)
    n = 4096 + 37                              # several tiles and a ragged tail
    x = rng.normal(size=(5, n)).astype(np.float32)
    y = net.forward(torch.as_tensor(x).cuda()).cpu().numpy()
    ps = unflatten(net.theta.cpu().numpy())
    yref, _ = M.forward(ps, bf16(x.T))
    for c in range(2):
        assert cosine(y[c], yref[:, c]) > 0.9999
        rel = np.linalg.norm(y[c] - yref[:, c]) / np.linalg.norm(yref[:, c])
        assert rel < 2e-2, rel


def test_mfma_gradients_match_oracle(G):
    say("learned: MFMA backward vs FP64 oracle")
    net = G.LearnedC2P(seed=4)
    rng = np.random.default_rng(8)
    nb = 1024
    x = rng.normal(size=(5, nb)).astype(np.float32)
    t = rng.normal(size=nb).astype(np.float32)
    _, grad = net.train_step(torch.as_tensor(x).cuda(), torch.as_tensor(t).cuda(), apply=False,
                             want_grad=True)
    g = grad.cpu().numpy().astype(np.float64)
    ps = unflatten(net.theta.cpu().numpy())
    y, cache = M.forward(ps, bf16(x.T))
    _, dy = M.loss_and_grad_out(y, t.astype(np.float64))
    gref = flat_grads(M.backward(ps, cache, dy))
    for (off, o, i), bo in zip(OFFS, BOFFS):
        for a, b in ((g[off:off + o * i], gref[off:off + o * i]), (g[bo:bo + o], gref[bo:bo + o])):
            c = cosine(a, b)
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            say(f"  tensor at {off}: cosine {c:.6f} rel {rel:.2e}")
            assert c > 0.999 and rel < 2e-2, (off, c, rel)
    # determinism: the same step twice gives bitwise the same gradient
    _, grad2 = net.train_step(torch.as_tensor(x).cuda(), torch.as_tensor(t).cuda(), apply=False,
                              want_grad=True)
    assert torch.equal(grad, grad2)


def test_adam_steps_match_oracle(G):
    """two training steps on the GPU (c2p_mlp_train_step with step >= 1) move
    the fp32 parameters and moments as the FP64 Adam of the oracle does with
    the same two gradients (learning rate 2e-3, bias correction of steps 1
    and 2)"""
    say("learned: two GPU Adam steps vs the oracle's Adam")
    net = G.LearnedC2P(seed=5)
    rng = np.random.default_rng(9)
    theta0 = net.theta.cpu().numpy().astype(np.float64)
    lr = 2e-3
    grads = []
    for step in range(2):
        x = rng.normal(size=(5, 512)).astype(np.float32)
        t = rng.normal(size=512).astype(np.float32)
        _, g = net.train_step(torch.as_tensor(x).cuda(), torch.as_tensor(t).cuda(), lr=lr,
                              want_grad=True)
        grads.append(g.cpu().numpy().astype(np.float64))
    assert net.step == 2
    ps = [[theta0.copy()]]
    opt = M.Adam([[theta0.copy(), np.zeros(1)]], lr=lr)
    params = [[theta0.copy(), np.zeros(1)]]
    for g in grads:
        opt.step(params, [[g, np.zeros(1)]])
    del ps
    th = net.theta.cpu().numpy().astype(np.float64)
    m = net.m.cpu().numpy().astype(np.float64)
    v = net.v.cpu().numpy().astype(np.float64)
    upd, upd_ref = th - theta0, params[0][0] - theta0
    live = np.abs(grads[0]) + np.abs(grads[1]) > 1e-20     # both moments resolved in fp32
    e_upd = float(np.max(np.abs(upd - upd_ref)[live]))
    say(f"  max |update - oracle update| {e_upd:.2e} (lr {lr}), {int(live.sum())} live parameters")
    assert int(live.sum()) > 8000
    assert e_upd <= 1e-4 * lr
    assert np.max(np.abs(upd_ref[live])) > 0.5 * lr          # the steps are not trivially small
    # first moments: 0.09 g1 + 0.1 g2 cancels where the two gradients have
    # opposite signs, so the fp32 moment (its coefficients 0.9f and 1 - 0.9f
    # are 3e-8 and 2.4e-7 off 0.9 and 0.1, each product and sum rounded to
    # 6e-8) is judged against the size of its terms; the second moments are
    # sums of positive terms and keep the relative bar
    terms = 0.09 * np.abs(grads[0]) + 0.1 * np.abs(grads[1])
    e_m = np.abs(m - opt.m[0][0])[live] / (terms[live] + 1e-30)
    say(f"  max |m - oracle m| / (0.09|g1| + 0.1|g2|) {np.max(e_m):.2e}")
    assert np.max(e_m) <= 1e-6
    np.testing.assert_allclose(v[live], opt.v[0][0][live], rtol=1e-5, atol=1e-20)
    # the bf16 copy follows the updated fp32 parameters
    tb = net.theta_h.cpu().numpy().astype(np.int16).view(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(tb.view(np.float32).astype(np.float64), bf16(th))


C4P = dict(gamma=5.0 / 3.0, rho_atm=1e-20, T_atm=1e-30, f_thr=1.0, M_max=1e30, c2p_tol=1e-12)


def _c4_device(G, n, seed):
    st = inputs.c2p_states(n, seed_offset=seed)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    w, bt, gam = d(st["w"]), d(st["bt"]), d(st["gam"])
    u = G.prim2con(w, bt, gam, G.MethodParams(**C4P))
    return st, w, bt, gam, u


def train_network(G, n_train=1 << 18, steps=1500, batch=4096, seed=0):
    p = G.MethodParams(**C4P)
    st, w, bt, gam, u = _c4_device(G, n_train, 300)
    net = G.LearnedC2P(seed=seed)
    raw, _ = net.features(u, bt, gam, p, standardise=False)
    net.fit_standardisation(raw)
    feats, target = net.features(u, bt, gam, p, w_true=w)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n_train, (batch,), device="cuda", generator=gen)
        lr = 2e-3 if it < steps * 0.7 else 5e-4
        loss, _ = net.train_step(feats[:, idx].contiguous(), target[idx].contiguous(), lr=lr)
        if it % 100 == 0 or it == steps - 1:
            losses.append(float(loss.item()))
    return net, losses


def test_learned_c2p_needs_fewer_evaluations_at_equal_error(G):
    say("learned: train on prim->cons pairs, compare with the plain solve")
    net, losses = train_network(G)
    say(f"  loss trace {['%.3g' % x for x in losses]}")
    assert losses[-1] < 0.5 * losses[0]
    p = G.MethodParams(**C4P)
    st, w, bt, gam, u = _c4_device(G, 1 << 16, 301)
    plain = G.c2p_batch(u.clone(), bt, gam, p, want_mu=True, want_nev=True, stats=True)
    learned = G.c2p_batch_learned(u.clone(), bt, gam, p, net, want_mu=True, want_nev=True, stats=True)
    eps = st["w"][4] / (2.0 / 3.0 * st["w"][0])
    mus = 1.0 / ((1 + eps + st["w"][4] / st["w"][0]) * st["W"])
    mu_p = plain["mu"].cpu().numpy()
    mu_l = learned["mu"].cpu().numpy()
    assert np.max(np.abs(mu_p - mus) / mus) < 1e-10
    assert np.max(np.abs(mu_l - mus) / mus) < 1e-10
    fl = learned["flags"].cpu().numpy().astype(np.uint16)
    assert not np.any(fl & O.F_C2P_FAIL)
    n_p = plain["nev"].double().mean().item()
    n_l = learned["nev"].double().mean().item()
    fb = float(np.mean((fl & O.F_BRACKET_FALLBACK) != 0))
    say(f"  mean master evaluations plain {n_p:.2f} learned {n_l:.2f}; fallback rate {fb:.4f}")
    assert n_l < n_p
    st_l = learned["stats"].cpu().numpy()
    assert st_l[0] == u.shape[1] and st_l[3] == 0
    # the split path (bracket kernel, then the plain kernel reading it) agrees
    split = G.c2p_batch_learned(u.clone(), bt, gam, p, net, want_mu=True, stats=True, split=True)
    assert np.max(np.abs(split["mu"].cpu().numpy() - mus) / mus) < 1e-10
    assert int(split["stats"][3].item()) == 0


def test_features_match_the_oracle_definition(G):
    """fp32 features of the GPU against the oracle's FP64 definition on the
    invariants of the same conserved states (no floor rule fires here)."""
    say("learned: features of 65536 states against the oracle definition")
    p = G.MethodParams(**C4P)
    st, w, bt, gam, u = _c4_device(G, 1 << 16, 302)
    net = G.LearnedC2P(seed=0)
    raw, _ = net.features(u, bt, gam, p, standardise=False)
    raw = raw.double().cpu().numpy()
    U = u.cpu().numpy()
    g = st["gam"]
    Gm = np.array([[g[0], g[1], g[2]], [g[1], g[3], g[4]], [g[2], g[4], g[5]]]).transpose(2, 0, 1)
    sg = np.sqrt(np.linalg.det(Gm))
    D = U[0] / sg
    r = (U[1:4] / sg / D).T
    B = st["bt"] / sg
    r2 = np.einsum("ni,nij,nj->n", r, np.linalg.inv(Gm), r)
    b2 = np.einsum("in,nij,jn->n", B, Gm, B) / D
    s = np.einsum("ni,in->n", r, B) / np.sqrt(D)
    q = U[4] / sg / D
    ref = M.features(D, q, r2, b2, s).T
    for c in range(5):
        err = np.max(np.abs(raw[c] - ref[c]) / np.maximum(np.abs(ref[c]), 1e-3))
        say(f"  feature {c}: max rel err {err:.2e}")
        assert err < 1e-5, (c, err)


STAR = dict(gamma=2.0, rho_atm=1.28e-13, T_atm=1.28e-11, f_thr=0.1, M_max=100.0, fofc=1, dmp_M=1.1)


def test_learned_stage_matches_plain_stage(G):
    """Two RK2 steps of the star (2^3 blocks of 16^3, FOFC+DMP) with the
    learned bracket in the stage inversion against the plain stage: the same
    decisions, the same state to the root-solve tolerance, no failures."""
    import copy
    say("learned stage: star 2^3 x 16^3, network trained on the mesh's own states")
    blocks, _ = inputs.star_blocks(n_per_side=2, nb=16)
    mp = G.MethodParams(**STAR)
    gp = G.DeviceMesh(copy.deepcopy(blocks), mp)
    gl = G.DeviceMesh(copy.deepcopy(blocks), mp)
    net = G.LearnedC2P(seed=0)
    u, bt, gam, w = gp.c2p_pairs(0)
    net.fit(u, bt, gam, mp, w, steps=2000)
    dt = float(gp.compute_dt(0.25).item())
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    stats_p = torch.zeros(4, dtype=torch.int64, device="cuda")
    for _ in range(2):
        gp.rk2_step(dt=dt, stats=stats_p)
        gl.rk2_step(dt=dt, mlp=net, stats=stats)
    torch.cuda.synchronize()
    n_s, n_ev, n_fb, n_fail = [int(x) for x in stats.cpu()]
    p_s, p_ev, p_fb, p_fail = [int(x) for x in stats_p.cpu()]
    say(f"  learned: solves {n_s}, evaluations/solve {n_ev / max(n_s, 1):.2f}, fallbacks {n_fb}, "
        f"failures {n_fail}; plain: evaluations/solve {p_ev / max(p_s, 1):.2f}")
    assert n_s == p_s == 4 * sum(b.nx * b.ny * b.nz for b in blocks)
    assert n_fail == 0 and p_fail == 0 and p_fb == 0
    for ib in range(len(blocks)):
        fp = gp.interior(gp.flags[ib], ib).cpu().numpy().astype(np.uint16)
        fl = gl.interior(gl.flags[ib], ib).cpu().numpy().astype(np.uint16)
        bad = (fp & ~np.uint16(O.F_BRACKET_FALLBACK)) != (fl & ~np.uint16(O.F_BRACKET_FALLBACK))
        assert np.mean(bad) < 0.01
        dil = bad.copy()
        for ax in range(3):
            dil = dil | np.roll(dil, 1, axis=ax) | np.roll(dil, -1, axis=ax)
        rho = gp.interior(gp.w0[ib], ib)[0].cpu().numpy()
        ok = ~dil & (rho > 1e-8)         # the star (atmosphere velocities are ill-conditioned)
        for name, a, b in (("U", gl.u0[ib], gp.u0[ib]), ("w", gl.w0[ib], gp.w0[ib])):
            ga = gl.interior(a, ib).cpu().numpy()
            pa = gp.interior(b, ib).cpu().numpy()
            assert np.all(np.isfinite(ga))
            for c in range(5):
                scale = np.max(np.abs(pa[c][ok])) if ok.any() else 1.0
                e = np.max(np.abs(ga[c][ok] - pa[c][ok])) / max(scale, 1e-300) if ok.any() else 0.0
                assert e < 1e-10, (ib, name, c, e)
    say("  learned and plain stages agree on the star")


@pytest.mark.parametrize("n", [1, 15, 17, 63, 65, 1000])
def test_learned_c2p_on_ragged_lengths(G, n):
    """lengths that leave the network's 16-state tiles and the 64-state waves
    partly filled: the fused and the split learned paths return the exact
    label's mu (1e-10, as the plain solve) with no unrecovered failure, and
    the flags other than the bracket-fallback bit equal the plain solve's"""
    say(f"learned C2P on {n} states (ragged tile and wave)")
    net = _trained(G)
    p = G.MethodParams(**C4P)
    st, w, bt, gam, u = _c4_device(G, n, 310 + n)
    eps = st["w"][4] / (2.0 / 3.0 * st["w"][0])
    mus = 1.0 / ((1 + eps + st["w"][4] / st["w"][0]) * st["W"])
    plain = G.c2p_batch(u.clone(), bt, gam, p, want_mu=True)
    fp = plain["flags"].cpu().numpy().astype(np.uint16)
    for split in (False, True):
        out = G.c2p_batch_learned(u.clone(), bt, gam, p, net, want_mu=True, stats=True, split=split)
        mu = out["mu"].cpu().numpy()
        assert mu.shape == (n,)
        assert np.max(np.abs(mu - mus) / mus) < 1e-10, split
        fl = out["flags"].cpu().numpy().astype(np.uint16)
        assert not np.any(fl & O.F_C2P_FAIL)
        np.testing.assert_array_equal(fl & ~np.uint16(O.F_BRACKET_FALLBACK), fp)
        stl = out["stats"].cpu().numpy()
        assert stl[0] == n and stl[3] == 0


def test_c2p_on_zero_states(G):
    """an empty batch is a valid call: nothing launched, nothing returned"""
    net = _trained(G)
    p = G.MethodParams(**C4P)
    e = lambda k: torch.empty((k, 0), dtype=torch.float64, device="cuda")
    for out in (G.c2p_batch(e(5), e(3), e(6), p, want_mu=True),
                G.c2p_batch_learned(e(5), e(3), e(6), p, net, want_mu=True),
                G.c2p_batch_learned(e(5), e(3), e(6), p, net, want_mu=True, split=True)):
        torch.cuda.synchronize()
        assert out["w"].shape == (5, 0) and out["mu"].shape == (0,)


_NET = {}


def _trained(G):
    """one trained network for the tests that only use it (trained once)"""
    if "net" not in _NET:
        _NET["net"], _ = train_network(G, steps=600)
    return _NET["net"]


def test_c2p_full_size_sampled_parity(G):
    """the learned-inversion workload at its full size: 2^24 states (the
    benchmark's states), plain and learned (fused) inversions over all of
    them in one launch each; a seeded sample of 65536 states against the
    oracle's inversion of the same states: the plain solve's flags equal and
    mu to 2e-12, the learned solve's flags equal but for the bracket-fallback
    bit and its mu to 2e-12 of the oracle's, no unrecovered failure"""
    n = 1 << 24
    say(f"C2P at full size: {n} states, plain and learned; 65536 sampled against the oracle")
    net = _trained(G)
    p = G.MethodParams(**C4P)
    s = inputs.c2p_states_torch(n, seed_offset=3, device="cuda")
    u = G.prim2con(s["w"], s["bt"], s["gam"], p)
    plain = G.c2p_batch(u.clone(), s["bt"], s["gam"], p, want_mu=True)
    learned = G.c2p_batch_learned(u.clone(), s["bt"], s["gam"], p, net, want_mu=True, stats=True)
    torch.cuda.synchronize()
    idx = torch.as_tensor(np.sort(np.random.default_rng(777).choice(n, size=1 << 16, replace=False)),
                          device="cuda")
    h = lambda t: np.ascontiguousarray(t[:, idx].cpu().numpy())
    po = O.Params(**C4P)
    _, wref, fref, nref, muref = O.c2p(h(u), h(s["bt"]), h(s["gam"]), po)
    fp = plain["flags"][idx].cpu().numpy().astype(np.uint16)
    fl = learned["flags"][idx].cpu().numpy().astype(np.uint16)
    mp = plain["mu"][idx].cpu().numpy()
    ml = learned["mu"][idx].cpu().numpy()
    np.testing.assert_array_equal(fp, fref)
    np.testing.assert_array_equal(fl & ~np.uint16(O.F_BRACKET_FALLBACK), fref)
    ep = np.max(np.abs(mp - muref) / muref)
    el = np.max(np.abs(ml - muref) / muref)
    say(f"  sampled mu against the oracle: plain {ep:.1e}, learned {el:.1e}")
    assert ep < 2e-12 and el < 2e-12
    assert int(learned["stats"][3].item()) == 0

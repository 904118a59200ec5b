"""Pins of the FP64 MLP oracle: backward against central finite differences,
the hard-swish activation and its derivative, Adam's bias-corrected first step, and the
bracket map."""
import numpy as np

from oracle import mlp as M


def test_hard_swish_and_its_derivative():
    """z clamp(z/6 + 1/2, 0, 1): 0 below -3, the identity above 3, the
    parabola z (z + 3) / 6 between; the derivative against central
    differences away from the two kinks"""
    z = np.linspace(-8, 8, 1601)
    z = z[(np.abs(z - 3) > 1e-3) & (np.abs(z + 3) > 1e-3)]
    h = 1e-6
    fd = (M.act(z + h) - M.act(z - h)) / (2 * h)
    np.testing.assert_allclose(M.dact(z), fd, rtol=1e-8, atol=1e-9)
    assert M.act(0.0) == 0.0 and M.act(3.0) == 3.0 and M.act(-3.0) == 0.0
    mid = z[np.abs(z) < 3]
    np.testing.assert_allclose(M.act(mid), mid * (mid + 3.0) / 6.0, rtol=1e-15, atol=1e-16)
    np.testing.assert_array_equal(M.act(z[z > 3]), z[z > 3])
    np.testing.assert_array_equal(M.act(z[z < -3]), 0.0 * z[z < -3])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = M.init_params(1)
    x = rng.normal(size=(7, 5))
    t = rng.normal(size=7)

    def loss_at(ps):
        y, _ = M.forward(ps, x)
        # fix the second target at the unperturbed first output (no gradient),
        # and the second output's input at the unperturbed last hidden layer
        # (its gradient stops at the read-out)
        e0 = y[:, 0] - t
        t1 = np.log(np.abs(y0_fixed - t) + M.LOG_ERR_C)
        y1 = h3_fixed @ ps[3][0][1] + ps[3][1][1]
        return 0.5 * np.mean(e0 * e0 + (y1 - t1) ** 2)

    y, cache = M.forward(params, x)
    y0_fixed = y[:, 0].copy()
    h3_fixed = cache[0][3].copy()
    loss, dy = M.loss_and_grad_out(y, t)
    assert abs(loss - loss_at(params)) < 1e-14
    grads = M.backward(params, cache, dy)
    h = 1e-6
    for li in range(4):
        for k in range(2):
            arr = params[li][k]
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + h
                lp = loss_at(params)
                arr[idx] = old - h
                lm = loss_at(params)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                g = grads[li][k][idx]
                assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (li, k, idx, g, fd)


def test_adam_first_step_is_sign_times_lr():
    params = [[np.array([[1.0, -2.0]]), np.array([0.5])]]
    grads = [[np.array([[0.3, -0.01]]), np.array([2.0])]]
    opt = M.Adam(params, lr=0.1, eps=0.0)
    opt.step(params, grads)
    np.testing.assert_allclose(params[0][0], [[0.9, -1.9]], rtol=1e-15)
    np.testing.assert_allclose(params[0][1], [0.4], rtol=1e-15)


def test_bracket_contains_guess_and_is_ordered():
    y = np.array([[0.0, -3.0], [-2.0, 0.0], [3.0, -8.0]])
    lo, hi = M.bracket(y)
    mid = 1 / (1 + np.exp(-y[:, 0]))
    assert np.all(lo < mid) and np.all(mid < hi) and np.all(lo > 0) and np.all(hi < 1)


def test_training_reduces_loss_on_a_smooth_map():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(512, 5))
    t = np.tanh(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    params = M.init_params(2)
    opt = M.Adam(params, lr=3e-3)
    first = None
    for it in range(300):
        y, cache = M.forward(params, x)
        loss, dy = M.loss_and_grad_out(y, t)
        mse = 0.5 * np.mean((y[:, 0] - t) ** 2)
        first = mse if first is None else first
        opt.step(params, M.backward(params, cache, dy))
    assert mse < 0.1 * first, (mse, first)

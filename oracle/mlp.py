"""FP64 oracle of the learned C2P guess network (not in the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A 5-64-64-64-2 multilayer perceptron with hard-swish activations maps five
invariants of a conserved state to an initial guess and a bracket half-width
for the root mu = 1/(hW) of the Kastaun master function.  The root solve
itself is unchanged and always finishes, so the network only decides where
the bracketed FP64 solve starts.

Features of a state (D, q = tau/D, r^2 = S_i S^i / D^2, b^2 = B^2/D,
s = r_i B^i / sqrt(D)) -- all invariant under changes of spatial basis:
    x0 = log10 D
    x1 = log10(1 + q)
    x2 = sqrt(r^2) / (1 + q)
    x3 = b^2 / (1 + q)
    x4 = s^2 / (r^2 b^2 + 1e-300)          (cos^2 of the angle between r and B)
then standardised: (x - mean) * scale.

Outputs: y0 = logit(mu) estimate; y1 = log of the expected absolute logit
error.  Bracket in logit space: y0 -/+ (k exp(y1) + delta_min), mapped back
with the logistic function.

Loss per sample: 0.5 (y0 - t)^2 + 0.5 (y1 - log(|y0 - t| + c))^2 with
t = logit(mu*), the second target using y0 without gradient; averaged over
the batch.  The second output is a linear read-out of the last hidden layer:
its loss trains only that read-out (W4[1], b4[1]), so the noisy error-scale
target does not pull the shared hidden layers away from the guess.
"""
import numpy as np

SIZES = [(64, 5), (64, 64), (64, 64), (2, 64)]
LOG_ERR_C = 1e-4


def act(z):
    """hard-swish (Howard et al. 2019): z clamp(z / 6 + 1/2, 0, 1)"""
    return z * np.clip(z / 6.0 + 0.5, 0.0, 1.0)


def dact(z):
    """its derivative: 0 below -3, 1 above 3, z / 3 + 1/2 between"""
    return np.where(z <= -3.0, 0.0, np.where(z >= 3.0, 1.0, z / 3.0 + 0.5))


def features(D, q, r2, b2, s):
    """raw invariants (n,) arrays -> (n, 5)"""
    x0 = np.log10(D)
    x1 = np.log10(1.0 + q)
    x2 = np.sqrt(r2) / (1.0 + q)
    x3 = b2 / (1.0 + q)
    x4 = s * s / (r2 * b2 + 1e-300)
    return np.stack([x0, x1, x2, x3, x4], axis=1)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    params = []
    for (o, i) in SIZES:
        W = rng.normal(size=(o, i)) * np.sqrt(2.0 / i)
        b = np.zeros(o)
        params.append([W, b])
    return params


def forward(params, x):
    """x (n, 5) standardised -> (y (n,2), cache)"""
    acts = [x]
    pre = []
    h = x
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        pre.append(z)
        if li < len(params) - 1:
            h = act(z)
            acts.append(h)
        else:
            h = z
    return h, (acts, pre)


def loss_and_grad_out(y, t):
    """loss and dL/dy for targets t = logit(mu*)"""
    n = y.shape[0]
    e0 = y[:, 0] - t
    t1 = np.log(np.abs(e0) + LOG_ERR_C)
    e1 = y[:, 1] - t1
    loss = 0.5 * np.mean(e0 * e0 + e1 * e1)
    dy = np.stack([e0, e1], axis=1) / n
    return loss, dy


def backward(params, cache, dy):
    """gradients [(dW, db)] for dy = dL/dy"""
    acts, pre = cache
    grads = [None] * len(params)
    g = dy
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        if li < len(params) - 1:
            g = g * dact(pre[li])
        dW = g.T @ acts[li]
        db = g.sum(axis=0)
        grads[li] = [dW, db]
        if li == len(params) - 1:
            g = g[:, :1] @ W[:1]        # the error-scale output stops here
        else:
            g = g @ W
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for li in range(len(params)):
            for k in range(2):
                g = grads[li][k]
                self.m[li][k] = self.b1 * self.m[li][k] + (1 - self.b1) * g
                self.v[li][k] = self.b2 * self.v[li][k] + (1 - self.b2) * g * g
                mh = self.m[li][k] / c1
                vh = self.v[li][k] / c2
                params[li][k] = params[li][k] - self.lr * mh / (np.sqrt(vh) + self.eps)


def bracket(y, k=4.0, delta_min=1e-3):
    """(mu_lo, mu_hi) from the network outputs"""
    half = k * np.exp(y[:, 1]) + delta_min
    lo = 1.0 / (1.0 + np.exp(-(y[:, 0] - half)))
    hi = 1.0 / (1.0 + np.exp(-(y[:, 0] + half)))
    return lo, hi

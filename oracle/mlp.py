"""FP64 reference of the per-feature scoring network (4 -> 64 -> 64 -> 2, SiLU).

Test infrastructure only.  Input row j holds four scale-free features of one
column (score z-statistic, minor-allele frequency, tau, log(lambda/lambda_max));
output 0 is the proposed standardised coefficient, output 1 the logit of the
column being active.  The loss per row is

    w_reg (o0 - t)^2 + w_pos a softplus(-o1) + (1 - a) softplus(o1),

averaged over the rows, with target coefficient t and activity a in {0, 1}.
Parity: pinned by central differences and a hand-written closed form
(tests/test_oracle_pins.py).
"""
import numpy as np

SHAPES = {"W1": (64, 4), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (2, 64), "b3": (2,)}
ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]


def n_params():
    return sum(int(np.prod(s)) for s in SHAPES.values())


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, k = {}, 0
    for name in ORDER:
        sz = int(np.prod(SHAPES[name]))
        out[name] = flat[k:k + sz].reshape(SHAPES[name])
        k += sz
    return out


def flatten(params):
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in ORDER])


def silu(a):
    return a / (1.0 + np.exp(-a))


def silu_grad(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def softplus(x):
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def forward(params, F):
    """F: (B, 4).  Returns outputs (B, 2) and the cache for backward."""
    a1 = F @ params["W1"].T + params["b1"]
    h1 = silu(a1)
    a2 = h1 @ params["W2"].T + params["b2"]
    h2 = silu(a2)
    o = h2 @ params["W3"].T + params["b3"]
    return o, (F, a1, h1, a2, h2)


def loss(params, F, t, a, w_reg=1.0, w_pos=1.0):
    o, _ = forward(params, F)
    per = (w_reg * (o[:, 0] - t) ** 2 + w_pos * a * softplus(-o[:, 1])
           + (1.0 - a) * softplus(o[:, 1]))
    return float(np.mean(per))


def backward(params, F, t, a, w_reg=1.0, w_pos=1.0):
    """Gradient of ``loss`` with respect to every parameter (dict of arrays)."""
    o, (F, a1, h1, a2, h2) = forward(params, F)
    B = F.shape[0]
    d_o = np.zeros_like(o)
    d_o[:, 0] = 2.0 * w_reg * (o[:, 0] - t) / B
    # d/dx softplus(-x) = -sigmoid(-x);  d/dx softplus(x) = sigmoid(x)
    d_o[:, 1] = (-w_pos * a * sigmoid(-o[:, 1]) + (1.0 - a) * sigmoid(o[:, 1])) / B
    g = {"W3": d_o.T @ h2, "b3": d_o.sum(axis=0)}
    d_h2 = d_o @ params["W3"]
    d_a2 = d_h2 * silu_grad(a2)
    g["W2"] = d_a2.T @ h1
    g["b2"] = d_a2.sum(axis=0)
    d_h1 = d_a2 @ params["W2"]
    d_a1 = d_h1 * silu_grad(a1)
    g["W1"] = d_a1.T @ F
    g["b1"] = d_a1.sum(axis=0)
    return g


def init_params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name in ORDER:
        shp = SHAPES[name]
        if name.startswith("W"):
            p[name] = rng.standard_normal(shp) * scale / np.sqrt(shp[1])
        else:
            p[name] = np.zeros(shp)
    return p

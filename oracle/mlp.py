"""FP64 reference of the cost-model MLP (test infrastructure only).

The network is 12 -> 64 -> 64 -> 3 with ReLU after the two hidden layers; the loss is the
masked mean squared error L = sum_{s,k} m_sk (y_sk - t_sk)^2 / sum m.  Parameters are one
flat vector laid out as W1[64][12], b1[64], W2[64][64], b2[64], W3[3][64], b3[3] (row-major,
output x input).  The gradient is the textbook backpropagation of that loss; Adam is the
update of Kingma and Ba (ICLR 2015) with bias correction.  Pinned by tests against central
finite differences and against Adam's closed-form first step.
"""
import numpy as np

IN, HID, OUT = 12, 64, 3
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)),
          ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def forward(p, X):
    P = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y, (X, a1, h1, a2, h2)


def loss(p, X, T, M):
    y, _ = forward(p, X)
    M = np.asarray(M, dtype=np.float64)
    return float((M * (y - T) ** 2).sum() / max(M.sum(), 1e-300))


def grad(p, X, T, M):
    """Gradient of the masked mean squared error with respect to the flat parameters."""
    P = unpack(p)
    y, (X, a1, h1, a2, h2) = forward(p, X)
    M = np.asarray(M, dtype=np.float64)
    dy = 2.0 * M * (y - np.asarray(T, dtype=np.float64)) / M.sum()
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dh2 = (dy @ P["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ P["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

Definitions written out plainly: y = W3 g(W2 g(W1 x + b1) + b2) + b3 with the exact GELU
g(z) = z (1 + erf(z / sqrt 2)) / 2, loss = mean over samples and outputs of (y - t)^2, its
gradient by the chain rule, and one bias-corrected Adam update (Kingma & Ba 2015).
Parameter vector order: W1[128][5], b1[128], W2[128][128], b2[128], W3[3][128], b3[3].
"""
import numpy as np
from scipy.special import erf

NIN, NHID, NOUT = 5, 128, 3
SHAPES = [("W1", (NHID, NIN)), ("b1", (NHID,)), ("W2", (NHID, NHID)), ("b2", (NHID,)),
          ("W3", (NOUT, NHID)), ("b3", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(p, X):
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ w["W1"].T + w["b1"]
    h1 = gelu(z1)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = gelu(z2)
    y = h2 @ w["W3"].T + w["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_grad(p, X, T):
    w = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    T = np.asarray(T, dtype=np.float64)
    dy = 2.0 * (y - T) / y.size
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dz2 = (dy @ w["W3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ w["W2"]) * gelu_grad(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return float(np.mean((y - T) ** 2)), pack(g)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

"""FP64 reference of the learned-r_max model (test infrastructure only).

The model is a 7 -> 64 -> 64 -> 1 multilayer perceptron with GELU
activations that predicts y = ln(r_max / r_max*) for a source from cheap
features; the FORA eps guarantee (Lemma 2) holds for any r_max, so the model
only moves work between the push and the walks.

Parameter vector layout (shared with the C ABI's documented layout):
mu[7], sigma[7], W1[64][7], b1[64], W2[64][64], b2[64], W3[64], b3.
"""
from __future__ import annotations

import math

import numpy as np

IN, H = 7, 64
MU, SIG = 0, 7
W1 = 14
B1 = W1 + H * IN
W2 = B1 + H
B2 = W2 + H * H
W3 = B2 + H
B3 = W3 + H
NPARAMS = B3 + 1
TRAIN0 = W1


def unpack(p):
    p = np.asarray(p, np.float64)
    return dict(mu=p[MU:MU + IN], sigma=p[SIG:SIG + IN],
                W1=p[W1:B1].reshape(H, IN), b1=p[B1:W2], W2=p[W2:B2].reshape(H, H),
                b2=p[B2:W3], W3=p[W3:B3], b3=p[B3])


def _phi(z):
    return np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def _cdf(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0)))


def gelu(z):
    return z * _cdf(z)


def gelu_grad(z):
    return _cdf(z) + z * _phi(z)


def forward(p, X):
    """Outputs y[N] and the intermediates of the forward pass."""
    P = unpack(p)
    X = np.asarray(X, np.float64)
    xs = (X - P["mu"]) / P["sigma"]
    z1 = xs @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    y = h2 @ P["W3"] + P["b3"]
    return y, dict(xs=xs, z1=z1, h1=h1, z2=z2, h2=h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def backward(p, X, t):
    """Gradient of the mean squared error with respect to all parameters
    (zero for mu and sigma, which are not trained), by the chain rule."""
    P = unpack(p)
    y, c = forward(p, X)
    N = y.shape[0]
    d3 = 2.0 * (y - np.asarray(t, np.float64)) / N          # dL/dy
    g = np.zeros(NPARAMS)
    g[W3:B3] = c["h2"].T @ d3
    g[B3] = d3.sum()
    d2 = np.outer(d3, P["W3"]) * gelu_grad(c["z2"])          # dL/dz2
    g[W2:B2] = (d2.T @ c["h1"]).ravel()
    g[B2:W3] = d2.sum(0)
    d1 = (d2 @ P["W2"]) * gelu_grad(c["z1"])                 # dL/dz1
    g[W1:B1] = (d1.T @ c["xs"]).ravel()
    g[B1:W2] = d1.sum(0)
    return g


def adam(p, g, m, v, lr, b1, b2, eps, step):
    """One bias-corrected Adam step (Kingma & Ba, ICLR 2015, Algorithm 1) on
    the trained parameters."""
    p, m, v = p.copy(), m.copy(), v.copy()
    sl = slice(TRAIN0, NPARAMS)
    m[sl] = b1 * m[sl] + (1 - b1) * g[sl]
    v[sl] = b2 * v[sl] + (1 - b2) * g[sl] ** 2
    mh = m[sl] / (1 - b1 ** step)
    vh = v[sl] / (1 - b2 ** step)
    p[sl] = p[sl] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as
    float32."""
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (r.astype(np.uint32) << 16).view(np.float32)
    nan = np.isnan(x)
    out = np.where(nan, np.float32(np.nan), out)
    return out.astype(np.float32)


def forward_bf16(p, X):
    """The BF16 inference pass: weights, standardised inputs and hidden
    activations rounded to BF16, sums in FP64."""
    pb = bf16_round(np.asarray(p, np.float32)).astype(np.float64)
    P = unpack(pb)
    X = np.asarray(X, np.float64)
    xs = bf16_round(((X - P["mu"]) / P["sigma"]).astype(np.float32)).astype(np.float64)
    h1 = bf16_round(gelu(xs @ P["W1"].T + P["b1"]).astype(np.float32)).astype(np.float64)
    h2 = bf16_round(gelu(h1 @ P["W2"].T + P["b2"]).astype(np.float32)).astype(np.float64)
    return h2 @ P["W3"] + P["b3"]


def features(g, srcs, alpha, eps, rmax_star):
    """The 7 source features: ln d(s); ln sum of the out-degrees of s's
    out-neighbours; the residue mass left on nodes over their threshold after
    the first synchronous push round at r_max* (each out-neighbour u holds
    (1-alpha)/d(s) and counts when that exceeds r_max* d(u); 0 if s is not
    pushed); ln n; ln m; alpha; eps."""
    deg = np.diff(g.rowptr.astype(np.int64))
    out = np.zeros((len(srcs), IN))
    for i, s in enumerate(np.asarray(srcs, np.int64)):
        nb = g.colidx[g.rowptr[s]:g.rowptr[s + 1]]
        dn = deg[nb].astype(np.float64)
        share = (1.0 - alpha) / deg[s]
        pushed = 1.0 > rmax_star * deg[s]
        out[i] = [math.log(deg[s]), math.log(dn.sum()),
                  (share * np.count_nonzero(share > rmax_star * dn)) if pushed else 0.0,
                  math.log(g.n), math.log(g.m), alpha, eps]
    return out

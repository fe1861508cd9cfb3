"""Plain FP64 reference of the message-passing network that proposes the
start block of Jacobi-Davidson, and of its training loss and gradients.

TEST INFRASTRUCTURE ONLY: the tests are its only users; the product library
never imports or executes anything here, and the two share no code.

The network is an engineering addition (the paper starts JD from one unit
vector, Algorithm 2); it can change only how many iterations JD needs,
never the answer, which the FP64 residual certificate decides.  Written out
plainly in numpy, dense where that is clearer, in the order below:

features (per vertex i, caller order; d = generalized degrees, A = D - G)
    f0 = 1,  f1 = log(1 + d_i),  f2 = (A f1)_i / d_i   (0 when d_i = 0),
    f_{3+c} = sqrt(3) u(seed, i R + c), c < R, u the SplitMix64 uniform
    variate in [-1, 1) of a counter (unit variance)
layer l < L (F_0 = 3 + R, F_l = H):
    Hc_l = [h_l | agg(h_l)],  agg(h) = D^{-1} A h   (rows with d = 0: 0)
    h_{l+1} = ReLU(Hc_l W_l + b_l),   W_l: 2 F_l x H
output:
    Y = Hc_L W_o + b_o,  W_o: 2H x p
    Yh = Y - Z (Z' Y),   Z = the normalized component indicators
loss against an orthonormal target X (n x k, orthogonal to Z):
    S = Yh'Yh,  C = Yh'X,  loss = 1 - trace(S^{-1} C C') / k
(the squared cosines of the principal angles between span X and span Yh,
averaged; 0 when span Yh contains span X, invariant to Yh -> Yh R).
Parameters are one flat vector: for each layer W (column-major, 2F_in x
F_out) then b (F_out), the output layer last.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Config:
    layers: int = 2
    hidden: int = 32
    random_channels: int = 4
    out_cols: int = 9

    @property
    def in_features(self) -> int:
        return 3 + self.random_channels

    def shapes(self):
        """(rows, cols) of each weight matrix, input layer first, output last."""
        dims = [self.in_features] + [self.hidden] * self.layers
        out = [(2 * dims[l], dims[l + 1]) for l in range(self.layers)]
        out.append((2 * dims[-1], self.out_cols))
        return out

    def num_params(self) -> int:
        return sum(r * c + c for r, c in self.shapes())


def splitmix_unit(seed: int, counters) -> np.ndarray:
    """SplitMix64 (Steele, Lea & Flood 2014) of (seed + (i + 1) * golden
    gamma), top 53 bits mapped to [-1, 1)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0) * 2.0 - 1.0


def unpack(cfg: Config, flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == cfg.num_params()
    out, at = [], 0
    for r, c in cfg.shapes():
        W = flat[at:at + r * c].reshape(c, r).T  # column-major storage
        at += r * c
        b = flat[at:at + c]
        at += c
        out.append((W, b))
    return out


def pack(cfg: Config, layers) -> np.ndarray:
    parts = []
    for W, b in layers:
        parts.append(np.asarray(W, dtype=np.float64).T.reshape(-1))
        parts.append(np.asarray(b, dtype=np.float64).reshape(-1))
    return np.concatenate(parts)


class Graph:
    """The pieces of G = D - A the network needs (caller order)."""

    def __init__(self, L):
        G = sp.csr_matrix(L.to_scipy(), dtype=np.float64)
        self.n = G.shape[0]
        self.d = np.asarray(G.diagonal()).copy()
        self.A = (sp.diags(self.d) - G).tocsr()
        self.A.eliminate_zeros()
        # component indicators, normalized
        ncomp, lab = sp.csgraph.connected_components(self.A, directed=False)
        Z = np.zeros((self.n, ncomp))
        Z[np.arange(self.n), lab] = 1.0
        self.Z = Z / np.sqrt(Z.sum(axis=0))

    def agg(self, h):
        """D^{-1} A h, rows of isolated vertices 0."""
        out = self.A @ h
        pos = self.d > 0
        out[pos] /= self.d[pos][:, None] if out.ndim == 2 else self.d[pos]
        out[~pos] = 0.0
        return out

    def agg_t(self, g):
        """(D^{-1} A)' g = A D^{-1} g."""
        s = np.zeros_like(g)
        pos = self.d > 0
        s[pos] = g[pos] / (self.d[pos][:, None] if g.ndim == 2 else self.d[pos])
        return self.A @ s


def features(cfg: Config, gr: Graph, seed: int) -> np.ndarray:
    n, R = gr.n, cfg.random_channels
    f = np.empty((n, 3 + R))
    f[:, 0] = 1.0
    f[:, 1] = np.log1p(gr.d)
    f[:, 2] = gr.agg(f[:, 1])
    cnt = np.arange(n, dtype=np.uint64)[:, None] * np.uint64(R) + np.arange(R, dtype=np.uint64)[None, :]
    f[:, 3:] = np.sqrt(3.0) * splitmix_unit(seed, cnt)
    return f


def forward(cfg: Config, params, gr: Graph, seed: int):
    layers = unpack(cfg, params)
    h = features(cfg, gr, seed)
    cache = []
    for W, b in layers[:-1]:
        Hc = np.concatenate([h, gr.agg(h)], axis=1)
        Zp = Hc @ W + b
        cache.append((Hc, Zp))
        h = np.maximum(Zp, 0.0)
    Wo, bo = layers[-1]
    Hc = np.concatenate([h, gr.agg(h)], axis=1)
    Y = Hc @ Wo + bo
    cache.append((Hc, None))
    Yh = Y - gr.Z @ (gr.Z.T @ Y)
    return Yh, cache


def subspace_loss(Yh, X):
    """loss = 1 - trace(S^{-1} C C') / k and its gradient with respect to Yh."""
    k = X.shape[1]
    S = Yh.T @ Yh
    C = Yh.T @ X
    Sinv = np.linalg.inv(S)
    M = C @ C.T
    loss = 1.0 - np.trace(Sinv @ M) / k
    B = Sinv @ M @ Sinv
    grad = (2.0 / k) * (Yh @ B - X @ (C.T @ Sinv))
    return loss, grad


def loss_and_grad(cfg: Config, params, gr: Graph, seed: int, X):
    """The training loss and its gradient (flat, like params)."""
    layers = unpack(cfg, params)
    Yh, cache = forward(cfg, params, gr, seed)
    loss, gY = subspace_loss(Yh, X)
    gY = gY - gr.Z @ (gr.Z.T @ gY)  # through the projection (symmetric)
    grads = [None] * len(layers)
    # output layer
    Hc, _ = cache[-1]
    Wo, _ = layers[-1]
    grads[-1] = (Hc.T @ gY, gY.sum(axis=0))
    gHc = gY @ Wo.T
    F = Hc.shape[1] // 2
    gh = gHc[:, :F] + gr.agg_t(gHc[:, F:])
    for l in range(len(layers) - 2, -1, -1):
        Hc, Zp = cache[l]
        W, _ = layers[l]
        gZ = gh * (Zp > 0.0)
        grads[l] = (Hc.T @ gZ, gZ.sum(axis=0))
        if l > 0:
            gHc = gZ @ W.T
            F = Hc.shape[1] // 2
            gh = gHc[:, :F] + gr.agg_t(gHc[:, F:])
    return float(loss), pack(cfg, grads)


def init_params(cfg: Config, seed: int) -> np.ndarray:
    """Glorot-uniform weights from SplitMix64 (counter = flat index), zero
    biases; an independent draw used only by the tests."""
    layers = []
    at = 0
    for r, c in cfg.shapes():
        a = np.sqrt(6.0 / (r + c))
        W = a * splitmix_unit(seed, np.arange(at, at + r * c)).reshape(c, r).T
        at += r * c + c
        layers.append((W, np.zeros(c)))
    return pack(cfg, layers)


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1), written out plainly
    in FP64: first and second moment averages of the gradient, their bias
    corrections by 1 - beta^step, then a step of lr times the corrected
    first moment over (the square root of the corrected second moment plus
    eps).  step counts from 1.  Returns (new params, new m, new v)."""
    g = np.asarray(grad, dtype=np.float64)
    m_new = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v_new = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m_new / (1.0 - beta1 ** step)
    v_hat = v_new / (1.0 - beta2 ** step)
    p_new = np.asarray(params, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p_new, m_new, v_new

"""fp64 reference of the learned warm start (TEST INFRASTRUCTURE ONLY).

The paper warm-starts GN from fractional solutions of an LP solver (Section 6,
"Randomized start and warm start"); the learned warm start replaces that solver
with a small message-passing network trained on GN's own results.  This module
is the plain reference of that network, written from its definition below; it
shares no code with the HIP kernels.

Definition (n vertices, hidden width H = 64):
  features  h0_i = [ w_i, deg_i / 10, w_i / max_{j in N[i]} w_j,
                     sum_{j in N(i)} w_j / (w_i + sum_{j in N(i)} w_j) ]
            (N[i] = N(i) + {i}, the closed neighbourhood)
  mean      M(H)_i = (1/deg_i) sum_{j in N(i)} H_j   (0 for isolated vertices)
  layer 1   X1 = [h0 | M(h0) | 0_8]   (n x 16),  h1 = ReLU(bf(X1) bf(W1) + b1)
  layer 2   H1 = bf(h1),  X2 = [H1 | bf(M(H1))] (n x 128),  h2 = ReLU(X2 bf(W2) + b2)
  head      z = h2 bf(u) + c,   p = sigmoid(z),
            x0 = clamp(p, 1e-3, 1) where |p - 1/2| > gate, else 1/2
  loss      L = mean_i [ softplus(z_i) - l_i z_i ]   (binary cross-entropy with labels l)
where bf(.) rounds to bfloat16 (round to nearest even), the precision the
matrix cores consume; products accumulate in full precision.  The backward
pass follows the chain rule of the same expression; the operands of its
matrix products are rounded to bfloat16 at the same places as the forward
(dpre2 and dpre1, the pre-activation gradients).  Passing rounding=False
gives the exact-arithmetic network (used for the finite-difference pins).

Parameter vector (fp32 master copy, flat): W1 [16 x 64] (rows 0-3 self
weights, rows 4-7 neighbour weights, rows 8-15 zero), b1 [64], W2 [128 x 64]
(rows 0-63 self, 64-127 neighbour), b2 [64], u [64], c [1].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

HID = 64
FEAT = 4
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_U, OFF_C = 0, 1024, 1088, 9280, 9344, 9408
NPARAMS = 9409


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) and return as float64 (via fp32 bits)."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    return (t[OFF_W1:OFF_B1].reshape(16, HID), t[OFF_B1:OFF_W2], t[OFF_W2:OFF_B2].reshape(128, HID),
            t[OFF_B2:OFF_U], t[OFF_U:OFF_C], t[OFF_C])


def init_params(seed: int = 0) -> np.ndarray:
    """He-style random init (float32), zero rows 8-15 of W1."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NPARAMS, dtype=np.float32)
    w1 = rng.standard_normal((16, HID)) * np.sqrt(2.0 / 8)
    w1[8:] = 0.0
    th[OFF_W1:OFF_B1] = w1.reshape(-1)
    th[OFF_W2:OFF_B2] = (rng.standard_normal((128, HID)) * np.sqrt(2.0 / 128)).reshape(-1)
    th[OFF_U:OFF_C] = rng.standard_normal(HID) * np.sqrt(1.0 / HID)
    return th


def _adj(n, row_ptr, col_idx):
    return sp.csr_matrix((np.ones(len(col_idx)), np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))


def features(n, row_ptr, col_idx, w) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    rp = np.asarray(row_ptr)
    out = np.zeros((n, FEAT))
    for i in range(n):
        nb = np.asarray(col_idx[rp[i]:rp[i + 1]])
        s = w[nb].sum() if nb.size else 0.0
        m = max(w[i], w[nb].max()) if nb.size else w[i]
        out[i] = [w[i], nb.size / 10.0, w[i] / m, s / (w[i] + s)]
    return out


def _mean_op(n, row_ptr, col_idx):
    A = _adj(n, row_ptr, col_idx)
    deg = np.diff(np.asarray(row_ptr)).astype(np.float64)
    inv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)
    return sp.diags(inv) @ A


def forward(n, row_ptr, col_idx, w, theta, rounding=True, gate=0.0):
    """Returns (x0, cache) with cache holding what backward needs."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, u, c = unpack(theta)
    Mop = _mean_op(n, row_ptr, col_idx)
    h0 = features(n, row_ptr, col_idx, w)
    X1 = np.zeros((n, 16))
    X1[:, 0:4] = h0
    X1[:, 4:8] = Mop @ h0
    X1r = rnd(X1)
    pre1 = X1r @ rnd(W1) + b1
    h1 = np.maximum(pre1, 0.0)
    H1 = rnd(h1)
    X2 = np.concatenate([H1, rnd(Mop @ H1)], axis=1)
    pre2 = X2 @ rnd(W2) + b2
    h2 = np.maximum(pre2, 0.0)
    z = h2 @ rnd(u) + c
    sig = 1.0 / (1.0 + np.exp(-z))
    x0 = np.where(np.abs(sig - 0.5) > gate, np.clip(sig, 1e-3, 1.0), 0.5)
    cache = dict(Mop=Mop, X1r=X1r, pre1=pre1, X2=X2, pre2=pre2, h2=h2, z=z, sig=sig)
    return x0, cache


def loss_and_grad(n, row_ptr, col_idx, w, theta, labels, rounding=True):
    """Binary cross-entropy of sigmoid(z) against labels and its gradient (flat)."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, u, c = unpack(theta)
    x0, C = forward(n, row_ptr, col_idx, w, theta, rounding)
    z = C["z"]
    lab = np.asarray(labels, dtype=np.float64)
    L = float(np.mean(np.logaddexp(0.0, z) - lab * z))
    dz = (C["sig"] - lab) / n
    g = np.zeros(NPARAMS)
    g[OFF_U:OFF_C] = C["h2"].T @ dz
    g[OFF_C] = dz.sum()
    dpre2 = np.outer(dz, rnd(u)) * (C["pre2"] > 0)
    dpre2r = rnd(dpre2)
    g[OFF_W2:OFF_B2] = (C["X2"].T @ dpre2r).reshape(-1)
    g[OFF_B2:OFF_U] = dpre2.sum(axis=0)
    dX2 = dpre2r @ rnd(W2).T
    dH1 = dX2[:, :HID] + C["Mop"].T @ dX2[:, HID:]
    dpre1 = dH1 * (C["pre1"] > 0)
    dpre1r = rnd(dpre1)
    gW1 = C["X1r"].T @ dpre1r
    gW1[8:] = 0.0
    g[OFF_W1:OFF_B1] = gW1.reshape(-1)
    g[OFF_B1:OFF_W2] = dpre1.sum(axis=0)
    return L, g, x0


def adam_step(theta, grad, m, v, t, lr=3e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): returns new (theta, m, v); t counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v

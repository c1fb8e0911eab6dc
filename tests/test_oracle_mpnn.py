"""Pins of the fp64 message-passing warm-start reference (oracle/mpnn.py).

The network is this implementation's own definition (the paper's warm start uses
an LP solver), so the pins check that the reference computes that definition:
hand-computed features, closed-form outputs for hand-set weights (which catch a
sum instead of a mean, swapped self/neighbour blocks, a transposed weight or a
missing bias), bfloat16 rounding against torch's conversion, the backward pass
against central differences and against torch autograd, and Adam against
torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mpnn as M
from helpers import graph_from_edges
from paper_2605_05330_amd import inputs as I


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 1e-30])])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(a), ref)


def test_features_by_hand():
    """Path a-b-c with w = (1, 4, 9) plus an isolated vertex d with w = 2."""
    g = graph_from_edges(4, [(0, 1), (1, 2)])
    f = M.features(4, g.row_ptr, g.col_idx, np.array([1.0, 4.0, 9.0, 2.0]))
    np.testing.assert_allclose(f, [[1, 0.1, 1 / 4, 4 / 5],
                                   [4, 0.2, 4 / 9, 10 / 14],
                                   [9, 0.1, 1, 4 / 13],
                                   [2, 0.0, 1, 0]], rtol=1e-15)


def _net(n=60, seed=0):
    g = I.unit_disk(n, 6, seed)
    w = I.weights_uniform01(n, seed).astype(np.float64)
    return g, w


def test_mean_aggregation_and_layout_closed_form():
    """Hand-set weights: layer 1 outputs h1 = (w_i, mean_{N(i)} deg_j/10, 1, 1, ...);
    layer 2 passes column 0 through the self block and column 1 through the
    neighbour block, so z = u0*bf(w_i) + u1*bf(mean_{N(i)} bf(mean_{N(j)} deg/10)) + c."""
    g, w = _net()
    n = g.n
    th = np.zeros(M.NPARAMS)
    W1 = np.zeros((16, 64))
    W1[0, 0] = 1.0            # self feature 0 (w) -> hidden 0
    W1[4 + 1, 1] = 1.0        # neighbour mean of feature 1 (deg/10) -> hidden 1
    th[M.OFF_W1:M.OFF_B1] = W1.reshape(-1)
    b1 = np.zeros(64)
    b1[2:] = 1.0
    th[M.OFF_B1:M.OFF_W2] = b1
    W2 = np.zeros((128, 64))
    W2[0, 0] = 1.0            # self block
    W2[64 + 1, 1] = 1.0       # neighbour block
    th[M.OFF_W2:M.OFF_B2] = W2.reshape(-1)
    u = np.zeros(64)
    u[0], u[1] = 0.5, 2.0
    th[M.OFF_U:M.OFF_C] = u
    th[M.OFF_C] = -0.25
    x0, C = M.forward(n, g.row_ptr, g.col_idx, w, th)
    deg = g.degrees().astype(np.float64)
    nbr = [g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]] for i in range(n)]
    mdeg = np.array([np.mean(deg[nb]) / 10 if len(nb) else 0.0 for nb in nbr])
    h1_1 = M.bf16(M.bf16(mdeg))                      # rounded X1 entry, then rounded h1
    m2 = np.array([np.mean(h1_1[nb]) if len(nb) else 0.0 for nb in nbr])
    z = 0.5 * M.bf16(M.bf16(w)) + 2.0 * M.bf16(m2) - 0.25
    np.testing.assert_allclose(C["z"], z, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(x0, np.clip(1 / (1 + np.exp(-z)), 1e-3, 1), rtol=1e-12)


def test_isolated_vertex_sees_zero_neighbourhood():
    g = graph_from_edges(3, [(0, 1)])
    th = M.init_params(1)
    x0, C = M.forward(3, g.row_ptr, g.col_idx, np.array([0.3, 0.6, 0.9]), th)
    assert np.all(C["X1r"][2, 4:8] == 0.0) and np.all(C["X2"][2, 64:] == 0.0)


def test_backward_matches_central_differences():
    g, w = _net(40, 3)
    th = M.init_params(3).astype(np.float64)
    lab = (I.rng_for(3, 5).random(40) < 0.4).astype(np.float64)
    L, gr, _ = M.loss_and_grad(40, g.row_ptr, g.col_idx, w, th, lab, rounding=False)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(np.arange(M.OFF_W1, M.OFF_W1 + 512), 30, replace=False),
                          rng.choice(np.arange(M.OFF_W2, M.OFF_B2), 60, replace=False),
                          np.arange(M.OFF_B1, M.OFF_B1 + 10), np.arange(M.OFF_B2, M.OFF_B2 + 10),
                          np.arange(M.OFF_U, M.OFF_U + 10), [M.OFF_C]])
    h = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (M.loss_and_grad(40, g.row_ptr, g.col_idx, w, tp, lab, rounding=False)[0]
              - M.loss_and_grad(40, g.row_ptr, g.col_idx, w, tm, lab, rounding=False)[0]) / (2 * h)
        assert abs(fd - gr[k]) <= 1e-6 * max(1.0, abs(gr[k])) + 1e-8, (k, fd, gr[k])


def test_backward_matches_torch_autograd():
    g, w = _net(80, 4)
    n = g.n
    th = M.init_params(4).astype(np.float64)
    lab = (I.rng_for(4, 5).random(n) < 0.4).astype(np.float64)
    L, gr, _ = M.loss_and_grad(n, g.row_ptr, g.col_idx, w, th, lab, rounding=False)
    t = torch.tensor(th, requires_grad=True)
    W1 = t[M.OFF_W1:M.OFF_B1].reshape(16, 64)
    b1 = t[M.OFF_B1:M.OFF_W2]
    W2 = t[M.OFF_W2:M.OFF_B2].reshape(128, 64)
    b2 = t[M.OFF_B2:M.OFF_U]
    u = t[M.OFF_U:M.OFF_C]
    c = t[M.OFF_C]
    Mop = torch.tensor(M._mean_op(n, g.row_ptr, g.col_idx).toarray())
    h0 = torch.tensor(M.features(n, g.row_ptr, g.col_idx, w))
    X1 = torch.cat([h0, Mop @ h0, torch.zeros(n, 8, dtype=torch.float64)], dim=1)
    h1 = torch.relu(X1 @ W1 + b1)
    h2 = torch.relu(torch.cat([h1, Mop @ h1], dim=1) @ W2 + b2)
    z = h2 @ u + c
    loss = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(lab))
    loss.backward()
    assert loss.item() == pytest.approx(L, rel=1e-12)
    g_ref = t.grad.numpy().copy()
    g_ref[M.OFF_W1 + 8 * 64:M.OFF_B1] = 0.0   # padding rows carry no gradient
    np.testing.assert_allclose(gr, g_ref, rtol=1e-9, atol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(2)
    th = rng.standard_normal(100)
    m = np.zeros(100)
    v = np.zeros(100)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 4):
        gr = rng.standard_normal(100)
        th, m, v = M.adam_step(th, gr, m, v, t)
        opt.zero_grad()
        p.grad = torch.tensor(gr)
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_gate_keeps_only_confident_vertices():
    g, w = _net(50, 8)
    th = M.init_params(8)
    th[M.OFF_C] = 3.0
    x_all, C = M.forward(50, g.row_ptr, g.col_idx, w, th)
    x_g, _ = M.forward(50, g.row_ptr, g.col_idx, w, th, gate=0.45)
    conf = np.abs(C["sig"] - 0.5) > 0.45
    assert np.array_equal(x_g[conf], x_all[conf]) and np.all(x_g[~conf] == 0.5)

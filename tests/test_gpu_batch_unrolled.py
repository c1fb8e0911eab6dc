"""Batched unrolled steps and adjoint (gn_batch_unrolled_forward / _backward):
bit-identical to the chained unrolled path (gn_unrolled_* with ckpt_every = 1)
on the batch's block-diagonal union graph, whose gradients are pinned against
the fp64 oracle by finite differences (test_gpu_grad.py)."""
import numpy as np
import pytest

from paper_2605_05330_amd import inputs as I

pytestmark = pytest.mark.gpu
F32 = np.float32


def _graphs():
    gs = [I.erdos_renyi(300, 6 / 299, 1), I.unit_disk(2000, 10, 2), I.barabasi_albert(500, 5, 3),
          I.hub_graph(900, [70, 150, 600], 3.0, 4), I.erdos_renyi(1, 0.0, 5), I.erdos_renyi(2, 1.0, 6),
          I.erdos_renyi(40, 0.2, 7), I.unit_disk(700, 8, 8)]
    ws = [I.weights_uniform01(g.n, 10 + k) for k, g in enumerate(gs)]
    return gs, ws


@pytest.mark.parametrize("with_w", [False, True])
def test_batch_unrolled_matches_union(gpu, with_w):
    import torch
    from paper_2605_05330_amd import libgn
    gs, ws = _graphs()
    B = libgn.Batch.from_graphs(gs, ws)
    U = B.graph_handle()
    N = B.total_n
    T = 20
    gammas = np.linspace(0.9, 1.5, T).astype(F32)
    rng = np.random.default_rng(0)
    x0 = torch.tensor(rng.uniform(0.05, 1.0, N).astype(F32), device="cuda")
    gxT = torch.tensor(rng.standard_normal(N).astype(F32), device="cuda")
    w = torch.tensor(rng.uniform(0.1, 2.0, N).astype(F32), device="cuda") if with_w else None

    ck = torch.empty(libgn.gn_unrolled_ckpt_floats(U, T, 1), device="cuda")
    xT_u, gw_u, gx0_u = (torch.empty(N, device="cuda") for _ in range(3))
    libgn.gn_unrolled_forward(U, w, gammas, 1, x0, xT_u, ck)
    libgn.gn_unrolled_backward(U, w, gammas, 1, ck, gxT, gw_u, gx0_u)

    store = torch.empty(libgn.gn_batch_unrolled_store_floats(B.handle, T), device="cuda")
    xT_b, gw_b, gx0_b = (torch.full((N,), float("nan"), device="cuda") for _ in range(3))
    libgn.gn_batch_unrolled_forward(B.handle, w, gammas, x0, xT_b, store)
    libgn.gn_batch_unrolled_backward(B.handle, w, gammas, store, gxT, gw_b, gx0_b)
    torch.cuda.synchronize()
    for a, b, name in ((xT_u, xT_b, "xT"), (gw_u, gw_b, "gw"), (gx0_u, gx0_b, "gx0")):
        ua = a.cpu().numpy().view(np.uint32)
        ub = b.cpu().numpy().view(np.uint32)
        assert np.array_equal(ua, ub), (name, int(np.sum(ua != ub)))
    # a second call with other gammas uploads the new table
    g2 = np.full(T, 1.2, F32)
    libgn.gn_unrolled_forward(U, w, g2, 1, x0, xT_u, ck)
    libgn.gn_batch_unrolled_forward(B.handle, w, g2, x0, xT_b, store)
    torch.cuda.synchronize()
    assert np.array_equal(xT_u.cpu().numpy().view(np.uint32), xT_b.cpu().numpy().view(np.uint32))


def test_batch_unrolled_zero_steps_and_limits(gpu):
    import torch
    from paper_2605_05330_amd import libgn
    gs, ws = _graphs()
    B = libgn.Batch.from_graphs(gs, ws)
    N = B.total_n
    x0 = torch.rand(N, device="cuda")
    xT = torch.empty(N, device="cuda")
    libgn.gn_batch_unrolled_forward(B.handle, None, np.zeros(0, F32), x0, xT, None)
    gxT = torch.randn(N, device="cuda")
    gw = torch.full((N,), 7.0, device="cuda")
    gx0 = torch.empty(N, device="cuda")
    libgn.gn_batch_unrolled_backward(B.handle, None, np.zeros(0, F32), None, gxT, gw, gx0)
    torch.cuda.synchronize()
    assert torch.equal(xT, x0) and torch.equal(gx0, gxT) and torch.count_nonzero(gw).item() == 0
    # a graph whose adjoint state (16 n bytes) exceeds one compute unit's LDS
    big = I.erdos_renyi(12000, 4 / 11999, 9)
    Bb = libgn.Batch.from_graphs([big, gs[0]], [I.weights_uniform01(big.n, 1), ws[0]])
    T = 4
    g = np.full(T, 1.0, F32)
    Nb = Bb.total_n
    store = torch.empty(libgn.gn_batch_unrolled_store_floats(Bb.handle, T), device="cuda")
    x0b, xTb = torch.rand(Nb, device="cuda"), torch.empty(Nb, device="cuda")
    libgn.gn_batch_unrolled_forward(Bb.handle, None, g, x0b, xTb, store)  # 8 n bytes: fits
    with pytest.raises(libgn.GNError):
        libgn.gn_batch_unrolled_backward(Bb.handle, None, g, store, torch.randn(Nb, device="cuda"),
                                         torch.empty(Nb, device="cuda"), torch.empty(Nb, device="cuda"))
    with pytest.raises(libgn.GNError):
        libgn.gn_batch_unrolled_forward(B.handle, None, np.array([1.0, float("nan")], F32), x0, xT, store)


def test_autograd_batch_matches_chained(gpu):
    import torch
    from paper_2605_05330_amd import libgn
    from paper_2605_05330_amd.autograd import gn_unrolled, gn_unrolled_batch
    gs, ws = _graphs()
    B = libgn.Batch.from_graphs(gs, ws)
    w0 = torch.tensor(np.concatenate(ws), device="cuda")
    gam = np.linspace(1.0, 1.4, 12).astype(F32)
    grads = []
    for batched in (False, True):
        w = w0.clone().requires_grad_(True)
        x0 = torch.full_like(w0, 0.5).requires_grad_(True)
        xT = gn_unrolled_batch(w, x0, B.handle, gam) if batched else gn_unrolled(w, x0, B.graph_handle(), gam, 1)
        (w * xT).sum().backward()
        grads.append((xT.detach().clone(), w.grad.clone(), x0.grad.clone()))
    for a, b in zip(*grads):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_batch_unrolled_many_graphs(gpu):
    """More graphs than compute units: the 512-thread kernels (two graphs per
    compute unit); same bit-identity with the chained path."""
    import torch
    from paper_2605_05330_amd import libgn
    gs = [I.erdos_renyi(20 + 7 * k, 5 / (19 + 7 * k), 100 + k) if k % 2 else I.unit_disk(30 + 5 * k, 8, 100 + k)
          for k in range(320)]
    ws = [I.weights_uniform01(g.n, 400 + k) for k, g in enumerate(gs)]
    B = libgn.Batch.from_graphs(gs, ws)
    U = B.graph_handle()
    N = B.total_n
    T = 8
    gammas = np.linspace(1.0, 1.5, T).astype(F32)
    rng = np.random.default_rng(1)
    x0 = torch.tensor(rng.uniform(0.05, 1.0, N).astype(F32), device="cuda")
    gxT = torch.tensor(rng.standard_normal(N).astype(F32), device="cuda")
    ck = torch.empty(libgn.gn_unrolled_ckpt_floats(U, T, 1), device="cuda")
    xT_u, gw_u, gx0_u = (torch.empty(N, device="cuda") for _ in range(3))
    libgn.gn_unrolled_forward(U, None, gammas, 1, x0, xT_u, ck)
    libgn.gn_unrolled_backward(U, None, gammas, 1, ck, gxT, gw_u, gx0_u)
    store = torch.empty(libgn.gn_batch_unrolled_store_floats(B.handle, T), device="cuda")
    xT_b, gw_b, gx0_b = (torch.empty(N, device="cuda") for _ in range(3))
    libgn.gn_batch_unrolled_forward(B.handle, None, gammas, x0, xT_b, store)
    libgn.gn_batch_unrolled_backward(B.handle, None, gammas, store, gxT, gw_b, gx0_b)
    torch.cuda.synchronize()
    for a, b in ((xT_u, xT_b), (gw_u, gw_b), (gx0_u, gx0_b)):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))

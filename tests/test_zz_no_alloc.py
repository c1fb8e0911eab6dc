"""gn_step_static (the step entry point that allocates nothing) against gn_step.

Both run the same kernels; the static variant keeps its state words in the
library's static device array instead of the graph's workspace.  Two calls in a
row, the second on a smaller graph, must each equal gn_step bit for bit (the
array keeps the first call's words; nothing from them may leak into the
second), and a graph above the array's capacity is refused with GN_E_SIZE
before any work is queued."""
import numpy as np
import pytest

from paper_2605_05330_amd import inputs as I

pytestmark = pytest.mark.gpu
F32 = np.float32


def _lib():
    from paper_2605_05330_amd import libgn
    return libgn


def _pair(g, w, x, gamma):
    import torch
    lg = _lib()
    G = lg.Graph(g.n, g.row_ptr, g.col_idx, w)
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=F32)).cuda()
    a, b = torch.full_like(xd, -7.0), torch.full_like(xd, -9.0)
    lg.gn_step(G.handle, gamma, xd, a)
    lg.gn_step_static(G.handle, gamma, xd, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_static_step_matches_step_twice_shrinking(gpu):
    big = I.barabasi_albert(200_000, 5, 0)            # every degree bin, 200k words
    wb = I.weights_uniform01(big.n, 0)
    r = I.rng_for(4, 8)
    xb = r.random(big.n) * 0.98 + 0.01
    xb[r.random(big.n) < 0.2] = np.exp2(-r.uniform(100, 140, 1))[0]   # some log-form states
    small = I.erdos_renyi(3001, 8 / 3000, 5)
    ws = I.weights_uniform01(small.n, 5)
    xs = I.rng_for(5, 9).random(small.n) * 0.98 + 0.01
    for g, w, x, gamma in ((big, wb, xb, 1.3), (small, ws, xs, 0.9)):
        a, b = _pair(g, w, x, gamma)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert np.all(a >= 0.0)


def test_static_step_capacity(gpu):
    import torch
    lg = _lib()
    cap = lg.gn_step_static_max_n()
    assert cap == 1 << 21
    n = cap + 1
    g = I.csr_from_edges(n, np.zeros(0), np.zeros(0))
    G = lg.Graph(n, g.row_ptr, g.col_idx, np.ones(n, F32))
    x = torch.full((n,), 0.5, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(lg.GNError) as e:
        lg.gn_step_static(G.handle, 1.5, x, y)
    assert e.value.status == lg.GN_E_SIZE
    lg.gn_step(G.handle, 1.5, x, y)          # the allocating entry point still takes it
    assert torch.all(y == 1.0)

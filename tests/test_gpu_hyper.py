"""Parity of GN under hyperedge constraints (gn_hyper_*) with the fp64 oracle
(oracle/hyper.py: the conflict multigraph run through the C oracle), through
the C ABI.

Step: element-wise within 1e-5 relative (fp32 sums of at most a few hundred
terms per vertex against fp64).  Solve: steps within 2 (threshold decisions of
the stopping test taken in fp32 and fp64), the same set, the same W(S)
exactly, statistics within fp32 rounding.  Instances: routes and stops where
pairs share several hyperedges (multiplicity > 1), rows and columns of an
assignment board (equal to the rook graph), hyperedges longer than a
wavefront, a check interval above 1, a run cut by max_steps.
"""
import numpy as np
import pytest

import oracle as O
from oracle import hyper as OH
from paper_2605_05330_amd import inputs

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2605_05330_amd import libgn
    return libgn


def _rook_hyperedges(N):
    ptr = np.arange(0, 2 * N * N + 1, N)
    members = np.concatenate([np.arange(N * i, N * i + N) for i in range(N)] +
                             [np.arange(j, N * N, N) for j in range(N)])
    return ptr, members


def _cases():
    a = inputs.clique_cover_instance(2000, 300, 3, 8, 1)
    b = inputs.clique_cover_instance(500, 8, 1, 3, 2)  # hyperedges of ~60-190 members
    return {"routes2000": (a.n, a.ptr, a.members), "long500": (b.n, b.ptr, b.members),
            "rook24": (24 * 24, *_rook_hyperedges(24))}


@pytest.mark.parametrize("case", ["routes2000", "long500", "rook24"])
@pytest.mark.parametrize("gamma", [0.9, 1.5])
def test_step_matches_oracle(gpu, case, gamma):
    import torch
    libgn = _lib()
    n, ptr, mem = _cases()[case]
    w = inputs.weights_uniform01(n, 5)
    x = inputs.rng_for(5, 21).random(n, dtype=np.float32)
    H = libgn.Hyper(n, ptr, mem, w)
    xi = torch.from_numpy(x).cuda()
    xo = torch.empty_like(xi)
    H.step(np.float32(gamma), xi, xo)
    ref, _ = OH.step(n, ptr, mem, w.astype(np.float64), float(np.float32(gamma)), x.astype(np.float64))
    np.testing.assert_allclose(xo.cpu().numpy(), ref, rtol=1e-5, atol=0)


def test_rows_and_columns_equal_the_rook_step(gpu):
    """Rows and columns as hyperedges: the same step as gn_rook_step on the board."""
    import torch
    libgn = _lib()
    N = 40
    ptr, mem = _rook_hyperedges(N)
    w, _ = inputs.rook_weights(N, 3)
    x = inputs.rng_for(3, 22).random(N * N, dtype=np.float32)
    H = libgn.Hyper(N * N, ptr, mem, w)
    R = libgn.Rook(N, N, w)
    xi = torch.from_numpy(x).cuda()
    a, b = torch.empty_like(xi), torch.empty_like(xi)
    H.step(1.2, xi, a)
    R.step(1.2, xi, b)
    np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-5, atol=0)


@pytest.mark.parametrize("case,check_every", [("routes2000", 1), ("long500", 1), ("rook24", 1), ("routes2000", 8)])
def test_solve_matches_oracle(gpu, case, check_every):
    import torch
    libgn = _lib()
    n, ptr, mem = _cases()[case]
    w = inputs.weights_uniform01(n, 6)
    H = libgn.Hyper(n, ptr, mem, w)
    x = torch.full((n,), 0.5, device="cuda")
    sel = torch.zeros(n, dtype=torch.uint8, device="cuda")
    sched = dict(gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=3000, tau=1e-4, check_every=check_every)
    res = H.solve(x, sel, **sched)
    ref = OH.solve(n, ptr, mem, w.astype(np.float64), np.full(n, 0.5),
                   **dict(sched, gamma0=float(np.float32(0.9))))
    assert res.binarised and ref.binarised
    assert abs(res.steps - ref.steps) <= 2 * check_every, (res.steps, ref.steps)
    if check_every > 1:
        assert res.steps % check_every == 0
    s = sel.cpu().numpy().astype(bool)
    assert np.array_equal(s, ref.sel)
    assert np.array_equal(s, x.cpu().numpy() > 0.5)
    assert res.set_objective == pytest.approx(ref.set_objective, rel=1e-12)
    assert res.set_size == ref.set_size and res.conflicts == ref.conflicts == 0
    assert res.uncovered == ref.uncovered == 0
    assert res.relaxed_objective == pytest.approx(ref.relaxed_objective, rel=1e-5)
    assert res.stab == pytest.approx(ref.stab, rel=1e-5)


def test_solve_independent_of_chain_length(gpu):
    """The steps run in captured chains with a progress mark before each
    chain's end; the chain length moves only where the host looks: every
    start's steps, states, sets and statistics are the same bits, for one
    start and for five, also when the budget ends the solve and when one
    handle's chains are rebuilt for another schedule."""
    import torch
    libgn = _lib()
    n, ptr, mem = _cases()[list(_cases())[0]]
    w = inputs.weights_uniform01(n, 8)
    H = libgn.Hyper(n, ptr, mem, w)
    u = 1.0 - inputs.rng_for(8, 29).random((5, n))
    x0 = np.clip(u, 1e-3, 1.0).astype(np.float32).reshape(-1)
    outs = {}
    try:
        for C in (64, 1, 8, 9, 100):
            libgn.gn_set_chunk_len(C)
            for ms in (3000, 23):
                for starts in (1, 5):
                    x = torch.from_numpy(x0[:starts * n].copy()).cuda()
                    sel = torch.zeros(starts * n, dtype=torch.uint8, device="cuda")
                    st, res, best = H.multi_solve(starts, x, sel, max_steps=ms)
                    key = (ms, starts)
                    o = ([(r.steps, r.binarised, r.fallback_count, r.set_objective, r.relaxed_objective, r.stab)
                          for r in res], x.cpu().numpy().view(np.uint32), sel.cpu().numpy())
                    if key not in outs:
                        outs[key] = o
                        continue
                    assert o[0] == outs[key][0], (C, key)
                    assert np.array_equal(o[1], outs[key][1]) and np.array_equal(o[2], outs[key][2])
    finally:
        libgn.gn_set_chunk_len(libgn.CHUNK_LEN_DEFAULT)
    assert max(r[0] for r in outs[(3000, 5)][0]) > 64
    assert all(r[0] == 23 and not r[1] for r in outs[(23, 1)][0])


def test_solve_cut_by_max_steps(gpu):
    import torch
    libgn = _lib()
    n, ptr, mem = _cases()["routes2000"]
    w = inputs.weights_uniform01(n, 6)
    H = libgn.Hyper(n, ptr, mem, w)
    x = torch.full((n,), 0.5, device="cuda")
    sel = torch.zeros(n, dtype=torch.uint8, device="cuda")
    res = H.solve(x, sel, max_steps=150)
    ref = OH.solve(n, ptr, mem, w.astype(np.float64), np.full(n, 0.5), gamma0=float(np.float32(0.9)),
                   max_steps=150)
    assert not res.binarised and not ref.binarised and res.steps == 150 == ref.steps
    np.testing.assert_allclose(x.cpu().numpy(), ref.x, rtol=1e-3, atol=1e-6)
    assert res.status == libgn.GN_NOT_CONVERGED


def test_solve_input_errors(gpu):
    import torch
    libgn = _lib()
    H = libgn.Hyper(3, np.array([0, 2, 3]), np.array([0, 1, 2]), np.ones(3, np.float32))
    sel = torch.zeros(3, dtype=torch.uint8, device="cuda")
    with pytest.raises(libgn.GNError) as e:
        H.solve(torch.tensor([0.5, float("nan"), 0.5], device="cuda"), sel)
    assert e.value.status == libgn.GN_E_ARG
    with pytest.raises(libgn.GNError) as e:
        H.solve(torch.tensor([0.5, 0.5, 0.0], device="cuda"), sel)  # vertex 2 alone with no mass
    assert e.value.status == libgn.GN_E_NOT_NORMALIZABLE
    x = torch.full((3,), 0.5, device="cuda")
    with pytest.raises(libgn.GNError):
        H.step(-1.0, x, torch.empty_like(x))
    with pytest.raises(libgn.GNError):
        H.step(1.0, x, x)


@pytest.mark.parametrize("n,ptr,mem,w", [
    (1, [0, 1], [0], [0.7]),                          # one vertex: selected at the first check, stab +inf
    (3, [0, 3], [0, 1, 2], [0.2, 0.9, 0.5]),          # one hyperedge: the heaviest vertex wins
    (4, [0, 1, 2, 3, 4], [0, 1, 2, 3], [0.3, 0.6, 0.9, 0.1]),  # singletons only: everything selected
])
def test_degenerate_instances(gpu, n, ptr, mem, w):
    import torch
    libgn = _lib()
    w = np.asarray(w, np.float32)
    H = libgn.Hyper(n, np.asarray(ptr), np.asarray(mem), w)
    x = torch.full((n,), 0.5, device="cuda")
    sel = torch.zeros(n, dtype=torch.uint8, device="cuda")
    res = H.solve(x, sel)
    ref = OH.solve(n, np.asarray(ptr), np.asarray(mem), w.astype(np.float64), np.full(n, 0.5),
                   gamma0=float(np.float32(0.9)))
    assert res.binarised and ref.binarised and abs(res.steps - ref.steps) <= 2
    assert np.array_equal(sel.cpu().numpy().astype(bool), ref.sel)
    assert res.set_objective == pytest.approx(ref.set_objective, rel=1e-12)
    if np.isinf(ref.stab):
        assert np.isinf(res.stab)
    else:
        assert res.stab == pytest.approx(ref.stab, rel=1e-5)


@pytest.mark.parametrize("case,starts", [("routes2000", 16), ("long500", 5)])
def test_multi_solve_matches_single_starts(gpu, case, starts):
    """Every start of a multi-start solve is the single-start solve from its
    point: the oracle's set and W(S), steps within 2; best is the heaviest
    binarised start."""
    import torch
    libgn = _lib()
    n, ptr, mem = _cases()[case]
    w = inputs.weights_uniform01(n, 7)
    H = libgn.Hyper(n, ptr, mem, w)
    u = 1.0 - inputs.rng_for(7, 23).random((starts, n))
    e = -np.log(u)
    x0 = np.clip(e / e.max(axis=1, keepdims=True), 1e-3, 1.0).astype(np.float32)
    x = torch.from_numpy(x0.reshape(-1)).cuda()
    sel = torch.zeros(starts * n, dtype=torch.uint8, device="cuda")
    st, res, best = H.multi_solve(starts, x, sel, max_steps=3000)
    s_all = sel.cpu().numpy().reshape(starts, n).astype(bool)
    for b in range(starts):
        ref = OH.solve(n, ptr, mem, w.astype(np.float64), x0[b].astype(np.float64), gamma0=float(np.float32(0.9)),
                       max_steps=3000)
        assert res[b].binarised == ref.binarised and abs(res[b].steps - ref.steps) <= 2
        assert np.array_equal(s_all[b], ref.sel)
        assert res[b].set_objective == pytest.approx(ref.set_objective, rel=1e-12)
    objs = [r.set_objective if r.binarised else -1 for r in res]
    assert best == int(np.argmax(objs))
    # one start through the multi-start call equals the single-start call
    x1 = torch.from_numpy(x0[3 % starts].copy()).cuda()
    s1 = torch.zeros(n, dtype=torch.uint8, device="cuda")
    r1 = H.solve(x1, s1, max_steps=3000)
    assert r1.steps == res[3 % starts].steps and r1.set_objective == res[3 % starts].set_objective
    assert np.array_equal(s1.cpu().numpy().astype(bool), s_all[3 % starts])

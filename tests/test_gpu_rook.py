"""Parity of the assignment solver (matrix cross-normalization, Section 2) with
the fp64 oracle run on the same graph in CSR form (the line graph of
K_{rows,cols}), through the C-ABI.

Tolerances:
  one step  |x_gpu - x_ref| <= 1e-5 |x_ref| + 1e-7.  The row and column sums are
            accumulated in fp64 and the neighbour sum (R_i - y) + (C_j - y) is
            rounded once to fp32, so the step's error is a few fp32 roundings,
            well inside the CSR step's bound.
  solve     identical assignments, steps within 2 of the oracle (the stopping test
            is a float decision on trajectories computed in different
            precisions), set objective equal to 1e-12 relative.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_05330_amd import inputs as I

pytestmark = pytest.mark.gpu

F32 = np.float32
RAMP = dict(gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=2000, tau=1e-4, check_every=1)


def _lib():
    from paper_2605_05330_amd import libgn
    return libgn


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _state(n, seed, zeros=0.0):
    r = I.rng_for(seed, 78)
    x = r.random(n) * 0.98 + 0.01
    if zeros:
        x[r.random(n) < zeros] = 0.0
    return x.astype(F32)


def _oracle_sched(s):
    o = dict(s)
    for k in ("gamma0", "gamma1", "tau"):
        o[k] = float(F32(o[k]))
    return o


def _step_parity(rows, cols, w, gamma, x):
    import torch
    R = _lib().Rook(rows, cols, w)
    xd = dev(x)
    out = torch.empty_like(xd)
    R.step(F32(gamma), xd, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    g = I.rook_rect(rows, cols)
    ref, _ = O.step(g.n, g.row_ptr, g.col_idx, w.reshape(-1).astype(np.float64), float(F32(gamma)),
                    x.astype(np.float64))
    bad = np.abs(got - ref) > 1e-5 * np.abs(ref) + 1e-7
    assert not bad.any(), (np.flatnonzero(bad)[:10], got[bad][:5], ref[bad][:5])
    return got, ref


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (5, 9), (16, 64), (17, 65), (37, 53), (70, 130)])
def test_step_matches_oracle(gpu, shape):
    """Single tiles, ragged tiles in both directions, several tiles of each kind."""
    rows, cols = shape
    w = I.rook_weights_rect(rows, cols, rows * 1000 + cols)
    for gamma in (0.9, 1.5):
        _step_parity(rows, cols, w, gamma, _state(rows * cols, rows + cols, zeros=0.1))


def test_step_single_row_is_simplex_projection(gpu):
    """1 x n: the graph is K_n, and at gamma = 1 one step gives x' = y / sum(y) in
    weighted space (the K_n case of Section 2)."""
    n = 40
    w = I.rook_weights_rect(1, n, 3)
    x = _state(n, 3)
    got, _ = _step_parity(1, n, w, 1.0, x)
    y = np.sqrt(w.reshape(-1).astype(np.float64)) * x
    np.testing.assert_allclose(got, y / y.sum(), rtol=1e-5, atol=1e-7)


def test_step_fallback_and_zero_support(gpu):
    """An all-zero row and column: the entry at their crossing has a zero closed
    neighbourhood and takes 1/2; the other zeros of that row and column stay 0."""
    rows, cols = 6, 5
    w = I.rook_weights_rect(rows, cols, 4)
    x = _state(rows * cols, 4).reshape(rows, cols)
    x[2, :] = 0.0
    x[:, 3] = 0.0
    got, ref = _step_parity(rows, cols, w, 1.3, x.reshape(-1))
    got = got.reshape(rows, cols)
    assert got[2, 3] == 0.5
    assert np.all(np.delete(got[2, :], 3) == 0.0) and np.all(np.delete(got[:, 3], 2) == 0.0)


def test_step_full_size_256(gpu):
    """The 256 x 256 assignment instance, every entry, against the oracle's CSR step
    on the 33.4M-entry rook graph."""
    w, _ = I.rook_weights(256, 0)
    _step_parity(256, 256, w.reshape(256, 256), 1.2, _state(256 * 256, 9))


def test_step_4096_sampled_entries(gpu):
    """The benchmark's 4096 x 4096 instance (split form), one step from a random
    state: 24 sampled entries against the oracle's step on each entry's star graph
    (the entry and its 8190 row and column mates), whose centre sees exactly its
    closed neighbourhood in the full instance."""
    import torch
    N = 4096
    w = I.rook_weights_rect(N, N, 0)
    x = _state(N * N, 21, zeros=0.05)
    R = _lib().Rook(N, N, w)
    xd = dev(x)
    out = torch.empty_like(xd)
    gamma = F32(1.3)
    R.step(gamma, xd, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    wf, xf = w.reshape(-1).astype(np.float64), x.astype(np.float64)
    rng = I.rng_for(22, 79)
    for _ in range(24):
        i, j = (int(t) for t in rng.integers(0, N, size=2))
        mates = np.concatenate([i * N + np.delete(np.arange(N), j), np.delete(np.arange(N), i) * N + j])
        ids = np.concatenate([[i * N + j], mates])
        m = len(mates)
        rp = np.concatenate([[0, m], m + np.arange(1, m + 1)]).astype(np.int32)
        ci = np.concatenate([np.arange(1, m + 1), np.zeros(m)]).astype(np.int32)
        ref, _ = O.step(m + 1, rp, ci, wf[ids], float(gamma), xf[ids])
        e = i * N + j
        assert abs(got[e] - ref[0]) <= 1e-5 * abs(ref[0]) + 1e-7, (i, j, got[e], ref[0])


def _solve(rows, cols, w, x0, **sch):
    import torch
    R = _lib().Rook(rows, cols, w)
    x = dev(np.asarray(x0, F32))
    sel = torch.zeros(rows * cols, dtype=torch.uint8, device="cuda")
    res = R.solve(x, sel, **sch)
    return res, x.cpu().numpy(), sel.cpu().numpy().astype(bool)


@pytest.mark.parametrize("shape", [(8, 8), (16, 16), (33, 33), (48, 48), (12, 20), (20, 12), (33, 70)])
def test_solve_matches_oracle(gpu, shape):
    rows, cols = shape
    w = I.rook_weights_rect(rows, cols, 7 * rows + cols)
    res, x, sel = _solve(rows, cols, w, np.full(rows * cols, 0.5), **RAMP)
    g = I.rook_rect(rows, cols)
    ref = O.solve(g.n, g.row_ptr, g.col_idx, w.reshape(-1).astype(np.float64), np.full(g.n, 0.5),
                  **_oracle_sched(RAMP))
    assert res.binarised and ref.binarised
    assert abs(res.steps - ref.steps) <= 2, (res.steps, ref.steps)
    assert np.array_equal(sel, ref.sel)
    assert res.conflicts == 0 and res.uncovered == 0
    assert res.set_size == min(rows, cols)
    S = sel.reshape(rows, cols)
    assert np.all(S.sum(axis=1) <= 1) and np.all(S.sum(axis=0) <= 1)
    assert res.set_objective == pytest.approx(ref.set_objective, rel=1e-12)
    assert res.stab == pytest.approx(ref.stab, rel=1e-5)


def test_solve_256_matches_csr_path(gpu):
    """At full size: the structured solver and the CSR solver on the rook graph
    reach the same permutation within 2 steps."""
    import torch
    w, _ = I.rook_weights(256, 0)
    res, x, sel = _solve(256, 256, w.reshape(256, 256), np.full(256 * 256, 0.5), **RAMP)
    g = I.rook(256)
    G = _lib().Graph(g.n, g.row_ptr, g.col_idx, w)
    xc = dev(np.full(g.n, 0.5, F32))
    sc = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
    rc = G.solve(xc, sc, **RAMP)
    assert res.binarised and rc.binarised
    assert abs(res.steps - rc.steps) <= 2, (res.steps, rc.steps)
    assert np.array_equal(sel, sc.cpu().numpy().astype(bool))
    P = sel.reshape(256, 256)
    assert np.all(P.sum(axis=0) == 1) and np.all(P.sum(axis=1) == 1)
    assert res.set_objective == pytest.approx(rc.set_objective, rel=1e-12)


def test_solve_fixed_steps_relaxed_objective(gpu):
    """tau = 0 never passes: after exactly 150 steps the relaxed objective matches
    the oracle to 1e-6 relative."""
    rows, cols = 24, 40
    w = I.rook_weights_rect(rows, cols, 5)
    S = dict(RAMP, max_steps=150, tau=0.0)
    res, x, sel = _solve(rows, cols, w, np.full(rows * cols, 0.5), **S)
    g = I.rook_rect(rows, cols)
    ref = O.solve(g.n, g.row_ptr, g.col_idx, w.reshape(-1).astype(np.float64), np.full(g.n, 0.5),
                  **_oracle_sched(S))
    assert not res.binarised and res.steps == 150 and ref.steps == 150
    assert res.relaxed_objective == pytest.approx(ref.relaxed_objective, rel=1e-6)
    np.testing.assert_allclose(x, ref.x, rtol=1e-4, atol=1e-6)


def test_solve_is_deterministic(gpu):
    rows, cols = 40, 40
    w = I.rook_weights_rect(rows, cols, 6)
    a = _solve(rows, cols, w, np.full(rows * cols, 0.5), **RAMP)
    b = _solve(rows, cols, w, np.full(rows * cols, 0.5), **RAMP)
    assert a[0].steps == b[0].steps and np.array_equal(a[1], b[1])


def test_solve_independent_of_chain_length(gpu):
    """The chain length moves only the progress marks the host waits on (at
    step 0 of every chain when it is 8 or less): steps, states and sets are
    identical, also when the budget ends the solve."""
    libgn = _lib()
    rows, cols = 40, 56
    w = I.rook_weights_rect(rows, cols, 17)
    outs = []
    try:
        for C in (64, 1, 8, 9, 33, 500):
            libgn.gn_set_chunk_len(C)
            for ms in (2000, 37):
                r, x, sel = _solve(rows, cols, w, np.full(rows * cols, 0.5), **dict(RAMP, max_steps=ms))
                outs.append((C, ms, r.steps, r.binarised, r.fallback_count, r.set_objective, x.view(np.uint32), sel))
    finally:
        libgn.gn_set_chunk_len(libgn.CHUNK_LEN_DEFAULT)
    ref = {o[1]: o for o in outs[:2]}
    assert ref[2000][3] and ref[2000][2] > 64 and not ref[37][3] and ref[37][2] == 37
    for o in outs[2:]:
        b = ref[o[1]]
        assert o[2:6] == b[2:6], (o[0], o[1])
        assert np.array_equal(o[6], b[6]) and np.array_equal(o[7], b[7])


def test_errors(gpu):
    libgn = _lib()
    with pytest.raises(libgn.GNError) as e:
        libgn.Rook(3, 3, np.array([1, 1, 1, 1, -1, 1, 1, 1, 1], F32))
    assert e.value.status == libgn.GN_E_WEIGHT
    with pytest.raises(libgn.GNError) as e:
        libgn.Rook(0, 3, np.zeros(0, F32))
    assert e.value.status == libgn.GN_E_ARG
    rows, cols = 5, 6
    w = I.rook_weights_rect(rows, cols, 2)
    x0 = np.full((rows, cols), 0.5, F32)
    x0[1, :] = 0.0
    x0[:, 4] = 0.0
    with pytest.raises(libgn.GNError) as e:
        _solve(rows, cols, w, x0.reshape(-1), **RAMP)
    assert e.value.status == libgn.GN_E_NOT_NORMALIZABLE
    x1 = np.full(rows * cols, 0.5, F32)
    x1[7] = -0.1
    with pytest.raises(libgn.GNError) as e:
        _solve(rows, cols, w, x1, **RAMP)
    assert e.value.status == libgn.GN_E_ARG


# large enough that each step runs as a reduction kernel plus the step kernel: with
# 32 x 64 tiles the tiles' re-reads of the partial sums exceed 16 bytes per entry
# when cols / 2 + 2 rows > 4096
SPLIT = (2100, 12)
assert SPLIT[1] / 2 + 2 * SPLIT[0] > 4096


def test_step_split_form_matches_oracle(gpu):
    rows, cols = SPLIT
    w = I.rook_weights_rect(rows, cols, 11)
    _step_parity(rows, cols, w, 1.1, _state(rows * cols, 11, zeros=0.05))


def test_solve_split_form_matches_csr_path(gpu):
    """The split form against the CSR solver on the same 53.2M-entry rook graph."""
    import torch
    rows, cols = SPLIT
    w = I.rook_weights_rect(rows, cols, 12)
    res, x, sel = _solve(rows, cols, w, np.full(rows * cols, 0.5), **RAMP)
    g = I.rook_rect(rows, cols)
    G = _lib().Graph(g.n, g.row_ptr, g.col_idx, w.reshape(-1))
    xc = dev(np.full(g.n, 0.5, F32))
    sc = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
    rc = G.solve(xc, sc, **RAMP)
    assert res.binarised and rc.binarised
    assert abs(res.steps - rc.steps) <= 2, (res.steps, rc.steps)
    assert np.array_equal(sel, sc.cpu().numpy().astype(bool))
    S = sel.reshape(rows, cols)
    assert res.set_size == cols and np.all(S.sum(axis=0) == 1) and np.all(S.sum(axis=1) <= 1)
    assert res.conflicts == 0 and res.uncovered == 0
    assert res.set_objective == pytest.approx(rc.set_objective, rel=1e-12)


def test_device_weights_and_zero_steps(gpu):
    """Weights handed over in device memory give the same instance; max_steps = 0
    returns the starting point, rounded, as not binarised."""
    import torch
    libgn = _lib()
    rows, cols = 20, 30
    w = I.rook_weights_rect(rows, cols, 13)
    a = _solve(rows, cols, w, np.full(rows * cols, 0.5), **RAMP)
    R = libgn.Rook(rows, cols, dev(w))
    x = dev(np.full(rows * cols, 0.5, F32))
    sel = torch.zeros(rows * cols, dtype=torch.uint8, device="cuda")
    r = R.solve(x, sel, **RAMP)
    assert r.steps == a[0].steps and np.array_equal(x.cpu().numpy(), a[1])
    x0 = _state(rows * cols, 14)
    res, x, sel = _solve(rows, cols, w, x0, **dict(RAMP, max_steps=0))
    assert res.steps == 0 and not res.binarised
    np.testing.assert_allclose(x, x0, rtol=1e-6, atol=0)  # |v x| / v: one rounding away from x0
    assert np.array_equal(sel, x0 > 0.5)

"""Parity of the HIP path (through the C-ABI) with the fp64 oracle.

Tolerances (fp32 kernel vs fp64 oracle):
  one step  |x_gpu - x_ref| <= 1e-5 |x_ref| + 1e-7, both from the same fp32 input.
            The neighbour sum is fp32 in the canonical 64-lane order: a lane adds at
            most ceil(deg/64) positive terms sequentially and the butterfly adds 6
            levels, so its relative error is below (ceil(deg/64) + 6) 2^-24 < 1e-5
            for every degree used here (<= 9001), plus a few roundings in the
            epilogue.
  solve     identical rounded sets on seeds whose trajectory has no near-tie, set
            objective equal to 1e-12 relative (same set, fp64 sums in different
            orders), steps within 2 of the oracle (the stopping test is a float
            decision on trajectories computed in different precisions),
            independence and maximality exact.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_05330_amd import inputs as I

pytestmark = pytest.mark.gpu

F32 = np.float32


def _lib():
    from paper_2605_05330_amd import libgn
    return libgn


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _graph(g, w):
    return _lib().Graph(g.n, g.row_ptr, g.col_idx, np.asarray(w, F32))


def _step_parity(g, w, gamma, x):
    import torch
    G = _graph(g, w)
    x32 = np.asarray(x, F32)
    xd = dev(x32)
    out = torch.empty_like(xd)
    G.step(F32(gamma), xd, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref, fb = O.step(g.n, g.row_ptr, g.col_idx, np.asarray(w, F32).astype(np.float64), float(F32(gamma)),
                     x32.astype(np.float64))
    err = np.abs(got - ref)
    bad = err > 1e-5 * np.abs(ref) + 1e-7
    assert not bad.any(), (np.flatnonzero(bad)[:10], got[bad][:5], ref[bad][:5])
    return got, ref


def _rand_state(n, seed, zeros=0.0):
    r = I.rng_for(seed, 77)
    x = r.random(n) * 0.98 + 0.01
    if zeros:
        x[r.random(n) < zeros] = 0.0
    return x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_step_er1000(gpu, seed):
    g = I.erdos_renyi(1000, 8 / 999, seed)
    w = I.weights_uniform01(1000, seed)
    for gamma in (0.9, 1.5):
        _step_parity(g, w, gamma, _rand_state(1000, seed, zeros=0.05))


def test_step_all_bins_ragged(gpu):
    """Degrees 0 .. 9001: every bin, multi-chunk LDS staging (> 4096), partial tail
    blocks in every bin."""
    g = I.hub_graph(12000, [10, 20, 40, 100, 300, 600, 1500, 5000, 9000], 3.0, 1)
    w = I.weights_uniform01(g.n, 1)
    info = _graph(g, w).info()
    assert all(v > 0 for k, v in info["bins"].items() if not k.startswith("unused")), info
    _step_parity(g, w, 1.3, _rand_state(g.n, 4, zeros=0.1))


def test_step_degree_sweep(gpu):
    """Every degree 0..130 and a few bin edges: a union of stars, one per degree."""
    degs = list(range(0, 131)) + [511, 512, 513, 4095, 4096, 4097]
    src, dst, off = [], [], 0
    for d in degs:
        src += [off] * d
        dst += list(range(off + 1, off + 1 + d))
        off += d + 1
    g = I.csr_from_edges(off, np.array(src), np.array(dst))
    w = I.weights_uniform01(g.n, 5)
    _step_parity(g, w, 1.1, _rand_state(g.n, 5))


def test_step_fallback_and_zero_support(gpu):
    """Safe division: nodes with an all-zero closed neighbourhood take 1/2; zeros with
    a positive neighbour stay 0 (support invariance)."""
    g = I.csr_from_edges(6, np.array([0, 1, 3]), np.array([1, 2, 4]))
    w = np.array([1, 2, 0.5, 1, 1, 3], F32)
    got, ref = _step_parity(g, w, 1.5, np.array([0.0, 0.4, 0.7, 0.0, 0.0, 0.9]))
    assert got[3] == 0.5 and got[4] == 0.5 and got[0] == 0.0 and got[5] == 1.0


def test_step_full_size_ba_and_rook(gpu):
    """Full-size one-step parity on the two at-scale workloads, all rows."""
    g = I.barabasi_albert(200_000, 5, 0)
    w = I.weights_uniform01(g.n, 0)
    _step_parity(g, w, 1.2, _rand_state(g.n, 8))
    r = I.rook(256)
    wr, _ = I.rook_weights(256, 0)
    _step_parity(r, wr, 1.2, _rand_state(r.n, 9))


def test_step_scale_invariance_bit_exact(gpu):
    """Section 2 property iv on the GPU: scaling x by 2^k gives bit-identical output."""
    import torch
    g = I.barabasi_albert(20_000, 4, 3)
    w = I.weights_uniform01(g.n, 3)
    G = _graph(g, w)
    x = dev(np.asarray(_rand_state(g.n, 3), F32))
    a, b = torch.empty_like(x), torch.empty_like(x)
    G.step(1.4, x, a)
    G.step(1.4, x * 8.0, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _solve_both(g, w, x0, **sch):
    import torch
    G = _graph(g, w)
    x = dev(np.asarray(x0, F32))
    sel = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
    res = G.solve(x, sel, **sch)
    osch = dict(sch)
    for k in ("gamma0", "gamma1", "tau"):
        if k in osch:
            osch[k] = float(F32(osch[k]))
    ref = O.solve(g.n, g.row_ptr, g.col_idx, np.asarray(w, F32).astype(np.float64),
                  np.asarray(x0, F32).astype(np.float64), **osch)
    return G, res, x.cpu().numpy(), sel.cpu().numpy().astype(bool), ref


SCHED_RAMP = dict(gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=2000, tau=1e-4, check_every=1)
SCHED_CONST = dict(gamma0=1.5, gamma1=1.5, ramp_steps=1, max_steps=2000, tau=1e-4, check_every=1)
PATHS = ["small", "chained"]


class _path:
    """gn_solve's two paths: "small" runs graphs up to the default work limit in
    one workgroup; "chained" (limit 0) runs every step as a launch of the fused
    step kernel, with its lagged stopping test, in replayed chains."""

    def __init__(self, which):
        self.limit = 0 if which == "chained" else None

    def __enter__(self):
        if self.limit is not None:
            _lib().gn_set_small_graph_limit(self.limit)

    def __exit__(self, *exc):
        lg = _lib()
        lg.gn_set_small_graph_limit(lg.SMALL_LIMIT_DEFAULT)


def _assert_solve_matches(res, x, sel, ref, steps_tol=2):
    assert res.binarised and ref.binarised
    assert res.conflicts == 0 and res.uncovered == 0
    assert abs(res.steps - ref.steps) <= steps_tol, (res.steps, ref.steps)
    assert np.array_equal(sel, ref.sel), int(np.sum(sel != ref.sel))
    assert res.set_objective == pytest.approx(ref.set_objective, rel=1e-12)
    assert res.set_size == int(ref.sel.sum())
    assert res.stab == pytest.approx(ref.stab, rel=1e-5)
    # final state within the stopping tolerance of the oracle's; S is its rounding
    assert np.max(np.abs(x - ref.x)) <= 2e-4
    assert np.array_equal(sel, x > 0.5)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("sched", ["ramp", "const"])
def test_solve_er1000(gpu, seed, sched, path):
    """ER n=1000, average degree 8, w uniform (0,1], x0 = 1/2, on both solve paths."""
    g = I.erdos_renyi(1000, 8 / 999, seed)
    w = I.weights_uniform01(1000, seed)
    S = SCHED_RAMP if sched == "ramp" else SCHED_CONST
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, w, np.full(1000, 0.5), **S)
    _assert_solve_matches(res, x, sel, ref)


@pytest.mark.parametrize("path", PATHS)
def test_solve_regrowth_from_deep_decay(gpu, path):
    """ER n=1500 (seed 109): vertices decay below 2^-300 while a neighbour holds the
    set and later regrow to replace it; the plain map needs 1459 steps here (a
    floor at 2^-100 would stop at 498).  The GPU carries those states in log form
    and must follow the same trajectory to the same set."""
    g = I.erdos_renyi(1500, 6 / 1499, 109)
    w = I.weights_uniform01(1500, 109)
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, w, np.full(1500, 0.5), **SCHED_RAMP)
    assert ref.steps == 1459
    _assert_solve_matches(res, x, sel, ref)
    assert sel[775] and not sel[276]


@pytest.mark.parametrize("path", PATHS)
def test_solve_same_steps_gives_same_relaxed_objective(gpu, path):
    """With the number of steps fixed (tau = 0 never passes), the relaxed objective
    after K steps matches the oracle to 1e-6 relative."""
    g = I.erdos_renyi(1000, 8 / 999, 11)
    w = I.weights_uniform01(1000, 11)
    S = dict(gamma0=0.9, gamma1=1.5, ramp_steps=1000, max_steps=150, tau=0.0, check_every=1)
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, w, np.full(1000, 0.5), **S)
    assert not res.binarised and res.steps == 150 and ref.steps == 150
    assert res.relaxed_objective == pytest.approx(ref.relaxed_objective, rel=1e-6)


@pytest.mark.parametrize("path", PATHS)
def test_solve_check_every(gpu, path):
    g = I.erdos_renyi(1000, 8 / 999, 2)
    w = I.weights_uniform01(1000, 2)
    S = dict(SCHED_CONST, check_every=8)
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, w, np.full(1000, 0.5), **S)
    assert res.binarised and res.steps % 8 == 0 and ref.steps % 8 == 0
    _assert_solve_matches(res, x, sel, ref, steps_tol=8)


def test_solve_ba200k_matches_oracle(gpu):
    """Barabasi-Albert n=200,000, m=5, gamma-pursuit: the at-scale plain-GN workload
    (881 steps of the plain map; vertices pass through the log form and one takes
    the safe-division reset)."""
    g = I.barabasi_albert(200_000, 5, 0)
    w = I.weights_uniform01(g.n, 0)
    G, res, x, sel, ref = _solve_both(g, w, np.full(g.n, 0.5), **SCHED_RAMP)
    assert ref.steps == 881
    _assert_solve_matches(res, x, sel, ref)


@pytest.mark.parametrize("kind", ["er", "ud"])
def test_solve_100k_matches_oracle(gpu, kind):
    """Above the single-workgroup limit (the chained fused-step path): ER n=100,000,
    average degree 6 (715 steps), and a unit-disk graph n=100,000, degree 10 (844
    steps), gamma-pursuit."""
    if kind == "er":
        g = I.erdos_renyi(100_000, 6 / 99_999, 31)
    else:
        g = I.unit_disk(100_000, 10, 32)
    w = I.weights_uniform01(g.n, 33)
    G, res, x, sel, ref = _solve_both(g, w, np.full(g.n, 0.5), **SCHED_RAMP)
    _assert_solve_matches(res, x, sel, ref)


def test_step_log_form_states(gpu):
    """One step from states far below 2^-100 (fp32 subnormals included): the GPU keeps
    them in log form; outputs at or above 2^-126 agree with the oracle's x' to
    3e-5 relative (the log form resolves 2^-17 in log2), larger ones to the
    one-step tolerance, and none becomes 0 while the oracle's is above 2^-149."""
    import torch
    g = I.erdos_renyi(4000, 8 / 3999, 12)
    w = I.weights_uniform01(g.n, 12)
    r = I.rng_for(12, 3)
    x = (r.random(g.n) * 0.98 + 0.01).astype(F32)
    tiny = r.random(g.n) < 0.4
    x[tiny] = np.exp2(-r.uniform(90, 148, tiny.sum())).astype(F32)
    G = _graph(g, w)
    xd = dev(x)
    out = torch.empty_like(xd)
    G.step(F32(1.3), xd, out)
    got = out.cpu().numpy().astype(np.float64)
    ref, _ = O.step(g.n, g.row_ptr, g.col_idx, w.astype(np.float64), float(F32(1.3)), x.astype(np.float64))
    deep = ref < 2.0 ** -100
    assert deep.sum() > 500
    norm = ref >= 2.0 ** -126
    rel = np.abs(got - ref) / ref
    assert np.all(rel[norm & deep] <= 3e-5), rel[norm & deep].max()
    assert np.all(rel[~deep] <= 1e-5 + 1e-7 / ref[~deep])
    assert np.all(got[ref > 2.0 ** -149] > 0)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [16, 48])
def test_solve_rook_csr_matches_oracle(gpu, N, path):
    """Assignment instances through the general CSR solver on both paths: the
    oracle's permutation (on 48 x 48 the plain map reaches it after the
    safe-division reset fires once), steps within 2, stab to 1e-5."""
    g = I.rook_rect(N, N)
    w = I.rook_weights_rect(N, N, 7 * N + N).reshape(-1)
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, w, np.full(g.n, 0.5), **SCHED_RAMP)
    _assert_solve_matches(res, x, sel, ref)
    assert res.fallback_count == ref.fallback_count
    P = sel.reshape(N, N)
    assert (P.sum(0) == 1).all() and (P.sum(1) == 1).all()


def test_solve_rook256_permutation(gpu):
    """Assignment instance 256x256: the result is a permutation matrix and the set is
    independent and maximal (properties that hold at any size)."""
    import torch
    r = I.rook(256)
    w, _ = I.rook_weights(256, 0)
    G = _graph(r, w)
    x = torch.full((r.n,), 0.5, device="cuda")
    sel = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    res = G.solve(x, sel, **SCHED_RAMP)
    assert res.binarised and res.conflicts == 0 and res.uncovered == 0
    P = sel.cpu().numpy().reshape(256, 256).astype(int)
    assert (P.sum(0) == 1).all() and (P.sum(1) == 1).all()
    assert res.set_objective == pytest.approx(float(w.astype(np.float64)[P.reshape(-1) == 1].sum()), rel=1e-12)


def test_objective_and_check_vs_oracle(gpu):
    import torch
    g = I.hub_graph(5000, [100, 700, 3000], 6.0, 2)
    w = I.weights_uniform01(g.n, 2)
    G = _graph(g, w)
    x = np.asarray(_rand_state(g.n, 2), F32)
    assert G.objective(dev(x)) == pytest.approx(O.objective(w.astype(np.float64), x.astype(np.float64)),
                                                rel=1e-12)
    rng = I.rng_for(2, 5)
    for p in (0.02, 0.2, 0.6):
        s = (rng.random(g.n) < p).astype(np.uint8)
        assert G.check(dev(s)) == O.check(g.n, g.row_ptr, g.col_idx, s)


@pytest.mark.parametrize("path", PATHS)
def test_solve_edge_cases(gpu, path):
    import torch
    lg = _lib()
    # empty graph
    G0 = lg.Graph(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, F32))
    r0 = G0.solve(torch.zeros(0, device="cuda"), torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert r0.binarised and r0.steps == 0
    # edgeless: one step to all ones
    g = I.csr_from_edges(5, np.zeros(0), np.zeros(0))
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, np.ones(5, F32), np.full(5, 0.3), **SCHED_CONST)
    assert res.binarised and res.steps == ref.steps == 1 and sel.all()
    assert res.stab == ref.stab == np.inf
    # K_2 with equal weights from the symmetric start never binarises
    k2 = I.csr_from_edges(2, np.array([0]), np.array([1]))
    with _path(path):
        G, res, x, sel, ref = _solve_both(k2, np.ones(2, F32), np.full(2, 0.5),
                                          **dict(SCHED_CONST, max_steps=300))
    assert res.status == lg.GN_NOT_CONVERGED and not res.binarised and res.steps == 300
    # max_steps = 0: nothing happens
    g = I.erdos_renyi(50, 0.1, 1)
    with _path(path):
        G, res, x, sel, ref = _solve_both(g, I.weights_uniform01(50, 1), np.full(50, 0.5),
                                          **dict(SCHED_CONST, max_steps=0))
    assert res.steps == 0 and not res.binarised and np.all(x == 0.5)


@pytest.mark.parametrize("path", PATHS)
def test_solve_rejects_bad_x0(gpu, path):
    """A start that is not normalizable, or has a negative entry, fails the
    solve with its status, and neither x nor sel is written (the outcome is
    decided on the device before the final rounding)."""
    import torch
    lg = _lib()
    g = I.csr_from_edges(4, np.array([0, 2]), np.array([1, 3]))
    G = _graph(g, np.ones(4, F32))
    for x0, status in (([0.5, 0.5, 0.0, 0.0], lg.GN_E_NOT_NORMALIZABLE), ([0.5, -0.1, 0.3, 0.3], lg.GN_E_ARG)):
        sel = torch.full((4,), 7, dtype=torch.uint8, device="cuda")
        x = dev(np.array(x0, F32))
        with _path(path), pytest.raises(lg.GNError) as e:
            G.solve(x, sel)
        assert e.value.status == status
        assert torch.equal(x.cpu(), torch.tensor(x0, dtype=torch.float32))  # untouched
        assert torch.equal(sel.cpu(), torch.full((4,), 7, dtype=torch.uint8))
    # the handle still solves afterwards
    x = dev(np.array([0.6, 0.4, 0.4, 0.6], F32))
    sel = torch.zeros(4, dtype=torch.uint8, device="cuda")
    with _path(path):
        r = G.solve(x, sel, **SCHED_RAMP)
    assert r.binarised and sel.cpu().tolist() == [1, 0, 0, 1]


def test_step_rejects_aliasing(gpu):
    import torch
    lg = _lib()
    g = I.erdos_renyi(30, 0.2, 0)
    G = _graph(g, I.weights_uniform01(30, 0))
    x = torch.full((30,), 0.5, device="cuda")
    with pytest.raises(lg.GNError):
        G.step(1.5, x, x)


def test_device_input_graph_create(gpu):
    """gn_graph_create from device-resident CSR + weights gives the same step."""
    import torch
    lg = _lib()
    g = I.erdos_renyi(2000, 6 / 1999, 4)
    w = I.weights_uniform01(g.n, 4)
    Gh = _graph(g, w)
    Gd = lg.Graph(g.n, dev(g.row_ptr), dev(g.col_idx), dev(w))
    x = dev(np.asarray(_rand_state(g.n, 1), F32))
    a, b = torch.empty_like(x), torch.empty_like(x)
    Gh.step(1.2, x, a)
    Gd.step(1.2, x, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(lg.GNError) as e:
        lg.Graph(3, dev(np.array([0, 1, 1, 1], np.int32)), dev(np.array([1], np.int32)), dev(np.ones(3, F32)))
    assert e.value.status == lg.GN_E_ASYMMETRIC


def test_repeat_solve_deterministic(gpu):
    import torch
    g = I.barabasi_albert(50_000, 5, 9)
    w = I.weights_uniform01(g.n, 9)
    G = _graph(g, w)
    outs = []
    for _ in range(2):
        x = torch.full((g.n,), 0.5, device="cuda")
        sel = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
        r = G.solve(x, sel, **SCHED_RAMP)
        outs.append((r, x.cpu(), sel.cpu()))
    assert outs[0][0] == outs[1][0]
    assert torch.equal(outs[0][1], outs[1][1]) and torch.equal(outs[0][2], outs[1][2])


def test_solve_independent_of_chain_length(gpu):
    """The number of step launches per replayed chain changes only how often the
    host looks at the stop flag: steps, states and sets are identical."""
    import torch
    libgn = _lib()
    g = I.erdos_renyi(3000, 7 / 2999, 21)
    w = I.weights_uniform01(g.n, 21)
    G = _graph(g, w)
    outs = []
    libgn.gn_set_small_graph_limit(0)   # every step a launch of the chained path
    try:
        for C in (1, 7, 32, 200):
            libgn.gn_set_chunk_len(C)
            x = dev(np.full(g.n, 0.5, F32))
            sel = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
            r = G.solve(x, sel, **SCHED_RAMP)
            outs.append((r.steps, r.fallback_count, x.cpu().numpy().view(np.uint32), sel.cpu().numpy()))
    finally:
        libgn.gn_set_chunk_len(libgn.CHUNK_LEN_DEFAULT)
        libgn.gn_set_small_graph_limit(libgn.SMALL_LIMIT_DEFAULT)
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[1] == outs[0][1]
        assert np.array_equal(o[2], outs[0][2]) and np.array_equal(o[3], outs[0][3])


def test_solve_independent_of_prune_interval(gpu):
    """How often the pruned lists are rebuilt, and where the chains start
    against those rebuilds, changes only which decayed vertices are still
    gathered: steps, states and sets are the bits of the full lists."""
    import torch
    libgn = _lib()
    g = I.barabasi_albert(20_000, 4, 23)
    w = I.weights_uniform01(g.n, 23)
    G = _graph(g, w)
    outs = []
    libgn.gn_set_small_graph_limit(0)
    try:
        for prune, C, P in ((libgn.PRUNE_NEVER, 32, 64), (libgn.PRUNE_ALWAYS, 7, 64), (libgn.PRUNE_ALWAYS, 32, 1),
                            (libgn.PRUNE_ALWAYS, 24, 64), (libgn.PRUNE_ALWAYS, 64, 16),
                            (libgn.PRUNE_ALWAYS, 9, 4096)):
            libgn.gn_set_pruning(prune)
            libgn.gn_set_chunk_len(C)
            libgn.gn_set_prune_interval(P)
            x = dev(np.full(g.n, 0.5, F32))
            sel = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
            r = G.solve(x, sel, **SCHED_RAMP)
            outs.append((r.steps, r.fallback_count, x.cpu().numpy().view(np.uint32), sel.cpu().numpy()))
    finally:
        libgn.gn_set_chunk_len(libgn.CHUNK_LEN_DEFAULT)
        libgn.gn_set_prune_interval(libgn.PRUNE_INTERVAL_DEFAULT)
        libgn.gn_set_pruning(libgn.PRUNE_WHERE_IT_PAYS)
        libgn.gn_set_small_graph_limit(libgn.SMALL_LIMIT_DEFAULT)
    assert outs[0][0] > 64
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[1] == outs[0][1]
        assert np.array_equal(o[2], outs[0][2]) and np.array_equal(o[3], outs[0][3])


@pytest.mark.parametrize("case", ["er1000", "hubs", "fits3000", "ud2500", "ud3000", "ba3000", "budget",
                                  "check_every"])
def test_small_graph_path_bitexact(gpu, case):
    """gn_solve runs small graphs in one workgroup (one launch, the graph's
    sliced column lines in LDS); forcing either path must give the same steps,
    states, sets, objectives and fallback counts."""
    import torch
    libgn = _lib()
    sch = dict(SCHED_RAMP)
    if case == "er1000":
        g = I.erdos_renyi(1000, 8 / 999, 0)
    elif case == "hubs":
        g = I.hub_graph(1200, [20, 60, 200, 700, 1100], 3.0, 5)  # rows of every class, one above 512
    elif case == "fits3000":
        g = I.erdos_renyi(3000, 6 / 2999, 6)   # CSR staged in LDS
    elif case == "ud2500":
        g = I.unit_disk(2500, 10, 9)
    elif case == "ud3000":
        g = I.unit_disk(3000, 10, 10)         # about 100 KB of LDS image
    elif case == "ba3000":
        g = I.barabasi_albert(3000, 5, 11)    # hubs: rows of degree > 128 in heavy slices
    elif case == "budget":
        g = I.erdos_renyi(900, 8 / 899, 7)
        sch["max_steps"] = 40
    else:
        g = I.erdos_renyi(900, 8 / 899, 8)
        sch["check_every"] = 5
    w = I.weights_uniform01(g.n, 3)
    G = _graph(g, w)
    outs = []
    try:
        for limit in (0, libgn.SMALL_LIMIT_DEFAULT):
            libgn.gn_set_small_graph_limit(limit)
            x = dev(np.full(g.n, 0.5, F32))
            sel = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
            r = G.solve(x, sel, **sch)
            outs.append((r, x.cpu().numpy().view(np.uint32), sel.cpu().numpy()))
    finally:
        libgn.gn_set_small_graph_limit(libgn.SMALL_LIMIT_DEFAULT)
    (ra, xa, sa), (rb, xb, sb) = outs
    assert (ra.steps, ra.binarised, ra.fallback_count) == (rb.steps, rb.binarised, rb.fallback_count)
    assert np.array_equal(xa, xb) and np.array_equal(sa, sb)
    assert ra.set_objective == rb.set_objective and ra.relaxed_objective == rb.relaxed_objective
    assert ra.stab == rb.stab and ra.uncovered == rb.uncovered and ra.conflicts == rb.conflicts
    if case == "budget":
        assert ra.steps == 40 and not ra.binarised


@pytest.mark.parametrize("case", ["regrowth", "hubs", "rook48", "sparse_start", "check_every", "ba200k"])
def test_pruned_lists_same_bits(gpu, case):
    """The chained solve reads pruned neighbour lists (vertices whose state is
    not ordinary dropped from their neighbours' lists, put back when they
    regrow).  With and without them: the same steps, states, sets, objectives,
    stab and fallback counts, bit for bit.  Cases: regrowth from deep decay
    (vertices leave and re-enter the lists), rows of every bin including one
    above 512 (its workgroup rewrites the entries), the 48x48 rook graph (rows of
    degree 94), a start with exact zeros and log-form values (unlisted from the
    first step), a stopping test every 5 steps, and the BA n=200,000 workload."""
    import torch
    libgn = _lib()
    sch = dict(SCHED_RAMP)
    x0 = None
    if case == "regrowth":
        g = I.erdos_renyi(1500, 6 / 1499, 109)
        w = I.weights_uniform01(g.n, 109)
    elif case == "hubs":
        g = I.hub_graph(1200, [20, 60, 200, 700, 1100], 3.0, 5)
        w = I.weights_uniform01(g.n, 3)
    elif case == "rook48":
        g = I.rook(48)
        w, _ = I.rook_weights(48, 48)
    elif case == "sparse_start":
        g = I.erdos_renyi(2000, 8 / 1999, 41)
        w = I.weights_uniform01(g.n, 41)
        rng = np.random.default_rng(41)
        x0 = (1.0 - rng.random(g.n)).astype(F32)
        u = rng.random(g.n)
        x0[u < 0.2] = 0.0
        x0[(u >= 0.2) & (u < 0.4)] = F32(1e-35)
    elif case == "check_every":
        g = I.unit_disk(5000, 10, 42)
        w = I.weights_uniform01(g.n, 42)
        sch = dict(SCHED_CONST, check_every=5)
    else:
        g = I.barabasi_albert(200_000, 5, 0)
        w = I.weights_uniform01(g.n, 0)
    if x0 is None:
        x0 = np.full(g.n, 0.5, F32)
    G = _graph(g, w)
    outs = []
    try:
        libgn.gn_set_small_graph_limit(0)
        for prune in (libgn.PRUNE_ALWAYS, libgn.PRUNE_NEVER):
            libgn.gn_set_pruning(prune)
            x = dev(x0)
            sel = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
            r = G.solve(x, sel, **sch)
            outs.append((r, x.cpu().numpy().view(np.uint32), sel.cpu().numpy()))
    finally:
        libgn.gn_set_pruning(libgn.PRUNE_WHERE_IT_PAYS)
        libgn.gn_set_small_graph_limit(libgn.SMALL_LIMIT_DEFAULT)
    (ra, xa, sa), (rb, xb, sb) = outs
    assert (ra.steps, ra.binarised, ra.fallback_count) == (rb.steps, rb.binarised, rb.fallback_count)
    assert np.array_equal(xa, xb) and np.array_equal(sa, sb)
    assert ra.set_objective == rb.set_objective and ra.relaxed_objective == rb.relaxed_objective
    assert ra.stab == rb.stab and ra.uncovered == rb.uncovered and ra.conflicts == rb.conflicts
    if case == "regrowth":
        assert ra.steps == 1459
    if case == "ba200k":
        assert ra.steps == 881


@pytest.mark.parametrize("gamma", [0.9, 1.5])
def test_relaxed_objective_grows_every_step(gpu, gamma):
    """Mass growth (Theorem 3): at a fixed gamma the weighted mass sum_i w_i x_i
    strictly increases at every step once x is the image of a step.  GPU steps on
    the 1000-vertex ER graph from a random interior start, the mass read with
    gn_objective after each of 60 steps.  It tracks the oracle's sequence to 1e-6
    relative, rises strictly wherever the oracle's rise exceeds 1e-6 relative (fp32
    rounding of x can hide smaller rises), and never falls by more than that."""
    import torch
    g = I.erdos_renyi(1000, 8 / 999, 0)
    w = I.weights_uniform01(g.n, 0)
    G = _lib().Graph(g.n, g.row_ptr, g.col_idx, w)
    x0 = (I.rng_for(0, 3).random(g.n) * 0.9 + 0.05).astype(F32)
    x = dev(x0)
    xr = x0.astype(np.float64)
    wf = w.astype(np.float64)
    F_prev = Fr_prev = None
    strict = 0
    for k in range(60):
        x1 = torch.empty_like(x)
        G.step(F32(gamma), x, x1)
        F = G.objective(x1)
        xr, _ = O.step(g.n, g.row_ptr, g.col_idx, wf, float(F32(gamma)), xr)
        Fr = float(np.dot(wf, xr))
        assert F == pytest.approx(Fr, rel=1e-6), (k, F, Fr)
        if k >= 1:
            assert Fr > Fr_prev, (k, Fr, Fr_prev)          # the invariant itself, in fp64
            if Fr - Fr_prev > 1e-6 * Fr:
                assert F > F_prev, (k, F, F_prev)
                strict += 1
            else:
                assert F >= F_prev - 1e-6 * F, (k, F, F_prev)
        F_prev, Fr_prev, x = F, Fr, x1
    assert strict >= 10

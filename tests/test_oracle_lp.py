"""Pins of the LP warm-start oracle (oracle/lp.py) against facts fixed outside it:
closed forms (softmax of one clique, the edge LP of an odd cycle), LP duality
against an independent LP solver (scipy's HiGHS), brute-force MWIS on perfect
formulations (interval graphs), and the invariants of the colouring."""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.special import softmax

from oracle import lp
from paper_2605_05330_amd import inputs


def cliques(n, groups):
    ptr = np.zeros(len(groups) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(g) for g in groups])
    return lp.Cliques(n, ptr, np.concatenate([np.asarray(sorted(g)) for g in groups]).astype(np.int64))


def lp_optimum(cl, c):
    A = np.zeros((cl.m, cl.n))
    for k in range(cl.m):
        A[k, cl.clique(k)] = 1.0
    r = linprog(-np.asarray(c, float), A_ub=A, b_ub=np.ones(cl.m), bounds=[(0, None)] * cl.n, method="highs")
    assert r.status == 0
    return -r.fun


def brute_mwis(cl, c):
    best = 0.0
    for mask in range(1 << cl.n):
        ok = all(sum((mask >> int(i)) & 1 for i in cl.clique(k)) <= 1 for k in range(cl.m))
        if ok:
            best = max(best, sum(c[i] for i in range(cl.n) if (mask >> i) & 1))
    return best


def run(cl, c, t0=1.0, drop=0.99, t_min=1e-4, passes=2000, check=10, tol=0.0, order=None):
    classes = lp.colour_classes(cl)
    K = int(classes.max()) + 1
    order = list(range(K)) if order is None else order
    return lp.solve(cl, c, t0, order, drop, t_min, passes, check, tol, 0.0, classes)


def test_single_clique_is_softmax():
    """One clique over all vertices: one update leaves x = softmax(c / T), its
    multiplier lam = T log sum exp(c / T), and D = lam."""
    c = np.array([0.3, 0.9, 0.5, 0.2])
    cl = cliques(4, [[0, 1, 2, 3]])
    T = 0.25
    Lam, lam = np.zeros(4), np.zeros(1)
    lp.update_clique(0, cl, c, Lam, lam, T)
    x = np.exp((c - Lam) / T)
    np.testing.assert_allclose(x, softmax(c / T), rtol=1e-14)
    assert lam[0] == pytest.approx(T * np.log(np.exp(c / T).sum()), rel=1e-14)
    D, P, xf = lp.evaluate(cl, c, Lam, lam, T)
    assert D == pytest.approx(lam[0], rel=1e-14)
    assert P == pytest.approx(c @ softmax(c / T), rel=1e-12)
    # annealed: the bound reaches max c, the LP (and MWIS) optimum
    _, res, _, _ = run(cl, c, passes=1500)
    assert res.dual == pytest.approx(0.9, abs=2e-3)


def test_odd_cycle_edge_lp_is_half():
    """Edge constraints of C5 with unit costs: LP* = 5/2 (all halves), above the
    integral optimum 2; the annealed bound and primal both reach 5/2."""
    cl = cliques(5, [[i, (i + 1) % 5] for i in range(5)])
    c = np.ones(5)
    assert lp_optimum(cl, c) == pytest.approx(2.5)
    xf, res, _, _ = run(cl, c, passes=1500)
    assert res.dual == pytest.approx(2.5, abs=5e-3)
    assert res.primal == pytest.approx(2.5, abs=5e-3)
    np.testing.assert_allclose(xf, 0.5, atol=5e-3)


def test_clamp_at_zero():
    """A singleton clique whose vertex is already held below 1 by another clique
    keeps lam = 0 (the projection onto lam >= 0)."""
    cl = cliques(2, [[0, 1], [0]])
    c = np.array([0.1, 1.0])
    T = 0.1
    Lam, lam = np.zeros(2), np.zeros(2)
    lp.update_clique(0, cl, c, Lam, lam, T)
    lp.update_clique(1, cl, c, Lam, lam, T)
    x0 = np.exp((c[0] - Lam[0]) / T)
    assert x0 < 1.0 and lam[1] == 0.0
    # the first update is the two-vertex softmax
    assert x0 == pytest.approx(softmax(c / T)[0], rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_weak_duality_and_convergence(seed):
    """At every check D(lam) >= LP* >= P(xf) and xf is feasible; annealed, D and P
    meet LP* (HiGHS) within 0.5%."""
    inst = inputs.clique_cover_instance(60, 25, 2, 4, seed)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    c = inputs.weights_uniform01(inst.n, seed).astype(np.float64)
    opt = lp_optimum(cl, c)
    classes = lp.colour_classes(cl)
    order = list(range(int(classes.max()) + 1))
    Lam, lam = np.zeros(cl.n), np.zeros(cl.m)
    for p in range(1200):
        T = lp.temperature(1.0, 0.99, 1e-4, p)
        lp.run_pass(cl, c, Lam, lam, classes, order, T)
        if p % 100 == 99:
            D, P, xf = lp.evaluate(cl, c, Lam, lam, T)
            assert D >= opt - 1e-9 and P <= opt + 1e-9
            for k in range(cl.m):
                assert xf[cl.clique(k)].sum() <= 1 + 1e-12
    assert D == pytest.approx(opt, rel=5e-3)
    assert P == pytest.approx(opt, rel=5e-3)


@pytest.mark.parametrize("seed", [0, 1])
def test_interval_graph_reaches_integral_optimum(seed):
    """Interval graphs with their maximal cliques as constraints are a perfect
    formulation: LP* equals the MWIS, found here by brute force."""
    rng = np.random.default_rng(seed)
    n = 12
    lo = rng.uniform(0, 10, n)
    hi = lo + rng.uniform(0.5, 3, n)
    groups = set()
    for pt in np.concatenate([lo, hi]):
        g = tuple(i for i in range(n) if lo[i] <= pt <= hi[i])
        if g:
            groups.add(g)
    groups = [g for g in groups if not any(set(g) < set(h) for h in groups)]
    cl = cliques(n, sorted(groups))
    assert all(any(i in g for g in groups) for i in range(n))
    c = rng.uniform(0.1, 1.0, n)
    best = brute_mwis(cl, c)
    assert lp_optimum(cl, c) == pytest.approx(best, rel=1e-9)
    _, res, _, _ = run(cl, c, passes=1500)
    assert res.dual == pytest.approx(best, rel=5e-3)


def test_colouring_first_fit():
    """Cliques of a class are disjoint, and a clique of class k meets some clique of
    every lower class among the cliques before it (first fit)."""
    inst = inputs.clique_cover_instance(300, 80, 2, 5, 3)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    cls = lp.colour_classes(cl)
    sets = [set(cl.clique(k).tolist()) for k in range(cl.m)]
    for a, b in itertools.combinations(range(cl.m), 2):
        if cls[a] == cls[b]:
            assert not sets[a] & sets[b]
    for k in range(cl.m):
        for q in range(int(cls[k])):
            assert any(cls[j] == q and sets[j] & sets[k] for j in range(k))


def test_order_within_class_is_irrelevant():
    """Updating a class's disjoint cliques in reverse order gives identical numbers."""
    inst = inputs.clique_cover_instance(200, 60, 2, 5, 4)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    c = inputs.weights_uniform01(inst.n, 4).astype(np.float64)
    cls = lp.colour_classes(cl)
    K = int(cls.max()) + 1
    A = (np.zeros(cl.n), np.zeros(cl.m))
    B = (np.zeros(cl.n), np.zeros(cl.m))
    for p in range(5):
        T = lp.temperature(0.5, 0.99, 1e-4, p)
        for r in range(K):
            ks = np.flatnonzero(cls == r)
            for k in ks:
                lp.update_clique(int(k), cl, c, A[0], A[1], T)
            for k in ks[::-1]:
                lp.update_clique(int(k), cl, c, B[0], B[1], T)
    assert np.array_equal(A[0], B[0]) and np.array_equal(A[1], B[1])


def test_stopping_rule():
    """With a gap tolerance the start stops at the first check whose gap is below it."""
    inst = inputs.clique_cover_instance(80, 30, 2, 4, 5)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    c = inputs.weights_uniform01(inst.n, 5).astype(np.float64)
    _, res, _, _ = run(cl, c, passes=3000, check=10, tol=1e-3)
    assert res.converged and res.gap <= 1e-3 and res.passes % 10 == 0
    _, prev, _, _ = run(cl, c, passes=res.passes - 10, check=10, tol=0.0)
    assert prev.gap > 1e-3


def test_bound_at_zero_multipliers_and_first_pass_temperature():
    """With lam = 0 the bound is the sum of the costs; the first pass runs at t0,
    so one pass over a single clique gives softmax(c / t0)."""
    inst = inputs.clique_cover_instance(40, 15, 2, 3, 6)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    c = inputs.weights_uniform01(inst.n, 6).astype(np.float64)
    D, _, _ = lp.evaluate(cl, c, np.zeros(cl.n), np.zeros(cl.m), 1.0)
    assert D == pytest.approx(c.sum(), rel=1e-14)
    one = cliques(3, [[0, 1, 2]])
    c3 = np.array([0.2, 0.7, 0.4])
    xf, res, _, _ = lp.solve(one, c3, 0.37, [0], 0.5, 1e-4, 1, 1, 0.0, 0.0)
    np.testing.assert_allclose(xf, softmax(c3 / 0.37), rtol=1e-13)
    assert res.passes == 1 and res.temperature == 0.37


def test_bound_from_multipliers_is_weak_duality():
    """D(lam) built from the multipliers alone: equal to the incremental form when
    Lam is exactly the sum of its cliques' multipliers, and above LP* (HiGHS) for
    arbitrary nonnegative multipliers, including ones whose incremental Lam has
    drifted."""
    inst = inputs.clique_cover_instance(50, 20, 2, 4, 7)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    c = inputs.weights_uniform01(inst.n, 7).astype(np.float64)
    opt = lp_optimum(cl, c)
    rng = np.random.default_rng(3)
    for _ in range(20):
        lam = rng.exponential(0.2, cl.m) * (rng.random(cl.m) < 0.7)
        Lam = np.zeros(cl.n)
        for k in range(cl.m):
            Lam[cl.clique(k)] += lam[k]
        D_inc, _, _ = lp.evaluate(cl, c, Lam, lam, 0.1)
        assert lp.bound(cl, c, lam) == pytest.approx(D_inc, rel=1e-14)
        assert lp.bound(cl, c, lam) >= opt - 1e-12
        # a drifted Lam (too large) understates the incremental bound; the rebuilt one does not
        D_drift, _, _ = lp.evaluate(cl, c, Lam + 0.5, lam, 0.1)
        assert D_drift < lp.bound(cl, c, lam)


def test_fair_share_lift():
    """One round on a clique of k members at zero gives each 1/k; a vertex takes the
    smallest share of its cliques; the lift never lowers a coordinate and keeps every
    clique sum at most 1."""
    cl = cliques(4, [[0, 1, 2, 3]])
    np.testing.assert_allclose(lp.lift(cl, np.zeros(4), 1), 0.25)
    cl = cliques(3, [[0, 1], [1, 2]])          # slack 1 - 0.2 = 0.8 in each clique
    x = lp.lift(cl, np.array([0.0, 0.2, 0.0]), 1)
    np.testing.assert_allclose(x, [0.4, 0.6, 0.4])
    inst = inputs.clique_cover_instance(80, 30, 2, 5, 4)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    x0 = np.random.default_rng(1).random(inst.n) * 0.05
    for rounds in (1, 2, 5):
        x = lp.lift(cl, x0, rounds)
        assert np.all(x >= x0)
        assert max(x[cl.clique(k)].sum() for k in range(cl.m)) <= 1 + 1e-12
        assert x.sum() > x0.sum()


@pytest.mark.parametrize("seed", [0, 1])
def test_annealed_solve_reaches_a_tenth_of_a_percent(seed):
    """The annealed schedule with best-so-far bounds meets the paper's stop (0.1%):
    D_best >= LP* >= P_best (HiGHS), both within 0.1%, and the warm start is the
    feasible point of P_best."""
    inst = inputs.clique_cover_instance(300, 60, 2, 5, seed)
    cl = lp.Cliques(inst.n, inst.ptr.astype(np.int64), inst.members.astype(np.int64))
    c = inputs.weights_uniform01(inst.n, seed).astype(np.float64)
    opt = lp_optimum(cl, c)
    classes = lp.colour_classes(cl)
    order = list(range(int(classes.max()) + 1))
    trace = []
    x, res, lam, _ = lp.solve(cl, c, 1.0, order, 0.99, 1e-4, 20000, 10, 1e-3, 0.0, classes, trace=trace,
                              anneal_tol=3e-3, stall=10)
    assert res.converged and res.gap <= 1e-3
    assert res.dual >= opt - 1e-9 and res.primal <= opt + 1e-9
    assert res.dual == pytest.approx(lp.bound(cl, c, lam), rel=0.2) or res.dual <= lp.bound(cl, c, lam)
    assert float(c @ x) == pytest.approx(res.primal, rel=1e-12)
    assert max(x[cl.clique(k)].sum() for k in range(cl.m)) <= 1 + 1e-12
    # the best-so-far bounds never move the wrong way
    assert all(b[1] <= a[1] + 1e-15 and b[2] >= a[2] - 1e-15 for a, b in zip(trace, trace[1:]))

"""Pins of the fp64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-derives a value with
the oracle's own formula: they use printed values (``tests/golden``), closed
forms, identities from other theorems, exhaustive search, or textbook
routines, chosen so that a dropped term, a wrong sign or index, or swapped
operands in the oracle fail at least one of them."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from helpers import (best_assignment_bruteforce, bits_to_mask, complete, cycle, dense_adjacency,
                     enumerate_mis, graph_from_edge_tokens, graph_from_edges, hypercube, petersen,
                     read_golden)
from paper_2605_05330_amd import inputs as I


def _step(g, w, gamma, x):
    return O.step(g.n, g.row_ptr, g.col_idx, w, gamma, x)


# ---------------------------------------------------------------- fixed points

def test_printed_fixed_point_7_nodes():
    """Appendix A: the 3-atom fixed point (0,1,0,1,0,1/4,3/4) of the unregularized map."""
    d = read_golden("fixed_point_7.txt")
    g = graph_from_edge_tokens(int(d["n"][0]), d["edges"])
    x = np.array([float(t) for t in d["x"]])
    x1, fb = _step(g, np.ones(g.n), 1.0, x)
    assert fb == 0
    assert np.array_equal(x1, x)  # exact: all values are dyadic


def test_path_fixed_point_and_zero_node_sum():
    """Appendix A: (1,0,1) on o-o-o is fixed, and the zero node's closed sum is 2."""
    d = read_golden("path3_fixed_point.txt")
    g = graph_from_edge_tokens(int(d["n"][0]), d["edges"])
    x = np.array([float(t) for t in d["x"]])
    x1, _ = _step(g, np.ones(3), 1.0, x)
    assert np.array_equal(x1, x)
    A = dense_adjacency(g)
    assert np.array_equal((A + np.eye(3)) @ x, np.array([float(t) for t in d["closed_sums"]]))


@pytest.mark.parametrize("make,d", [(lambda: cycle(5), 2), (lambda: cycle(9), 2), (petersen, 3),
                                    (lambda: complete(4), 3), (lambda: hypercube(3), 3),
                                    (lambda: hypercube(4), 4)])
def test_regular_uniform_atom(make, d):
    """Appendix A: a d-regular graph is normalized by the uniform vector 1/(d+1)."""
    g = make()
    x = np.full(g.n, 1.0 / (d + 1))
    x1, _ = _step(g, np.ones(g.n), 1.0, x)
    np.testing.assert_allclose(x1, x, rtol=0, atol=1e-15)


@pytest.mark.parametrize("gamma", [0.5, 1.3, 2.0])
def test_regular_uniform_wrgn_fixed_point(gamma):
    """WRGN with uniform weights on a d-regular graph: 1/(1 + gamma d) is fixed, since
    x_i/(x_i + gamma sum_j (v_j/v_i) x_j) = 1/(1 + gamma d) for uniform x and v."""
    g = petersen()
    w = np.full(g.n, 2.5)
    x = np.full(g.n, 1.0 / (1.0 + 3 * gamma))
    x1, _ = _step(g, w, gamma, x)
    np.testing.assert_allclose(x1, x, rtol=1e-14)


def test_complete_graph_simplex_projection():
    """Section 2: on K_n one GN step is x / sum(x), a projection onto the simplex."""
    g = complete(6)
    x = np.array([0.3, 0.1, 0.7, 0.2, 0.05, 0.9])
    x1, _ = _step(g, np.ones(6), 1.0, x)
    np.testing.assert_allclose(x1, x / x.sum(), rtol=1e-15)
    assert abs(x1.sum() - 1.0) < 1e-15


def test_gamma_zero_gives_all_ones():
    """Appendix H footnote: gamma = 0 removes the edges and one step gives x = 1."""
    g = I.erdos_renyi(40, 0.2, 3)
    w = I.weights_uniform01(40, 3)
    x = I.rng_for(3, 9).random(40) + 0.01
    x1, _ = _step(g, w, 0.0, x)
    assert np.array_equal(x1, np.ones(40))


def test_isolated_vertices_go_to_one():
    """No neighbours: x_i / x_i = 1 (isolated vertices belong to every MIS)."""
    g = graph_from_edges(5, [(0, 1)])
    x1, _ = _step(g, np.array([1.0, 2.0, 3.0, 0.5, 0.25]), 1.5, np.array([0.4, 0.6, 0.3, 0.01, 0.9]))
    assert np.array_equal(x1[2:], np.ones(3))


# ------------------------------------------------------------ weighted K_2 (App. H)

def test_k2_interior_limit_below_gamma_b():
    """Appendix H: for gamma < 1/sqrt(w0) the limit is the interior point (I+gamma A)^-1 v."""
    d = read_golden("k2_interior_limit.txt")
    w0, gamma = float(d["w0"][0]), float(d["gamma"][0])
    g = complete(2)
    w = np.array([w0, 1.0])
    x = np.array([0.5, 0.5])
    for _ in range(400):
        x, _ = _step(g, w, gamma, x)
    np.testing.assert_allclose(x, [float(t) for t in d["x"]], atol=5e-7)
    # same point as the dense linear solve
    v = np.sqrt(w)
    y = np.linalg.solve(np.array([[1.0, gamma], [gamma, 1.0]]), v)
    np.testing.assert_allclose(x, y / v, rtol=1e-12)


@pytest.mark.parametrize("w0", [2.0, 4.0])
def test_k2_phase_transitions(w0):
    """Appendix H: above gamma_B = 1/sqrt(w0) the heavy node wins from any start; above
    gamma_D = sqrt(w0) the light MIS {1} is gamma-stable too (stab = gamma/sqrt(w0))."""
    g = complete(2)
    w = np.array([w0, 1.0])
    gb, gd = 1 / math.sqrt(w0), math.sqrt(w0)
    for x0 in ([0.5, 0.5], [0.05, 0.95]):
        r = O.solve(2, g.row_ptr, g.col_idx, w, x0, gamma0=0.5 * (gb + gd), gamma1=0.5 * (gb + gd),
                    ramp_steps=1, max_steps=5000)
        assert r.binarised and list(r.sel) == [True, False]
    # stab of {1} (node 0 outside) is gamma * sqrt(w1/w0)
    assert O.stab(2, g.row_ptr, g.col_idx, w, 1.1 * gd, [0, 1]) == pytest.approx(1.1, rel=1e-15)
    r = O.solve(2, g.row_ptr, g.col_idx, w, [0.01, 0.99], gamma0=1.5 * gd, gamma1=1.5 * gd,
                ramp_steps=1, max_steps=5000)
    assert r.binarised and list(r.sel) == [False, True]


def test_k2_equal_weights_symmetric_start_never_binarises():
    """Appendix H, w0 = 1, gamma > 1: the apex 1/2 is a fixed point; the symmetric start
    stays there, so the solve reports no binarisation."""
    g = complete(2)
    r = O.solve(2, g.row_ptr, g.col_idx, np.ones(2), [0.5, 0.5], gamma0=1.5, gamma1=1.5,
                ramp_steps=1, max_steps=300)
    assert r.status == O.NOT_CONVERGED and not r.binarised
    np.testing.assert_allclose(r.x, [0.4, 0.4], rtol=1e-15)  # 1/(1+gamma) after one step, fixed


# ------------------------------------------------------------ identities

def _sparse(g):
    return sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))


def test_preconditioned_gradient_identity():
    """Appendix D: y^{k+1} - y^k = -diag(y^{k+1} / v) grad E(y^k), grad E = (I+gamma A) y - v."""
    g = I.erdos_renyi(300, 0.03, 11)
    w = I.weights_uniform01(300, 11).astype(np.float64)
    v = np.sqrt(w)
    x = I.rng_for(11, 5).random(300) * 0.9 + 0.05
    gamma = 1.3
    x1, _ = _step(g, w, gamma, x)
    y0, y1 = v * x, v * x1
    grad = y0 + gamma * (_sparse(g) @ y0) - v
    np.testing.assert_allclose(y1 - y0, -(y1 / v) * grad, rtol=1e-11, atol=1e-14)


def test_replicator_identity():
    """Theorem 5: M_v(y^{k+1}) equals the mean fitness fbar(p^k), p = v y / M_v,
    f_i = v_i / ((I + gamma A)(p / v))_i; and p^{k+1} = p^k f / fbar."""
    g = I.unit_disk(400, 8, 2)
    w = I.weights_uniform01(400, 2).astype(np.float64)
    v = np.sqrt(w)
    x = I.rng_for(2, 5).random(400) * 0.8 + 0.1
    gamma = 1.2
    y = v * x
    M = float(np.dot(v, y))
    p = v * y / M
    q = p / v
    f = v / (q + gamma * (_sparse(g) @ q))
    fbar = float(np.dot(p, f))
    x1, _ = _step(g, w, gamma, x)
    assert O.objective(w, x1) == pytest.approx(fbar, rel=1e-13)
    np.testing.assert_allclose(v * (v * x1) / O.objective(w, x1), p * f / fbar, rtol=1e-12)


def test_scale_invariance_bit_exact():
    """Section 2 property iv: the map is projective; scaling by 2^k is exact in binary."""
    g = I.barabasi_albert(500, 3, 4)
    w = I.weights_uniform01(500, 4).astype(np.float64)
    x = I.rng_for(4, 5).random(500) * 0.9 + 0.05
    base, _ = _step(g, w, 1.4, x)
    for k in (-3, 5, 20):
        xs, _ = _step(g, w, 1.4, x * 2.0 ** k)
        assert np.array_equal(xs, base)


def test_energy_closed_form_at_mis():
    """Section 5 (weight-tilted Motzkin-Straus) / Appendix B: at the binary point of a
    MIS M, y = v 1_M and E(y) = 1/2 W(M) - W(M) = -W(M)/2."""
    g = petersen()
    w = I.weights_uniform01(10, 1).astype(np.float64)
    sets, W = enumerate_mis(g, w)
    for s, wt in zip(sets[:5], W[:5]):
        sel = np.array([(s >> i) & 1 for i in range(10)], dtype=np.float64)
        y = np.sqrt(w) * sel
        assert O.energy(10, g.row_ptr, g.col_idx, w, 1.7, y) == pytest.approx(-wt / 2, rel=1e-14)


# ------------------------------------------------------------ invariants of the iteration

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_energy_descent_and_mass_growth_constant_gamma(seed):
    """Theorem 1: E(y) strictly decreases at fixed gamma; Theorem 3: the weighted mass
    sum w x strictly increases once x is the image of a step (k >= 1); x stays in [0,1]
    (property i)."""
    g = I.erdos_renyi(200, 8 / 199, seed)
    w = I.weights_uniform01(200, seed).astype(np.float64)
    v = np.sqrt(w)
    gamma = 1.5
    x = I.rng_for(seed, 3).random(200) * 0.9 + 0.05
    E_prev = O.energy(200, g.row_ptr, g.col_idx, w, gamma, v * x)
    F_prev = None
    for k in range(60):
        x1, fb = _step(g, w, gamma, x)
        assert fb == 0
        assert np.all((x1 >= 0) & (x1 <= 1))
        E = O.energy(200, g.row_ptr, g.col_idx, w, gamma, v * x1)
        if not np.array_equal(x1, x):
            assert E < E_prev
        F = O.objective(w, x1)
        if k >= 1 and not np.array_equal(x1, x):
            assert F > F_prev
        E_prev, F_prev, x = E, F, x1


def test_support_invariance_and_fallback():
    """Section 2 property ii: zeros stay zero.  Code appendix safe division: a node whose
    closed-neighbourhood sum is <= 1e-9 is reset to 1/2."""
    g = graph_from_edges(6, [(0, 1), (1, 2), (3, 4)])
    w = np.array([1.0, 2.0, 0.5, 1.0, 1.0, 3.0])
    x = np.array([0.0, 0.4, 0.7, 0.0, 0.0, 0.9])
    x1, fb = _step(g, w, 1.5, x)
    assert x1[0] == 0.0
    # nodes 3 and 4 have an all-zero closed neighbourhood
    assert fb == 2 and x1[3] == 0.5 and x1[4] == 0.5
    assert x1[5] == 1.0


def test_gamma_schedule():
    """Section 6 / code appendix: linear ramp gamma0 -> gamma1 over T steps, p = k/(T-1)."""
    assert O.gamma(0.9, 1.5, 1000, 0) == 0.9
    assert O.gamma(0.9, 1.5, 1000, 999) == 1.5
    assert O.gamma(0.9, 1.5, 1000, 5000) == 1.5
    assert O.gamma(0.9, 1.5, 1000, 333) == pytest.approx(0.9 + 0.6 * 333 / 999, rel=1e-15)
    assert O.gamma(1.1, 1.1, 1, 7) == 1.1


# ------------------------------------------------------------ limits: brute force

@pytest.mark.parametrize("seed", range(12))
def test_limit_is_stable_mis_bruteforce(seed):
    """Theorem 4: the iteration converges to a gamma-stable MIS, and every MWIS is
    gamma-stable with stab >= gamma.  Exhaustive MIS enumeration on n <= 16."""
    rng = I.rng_for(seed, 42)
    n = int(rng.integers(8, 17))
    g = I.erdos_renyi(n, 0.3, seed)
    w = I.weights_uniform01(n, seed).astype(np.float64)
    sets, W = enumerate_mis(g, w)
    gamma = 1.5
    r = O.solve(n, g.row_ptr, g.col_idx, w, np.full(n, 0.5), gamma0=gamma, gamma1=gamma,
                ramp_steps=1, max_steps=20000)
    assert r.binarised
    assert bits_to_mask(r.sel) in sets
    assert r.conflicts == 0 and r.uncovered == 0
    assert r.set_objective == pytest.approx(W[sets.index(bits_to_mask(r.sel))], rel=1e-14)
    assert r.stab > 1.0
    best = int(np.argmax(W))
    mwis = np.array([(sets[best] >> i) & 1 for i in range(n)], dtype=np.uint8)
    assert O.stab(n, g.row_ptr, g.col_idx, w, gamma, mwis) >= gamma * (1 - 1e-12)
    # the stop is at a true limit: many more steps do not change the set
    r2 = O.solve(n, g.row_ptr, g.col_idx, w, r.x, gamma0=gamma, gamma1=gamma, ramp_steps=1,
                 max_steps=3000, tau=0.0)
    assert np.array_equal(r2.sel, r.sel)


def test_rounded_set_is_independent_after_any_step():
    """For gamma >= 1, two adjacent nodes cannot both exceed 1/2 after a step:
    y_i > gamma y_j and y_j > gamma y_i cannot hold together."""
    g = I.unit_disk(500, 12, 8)
    w = I.weights_uniform01(500, 8).astype(np.float64)
    x = I.rng_for(8, 1).random(500)
    for gamma in (1.0, 1.2):
        x1, _ = _step(g, w, gamma, x)
        assert O.check(500, g.row_ptr, g.col_idx, (x1 > 0.5).astype(np.uint8))[0] == 0


# ------------------------------------------------------------ assignment (rook graphs)

@pytest.mark.parametrize("N,seed", [(3, 0), (4, 1), (5, 2), (6, 3), (7, 4), (8, 5)])
def test_rook_converges_to_permutation(N, seed):
    """Abstract / Section 2 (cross-normalization): on the rook graph every MIS is a
    permutation matrix; the objective is at most the optimal assignment (brute force
    over N! for N <= 7, scipy's LAP solver for N = 8)."""
    g = I.rook(N)
    w, C = I.rook_weights(N, seed, temperature=0.1)
    w = w.astype(np.float64)
    r = O.solve(g.n, g.row_ptr, g.col_idx, w, np.full(g.n, 0.5), max_steps=4000)
    assert r.binarised
    P = r.sel.reshape(N, N).astype(int)
    assert (P.sum(0) == 1).all() and (P.sum(1) == 1).all()
    Wm = w.reshape(N, N)
    if N <= 7:
        best = best_assignment_bruteforce(Wm)
    else:
        from scipy.optimize import linear_sum_assignment
        ri, cj = linear_sum_assignment(-Wm)
        best = float(Wm[ri, cj].sum())
    assert r.set_objective <= best * (1 + 1e-12)


# ------------------------------------------------------------ checks and validation

def test_check_objective_stab_by_hand():
    g = graph_from_edges(4, [(0, 1), (1, 2), (2, 3)])   # path a-b-c-d
    w = np.array([1.0, 4.0, 9.0, 1.0])
    assert O.check(4, g.row_ptr, g.col_idx, [1, 0, 1, 0]) == (0, 0)
    assert O.check(4, g.row_ptr, g.col_idx, [1, 1, 1, 0]) == (2, 0)
    assert O.check(4, g.row_ptr, g.col_idx, [1, 0, 0, 0]) == (0, 2)
    # S = {0, 2}: node 1 sees sqrt(1/4) + sqrt(9/4) = 2, node 3 sees sqrt(9/1) = 3
    assert O.stab(4, g.row_ptr, g.col_idx, w, 1.5, [1, 0, 1, 0]) == pytest.approx(3.0, rel=1e-15)
    assert O.objective(w, np.array([1.0, 0.5, 0.0, 0.25])) == pytest.approx(3.25, rel=1e-15)


def test_validation_codes():
    ok = graph_from_edges(3, [(0, 1), (1, 2)])
    w = np.ones(3)
    assert O.validate(3, ok.row_ptr, ok.col_idx, w) == O.OK
    # asymmetric: 0->1 without 1->0
    assert O.validate(3, [0, 1, 1, 1], [1], w) == O.E_ASYMMETRIC
    assert O.validate(3, [0, 1, 2, 2], [0, 1], w) == O.E_SELF_LOOP
    assert O.validate(3, [0, 2, 3, 3], [1, 1, 0], w) == O.E_CSR           # duplicate
    assert O.validate(3, [0, 1, 2, 2], [5, 0], w) == O.E_CSR              # out of range
    assert O.validate(3, [0, 2, 1, 2], [1, 0], w) == O.E_CSR              # non-monotone
    assert O.validate(3, ok.row_ptr, ok.col_idx, [1.0, 0.0, 1.0]) == O.E_WEIGHT
    assert O.validate(3, ok.row_ptr, ok.col_idx, [1.0, np.nan, 1.0]) == O.E_WEIGHT
    assert O.is_normalizable(3, ok.row_ptr, ok.col_idx, [0.0, 0.0, 0.3]) == O.E_NOT_NORMALIZABLE
    assert O.is_normalizable(3, ok.row_ptr, ok.col_idx, [0.0, 0.1, 0.0]) == O.OK
    assert O.is_normalizable(3, ok.row_ptr, ok.col_idx, [0.0, -0.1, 1.0]) == O.E_ARG


def test_solve_rejects_non_normalizable_start():
    g = graph_from_edges(3, [(0, 1)])
    r = O.solve(3, g.row_ptr, g.col_idx, np.ones(3), [0.5, 0.5, 0.0])
    assert r.status == O.E_NOT_NORMALIZABLE


def test_empty_and_edgeless_graphs():
    r = O.solve(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0))
    assert r.steps == 0 and r.set_size == 0 and r.binarised
    g = graph_from_edges(4, [])
    r = O.solve(4, g.row_ptr, g.col_idx, np.ones(4), np.full(4, 0.3))
    assert r.binarised and r.steps == 1 and r.sel.all()


def test_stopping_rule_is_first_passing_check():
    """The solve stops at the first check step whose state passes the test."""
    g = I.erdos_renyi(120, 6 / 119, 5)
    w = I.weights_uniform01(120, 5).astype(np.float64)
    x0 = np.full(120, 0.5)
    r = O.solve(120, g.row_ptr, g.col_idx, w, x0, gamma0=1.3, gamma1=1.3, ramp_steps=1)
    assert r.binarised and r.steps > 1
    xs = O.unrolled_forward(120, g.row_ptr, g.col_idx, w, np.full(r.steps, 1.3), x0)
    for k in (r.steps - 1, r.steps):
        res, unc, grow = O.binarisation(120, g.row_ptr, g.col_idx, w, 1.3, xs[k])
        passed = res <= 1e-4 and unc == 0 and grow == 0
        assert passed == (k == r.steps)
    np.testing.assert_array_equal(xs[r.steps], r.x)


# ------------------------------------------------------------ reverse mode

def _fd_grad_w(g, w, gammas, x0, c, h=1e-6):
    out = np.zeros(g.n)
    for i in range(g.n):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fp = c @ O.unrolled_forward(g.n, g.row_ptr, g.col_idx, wp, gammas, x0)[-1]
        fm = c @ O.unrolled_forward(g.n, g.row_ptr, g.col_idx, wm, gammas, x0)[-1]
        out[i] = (fp - fm) / (2 * h)
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_vjp_matches_central_differences(seed):
    """Reverse mode through T = 50 steps vs fp64 central differences, n = 30."""
    g = I.unit_disk(30, 5, seed)
    w = I.weights_uniform(30, 0.5, 1.5, seed).astype(np.float64)
    x0 = np.full(30, 0.5)
    gammas = np.full(50, 1.5)
    c = I.rng_for(seed, 8).random(30)
    gw, gx0 = O.unrolled_vjp(30, g.row_ptr, g.col_idx, w, gammas, x0, c)
    fd = _fd_grad_w(g, w, gammas, x0, c)
    np.testing.assert_allclose(gw, fd, rtol=2e-6, atol=1e-9)
    fdx = np.zeros(30)
    h = 1e-6
    for i in range(30):
        xp, xm = x0.copy(), x0.copy()
        xp[i] += h
        xm[i] -= h
        fdx[i] = (c @ O.unrolled_forward(30, g.row_ptr, g.col_idx, w, gammas, xp)[-1]
                  - c @ O.unrolled_forward(30, g.row_ptr, g.col_idx, w, gammas, xm)[-1]) / (2 * h)
    np.testing.assert_allclose(gx0, fdx, rtol=2e-5, atol=5e-9)  # FD round-off ~ eps|L|/h


def test_single_step_vjp_is_jacobian_transpose():
    """Lemma (Jacobian) of Appendix F: dN_B(x)_i/dx_j = (delta_ij (Bx)_i - x_i B_ij)/(Bx)_i^2
    with B = I + gamma V^-1 A V; one reverse step must return J^T gbar."""
    g = I.erdos_renyi(25, 0.25, 6)
    w = I.weights_uniform01(25, 6).astype(np.float64)
    v = np.sqrt(w)
    x = I.rng_for(6, 2).random(25) + 0.05
    gamma = 1.25
    A = dense_adjacency(g)
    B = np.eye(25) + gamma * (A * v[None, :] / v[:, None])
    Bx = B @ x
    J = (np.diag(Bx) - x[:, None] * B) / (Bx[:, None] ** 2)
    gbar = I.rng_for(6, 4).standard_normal(25)
    _, gx0 = O.unrolled_vjp(25, g.row_ptr, g.col_idx, w, [gamma], x, gbar)
    np.testing.assert_allclose(gx0, J.T @ gbar, rtol=1e-12, atol=1e-14)


def test_batched_reference_is_per_graph():
    """Section 2 property iii: components do not interact, so the batched reference is
    the per-graph solve; a block-diagonal union solved as one graph agrees."""
    gs = [I.erdos_renyi(60 + 10 * k, 6 / (59 + 10 * k), k) for k in range(4)]
    ns, nnzs, rp, ci = I.concat_graphs(gs)
    w = np.concatenate([I.weights_uniform01(gg.n, k) for k, gg in enumerate(gs)]).astype(np.float64)
    x0 = np.full(len(w), 0.5)
    per = O.solve_batch(ns, rp, ci, w, x0, gamma0=1.4, gamma1=1.4, ramp_steps=1, max_steps=3000,
                        tau=0.0)
    # union graph with global indices
    from paper_2605_05330_amd.inputs import csr_from_edges, edges_of
    src, dst, off = [], [], 0
    for gg in gs:
        a, b = edges_of(gg)
        src.append(a + off)
        dst.append(b + off)
        off += gg.n
    U = csr_from_edges(off, np.concatenate(src), np.concatenate(dst))
    xs = O.unrolled_forward(U.n, U.row_ptr, U.col_idx, w, np.full(3000, 1.4), x0)[-1]
    np.testing.assert_array_equal(np.concatenate([p.x for p in per]), xs)


def test_support_invariance_over_long_runs():
    """Section 2 property ii: supp(N(x)) = supp(x).  Positive states are computed at
    their own magnitude far below any fp32 range and are held at fp64's smallest
    normal number 2^-1022 only where fp64 would underflow; exact zeros stay 0."""
    g = I.erdos_renyi(300, 8 / 299, 21)
    w = I.weights_uniform01(300, 21).astype(np.float64)
    x = I.rng_for(21, 1).random(300) * 0.9 + 0.05
    deg = g.degrees()
    zeros = [i for i in range(300) if deg[i] > 0][:20:2]   # spaced out: each keeps positive neighbours
    x[zeros] = 0.0
    assert O.is_normalizable(300, g.row_ptr, g.col_idx, x) == O.OK
    assert O.x_floor() == 2.0 ** -1022
    xs = O.unrolled_forward(300, g.row_ptr, g.col_idx, w, np.full(3000, 1.5), x)
    pos = np.setdiff1d(np.arange(300), zeros)
    assert np.all(xs[:, pos] >= 2.0 ** -1022)     # positives never underflow to 0
    assert np.any((xs[:, pos] > 0) & (xs[:, pos] < 2.0 ** -300))   # and are carried far below fp32's range
    # a value above the floor is the quotient itself: x' = y / s exactly as fp64 rounds it
    v = np.sqrt(w)
    A = _sparse(g)
    for k in (10, 200, 2999):
        y = v * xs[k]
        s_k = y + 1.5 * (A @ y)
        q = y / s_k
        above = (q >= 2.0 ** -1022) & (s_k > 1e-9)
        np.testing.assert_array_equal(xs[k + 1, above], q[above])
    # zeros stay 0 as long as their closed-neighbourhood sum is above the 1e-9 reset
    for k in range(3000):
        s_k = 1.5 * (A @ (v * xs[k]))
        live = [z for z in zeros if s_k[z] > 1e-9]
        assert np.all(xs[k + 1, live] == 0.0)


def _floor_cases():
    """Instances whose solves take vertices below 2^-300 and back (ER n = 1500,
    seed 109; rook 16 x 16 and 48 x 48 with the test weights of those shapes)."""
    er = I.erdos_renyi(1500, 6 / 1499, 109)
    yield "er1500", er, I.weights_uniform01(1500, 109)
    for N in (16, 48):
        yield f"rook{N}", I.rook_rect(N, N), I.rook_weights_rect(N, N, 7 * N + N).reshape(-1)


SCHED_RAMP = dict(gamma0=float(np.float32(0.9)), gamma1=1.5, ramp_steps=1000, max_steps=2000, tau=1e-4)


def test_result_does_not_depend_on_a_deep_floor():
    """The support floor is where fp64 runs out (2^-1022), not a level chosen in the
    method's range: holding positives at 2^-100 or 2^-300 changes steps (and on rook
    48 x 48 the permutation), while moving the floor between 2^-1000, 2^-1010 and
    2^-1022 changes neither the set nor, except on the rook instance that takes the
    safe-division reset at the bottom of its range, the step count."""
    steps = {}
    try:
        for name, g, w in _floor_cases():
            w = w.astype(np.float64)
            for f in (2.0 ** -100, 2.0 ** -1000, 2.0 ** -1010, 2.0 ** -1022):
                O.set_x_floor(f)
                r = O.solve(g.n, g.row_ptr, g.col_idx, w, np.full(g.n, 0.5), **SCHED_RAMP)
                assert r.binarised and r.conflicts == 0 and r.uncovered == 0
                steps[name, f] = (r.steps, r.sel.tobytes())
    finally:
        O.set_x_floor(0.0)
    assert O.x_floor() == 2.0 ** -1022
    for name in ("er1500", "rook16", "rook48"):
        deep = [steps[name, f] for f in (2.0 ** -1000, 2.0 ** -1010, 2.0 ** -1022)]
        assert all(d[1] == deep[-1][1] for d in deep)                 # same set
        assert steps[name, 2.0 ** -100][0] != deep[-1][0]            # a 2^-100 floor is not the map
    assert steps["er1500", 2.0 ** -1000][0] == steps["er1500", 2.0 ** -1022][0] == 1459
    assert steps["rook16", 2.0 ** -1000][0] == steps["rook16", 2.0 ** -1022][0] == 402
    assert steps["rook48", 2.0 ** -100][1] != steps["rook48", 2.0 ** -1022][1]   # another permutation


def test_frozen_vertex_regrows_to_stable_set():
    """Theorem 4 convergence needs support invariance: on this graph a light vertex
    decays below 1e-70 while its neighbour is selected and must later regrow to
    replace it; the solve ends on a gamma-stable set that a long continuation keeps."""
    g = I.erdos_renyi(1500, 6 / 1499, 109)
    w = I.weights_uniform01(1500, 109).astype(np.float64)
    r = O.solve(1500, g.row_ptr, g.col_idx, w, np.full(1500, 0.5), gamma0=0.9, gamma1=1.5, ramp_steps=1000,
                max_steps=3000)
    assert r.binarised and r.sel[775] and not r.sel[276]
    assert r.growing == 0 and r.stab > 1.0 - 1e-3
    r2 = O.solve(1500, g.row_ptr, g.col_idx, w, r.x, gamma0=1.5, gamma1=1.5, ramp_steps=1, max_steps=2000,
                 tau=0.0)
    assert np.array_equal(r2.sel, r.sel)


def test_random_start_by_hand():
    """u = exp(-k): e = k, so x = k / k_max clamped to [1e-3, 1]; u = 1 gives e = 0,
    clamped up to 1e-3; the largest draw maps to exactly 1."""
    k = np.array([0.0, 0.5, 1.0, 2.0, 4.0, 1e-4])
    x = O.random_start(np.exp(-k))
    np.testing.assert_allclose(x, [1e-3, 0.125, 0.25, 0.5, 1.0, 1e-3], rtol=1e-12)
    assert x[4] == 1.0
    assert np.array_equal(O.random_start(np.ones(5)), np.ones(5))


def test_random_start_is_scale_free_draw():
    """-log U with U uniform is Exp(1): the mean of e over many draws is 1 (within 1%),
    and the normalised start is a point of (0, 1] with one coordinate at 1."""
    u = 1.0 - I.rng_for(3, 40).random(200_000)
    e = -np.log(u)
    assert abs(e.mean() - 1.0) < 0.01
    x = O.random_start(u)
    assert x.max() == 1.0 and x.min() >= 1e-3


def test_all_core_build_is_bit_identical():
    """The all-core build of the oracle (the benchmark's second CPU baseline) runs
    the rows of a step and of the stopping test on several threads; each row keeps
    its CSR order and the cross-row reductions are max and counts, so every output
    is bit-identical to the single-thread build (ER n=1500 seed 109, which
    regrows from deep decay, and rook 48 x 48, which takes the safe-division reset)."""
    for name, g, w in _floor_cases():
        if name == "rook16":
            continue
        w = w.astype(np.float64)
        a = O.solve(g.n, g.row_ptr, g.col_idx, w, np.full(g.n, 0.5), **SCHED_RAMP)
        b = O.solve(g.n, g.row_ptr, g.col_idx, w, np.full(g.n, 0.5), omp=True, **SCHED_RAMP)
        assert (a.steps, a.fallback_count, a.growing) == (b.steps, b.fallback_count, b.growing)
        assert np.array_equal(a.x.view(np.uint64), b.x.view(np.uint64))
        assert a.stab == b.stab and a.residual == b.residual and a.relaxed_objective == b.relaxed_objective

"""Fractional warm start from the clique LP relaxation (TEST INFRASTRUCTURE ONLY).

Imported by ``tests/`` and the benchmark's CPU-baseline leg; the product path
never imports it.  Plain fp64 numpy, written from the paper's description of
its warm start (Section 6, "Randomized start and warm start"): fractional
solutions of the MWIS LP relaxation over clique constraints, computed by a
Bregman-Sinkhorn scheme run alone (no rounding), stopped at a fractional
duality gap of 0.1%, with diversity across starts from a randomized clique
order and jittered initial temperatures, the temperature dropping by a factor
0.99.  The paper gives no formulas for the solver (it ran a modified external
code); the steps below are this project's reading of an entropy-smoothed
clique LP solved by exact block-coordinate minimisation of its dual.

Problem.  Costs c > 0 on n vertices and cliques C_1..C_m covering every vertex:
    LP* = max c.x  s.t.  sum_{i in C} x_i <= 1 for every clique C,  x >= 0.
(x <= 1 follows from the cover.)  With multipliers lam_C >= 0 and
Lam_i = sum_{C contains i} lam_C, every lam gives the upper bound
    D(lam) = sum_C lam_C + sum_i max(0, c_i - Lam_i)  >=  LP*.
At temperature T the smoothed primal is x_i = exp((c_i - Lam_i) / T).

Clique update at T (exact minimisation of the smoothed dual in lam_C >= 0):
    L = log sum_{i in C} exp((c_i - Lam_i) / T),
    lam_C' = max(0, lam_C + T L),   Lam_i += lam_C' - lam_C  for i in C,
after which sum_{i in C} x_i = 1 (or < 1 with lam_C' = 0).

Parallel order.  Cliques are coloured first-fit in input order: clique k takes
the smallest class none of whose cliques shares a vertex with it.  Cliques of a
class are disjoint, so updating them one after the other or all at once gives
the same numbers.  A pass visits the classes in a per-start order (the caller's
permutation: the randomized clique order); pass p runs at
T_p = max(t_min, t0 * drop^p).

Check (after pass p when (p + 1) % check_every == 0, and after the last pass),
at the pass's T:  x_i = exp(min((c_i - Lam_i) / T, 60)) (the cap only keeps
sums finite), S_C = sum_{i in C} x_i, xf_i = x_i / max(1, max_{C contains i} S_C)
(feasible), then `lift_rounds` rounds of a fair-share lift that hands every
clique's slack 1 - sum_{i in C} xf_i out equally to its members, each member
rising by the smallest share of its cliques (still feasible); P = c.xl of the
lifted point.  The bound is taken from the multipliers themselves,
D = sum lam_C + sum_i max(0, c_i - sum_{C contains i} lam_C), so a drift of the
incrementally kept Lam cannot make it invalid.  The start keeps the smallest D
and the largest P over its checks (and the point of that P) and stops when
(D_best - P_best) / D_best <= gap_tol.  Its warm start is max(x_best, x_floor)
(GN needs a positive start).

Temperatures.  anneal_tol <= 0: T_p = max(t_min, t0 drop^p) (the drop every
pass).  anneal_tol > 0: the temperature is held within a check interval; at a
check it drops by drop^check_every (not below t_min) when the smoothed primal's
worst clique excess max_C S_C - 1 is at most anneal_tol, or when P_best has not
improved by a relative 5e-5 for `stall` checks; the primal stays near-feasible
at every temperature before it cools, which the feasible point needs to come
close to LP*.

Pinned by tests/test_oracle_lp.py (closed forms, LP duality against an
independent LP solver, brute force on perfect formulations).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

EXP_CAP = 60.0


@dataclass
class Cliques:
    """Clique constraints in CSR form: clique k is members[ptr[k]:ptr[k+1]]."""
    n: int
    ptr: np.ndarray
    members: np.ndarray

    @property
    def m(self) -> int:
        return len(self.ptr) - 1

    def clique(self, k: int) -> np.ndarray:
        return self.members[self.ptr[k]:self.ptr[k + 1]]


@dataclass
class LPResult:
    passes: int
    temperature: float
    dual: float       # smallest bound over the checks
    primal: float     # largest feasible value over the checks
    gap: float
    converged: bool


STALL_REL = 5e-5   # a check "improves" P_best when it raises it by more than this fraction


def colour_classes(cl: Cliques) -> np.ndarray:
    """First-fit class of every clique, in input order (disjoint cliques per class)."""
    used: list[set[int]] = [set() for _ in range(cl.n)]  # classes already touching vertex i
    cls = np.zeros(cl.m, dtype=np.int64)
    for k in range(cl.m):
        taken = set()
        for i in cl.clique(k):
            taken |= used[int(i)]
        c = 0
        while c in taken:
            c += 1
        cls[k] = c
        for i in cl.clique(k):
            used[int(i)].add(c)
    return cls


def temperature(t0: float, drop: float, t_min: float, p: int) -> float:
    return max(t_min, t0 * drop ** p)


def update_clique(k: int, cl: Cliques, c: np.ndarray, Lam: np.ndarray, lam: np.ndarray, T: float) -> None:
    """The clique update of the smoothed dual (log-sum-exp with its maximum taken out)."""
    idx = cl.clique(k)
    a = (c[idx] - Lam[idx]) / T
    amax = a.max()
    L = amax + np.log(np.exp(a - amax).sum())
    new = max(0.0, lam[k] + T * L)
    Lam[idx] += new - lam[k]
    lam[k] = new


def run_pass(cl: Cliques, c, Lam, lam, classes: np.ndarray, order, T: float) -> None:
    for r in order:
        for k in np.flatnonzero(classes == r):
            update_clique(int(k), cl, c, Lam, lam, T)


def evaluate(cl: Cliques, c, Lam, lam, T: float):
    """(dual bound D, feasible primal value P, feasible point xf)."""
    x = np.exp(np.minimum((c - Lam) / T, EXP_CAP))
    mx = np.ones(cl.n)
    for k in range(cl.m):
        idx = cl.clique(k)
        mx[idx] = np.maximum(mx[idx], x[idx].sum())
    xf = x / mx
    D = lam.sum() + np.maximum(0.0, c - Lam).sum()
    return D, float(c @ xf), xf


def bound(cl: Cliques, c, lam) -> float:
    """D(lam) = sum lam_C + sum_i max(0, c_i - sum_{C contains i} lam_C)."""
    Lam = np.zeros(cl.n)
    for k in range(cl.m):
        Lam[cl.clique(k)] += lam[k]
    return float(lam.sum() + np.maximum(0.0, c - Lam).sum())


def lift(cl: Cliques, x, rounds: int) -> np.ndarray:
    """Fair-share lift of a feasible point: in each round every clique's slack
    1 - sum_{i in C} x_i is split equally among its members, and every vertex
    rises by the smallest share of its cliques (all at once)."""
    x = np.array(x, dtype=np.float64, copy=True)
    for _ in range(rounds):
        share = np.empty(cl.m)
        for k in range(cl.m):
            idx = cl.clique(k)
            share[k] = max(0.0, 1.0 - x[idx].sum()) / idx.size
        up = np.full(cl.n, np.inf)
        for k in range(cl.m):
            idx = cl.clique(k)
            up[idx] = np.minimum(up[idx], share[k])
        x += up
    return x


def check(cl: Cliques, c, Lam, lam, T: float, lift_rounds: int):
    """(bound D(lam), lifted feasible value P, lifted point, worst clique excess of x)."""
    x = np.exp(np.minimum((c - Lam) / T, EXP_CAP))
    S = np.array([x[cl.clique(k)].sum() for k in range(cl.m)])
    _, _, xf = evaluate(cl, c, Lam, lam, T)
    xl = lift(cl, xf, lift_rounds)
    return bound(cl, c, lam), float(c @ xl), xl, float(S.max() - 1.0)


def solve(cl: Cliques, c: np.ndarray, t0: float, order, drop: float, t_min: float, max_passes: int,
          check_every: int, gap_tol: float, x_floor: float, classes: np.ndarray | None = None,
          trace: list | None = None, anneal_tol: float = 0.0, stall: int = 10, lift_rounds: int = 2):
    """One start: (warm start max(x_best, x_floor), LPResult, lam, Lam).  trace, when
    given, receives (passes, D_best, P_best, gap, T, excess) of every check."""
    c = np.asarray(c, dtype=np.float64)
    if classes is None:
        classes = colour_classes(cl)
    Lam = np.zeros(cl.n)
    lam = np.zeros(cl.m)
    T = float(t0)
    D_best, P_best, x_best, quiet = np.inf, -np.inf, None, 0
    for p in range(max_passes):
        if anneal_tol <= 0.0:
            T = temperature(t0, drop, t_min, p)
        run_pass(cl, c, Lam, lam, classes, order, T)
        last = p + 1 == max_passes
        if (p + 1) % check_every == 0 or last:
            D, P, xl, excess = check(cl, c, Lam, lam, T, lift_rounds)
            quiet = 0 if P > P_best * (1.0 + STALL_REL) else quiet + 1
            if P > P_best:
                P_best, x_best = P, xl
            D_best = min(D_best, D)
            gap = (D_best - P_best) / D_best
            if trace is not None:
                trace.append((p + 1, D_best, P_best, gap, T, excess))
            if gap <= gap_tol or last:
                return (np.maximum(x_best, x_floor), LPResult(p + 1, T, D_best, P_best, gap, gap <= gap_tol),
                        lam, Lam)
            if anneal_tol > 0.0 and (excess <= anneal_tol or quiet >= stall):
                T = max(t_min, T * drop ** check_every)
                quiet = 0
    raise AssertionError("unreachable")

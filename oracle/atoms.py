"""Census of GN atoms on small connected graphs (TEST INFRASTRUCTURE ONLY).

Appendix A ("fractional atoms"): a fixed point of GN with full support on a
connected graph is an atom; with B = A + I, the atoms of a connected graph are
the solutions x > 0 of B x = 1 (every closed-neighbourhood sum equals 1).  A
connected graph is *atomic* when it has at least one atom.  Its atomic spectrum
is discrete (the single point B^-1 1) when det(B) != 0 and continuous (an affine
space cut by the open cube) when det(B) = 0.  Table atoms_10 counts, for each
number of vertices n, the connected graphs up to isomorphism and the atomic
ones split into irregular / regular (all degrees equal) x discrete / continuous.

This module computes that census from the definition, slowly and plainly, with
no code in common with the GPU kernel:
  * enumeration: every labelled graph on n vertices, its canonical form is the
    smallest edge bitmask over all n! relabellings, one graph per form;
  * connectedness by breadth-first search;
  * det(B) and, when B is invertible, B^-1 1 in exact rational arithmetic
    (fractions.Fraction, Gaussian elimination);
  * when B is singular, the existence of x > 0 with B x = 1 by the linear
    program  max t  s.t.  B x = 1, x_i >= t, t <= 1  (scipy's HiGHS, fp64):
    atomic iff t* > 1e-9.  (B x = 1 with x >= 0 bounds x by 1, since B has a unit
    diagonal and non-negative entries, so t* is finite; a positive optimum of
    a 0/1 system this small is far above the threshold.)
Practical up to n = 6 (2^15 labelled graphs times 720 relabellings).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from fractions import Fraction

import numpy as np


@dataclass
class Census:
    """Counts for one n: connected graphs up to isomorphism, then the atomic ones."""
    n: int
    graphs: int                 # all graphs up to isomorphism (connected or not)
    connected: int
    irregular_discrete: int
    irregular_continuous: int
    regular_discrete: int
    regular_continuous: int

    @property
    def atomic(self) -> int:
        return self.irregular_discrete + self.irregular_continuous + self.regular_discrete + self.regular_continuous


def pairs(n: int) -> list[tuple[int, int]]:
    """Vertex pairs (i < j) in lexicographic order: bit k of an edge mask is pair k."""
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def canonical_forms(n: int) -> np.ndarray:
    """One edge mask per isomorphism class of graphs on n vertices: the smallest
    mask over all relabellings of every labelled graph, deduplicated."""
    P = pairs(n)
    m = len(P)
    codes = np.arange(1 << m, dtype=np.int64)
    best = codes.copy()
    index = {p: k for k, p in enumerate(P)}
    for perm in itertools.permutations(range(n)):
        # bit k of the relabelled mask is the bit of the pair perm maps onto pair k
        out = np.zeros_like(codes)
        for k, (i, j) in enumerate(P):
            a, b = perm[i], perm[j]
            src = index[(min(a, b), max(a, b))]
            out |= ((codes >> src) & 1) << k
        np.minimum(best, out, out=best)
    return np.unique(best)


def adjacency(n: int, mask: int) -> list[list[int]]:
    A = [[0] * n for _ in range(n)]
    for k, (i, j) in enumerate(pairs(n)):
        if (mask >> k) & 1:
            A[i][j] = A[j][i] = 1
    return A


def is_connected(A: list[list[int]]) -> bool:
    n = len(A)
    seen, stack = {0}, [0]
    while stack:
        i = stack.pop()
        for j in range(n):
            if A[i][j] and j not in seen:
                seen.add(j)
                stack.append(j)
    return len(seen) == n


def solve_exact(B: list[list[int]]):
    """(det B, B^-1 1) over the rationals; the solution is None when det B = 0."""
    n = len(B)
    M = [[Fraction(B[i][j]) for j in range(n)] + [Fraction(1)] for i in range(n)]
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return Fraction(0), None
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for j in range(c, n + 1):
                M[r][j] -= f * M[c][j]
    x = [Fraction(0)] * n
    for c in range(n - 1, -1, -1):
        x[c] = (M[c][n] - sum(M[c][j] * x[j] for j in range(c + 1, n))) / M[c][c]
    return det, x


def positive_solution_exists(B: list[list[int]]) -> bool:
    """Whether some x > 0 solves B x = 1: the LP max t, B x = 1, x >= t, t <= 1."""
    from scipy.optimize import linprog

    n = len(B)
    c = np.zeros(n + 1)
    c[n] = -1.0  # maximise t
    A_eq = np.hstack([np.array(B, dtype=np.float64), np.zeros((n, 1))])
    b_eq = np.ones(n)
    A_ub = np.hstack([-np.eye(n), np.ones((n, 1))])  # t - x_i <= 0
    b_ub = np.zeros(n)
    bounds = [(None, None)] * n + [(None, 1.0)]
    r = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq, bounds=bounds, method="highs")
    return r.status == 0 and -r.fun > 1e-9


def classify(A: list[list[int]]):
    """None for a non-atomic graph, else (regular, discrete)."""
    n = len(A)
    B = [[A[i][j] + (1 if i == j else 0) for j in range(n)] for i in range(n)]
    det, x = solve_exact(B)
    degrees = {sum(row) for row in A}
    regular = len(degrees) == 1
    if det != 0:
        return (regular, True) if all(v > 0 for v in x) else None
    return (regular, False) if positive_solution_exists(B) else None


def census(n: int) -> Census:
    forms = canonical_forms(n)
    out = Census(n, len(forms), 0, 0, 0, 0, 0)
    for mask in forms:
        A = adjacency(n, int(mask))
        if not is_connected(A):
            continue
        out.connected += 1
        cls = classify(A)
        if cls is None:
            continue
        regular, discrete = cls
        if regular and discrete:
            out.regular_discrete += 1
        elif regular:
            out.regular_continuous += 1
        elif discrete:
            out.irregular_discrete += 1
        else:
            out.irregular_continuous += 1
    return out

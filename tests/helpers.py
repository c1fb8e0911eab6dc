"""Test helpers: tiny graphs, fixture parsing and brute-force enumeration.

Nothing here implements the GN method; these are independent references used to
pin the oracle (exhaustive search, textbook assignment) and to build inputs."""
from __future__ import annotations

import itertools
import os

import numpy as np

from paper_2605_05330_amd.inputs import Graph, csr_from_edges

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def graph_from_edge_tokens(n: int, toks: list[str]) -> Graph:
    src, dst = [], []
    for t in toks:
        a, b = t.split("-")
        src.append(int(a))
        dst.append(int(b))
    return csr_from_edges(n, np.array(src), np.array(dst))


def graph_from_edges(n: int, edges) -> Graph:
    edges = list(edges)
    if not edges:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    e = np.array(edges, dtype=np.int64)
    return csr_from_edges(n, e[:, 0], e[:, 1])


def complete(n: int) -> Graph:
    return graph_from_edges(n, itertools.combinations(range(n), 2))


def cycle(n: int) -> Graph:
    return graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def petersen() -> Graph:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return graph_from_edges(10, outer + spokes + inner)


def hypercube(d: int) -> Graph:
    n = 1 << d
    return graph_from_edges(n, [(i, i ^ (1 << b)) for i in range(n) for b in range(d) if i < i ^ (1 << b)])


def dense_adjacency(g: Graph) -> np.ndarray:
    A = np.zeros((g.n, g.n))
    for i in range(g.n):
        A[i, g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]] = 1.0
    return A


def enumerate_mis(g: Graph, w: np.ndarray):
    """All maximal independent sets of a graph with n <= 20 by exhaustive search.
    Returns (list of bitmasks, weights)."""
    n = g.n
    assert n <= 20
    S = np.arange(1 << n, dtype=np.int64)
    ok = np.ones(S.shape, dtype=bool)
    A = dense_adjacency(g)
    for i in range(n):
        for j in range(i + 1, n):
            if A[i, j]:
                ok &= ~(((S >> i) & 1).astype(bool) & ((S >> j) & 1).astype(bool))
    nbmask = [int(sum(1 << j for j in range(n) if A[i, j])) for i in range(n)]
    for i in range(n):
        has_i = ((S >> i) & 1).astype(bool)
        covered = (S & nbmask[i]) != 0
        ok &= has_i | covered
    sets = S[ok]
    weights = np.array([sum(float(w[i]) for i in range(n) if (s >> i) & 1) for s in sets])
    return [int(s) for s in sets], weights


def bits_to_mask(sel) -> int:
    return int(sum(1 << i for i, b in enumerate(sel) if b))


def best_assignment_bruteforce(W: np.ndarray) -> float:
    N = W.shape[0]
    best = -np.inf
    for perm in itertools.permutations(range(N)):
        best = max(best, float(sum(W[i, perm[i]] for i in range(N))))
    return best

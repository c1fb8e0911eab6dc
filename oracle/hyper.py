"""GN under hyperedge constraints (TEST INFRASTRUCTURE ONLY).

Imported by ``tests/`` only.  The paper leaves the extension of GN to
hypergraph constraints to future work (Conclusion) and gives no formula.  This
project's reading takes the hyperedges as clique constraints (at most one
selected vertex per hyperedge: the form of the paper's instances, Section 6)
and normalises every vertex by the mass of the hyperedges holding it, as the
paper's cross-normalization of the assignment problem (Section 2) does with
rows and columns:

    s_i = y_i + gamma * sum_{e contains i} (Y_e - y_i),   Y_e = sum_{j in e} y_j.

That is the WRGN step on the conflict graph whose edge (i, j) carries the
number of hyperedges holding both (A = H^T H - diag, H the incidence matrix).
The oracle writes that multigraph out as CSR, one entry per shared hyperedge,
and hands it to the fp64 C oracle (``oracle.step`` / ``oracle.solve``), whose
sums over CSR entries then count every shared hyperedge: the step, the
stopping test (uncovered, growing), the conflicts (pairs per shared hyperedge)
and the stability sum all take the multiplicity as the weight.

Pinned by tests/test_oracle_hyper.py: the expansion equals the simple conflict
graph when no pair shares two hyperedges and the rook graph for rows and
columns; a pair in two hyperedges doubles its weight (closed form on K2).
"""
from __future__ import annotations

import numpy as np

import oracle as O


def multigraph(n: int, ptr, members) -> tuple[np.ndarray, np.ndarray]:
    """CSR (int32) of the conflict multigraph: for every hyperedge and every
    ordered pair (i, j), i != j, of its members one entry j in row i; rows
    sorted by column, repeats kept."""
    rows, cols = [], []
    for e in range(len(ptr) - 1):
        mem = np.asarray(members[ptr[e]:ptr[e + 1]], dtype=np.int64)
        for i in mem:
            for j in mem:
                if i != j:
                    rows.append(int(i))
                    cols.append(int(j))
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return rp.astype(np.int32), cols.astype(np.int32)


def step(n, ptr, members, w, gamma, x):
    rp, ci = multigraph(n, ptr, members)
    return O.step(n, rp, ci, w, gamma, x)


def solve(n, ptr, members, w, x0, **sched):
    rp, ci = multigraph(n, ptr, members)
    return O.solve(n, rp, ci, w, x0, **sched)

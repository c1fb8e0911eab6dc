"""Seeded synthetic inputs: graphs (CSR) and vertex weights.

This module is shared by the HIP path's tests and benchmark and by the oracle's
tests.  It builds problem data only -- simple undirected graphs and positive
vertex weights, the input ``G = (A, w)`` of the MWIS problem (Section 2 and the
WRGN definition: ``A`` symmetric with zero diagonal, ``w`` strictly positive) --
and contains none of the method's arithmetic.

Every generator is a pure function of its arguments: the random streams are
numpy ``PCG64`` generators seeded with ``SeedSequence([seed, stream])``.

Graph families (stand-ins for the paper's AVR / MSCD conflict graphs, which are
not available):

* Erdos-Renyi ``G(n, p)``: each unordered pair independently with probability p.
* Barabasi-Albert: seed clique ``K_{m+1}``, every later vertex attaches to ``m``
  distinct earlier vertices chosen with probability proportional to degree.
* 2-D unit-disk: ``n`` points uniform in the unit square, an edge when the
  Euclidean distance is at most ``r``.
* Rook graph of an ``N x N`` board: the line graph of ``K_{N,N}`` used for the
  assignment problem; cell ``(i, j)`` has index ``N*i + j`` and conflicts with
  every other cell of its row and of its column.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Graph", "rng_for", "csr_from_edges", "erdos_renyi", "barabasi_albert",
    "unit_disk", "rook", "weights_uniform01", "weights_uniform", "rook_weights",
    "concat_graphs", "batch_sizes_loguniform", "edges_of",
]


@dataclass
class Graph:
    """Simple undirected graph in CSR form (int32), columns sorted per row."""
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def rng_for(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, dedup: bool = False) -> Graph:
    """Symmetric CSR from undirected edges ``src[k] -- dst[k]`` (no loops; duplicates
    must be absent unless ``dedup``, which drops repeated pairs and loops)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if dedup and src.size:
        a, b = np.minimum(src, dst), np.maximum(src, dst)
        keep = a != b
        pairs = np.unique(np.stack([a[keep], b[keep]], axis=1), axis=0)
        src, dst = pairs[:, 0], pairs[:, 1]
    rows = np.concatenate([src, dst])
    cols = np.concatenate([dst, src])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=n) if n > 0 else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), cols.astype(np.int32))


def edges_of(g: Graph) -> tuple[np.ndarray, np.ndarray]:
    """Undirected edge list (i < j) of a CSR graph."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cols = g.col_idx.astype(np.int64)
    keep = rows < cols
    return rows[keep], cols[keep]


def _pair_from_linear(idx: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Map a linear index over the pairs i<j (row-major) to (i, j)."""
    # number of pairs before row i: i*n - i*(i+1)/2
    idx = idx.astype(np.int64)
    nf = float(n)
    i = np.floor((2 * nf - 1 - np.sqrt((2 * nf - 1) ** 2 - 8.0 * idx)) / 2).astype(np.int64)
    i = np.clip(i, 0, n - 2)
    before = i * n - i * (i + 1) // 2
    # fix float rounding at row boundaries
    for _ in range(2):
        hi = idx >= before + (n - 1 - i)
        i = np.where(hi, i + 1, i)
        before = i * n - i * (i + 1) // 2
        lo = idx < before
        i = np.where(lo, i - 1, i)
        before = i * n - i * (i + 1) // 2
    j = idx - before + i + 1
    return i, j


def erdos_renyi(n: int, p: float, seed: int, stream: int = 0) -> Graph:
    """``G(n, p)``: the number of edges is Binomial(n(n-1)/2, p) and the edge set is a
    uniform subset of that size, which is the same distribution as independent pairs."""
    rng = rng_for(seed, stream)
    npairs = n * (n - 1) // 2
    if npairs == 0 or p <= 0.0:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    m = int(rng.binomial(npairs, min(p, 1.0)))
    lin = rng.choice(npairs, size=m, replace=False)
    i, j = _pair_from_linear(np.sort(lin), n)
    return csr_from_edges(n, i, j)


def barabasi_albert(n: int, m: int, seed: int, stream: int = 0) -> Graph:
    """Preferential attachment with a ``K_{m+1}`` seed; each new vertex takes ``m``
    distinct targets drawn proportionally to current degree."""
    if n <= m + 1:
        iu = np.triu_indices(n, 1)
        return csr_from_edges(n, iu[0], iu[1])
    rng = rng_for(seed, stream)
    n_edges = (m + 1) * m // 2 + (n - m - 1) * m
    src = np.empty(n_edges, dtype=np.int64)
    dst = np.empty(n_edges, dtype=np.int64)
    ends = np.empty(2 * n_edges, dtype=np.int64)   # every edge endpoint, degree-proportional pool
    iu = np.triu_indices(m + 1, 1)
    e0 = len(iu[0])
    src[:e0] = iu[0]
    dst[:e0] = iu[1]
    ends[0:2 * e0:2] = iu[0]
    ends[1:2 * e0:2] = iu[1]
    e = e0
    pool = 2 * e0
    draws = rng.random(size=(n - m - 1, 4 * m))
    for t in range(m + 1, n):
        row = draws[t - m - 1]
        chosen: list[int] = []
        k = 0
        while len(chosen) < m:
            if k < row.shape[0]:
                u = row[k]
            else:
                u = rng.random()
            k += 1
            c = int(ends[int(u * pool)])
            if c not in chosen:
                chosen.append(c)
        for c in chosen:
            src[e] = c
            dst[e] = t
            ends[pool] = c
            ends[pool + 1] = t
            e += 1
            pool += 2
    return csr_from_edges(n, src, dst)


def unit_disk(n: int, avg_degree: float, seed: int, stream: int = 0) -> Graph:
    """Points uniform in [0,1)^2, radius ``r = sqrt(avg_degree / (pi (n-1)))`` (boundary
    effects make the realised mean degree slightly lower)."""
    from scipy.spatial import cKDTree
    rng = rng_for(seed, stream)
    pts = rng.random(size=(n, 2))
    if n < 2:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    r = math.sqrt(avg_degree / (math.pi * (n - 1)))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    if pairs.size == 0:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    return csr_from_edges(n, pairs[:, 0], pairs[:, 1])


def rook(N: int) -> Graph:
    """Rook graph of an N x N board, built directly in sorted CSR order."""
    n = N * N
    deg = 2 * (N - 1)
    row_ptr = (np.arange(n + 1, dtype=np.int64) * deg)
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("board too large for int32 CSR")
    i = np.arange(N, dtype=np.int64)[:, None]
    j = np.arange(N, dtype=np.int64)[None, :]
    cols = np.empty((N, N, deg), dtype=np.int32)
    k = np.arange(N, dtype=np.int64)
    # column mates above (k < i), row mates (k != j), column mates below (k > i)
    for a in range(N):
        for_col = k * N  # cells (k, b) have index k*N + b
        above = for_col[:a]
        below = for_col[a + 1:]
        rowmates = a * N + k
        for b in range(N):
            seg = np.concatenate([above + b, np.delete(rowmates, b), below + b])
            cols[a, b, :] = seg
    del i, j
    return Graph(n, row_ptr.astype(np.int32), cols.reshape(-1))


def rook_rect(rows: int, cols: int) -> Graph:
    """Line graph of K_{rows,cols} (a rows x cols rook board): cell (a, b) = a*cols + b,
    adjacent to the other cells of its row and of its column; sorted CSR."""
    n = rows * cols
    deg = (rows - 1) + (cols - 1)
    if n * deg > np.iinfo(np.int32).max:
        raise ValueError("board too large for int32 CSR")
    out = np.empty((rows, cols, deg), dtype=np.int32)
    kr = np.arange(rows, dtype=np.int64) * cols
    kc = np.arange(cols, dtype=np.int64)
    for a in range(rows):
        above, below = kr[:a], kr[a + 1:]
        for b in range(cols):
            out[a, b, :] = np.concatenate([above + b, np.delete(a * cols + kc, b), below + b])
    return Graph(n, (np.arange(n + 1, dtype=np.int64) * deg).astype(np.int32), out.reshape(-1))


def rook_weights_rect(rows: int, cols: int, seed: int, temperature: float = 0.1, stream: int = 1) -> np.ndarray:
    """Assignment weights w = exp(-C / T), C uniform [0, 1) fp32, as a rows x cols
    float32 matrix (row-major = cell order)."""
    C = rng_for(seed, stream).random(size=(rows, cols), dtype=np.float32)
    return np.exp(-C.astype(np.float64) / temperature).astype(np.float32)


def hub_graph(n: int, hub_degrees, background_degree: float, seed: int, stream: int = 0) -> Graph:
    """Sparse ER background of the given mean degree plus one hub per entry of
    ``hub_degrees``, each joined to that many distinct random vertices: a
    ragged degree mix from 0 to the largest hub degree."""
    rng = rng_for(seed, stream)
    bg = erdos_renyi(n, background_degree / max(n - 1, 1), seed, stream + 100)
    s0, d0 = edges_of(bg)
    srcs, dsts = [s0], [d0]
    hubs = rng.choice(n, size=len(hub_degrees), replace=False)
    for h, d in zip(hubs, hub_degrees):
        others = rng.choice(n - 1, size=int(d), replace=False)
        others = others + (others >= h)
        srcs.append(np.full(int(d), h, dtype=np.int64))
        dsts.append(others.astype(np.int64))
    return csr_from_edges(n, np.concatenate(srcs), np.concatenate(dsts), dedup=True)


def weights_uniform01(n: int, seed: int, stream: int = 1) -> np.ndarray:
    """w = 1 - u with u uniform on [0, 1) in fp32: values in (0, 1], exact in fp32."""
    u = rng_for(seed, stream).random(size=n, dtype=np.float32)
    return (np.float32(1.0) - u).astype(np.float32)


def weights_uniform(n: int, lo: float, hi: float, seed: int, stream: int = 1) -> np.ndarray:
    """w uniform on (lo, hi]: ``hi - (hi - lo) * u`` rounded to fp32."""
    u = rng_for(seed, stream).random(size=n)
    return (hi - (hi - lo) * u).astype(np.float32)


def rook_weights(N: int, seed: int, temperature: float = 0.1, stream: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Assignment weights ``w = exp(-C / T)`` with C uniform [0, 1) (fp32), w rounded to
    fp32.  Returns (w as an N*N vector in cell order, C as an N x N matrix)."""
    C = rng_for(seed, stream).random(size=(N, N), dtype=np.float32)
    w = np.exp(-C.astype(np.float64) / temperature).astype(np.float32)
    return w.reshape(-1), C


def batch_sizes_loguniform(count: int, lo: int, hi: int, seed: int, stream: int = 7) -> np.ndarray:
    """n_g = floor(exp(U(ln lo, ln hi)))."""
    u = rng_for(seed, stream).random(size=count)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def concat_graphs(graphs: list[Graph]) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Concatenate graphs into per-graph sizes and *local* CSR arrays back to back.

    Returns (n[count] int32, nnz[count] int64, row_ptr_cat int32 (sum(n)+count entries:
    each graph's own row_ptr, starting at 0), col_idx_cat int32 (local column ids))."""
    ns = np.array([g.n for g in graphs], dtype=np.int32)
    nnzs = np.array([g.nnz for g in graphs], dtype=np.int64)
    rp = np.concatenate([g.row_ptr for g in graphs]).astype(np.int32) if graphs else np.zeros(0, np.int32)
    ci = np.concatenate([g.col_idx for g in graphs]).astype(np.int32) if graphs else np.zeros(0, np.int32)
    return ns, nnzs, rp, ci


def batch_workload(count: int = 4096, seed: int = 0, n_lo: int = 50, n_hi: int = 5000):
    """Many independent graphs of uneven sizes: n_g = floor(exp(U(ln n_lo, ln n_hi))),
    the first half Erdos-Renyi with mean degree 6, the second half unit-disk with
    radius set for mean degree 10; weights uniform (0, 1].  Graph g uses seed
    (seed, g).  Returns (graphs, weights)."""
    ns = batch_sizes_loguniform(count, n_lo, n_hi, seed)
    graphs, weights = [], []
    half = count // 2
    for g in range(count):
        n = int(ns[g])
        gseed = seed * 1_000_003 + g
        if g < half:
            gr = erdos_renyi(n, 6.0 / max(n - 1, 1), gseed)
        else:
            gr = unit_disk(n, 10.0, gseed)
        graphs.append(gr)
        weights.append(weights_uniform01(n, gseed))
    return graphs, weights


@dataclass
class CliqueInstance:
    """MWIS instance given by clique constraints (the form of the paper's AVR /
    MSCD benchmarks): clique k is members[ptr[k]:ptr[k+1]] (sorted, distinct);
    every vertex lies in at least one clique.  ``graph`` is the conflict graph,
    an edge between two vertices that share a clique."""
    n: int
    ptr: np.ndarray      # int32 [m+1]
    members: np.ndarray  # int32 [ptr[-1]]
    graph: Graph

    @property
    def m(self) -> int:
        return len(self.ptr) - 1


def clique_cover_instance(n: int, items: int, k_lo: int, k_hi: int, seed: int, stream: int = 11,
                          zipf: float = 0.0) -> CliqueInstance:
    """Routes and stops: vertex i (a route) covers k_i ~ U{k_lo..k_hi} distinct
    items (stops), drawn without replacement with probability proportional to
    (rank + 1)^-zipf (zipf = 0: uniform); the routes covering an item form a
    clique.  Empty items are dropped; cliques keep item order."""
    rng = rng_for(seed, stream)
    p = (np.arange(items, dtype=np.float64) + 1.0) ** -float(zipf)
    p /= p.sum()
    k = rng.integers(k_lo, k_hi + 1, size=n)
    rows, cols = [], []
    for i in range(n):
        its = rng.choice(items, size=int(k[i]), replace=False, p=p)
        rows.append(np.full(its.size, i, dtype=np.int64))
        cols.append(its.astype(np.int64))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    order = np.lexsort((r, c))                # by item, then vertex
    r, c = r[order], c[order]
    sizes = np.bincount(c, minlength=items)
    sizes = sizes[sizes > 0]
    ptr = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    members = r.astype(np.int32)
    # conflict graph: all pairs inside each clique
    src, dst = [], []
    for q in range(sizes.size):
        mem = members[ptr[q]:ptr[q + 1]].astype(np.int64)
        if mem.size > 1:
            a, b = np.triu_indices(mem.size, 1)
            src.append(mem[a])
            dst.append(mem[b])
    g = csr_from_edges(n, np.concatenate(src) if src else np.zeros(0, np.int64),
                       np.concatenate(dst) if dst else np.zeros(0, np.int64), dedup=True)
    return CliqueInstance(n, ptr.astype(np.int32), members, g)


def class_orders(starts: int, n_classes: int, seed: int, stream: int = 12) -> np.ndarray:
    """One uniformly random permutation of the clique classes per start (int32
    [starts, n_classes]): the randomized clique order of the LP warm start."""
    rng = rng_for(seed, stream)
    return np.stack([rng.permutation(n_classes) for _ in range(starts)]).astype(np.int32)


def jittered_temperatures(starts: int, lo: float, hi: float, seed: int, stream: int = 13) -> np.ndarray:
    """Initial temperatures uniform on [lo, hi) per start, fp32."""
    u = rng_for(seed, stream).random(size=starts)
    return (lo + (hi - lo) * u).astype(np.float32)

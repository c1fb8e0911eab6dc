"""The atom census's shared code (gn_atoms.h: per-graph classification and the
cycle-type enumeration) run on the host, summed by Burnside's lemma, against the
paper's Table atoms_10 (Appendix A) for n = 1..7 and against the oracle's
isomorphism-free census for n = 1..6.  No GPU involved."""
import os
import shutil
import subprocess

import pytest

from oracle import atoms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _table():
    rows = {}
    with open(os.path.join(ROOT, "tests", "golden", "atoms_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(t) for t in line.split()]
                rows[v[0]] = v[1:6]
    return rows


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_census_matches_table_and_oracle(tmp_path):
    exe = tmp_path / "atoms_check"
    cmd = ["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "paper_2605_05330_amd", "csrc"),
           os.path.join(ROOT, "tests", "atoms_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe), "7"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout
    got = {}
    for line in out.stdout.split("\n"):
        if line.strip():
            v = [int(t) for t in line.split()]
            got[v[0]] = v[1:]
    table = _table()
    for n in range(1, 8):
        assert got[n] == table[n], n
    for n in range(1, 7):
        c = atoms.census(n)
        assert got[n] == [c.connected, c.irregular_discrete, c.irregular_continuous, c.regular_discrete,
                          c.regular_continuous], n


def _circulant(n, steps):
    m, k = 0, 0
    for i in range(n):
        for j in range(i + 1, n):
            if min(j - i, n - (j - i)) in steps:
                m |= 1 << k
            k += 1
    return m


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("n", [9, 10])
def test_host_classification_matches_oracle(tmp_path, n):
    """At n = 9 and 10 the census packs the adjacency rows at an n-bit stride
    (81 and 100 bits).  Its per-graph classification (connected, regular, not
    atomic / discrete / continuous) is compared with the oracle's exact
    rational solve and LP on n-vertex graphs: the circulants, random graphs
    over a range of densities, and, from a larger random pool, graphs the host
    code puts in each class (the oracle then decides each of them
    independently)."""
    exe = tmp_path / "atoms_check"
    cmd = ["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "paper_2605_05330_amd", "csrc"),
           os.path.join(ROOT, "tests", "atoms_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def host(masks):
        out = subprocess.run([str(exe), "classify", str(n)], input="\n".join(map(str, masks)) + "\n",
                             capture_output=True, text=True, timeout=300)
        assert out.returncode == 0
        return [tuple(int(t) for t in line.split()) for line in out.stdout.split("\n") if line.strip()]

    import numpy as np
    rng = np.random.default_rng(2605 + n)
    m = n * (n - 1) // 2
    weights = 1 << np.arange(m, dtype=np.int64)
    steps = list(range(1, n // 2 + 1))
    fixed = [_circulant(n, {d for b, d in enumerate(steps) if (s >> b) & 1}) for s in range(1 << len(steps))]
    fixed += [int(((rng.random(m) < p) * weights).sum()) for p in (0.2, 0.35, 0.5, 0.65, 0.8, 0.95) for _ in range(60)]
    pool = [int(((rng.random(m) < p) * weights).sum()) for p in (0.5, 0.7, 0.8, 0.9) for _ in range(50000)]
    picked, per_class = [], {}
    for g, (conn, reg, cls) in zip(pool, host(pool)):
        key = (reg, cls)
        if conn and cls >= 0 and per_class.get(key, 0) < 25:
            per_class[key] = per_class.get(key, 0) + 1
            picked.append(g)
    masks = fixed + picked
    seen = {"disconnected": 0, "not atomic": 0, "discrete": 0, "continuous": 0}
    for g, (conn, reg, cls) in zip(masks, host(masks)):
        A = atoms.adjacency(n, g)
        assert conn == int(atoms.is_connected(A)), g
        if not conn:
            seen["disconnected"] += 1
            continue
        assert reg == int(len({sum(row) for row in A}) == 1), g
        ref = atoms.classify(A)
        assert cls == (-1 if ref is None else (0 if ref[1] else 1)), g
        seen["not atomic" if ref is None else ("discrete" if ref[1] else "continuous")] += 1
    assert min(seen.values()) >= 5, seen


def test_marked_vertex_form_of_the_labelled_count():
    """The census counts the labelled graphs of Burnside's identity term in a
    two-level marked-vertex form: mark a vertex of maximum degree d, relabel it
    0 with neighbours A = {1..d}; mark a vertex of largest degree within A,
    relabel it 1 with neighbours {0} u {2..a+1} u {d+1..d+b}; then sum
    n C(n-1, d) d C(d-1, a) C(n-1-d, b) P(G) / (k(G) k'(G)) over the graphs
    with those neighbourhoods, no degree above d and no vertex of A above
    vertex 1's degree (k: the vertices of degree d; k': those of A with
    vertex 1's degree).  Checked here against plain enumeration of every
    labelled graph, with the oracle deciding connectivity and the atomic class
    (n = 4, 5: all classes; n = 6: connected graphs)."""
    from fractions import Fraction
    from math import comb

    def key(A, full):
        if not atoms.is_connected(A):
            return None
        if not full:
            return "connected"
        c = atoms.classify(A)
        return "connected" if c is None else ("regular" if c[0] else "irregular", "discrete" if c[1] else "continuous")

    def add(acc, k, w):
        acc[k] = acc.get(k, 0) + w
        if k != "connected":
            acc["connected"] = acc.get("connected", 0) + w

    for n, full in ((4, True), (5, True), (6, False)):
        P = atoms.pairs(n)
        plain = {}
        for mask in range(1 << len(P)):
            k = key(atoms.adjacency(n, mask), full)
            if k is not None:
                add(plain, k, 1)
        marked = {}
        rest = [(i, j) for (i, j) in P if i >= 2]
        for d in range(1, n):
            for a in range(d):
                for b in range(n - d):
                    if 1 + a + b > d:
                        continue
                    fac = n * comb(n - 1, d) * d * comb(d - 1, a) * comb(n - 1 - d, b)
                    for sub in range(1 << len(rest)):
                        A = [[0] * n for _ in range(n)]
                        for j in range(1, d + 1):
                            A[0][j] = A[j][0] = 1
                        for j in list(range(2, a + 2)) + list(range(d + 1, d + 1 + b)):
                            A[1][j] = A[j][1] = 1
                        for bit, (i, j) in enumerate(rest):
                            if (sub >> bit) & 1:
                                A[i][j] = A[j][i] = 1
                        deg = [sum(r) for r in A]
                        if max(deg[1:]) > d or max(deg[1:d + 1]) > deg[1]:
                            continue
                        k = key(A, full)
                        if k is None:
                            continue
                        kk = sum(1 for v in range(1, d + 1) if deg[v] == deg[1])
                        add(marked, k, Fraction(fac, deg.count(d) * kk))
        assert marked == plain, (n, marked, plain)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_nullity_one_line_test_matches_subset_search(tmp_path):
    """Singular systems of nullity one are decided in closed form (the
    solutions of B x = 1 are a line; a positive point exists iff an interval
    of the line parameter is non-empty).  On random graphs of 8, 9 and 10
    vertices whose B, or twin quotient's B, has nullity one, the test agrees
    with the subset search over bases, and both outcomes occur."""
    exe = tmp_path / "atoms_check"
    cmd = ["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "paper_2605_05330_amd", "csrc"),
           os.path.join(ROOT, "tests", "atoms_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    for n in (8, 9, 10):
        out = subprocess.run([str(exe), "linecheck", str(n), "1500000", str(n)], capture_output=True, text=True,
                             timeout=300)
        assert out.returncode == 0
        tested, agree, positive = (int(t) for t in out.stdout.split())
        assert tested >= 1000 and agree == tested and 0 < positive < tested, (n, tested, agree, positive)

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
def test_host_classification_9_vertices_matches_oracle(tmp_path):
    """The census at n = 9 packs the adjacency rows at a 9-bit stride (81 bits).
    Its per-graph classification (connected, regular, not atomic / discrete /
    continuous) is compared with the oracle's exact rational solve and LP on
    9-vertex graphs: the 16 circulants, random graphs over a range of
    densities, and, from a larger random pool, graphs the host code puts in
    each class (the oracle then decides each of them independently)."""
    exe = tmp_path / "atoms_check"
    cmd = ["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "paper_2605_05330_amd", "csrc"),
           os.path.join(ROOT, "tests", "atoms_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def host(masks):
        out = subprocess.run([str(exe), "classify", "9"], input="\n".join(map(str, masks)) + "\n",
                             capture_output=True, text=True, timeout=300)
        assert out.returncode == 0
        return [tuple(int(t) for t in line.split()) for line in out.stdout.split("\n") if line.strip()]

    import numpy as np
    rng = np.random.default_rng(2605)
    weights = 1 << np.arange(36, dtype=np.int64)
    fixed = [_circulant(9, set(s)) for s in range(16) for s in [[d for d in (1, 2, 3, 4) if (s >> (d - 1)) & 1]]]
    fixed += [int(((rng.random(36) < p) * weights).sum()) for p in (0.2, 0.35, 0.5, 0.65, 0.8, 0.95) for _ in range(60)]
    pool = [int(((rng.random(36) < p) * weights).sum()) for p in (0.5, 0.7, 0.8, 0.9) for _ in range(50000)]
    picked, per_class = [], {}
    for m, (conn, reg, cls) in zip(pool, host(pool)):
        key = (reg, cls)
        if conn and cls >= 0 and per_class.get(key, 0) < 25:
            per_class[key] = per_class.get(key, 0) + 1
            picked.append(m)
    masks = fixed + picked
    seen = {"disconnected": 0, "not atomic": 0, "discrete": 0, "continuous": 0}
    for m, (conn, reg, cls) in zip(masks, host(masks)):
        A = atoms.adjacency(9, m)
        assert conn == int(atoms.is_connected(A)), m
        if not conn:
            seen["disconnected"] += 1
            continue
        assert reg == int(len({sum(row) for row in A}) == 1), m
        ref = atoms.classify(A)
        assert cls == (-1 if ref is None else (0 if ref[1] else 1)), m
        seen["not atomic" if ref is None else ("discrete" if ref[1] else "continuous")] += 1
    assert min(seen.values()) >= 5, seen

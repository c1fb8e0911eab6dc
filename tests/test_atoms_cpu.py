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

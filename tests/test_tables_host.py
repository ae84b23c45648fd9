"""Host table builder of the library (csrc/tables.cpp) on the CPU: a small harness built
with g++ prints the tables of seeded balanced hierarchies, which must equal tables
derived here by brute force from the oct coordinates (Morton order, same-level
neighbour octs, parent cells, coarse neighbour cells at faces towards a coarser leaf,
child marks and leaf counts); malformed hierarchies are rejected with a reason.  Every
case runs twice: with a plain build and with AddressSanitizer and UndefinedBehaviorSanitizer
(any report aborts the harness, which fails the test)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from synth.hierarchy import random_balanced_hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_1112_amd", "csrc")
OFF = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


SANITIZE = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module", params=["plain", "asan_ubsan"])
def harness(request, tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tables") / f"tables_dump_{request.param}")
    extra = SANITIZE if request.param == "asan_ubsan" else []
    subprocess.run(["g++", "-O1", "-std=c++17"] + extra + ["-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "tables_dump.cpp"), os.path.join(CSRC, "tables.cpp"),
                    "-o", exe], check=True)
    return exe


def _dump(harness, tmp_path, levels):
    path = tmp_path / "h.bin"
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(levels)))
        for lvl, octs in levels:
            a = np.ascontiguousarray(np.asarray(octs, dtype=np.int32).reshape(-1, 3))
            f.write(struct.pack("<iq", lvl, len(a)))
            f.write(a.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")
    run = subprocess.run([harness, str(path)], capture_output=True, text=True, env=env)
    assert run.returncode == 0, (run.returncode, run.stderr[-4000:])
    out = run.stdout.splitlines()
    if out and out[0].startswith("ERR"):
        return out[0]
    tabs, k = {}, 0
    while k < len(out):
        lvl, n_oct, n_leaf = (int(x) for x in out[k].split())
        arr = [np.array(out[k + j].split(), dtype=np.int64) if out[k + j] else np.zeros(0, np.int64)
               for j in range(1, 6)]
        tabs[lvl] = dict(n_oct=n_oct, n_leaf=n_leaf, ijk=arr[0].reshape(-1, 3), nbr=arr[1].reshape(-1, 6),
                         cnb=arr[2].reshape(-1, 6), parent=arr[3], child=arr[4])
        k += 6
    return tabs


def _morton(i, j, k):
    key = 0
    for b in range(21):
        key |= ((i >> b) & 1) << (3 * b) | ((j >> b) & 1) << (3 * b + 1) | ((k >> b) & 1) << (3 * b + 2)
    return key


def _brute(levels):
    """Tables of every level from the coordinates alone."""
    out = {}
    for idx, (lvl, octs) in enumerate(levels):
        n_side = 1 << (lvl - 1)
        ijk = sorted((tuple(int(v) for v in o) for o in np.asarray(octs).reshape(-1, 3)), key=lambda c: _morton(*c))
        pos = {c: o for o, c in enumerate(ijk)}
        n = len(ijk)
        nbr = -np.ones((n, 6), np.int64)
        cnb = -np.ones((n, 6), np.int64)
        parent = -np.ones(n, np.int64)
        for o, (I, J, K) in enumerate(ijk):
            for d, (dx, dy, dz) in enumerate(OFF):
                a, b, c = I + dx, J + dy, K + dz
                if min(a, b, c) < 0 or max(a, b, c) >= n_side:
                    continue
                nbr[o, d] = pos.get((a, b, c), -1)
                if idx > 0 and nbr[o, d] < 0:
                    cpos = out[levels[idx - 1][0]]["pos"]
                    cnb[o, d] = 8 * cpos[(a >> 1, b >> 1, c >> 1)] + ((a & 1) | (b & 1) << 1 | (c & 1) << 2)
            if idx > 0:
                cpos = out[levels[idx - 1][0]]["pos"]
                parent[o] = 8 * cpos[(I >> 1, J >> 1, K >> 1)] + ((I & 1) | (J & 1) << 1 | (K & 1) << 2)
        out[lvl] = dict(n_oct=n, n_leaf=8 * n, ijk=np.array(ijk, np.int64).reshape(-1, 3), nbr=nbr, cnb=cnb,
                        parent=parent, child=-np.ones(8 * n, np.int64), pos=pos)
        if idx > 0:
            coarse = out[levels[idx - 1][0]]
            for o in range(n):
                coarse["child"][parent[o]] = o
            coarse["n_leaf"] -= n
    return out


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tables_equal_brute_force(harness, tmp_path, seed):
    h = random_balanced_hierarchy(seed, 3, 6, p_refine=0.5)
    levels = [(l, h.octs[l]) for l in sorted(h.octs)]
    assert len(levels) == 4
    got, ref = _dump(harness, tmp_path, levels), _brute(levels)
    assert not isinstance(got, str), got
    for l in ref:
        for name in ("n_oct", "n_leaf"):
            assert got[l][name] == ref[l][name], (l, name)
        for name in ("ijk", "nbr", "cnb", "parent", "child"):
            assert np.array_equal(got[l][name], ref[l][name]), (l, name)


def _full(level):
    n = 1 << (level - 1)
    return np.array([(i, j, k) for k in range(n) for j in range(n) for i in range(n)], np.int32)


@pytest.mark.parametrize("case,reason", [
    ("duplicate", "duplicate oct"),
    ("out_of_range", "out of range"),
    ("base_incomplete", "base level"),
    ("no_parent", "without a parent"),
    ("unbalanced", "unbalanced"),
])
def test_malformed_hierarchies_rejected(harness, tmp_path, case, reason):
    base = _full(2)  # 2^3 octs: the coarse box of 4^3 cells
    if case == "duplicate":
        levels = [(2, base), (3, np.array([[0, 0, 0], [0, 0, 0]]))]
    elif case == "out_of_range":
        levels = [(2, base), (3, np.array([[4, 0, 0]]))]
    elif case == "base_incomplete":
        levels = [(2, base[:-1])]
    elif case == "no_parent":
        # level 4 oct under a level-3 cell that is not refined
        levels = [(2, base), (3, np.array([[0, 0, 0]])), (4, np.array([[6, 6, 6]]))]
    else:
        # a level-4 oct next to a level-2 leaf: its parent's face neighbour at level 3 is missing
        levels = [(2, base), (3, np.array([[1, 1, 1]])), (4, np.array([[3, 2, 2]]))]
    got = _dump(harness, tmp_path, levels)
    assert isinstance(got, str) and got.startswith("ERR") and reason in got, got

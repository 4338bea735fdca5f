"""The pins are strong enough: plant plausible mistakes in a copy of the oracle
source (on the CPU, in a temporary directory) and check that every mutant
fails at least one pin.  The real oracle is never modified."""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from tests import bruteforce

SRC = os.path.join(os.path.dirname(oracle.__file__), "afps_oracle.c")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")

MUTANTS = {
    "drop_dz": ("return xy + zz;", "return xy;"),
    "wrong_sign": ("float dy = p[1] - q[1];", "float dy = p[1] + q[1];"),
    "wrong_coordinate": ("float dz = p[2] - q[2];", "float dz = p[2] - q[1];"),
    "transposed_operand": ("float d = squared_distance(pts + 3 * (int64_t)j, sample);",
                           "float d = squared_distance(pts + 3 * (int64_t)j, pts + 3 * (int64_t)(j - (j > 0)));"),
    "tie_to_highest": ("if (dist[j] > dist[far])", "if (dist[j] >= dist[far])"),
    "update_reversed": ("dist[j] = d < dist[j] ? d : dist[j];", "dist[j] = d > dist[j] ? d : dist[j];"),
    "sample_split_floor": ("*first_sample = s * qc + (s < rc ? s : rc);",
                           "*first_sample = s * qc + (s < rc ? 0 : rc);"),
    "point_split_last": ("*num_points = qn + (s < rn ? 1 : 0);",
                         "*num_points = qn + (s >= m - rn ? 1 : 0);"),
    "window_floor_ceil_swapped": ("below = k / 2;                                 /* the sample and k neighbours */\n        above = k - k / 2;",
                                  "below = k - k / 2;\n        above = k / 2;"),
    "window_excludes_top": ("*hi = to > n - 1 ? n - 1 : (int32_t)to;", "*hi = to > n - 1 ? n - 1 : (int32_t)to - 1;"),
    "start_not_local": ("int32_t pick = start % n;", "int32_t pick = 0;"),
    "initial_1e9": ("INITIAL_DISTANCE = 1e10f;", "INITIAL_DISTANCE = 1e9f;"),
    "local_output_index": ("out[t] = first + pick;", "out[t] = pick;"),
    "npdu_full_first_pass": ("const int whole = k < 0 || (t == 1 && (flags & ORACLE_NPDU_FIRST_FULL));",
                             "const int whole = k < 0 || t == 1;"),
    "first_full_every_iteration": ("(t == 1 && (flags & ORACLE_NPDU_FIRST_FULL))",
                                   "(flags & ORACLE_NPDU_FIRST_FULL)"),
    "shift_wrong_way": ("            to -= from;", "            to += from;"),
    "shift_never_left": ("            from -= to - (n - 1);", "            from -= 0;"),
    "self_window_not_reduced": ("below = (k - 1) / 2;", "below = k / 2;"),
}


def _pins_pass(lib) -> bool:
    with open(GOLDEN) as f:
        for case in json.load(f)["cases"]:
            pts = np.array(case["points"], dtype=np.float32)
            try:
                got = oracle.afps(pts, case["c"], case["m"], case["k"], case["start"], lib=lib,
                                  flags=case.get("flags", 0))
            except oracle.OracleError:
                return False
            if got.tolist() != case["expected"]:
                return False
    rng = np.random.default_rng(99)
    for _ in range(40):
        n = int(rng.integers(2, 40))
        pts = rng.random((n, 3), dtype=np.float32)
        c = int(rng.integers(1, n + 1))
        m = int(rng.integers(1, c + 1))
        k = [None, 0, 1, 3, 6][int(rng.integers(0, 5))]
        start = int(rng.integers(0, n))
        try:
            got = oracle.afps(pts, c, m, k, start, lib=lib)
        except oracle.OracleError:
            return False
        if got.tolist() != bruteforce.afps(pts, c, m, k, start).tolist():
            return False
    for flags in (1, 2, 4, 7):                  # the alternative NPDU readings
        for _ in range(12):
            n = int(rng.integers(2, 40))
            pts = rng.random((n, 3), dtype=np.float32)
            c = int(rng.integers(1, n + 1))
            m = int(rng.integers(1, c + 1))
            k = [1, 2, 3, 6][int(rng.integers(0, 4))]
            start = int(rng.integers(0, n))
            try:
                got = oracle.afps(pts, c, m, k, start, lib=lib, flags=flags)
            except oracle.OracleError:
                return False
            if got.tolist() != bruteforce.afps(pts, c, m, k, start, flags).tolist():
                return False
    return True


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


def test_unmutated_copy_passes(workdir):
    path = str(workdir / "liboracle_copy.so")
    shutil.copy(SRC, str(workdir / "copy.c"))
    oracle.build(path, str(workdir / "copy.c"))
    assert _pins_pass(oracle.load(path))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, "mutation anchor not found: " + name
    src = workdir / (name + ".c")
    src.write_text(text.replace(old, new))
    path = str(workdir / ("lib" + name + ".so"))
    oracle.build(path, str(src))
    assert not _pins_pass(oracle.load(path)), "pins did not catch mutant " + name

"""The oracle's spherical-harmonic matrices against the values the paper
prints for its worked examples (text fixtures under tests/golden/, each
naming the equation it copies the numbers from)."""

import os

import numpy as np
import pytest

from oracle import sh

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _entries(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        f = line.split()
        out.append((f[0], tuple(map(int, f[1:4])), tuple(map(int, f[4:7])), float(f[7])))
    return out


def _matrices():
    S = sh.system_matrices(1)
    return {
        "Ax": S["A"][0],
        "Omz": S["Om"][2],
        "AxAx": S["AA"][0, 0],
        "G1": S["AOm"][1, 2] - S["AOm"][2, 1],
        "G2": S["AAOm"][0, 1, 2] - S["AAOm"][0, 2, 1],
        "C": np.diag(S["C"]) if np.ndim(S["C"]) == 1 else S["C"],
    }


@pytest.mark.parametrize("fixture", ["convergence_study_lmax1.txt", "shock_system_lmax1.txt"])
def test_printed_entries(fixture):
    mats = _matrices()
    ent = _entries(fixture)
    assert ent
    for mat, row, col, val in ent:
        M = mats[mat]
        got = M[sh.lms_index(*row), sh.lms_index(*col)]
        assert abs(got - val) < 1e-13, (fixture, mat, row, col, got, val)


def test_convergence_rows_have_no_other_entries():
    """The printed convergence-study system lists every non-zero of A^x and
    Omega^z at l_max = 1."""
    mats = _matrices()
    listed = {}
    for mat, row, col, _ in _entries("convergence_study_lmax1.txt"):
        listed.setdefault(mat, set()).add((sh.lms_index(*row), sh.lms_index(*col)))
    for mat, pos in listed.items():
        M = mats[mat]
        for i in range(M.shape[0]):
            for j in range(M.shape[1]):
                if (i, j) not in pos:
                    assert abs(M[i, j]) < 1e-14, (mat, i, j, M[i, j])

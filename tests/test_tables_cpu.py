"""The compile-time 1-D basis tables of the (x, ln p) kernels (basis.hpp,
written out by hand in closed form) against the oracle's Lagrange basis on
the Gauss-Lobatto nodes and Gauss rule: phi, its derivative, the exact mass
matrix, the test matrices with the inverse mass folded in, and the lifts.
basis.hpp is plain C++: it is compiled here with the host compiler."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_05110_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "basis.hpp"
template <int K> void dump() {
  using B = vfp::CBasis<K>;
  constexpr int K1 = K + 1;
  auto m = [](const char* n, const double (*a)[K1], int rows) {
    std::printf("%s", n);
    for (int i = 0; i < rows; ++i)
      for (int j = 0; j < K1; ++j) std::printf(" %.17g", a[i][j]);
    std::printf("\n");
  };
  std::printf("K %d\n", K);
  m("phi", B::phi, K1); m("dphi", B::dphi, K1); m("mass", B::mass, K1);
  m("tst", B::tst, K1); m("dtst", B::dtst, K1); m("lift", B::lift, 2);
}
int main() { dump<1>(); dump<2>(); return 0; }
"""


def _compile_and_run(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "dump.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "dump"
    subprocess.run([cxx, "-std=c++17", "-O0", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    tables, k = {}, None
    for line in out.splitlines():
        f = line.split()
        if f[0] == "K":
            k = int(f[1])
            tables[k] = {}
        else:
            tables[k][f[0]] = np.array([float(v) for v in f[1:]])
    return tables


def test_basis_tables_match_oracle(tmp_path):
    tables = _compile_and_run(tmp_path)
    for k in (1, 2):
        K1 = k + 1
        g, w = dg.gauss_rule(K1)
        phi, dphi = dg.lagrange(dg.lobatto_nodes(k), g)            # [q][j]
        mass = phi.T @ np.diag(w) @ phi
        minv = np.linalg.inv(mass)
        tst = minv @ phi.T @ np.diag(w)                             # [i][q]
        dtst = minv @ dphi.T @ np.diag(w)
        lift = np.stack([minv[:, 0], minv[:, k]])
        want = {"phi": phi, "dphi": dphi, "mass": mass, "tst": tst, "dtst": dtst, "lift": lift}
        for name, ref in want.items():
            got = tables[k][name].reshape(ref.shape)
            np.testing.assert_allclose(got, ref, atol=1e-14, err_msg=f"k={k} {name}")

"""Pins of the oracle's spherical-harmonic algebra against what the paper fixes.

The oracle builds every matrix by sphere quadrature; these tests compare with
the paper's closed forms (retyped here from the equations cited), its
explicit tables, and algebraic identities.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sl
from numpy.polynomial import legendre as npleg

from oracle import sh

LMAXES = [1, 2, 3, 5]


def _random_dirs(n=50, seed=0):
    g = np.random.default_rng(seed)
    v = g.standard_normal((3, n))
    return v / np.linalg.norm(v, axis=0)


def test_index_map_order():
    # eq. ordering-expansion-coefficients: (f000, f110, f100, f111, f220, f210, f200, f211, f221)
    want = [(0, 0, 0), (1, 1, 0), (1, 0, 0), (1, 1, 1), (2, 2, 0), (2, 1, 0),
            (2, 0, 0), (2, 1, 1), (2, 2, 1)]
    assert sh.lms_list(2) == want


def test_real_harmonics_table():
    """App. A, table of real spherical harmonics for l <= 2 (theta from x)."""
    X = _random_dirs()
    ct = X[0]
    st = np.sqrt(1 - ct ** 2)
    phi = np.arctan2(X[2], X[1])
    pi = math.pi
    table = {
        (0, 0, 0): np.full_like(ct, math.sqrt(1 / (4 * pi))),
        (1, 0, 0): math.sqrt(3 / (4 * pi)) * ct,
        (1, 1, 0): -math.sqrt(3 / (4 * pi)) * st * np.cos(phi),
        (1, 1, 1): -math.sqrt(3 / (4 * pi)) * st * np.sin(phi),
        (2, 0, 0): 0.25 * math.sqrt(5 / pi) * (3 * ct ** 2 - 1),
        (2, 1, 0): -0.5 * math.sqrt(15 / pi) * st * ct * np.cos(phi),
        (2, 1, 1): -0.5 * math.sqrt(15 / pi) * st * ct * np.sin(phi),
        (2, 2, 0): 0.25 * math.sqrt(15 / pi) * st ** 2 * np.cos(2 * phi),
        (2, 2, 1): 0.25 * math.sqrt(15 / pi) * st ** 2 * np.sin(2 * phi),
    }
    Y = sh.real_sph_harm(2, X)
    for lms, ref in table.items():
        np.testing.assert_allclose(Y[sh.lms_index(*lms)], ref, atol=1e-14)


@pytest.mark.parametrize("lmax", LMAXES)
def test_orthonormal(lmax):
    """App. A: int Y_l'm's' Y_lms dOmega = delta."""
    pts, w = sh.sphere_quadrature(2 * lmax + 2)
    Y = sh.real_sph_harm(lmax, pts)
    np.testing.assert_allclose(Y @ (w[:, None] * Y.T), np.eye(Y.shape[0]), atol=1e-13)


def _Ax_closed(lmax):
    """eq. representation-matrix-Ax."""
    n = (lmax + 1) ** 2
    M = np.zeros((n, n))
    for (l, m, s) in sh.lms_list(lmax):
        j = sh.lms_index(l, m, s)
        if l + 1 <= lmax:
            M[sh.lms_index(l + 1, m, s), j] = math.sqrt(
                (l + m + 1) * (l - m + 1) / ((2 * l + 3) * (2 * l + 1)))
        if l - 1 >= m:
            M[sh.lms_index(l - 1, m, s), j] = math.sqrt(
                (l + m) * (l - m) / ((2 * l + 1) * (2 * l - 1)))
    return M


def _Omx_closed(lmax):
    """eq. representation-matrix-Omegax."""
    n = (lmax + 1) ** 2
    M = np.zeros((n, n))
    for (l, m, s) in sh.lms_list(lmax):
        for sp in (0, 1):
            if m == 0 and sp == 1:
                continue
            i = sh.lms_index(l, m, sp)
            j = sh.lms_index(l, m, s)
            M[i, j] = m * ((sp == 0 and s == 1) / math.sqrt(1 + (m == 0))
                           - (sp == 1 and s == 0) / math.sqrt(1 + (m == 0)))
    return M


@pytest.mark.parametrize("lmax", LMAXES)
def test_Ax_Omx_closed_forms(lmax):
    A = sh.direction_matrices(lmax)
    Om = sh.rotation_generators(lmax)
    np.testing.assert_allclose(A[0], _Ax_closed(lmax), atol=1e-13)
    np.testing.assert_allclose(Om[0], _Omx_closed(lmax), atol=1e-13)


@pytest.mark.parametrize("lmax", LMAXES)
def test_symmetry_and_commutators(lmax):
    """A symmetric, Omega antisymmetric (Sec. 2.1); angular-momentum algebra."""
    A = sh.direction_matrices(lmax)
    Om = sh.rotation_generators(lmax)
    for a in range(3):
        np.testing.assert_allclose(A[a], A[a].T, atol=1e-14)
        np.testing.assert_allclose(Om[a], -Om[a].T, atol=1e-13)
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        np.testing.assert_allclose(Om[a] @ Om[b] - Om[b] @ Om[a], -Om[c], atol=1e-12)


@pytest.mark.parametrize("lmax", LMAXES)
def test_rotation_relations(lmax):
    """eq. real-direction-op-matrices-and-rotations and the Omega analogue."""
    A = sh.direction_matrices(lmax)
    Om = sh.rotation_generators(lmax)
    Rz = sl.expm(math.pi / 2 * Om[2])
    Rx = sl.expm(math.pi / 2 * Om[0])
    np.testing.assert_allclose(Rz.T @ A[0] @ Rz, A[1], atol=1e-12)
    np.testing.assert_allclose(Rx.T @ A[1] @ Rx, A[2], atol=1e-12)
    np.testing.assert_allclose(Rz.T @ Om[0] @ Rz, Om[1], atol=1e-12)
    np.testing.assert_allclose(Rx.T @ Om[1] @ Rx, Om[2], atol=1e-12)
    np.testing.assert_allclose(sl.expm(-math.pi / 2 * Om[2]), Rz.T, atol=1e-12)


def _u(lp, mp, l, m):
    """eq. complex-rotation; sum over k with non-negative factorial arguments."""
    if lp != l:
        return 0.0
    tot = 0.0
    for k in range(0, 2 * l + 1):
        args = (l - mp - k, l - m - k, mp + m + k)
        if min(args) < 0:
            continue
        tot += (-1) ** k * math.sqrt(math.factorial(l + mp) * math.factorial(l - mp)
                                     * math.factorial(l + m) * math.factorial(l - m)) / (
            math.factorial(k) * math.factorial(args[0]) * math.factorial(args[1])
            * math.factorial(args[2]))
    return (-1) ** (l - mp) / 2 ** l * tot


@pytest.mark.parametrize("lmax", [1, 2, 3, 4])
def test_rotation_matrix_z_closed_form(lmax):
    """eq. representation-matrix-Uz equals expm(pi/2 Omega^z)."""
    n = (lmax + 1) ** 2
    M = np.zeros((n, n))
    for (lp, mp, sp) in sh.lms_list(lmax):
        for (l, m, s) in sh.lms_list(lmax):
            v = 0.0
            if sp == 0 and s == 0:
                v = (_u(lp, mp, l, m) + (-1) ** m * _u(lp, mp, l, -m)) / math.sqrt(
                    (1 + (mp == 0)) * (1 + (m == 0)))
            elif sp == 1 and s == 1:
                v = _u(lp, mp, l, m) - (-1) ** m * _u(lp, mp, l, -m)
            M[sh.lms_index(lp, mp, sp), sh.lms_index(l, m, s)] = v
    Om = sh.rotation_generators(lmax)
    np.testing.assert_allclose(sl.expm(math.pi / 2 * Om[2]), M, atol=1e-12)


@pytest.mark.parametrize("lmax", [1, 2, 3, 4])
def test_rotation_matrix_x_closed_form_transposed(lmax):
    """eq. representation-matrix-Ux as printed equals expm(-pi/2 Omega^x), i.e.
    it is the transpose of expm(+pi/2 Omega^x) (a sign reading of that eq.)."""
    n = (lmax + 1) ** 2
    M = np.zeros((n, n))
    for (lp, mp, sp) in sh.lms_list(lmax):
        for (l, m, s) in sh.lms_list(lmax):
            if lp != l or mp != m:
                continue
            c, si = math.cos(math.pi / 2 * m), math.sin(math.pi / 2 * m)
            v = 0.0
            if sp == 0 and s == 0:
                v = (c + (mp == 0) * (m == 0)) / math.sqrt((1 + (mp == 0)) * (1 + (m == 0)))
            if sp == 1 and s == 0:
                v += si / math.sqrt(1 + (mp == 0))
            if sp == 0 and s == 1:
                v -= si / math.sqrt(1 + (m == 0))
            if sp == 1 and s == 1:
                v += c
            M[sh.lms_index(lp, mp, sp), sh.lms_index(l, m, s)] = v
    Om = sh.rotation_generators(lmax)
    np.testing.assert_allclose(sl.expm(-math.pi / 2 * Om[0]), M, atol=1e-12)
    np.testing.assert_allclose(sl.expm(math.pi / 2 * Om[0]), M.T, atol=1e-12)


@pytest.mark.parametrize("lmax", LMAXES)
def test_equal_spectra_and_lambda_max(lmax):
    """Same eigenvalues for A^x, A^y, A^z (Sec. 3.2); those of A^x are the
    roots of the Legendre polynomials of degree m..l_max+1 blocks, the
    largest being the largest root of P_{l_max+1}."""
    A = sh.direction_matrices(lmax)
    ev = [np.sort(np.linalg.eigvalsh(A[a])) for a in range(3)]
    np.testing.assert_allclose(ev[0], ev[1], atol=1e-12)
    np.testing.assert_allclose(ev[0], ev[2], atol=1e-12)
    c = np.zeros(lmax + 2)
    c[-1] = 1
    assert abs(ev[0][-1] - npleg.legroots(c).max()) < 1e-12


def test_collision_matrix():
    C = sh.collision_matrix(3)
    want = [l * (l + 1) / 2 for (l, m, s) in sh.lms_list(3)]
    np.testing.assert_array_equal(np.diag(C), want)


def test_shock_block_lmax1():
    """eq. actual-soe-for-sapphire (l_max = 1, B and U along x).

    In ln-p form and reading the U' coefficient of the gamma m/sqrt(3) and
    -2/(sqrt(3)V) entries as dU/dt = U U' (the general system has dU/dt
    there): (A^x A^x)_t restricted to (f000, f100) is diag(1/3, 3/5);
    (A^y Omega^z - A^z Omega^y)_t couples f000 <- f100 with -2/sqrt(3); and
    (A^x(A^y Omega^z - A^z Omega^y))_t gives -2/5 on f100 (truncation after
    multiplying -- the printed -2/5 is reached only that way)."""
    S = sh.system_matrices(1)
    i0, i1 = sh.lms_index(0, 0, 0), sh.lms_index(1, 0, 0)
    AA = S["AA"][0, 0]
    assert abs(AA[i0, i0] - 1 / 3) < 1e-14 and abs(AA[i1, i1] - 3 / 5) < 1e-14
    assert abs(AA[i0, i1]) < 1e-14
    G1 = S["AOm"][1, 2] - S["AOm"][2, 1]
    assert abs(G1[i0, i1] + 2 / math.sqrt(3)) < 1e-13
    assert abs(G1[i1, i1]) < 1e-14 and abs(G1[i0, i0]) < 1e-14
    G2 = S["AAOm"][0, 1, 2] - S["AAOm"][0, 2, 1]
    assert abs(G2[i1, i1] + 0.4) < 1e-13
    # truncating first gives -2/3 instead: the rule matters
    A, Om = sh.direction_matrices(1), sh.rotation_generators(1)
    G2_first = A[0] @ (A[1] @ Om[2] - A[2] @ Om[1])
    assert abs(G2_first[i1, i1] + 2 / 3) < 1e-13
    # beta^x block [[U, V/sqrt3],[V/sqrt3, U]] comes from A^x
    assert abs(S["A"][0][i0, i1] - 1 / math.sqrt(3)) < 1e-14


def test_convergence_study_equations():
    """eq. convergence-study-explicit-equations: with B along z the system
    d_t f + V A^x d_x f - omega Omega^z f = 0 at l_max=1 reads
    d_t f110 = omega f100, d_t f100 = -omega f110 - V/sqrt3 d_x f000, f111 frozen."""
    A = sh.direction_matrices(1)
    Om = sh.rotation_generators(1)
    i000, i110, i100, i111 = (sh.lms_index(0, 0, 0), sh.lms_index(1, 1, 0),
                              sh.lms_index(1, 0, 0), sh.lms_index(1, 1, 1))
    assert abs(Om[2][i110, i100] - 1) < 1e-14
    assert abs(Om[2][i100, i110] + 1) < 1e-14
    assert np.abs(Om[2][i111]).max() < 1e-14 and np.abs(Om[2][:, i111]).max() < 1e-14
    assert np.abs(Om[2][i000]).max() < 1e-14
    assert abs(A[0][i100, i000] - 1 / math.sqrt(3)) < 1e-14

"""Real spherical harmonics and the system matrices A^a, Omega^a, C (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Route.  Every matrix is computed by sphere quadrature of its defining integral,
never from the paper's closed forms (those serve as independent pins in the
tests):

* Y_lms is the real harmonic of App. A (eq. spherical-harmonics,
  eq. normalisation-spherical-harmonics, eq. associated-legendre-polynomials):
  Condon-Shortley phase inside P_l^m, theta measured from the x axis, so that
  p = p (cos theta, sin theta cos phi, sin theta sin phi) (Sec. 1).
* A^a_ij = int Y_i (p_a / p) Y_j dOmega   (the direction operators, Sec. 2.1).
* Omega^a_ij = int Y_i [(p x grad_p)_a Y_j] dOmega  (angular-momentum
  generators; the x component is the azimuthal derivative d/dphi, which is
  what eq. representation-matrix-Omegax states).
* C = diag(l(l+1)/2)  (eq. real-C-matrix).
* Products such as A^a A^b are formed from matrices built for L = l_max + 1
  and then cut to n x n (the truncation rule stated after eq. real-C-matrix).

Ordering follows eq. ordering-expansion-coefficients: j(l,m,s) = l(l+1) +
(-1)^(s+1) m.
"""

from __future__ import annotations

import functools
import math

import numpy as np
from numpy.polynomial import legendre as npleg


def lms_index(l: int, m: int, s: int) -> int:
    """Index map j(l,m,s) = l(l+1) + (-1)^(s+1) m, zero based (Sec. 2.1)."""
    return l * (l + 1) + (m if s == 1 else -m)


def lms_list(lmax: int):
    """All (l, m, s) triples ordered by the index map, length (lmax+1)^2."""
    out = [None] * ((lmax + 1) ** 2)
    for l in range(lmax + 1):
        for m in range(l + 1):
            for s in ((0,) if m == 0 else (0, 1)):
                out[lms_index(l, m, s)] = (l, m, s)
    return out


def _norm(l: int, m: int) -> float:
    """N_lm of eq. normalisation-spherical-harmonics."""
    return math.sqrt((2 * l + 1) / (2 * math.pi * (1 + (m == 0)))
                     * math.factorial(l - m) / math.factorial(l + m))


def _legendre_deriv(l: int, order: int, x):
    """d^order P_l / dx^order evaluated at x (P_l as in eq. legendre-polynomials)."""
    if order > l:
        return np.zeros_like(x)
    c = np.zeros(l + 1)
    c[l] = 1.0
    return npleg.legval(x, npleg.legder(c, order)) if order else npleg.legval(x, c)


def real_sph_harm(lmax: int, pts):
    """Y_lms at unit vectors pts (3, N) -> (n, N).

    Written as a polynomial in Cartesian components: with x = cos theta,
    y + i z = sin theta e^{i phi}, so sin^m theta (cos m phi, sin m phi) =
    (Re, Im) (y + i z)^m and P_l^m(x) = (-1)^m sin^m theta d^m P_l/dx^m.
    """
    x, y, z = pts
    w = y + 1j * z
    out = np.zeros(((lmax + 1) ** 2, x.shape[0]))
    for (l, m, s) in lms_list(lmax):
        radial = _norm(l, m) * (-1) ** m * _legendre_deriv(l, m, x)
        ang = w ** m
        out[lms_index(l, m, s)] = radial * (ang.imag if s else ang.real)
    return out


def directions(theta, phi):
    """Unit vectors (3, N) for polar angle theta from the x axis and azimuth
    phi about it (Sec. 1)."""
    theta = np.asarray(theta, float).ravel()
    phi = np.asarray(phi, float).ravel()
    return np.stack([np.cos(theta), np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi)])


def reconstruct(zeta, lmax: int, theta, phi):
    """f(node, d) = sum_lms zeta[node, lms] Y_lms(theta_d, phi_d)
    (eq. spherical-harmonic-exp): array (rows, ndir)."""
    n = (lmax + 1) ** 2
    Z = np.asarray(zeta, float).reshape(-1, n)
    return Z @ real_sph_harm(lmax, directions(theta, phi))


def real_sph_harm_grad(lmax: int, pts):
    """Cartesian gradient (3, n, N) of the polynomial extension used above.

    Only tangential components are used (through p x grad), for which any
    smooth extension off the sphere gives the same result.
    """
    x, y, z = pts
    w = y + 1j * z
    n = (lmax + 1) ** 2
    g = np.zeros((3, n, x.shape[0]))
    for (l, m, s) in lms_list(lmax):
        c = _norm(l, m) * (-1) ** m
        d0 = _legendre_deriv(l, m, x)
        d1 = _legendre_deriv(l, m + 1, x)
        ang = w ** m
        dang = m * w ** (m - 1) if m > 0 else np.zeros_like(w)
        j = lms_index(l, m, s)
        pick = (lambda v: v.imag) if s else (lambda v: v.real)
        g[0, j] = c * d1 * pick(ang)
        g[1, j] = c * d0 * pick(dang)
        g[2, j] = c * d0 * pick(1j * dang)
    return g


def sphere_quadrature(degree: int):
    """Gauss-Legendre in cos(theta) x uniform phi rule, exact to `degree`.

    Returns (pts (3,N), weights (N,)) with theta measured from the x axis.
    """
    nt = degree // 2 + 2
    nphi = degree + 2
    ct, wt = npleg.leggauss(nt)
    phi = 2 * math.pi * np.arange(nphi) / nphi
    CT, PH = np.meshgrid(ct, phi, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    pts = np.stack([CT.ravel(), (ST * np.cos(PH)).ravel(), (ST * np.sin(PH)).ravel()])
    wts = (wt[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).ravel()
    return pts, wts


@functools.lru_cache(maxsize=None)
def _base_matrices(L: int):
    """(A[3], Omega[3]) for truncation degree L, by quadrature."""
    pts, wts = sphere_quadrature(2 * L + 4)
    Y = real_sph_harm(L, pts)
    G = real_sph_harm_grad(L, pts)
    A = np.einsum("iq,aq,jq,q->aij", Y, pts, Y, wts)
    # (p x grad)_a = eps_abc p_b d_c
    pxg = np.stack([pts[1] * G[2] - pts[2] * G[1],
                    pts[2] * G[0] - pts[0] * G[2],
                    pts[0] * G[1] - pts[1] * G[0]])
    Om = np.einsum("iq,ajq,q->aij", Y, pxg, wts)
    A[np.abs(A) < 1e-12] = 0.0
    Om[np.abs(Om) < 1e-12] = 0.0
    return A, Om


def direction_matrices(lmax: int):
    """A^x, A^y, A^z for l_max, shape (3, n, n)."""
    return _base_matrices(lmax)[0].copy()


def rotation_generators(lmax: int):
    """Omega^x, Omega^y, Omega^z for l_max, shape (3, n, n)."""
    return _base_matrices(lmax)[1].copy()


def collision_matrix(lmax: int):
    """C = diag(l(l+1)/2), eq. real-C-matrix."""
    return np.diag([l * (l + 1) / 2.0 for (l, m, s) in lms_list(lmax)])


EPS = np.zeros((3, 3, 3))
for _a, _b, _c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    EPS[_a, _b, _c] = 1.0
    EPS[_a, _c, _b] = -1.0


@functools.lru_cache(maxsize=None)
def system_matrices(lmax: int):
    """Everything eq. real-system-of-equations needs, as a dict of arrays.

    Keys: A (3,n,n), Om (3,n,n), C (n,n), AA (3,3,n,n) = (A^a A^b)_t,
    AOm (3,3,n,n) = (A^b Omega^c)_t, AAOm (3,3,3,n,n) = (A^a A^c Omega^d)_t.
    Products use the L = l_max + 1 matrices then truncate to n x n.
    """
    n = (lmax + 1) ** 2
    A, Om = _base_matrices(lmax)
    AL, OmL = _base_matrices(lmax + 1)
    AA = np.einsum("aij,bjk->abik", AL, AL)[:, :, :n, :n]
    AOm = np.einsum("bij,cjk->bcik", AL, OmL)[:, :, :n, :n]
    AAOm = np.einsum("aij,cjk,dkl->acdil", AL, AL, OmL)[:, :, :, :n, :n]
    return {"A": A[:, :n, :n].copy(), "Om": Om[:, :n, :n].copy(),
            "C": collision_matrix(lmax), "AA": AA.copy(), "AOm": AOm.copy(),
            "AAOm": AAOm.copy(), "n": n, "lmax": lmax}

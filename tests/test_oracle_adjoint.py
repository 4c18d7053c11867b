"""Pins of the oracle's reverse mode (the discrete adjoint of classical RK4
and the scattering-frequency gradient).

These check the oracle against the mathematics, not against itself:
  * the transpose identity <dJ/dz0, dz0> = <g, dzN> for J = <g, z_N>, with dzN
    from the forward (linear part) -- any dropped or mis-ordered stage breaks it;
  * the scattering gradient against central finite differences of the
    forward run;
  * the scattering gradient of a uniform state against the closed form
    d/dnu R(-dt nu l(l+1)/2)^N, R the RK4 stability polynomial.
"""

import math
from dataclasses import replace

import numpy as np
import pytest

from oracle import dg, sh
from paper_2501_05110_amd import workloads as W


def _small_shock(nx=6, np_=4, k=1, lmax=1):
    return W.shock_workload("s", nx, np_, k, lmax, steps=0, seed=11)


@pytest.mark.parametrize("k,lmax", [(1, 1), (2, 2)])
def test_rk4_gradient_transpose_identity(k, lmax):
    wl = _small_shock(5, 3, k, lmax)
    S = dg.assemble(wl)
    rng = np.random.default_rng(3)
    N = wl.ndofs
    z0 = rng.standard_normal(N)
    g = rng.standard_normal(N)
    dt, n = 2e-3, 7
    dz0, _ = dg.rk4_gradient(S, z0, dt, n, g)
    d = rng.standard_normal(N)
    dzN = dg.rk4(S, d, dt, n, with_source=False)
    lhs, rhs = float(dz0 @ d), float(g @ dzN)
    assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + np.linalg.norm(g) * np.linalg.norm(dzN))


def test_rk4_gradient_nu_central_differences():
    """dJ/dnu along seeded directions, scaled to nu, against central
    differences (h = 1e-5 relative; the error is O(h^2) ~ 1e-10).  The flux
    splitting does not depend on nu, so no upwind sign can flip between the
    two evaluations."""
    wl = _small_shock(6, 4, 1, 1)
    nu = np.asarray(wl.nu, float)
    rng = np.random.default_rng(5)
    z0 = rng.standard_normal(wl.ndofs)
    g = rng.standard_normal(wl.ndofs)
    dt, n = 5e-3, 12
    S = dg.assemble(wl)
    _, gnu = dg.rk4_gradient(S, z0, dt, n, g, dsys=dg.collision_system(wl))
    h = 1e-5
    for j in range(3):
        d = nu * rng.standard_normal(nu.shape)
        Jp = g @ dg.rk4(dg.assemble(replace(wl, nu=nu + h * d)), z0, dt, n)
        Jm = g @ dg.rk4(dg.assemble(replace(wl, nu=nu - h * d)), z0, dt, n)
        fd = (Jp - Jm) / (2 * h)
        ad = float(gnu @ d)
        assert abs(fd - ad) <= 1e-7 * max(abs(ad), 1e-12), (j, fd, ad)


def test_rk4_gradient_nu_uniform_closed_form():
    """Pure scattering of a uniform state c (every cell, every node): after N
    steps each coefficient is c R(z)^N with z = -dt nu l(l+1)/2, so for
    J = sum g . z_N with g uniform,
        dJ/dnu_c = sum_{b, lms} g c N R(z)^(N-1) R'(z) (-dt l(l+1)/2)
    per cell (the cells decouple)."""
    nu, dt, N = 0.7, 0.04, 25
    wl = W.Workload(name="u", lmax=2, k=1, axes=("x",),
                    nodes=(W.uniform_nodes(-1.0, 1.0, 5),), bc=((W.PERIODIC, W.PERIODIC),),
                    terms=frozenset({W.COLLISION}), p_fixed=math.sqrt(3), flow=W.zero_flow,
                    magnetic=None, nu=nu)
    S = dg.assemble(wl)
    rng = np.random.default_rng(8)
    c = rng.standard_normal(wl.n_lms)
    gl = rng.standard_normal(wl.n_lms)
    z0 = np.tile(c, (wl.ncells, wl.n_basis, 1)).ravel()
    g = np.tile(gl, (wl.ncells, wl.n_basis, 1)).ravel()
    _, gnu = dg.rk4_gradient(S, z0, dt, N, g, dsys=dg.collision_system(wl))
    ll = np.array([l * (l + 1) / 2 for (l, m, s) in sh.lms_list(2)])
    z = -dt * nu * ll
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    dR = 1 + z + z ** 2 / 2 + z ** 3 / 6
    per_cell = wl.n_basis * np.sum(gl * c * N * R ** (N - 1) * dR * (-dt * ll))
    np.testing.assert_allclose(gnu, per_cell, rtol=1e-12)

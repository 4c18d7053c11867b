"""Pins of the oracle's Theta-method step (eq. theta-method,
eq. system-matrix-rhs) against closed forms and limits that do not use its
own formula:

* Theta = 0 is the forward Euler method (the paper's own remark): one step
  equals zeta + dt L(zeta) from the oracle's `apply`;
* pure scattering of a uniform state: each mode is multiplied per step by
  the Theta-method's amplification factor (1 - (1-Theta) z) / (1 + Theta z)
  at z = dt nu l(l+1)/2 (textbook linear-stability result);
* Crank-Nicolson (Theta = 1/2) on a rigid rotation (uniform B along z): the
  Cayley transform of a rotation generator is the rotation by
  2 atan(omega dt / 2) per step, so the l = 1 block turns by exactly that
  angle and keeps its length;
* backward Euler (Theta = 1) with a huge step lands on the steady state
  D zeta = h (sparse LU of D).
"""

import math

import numpy as np
import pytest

from oracle import dg, sh
from paper_2501_05110_amd import workloads as W


def _uniform_wl(axes, lmax, k, n=4, B=None, nu=0.0, p=math.sqrt(3)):
    nodes = tuple(W.uniform_nodes(-1.0, 1.0 + 0.1 * i, n + i) for i in range(len(axes)))
    return W.Workload(name="u", lmax=lmax, k=k, axes=axes, nodes=nodes,
                      bc=((W.PERIODIC, W.PERIODIC),) * len(axes),
                      terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION}),
                      p_fixed=p, flow=W.zero_flow,
                      magnetic=None if B is None else W.uniform_field(B), nu=nu)


def test_theta_zero_is_forward_euler():
    wl = W.shock_workload("t0", 10, 4, 2, 3, seed=3)
    S = dg.assemble(wl)
    z = np.random.default_rng(1).standard_normal(wl.ndofs)
    dt = 2e-3
    got = dg.theta_step(S, z, dt, 0.0)
    want = z + dt * dg.apply(S, z)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.max(np.abs(want)))


@pytest.mark.parametrize("theta", [0.5, 1.0, 0.3])
def test_scattering_amplification_factor(theta):
    nu, dt, N = 0.8, 0.7, 12            # dt far beyond the explicit limit
    wl = _uniform_wl(("x",), 3, 1, nu=nu)
    wl.terms = frozenset({W.COLLISION})
    S = dg.assemble(wl)
    c = np.random.default_rng(4).standard_normal(wl.n_lms)
    z = np.tile(c, (wl.ncells, wl.n_basis, 1))
    out = dg.theta_step(S, z, dt, theta, N).reshape(wl.shape)[2, 1]
    ll = np.array([l * (l + 1) / 2 for (l, m, s) in sh.lms_list(3)])
    zz = dt * nu * ll
    g = (1 - (1 - theta) * zz) / (1 + theta * zz)
    np.testing.assert_allclose(out, c * g ** N, rtol=1e-12, atol=1e-15)


def test_crank_nicolson_rotation_is_cayley():
    B, dt, N = 0.9, 0.4, 25
    wl = _uniform_wl(("x",), 1, 2, B=(0.0, 0.0, B))
    wl.terms = frozenset({W.ROTATION})
    S = dg.assemble(wl)
    c = np.array([0.3, 1.0, -0.5, 0.7])          # f000, f110, f100, f111
    z = np.tile(c, (wl.ncells, wl.n_basis, 1))
    out = dg.theta_step(S, z, dt, 0.5, N).reshape(wl.shape)[1, 2]
    w = B / 2.0                                   # omega = B / gamma, gamma = 2
    ang = N * 2.0 * math.atan(w * dt / 2.0)
    f110 = c[1] * math.cos(ang) + c[2] * math.sin(ang)
    f100 = -c[1] * math.sin(ang) + c[2] * math.cos(ang)
    np.testing.assert_allclose(out, [c[0], f110, f100, c[3]], atol=1e-13)
    assert abs(math.hypot(out[1], out[2]) - math.hypot(c[1], c[2])) < 1e-13


def test_backward_euler_huge_step_is_steady_state():
    wl = W.shock_workload("be", 12, 5, 1, 1, seed=5, lnp=(0.0, 3.0))
    S = dg.assemble(wl)
    zs = dg.steady_state(S)
    z0 = np.random.default_rng(2).standard_normal(wl.ndofs) * 1e-3
    z1 = dg.theta_step(S, z0, 1e9, 1.0)
    assert np.max(np.abs(z1 - zs)) <= 1e-6 * np.max(np.abs(zs))

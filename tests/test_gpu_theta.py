"""Theta-method steps (eq. theta-method / eq. system-matrix-rhs) of the HIP
library against the oracle's sparse-LU solution of the same system.

The library solves the system by restarted GMRES to a relative residual tol
on the M^{-1}-scaled form; with tol = 1e-13 and time steps 10-20 times the
explicit limit, the condition number of I - dt Theta L0 stays below ~1e2, so
after a few steps the states agree to ~1e-11.  The bar written here is
THETA_TOL = 1e-10 (relative, infinity norm).
"""

import numpy as np
import pytest

from oracle import dg
from paper_2501_05110_amd import workloads as W

from gpu_cases import CASES, _say, rel_inf, shock

pytestmark = pytest.mark.gpu
THETA_TOL = 1e-10


def _gpu_theta(op, z, dt, theta, n, **kw):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(z).ravel()).cuda()
    st = op.theta_advance(u, dt, n, theta=theta, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st


@pytest.mark.parametrize("name,theta,cfl_mult", [
    ("shock_k2_l3", 0.5, 10.0), ("shock_k2_l3", 1.0, 20.0), ("shock_k1_l5", 0.5, 10.0),
    ("uniform2d", 1.0, 10.0), ("cube_k1_l3", 0.5, 10.0), ("c1", 0.5, 20.0)])
def test_theta_parity(lib, cuda, name, theta, cfl_mult):
    from paper_2501_05110_amd.vfp import Operator
    wl = CASES[name]()
    op = Operator(wl)
    dt = cfl_mult * op.cfl_dt(0.2)
    z = W.random_state(wl, 31)
    n = 3
    _say(f"[theta] {name}: theta={theta} dt={dt:.4e} ({cfl_mult}x the explicit step) ndofs={wl.ndofs}")
    got, st = _gpu_theta(op, z, dt, theta, n, tol=1e-13, restart=40, max_iters=2000)
    want = dg.theta_step(dg.assemble(wl), z, dt, theta, n)
    err = rel_inf(got, want)
    _say(f"   iterations={st['iterations']} residual={st['residual']:.2e} rel_inf={err:.3e}")
    assert st["converged"] and st["residual"] <= 1e-13
    assert err <= THETA_TOL, (name, theta, err)


def test_theta_zero_is_the_stage_kernel(lib, cuda):
    """Theta = 0 is forward Euler: zeta + dt L(zeta), no Krylov iteration."""
    from paper_2501_05110_amd.vfp import Operator
    wl = shock(14, 5, 2, 3)
    op = Operator(wl)
    dt = op.cfl_dt(0.2)
    z = W.random_state(wl, 5)
    got, st = _gpu_theta(op, z, dt, 0.0, 1)
    S = dg.assemble(wl)
    want = z.ravel() + dt * dg.apply(S, z)
    assert st["iterations"] == 0
    assert rel_inf(got, want) <= 1e-12


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_theta_scattering_closed_form(lib, cuda, theta):
    """Uniform state, scattering only: each mode scales per step by
    (1 - (1-Theta) z)/(1 + Theta z), z = dt nu l(l+1)/2."""
    from oracle import sh
    from paper_2501_05110_amd.vfp import Operator
    wl = W.Workload(name="scat", lmax=3, k=1, axes=("x",), nodes=(W.uniform_nodes(-1.0, 1.0, 6),),
                    bc=((W.PERIODIC, W.PERIODIC),), terms=frozenset({W.COLLISION}), p_fixed=3 ** 0.5,
                    flow=W.zero_flow, magnetic=None, nu=0.8)
    op = Operator(wl)
    c = np.random.default_rng(4).standard_normal(wl.n_lms)
    z = np.tile(c, (wl.ncells, wl.n_basis, 1))
    dt, N = 0.7, 12
    got, st = _gpu_theta(op, z, dt, theta, N, tol=1e-14)
    ll = np.array([l * (l + 1) / 2 for (l, m, s) in sh.lms_list(3)])
    g = (1 - (1 - theta) * dt * 0.8 * ll) / (1 + theta * dt * 0.8 * ll)
    want = np.broadcast_to(c * g ** N, wl.shape)
    np.testing.assert_allclose(got.reshape(wl.shape), want, rtol=1e-12, atol=1e-14)
    assert st["converged"]


def test_theta_rejects_bad_arguments(lib, cuda):
    import torch
    from paper_2501_05110_amd.vfp import Operator, VFPError
    op = Operator(shock(4, 3, 1, 1))
    u = torch.zeros(op.ndofs, dtype=torch.float64, device="cuda")
    for kw in ({"theta": 1.5}, {"theta": -0.1}, {"tol": 0.0}, {"restart": 0}, {"restart": 65},
               {"max_iters": 0}, {"precond": 7}):
        with pytest.raises(VFPError):
            op.theta_advance(u, 0.1, 1, **kw)
    small = torch.empty(8, dtype=torch.float64, device="cuda")
    with pytest.raises(VFPError):
        op.theta_advance(u, 0.1, 1, work=small)


def test_theta_collision_preconditioner(lib, cuda):
    """Strong scattering (nu0 = 200): the collision-diagonal right
    preconditioner gives the same step (oracle's sparse LU) in fewer Krylov
    iterations; on scattering alone it is the exact inverse (one iteration
    per step)."""
    from paper_2501_05110_amd.vfp import Operator
    wl = shock(16, 6, 2, 3, nu0=200.0)
    op = Operator(wl)
    dt = 10.0 * op.cfl_dt(0.2)
    z = W.random_state(wl, 37)
    want = dg.theta_step(dg.assemble(wl), z, dt, 1.0, 2)
    its = {}
    for pc in (None, "collision"):
        got, st = _gpu_theta(op, z, dt, 1.0, 2, tol=1e-13, restart=40, max_iters=3000, precond=pc)
        err = rel_inf(got, want)
        its[pc] = st["iterations"]
        _say(f"[theta-pc] precond={pc} iterations={st['iterations']} residual={st['residual']:.2e} rel_inf={err:.3e}")
        assert st["converged"] and err <= THETA_TOL
    assert its["collision"] < its[None]
    scat = W.Workload(name="scat", lmax=3, k=1, axes=("x",), nodes=(W.uniform_nodes(-1.0, 1.0, 6),),
                      bc=((W.PERIODIC, W.PERIODIC),), terms=frozenset({W.COLLISION}), p_fixed=3 ** 0.5,
                      flow=W.zero_flow, magnetic=None, nu=0.8)
    ops = Operator(scat)
    c = np.random.default_rng(4).standard_normal(scat.n_lms)
    zs = np.tile(c, (scat.ncells, scat.n_basis, 1))
    _, st = _gpu_theta(ops, zs, 0.7, 0.5, 3, tol=1e-13, precond="collision")
    _say(f"   scattering only: iterations={st['iterations']} for 3 steps")
    assert st["converged"] and st["iterations"] <= 3


def test_theta_short_restarts_and_iteration_cap(lib, cuda):
    """Restarts every 4 Krylov vectors (so the next iteration is often queued
    across a restart boundary) still give the oracle's step, and an
    iteration cap stops the solve after exactly that many iterations with a
    finite state (a queued iteration that is not used is not counted)."""
    from paper_2501_05110_amd.vfp import Operator
    wl = shock(16, 6, 2, 3)
    op = Operator(wl)
    dt = 10.0 * op.cfl_dt(0.2)
    z = W.random_state(wl, 53)
    want = dg.theta_step(dg.assemble(wl), z, dt, 0.5, 2)
    got, st = _gpu_theta(op, z, dt, 0.5, 2, tol=1e-12, restart=4, max_iters=5000)
    err = rel_inf(got, want)
    _say(f"[theta restarts] restart=4: iterations={st['iterations']} residual={st['residual']:.2e} rel_inf={err:.3e}")
    assert st["converged"] and err <= THETA_TOL
    capped, st2 = _gpu_theta(op, z, dt, 0.5, 1, tol=1e-14, restart=4, max_iters=7)
    _say(f"   capped: iterations={st2['iterations']} converged={st2['converged']} residual={st2['residual']:.2e}")
    assert st2["iterations"] == 7 and not st2["converged"]
    assert np.isfinite(capped).all()


def _x_transport(nx=40, k=2, lmax=3, U=(0.3, 0.0, 0.0)):
    """Advection along one axis only (fixed p, uniform flow, zero inflow /
    continuous ends): the system is block-tridiagonal along x."""
    return W.Workload(name="xtransport", lmax=lmax, k=k, axes=("x",), nodes=(W.uniform_nodes(-2.0, 2.0, nx),),
                      bc=((W.ZERO_INFLOW, W.CONTINUOUS),), terms=frozenset({W.ADVECTION}), p_fixed=0.5,
                      flow=W.uniform_flow(U), magnetic=None, nu=0.0)


def test_xline_preconditioner_exact_along_x(lib, cuda):
    """VFP_PRECOND_XLINE inverts the block-tridiagonal part along axis 0
    exactly: on transport along x alone that is the whole system, so each
    Crank-Nicolson step converges in one Krylov iteration, at a Courant
    number of 50, and matches the oracle's sparse-LU step."""
    from paper_2501_05110_amd.vfp import Operator
    wl = _x_transport()
    op = Operator(wl)
    dt = 50.0 * op.cfl_dt(1.0)
    z = W.random_state(wl, 41)
    want = dg.theta_step(dg.assemble(wl), z, dt, 0.5, 3)
    got, st = _gpu_theta(op, z, dt, 0.5, 3, tol=1e-13, restart=30, max_iters=500, precond="xline")
    err = rel_inf(got, want)
    _say(f"[xline exact] iterations={st['iterations']} residual={st['residual']:.2e} rel_inf={err:.3e}")
    assert st["converged"] and st["iterations"] <= 3
    assert err <= THETA_TOL


def test_xline_preconditioner_dsa_paper_setup(lib, cuda):
    """The paper's DSA setup (Table sapphire-simulation-parameters: l_max =
    1, Crank-Nicolson with dt = 1, the stretched x grid of Fig. shock-grid),
    coarsened to 16 cells in ln p and a coarser shock spacing: two steps with
    the x-line preconditioner against the oracle's sparse-LU steps.  At
    dt = 1 the x Courant number reaches ~25 in the shock cells; the
    unpreconditioned GMRES needs an order of magnitude more iterations."""
    from paper_2501_05110_amd.vfp import Operator
    wl = W.paper_dsa_workload(np_=16, dx_shock=0.04, grow=0.04)
    op = Operator(wl)
    z = W.random_state(wl, 43, 1e-2)
    dt, nst = 1.0, 2
    want = dg.theta_step(dg.assemble(wl), z, dt, 0.5, nst)
    got, st = _gpu_theta(op, z, dt, 0.5, nst, tol=1e-13, restart=40, max_iters=2000, precond="xline")
    err = rel_inf(got, want)
    _say(f"[xline dsa] {wl.name} ndofs={wl.ndofs}: iterations={st['iterations']} residual={st['residual']:.2e} "
         f"rel_inf={err:.3e}")
    assert st["converged"] and err <= 1e-9
    _, st0 = _gpu_theta(op, z, dt, 0.5, nst, tol=1e-13, restart=40, max_iters=2000)
    _say(f"   without a preconditioner: iterations={st0['iterations']} converged={st0['converged']}")
    assert st["iterations"] * 5 <= st0["iterations"]


@pytest.mark.parametrize("nx,k,lmax", [(37, 1, 1), (5, 3, 1), (23, 2, 1)])
def test_xline_quad_lanes_match_rowwise(lib, cuda, monkeypatch, nx, k, lmax):
    """Blocks of at most 16 unknowns are solved with four lanes per row and
    a ring of prefetched cells; that solve rounds exactly as the one lane
    per row solve (VFP_XLINE_ROWS=1), so the Theta steps agree bit for bit
    (b = 8, 16 and 12; a line shorter than the ring; lengths that are not a
    multiple of it), and both match the oracle's sparse-LU step."""
    from paper_2501_05110_amd.vfp import Operator
    wl = _x_transport(nx=nx, k=k, lmax=lmax)
    op = Operator(wl)
    dt = 30.0 * op.cfl_dt(1.0)
    z = W.random_state(wl, 47)
    want = dg.theta_step(dg.assemble(wl), z, dt, 0.5, 2)
    out = {}
    for rows in ("0", "1"):
        monkeypatch.setenv("VFP_XLINE_ROWS", rows)
        out[rows] = _gpu_theta(op, z, dt, 0.5, 2, tol=1e-13, restart=30, max_iters=500, precond="xline")
    (g0, s0), (g1, s1) = out["0"], out["1"]
    b = (k + 1) * (lmax + 1) ** 2
    _say(f"[xline lanes] nx={nx} b={b}: iterations {s0['iterations']} / {s1['iterations']}, "
         f"rel_inf={rel_inf(g0, want):.3e}")
    assert np.array_equal(g0, g1) and s0["iterations"] == s1["iterations"]
    assert s0["converged"] and rel_inf(g0, want) <= THETA_TOL


def test_xline_preconditioner_periodic_and_rejected(lib, cuda):
    """A periodic axis 0 whose length is not a multiple of 3 (the wrap left
    out of the preconditioner, the last cell probed with a colour of its
    own): still the oracle's step; and blocks above 48 unknowns per cell are
    refused."""
    from paper_2501_05110_amd.vfp import Operator, VFPError
    wl = W.Workload(name="xper", lmax=3, k=2, axes=("x",), nodes=(W.uniform_nodes(-2.0, 2.0, 10),),
                    bc=((W.PERIODIC, W.PERIODIC),), terms=frozenset({W.ADVECTION, W.COLLISION}), p_fixed=0.5,
                    flow=W.uniform_flow((0.3, 0.0, 0.0)), magnetic=None, nu=0.5)
    op = Operator(wl)
    dt = 20.0 * op.cfl_dt(0.2)
    z = W.random_state(wl, 47)
    want = dg.theta_step(dg.assemble(wl), z, dt, 0.5, 2)
    got, st = _gpu_theta(op, z, dt, 0.5, 2, tol=1e-13, restart=40, max_iters=1000, precond="xline")
    err = rel_inf(got, want)
    _say(f"[xline periodic] iterations={st['iterations']} rel_inf={err:.3e}")
    assert st["converged"] and err <= THETA_TOL
    big = Operator(shock(6, 3, 2, 3))          # 9 x 16 = 144 unknowns per cell
    with pytest.raises(VFPError):
        big.theta_precond_size("xline")

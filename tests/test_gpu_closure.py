"""The closure example of Sec. 4.3 on the library: free streaming of an
isotropic Gaussian (gamma = 2, nu = 0) along x, advanced to t = 12/sqrt(3)
and reconstructed at x = 6 sigma over the sphere (vfp_reconstruct), against
the characteristic solution f = exp(-(x - V cos(theta) t)^2 / 2) / sqrt(2 pi).
Truncating the expansion closes the system; the error over the sphere falls
as l_max grows up to the paper's l_max = 11, which reproduces the beam, and
the GPU state matches the oracle's (l_max = 3 here; l_max 9 and 11 on a
smaller grid below)."""

import math

import numpy as np
import pytest

from oracle import dg, sh
from paper_2501_05110_amd import workloads as W

from gpu_cases import _say, rel_inf

pytestmark = pytest.mark.gpu

P = math.sqrt(3.0)             # gamma = 2
V = P / 2.0
T_F = 12.0 / math.sqrt(3.0)
DT = 1.0 / (100.0 * math.sqrt(3.0))
X0 = 6.0                       # 6 sigma


def _workload(lmax):
    return W.Workload(name=f"closure_l{lmax}", lmax=lmax, k=2, axes=("x",),
                      nodes=(W.uniform_nodes(-15.0, 15.0, 256),), bc=((W.ZERO_INFLOW, W.ZERO_INFLOW),),
                      terms=frozenset({W.ADVECTION, W.COLLISION}), p_fixed=P, flow=W.zero_flow,
                      magnetic=None, nu=0.0)


def _initial(wl):
    n = wl.n_lms

    def f0(X, p):
        out = np.zeros((n, X.shape[1]))
        out[0] = math.sqrt(4 * math.pi) * np.exp(-X[0] ** 2 / 2) / math.sqrt(2 * math.pi)
        return out
    return dg.project(wl, f0)


def test_closure_example(lib, cuda):
    import torch
    from paper_2501_05110_amd import vfp
    pts, wts = sh.sphere_quadrature(40)
    theta = np.arccos(np.clip(pts[0], -1, 1))
    phi = np.arctan2(pts[2], pts[1])
    exact = np.exp(-(X0 - V * np.cos(theta) * T_F) ** 2 / 2) / math.sqrt(2 * math.pi)
    h = 30.0 / 256
    cell = int((X0 + 15.0) // h)
    eta = 2 * ((X0 + 15.0) / h - cell) - 1
    Lx, _ = dg.lagrange(dg.lobatto_nodes(2), np.array([eta]))
    nsteps = int(round(T_F / DT))
    errs = []
    for lmax in (1, 3, 5, 7, 9, 11):
        wl = _workload(lmax)
        op = vfp.Operator(wl)
        z0 = _initial(wl)
        u = torch.from_numpy(z0.ravel().copy()).cuda()
        work = torch.empty(2 * wl.ndofs, dtype=torch.float64, device="cuda")
        op.advance(u, T_F / nsteps, nsteps, work)
        Y = torch.from_numpy(vfp.sh_eval(lmax, theta, phi)).cuda()
        rows = wl.ndofs // wl.n_lms
        f = torch.empty(rows * theta.size, dtype=torch.float64, device="cuda")
        op.reconstruct(u, Y, f)
        torch.cuda.synchronize()
        fr = f.cpu().numpy().reshape(wl.ncells, wl.n_basis, theta.size)[cell]   # (nodes, directions)
        fnum = Lx[0] @ fr
        err = math.sqrt(np.sum(wts * (fnum - exact) ** 2) / np.sum(wts * exact ** 2))
        errs.append(err)
        _say(f"[closure] l_max={lmax} steps={nsteps} relative L2 error over the sphere at x=6: {err:.4f}")
        if lmax == 3:
            want = dg.rk4(dg.assemble(wl), z0.ravel(), T_F / nsteps, nsteps)
            perr = rel_inf(u.cpu().numpy(), want)
            _say(f"   state vs oracle rel_inf={perr:.2e}")
            assert perr <= 1e-10
        op.close()
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[0] > 0.5 and errs[-1] < 0.05, errs


@pytest.mark.parametrize("lmax,k", [(9, 2), (11, 2), (11, 1)])
def test_high_lmax_parity(lib, cuda, lmax, k):
    """l_max 9 and 11 on a line along x with B along x, scattering, a flow
    and a source: apply and 100 steps against the oracle."""
    import torch
    from paper_2501_05110_amd import vfp
    from gpu_cases import APPLY_TOL, STEPS_TOL, gpu_apply
    wl = W.Workload(name=f"line_l{lmax}", lmax=lmax, k=k, axes=("x",),
                    nodes=(np.linspace(-2.0, 3.0, 24) ** 1.0,), bc=((W.ZERO_INFLOW, W.CONTINUOUS),),
                    terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION, W.SOURCE}), p_fixed=P,
                    flow=W.uniform_flow([0.1, 0.0, 0.0]), magnetic=W.uniform_field((0.7, 0.0, 0.0)), nu=0.05,
                    source=lambda X, p: np.exp(-X[0] ** 2))
    op = vfp.Operator(wl)
    S = dg.assemble(wl)
    z = W.random_state(wl, 61)
    for ws in (True, False):
        err = rel_inf(gpu_apply(op, z, ws), dg.apply(S, z, ws))
        _say(f"[l_max {lmax}, k {k}] apply with_source={ws} rel_inf={err:.3e}")
        assert err <= APPLY_TOL
    dt = op.cfl_dt(0.2)
    u = torch.from_numpy(z.ravel().copy()).cuda()
    work = torch.empty(2 * wl.ndofs, dtype=torch.float64, device="cuda")
    op.advance(u, dt, 100, work)
    torch.cuda.synchronize()
    err = rel_inf(u.cpu().numpy(), dg.rk4(S, z, dt, 100))
    _say(f"   100 steps rel_inf={err:.3e}")
    assert err <= STEPS_TOL
    op.close()

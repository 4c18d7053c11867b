"""Diffusive shock acceleration (Sec. 4.4) reached by time stepping on the
library: a parallel shock of compression r = 4 with continuous injection,
advanced from f = 0 until the spectrum behind the shock is steady for ln p up
to 4; its slope is -3r/(r-1) = -4 (eq. particle-spectrum-shock-rest-frame)
within 2 %.  Scattering nu = 10 shortens the acceleration time (kappa =
V^2/(3 nu)) while keeping the shock width w far below kappa/U."""

import math

import numpy as np
import pytest

from paper_2501_05110_amd import workloads as W

from gpu_cases import _say

pytestmark = pytest.mark.gpu


def _dsa_grid(L=40.0, h0=0.01, grow=1.08, n_fine=6):
    pos = [0.0]
    h = h0
    while pos[-1] < L:
        pos.append(pos[-1] + h)
        if len(pos) > n_fine:
            h *= grow
    pos = np.array(pos)
    pos[-1] = L
    return np.concatenate([-pos[::-1], pos[1:]])


def _slope(z, wl, xn, pn, lo, hi):
    nx, npc = len(xn) - 1, len(pn) - 1
    f = z.reshape(wl.shape)[:, :, 0].reshape(npc, nx, 2, 2)     # [ip][ix][jp][jx]
    xc = 0.5 * (xn[:-1] + xn[1:])
    sel = np.where((xc > 0.5) & (xc < 3))[0]
    fp = f[:, sel].mean(axis=(1, 3)).ravel()
    lnp = np.stack([pn[:-1], pn[1:]], 1).ravel()
    m = (lnp > lo) & (lnp < hi)
    return np.polyfit(lnp[m], np.log(fp[m]), 1)[0]


def test_dsa_slope_by_time_stepping(lib, cuda):
    import torch
    from paper_2501_05110_amd import vfp
    r, U1, w, nu = 4.0, 0.05, 0.02, 10.0
    xn = _dsa_grid()
    pn = np.linspace(0.0, 5.0, 41)
    wl = W.Workload(name="dsa", lmax=1, k=1, axes=("x", "lnp"), nodes=(xn, pn),
                    bc=((W.ZERO_INFLOW, W.CONTINUOUS), (W.ZERO_INFLOW, W.ZERO_INFLOW)),
                    terms=frozenset({W.ADVECTION, W.MOMENTUM, W.ROTATION, W.COLLISION, W.SOURCE}),
                    flow=W.shock_flow(U1 / r, r, w), magnetic=W.uniform_field((1.0, 0, 0)),
                    nu=nu, source=W.gaussian_source(0.1, 0.0, 0.5, 0.05, 1 / 8))
    op = vfp.Operator(wl)
    dt = op.cfl_dt(0.2)
    u = torch.zeros(wl.ndofs, dtype=torch.float64, device="cuda")
    work = torch.empty(2 * wl.ndofs, dtype=torch.float64, device="cuda")
    want = -3 * r / (r - 1)
    t = 0.0
    for T in (1000.0, 2500.0):
        n = int(round((T - t) / dt))
        op.advance(u, dt, n, work)
        torch.cuda.synchronize()
        t += n * dt
        z = u.cpu().numpy()
        s1, s2 = _slope(z, wl, xn, pn, 1.0, 2.5), _slope(z, wl, xn, pn, 1.5, 4.0)
        _say(f"[dsa] t={t:.0f} ({n} steps) slope ln p in [1, 2.5]: {s1:.4f}, in [1.5, 4]: {s2:.4f} (theory {want})")
    assert np.all(np.isfinite(z))
    assert abs(s1 - want) < 0.02 * abs(want) and abs(s2 - want) < 0.02 * abs(want), (s1, s2)

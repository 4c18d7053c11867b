"""Gradients with respect to the planar flow and the shock-profile parameters.

* Flow sensitivities dJ/dU, dJ/dU', dJ/d(dU/dt) at sampled x Gauss points and
  dJ/dU at sampled x faces, from the library's reverse sweep, against
  central differences of the oracle's forward run with that one flow value
  perturbed (the oracle samples the flow callable at the same points).
* dJ/d(r, w) (and dJ/dnu per cell) through advance_with_grad and
  planar_shock_fields, against central differences of the oracle in 16 seeded
  directions of (nu, r, w) -- 1e-6 relative -- with nu perturbed in log space
  and no upwind decision reversed between the two sides of a difference.
The sampled points include ones inside the shock, where the ln p face
matrix is indefinite (the spectral-derivative branch).
"""

from dataclasses import replace

import numpy as np
import pytest

from oracle import dg
from paper_2501_05110_amd import workloads as W

from gpu_cases import _say, shock

pytestmark = pytest.mark.gpu
FD_TOL = 1e-6


def _perturbed(base, which, x0, h):
    def flow(X):
        U, dU, a = base(X)
        hit = np.abs(X[0] - x0) < 1e-12
        if which == "u" or which == "uf":
            U[0][hit] += h
        elif which == "du":
            dU[0, 0][hit] += h
        else:
            a[0][hit] += h
        return U, dU, a
    flow.kind = base.kind
    return flow


def _upwind_signs(wl):
    """Signs of the eigenvalues of n.beta at every face point of every cell
    (0 where an eigenvalue vanishes to rounding): the upwind decisions."""
    g = dg.Grid(wl)
    out = []
    for c in range(g.ncells):
        idx = g.cell_multi(c)
        for a in range(g.d):
            for side in (0, 1):
                _, _, eta, _ = g.face_tables(a, side)
                XF, pF = g.points(idx, eta)
                beta, _ = g.coefficients(c, XF, pF)
                lam = np.linalg.eigvalsh(beta[a])            # [point, n]
                tol = 1e-12 * max(1.0, float(np.abs(lam).max()))
                out.append(np.where(np.abs(lam) <= tol, 0.0, np.sign(lam)).ravel())
    return np.concatenate(out)


def _oracle_J(wl, z0, dt, n, g):
    return float(g @ dg.rk4(dg.assemble(wl), z0, dt, n))


def test_flow_sensitivities_vs_oracle(lib, cuda):
    import torch
    from paper_2501_05110_amd.vfp import Operator
    # a wider shock (w = L/20) so that several Gauss points see a gradient
    wl = W.shock_workload("fg", 12, 5, 2, 3, w_frac=0.05, seed=6)
    op = Operator(wl)
    dt = op.cfl_dt(0.2)
    n = 6
    rng = np.random.default_rng(21)
    z0 = rng.standard_normal(wl.ndofs)
    g = rng.standard_normal(wl.ndofs)
    N = op.ndofs
    tz0 = torch.from_numpy(z0).cuda()
    tape = torch.empty(4 * n * N, dtype=torch.float64, device="cuda")
    op.advance_tape(tz0, dt, n, tape)
    mu = torch.from_numpy(g.copy()).cuda()
    op.mass(mu, mu, inverse=True)
    work = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    slots = torch.zeros(op.field_grad_size(), dtype=torch.float64, device="cuda")
    op.adjoint_steps(tz0, tape, dt, n, mu, None, work, field_slots=slots)
    nx = wl.ncells_axis[0]
    nq = nx * (wl.k + 1)
    gu, gd, ga = (torch.empty(nq, dtype=torch.float64, device="cuda") for _ in range(3))
    gf = torch.empty(nx + 1, dtype=torch.float64, device="cuda")
    op.field_grad_reduce(slots, gu, gd, ga, gf)
    torch.cuda.synchronize()
    got = {"u": gu.cpu().numpy(), "du": gd.cpu().numpy(), "a": ga.cpu().numpy(), "uf": gf.cpu().numpy()}
    xv = op.points(0, 0)
    xf = op.points(1, 0)
    # U at Gauss points near and far from the shock; U' and dU/dt only where
    # |U'| is far above the perturbation (where U' = 0 the ln p face matrix
    # vanishes and the flux has a kink, which a central difference straddles)
    _, dUv, _ = W.shock_profile(xv, wl.meta["U0"], wl.meta["r"], wl.meta["w"])
    iq = [int(np.argmin(np.abs(xv - x))) for x in (-0.5, 0.2, 0.9, -6.0)]
    ig = [i for i in np.argsort(-np.abs(dUv))[:6] if abs(dUv[i]) > 1e-3]
    assert len(ig) >= 4
    jf = [int(np.argmin(np.abs(xf - x))) for x in (0.0, -1.6, 5.0)] + [0, nx]
    h = 1e-6
    worst = 0.0
    for which, idxs, xs in (("u", iq, xv), ("du", ig, xv), ("a", ig, xv), ("uf", jf, xf)):
        for i in idxs:
            Jp = _oracle_J(replace(wl, flow=_perturbed(wl.flow, which, xs[i], h)), z0, dt, n, g)
            Jm = _oracle_J(replace(wl, flow=_perturbed(wl.flow, which, xs[i], -h)), z0, dt, n, g)
            fd = (Jp - Jm) / (2 * h)
            gv = got[which][i]
            scale = max(abs(fd), 1e-3 * max(np.max(np.abs(got[which])), 1e-30))
            err = abs(gv - fd) / scale
            worst = max(worst, err)
            _say(f"[field] {which}[{i}] x={xs[i]:+.4f}: gpu={gv:+.8e} fd={fd:+.8e} rel={err:.2e}")
            assert err <= FD_TOL, (which, i, gv, fd)
    _say(f"   worst {worst:.2e}")


def test_profile_and_nu_gradient_directions(lib, cuda):
    """J = 0.5 |f_000 at the trace x = +L/2 - target|^2 after n steps; the
    gradient in (nu per cell, r, w) along seeded directions against central
    differences of the oracle (parameters perturbed by 1e-5 relative).  (r, w)
    are the flow profile's; the source is held fixed."""
    import torch
    from paper_2501_05110_amd import vfp
    wl = shock(16, 6, 2, 3, seed=8)
    U0, r0, w0 = wl.meta["U0"], wl.meta["r"], wl.meta["w"]
    op = vfp.Operator(wl)
    dt = op.cfl_dt(0.2)
    n = 20
    z0 = W.random_state(wl, 8, 1e-2).ravel()
    nu0 = np.asarray(wl.nu, float)
    nx, npc = wl.ncells_axis
    ix = nx * 3 // 4
    K1 = wl.k + 1
    sel = np.zeros(wl.shape, bool)
    for jp in range(npc):
        for bq in range(K1):
            sel[jp * nx + ix, bq * K1, 0] = True
    target = np.random.default_rng(9).standard_normal(int(sel.sum())) * 1e-2
    tsel = torch.from_numpy(sel.ravel()).cuda()
    ttarget = torch.from_numpy(target).cuda()

    tU0 = torch.tensor(U0, dtype=torch.float64, device="cuda")
    tr = torch.tensor(r0, dtype=torch.float64, device="cuda", requires_grad=True)
    tw = torch.tensor(w0, dtype=torch.float64, device="cuda", requires_grad=True)
    tnu = torch.from_numpy(nu0.copy()).cuda().requires_grad_(True)
    u0 = torch.from_numpy(z0).cuda()
    flow = vfp.planar_shock_fields(op, tU0, tr, tw)
    uN = vfp.advance_with_grad(op, u0, tnu, dt, n, seg=6, flow=flow)
    loss = 0.5 * ((uN[tsel] - ttarget) ** 2).sum()
    loss.backward()
    g_nu, g_r, g_w = tnu.grad.cpu().numpy(), float(tr.grad), float(tw.grad)
    _say(f"[profile] J={float(loss.detach()):.6e} dJ/dr={g_r:+.6e} dJ/dw={g_w:+.6e} |dJ/dnu|={np.abs(g_nu).max():.3e}")

    def J(nu, r, w):
        # the profile (r, w) changes; the injection keeps its width (the
        # source is an input of its own, not a function of the profile)
        wl2 = replace(wl, flow=W.shock_flow(U0, r, w), nu=nu)
        zN = dg.rk4(dg.assemble(wl2), z0, dt, n).reshape(wl.shape)
        return 0.5 * float(np.sum((zN[sel] - target) ** 2))

    # 16 directions; every fourth leaves out nu, r or w in turn.  nu moves in
    # log space (nu exp(+-h d) = nu (1 +- h d) to first order, d scaled per
    # cell), so the directional derivative is g_nu . (nu d).
    rng = np.random.default_rng(33)
    h = 1e-5
    for d in range(16):
        dl = rng.standard_normal(nu0.shape) * (d % 4 != 0)
        dr = r0 * rng.standard_normal() * (d % 4 != 1)
        dw = w0 * rng.standard_normal() * (d % 4 != 2)
        nup, num = nu0 * np.exp(h * dl), nu0 * np.exp(-h * dl)
        pp, pm = (r0 + h * dr, w0 + h * dw), (r0 - h * dr, w0 - h * dw)
        # the two sides of the difference take the same upwind decisions: no
        # eigenvalue of n.beta changes sign (one that reaches 0 exactly, where
        # the tanh tail rounds to 0, multiplies a zero matrix and does not count)
        sp_ = _upwind_signs(replace(wl, flow=W.shock_flow(U0, *pp)))
        sm_ = _upwind_signs(replace(wl, flow=W.shock_flow(U0, *pm)))
        assert not np.any(sp_ * sm_ < 0), f"direction {d}: an upwind decision flips"
        fd = (J(nup, *pp) - J(num, *pm)) / (2 * h)
        ad = float(g_nu @ (nu0 * dl)) + g_r * dr + g_w * dw
        err = abs(fd - ad) / max(abs(fd), 1e-30)
        _say(f"   direction {d}: adjoint={ad:+.10e} fd={fd:+.10e} rel={err:.2e}")
        assert err <= FD_TOL, (d, ad, fd)


def _flip_signs(wl, U0, r, w, xv, xf, pv_face, V_face_x):
    """Signs (0 within rounding of zero) of every upwind speed of the planar
    (x, ln p) shock: the x-face speeds U(x_F) + lambda V(p) at every x face
    and p Gauss point, and the eigenvalues of beta^{ln p} = -(gamma m/p)
    dU/dt A^x - U' (A^x A^x)_t at every p face and x Gauss point."""
    from oracle import sh
    S = sh.system_matrices(wl.lmax)
    lam = np.linalg.eigvalsh(S["A"][0])
    Uf, _, _ = W.shock_profile(xf, U0, r, w)
    sx = Uf[:, None, None] + lam[None, :, None] * V_face_x[None, None, :]
    Uv, dU, a = W.shock_profile(xv, U0, r, w)
    p = pv_face
    gam = np.sqrt(1 + p * p)
    B = (-(gam / p)[None, :, None, None] * a[:, None, None, None] * S["A"][0][None, None]
         - dU[:, None, None, None] * S["AA"][0, 0][None, None])
    lp = np.linalg.eigvalsh(B.reshape(-1, *B.shape[2:]))
    out = []
    for v in (sx.ravel(), lp.ravel()):
        tol = 1e-12 * max(1.0, float(np.abs(v).max()))
        out.append(np.where(np.abs(v) <= tol, 0.0, np.sign(v)))
    return np.concatenate(out)


@pytest.mark.timeout(600)
def test_c5_gradient_directions_full_size(lib, cuda):
    """The adjoint configuration at its own size: the 512 x 64 shock (k = 2,
    l_max = 3; 4,718,592 DoF), 1000 steps, sqrt(N) = 32-step checkpoints.
    J = 0.5 |f_000 on the trace x = +L/2 (the downstream cell's lower face
    nodes) - target|^2.  The gradient in (nu per cell, r, w) along 16 seeded
    directions against central differences of the library's own forward run
    (pinned to the oracle at 1e-10 after 1000 steps), nu perturbed in log
    space, with no upwind speed changing sign between the two sides of any
    difference.  The U' and dU/dt sensitivities are formed on the shock's
    support only (vfp_field_grad_support), as the benchmark times them."""
    import torch
    from paper_2501_05110_amd import vfp
    wl = W.config5()
    U0, r0, w0 = wl.meta["U0"], wl.meta["r"], wl.meta["w"]
    op = vfp.Operator(wl)
    dt = op.cfl_dt(0.2)
    n = 1000
    seg = vfp.checkpoint_segment(n)
    assert seg == 32
    N = op.ndofs
    z0 = torch.from_numpy(np.ascontiguousarray(wl.meta["init"]).ravel()).cuda()
    nu0 = np.asarray(wl.nu, float)
    nx, npc = wl.ncells_axis
    K1 = wl.k + 1
    ix = nx * 3 // 4                       # cells right of x = +L/2
    sel = np.zeros(wl.shape, bool)
    for jp in range(npc):
        for bq in range(K1):
            sel[jp * nx + ix, bq * K1, 0] = True
    tsel = torch.from_numpy(sel.ravel()).cuda()
    target = torch.from_numpy(np.random.default_rng(55).standard_normal(int(sel.sum())) * 1e-3).cuda()
    _say(f"[c5] ndofs={N} steps={n} seg={seg} dt={dt:.4e}")

    tU0 = torch.tensor(U0, dtype=torch.float64, device="cuda")
    tr = torch.tensor(r0, dtype=torch.float64, device="cuda", requires_grad=True)
    tw = torch.tensor(w0, dtype=torch.float64, device="cuda", requires_grad=True)
    tnu = torch.from_numpy(nu0.copy()).cuda().requires_grad_(True)
    support = vfp.planar_shock_support(op, w0)
    _say(f"   U' support: {int(support.sum())} of {support.size} x cells")
    uN = vfp.advance_with_grad(op, z0, tnu, dt, n, seg=seg, flow=vfp.planar_shock_fields(op, tU0, tr, tw),
                               flow_support=support)
    loss = 0.5 * ((uN[tsel] - target) ** 2).sum()
    loss.backward()
    g_nu, g_r, g_w = tnu.grad.cpu().numpy(), float(tr.grad), float(tw.grad)
    _say(f"   J={float(loss.detach()):.6e} dJ/dr={g_r:+.6e} dJ/dw={g_w:+.6e} |dJ/dnu|={np.abs(g_nu).max():.3e}")

    work = torch.empty(2 * N, dtype=torch.float64, device="cuda")

    def J(nu, r, w):
        fl = vfp.planar_shock_fields(op, tU0, torch.tensor(r, dtype=torch.float64, device="cuda"),
                                     torch.tensor(w, dtype=torch.float64, device="cuda"))
        op.set_flow_planar(*(t.cpu().numpy() for t in fl))
        op.set_scattering(nu)
        u = z0.clone()
        op.advance(u, dt, n, work)
        return 0.5 * float(((u[tsel] - target) ** 2).sum())

    xv = op.points(0, 0)
    xf = op.points(1, 0)
    pq = np.exp(op.points(0, 1))                  # p at the ln p Gauss points (x faces)
    pf = np.exp(op.points(1, 1))                  # p at the ln p faces
    Vq = pq / np.sqrt(1 + pq * pq)
    rng = np.random.default_rng(34)
    h = 1e-5
    worst = 0.0
    for d in range(16):
        dl = rng.standard_normal(nu0.shape) * (d % 4 != 0)
        dr = r0 * rng.standard_normal() * (d % 4 != 1)
        dw = w0 * rng.standard_normal() * (d % 4 != 2)
        pp, pm = (r0 + h * dr, w0 + h * dw), (r0 - h * dr, w0 - h * dw)
        sp_ = _flip_signs(wl, U0, *pp, xv, xf, pf, Vq)
        sm_ = _flip_signs(wl, U0, *pm, xv, xf, pf, Vq)
        assert not np.any(sp_ * sm_ < 0), f"direction {d}: an upwind decision flips"
        fd = (J(nu0 * np.exp(h * dl), *pp) - J(nu0 * np.exp(-h * dl), *pm)) / (2 * h)
        ad = float(g_nu @ (nu0 * dl)) + g_r * dr + g_w * dw
        err = abs(fd - ad) / max(abs(fd), 1e-30)
        worst = max(worst, err)
        _say(f"   direction {d}: adjoint={ad:+.10e} fd={fd:+.10e} rel={err:.2e}")
        assert err <= FD_TOL, (d, ad, fd)
    _say(f"   worst {worst:.2e}")
    op.close()


def test_support_keeps_profile_gradient(lib, cuda):
    """Forming the U' and dU/dt sensitivities on the shock's support only
    leaves dJ/d(nu, r, w) unchanged: outside it those sensitivities meet
    parameter derivatives that are exactly zero."""
    import torch
    from paper_2501_05110_amd import vfp
    wl = W.shock_workload("sup", 40, 6, 2, 3, w_frac=0.01, seed=8)
    U0, r0, w0 = wl.meta["U0"], wl.meta["r"], wl.meta["w"]
    op = vfp.Operator(wl)
    dt = op.cfl_dt(0.2)
    z0 = torch.from_numpy(W.random_state(wl, 8, 1e-2).ravel()).cuda()
    g = torch.from_numpy(np.random.default_rng(4).standard_normal(wl.ndofs)).cuda()
    support = vfp.planar_shock_support(op, w0)
    assert 0 < support.sum() < support.size
    out = []
    for sup in (None, support):
        tr = torch.tensor(r0, dtype=torch.float64, device="cuda", requires_grad=True)
        tw = torch.tensor(w0, dtype=torch.float64, device="cuda", requires_grad=True)
        tnu = torch.from_numpy(np.asarray(wl.nu, float).copy()).cuda().requires_grad_(True)
        fl = vfp.planar_shock_fields(op, torch.tensor(U0, dtype=torch.float64, device="cuda"), tr, tw)
        uN = vfp.advance_with_grad(op, z0, tnu, dt, 12, seg=4, flow=fl, flow_support=sup)
        (uN * g).sum().backward()
        out.append((float(tr.grad), float(tw.grad), tnu.grad.cpu().numpy()))
    _say(f"[support] {int(support.sum())}/{support.size} cells: dJ/dr {out[0][0]:+.12e} vs {out[1][0]:+.12e}, "
         f"dJ/dw {out[0][1]:+.12e} vs {out[1][1]:+.12e}")
    assert abs(out[0][0] - out[1][0]) <= 1e-12 * abs(out[0][0])
    assert abs(out[0][1] - out[1][1]) <= 1e-12 * abs(out[0][1])
    np.testing.assert_allclose(out[1][2], out[0][2], rtol=1e-12, atol=0)
    op.close()


@pytest.mark.parametrize("nx,npc,k,lmax", [(40, 6, 2, 3), (37, 5, 2, 3), (29, 4, 1, 1), (31, 3, 2, 2)])
def test_support_tiles_bit_identical(lib, cuda, nx, npc, k, lmax):
    """With a support set, only the tiles that hold a support cell run the
    U'/dU/dt part: every slot of a support cell and every U / U_face slot is
    bit-identical to the run without a support; the U'/dU/dt slots of the
    other cells are either that same value (a tile shared with a support
    cell) or untouched (zero), and some are untouched.  Odd nx puts tiles
    across p rows and leaves a partial last tile; l_max = 2 gives tiles of
    7 cells."""
    import torch
    from paper_2501_05110_amd import vfp
    wl = W.shock_workload("tiles", nx, npc, k, lmax, w_frac=0.02, seed=9)
    op = vfp.Operator(wl)
    g = torch.Generator(device="cuda").manual_seed(11)
    mu = torch.randn(op.ndofs, dtype=torch.float64, device="cuda", generator=g)
    fwd = torch.randn(op.ndofs, dtype=torch.float64, device="cuda", generator=g)
    support = vfp.planar_shock_support(op, wl.meta["w"])
    assert 0 < support.sum() < support.size
    got = []
    for sup in (None, support):
        op.field_grad_support(sup)
        slots = torch.zeros(op.field_grad_size(), dtype=torch.float64, device="cuda")
        op.field_grad_stage(mu, fwd, 0.25, slots)
        op.field_grad_stage(fwd, mu, -0.5, slots)
        torch.cuda.synchronize()
        got.append(slots.cpu().numpy().reshape(op.ncells, -1))
    full, part = got
    K1 = k + 1
    ns = full.shape[1]
    assert ns == 7 * K1 + 2
    p1 = np.zeros(ns, bool)                     # the U' / dU/dt slots
    for q in range(K1):
        p1[3 * q + 1] = p1[3 * q + 2] = True
    p1[3 * K1 + 2:] = True
    on = np.asarray(support, bool)[np.arange(op.ncells) % nx]
    keep = ~p1[None, :] | on[:, None]
    _say(f"[tiles] {nx}x{npc} k={k} l_max={lmax}: {int(support.sum())}/{nx} x cells in the support")
    assert np.array_equal(part[keep], full[keep])
    rest, ref = part[~keep], full[~keep]
    assert np.all((rest == 0) | (rest == ref))
    assert np.any((rest == 0) & (ref != 0))
    assert np.abs(full[on][:, p1]).max() > 0
    op.close()


@pytest.mark.parametrize("nx,npc,k,lmax", [(14, 5, 2, 3), (11, 4, 1, 2), (9, 3, 2, 1)])
def test_nu_gradient_same_with_flow(lib, cuda, nx, npc, k, lmax):
    """With the flow sensitivities requested, dJ/dnu per cell is formed in
    their launch (which reads the same adjoint and forward stage inputs)
    instead of in the adjoint stages: the adjoint state must come out
    bit-identical and dJ/dnu equal to rounding (the per-cell products are the
    same; only the order of the 16-lane sum may differ with the adjoint's
    launch shape)."""
    import torch
    from paper_2501_05110_amd.vfp import Operator
    wl = shock(nx, npc, k, lmax, seed=12, w_frac=0.05)
    op = Operator(wl)
    dt = op.cfl_dt(0.2)
    n = 5
    rng = np.random.default_rng(31)
    N = op.ndofs
    tz0 = torch.from_numpy(rng.standard_normal(N)).cuda()
    g = torch.from_numpy(rng.standard_normal(N)).cuda()
    tape = torch.empty(4 * n * N, dtype=torch.float64, device="cuda")
    op.advance_tape(tz0, dt, n, tape)
    out = {}
    for mode in ("no_flow", "flow"):
        _say(f"[nu/flow] {nx}x{npc} k={k} lmax={lmax} {mode}")
        mu = g.clone()
        op.mass(mu, mu, inverse=True)
        work = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        gnu = torch.zeros(op.ncells, dtype=torch.float64, device="cuda")
        slots = torch.zeros(op.field_grad_size(), dtype=torch.float64, device="cuda") \
            if mode != "no_flow" else torch.zeros(1, dtype=torch.float64, device="cuda")
        op.adjoint_steps(tz0, tape, dt, n, mu, gnu, work, field_slots=slots if mode != "no_flow" else None)
        torch.cuda.synchronize()
        out[mode] = (mu.cpu().numpy(), gnu.cpu().numpy(), slots.cpu().numpy())
    (m0, g0, _), (m1, g1, s1) = out["no_flow"], out["flow"]
    assert np.array_equal(m0, m1)
    assert np.abs(s1).max() > 0
    scale = np.abs(g0).max()
    assert scale > 0
    err = np.abs(g1 - g0).max() / scale
    _say(f"   max |dJ/dnu| {scale:.3e}, rel diff {err:.1e}")
    assert err <= 1e-13

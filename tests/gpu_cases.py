"""Shared GPU-test helpers: tolerances, seeded workloads of the parity
cases, and a host round trip through the library's apply."""

import sys

import numpy as np

from paper_2501_05110_amd import workloads as W

APPLY_TOL = 1e-12
STEPS_TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def gpu_apply(op, z, with_source=True):
    import torch
    zin = torch.from_numpy(np.ascontiguousarray(z).ravel()).cuda()
    zout = torch.empty_like(zin)
    op.apply(zin, zout, with_source)
    torch.cuda.synchronize()
    return zout.cpu().numpy()


def shock(nx, np_, k, lmax, seed=2, **kw):
    return W.shock_workload(f"shock_{nx}x{np_}_k{k}_l{lmax}", nx, np_, k, lmax, seed=seed, **kw)


def uniform2d(lmax=3, k=1):
    return W.Workload(
        name="xy", lmax=lmax, k=k, axes=("x", "y"),
        nodes=(np.linspace(-1, 1, 14), np.linspace(0, 2.2, 10) ** 1.1),
        bc=((W.ZERO_INFLOW, W.CONTINUOUS), (W.PERIODIC, W.PERIODIC)),
        terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION}), p_fixed=1.3,
        flow=W.uniform_flow([0.1, -0.05, 0.02]), magnetic=W.uniform_field((0.3, -0.6, 1.1)), nu=0.7)


def planar1d(lmax=3, k=2):
    return W.Workload(
        name="x_planar", lmax=lmax, k=k, axes=("x",), nodes=(np.linspace(-3, 3, 41),),
        bc=((W.ZERO_INFLOW, W.CONTINUOUS),),
        terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION}), p_fixed=2.0,
        flow=W.shock_flow(0.1, 4.0, 0.3), magnetic=W.uniform_field((0.5, 0.2, 0.0)), nu=0.4)


def cube(n=(5, 4, 3), lmax=5, k=2):
    return W.config3(n, lmax=lmax, k=k)


def box_mixed(lmax=3, k=2):
    """Three spatial axes with every boundary kind, a uniform flow, a uniform
    B, scattering per cell and a source: the branches of the 3-D kernel that
    the periodic box does not reach."""
    n = (6, 5, 4)
    nodes = (np.linspace(-1.0, 1.0, n[0] + 1), np.linspace(0.0, 1.5, n[1] + 1) ** 1.2,
             np.linspace(-0.5, 0.7, n[2] + 1))
    nu = 0.2 + np.random.default_rng(41).uniform(0.0, 1.0, int(np.prod(n)))
    return W.Workload(
        name="box_mixed", lmax=lmax, k=k, axes=("x", "y", "z"), nodes=nodes,
        bc=((W.ZERO_INFLOW, W.CONTINUOUS), (W.PERIODIC, W.PERIODIC), (W.CONTINUOUS, W.ZERO_INFLOW)),
        terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION, W.SOURCE}), p_fixed=1.3,
        flow=W.uniform_flow([0.1, -0.05, 0.02]), magnetic=W.uniform_field((0.3, -0.6, 1.1)), nu=nu,
        source=lambda X, p: np.exp(-(X[0] ** 2 + (X[2] - 0.1) ** 2)))


def line(k, lmax=3, n=23):
    """1-D x with a planar flow and zero-inflow / continuous ends."""
    return W.Workload(
        name=f"line_k{k}_l{lmax}", lmax=lmax, k=k, axes=("x",), nodes=(np.linspace(-3, 3, n + 1) ** 1.0,),
        bc=((W.ZERO_INFLOW, W.CONTINUOUS),),
        terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION}), p_fixed=2.0,
        flow=W.shock_flow(0.1, 4.0, 0.3), magnetic=W.uniform_field((0.5, 0.2, 0.0)), nu=0.4)


# degrees above 2 (forward operator, general kernels): k <= 5 on one axis,
# k = 3 on two
HIGH_K_CASES = {
    "line_k3_l3": lambda: line(3),
    "line_k4_l5": lambda: line(4, 5, 17),
    "line_k5_l7": lambda: line(5, 7, 13),
    "line_k5_periodic_l3": lambda: W.Workload(
        name="line_k5_periodic", lmax=3, k=5, axes=("x",), nodes=(W.uniform_nodes(-0.5, 0.5, 19),),
        bc=((W.PERIODIC, W.PERIODIC),), terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION}),
        p_fixed=3 ** 0.5, flow=W.zero_flow, magnetic=W.uniform_field((0.0, 0.0, 1.0)), nu=1.0),
    "uniform2d_k3_l3": lambda: uniform2d(3, 3),
    "shock_k3_l3": lambda: shock(11, 6, 3, 3),
}

# momentum axis p itself (general kernels, forward and adjoint)
P_AXIS_CASES = {
    "shock_p_k2_l3": lambda: shock(13, 7, 2, 3, paxis="p", lnp=(-1.0, 2.5)),
    "shock_p_k1_l5": lambda: shock(10, 6, 1, 5, paxis="p", lnp=(-1.0, 2.5)),
    "shock_p_k3_l1": lambda: shock(9, 5, 3, 1, paxis="p", lnp=(-1.0, 2.5)),
    "shock_p_k2_l3_tiles": lambda: shock(16, 7, 2, 3, paxis="p", lnp=(-1.0, 2.5)),
}

def swirl(axes, n, k, lmax, bc, source=True):
    """Spatial axes with the flow, and the scattering rate, given at the
    points (both vary inside every cell), a uniform B and (optionally) a
    source.  On a periodic axis the flow is periodic too (its period is that
    axis' length, and it has no linear part); otherwise it also has a
    divergence."""
    lo, hi = (-1.2, -0.9, -0.6), (1.5, 1.4, 0.9)
    nodes = tuple(np.linspace(lo[a], hi[a], n[a] + 1) ** 1.0 for a in range(len(axes)))
    per = [a for a in range(len(axes)) if bc[a][0] == W.PERIODIC and a < 2]
    length = hi[per[0]] - lo[per[0]] if per else 2.0
    stretch = 0.0 if per else 1.0
    return W.Workload(
        name=f"swirl{len(axes)}d_k{k}_l{lmax}", lmax=lmax, k=k, axes=axes, nodes=nodes, bc=bc,
        terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION} | ({W.SOURCE} if source else set())),
        p_fixed=1.3, flow=W.swirl_flow(U0=(0.12, -0.07, 0.05), amp=0.2, length=length, stretch=stretch),
        magnetic=W.uniform_field((0.3, -0.6, 1.1)), nu=W.varying_scattering(0.7, 0.4, 2.0),
        source=lambda X, p: np.exp(-(X[0] ** 2 + (X[1] - 0.1) ** 2 + X[2] ** 2)))


def field_B(X):
    """A magnetic field that varies along x."""
    return np.stack([1.0 + 0.3 * np.sin(2.0 * X[0]), 0.2 * np.cos(1.5 * X[0]), 0.1 + 0.0 * X[0]])


def shock_fields(nx, np_, k, lmax, B=True, nu=True, seed=2):
    """The shock with B(x) at the points and/or nu(x, p) at the points."""
    from dataclasses import replace
    wl = shock(nx, np_, k, lmax, seed=seed)
    kw = {}
    if B:
        kw["magnetic"] = field_B
    if nu:
        kw["nu"] = W.varying_scattering(1.0, 0.5, 7.0)
    return replace(wl, name=wl.name + ("_B" if B else "") + ("_nu" if nu else ""), **kw)


_ZI, _CO, _PE = W.ZERO_INFLOW, W.CONTINUOUS, W.PERIODIC

# fields given at the points: flow on 1-3 spatial axes, B with a momentum
# axis, nu inside the cells (general kernels, forward and adjoint)
FIELD_CASES = {
    "swirl1d_k2_l7": lambda: swirl(("x",), (21,), 2, 7, ((_ZI, _CO),)),
    "swirl2d_k2_l3": lambda: swirl(("x", "y"), (13, 10), 2, 3, ((_ZI, _CO), (_PE, _PE))),
    "swirl2d_k1_l5": lambda: swirl(("x", "y"), (17, 9), 1, 5, ((_ZI, _ZI), (_CO, _ZI))),
    "swirl2d_k2_l3_tiles": lambda: swirl(("x", "y"), (40, 33), 2, 3, ((_ZI, _CO), (_ZI, _ZI))),
    "swirl3d_k1_l3": lambda: swirl(("x", "y", "z"), (6, 5, 4), 1, 3, ((_ZI, _CO), (_PE, _PE), (_CO, _ZI))),
    "swirl3d_k2_l2": lambda: swirl(("x", "y", "z"), (4, 4, 3), 2, 2, ((_PE, _PE), (_ZI, _CO), (_PE, _PE))),
    "shock_B_k2_l3": lambda: shock_fields(13, 8, 2, 3, nu=False),
    "shock_nu_k2_l3": lambda: shock_fields(12, 7, 2, 3, B=False),
    "shock_B_nu_k1_l5": lambda: shock_fields(11, 6, 1, 5),
}

CASES = {
    "c1": lambda: W.config1(),
    "shock_k2_l3": lambda: shock(25, 11, 2, 3),
    "shock_k1_l3": lambda: shock(19, 7, 1, 3),
    "shock_k2_l1": lambda: shock(13, 9, 2, 1),
    "shock_k1_l5": lambda: shock(11, 6, 1, 5),
    "shock_k2_l7": lambda: shock(9, 5, 2, 7),
    # x rows of whole workgroup tiles (4 cells at l_max = 3, 16 at l_max = 1),
    # and one tile per row
    "shock_k2_l3_tiles": lambda: shock(32, 6, 2, 3),
    "shock_k1_l1_tiles": lambda: shock(32, 5, 1, 1),
    "shock_k2_l3_row": lambda: shock(4, 3, 2, 3),
    "uniform2d": lambda: uniform2d(),
    "uniform2d_k2_l2": lambda: uniform2d(2, 2),
    "planar1d": lambda: planar1d(),
    "cube_k2_l5": lambda: cube(),
    "cube_k1_l3": lambda: cube((4, 3, 5), 3, 1),
    "box_mixed_k2_l3": lambda: box_mixed(),
    "box_mixed_k1_l7": lambda: box_mixed(7, 1),
}

"""Seeded synthetic workloads shaped like the paper's examples.

This module holds inputs only -- grids, background-field profiles, source
shapes, scattering rates and seeded random states -- and none of the
discretisation's arithmetic.  Both the HIP library (through its Python
binding) and the CPU oracle draw their inputs from here, so that the two see
identical data.

Units are the code units of Table 1 (q = m = c = 1 for protons), so that
gamma = sqrt(1 + p^2), V = p / gamma.

Field callables take spatial points X of shape (3, N) (axes that a run does not
simulate are zero) and return arrays over N:

* flow(X) -> (U (3,N), dU (3,3,N) with dU[a,b] = dU_b/dx^a, dUdt (3,N))
* magnetic(X) -> B (3,N)
* source(X, p) -> isotropic source s (N,)   (the s of eq. monoenergetic-point-source)
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20250110

# term names, matching the term switches of eq. vfp-terms-names
ADVECTION, MOMENTUM, ROTATION, COLLISION, SOURCE = (
    "advection", "momentum", "rotation", "collision", "source")

# boundary kinds (Sec. 3.3 and eq. continuous-bc)
PERIODIC, ZERO_INFLOW, CONTINUOUS = "periodic", "zero_inflow", "continuous"


def rng(config_index: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config_index + 1000 * extra)


# ---------------------------------------------------------------- fields --

def zero_flow(X):
    N = X.shape[1]
    return np.zeros((3, N)), np.zeros((3, 3, N)), np.zeros((3, N))


zero_flow.kind = ("uniform", np.zeros(3))


def uniform_flow(U):
    U = np.asarray(U, dtype=float)

    def flow(X):
        N = X.shape[1]
        return (np.repeat(U[:, None], N, axis=1), np.zeros((3, 3, N)),
                np.zeros((3, N)))
    flow.kind = ("uniform", U)
    return flow


def shock_profile(x, U0, r, w):
    """Planar tanh shock U(x) = U0[(r+1)/2 - (r-1)/2 tanh(x/w)] along x.

    Returns (U, dU/dx, dU/dt).  The flow is steady, so its material
    derivative is dU/dt = U dU/dx.  U0 is the downstream speed; the upstream
    speed is r U0.
    """
    t = np.tanh(x / w)
    U = U0 * ((r + 1) / 2 - (r - 1) / 2 * t)
    dU = -U0 * (r - 1) / (2 * w) * (1 - t * t)
    return U, dU, U * dU


def shock_flow(U0, r, w):
    def flow(X):
        N = X.shape[1]
        Ux, dUx, aUx = shock_profile(X[0], U0, r, w)
        U = np.zeros((3, N))
        dU = np.zeros((3, 3, N))
        a = np.zeros((3, N))
        U[0], dU[0, 0], a[0] = Ux, dUx, aUx
        return U, dU, a
    flow.kind = ("planar_x",)
    return flow


def swirl_flow(U0=(0.1, -0.05, 0.02), amp=0.15, length=2.0, stretch=1.0):
    """A steady flow that varies along x and y:
    U_x = U0_x + amp sin(2 pi y / L) + stretch amp x / (2L),
    U_y = U0_y + amp cos(2 pi x / L) - 0.3 stretch amp y / L,
    U_z = U0_z + amp/2 sin(2 pi (x + y) / L);
    divergence-free in (x, y) for stretch = 0 (then also periodic in x and y
    with period L).  Returns U, dU[a, b] = dU_b/dx^a and the material
    derivative U.grad U."""
    U0 = np.asarray(U0, dtype=float)
    k = 2 * math.pi / length

    def flow(X):
        x, y = X[0], X[1]
        N = X.shape[1]
        U = np.zeros((3, N))
        dU = np.zeros((3, 3, N))
        U[0] = U0[0] + amp * np.sin(k * y) + stretch * amp * x / (2 * length)
        U[1] = U0[1] + amp * np.cos(k * x) - 0.3 * stretch * amp * y / length
        U[2] = U0[2] + 0.5 * amp * np.sin(k * (x + y))
        dU[0, 0] = stretch * amp / (2 * length)
        dU[1, 0] = amp * k * np.cos(k * y)
        dU[0, 1] = -amp * k * np.sin(k * x)
        dU[1, 1] = -0.3 * stretch * amp / length
        dU[0, 2] = dU[1, 2] = 0.5 * amp * k * np.cos(k * (x + y))
        a = np.einsum("an,abn->bn", U, dU)
        return U, dU, a
    flow.kind = ("points",)
    return flow


def varying_scattering(nu0=0.7, amp=0.4, length=2.0):
    """nu(x, p) = nu0 (1 + amp sin(2 pi x / L) cos(2 pi y / L)) p^(-1/3):
    varies inside every cell."""
    k = 2 * math.pi / length

    def nu(X, p):
        return nu0 * (1 + amp * np.sin(k * X[0]) * np.cos(k * X[1])) * np.power(p, -1.0 / 3.0)
    return nu


def uniform_field(B):
    B = np.asarray(B, dtype=float)

    def field(X):
        return np.repeat(B[:, None], X.shape[1], axis=1)
    field.kind = ("uniform", B)
    return field


@dataclass
class FourierField:
    """B = B0 + sum over axes a and modes n of A_{a,n} cos(2 pi n x_a / L + phi_{a,n}).

    Each A_{a,n} is perpendicular to e_a, so div B = 0.
    """
    B0: np.ndarray
    amp: np.ndarray      # (3 axes, nmodes, 3 components)
    phase: np.ndarray    # (3, nmodes)
    length: float
    kind = ("points",)

    def __call__(self, X):
        B = np.repeat(np.asarray(self.B0, float)[:, None], X.shape[1], axis=1)
        nm = self.amp.shape[1]
        for a in range(3):
            for k in range(nm):
                c = np.cos(2 * math.pi * (k + 1) * X[a] / self.length + self.phase[a, k])
                B += self.amp[a, k][:, None] * c[None, :]
        return B


def random_fourier_field(seed, B0=(0.0, 0.0, 1.0), nmodes=8, length=20.0,
                         rms=0.5, box=(-10.0, 10.0), grid=48):
    g = np.random.default_rng(seed)
    amp = g.standard_normal((3, nmodes, 3))
    for a in range(3):
        amp[a, :, a] = 0.0
    phase = g.uniform(0, 2 * math.pi, (3, nmodes))
    fld = FourierField(np.zeros(3), amp, phase, length)
    # rescale so that the rms of |delta B| over the cell centres is `rms`
    h = (box[1] - box[0]) / grid
    c = box[0] + h * (np.arange(grid) + 0.5)
    X = np.stack([m.ravel() for m in np.meshgrid(c, c, c, indexing="ij")])
    dB = fld(X)
    scale = rms / math.sqrt(np.mean(np.sum(dB * dB, axis=0)))
    return FourierField(np.asarray(B0, float), amp * scale, phase, length)


def gaussian_source(Q, x0, lnp0, sigma_x, sigma_lnp):
    """Isotropic injection: a Gaussian in (x, ln p) with total rate Q."""
    def source(X, p):
        lp = np.log(p)
        return (Q / (2 * math.pi * sigma_x * sigma_lnp)
                * np.exp(-(X[0] - x0) ** 2 / (2 * sigma_x ** 2))
                * np.exp(-(lp - lnp0) ** 2 / (2 * sigma_lnp ** 2)))
    return source


# ------------------------------------------------------------- workloads --

@dataclass
class Workload:
    """One run: grid, discretisation, physics switches and input fields."""
    name: str
    lmax: int
    k: int
    axes: tuple                 # e.g. ("x",), ("x","lnp"), ("x","y","z")
    nodes: tuple                # per-axis cell boundaries (monotone arrays)
    bc: tuple                   # per-axis (lo, hi) boundary kinds
    terms: frozenset
    p_fixed: float = None       # momentum magnitude if there is no ln p axis
    flow: object = zero_flow
    magnetic: object = None
    nu: object = 0.0            # float, per-cell array (len = ncells) or nu(X, p) at the points
    source: object = None
    mass: float = 1.0
    charge: float = 1.0
    steps: int = 0
    courant: float = 0.2
    meta: dict = field(default_factory=dict)

    @property
    def ncells_axis(self):
        return tuple(len(n) - 1 for n in self.nodes)

    @property
    def ncells(self):
        return int(np.prod(self.ncells_axis))

    @property
    def n_lms(self):
        return (self.lmax + 1) ** 2

    @property
    def n_basis(self):
        return (self.k + 1) ** len(self.axes)

    @property
    def ndofs(self):
        return self.ncells * self.n_basis * self.n_lms

    @property
    def shape(self):
        return (self.ncells, self.n_basis, self.n_lms)


def uniform_nodes(lo, hi, n):
    return np.linspace(lo, hi, n + 1)


def equidistant_node_coords(wl: Workload, axis: int):
    """Coordinates of the k+1 equidistant nodes of every cell along `axis`,
    shape (ncells_axis, k+1).  Used to sample initial data at nodes."""
    nd = wl.nodes[axis]
    t = np.linspace(0.0, 1.0, wl.k + 1)
    return nd[:-1, None] + (nd[1:] - nd[:-1])[:, None] * t[None, :]


def nodal_state(wl: Workload, func):
    """State vector [cell][basis][lms] holding func at the equidistant nodes.

    func(coords: dict axis->array (M,)) -> (n_lms, M) values.
    """
    K1 = wl.k + 1
    naxis = wl.ncells_axis
    grids = [equidistant_node_coords(wl, a) for a in range(len(wl.axes))]
    # multi-index over (cells..., nodes...) flattened in [cell][basis] order
    coords = {}
    d = len(wl.axes)
    cell_idx = np.indices(naxis[::-1]).reshape(d, -1)[::-1]     # axis0 fastest
    node_idx = np.indices((K1,) * d).reshape(d, -1)[::-1]
    for a, name in enumerate(wl.axes):
        c = grids[a][cell_idx[a][:, None], node_idx[a][None, :]]
        coords[name] = c.ravel()
    vals = func(coords)                       # (n_lms, ncells*nb)
    return np.ascontiguousarray(vals.T.reshape(wl.shape))


def random_state(wl: Workload, seed: int, scale: float = 1.0):
    return scale * np.random.default_rng(seed).standard_normal(wl.shape)


# C1: 1-D x, fixed p, periodic, k=1, l_max=3, gamma=2, U=0, B=e_z, nu=1
def config1(ncells=64):
    p = math.sqrt(3.0)                     # gamma = 2
    wl = Workload(
        name="1d_x_lmax3_k1", lmax=3, k=1, axes=("x",),
        nodes=(uniform_nodes(-0.5, 0.5, ncells),),
        bc=((PERIODIC, PERIODIC),),
        terms=frozenset({ADVECTION, ROTATION, COLLISION}),
        p_fixed=p, flow=zero_flow, magnetic=uniform_field((0.0, 0.0, 1.0)),
        nu=1.0, steps=100)
    c = rng(1).standard_normal(wl.n_lms)
    wl.meta["init"] = nodal_state(
        wl, lambda X: c[:, None] * np.exp(-X["x"] ** 2 / (2 * 0.1 ** 2))[None, :])
    return wl


def shock_workload(name, nx, np_, k, lmax, U0=0.1, r=4.0, L=10.0, w_frac=0.01,
                   nu0=1.0, lnp=(0.0, 10.0), seed=2, steps=2000, Q=0.1,
                   lnp_inj=0.5, sigma_lnp=1.0 / 8, init=True, paxis="lnp"):
    """paxis: "lnp" (cells uniform in ln p over `lnp`) or "p" (the momentum
    axis is p itself, cells uniform in p over exp(lnp))."""
    w = w_frac * L
    xn = uniform_nodes(-L, L, nx)
    if paxis == "lnp":
        pn = uniform_nodes(lnp[0], lnp[1], np_)
        pc = np.exp(0.5 * (pn[:-1] + pn[1:]))
    else:
        pn = uniform_nodes(math.exp(lnp[0]), math.exp(lnp[1]), np_)
        pc = 0.5 * (pn[:-1] + pn[1:])
    nu_cell = np.repeat((nu0 * pc ** (-1.0 / 3.0))[:, None], nx, axis=1).ravel()
    wl = Workload(
        name=name, lmax=lmax, k=k, axes=("x", paxis), nodes=(xn, pn),
        bc=((ZERO_INFLOW, CONTINUOUS), (ZERO_INFLOW, ZERO_INFLOW)),
        terms=frozenset({ADVECTION, MOMENTUM, ROTATION, COLLISION, SOURCE}),
        flow=shock_flow(U0, r, w), magnetic=uniform_field((1.0, 0.0, 0.0)),
        nu=nu_cell, source=gaussian_source(Q, 0.0, lnp_inj, w, sigma_lnp),
        steps=steps,
        meta={"U0": U0, "r": r, "w": w, "L": L, "nu0": nu0})
    if init:
        wl.meta["init"] = random_state(wl, SEED_BASE + seed, 1e-3)
    return wl


def paper_shock_x_nodes(shock_halfwidth=0.04, dx_shock=0.01, grow=0.01, half_length=280.0):
    """The stretched x grid of Sec. 4.4 (Fig. shock-grid): cells of
    dx_shock across |x| <= shock_halfwidth, then cell i outside has width
    sinh(grow i) (never below dx_shock), out to |x| = half_length."""
    pos = list(np.arange(0.0, shock_halfwidth + 1e-12, dx_shock))
    i = 1
    while pos[-1] < half_length:
        pos.append(pos[-1] + max(dx_shock, math.sinh(grow * i)))
        i += 1
    pos = np.array(pos)
    pos[-1] = half_length
    return np.concatenate([-pos[::-1], pos[1:]])


def paper_dsa_workload(np_=256, k=1, dx_shock=0.01, grow=0.01):
    """The diffusive-shock-acceleration run of Sec. 4.4 with the parameters
    of Table sapphire-simulation-parameters: U1 = 1/60, r = 4, shock width
    1/25 (tanh profile of eq. sapphire-velocity-profile), nu = 1, B = e_x,
    Q = 0.1, p0 = 2, sigma_x = sigma_p = 1/8 (the source of
    eq. monoenergetic-point-source, Gaussian in p), l_max = 1, the domain
    [-280, 280] x [ln 0.1, ln 100] with the stretched x grid and np_ cells in
    ln p; zero inflow upstream and at both p ends, "continuous" downstream."""
    U1, r, Ls, Q, p0, sx, sp = 1.0 / 60.0, 4.0, 1.0 / 25.0, 0.1, 2.0, 1.0 / 8.0, 1.0 / 8.0

    def source(X, p):
        return (Q / (2 * math.pi * sx * sp) * np.exp(-X[0] ** 2 / (2 * sx * sx))
                * np.exp(-(p - p0) ** 2 / (2 * sp * sp)))
    xn = paper_shock_x_nodes(Ls, dx_shock, grow)
    pn = uniform_nodes(math.log(0.1), math.log(100.0), np_)
    return Workload(
        name=f"dsa_paper_{len(xn) - 1}x{np_}_k{k}", lmax=1, k=k, axes=("x", "lnp"), nodes=(xn, pn),
        bc=((ZERO_INFLOW, CONTINUOUS), (ZERO_INFLOW, ZERO_INFLOW)),
        terms=frozenset({ADVECTION, MOMENTUM, ROTATION, COLLISION, SOURCE}),
        flow=shock_flow(U1 / r, r, Ls), magnetic=uniform_field((1.0, 0.0, 0.0)), nu=1.0, source=source,
        meta={"U1": U1, "r": r, "Q": Q, "p0": p0})


# C2: 2-D (x, ln p) parallel shock, 1024 x 128, k=2, l_max=3
def config2(nx=1024, np_=128, steps=2000):
    return shock_workload("shock2d_x_lnp_1024x128_k2_lmax3", nx, np_, 2, 3,
                          steps=steps, seed=2)


# C3: 3-D x,y,z periodic, 48^3, k=2, l_max=5, fixed p (gamma=2)
def config3(ncell=48, steps=500, lmax=5, k=2):
    p = math.sqrt(3.0)
    nc = (ncell,) * 3 if np.isscalar(ncell) else tuple(ncell)
    nodes = tuple(uniform_nodes(-10.0, 10.0, m) for m in nc)
    B = random_fourier_field(SEED_BASE + 3)
    wl = Workload(
        name=f"3d_xyz_{'x'.join(map(str, nc))}_k{k}_lmax{lmax}", lmax=lmax, k=k, axes=("x", "y", "z"),
        nodes=nodes, bc=((PERIODIC, PERIODIC),) * 3,
        terms=frozenset({ADVECTION, ROTATION, COLLISION}),
        p_fixed=p, flow=zero_flow, magnetic=B, nu=0.1, steps=steps)
    xc = np.random.default_rng(SEED_BASE + 3 + 7).uniform(-10, 10, 3)
    n = wl.n_lms

    def f0(X):
        r2 = (X["x"] - xc[0]) ** 2 + (X["y"] - xc[1]) ** 2 + (X["z"] - xc[2]) ** 2
        out = np.zeros((n, r2.shape[0]))
        out[0] = np.exp(-r2 / (2 * 1.5 ** 2))
        return out
    wl.meta["init_func"] = f0
    wl.meta["B_field"] = B
    return wl


# C4: a batch of independent shock runs of mixed sizes and orders; the
# states are not generated here (about 2e9 DoF in total): callers draw them
# on the device.
def config4(nruns=256, steps=100, seed=4):
    g = np.random.default_rng(SEED_BASE + seed)
    runs = []
    for i in range(nruns):
        nx = int(g.integers(128, 1025))
        np_ = int(g.integers(32, 129))
        k = int(g.integers(1, 3))
        lmax = int(g.choice([1, 3, 5, 7]))
        r = float(g.uniform(2.0, 4.0))
        nu0 = float(np.exp(g.uniform(np.log(0.1), np.log(10.0))))
        runs.append(shock_workload(f"batch_{i}_{nx}x{np_}_k{k}_lmax{lmax}", nx, np_, k, lmax, r=r,
                                   nu0=nu0, seed=seed, steps=steps, init=False))
    return runs


# Many small shock runs (16-64 x 8-16 cells, mixed k and l_max): the regime
# where one launch per run is launch-bound.
def batch_small(nruns=512, steps=50, seed=7):
    g = np.random.default_rng(SEED_BASE + seed)
    runs = []
    for i in range(nruns):
        nx = int(g.integers(16, 65))
        np_ = int(g.integers(8, 17))
        k = int(g.integers(1, 3))
        lmax = int(g.choice([1, 3, 5, 7]))
        r = float(g.uniform(2.0, 4.0))
        runs.append(shock_workload(f"small_{i}_{nx}x{np_}_k{k}_lmax{lmax}", nx, np_, k, lmax, r=r,
                                   seed=seed, steps=steps, init=False))
    return runs


# C5: adjoint case, C2 physics on 512 x 64 cells
def config5(nx=512, np_=64, steps=1000):
    return shock_workload("shock2d_x_lnp_512x64_k2_lmax3", nx, np_, 2, 3,
                          steps=steps, seed=5)

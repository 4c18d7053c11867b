"""Assembled DG system M dzeta/dt + D zeta = h, stepped with classical RK4.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This is the plain definition of the semi-discrete operator of Sec. 3:

* basis: tensor products of 1-D Lagrange polynomials on Gauss-Lobatto nodes
  (eq. lagrange-polynomial; for k <= 2 these are the equidistant nodes);
* mass, DG matrix and load vector of eq. definition-mass-and-dg-matrix, with
  the volume term of eq. linear-system-degrees-of-freedom
  (phi.(R - div beta) f  -  (grad phi . beta) f);
* interior faces: the upwind flux of eq. definition-upwind-flux,
  J = W(Lambda+ W^T f1 + Lambda- W^T f2), with the jump of the test functions
  (eq. numerical-at-interface) and n_F pointing from T1 to T2;
* boundary faces: zero inflow J = W Lambda+ W^T f (eq. definition-boundary-flux)
  or "continuous" J = (n.beta) f (eq. continuous-bc); periodic axes wrap;
* integrals by Gauss-Legendre quadrature with k+1 points per axis (a reading:
  the paper writes exact integrals);
* advection matrices and reaction matrix of eq. definitions-advection-reaction-eq
  with the momentum axis taken as ln p (beta^{ln p} = beta^p / p) -- a reading of
  "momentum terms adapted accordingly" (Sec. 4, term list);
* time stepping: classical RK4 on dzeta/dt = M^{-1}(h - D zeta), and the
  Theta-method of eq. theta-method / eq. system-matrix-rhs by sparse LU.

Nothing is blocked, fused or reordered; per-cell loops are plain Python.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as npleg

from . import sh

SPATIAL = {"x": 0, "y": 1, "z": 2}


# ------------------------------------------------------------ 1-D basis --

def lobatto_nodes(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto points on [-1, 1]: +-1 and the roots of P_k'."""
    if k == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(k + 1)
    c[k] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(c)).real)
    return np.concatenate([[-1.0], inner, [1.0]])


def gauss_rule(q: int):
    """q-point Gauss-Legendre rule on [-1, 1]."""
    return npleg.leggauss(q)


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values (len(x), k+1) and derivatives of the Lagrange polynomials."""
    K1 = len(nodes)
    x = np.atleast_1d(np.asarray(x, float))
    val = np.ones((len(x), K1))
    der = np.zeros((len(x), K1))
    for i in range(K1):
        for j in range(K1):
            if j == i:
                continue
            val[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
        # derivative by the product rule
        for m in range(K1):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(K1):
                if j in (i, m):
                    continue
                term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            der[:, i] += term
    return val, der


# -------------------------------------------------------- coefficients --

@dataclass
class Physics:
    lmax: int
    terms: frozenset
    mass: float = 1.0
    charge: float = 1.0


def point_coefficients(phys: Physics, axes, X, p, flow, magnetic, nu):
    """beta^alpha (d, N, n, n) and G = R - div(beta) (N, n, n) at N points."""
    beta, R, div = point_terms(phys, axes, X, p, flow, magnetic, nu)
    return beta, R - div


def point_terms(phys: Physics, axes, X, p, flow, magnetic, nu):
    """beta^alpha (d, N, n, n), R (N, n, n) and div(beta) (N, n, n) at N points.

    X: (3, N) spatial coordinates; p: (N,) momentum magnitudes; nu: (N,).
    Eq. definitions-advection-reaction-eq on a "p" axis; on an "lnp" axis
    d/dp is replaced by d/d ln p.
    """
    S = sh.system_matrices(phys.lmax)
    n = S["n"]
    N = X.shape[1]
    A, Om, C = S["A"], S["Om"], S["C"]
    AA, AOm, AAOm = S["AA"], S["AOm"], S["AAOm"]
    eps = sh.EPS
    m_, q_ = phys.mass, phys.charge
    gam = np.sqrt(1.0 + (p / m_) ** 2)
    V = p / (gam * m_)
    U, dU, a = flow(X)
    on = phys.terms
    beta = np.zeros((len(axes), N, n, n))
    R = np.zeros((N, n, n))
    div = np.zeros((N, n, n))
    I = np.eye(n)
    for ax, name in enumerate(axes):
        if name in SPATIAL:
            c = SPATIAL[name]
            if "advection" in on:
                beta[ax] = U[c][:, None, None] * I + V[:, None, None] * A[c]
                div += dU[c, c][:, None, None] * I
        elif name == "lnp":
            if "momentum" in on:
                # beta^p / p = -(gamma m / p) dU_a/dt A^a - dU_b/dx^a (A^a A^b)_t
                for aa in range(3):
                    beta[ax] -= (gam * m_ / p * a[aa])[:, None, None] * A[aa]
                    for bb in range(3):
                        beta[ax] -= dU[aa, bb][:, None, None] * AA[aa, bb]
                # d/d ln p of beta^{ln p}: only gamma m / p depends on p,
                # d(gamma m/p)/d ln p = -m/(gamma p)
                for aa in range(3):
                    div += (m_ / (gam * p) * a[aa])[:, None, None] * A[aa]
        elif name == "p":
            if "momentum" in on:
                # beta^p = -gamma m dU_a/dt A^a - p dU_b/dx^a (A^a A^b)_t
                # (eq. definitions-advection-reaction-eq, the fourth component)
                for aa in range(3):
                    beta[ax] -= (gam * m_ * a[aa])[:, None, None] * A[aa]
                    for bb in range(3):
                        beta[ax] -= (p * dU[aa, bb])[:, None, None] * AA[aa, bb]
                # d/dp of beta^p, with d(gamma m)/dp = p/(gamma m) = V
                for aa in range(3):
                    div -= (V * a[aa])[:, None, None] * A[aa]
                    for bb in range(3):
                        div -= dU[aa, bb][:, None, None] * AA[aa, bb]
        else:
            raise ValueError(name)
    if "momentum" in on:
        for aa in range(3):
            for bb in range(3):
                for cc in range(3):
                    e = eps[aa, bb, cc]
                    if e:
                        R += (e / V * a[aa])[:, None, None] * AOm[bb, cc]
        for aa in range(3):
            for bb in range(3):
                for cc in range(3):
                    for dd in range(3):
                        e = eps[bb, cc, dd]
                        if e:
                            R += (e * dU[aa, bb])[:, None, None] * AAOm[aa, cc, dd]
    if "rotation" in on and magnetic is not None:
        B = magnetic(X)
        for aa in range(3):
            omega = q_ * B[aa] / (gam * m_)
            R -= omega[:, None, None] * Om[aa]
    if "collision" in on:
        R += nu[:, None, None] * C
    return beta, R, div


# ------------------------------------------------------------ the system --

@dataclass
class System:
    D: sp.csr_matrix
    M: sp.csr_matrix
    Minv: sp.csr_matrix
    h: np.ndarray
    rows_cells: np.ndarray      # cells whose rows were assembled
    shape: tuple                # (ncells, nb, n)


class Grid:
    """Tensor grid bookkeeping for a Workload-like object."""

    def __init__(self, wl):
        self.wl = wl
        self.axes = tuple(wl.axes)
        self.d = len(self.axes)
        self.k = wl.k
        self.K1 = wl.k + 1
        self.n = (wl.lmax + 1) ** 2
        self.nb = self.K1 ** self.d
        self.nodes = [np.asarray(nd, float) for nd in wl.nodes]
        self.N = [len(nd) - 1 for nd in self.nodes]
        self.ncells = int(np.prod(self.N))
        self.ref_nodes = lobatto_nodes(self.k)
        self.gq, self.gw = gauss_rule(self.K1)
        self.Lq, self.Dq = lagrange(self.ref_nodes, self.gq)        # (q, j)
        self.Lend, _ = lagrange(self.ref_nodes, np.array([-1.0, 1.0]))  # (2, j)
        self.phys = Physics(wl.lmax, frozenset(wl.terms), wl.mass, wl.charge)
        nu = wl.nu
        # nu is a constant, one value per cell, or a function nu(X, p)
        # sampled at the quadrature points like the other coefficients
        self.nu_fn = nu if callable(nu) else None
        self.nu_cell = (None if self.nu_fn else
                        np.full(self.ncells, float(nu)) if np.isscalar(nu) else np.asarray(nu, float))

    def cell_multi(self, c):
        idx = []
        for a in range(self.d):
            idx.append(c % self.N[a])
            c //= self.N[a]
        return idx

    def cell_flat(self, idx):
        c = 0
        for a in reversed(range(self.d)):
            c = c * self.N[a] + idx[a]
        return c

    def basis_multi(self):
        """(nb, d) node multi-indices, axis 0 fastest."""
        return np.indices((self.K1,) * self.d).reshape(self.d, -1)[::-1].T

    def points(self, idx, eta):
        """Physical points for reference coords eta (d, Q) in cell idx.

        Returns X (3, Q) spatial coordinates and p (Q,) momentum magnitudes.
        """
        Q = eta.shape[1]
        X = np.zeros((3, Q))
        p = np.full(Q, np.nan if self.wl.p_fixed is None else float(self.wl.p_fixed))
        for a, name in enumerate(self.axes):
            lo, hi = self.nodes[a][idx[a]], self.nodes[a][idx[a] + 1]
            xi = lo + (1.0 + eta[a]) * (hi - lo) / 2.0
            if name in SPATIAL:
                X[SPATIAL[name]] = xi
            elif name == "lnp":
                p = np.exp(xi)
            else:
                p = xi
        return X, p

    def widths(self, idx):
        return np.array([self.nodes[a][idx[a] + 1] - self.nodes[a][idx[a]]
                         for a in range(self.d)])

    def coefficients(self, c, X, p):
        nu = self.nu_fn(X, p) if self.nu_fn else np.full(X.shape[1], self.nu_cell[c])
        return point_coefficients(self.phys, self.axes, X, p, self.wl.flow,
                                  self.wl.magnetic, nu)

    def volume_tables(self):
        """Reference values at the (k+1)^d Gauss points: phi (Q, nb), dphi_ref
        (d, Q, nb), eta (d, Q), weights (Q,)."""
        bm = self.basis_multi()
        # point multi-indices of the rule (len(gq) points per axis, axis 0
        # fastest, as the basis); the method's rule has k+1 points
        nq = len(self.gq)
        qm = np.indices((nq,) * self.d).reshape(self.d, -1)[::-1].T
        Q = len(qm)
        phi = np.ones((Q, self.nb))
        dphi = np.ones((self.d, Q, self.nb))
        w = np.ones(Q)
        eta = np.zeros((self.d, Q))
        for a in range(self.d):
            qa = qm[:, a]
            ja = bm[:, a]
            phi *= self.Lq[qa][:, ja]
            w *= self.gw[qa]
            eta[a] = self.gq[qa]
            for b in range(self.d):
                dphi[b] *= (self.Dq if a == b else self.Lq)[qa][:, ja]
        return phi, dphi, eta, w

    def face_tables(self, axis, side):
        """Face points on side (0 = lo, 1 = hi) of `axis`: phi of the cell at
        the face (Qf, nb), phi of the neighbour at its opposite face, eta
        (d, Qf) in this cell, weights (Qf,)."""
        bm = self.basis_multi()
        other = [a for a in range(self.d) if a != axis]
        qm = (np.indices((len(self.gq),) * len(other)).reshape(len(other), -1)[::-1].T
              if other else np.zeros((1, 0), int))
        Qf = qm.shape[0]
        phi_in = np.ones((Qf, self.nb))
        phi_out = np.ones((Qf, self.nb))
        w = np.ones(Qf)
        eta = np.zeros((self.d, Qf))
        for t, a in enumerate(other):
            qa = qm[:, t]
            phi_in *= self.Lq[qa][:, bm[:, a]]
            phi_out *= self.Lq[qa][:, bm[:, a]]
            w *= self.gw[qa]
            eta[a] = self.gq[qa]
        eta[axis] = -1.0 if side == 0 else 1.0
        phi_in *= self.Lend[side][bm[:, axis]][None, :]
        phi_out *= self.Lend[1 - side][bm[:, axis]][None, :]
        return phi_in, phi_out, eta, w


def _split(B):
    """Upwind split B = B+ + B- via the eigen-decomposition (W orthogonal)."""
    lam, W = np.linalg.eigh(B)
    Bp = np.einsum("...ij,...j,...kj->...ik", W, np.maximum(lam, 0.0), W)
    Bm = np.einsum("...ij,...j,...kj->...ik", W, np.minimum(lam, 0.0), W)
    return Bp, Bm


def assemble(wl, cells=None) -> System:
    """Assemble M, D, h (rows of `cells` only; all cells by default)."""
    g = Grid(wl)
    n, nb, d = g.n, g.nb, g.d
    ndof = g.ncells * nb * n
    cells = np.arange(g.ncells) if cells is None else np.asarray(cells)
    phiV, dphiV, etaV, wV = g.volume_tables()
    faces = {(a, s): g.face_tables(a, s) for a in range(d) for s in (0, 1)}
    rows, cols, vals = [], [], []
    mrows, mcols, mvals, irows, icols, ivals = [], [], [], [], [], []
    h = np.zeros(ndof)
    In = np.eye(n)
    src_on = "source" in g.phys.terms and wl.source is not None
    s000 = math.sqrt(4.0 * math.pi)

    def put(rc, cc, block):
        r0, c0 = rc * nb * n, cc * nb * n
        nz = np.nonzero(block)
        rows.append(r0 + nz[0])
        cols.append(c0 + nz[1])
        vals.append(block[nz])

    for c in cells:
        idx = g.cell_multi(int(c))
        hw = g.widths(idx)
        J = np.prod(hw / 2.0)
        X, p = g.points(idx, etaV)
        beta, G = g.coefficients(c, X, p)
        wJ = wV * J
        dphi = dphiV * (2.0 / hw)[:, None, None]
        blk = np.einsum("q,qi,qj,qac->iajc", wJ, phiV, phiV, G)
        blk -= np.einsum("q,dqi,qj,dqac->iajc", wJ, dphi, phiV, beta)
        # faces
        own = {c: blk}
        for a in range(d):
            for side in (0, 1):
                phi_in, phi_out, etaF, wF = faces[(a, side)]
                JF = np.prod(np.delete(hw, a) / 2.0) if d > 1 else 1.0
                XF, pF = g.points(idx, etaF)
                betaF, _ = g.coefficients(c, XF, pF)
                B = betaF[a]
                nidx = list(idx)
                nidx[a] += 1 if side == 1 else -1
                kind = wl.bc[a][side]
                if 0 <= nidx[a] < g.N[a] or kind == "periodic":
                    nidx[a] %= g.N[a]
                    cn = g.cell_flat(nidx)
                    Bp, Bm = _split(B)
                    wf = wF * JF
                    if side == 1:      # this cell is T1, neighbour is T2
                        self_blk = np.einsum("q,qi,qj,qac->iajc", wf, phi_in, phi_in, Bp)
                        nb_blk = np.einsum("q,qi,qj,qac->iajc", wf, phi_in, phi_out, Bm)
                    else:              # this cell is T2, neighbour is T1
                        self_blk = -np.einsum("q,qi,qj,qac->iajc", wf, phi_in, phi_in, Bm)
                        nb_blk = -np.einsum("q,qi,qj,qac->iajc", wf, phi_in, phi_out, Bp)
                    own[c] = own[c] + self_blk
                    own[cn] = own.get(cn, 0) + nb_blk
                else:
                    Bn = B if side == 1 else -B
                    if kind == "zero_inflow":
                        Bn = _split(Bn)[0]
                    elif kind != "continuous":
                        raise ValueError(kind)
                    own[c] = own[c] + np.einsum("q,qi,qj,qac->iajc", wF * JF,
                                                phi_in, phi_in, Bn)
        for cc, b in own.items():
            put(int(c), int(cc), b.reshape(nb * n, nb * n))
        # mass block and its inverse (the basis mass matrix times I_n)
        Mt = np.einsum("q,qi,qj->ij", wJ, phiV, phiV)
        Mi = np.linalg.inv(Mt)
        Mfull = np.kron(Mt, In)
        Mifull = np.kron(Mi, In)
        base = int(c) * nb * n
        r_, c_ = np.nonzero(Mfull)
        mrows.append(base + r_); mcols.append(base + c_); mvals.append(Mfull[r_, c_])
        r_, c_ = np.nonzero(Mifull)
        irows.append(base + r_); icols.append(base + c_); ivals.append(Mifull[r_, c_])
        if src_on:
            sv = s000 * wl.source(X, p)
            hc = np.einsum("q,qi,q->i", wJ, phiV, sv)
            h[base + np.arange(nb) * n] = hc

    def csr(rr, cc, vv):
        if not rr:
            return sp.csr_matrix((ndof, ndof))
        return sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))),
                             shape=(ndof, ndof))

    return System(csr(rows, cols, vals), csr(mrows, mcols, mvals),
                  csr(irows, icols, ivals), h, cells, (g.ncells, nb, n))


# ----------------------------------------------------------- operators --

def apply(sysm: System, zeta, with_source=True):
    """M^{-1}(h - D zeta) as a flat vector (rows of assembled cells only)."""
    z = np.asarray(zeta, float).ravel()
    r = -(sysm.D @ z)
    if with_source:
        r = r + sysm.h
    return sysm.Minv @ r


def apply_adjoint(sysm: System, lam):
    """Euclidean adjoint of the linear part of `apply`: -D^T M^{-1} lam."""
    return -(sysm.D.T @ (sysm.Minv @ np.asarray(lam, float).ravel()))


def rk4(sysm: System, zeta, dt, nsteps, with_source=True):
    """Classical RK4 (nodes 0, 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6)."""
    z = np.asarray(zeta, float).ravel().copy()
    for _ in range(nsteps):
        k1 = apply(sysm, z, with_source)
        k2 = apply(sysm, z + 0.5 * dt * k1, with_source)
        k3 = apply(sysm, z + 0.5 * dt * k2, with_source)
        k4 = apply(sysm, z + dt * k3, with_source)
        z = z + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return z


def collision_system(wl) -> System:
    """The collision part alone with nu = 1 in every cell: its D is
    sum_c (M_c x C) restricted to cell c, so that d D / d nu_c is that block
    (the nu C term of R in eq. definitions-advection-reaction-eq, integrated
    as in eq. definition-mass-and-dg-matrix)."""
    from dataclasses import replace
    return assemble(replace(wl, terms=frozenset({"collision"}), nu=1.0, source=None))


def rk4_gradient(sysm: System, zeta0, dt, nsteps, dJ_dzN, dsys=None, with_source=True):
    """Reverse mode of `rk4` for a loss J(zeta_N) with dJ/dzeta_N given.

    Returns (dJ/dzeta_0, dJ/dnu) where dJ/dnu (one value per cell) is formed
    when `dsys` (from `collision_system`) is given: d apply(x)/d nu_c is
    -M^{-1} (dD/dnu_c) x.  Each classical RK4 stage is transposed in turn;
    the forward states are kept for every step.
    """
    z = np.asarray(zeta0, float).ravel().copy()
    states = []
    for _ in range(nsteps):
        states.append(z.copy())
        k1 = apply(sysm, z, with_source)
        k2 = apply(sysm, z + 0.5 * dt * k1, with_source)
        k3 = apply(sysm, z + 0.5 * dt * k2, with_source)
        k4 = apply(sysm, z + dt * k3, with_source)
        z = z + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    ncells, nb, n = sysm.shape
    gnu = np.zeros(ncells) if dsys is not None else None

    def dnu(kbar, x):
        if gnu is None:
            return
        t = -(sysm.Minv @ (dsys.D @ x))
        gnu[:] += (kbar * t).reshape(ncells, nb * n).sum(axis=1)

    zbar = np.asarray(dJ_dzN, float).ravel().copy()
    for zs in reversed(states):
        k1 = apply(sysm, zs, with_source)
        x2 = zs + 0.5 * dt * k1
        k2 = apply(sysm, x2, with_source)
        x3 = zs + 0.5 * dt * k2
        k3 = apply(sysm, x3, with_source)
        x4 = zs + dt * k3
        kb1, kb2, kb3, kb4 = dt / 6.0 * zbar, dt / 3.0 * zbar, dt / 3.0 * zbar, dt / 6.0 * zbar
        znew = zbar.copy()
        dnu(kb4, x4)
        xb4 = apply_adjoint(sysm, kb4)
        znew += xb4
        kb3 = kb3 + dt * xb4
        dnu(kb3, x3)
        xb3 = apply_adjoint(sysm, kb3)
        znew += xb3
        kb2 = kb2 + 0.5 * dt * xb3
        dnu(kb2, x2)
        xb2 = apply_adjoint(sysm, kb2)
        znew += xb2
        kb1 = kb1 + 0.5 * dt * xb2
        dnu(kb1, zs)
        znew += apply_adjoint(sysm, kb1)
        zbar = znew
    return zbar, gnu


def theta_step(sysm: System, zeta, dt, theta, nsteps=1):
    """Theta-method (eq. theta-method) with time-independent D and h: each
    step solves the linear system of eq. system-matrix-rhs,
        (M + dt theta D) zeta^n = (M - dt (1 - theta) D) zeta^{n-1} + dt h,
    by a sparse LU factorisation of its matrix (direct, so the result is the
    system's exact solution up to rounding)."""
    z = np.asarray(zeta, float).ravel().copy()
    lhs = (sysm.M + (dt * theta) * sysm.D).tocsc()
    rhs_op = sysm.M - (dt * (1.0 - theta)) * sysm.D
    lu = spla.splu(lhs)
    for _ in range(nsteps):
        z = lu.solve(rhs_op @ z + dt * sysm.h)
    return z


def steady_state(sysm: System):
    """Solve D zeta = h (sparse LU)."""
    return spla.spsolve(sysm.D.tocsc(), sysm.h)


def load_vector(wl, func):
    """int_T phi_i . func over every cell (the form of h in
    eq. definition-mass-and-dg-matrix for a general vector source).

    func(X (3,N), p (N,)) -> (n, N).  Returns (ncells, nb, n).
    """
    g = Grid(wl)
    phiV, _, etaV, wV = g.volume_tables()
    out = np.zeros((g.ncells, g.nb, g.n))
    for c in range(g.ncells):
        idx = g.cell_multi(c)
        J = np.prod(g.widths(idx) / 2.0)
        X, p = g.points(idx, etaV)
        out[c] = np.einsum("q,qi,aq->ia", wV * J, phiV, func(X, p))
    return out


def project(wl, func):
    """L^2 projection of func onto V_h (eq. zeta-initial-condition).

    func(X (3,N), p (N,)) -> (n, N).  Returns (ncells, nb, n).
    """
    g = Grid(wl)
    phiV, _, etaV, wV = g.volume_tables()
    rhs = load_vector(wl, func)
    out = np.zeros_like(rhs)
    for c in range(g.ncells):
        J = np.prod(g.widths(g.cell_multi(c)) / 2.0)
        Mt = np.einsum("q,qi,qj->ij", wV * J, phiV, phiV)
        out[c] = np.linalg.solve(Mt, rhs[c])
    return out


def l2_error(wl, zeta, func, extra=3):
    """sqrt(int |f_h - func|^2) summed over lms, with a (k+1+extra)-point
    Gauss rule per axis.  func(X, p) -> (n, N)."""
    g = Grid(wl)
    q, w = gauss_rule(g.K1 + extra)
    d = g.d
    qm = np.indices((len(q),) * d).reshape(d, -1)[::-1].T
    eta = np.stack([q[qm[:, a]] for a in range(d)])
    wq = np.prod(np.stack([w[qm[:, a]] for a in range(d)]), axis=0)
    fh = evaluate(wl, zeta, eta)                       # (ncells, Q, n)
    tot = 0.0
    for c in range(g.ncells):
        idx = g.cell_multi(c)
        J = np.prod(g.widths(idx) / 2.0)
        X, p = g.points(idx, eta)
        diff = fh[c] - func(X, p).T
        tot += np.sum(wq * J * np.sum(diff * diff, axis=1))
    return math.sqrt(tot)


def evaluate(wl, zeta, eta_points):
    """f_h at reference points eta (d, Q) of every cell -> (ncells, Q, n)."""
    g = Grid(wl)
    bm = g.basis_multi()
    z = np.asarray(zeta, float).reshape(g.ncells, g.nb, g.n)
    phi = np.ones((eta_points.shape[1], g.nb))
    for a in range(g.d):
        v, _ = lagrange(g.ref_nodes, eta_points[a])
        phi *= v[:, bm[:, a]]
    return np.einsum("qb,cbn->cqn", phi, z)

"""Thin ctypes binding of libvfp.so (include/vfp.h).

Argument marshalling only: every step of the operator runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  The
binding fails loudly if the library is missing -- there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvfp.so")

AXIS = {"x": 0, "y": 1, "z": 2, "lnp": 3, "p": 4}
TERM = {"advection": 1, "momentum": 2, "rotation": 4, "collision": 8, "source": 16}
BC = {"periodic": 0, "zero_inflow": 1, "continuous": 2}
PTS_VOLUME, PTS_FACE, PTS_NODE = 0, 1, 2

_lib = None


class VFPError(RuntimeError):
    pass


class ThetaOpts(C.Structure):
    """vfp_theta_opts"""
    _fields_ = [("theta", C.c_double), ("tol", C.c_double), ("restart", C.c_int), ("max_iters", C.c_int),
                ("precond", C.c_int)]


class ThetaStats(C.Structure):
    """vfp_theta_stats"""
    _fields_ = [("iterations", C.c_int64), ("residual", C.c_double), ("converged", C.c_int)]


def load(path: str = None):
    """Load the built library (never builds it)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("VFP_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise VFPError(f"{path} is missing: build it with `python -m paper_2501_05110_amd.build`")
    # torch's bundled HIP runtime carries the same SONAME as the one libvfp
    # links against; loading torch first makes the process use one runtime.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I, D, U, L = C.c_void_p, C.c_int, C.c_double, C.c_uint, C.c_int64
    dp = C.POINTER(C.c_double)
    sig = {
        "vfp_last_error": (C.c_char_p, []),
        "vfp_create": (I, [C.POINTER(P), I, I, I, C.POINTER(I), U, D, D]),
        "vfp_destroy": (None, [P]),
        "vfp_set_mesh": (I, [P, C.POINTER(I), C.POINTER(dp), C.POINTER(I), C.POINTER(I)]),
        "vfp_set_momentum": (I, [P, D]),
        "vfp_query_points": (I, [P, I, I, dp, C.POINTER(L)]),
        "vfp_set_flow_uniform": (I, [P, dp]),
        "vfp_set_flow_planar": (I, [P, dp, dp, dp, dp]),
        "vfp_set_flow_points": (I, [P, dp, dp, C.POINTER(dp)]),
        "vfp_set_magnetic_uniform": (I, [P, dp]),
        "vfp_set_magnetic_points": (I, [P, dp]),
        "vfp_set_scattering": (I, [P, D, dp]),
        "vfp_set_scattering_points": (I, [P, dp]),
        "vfp_set_source_points": (I, [P, dp]),
        "vfp_ndofs": (I, [P, C.POINTER(L)]),
        "vfp_cfl_dt": (I, [P, D, dp]),
        "vfp_autotune": (I, [P, P, P, I, C.POINTER(I), P]),
        "vfp_apply": (I, [P, P, P, I, P]),
        "vfp_stage": (I, [P, P, P, P, D, P]),
        "vfp_advance": (I, [P, P, D, L, P, P]),
        "vfp_mass": (I, [P, P, P, I, P]),
        "vfp_apply_adjoint": (I, [P, P, P, P, P]),
        "vfp_apply_adjoint_noalloc": (I, [P, P, P, P]),
        "vfp_adjoint_stage": (I, [P, P, P, P, D, P, P, P, P]),
        "vfp_advance_tape": (I, [P, P, D, L, P, P]),
        "vfp_adjoint_steps": (I, [P, P, P, D, L, P, P, P, P, P]),
        "vfp_forward_checkpoints": (I, [P, P, D, L, L, P, P, P]),
        "vfp_adjoint_checkpointed": (I, [P, P, D, L, L, P, P, P, P, P, P]),
        "vfp_field_grad_size": (I, [P, C.POINTER(L)]),
        "vfp_field_grad_support": (I, [P, C.POINTER(C.c_ubyte)]),
        "vfp_field_grad_stage": (I, [P, P, P, D, P, P]),
        "vfp_field_grad_reduce": (I, [P, P, P, P, P, P, P]),
        "vfp_sh_eval": (I, [I, L, dp, dp, dp]),
        "vfp_reconstruct": (I, [P, P, P, L, P, P]),
        "vfp_theta_work_size": (I, [P, I, C.POINTER(L)]),
        "vfp_theta_precond_size": (I, [P, I, C.POINTER(L)]),
        "vfp_theta_advance": (I, [P, P, D, L, C.POINTER(ThetaOpts), P, L, C.POINTER(ThetaStats), P]),
        "vfp_batch_create": (I, [C.POINTER(P), C.POINTER(P), I, U]),
        "vfp_batch_destroy": (None, [P]),
        "vfp_batch_bind": (I, [P, C.POINTER(P), C.POINTER(P), dp]),
        "vfp_batch_advance": (I, [P, L, P]),
        "vfp_batch_autotune": (I, [P, I, P]),
        "vfp_batch_nclasses": (I, [P]),
        "vfp_batch_class_info": (I, [P, I, C.POINTER(I)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["vfp_last_error", "vfp_create", "vfp_destroy", "vfp_set_mesh", "vfp_set_momentum",
            "vfp_query_points", "vfp_set_flow_uniform", "vfp_set_flow_planar", "vfp_set_flow_points",
            "vfp_set_magnetic_uniform", "vfp_set_magnetic_points", "vfp_set_scattering",
            "vfp_set_scattering_points",
            "vfp_set_source_points", "vfp_ndofs", "vfp_cfl_dt", "vfp_autotune", "vfp_apply", "vfp_stage",
            "vfp_advance", "vfp_mass", "vfp_apply_adjoint", "vfp_apply_adjoint_noalloc", "vfp_adjoint_stage", "vfp_advance_tape",
            "vfp_adjoint_steps", "vfp_forward_checkpoints", "vfp_adjoint_checkpointed",
            "vfp_batch_create", "vfp_batch_destroy", "vfp_batch_bind", "vfp_batch_advance",
            "vfp_batch_autotune", "vfp_batch_nclasses", "vfp_batch_class_info",
            "vfp_field_grad_size", "vfp_field_grad_support", "vfp_field_grad_stage", "vfp_field_grad_reduce",
            "vfp_theta_work_size", "vfp_theta_precond_size", "vfp_theta_advance", "vfp_sh_eval",
            "vfp_reconstruct"]


def _check(rc):
    if rc != 0:
        msg = _lib.vfp_last_error().decode()
        raise VFPError(f"vfp error {rc}: {msg}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Operator:
    """The DG operator of one run (a context of the C library)."""

    def __init__(self, wl):
        lib = load()
        self.wl = wl
        self._ctx = C.c_void_p()
        kinds = (C.c_int * len(wl.axes))(*[AXIS[a] for a in wl.axes])
        mask = 0
        for t in wl.terms:
            mask |= TERM[t]
        _check(lib.vfp_create(C.byref(self._ctx), wl.lmax, wl.k, len(wl.axes), kinds, mask,
                              float(wl.mass), float(wl.charge)))
        d = len(wl.axes)
        self._nodes = [_f64(n) for n in wl.nodes]
        nc = (C.c_int * d)(*[len(n) - 1 for n in self._nodes])
        nptr = (C.POINTER(C.c_double) * d)(*[_dptr(n) for n in self._nodes])
        lo = (C.c_int * d)(*[BC[b[0]] for b in wl.bc])
        hi = (C.c_int * d)(*[BC[b[1]] for b in wl.bc])
        _check(lib.vfp_set_mesh(self._ctx, nc, nptr, lo, hi))
        self.mom = "lnp" in wl.axes or "p" in wl.axes
        if not self.mom:
            _check(lib.vfp_set_momentum(self._ctx, float(wl.p_fixed)))
        self._set_fields()
        n = C.c_int64()
        _check(lib.vfp_ndofs(self._ctx, C.byref(n)))
        self.ndofs = n.value
        self.shape = wl.shape

    # -- field sampling at the points the library reports ----------------
    def points(self, which, axis):
        cnt = C.c_int64()
        _check(_lib.vfp_query_points(self._ctx, which, axis, None, C.byref(cnt)))
        out = np.zeros(cnt.value)
        _check(_lib.vfp_query_points(self._ctx, which, axis, _dptr(out), C.byref(cnt)))
        return out

    def volume_points(self):
        """Spatial coordinates X (3, ncells*nb) and momenta p of every volume
        point, ordered [cell][q]."""
        wl = self.wl
        d = len(wl.axes)
        K1 = wl.k + 1
        ncx = wl.ncells_axis
        coords = [self.points(PTS_VOLUME, a).reshape(ncx[a], K1) for a in range(d)]
        cell_idx = np.indices(ncx[::-1]).reshape(d, -1)[::-1]
        q_idx = np.indices((K1,) * d).reshape(d, -1)[::-1]
        X = np.zeros((3, wl.ncells * wl.n_basis))
        p = np.full(X.shape[1], np.nan if wl.p_fixed is None else float(wl.p_fixed))
        for a, name in enumerate(wl.axes):
            v = coords[a][cell_idx[a][:, None], q_idx[a][None, :]].ravel()
            if name == "lnp":
                p = np.exp(v)
            elif name == "p":
                p = v
            else:
                X[AXIS[name]] = v
        return X, p

    def face_points(self, axis):
        """Spatial coordinates X (3, nfaces*nqf) of the Gauss points of the
        faces normal to `axis`, ordered [face][qf]: faces over (N_axis + 1)
        positions on that axis and N_b cells on the others (axis 0 fastest),
        qf over the other axes' Gauss points (first other axis fastest)."""
        wl = self.wl
        d = len(wl.axes)
        K1 = wl.k + 1
        ncx = list(wl.ncells_axis)
        ext = [ncx[b] + (1 if b == axis else 0) for b in range(d)]
        f_idx = np.indices(ext[::-1]).reshape(d, -1)[::-1]          # (d, nfaces), axis 0 fastest
        others = [b for b in range(d) if b != axis]
        q_idx = (np.indices((K1,) * len(others)).reshape(len(others), -1)[::-1]
                 if others else np.zeros((0, 1), int))
        nf, nqf = f_idx.shape[1], q_idx.shape[1]
        X = np.zeros((3, nf * nqf))
        for b, name in enumerate(wl.axes):
            if b == axis:
                v = np.repeat(self.points(PTS_FACE, b)[f_idx[b]], nqf)
            else:
                t = others.index(b)
                vol = self.points(PTS_VOLUME, b).reshape(ncx[b], K1)
                v = vol[f_idx[b][:, None], q_idx[t][None, :]].ravel()
            X[AXIS[name]] = v
        return X

    def _set_fields(self):
        wl, lib, ctx = self.wl, _lib, self._ctx
        kind = getattr(wl.flow, "kind", None)
        if kind is None:
            raise VFPError("flow callable has no .kind (uniform or planar_x)")
        if kind[0] == "uniform":
            _check(lib.vfp_set_flow_uniform(ctx, _dptr(_f64(kind[1]))))
        elif kind[0] == "planar_x":
            xv = self.points(PTS_VOLUME, 0)
            xf = self.points(PTS_FACE, 0)

            def sample(x):
                X = np.zeros((3, x.shape[0]))
                X[0] = x
                U, dU, a = wl.flow(X)
                return _f64(U[0]), _f64(dU[0, 0]), _f64(a[0])
            u, du, a = sample(xv)
            uf = sample(xf)[0]
            _check(lib.vfp_set_flow_planar(ctx, _dptr(u), _dptr(du), _dptr(a), _dptr(uf)))
        elif kind[0] == "points":
            X, _ = self.volume_points()
            U, dU, _ = wl.flow(X)
            Up = _f64(U.T)                                   # [cell*q][3]
            G = _f64(np.transpose(dU, (2, 0, 1)))            # [cell*q][a][b]
            self._uface = []
            for a in range(len(wl.axes)):
                Uf, _, _ = wl.flow(self.face_points(a))
                self._uface.append(_f64(Uf.T))
            fp = (C.POINTER(C.c_double) * len(self._uface))(*[_dptr(x) for x in self._uface])
            _check(lib.vfp_set_flow_points(ctx, _dptr(Up), _dptr(G), fp))
        else:
            raise VFPError(f"flow kind {kind}")
        if wl.magnetic is not None:
            mk = getattr(wl.magnetic, "kind", ("points",))
            if mk[0] == "uniform":
                _check(lib.vfp_set_magnetic_uniform(ctx, _dptr(_f64(mk[1]))))
            else:
                X, _ = self.volume_points()
                B = _f64(wl.magnetic(X).T)          # [cell*q][3]
                _check(lib.vfp_set_magnetic_points(ctx, _dptr(B)))
        if callable(wl.nu):
            X, p = self.volume_points()
            _check(lib.vfp_set_scattering_points(ctx, _dptr(_f64(wl.nu(X, p)))))
        elif np.isscalar(wl.nu):
            _check(lib.vfp_set_scattering(ctx, float(wl.nu), None))
        else:
            nu = _f64(wl.nu)
            if nu.shape != (wl.ncells,):
                raise VFPError("nu must be a scalar or one value per cell")
            _check(lib.vfp_set_scattering(ctx, 0.0, _dptr(nu)))
        if wl.source is not None and "source" in wl.terms:
            X, p = self.volume_points()
            s = _f64(wl.source(X, p))
            _check(lib.vfp_set_source_points(ctx, _dptr(s)))

    def set_scattering(self, nu):
        if np.isscalar(nu):
            _check(_lib.vfp_set_scattering(self._ctx, float(nu), None))
        else:
            _check(_lib.vfp_set_scattering(self._ctx, 0.0, _dptr(_f64(nu))))

    # -- compute ------------------------------------------------------------
    def _t(self, x, name, size=None, optional=False):
        import torch
        if x is None and optional:
            return None
        size = self.ndofs if size is None else size
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64 \
                or not x.is_contiguous() or x.numel() < size:
            raise VFPError(f"{name} must be a contiguous float64 CUDA tensor of >= {size} elements")
        return C.c_void_p(x.data_ptr())

    def autotune(self, u, work, reps=5, stream=None):
        """Time the stage kernel's launch shapes (vfp_autotune) and keep the
        fastest; returns {"shape", "lanes", "tile_map"}."""
        ch = (C.c_int * 3)()
        _check(_lib.vfp_autotune(self._ctx, self._t(u, "u"), self._t(work, "work"), int(reps), ch,
                                 _stream_handle(stream)))
        return {"shape": ch[0], "lanes": ch[1], "tile_map": ch[2]}

    def apply(self, zin, zout, with_source=True, stream=None):
        _check(_lib.vfp_apply(self._ctx, self._t(zin, "in"), self._t(zout, "out"),
                              int(bool(with_source)), _stream_handle(stream)))

    def stage(self, w_in, u, w_out, cdt, stream=None):
        _check(_lib.vfp_stage(self._ctx, self._t(w_in, "w_in"), self._t(u, "u"),
                              self._t(w_out, "w_out"), float(cdt), _stream_handle(stream)))

    def advance(self, u, dt, nsteps, work, stream=None):
        import torch
        if work.numel() < 2 * self.ndofs:
            raise VFPError("work needs 2*ndofs doubles")
        _check(_lib.vfp_advance(self._ctx, self._t(u, "u"), float(dt), int(nsteps),
                                self._t(work, "work"), _stream_handle(stream)))

    # -- adjoint ------------------------------------------------------------
    def mass(self, zin, zout, inverse=False, stream=None):
        _check(_lib.vfp_mass(self._ctx, self._t(zin, "in"), self._t(zout, "out"), int(bool(inverse)),
                             _stream_handle(stream)))

    def apply_adjoint(self, zin, zout, work=None, stream=None):
        """zout = -D^T M^{-1} zin; work (ndofs doubles) is the call's scratch,
        taken from torch's allocator when not given."""
        import torch
        if work is None:
            work = torch.empty(self.ndofs, dtype=torch.float64, device=zin.device)
        _check(_lib.vfp_apply_adjoint(self._ctx, self._t(zin, "in"), self._t(zout, "out"),
                                      self._t(work, "work"), _stream_handle(stream)))

    def adjoint_stage(self, mu_in, acc_in, fwd, cdt, t_out, acc_out, grad_nu=None, stream=None):
        _check(_lib.vfp_adjoint_stage(
            self._ctx, self._t(mu_in, "mu_in"), self._t(acc_in, "acc_in"),
            self._t(fwd, "fwd", optional=True), float(cdt), self._t(t_out, "t_out", optional=True),
            self._t(acc_out, "acc_out"), self._t(grad_nu, "grad_nu", self.ncells, optional=True),
            _stream_handle(stream)))

    def advance_tape(self, u0, dt, nsteps, tape, stream=None):
        _check(_lib.vfp_advance_tape(self._ctx, self._t(u0, "u0"), float(dt), int(nsteps),
                                     self._t(tape, "tape", 4 * nsteps * self.ndofs),
                                     _stream_handle(stream)))

    def adjoint_steps(self, u0, tape, dt, nsteps, mu, grad_nu, work, field_slots=None, stream=None):
        _check(_lib.vfp_adjoint_steps(
            self._ctx, self._t(u0, "u0"), self._t(tape, "tape", 4 * nsteps * self.ndofs), float(dt),
            int(nsteps), self._t(mu, "mu"), self._t(grad_nu, "grad_nu", self.ncells, optional=True),
            self._slots(field_slots), self._t(work, "work", 3 * self.ndofs), _stream_handle(stream)))

    def forward_checkpoints(self, u, dt, nsteps, seg, ckpt, work, stream=None):
        nseg = -(-nsteps // seg)
        _check(_lib.vfp_forward_checkpoints(
            self._ctx, self._t(u, "u"), float(dt), int(nsteps), int(seg),
            self._t(ckpt, "ckpt", nseg * self.ndofs), self._t(work, "work", 2 * self.ndofs),
            _stream_handle(stream)))

    def adjoint_checkpointed(self, ckpt, dt, nsteps, seg, tape, lam, grad_nu, work, field_slots=None,
                             stream=None):
        nseg = -(-nsteps // seg)
        _check(_lib.vfp_adjoint_checkpointed(
            self._ctx, self._t(ckpt, "ckpt", nseg * self.ndofs), float(dt), int(nsteps), int(seg),
            self._t(tape, "tape", 4 * min(seg, nsteps) * self.ndofs), self._t(lam, "lam"),
            self._t(grad_nu, "grad_nu", self.ncells, optional=True),
            self._slots(field_slots), self._t(work, "work", 3 * self.ndofs), _stream_handle(stream)))

    def _slots(self, slots):
        return None if slots is None else self._t(slots, "field_slots", self.field_grad_size())

    def field_grad_size(self):
        n = C.c_int64()
        _check(_lib.vfp_field_grad_size(self._ctx, C.byref(n)))
        return n.value

    def field_grad_stage(self, mu, fwd, cdt, slots, stream=None):
        _check(_lib.vfp_field_grad_stage(self._ctx, self._t(mu, "mu"), self._t(fwd, "fwd"), float(cdt),
                                         self._t(slots, "slots", self.field_grad_size()),
                                         _stream_handle(stream)))

    def field_grad_reduce(self, slots, g_u, g_dudx, g_dudt, g_uface, stream=None):
        nq = self.wl.ncells_axis[0] * (self.wl.k + 1)
        _check(_lib.vfp_field_grad_reduce(
            self._ctx, self._t(slots, "slots", self.field_grad_size()), self._t(g_u, "g_u", nq),
            self._t(g_dudx, "g_dudx", nq), self._t(g_dudt, "g_dudt", nq),
            self._t(g_uface, "g_uface", self.wl.ncells_axis[0] + 1), _stream_handle(stream)))

    def reconstruct(self, zeta, Y, out, stream=None):
        """out[row, d] = sum_lms zeta[row, lms] Y[d, lms] at every basis node
        (vfp_reconstruct); Y: device table (ndir, n), e.g. from sh_eval."""
        if Y.numel() == 0 or Y.numel() % self.wl.n_lms:
            raise VFPError(f"Y must hold ndir x {self.wl.n_lms} values")
        ndir = Y.numel() // self.wl.n_lms
        rows = self.ndofs // self.wl.n_lms
        _check(_lib.vfp_reconstruct(self._ctx, self._t(zeta, "zeta"), self._t(Y, "Y", ndir * self.wl.n_lms),
                                    int(ndir), self._t(out, "out", rows * ndir), _stream_handle(stream)))

    def theta_work_size(self, restart=30):
        n = C.c_int64()
        _check(_lib.vfp_theta_work_size(self._ctx, int(restart), C.byref(n)))
        return n.value

    def theta_precond_size(self, precond):
        n = C.c_int64()
        pc = {None: 0, "none": 0, "collision": 1, "xline": 2}.get(precond, precond)
        _check(_lib.vfp_theta_precond_size(self._ctx, int(pc), C.byref(n)))
        return n.value

    def theta_advance(self, u, dt, nsteps, theta=0.5, tol=1e-12, restart=30, max_iters=1000, work=None,
                      precond=None, stream=None):
        """nsteps Theta-method steps in place on u (vfp_theta_advance);
        returns {"iterations", "residual", "converged"}.  work: device
        tensor of >= theta_work_size(restart) + theta_precond_size(precond)
        doubles (allocated if None); precond: None, "collision"
        (VFP_PRECOND_COLLISION) or "xline" (VFP_PRECOND_XLINE)."""
        import torch
        pc = {None: 0, "none": 0, "collision": 1, "xline": 2}.get(precond, precond)
        need = self.theta_work_size(restart) + self.theta_precond_size(pc)
        if work is None:
            work = torch.empty(need, dtype=torch.float64, device=u.device)
        opts = ThetaOpts(float(theta), float(tol), int(restart), int(max_iters), int(pc))
        st = ThetaStats()
        _check(_lib.vfp_theta_advance(self._ctx, self._t(u, "u"), float(dt), int(nsteps), C.byref(opts),
                                      self._t(work, "work", need), int(work.numel()), C.byref(st),
                                      _stream_handle(stream)))
        return {"iterations": int(st.iterations), "residual": float(st.residual), "converged": bool(st.converged)}

    def field_grad_support(self, xcells=None):
        """Form the U' and dU/dt sensitivities only on the x cells marked
        True (vfp_field_grad_support); None: everywhere."""
        if xcells is None:
            _check(_lib.vfp_field_grad_support(self._ctx, None))
            return
        m = np.ascontiguousarray(np.asarray(xcells, dtype=bool).astype(np.uint8))
        if m.size != self.wl.ncells_axis[0]:
            raise VFPError("one flag per x cell")
        _check(_lib.vfp_field_grad_support(self._ctx, m.ctypes.data_as(C.POINTER(C.c_ubyte))))

    def set_flow_planar(self, u, dudx, dudt, u_face):
        """Replace the planar flow profile (host arrays at the x Gauss points
        and x faces)."""
        _check(_lib.vfp_set_flow_planar(self._ctx, _dptr(_f64(u)), _dptr(_f64(dudx)), _dptr(_f64(dudt)),
                                        _dptr(_f64(u_face))))

    @property
    def ncells(self):
        return self.wl.ncells

    def cfl_dt(self, courant=None):
        c = self.wl.courant if courant is None else courant
        dt = C.c_double()
        _check(_lib.vfp_cfl_dt(self._ctx, float(c), C.byref(dt)))
        return dt.value

    def close(self):
        if self._ctx:
            _lib.vfp_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many runs advanced together (vfp_batch_*): one launch per stage and
    (k, l_max) class walks the tiles of all runs of that class."""

    def __init__(self, ops, graph=True):
        lib = load()
        self.ops = list(ops)
        arr = (C.c_void_p * len(self.ops))(*[op._ctx.value for op in self.ops])
        self._b = C.c_void_p()
        _check(lib.vfp_batch_create(C.byref(self._b), arr, len(self.ops), 1 if graph else 0))

    def bind(self, u, work, dt):
        """u[r], work[r]: float64 CUDA tensors (ndofs, 2 ndofs); dt[r]."""
        n = len(self.ops)
        up = (C.c_void_p * n)(*[op._t(x, "u").value for op, x in zip(self.ops, u)])
        wp = (C.c_void_p * n)(*[op._t(x, "work", 2 * op.ndofs).value for op, x in zip(self.ops, work)])
        dts = _f64([float(d) for d in dt])
        self._keep = (list(u), list(work))
        _check(_lib.vfp_batch_bind(self._b, up, wp, _dptr(dts)))

    def advance(self, nsteps, stream=None):
        _check(_lib.vfp_batch_advance(self._b, int(nsteps), _stream_handle(stream)))

    def autotune(self, reps=3, stream=None):
        _check(_lib.vfp_batch_autotune(self._b, int(reps), _stream_handle(stream)))

    def classes(self):
        out = []
        for i in range(_lib.vfp_batch_nclasses(self._b)):
            info = (C.c_int * 8)()
            _check(_lib.vfp_batch_class_info(self._b, i, info))
            out.append(dict(zip(("k", "lmax", "nrot", "runs", "batched", "tiles", "lanes", "tile_map"),
                                list(info))))
        return out

    def close(self):
        if self._b:
            _lib.vfp_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sh_eval(lmax: int, theta, phi):
    """Y[d, lms] = Y_lms(theta[d], phi[d]) from the library's host routine
    (vfp_sh_eval), as a numpy array (ndir, (lmax+1)^2)."""
    import numpy as np
    load()
    th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    ph = np.ascontiguousarray(phi, dtype=np.float64).ravel()
    if th.shape != ph.shape:
        raise VFPError("theta and phi must have the same length")
    Y = np.zeros((th.size, (lmax + 1) ** 2))
    _check(_lib.vfp_sh_eval(int(lmax), th.size, _dptr(th), _dptr(ph), _dptr(Y)))
    return Y


def checkpoint_segment(nsteps: int) -> int:
    """Segment length for sqrt(N) checkpointing."""
    return max(1, int(math.ceil(math.sqrt(max(nsteps, 1)))))


def grad_segment(op: "Operator", nsteps: int, device=None, reserve: int = 16 << 30) -> int:
    """Steps per checkpoint segment for a reverse pass on `device`: the whole
    stage tape (nsteps, no replay) when its 4 nsteps + 1 state vectors fit in
    the device's free memory with `reserve` bytes to spare, else sqrt(N)
    checkpointing (one replay of the forward run)."""
    import torch
    need = (4 * max(nsteps, 1) + 1) * op.ndofs * 8
    free, _ = torch.cuda.mem_get_info(device)
    # memory torch's caching allocator holds but does not use is free to it
    free += torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)
    return max(nsteps, 1) if need + reserve <= free else checkpoint_segment(nsteps)


class _AdvanceFn:
    """Namespace for the autograd function (built lazily so that importing
    this module does not need torch)."""
    fn = None


def planar_shock_fields(op: "Operator", U0, r, w):
    """The tanh shock U(x) = U0[(r+1)/2 - (r-1)/2 tanh(x/w)] (U0 the
    downstream speed) at the library's x Gauss points and x faces, as
    differentiable torch tensors (u, dU/dx, dU/dt = U dU/dx, u_face) of the
    parameters (torch scalars on the GPU)."""
    import torch
    xv = torch.from_numpy(op.points(PTS_VOLUME, 0)).to(U0.device)
    xf = torch.from_numpy(op.points(PTS_FACE, 0)).to(U0.device)

    def prof(x):
        t = torch.tanh(x / w)
        U = U0 * ((r + 1) / 2 - (r - 1) / 2 * t)
        dU = -U0 * (r - 1) / (2 * w) * (1 - t * t)
        return U, dU
    u, du = prof(xv)
    uf, _ = prof(xf)
    return u, du, u * du, uf


def planar_shock_support(op: "Operator", w):
    """x cells where the tanh shock of width w has a gradient at one of its
    Gauss points with a wide margin (|x| < 25 w; beyond ~19 w, 1 - tanh^2
    rounds to 0 in double precision, and with it U', U U' and all their
    derivatives in the profile's parameters): the support for
    field_grad_support."""
    K1 = op.wl.k + 1
    xv = op.points(PTS_VOLUME, 0).reshape(-1, K1)
    return np.any(np.abs(xv) < 25.0 * float(w), axis=1)


def advance_with_grad(op: "Operator", u0, nu_cell, dt: float, nsteps: int, seg: int = None, flow=None,
                      flow_support=None):
    """u_N = RK4^N(u0) with the scattering frequency nu_cell (one value per
    cell) and, optionally, the planar flow flow = (u, dudx, dudt, u_face) as
    differentiable inputs: backward returns their gradients from the discrete
    adjoint of the library (the flow sensitivities from vfp_field_grad_*).
    flow_support: optional flags per x cell (vfp_field_grad_support) where
    the flow's parameters move U' and dU/dt (planar_shock_support for the
    tanh shock); the other cells skip those sensitivities.
    seg: steps per checkpoint segment; with seg >= nsteps the forward keeps
    the whole stage tape (4 nsteps vectors) and the reverse pass replays
    nothing.  Default: the whole tape when it fits in free device memory,
    else ceil(sqrt(nsteps)) (grad_segment)."""
    import torch
    if _AdvanceFn.fn is None:
        class AdvanceFn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, u0, nu, u_q, du_q, a_q, u_f, op, dt, nsteps, seg, has_flow, support):
                if has_flow:
                    op.set_flow_planar(*(t.detach().cpu().numpy() for t in (u_q, du_q, a_q, u_f)))
                op.set_scattering(nu.detach().cpu().numpy())
                N = op.ndofs
                u = u0.detach().clone().contiguous()
                if seg >= nsteps and nsteps > 0:
                    # whole stage tape: slot 4 nsteps - 1 is the final state
                    ckpt = torch.empty((4 * nsteps + 1) * N, dtype=torch.float64, device=u.device)
                    ckpt[:N].copy_(u)
                    op.advance_tape(ckpt[:N], dt, nsteps, ckpt[N:])
                    u = ckpt[4 * nsteps * N:].clone()
                else:
                    nseg = -(-nsteps // seg)
                    ckpt = torch.empty(max(nseg, 1) * N, dtype=torch.float64, device=u.device)
                    work = torch.empty(2 * N, dtype=torch.float64, device=u.device)
                    op.forward_checkpoints(u, dt, nsteps, seg, ckpt, work)
                ctx.op, ctx.dt, ctx.nsteps, ctx.seg, ctx.has_flow = op, dt, nsteps, seg, has_flow
                ctx.support = support
                ctx.nu = nu.detach().cpu().numpy().copy()
                ctx.flow = tuple(t.detach().cpu().numpy().copy() for t in (u_q, du_q, a_q, u_f)) \
                    if has_flow else None
                ctx.save_for_backward(ckpt)
                return u

            @staticmethod
            def backward(ctx, g):
                (ckpt,) = ctx.saved_tensors
                op, N = ctx.op, ctx.op.ndofs
                if ctx.has_flow:
                    op.set_flow_planar(*ctx.flow)
                    op.field_grad_support(ctx.support)
                op.set_scattering(ctx.nu)
                dev = g.device
                lam = g.detach().to(torch.float64).contiguous().clone()
                grad_nu = torch.zeros(op.ncells, dtype=torch.float64, device=dev)
                slots = torch.zeros(op.field_grad_size(), dtype=torch.float64, device=dev) \
                    if ctx.has_flow else None
                if ctx.nsteps > 0 and ctx.seg >= ctx.nsteps:
                    work = torch.empty(3 * N, dtype=torch.float64, device=dev)
                    op.mass(lam, lam, inverse=True)
                    op.adjoint_steps(ckpt[:N], ckpt[N:], ctx.dt, ctx.nsteps, lam, grad_nu, work,
                                     field_slots=slots)
                    op.mass(lam, lam, inverse=False)
                elif ctx.nsteps > 0:
                    tape = torch.empty(4 * min(ctx.seg, ctx.nsteps) * N, dtype=torch.float64, device=dev)
                    work = torch.empty(3 * N, dtype=torch.float64, device=dev)
                    op.adjoint_checkpointed(ckpt, ctx.dt, ctx.nsteps, ctx.seg, tape, lam, grad_nu, work,
                                            field_slots=slots)
                gf = (None, None, None, None)
                if ctx.has_flow:
                    nq = op.wl.ncells_axis[0] * (op.wl.k + 1)
                    gu, gd, ga = (torch.empty(nq, dtype=torch.float64, device=dev) for _ in range(3))
                    gfc = torch.empty(op.wl.ncells_axis[0] + 1, dtype=torch.float64, device=dev)
                    op.field_grad_reduce(slots, gu, gd, ga, gfc)
                    gf = (gu, gd, ga, gfc)
                return (lam, grad_nu) + gf + (None, None, None, None, None, None)
        _AdvanceFn.fn = AdvanceFn
    import torch as _t
    seg = grad_segment(op, nsteps, u0.device) if seg is None else int(seg)
    if flow is None:
        z = _t.zeros(1, dtype=_t.float64, device=u0.device)
        return _AdvanceFn.fn.apply(u0, nu_cell, z, z, z, z, op, float(dt), int(nsteps), seg, False, None)
    return _AdvanceFn.fn.apply(u0, nu_cell, *flow, op, float(dt), int(nsteps), seg, True, flow_support)

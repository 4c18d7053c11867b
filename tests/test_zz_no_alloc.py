"""vfp_apply_adjoint_noalloc (the allocation-free form of vfp_apply_adjoint
for callers that cannot allocate device memory) against vfp_apply_adjoint
with a caller work vector: same kernels, so the results must agree to the
bit.  Two calls in a row share the library's scratch array, the second on a
smaller problem; a problem above the array's size is refused before any
launch."""

import ctypes as C

import numpy as np
import pytest

from paper_2501_05110_amd import workloads as W

from gpu_cases import _say, shock

pytestmark = pytest.mark.gpu


def _noalloc(lib, op, zin, zout):
    import torch
    fn = lib.vfp_apply_adjoint_noalloc
    fn.restype = C.c_int
    fn.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    return fn(op._ctx, C.c_void_p(zin.data_ptr()), C.c_void_p(zout.data_ptr()),
              C.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_apply_adjoint(lib, cuda):
    import torch
    from paper_2501_05110_amd.vfp import Operator
    for wl in (shock(25, 11, 2, 3), shock(12, 5, 1, 5, seed=3)):
        _say(f"[noalloc] {wl.name}: ndofs={wl.ndofs}")
        op = Operator(wl)
        lam = torch.from_numpy(W.random_state(wl, 77).ravel().copy()).cuda()
        want = torch.empty_like(lam)
        work = torch.empty_like(lam)
        op.apply_adjoint(lam, want, work=work)
        got = torch.full_like(lam, float("nan"))
        assert _noalloc(lib, op, lam, got) == 0, lib.vfp_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert torch.isfinite(got).all()
        op.close()


def test_noalloc_refuses_above_limit(lib, cuda):
    import torch
    from paper_2501_05110_amd.vfp import Operator
    wl = shock(1024, 64, 2, 3)           # 9,437,184 DoF > 8,388,608
    _say(f"[noalloc] limit: ndofs={wl.ndofs}")
    op = Operator(wl)
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = _noalloc(lib, op, z, z)
    assert rc == -1
    assert b"allocation-free limit" in lib.vfp_last_error()
    op.close()

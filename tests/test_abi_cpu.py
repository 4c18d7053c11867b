"""Host-side checks of the C ABI that need no GPU: every function declared in
include/vfp.h is exported, and argument validation reports errors through
status codes and vfp_last_error()."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2501_05110_amd import vfp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vfp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vfp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_functions(lib):
    assert sorted(vfp.exported_symbols()) == declared_functions()


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _create(lib, lmax=3, k=2, axes=(0, 3), mask=31, mass=1.0, charge=1.0):
    ctx = C.c_void_p()
    kinds = (C.c_int * len(axes))(*axes)
    rc = lib.vfp_create(C.byref(ctx), lmax, k, len(axes), kinds, mask, mass, charge)
    return rc, ctx


@pytest.mark.parametrize("kw,needle", [
    (dict(lmax=0), "lmax"), (dict(lmax=12), "lmax"), (dict(k=0), "k="), (dict(k=6), "k="),
    (dict(axes=()), "naxes"), (dict(axes=(0, 1, 2, 3)), "naxes"), (dict(axes=(3, 0)), "ln p"),
    (dict(axes=(1,)), "x, y, z"), (dict(axes=(0, 1, 2, 3)[:3] + ()), None),
    (dict(mass=0.0), "mass"), (dict(mask=64), "term"), (dict(axes=(3,)), "spatial"),
])
def test_create_validation(lib, kw, needle):
    rc, ctx = _create(lib, **kw)
    if needle is None:
        assert rc == 0
        lib.vfp_destroy(ctx)
        return
    assert rc == -1
    assert needle in lib.vfp_last_error().decode()


@pytest.mark.parametrize("lmax,k,axes,rc_want", [
    (11, 2, (0,), 0), (8, 1, (0,), 0), (9, 2, (0, 1), -5), (11, 2, (0, 3), -5), (9, 3, (0,), -5)])
def test_create_high_lmax_scope(lib, lmax, k, axes, rc_want):
    """l_max 8..11: one spatial axis x at fixed p with k <= 2 (VFP_EUNSUPPORTED
    otherwise)."""
    rc, ctx = _create(lib, lmax=lmax, k=k, axes=axes)
    assert rc == rc_want, lib.vfp_last_error().decode()
    if rc == 0:
        lib.vfp_destroy(ctx)


@pytest.mark.parametrize("k,axes,rc_want", [
    (5, (0,), 0), (3, (0, 3), 0), (3, (0, 1), 0), (4, (0, 3), -5), (3, (0, 1, 2), -5), (2, (0, 1, 2), 0)])
def test_create_degree_per_axes(lib, k, axes, rc_want):
    """k <= 5 on one axis, 3 on two, 2 on three (VFP_EUNSUPPORTED beyond)."""
    rc, ctx = _create(lib, k=k, axes=axes)
    assert rc == rc_want, lib.vfp_last_error().decode()
    if rc == 0:
        lib.vfp_destroy(ctx)


def test_calls_out_of_order(lib):
    rc, ctx = _create(lib)
    assert rc == 0
    U = (C.c_double * 3)(0.1, 0, 0)
    assert lib.vfp_set_flow_uniform(ctx, U) == -4
    assert "set_mesh" in lib.vfp_last_error().decode()
    n = C.c_int64()
    assert lib.vfp_ndofs(ctx, C.byref(n)) == -4
    assert lib.vfp_apply(ctx, None, None, 1, None) == -4
    # every compute call checks the state first
    assert lib.vfp_apply_adjoint(ctx, None, None, None, None) == -4
    assert lib.vfp_mass(ctx, None, None, 1, None) == -4
    assert lib.vfp_adjoint_stage(ctx, None, None, None, 0.1, None, None, None, None) == -4
    assert lib.vfp_advance_tape(ctx, None, 0.1, 1, None, None) == -4
    assert lib.vfp_adjoint_steps(ctx, None, None, 0.1, 1, None, None, None, None, None) == -4
    assert lib.vfp_forward_checkpoints(ctx, None, 0.1, 1, 1, None, None, None) == -4
    assert lib.vfp_adjoint_checkpointed(ctx, None, 0.1, 1, 1, None, None, None, None, None, None) == -4
    ns = C.c_int64()
    assert lib.vfp_field_grad_size(ctx, C.byref(ns)) == -4
    assert lib.vfp_field_grad_stage(ctx, None, None, 0.1, None, None) == -4
    assert lib.vfp_field_grad_reduce(ctx, None, None, None, None, None, None) == -4
    # a batch needs ready contexts
    b = C.c_void_p()
    arr = (C.c_void_p * 1)(ctx.value)
    assert lib.vfp_batch_create(C.byref(b), arr, 1, 0) == -4
    assert lib.vfp_batch_create(C.byref(b), arr, 0, 0) == -1
    assert lib.vfp_batch_create(C.byref(b), arr, 1, 8) == -1
    assert lib.vfp_batch_create(None, arr, 1, 0) == -1
    assert lib.vfp_batch_advance(None, 1, None) == -1
    assert lib.vfp_batch_nclasses(None) == 0
    lib.vfp_batch_destroy(None)
    assert lib.vfp_set_momentum(ctx, 1.0) == -1       # ln p axis: momentum is a coordinate
    lib.vfp_destroy(ctx)
    lib.vfp_destroy(None)


def test_mesh_validation_and_points(lib):
    rc, ctx = _create(lib, lmax=1, k=2, axes=(0,))
    assert rc == 0
    bad = np.array([0.0, 1.0, 0.5])
    arr = (C.POINTER(C.c_double) * 1)(bad.ctypes.data_as(C.POINTER(C.c_double)))
    nc = (C.c_int * 1)(2)
    per = (C.c_int * 1)(0)
    zin = (C.c_int * 1)(1)
    assert lib.vfp_set_mesh(ctx, nc, arr, per, per) == -1
    assert "increasing" in lib.vfp_last_error().decode()
    good = np.array([0.0, 1.0, 3.0])
    arr = (C.POINTER(C.c_double) * 1)(good.ctypes.data_as(C.POINTER(C.c_double)))
    assert lib.vfp_set_mesh(ctx, nc, arr, per, zin) == -1      # periodic on one end only
    rc = lib.vfp_set_mesh(ctx, nc, arr, zin, zin)
    assert rc in (0, -3)          # -3 (EDEVICE) on a machine without a GPU
    n = C.c_int64()
    assert lib.vfp_ndofs(ctx, C.byref(n)) == 0 and n.value == 2 * 3 * 4
    cnt = C.c_int64()
    assert lib.vfp_query_points(ctx, 0, 0, None, C.byref(cnt)) == 0 and cnt.value == 6
    pts = np.zeros(6)
    assert lib.vfp_query_points(ctx, 0, 0, pts.ctypes.data_as(C.POINTER(C.c_double)), C.byref(cnt)) == 0
    g = np.sqrt(0.6)
    want = np.concatenate([0.5 + 0.5 * np.array([-g, 0, g]), 2.0 + np.array([-g, 0, g])])
    np.testing.assert_allclose(pts, want, atol=1e-15)
    assert lib.vfp_query_points(ctx, 1, 0, pts.ctypes.data_as(C.POINTER(C.c_double)), C.byref(cnt)) == 0
    np.testing.assert_allclose(pts[:3], good)
    assert lib.vfp_query_points(ctx, 0, 1, None, C.byref(cnt)) == -1
    lib.vfp_destroy(ctx)

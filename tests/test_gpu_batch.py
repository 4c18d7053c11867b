"""Batched runs: every run of a batch must equal the same run advanced alone
(bit for bit: the arithmetic per cell is the same, only the launch differs),
with and without the captured graph and after autotuning; sampled runs also
match the oracle after many steps."""

import numpy as np
import pytest

from oracle import dg
from paper_2501_05110_amd import workloads as W

from gpu_cases import STEPS_TOL, _say, planar1d, rel_inf, shock, uniform2d

pytestmark = pytest.mark.gpu


def _runs():
    g = np.random.default_rng(77)
    wls = []
    for i, (k, lmax) in enumerate([(2, 3), (2, 3), (1, 1), (2, 1), (1, 3), (2, 5), (1, 7), (2, 3),
                                   (1, 1), (2, 7)]):
        nx = int(g.integers(5, 40))
        np_ = int(g.integers(3, 12))
        wls.append(W.shock_workload(f"b{i}", nx, np_, k, lmax, r=float(g.uniform(2, 4)),
                                    nu0=float(np.exp(g.uniform(-2, 2))), seed=10 + i))
    wls.append(uniform2d())          # not an (x, ln p) run: launched one by one
    wls.append(planar1d())
    return wls


def _setup(wls):
    import torch
    from paper_2501_05110_amd.vfp import Operator
    ops = [Operator(wl) for wl in wls]
    z0 = [np.random.default_rng(100 + i).standard_normal(op.ndofs) for i, op in enumerate(ops)]
    dts = [op.cfl_dt(0.2) * (0.9 + 0.01 * i) for i, op in enumerate(ops)]
    u = [torch.from_numpy(z).cuda() for z in z0]
    work = [torch.empty(2 * op.ndofs, dtype=torch.float64, device="cuda") for op in ops]
    return ops, z0, dts, u, work


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_runs(lib, cuda, graph):
    import torch
    from paper_2501_05110_amd.vfp import Batch
    wls = _runs()
    ops, z0, dts, u, work = _setup(wls)
    b = Batch(ops, graph=graph)
    b.bind(u, work, dts)
    cls = b.classes()
    _say(f"[batch] graph={graph} classes={cls}")
    assert sum(c["runs"] for c in cls) == len(ops)
    assert any(c["batched"] and c["runs"] > 1 for c in cls)
    b.advance(7)
    b.advance(5)
    b.autotune(reps=2)
    _say(f"   tuned: {b.classes()}")
    b.advance(6)
    torch.cuda.synchronize()
    for i, op in enumerate(ops):
        ref = torch.from_numpy(z0[i]).cuda()
        wk = torch.empty(2 * op.ndofs, dtype=torch.float64, device="cuda")
        op.advance(ref, dts[i], 18, wk)
        torch.cuda.synchronize()
        same = torch.equal(ref, u[i])
        if not same:
            _say(f"   run {i} ({wls[i].name}) max diff {float((ref - u[i]).abs().max()):.3e}")
        assert same, i
    b.close()


def test_batch_sample_matches_oracle(lib, cuda):
    """Two runs of a batch, 200 steps, against the oracle's classical RK4."""
    import torch
    from paper_2501_05110_amd.vfp import Batch
    wls = [shock(14, 6, 2, 3, seed=3), shock(11, 5, 1, 5, seed=4), shock(9, 7, 2, 3, seed=5)]
    ops, z0, dts, u, work = _setup(wls)
    b = Batch(ops)
    b.bind(u, work, dts)
    n = 200
    b.advance(n)
    torch.cuda.synchronize()
    for i in (0, 1):
        want = dg.rk4(dg.assemble(wls[i]), z0[i], dts[i], n)
        err = rel_inf(u[i].cpu().numpy(), want)
        _say(f"[batch oracle] run {i}: rel_inf={err:.3e}")
        assert err <= STEPS_TOL
    b.close()


def test_batch_refuses_runs_set_up_after_bind(lib, cuda):
    """The stage descriptors copy each run's field pointers and values when
    the batch is bound; a set-up call on a run afterwards (which may free
    and reallocate those fields) makes advance and autotune refuse to launch
    until the batch is bound again."""
    import torch
    from paper_2501_05110_amd.vfp import Batch, VFPError
    wls = [shock(10, 4, 2, 3, seed=3), shock(9, 5, 1, 1, seed=4)]
    ops, z0, dts, u, work = _setup(wls)
    b = Batch(ops)
    b.bind(u, work, dts)
    b.advance(1)
    ops[1].set_scattering(np.full(wls[1].ncells, 2.0))   # reallocates nu per cell
    before = [x.clone() for x in u]
    with pytest.raises(VFPError, match="bind again"):
        b.advance(1)
    with pytest.raises(VFPError, match="bind again"):
        b.autotune(reps=1)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(u, before))
    b.bind(u, work, dts)
    b.advance(1)
    torch.cuda.synchronize()
    b.close()


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("case", [(40, 9, 2, 3), (21, 7, 1, 5), (13, 6, 2, 1), (9, 5, 2, 7)])
def test_workgroup_shapes_agree(lib, cuda, shape, case, monkeypatch):
    """The (x, ln p) stage kernel in each workgroup shape (cells per tile,
    lanes per workgroup) gives the default shape's results bit for bit
    (apply and 20 steps); vfp_autotune keeps them too."""
    import torch
    from paper_2501_05110_amd.vfp import Operator
    wl = shock(*case, seed=6)
    z = torch.from_numpy(np.random.default_rng(3).standard_normal(wl.ndofs)).cuda()
    outs = []
    for sh in (0, shape):
        monkeypatch.setenv("VFP_SHOCK_SHAPE", str(sh))
        op = Operator(wl)
        a = torch.empty_like(z)
        op.apply(z, a)
        u = z.clone()
        work = torch.empty(2 * wl.ndofs, dtype=torch.float64, device="cuda")
        op.advance(u, op.cfl_dt(0.2), 20, work)
        torch.cuda.synchronize()
        outs.append((a, u))
        if sh == shape:
            chosen = op.autotune(z, work[:wl.ndofs], reps=2)
            _say(f"[shapes] {case} shape {shape}: autotune chose {chosen}")
            b = torch.empty_like(z)
            op.apply(z, b)
            torch.cuda.synchronize()
            assert torch.equal(a, b)
        op.close()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])

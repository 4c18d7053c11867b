"""Benchmark: explicit time stepping of the DG x spherical-harmonic operator.

Workload: the 2-D (x, ln p) parallel shock -- 1024 x 128 cells, DG degree 2,
l_max = 3 (18,874,368 FP64 degrees of freedom), tanh flow profile with r = 4,
B along x, nu ~ p^(-1/3) per cell, Gaussian injection -- advanced with the
four-stage fourth-order Runge-Kutta scheme at Courant number 0.2.  A step is
one full Runge-Kutta step (four fused stage launches over all cells).

Prints one JSON line: DoF-updates/s over the timed steps, the stage kernel's
HBM roofline fraction (algorithmic bytes / measured launch time, against
8 TB/s), and the CPU oracle's rate on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--warmup-seconds S] [--gpus 1] [--no-cpu] [--no-adjoint]
                  [--no-batch] [--no-other] [--no-theta] [--batch-small] [--copy-probe]

It also reports the adjoint: a 1000-step forward run of the 512 x 64 shock
and its reverse pass (gradients w.r.t. the initial state and nu per cell,
and with the flow sensitivities for the shock profile), from sqrt(N)
checkpoints and from the whole stage tape (151 GB here; the default where
it fits), with the reverse / forward time ratios, and the batched path:
256 shock runs of 128-1024 x 32-128 cells, mixed k and l_max, advanced by
one launch per stage and class (workgroup shape and tile order autotuned
per class) against one run per launch sequence on the same GPU
(--batch-small: 512 small runs), and the stage throughput of the 3-D box
(48^3, k=2, l_max=5) and the 1-D line (64 cells, k=1, l_max=3), and
Theta-method steps (Crank-Nicolson, backward Euler) of the 512 x 64 shock at
10 times the explicit time step and the Sec. 4.4 run on its 410 x 256 grid
by implicit steps with the x-line preconditioner, and (with the other
configurations) the reconstruction of f in 64 directions, a k = 5 line, the
shock on a linear p axis and the 1024 x 128 stage with a shock wide enough
that the flow gradient is nonzero on every x column.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_shock_kernel_shock2d_1024x128.json")


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    passes (scaled by a plain copy's counts), or None when the kernel sources
    have changed since those counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(budget_s=12.0):
    """The oracle (assembled CSR + classical RK4) on a reduced grid with the
    same per-cell structure: 64 x 8 cells of the same shock, k=2, l_max=3.
    SciPy's CSR product runs on one thread."""
    import numpy as np
    from oracle import dg
    from paper_2501_05110_amd import workloads as W

    wl = W.config2(nx=64, np_=8)
    t0 = time.perf_counter()
    S = dg.assemble(wl)
    t_asm = time.perf_counter() - t0
    z = wl.meta["init"].ravel().copy()
    # dt as the GPU run would use it on this grid is irrelevant for the rate
    dt = 1e-3
    steps = 0
    t0 = time.perf_counter()
    while True:
        z = dg.rk4(S, z, dt, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    rate = wl.ndofs * steps / el
    return {"value": rate, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"same shock on 64x8 cells ({wl.ndofs} DoF), {steps} classical RK4 steps "
                      f"in {el:.1f} s after {t_asm:.1f} s assembly; per-DoF rate of the "
                      f"1024x128 workload's structure",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def adjoint_timing(steps=1000):
    """Forward run and checkpointed reverse pass (dJ/du0 and dJ/dnu per cell)
    of the 512 x 64 shock, k=2, l_max=3; returns times and their ratio."""
    import numpy as np
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    wl = W.config5(steps=steps)
    op = vfp.Operator(wl)
    N = op.ndofs
    dt = op.cfl_dt(wl.courant)
    # the mode a reverse pass takes by default on this GPU (advance_with_grad)
    default_mode = "full_tape" if vfp.grad_segment(op, steps, torch.device("cuda:0")) >= steps else "checkpointed"
    seg = vfp.checkpoint_segment(steps)
    nseg = -(-steps // seg)
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(np.ascontiguousarray(wl.meta["init"]).ravel()).to(dev)
    work = torch.empty(3 * N, dtype=torch.float64, device=dev)
    ckpt = torch.empty(nseg * N, dtype=torch.float64, device=dev)
    tape = torch.empty(4 * seg * N, dtype=torch.float64, device=dev)
    gnu = torch.zeros(wl.ncells, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    u = u0.clone()
    op.advance(u, dt, 5, work)                       # warm-up
    u.copy_(u0)
    t_fwd = timed(lambda: op.advance(u, dt, steps, work))
    u.copy_(u0)
    t_ck = timed(lambda: op.forward_checkpoints(u, dt, steps, seg, ckpt, work))
    lam0 = torch.randn(N, dtype=torch.float64, device=dev,
                       generator=torch.Generator(device=dev).manual_seed(5))
    lam = lam0.clone()
    t_rev = timed(lambda: op.adjoint_checkpointed(ckpt, dt, steps, seg, tape, lam, gnu, work))
    # the same with the flow sensitivities (for dJ/d(r, w)) and their reduction;
    # U' and dU/dt move with (r, w) only inside the shock (the support)
    op.field_grad_support(vfp.planar_shock_support(op, wl.meta["w"]))
    slots = torch.zeros(op.field_grad_size(), dtype=torch.float64, device=dev)
    nq = wl.ncells_axis[0] * (wl.k + 1)
    gf = [torch.empty(nq, dtype=torch.float64, device=dev) for _ in range(3)]
    gfc = torch.empty(wl.ncells_axis[0] + 1, dtype=torch.float64, device=dev)
    lam = lam0.clone()

    def full():
        op.adjoint_checkpointed(ckpt, dt, steps, seg, tape, lam, gnu, work, field_slots=slots)
        op.field_grad_reduce(slots, *gf, gfc)
    t_full = timed(full)
    if not (torch.isfinite(lam).all() and torch.isfinite(gnu).all() and torch.isfinite(slots).all()):
        raise RuntimeError("adjoint produced non-finite values")
    del tape, ckpt
    torch.cuda.empty_cache()
    # the same gradients from a full stage tape (4 vectors per step: 151 GB
    # here, within one MI355X's HBM): the forward writes every stage output
    # to its own slot (no extra traffic) and the reverse replays nothing
    taped = {}
    need = 4 * steps * N * 8
    free, _ = torch.cuda.mem_get_info()
    if need < free - (8 << 30):
        full_tape = torch.empty(4 * steps * N, dtype=torch.float64, device=dev)
        t_tf = timed(lambda: op.advance_tape(u0, dt, steps, full_tape))
        mu = lam0.clone()
        op.mass(mu, mu, inverse=True)
        t_tr = timed(lambda: op.adjoint_steps(u0, full_tape, dt, steps, mu, gnu, work))
        slots.zero_()
        mu = lam0.clone()
        op.mass(mu, mu, inverse=True)
        t_trf = timed(lambda: op.adjoint_steps(u0, full_tape, dt, steps, mu, gnu, work, field_slots=slots))
        del full_tape
        taped = {"tape_GB": need / 1e9, "forward_taped_s": t_tf, "reverse_s": t_tr, "reverse_with_flow_s": t_trf,
                 "reverse_over_forward": t_tr / t_fwd, "reverse_with_flow_over_forward": t_trf / t_fwd}
    if default_mode == "full_tape" and taped:
        dflt = {"mode": default_mode, "reverse_over_forward": taped["reverse_over_forward"],
                "reverse_with_flow_over_forward": taped["reverse_with_flow_over_forward"]}
    else:
        dflt = {"mode": "checkpointed", "reverse_over_forward": t_rev / t_fwd,
                "reverse_with_flow_over_forward": t_full / t_fwd}
    return {"workload": wl.name, "ndofs": N, "steps": steps, "segment": seg, "default": dflt,
            "forward_s": t_fwd, "forward_checkpointed_s": t_ck, "reverse_s": t_rev,
            "reverse_over_forward": t_rev / t_fwd,
            "reverse_with_flow_s": t_full, "reverse_with_flow_over_forward": t_full / t_fwd,
            "full_tape": taped,
            "note": "reverse = replay of each segment into a stage tape + adjoint stages with the "
                    "fused dJ/dnu accumulation (dJ/du0, dJ/dnu for 32768 cells); with_flow adds the "
                    "planar-flow sensitivities that give dJ/d(r, w), whose launches then also form dJ/dnu (the adjoint "
                    "stages skip the forward state)"}


def batch_timing(full=False, steps=None):
    """Many independent shock runs advanced by the batched path (one launch
    per stage and (k, l_max) class, graph replay, autotuned workgroup shape and
    tile order) and,
    on the same GPU and buffers, one run per launch sequence.  full: the 256
    runs of mixed size, k and l_max (about 2.3e9 DoF); else 512 small runs."""
    import numpy as np
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    wls = W.config4() if full else W.batch_small()
    steps = steps or (20 if full else 50)
    t0 = time.perf_counter()
    ops = [vfp.Operator(wl) for wl in wls]
    t_setup = time.perf_counter() - t0
    N = [op.ndofs for op in ops]
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(4)
    u = [torch.randn(n, dtype=torch.float64, device=dev, generator=gen) * 1e-3 for n in N]
    work = [torch.empty(2 * n, dtype=torch.float64, device=dev) for n in N]
    dts = [op.cfl_dt(0.2) for op in ops]
    b = vfp.Batch(ops, graph=True)
    b.bind(u, work, dts)
    b.autotune(reps=2)
    stream = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    b.advance(2)
    t_b = timed(lambda: b.advance(steps))

    def per_run():
        for i, op in enumerate(ops):
            op.advance(u[i], dts[i], steps, work[i])
    # the runs advanced alone get the same tuning: each run's own launch shape
    for i, op in enumerate(ops):
        op.autotune(u[i], work[i][:N[i]], reps=2)
        op.advance(u[i], dts[i], 2, work[i])
    t_s = timed(per_run)
    for x in u:
        if not torch.isfinite(x).all():
            raise RuntimeError("batched state is not finite")
    tot = sum(N)
    cls = b.classes()
    b.close()
    return {"workload": "batch_256_mixed" if full else "batch_512_small", "runs": len(ops), "ndofs": tot,
            "steps": steps, "batched_dofs_per_s": tot * steps / t_b, "per_run_dofs_per_s": tot * steps / t_s,
            "speedup": t_s / t_b, "setup_s": t_setup,
            "classes": [{k: c[k] for k in ("k", "lmax", "runs", "tiles", "lanes", "tile_map")} for c in cls],
            "note": "batched: one launch per stage and (k, l_max) class, graph replay, workgroup shape and tile "
                    "order tuned per class; alone: each run's stages launched in sequence, launch shape tuned "
                    "per run"}


def dsa_paper_timing():
    """The run of Sec. 4.4 on the paper's grid (410 x 256 cells, k = 1,
    1,679,360 DoF) by implicit steps with the x-line preconditioner: Crank-
    Nicolson with the paper's dt = 1 (20 steps from f = 0), and backward Euler
    with dt = 1e7 until the state is stationary (the steady state whose
    spectrum the paper reports; tests/test_gpu_dsa.py checks it against the
    oracle's)."""
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    wl = W.paper_dsa_workload()
    t0 = time.perf_counter()
    op = vfp.Operator(wl)
    t_setup = time.perf_counter() - t0
    N = op.ndofs
    work = torch.empty(op.theta_work_size(64) + op.theta_precond_size("xline"), dtype=torch.float64, device="cuda")
    u = torch.zeros(N, dtype=torch.float64, device="cuda")
    op.theta_advance(u, 1.0, 1, theta=0.5, tol=1e-10, restart=40, max_iters=400, work=work, precond="xline")
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cn = op.theta_advance(u, 1.0, 20, theta=0.5, tol=1e-10, restart=40, max_iters=400, work=work, precond="xline")
    torch.cuda.synchronize()
    t_cn = (time.perf_counter() - t0) / 20
    u.zero_()
    prev = u.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, steps = 0, 0
    for steps in range(1, 13):
        st = op.theta_advance(u, 1e7, 1, theta=1.0, tol=1e-11, restart=64, max_iters=3000, work=work,
                              precond="xline")
        its += st["iterations"]
        change = float((u - prev).abs().max() / u.abs().max())
        prev.copy_(u)
        if change == 0.0:
            break
    torch.cuda.synchronize()
    t_ss = time.perf_counter() - t0
    op.close()
    return {"workload": wl.name, "ndofs": N, "setup_s": t_setup,
            "crank_nicolson_dt1": {"s_per_step": t_cn, "iterations_per_step": cn["iterations"] / 20,
                                   "converged": cn["converged"]},
            "steady_state_backward_euler_dt1e7": {"steps": steps, "iterations": its, "s": t_ss,
                                                  "stationary": change == 0.0},
            "note": "x-line block-tridiagonal preconditioner (VFP_PRECOND_XLINE), GMRES restart 40/64, "
                    "tol 1e-10 / 1e-11"}


def extension_timing():
    """The rows beyond the explicit (x, ln p) path, each with its HBM roofline
    fraction (algorithmic bytes per launch / launch time / 8 TB/s):
    * reconstruction of f in 64 directions from the 1024 x 128 shock state
      (reads the state and the table, writes rows x 64 values);
    * a 1-D line at k = 5 (8192 cells, l_max = 7) and the 512 x 64 shock on a
      linear p axis (k = 2, l_max = 3), both on the general kernels: stage
      launches, 16 B/DoF for the first stage and 24 B/DoF for the others;
    * the 1024 x 128 shock with a width of 2.5 (w_frac 0.25) instead of 0.1,
      so that U' is nonzero on every x column and the stage kernel takes the
      momentum terms everywhere (with the benchmark's width it skips them on
      the columns where 1 - tanh^2(x/w) rounds to 0); its bytes per launch
      include the input fields as the benchmark line's do."""
    import math
    import numpy as np
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    out = {}
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    wl = W.config2(steps=1)
    op = vfp.Operator(wl)
    ndir = 64
    g = np.random.default_rng(11)
    th, ph = np.arccos(g.uniform(-1, 1, ndir)), g.uniform(0, 2 * math.pi, ndir)
    Y = torch.from_numpy(vfp.sh_eval(wl.lmax, th, ph)).cuda()
    z = torch.from_numpy(np.ascontiguousarray(wl.meta["init"]).ravel()).cuda()
    rows = op.ndofs // wl.n_lms
    f = torch.empty(rows * ndir, dtype=torch.float64, device="cuda")
    t = timed(lambda: op.reconstruct(z, Y, f), 20)
    bts = 8 * (op.ndofs + Y.numel() + rows * ndir)
    out["reconstruct_shock2d_1024x128_64dirs"] = {
        "us_per_launch": t * 1e6, "bytes_per_launch": bts, "achieved_GBs": bts / t / 1e9,
        "frac": bts / t / 1e9 / HBM_PEAK_GBS}
    op.close()
    del f, z

    cases = (
        ("line1d_8192_k5_lmax7", W.Workload(
            name="line_k5", lmax=7, k=5, axes=("x",), nodes=(W.uniform_nodes(-10.0, 10.0, 8192),),
            bc=((W.PERIODIC, W.PERIODIC),), terms=frozenset({W.ADVECTION, W.ROTATION, W.COLLISION}),
            p_fixed=math.sqrt(3.0), flow=W.zero_flow, magnetic=W.uniform_field((0.0, 0.0, 1.0)), nu=1.0)),
        ("shock2d_x_p_512x64_k2_lmax3", W.shock_workload("shock_p", 512, 64, 2, 3, paxis="p",
                                                         lnp=(-1.0, 2.5), init=False)),
        ("shock2d_x_lnp_1024x128_k2_lmax3_wide_shock", W.shock_workload("shock_wide", 1024, 128, 2, 3,
                                                                       w_frac=0.25, init=False)),
    )
    for name, wl in cases:
        op = vfp.Operator(wl)
        N = op.ndofs
        u = torch.from_numpy(W.random_state(wl, 5, 1e-3).ravel()).cuda()
        work = torch.empty(2 * N, dtype=torch.float64, device="cuda")
        dt = op.cfl_dt(0.2) / wl.k
        steps = 20
        t = timed(lambda: op.advance(u, dt, steps, work), 1) / steps
        bts = N * (16 + 3 * 24) / 4
        if name.endswith("wide_shock"):
            bts += 8 * wl.ncells + 8 * wl.ncells * wl.n_basis + 8 * (1024 * 3 * 4 + 1025 + 128 * 3 * 4 + 129)
        out[name] = {"ndofs": N, "dofs_per_s": N / t, "us_per_launch": t / 4 * 1e6,
                     "bytes_per_launch": bts, "achieved_GBs": bts / (t / 4) / 1e9,
                     "frac": bts / (t / 4) / 1e9 / HBM_PEAK_GBS}
        if not torch.isfinite(u).all():
            raise RuntimeError(f"{name}: state is not finite")
        op.close()
    return out


def theta_timing(steps=5, cfl_mult=10.0):
    """Theta-method steps (Crank-Nicolson and backward Euler) of the 512 x 64
    shock, k=2, l_max=3, at 10 times the explicit time step: restarted GMRES
    (30 vectors, relative residual 1e-10) whose operator is the fused stage
    kernel; against the explicit Runge-Kutta run over the same time."""
    import numpy as np
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    import math
    wl = W.config5(steps=steps)
    op = vfp.Operator(wl)
    N = op.ndofs
    dt_exp = op.cfl_dt(wl.courant)
    dt = cfl_mult * dt_exp
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(np.ascontiguousarray(wl.meta["init"]).ravel()).to(dev)
    work = torch.empty(op.theta_work_size(30), dtype=torch.float64, device=dev)
    res = {"workload": wl.name, "ndofs": N, "steps": steps, "dt_over_explicit": cfl_mult}
    for name, theta in (("crank_nicolson", 0.5), ("backward_euler", 1.0)):
        u = u0.clone()
        op.theta_advance(u, dt, 1, theta=theta, tol=1e-10, restart=30, work=work)   # warm-up
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = op.theta_advance(u, dt, steps, theta=theta, tol=1e-10, restart=30, work=work)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        if not (st["converged"] and torch.isfinite(u).all()):
            raise RuntimeError(f"Theta-method {name} did not converge: {st}")
        res[name] = {"s_per_step": t / steps, "iterations_per_step": st["iterations"] / steps,
                     "residual": st["residual"]}
    # strong scattering (nu0 = 300): explicit steps are limited by the
    # reaction stiffness as well; the collision-diagonal preconditioner
    # inverts the stiff part exactly
    wl_s = W.shock_workload("shock_512x64_nu300", 512, 64, 2, 3, nu0=300.0, init=False)
    op_s = vfp.Operator(wl_s)
    nu_max = float(np.max(wl_s.nu))
    dt_cfl = op_s.cfl_dt(wl_s.courant)
    dt_rk = min(dt_cfl, 0.9 * 2.785 / (nu_max * wl_s.lmax * (wl_s.lmax + 1) / 2))
    stiff = {"nu_max": nu_max, "dt_cfl": dt_cfl, "dt_explicit_stable": dt_rk, "dt_implicit": cfl_mult * dt_cfl}
    us0 = torch.from_numpy(W.random_state(wl_s, 9, 1e-3).ravel()).to(dev)
    for name, pc in (("crank_nicolson", None), ("crank_nicolson_precond", "collision")):
        u = us0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = op_s.theta_advance(u, cfl_mult * dt_cfl, 2, theta=0.5, tol=1e-10, restart=30, work=work,
                                precond=pc)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / 2
        if not st["converged"]:
            raise RuntimeError(f"stiff Theta-method {name} did not converge: {st}")
        stiff[name] = {"s_per_step": t, "iterations_per_step": st["iterations"] / 2,
                       "s_per_unit_time": t / (cfl_mult * dt_cfl)}
    u = us0.clone()
    w2 = torch.empty(2 * N, dtype=torch.float64, device=dev)
    nrk = int(math.ceil(cfl_mult * dt_cfl / dt_rk)) * 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op_s.advance(u, dt_rk, nrk, w2)
    torch.cuda.synchronize()
    stiff["explicit_rk4_s_per_unit_time"] = (time.perf_counter() - t0) / (nrk * dt_rk)
    res["stiff_scattering"] = stiff
    op_s.close()

    u = u0.clone()
    op.advance(u, dt_exp, 5, w2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.advance(u, dt_exp, int(cfl_mult) * steps, w2)
    torch.cuda.synchronize()
    res["explicit_rk4_s_per_equal_time"] = (time.perf_counter() - t0) / steps
    return res


def other_configs():
    """The 3-D periodic box (48^3 cells, k=2, l_max=5, B with random Fourier
    modes; 107,495,424 DoF) and the 1-D periodic line (64 cells, k=1,
    l_max=3; 2,048 DoF): stage throughput, and for the box its HBM roofline
    fraction (stage bytes: 22 B/DoF on average plus B at the volume points)."""
    import numpy as np
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    out = {}
    stream = torch.cuda.current_stream()
    for name, wl, steps in (("box3d_48_k2_lmax5", W.config3(), 20), ("line1d_64_k1_lmax3", W.config1(), 100)):
        # (the line: 100 steps, the configuration's run length)
        op = vfp.Operator(wl)
        N = op.ndofs
        dt = op.cfl_dt(wl.courant)
        if "init" in wl.meta:
            u = torch.from_numpy(np.ascontiguousarray(wl.meta["init"]).ravel()).cuda()
        else:
            u = torch.from_numpy(np.ascontiguousarray(W.nodal_state(wl, wl.meta["init_func"])).ravel()).cuda()
        work = torch.empty(2 * N, dtype=torch.float64, device="cuda")
        t_w = time.perf_counter()
        while True:                      # untimed warm-up, at least 0.5 s of kernel time
            op.advance(u, dt, 3, work)
            torch.cuda.synchronize()
            if time.perf_counter() - t_w > 0.5:
                break
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        op.advance(u, dt, steps, work)
        e1.record(stream)
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        if not torch.isfinite(u).all():
            raise RuntimeError(f"{name}: state is not finite")
        rec = {"ndofs": N, "steps": steps, "dofs_per_s": N * steps / secs, "us_per_step": secs / steps * 1e6}
        if name.startswith("line"):
            rec["path"] = "one launch for all steps (the state in one workgroup's LDS)"
            rec["steps"] = steps
        if name.startswith("box"):
            per_launch = secs / (4 * steps)
            fields = 8 * wl.ncells * wl.n_basis * 3
            bts = N * (16 + 24 * 3) / 4 + fields
            rec.update({"us_per_launch": per_launch * 1e6, "bytes_per_launch": bts,
                        "achieved_GBs": bts / per_launch / 1e9, "frac": bts / per_launch / 1e9 / HBM_PEAK_GBS,
                        "kernel": "stage_kernel<3,2,5,false,false,false>"})
        out[name] = rec
        op.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warmup-seconds", type=float, default=2.0,
                    help="keep warming up (untimed) until this much time has passed")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the 3-D box and 1-D line legs")
    ap.add_argument("--no-theta", action="store_true", help="skip the Theta-method (implicit) leg")
    ap.add_argument("--batch-small", action="store_true",
                    help="also time 512 small runs (16-64 x 8-16 cells), where one launch per run is launch-bound")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the stage kernel's default launch shape (no vfp_autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              f"the multi-GPU decomposition is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2501_05110_amd import vfp, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    wl = W.config2()
    op = vfp.Operator(wl)
    N = op.ndofs
    dt = op.cfl_dt(wl.courant)
    u = torch.from_numpy(np.ascontiguousarray(wl.meta["init"]).ravel()).to(dev)
    work = torch.empty(2 * N, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)   # plain elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b

    # launch shape of the stage kernel: the library times its workgroup
    # shapes and tile orders on this state and keeps the fastest
    tuned = op.autotune(u, work[:N], reps=10) if not args.no_autotune else None

    # untimed warm-up: the requested steps, then more until the kernel has
    # run for --warmup-seconds (the GPU's clocks ramp up over the first
    # second of sustained work; a short warm-up leaves the timed steps on a
    # cold clock)
    t_w = time.perf_counter()
    op.advance(u, dt, args.warmup, work)
    torch.cuda.synchronize()
    warm_steps = args.warmup
    while time.perf_counter() - t_w < args.warmup_seconds:
        op.advance(u, dt, 100, work)
        torch.cuda.synchronize()
        warm_steps += 100
    warm_s = time.perf_counter() - t_w

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    op.advance(u, dt, args.steps, work)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    if not torch.isfinite(u).all():
        print("state is not finite after the timed steps", file=sys.stderr)
        sys.exit(1)

    # context for the roofline: what a plain streaming kernel (torch.mul on
    # 1 GiB, reading 1 GiB and writing 1 GiB) reaches on this GPU
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * a.numel() * 8 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del a, b

    secs = gpu_ms / 1e3
    launches = 4 * args.steps
    per_launch_s = secs / launches
    ncells = wl.ncells
    nb = wl.n_basis
    # algorithmic bytes per stage launch: stage 1 reads u and writes w (16 B/DoF),
    # stages 2-4 read w_in and u and write w_out (24 B/DoF); plus the input
    # fields at the resolution they cross the ABI (nu per cell, s at the volume
    # points, the 1-D profiles)
    field_bytes = 8 * ncells + 8 * ncells * nb + 8 * (1024 * 3 * 4 + 1025 + 128 * 3 * 4 + 129)
    bytes_per_launch = N * (16 + 24 * 3) / 4 + field_bytes
    achieved = bytes_per_launch / per_launch_s / 1e9
    out = {
        "metric": "DG-SH operator DoF-updates/s (FP64)",
        "value": N * args.steps / secs,
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": list(wl.ncells_axis), "k": wl.k,
                   "lmax": wl.lmax, "ndofs": N, "dt": dt, "courant": wl.courant,
                   "stage_launches": launches, "wall_s": wall,
                   "warmup_steps_run": warm_steps, "warmup_s": warm_s, "launch_shape": tuned},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "shock_kernel<2,3,1,false,false>",
                     "bytes_per_launch": bytes_per_launch, "us_per_launch": per_launch_s * 1e6,
                     "copy_GBs": copy_gbs},
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing()
    if not args.no_batch:
        out["batch"] = batch_timing(full=True)
    if args.batch_small:
        out["batch_small"] = batch_timing(full=False)
    if not args.no_other:
        out["other_configs"] = other_configs()
    if not args.no_theta:
        out["theta"] = theta_timing()
        out["dsa_paper"] = dsa_paper_timing()
    if not args.no_other:
        out["extensions"] = extension_timing()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

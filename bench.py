"""Benchmark of the SEM Burgers hot path on one MI355X.

Main timed step (the metric's workload): on the 3-D periodic unit cube with 32^3 hexahedral
elements of order N = 7 (33,718,272 unique DOF, FP64), one step applies F(u) and J(u)^T w once each.
`value` is DOF processed per second by that pair, in GDOF/s.  Per-operator GDOF/s (F, J v, J^T),
the J^T/F cost ratio, the FP32 variant, adjoint gradients/s of the 64-IC 2-D configuration and the
batched-vs-plain gradient/s of the 128 uneven 2-D problems are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu] [--calib-copy]
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E datasheet peak
HBM_RESERVE = 80e9  # HBM left free beside stored stage states (segment recompute storage, fields)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fast3d_jact_32cube_n7.md")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1806_01422_amd", "csrc", f) for f in ("kern_fast3d.hip", "fast_common.h")]


def measured_traffic():
    """HBM bytes per J^T apply from the committed FETCH_SIZE/WRITE_SIZE counter summary, or None
    when that summary is absent or was taken on a different version of the kernel source."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRCS)).hexdigest()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("source_sha256:",
                                                                                      "traffic_bytes_per_launch:")))
    if fields.get("source_sha256", "").strip() != src or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def event_time_ms(fn, reps, trials=1, warmup=1):
    """Milliseconds per call of fn: HIP events on the current stream around reps back-to-back calls,
    after warmup calls (first-call set-up such as module load and graph capture stays out); the
    median over trials."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    per = []
    for _ in range(trials):
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        per.append(s.elapsed_time(e) / reps)
    return float(np.median(per))


def c3_inputs(ctx, dtype):
    cfg = wl.C3
    xs = [ctx.node_coords(k) for k in range(3)]
    u = wl.fourier_field(xs, cfg.L, wl.C3_K, wl.C3_SEEDS["u"])[None]
    w = wl.normal_field(ctx.shape, wl.C3_SEEDS["w"])
    v = wl.normal_field(ctx.shape, wl.C3_SEEDS["v"])
    cv = lambda a: torch.from_numpy(a).to(device="cuda", dtype=dtype)  # noqa: E731
    return cv(u), cv(v), cv(w)


def cpu_baseline(target_s=12.0):
    """The CPU oracle (FP64, OpenMP) on the host cores: F and J^T on the full 3-D field."""
    import oracle
    cfg = wl.C3
    m = oracle.Mesh(3, cfg.N, list(cfg.E), list(cfg.L), cfg.nu)
    xs = [m.coords(k) for k in range(3)]
    u = wl.fourier_field(xs, cfg.L, wl.C3_K, wl.C3_SEEDS["u"])[None]
    w = wl.normal_field(m.shape, wl.C3_SEEDS["w"])
    reps, t_total, t0 = 0, 0.0, time.time()
    while t_total < target_s and reps < 20:
        t = time.time()
        m.rhs(u)
        m.jact_vec(u, w)
        t_total += time.time() - t
        reps += 1
    dof = m.ndof
    return {"value": round(dof * reps / t_total / 1e9, 5), "unit": "GDOF/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{reps} x (F + J^T) on the full 32^3 N=7 FP64 field ({dof} DOF), "
                      f"{t_total:.1f} s total on {oracle.num_threads()} threads"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_detail():
    """The CPU oracle on the host in more detail: the 2-D single applies (median of 20) and one
    3-D F + J^T pair on one thread and on all threads, and the C4 and C5 gradients extrapolated
    from stated samples."""
    import oracle

    def med(fn, n):
        ts = []
        for _ in range(n):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    allt = oracle.num_threads()
    out = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "omp_threads_all": allt,
           "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}
    cfg = wl.C2
    m2 = oracle.Mesh(2, cfg.N, list(cfg.E), list(cfg.L), cfg.nu)
    xs = [m2.coords(k) for k in range(2)]
    u2 = wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C2_SEEDS["u"])[None]
    w2 = wl.normal_field(m2.shape, wl.C2_SEEDS["w"])
    cfg3 = wl.C3
    m3 = oracle.Mesh(3, cfg3.N, list(cfg3.E), list(cfg3.L), cfg3.nu)
    xs3 = [m3.coords(k) for k in range(3)]
    u3 = wl.fourier_field(xs3, cfg3.L, wl.C3_K, wl.C3_SEEDS["u"])[None]
    w3 = wl.normal_field(m3.shape, wl.C3_SEEDS["w"])
    try:
        for label, nt in (("all_threads", 0), ("one_thread", 1)):
            oracle.set_threads(nt)
            f = med(lambda: m2.rhs(u2), 20)
            jt = med(lambda: m2.jact_vec(u2, w2), 20)
            t = time.perf_counter()
            m3.rhs(u3)
            m3.jact_vec(u3, w3)
            t3 = time.perf_counter() - t
            out[label] = {"threads": oracle.num_threads(),
                          "c2_f_us": round(f * 1e6, 1), "c2_jt_us": round(jt * 1e6, 1),
                          "c2_f_gdofs": round(m2.ndof / f / 1e9, 5), "c2_jt_gdofs": round(m2.ndof / jt / 1e9, 5),
                          "c3_f_plus_jt_gdofs": round(m3.ndof / t3 / 1e9, 5), "c3_sample": "one F + J^T pair"}
    finally:
        oracle.set_threads(0)
    del m3, u3, w3
    # C4: one initial condition, 20 of the 500 steps, forward + adjoint; scaled to 500 steps
    n4, k4 = 20, 10
    u4 = wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_IC_SEED0)[None]
    tg4 = wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_TARGET_SEED0)[None]
    t = time.perf_counter()
    uT, ck = m2.rk4_forward(u4, wl.C4_DT, n4, k4)
    m2.rk4_adjoint(ck, wl.C4_DT, n4, k4, uT - tg4)
    t4 = (time.perf_counter() - t) * wl.C4_STEPS / n4
    out["c4"] = {"gradients_per_s": round(1.0 / t4, 4),
                 "sample": f"one IC, {n4} of {wl.C4_STEPS} steps (ckpt every {k4}) on all threads, "
                           f"scaled by steps; the 64 ICs are independent, so gradients/s is per IC"}
    # C5 plain loop: the first 8 problems, 10 steps, forward + adjoint; scaled by DOF and steps
    probs = wl.c5_problems()
    sub, n5, k5 = probs[:8], 10, 5
    dof_sub, dof_all = 0, 0
    t5 = 0.0
    for i, p in enumerate(probs):
        dof_all += 2 * (p.N * p.E) ** 2
        if i >= len(sub):
            continue
        m = oracle.Mesh(2, p.N, [p.E, p.E], [1.0, 1.0], p.nu)
        xp = [m.coords(k) for k in range(2)]
        up = wl.fourier_field(xp, [1.0, 1.0], wl.C5_K, p.ic_seed)[None]
        tp = wl.fourier_field(xp, [1.0, 1.0], wl.C5_K, p.target_seed)[None]
        t = time.perf_counter()
        uT, ck = m.rk4_forward(up, p.dt, n5, k5)
        m.rk4_adjoint(ck, p.dt, n5, k5, uT - tp)
        t5 += time.perf_counter() - t
        dof_sub += m.ndof
    t_all = t5 * (dof_all / dof_sub) * (wl.C5_STEPS / n5)
    out["c5_plain"] = {"gradients_per_s": round(len(probs) / t_all, 4),
                       "sample": f"problems 0..{len(sub) - 1} ({dof_sub} of {dof_all} DOF), {n5} of {wl.C5_STEPS} "
                                 f"steps, forward + adjoint on all threads, scaled by DOF and steps"}
    return out


def gradient_c4(P, nsteps=wl.C4_STEPS, K=wl.C4_CKPT, stored_tail=0):
    """Misfit gradients of the 64 ICs through autograd: uniform checkpoints every K steps, the
    last stored_tail segments kept whole (every stage state) by the forward sweep."""
    cfg = wl.C4
    ctx = P.Context(2, cfg.N, cfg.E, cfg.L, cfg.nu, batch=cfg.batch)
    xs = [ctx.node_coords(k) for k in range(2)]
    u0 = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_IC_SEED0 + b) for b in range(cfg.batch)])
    tg = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_TARGET_SEED0 + b) for b in range(cfg.batch)])
    U0, TG = torch.from_numpy(u0).cuda(), torch.from_numpy(tg).cuda()

    def grad():
        x = U0.clone().requires_grad_(True)
        yT = P.trajectory(x, ctx, wl.C4_DT, nsteps, K, stored_tail=stored_tail)
        loss = 0.5 * ((yT - TG) ** 2).sum()
        loss.backward()
        return x.grad

    g = grad()  # warm-up (graph capture, allocations); its gradient is returned
    ms = event_time_ms(grad, 1)
    ctx.close()
    return cfg.batch / (ms / 1e3), ms, g


def apply_2d(P):
    """Single-apply throughput of F, J v and J^T w on the 2-D 64x64 N=7 FP64 mesh (nu = 1e-3), for one
    field and for the 64 fields of the adjoint-gradient configuration; HBM fraction from the
    algorithmic bytes (F, J v: 16 B/DOF and 24 B/DOF; J^T: 24 B/DOF)."""
    cfg = wl.C2
    out = {"workload": "2-D 64x64 N=7 FP64, nu=1e-3: one field, and 64 fields (the gradient batch)",
           "note": "one field (6.4-9.6 MB per apply) stays in the 256 MB last-level cache and is bound by launch "
                   "and latency, so its HBM fraction is not meaningful; 64 fields (411-617 MB) are HBM-bound",
           "timing": "HIP events, 100 applies after 10 warm-up applies, median of 5 trials"}
    for batch in (1, wl.C4.batch):
        ctx = P.Context(2, cfg.N, cfg.E, cfg.L, cfg.nu, batch=batch)
        xs = [ctx.node_coords(k) for k in range(2)]
        u = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_IC_SEED0 + b) for b in range(batch)])
        U = torch.from_numpy(u).cuda()
        V = torch.from_numpy(wl.normal_field(ctx.shape, wl.C2_SEEDS["v"])).cuda()
        W = torch.from_numpy(wl.normal_field(ctx.shape, wl.C2_SEEDS["w"])).cuda()
        F, JV, JT = ctx.empty(), ctx.empty(), ctx.empty()
        reps = 100
        t_f = event_time_ms(lambda: ctx.rhs(U, F), reps, trials=5, warmup=10)
        t_jv = event_time_ms(lambda: ctx.jac_vec(U, V, JV), reps, trials=5, warmup=10)
        t_jt = event_time_ms(lambda: ctx.jact_vec(U, W, JT), reps, trials=5, warmup=10)
        dof = ctx.ndof * batch
        out[f"fields_{batch}"] = {
            "dof": dof, "kernel_path": ctx.path, "f_us": round(t_f * 1e3, 2), "jv_us": round(t_jv * 1e3, 2),
            "jt_us": round(t_jt * 1e3, 2), "f_gdofs": round(dof / t_f / 1e6, 2), "jv_gdofs": round(dof / t_jv / 1e6, 2),
            "jt_gdofs": round(dof / t_jt / 1e6, 2),
            "f_hbm_frac": round(16.0 * dof / (t_f / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "jt_hbm_frac": round(24.0 * dof / (t_jt / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        ctx.close()
        del U, V, W, F, JV, JT
        torch.cuda.empty_cache()
    return out


def c5_sets(P):
    probs = wl.c5_problems()
    specs = [dict(dim=2, order=p.N, elems=(p.E, p.E), length=(1.0, 1.0), nu=p.nu, dt=p.dt) for p in probs]
    return probs, specs


def gradient_c5(P, nsteps=wl.C5_STEPS, K=50, iters=wl.C5_ITERS, alpha=wl.C5_ALPHA, plain_iters=2):
    """Gradient descent on the initial conditions of all 128 problems: `iters` iterations of
    u0 <- u0 - alpha d / max|d| per problem, d = W g, g the misfit gradient (forward + adjoint over
    `nsteps` RK4 steps, checkpoint every K) and W = M / mean(M).  Batched: the packed set (autotuned
    launches, graph-captured steps).  Plain: one context per problem, launched one after another;
    it runs `plain_iters` iterations (the cost of an iteration does not depend on the iterate) and
    its iterate there is compared with the batched loop's, value by value.  Both run the same
    kernels and the same elementwise update, so the iterates are bitwise equal."""
    probs, specs = c5_sets(P)
    B = P.Batch(specs)
    step_ms = B.autotune()  # launch shape chosen by timing the captured RK4 step
    u0 = B.empty()
    tg = B.empty()
    nodes = []
    for i, p in enumerate(probs):
        ctxi = P.Context(2, p.N, (p.E, p.E), (1.0, 1.0), p.nu)
        xs = [ctxi.node_coords(k) for k in range(2)]
        B.view(u0, i).copy_(torch.from_numpy(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.ic_seed)[None]))
        B.view(tg, i).copy_(torch.from_numpy(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.target_seed)[None]))
        nodes.append(ctxi.nodes)
        ctxi.close()
    # W = M / mean(M): on the unit square mean(M) = 1 / nodes
    wB = B.mass()
    for i in range(len(probs)):
        B.view(wB, i).mul_(float(nodes[i]))

    sizes = torch.tensor([int(B.offsets[i + 1] - B.offsets[i]) for i in range(len(probs))], device="cuda")

    def step(u, g, w, views=None):
        # views: the packed set's problem slices (one scale per problem), else one problem
        d = w * g
        if views is None:
            scale = alpha / d.abs().max()
        else:
            mx = torch.stack([views(d, i).abs().max() for i in range(len(probs))])
            scale = torch.repeat_interleave(alpha / mx, sizes)
        d.mul_(scale)
        u.sub_(d)

    def batched_loop(n_it, record=None):
        u = u0.clone()
        for it in range(n_it):
            uT, ck = B.rk4_forward(u, nsteps, K)
            r = uT - tg
            if record is not None:
                record.append(0.5 * (r * r).sum())
            g = B.rk4_adjoint(ck, nsteps, K, r)
            step(u, g, wB, B.view)
        return u

    ctxs = [P.Context(2, p.N, (p.E, p.E), (1.0, 1.0), p.nu) for p in probs]
    wps = [c.mass() * float(n) for c, n in zip(ctxs, nodes)]
    views = [(B.view(u0, i).contiguous(), B.view(tg, i).contiguous()) for i in range(len(probs))]

    def plain_loop(n_it):
        us = [ui.clone() for ui, _ in views]
        for it in range(n_it):
            for c, p, u, (_, ti), w in zip(ctxs, probs, us, views, wps):
                uT, ck = c.rk4_forward(u, p.dt, nsteps, K)
                g = c.rk4_adjoint(ck, p.dt, nsteps, K, uT - ti)
                step(u, g, w)
        return us

    phis = []
    ub = batched_loop(iters, phis)  # warm-up and the objective history
    phis = [float(v) for v in phis]
    finite = bool(torch.isfinite(ub).all())
    ub2 = batched_loop(plain_iters)
    up2 = plain_loop(plain_iters)
    # a non-finite value anywhere makes the difference NaN (Python's max would skip it)
    diff = float(torch.stack([(B.view(ub2, i) - up2[i]).abs().max() for i in range(len(probs))]).max())
    tb = event_time_ms(lambda: batched_loop(iters), 1, warmup=0)
    tp = event_time_ms(lambda: plain_loop(plain_iters), 1, warmup=0)
    ng_b, ng_p = len(probs) * iters, len(probs) * plain_iters
    out = {"workload": f"{len(probs)} uneven 2-D problems, {iters} gradient-descent iterations on the initial "
                       f"conditions, {nsteps} RK4 steps each (checkpoint every {K}); mass-weighted direction, step normalised to "
                       f"max change {alpha} per problem and iteration",
           "batched_gradients_per_s": round(ng_b / (tb / 1e3), 2),
           "plain_gradients_per_s": round(ng_p / (tp / 1e3), 2),
           "batched_over_plain": round((tp / ng_p) / (tb / ng_b), 3),
           "batched_loop_s": round(tb / 1e3, 3), "plain_iterations_timed": plain_iters,
           "max_abs_iterate_diff_after_plain_iterations": diff, "iterates_finite": finite,
           "objective_first_last": [round(phis[0], 6), round(phis[-1], 6)],
           "objective_decreased_every_iteration": all(b < a for a, b in zip(phis, phis[1:])),
           "problems": len(probs), "total_dof": int(B.total), "autotuned_rk4_step_ms": round(step_ms, 4)}
    for c in ctxs:
        c.close()
    del up2, views, wps
    torch.cuda.empty_cache()

    # one gradient with every stage state of all steps kept by the forward sweep (4 states per
    # step), when free HBM holds them beside the same reserve as the 64-IC gradient: the adjoint
    # then recomputes nothing
    def batched_grad():
        uT, ck = B.rk4_forward(u0, nsteps, K)
        return B.rk4_adjoint(ck, nsteps, K, uT - tg)

    st_bytes = nsteps * 4 * 8 * int(B.total)
    if torch.cuda.mem_get_info()[0] - HBM_RESERVE >= st_bytes:
        def batched_stored():
            uT, st = B.rk_forward_stored(u0, nsteps)
            return B.rk_adjoint_stored(st, nsteps, uT - tg)

        gb = batched_grad()
        gs = batched_stored()
        tg1 = event_time_ms(batched_grad, 1)
        ts = event_time_ms(batched_stored, 1)
        out.update({"one_gradient_gradients_per_s": round(len(probs) / (tg1 / 1e3), 2),
                    "all_stages_stored_gradients_per_s": round(len(probs) / (ts / 1e3), 2),
                    "all_stages_stored_bytes": st_bytes,
                    "all_stages_stored_max_abs_gradient_diff": float((gs - gb).abs().max())})
        del gb, gs
    B.close()
    return out


def rk_adjoint_ratio(P, nsteps=10):
    """Forward and discrete-adjoint time per step of RK-3 and RK4 on the 3-D 32^3 N=7 FP64 field:
    checkpoints every step (the adjoint recomputes only stage states) and every 5 steps (segment
    recompute as well), and every stage stored by the forward sweep (no recompute)."""
    cfg = wl.C3
    ctx = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float64)
    U, _, W = c3_inputs(ctx, torch.float64)
    dt = 1e-4
    out = {"workload": f"3-D 32^3 N=7 FP64, {nsteps} steps, dt={dt}"}
    for scheme in ("rk3", "rk4"):
        res = {}
        for K in (1, 5):
            uT, ck = ctx.rk_forward(U, dt, nsteps, K, scheme=scheme)  # warm-up (graph capture)
            work = torch.empty(ctx.workspace_bytes(K) // 8, dtype=torch.float64, device="cuda")
            ctx.rk_adjoint(ck, dt, nsteps, K, W, scheme=scheme, work=work)
            t_f = event_time_ms(lambda: ctx.rk_forward(U, dt, nsteps, K, scheme=scheme), 3) / nsteps
            t_a = event_time_ms(lambda: ctx.rk_adjoint(ck, dt, nsteps, K, W, scheme=scheme, work=work), 3) / nsteps
            res[f"K{K}"] = {"forward_ms_per_step": round(t_f, 4), "adjoint_ms_per_step": round(t_a, 4),
                            "adjoint_over_forward": round(t_a / t_f, 3)}
            del ck, work
        # every stage stored by the forward sweep: the adjoint applies only the J^T products
        uT, st = ctx.rk_forward_stored(U, dt, nsteps, scheme=scheme)
        ctx.rk_adjoint_stored(st, dt, nsteps, W, scheme=scheme)
        t_f = event_time_ms(lambda: ctx.rk_forward_stored(U, dt, nsteps, scheme=scheme), 3) / nsteps
        t_a = event_time_ms(lambda: ctx.rk_adjoint_stored(st, dt, nsteps, W, scheme=scheme), 3) / nsteps
        res["stored_stages"] = {"forward_ms_per_step": round(t_f, 4), "adjoint_ms_per_step": round(t_a, 4),
                                "adjoint_over_forward": round(t_a / t_f, 3),
                                "stage_states_gb": round(st.numel() * 8 / 1e9, 2)}
        del uT, st
        torch.cuda.empty_cache()
        out[scheme] = res
    ctx.close()
    torch.cuda.empty_cache()
    return out


def revolve_measure(P, nsteps=40):
    """RK-3 on the 3-D 32^3 N=7 FP64 field with binomial checkpointing in a few state slots:
    forward and adjoint time per step, forward steps the schedule recomputes, memory in states."""
    cfg = wl.C3
    ctx = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float64)
    U, _, W = c3_inputs(ctx, torch.float64)
    dt = 1e-4
    out = {"workload": f"3-D 32^3 N=7 FP64, RK-3, {nsteps} steps, dt={dt}"}
    for snaps in (4, 8):
        _, adv = P.revolve_plan(nsteps, snaps)
        uT, ck = ctx.rk_forward_revolve(U, dt, nsteps, snaps, scheme="rk3")
        work = torch.empty(ctx.workspace_bytes(1) * snaps // 8, dtype=torch.float64, device="cuda")
        t_f = event_time_ms(lambda: ctx.rk_forward_revolve(U, dt, nsteps, snaps, scheme="rk3"), 2) / nsteps
        t_a = event_time_ms(lambda: ctx.rk_adjoint_revolve(ck, dt, nsteps, snaps, W, scheme="rk3", work=work),
                            2) / nsteps
        out[f"snaps{snaps}"] = {"forward_ms_per_step": round(t_f, 4), "adjoint_ms_per_step": round(t_a, 4),
                                "adjoint_over_forward": round(t_a / t_f, 3), "schedule_forward_steps": adv,
                                "state_slots": snaps, "store_all_states": nsteps}
        del ck, work
    ctx.close()
    torch.cuda.empty_cache()
    return out


def cn_measure(P, nsteps=4, K=2, dt=2e-4):
    """Crank-Nicolson on the 3-D 32^3 N=7 FP64 field: forward (Newton-Krylov per step) and
    discrete adjoint (one GMRES solve with J^T per step plus the segment recompute)."""
    cfg = wl.C3
    ctx = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float64)
    U, _, W = c3_inputs(ctx, torch.float64)
    work = torch.empty(ctx.cn_workspace_bytes(K) // 8, dtype=torch.float64, device="cuda")
    uT, ck, _ = ctx.cn_forward(U, dt, nsteps, K, work=work)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uT, ck, sf = ctx.cn_forward(U, dt, nsteps, K, work=work)
    t_f = (time.perf_counter() - t0) * 1e3 / nsteps
    t0 = time.perf_counter()
    lam, sa = ctx.cn_adjoint(ck, dt, nsteps, K, W, work=work)
    t_a = (time.perf_counter() - t0) * 1e3 / nsteps
    ctx.close()
    del U, W, work, ck, uT, lam
    torch.cuda.empty_cache()
    return {"workload": f"3-D 32^3 N=7 FP64, Crank-Nicolson, {nsteps} steps, dt={dt}, checkpoint every {K}",
            "forward_ms_per_step": round(t_f, 3), "adjoint_ms_per_step": round(t_a, 3),
            "adjoint_over_forward": round(t_a / t_f, 3), "forward_stats": sf, "adjoint_stats": sa,
            "note": "the adjoint includes recomputing each segment's states (Newton solves)"}


def lmvm_measure(P):
    """The optimiser on the GPU: the 1-D optimal-initial-condition recovery (Cole-Hopf target at
    T = 4, Gaussian-perturbed first guess, E=16 N=8 nu=0.01, RK4 dt=5e-3, 30 iterations).  The
    objective history comes from the 30-iteration run; the initial-condition error after k
    iterations from runs stopped at k (the driver is deterministic, so run k ends at the k-th
    iterate of the long run)."""
    out = {}
    nu, T, dt = 0.01, 4.0, 5e-3
    c = P.Context(1, 8, [16], [4.0], nu)
    x = torch.from_numpy(c.node_coords(0))

    def ch(t):
        ex = np.exp(-nu * np.pi ** 2 * t)
        return 2 * nu * np.pi * torch.sin(np.pi * x) * ex / (2.0 + ex * torch.cos(np.pi * x))
    exact0 = ch(0.0)[None, None].to("cuda", torch.float64)
    target = ch(T)[None, None].to("cuda", torch.float64)
    guess = exact0 + torch.exp(-4 * (x - 2) ** 2)[None, None].to("cuda", torch.float64)
    n = int(round(T / dt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, hist, st = c.lmvm_initial_condition(guess, target, dt, n, 50, scheme="rk4", opts={"max_iters": 30})
    t1 = time.perf_counter() - t0
    e0 = float((guess - exact0).norm())
    ic_err = {"0": 1.0}
    for k in (1, 2, 5, 10, 20):
        uk, _, _ = c.lmvm_initial_condition(guess, target, dt, n, 50, scheme="rk4", opts={"max_iters": k})
        ic_err[str(k)] = round(float((uk - exact0).norm()) / e0, 4)
    ic_err[str(st["iters"])] = round(float((u - exact0).norm()) / e0, 4)
    out["recovery_1d"] = {"iterations": st["iters"], "evaluations": st["evals"], "seconds": round(t1, 3),
                          "objective_history": [round(h, 8) for h in hist],
                          "ic_error_l2_relative_after_k_iterations": ic_err,
                          "note": "the misfit at T falls ~600x while the initial condition stays ~95% off: over "
                                  "T = 4 the unit Gaussian bump steepens and is damped, so its detail is not "
                                  "observable at T; the recovery outcome is parity-unpinned"}
    c.close()
    torch.cuda.empty_cache()
    return out


def profile_case(P, case):
    """A short, fixed workload for rocprofv3 kernel traces."""
    if case == "c5_steps":
        probs, specs = c5_sets(P)
        B = P.Batch(specs)
        B.autotune()
        u = B.empty().normal_(0, 0.01)
        for _ in range(3):
            uT, ck = B.rk4_forward(u, 20, 10)
            B.rk4_adjoint(ck, 20, 10, uT)
    elif case == "c4_gradient":
        gradient_c4(P, nsteps=100)
    else:
        cfg = wl.C3
        ctx = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float64)
        U, _, W = c3_inputs(ctx, torch.float64)
        for scheme in ("rk4", "rk3"):
            uT, ck = ctx.rk_forward(U, 1e-4, 10, 5, scheme=scheme)
            ctx.rk_adjoint(ck, 1e-4, 10, 5, W, scheme=scheme)
    torch.cuda.synchronize()
    log(f"profile case {case} done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="comma-separated extra measurements to run (fp32, fp64_rates, c2_apply, c4_adjoint, c5_batched, "
                         "rk_adjoint, revolve, crank_nicolson, lmvm), or all")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain elementwise copy of one field (known bytes) for counter calibration")
    ap.add_argument("--profile-case", choices=("c5_steps", "c4_gradient", "rk3d_steps"),
                    help="run only a short workload for a profiler (no JSON contract): the batched set's "
                         "RK4 steps and adjoint, the 64-IC misfit gradient over 100 steps (warm-up plus "
                         "one timed gradient), or RK4 steps and adjoint on the 3-D field")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path runs on one MI355X, "
              "with no sharding or collectives", file=sys.stderr)
        sys.exit(2)
    import paper_1806_01422_amd as P

    if args.profile_case:
        profile_case(P, args.profile_case)
        return

    cfg = wl.C3
    ctx = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float64)
    dof = ctx.ndof
    U, V, W = c3_inputs(ctx, torch.float64)
    F, JT, JV = ctx.empty(), ctx.empty(), ctx.empty()

    def step():
        ctx.rhs(U, F)
        ctx.jact_vec(U, W, JT)

    log(f"3-D 32^3 N=7 FP64: {dof} DOF; warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    s.record()
    for _ in range(args.steps):
        step()
    e.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = s.elapsed_time(e) / args.steps
    value = dof / (ms_step / 1e3) / 1e9  # DOF through F + J^T per second
    log(f"step (F + J^T): {ms_step:.4f} ms  ({value:.2f} GDOF/s), wall {wall:.3f} s")

    # single operators: 100 back-to-back applies after 10 warm-up applies, median of 5 trials
    reps = 100
    t_f = event_time_ms(lambda: ctx.rhs(U, F), reps, trials=5, warmup=10)
    t_jt = event_time_ms(lambda: ctx.jact_vec(U, W, JT), reps, trials=5, warmup=10)
    t_jv = event_time_ms(lambda: ctx.jac_vec(U, V, JV), reps, trials=5, warmup=10)
    bytes_jt = 24.0 * dof  # read u and w, write J^T w (FP64)
    achieved = bytes_jt / (t_jt / 1e3) / 1e9
    # reference: a plain elementwise streaming kernel over one field (read 8 B, write 8 B per DOF)
    t_copy = event_time_ms(lambda: torch.neg(U, out=JV), reps, trials=5, warmup=10)
    copy_gbs = 16.0 * dof / (t_copy / 1e3) / 1e9
    out = {
        "metric": "GDOF/s for F(u) and J^T w (FP64), J^T/F cost ratio, gradient/s batched vs plain",
        "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3-D periodic viscous Burgers, unit cube, 32^3 hex elements, order N=7 "
                               "(8 GLL points per direction), nu=1e-3; step = F(u) + J(u)^T w",
                   "elements": [32, 32, 32], "order": 7, "dof": dof, "fields": "u: seeded Fourier |k|<=6, "
                   "1/|k|^2 spectrum, max|u|=1; w, v: seeded N(0,1)"},
        "f_gdofs": round(dof / t_f / 1e6, 3), "jt_gdofs": round(dof / t_jt / 1e6, 3),
        "jv_gdofs": round(dof / t_jv / 1e6, 3), "jt_over_f": round(t_jt / t_f, 4),
        "f_ms": round(t_f, 5), "jt_ms": round(t_jt, 5), "jv_ms": round(t_jv, 5),
        "roofline": {"bound": "hbm", "kernel": "J^T w apply: fast3d_kernel (J^T, faces completed in the kernel)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic()},
        "f_hbm_frac": round(16.0 * dof / (t_f / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "stream_copy": {"gbs": round(copy_gbs, 1), "jt_frac": round(achieved / copy_gbs, 4),
                        "f_frac": round(16.0 * dof / (t_f / 1e3) / 1e9 / copy_gbs, 4)},
    }
    if args.calib_copy:
        # A plain copy of one field (read 8 B, write 8 B per DOF): the reference dispatch against
        # which the FETCH_SIZE / WRITE_SIZE counters are scaled.
        for _ in range(5):
            torch.neg(U, out=JV)
        torch.cuda.synchronize()
        log(f"calibration copy: 5 x {8 * dof} bytes read and written")
    ctx.close()
    del U, V, W, F, JT, JV
    torch.cuda.empty_cache()

    chosen = set(args.extras.split(","))

    def want(name):
        return not args.no_extras and ("all" in chosen or name in chosen)

    if want("fp32"):
        c32 = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float32)
        U32, _, W32 = c3_inputs(c32, torch.float32)
        t_f32 = event_time_ms(lambda: c32.rhs(U32), reps, trials=5, warmup=10)
        t_jt32 = event_time_ms(lambda: c32.jact_vec(U32, W32), reps, trials=5, warmup=10)
        c64 = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=torch.float64)
        U64, _, W64 = c3_inputs(c64, torch.float64)
        f64, j64 = c64.rhs(U64), c64.jact_vec(U64, W64)
        e_f = float((c32.rhs(U32).double() - f64).abs().max() / f64.abs().max())
        e_j = float((c32.jact_vec(U32, W32).double() - j64).abs().max() / j64.abs().max())
        out["fp32"] = {"f_gdofs": round(dof / t_f32 / 1e6, 3), "jt_gdofs": round(dof / t_jt32 / 1e6, 3),
                       "f_rel_err_vs_fp64": e_f, "jt_rel_err_vs_fp64": e_j}
        c32.close(), c64.close()
        del U32, W32, U64, W64, f64, j64
        torch.cuda.empty_cache()
        log("fp32 done")
    if want("fp64_rates"):
        # the diagnostic behind contracting on the vector units: matrix-core and vector FP64 rates,
        # alone and interleaved in one instruction stream
        r = P.probe_fp64_rates()
        out["fp64_rates"] = {k: round(v, 2) for k, v in r.items()}
        out["fp64_rates"]["unit"] = "TFLOP/s"
        out["fp64_rates"]["note"] = ("4096 x 256 threads: v_mfma_f64_16x16x4f64 with four accumulators, v_fma_f64 "
                                     "with eight chains, and both in one loop; dense FP64 peak 78.6 TFLOP/s")
    if want("c2_apply"):
        out["c2_apply"] = apply_2d(P)
        log("2-D apply done")
    if want("c4_adjoint"):
        gps, ms, g_plain = gradient_c4(P)
        torch.cuda.empty_cache()
        # as many of the last segments kept whole as free HBM holds beside the reserve: one segment
        # is 50 steps x 4 states x 205.5 MB = 41.1 GB (4 segments on an idle 288 GB MI355X)
        seg_bytes = wl.C4_CKPT * 4 * 8 * 401408 * wl.C4.batch
        tail = int(max(0, min(wl.C4_STEPS // wl.C4_CKPT, (torch.cuda.mem_get_info()[0] - HBM_RESERVE) // seg_bytes)))
        gps_t, ms_t, g_tail = gradient_c4(P, stored_tail=tail)
        out["c4_adjoint"] = {"gradients_per_s": round(gps, 3), "ms_per_batch_of_64": round(ms, 2),
                             "steps": wl.C4_STEPS, "ckpt_every": wl.C4_CKPT,
                             "stored_tail_segments": tail, "stored_tail_bytes": tail * seg_bytes,
                             "gradients_per_s_stored_tail": round(gps_t, 3),
                             "ms_per_batch_of_64_stored_tail": round(ms_t, 2),
                             "stored_tail_max_abs_gradient_diff": float((g_tail - g_plain).abs().max()),
                             "workload": "2-D 64x64 N=7, 64 ICs, RK4 dt=2e-4, misfit gradient via autograd"}
        torch.cuda.empty_cache()
        log("c4 done")
    if want("c5_batched"):
        out["c5_batched"] = gradient_c5(P)
        log("c5 done")
    if want("rk_adjoint"):
        out["rk_adjoint"] = rk_adjoint_ratio(P)
        log("rk adjoint ratio done")
    if want("revolve"):
        out["revolve"] = revolve_measure(P)
        log("revolve done")
    if want("crank_nicolson"):
        out["crank_nicolson"] = cn_measure(P)
        log("crank-nicolson done")
    if want("lmvm"):
        out["lmvm"] = lmvm_measure(P)
        log("lmvm done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_oracle"] = cpu_oracle_detail()
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the cell-centred multigrid hot path on one MI355X.

A step is one whole solve to tolerance (V(2,2) cycles of red-black
Gauss-Seidel, four-cell restriction, centred-slope prolongation, 2x2 bottom
solve, FP64 stop test) of the headline workload, the largest single-GPU
configuration of the plain FP64 V-cycle:

  Poisson on 8192 x 8192 cells, homogeneous Dirichlet sides, f = sum of 64
  seeded Fourier modes (|k| <= 32, N(0,1) amplitudes), relative residual 1e-10.

Inputs are generated on the host, uploaded once, and resident in HBM when the
timed region starts.  The printed JSON line reports grid-points x V-cycles per
second over the K timed solves, the roofline of the dominant kernel (measured
with HIP events in a separate pass of the same K solves), the FP64 CPU oracle
timed on a bounded sample of the same workload, and in `also` the other
workloads (4096^2 periodic, the mixed, batched and learned forms, the next
rows) and a streaming probe of this device.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import tempfile
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def upload(cc, torch, fv):
    n = fv.shape[0]
    f = cc.field(n)
    f[1:n + 1, 1:n + 1] = torch.from_numpy(fv).cuda()
    return f


def run_solves(cc, torch, plan, f, phi, steps, profile=False):
    """Time `steps` solves; returns (seconds, results)."""
    if profile:
        cc.ccmg_plan_profile(plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [cc.ccmg_solve(plan, f, phi) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if profile:
        stats = cc.ccmg_plan_kernel_stats(plan)
        cc.ccmg_plan_profile(plan, False)
    return dt, res, stats


def measure(cc, torch, n, bc, fv, steps, warmup, fused_shape=None):
    prob = cc.Problem(n=n, bc=bc, rtol=1e-10)
    plan = cc.Plan(prob)
    f = upload(cc, torch, fv)
    phi = cc.field(n)
    cc.ccmg_plan_autotune(plan, f, phi)  # launch shapes per level, before any timing
    if fused_shape:  # a fixed shape for the fused launch (reproducible counter runs)
        cc.ccmg_plan_set_shape(plan, 0, 2, fused_shape[0], fused_shape[1])
    shapes = cc.ccmg_plan_shapes(plan)
    fused_shape = cc.ccmg_plan_fused_shape(plan, 2)
    # levels 1 .. (those above the 32^2 tail) run as visits where ty > 0
    visits = [cc.ccmg_plan_shape(plan, lv, 5) for lv in range(1, n.bit_length() - 1 - 5)]
    for _ in range(warmup):
        r = cc.ccmg_solve(plan, f, phi)
        assert r.status == cc.OK, r
    dt, res, _ = run_solves(cc, torch, plan, f, phi, steps)
    cycles = sum(r.cycles for r in res)
    assert all(r.status == cc.OK and r.rel_resid <= 1e-10 for r in res)
    # kernel durations: a second pass of the same solves with HIP events around
    # the finest-level launches
    _, _, stats = run_solves(cc, torch, plan, f, phi, steps, profile=True)
    out = dict(n=n, bc=bc, seconds=dt, solves=steps, cycles=cycles,
               cycles_per_solve=cycles / steps, ms_per_solve=1e3 * dt / steps,
               pts_cycles_per_s=n * n * cycles / dt, rel_resid=res[-1].rel_resid,
               history=res[-1].history, kernels=stats, shapes=shapes, fused_shape=fused_shape, visits=visits)
    del plan, f, phi
    torch.cuda.empty_cache()
    return out


def time_form(cc, torch, prob, fv, steps, warmup):
    """Time-to-tolerance of one problem: autotune, warm up, then `steps` solves."""
    plan = cc.Plan(prob)
    f = upload(cc, torch, fv)
    phi = cc.field(prob.n)
    cc.ccmg_plan_autotune(plan, f, phi)
    for _ in range(warmup):
        r = cc.ccmg_solve(plan, f, phi)
        assert r.status == cc.OK, r
    dt, res, _ = run_solves(cc, torch, plan, f, phi, steps)
    assert all(r.status == cc.OK and r.rel_resid <= prob.rtol for r in res)
    _, _, stats = run_solves(cc, torch, plan, f, phi, max(2, steps // 2), profile=True)
    out = dict(ms=1e3 * dt / steps, cycles=res[-1].cycles, inner_cycles=res[-1].inner_cycles,
               rel_resid=res[-1].rel_resid,
               kernels=[dict(name=k["name"], avg_ms=round(k["ms"] / k["launches"], 5),
                             gbs=round(k["bytes"] / k["launches"] / (k["ms"] / k["launches"] * 1e-3) / 1e9, 1))
                        for k in stats if k["launches"] > 0])
    del plan, f, phi
    torch.cuda.empty_cache()
    return out


def mixed_vs_plain(cc, torch, W, steps):
    """Mixed precision against the plain FP64 form on the same problems: the
    Crank-Nicolson Helmholtz solves (1 - (k dt/2) Lap) phi = g on 8192^2
    (k dt / h^2 = 0.1, 1, 10; g a Gaussian random field of correlation length
    0.05, periodic), the 4096^2 periodic Poisson problem and the 8192^2
    Dirichlet headline problem."""
    out = {}
    n = 8192
    g = W.gaussian_random_field(n, seed=0)
    for c in (0.1, 1.0, 10.0):
        beta = c / (2.0 * n * n)
        row = {}
        for name, prec in (("plain_fp64", cc.FP64), ("mixed", cc.MIXED)):
            prob = cc.Problem(n=n, bc="P", alpha=1.0, beta=beta, rtol=1e-10, prec=prec)
            row[name] = time_form(cc, torch, prob, g, steps, 1)
        row["speedup"] = round(row["plain_fp64"]["ms"] / row["mixed"]["ms"], 3)
        out[f"helmholtz_8192_c{c}"] = row
        log(f"helmholtz 8192^2 c={c}: plain {row['plain_fp64']['ms']:.3f} ms ({row['plain_fp64']['cycles']} cyc), "
            f"mixed {row['mixed']['ms']:.3f} ms ({row['mixed']['cycles']} steps), x{row['speedup']}")
    del g
    n = 4096
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    row = {}
    for name, prec in (("plain_fp64", cc.FP64), ("mixed", cc.MIXED)):
        row[name] = time_form(cc, torch, cc.Problem(n=n, bc="P", rtol=1e-10, prec=prec), fv, steps, 2)
    row["speedup"] = round(row["plain_fp64"]["ms"] / row["mixed"]["ms"], 3)
    out["poisson_4096_periodic"] = row
    log(f"poisson 4096^2: plain {row['plain_fp64']['ms']:.3f} ms, mixed {row['mixed']['ms']:.3f} ms, x{row['speedup']}")
    del fv
    n = 8192
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    row = {}
    for name, prec in (("plain_fp64", cc.FP64), ("mixed", cc.MIXED)):
        row[name] = time_form(cc, torch, cc.Problem(n=n, bc="D", rtol=1e-10, prec=prec), fv, steps, 1)
    row["speedup"] = round(row["plain_fp64"]["ms"] / row["mixed"]["ms"], 3)
    out["poisson_8192_dirichlet"] = row
    log(f"poisson 8192^2 Dirichlet: plain {row['plain_fp64']['ms']:.3f} ms, mixed {row['mixed']['ms']:.3f} ms, "
        f"x{row['speedup']}")
    return out


def cn_diffusion(cc, torch, steps):
    """Crank-Nicolson diffusion steps (the paper's Gaussian test problem,
    t0 = 1e-4, phi1 = 1, phi2 = 2, k = 1, C = dt k / dx^2 = 2) on 8192^2 with
    Neumann sides: per step the right-hand side kernel and a solve from the
    old level to 1e-10, plain FP64 and mixed precision."""
    n = 8192
    h = 1.0 / n
    dt = 2.0 * h * h
    x = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) * h
    r2 = (x[None, :] - 0.5) ** 2 + (x[:, None] - 0.5) ** 2
    g0 = (1e-4 / (0.0 + 1e-4)) * torch.exp(-0.25 * r2 / 1e-4) + 1.0
    out = {}
    for name, prec in (("plain_fp64", cc.FP64), ("mixed", cc.MIXED)):
        plan = cc.Plan(cc.Problem(n=n, bc=("N",) * 4, alpha=1.0, beta=dt / 2, rtol=1e-10, prec=prec))
        phi, work = cc.field(n), cc.field(n)
        phi[1:n + 1, 1:n + 1] = g0
        cc.ccmg_plan_autotune(plan, phi, work)
        for _ in range(2):
            r = cc.ccmg_cn_step(plan, phi, work)
            assert r.status == cc.OK, r
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc = 0
        for _ in range(steps):
            r = cc.ccmg_cn_step(plan, phi, work)
            assert r.status == cc.OK, r
            cyc += r.cycles
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        cc.ccmg_plan_profile(plan, True)
        for _ in range(3):
            cc.ccmg_cn_step(plan, phi, work)
        st = {k["name"]: k for k in cc.ccmg_plan_kernel_stats(plan)}
        cc.ccmg_plan_profile(plan, False)
        # the right-hand side pass (FP64 solves with the fused launch form it in
        # their first pre-smoothing launch instead: no separate pass)
        k = st["cn_rhs"]
        rhs = None
        if k["launches"] > 0:
            avg = k["ms"] / k["launches"]
            rhs = dict(avg_ms=round(avg, 5), gbs=round(k["bytes"] / k["launches"] / (avg * 1e-3) / 1e9, 1))
        out[name] = dict(ms_per_step=round(1e3 * dt_s / steps, 3), cycles_per_step=cyc / steps,
                         cell_steps_per_s=n * n * steps / dt_s, cn_rhs=rhs)
        del plan, phi, work
        torch.cuda.empty_cache()
    out["speedup_mixed"] = round(out["plain_fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 3)
    rhs = out["mixed"]["cn_rhs"]
    log(f"CN diffusion 8192^2: plain {out['plain_fp64']['ms_per_step']} ms/step "
        f"({out['plain_fp64']['cycles_per_step']:.1f} cyc; right-hand side "
        f"{'in the first launch' if out['plain_fp64']['cn_rhs'] is None else 'a separate pass'}), "
        f"mixed {out['mixed']['ms_per_step']} ms/step" + (f", rhs kernel {rhs['gbs']} GB/s" if rhs else ""))
    return out


def side_data_solves(cc, torch, W, reps):
    """Inhomogeneous side data on the 4096^2 Fourier-mode right-hand side:
    Dirichlet values on x-lo / y-hi and Neumann derivatives on x-hi / y-lo
    (smooth periodic profiles along each side), time to 1e-10 against the same
    solve with homogeneous sides."""
    n = 4096
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    t = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n
    b = [torch.sin(2 * torch.pi * t) + 0.5, torch.cos(4 * torch.pi * t), 0.3 * torch.sin(6 * torch.pi * t),
         1.0 - t * 0.0]
    plan = cc.Plan(cc.Problem(n=n, bc=("D", "N", "N", "D"), rtol=1e-10))
    f = upload(cc, torch, fv)
    phi, work = cc.field(n), cc.field(n)
    cc.ccmg_plan_autotune(plan, f, phi)
    out = {}
    for name, data in (("homogeneous", None), ("with_data", b)):
        best, cyc = float("inf"), 0
        for _ in range(reps + 1):
            phi.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = cc.ccmg_solve_bc(plan, f, phi, data, work)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            assert r.status == cc.OK, r
            cyc = r.cycles
        out[name] = dict(ms=round(1e3 * best, 3), cycles=cyc)
    # (the tolerance is relative to the shifted right-hand side, which the data
    # enlarge: the two solves are different problems, not a speed comparison)
    log(f"side data 4096^2: homogeneous {out['homogeneous']['ms']} ms ({out['homogeneous']['cycles']} cycles), "
        f"with data {out['with_data']['ms']} ms ({out['with_data']['cycles']} cycles)")
    del plan, f, phi, work
    torch.cuda.empty_cache()
    return out


def bottom_solver(cc, torch, W, steps):
    """The bottom of the V-cycle on the 4096^2 periodic Poisson problem (FP64
    and mixed): 50 relaxations on 2 x 2 against an exact solve
    on 4 x 4 or 8 x 8 (inverse operator from LDS).  Time to 1e-10, best of
    two alternating rounds of `steps` solves each."""
    n = 4096
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    f = upload(cc, torch, fv)
    phi = cc.field(n)
    out = {}
    for pname, prec in (("fp64", cc.FP64), ("mixed", cc.MIXED)):
        plans = {}
        for nb in (2, 4, 8):
            plan = cc.Plan(cc.Problem(n=n, bc="P", rtol=1e-10, prec=prec))
            cc.ccmg_plan_set_bottom(plan, nb)
            cc.ccmg_plan_autotune(plan, f, phi)
            cc.ccmg_solve(plan, f, phi)
            plans[nb] = plan
        best = {nb: float("inf") for nb in plans}
        cyc = {}
        for _ in range(2):
            for nb, plan in plans.items():
                dt, res, _ = run_solves(cc, torch, plan, f, phi, steps)
                assert all(r.status == cc.OK and r.rel_resid <= 1e-10 for r in res)
                best[nb] = min(best[nb], 1e3 * dt / steps)
                cyc[nb] = res[-1].cycles
        out[pname] = {f"n_bottom_{nb}": dict(ms=round(best[nb], 4), cycles=cyc[nb]) for nb in plans}
        log(f"bottom 4096^2 {pname}: " + ", ".join(f"{nb}^2 {best[nb]:.3f} ms ({cyc[nb]} cyc)" for nb in plans))
        del plans
    del f, phi
    torch.cuda.empty_cache()
    return out


def projection(cc, torch, reps):
    """Cell-centred approximate projection on 4096^2 (doubly periodic): the
    paper's convergence field (Minion's divergence-free u, v) plus the
    gradient of 0.1 sin(2 pi x) cos(4 pi y); time per projection (divergence,
    Poisson solve to 1e-10, gradient correction) and the error against the
    divergence-free part."""
    n = 4096
    t = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n
    X, Y = t[None, :], t[:, None]
    ud = 1 - 2 * torch.cos(2 * np.pi * X) * torch.sin(2 * np.pi * Y)
    vd = 1 + 2 * torch.sin(2 * np.pi * X) * torch.cos(2 * np.pi * Y)
    gx = 0.2 * np.pi * torch.cos(2 * np.pi * X) * torch.cos(4 * np.pi * Y)
    gy = -0.4 * np.pi * torch.sin(2 * np.pi * X) * torch.sin(4 * np.pi * Y)
    plan = cc.Plan(cc.Problem(n=n, bc=("P",) * 4, rtol=1e-10))
    u, v, phi, work = (cc.field(n) for _ in range(4))
    u[1:n + 1, 1:n + 1] = ud + gx
    cc.ccmg_plan_autotune(plan, u, work)
    best, cyc = float("inf"), 0
    for rep in range(reps + 1):
        u[1:n + 1, 1:n + 1] = ud + gx
        v[1:n + 1, 1:n + 1] = vd + gy
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cc.ccmg_project(plan, u, v, phi, work)
        torch.cuda.synchronize()
        if rep > 0:
            best = min(best, time.perf_counter() - t0)
        assert r.status == cc.OK, r
        cyc = r.cycles
    err = max((u[1:n + 1, 1:n + 1] - ud).abs().max().item(), (v[1:n + 1, 1:n + 1] - vd).abs().max().item())
    cc.ccmg_plan_profile(plan, True)
    u[1:n + 1, 1:n + 1] = ud + gx
    v[1:n + 1, 1:n + 1] = vd + gy
    cc.ccmg_project(plan, u, v, phi, work)
    st = {k["name"]: k for k in cc.ccmg_plan_kernel_stats(plan)}
    cc.ccmg_plan_profile(plan, False)
    kern = {name: dict(avg_ms=round(st[name]["ms"] / st[name]["launches"], 5),
                       gbs=round(st[name]["bytes"] / st[name]["ms"] * 1e-6, 1))
            for name in ("divergence", "subtract_gradient")}
    out = dict(ms=round(1e3 * best, 3), cycles=cyc, max_error_vs_divergence_free=err, kernels=kern)
    log(f"projection 4096^2: {out['ms']} ms ({cyc} cycles), error {err:.2e}, "
        f"divergence {kern['divergence']['gbs']} GB/s, gradient {kern['subtract_gradient']['gbs']} GB/s")
    del plan, u, v, phi, work
    torch.cuda.empty_cache()
    return out


def batched_vs_sequential(cc, torch, W, reps):
    """The batched workload: 512 independent Poisson problems, sizes uniform in
    {32, ..., 1024}^2, per-axis periodic / Dirichlet sides, 16 seeded Fourier
    modes |k| <= 8 (zero mean), to 1e-10 -- one batched solve (graph-replayed
    steps, FP32 cycles + FP64 refinement) against the same 512 problems solved
    one after another with plain FP64 plans."""
    items = W.batch(seed=0)
    cells = sum(it.n * it.n for it in items)
    fs, phis = [], []
    for it in items:
        fs.append(upload(cc, torch, it.f))
        phis.append(cc.field(it.n))
    probs = [cc.Problem(n=it.n, bc=it.bc, rtol=1e-10, prec=cc.MIXED) for it in items]
    batch = cc.Batch(probs)
    cc.ccmg_batch_autotune(batch, fs, phis)
    shapes = cc.ccmg_batch_shapes(batch)
    res, info = cc.ccmg_batch_solve(batch, fs, phis)  # warm-up
    assert info["converged"] == len(items), info
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    for _ in range(reps):
        res, info = cc.ccmg_batch_solve(batch, fs, phis)
        steps += info["steps"]
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    assert info["converged"] == len(items) and all(r.rel_resid <= 1e-10 for r in res)
    del batch
    torch.cuda.empty_cache()
    # sequential plain FP64 solves (one plan per size and side pairing)
    plans = {}
    for it, f in zip(items, fs):
        key = (it.n, it.bc)
        if key not in plans:
            plans[key] = cc.Plan(cc.Problem(n=it.n, bc=it.bc, rtol=1e-10))
            cc.ccmg_plan_autotune(plans[key], f, cc.field(it.n))
    for it, f, phi in zip(items, fs, phis):  # warm-up
        cc.ccmg_solve(plans[(it.n, it.bc)], f, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_cycles = 0
    for it, f, phi in zip(items, fs, phis):
        r = cc.ccmg_solve(plans[(it.n, it.bc)], f, phi)
        assert r.status == cc.OK
        seq_cycles += r.cycles
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out = dict(problems=len(items), cells=cells, batched_ms=round(1e3 * tb, 3), batched_steps=steps // reps,
               sequential_plain_fp64_ms=round(1e3 * ts, 3), sequential_cycles=seq_cycles,
               speedup=round(ts / tb, 3), batched_cells_steps_per_s=cells * (steps / reps) / tb,
               shapes=shapes)
    log(f"batched 512: {1e3 * tb:.2f} ms ({steps // reps} steps) vs sequential plain {1e3 * ts:.2f} ms, "
        f"x{ts / tb:.2f}")
    del plans, fs, phis
    torch.cuda.empty_cache()
    return out


def learned_vs_plain(cc, torch, W, train_seeds, train_steps, eval_seeds=256):
    """The learned form: periodic Poisson 1024^2 with Gaussian-blob right-hand
    sides.  Training pairs from plain multigrid solves of seeds 0..train_seeds-1,
    training on the GPU, then time to 1e-10 (guess time included) on unseen
    seeds 100000..100000+eval_seeds-1 for: the zero guess, the learned guess,
    the learned guess's decoder run on a zero network output (network weights
    all zero), and k = 1, 2 V-cycles of the averaged problem on the network's
    grid plus the same prolongations (non-learned guesses of about the
    network's cost)."""
    from paper_1306_6883_amd import learned as L
    n = 1024
    net = L.new_net(batch=32, n_max=n, seed=0)
    plan = cc.Plan(L.periodic_poisson(n))
    t0 = time.perf_counter()
    data = L.make_dataset(net, n, range(train_seeds), plan=plan)
    t_data = time.perf_counter() - t0
    log(f"learned: {train_seeds} plain-MG training solves in {t_data:.1f} s ({data.cycles:.1f} cycles each)")
    t0 = time.perf_counter()
    hist = L.train(net, data, steps=train_steps, batch=32, lr=1e-3, lr_final=1e-5, warmup=200)
    t_train = time.perf_counter() - t0
    del data
    ev = L.make_dataset(net, n, range(100000, 100000 + eval_seeds), plan=plan)
    err = L.target_error(net, ev)
    del ev
    log(f"learned: {train_steps} Adam steps (batch 32) in {t_train:.1f} s, loss {hist[-1][1]:.3e}, "
        f"held-out error on the network grid {err:.4f}")
    cmp = L.compare_guesses(net, n, range(100000, 100000 + eval_seeds), plan=plan, reps=2)
    guesses = {k: dict(ms=round(float(np.mean(cmp.ms[k])), 4), cycles=round(float(np.mean(cmp.cycles[k])), 3),
                       guess_ms=round(cmp.guess_ms[k], 4)) for k in cmp.ms}
    mz = guesses["zero"]["ms"]
    for k, g in guesses.items():
        g["speedup_vs_zero"] = round(mz / g["ms"], 3)
    out = dict(n=n, train_solves=train_seeds, train_steps=train_steps, dataset_s=round(t_data, 1),
               train_s=round(t_train, 1), final_loss=hist[-1][1], heldout_error=round(err, 5),
               eval_seeds=f"100000..{100000 + eval_seeds - 1}", coarse_iters=cc.COARSE_ITERS,
               cycles_zero=guesses["zero"]["cycles"], cycles_learned=guesses["learned"]["cycles"],
               ms_zero=mz, ms_learned=guesses["learned"]["ms"], guess_ms=guesses["learned"]["guess_ms"],
               speedup=guesses["learned"]["speedup_vs_zero"], guesses=guesses, all_reached_tol=True)
    log("learned 1024^2 (" + out["eval_seeds"] + "): " +
        ", ".join(f"{k} {g['cycles']:.2f} cyc {g['ms']:.3f} ms (guess {g['guess_ms']:.3f})" for k, g in guesses.items()))
    del net, plan
    torch.cuda.empty_cache()
    return out


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
# counter summaries of the fused finest launch, per workload
PMC_SUMMARY = {8192: os.path.join(PROFILES, "march_finest_fused_dirichlet8192_pmc.md"),
               4096: os.path.join(PROFILES, "march_finest_fused_poisson4096_pmc.md")}


def measured_traffic(kernel: str, shape, summary: str):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's reading), or
    None when there is none, the kernel's sources changed since, or the
    autotuner chose another launch shape (rows per band, waves per workgroup)
    than the one the counters were taken with."""
    import hashlib
    try:
        text = open(summary).read()
    except (OSError, TypeError):
        return None
    fields = dict(re.findall(r"^\s+(\w+): (.+)$", text, flags=re.M))
    if fields.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for rel in fields.get("source_files", "").split():
        with open(os.path.join(root, rel), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != fields.get("source_sha256"):
        return None
    # one counter pair per launch shape the autotuner picks at this size
    key = f"traffic_bytes_per_launch_{shape[0]}_{shape[1]}" if shape is not None else None
    if key not in fields:
        return None
    return float(fields[key])


def roofline_of(meas):
    ks = [k for k in meas["kernels"] if k["launches"] > 0]
    dom = max(ks, key=lambda k: k["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom["name"], meas.get("fused_shape"), PMC_SUMMARY.get(meas["n"]))
    # the counters' bytes over the same launch time (HBM traffic actually moved)
    traffic_gbs = round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom["name"],
                avg_launch_ms=round(avg_ms, 5), bytes_per_launch=bytes_per_launch,
                traffic_gbs=traffic_gbs,
                traffic_frac=round(traffic_gbs / HBM_PEAK_GBS, 4) if traffic_gbs else None,
                all_kernels=[dict(name=k["name"], launches=k["launches"],
                                  avg_ms=round(k["ms"] / k["launches"], 5),
                                  gbs=round(k["bytes"] / k["launches"] / (k["ms"] / k["launches"] * 1e-3) / 1e9, 1))
                             for k in ks])


def cpu_baseline(fv, n, bc, budget_s=10.0):
    """The FP64 CPU oracle on a bounded sample of the same workload: whole
    solves to 1e-10 repeated until about `budget_s` seconds have passed (at
    least one)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p = oracle.Problem(n=n, h=1.0 / n, bc=bc, rtol=1e-10)
    f = oracle.embed(fv)
    solves = cycles = 0
    t0 = time.perf_counter()
    while True:
        _, r = oracle.solve(p, f)
        solves += 1
        cycles += r.cycles
        dt = time.perf_counter() - t0
        if dt >= budget_s or solves >= 50:
            break
    return {"value": n * n * cycles / dt, "unit": "grid-pts*V-cycles/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{solves} whole {n}^2 {SIDE_NAMES[bc]} solves to 1e-10 ({cycles} V(2,2) cycles), "
                      f"plain C + OpenMP, {dt:.1f} s ({dt / solves:.2f} s per solve)"}


SIDE_NAMES = {"DDDD": "Dirichlet", "PPPP": "periodic"}


def cpu_single_thread(fv, n, bc):
    """One whole oracle solve of the same problem on one thread (a child
    process with OMP_NUM_THREADS=1: the thread count is fixed when the
    OpenMP runtime starts), and the host's CPU model and thread count."""
    fpath = os.path.join(tempfile.mkdtemp(), "f.npy")
    np.save(fpath, fv)
    code = ("import sys, time, json, numpy as np, oracle; f = oracle.embed(np.load(sys.argv[1])); "
            "n = f.shape[0] - 2; p = oracle.Problem(n=n, h=1.0 / n, bc=sys.argv[2], rtol=1e-10); "
            "t = time.perf_counter(); _, r = oracle.solve(p, f); dt = time.perf_counter() - t; "
            "print(json.dumps([r.cycles, dt]))")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code, fpath, bc], env=env, capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.abspath(__file__)), timeout=300)
    os.remove(fpath)
    cycles, dt = json.loads(out.stdout.strip().splitlines()[-1])
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=n * n * cycles / dt, unit="grid-pts*V-cycles/s", threads=1,
                sample=f"one {n}^2 {SIDE_NAMES[bc]} solve to 1e-10 ({cycles} cycles), {dt:.1f} s",
                host_cpu=model, host_threads=os.cpu_count())


def stream_probe(cc, torch, n):
    """What this device's memory delivers for the fused launch's compulsory
    pattern: c = a + b over three FP64 arrays of n^2 values (the library's
    streaming probe: the fastest of its launch shapes, ordinary or
    nontemporal accesses, HIP events over 20 launches each)."""
    a = torch.full((n * n,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.full_like(a, 2.0)
    c = torch.empty_like(a)
    ms, cfg = cc.ccmg_probe_stream(a, b, c, reps=20)
    assert float(c[-1]) == 3.0
    gbs = 3 * 8 * n * n / (ms * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    return dict(n=n, bytes_per_launch=3 * 8 * n * n, ms=round(ms, 5), gbs=round(gbs, 1),
                frac_of_peak=round(gbs / HBM_PEAK_GBS, 4), workgroups_per_cu=cfg % 1000,
                nontemporal=cfg >= 1000)


def fmg_start(cc, torch, W, steps):
    """Time to 1e-10 from the full multigrid start (CCMG_OPT_FMG = 1: one
    V-cycle per level below the finest, starting from the coarse tail's
    32^2 level) against the plain zero start, on the headline problem (8192^2
    Dirichlet) and the 4096^2 periodic one; best of two alternating rounds of
    `steps` solves each."""
    out = {}
    for n, side, name in ((8192, "D", "dirichlet_8192"), (4096, "P", "periodic_4096")):
        fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
        f = upload(cc, torch, fv)
        phi = cc.field(n)
        plans = {}
        for mode in ("plain", "fmg"):
            plan = cc.Plan(cc.Problem(n=n, bc=side, rtol=1e-10))
            if mode == "fmg":
                cc.ccmg_plan_set_option(plan, cc.OPT_FMG, 1)
            cc.ccmg_plan_autotune(plan, f, phi)
            cc.ccmg_solve(plan, f, phi)
            plans[mode] = plan
        best = {k: float("inf") for k in plans}
        last = {}
        for _ in range(2):
            for mode, plan in plans.items():
                dt, res, _ = run_solves(cc, torch, plan, f, phi, steps)
                assert all(r.status == cc.OK and r.rel_resid <= 1e-10 for r in res)
                best[mode] = min(best[mode], 1e3 * dt / steps)
                last[mode] = res[-1]
        out[name] = {mode: dict(ms=round(best[mode], 4), cycles=last[mode].cycles,
                                rel_resid0=last[mode].rel_resid0, rel_resid=last[mode].rel_resid) for mode in plans}
        out[name]["speedup"] = round(best["plain"] / best["fmg"], 3)
        log(f"FMG start {n}^2 {side}: plain {best['plain']:.3f} ms ({last['plain'].cycles} cyc), "
            f"FMG {best['fmg']:.3f} ms ({last['fmg'].cycles} cyc), x{out[name]['speedup']}")
        del plans, f, phi
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the headline workload (no other legs)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess leg")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned-guess leg and print its result (profiling aid)")
    ap.add_argument("--learned-solves", type=int, default=20000, help="training solves of the learned leg")
    ap.add_argument("--learned-steps", type=int, default=30000, help="training steps of the learned leg")
    ap.add_argument("--learned-eval", type=int, default=256, help="held-out seeds the learned leg evaluates on")
    ap.add_argument("--next-rows-only", action="store_true",
                    help="only the Crank-Nicolson, side-data and projection legs (one JSON line of their own)")
    ap.add_argument("--fmg-only", action="store_true",
                    help="only the full multigrid start leg (one JSON line of its own; profiling aid)")
    ap.add_argument("--fused-shape", type=str, default=None,
                    help="TY,WPB: rows per band and waves per workgroup of the headline's fused launch, "
                         "instead of the autotuner's choice (for counter runs)")
    ap.add_argument("--workload", choices=("dirichlet8192", "periodic4096"), default="dirichlet8192",
                    help="the measured workload of a --quick run (counter runs of the 4096^2 line)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not part of it"}))
        sys.exit(2)

    import torch
    import paper_1306_6883_amd as cc
    import workloads as W

    torch.cuda.set_device(0)
    if args.probe_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
        del a, b

    if args.learned_only:
        print(json.dumps({"learned": learned_vs_plain(cc, torch, W, args.learned_solves, args.learned_steps,
                                                      args.learned_eval)}), flush=True)
        return
    if args.fmg_only:
        print(json.dumps({"fmg_start": fmg_start(cc, torch, W, 10)}), flush=True)
        return
    if args.next_rows_only:
        print(json.dumps({"cn_diffusion": cn_diffusion(cc, torch, 10), "side_data": side_data_solves(cc, torch, W, 5),
                          "projection": projection(cc, torch, 5), "bottom_solver": bottom_solver(cc, torch, W, 20),
                          "fmg_start": fmg_start(cc, torch, W, 10)}),
              flush=True)
        return
    if args.workload == "periodic4096" and not args.quick:
        print(json.dumps({"error": "--workload periodic4096 is for --quick counter runs"}))
        sys.exit(2)
    n, side = (8192, "D") if args.workload == "dirichlet8192" else (4096, "P")
    log("generating inputs")
    f_head = W.fourier_modes(n, seed=0, count=64, kmax=32)

    log(f"{n}^2 {'Dirichlet' if side == 'D' else 'periodic'}: {args.warmup} warmup + {args.steps} timed solves")
    fshape = tuple(int(x) for x in args.fused_shape.split(",")) if args.fused_shape else None
    m = measure(cc, torch, n, side, f_head, args.steps, args.warmup, fused_shape=fshape)
    log(f"{m['ms_per_solve']:.3f} ms/solve, {m['cycles_per_solve']:.1f} cycles, "
        f"{m['pts_cycles_per_s'] / 1e9:.2f} G pts*cycles/s")
    rl = roofline_of(m)
    log(f"dominant kernel {rl['kernel']} {m['fused_shape']}: {rl['avg_launch_ms']:.4f} ms, {rl['achieved']} GB/s "
        f"({rl['frac']:.3f})" + (f"; counter bytes {rl['traffic_gbs']} GB/s ({rl['traffic_frac']:.3f})"
                                  if rl["traffic_gbs"] else ""))

    also = {}
    if not args.quick:
        also["stream_probe"] = [stream_probe(cc, torch, k) for k in (8192, 4096)]
        log("stream probe (read 2, write 1): " + ", ".join(f"{p['n']}^2 {p['gbs']} GB/s" for p in also["stream_probe"]))
        n4 = 4096
        f4 = W.fourier_modes(n4, seed=0, count=64, kmax=32)
        log(f"{n4}^2 periodic: {args.warmup} warmup + {args.steps} timed solves")
        m4 = measure(cc, torch, n4, "P", f4, args.steps, args.warmup)
        rl4 = roofline_of(m4)
        also["periodic_4096"] = dict(ms_per_solve=round(m4["ms_per_solve"], 4),
                                     cycles_per_solve=m4["cycles_per_solve"],
                                     value=m4["pts_cycles_per_s"], rel_resid=m4["rel_resid"],
                                     roofline=rl4, fused_shape=m4["fused_shape"], visits=m4["visits"])
        log(f"{n4}^2: {m4['ms_per_solve']:.3f} ms/solve, {m4['pts_cycles_per_s'] / 1e9:.2f} G; "
            f"{rl4['kernel']} {rl4['achieved']} GB/s" +
            (f", counter bytes {rl4['traffic_gbs']} GB/s" if rl4["traffic_gbs"] else ""))
        del f4
        also["mixed_precision"] = mixed_vs_plain(cc, torch, W, max(args.steps // 4, 3))
        also["batched"] = batched_vs_sequential(cc, torch, W, 3)
        also["cn_diffusion"] = cn_diffusion(cc, torch, 10)
        also["side_data"] = side_data_solves(cc, torch, W, 5)
        also["projection"] = projection(cc, torch, 5)
        also["bottom_solver"] = bottom_solver(cc, torch, W, 20)
        also["fmg_start"] = fmg_start(cc, torch, W, 10)
        if not args.no_learned:
            also["learned"] = learned_vs_plain(cc, torch, W, args.learned_solves, args.learned_steps,
                                               args.learned_eval)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle sample")
        cpu = cpu_baseline(f_head, n, "DDDD")
        log(f"oracle: {cpu['value'] / 1e9:.3f} G pts*cycles/s on {cpu['cores']} threads ({cpu['sample']})")
        if not args.quick:
            also["cpu_oracle_1_thread"] = cpu_single_thread(f_head, n, "DDDD")
            log(f"oracle, 1 thread: {also['cpu_oracle_1_thread']['value'] / 1e9:.3f} G pts*cycles/s "
                f"({also['cpu_oracle_1_thread']['host_cpu']})")

    line = {
        "metric": "time-to-1e-10 residual & grid-pts*V-cycles/s (HBM % peak), plain vs mixed/batched/learned",
        "value": m["pts_cycles_per_s"],
        "unit": "grid-pts*V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain FP64 V(2,2) Poisson {n}^2 "
                               f"{'homogeneous Dirichlet' if side == 'D' else 'periodic'}, 64 Fourier modes |k|<=32, "
                               "seed 0, to relative residual 1e-10",
                   "n": n, "bc": "Dirichlet" if side == "D" else "periodic", "rtol": 1e-10,
                   "cycles_per_solve": m["cycles_per_solve"], "time_to_tol_ms": m["ms_per_solve"]},
        "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": {k: rl[k] for k in ("kernel", "avg_launch_ms", "bytes_per_launch", "traffic_gbs", "traffic_frac",
                                                        "all_kernels")},
        "launch_shapes": {"levels": "finest first; (rows per band, waves per workgroup) of the nu1 and nu2 launches",
                          "value": m["shapes"], "fused": m["fused_shape"],
                          "visits": "levels 1, 2, ...: shape of the visit launch, (0, 1) where the level runs "
                                    "its two launches", "visit_value": m["visits"]},
        "cpu_baseline": cpu,
        "also": also,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

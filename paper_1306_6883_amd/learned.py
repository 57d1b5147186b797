"""Training and evaluation of the learned initial guess.

The network (six linear dilated 3x3 convolutions on a 128 x 128 grid, see
include/ccmg.h) learns the map from a right-hand side to the solution of the
periodic Poisson problem, both averaged onto its grid and divided by the RMS
of the right-hand side.  Its training pairs come from the plain multigrid
solver itself; every solve, encode, forward, backward, Adam step and guess
runs in the library's kernels.  PyTorch only holds the device arrays and makes
the synthetic right-hand sides.

The guess is then used by ccmg_solve_learned: plain multigrid continues from
it to the same tolerance, so a poor guess costs cycles, never accuracy.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

import workloads as W

from . import (NET_G, OK, Net, Plan, Problem, ccmg_net_encode, ccmg_net_forward, ccmg_net_get_params,
               ccmg_net_guess, ccmg_net_param_count, ccmg_net_set_params, ccmg_net_train_step,
               ccmg_plan_autotune, ccmg_solve, ccmg_solve_learned, field)

# layer shapes in parameter order: (out channels, taps, in channels)
_LAYERS = [(32, 9, 1), (32, 9, 32), (32, 9, 32), (32, 9, 32), (32, 9, 32), (1, 9, 32)]


def periodic_poisson(n: int, rtol: float = 1e-10) -> Problem:
    """The learned form's problem: Lap phi = f on the unit square, periodic
    (alpha = 0, beta = -1 in (alpha - beta Lap) phi = f)."""
    return Problem(n=n, bc="P", alpha=0.0, beta=-1.0, rtol=rtol)


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """Random parameters: each layer N(0, 1 / fan_in) so that the linear stack
    keeps the input's scale."""
    g = np.random.default_rng(np.random.SeedSequence([0x6E6574, seed]))
    parts = [g.normal(0.0, 1.0 / math.sqrt(k * ci), size=co * k * ci) for co, k, ci in _LAYERS]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == ccmg_net_param_count()
    return torch.as_tensor(p, device=device)


@dataclass
class Dataset:
    x: torch.Tensor       # [S, G, G] encoded right-hand sides
    t: torch.Tensor       # [S, G, G] encoded solutions (same scale as x's source)
    seeds: list
    solve_ms: float       # total time of the plain solves that made the targets
    cycles: float         # mean V-cycles per solve


def make_dataset(net: Net, n: int, seeds, chunk: int = 64, plan: Plan | None = None,
                 log=None) -> Dataset:
    """Solve the blob problem of every seed with plain multigrid (zero guess)
    and encode (f, phi) for the network."""
    seeds = list(seeds)
    dev = net.device
    plan = plan or Plan(periodic_poisson(n), device=dev)
    X = torch.empty((len(seeds), NET_G, NET_G), dtype=torch.float32, device=dev)
    T = torch.empty_like(X)
    f = field(n, device=dev)
    phi = field(n, device=dev)
    tuned = False
    total_ms, cyc = 0.0, 0
    t0 = time.time()
    for c0 in range(0, len(seeds), chunk):
        F = W.gaussian_blobs_torch(n, seeds[c0:c0 + chunk], device=dev)
        for i in range(F.shape[0]):
            f[1:n + 1, 1:n + 1] = F[i]
            if not tuned:
                ccmg_plan_autotune(plan, f, phi)
                tuned = True
            r = ccmg_solve(plan, f, phi)
            if r.status != OK:
                raise RuntimeError(f"plain multigrid did not converge for seed {seeds[c0 + i]}: {r}")
            total_ms += r.ms
            cyc += r.cycles
            k = c0 + i
            ccmg_net_encode(net, f, f, X[k])
            ccmg_net_encode(net, phi, f, T[k])
        if log and (c0 // chunk) % 50 == 0:
            log(f"dataset {c0 + F.shape[0]}/{len(seeds)} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize(dev)
    return Dataset(X, T, seeds, total_ms, cyc / max(1, len(seeds)))


def train(net: Net, data: Dataset, steps: int, batch: int = 32, lr: float = 1e-3, lr_final: float = 1e-5,
          warmup: int = 100, seed: int = 0, log=None, log_every: int = 250):
    """Adam with a linear warm-up then a cosine decay; minibatches drawn without
    replacement each epoch.  Returns the loss history [(step, loss)]."""
    S = data.x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(S, generator=g)
    pos = 0
    hist = []
    xb = torch.empty((batch, NET_G, NET_G), dtype=torch.float32, device=net.device)
    tb = torch.empty_like(xb)
    t0 = time.time()
    for k in range(steps):
        if pos + batch > S:
            perm = torch.randperm(S, generator=g)
            pos = 0
        idx = perm[pos:pos + batch].to(net.device)
        pos += batch
        torch.index_select(data.x, 0, idx, out=xb)
        torch.index_select(data.t, 0, idx, out=tb)
        if k < warmup:
            rate = lr * (k + 1) / warmup
        else:
            u = (k - warmup) / max(1, steps - warmup)
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * u))
        want = (k % log_every == 0) or k == steps - 1
        loss = ccmg_net_train_step(net, xb, tb, rate, want_loss=want)
        if want:
            hist.append((k, loss))
            if log:
                log(f"step {k} loss {loss:.4e} lr {rate:.2e} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize(net.device)
    return hist


def target_error(net: Net, data: Dataset, batch: int | None = None) -> float:
    """Relative L2 error of the network against the encoded targets."""
    b = batch or net.batch
    num = den = 0.0
    for c0 in range(0, data.x.shape[0], b):
        x = data.x[c0:c0 + b].contiguous()
        y = ccmg_net_forward(net, x)
        t = data.t[c0:c0 + b]
        num += float(((y - t) ** 2).sum())
        den += float((t ** 2).sum())
    return math.sqrt(num / den)


@dataclass
class Comparison:
    seeds: list
    cycles_zero: list
    cycles_learned: list
    ms_zero: list
    ms_learned: list
    guess_error: list     # ||guess - phi|| / ||phi|| at full resolution (means removed)
    rel_resid_guess: list
    used: list


def compare(net: Net, n: int, seeds, plan: Plan | None = None, reps: int = 1) -> Comparison:
    """Time to tolerance from a zero guess against the learned solve (guess
    time included), on the same problems and the same plan."""
    dev = net.device
    plan = plan or Plan(periodic_poisson(n), device=dev, stream=net.stream)
    f = field(n, device=dev)
    phi = field(n, device=dev)
    phi_ref = field(n, device=dev)
    out = Comparison(list(seeds), [], [], [], [], [], [], [])
    for s in seeds:
        f[1:n + 1, 1:n + 1] = W.gaussian_blobs_torch(n, [s], device=dev)[0]
        best_z = best_l = float("inf")
        for _ in range(reps):
            phi_ref.zero_()
            rz = ccmg_solve(plan, f, phi_ref)
            best_z = min(best_z, rz.ms)
            phi.zero_()
            rl, used = ccmg_solve_learned(plan, net, f, phi)
            best_l = min(best_l, rl.ms)
        if rz.status != OK or rl.status != OK:
            raise RuntimeError(f"seed {s}: zero-guess status {rz.status}, learned status {rl.status}")
        # the guess alone, for its error
        g = field(n, device=dev)
        ccmg_net_guess(net, f, g)
        gv = g[1:n + 1, 1:n + 1]
        pv = phi_ref[1:n + 1, 1:n + 1]
        d = (gv - gv.mean()) - (pv - pv.mean())
        out.guess_error.append(float(d.norm() / (pv - pv.mean()).norm()))
        out.cycles_zero.append(rz.cycles)
        out.cycles_learned.append(rl.cycles)
        out.ms_zero.append(best_z)
        out.ms_learned.append(best_l)
        out.rel_resid_guess.append(rl.rel_resid0)
        out.used.append(used)
    return out


def params_of(net: Net) -> torch.Tensor:
    return ccmg_net_get_params(net)


def new_net(batch: int = 32, n_max: int = 1024, seed: int = 0, device=None) -> Net:
    net = Net(batch=batch, n_max=n_max, device=device)
    ccmg_net_set_params(net, init_params(seed, device=net.device))
    return net

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
               ccmg_net_get_state, ccmg_net_guess, ccmg_net_param_count, ccmg_net_set_params, ccmg_net_set_state,
               ccmg_net_train_step,
               ccmg_plan_autotune, ccmg_prolong_add, ccmg_restrict, ccmg_solve, ccmg_solve_learned, ccmg_vcycle,
               field)

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
          warmup: int = 100, seed: int = 0, log=None, log_every: int = 250, start: int = 0,
          stop: int | None = None, checkpoint: str | None = None, checkpoint_every: int = 0):
    """Adam with a linear warm-up then a cosine decay over `steps` steps;
    minibatches drawn without replacement, a fresh permutation per epoch
    (seeded by the epoch).  Runs steps start .. stop - 1 of that schedule
    (stop defaults to steps): a net restored with load_checkpoint at step
    `start` continues exactly as an uninterrupted run would.  With
    `checkpoint`, the state is saved there every `checkpoint_every` steps and
    at the end.  Returns the loss history [(step, loss)]."""
    S = data.x.shape[0]
    per_epoch = S // batch
    if per_epoch < 1:
        raise ValueError("fewer training samples than one batch")
    hist = []
    xb = torch.empty((batch, NET_G, NET_G), dtype=torch.float32, device=net.device)
    tb = torch.empty_like(xb)
    t0 = time.time()
    perm, epoch = None, -1
    stop = steps if stop is None else stop
    for k in range(start, stop):
        e = k // per_epoch
        if e != epoch:
            epoch = e
            g = torch.Generator(device="cpu").manual_seed(seed * 1000003 + epoch)
            perm = torch.randperm(S, generator=g)
        pos = (k % per_epoch) * batch
        idx = perm[pos:pos + batch].to(net.device)
        torch.index_select(data.x, 0, idx, out=xb)
        torch.index_select(data.t, 0, idx, out=tb)
        if k < warmup:
            rate = lr * (k + 1) / warmup
        else:
            u = (k - warmup) / max(1, steps - warmup)
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * u))
        want = (k % log_every == 0) or k == stop - 1
        loss = ccmg_net_train_step(net, xb, tb, rate, want_loss=want)
        if want:
            hist.append((k, loss))
            if log:
                log(f"step {k} loss {loss:.4e} lr {rate:.2e} ({time.time() - t0:.1f} s)")
        if checkpoint and checkpoint_every and (k + 1) % checkpoint_every == 0:
            save_checkpoint(net, checkpoint)
    if checkpoint:
        save_checkpoint(net, checkpoint)
    torch.cuda.synchronize(net.device)
    return hist


def save_checkpoint(net: Net, path: str) -> None:
    """Parameters, Adam moments and step counter to an .npz file (plain
    arrays, no pickled objects)."""
    state, step = ccmg_net_get_state(net)
    torch.cuda.synchronize(net.device)
    tmp = path + ".tmp.npz"
    np.savez(tmp, state=state.cpu().numpy(), step=np.array([step], dtype=np.int64))
    import os
    os.replace(tmp, path)


def load_checkpoint(net: Net, path: str) -> int:
    """Restore a state saved by save_checkpoint; returns its step counter."""
    with np.load(path, allow_pickle=False) as z:
        state = torch.as_tensor(z["state"], dtype=torch.float32).to(net.device).contiguous()
        step = int(z["step"][0])
    ccmg_net_set_state(net, state, step)
    torch.cuda.synchronize(net.device)
    return step


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


@dataclass
class GuessComparison:
    """Time to tolerance (guess included) and V-cycles per problem for each
    way of starting the solve, and each guess's own cost."""
    seeds: list
    ms: dict          # name -> [ms per seed]
    cycles: dict      # name -> [cycles per seed]
    guess_ms: dict    # name -> median ms of the guess alone


class CoarseGuess:
    """A non-learned guess of the same shape as the learned one: the right-hand
    side averaged onto the network's grid (multigrid restriction), k V-cycles
    of the Poisson problem there from zero, then multigrid prolongations back
    to the full grid -- every step through the library's entry points."""

    def __init__(self, plan: Plan, k: int):
        n = plan.n
        self.plan, self.k, self.n = plan, k, n
        self.levels = int(round(math.log2(n // NET_G)))
        dev = plan.workspace.device
        self.coarse_plan = Plan(periodic_poisson(NET_G), device=dev, stream=plan.stream)
        self.f = [None] + [field(n >> l, device=dev) for l in range(1, self.levels + 1)]
        self.e = [None] + [field(n >> l, device=dev) for l in range(1, self.levels + 1)]
        self.zero = [field(n >> l, device=dev) for l in range(self.levels)]

    def __call__(self, f: torch.Tensor, phi: torch.Tensor) -> None:
        L = self.levels
        src = f
        for l in range(L):
            ccmg_restrict(self.plan, l, src, self.f[l + 1])
            src = self.f[l + 1]
        self.e[L].zero_()
        for _ in range(self.k):
            ccmg_vcycle(self.coarse_plan, self.f[L], self.e[L])
        for l in range(L - 1, -1, -1):
            ccmg_prolong_add(self.plan, l, self.e[l + 1], self.zero[l], phi if l == 0 else self.e[l])


def compare_guesses(net: Net, n: int, seeds, plan: Plan | None = None, reps: int = 1, coarse_k=(1, 2)):
    """Zero guess, the learned guess, the learned guess's decoder run on a zero
    network output (a network with all weights zero: 32 relaxations on the
    network's grid, then the prolongations), and k V-cycles of the averaged
    problem on the network's grid plus the prolongations: the time to
    tolerance of each (guess included) and its V-cycles, on the same
    problems and the same plan."""
    dev = net.device
    plan = plan or Plan(periodic_poisson(n), device=dev, stream=net.stream)
    zero_net = Net(batch=1, n_max=n, device=dev, stream=net.stream)
    ccmg_net_set_params(zero_net, torch.zeros(ccmg_net_param_count(), dtype=torch.float32, device=dev))
    coarse = {k: CoarseGuess(plan, k) for k in coarse_k}
    f = field(n, device=dev)
    phi = field(n, device=dev)
    names = ["zero", "learned", "decoder_only"] + [f"coarse_vcycles_{k}" for k in coarse_k]
    out = GuessComparison(list(seeds), {k: [] for k in names}, {k: [] for k in names}, {})
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gtimes = {k: [] for k in names}

    def timed_guess(fn):
        e0.record(plan.stream)
        fn()
        e1.record(plan.stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    with torch.cuda.stream(plan.stream):
        for s in seeds:
            f[1:n + 1, 1:n + 1] = W.gaussian_blobs_torch(n, [s], device=dev)[0]
            best = {k: float("inf") for k in names}
            cyc = {}
            for _ in range(reps):
                phi.zero_()
                r = ccmg_solve(plan, f, phi)
                best["zero"] = min(best["zero"], r.ms)
                cyc["zero"] = r.cycles
                for name, nt in (("learned", net), ("decoder_only", zero_net)):
                    phi.zero_()
                    r, used = ccmg_solve_learned(plan, nt, f, phi)
                    if not used:
                        raise RuntimeError(f"seed {s}: {name} guess discarded")
                    best[name] = min(best[name], r.ms)
                    cyc[name] = r.cycles
                for k, g in coarse.items():
                    name = f"coarse_vcycles_{k}"
                    phi.zero_()
                    gms = timed_guess(lambda: g(f, phi))
                    r = ccmg_solve(plan, f, phi, use_guess=True)
                    if r.status != OK:
                        raise RuntimeError(f"seed {s}: {name} status {r.status}")
                    best[name] = min(best[name], gms + r.ms)
                    cyc[name] = r.cycles
                    gtimes[name].append(gms)
                for name, nt in (("learned", net), ("decoder_only", zero_net)):
                    gtimes[name].append(timed_guess(lambda: ccmg_net_guess(nt, f, phi)))
            for k in names:
                out.ms[k].append(best[k])
                out.cycles[k].append(cyc[k])
    out.guess_ms = {k: float(np.median(v)) for k, v in gtimes.items() if v}
    out.guess_ms["zero"] = 0.0
    return out


def params_of(net: Net) -> torch.Tensor:
    return ccmg_net_get_params(net)


def new_net(batch: int = 32, n_max: int = 1024, seed: int = 0, device=None) -> Net:
    net = Net(batch=batch, n_max=n_max, device=device)
    ccmg_net_set_params(net, init_params(seed, device=net.device))
    return net

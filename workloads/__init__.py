"""Seeded synthetic inputs for the multigrid workloads.

Shared by the tests, the smoke check and the benchmark, and by both the HIP
path and the CPU oracle.  This module only draws and evaluates right-hand
sides; it contains none of the solver's arithmetic.

Every generator returns float64 arrays of valid cells indexed [j, i]
(y rows, x contiguous) with cell centres x_i = xmin + (i + 1/2) h.  Random
numbers come from ``numpy.random.default_rng(SeedSequence([workload_id, seed]))``
so a (workload, seed) pair always yields the same bytes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# workload ids used in the seed sequence
W_SINE_NOISE = 1
W_FOURIER = 2
W_GRF = 3
W_BATCH = 4
W_BLOBS = 5


def rng(workload: int, seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([workload, seed]))


def centres(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


def sine_noise(n: int, seed: int = 0, sigma: float = 1e-2) -> np.ndarray:
    """Dirichlet unit-square workload: f = Lap of sin(2 pi x) sin(2 pi y) at cell
    centres plus i.i.d. N(0, sigma^2) noise per cell."""
    x = centres(n)
    s = np.sin(2 * np.pi * x)
    f = -8.0 * np.pi**2 * np.outer(s, s)
    return f + rng(W_SINE_NOISE, seed).normal(0.0, sigma, size=(n, n))


def _modes(r: np.random.Generator, count: int, kmax: int):
    """`count` distinct integer wave vectors with 0 < |k| <= kmax, k and -k
    identified; amplitudes N(0, 1); phases U[0, 2 pi)."""
    cand = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
            if 0 < kx * kx + ky * ky <= kmax * kmax and (kx > 0 or (kx == 0 and ky > 0))]
    idx = r.choice(len(cand), size=count, replace=False)
    ks = np.array([cand[i] for i in idx], dtype=np.int64)
    amp = r.normal(0.0, 1.0, size=count)
    ph = r.uniform(0.0, 2 * np.pi, size=count)
    return ks, amp, ph


def fourier_modes(n: int, seed: int = 0, count: int = 64, kmax: int = 32,
                  workload: int = W_FOURIER) -> np.ndarray:
    """Sum of `count` seeded Fourier modes a cos(2 pi k.x + theta), zero discrete mean.
    Evaluated separably as a rank-2*count product so large n stays cheap."""
    ks, amp, ph = _modes(rng(workload, seed), count, kmax)
    x = centres(n)
    ax = 2 * np.pi * np.outer(ks[:, 0], x) + ph[:, None]     # (count, n) in x
    ay = 2 * np.pi * np.outer(ks[:, 1], x)                   # (count, n) in y
    # cos(ax + ay) = cos ax cos ay - sin ax sin ay ; f[j, i] = sum_m a_m (...)
    left = np.concatenate([np.cos(ay), -np.sin(ay)], axis=0).T          # (n, 2c) over y
    right = np.concatenate([amp[:, None] * np.cos(ax), amp[:, None] * np.sin(ax)], axis=0)
    f = left @ right
    return f - f.mean()


def gaussian_random_field(n: int, seed: int = 0, corr: float = 0.05) -> np.ndarray:
    """White noise filtered by exp(-(2 pi |k| corr)^2 / 4) (Gaussian covariance
    exp(-r^2 / (2 corr^2))), scaled to unit standard deviation."""
    w = rng(W_GRF, seed).standard_normal((n, n))
    W = np.fft.rfft2(w)
    ky = np.fft.fftfreq(n, d=1.0 / n)[:, None]
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, :]
    W *= np.exp(-((2 * np.pi * corr) ** 2) * (kx * kx + ky * ky) / 4.0)
    g = np.fft.irfft2(W, s=(n, n))
    return (g - g.mean()) / g.std()


def blob_params(seed: int):
    """(centres [nb, 2], widths [nb], amplitudes [nb]) of the blob workload."""
    r = rng(W_BLOBS, seed)
    nb = int(r.integers(1, 9))
    c = r.uniform(0.0, 1.0, size=(nb, 2))
    w = r.uniform(0.01, 0.1, size=nb)
    a = r.normal(0.0, 1.0, size=nb)
    return c, w, a


def gaussian_blobs(n: int, seed: int) -> np.ndarray:
    """Periodic sum of 1-8 Gaussian blobs (uniform centres, widths U[0.01, 0.1],
    amplitudes N(0, 1)), minimum-image distance, zero mean."""
    c, w, a = blob_params(seed)
    nb = len(a)
    x = centres(n)
    f = np.zeros((n, n))
    for b in range(nb):
        dx = x - c[b, 0]
        dx -= np.round(dx)
        dy = x - c[b, 1]
        dy -= np.round(dy)
        f += a[b] * np.outer(np.exp(-dy**2 / (2 * w[b] ** 2)), np.exp(-dx**2 / (2 * w[b] ** 2)))
    return f - f.mean()


def gaussian_blobs_torch(n: int, seeds, device="cuda"):
    """gaussian_blobs for several seeds at once, built on a torch device:
    a [len(seeds), n, n] float64 tensor (the same fields up to rounding)."""
    import torch

    ps = [blob_params(s) for s in seeds]
    m = max(len(p[2]) for p in ps)
    C = np.zeros((len(ps), m, 2))
    Wd = np.ones((len(ps), m))
    A = np.zeros((len(ps), m))
    for i, (c, w, a) in enumerate(ps):
        C[i, :len(a)], Wd[i, :len(a)], A[i, :len(a)] = c, w, a
    dev = torch.device(device)
    C, Wd, A = (torch.as_tensor(v, device=dev) for v in (C, Wd, A))
    x = torch.as_tensor(centres(n), device=dev)
    dx = x[None, None, :] - C[:, :, 0:1]
    dx = dx - torch.round(dx)
    dy = x[None, None, :] - C[:, :, 1:2]
    dy = dy - torch.round(dy)
    gx = torch.exp(-dx**2 / (2 * Wd[:, :, None] ** 2))                 # [B, m, n]
    gy = torch.exp(-dy**2 / (2 * Wd[:, :, None] ** 2)) * A[:, :, None]
    f = torch.bmm(gy.transpose(1, 2).contiguous(), gx.contiguous())    # [B, n(y), n(x)]
    return f - f.mean(dim=(1, 2), keepdim=True)


@dataclass
class BatchItem:
    n: int
    bc: tuple          # (xlo, xhi, ylo, yhi) as 'P' / 'D'
    f: np.ndarray


def batch_sizes(seed: int, count: int = 512, sizes=(32, 64, 128, 256, 512, 1024)):
    """Sizes and BCs of the batched workload, without the right-hand sides."""
    r = rng(W_BATCH, seed)
    ns = r.choice(np.array(sizes), size=count)
    bx = r.integers(0, 2, size=count)
    by = r.integers(0, 2, size=count)
    out = []
    for i in range(count):
        ax = "P" if bx[i] == 0 else "D"
        ay = "P" if by[i] == 0 else "D"
        out.append((int(ns[i]), (ax, ax, ay, ay)))
    return out


def batch(seed: int = 0, count: int = 512, sizes=(32, 64, 128, 256, 512, 1024),
          modes: int = 16, kmax: int = 8) -> list:
    """Batched workload: per problem a size, per-axis periodic/Dirichlet BC and
    `modes` Fourier modes with |k| <= kmax (zero mean)."""
    items = []
    for i, (n, bc) in enumerate(batch_sizes(seed, count, sizes)):
        f = fourier_modes(n, seed=seed * 100003 + i, count=modes, kmax=kmax, workload=W_BATCH)
        items.append(BatchItem(n, bc, f))
    return items

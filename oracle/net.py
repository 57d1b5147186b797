"""FP64 NumPy oracle of the learned initial guess's network (TEST
INFRASTRUCTURE ONLY; part of the oracle, shares nothing with the HIP path).

Network: six 3x3 convolutions with circular padding and dilations
1, 2, 4, 8, 16, 32 on a G x G grid, channels 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1,
no biases, no activations (the map right-hand side -> solution is linear).
A convolution here is the cross-correlation

    out[y, x, co] = sum_{tap, ci} W[co, tap, ci] * in[y + dy(tap) d, x + dx(tap) d, ci]

with tap = 3 (dy + 1) + (dx + 1), indices taken modulo G.  Loss: mean squared
error.  `bf=True` applies the roundings of the GPU path (bfloat16, round to
nearest even), with sums kept in FP64.  Forward: the first and last layers'
weights unrounded; those of the 32 -> 32 layers carried as a bfloat16 pair
(hi = bf16(w), lo = bf16(w - hi)) whose lo part multiplies only the
activations' hi part; the activations between layers carried as a pair of
bfloat16 values (hi = bf16(v), lo = bf16(v - hi)); the network input
unrounded.  Backward: weights rounded to bfloat16 (hi only); the output
gradient and the back-propagated activation gradients rounded to bfloat16;
the weight gradients of the 32 -> 32 layers formed from the activations'
hi parts, those of the first and last layer from the full input / pair.

Parameter vector layout: W1 [32, 9], W2..W5 [32, 9, 32], W6 [9, 32].
"""
from __future__ import annotations

import numpy as np

G = 128
C = 32
DIL = [1, 2, 4, 8, 16, 32]
TAPS = [(ty - 1, tx - 1) for ty in range(3) for tx in range(3)]
SIZES = [C * 9] + [C * 9 * C] * 4 + [9 * C]


def param_count() -> int:
    return sum(SIZES)


def split(params: np.ndarray):
    """Parameter vector -> list of weight arrays with shapes [Cout, 9, Cin]."""
    out, o = [], 0
    for l, sz in enumerate(SIZES):
        w = params[o:o + sz]
        o += sz
        if l == 0:
            out.append(w.reshape(C, 9, 1))
        elif l == 5:
            out.append(w.reshape(9, C).reshape(1, 9, C))
        else:
            out.append(w.reshape(C, 9, C))
    return out


def join(ws) -> np.ndarray:
    parts = []
    for l, w in enumerate(ws):
        parts.append(w.reshape(C, 9) if l == 0 else (w.reshape(9, C) if l == 5 else w.reshape(-1)))
    return np.concatenate([p.reshape(-1) for p in parts])


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (through float32, round to nearest even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_pair(a: np.ndarray) -> np.ndarray:
    """v carried as hi + lo, both bfloat16 (about 16 significant bits)."""
    hi = bf16(a)
    return hi + bf16(np.asarray(a, dtype=np.float64) - hi)


def shifted(a: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[b, y, x] = a[b, (y + dy) % G, (x + dx) % G]."""
    return np.roll(a, shift=(-dy, -dx), axis=(1, 2))


def conv(a: np.ndarray, w: np.ndarray, d: int) -> np.ndarray:
    """a: [B, G, G, Cin], w: [Cout, 9, Cin] -> [B, G, G, Cout]."""
    out = np.zeros(a.shape[:3] + (w.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        out += shifted(a, dy * d, dx * d) @ w[:, t, :].T
    return out


def conv_t(g: np.ndarray, w: np.ndarray, d: int) -> np.ndarray:
    """Adjoint of conv in its input: g: [B, G, G, Cout] -> [B, G, G, Cin]."""
    out = np.zeros(g.shape[:3] + (w.shape[2],))
    for t, (dy, dx) in enumerate(TAPS):
        out += shifted(g, -dy * d, -dx * d) @ w[:, t, :]
    return out


def conv_w(g: np.ndarray, a: np.ndarray, d: int) -> np.ndarray:
    """Gradient in the weights: [Cout, 9, Cin] = sum_p g[p, co] a[p + off, ci]."""
    B = g.shape[0]
    out = np.zeros((g.shape[3], 9, a.shape[3]))
    gf = g.reshape(-1, g.shape[3])
    for t, (dy, dx) in enumerate(TAPS):
        out[:, t, :] = gf.T @ shifted(a, dy * d, dx * d).reshape(-1, a.shape[3])
    return out


def forward(params: np.ndarray, x: np.ndarray, bf: bool = False):
    """x: [B, G, G] -> (y [B, G, G], layer inputs a0 .. a5, their hi parts).
    Without `bf` the hi parts are the inputs themselves."""
    ws = split(params)
    a = [x[..., None]]
    hi = [x[..., None]]
    for l in range(5):
        if bf and l > 0:
            wh = bf16(ws[l])
            v = conv(a[-1], wh, DIL[l]) + conv(hi[-1], bf16(ws[l] - wh), DIL[l])
        else:
            v = conv(a[-1], ws[l], DIL[l])
        if bf:
            h = bf16(v)
            a.append(h + bf16(v - h))
            hi.append(h)
        else:
            a.append(v)
            hi.append(v)
    y = conv(a[-1], ws[5], DIL[5])[..., 0]
    return y, a, hi


def loss_grad(params: np.ndarray, x: np.ndarray, t: np.ndarray, bf: bool = False):
    """Mean squared error and its gradient in every parameter."""
    r = bf16 if bf else (lambda v: v)
    ws = [r(w) for w in split(params)]
    y, a, hi = forward(params, x, bf)
    n = y.size
    loss = float(np.mean((y - t) ** 2))
    g = r(2.0 * (y - t) / n)[..., None]
    grads = [None] * 6
    grads[5] = conv_w(g, a[5], DIL[5])
    g = r(conv_t(g, ws[5], DIL[5]))
    for l in range(4, 0, -1):
        grads[l] = conv_w(g, hi[l], DIL[l])
        g = r(conv_t(g, ws[l], DIL[l]))
    grads[0] = conv_w(g, a[0], DIL[0])
    return loss, join(grads)


def conv_fft(a: np.ndarray, w: np.ndarray, d: int) -> np.ndarray:
    """The same convolution through the convolution theorem (an independent
    computation, used to pin `conv`)."""
    B, H, W_, Ci = a.shape
    k = np.zeros((w.shape[0], Ci, H, W_))
    for t, (dy, dx) in enumerate(TAPS):
        k[:, :, (-dy * d) % H, (-dx * d) % W_] += w[:, t, :]
    A = np.fft.fft2(np.moveaxis(a, 3, 1))                   # [B, Ci, H, W]
    K = np.fft.fft2(k)                                      # [Co, Ci, H, W]
    out = np.einsum("bihw,oihw->bohw", A, K)
    return np.moveaxis(np.real(np.fft.ifft2(out)), 1, 3)


def prolong_periodic(c: np.ndarray) -> np.ndarray:
    """One multigrid prolongation of a periodic coarse grid (no ghosts):
    centred slopes, offsets of a quarter coarse width, no xy term."""
    nc = c.shape[0]
    e = c
    mx = 0.5 * (np.roll(c, -1, axis=1) - np.roll(c, 1, axis=1))
    my = 0.5 * (np.roll(c, -1, axis=0) - np.roll(c, 1, axis=0))
    f = np.zeros((2 * nc, 2 * nc))
    for b in (0, 1):
        for a_ in (0, 1):
            dx = 0.25 if a_ else -0.25
            dy = 0.25 if b else -0.25
            f[b::2, a_::2] = (e + dx * mx) + dy * my
    return f


def block_mean(a: np.ndarray, r: int) -> np.ndarray:
    n = a.shape[0]
    return a.reshape(n // r, r, n // r, r).mean(axis=(1, 3))

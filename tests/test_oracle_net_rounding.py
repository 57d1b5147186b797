"""Pins of the network oracle's emulated roundings (CPU).

`net.loss_grad(bf=True)` is what the GPU's per-layer gradients are compared
with.  Its rounding points (module docstring of oracle/net.py) are pinned two
ways, neither of which restates its code:

1. A worked example with exact values.  A chain network (one non-zero weight
   per layer, centre tap, channel 0) on a single non-zero pixel makes every
   quantity a scalar; weights, input and target are dyadic numbers chosen so
   that each rounding point leaves its own mark (two of them ties that go to
   the even neighbour).  The expected gradients were derived by hand from the
   bfloat16 format (8 significant bits, round to nearest, ties to even) and
   are written below as literals with the derivation.

2. A bound.  For any instance, |grad_bf - grad_exact| is at most a running
   error bound built from the rounding points (unit roundoff u = 2^-8 for one
   bfloat16, 2^-16 for a hi + lo pair), propagated with absolute values
   through the same convolutions (themselves pinned in test_oracle_net.py).
   The target is chosen so that the output gradient 2 (y - t) / n is exactly
   representable, which makes every error of the last layer's gradient second
   order: a lo part dropped there shows up at once.

The checks are written as `check_*(N)` so that the mutation tests can run them
on a module with a planted mistake."""
import numpy as np
import pytest

from oracle import net

U = 2.0 ** -8      # bfloat16: |bf16(v) - v| <= U |v|
U2 = 2.0 ** -16    # hi + lo pair: |pair(v) - v| <= U2 |v|
SLACK = 1.0 + 1e-9  # FP64 rounding of the bound's own sums

# ------------------------------------------------------------ worked example
# chain weights W1..W6 (centre tap, channel 0 -> 0) and the input value
W_CHAIN = [1.0, 1.0, 1.0 + 2.0 ** -9, 3.0, 1.0, 3.0 + 2.0 ** -8]
X0 = 1.0 + 2.0 ** -12
PIX = (5, 9)
Q = 1.0 + 2.0 ** -7 + 2.0 ** -9   # wanted output gradient 2 (y - t) / n (not a bfloat16)
# Forward (weights of W2..W5 as pairs wh + wl, activations as pairs, input and
# W1, W6 unrounded):
#   a1 = 1 + 2^-12            (pair exact; hi1 = 1)
#   a2 = a1                   (hi2 = 1)
#   a3 = a2*1 + hi2*2^-9 = 1 + 2^-9 + 2^-12   (W3: wh = 1, wl = 2^-9; the
#        a2_lo * wl term is not formed; hi3 = 1, lo3 = 9*2^-12 exact)
#   a4 = 3 a3 = 3 + 27*2^-12  (hi4 = 3, lo4 = 27*2^-12: five bits, exact)
#   a5 = a4                   (hi5 = 3)
#   y  = W6 a5
# Backward (weights rounded to one bfloat16: W3 -> 1, W6 -> 3):
#   g6 = bf16(Q) = 1 + 2^-7                    (2^-9 below half a unit, 2^-8)
#   dW6 = g6 a5                                (the pair)
#   g5 = bf16(g6 * 3) = bf16(3.0234375) = 3.03125   (tie: 3 + 2^-6 is odd, 3 + 2^-5 even)
#   dW5 = g5 hi4 = 9.09375
#   g4 = bf16(g5 * 1) = 3.03125;  dW4 = g4 hi3 = 3.03125
#   g3 = bf16(g4 * 3) = bf16(9.09375) = 9.125       (tie: 1.0010001b x 2^3 is odd)
#   dW3 = g3 hi2 = 9.125;  g2 = bf16(9.125 * 1) = 9.125
#   dW2 = g2 hi1 = 9.125;  g1 = 9.125
#   dW1 = g1 x0                                (the input, unrounded)
EXPECT_BF = [9.125 * (1.0 + 2.0 ** -12), 9.125, 9.125, 3.03125, 9.09375,
             (1.0 + 2.0 ** -7) * (3.0 + 27 * 2.0 ** -12)]


def chain_instance(N):
    """Parameters, input and target of the worked example (batch 1, G x G)."""
    ws = []
    for l in range(6):
        w = np.zeros((net.C, 9, net.C)) if 0 < l < 5 else (np.zeros((net.C, 9, 1)) if l == 0
                                                             else np.zeros((1, 9, net.C)))
        w[0, 4, 0] = W_CHAIN[l]
        ws.append(w)
    p = net.join(ws)
    x = np.zeros((1, net.G, net.G))
    x[0][PIX] = X0
    y = N.forward(p, x, bf=True)[0]
    n = y.size
    t = np.zeros_like(y)
    t[0][PIX] = y[0][PIX] - (n / 2) * Q  # so that 2 (y - t) / n == Q exactly
    assert 2.0 * (y[0][PIX] - t[0][PIX]) / n == Q
    return p, x, t


def chain_entry(N, g, l):
    """The single non-zero entry of layer l's gradient; all others must be 0."""
    w = net.split(g)[l]
    v = w[0, 4, 0]
    rest = w.copy()
    rest[0, 4, 0] = 0.0
    assert not np.any(rest), f"layer {l + 1} has other non-zero entries"
    return v


def check_worked_example(N):
    p, x, t = chain_instance(N)
    _, g = N.loss_grad(p, x, t, bf=True)
    got = [chain_entry(N, g, l) for l in range(6)]
    for l in range(6):
        assert got[l] == EXPECT_BF[l], (l + 1, got[l], EXPECT_BF[l])


def check_worked_example_unrounded(N):
    """Without the roundings the same instance gives the exact chain rule:
    dW_k = g_k a_{k-1} with g_k the product of the weights above layer k."""
    p, x, t = chain_instance(N)
    _, g = N.loss_grad(p, x, t, bf=False)
    ye = N.forward(p, x, bf=False)[0]
    n = ye.size
    ge = 2.0 * (ye[0][PIX] - t[0][PIX]) / n
    a = [X0]
    for w in W_CHAIN[:5]:
        a.append(a[-1] * w)
    up = ge
    want = [0.0] * 6
    for l in range(5, -1, -1):
        want[l] = up * a[l]
        up *= W_CHAIN[l]
    for l in range(6):
        assert abs(chain_entry(N, g, l) - want[l]) <= 1e-15 * abs(want[l]), (l + 1,)


# ------------------------------------------------------------------- bound
def random_instance(seed, positive, gs):
    """Random weights (N(0, 1/fan-in), or their absolute values) and input on
    a gs x gs grid, batch 2, and per-pixel factors c in +-[0.5, 1.5] (positive
    only if `positive`) that place the target: 2 (y - t) / n = bf16(c 2 y / n),
    a bfloat16 value of the size of 2 y / n (y - t is not a small difference of
    large numbers)."""
    g = np.random.default_rng(seed)
    p = np.concatenate([g.normal(0, 1 / np.sqrt(k * ci), co * k * ci)
                        for co, k, ci in [(32, 9, 1)] + [(32, 9, 32)] * 4 + [(1, 9, 32)]])
    x = g.standard_normal((2, gs, gs))
    c = g.uniform(0.5, 1.5, (2, gs, gs))
    if positive:
        p, x = np.abs(p), np.abs(x)
    else:
        c *= g.choice([-1.0, 1.0], (2, gs, gs))
    return p, x, c


def gradient_bound(N, p, x, c):
    """(exact gradient, bound on |grad_bf - grad_exact|, bf gradient), per
    parameter vector.  Layer k maps a_{k-1} to a_k with W_k = split(p)[k-1].
    Only N.forward and N.loss_grad come from the module under test; the
    bound's own convolutions and roundings are the pinned ones of `net`."""
    ws = net.split(p)
    yb, ab, hb = N.forward(p, x, bf=True)
    ye, ae, _ = N.forward(p, x, bf=False)
    n = yb.size
    q = net.bf16(c * 2.0 * yb / n)
    t = yb - (n / 2) * q                      # 2 (yb - t) / n == q up to 2^-50: bf16 keeps q
    _, gex = N.loss_grad(p, x, t, bf=False)
    _, gbf = N.loss_grad(p, x, t, bf=True)
    A = lambda v: np.abs(v)
    # forward: delta_k >= |a_k^bf - a_k^exact|
    delta = [np.zeros_like(ae[0]), U2 * A(ae[1]) * SLACK]
    for k in range(2, 6):
        W = ws[k - 1]
        wh = net.bf16(W)
        wl = net.bf16(W - wh)
        rho = W - wh - wl
        d = net.DIL[k - 1]
        e = (net.conv(delta[k - 1], A(W), d) + net.conv(A(ab[k - 1] - hb[k - 1]), A(wl), d)
             + net.conv(A(ab[k - 1]), A(rho), d))
        delta.append((U2 * A(ae[k]) + (1 + U2) * e) * SLACK)
    dy = net.conv(delta[5], A(ws[5]), net.DIL[5])[..., 0] * SLACK
    # backward: eps_k >= |g_k^bf - g_k^exact|, g_k the gradient at a_k (k = 5..1), g_6 at y
    g_ex = {6: (2.0 * (ye - t) / n)[..., None]}
    eps = {6: (2.0 * dy / n + 1e-15 * A(q))[..., None] * SLACK}
    for k in range(5, 0, -1):
        W = ws[k]
        d = net.DIL[k]
        g_ex[k] = net.conv_t(g_ex[k + 1], W, d)
        e = net.conv_t(eps[k + 1], A(net.bf16(W)), d) + net.conv_t(A(g_ex[k + 1]), A(net.bf16(W) - W), d)
        eps[k] = (U * A(g_ex[k]) + (1 + U) * e) * SLACK
    # weight gradients: layer 6 from the pair a5, layers 2..5 from the hi parts, layer 1 from x
    bound = [None] * 6
    for k in range(6, 0, -1):
        d = net.DIL[k - 1]
        if k == 1:
            used, dev = ae[0], np.zeros_like(ae[0])
        elif k == 6:
            used, dev = ab[5], delta[5]
        else:
            used, dev = hb[k - 1], A(hb[k - 1] - ab[k - 1]) + delta[k - 1]
        b = net.conv_w(eps[k], A(used), d) + net.conv_w(A(g_ex[k]), dev, d)
        b += 1e-13 * net.conv_w(A(g_ex[k]), A(ae[k - 1]), d)  # FP64 sums of both gradients
        bound[k - 1] = b * SLACK
    return gex, net.join(bound), gbf


def check_bound(N, seed, positive, gs=8):
    gex, bnd, gbf = gradient_bound(N, *random_instance(seed, positive, gs))
    err = np.abs(gbf - gex)
    o = 0
    for l, sz in enumerate(net.SIZES):
        sl = slice(o, o + sz)
        worst = np.max(err[sl] - bnd[sl])
        assert worst <= 0.0, (l + 1, worst, float(np.max(err[sl])), float(np.max(bnd[sl])))
        o += sz


def test_worked_example_every_rounding_point():
    check_worked_example(net)


def test_worked_example_without_rounding_is_the_chain_rule():
    check_worked_example_unrounded(net)


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("positive", [True, False])
def test_rounded_gradient_within_the_running_error_bound(seed, positive):
    check_bound(net, seed, positive)


def test_last_layer_bound_is_second_order():
    """With a representable output gradient and cancellation-free data the
    last layer's bound stays near the pair's precision (a few 2^-16 of the
    gradient), far below what one bfloat16 rounding (2^-8) would need: the
    bound above can tell a pair from a single bfloat16."""
    gex, bnd, _ = gradient_bound(net, *random_instance(3, True, 8))
    o = sum(net.SIZES[:5])
    rel = np.max(bnd[o:] / np.abs(gex[o:]))
    assert rel < 2.0 ** -12, rel


def test_rounded_gradient_relative_error_per_layer():
    """On a signed random instance the per-layer relative error of the
    rounded gradient (norm of the difference over the norm) stays below
    2^-5: the back-propagated gradients carry one bfloat16 each."""
    gex, _, gbf = gradient_bound(net, *random_instance(4, False, 16))
    o = 0
    for l, sz in enumerate(net.SIZES):
        e = np.linalg.norm(gbf[o:o + sz] - gex[o:o + sz]) / np.linalg.norm(gex[o:o + sz])
        assert e < 2.0 ** -5, (l + 1, e)
        o += sz

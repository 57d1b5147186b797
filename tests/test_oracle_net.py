"""Pins of the network oracle (CPU): the convolution against the convolution
theorem, its adjoint, and the loss gradient against central differences."""
import numpy as np
import pytest

from oracle import net as N

GS = 16  # small grid for the checks: the oracle's functions take any grid size


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_conv_matches_fft_convolution(d):
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, GS, GS, 3))
    w = rng.standard_normal((4, 9, 3))
    assert np.allclose(N.conv(a, w, d), N.conv_fft(a, w, d), atol=1e-12)


def test_conv_tap_convention():
    """tap 3*(dy+1)+(dx+1) reads in[y + dy d, x + dx d]: a unit impulse moves opposite."""
    a = np.zeros((1, GS, GS, 1))
    a[0, 5, 7, 0] = 1.0
    w = np.zeros((1, 9, 1))
    w[0, 5, 0] = 1.0  # tap (dy, dx) = (0, +1)
    out = N.conv(a, w, 2)
    assert out[0, 5, 5, 0] == 1.0 and out.sum() == 1.0


@pytest.mark.parametrize("d", [1, 4])
def test_conv_t_is_adjoint(d):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, GS, GS, 3))
    g = rng.standard_normal((2, GS, GS, 5))
    w = rng.standard_normal((5, 9, 3))
    assert np.isclose(np.sum(N.conv(a, w, d) * g), np.sum(a * N.conv_t(g, w, d)), rtol=1e-12)
    # weight gradient: d/dw <conv(a, w), g> = conv_w(g, a)
    dw = N.conv_w(g, a, d)
    e = rng.standard_normal(w.shape)
    assert np.isclose(np.sum(N.conv(a, e, d) * g), np.sum(dw * e), rtol=1e-12)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(N.param_count()) * 0.1
    x = rng.standard_normal((2, GS, GS))
    t = rng.standard_normal((2, GS, GS))
    loss, g = N.loss_grad(p, x, t)
    for k in rng.choice(p.size, size=24, replace=False):
        e = np.zeros_like(p)
        e[k] = 1e-6
        fd = (N.loss_grad(p + e, x, t)[0] - N.loss_grad(p - e, x, t)[0]) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 3.14159265, -2.5e-3])
    r = N.bf16(v)
    # exact bf16 values survive; ties go to even; relative error <= 2^-8
    assert N.bf16(np.array([1.0 + 2 ** -7]))[0] == 1.0 + 2 ** -7
    assert N.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie -> even (1.0)
    assert N.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6  # tie -> even
    assert np.all(np.abs(r - v) <= 2 ** -8 * np.abs(v))


def test_prolongation_matches_multigrid_oracle():
    """The decoder's prolongation is the multigrid one (periodic sides)."""
    import oracle
    rng = np.random.default_rng(3)
    c = rng.standard_normal((8, 8))
    fine = oracle.field_zeros(16)
    oracle.prolong_add(oracle.embed(c), fine, "PPPP")
    assert np.allclose(N.prolong_periodic(c), oracle.interior(fine), atol=1e-15)


def test_bf16_pair_keeps_about_16_bits():
    v = np.random.default_rng(4).standard_normal(10000) * 10.0 ** np.random.default_rng(5).uniform(-5, 5, 10000)
    p = N.bf16_pair(v)
    assert np.all(np.abs(p - v) <= 2.0 ** -16 * np.abs(v))


def test_rounded_forward_stays_within_the_pairs_precision():
    """Each layer's weights and activations keep about 16 bits (hi + lo
    pairs), so six layers of the rounded forward stay within a few 2^-16 of
    the unrounded one; rounding the weights to one bfloat16 (2^-9) would not."""
    g = np.random.default_rng(6)
    p = np.concatenate([g.normal(0, 1 / np.sqrt(k * ci), co * k * ci)
                        for co, k, ci in [(32, 9, 1)] + [(32, 9, 32)] * 4 + [(1, 9, 32)]])
    p = p.astype(np.float32).astype(np.float64)
    x = g.standard_normal((1, N.G, N.G)).astype(np.float32).astype(np.float64)
    y = N.forward(p, x)[0]
    e = np.linalg.norm(N.forward(p, x, bf=True)[0] - y) / np.linalg.norm(y)
    assert e < 6 * 2.0 ** -16
    e1 = np.linalg.norm(N.forward(N.bf16(p), x)[0] - y) / np.linalg.norm(y)
    assert e1 > 10 * e

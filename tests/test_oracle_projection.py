"""Pins of the oracle's cell-centred approximate projection (Sec. 3.5,
incompressible flow; CPU only): Lap phi = D U*, U = U* - G phi with D, G
centred differences across two cells and Lap the 5-point operator on the
doubly periodic unit square.

* A discrete curl (u = D_y psi, v = -D_x psi) has D U = 0 exactly (centred
  differences commute on a periodic grid): the projection leaves it unchanged.
* Fourier modes diagonalise D, G and Lap, so the projection of U* = G phi0
  for a mode phi0 is G phi0 (1 - r) with r the ratio of the symbols of D G
  and Lap, in closed form.
* The paper's convergence field (Minion's divergence-free u, v) plus a smooth
  gradient: the projection recovers the divergence-free part at second order
  as h halves."""
import numpy as np

import oracle


def grid(n):
    t = (np.arange(n) + 0.5) / n
    return np.meshgrid(t, t)


def centred(a, axis):
    """(a[k+1] - a[k-1]) / 2h along `axis` (1 = x, 0 = y), periodic."""
    n = a.shape[0]
    return (np.roll(a, -1, axis=axis) - np.roll(a, 1, axis=axis)) * n / 2.0


def test_discrete_curl_is_left_unchanged():
    n = 64
    X, Y = grid(n)
    psi = np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y) + 0.3 * np.cos(6 * np.pi * X + 1.0)
    u0, v0 = centred(psi, 0), -centred(psi, 1)
    f = oracle.divergence(n, 1.0 / n, oracle.embed(u0), oracle.embed(v0))
    assert np.abs(oracle.interior(f)).max() < 1e-11
    u, v, phi, r = oracle.project(n, oracle.embed(u0.copy()), oracle.embed(v0.copy()))
    assert np.abs(oracle.interior(u) - u0).max() < 1e-12 and np.abs(oracle.interior(v) - v0).max() < 1e-12


def test_gradient_of_a_mode_in_closed_form():
    n = 64
    h = 1.0 / n
    X, Y = grid(n)
    kx, ky = 3, 2
    phi0 = np.cos(2 * np.pi * (kx * X + ky * Y))
    gx, gy = centred(phi0, 1), centred(phi0, 0)
    sx, sy = np.sin(2 * np.pi * kx * h), np.sin(2 * np.pi * ky * h)
    dg = -(sx ** 2 + sy ** 2) / h ** 2                       # symbol of D G
    lap = -(4 / h ** 2) * (np.sin(np.pi * kx * h) ** 2 + np.sin(np.pi * ky * h) ** 2)  # of Lap
    r = dg / lap
    u, v, phi, res = oracle.project(n, oracle.embed(gx.copy()), oracle.embed(gy.copy()), rtol=1e-13)
    assert res.status == oracle.OK
    assert np.abs(oracle.interior(phi) - r * phi0).max() < 1e-11
    assert np.abs(oracle.interior(u) - (1 - r) * gx).max() < 1e-10
    assert np.abs(oracle.interior(v) - (1 - r) * gy).max() < 1e-10


def test_minion_field_recovered_at_second_order():
    errs = []
    for n in (32, 64, 128):
        X, Y = grid(n)
        ud = 1 - 2 * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        vd = 1 + 2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        # plus the gradient of phi0 = 0.1 sin(2 pi x) cos(4 pi y)
        gx = 0.2 * np.pi * np.cos(2 * np.pi * X) * np.cos(4 * np.pi * Y)
        gy = -0.4 * np.pi * np.sin(2 * np.pi * X) * np.sin(4 * np.pi * Y)
        u, v, phi, r = oracle.project(n, oracle.embed(ud + gx), oracle.embed(vd + gy))
        assert r.status == oracle.OK
        errs.append(max(np.abs(oracle.interior(u) - ud).max(), np.abs(oracle.interior(v) - vd).max()))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5

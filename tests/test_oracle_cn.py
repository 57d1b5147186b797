"""Pins of the oracle's Crank-Nicolson diffusion step (Sec. 3.4, implicit
diffusion; CPU only).  No value of the paper's Gaussian test is printed (it
is shown as a figure), so the pins come from the mathematics:

* cell-centred sin / cos / Fourier modes are exact eigenvectors of the
  discrete Laplacian with the homogeneous side rules, so one step multiplies
  such a mode by (1 + beta lam) / (1 - beta lam) (beta = k dt / 2), and the
  right-hand side alone by (1 + beta lam);
* the Gaussian of the paper's test problem (t0 = 1e-4, phi1 = 1, phi2 = 2,
  k = 1, C = dt k / dx^2 = 2) is an exact solution of the continuous
  equation: the discrete steps follow it, second order as dx halves at fixed
  C (dt ~ dx^2);
* with Neumann sides the step conserves the total of phi (the discrete
  Laplacian sums to zero)."""
import numpy as np
import pytest

import oracle


def modes(n, bc):
    """(phi, lam): one separable eigenvector of the discrete Laplacian for the
    side types `bc` and its eigenvalue, in closed form."""
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    if bc == "NNNN":
        fx, fy = np.cos(3 * np.pi * x), np.cos(2 * np.pi * x)
        lam = -(4 / h ** 2) * (np.sin(3 * np.pi * h / 2) ** 2 + np.sin(2 * np.pi * h / 2) ** 2)
    elif bc == "PPPP":
        fx, fy = np.cos(2 * np.pi * 3 * x), np.sin(2 * np.pi * 2 * x)
        lam = -(4 / h ** 2) * (np.sin(3 * np.pi * h) ** 2 + np.sin(2 * np.pi * h) ** 2)
    elif bc == "DDDD":
        fx, fy = np.sin(3 * np.pi * x), np.sin(np.pi * x)
        lam = -(4 / h ** 2) * (np.sin(3 * np.pi * h / 2) ** 2 + np.sin(np.pi * h / 2) ** 2)
    else:  # Dirichlet in x, Neumann in y
        fx, fy = np.sin(2 * np.pi * x), np.cos(np.pi * x)
        lam = -(4 / h ** 2) * (np.sin(2 * np.pi * h / 2) ** 2 + np.sin(np.pi * h / 2) ** 2)
    return np.outer(fy, fx), lam


def gaussian(n, t, k=1.0, t0=1e-4, phi1=1.0, phi2=2.0):
    """The test problem's exact solution at cell centres (rows = y)."""
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    return (phi2 - phi1) * t0 / (t + t0) * np.exp(-0.25 * r2 / (k * (t + t0))) + phi1


@pytest.mark.parametrize("bc", ["NNNN", "PPPP", "DDDD", "DDNN"])
@pytest.mark.parametrize("c", [0.5, 2.0, 10.0])
def test_cn_step_multiplies_an_eigenmode_by_the_closed_form_factor(bc, c):
    n = 64
    h = 1.0 / n
    beta = c * h * h / 2  # k dt / 2 with k = 1, dt = c h^2
    phi0, lam = modes(n, bc)
    rhs = oracle.cn_rhs(n, h, beta, bc, oracle.embed(phi0.copy()))
    assert np.abs(oracle.interior(rhs) - (1 + beta * lam) * phi0).max() < 1e-13
    p = oracle.Problem(n=n, h=h, alpha=1.0, beta=beta, bc=bc, rtol=1e-13)
    phi, r = oracle.cn_step(p, oracle.embed(phi0.copy()))
    assert r.status == oracle.OK
    g = (1 + beta * lam) / (1 - beta * lam)
    assert np.abs(oracle.interior(phi) - g * phi0).max() < 1e-12


def run_gaussian(n, t_end=0.005, C=2.0, bc="NNNN"):
    h = 1.0 / n
    steps = int(np.ceil(t_end / (C * h * h)))
    dt = t_end / steps  # k = 1; C <= 2
    p = oracle.Problem(n=n, h=h, alpha=1.0, beta=dt / 2, bc=bc, rtol=1e-12)
    phi = oracle.embed(gaussian(n, 0.0))
    total0 = oracle.interior(phi).sum()
    for _ in range(steps):
        phi, r = oracle.cn_step(p, phi)
        assert r.status == oracle.OK
    return oracle.interior(phi), total0


def test_cn_gaussian_follows_the_exact_solution_to_second_order():
    errs = {}
    for n in (64, 128, 256):
        got, _ = run_gaussian(n)
        errs[n] = np.abs(got - gaussian(n, 0.005)).max()
    amp = 1e-4 / (0.005 + 1e-4)  # peak height above phi1 at t_end
    assert errs[128] < 2e-3 * amp  # within 0.2% of the peak on the paper's 128^2 grid
    assert errs[64] / errs[128] > 3.0 and errs[128] / errs[256] > 3.0


def test_cn_conserves_the_total_with_neumann_sides():
    got, total0 = run_gaussian(64, t_end=0.002)
    assert abs(got.sum() - total0) <= 1e-12 * total0


def test_cn_step_requires_alpha_one():
    p = oracle.Problem(n=8, h=1 / 8, alpha=0.5, beta=0.1, bc="NNNN")
    with pytest.raises(ValueError):
        oracle.cn_step(p, oracle.field_zeros(8))

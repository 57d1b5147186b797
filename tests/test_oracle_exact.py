"""Pins of the array-form operator of the exact-solution module (CPU).

`exact.apply_operator` and `exact.relative_residual` are the host-side check
of every full-size GPU test: the returned field's residual is recomputed with
them.  They restate the operator of Eq. (helmholtz), (alpha - beta Lap_h) phi,
with the ghost equations of Sec. 3.3 (Dirichlet ghost = -cell, Neumann
ghost = +cell) and periodic wrapping, in whole-array form.  Two independent
forms pin them: the dense matrix assembled entry by entry (`exact.assemble`,
itself pinned by symmetry, closed-form eigenvalues and the dense/transform
agreement in test_oracle_pins.py) and the C oracle's residual (`og_residual`),
for all 25 pairings of side types, Poisson and Helmholtz.

The checks are written as `check_*(E, ...)` so that the mutation tests can run
them on a module with a planted mistake."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import exact

AXES = [("P", "P"), ("D", "D"), ("N", "N"), ("D", "N"), ("N", "D")]
ALL_BC = [ax + ay for ax, ay in itertools.product(AXES, AXES)]
OPS = [(0.0, -1.0), (1.0, 0.37), (2.5, -0.01)]


def check_apply_operator_equals_assembled(E, bc, ab, n=8):
    """(alpha - beta Lap_h) phi in array form equals the assembled matrix
    times phi, cell by cell (<= 1e-13 of the largest entry)."""
    h = 1.0 / n
    phi = np.random.default_rng(n + 7 * len(bc)).standard_normal((n, n))
    A = exact.assemble(n, h, ab[0], ab[1], bc)
    want = (A @ phi.reshape(-1)).reshape(n, n)
    got = E.apply_operator(phi, h, ab[0], ab[1], bc)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), (bc, ab)


def check_relative_residual_equals_assembled(E, bc, ab, n=8):
    """||f - A phi|| / ||f|| with A the assembled matrix (<= 1e-13 relative)."""
    h = 1.0 / n
    g = np.random.default_rng(3 * n + len(bc))
    phi = g.standard_normal((n, n))
    f = g.standard_normal((n, n))
    A = exact.assemble(n, h, ab[0], ab[1], bc)
    r = f.reshape(-1) - A @ phi.reshape(-1)
    want = np.linalg.norm(r) / np.linalg.norm(f)
    got = E.relative_residual(phi, f, h, ab[0], ab[1], bc)
    assert abs(got - want) <= 1e-13 * want, (bc, ab, got, want)


def check_residual_equals_c_oracle(E, bc, ab, n=16):
    """f - (alpha - beta Lap_h) phi equals the C oracle's residual (its own
    ghost fill and stencil), cell by cell."""
    h = 1.0 / n
    g = np.random.default_rng(5 * n + len(bc))
    phi = g.standard_normal((n, n))
    f = g.standard_normal((n, n))
    prob = oracle.Problem(n=n, h=h, alpha=ab[0], beta=ab[1], bc=bc)
    want = oracle.interior(oracle.residual(prob, oracle.embed(phi), oracle.embed(f)))
    got = f - E.apply_operator(phi, h, ab[0], ab[1], bc)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), (bc, ab)


def check_exact_solutions_have_rounding_residual(E):
    """The dense solution's relative residual is at rounding level, a zero
    field's is exactly 1, and the operator multiplies a periodic Fourier mode
    by its closed-form eigenvalue alpha - beta lam."""
    n, h = 8, 1.0 / 8
    for bc, ab in (("DDDD", (0.0, -1.0)), ("DNPP", (1.0, 0.37)), ("NDND", (0.0, -1.0))):
        f = np.random.default_rng(11).standard_normal((n, n))
        if exact.is_singular(ab[0], bc):
            f -= f.mean()
        x = exact.dense_solve(f, h, ab[0], ab[1], bc)
        assert E.relative_residual(x, f, h, ab[0], ab[1], bc) <= 1e-13
        assert E.relative_residual(np.zeros((n, n)), f, h, ab[0], ab[1], bc) == 1.0
    # periodic Fourier mode cos(2 pi (kx x + ky y)): an eigenvector of Lap_h
    # with eigenvalue -(4/h^2)(sin^2(pi kx h) + sin^2(pi ky h))
    kx, ky = 2, 3
    xc = (np.arange(n) + 0.5) * h
    mode = np.cos(2 * np.pi * (kx * xc[None, :] + ky * xc[:, None]))
    lam = -(4 / h**2) * (np.sin(np.pi * kx * h) ** 2 + np.sin(np.pi * ky * h) ** 2)
    for alpha, beta in ((0.0, -1.0), (1.0, 0.37)):
        got = E.apply_operator(mode, h, alpha, beta, "PPPP")
        assert np.max(np.abs(got - (alpha - beta * lam) * mode)) <= 1e-12 * abs(alpha - beta * lam)


@pytest.mark.parametrize("bc", ALL_BC)
@pytest.mark.parametrize("ab", OPS)
def test_apply_operator_equals_assembled_matrix(bc, ab):
    check_apply_operator_equals_assembled(exact, bc, ab)


@pytest.mark.parametrize("bc", ALL_BC)
@pytest.mark.parametrize("ab", OPS[:2])
def test_relative_residual_equals_assembled_matrix(bc, ab):
    check_relative_residual_equals_assembled(exact, bc, ab)


@pytest.mark.parametrize("bc", ALL_BC)
@pytest.mark.parametrize("ab", OPS[:2])
def test_residual_equals_c_oracle(bc, ab):
    check_residual_equals_c_oracle(exact, bc, ab)


def test_exact_solutions_have_rounding_residual():
    check_exact_solutions_have_rounding_residual(exact)

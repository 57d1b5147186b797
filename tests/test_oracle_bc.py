"""Pins of the oracle's inhomogeneous side data (Sec. 3.3: the boundary
value enters the ghost cell's expression; CPU only).

* The definition written out: the discrete problem with the ghost cells as
  unknowns of their own (interior 5-point rows plus one ghost equation per
  ghost) is assembled and solved densely at n = 8; the oracle's solve (the
  data moved to the right-hand side, homogeneous V-cycles) must agree.
* Linear functions are reproduced exactly: their 5-point Laplacian is zero
  and the second-order ghost rules are exact for them.
* A smooth manufactured solution with data on every side converges at
  second order."""
import numpy as np
import pytest

import oracle


def centres(n):
    return (np.arange(n) + 0.5) / n


def side_data(bc, phi_fn, dx_fn, dy_fn, n):
    """Dirichlet values or Neumann derivatives of an exact solution on the
    four sides (x-lo, x-hi along y; y-lo, y-hi along x)."""
    t = centres(n)
    out = []
    for s, code in enumerate(bc):
        if code == "P":
            out.append(None)
            continue
        if s < 2:
            X = np.full(n, 0.0 if s == 0 else 1.0)
            out.append(phi_fn(X, t) if code == "D" else dx_fn(X, t))
        else:
            Y = np.full(n, 0.0 if s == 2 else 1.0)
            out.append(phi_fn(t, Y) if code == "D" else dy_fn(t, Y))
    return out


def extended_dense_solve(n, alpha, beta, bc, f, b):
    """Unknowns: the n^2 valid cells and the 4n ghosts.  Rows: (alpha - beta
    Lap) phi = f on valid cells, reading ghosts as unknowns; for each ghost
    its side rule (Dirichlet: (ghost + adjacent) / 2 = v; Neumann:
    (adjacent - ghost) / h = d on a lo side, (ghost - adjacent) / h = d on a
    hi side; periodic: ghost = the opposite cell)."""
    h = 1.0 / n
    c = beta / (h * h)
    nv = n * n
    gid = {}
    for s in range(4):
        for k in range(n):
            gid[(s, k)] = nv + s * n + k
    N = nv + 4 * n
    A = np.zeros((N, N))
    rhs = np.zeros(N)

    def ref(i, j):  # unknown index of cell (i, j), valid or ghost
        if 0 <= i < n and 0 <= j < n:
            return j * n + i
        if i < 0:
            return gid[(0, j)]
        if i >= n:
            return gid[(1, j)]
        if j < 0:
            return gid[(2, i)]
        return gid[(3, i)]

    for j in range(n):
        for i in range(n):
            k = j * n + i
            A[k, k] = alpha + 4 * c
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                A[k, ref(i + di, j + dj)] -= c
            rhs[k] = f[j, i]
    codes = oracle.bc_codes(bc)
    for s in range(4):
        for k in range(n):
            g = gid[(s, k)]
            if s == 0:
                adj, opp = k * n + 0, k * n + n - 1
            elif s == 1:
                adj, opp = k * n + n - 1, k * n + 0
            elif s == 2:
                adj, opp = 0 * n + k, (n - 1) * n + k
            else:
                adj, opp = (n - 1) * n + k, 0 * n + k
            if codes[s] == oracle.PERIODIC:
                A[g, g], A[g, opp] = 1.0, -1.0
            elif codes[s] == oracle.DIRICHLET:
                A[g, g], A[g, adj] = 0.5, 0.5
                rhs[g] = b[s][k]
            else:
                lo = s in (0, 2)
                A[g, g], A[g, adj] = (-1.0 / h, 1.0 / h) if lo else (1.0 / h, -1.0 / h)
                rhs[g] = b[s][k]
    x = np.linalg.solve(A, rhs)
    return x[:nv].reshape(n, n)


@pytest.mark.parametrize("bc", ["DDDD", "NNDD", "DNDN", "PPDN", "DDPP"])
@pytest.mark.parametrize("ab", [(0.0, -1.0), (1.0, 0.02)])
def test_side_data_solve_matches_the_extended_dense_system(bc, ab):
    n = 8
    h = 1.0 / n
    alpha, beta = ab
    rng = np.random.default_rng(7)
    f = rng.standard_normal((n, n))
    b = [None if code == "P" else rng.standard_normal(n) for code in bc]
    want = extended_dense_solve(n, alpha, beta, bc, f, b)
    p = oracle.Problem(n=n, h=h, alpha=alpha, beta=beta, bc=bc, rtol=1e-13)
    phi, r = oracle.solve_bc(p, oracle.embed(f), b)
    assert r.status == oracle.OK
    assert np.abs(oracle.interior(phi) - want).max() <= 1e-10 * np.abs(want).max()


# (all-Neumann Poisson is singular: its data fix phi only up to a constant,
# which the test below covers)
@pytest.mark.parametrize("bc,ab", [(bc, ab) for bc in ["DDDD", "NNDD", "DNND", "NNNN", "PPDN"]
                                   for ab in [(0.0, -1.0), (1.0, 0.01)]
                                   if not (bc == "NNNN" and ab[0] == 0.0)])
def test_linear_functions_are_reproduced(bc, ab):
    n = 32
    h = 1.0 / n
    alpha, beta = ab
    if bc.startswith("PP"):
        lin = lambda X, Y: 0.3 - 0.6 * Y  # periodic in x: no x slope
        dx, dy = (lambda X, Y: 0.0 * X), (lambda X, Y: -0.6 + 0.0 * X)
    else:
        lin = lambda X, Y: 0.3 + 1.7 * X - 0.6 * Y
        dx, dy = (lambda X, Y: 1.7 + 0.0 * X), (lambda X, Y: -0.6 + 0.0 * X)
    t = centres(n)
    X, Y = np.meshgrid(t, t)
    f = alpha * lin(X, Y)  # Lap of a linear function is zero
    b = side_data(bc, lin, dx, dy, n)
    p = oracle.Problem(n=n, h=h, alpha=alpha, beta=beta, bc=bc, rtol=1e-13)
    phi, r = oracle.solve_bc(p, oracle.embed(f), b)
    assert r.status == oracle.OK
    assert np.abs(oracle.interior(phi) - lin(X, Y)).max() < 1e-11


def test_linear_function_singular_neumann():
    n = 32
    t = centres(n)
    X, Y = np.meshgrid(t, t)
    lin = 0.3 + 1.7 * X - 0.6 * Y
    b = [np.full(n, 1.7), np.full(n, 1.7), np.full(n, -0.6), np.full(n, -0.6)]
    p = oracle.Problem(n=n, h=1.0 / n, bc="NNNN", rtol=1e-13)
    phi, r = oracle.solve_bc(p, oracle.field_zeros(n), b)
    got = oracle.interior(phi)
    assert r.status == oracle.OK
    assert np.abs((got - got.mean()) - (lin - lin.mean())).max() < 1e-11


def test_ghosts_carry_the_data():
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(3)
    a = oracle.embed(rng.standard_normal((n, n)))
    b = [rng.standard_normal(n) for _ in range(4)]
    oracle.fill_bc(a, h, "DNND", b)
    # x-lo Dirichlet: the face value is the mean of ghost and cell
    assert np.allclose(0.5 * (a[1:-1, 0] + a[1:-1, 1]), b[0], rtol=0, atol=1e-14)
    # x-hi Neumann: (ghost - cell) / h is the derivative
    assert np.allclose((a[1:-1, -1] - a[1:-1, -2]) / h, b[1], rtol=0, atol=1e-12)
    # y-lo Neumann: (cell - ghost) / h
    assert np.allclose((a[1, 1:-1] - a[0, 1:-1]) / h, b[2], rtol=0, atol=1e-12)
    # y-hi Dirichlet
    assert np.allclose(0.5 * (a[-1, 1:-1] + a[-2, 1:-1]), b[3], rtol=0, atol=1e-14)


def test_manufactured_solution_converges_at_second_order():
    """phi = exp(0.7 x) cos(1.3 y) + x y: Lap phi = (0.49 - 1.69) exp(0.7x) cos(1.3y);
    Dirichlet data on x-lo, y-hi, Neumann derivatives on x-hi, y-lo."""
    phi_fn = lambda X, Y: np.exp(0.7 * X) * np.cos(1.3 * Y) + X * Y
    dx = lambda X, Y: 0.7 * np.exp(0.7 * X) * np.cos(1.3 * Y) + Y
    dy = lambda X, Y: -1.3 * np.exp(0.7 * X) * np.sin(1.3 * Y) + X
    lap = lambda X, Y: (0.49 - 1.69) * np.exp(0.7 * X) * np.cos(1.3 * Y)
    bc = "DNND"
    errs = []
    for n in (16, 32, 64):
        t = centres(n)
        X, Y = np.meshgrid(t, t)
        p = oracle.Problem(n=n, h=1.0 / n, bc=bc, rtol=1e-12)
        phi, r = oracle.solve_bc(p, oracle.embed(lap(X, Y)), side_data(bc, phi_fn, dx, dy, n))
        assert r.status == oracle.OK
        errs.append(np.sqrt(np.mean((oracle.interior(phi) - phi_fn(X, Y)) ** 2)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5

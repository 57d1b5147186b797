"""Pins of the oracle's exact bottom solve (CPU): the V-cycle may end on a
level of n_bottom x n_bottom cells solved directly instead of relaxing on the
2 x 2 grid (the paper's Sec. 3.3 leaves the coarsest solve open).  The pins
compare with numpy's dense solver on a matrix assembled separately in Python
(oracle.exact) and with the fixed point of the cycle."""
import numpy as np
import pytest

import oracle
from oracle import exact

BCS = ["DDDD", "NNNN", "PPPP", "DNPP", "PPND", "NDDN"]
ABS = [(0.0, -1.0), (1.0, 0.5 / 64), (3.0, 0.02)]


def rand_f(n, seed, singular):
    f = np.random.default_rng(seed).standard_normal((n, n))
    if singular:
        f -= f.mean()
    return f


@pytest.mark.parametrize("n", [4, 8])
@pytest.mark.parametrize("ab", ABS)
@pytest.mark.parametrize("bc", BCS)
def test_direct_bottom_on_the_top_level_is_the_dense_solution(bc, ab, n):
    """With n_bottom = n one cycle is the exact solve, whatever the start
    (the zero-mean solution for a singular problem)."""
    h = 1.0 / n
    p = oracle.Problem(n=n, h=h, alpha=ab[0], beta=ab[1], bc=bc, n_bottom=n)
    f = rand_f(n, 7, p.singular)
    phi = oracle.embed(np.random.default_rng(8).standard_normal((n, n)))
    oracle.vcycle(p, phi, oracle.embed(f))
    x = exact.dense_solve(f, h, *ab, bc)
    got = oracle.interior(phi)
    assert np.linalg.norm(got - x) / np.linalg.norm(x) < 1e-12
    if p.singular:
        assert abs(got.mean()) < 1e-14 * np.abs(got).max()


@pytest.mark.parametrize("nb", [4, 8, 16])
@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "DNPP", "NNNN"])
def test_direct_bottom_cycles_converge_to_the_dense_solution(bc, nb):
    n, h = 32, 1.0 / 32
    p = oracle.Problem(n=n, h=h, bc=bc, rtol=1e-13, max_cycles=60, n_bottom=nb)
    f = rand_f(n, 9, p.singular)
    phi, res = oracle.solve(p, oracle.embed(f))
    assert res.status == oracle.OK
    x = exact.dense_solve(f, h, p.alpha, p.beta, bc)
    assert np.linalg.norm(oracle.interior(phi) - x) / np.linalg.norm(x) < 1e-11


@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "NDDN"])
def test_direct_bottom_keeps_the_cycle_rate(bc):
    """An exact coarsest solve is at least as good as 50 relaxations on 2 x 2:
    the cycle count to 1e-10 at 64^2 does not grow, and the two-grid limit
    (n_bottom = n / 2) converges at a rate below 0.2 per cycle."""
    n, h = 64, 1.0 / 64
    f = rand_f(n, 10, bc in ("PPPP",))
    counts = {}
    for nb in (2, 4, 8, 32):
        p = oracle.Problem(n=n, h=h, bc=bc, n_bottom=nb)
        _, res = oracle.solve(p, oracle.embed(f))
        assert res.status == oracle.OK
        counts[nb] = res.cycles
        if nb == 32:
            rates = np.array(res.history[1:]) / np.array(res.history[:-1])
            assert rates.max() < 0.2
    assert max(counts.values()) <= counts[2]


def test_relaxation_bottom_unchanged_by_the_option():
    """n_bottom = 2 (and any size that is not a level) is the 2 x 2 relaxation
    bottom: the same iterates as the default."""
    n, h = 32, 1.0 / 32
    f = oracle.embed(rand_f(n, 11, False))
    ref, _ = oracle.solve(oracle.Problem(n=n, h=h, max_cycles=3, rtol=0.0), f)
    for nb in (2, 0, 64):
        got, _ = oracle.solve(oracle.Problem(n=n, h=h, max_cycles=3, rtol=0.0, n_bottom=nb), f)
        assert np.array_equal(got, ref)

"""Pins of the oracle's full multigrid start (og_fmg, CPU): facts that a
correct nested iteration must satisfy, independent of how it is coded.

FMG is not in the paper (its Sec. 3.3 cycles from a zero guess and leaves the
coarse solve open); it is the standard scheme of the multigrid literature
(Brandt 1977; Briggs, Henson and McCormick, "A Multigrid Tutorial", Ch. 3),
whose defining property is that one pass leaves an algebraic error below the
discretization error."""
import os

import numpy as np
import pytest

import oracle
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = [t.strip() for t in line.split("=", 1)]
        out[k] = v
    return out


def ex6(n):
    """The paper's Poisson test problem (Sec. 3.3.1) on n^2 cells."""
    g = read_golden("ex6_poisson.txt")
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    env = {"x": X, "y": Y}
    p = oracle.Problem(n=n, h=h, alpha=float(g["alpha"]), beta=float(g["beta"]), bc=tuple(g["bc"].split()),
                       rtol=1e-12)
    return p, eval(g["rhs"], {}, env), eval(g["solution"], {}, env)


def l2(h, e):
    return np.sqrt(h * h * np.sum(e * e))


@pytest.mark.parametrize("n", [32, 64, 128, 256])
def test_fmg_reaches_discretization_accuracy(n):
    """One FMG pass (one V(2,2) per level) leaves an algebraic error (against
    the exact discrete solution) below the discretization error (against the
    analytic solution of the paper's test problem); two V-cycles per level
    leave it far below.  Observed ratios: 0.20-0.48 and 0.011-0.020."""
    p, f, u = ex6(n)
    uh, res = oracle.solve(p, oracle.embed(f))
    assert res.status == oracle.OK
    disc = l2(p.h, oracle.interior(uh) - u)
    one = oracle.interior(oracle.fmg(p, oracle.embed(f), top_n=2, ncyc=1))
    two = oracle.interior(oracle.fmg(p, oracle.embed(f), top_n=2, ncyc=2))
    assert l2(p.h, one - oracle.interior(uh)) <= 0.6 * disc
    assert l2(p.h, two - oracle.interior(uh)) <= 0.05 * disc
    # and the total error stays at the discretization error's size
    assert l2(p.h, one - u) <= 1.6 * disc
    assert l2(p.h, two - u) <= 1.05 * disc


@pytest.mark.parametrize("bc,ab", [("DDDD", (0.0, -1.0)), ("PPPP", (0.0, -1.0)), ("NNNN", (0.0, -1.0)),
                                   ("DNPP", (1.0, 0.5 / 64)), ("NDDN", (0.0, -1.0))])
def test_fmg_with_many_cycles_is_the_discrete_solution(bc, ab):
    """With enough V-cycles per level FMG converges to the exact discrete
    solution (dense or transform solve of the assembled operator)."""
    n = 32
    p = oracle.Problem(n=n, h=1.0 / n, alpha=ab[0], beta=ab[1], bc=tuple(bc))
    f = np.random.default_rng(3).standard_normal((n, n))
    if p.singular:
        f -= f.mean()
    want = exact.dense_solve(f, 1.0 / n, ab[0], ab[1], tuple(bc))
    got = oracle.interior(oracle.fmg(p, oracle.embed(f), top_n=4, ncyc_top=20, ncyc=20))
    if p.singular:
        got = got - got.mean()
        want = want - want.mean()
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def test_fmg_is_linear_in_f():
    """Every step is linear in f (restriction, V-cycles from a guess that is
    itself linear in f, prolongation), so FMG(a f1 + b f2) = a FMG(f1) + b FMG(f2)."""
    n = 64
    p = oracle.Problem(n=n, h=1.0 / n, bc=("D", "N", "D", "D"))
    rng = np.random.default_rng(5)
    f1, f2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    a, b = 0.75, -2.5
    lhs = oracle.fmg(p, oracle.embed(a * f1 + b * f2), top_n=8)
    rhs = a * oracle.fmg(p, oracle.embed(f1), top_n=8) + b * oracle.fmg(p, oracle.embed(f2), top_n=8)
    assert np.max(np.abs(oracle.interior(lhs - rhs))) <= 1e-12 * np.max(np.abs(oracle.interior(rhs)))


@pytest.mark.parametrize("bc", ["DDDD", "PPPP"])
def test_fmg_start_saves_cycles(bc):
    """V-cycles from the FMG start (from 32^2 up) reach the paper's
    tolerance in at most 8 cycles where a zero start needs at least 11
    (smooth right-hand side, 256^2)."""
    n = 256
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    f = np.sin(2 * np.pi * 3 * X) * np.cos(2 * np.pi * 5 * Y) + 0.5 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * 7 * Y)
    if bc == "DDDD":
        f = f + 1.0
    else:
        f = f - f.mean()
    p = oracle.Problem(n=n, h=1.0 / n, bc=tuple(bc), rtol=1e-10)
    _, r0 = oracle.solve(p, oracle.embed(f))
    guess = oracle.fmg(p, oracle.embed(f), top_n=32)
    _, r1 = oracle.solve(p, oracle.embed(f), guess.copy())
    assert r0.status == r1.status == oracle.OK
    assert r0.cycles >= 11 and r1.cycles <= 8
    assert r1.rel_resid0 < 1e-2


def test_fmg_rejects_bad_arguments():
    p = oracle.Problem(n=16, h=1.0 / 16)
    f = oracle.embed(np.ones((16, 16)))
    for kw in ({"top_n": 3}, {"top_n": 32}, {"ncyc": -1}, {"ncyc_top": -1}):
        with pytest.raises(ValueError):
            oracle.fmg(p, f, **kw)

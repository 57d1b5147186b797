"""Inhomogeneous side data through the C ABI against the oracle: the shifted
right-hand side and the ghost fill element by element, whole solves
iterate-level, linear data reproduced exactly up to the benchmark's size,
and the mixed-precision plan."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
from test_oracle_bc import centres, side_data

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


def dev_field(a, pad=3):
    n = a.shape[0] - 2
    t = torch.zeros((n + 2, n + 2 + pad), dtype=torch.float64, device="cuda")
    t[:, :n + 2] = torch.from_numpy(a).cuda()
    return t


def host(t):
    n = t.shape[0] - 2
    return t[:, :n + 2].cpu().numpy()


def dev_sides(b):
    return [None if v is None else torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in b]


def rand_sides(bc, n, seed):
    rng = np.random.default_rng(seed)
    return [None if code == "P" else rng.standard_normal(n) for code in bc]


@pytest.mark.parametrize("bc", ["DDDD", "NNNN", "DNND", "PPDN", "NDPP"])
@pytest.mark.parametrize("n", [2, 8, 64, 512])
def test_bc_rhs_and_ghosts_match_oracle(bc, n):
    h = 1.0 / n
    beta = -1.0
    rng = np.random.default_rng(n)
    f = oracle.embed(rng.standard_normal((n, n)))
    b = rand_sides(bc, n, n + 1)
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=0.0, beta=beta))
    d_f, d_o = dev_field(f), dev_field(oracle.field_zeros(n))
    cc.ccmg_bc_rhs(plan, d_f, d_o, dev_sides(b))
    torch.cuda.synchronize()
    want = oracle.interior(oracle.bc_rhs(n, h, beta, bc, b, f))
    got = oracle.interior(host(d_o))
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    phi = oracle.embed(rng.standard_normal((n, n)))
    d_phi = dev_field(phi)
    cc.ccmg_fill_ghosts_bc(plan, d_phi, dev_sides(b))
    torch.cuda.synchronize()
    ref = oracle.fill_bc(phi.copy(), h, bc, b)
    g = host(d_phi)
    for sl in (np.s_[1:-1, 0], np.s_[1:-1, -1], np.s_[0, 1:-1], np.s_[-1, 1:-1]):
        assert np.abs(g[sl] - ref[sl]).max() <= 1e-14 * max(1.0, np.abs(ref[sl]).max())


@pytest.mark.parametrize("bc", ["DDDD", "DNND", "PPDN"])
@pytest.mark.parametrize("ab", [(0.0, -1.0), (1.0, 0.5 / 256 ** 2)])
def test_solve_bc_matches_oracle(bc, ab):
    """Iterate level: the GPU's solve with side data against the oracle's
    (same cycles, up to one)."""
    n = 256
    h = 1.0 / n
    alpha, beta = ab
    rng = np.random.default_rng(11)
    f = rng.standard_normal((n, n))
    b = rand_sides(bc, n, 12)
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=alpha, beta=beta, rtol=1e-10))
    d_f, d_phi, d_w = dev_field(oracle.embed(f)), dev_field(oracle.field_zeros(n)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve_bc(plan, d_f, d_phi, dev_sides(b), d_w)
    po = oracle.Problem(n=n, h=h, alpha=alpha, beta=beta, bc=bc, rtol=1e-10)
    ref, ro = oracle.solve_bc(po, oracle.embed(f), b)
    assert r.status == cc.OK and ro.status == oracle.OK
    assert abs(r.cycles - ro.cycles) <= 1
    got = host(d_phi)
    g, w = oracle.interior(got), oracle.interior(ref)
    assert np.linalg.norm(g - w) / np.linalg.norm(w) <= 1e-9
    # the returned ghosts carry the data
    again = oracle.fill_bc(got.copy(), h, bc, b)
    assert np.abs(again[1:-1, 0] - got[1:-1, 0]).max() <= 1e-12 * max(1.0, np.abs(got).max())


@pytest.mark.parametrize("bc,n", [("DDDD", 512), ("NNDD", 512), ("PPDD", 512), ("DNND", 64), ("PPDN", 64),
                                  ("NDDN", 64)])
@pytest.mark.parametrize("ab", [(0.0, -1.0), (1.0, 0.37 / 64 ** 2)])
def test_solve_bc_against_exact_discrete_solution(bc, n, ab):
    """The solve with side data against the exact solution of the discrete
    problem: the data's part of each ghost moved to the right-hand side by
    the (pinned) oracle, then that homogeneous problem solved exactly -- by
    the fast transforms when each axis has one side type, else by the dense
    matrix.  Relative error <= 1e-9, and the FP64 residual of the returned
    field recomputed on the host <= the tolerance of the shifted right-hand
    side.  The tolerance is the paper's 1e-11 (Sec. 3.3.1): with white-noise
    f and mixed Dirichlet / Neumann sides the error of any iterate at 1e-10
    can be ||A^-1|| ||f|| / ||phi*|| ~ 1.6e3 times its residual, and the
    oracle's own solve stops at 1.4e-9 (DNND, 64^2) -- the same as the GPU's."""
    h = 1.0 / n
    alpha, beta = ab
    rng = np.random.default_rng(n + len(bc))
    f = rng.standard_normal((n, n))
    b = rand_sides(bc, n, 21)
    if exact.is_singular(alpha, bc):
        # Neumann data compatible with f: the shifted right-hand side sums to 0
        fs = oracle.interior(oracle.bc_rhs(n, h, beta, bc, b, oracle.embed(f)))
        f = f - fs.mean()
    fs = oracle.interior(oracle.bc_rhs(n, h, beta, bc, b, oracle.embed(f)))
    if bc[0] == bc[1] and bc[2] == bc[3]:
        want = exact.transform_solve(fs, h, alpha, beta, bc)
    else:
        want = exact.dense_solve(fs, h, alpha, beta, bc)
    rtol = 1e-11
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=alpha, beta=beta, rtol=rtol))
    d_f, d_phi, d_w = dev_field(oracle.embed(f)), dev_field(oracle.field_zeros(n)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve_bc(plan, d_f, d_phi, dev_sides(b), d_w)
    assert r.status == cc.OK and r.rel_resid <= rtol, r
    got = oracle.interior(host(d_phi))
    assert exact.relative_residual(got, fs, h, alpha, beta, bc) <= 1.05 * rtol
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= 1e-9, err


@pytest.mark.parametrize("prec", [cc.FP64, cc.MIXED])
def test_linear_data_reproduced_at_full_size(prec):
    """Laplace on 4096^2 with the side data of a linear function (Dirichlet on
    x-lo and y-hi, Neumann on x-hi and y-lo), autotuned plan: the solution is
    that function at the cell centres (relative error <= 1e-9).  Tolerance
    1e-11, the paper's (Sec. 3.3.1): the right-hand side is only the data's
    part next to the sides, and at 1e-10 the error of any iterate can exceed
    1e-9 (1.6e-9 seen)."""
    n = 4096
    bc = "DNND"
    lin = lambda X, Y: 0.3 + 1.7 * X - 0.6 * Y
    dx, dy = (lambda X, Y: 1.7 + 0.0 * X), (lambda X, Y: -0.6 + 0.0 * X)
    b = side_data(bc, lin, dx, dy, n)
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), rtol=1e-11, prec=prec))
    d_f = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
    d_phi, d_w = torch.zeros_like(d_f), torch.zeros_like(d_f)
    cc.ccmg_plan_autotune(plan, d_f, d_phi)
    r = cc.ccmg_solve_bc(plan, d_f, d_phi, dev_sides(b), d_w)
    assert r.status == cc.OK and r.rel_resid <= 1e-11
    t = torch.from_numpy(centres(n)).cuda()
    want = 0.3 + 1.7 * t[None, :] - 0.6 * t[:, None]
    # the linear function is the exact discrete solution: relative error
    err = ((d_phi[1:n + 1, 1:n + 1] - want).norm() / want.norm()).item()
    assert err <= 1e-9, err


def test_data_on_a_periodic_side_is_rejected():
    n = 16
    plan = cc.Plan(cc.Problem(n=n, bc=("P", "P", "D", "D")))
    d_f, d_o = dev_field(oracle.field_zeros(n)), dev_field(oracle.field_zeros(n))
    b = dev_sides([np.ones(n), None, None, None])
    with pytest.raises(Exception):
        cc.ccmg_bc_rhs(plan, d_f, d_o, b)

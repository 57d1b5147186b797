"""Full multigrid through the C ABI (ccmg_fmg, and the FMG start of
ccmg_solve) against the oracle's og_fmg: the same restrictions, coarse
V-cycles, prolongations and per-level V-cycles, element by element."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


def dev_field(a):
    n = a.shape[0] - 2
    t = torch.zeros((n + 2, n + 2 + 5), dtype=torch.float64, device="cuda")
    t[:, :n + 2] = torch.from_numpy(a).cuda()
    return t


def valid(t):
    n = t.shape[0] - 2
    return t[1:n + 1, 1:n + 1].cpu().numpy()


def rhs(n, seed, singular):
    f = W.fourier_modes(n, seed=seed, count=16, kmax=8) + np.random.default_rng(seed).standard_normal((n, n)) * 0.1
    return f - f.mean() if singular else f + 0.3


@pytest.mark.parametrize("bc", ["DDDD", "NNDD", "DNPP", "PPPP", "NNNN"])
@pytest.mark.parametrize("n", [16, 32, 64, 128, 512])
@pytest.mark.parametrize("cyc", [(1, 1), (2, 1), (1, 2), (1, 0)])
def test_fmg_matches_oracle(bc, n, cyc):
    """ccmg_fmg = og_fmg started on the coarse tail's top level (32^2, or the
    finest level if smaller), to rounding; singular problems up to their mean
    (the oracle pins the mean of phi after each V-cycle, the GPU does not: a
    V-cycle commutes with adding a constant there)."""
    ncyc_top, ncyc = cyc
    prob = cc.Problem(n=n, bc=tuple(bc))
    singular = "D" not in bc
    f = rhs(n, 7, singular)
    plan = cc.Plan(prob)
    phi = dev_field(np.full((n + 2, n + 2), np.nan))  # not read
    cc.ccmg_fmg(plan, dev_field(oracle.embed(f)), phi, ncyc_top=ncyc_top, ncyc=ncyc)
    torch.cuda.synchronize()
    op = oracle.Problem(n=n, h=1.0 / n, bc=tuple(bc))
    want = oracle.interior(oracle.fmg(op, oracle.embed(f), top_n=min(n, 32), ncyc_top=ncyc_top, ncyc=ncyc))
    got = valid(phi)
    if singular:
        got, want = got - got.mean(), want - want.mean()
    assert np.isfinite(got).all()
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_fmg_helmholtz_and_ghosts():
    n, bc = 256, ("D", "N", "P", "P")
    prob = cc.Problem(n=n, bc=bc, alpha=1.0, beta=0.5 / n)
    f = rhs(n, 3, False)
    plan = cc.Plan(prob)
    phi = dev_field(np.zeros((n + 2, n + 2)))
    cc.ccmg_fmg(plan, dev_field(oracle.embed(f)), phi, ncyc_top=2, ncyc=1)
    torch.cuda.synchronize()
    op = oracle.Problem(n=n, h=1.0 / n, alpha=1.0, beta=0.5 / n, bc=bc)
    want = oracle.fmg(op, oracle.embed(f), top_n=32, ncyc_top=2, ncyc=1)
    got = phi[:, :n + 2].cpu().numpy()
    assert np.max(np.abs(oracle.interior(got) - oracle.interior(want))) <= 1e-11 * np.max(np.abs(want))
    # ghost cells filled by the side rules (corners are never written)
    filled = oracle.fill(got.copy(), bc)
    assert np.array_equal(got[1:-1, :], filled[1:-1, :]) and np.array_equal(got[:, 1:-1], filled[:, 1:-1])


def test_fmg_rejects_bad_arguments():
    plan = cc.Plan(cc.Problem(n=64, bc="D"))
    f, phi = dev_field(np.zeros((66, 66))), dev_field(np.zeros((66, 66)))
    for kw in ({"ncyc_top": 0}, {"ncyc_top": 17}, {"ncyc": -1}, {"ncyc": 17}):
        with pytest.raises(cc.CcmgError):
            cc.ccmg_fmg(plan, f, phi, **kw)
    mixed = cc.Plan(cc.Problem(n=64, bc="D", prec=cc.MIXED))
    with pytest.raises(cc.CcmgError):
        cc.ccmg_fmg(mixed, f, phi)


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "NDDN"])
@pytest.mark.parametrize("n", [512, 2048])
def test_solve_with_fmg_start(bc, n, fused):
    """ccmg_solve with CCMG_OPT_FMG: reaches the tolerance in fewer V-cycles
    than from zero, with the same solution (both within the tolerance of the
    exact discrete one, so they agree to about rtol times the conditioning);
    the residual after its first cycle is the oracle's FMG result's.  With
    the fused finest launch the finest prolongation happens inside the first
    pre-smoothing and the start's own residual is not formed (NaN)."""
    singular = "D" not in bc
    f = rhs(n, 11, singular)
    df = dev_field(oracle.embed(f))
    plain = cc.Plan(cc.Problem(n=n, bc=tuple(bc), rtol=1e-10))
    p0 = dev_field(np.zeros((n + 2, n + 2)))
    r0 = cc.ccmg_solve(plain, df, p0)
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), rtol=1e-10))
    cc.ccmg_plan_set_option(plan, cc.OPT_FMG, 1)
    cc.ccmg_plan_set_option(plan, cc.OPT_FUSED, fused)
    assert cc.ccmg_plan_get_option(plan, cc.OPT_FMG) == 1.0
    p1 = dev_field(np.zeros((n + 2, n + 2)))
    r1 = cc.ccmg_solve(plan, df, p1)
    assert r0.status == r1.status == cc.OK
    assert r1.rel_resid <= 1e-10 and r1.cycles <= r0.cycles - 3
    a, b = valid(p0), valid(p1)
    if singular:
        assert abs(b.mean()) <= 1e-12 * np.abs(b).max()
    assert np.max(np.abs(a - b)) <= 1e-7 * np.max(np.abs(a))
    # og_fmg's V-cycle on the finest level is the solve's first cycle: the
    # residual after it is the oracle's FMG result's
    if n == 512:
        op = oracle.Problem(n=n, h=1.0 / n, bc=tuple(bc))
        g = oracle.fmg(op, oracle.embed(f), top_n=32, ncyc_top=1, ncyc=1)
        rho = oracle.norm(oracle.residual(op, g.copy(), oracle.embed(f)), 1.0 / n) / oracle.norm(oracle.embed(f),
                                                                                                 1.0 / n)
        # (the start itself is the prolongated coarse solution: the fine-grid
        # noise of this f is still in its residual)
        if fused:
            assert np.isnan(r1.rel_resid0)
        else:
            assert 0.0 < r1.rel_resid0 < 1.0
        assert abs(r1.history[1] - rho) <= 1e-6 * rho


def test_solve_with_fmg_start_zero_and_nonfinite_rhs():
    """The FMG pass is queued before f's statistics are checked; a zero f
    still gives phi = 0 and OK, a non-finite f ENONFINITE, and the plan
    solves normally afterwards."""
    n = 256
    plan = cc.Plan(cc.Problem(n=n, bc="D", rtol=1e-10))
    cc.ccmg_plan_set_option(plan, cc.OPT_FMG, 1)
    phi = dev_field(np.full((n + 2, n + 2), 3.0))
    r = cc.ccmg_solve(plan, dev_field(np.zeros((n + 2, n + 2))), phi)
    assert r.status == cc.OK and torch.count_nonzero(phi[:, :n + 2]).item() == 0
    bad = np.zeros((n + 2, n + 2))
    bad[5, 7] = np.inf
    with pytest.raises(cc.CcmgError):
        cc.ccmg_solve(plan, dev_field(bad), phi)
    f = rhs(n, 2, False)
    r = cc.ccmg_solve(plan, dev_field(oracle.embed(f)), phi)
    assert r.status == cc.OK and r.rel_resid <= 1e-10

"""FP64 solves whose finest level runs the post-smoothing of one V-cycle and
the pre-smoothing of the next in one launch: the same iterates, residual
history and result as the unfused cycles, for every side type, plus the path
where the last cycle's post-smoothed iterate was not kept."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
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


def solve(n, bc, fv, guess=None, options=None, **kw):
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), rtol=1e-10, **kw))
    for opt, v in (options or {}).items():
        cc.ccmg_plan_set_option(plan, opt, v)
    f = dev_field(oracle.embed(fv))
    phi = dev_field(oracle.embed(guess) if guess is not None else oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, f, phi, use_guess=guess is not None)
    return r, phi, plan


@pytest.mark.parametrize("bc", ["DDDD", "NNDD", "DNPP", "PPDD", "PPPP", "NNNN"])
@pytest.mark.parametrize("n", [64, 512])
@pytest.mark.parametrize("visit", [1, 2])
def test_fused_solve_matches_unfused(bc, n, visit):
    """visit = 2: also the first fused launch that recomputes the first
    pre-smoothing, and every coarse level as a visit (both forms)."""
    fv = W.fourier_modes(n, seed=4, count=16, kmax=8)
    if not exact.is_singular(0.0, bc):
        fv = fv + 0.3  # a mean, where the problem allows one
    r0, p0, _ = solve(n, bc, fv, options={cc.OPT_FUSED: 0, cc.OPT_VISIT: visit})
    r1, p1, plan = solve(n, bc, fv, options={cc.OPT_VISIT: visit})
    assert r0.status == r1.status == cc.OK
    assert r0.cycles == r1.cycles
    a, b = valid(p0), valid(p1)
    if exact.is_singular(0.0, bc):
        # the unfused cycles shift phi by its mean between cycles: rounding only
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        assert np.allclose(r0.history, r1.history, rtol=1e-4, atol=0)  # residuals near the FP64 floor
    else:
        assert np.array_equal(a, b)
        # the norm's per-tile sums follow the tiles of a different launch
        assert np.allclose(r0.history, r1.history, rtol=1e-12, atol=0)
    cc.ccmg_plan_profile(plan, True)
    phi = dev_field(oracle.field_zeros(n))
    cc.ccmg_solve(plan, dev_field(oracle.embed(fv)), phi)
    stats = {k["name"]: k for k in cc.ccmg_plan_kernel_stats(plan)}
    cc.ccmg_plan_profile(plan, False)
    assert stats["finest_fused"]["launches"] + stats["finest_fused_first"]["launches"] >= r1.cycles - 1
    assert stats["finest_fused_first"]["launches"] == (1 if visit == 2 else 0)
    assert 1 <= stats["finest_pre"]["launches"] <= 2


@pytest.mark.parametrize("n", [1024, 2048])
def test_edge_strip_bands_leave_iterates_unchanged(n):
    """With Dirichlet or Neumann x sides, bands of 64 rows or more are halved
    in the two edge strips (their tiles apply the ghost rule in every stage).
    That is only another cut of the level into tiles: the solve's iterates are
    bitwise those of bands too short to be split, on every level and in the
    fused launch (ragged last bands included: 2048 rows in bands of 342 and
    edge bands of 172)."""
    fv = W.fourier_modes(n, seed=6, count=16, kmax=8) + 0.2
    outs = []
    for ty_fused, ty_levels in ((16, (16, 8)), (342, (128, 256)), (128, (64, 96))):
        plan = cc.Plan(cc.Problem(n=n, bc=("D", "N", "N", "D"), rtol=1e-10))
        cc.ccmg_plan_set_shape(plan, 0, 2, ty_fused, 1)
        for level in range(4):
            cc.ccmg_plan_set_shape(plan, level, 0, ty_levels[0], 1)
            cc.ccmg_plan_set_shape(plan, level, 1, ty_levels[1], 2)
        phi = dev_field(oracle.field_zeros(n))
        r = cc.ccmg_solve(plan, dev_field(oracle.embed(fv)), phi)
        assert r.status == cc.OK
        outs.append((valid(phi), r.cycles))
    for o, cyc in outs[1:]:
        assert cyc == outs[0][1]
        assert np.array_equal(o, outs[0][0])


@pytest.mark.parametrize("bc", ["DDDD", "PPPP"])
def test_fused_solve_with_guess_and_helmholtz(bc):
    n = 256
    fv = W.gaussian_random_field(n, seed=3)
    fv -= fv.mean()
    guess = 0.01 * np.random.default_rng(2).standard_normal((n, n))
    for kw in ({}, {"alpha": 1.0, "beta": 0.5 / (n * n)}):
        r0, p0, _ = solve(n, bc, fv, guess, options={cc.OPT_FUSED: 0}, **kw)
        r1, p1, _ = solve(n, bc, fv, guess, **kw)
        assert r0.status == r1.status == cc.OK and r0.cycles == r1.cycles
        a, b = valid(p0), valid(p1)
        if exact.is_singular(kw.get("alpha", 0.0), bc):
            # the unfused cycles shift phi by its mean between cycles: rounding only
            assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        else:
            # products fuse into sums only within an expression, so values kept
            # in registers across stages round as after a store: the same bits
            assert np.array_equal(a, b)


@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "DNPP"])
def test_fused_solve_when_last_iterate_was_not_kept(bc):
    """With no post-smoothed iterate kept past the first cycles, the solve
    returns the next cycle's pre-smoothed iterate, checked by its own residual."""
    n = 512
    fv = W.fourier_modes(n, seed=9, count=16, kmax=8)
    r, p, _ = solve(n, bc, fv, options={cc.OPT_FUSED_KEEP: 0})
    assert r.status == cc.OK and r.rel_resid <= 1e-10
    got = valid(p)
    h = 1.0 / n
    assert exact.relative_residual(got, fv, h, 0.0, -1.0, bc) <= 1e-10
    r2, p2, _ = solve(n, bc, fv)
    ref = valid(p2)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9
    if exact.is_singular(0.0, bc):
        assert abs(got.mean()) < 1e-13 * np.abs(got).max()


def test_fused_not_used_for_other_smoothing_counts():
    n = 256
    fv = W.fourier_modes(n, seed=1, count=8, kmax=4)
    r, p, plan = solve(n, "DDDD", fv, nu1=1, nu2=3)
    assert r.status == cc.OK
    cc.ccmg_plan_profile(plan, True)
    cc.ccmg_solve(plan, dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n)))
    stats = {k["name"]: k for k in cc.ccmg_plan_kernel_stats(plan)}
    cc.ccmg_plan_profile(plan, False)
    assert stats["finest_fused"]["launches"] == 0


@pytest.mark.parametrize("c", [0.1, 10.0])
def test_kernel_stats_count_only_launches_that_ran(c):
    """A well-conditioned Helmholtz solve converges in two or three cycles;
    the launches queued ahead for the next cycle exit at once (the device
    flags convergence first) and are left out of the timing statistics, so
    the finest-level launches counted are exactly one per cycle plus the
    first pre-smoothing."""
    n = 1024
    fv = W.gaussian_random_field(n, seed=4)
    r, _, plan = solve(n, "PPPP", fv, options={cc.OPT_VISIT: 2}, alpha=1.0, beta=c / (2.0 * n * n))
    cc.ccmg_plan_profile(plan, True)
    phi = dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, dev_field(oracle.embed(fv)), phi)
    stats = {k["name"]: k for k in cc.ccmg_plan_kernel_stats(plan)}
    cc.ccmg_plan_profile(plan, False)
    assert r.status == cc.OK
    counted = sum(stats[k]["launches"] for k in ("finest_pre", "finest_post", "finest_fused", "finest_fused_first"))
    assert counted == r.cycles + 1, (counted, r.cycles)
    # from zero (recomputing forms on), the first cycle's end recomputes its
    # pre-smoothing (not stored)
    assert stats["finest_fused_first"]["launches"] == (1 if r.cycles >= 2 else 0)


def test_plan_options_round_trip_and_reject_bad_values():
    plan = cc.Plan(cc.Problem(n=64, bc="D"))
    assert cc.ccmg_plan_get_option(plan, cc.OPT_FUSED) == 1.0
    assert cc.ccmg_plan_get_option(plan, cc.OPT_FUSED_KEEP) == 1.0
    assert cc.ccmg_plan_get_option(plan, cc.OPT_MIXED_INNER) == 3.0
    cc.ccmg_plan_set_option(plan, cc.OPT_MIXED_INNER, 5)
    assert cc.ccmg_plan_get_option(plan, cc.OPT_MIXED_INNER) == 5.0
    for opt, bad in ((cc.OPT_FUSED, 2), (cc.OPT_FUSED_KEEP, -1), (cc.OPT_MIXED_INNER, 0), (cc.OPT_MIXED_INNER, 2.5),
                     (cc.OPT_MIXED_INNER, 9), (99, 1), (cc.OPT_FUSED_KEEP, float("nan"))):
        with pytest.raises(cc.CcmgError):
            cc.ccmg_plan_set_option(plan, opt, bad)


@pytest.mark.parametrize("max_cycles", [1, 2, 100])
def test_statistics_from_the_first_cycle(max_cycles):
    """FP64 solves from zero with the fused launch take f's statistics from
    the first pre-smoothing launch's own loads and check them once the first
    cycle has run: a zero f still gives phi = 0 and OK, a non-finite f
    ENONFINITE, an incompatible singular f EINCOMPAT, and the plan then solves
    as before (its ||f|| summed per tile instead of per workgroup: the
    residual history agrees with the separate pass's to rounding)."""
    n = 512
    plan = cc.Plan(cc.Problem(n=n, bc="DDDD", rtol=1e-10, max_cycles=max_cycles))
    phi = dev_field(np.full((n + 2, n + 2), 5.0))
    r = cc.ccmg_solve(plan, dev_field(oracle.field_zeros(n)), phi)
    assert r.status == cc.OK and r.cycles == 0 and torch.count_nonzero(phi[:, :n + 2]).item() == 0
    for bad in (np.nan, np.inf, -np.inf):
        fv = np.zeros((n, n))
        fv[100, 7] = bad
        with pytest.raises(cc.CcmgError) as e:
            cc.ccmg_solve(plan, dev_field(oracle.embed(fv)), phi)
        assert e.value.status == cc.ENONFINITE
    per = cc.Plan(cc.Problem(n=n, bc="PPPP", rtol=1e-10, max_cycles=max_cycles))
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(per, dev_field(oracle.embed(np.ones((n, n)))), phi)
    assert e.value.status == cc.EINCOMPAT
    fv = W.fourier_modes(n, seed=8, count=16, kmax=8) + 0.1
    r1, p1, _ = solve(n, "DDDD", fv, options={})
    r0, p0, _ = solve(n, "DDDD", fv, options={cc.OPT_FUSED: 0})
    assert r1.status == r0.status == cc.OK and r1.cycles == r0.cycles
    assert np.allclose(r1.history, r0.history, rtol=1e-13, atol=0)
    assert np.array_equal(valid(p1), valid(p0))
    d_phi = dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, dev_field(oracle.embed(fv)), d_phi)
    assert r.status == (cc.OK if max_cycles == 100 else cc.NOT_CONVERGED) and r.cycles == min(max_cycles, r1.cycles)
    assert abs(r.history[1] - r1.history[1]) <= 1e-12 * r1.history[1]


@pytest.mark.parametrize("bc", ["DDNN", "DNPP"])
def test_guess_residual_from_the_first_launch(bc):
    """Non-singular FP64 solves from a guess take the guess's residual norm
    (and f's statistics) in the first pre-smoothing launch and read it with
    the first cycle's: the same iterates as the unfused solve (which takes
    them in separate passes before the first cycle), its history to rounding;
    a guess already within the tolerance returns unchanged after 0 cycles,
    a non-finite guess gives ENONFINITE."""
    n = 512
    kw = {"alpha": 1.0, "beta": 2.0 / (2.0 * n * n)}
    fv = W.gaussian_random_field(n, seed=6)
    guess = 0.5 * np.random.default_rng(3).standard_normal((n, n))
    r0, p0, _ = solve(n, bc, fv, guess, options={cc.OPT_FUSED: 0}, **kw)
    r1, p1, plan = solve(n, bc, fv, guess, **kw)
    assert r0.status == r1.status == cc.OK and r0.cycles == r1.cycles
    assert np.array_equal(valid(p0), valid(p1))
    assert np.allclose(r0.history, r1.history, rtol=1e-12, atol=0)
    assert abs(r1.rel_resid0 - r0.rel_resid0) <= 1e-12 * r0.rel_resid0
    # the converged field as the guess: 0 cycles, the field unchanged
    f = dev_field(oracle.embed(fv))
    before = p1.clone()
    r = cc.ccmg_solve(plan, f, p1, use_guess=True)
    assert r.status == cc.OK and r.cycles == 0 and r.rel_resid0 <= 1e-10
    assert torch.equal(p1[1:n + 1, 1:n + 1], before[1:n + 1, 1:n + 1])
    bad = p1.clone()
    bad[200, 300] = float("nan")
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(plan, f, bad, use_guess=True)
    assert e.value.status == cc.ENONFINITE
    r = cc.ccmg_solve(plan, f, p1, use_guess=True)  # the plan goes on as before
    assert r.status == cc.OK and r.cycles == 0

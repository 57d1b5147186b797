"""Mixed-precision form (FP32 V-cycles, FP64 residual and correction) against
the FP64 oracle: the converged iterate meets the same FP64 tolerances as the
plain form."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
import workloads as W

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


def mixed_plan(n, bc, alpha=0.0, beta=-1.0, **kw):
    return cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=alpha, beta=beta, prec=cc.MIXED, **kw))


@pytest.mark.parametrize("bc", ["PPPP", "DDDD", "NNNN", "DNPP", "PPDD"])
@pytest.mark.parametrize("n", [8, 32, 64, 256, 1024])
def test_mixed_solve_meets_fp64_tolerance(bc, n):
    h = 1.0 / n
    sing = exact.is_singular(0.0, bc)
    fv = np.random.default_rng(21).standard_normal((n, n))
    if sing:
        fv -= fv.mean()
    plan = mixed_plan(n, bc)
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, d_f, d_phi)
    assert r.status == cc.OK and r.rel_resid <= 1e-10
    got = oracle.interior(host(d_phi))
    # the FP64 residual of the returned field, recomputed on the host
    assert exact.relative_residual(got, fv, h, 0.0, -1.0, bc) <= 1.5e-10
    _, ro = oracle.solve(oracle.Problem(n=n, h=h, bc=bc, rtol=1e-10), oracle.embed(fv))
    assert r.cycles <= ro.cycles + 2
    if bc[0] == bc[1] and bc[2] == bc[3]:
        x = exact.transform_solve(fv, h, 0.0, -1.0, bc)
        assert np.linalg.norm(got - x) / np.linalg.norm(x) < 1e-9
    if sing:
        assert abs(got.mean()) < 1e-13 * np.abs(got).max()


@pytest.mark.parametrize("bc", ["PPPP", "DDDD", "DNPP"])
def test_mixed_step_matches_fp64_vcycle(bc):
    """One refinement step = phi + (FP32 V-cycle for A e = r from 0); the FP64
    V-cycle from phi is phi + B r with the same B, so the two agree to FP32
    rounding of the correction."""
    n = 256
    h = 1.0 / n
    fv = np.random.default_rng(22).standard_normal((n, n))
    if "D" not in bc:
        fv -= fv.mean()
    phi0 = oracle.embed(np.random.default_rng(23).standard_normal((n, n)))
    plan = mixed_plan(n, bc)
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(phi0)
    cc.ccmg_vcycle(plan, d_f, d_phi)
    got = oracle.interior(host(d_phi))
    ref = phi0.copy()
    oracle.vcycle(oracle.Problem(n=n, h=h, bc=bc), ref, oracle.embed(fv))
    corr = oracle.interior(ref) - oracle.interior(phi0)
    err = np.linalg.norm(got - oracle.interior(ref)) / np.linalg.norm(corr)
    assert err < 1e-4, err


@pytest.mark.parametrize("c", [0.1, 1.0, 10.0])
def test_mixed_crank_nicolson_helmholtz(c):
    """(1 - (k dt / 2) Lap) phi = g with k dt / h^2 = c, g a Gaussian random field."""
    n = 1024
    h = 1.0 / n
    beta = c * h * h / 2
    g = W.gaussian_random_field(n, seed=1)
    plan = mixed_plan(n, "PPPP", alpha=1.0, beta=beta)
    d_f, d_phi = dev_field(oracle.embed(g)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, d_f, d_phi)
    assert r.status == cc.OK and r.rel_resid <= 1e-10
    x = exact.transform_solve(g, h, 1.0, beta, "PPPP")
    got = oracle.interior(host(d_phi))
    assert np.linalg.norm(got - x) / np.linalg.norm(x) < 1e-9
    assert exact.relative_residual(got, g, h, 1.0, beta, "PPPP") <= 1.5e-10


def test_mixed_large_poisson_periodic():
    n = 4096
    h = 1.0 / n
    fv = W.fourier_modes(n, seed=0)
    plan = mixed_plan(n, "PPPP")
    d_f, d_phi = dev_field(oracle.embed(fv), pad=0), dev_field(oracle.field_zeros(n), pad=0)
    cc.ccmg_plan_autotune(plan, d_f, d_phi)
    r = cc.ccmg_solve(plan, d_f, d_phi)
    assert r.status == cc.OK and r.rel_resid <= 1e-10
    got = oracle.interior(host(d_phi))
    x = exact.transform_solve(fv, h, 0.0, -1.0, "PPPP")
    assert np.linalg.norm(got - x) / np.linalg.norm(x) < 1e-9


def test_mixed_guess_and_history():
    n = 128
    fv = np.random.default_rng(24).standard_normal((n, n))
    plan = mixed_plan(n, "DDDD")
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    r1 = cc.ccmg_solve(plan, d_f, d_phi)
    assert r1.history[0] == 1.0 and all(np.diff(np.log(r1.history)) < 0)
    r2 = cc.ccmg_solve(plan, d_f, d_phi, use_guess=True)
    assert r2.cycles == 0 and r2.rel_resid0 <= 1e-10
    plan1 = mixed_plan(n, "DDDD", max_cycles=2)
    r3 = cc.ccmg_solve(plan1, d_f, dev_field(oracle.field_zeros(n)))
    assert r3.status == cc.NOT_CONVERGED and r3.cycles == 2


@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "DNPP"])
def test_mixed_tile_kernel_matches_row_march(bc):
    """The FP32 inner cycles give the same iterate whether the levels below the
    finest run as row-march bands or as 2-D LDS tiles (bitwise; singular
    problems to rounding, their coarse means being sums grouped by tile)."""
    n = 1024
    fv = np.random.default_rng(33).standard_normal((n, n))
    if exact.is_singular(0.0, bc):
        fv -= fv.mean()
    outs = []
    for mode in ("march", "tile"):
        plan = mixed_plan(n, bc)
        for level in range(1, 4):  # 512, 256, 128 (the tail starts at 64 or 32)
            for kind in (0, 1):
                if mode == "tile":
                    cc.ccmg_plan_set_shape(plan, level, kind, 0, 1)
                else:
                    cc.ccmg_plan_set_shape(plan, level, kind, 16, 1)
        d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
        r = cc.ccmg_solve(plan, d_f, d_phi)
        assert r.status == cc.OK and r.rel_resid <= 1e-10
        outs.append((host(d_phi), r.cycles))
    assert outs[0][1] == outs[1][1]
    if exact.is_singular(0.0, bc):
        a, b = outs[0][0], outs[1][0]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    else:
        assert np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("bc", ["PPPP", "DDDD", "DNPP"])
@pytest.mark.parametrize("m", [1, 2, 3])
def test_mixed_steps_with_inner_cycles_match_oracle(bc, m):
    """Refinement steps of several FP32 V-cycles from a zero correction: the
    first step runs min(2, m) cycles, the second (its contraction now known,
    the tolerance far away) m; from phi = 0 the two steps together equal
    min(2, m) + m oracle V-cycles from zero, to FP32 rounding."""
    n = 256
    h = 1.0 / n
    sing = exact.is_singular(0.0, bc)
    fv = np.random.default_rng(41).standard_normal((n, n))
    if sing:
        fv -= fv.mean()
    plan = mixed_plan(n, bc, max_cycles=2, rtol=1e-14)  # the tolerance asks for more cycles
    cc.ccmg_plan_set_option(plan, cc.OPT_MIXED_INNER, m)
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, d_f, d_phi)
    total = min(2, m) + m
    assert r.status == cc.NOT_CONVERGED and r.cycles == 2 and r.inner_cycles == total
    ref = oracle.field_zeros(n)
    for _ in range(total):
        oracle.vcycle(oracle.Problem(n=n, h=h, bc=bc), ref, oracle.embed(fv))
    got, want = oracle.interior(host(d_phi)), oracle.interior(ref)
    if sing:
        got, want = got - got.mean(), want - want.mean()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < 1e-4, err


@pytest.mark.parametrize("bc", ["PPPP", "DDDD", "NNNN", "DNPP"])
def test_mixed_inner_cycles_against_one_cycle_steps(bc):
    """Several FP32 cycles per refinement step reach the same FP64 tolerance
    and the same solution as one cycle per step, in fewer steps and about the
    same number of FP32 cycles; the fused launch joins the inner cycles."""
    n = 1024
    h = 1.0 / n
    sing = exact.is_singular(0.0, bc)
    fv = W.gaussian_random_field(n, seed=5)
    if sing:
        fv -= fv.mean()
    outs = {}
    for m in ("1", "3"):
        plan = mixed_plan(n, bc)
        cc.ccmg_plan_set_option(plan, cc.OPT_MIXED_INNER, int(m))
        d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
        r = cc.ccmg_solve(plan, d_f, d_phi)
        assert r.status == cc.OK and r.rel_resid <= 1e-10
        got = oracle.interior(host(d_phi))
        assert exact.relative_residual(got, fv, h, 0.0, -1.0, bc) <= 1.5e-10
        cc.ccmg_plan_profile(plan, True)
        cc.ccmg_solve(plan, d_f, dev_field(oracle.field_zeros(n)))
        stats = {k["name"]: k for k in cc.ccmg_plan_kernel_stats(plan)}
        cc.ccmg_plan_profile(plan, False)
        outs[m] = (r, got, stats)
    (r1, g1, s1), (r3, g3, s3) = outs["1"], outs["3"]
    assert r1.inner_cycles == r1.cycles and s1["mixed_finest_fused"]["launches"] == 0
    assert r3.cycles < r1.cycles
    assert r3.inner_cycles <= r1.inner_cycles + 3
    assert s3["mixed_finest_fused"]["launches"] >= r3.inner_cycles - r3.cycles
    assert np.linalg.norm(g3 - g1) / np.linalg.norm(g1) < 1e-9
    if sing:
        assert abs(g3.mean()) < 1e-13 * np.abs(g3).max()


@pytest.mark.parametrize("max_cycles", [1, 100])
def test_mixed_statistics_and_start_residual_from_the_start_pass(max_cycles):
    """MIXED solves take f's statistics in the start pass (the FP64 residual
    rounded to FP32) and check them, with the start's residual, once the
    first step has run: zero f gives phi = 0 and OK, a non-finite f or guess
    ENONFINITE, an incompatible singular f EINCOMPAT, a guess within the
    tolerance returns unchanged after 0 steps, and a plan goes on solving."""
    n = 256
    plan = mixed_plan(n, "DDNN", rtol=1e-10, max_cycles=max_cycles)
    phi = dev_field(np.full((n + 2, n + 2), 4.0))
    r = cc.ccmg_solve(plan, dev_field(oracle.field_zeros(n)), phi)
    assert r.status == cc.OK and r.cycles == 0 and torch.count_nonzero(phi[:, :n + 2]).item() == 0
    bad = np.zeros((n, n))
    bad[17, 3] = np.inf
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(plan, dev_field(oracle.embed(bad)), phi)
    assert e.value.status == cc.ENONFINITE
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(mixed_plan(n, "PPPP", max_cycles=max_cycles), dev_field(oracle.embed(np.ones((n, n)))), phi)
    assert e.value.status == cc.EINCOMPAT
    fv = W.fourier_modes(n, seed=2, count=16, kmax=8) + 0.1
    f = dev_field(oracle.embed(fv))
    phi = dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, f, phi)
    if max_cycles == 1:
        assert r.status == cc.NOT_CONVERGED and r.cycles == 1
        return
    assert r.status == cc.OK and r.rel_resid <= 1e-10 and r.rel_resid0 == 1.0
    before = phi.clone()
    r = cc.ccmg_solve(plan, f, phi, use_guess=True)
    assert r.status == cc.OK and r.cycles == 0 and r.rel_resid0 <= 1e-10
    assert torch.equal(phi[1:n + 1, 1:n + 1], before[1:n + 1, 1:n + 1])
    nan_guess = phi.clone()
    nan_guess[9, 9] = float("nan")
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(plan, f, nan_guess, use_guess=True)
    assert e.value.status == cc.ENONFINITE

"""Crank-Nicolson diffusion steps (Sec. 3.4) through the C ABI against the
oracle: the right-hand side kernel element by element, whole steps of the
paper's Gaussian test problem, the closed-form factor of an eigenmode at the
benchmark's full size, and the mixed-precision plan."""
import numpy as np
import pytest
import torch

import oracle
from test_oracle_cn import gaussian, modes

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


def cn_plan(n, bc, c, prec=cc.FP64, rtol=1e-12):
    h = 1.0 / n
    return cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=1.0, beta=c * h * h / 2, rtol=rtol, prec=prec))


@pytest.mark.parametrize("bc", ["NNNN", "PPPP", "DDDD", "DNPP", "PPDN"])
@pytest.mark.parametrize("n", [2, 8, 64, 512])
def test_cn_rhs_matches_oracle(bc, n):
    """Several row bands and column blocks, a ragged last block (n < 256)."""
    h = 1.0 / n
    c = 3.0
    phi = oracle.embed(np.random.default_rng(n).standard_normal((n, n)))
    plan = cn_plan(n, bc, c)
    d_phi, d_f = dev_field(phi), dev_field(oracle.field_zeros(n))
    cc.ccmg_cn_rhs(plan, d_phi, d_f)
    torch.cuda.synchronize()
    want = oracle.interior(oracle.cn_rhs(n, h, c * h * h / 2, bc, phi.copy()))
    got = oracle.interior(host(d_f))
    assert np.abs(got - want).max() <= 1e-14 * (1 + 4 * c) * np.abs(oracle.interior(phi)).max() * 4
    # ghosts of f untouched
    assert np.all(host(d_f)[0, :] == 0) and np.all(host(d_f)[:, 0] == 0)


@pytest.mark.parametrize("bc", ["NNNN", "PPPP", "DDNN"])
def test_cn_gaussian_steps_match_oracle_and_the_exact_solution(bc):
    """The paper's test problem on 128^2 with C = 2 up to t = 0.005: every
    step's result against the oracle's step, and (Neumann, periodic sides)
    the end state against the exact Gaussian (within 0.2% of its peak)."""
    n = 128
    h = 1.0 / n
    t_end = 0.005
    steps = int(np.ceil(t_end / (2.0 * h * h)))
    dt = t_end / steps
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=1.0, beta=dt / 2, rtol=1e-12))
    po = oracle.Problem(n=n, h=h, alpha=1.0, beta=dt / 2, bc=bc, rtol=1e-12)
    ref = oracle.embed(gaussian(n, 0.0))
    d_phi, d_work = dev_field(ref.copy()), dev_field(oracle.field_zeros(n))
    for s in range(steps):
        r = cc.ccmg_cn_step(plan, d_phi, d_work)
        ref, ro = oracle.cn_step(po, ref)
        assert r.status == cc.OK and ro.status == oracle.OK
        if s % 10 == 0 or s == steps - 1:
            got = oracle.interior(host(d_phi))
            assert np.abs(got - oracle.interior(ref)).max() <= 1e-10 * np.abs(oracle.interior(ref)).max()
    if "D" not in bc:  # homogeneous Dirichlet sides hold 0, not the background 1 of the exact Gaussian
        amp = 1e-4 / (t_end + 1e-4)
        assert np.abs(oracle.interior(host(d_phi)) - gaussian(n, t_end)).max() < 2e-3 * amp


@pytest.mark.parametrize("prec", [cc.FP64, cc.MIXED])
def test_cn_step_eigenmode_factor_at_full_size(prec):
    """8192^2 Neumann, C = 2, the benchmark's launch configuration (autotuned
    plan): one step multiplies a discrete eigenmode by the closed-form factor."""
    n = 8192
    c = 2.0
    h = 1.0 / n
    beta = c * h * h / 2
    phi0, lam = modes(n, "NNNN")
    g = (1 + beta * lam) / (1 - beta * lam)
    plan = cn_plan(n, "NNNN", c, prec=prec, rtol=1e-10)
    d_phi = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
    d_phi[1:n + 1, 1:n + 1] = torch.from_numpy(phi0).cuda()
    d_work = torch.zeros_like(d_phi)
    cc.ccmg_plan_autotune(plan, d_phi, d_work)
    d_phi[1:n + 1, 1:n + 1] = torch.from_numpy(phi0).cuda()
    r = cc.ccmg_cn_step(plan, d_phi, d_work)
    assert r.status == cc.OK and r.rel_resid <= 1e-10
    got = d_phi[1:n + 1, 1:n + 1].cpu().numpy()
    assert np.abs(got - g * phi0).max() <= 1e-9


def test_cn_mixed_plan_matches_fp64_plan():
    n = 256
    phi0 = np.random.default_rng(5).standard_normal((n, n))
    outs = []
    for prec in (cc.FP64, cc.MIXED):
        plan = cn_plan(n, "DNPP", 10.0, prec=prec, rtol=1e-11)
        d_phi, d_work = dev_field(oracle.embed(phi0)), dev_field(oracle.field_zeros(n))
        r = cc.ccmg_cn_step(plan, d_phi, d_work)
        assert r.status == cc.OK
        outs.append(oracle.interior(host(d_phi)))
    assert np.abs(outs[0] - outs[1]).max() <= 1e-9 * np.abs(outs[0]).max()


def test_cn_step_rejects_bad_arguments():
    n = 32
    plan = cc.Plan(cc.Problem(n=n, bc=("N",) * 4, alpha=0.5, beta=0.01))
    d_phi, d_work = dev_field(oracle.field_zeros(n)), dev_field(oracle.field_zeros(n))
    with pytest.raises(Exception):
        cc.ccmg_cn_step(plan, d_phi, d_work)  # alpha != 1
    plan1 = cn_plan(n, "NNNN", 1.0)
    with pytest.raises(Exception):
        cc.ccmg_cn_rhs(plan1, d_phi, d_phi)  # in place


@pytest.mark.parametrize("bc", ["NNNN", "DDDD", "DNPP", "PPPP"])
@pytest.mark.parametrize("n", [64, 1024])
def test_cn_step_forms_the_rhs_in_its_first_launch(bc, n):
    """FP64 steps with the fused launch form the right-hand side in the first
    pre-smoothing launch (from the old level it loads anyway): d_work ends up
    holding exactly ccmg_cn_rhs's right-hand side, and the new level is bitwise
    that of the separate pass followed by ccmg_solve from the old level."""
    h = 1.0 / n
    c = 2.0
    phi0 = oracle.embed(np.random.default_rng(n + 1).standard_normal((n, n)) + 1.0)
    plan = cn_plan(n, bc, c, rtol=1e-10)
    d_phi, d_work = dev_field(phi0), dev_field(np.full((n + 2, n + 2), 7.0))
    r1 = cc.ccmg_cn_step(plan, d_phi, d_work)
    ref = cn_plan(n, bc, c, rtol=1e-10)
    cc.ccmg_plan_set_option(ref, cc.OPT_FUSED, 0)  # (the two-pass form)
    e_phi, e_f = dev_field(phi0), dev_field(oracle.field_zeros(n))
    cc.ccmg_cn_rhs(ref, e_phi, e_f)
    plan2 = cn_plan(n, bc, c, rtol=1e-10)
    r0 = cc.ccmg_solve(plan2, e_f, e_phi, use_guess=True)
    torch.cuda.synchronize()
    assert r1.status == r0.status == cc.OK and r1.cycles == r0.cycles
    assert np.array_equal(oracle.interior(host(d_work)), oracle.interior(host(e_f)))
    assert np.array_equal(oracle.interior(host(d_phi)), oracle.interior(host(e_phi)))
    assert abs(r1.rel_resid0 - r0.rel_resid0) <= 1e-12 * r0.rel_resid0

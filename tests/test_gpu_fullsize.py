"""The benchmark's workloads at their full sizes, in the launch configuration
the benchmark times (autotuned plans, fused finest launches), checked against
what the oracle side fixes at any size: the FP64 residual of the returned
field recomputed on the host, and the exact discrete solution from the fast
transforms (FFT periodic, DST Dirichlet) -- relative residual <= 1e-10,
solution error <= 1e-9.  The batched workload is checked problem by problem
against the CPU oracle's own multigrid solves."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


def to_dev(fv):
    n = fv.shape[0]
    t = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
    t[1:n + 1, 1:n + 1] = torch.from_numpy(fv).cuda()
    return t


def valid(t):
    n = t.shape[0] - 2
    return t[1:n + 1, 1:n + 1].cpu().numpy()


def check_against_transforms(prob, fv, bc, sol_tol=1e-9, setup=None):
    n = prob.n
    plan = cc.Plan(prob)
    if setup is not None:  # plan options, set before tuning as the benchmark does
        setup(plan)
    f, phi = to_dev(fv), to_dev(np.zeros((n, n)))
    cc.ccmg_plan_autotune(plan, f, phi)
    r = cc.ccmg_solve(plan, f, phi)
    assert r.status == cc.OK and r.rel_resid <= 1e-10, r
    got = valid(phi)
    del plan, f, phi
    torch.cuda.empty_cache()
    h = 1.0 / n
    # the residual of the returned field, recomputed in FP64 on the host
    assert exact.relative_residual(got, fv, h, prob.alpha, prob.beta, bc) <= 1.05e-10
    x = exact.transform_solve(fv, h, prob.alpha, prob.beta, bc)
    if exact.is_singular(prob.alpha, bc):
        assert abs(got.mean()) <= 1e-13 * np.abs(got).max()
    err = np.linalg.norm(got - x) / np.linalg.norm(x)
    assert err <= sol_tol, err
    return r


def test_plain_poisson_4096_periodic():
    """4096^2 periodic, 64 Fourier modes |k| <= 32, seed 0."""
    n = 4096
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    r = check_against_transforms(cc.Problem(n=n, bc="P", rtol=1e-10), fv, "PPPP")
    assert r.cycles <= 13


def test_plain_poisson_8192_dirichlet():
    """The headline: 8192^2 Dirichlet, 64 Fourier modes |k| <= 32, seed 0."""
    n = 8192
    print(f"plain FP64 Poisson n={n} Dirichlet", flush=True)
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    check_against_transforms(cc.Problem(n=n, bc="D", rtol=1e-10), fv, "DDDD")


@pytest.mark.parametrize("c", [0.1, 1.0, 10.0])
def test_mixed_crank_nicolson_8192(c):
    """(1 - (k dt / 2) Lap) phi = g, k dt / h^2 = c, Gaussian random field g."""
    n = 8192
    g = W.gaussian_random_field(n, seed=0)
    prob = cc.Problem(n=n, bc="P", alpha=1.0, beta=c / (2.0 * n * n), rtol=1e-10, prec=cc.MIXED)
    check_against_transforms(prob, g, "PPPP")


@pytest.mark.parametrize("c", [0.1, 1.0, 10.0])
def test_plain_fp64_helmholtz_8192(c):
    """The same Crank-Nicolson Helmholtz solves in plain FP64 (the baseline
    of the mixed form's speed-up), autotuned, fused finest launches."""
    n = 8192
    print(f"plain FP64 Helmholtz n={n} c={c}", flush=True)
    g = W.gaussian_random_field(n, seed=0)
    prob = cc.Problem(n=n, bc="P", alpha=1.0, beta=c / (2.0 * n * n), rtol=1e-10, prec=cc.FP64)
    check_against_transforms(prob, g, "PPPP")


def test_mixed_poisson_8192_dirichlet():
    """The mixed form on the 8192^2 Dirichlet Poisson workload (FP32 cycles,
    FP64 refinement), against the DST solve."""
    n = 8192
    print(f"mixed Poisson n={n} Dirichlet", flush=True)
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    check_against_transforms(cc.Problem(n=n, bc="D", rtol=1e-10, prec=cc.MIXED), fv, "DDDD")


def test_mixed_poisson_4096_periodic():
    """The mixed form on the 4096^2 periodic Poisson workload (singular: the
    returned field has zero mean), against the FFT solve."""
    n = 4096
    print(f"mixed Poisson n={n} periodic", flush=True)
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    check_against_transforms(cc.Problem(n=n, bc="P", rtol=1e-10, prec=cc.MIXED), fv, "PPPP")


@pytest.mark.parametrize("n,side,bc",[(8192, "D", "DDDD"), (4096, "P", "PPPP")])
def test_full_multigrid_start_full_size(n, side, bc):
    """The full multigrid start (CCMG_OPT_FMG = 1) on the benchmark's two
    problems (64 Fourier modes |k| <= 32, seed 0), autotuned with the option
    set, fused finest launches: the same bar as the zero start, in fewer
    cycles."""
    print(f"FMG start n={n} {bc}", flush=True)
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    r = check_against_transforms(cc.Problem(n=n, bc=side, rtol=1e-10), fv, bc,
                                 setup=lambda plan: cc.ccmg_plan_set_option(plan, cc.OPT_FMG, 1))
    assert r.cycles <= 9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nb", [4, 8])
def test_exact_bottom_full_size(nb, prec):
    """The exact 4^2 or 8^2 bottom solve on the benchmark's 4096^2 periodic
    problem, FP64 and mixed, autotuned: the returned field (zero mean) against
    the FFT solve."""
    n = 4096
    print(f"exact bottom {nb}^2 n={n} {prec}", flush=True)
    fv = W.fourier_modes(n, seed=0, count=64, kmax=32)
    prob = cc.Problem(n=n, bc="P", rtol=1e-10, prec=cc.FP64 if prec == "fp64" else cc.MIXED)
    check_against_transforms(prob, fv, "PPPP", setup=lambda plan: cc.ccmg_plan_set_bottom(plan, nb))


def test_batched_512_against_oracle_solves():
    """The 512-problem batch (sizes 32..1024, per-axis periodic / Dirichlet,
    16 modes |k| <= 8), one batched solve, each result against the CPU
    oracle's solve of the same problem."""
    items = W.batch(seed=0)
    fs = [to_dev(it.f) for it in items]
    phis = [to_dev(np.zeros((it.n, it.n))) for it in items]
    batch = cc.Batch([cc.Problem(n=it.n, bc=it.bc, rtol=1e-10, prec=cc.MIXED) for it in items])
    cc.ccmg_batch_autotune(batch, fs, phis)
    res, info = cc.ccmg_batch_solve(batch, fs, phis)
    assert info["converged"] == len(items)
    worst = 0.0
    for it, r, phi in zip(items, res, phis):
        assert r.status == cc.OK and r.rel_resid <= 1e-10
        got = valid(phi)
        ref, ro = oracle.solve(oracle.Problem(n=it.n, h=1.0 / it.n, bc=it.bc, rtol=1e-10), oracle.embed(it.f))
        assert ro.status == 0
        ref = oracle.interior(ref)
        if "D" not in it.bc:  # singular: both return the zero-mean representative
            ref = ref - ref.mean()
        worst = max(worst, np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert worst <= 1e-9, worst


@pytest.mark.parametrize("bc,prec", [("PPPP", "fp64"), ("DNDN", "mixed")])
def test_maximum_size_16384(bc, prec):
    """The largest grid a plan accepts (16384^2, 2 GiB per field), autotuned.
    A white-noise right-hand side: smooth data would put the FP64 residual
    floor of even the exact solution near 1e-10 at this size, rough data keep
    it far below.  Checked by what holds at any size: the returned field's
    residual recomputed in FP64 on the host, zero mean when singular."""
    n = 16384
    print(f"max size n={n} bc={bc} prec={prec}", flush=True)
    fv = np.random.default_rng(5).standard_normal((n, n))
    if exact.is_singular(0.0, bc):
        fv -= fv.mean()
    prob = cc.Problem(n=n, bc=tuple(bc), rtol=1e-10, prec=cc.FP64 if prec == "fp64" else cc.MIXED)
    plan = cc.Plan(prob)
    f, phi = to_dev(fv), to_dev(np.zeros((n, n)))
    cc.ccmg_plan_autotune(plan, f, phi)
    r = cc.ccmg_solve(plan, f, phi)
    assert r.status == cc.OK and r.rel_resid <= 1e-10, r
    got = valid(phi)
    del plan, f, phi
    torch.cuda.empty_cache()
    assert exact.relative_residual(got, fv, 1.0 / n, 0.0, -1.0, bc) <= 1.05e-10
    if exact.is_singular(0.0, bc):
        assert abs(got.mean()) <= 1e-13 * np.abs(got).max()

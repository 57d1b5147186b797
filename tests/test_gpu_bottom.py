"""Exact bottom solve (ccmg_plan_set_bottom): the V-cycle ends on a 4 x 4 or
8 x 8 level with phi = A^-1 f.  Compared with the oracle's cycle that ends the
same way (a dense Gaussian elimination there, the inverse from Gauss-Jordan
on the GPU), cycle by cycle; whole solves against the exact discrete
solution; FP64 and mixed plans; the argument checks."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")

BCS = ["DDDD", "NNNN", "PPPP", "DNPP", "PPND", "NDDN"]
ABS = [(0.0, -1.0), (1.0, 0.5 / 64)]


def dev_field(a, pad=3):
    n = a.shape[0] - 2
    t = torch.zeros((n + 2, n + 2 + pad), dtype=torch.float64, device="cuda")
    t[:, :n + 2] = torch.from_numpy(a).cuda()
    return t


def host(t):
    n = t.shape[0] - 2
    return t[:, :n + 2].cpu().numpy()


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def make(n, bc, ab, nb, prec=cc.FP64, **kw):
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=ab[0], beta=ab[1], prec=prec, **kw))
    cc.ccmg_plan_set_bottom(plan, nb)
    return plan


@pytest.mark.parametrize("ab", ABS)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n,nb", [(4, 4), (8, 4), (8, 8), (32, 4), (32, 8), (64, 4), (64, 8), (512, 4), (512, 8)])
def test_vcycle_iterates_match_oracle(n, nb, bc, ab):
    """Three cycles from a random start; the levels above the bottom are the
    ones the relaxation-bottom parity tests cover, so differences are the two
    inverses' rounding, carried up the hierarchy."""
    print(f"bottom vcycle n={n} bc={bc} ab={ab} nb={nb}", flush=True)
    plan = make(n, bc, ab, nb)
    p = oracle.Problem(n=n, h=1.0 / n, alpha=ab[0], beta=ab[1], bc=bc, n_bottom=nb)
    fv = np.random.default_rng(21).standard_normal((n, n))
    if p.singular:
        fv -= fv.mean()
    f = oracle.embed(fv)
    ref = oracle.embed(np.random.default_rng(22).standard_normal((n, n)))
    d_f, d_phi = dev_field(f), dev_field(ref)
    for k in range(3):
        cc.ccmg_vcycle(plan, d_f, d_phi)
        oracle.vcycle(p, ref, f)
        e = rel_max(oracle.interior(host(d_phi)), oracle.interior(ref))
        assert e < 1e-11, (k, e)


@pytest.mark.parametrize("nb", [4, 8])
@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "DNPP", "NNNN"])
def test_bottom_on_the_finest_level_is_the_exact_solution(bc, nb):
    """n = n_bottom: one cycle is the direct solve (zero mean if singular)."""
    n = nb
    ab = (0.0, -1.0)
    plan = make(n, bc, ab, nb)
    fv = np.random.default_rng(23).standard_normal((n, n))
    if exact.is_singular(*ab[:1], bc):
        fv -= fv.mean()
    d_f = dev_field(oracle.embed(fv))
    d_phi = dev_field(oracle.embed(np.random.default_rng(24).standard_normal((n, n))))
    cc.ccmg_vcycle(plan, d_f, d_phi)
    x = exact.dense_solve(fv, 1.0 / n, *ab, bc)
    assert rel_max(oracle.interior(host(d_phi)), x) < 1e-13


@pytest.mark.parametrize("prec", [cc.FP64, cc.MIXED])
@pytest.mark.parametrize("bc", ["DDDD", "PPPP", "PPND"])
@pytest.mark.parametrize("n", [256, 2048])
def test_solve_with_exact_bottom(n, bc, prec):
    """Whole solves: same tolerance, no more cycles than the relaxation
    bottom, and the oracle's cycle count."""
    print(f"bottom solve n={n} bc={bc} prec={prec}", flush=True)
    fv = W.fourier_modes(n, seed=4, count=16, kmax=8)
    singular = exact.is_singular(0.0, bc)
    if singular:
        fv = fv - fv.mean()
    out = {}
    for nb in (2, 8):
        plan = make(n, bc, (0.0, -1.0), nb, prec=prec)
        d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
        r = cc.ccmg_solve(plan, d_f, d_phi)
        assert r.status == cc.OK and r.rel_resid <= 1e-10
        out[nb] = (r, oracle.interior(host(d_phi)))
    assert out[8][0].cycles <= out[2][0].cycles
    assert rel_max(out[8][1], out[2][1]) < 1e-8
    if prec == cc.FP64 and n == 256:
        _, ro = oracle.solve(oracle.Problem(n=n, h=1.0 / n, bc=bc, n_bottom=8), oracle.embed(fv))
        assert ro.cycles == out[8][0].cycles


def test_helmholtz_cn_and_projection_with_exact_bottom():
    """The other entry points of a plan use the same bottom."""
    n = 256
    h = 1.0 / n
    plan = make(n, "NNNN", (1.0, 2.0 * h * h), 4)
    x = W.gaussian_random_field(n, seed=5)
    phi = dev_field(oracle.embed(x))
    work = dev_field(oracle.field_zeros(n))
    r = cc.ccmg_cn_step(plan, phi, work)
    assert r.status == cc.OK
    ref = oracle.embed(x.copy())
    oracle.cn_step(oracle.Problem(n=n, h=h, alpha=1.0, beta=2.0 * h * h, bc="NNNN", n_bottom=4), ref)
    assert rel_max(oracle.interior(host(phi)), oracle.interior(ref)) < 1e-9


def test_set_bottom_rejects_bad_arguments():
    plan = cc.Plan(cc.Problem(n=64, bc="P"))
    for nb in (0, 1, 3, 16, 32, 64):
        with pytest.raises(cc.CcmgError):
            cc.ccmg_plan_set_bottom(plan, nb)
    small = cc.Plan(cc.Problem(n=4, bc="D"))
    with pytest.raises(cc.CcmgError):
        cc.ccmg_plan_set_bottom(small, 8)
    # indefinite: alpha and beta of opposite signs
    ind = cc.Plan(cc.Problem(n=64, bc="D", alpha=1.0, beta=-1.0))
    with pytest.raises(cc.CcmgError):
        cc.ccmg_plan_set_bottom(ind, 8)


def test_relaxation_bottom_restored_bitwise():
    """n_bottom = 2 after 8: the same iterates as a plan never changed."""
    n, bc = 128, "DNPP"
    fv = np.random.default_rng(25).standard_normal((n, n))
    res = []
    for steps in ([], [8, 2]):
        plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), max_cycles=4, rtol=0.0))
        for nb in steps:
            cc.ccmg_plan_set_bottom(plan, nb)
        d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
        cc.ccmg_solve(plan, d_f, d_phi)
        res.append(host(d_phi))
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("nb", [4, 8])
def test_autotune_keeps_the_inverse(nb):
    """Autotuning clears the plan's scratch, not the bottom's inverse: a tuned
    plan converges like an untuned one, to the same iterate."""
    n, bc = 512, "PPPP"
    fv = W.fourier_modes(n, seed=6, count=64, kmax=32)
    fv = fv - fv.mean()
    got = []
    for tune in (False, True):
        plan = make(n, bc, (0.0, -1.0), nb)
        d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
        if tune:
            cc.ccmg_plan_autotune(plan, d_f, d_phi)
        r = cc.ccmg_solve(plan, d_f, d_phi)
        assert r.status == cc.OK
        got.append((r.cycles, oracle.interior(host(d_phi))))
    assert got[0][0] == got[1][0]
    assert rel_max(got[1][1], got[0][1]) < 1e-11

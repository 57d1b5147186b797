"""Two levels' pre-smoothing in one launch (2-D tiles with halos for both
levels): the same iterates as the levels' own launches -- bitwise for
non-singular problems; for singular ones the coarse right-hand side's mean
(zero up to rounding) is not removed between the two levels, so there they
agree to rounding -- for FP64 and mixed plans, Poisson and Helmholtz."""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import exact
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


def dev_field(a, pad=5):
    n = a.shape[0] - 2
    t = torch.zeros((n + 2, n + 2 + pad), dtype=torch.float64, device="cuda")
    t[:, :n + 2] = torch.from_numpy(a).cuda()
    return t


def host(t):
    n = t.shape[0] - 2
    return t[:, :n + 2].cpu().numpy()


def solve(n, bc, fv, monkeypatch, pair, **kw):
    monkeypatch.setenv("CCMG_PAIR", "1" if pair else "0")
    plan = cc.Plan(cc.Problem(n=n, bc=tuple(bc), rtol=1e-10, **kw))
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, d_f, d_phi)
    return r, host(d_phi)


@pytest.mark.parametrize("bc", ["DDDD", "DNDN", "PPDN", "PPPP", "NNNN"])
@pytest.mark.parametrize("n", [256, 1024])
@pytest.mark.parametrize("prec", [cc.FP64, cc.MIXED])
def test_pair_matches_separate_launches(bc, n, prec, monkeypatch):
    fv = W.fourier_modes(n, seed=3, count=16, kmax=8)
    if exact.is_singular(0.0, bc):
        fv = fv - fv.mean()
    r0, p0 = solve(n, bc, fv, monkeypatch, False, prec=prec)
    r1, p1 = solve(n, bc, fv, monkeypatch, True, prec=prec)
    assert r0.status == r1.status == cc.OK
    assert r0.cycles == r1.cycles
    if exact.is_singular(0.0, bc):
        assert np.abs(p1 - p0).max() <= (1e-11 if prec == cc.FP64 else 1e-9) * np.abs(p0).max()
        # residuals well above the FP64 floor agree closely; near the floor
        # (last cycles) rounding differences are relatively large
        h0, h1 = np.array(r0.history), np.array(r1.history)
        big = h0 > 1e-8
        # (mixed: FP32 corrections, whose rounding moves the residual more)
        assert np.allclose(h0[big], h1[big], rtol=1e-6 if prec == cc.FP64 else 1e-2, atol=0)
    else:
        assert np.array_equal(p0, p1) and r0.history == r1.history


@pytest.mark.parametrize("bc", ["DDPP", "PPPP", "NNDD"])
def test_pair_helmholtz_and_oracle(bc, monkeypatch):
    n = 512
    h = 1.0 / n
    alpha, beta = 1.0, 2.0 * h * h
    fv = W.gaussian_random_field(n, seed=2)
    r, p = solve(n, bc, fv, monkeypatch, True, alpha=alpha, beta=beta)
    assert r.status == cc.OK and r.rel_resid <= 1e-10
    x = exact.transform_solve(fv, h, alpha, beta, bc)
    assert np.linalg.norm(oracle.interior(p) - x) / np.linalg.norm(x) < 1e-9

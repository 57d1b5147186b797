"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Kernel-level steps (one relaxation launch, residual, restriction,
prolongation, ghost fill) are compared element by element with the oracle's
own step on the same seeded input; V-cycles iterate by iterate; solves
against the oracle's solve and the exact discrete solution."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")

BCS = ["PPPP", "DDDD", "NNNN", "DNPP", "PPND", "DDNN"]
SIZES = [2, 4, 8, 32, 64, 128, 256, 512]


def dev_field(a):
    """oracle field (n+2, n+2) -> device tensor with a padded pitch (ghosts copied)."""
    n = a.shape[0] - 2
    t = torch.zeros((n + 2, n + 2 + 5), dtype=torch.float64, device="cuda")
    t[:, :n + 2] = torch.from_numpy(a).cuda()
    return t


def host(t):
    n = t.shape[0] - 2
    return t[:, :n + 2].cpu().numpy()


def rand(n, seed, scale=1.0):
    return oracle.embed(np.random.default_rng(seed).standard_normal((n, n)) * scale)


def rel_max(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def plan_for(n, bc, alpha=0.0, beta=-1.0, **kw):
    return cc.Plan(cc.Problem(n=n, bc=tuple(bc), alpha=alpha, beta=beta, **kw))


def oprob(n, bc, alpha=0.0, beta=-1.0, **kw):
    return oracle.Problem(n=n, h=1.0 / n, alpha=alpha, beta=beta, bc=tuple(bc), **kw)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [4, 8, 64, 256, 512])
@pytest.mark.parametrize("iters", [1, 2])
def test_smooth_matches_oracle(bc, n, iters):
    plan = plan_for(n, bc)
    phi, f = rand(n, 1), rand(n, 2, n * n)
    out = dev_field(np.zeros_like(phi))
    cc.ccmg_smooth(plan, 0, iters, dev_field(f), dev_field(phi), out)
    torch.cuda.synchronize()
    want = oracle.smooth(oprob(n, bc), phi.copy(), f, iters)
    got = host(out)
    assert rel_max(oracle.interior(got), oracle.interior(want)) < 1e-13


@pytest.mark.parametrize("bc", ["PPPP", "DNDN"])
def test_smooth_helmholtz_and_coarse_level(bc):
    n, level = 512, 2  # level 2 of a 512 plan: 128 cells, h = 4/512
    plan = plan_for(n, bc, alpha=1.0, beta=0.5 * 1.0 / n)
    m = n >> level
    phi, f = rand(m, 3), rand(m, 4)
    out = dev_field(np.zeros_like(phi))
    cc.ccmg_smooth(plan, level, 2, dev_field(f), dev_field(phi), out)
    p = oracle.Problem(n=n, h=1.0 / n, alpha=1.0, beta=0.5 / n, bc=tuple(bc))
    want = oracle.smooth(p, phi.copy(), f, 2, level=level)
    assert rel_max(oracle.interior(host(out)), oracle.interior(want)) < 1e-13


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [2, 8, 128, 512])
def test_residual_matches_oracle(bc, n):
    plan = plan_for(n, bc, alpha=0.3, beta=-0.7)
    phi, f = rand(n, 5), rand(n, 6, n * n)
    r = dev_field(np.zeros_like(phi))
    cc.ccmg_residual(plan, 0, dev_field(f), dev_field(phi), r)
    want = oracle.residual(oprob(n, bc, 0.3, -0.7), phi.copy(), f)
    got = oracle.interior(host(r))
    assert np.max(np.abs(got - oracle.interior(want))) < 1e-12 * np.max(np.abs(oracle.interior(f)))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [4, 64, 256, 512])
def test_restrict_residual_matches_oracle(bc, n):
    plan = plan_for(n, bc)
    phi, f = rand(n, 7), rand(n, 8, n * n)
    fc = dev_field(oracle.field_zeros(n // 2))
    cc.ccmg_restrict_residual(plan, 0, dev_field(f), dev_field(phi), fc)
    p = oprob(n, bc)
    want = oracle.restrict(oracle.residual(p, phi.copy(), f))
    got = oracle.interior(host(fc))
    assert np.max(np.abs(got - oracle.interior(want))) < 1e-12 * np.max(np.abs(oracle.interior(f)))


@pytest.mark.parametrize("n,level", [(4, 0), (8, 1), (64, 0), (64, 1), (512, 0), (512, 1), (2048, 0), (2048, 1)])
def test_restrict_matches_oracle(n, level):
    """The standalone four-cell average (Sec. 3.3) equals the oracle's
    restriction bit for bit (same additions in the same order), on the finest
    level and the one below it, down to the 2 x 2 level that ends the
    hierarchy; the coarse ghosts and the fine array are left alone."""
    plan = plan_for(n, "DDDD")
    nl = n >> level
    fine = rand(nl, 30 + nl)
    d_fine = dev_field(fine)
    coarse = dev_field(np.full((nl // 2 + 2, nl // 2 + 2), 7.0))
    cc.ccmg_restrict(plan, level, d_fine, coarse)
    want = oracle.restrict(fine.copy())
    got = host(coarse)
    assert np.array_equal(oracle.interior(got), oracle.interior(want))
    assert np.all(got[0, :] == 7.0) and np.all(got[-1, :] == 7.0) and np.all(got[:, 0] == 7.0)
    assert np.array_equal(host(d_fine), fine)


def test_restrict_rejects_bad_arguments():
    plan = plan_for(64, "PPPP")
    fine = dev_field(oracle.field_zeros(64))
    with pytest.raises(cc.CcmgError):  # overlapping arrays
        cc.ccmg_restrict(plan, 0, fine, fine[:34, :34])
    with pytest.raises(cc.CcmgError):  # no level below the coarsest
        cc.ccmg_restrict(plan_for(2, "PPPP"), 0, dev_field(oracle.field_zeros(2)), dev_field(oracle.field_zeros(1)))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [4, 8, 64, 256, 512])
def test_prolong_add_matches_oracle(bc, n):
    plan = plan_for(n, bc)
    ec, phi = rand(n // 2, 9), rand(n, 10)
    out = dev_field(np.zeros_like(phi))
    cc.ccmg_prolong_add(plan, 0, dev_field(ec), dev_field(phi), out)
    want = oracle.prolong_add(ec.copy(), phi.copy(), tuple(bc))
    assert rel_max(oracle.interior(host(out)), oracle.interior(want)) < 1e-14


@pytest.mark.parametrize("bc", BCS)
def test_fill_ghosts_matches_oracle(bc):
    n = 64
    a = rand(n, 11)
    t = dev_field(a)
    cc.ccmg_fill_ghosts(plan_for(n, bc), 0, t)
    want = oracle.fill(a.copy(), tuple(bc))
    got = host(t)
    mask = np.ones_like(a, dtype=bool)
    mask[[0, 0, -1, -1], [0, -1, 0, -1]] = False  # corners are never read
    assert np.array_equal(got[mask], want[mask])


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", SIZES)
def test_vcycle_iterates_match_oracle(bc, n):
    """Three V-cycles from a random guess, compared after each cycle."""
    plan = plan_for(n, bc)
    p = oprob(n, bc)
    f = oracle.embed(np.random.default_rng(12).standard_normal((n, n)))
    if p.singular:
        f = oracle.embed(oracle.interior(f) - oracle.interior(f).mean())
    phi = rand(n, 13)
    d_f, d_phi = dev_field(f), dev_field(phi)
    ref = phi.copy()
    for k in range(3):
        cc.ccmg_vcycle(plan, d_f, d_phi)
        oracle.vcycle(p, ref, f)
        got = oracle.interior(host(d_phi))
        assert rel_max(got, oracle.interior(ref)) < 1e-11, (k, rel_max(got, oracle.interior(ref)))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [2, 8, 32, 64, 256, 1024])
def test_solve_matches_oracle_and_exact(bc, n):
    p = oprob(n, bc, rtol=1e-10)
    fv = np.random.default_rng(14).standard_normal((n, n))
    if p.singular:
        fv -= fv.mean()
    phi_o, ro = oracle.solve(p, oracle.embed(fv))
    plan = plan_for(n, bc)
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    rg = cc.ccmg_solve(plan, d_f, d_phi)
    assert rg.status == cc.OK and ro.status == oracle.OK
    assert rg.rel_resid <= 1e-10
    assert abs(rg.cycles - ro.cycles) <= 1
    got = host(d_phi)
    x = exact.dense_solve(fv, 1.0 / n, 0.0, -1.0, tuple(bc)) if n <= 8 else None
    if x is None and bc[0] == bc[1] and bc[2] == bc[3]:
        x = exact.transform_solve(fv, 1.0 / n, 0.0, -1.0, tuple(bc))
    if x is not None:
        err = np.linalg.norm(oracle.interior(got) - x) / np.linalg.norm(x)
        assert err < 1e-9, err
    err_o = np.linalg.norm(oracle.interior(got) - oracle.interior(phi_o)) / np.linalg.norm(oracle.interior(phi_o))
    assert err_o < 1e-9
    # residual recomputed on the host from the returned field
    assert exact.relative_residual(oracle.interior(got), fv, 1.0 / n, 0.0, -1.0, tuple(bc)) <= 1.5e-10


def test_solve_ghosts_filled_and_zero_mean():
    n, bc = 128, "PPPP"
    fv = W.fourier_modes(n, seed=3, count=16, kmax=8)
    plan = plan_for(n, bc)
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, d_f, d_phi)
    assert r.status == cc.OK
    got = host(d_phi)
    filled = oracle.fill(got.copy(), bc)
    assert np.array_equal(got[1:-1, :], filled[1:-1, :]) and np.array_equal(got[:, 1:-1], filled[:, 1:-1])
    assert abs(oracle.interior(got).mean()) < 1e-14 * np.max(np.abs(got))


def test_c1_sine_noise_64_to_1e11():
    """64x64 Dirichlet, f from sin(2 pi x) sin(2 pi y) plus seeded N(0, 1e-2) noise,
    V(2,2), 50 bottom relaxations, relative residual 1e-11."""
    n = 64
    fv = W.sine_noise(n, seed=0)
    p = oprob(n, "DDDD", rtol=1e-11)
    phi_o, ro = oracle.solve(p, oracle.embed(fv))
    plan = plan_for(n, "DDDD", rtol=1e-11)
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    rg = cc.ccmg_solve(plan, d_f, d_phi)
    assert rg.status == cc.OK and rg.rel_resid <= 1e-11
    assert rg.cycles == ro.cycles
    np.testing.assert_allclose(rg.history[:rg.cycles + 1], ro.history[:ro.cycles + 1], rtol=1e-6)
    x = exact.transform_solve(fv, 1.0 / n, 0.0, -1.0, "DDDD")
    assert np.linalg.norm(oracle.interior(host(d_phi)) - x) / np.linalg.norm(x) < 1e-9


@pytest.mark.parametrize("c", [0.1, 1.0, 10.0])
def test_helmholtz_solve(c):
    """(1 - beta Lap) phi = g with beta = c h^2 / 2 (Crank-Nicolson diffusion form)."""
    n = 256
    h = 1.0 / n
    beta = c * h * h / 2
    g = W.gaussian_random_field(n, seed=0)
    plan = plan_for(n, "PPPP", alpha=1.0, beta=beta)
    d_f, d_phi = dev_field(oracle.embed(g)), dev_field(oracle.field_zeros(n))
    r = cc.ccmg_solve(plan, d_f, d_phi)
    assert r.status == cc.OK
    x = exact.transform_solve(g, h, 1.0, beta, "PPPP")
    assert np.linalg.norm(oracle.interior(host(d_phi)) - x) / np.linalg.norm(x) < 1e-9


def test_solve_with_guess_and_zero_rhs():
    n = 64
    plan = plan_for(n, "DDDD")
    fv = np.random.default_rng(15).standard_normal((n, n))
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    r1 = cc.ccmg_solve(plan, d_f, d_phi)
    r2 = cc.ccmg_solve(plan, d_f, d_phi, use_guess=True)
    assert r2.cycles == 0 and r2.rel_resid0 <= 1e-10
    z = dev_field(oracle.field_zeros(n))
    d_phi.fill_(3.0)
    r3 = cc.ccmg_solve(plan, z, d_phi, use_guess=True)
    assert r3.status == cc.OK and float(d_phi[:, :n + 2].abs().max()) == 0.0


def test_error_paths():
    n = 64
    plan = plan_for(n, "PPPP")
    fv = np.ones((n, n))
    d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(plan, d_f, d_phi)
    assert e.value.status == cc.EINCOMPAT
    fv = np.zeros((n, n))
    fv[3, 4] = np.nan
    with pytest.raises(cc.CcmgError) as e:
        cc.ccmg_solve(plan_for(n, "DDDD"), dev_field(oracle.embed(fv)), d_phi)
    assert e.value.status == cc.ENONFINITE
    p1 = plan_for(n, "DDDD", max_cycles=1)
    fv = np.random.default_rng(16).standard_normal((n, n))
    r = cc.ccmg_solve(p1, dev_field(oracle.embed(fv)), d_phi)
    assert r.status == cc.NOT_CONVERGED and r.cycles == 1 and len(r.history) == 2


def test_deterministic_bitwise():
    n = 512
    fv = W.fourier_modes(n, seed=1, count=16, kmax=8)
    plan = plan_for(n, "PPPP")
    outs = []
    for _ in range(2):
        d_f, d_phi = dev_field(oracle.embed(fv)), dev_field(oracle.field_zeros(n))
        r = cc.ccmg_solve(plan, d_f, d_phi)
        outs.append((host(d_phi), r.history))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


@pytest.mark.parametrize("bc", ["PPPP", "DNDD"])
def test_tile_shape_invariance(bc):
    """Every cell's arithmetic is independent of how a level is cut into tiles:
    three V-cycles give bitwise-identical iterates for any launch shapes (row
    march bands, or the 2-D LDS tile kernel below the finest level), and
    after autotuning.  Singular problems (all periodic) also remove the mean of
    each coarse right-hand side, a sum whose grouping follows the tiles, so
    there the iterates agree to rounding instead."""
    n = 1024
    plan = plan_for(n, bc)
    fv = W.fourier_modes(n, seed=5, count=16, kmax=8)
    f = dev_field(oracle.embed(fv))
    start = rand(n, 17)
    outs = []
    for shapes in ([(8, 1), (8, 4)], [(64, 2), (16, 1)], [(256, 4), (128, 2)], "tile", "auto"):
        if shapes == "auto":
            cc.ccmg_plan_autotune(plan, f, dev_field(start))
        elif shapes == "tile":  # the 2-D LDS tile kernel on the levels between the finest and the tail
            cc.ccmg_plan_set_shape(plan, 0, 0, 64, 1)
            cc.ccmg_plan_set_shape(plan, 0, 1, 128, 1)
            for level in range(1, 4):  # 512^2 .. 128^2 (the tail starts at 64^2 or 32^2)
                cc.ccmg_plan_set_shape(plan, level, 0, 0, 1)
                cc.ccmg_plan_set_shape(plan, level, 1, 0, 1)
            assert [s[0] for s in cc.ccmg_plan_shapes(plan)[1:4]] == [0] * 3
        else:
            for level in range(5):
                cc.ccmg_plan_set_shape(plan, level, 0, *shapes[0])
                cc.ccmg_plan_set_shape(plan, level, 1, *shapes[1])
        phi = dev_field(start)
        for _ in range(3):
            cc.ccmg_vcycle(plan, f, phi)
        outs.append(host(phi))
    singular = "D" not in bc
    for o in outs[1:]:
        if singular:
            assert rel_max(o, outs[0]) < 1e-12
        else:
            assert np.array_equal(o, outs[0])
    assert len(cc.ccmg_plan_shapes(plan)) == 10


def test_pitch_bounds_rejected_before_any_launch():
    """A pitch below n + 2, or one that makes an array of 2^31 elements or
    more, is refused by the host checks (the kernels form 32-bit row
    offsets); nothing is launched, so small real buffers are safe here."""
    n = 64
    plan = plan_for(n, "DDDD")
    f = dev_field(oracle.embed(rand(n, 1)))
    phi = dev_field(oracle.field_zeros(n))
    phi2 = dev_field(oracle.field_zeros(n))
    L = cc.lib()
    big = (2 ** 31) // (n + 2) + 1
    for pitch in (n + 1, big):
        assert L.ccmg_solve(plan.handle, f.data_ptr(), phi.data_ptr(), pitch, 0, None) == cc.EINVAL
        assert L.ccmg_smooth(plan.handle, 0, 1, f.data_ptr(), phi.data_ptr(), phi2.data_ptr(), pitch) == cc.EINVAL
    torch.cuda.synchronize()

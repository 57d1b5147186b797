"""Batched solves: many independent problems of different sizes and side types
in one sequence of launches (graph-replayed), each checked against the FP64
oracle / exact solution and against solving it alone."""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


def dev_field(a, pad=0):
    n = a.shape[0] - 2
    t = torch.zeros((n + 2, n + 2 + pad), dtype=torch.float64, device="cuda")
    t[:, :n + 2] = torch.from_numpy(a).cuda()
    return t


def host(t):
    n = t.shape[0] - 2
    return t[:, :n + 2].cpu().numpy()


def make_batch(seed, count, sizes, modes=16, kmax=8):
    items = W.batch(seed=seed, count=count, sizes=sizes, modes=modes, kmax=kmax)
    probs = [cc.Problem(n=it.n, bc=it.bc, rtol=1e-10, prec=cc.MIXED) for it in items]
    return items, probs


def check_against_exact(it, phi_host):
    n = it.n
    got = oracle.interior(phi_host)
    assert exact.relative_residual(got, it.f, 1.0 / n, 0.0, -1.0, it.bc) <= 1.5e-10
    x = exact.transform_solve(it.f, 1.0 / n, 0.0, -1.0, it.bc)
    err = np.linalg.norm(got - x) / np.linalg.norm(x)
    assert err < 1e-9, (n, it.bc, err)


def test_batch_mixed_sizes_and_sides():
    items, probs = make_batch(seed=3, count=24, sizes=(8, 32, 64, 128, 256, 512))
    batch = cc.Batch(probs)
    fs = [dev_field(oracle.embed(it.f), pad=i % 3) for i, it in enumerate(items)]
    phis = [dev_field(oracle.field_zeros(it.n), pad=i % 3) for i, it in enumerate(items)]
    res, info = cc.ccmg_batch_solve(batch, fs, phis)
    assert info["status"] == cc.OK and info["converged"] == len(items)
    for it, r, phi in zip(items, res, phis):
        assert r.status == cc.OK and r.rel_resid <= 1e-10
        check_against_exact(it, host(phi))
        # the returned field has its ghost cells filled
        h = host(phi)
        filled = oracle.fill(h.copy(), it.bc)
        assert np.array_equal(h[1:-1, :], filled[1:-1, :]) and np.array_equal(h[:, 1:-1], filled[:, 1:-1])


def test_batch_matches_single_mixed_solves():
    """Each problem of a batch takes the same steps as solving it alone with a
    MIXED plan that runs one FP32 V-cycle per refinement step, as the batch
    does (the same arithmetic; tile shapes may differ, so compare to
    rounding)."""
    items, probs = make_batch(seed=4, count=8, sizes=(64, 128, 256))
    batch = cc.Batch(probs)
    fs = [dev_field(oracle.embed(it.f)) for it in items]
    phis = [dev_field(oracle.field_zeros(it.n)) for it in items]
    res, info = cc.ccmg_batch_solve(batch, fs, phis)
    for i, (it, r, phi, p) in enumerate(zip(items, res, phis, probs)):
        plan = cc.Plan(p)
        cc.ccmg_plan_set_option(plan, cc.OPT_MIXED_INNER, 1)
        one = dev_field(oracle.field_zeros(it.n))
        r1 = cc.ccmg_solve(plan, fs[i], one)
        assert r1.cycles == r.cycles
        np.testing.assert_allclose(r.history, r1.history, rtol=1e-6)
        a, b = oracle.interior(host(phi)), oracle.interior(host(one))
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-11


def test_batch_repeat_guess_and_autotune():
    items, probs = make_batch(seed=5, count=12, sizes=(32, 64, 128, 256))
    batch = cc.Batch(probs)
    fs = [dev_field(oracle.embed(it.f)) for it in items]
    scratch = [dev_field(oracle.field_zeros(it.n)) for it in items]
    cc.ccmg_batch_autotune(batch, fs, scratch)
    shp = cc.ccmg_batch_shapes(batch)
    assert shp["sizes"] == sorted(shp["sizes"], reverse=True) and all(t >= 8 for t in shp["ty"])
    phis = [dev_field(oracle.field_zeros(it.n)) for it in items]
    res1, info1 = cc.ccmg_batch_solve(batch, fs, phis)
    out1 = [host(p) for p in phis]
    res2, info2 = cc.ccmg_batch_solve(batch, fs, phis)  # same arrays: descriptors reused
    out2 = [host(p) for p in phis]
    for a, b in zip(out1, out2):
        assert np.array_equal(a, b)  # deterministic
    assert info2["steps"] == info1["steps"]
    res3, info3 = cc.ccmg_batch_solve(batch, fs, phis, use_guess=True)
    assert all(r.cycles == 0 for r in res3) and info3["steps"] == 0
    for it, phi in zip(items, phis):
        check_against_exact(it, host(phi))


def test_batch_skips_converged_and_reports_each():
    """Problems that converge early stop working while the rest continue; one
    problem with max_cycles = 1 reports NOT_CONVERGED with its history."""
    items, probs = make_batch(seed=6, count=6, sizes=(64, 256))
    probs[0] = cc.Problem(n=items[0].n, bc=items[0].bc, rtol=1e-3, prec=cc.MIXED)
    probs[1] = cc.Problem(n=items[1].n, bc=items[1].bc, rtol=1e-10, max_cycles=1, prec=cc.MIXED)
    batch = cc.Batch(probs)
    fs = [dev_field(oracle.embed(it.f)) for it in items]
    phis = [dev_field(oracle.field_zeros(it.n)) for it in items]
    res, info = cc.ccmg_batch_solve(batch, fs, phis)
    assert res[0].status == cc.OK and res[0].rel_resid <= 1e-3 and res[0].cycles < res[2].cycles
    assert res[1].status == cc.NOT_CONVERGED and res[1].cycles == 1 and len(res[1].history) == 2
    assert info["status"] == cc.NOT_CONVERGED
    for it, r, phi in list(zip(items, res, phis))[2:]:
        assert r.status == cc.OK
        check_against_exact(it, host(phi))


def test_batch_rejects_other_cycle_shapes():
    with pytest.raises(cc.CcmgError):
        cc.Batch([cc.Problem(n=64, nu1=1, prec=cc.MIXED)])


def test_graph_replays_match_eager_launches():
    """Every replay of the captured step graphs gives the same bits as issuing
    the same launches directly, across several solves with other work and
    synchronisations in between."""
    items, probs = make_batch(seed=7, count=10, sizes=(32, 64, 128, 256))
    batch = cc.Batch(probs)
    fs = [dev_field(oracle.embed(it.f)) for it in items]
    phis = [dev_field(oracle.field_zeros(it.n)) for it in items]
    cc.ccmg_batch_set_option(batch, cc.BATCH_OPT_EAGER, 1)
    res_e, _ = cc.ccmg_batch_solve(batch, fs, phis)
    eager = [host(p) for p in phis]
    cc.ccmg_batch_set_option(batch, cc.BATCH_OPT_EAGER, 0)
    for rep in range(3):
        for p in phis:
            p.fill_(float(rep))  # unrelated eager work between replays
        torch.cuda.synchronize()
        res_g, _ = cc.ccmg_batch_solve(batch, fs, phis)
        for a, b, ra, rb in zip(eager, phis, res_e, res_g):
            hb = host(b)
            for c in ((0, 0), (0, -1), (-1, 0), (-1, -1)):  # corner ghosts are never written
                hb[c] = a[c]
            assert np.array_equal(a, hb)
            assert ra.history == rb.history


def test_zero_rhs_with_guess_returns_zero_like_a_single_solve():
    """A problem with f = 0 in a batch, started from a non-zero guess, returns
    phi = 0 (valid and ghost cells) with status OK, zero cycles and a zero
    relative residual -- what ccmg_solve returns for it; the other problems of
    the batch are unaffected."""
    items, probs = make_batch(seed=11, count=4, sizes=(32, 64))
    fs = [dev_field(oracle.embed(it.f)) for it in items]
    fs[1] = dev_field(oracle.field_zeros(items[1].n))
    rng = np.random.default_rng(12)
    phis = [dev_field(oracle.embed(rng.standard_normal((it.n, it.n)))) for it in items]
    batch = cc.Batch(probs)
    res, info = cc.ccmg_batch_solve(batch, fs, phis, use_guess=True)
    assert res[1].status == cc.OK and res[1].cycles == 0 and res[1].rel_resid == 0.0
    assert not np.any(host(phis[1]))
    one = cc.Plan(probs[1])
    single = dev_field(oracle.embed(rng.standard_normal((items[1].n, items[1].n))))
    r1 = cc.ccmg_solve(one, fs[1], single, use_guess=True)
    assert r1.status == cc.OK and r1.cycles == 0 and not np.any(host(single))
    for i in (0, 2, 3):
        assert res[i].status == cc.OK and res[i].rel_resid <= 1e-10
        check_against_exact(items[i], host(phis[i]))

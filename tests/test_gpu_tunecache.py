"""The autotune cache on the device: a second plan of the same problem takes
the stored shapes instead of timing again, and solves to the same bits; a
different problem misses."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")
from paper_1306_6883_amd import tunecache as T  # noqa: E402


def test_cache_hit_gives_same_shapes_and_bits(tmp_path):
    path = str(tmp_path / "tune.json")
    n = 512
    prob = cc.Problem(n=n, bc=("D", "D", "P", "P"), rtol=1e-10)
    f = torch.from_numpy(oracle.embed(W.fourier_modes(n, seed=3, count=16, kmax=8))).cuda()
    a = cc.Plan(prob)
    sa, hit = T.tuned(a, f, cc.field(n), path)
    assert not hit
    b = cc.Plan(prob)
    sb, hit = T.tuned(b, f, cc.field(n), path)
    assert hit and sa == sb == T.shapes_of(b)
    pa, pb = cc.field(n), cc.field(n)
    ra, rb = cc.ccmg_solve(a, f, pa), cc.ccmg_solve(b, f, pb)
    assert ra.status == rb.status == cc.OK and ra.cycles == rb.cycles
    assert torch.equal(pa, pb)
    # another problem is another key
    c = cc.Plan(cc.Problem(n=n, bc="P", rtol=1e-10))
    fc = f.clone()
    fc[1:n + 1, 1:n + 1] -= fc[1:n + 1, 1:n + 1].mean()
    _, hit = T.tuned(c, fc, cc.field(n), path)
    assert not hit
    assert len(T._load(path)) == 2

"""Plain V-cycles under HIP graph capture: ccmg_vcycle (plan workspace) and
ccmg_vcycle_noalloc (static scratch) enqueue only kernel launches, so a fixed
number of cycles can be captured once and replayed.  Every replay -- with
unrelated eager work and synchronisations between replays -- must give the
bits of the same cycles issued eagerly."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


def rand_field(n, seed, zero_mean):
    v = np.random.default_rng(seed).standard_normal((n, n))
    if zero_mean:
        v -= v.mean()
    return torch.from_numpy(oracle.embed(v)).cuda()


@pytest.mark.parametrize("sides", [("P",) * 4, ("D", "N", "D", "D")])
@pytest.mark.parametrize("noalloc", [False, True])
def test_captured_vcycles_replay_bitwise(sides, noalloc):
    n, cycles = 512, 3
    singular = "D" not in sides
    prob = cc.Problem(n=n, bc=sides)
    s = torch.cuda.Stream()
    f = rand_field(n, 1, singular)
    phi0 = rand_field(n, 2, False)
    plan = None if noalloc else cc.Plan(prob, stream=s)

    def cycle(phi):
        if noalloc:
            cc.ccmg_vcycle_noalloc(prob, f, phi, stream=s)
        else:
            cc.ccmg_vcycle(plan, f, phi)

    # eager reference (this also makes the first call's one-time set-up happen outside capture)
    ref = phi0.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        for _ in range(cycles):
            cycle(ref)
    s.synchronize()
    # capture
    phi = phi0.clone()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        for _ in range(cycles):
            cycle(phi)
    for rep in range(3):
        phi.copy_(phi0)
        junk = torch.full((1 << 20,), float(rep), device="cuda")  # unrelated eager work
        junk.mul_(2.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(phi, ref), rep
        del junk

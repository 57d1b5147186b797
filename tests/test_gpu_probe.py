"""The streaming probe (diagnostics beside the nameplate bandwidth): c = a + b
element by element after every launch shape it sweeps, for even sizes from
one 16-byte pair up, and its argument checks (rejected on the host, before
any launch)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1306_6883_amd")


@pytest.mark.parametrize("count", [2, 1002, (1 << 20) + 6])
def test_probe_adds_elementwise(count):
    rng = np.random.default_rng(count)
    a = torch.from_numpy(rng.standard_normal(count)).cuda()
    b = torch.from_numpy(rng.standard_normal(count)).cuda()
    c = torch.full_like(a, float("nan"))
    ms, cfg = cc.ccmg_probe_stream(a, b, c, reps=2)
    torch.cuda.synchronize()
    assert ms > 0.0
    assert cfg % 1000 in (2, 4, 8, 32, 128) and cfg // 1000 in (0, 1)
    assert np.array_equal(c.cpu().numpy(), a.cpu().numpy() + b.cpu().numpy())


def test_probe_rejects_bad_arguments():
    a = torch.zeros(10, dtype=torch.float64, device="cuda")
    b, c = torch.zeros_like(a), torch.zeros_like(a)
    with pytest.raises(cc.CcmgError):  # odd count
        cc.ccmg_probe_stream(a[:9], b[:9], c[:9])
    with pytest.raises(cc.CcmgError):  # arrays 8-byte but not 16-byte aligned
        cc.ccmg_probe_stream(a[1:9], b[1:9], c[1:9])
    with pytest.raises(cc.CcmgError):
        cc.ccmg_probe_stream(a, b, c, reps=0)
    with pytest.raises(ValueError):
        cc.ccmg_probe_stream(a, b[:8], c)
    with pytest.raises(ValueError):
        cc.ccmg_probe_stream(a.float(), b.float(), c.float())

"""Learned initial guess on the GPU: every kernel of the network's forward and
backward pass against the FP64 network oracle (with the same BF16 rounding
points emulated), the Adam step, the encoder and decoder, the learned solve's
fallbacks, and the gain of a briefly trained network."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import net as ON

pytestmark = pytest.mark.gpu

G = ON.G


@pytest.fixture(scope="module")
def M():
    import paper_1306_6883_amd as M
    return M


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_inputs(nb, seed):
    g = np.random.default_rng(seed)
    p = np.concatenate([g.normal(0, 1 / math.sqrt(k * ci), co * k * ci)
                        for co, k, ci in [(32, 9, 1)] + [(32, 9, 32)] * 4 + [(1, 9, 32)]]).astype(np.float32)
    x = g.standard_normal((nb, G, G)).astype(np.float32)
    t = (0.1 * g.standard_normal((nb, G, G))).astype(np.float32)
    return p, x, t


def dev(a):
    return torch.as_tensor(a, device="cuda").contiguous()


def test_param_count(M):
    assert M.ccmg_net_param_count() == ON.param_count() == 37440


def test_forward_matches_oracle(M):
    p, x, _ = make_inputs(2, 1)
    net = M.Net(batch=4, n_max=256)
    M.ccmg_net_set_params(net, dev(p))
    y = M.ccmg_net_forward(net, dev(x)).cpu().numpy()
    yb = ON.forward(p.astype(np.float64), x.astype(np.float64), bf=True)[0]
    y64 = ON.forward(p.astype(np.float64), x.astype(np.float64), bf=False)[0]
    e_bf, e_64 = rel(y, yb), rel(y, y64)
    print(f"forward: rel err vs BF16-emulated oracle {e_bf:.2e}, vs FP64 oracle {e_64:.2e}")
    # same rounding points: differences only from FP32 sums flipping a rounding
    assert e_bf < 2e-4
    # weights and activations of the 32 -> 32 layers as BF16 pairs (about 16
    # bits each), first and last layer in FP32
    assert e_64 < 2e-4


def test_loss_and_every_layer_gradient_match_oracle(M):
    p, x, t = make_inputs(2, 2)
    net = M.Net(batch=4, n_max=256)
    M.ccmg_net_set_params(net, dev(p))
    loss, g = M.ccmg_net_loss_grad(net, dev(x), dev(t))
    g = g.cpu().numpy()
    lb, gb = ON.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), bf=True)
    assert abs(loss - lb) <= 1e-3 * lb
    # Same rounding points; the GPU sums in FP32 (the oracle in FP64), so a
    # back-propagated value within ~sqrt(288) 2^-24 of a bfloat16 midpoint
    # rounds the other way (one bfloat16 unit, 2^-8): about 1e-3 of the values
    # per layer, ~1e-4 of a layer's norm, accumulating over the five rounded
    # stages below the output -- bound 1e-3 (seen: <= 2.7e-4).
    o = 0
    for l, sz in enumerate(ON.SIZES):
        e = rel(g[o:o + sz], gb[o:o + sz])
        print(f"layer {l + 1}: gradient rel err {e:.2e}")
        assert e < 1e-3, l
        o += sz


def test_gradient_matches_central_difference_on_device(M):
    """In the GPU's own arithmetic: the loss change along the gradient matches
    the gradient's squared norm (central difference over a step that changes
    the loss by about 5%: small enough for higher orders to vanish, large
    enough that BF16 rounding of the weights is noise)."""
    p, x, t = make_inputs(2, 3)
    net = M.Net(batch=4, n_max=256)
    P = dev(p)
    M.ccmg_net_set_params(net, P)
    l0, g = M.ccmg_net_loss_grad(net, dev(x), dev(t))
    eps = 0.05 * l0 / float(g.norm()) ** 2
    M.ccmg_net_set_params(net, (P - eps * g).contiguous())
    lm, _ = M.ccmg_net_loss_grad(net, dev(x), dev(t))
    M.ccmg_net_set_params(net, (P + eps * g).contiguous())
    lp, _ = M.ccmg_net_loss_grad(net, dev(x), dev(t))
    pred = eps * float(g.norm()) ** 2
    assert lm < l0 < lp
    assert abs((lp - lm) / 2 - pred) < 0.03 * pred


def test_adam_steps(M):
    p, x, t = make_inputs(2, 4)
    net = M.Net(batch=4, n_max=256)
    M.ccmg_net_set_params(net, dev(p))
    w = p.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lr = 1e-3
    for k in range(1, 3):
        _, g = M.ccmg_net_loss_grad(net, dev(x), dev(t))
        g = g.cpu().numpy().astype(np.float64)
        M.ccmg_net_train_step(net, dev(x), dev(t), lr)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        w = w - lr * (m / (1 - 0.9 ** k)) / (np.sqrt(v / (1 - 0.999 ** k)) + 1e-8)
        got = M.ccmg_net_get_params(net).cpu().numpy()
        assert np.max(np.abs(got - w)) < 1e-5, k


def test_train_step_reduces_loss(M):
    p, x, t = make_inputs(4, 5)
    net = M.Net(batch=4, n_max=256)
    M.ccmg_net_set_params(net, dev(p))
    X, T = dev(x), dev(t)
    losses = [M.ccmg_net_train_step(net, X, T, 1e-3) for _ in range(30)]
    assert losses[-1] < 0.5 * losses[0]


@pytest.mark.parametrize("n", [256, 1024])
def test_encode_matches_block_mean(M, n):
    net = M.Net(batch=1, n_max=1024)
    fv = W.gaussian_blobs(n, 7)
    av = np.random.default_rng(0).standard_normal((n, n))
    f, a = M.to_field(fv), M.to_field(av)
    xa = M.ccmg_net_encode(net, a, f).cpu().numpy()
    ref = ON.block_mean(av, n // G) / math.sqrt(np.mean(fv ** 2))
    assert np.max(np.abs(xa - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,iters,length", [(256, 0, 1.0), (512, 0, 2.0), (1024, 0, 1.0), (256, 3, 1.0),
                                             (1024, 5, 0.5)])
def test_guess_is_relaxed_prolonged_network_output(M, n, iters, length):
    """The guess = network output in physical units, `iters` red-black
    Gauss-Seidel iterations on the network's grid (FP32 on the device, FP64 in
    the oracle), then multigrid prolongations."""
    import oracle
    p, _, _ = make_inputs(1, 6)
    net = M.Net(batch=1, n_max=1024)
    M.ccmg_net_set_params(net, dev(p))
    fv = W.gaussian_blobs(n, 8)
    f = M.to_field(fv)
    phi = M.field(n)
    M.ccmg_net_guess(net, f, phi, length=length, coarse_iters=iters)
    # the guess skips the RMS normalisation (it cancels in a linear network):
    # encode against a scale field of RMS exactly 1
    ones = M.to_field(np.ones((n, n)))
    x = M.ccmg_net_encode(net, f, ones)
    y = M.ccmg_net_forward(net, x[None].contiguous())[0].cpu().numpy().astype(np.float64)
    c = y * length ** 2
    if iters:
        prob = oracle.Problem(n=G, h=length / G, alpha=0.0, beta=-1.0, bc="PPPP")
        cf = oracle.embed(c)
        oracle.smooth(prob, cf, oracle.embed(x.cpu().numpy().astype(np.float64)), iters)
        c = oracle.interior(cf).copy()
    while c.shape[0] < n:
        c = ON.prolong_periodic(c)
    got = phi[1:n + 1, 1:n + 1].cpu().numpy()
    # FP32 scaling and relaxation on the device
    assert np.max(np.abs(got - c)) <= 2e-6 * np.max(np.abs(c))


def test_guess_ignores_the_scale_of_f(M):
    """Scaling f by a power of two scales the guess exactly (linear network,
    no normalisation at inference, every rounding scale-invariant)."""
    p, _, _ = make_inputs(1, 7)
    net = M.Net(batch=1, n_max=512)
    M.ccmg_net_set_params(net, dev(p))
    fv = W.gaussian_blobs(512, 11)
    g1, g2 = M.field(512), M.field(512)
    M.ccmg_net_guess(net, M.to_field(fv), g1)
    M.ccmg_net_guess(net, M.to_field(fv * 2.0 ** -10), g2)
    a, b = g2.cpu().numpy() * 2.0 ** 10, g1.cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_learned_solve_converges_with_untrained_and_broken_weights(M):
    """Plain multigrid always finishes from the guess: random weights, huge
    weights (guess discarded) and non-finite weights (guess discarded)."""
    from paper_1306_6883_amd import learned as L
    n = 256
    plan = M.Plan(L.periodic_poisson(n))
    net = M.Net(batch=1, n_max=n)
    f = M.to_field(W.gaussian_blobs(n, 9))
    ref = M.field(n)
    rz = M.ccmg_solve(plan, f, ref)
    p = L.init_params(3)
    for scale, expect_used in [(0.5, None), (1e6, False), (float("nan"), False)]:
        M.ccmg_net_set_params(net, (p * scale).contiguous())
        phi = M.field(n)
        r, used = M.ccmg_solve_learned(plan, net, f, phi)
        assert r.status == M.OK and r.rel_resid <= 1e-10
        if expect_used is None:
            expect_used = bool(r.rel_resid0 <= 1e6)
        assert used == expect_used, (scale, r.rel_resid0)
        d = (phi - ref)[1:n + 1, 1:n + 1]
        assert float(d.norm() / ref[1:n + 1, 1:n + 1].norm()) < 1e-9
    assert rz.status == M.OK


def test_learned_solve_rejects_bad_arguments(M):
    from paper_1306_6883_amd import learned as L
    plan = M.Plan(L.periodic_poisson(128))
    net = M.Net(batch=1, n_max=256)
    f, phi = M.field(128), M.field(128)
    with pytest.raises(M.CcmgError):
        M.ccmg_solve_learned(plan, net, f, phi)        # n below the decoder's minimum
    plan2 = M.Plan(L.periodic_poisson(512))
    with pytest.raises(M.CcmgError):
        M.ccmg_solve_learned(plan2, net, M.field(512), M.field(512))  # n above n_max
    helm = M.Plan(M.Problem(n=256, bc="P", alpha=1.0, beta=-1.0))
    with pytest.raises(M.CcmgError):
        M.ccmg_solve_learned(helm, net, M.field(256), M.field(256))  # not the trained problem
    for sides in ("D", ("P", "P", "D", "D"), ("N", "N", "P", "P")):
        other = M.Plan(M.Problem(n=256, bc=sides))
        with pytest.raises(M.CcmgError) as e:
            M.ccmg_solve_learned(other, net, M.field(256), M.field(256))  # trained on periodic sides only
        assert e.value.status == M.EINVAL


def test_trained_network_gains_over_zero_guess(M):
    """A network trained on the GPU on plain-multigrid solutions (training
    seeds 0..4095) guesses unseen problems (seeds 100000..100255) well enough
    to save V-cycles, and every solve from a guess still reaches the
    tolerance.  Beside it, for attribution: the same decoder run on a zero
    network output, and non-learned guesses of about the network's cost
    (k V-cycles of the averaged problem on the network's grid, then the
    prolongations)."""
    from paper_1306_6883_amd import learned as L
    n = 1024
    net = L.new_net(batch=32, n_max=n, seed=0)
    plan = M.Plan(L.periodic_poisson(n))
    data = L.make_dataset(net, n, range(4096), plan=plan)
    hist = L.train(net, data, steps=16000, batch=32, lr=1e-3, lr_final=1e-5, warmup=200)
    print("loss", hist[0], hist[-1], "plain cycles", data.cycles)
    assert hist[-1][1] < 1e-3 * hist[0][1]
    cmp = L.compare(net, n, range(100000, 100008), plan=plan)
    print("guess error", np.round(cmp.guess_error, 4))
    assert all(cmp.used)
    assert np.mean(cmp.guess_error) < 0.05
    g = L.compare_guesses(net, n, range(100000, 100256), plan=plan)
    for k in g.ms:
        print(f"{k}: cycles {np.mean(g.cycles[k]):.2f}, ms {np.mean(g.ms[k]):.3f} (guess {g.guess_ms[k]:.3f})")
    assert len(g.cycles["learned"]) == 256
    assert np.mean(g.cycles["learned"]) <= np.mean(g.cycles["zero"]) - 1
    assert np.mean(g.cycles["decoder_only"]) <= np.mean(g.cycles["zero"])


def test_checkpoint_resume_continues_exactly(M, tmp_path):
    """Training stopped at step 17 of a 40-step schedule, checkpointed
    (parameters, Adam moments, step counter) and resumed in a fresh net ends
    with the same parameters, bit for bit, as an uninterrupted run."""
    from paper_1306_6883_amd import learned as L
    n = 256
    plan = M.Plan(L.periodic_poisson(n))
    a = L.new_net(batch=8, n_max=n, seed=1)
    data = L.make_dataset(a, n, range(48), plan=plan)
    L.train(a, data, steps=40, batch=8, warmup=10)
    b = L.new_net(batch=8, n_max=n, seed=1)
    path = str(tmp_path / "net.npz")
    L.train(b, data, steps=40, batch=8, warmup=10, stop=17, checkpoint=path)
    c = L.new_net(batch=8, n_max=n, seed=5)  # other weights: all of them come from the checkpoint
    assert L.load_checkpoint(c, path) == 17
    L.train(c, data, steps=40, batch=8, warmup=10, start=17)
    pa, pc = M.ccmg_net_get_params(a), M.ccmg_net_get_params(c)
    assert torch.equal(pa, pc)
    sa, ka = M.ccmg_net_get_state(a)
    sc, kc = M.ccmg_net_get_state(c)
    assert ka == kc == 40 and torch.equal(sa, sc)
    with pytest.raises(ValueError):
        M.ccmg_net_set_state(c, sa[:10].contiguous(), 3)

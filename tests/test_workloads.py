"""Seeded input generators: determinism and the stated statistics."""
import numpy as np

import workloads as W


def test_fourier_modes_direct_evaluation():
    n = 32
    f = W.fourier_modes(n, seed=3, count=8, kmax=4)
    ks, amp, ph = W._modes(W.rng(W.W_FOURIER, 3), 8, 4)
    x = W.centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    g = sum(a * np.cos(2 * np.pi * (k[0] * X + k[1] * Y) + t) for k, a, t in zip(ks, amp, ph))
    assert np.allclose(f, g - g.mean(), atol=1e-12)
    assert abs(f.mean()) < 1e-14
    assert len({tuple(k) for k in ks}) == 8 and np.all((ks**2).sum(1) <= 16)


def test_generators_deterministic():
    for fn in (lambda: W.sine_noise(16, 0), lambda: W.gaussian_blobs(32, 100000),
               lambda: W.gaussian_random_field(32, 1), lambda: W.fourier_modes(16, 2)):
        assert np.array_equal(fn(), fn())


def test_grf_unit_std_zero_mean():
    g = W.gaussian_random_field(128, 0)
    assert abs(g.std() - 1) < 1e-12 and abs(g.mean()) < 1e-12


def test_blobs_zero_mean_periodic():
    f = W.gaussian_blobs(64, 5)
    assert abs(f.mean()) < 1e-14
    # minimum-image distance: the field is smooth across the periodic seam
    assert np.max(np.abs(f[:, 0] - f[:, -1])) < 0.5 * np.max(np.abs(f)) + 1e-12


def test_batch_sizes_and_bcs():
    items = W.batch_sizes(0)
    assert len(items) == 512
    ns = {n for n, _ in items}
    assert ns <= {32, 64, 128, 256, 512, 1024} and len(ns) == 6
    for _, bc in items:
        assert bc[0] == bc[1] and bc[2] == bc[3] and set(bc) <= {"P", "D"}


def test_blob_fields_built_with_torch_match_numpy():
    """The batched torch generator gives the same fields as the numpy one."""
    import workloads as W
    F = W.gaussian_blobs_torch(64, [3, 4, 100000], device="cpu").numpy()
    for k, s in enumerate([3, 4, 100000]):
        ref = W.gaussian_blobs(64, s)
        assert np.max(np.abs(F[k] - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert abs(F[k].mean()) < 1e-15

"""The seeded input generators: reproducible, right shapes, right second moments."""
import numpy as np

from paper_2605_23812_amd import inputs


def test_grf_reproducible_and_shaped():
    a = inputs.grf_perturbations(3, 32, 0.1, 1e-2, seed=5)
    b = inputs.grf_perturbations(3, 32, 0.1, 1e-2, seed=5)
    assert a.shape == (3, 2 * 64 * 32)
    assert np.array_equal(a, b)
    # a draw does not depend on how many draws were requested
    c = inputs.grf_perturbations(5, 32, 0.1, 1e-2, seed=5)
    assert np.array_equal(a, c[:3])


def test_grf_variance_and_squared_exponential_correlation():
    ny, nx, h, ell, sigma = 256, 256, 1.0 / 128, 0.05, 1.0
    f = np.stack([inputs.grf_field(1, (k, 0), ny, nx, h, ell, sigma) for k in range(12)])
    assert abs(f.var() - sigma ** 2) < 0.1
    for lag in (3, 6, 9):
        r = lag * h
        corr = np.mean(f[:, :, :-lag] * f[:, :, lag:]) / f.var()
        assert abs(corr - np.exp(-r * r / ell ** 2)) < 0.06, (lag, corr)


def test_initial_field_profile():
    u0, v0 = inputs.initial_field(8, amp=0.0)
    assert u0.shape == (16, 33) and v0.shape == (17, 32)
    y = -1 + (np.arange(16) + 0.5) / 8
    assert np.allclose(u0[:, 5], np.where(y > 0, 4 * y * (1 - y), 0.0))
    assert not v0.any()

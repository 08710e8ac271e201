"""Pins of the eigen-ensemble oracle (CPU).

* two cells: B = s^2 [[1, e], [e, 1]] with e = exp(-d^2 / a^2) has eigenvalues s^2 (1 +- e) and
  eigenvectors (1, +-1) / sqrt(2);
* a uniform variance on a rectangle of cells: the spectrum of B is the set of products of the
  spectra of the two 1-D kernel matrices (Kronecker structure);
* eq. ensemble_covariance: with every mode kept, E E^T / (N - 1) = B; truncated, the error in the
  2-norm is the first dropped eigenvalue (Eckart-Young) and the members are orthogonal with
  |E_k|^2 = (N - 1) mu_k;
* the taper: sigma_max^2 at the centre of the region, zero at its corners, mirror-symmetric;
* the separable product D (Ky kron Kx) D v equals the dense B v;
* the reconstruction error: 0 inside the span, 1 orthogonal to it, 1/2 for a mode inside plus a
  mode outside of equal norm.
"""
import numpy as np
import pytest

from oracle import eigen as OE_
from oracle import envar as OE


def test_two_cells_closed_form():
    d, a, s2 = 0.05, 0.07, 0.01
    x, y = np.array([0.3, 0.3 + d]), np.array([0.1, 0.1])
    B = OE_.covariance(x, y, np.array([s2, s2]), a, a)
    e = np.exp(-d * d / (a * a))
    mu, V = OE_.eigenpairs(B, 2)
    assert np.allclose(mu, [s2 * (1 + e), s2 * (1 - e)], rtol=1e-14, atol=0)
    assert np.allclose(np.abs(V), 1 / np.sqrt(2), rtol=1e-14)
    assert V[0, 0] * V[0, 1] > 0 and V[1, 0] * V[1, 1] < 0


def test_uniform_rectangle_spectrum_is_kronecker():
    p = OE.Problem(inv_h=16, region="box", box=(1.3, 1.7, -0.5, -0.2))
    x, y = OE_.cell_coords(p)
    s2 = 0.01
    B = OE_.covariance(x, y, np.full(x.shape, s2), 0.07, 0.11)
    xs, ys = np.unique(x), np.unique(y)
    assert xs.size * ys.size == x.size
    kx = np.linalg.eigvalsh(np.exp(-(xs[:, None] - xs[None, :]) ** 2 / 0.07 ** 2))
    ky = np.linalg.eigvalsh(np.exp(-(ys[:, None] - ys[None, :]) ** 2 / 0.11 ** 2))
    want = np.sort(s2 * np.outer(kx, ky).ravel())[::-1]
    mu, _ = OE_.eigenpairs(B, x.size)
    assert np.abs(mu - want).max() <= 1e-13 * want[0]


@pytest.mark.parametrize("taper", ["none", "ellipse"])
def test_ensemble_covariance_and_truncation(taper):
    p = OE.Problem(inv_h=16, region="cavity")
    x, y = OE_.cell_coords(p)
    sig2 = OE_.taper_variance(p, 0.01, taper)
    B = OE_.covariance(x, y, sig2)
    n = x.size
    E, mu = OE_.eigen_ensemble(B, n)
    assert np.abs(E.T @ E / (n - 1) - B).max() <= 1e-13 * np.abs(B).max()  # eq. ensemble_covariance
    N = 20
    E, mu = OE_.eigen_ensemble(B, N)
    mu_all = np.sort(np.linalg.eigvalsh(B))[::-1]
    err = np.linalg.norm(B - E.T @ E / (N - 1), 2)
    assert abs(err - mu_all[N]) <= 1e-12 * mu_all[0]
    G = E @ E.T
    assert np.allclose(np.diag(G), (N - 1) * mu, rtol=1e-12)
    assert np.abs(G - np.diag(np.diag(G))).max() <= 1e-12 * G.max()
    assert np.all(np.diff(mu) <= 0)


def test_taper_shape():
    p = OE.Problem(inv_h=16, region="box", box=(1.3, 1.8, -0.7, -0.1))
    x, y = OE_.cell_coords(p)
    s2 = OE_.taper_variance(p, 0.01)
    xs, ys = np.unique(x), np.unique(y)
    nx, ny = xs.size, ys.size
    grid = s2.reshape(ny, nx)
    assert np.allclose(grid, grid[::-1, :], rtol=0, atol=1e-18) and np.allclose(grid, grid[:, ::-1], atol=1e-18)
    assert grid[0, 0] == 0.0 and grid[-1, -1] == 0.0
    # the centre cell sits at r^2 = (h / 2)^2 / rx^2 + (h / 2)^2 / ry^2 from the centre for even counts
    h = p.grid().h
    rx, ry = nx * h / 2, ny * h / 2
    c = grid[ny // 2, nx // 2]
    r2 = (0.5 * h / rx) ** 2 * (nx % 2 == 0) + (0.5 * h / ry) ** 2 * (ny % 2 == 0)
    assert abs(c - 0.01 * (1 - r2) ** 2) <= 1e-15 and grid.max() == c
    assert np.all(s2 <= 0.01) and np.all(s2 >= 0.0)


def test_separable_product_matches_dense():
    p = OE.Problem(inv_h=16, region="column")
    x, y = OE_.cell_coords(p)
    sig2 = OE_.taper_variance(p, 0.01)
    B = OE_.covariance(x, y, sig2, 0.07, 0.09)
    v = np.random.default_rng(0).standard_normal(x.size)
    assert np.abs(OE_.apply_separable(p, sig2, v, 0.07, 0.09) - B @ v).max() <= 1e-14 * np.abs(B @ v).max()


def test_reconstruction_error_limits():
    p = OE.Problem(inv_h=16, region="cavity")
    x, y = OE_.cell_coords(p)
    B = OE_.covariance(x, y, OE_.taper_variance(p))
    mu, V = OE_.eigenpairs(B, 12)
    inside = 0.3 * V[0] - 2.0 * V[4]
    assert OE_.reconstruction_error(inside, V[:10]) <= 1e-28
    assert abs(OE_.reconstruction_error(V[11], V[:10]) - 1.0) <= 1e-14
    assert abs(OE_.reconstruction_error(V[1] + V[10], V[:10]) - 0.5) <= 1e-14
    rows = OE_.control_rows(V[:3], component=1)
    assert rows.shape == (3, p.m) and np.all(rows[:, :x.size] == 0) and np.array_equal(rows[:, x.size:], V[:3])

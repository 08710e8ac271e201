"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds no arithmetic of the method itself: it only draws random
numbers and lays out the initial fields, with the sizes and structure of the
paper's workloads (Sec. 4). Every draw uses numpy's Philox counter-based
generator keyed by (seed, stream), so a draw never depends on how many other
draws were made.

* ``grf_perturbations`` : control perturbations delta f_i, random draws from a
  zero-mean Gaussian with the squared-exponential covariance of eq.
  (covarianceB) with a_x = a_y = ell, c_xy = inf and a uniform variance:
  C(r) = sigma^2 exp(-r^2 / ell^2). (The paper's own ensemble takes the
  leading eigenvectors of that covariance instead; random draws are the
  common alternative it names in Sec. 3.3.2.) The field is white noise
  convolved with the separable kernel exp(-2 r^2 / ell^2), normalised to
  variance sigma^2; components x and y are independent. Layout per row:
  [f_x over the region cells, row-major, then f_y] with the region a
  rectangle of ``ny`` x ``nx`` cells.
* ``initial_field`` : parabolic channel profile 4 y (1 - y) above y = 0 and
  rest in the cavity, plus i.i.d. N(0, amp^2) noise on every face; each
  solver imposes its own boundary values on it.
"""
import numpy as np

DEFAULT_SEED = 2605238120


def _rng(seed, *stream):
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), *map(int, stream)])))


def region_shape(inv_h, region="column"):
    """(ny, nx) of the rectangular control region for the cavity geometry."""
    n = int(inv_h)
    if region == "column":
        return 2 * n, n
    if region == "cavity":
        return n, n
    raise ValueError("region shape is only defined for 'column' and 'cavity'")


def _kernel_1d(ell, h):
    half = int(np.ceil(3.0 * ell / h))
    x = np.arange(-half, half + 1) * h
    return np.exp(-2.0 * x * x / (ell * ell))


def grf_field(seed, stream, ny, nx, h, ell, sigma):
    """One zero-mean GRF sample on an ny x nx cell grid of spacing h."""
    k = _kernel_1d(ell, h)
    pad = len(k) // 2
    w = _rng(seed, *stream).standard_normal((ny + 2 * pad, nx + 2 * pad))
    a = np.apply_along_axis(lambda r: np.convolve(r, k, mode="valid"), 1, w)
    a = np.apply_along_axis(lambda c: np.convolve(c, k, mode="valid"), 0, a)
    norm = np.sqrt(np.sum(k * k) ** 2)  # variance of the separable sum of unit white noise
    return sigma * a / norm


def grf_perturbations(n_members, inv_h, ell, sigma, seed=DEFAULT_SEED, region="column", shape=None):
    """(n_members, m) FP64 array of perturbation rows delta f_i."""
    ny, nx = shape if shape is not None else region_shape(inv_h, region)
    h = 1.0 / inv_h
    out = np.empty((n_members, 2 * ny * nx))
    for i in range(n_members):
        fx = grf_field(seed, (i, 0), ny, nx, h, ell, sigma)
        fy = grf_field(seed, (i, 1), ny, nx, h, ell, sigma)
        out[i] = np.concatenate([fx.ravel(), fy.ravel()])
    return out


def box_dims(inv_h, geometry="cavity", length=4.0):
    """(NX, NY, y0) of the bounding box of the MAC grid ("paper": a channel of height 1/2 over the
    unit cavity)."""
    n = int(inv_h)
    if geometry == "cavity":
        return int(round(length * n)), 2 * n, -1.0
    if geometry == "paper":
        return int(round(length * n)), n + n // 2, -1.0
    if geometry == "channel":
        return int(round(length * n)), n, 0.0
    raise ValueError(geometry)


def initial_field(inv_h, amp=1e-3, seed=DEFAULT_SEED, geometry="cavity", length=4.0):
    """(u0 (NY, NX+1), v0 (NY+1, NX)) raw initial face fields before boundary values: the inflow
    profile (parabola, or uniform for "paper") in the channel plus seeded noise of size amp."""
    NX, NY, y0 = box_dims(inv_h, geometry, length)
    h = 1.0 / inv_h
    y = y0 + (np.arange(NY) + 0.5) * h
    prof = np.where(y > 0.0, 1.0 if geometry == "paper" else 4.0 * y * (1.0 - y), 0.0)
    rng = _rng(seed, 1 << 20)
    u0 = prof[:, None] + amp * rng.standard_normal((NY, NX + 1))
    v0 = amp * rng.standard_normal((NY + 1, NX))
    return u0, v0

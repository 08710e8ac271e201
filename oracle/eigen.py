"""Oracle of the deterministic eigen-ensemble (Sec. 3.3.2, eq. covarianceB and eq. eigenvm1) and of
the reconstruction error of App. A (eq. reconstruction_error).

TEST INFRASTRUCTURE ONLY (see the package header).

* ``taper_variance``  : sigma_i^2 over the control cells: sigma_max^2 (1 - r^2)^2 inside the ellipse
                        inscribed in the region's bounding rectangle, 0 outside (r the elliptic radius,
                        1 on the ellipse), or sigma_max^2 everywhere ("none").
* ``covariance``      : the dense B of eq. covarianceB with c_xy = infinity (no cross term):
                        B_ij = sigma_i sigma_j exp(-(x_i - x_j)^2 / a_x^2 - (y_i - y_j)^2 / a_y^2).
* ``eigen_ensemble``  : the N leading eigenpairs of B (eigenvalues decreasing) and
                        E = V_N diag(mu_N)^(1/2) sqrt(N - 1) (eq. eigenvm1). With M_f = h^2 I the
                        M_f-orthonormal eigenvectors are U = V / h with eigenvalues Sigma = h^2 mu, so
                        U Sigma^(1/2) = V mu^(1/2): E does not depend on h through M_f. Returned E is
                        [N][n_cells] (row k = the k-th member's scalar field).
* ``control_rows``    : the members as control rows [N][m], driving one forcing component.
* ``apply_separable`` : B v from the Kronecker structure of the kernel on a rectangle of cells
                        (a second formula for B, used at sizes where the dense B does not fit).
* ``reconstruction_error``: eq. reconstruction_error for the orthonormal basis V_N (M_f = h^2 I
                        cancels): |f - V V^T f|^2 / |f|^2.
"""
import numpy as np


def cell_coords(p):
    """(x, y) centres of the control cells, in control order (row-major over (j, i))."""
    g = p.grid()
    cells = p.cells()
    return np.array([g.xc[i] for _, i in cells]), np.array([g.yc[j] for j, _ in cells])


def taper_variance(p, sigma2_max=0.01, taper="ellipse"):
    """sigma_i^2 of every control cell (the shape of Sec. 4.2: largest at the centre of the
    actuation region, decreasing smoothly to zero at its boundary)."""
    x, y = cell_coords(p)
    if taper == "none":
        return np.full(x.shape, float(sigma2_max))
    h = p.grid().h
    x0, x1 = x.min() - 0.5 * h, x.max() + 0.5 * h
    y0, y1 = y.min() - 0.5 * h, y.max() + 0.5 * h
    r2 = ((x - 0.5 * (x0 + x1)) / (0.5 * (x1 - x0))) ** 2 + ((y - 0.5 * (y0 + y1)) / (0.5 * (y1 - y0))) ** 2
    return np.where(r2 < 1.0, sigma2_max * (1.0 - r2) ** 2, 0.0)


def covariance(x, y, sig2, a_x=0.07, a_y=0.07):
    """Dense B of eq. covarianceB (c_xy = infinity)."""
    s = np.sqrt(np.asarray(sig2, dtype=np.float64))
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    return s[:, None] * s[None, :] * np.exp(-dx ** 2 / a_x ** 2 - dy ** 2 / a_y ** 2)


def eigenpairs(B, N):
    """The N leading eigenpairs of the symmetric B: mu [N] decreasing, V [N][n] orthonormal rows."""
    mu, V = np.linalg.eigh(B)
    order = np.argsort(mu)[::-1][:N]
    return mu[order], V[:, order].T.copy()


def eigen_ensemble(B, N):
    """(E [N][n], mu [N]) with E_k = V_k sqrt(mu_k) sqrt(N - 1) (eq. eigenvm1)."""
    mu, V = eigenpairs(B, N)
    return V * (np.sqrt(np.maximum(mu, 0.0)) * np.sqrt(N - 1.0))[:, None], mu


def control_rows(Es, component=1):
    """Control rows [N][m] = [f_x over the cells, f_y over the cells] with the members in one component
    (1 = y, the paper's y-momentum forcing of Sec. 4.1)."""
    N, n = Es.shape
    out = np.zeros((N, 2 * n))
    out[:, component * n:(component + 1) * n] = Es
    return out


def apply_separable(p, sig2, v, a_x=0.07, a_y=0.07):
    """B v for a control region that fills a rectangle of cells: with D = diag(sigma) and the kernel
    exp(-dx^2/a_x^2) exp(-dy^2/a_y^2) = Kx (x) Ky on the rectangle, B v = D (Ky kron Kx) D v."""
    g = p.grid()
    cells = p.cells()
    js = sorted({j for j, _ in cells})
    is_ = sorted({i for _, i in cells})
    ny, nx = len(js), len(is_)
    assert ny * nx == len(cells), "the region is not a full rectangle of cells"
    xs, ys = g.xc[is_], g.yc[js]
    Kx = np.exp(-(xs[:, None] - xs[None, :]) ** 2 / a_x ** 2)
    Ky = np.exp(-(ys[:, None] - ys[None, :]) ** 2 / a_y ** 2)
    s = np.sqrt(np.asarray(sig2, dtype=np.float64))
    w = (s * np.asarray(v, dtype=np.float64)).reshape(ny, nx)
    return s * (Ky @ w @ Kx.T).reshape(-1)


def reconstruction_error(f, V):
    """eq. reconstruction_error: the share of f's energy outside the span of the orthonormal rows V."""
    f = np.asarray(f, dtype=np.float64)
    V = np.atleast_2d(np.asarray(V, dtype=np.float64))
    r = f - V.T @ (V @ f)
    return float(r @ r) / float(f @ f)

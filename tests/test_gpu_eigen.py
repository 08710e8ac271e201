"""The deterministic eigen-ensemble on the GPU against the oracle (needs an MI355X; calls the C ABI
through the binding).

Eigenvectors are unique only up to sign and, for repeated eigenvalues, up to a rotation inside the
eigenspace; the comparison therefore uses what is unique: the eigenvalues, the ensemble covariance
E E^T / (N - 1) (the spectral projector scaled by the eigenvalues; unique when mu_N > mu_N+1), and,
for every returned member, the residual of the oracle's B applied to it.

* small regions (cavity and column at h = 1/32, the paper's actuation window at h = 1/64) with and
  without the variance taper against the dense oracle;
* the column region at h = 1/128 (32,768 cells, 64 members): residuals with the oracle's separable
  product, orthogonality, and the leading eigenvalues against ARPACK on the same operator;
* the reconstruction error against the oracle's formula and its limits;
* argument errors.
"""
import numpy as np
import pytest

from oracle import eigen as OG
from oracle import envar as OE
from paper_2605_23812_amd import envar as E

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


REGIONS = {
    "cavity32": (32, "cavity", E.REGION_CAVITY, (0.0, 0.0, 0.0, 0.0)),
    "column32": (32, "column", E.REGION_COLUMN, (0.0, 0.0, 0.0, 0.0)),
    "window64": (64, "box", E.REGION_BOX, (1.25 - 0.32, 1.25 + 0.15, -0.60, 0.15)),
}


def _problems(name):
    n, reg, creg, box = REGIONS[name]
    return OE.Problem(inv_h=n, region=reg, box=box), E.Problem(inv_h=n, region=creg, box=box)


# N sits at a gap of the spectrum (the square cavity's 20th and 21st eigenvalues are equal)
@pytest.mark.parametrize("name,taper,N,a", [("cavity32", E.TAPER_ELLIPSE, 21, 0.07), ("column32", E.TAPER_NONE, 12, 0.07),
                                            ("column32", E.TAPER_ELLIPSE, 32, 0.1),
                                            ("window64", E.TAPER_ELLIPSE, 20, 0.07)])
def test_eigen_ensemble_matches_oracle(name, taper, N, a):
    op, p = _problems(name)
    x, y = OG.cell_coords(op)
    sig2 = OG.taper_variance(op, 0.01, "ellipse" if taper == E.TAPER_ELLIPSE else "none")
    B = OG.covariance(x, y, sig2, a, a)
    mu_all = np.sort(np.linalg.eigvalsh(B))[::-1]
    Er, mur = OG.eigen_ensemble(B, N)
    gap = (mu_all[N - 1] - mu_all[N]) / mu_all[0]
    _say(name, "cells", x.size, "N", N, "mu_N / mu_1", mu_all[N - 1] / mu_all[0], "gap", gap)
    Eg, mug, info = E.eigen_ensemble(p, N, a_x=a, a_y=a, taper=taper, component=1)
    torch.cuda.synchronize()
    Eg, mug = Eg.cpu().numpy(), mug.cpu().numpy()
    _say(" info", info, "mu err", np.abs(mug - mur).max() / mur[0])
    n = x.size
    assert info["converged"] == 1 and info["orth_err"] < 1e-12
    assert np.all(Eg[:, :n] == 0.0)  # only the y component is driven
    Ey = Eg[:, n:]
    assert np.abs(mug - mur).max() <= 1e-12 * mur[0]
    # every member is an eigenvector of the oracle's B with its eigenvalue
    for k in range(N):
        v = Ey[k] / np.linalg.norm(Ey[k])
        r = np.linalg.norm(B @ v - mug[k] * v) / mur[0]
        assert r <= 1e-9, (k, r)
    # the ensemble covariance (unique when the N-th eigenvalue is separated); Davis-Kahan bounds the
    # subspace angle by the block residual (<= sqrt(N) tol mu_1, tol = 1e-10) over the gap
    assert gap > 1e-6
    Pg, Pr = Ey.T @ Ey / (N - 1), Er.T @ Er / (N - 1)
    err = np.abs(Pg - Pr).max() / np.abs(Pr).max()
    _say(" ensemble covariance rel err", err, "bound", 10 * np.sqrt(N) * 1e-10 / gap)
    assert err <= 10 * np.sqrt(N) * 1e-10 / gap
    G = Ey @ Ey.T
    assert np.allclose(np.diag(G), (N - 1) * mug, rtol=1e-10)


def test_eigen_ensemble_full_size_column_h128():
    from scipy.sparse.linalg import LinearOperator, eigsh

    n, N = 128, 64
    op = OE.Problem(inv_h=n, region="column")
    p = E.Problem(inv_h=n, region=E.REGION_COLUMN)
    sig2 = OG.taper_variance(op, 0.01)
    Eg, mug, info = E.eigen_ensemble(p, N, component=1)
    torch.cuda.synchronize()
    Eg, mug = Eg.cpu().numpy(), mug.cpu().numpy()
    ncc = sig2.size
    _say("h=1/128 column: cells", ncc, "info", info)
    assert info["converged"] == 1 and info["orth_err"] < 1e-12 and np.all(Eg[:, :ncc] == 0.0)
    Ey = Eg[:, ncc:]
    for k in range(N):
        v = Ey[k] / np.linalg.norm(Ey[k])
        r = np.linalg.norm(OG.apply_separable(op, sig2, v) - mug[k] * v) / mug[0]
        assert r <= 1e-9, (k, r)
    V = Ey / np.linalg.norm(Ey, axis=1)[:, None]
    assert np.abs(V @ V.T - np.eye(N)).max() <= 1e-12
    A = LinearOperator((ncc, ncc), matvec=lambda v: OG.apply_separable(op, sig2, v), dtype=np.float64)
    ref = np.sort(eigsh(A, k=N + 8, which="LA", tol=1e-13, v0=np.ones(ncc))[0])[::-1][:N]
    _say(" eigenvalue rel err vs ARPACK", np.abs(mug - ref).max() / ref[0])
    assert np.abs(mug - ref).max() <= 1e-11 * ref[0]


def test_reconstruction_error_matches_oracle():
    op, p = _problems("column32")
    N = 16
    Eg, mug, _ = E.eigen_ensemble(p, N)
    rng = np.random.default_rng(3)
    m = E.control_dim(p)
    x, y = OG.cell_coords(op)
    n = x.size
    # a smooth reference forcing in the y component, plus a little noise in both
    f = np.concatenate([1e-3 * rng.standard_normal(n),
                        np.sin(3.0 * x) * np.cos(2.0 * y) + 1e-3 * rng.standard_normal(n)])
    out = E.recon_error(Eg, torch.tensor(f, device="cuda")).cpu().numpy()[0]
    Eh = Eg.cpu().numpy()
    ref = OG.reconstruction_error(f, Eh / np.linalg.norm(Eh, axis=1)[:, None])
    _say("E_rec gpu", out, "oracle", ref)
    assert abs(out - ref) <= 1e-12 * max(ref, 1e-300) + 1e-15
    inside = 0.7 * Eh[0] - 0.2 * Eh[5]
    assert E.recon_error(Eg, torch.tensor(inside, device="cuda")).cpu().numpy()[0] <= 1e-24
    xonly = np.concatenate([np.ones(n), np.zeros(n)])
    assert abs(E.recon_error(Eg, torch.tensor(xonly, device="cuda")).cpu().numpy()[0] - 1.0) <= 1e-15
    assert m == 2 * n


def test_eigen_argument_errors():
    _, p = _problems("cavity32")
    with pytest.raises(E.EnvarError) as ei:
        E.eigen_ensemble(p, 1)
    assert ei.value.code == E.EINVAL
    with pytest.raises(E.EnvarError) as ei:
        E.eigen_ensemble(p, 8, component=2)
    assert ei.value.code == E.EINVAL
    tiny = E.Problem(inv_h=16, region=E.REGION_BOX, box=(1.3, 1.42, -0.2, -0.09))  # 2 x 2 cells
    with pytest.raises(E.EnvarError) as ei:
        E.eigen_ensemble(tiny, 5, taper=E.TAPER_NONE)
    assert ei.value.code == E.EINVAL
    Eg, mug, info = E.eigen_ensemble(tiny, 4, taper=E.TAPER_NONE)  # the whole space: exact in one iteration
    torch.cuda.synchronize()
    op = OE.Problem(inv_h=16, region="box", box=(1.3, 1.42, -0.2, -0.09))
    x, y = OG.cell_coords(op)
    mur = np.sort(np.linalg.eigvalsh(OG.covariance(x, y, np.full(x.size, 0.01))))[::-1]
    assert np.abs(mug.cpu().numpy() - mur).max() <= 1e-14 * mur[0] and info["converged"] == 1

"""GPU anomaly reduction vs textbook least squares (needs an MI355X).

g = X^+ dJ for X_i = f_i - f_0: compared with numpy.linalg.lstsq on the same
seeded rows (FP64 MFMA: 1e-10 relative; FP32 MFMA: cosine >= 0.999999), for
n <= m (Gram path) and n > m (normal-equation path), at the size edges of the
Cholesky variants and at the largest supported system (1024), the closed form of
an antithetic quadratic cost, repeated members (rank-deficient X: the
minimum-norm solution) and a non-finite cost (reported, not returned); FP64 anomalies formed where
they are read, from aligned and unaligned control rows, bit for bit.
"""
import numpy as np
import pytest

from paper_2605_23812_amd import envar as E

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(rows, J, precision):
    c = torch.tensor(rows, dtype=torch.float64, device="cuda")
    j = torch.tensor(J, dtype=torch.float64, device="cuda")
    g = E.gradient(c, j, precision)
    torch.cuda.synchronize()
    return g.cpu().numpy()


# n (or m when n > m) spans every Cholesky variant: four waves of 16 rows each (<= 64), 32-column
# panels with MFMA trailing updates (<= 256), 32-column panels on the vector units (<= 448) and the
# unblocked global-memory kernel. The four-wave
# factor is hit at every wave boundary (16, 32, 48), with a partly filled fourth wave (49, 63) and
# full (64).
@pytest.mark.parametrize("n,m", [(8, 4096), (64, 5000), (17, 333), (130, 1024), (1, 50), (16, 8), (40, 33),
                                 (256, 2048), (200, 100), (300, 1500), (500, 3000),
                                 (16, 700), (32, 700), (48, 700), (49, 700), (63, 700)])
def test_gradient_fp64_matches_lstsq(n, m):
    rng = np.random.default_rng(n * 1000 + m)
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    J = rng.standard_normal(n + 1)
    g = _run(rows, J, E.FP64)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    print("fp64 gradient", n, m, np.abs(g - ref).max() / np.abs(ref).max(), flush=True)
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()


# the edges of the Cholesky variants (one wave <= 64 < MFMA panels <= 256 < vector panels <= 448 <
# unblocked) and the largest supported system, in the Gram (n <= m) and normal-equation (n > m)
# forms; inside the MFMA range, panel counts with a full last panel (96), one row past it (97) and
# ragged trailing tiles (161, 223, 255)
@pytest.mark.parametrize("n,m", [(65, 200), (96, 500), (97, 400), (161, 700), (223, 900), (255, 1000), (257, 600),
                                 (448, 900), (449, 900), (1024, 2048), (1100, 1024)])
def test_gradient_fp64_at_solver_size_edges(n, m):
    rng = np.random.default_rng(7 * n + m)
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    J = rng.standard_normal(n + 1)
    g = _run(rows, J, E.FP64)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print("fp64 gradient at size edge", n, m, err, flush=True)
    assert err <= 1e-9


# An FP64 gradient over at least as many controls as members forms the anomalies where the Gram and
# the final product read them, with 16-byte loads from aligned control rows and element loads from
# rows that are not (a view one element into a buffer). The two must agree bit for bit (the same
# differences, summed in the same order), with the Cholesky solve and the pseudo-inverse, and match
# lstsq. 64- and 128-row Gram blocks, a partial last block, an odd m (element loads either way).
@pytest.mark.parametrize("n,m", [(8, 4096), (64, 5000), (130, 1024), (256, 2048), (17, 333), (17, 334)])
def test_gradient_fp64_onfly_anomalies_aligned_and_not(n, m):
    rng = np.random.default_rng(11 * n + m)
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    J = rng.standard_normal(n + 1)
    a = torch.tensor(rows, dtype=torch.float64, device="cuda")
    buf = torch.zeros((n + 1) * m + 1, dtype=torch.float64, device="cuda")
    b = buf[1:].view(n + 1, m)
    b.copy_(a)
    assert a.data_ptr() % 16 == 0 and b.data_ptr() % 16 == 8
    j = torch.tensor(J, dtype=torch.float64, device="cuda")
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    for precision in (E.FP64, E.FP64 | E.GRADIENT_PINV):
        ga = E.gradient(a, j, precision)
        gb = E.gradient(b, j, precision)
        torch.cuda.synchronize()
        ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
        err = np.abs(ga - ref).max() / np.abs(ref).max()
        print("fp64 gradient, aligned against unaligned control rows:", n, m, precision, "lstsq", err, flush=True)
        assert np.array_equal(ga, gb)
        assert err <= 1e-9


@pytest.mark.parametrize("n,m", [(8, 4096), (64, 65536), (256, 65536)])
def test_gradient_fp32_mfma_cosine(n, m):
    rng = np.random.default_rng(n + m)
    rows = rng.standard_normal((n + 1, m)) * 5e-3
    J = rng.standard_normal(n + 1) * 1e-3
    g = _run(rows, J, E.MIXED)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    cos = g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref))
    print("fp32 gradient", n, m, cos, np.linalg.norm(g - ref) / np.linalg.norm(ref), flush=True)
    assert cos >= 0.999999


def test_gradient_exact_on_antithetic_quadratic():
    m = 24
    rng = np.random.default_rng(3)
    A = rng.standard_normal((m, m))
    Q = A @ A.T / m + np.eye(m)
    b = rng.standard_normal(m)
    f0 = rng.standard_normal(m)
    D = rng.standard_normal((m, m)) * 0.1
    rows = np.vstack([f0, f0 + D, f0 - D])
    J = np.array([0.5 * r @ Q @ r + b @ r for r in rows])
    g = _run(rows, J, E.FP64)
    grad = Q @ f0 + b
    assert np.abs(g - grad).max() <= 1e-9 * np.abs(grad).max()


@pytest.mark.parametrize("precision,tol", [(E.FP64, 1e-8), (E.MIXED, 1e-5)])
def test_gradient_with_repeated_members_is_minimum_norm(precision, tol):
    rng = np.random.default_rng(77)
    n, m = 12, 3000
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    rows[7] = rows[3]  # a repeated member with the same cost: X has rank n - 1
    rows[11] = rows[2]
    J = rng.standard_normal(n + 1)
    J[7], J[11] = J[3], J[2]
    g = _run(rows, J, precision)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)  # minimum-norm solution
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print("repeated members", precision, err, flush=True)
    assert err <= tol


def test_gradient_with_repeated_members_in_the_panel_range():
    """Rank-deficient X at n = 150 (32-column MFMA panels): the minimum-norm solution."""
    rng = np.random.default_rng(78)
    n, m = 150, 4000
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    for a, b in ((40, 3), (120, 77), (150, 149)):
        rows[a] = rows[b]
    J = rng.standard_normal(n + 1)
    for a, b in ((40, 3), (120, 77), (150, 149)):
        J[a] = J[b]
    g = _run(rows, J, E.FP64)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print("repeated members, n = 150", err, flush=True)
    assert err <= 1e-8


def test_mixed_gradient_of_a_nearly_dependent_ensemble_is_the_fp64_gradient():
    """Eight pairs of members that differ by 1e-5 of their perturbation: the FP32 Gram's rounding
    (about 1e-7 of its largest entries) swamps the pairs' small eigenvalues (about 1e-10 of the
    largest), so the FP32 factor fails; the call then forms the system again in FP64 from the
    control rows, which is the FP64 gradient's own arithmetic: the results agree to the bit."""
    rng = np.random.default_rng(79)
    n, m = 48, 6000
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    for a in range(8):
        i, j = 1 + 2 * a, 2 + 2 * a
        rows[j] = rows[i] + 1e-5 * (rows[i] - rows[0]) * rng.standard_normal(m)
    J = rng.standard_normal(n + 1)
    g64 = _run(rows, J, E.FP64)
    gmx = _run(rows, J, E.MIXED)
    # the FP64 gradient is the ridged solution X^T (G + 1e-12 tr(G)/n I)^-1 dJ (the pairs'
    # eigenvalues are about 100 times the ridge, so it moves them by about 1%): checked against
    # numpy to the conditioning of G + ridge (about 1e10)
    X = rows[1:] - rows[0]
    G = X @ X.T
    ref = X.T @ np.linalg.solve(G + 1e-12 * np.trace(G) / n * np.eye(n), J[1:] - J[0])
    err = np.abs(g64 - ref).max() / np.abs(ref).max()
    print("nearly dependent: FP64 vs numpy (ridged)", err, " mixed vs FP64 max |diff|", np.abs(gmx - g64).max(),
          flush=True)
    assert err <= 1e-5
    assert np.array_equal(gmx, g64)


@pytest.mark.parametrize("n,m", [(40, 500), (150, 4000), (200, 100)])
def test_pseudo_inverse_gradient_matches_lstsq(n, m):
    """precision | GRADIENT_PINV: the eigen-pseudo-inverse of the Gram (Jacobi), in FP64, for the
    Gram (n <= m) and normal-equation (n > m) forms; mixed precision with the flag runs on the FP64
    Gram and gives the same bits."""
    rng = np.random.default_rng(11 * n + m)
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    J = rng.standard_normal(n + 1)
    g = _run(rows, J, E.FP64 | E.GRADIENT_PINV)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print("pseudo-inverse gradient", n, m, err, flush=True)
    assert err <= 1e-9
    if n <= m:
        assert np.array_equal(_run(rows, J, E.MIXED | E.GRADIENT_PINV), g)


def test_pseudo_inverse_gradient_with_repeated_members_is_minimum_norm():
    rng = np.random.default_rng(80)
    n, m = 100, 3000
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    J = rng.standard_normal(n + 1)
    for a, b in ((40, 3), (70, 12), (99, 98)):
        rows[a] = rows[b]
        J[a] = J[b]
    g = _run(rows, J, E.FP64 | E.GRADIENT_PINV)
    X = rows[1:] - rows[0]
    ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print("pseudo-inverse, repeated members", err, flush=True)
    assert err <= 1e-9


def test_gradient_reports_a_non_finite_cost():
    rng = np.random.default_rng(5)
    rows = rng.standard_normal((9, 500)) * 1e-2
    J = rng.standard_normal(9)
    J[4] = np.nan
    for precision in (E.FP64, E.MIXED):
        with pytest.raises(E.EnvarError) as ei:
            _run(rows, J, precision)
        assert ei.value.code == E.EDIVERGED
    assert np.all(np.isfinite(_run(rows[:4], J[:4], E.FP64)))  # the library still works

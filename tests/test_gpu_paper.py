"""The paper's geometry (Sec. 2, Table tabgeometry, boundary conditions of Sec. 4.4) on the GPU
against the oracle (needs an MI355X; calls the C ABI through the binding).

* the forward at h = 1/32, Re = 6250, with y-only forcing rows on the paper's actuation window
  (Sec. 4.1), FP64 and mixed precision: costs and final fields;
* the lid-sensor series in that geometry;
* the eigen-ensemble of the actuation window against the dense oracle.
"""
import numpy as np
import pytest

from oracle import eigen as OG
from oracle import envar as OE
from oracle import gn as OGN
from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WINDOW = (1.25 - 0.32, 1.25 + 0.15, -0.60, 0.15)


def _say(*a):
    print(*a, flush=True)


def _setup(n=32, spin=40, Re=6250.0):
    op = OE.Problem(inv_h=n, Re=Re, geometry="paper", region="box", box=WINDOW)
    p = E.Problem(inv_h=n, Re=Re, geometry=E.CAVITY_PAPER, region=E.REGION_BOX, box=WINDOW)
    u0, v0 = inputs.initial_field(n, amp=1e-3, geometry="paper")
    st = OE.spinup(op, OE.initial_state(op, u0, v0), spin)
    return op, p, st


def _y_rows(op, N, scale, seed):
    """Seeded y-only forcing rows on the control cells (the x half zero)."""
    rng = np.random.default_rng(seed)
    n = len(op.cells())
    rows = np.zeros((N, 2 * n))
    rows[:, n:] = scale * rng.standard_normal((N, n))
    return rows


@pytest.mark.parametrize("precision,tol", [(E.FP64, 1e-10), (E.MIXED, 1e-6)])
def test_paper_geometry_forward_matches_oracle(precision, tol):
    n, horizon = 32, 12
    op, p, st = _setup(n)
    p.precision = precision
    assert E.control_dim(p) == op.m
    rows = np.vstack([np.zeros(op.m), _y_rows(op, 2, 1e-2, 5)])
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    J, F, stats = E.forward(p, state, torch.tensor(rows, device="cuda"), horizon, fields=True)
    torch.cuda.synchronize()
    J = J.cpu().numpy()
    u, v = E.split_fields(p, F)
    for i in range(rows.shape[0]):
        Jr, sr = OE.forward_member(op, st, rows[i], horizon, return_state=True)
        _say("member", i, "J", J[i], "oracle", Jr, "rel", abs(J[i] - Jr) / abs(Jr))
        assert abs(J[i] - Jr) <= tol * abs(Jr)
        assert np.abs(u[i] - sr.u).max() <= tol * np.abs(sr.u).max()
        assert np.abs(v[i] - sr.v).max() <= tol * np.abs(sr.u).max()
    assert stats["unconverged"] == 0


def test_paper_geometry_sensor_series_match_oracle():
    n, horizon, every = 32, 12, 3
    op, p, st = _setup(n)
    rows = np.vstack([np.zeros(op.m), _y_rows(op, 2, 1e-2, 6)])
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    J, series, _ = E.forward_obs(p, state, torch.tensor(rows, device="cuda"), horizon, every)
    torch.cuda.synchronize()
    Jr, Sr = OGN.forward_obs(op, st, rows, horizon, every)
    s = series.cpu().numpy()
    _say("paper geometry series max |gpu - oracle|", np.abs(s - Sr).max(), "scale", np.abs(Sr).max())
    assert np.abs(s - Sr).max() <= 1e-10 * np.abs(Sr).max()
    assert np.all(np.abs(J.cpu().numpy() - Jr) <= 1e-10 * np.abs(Jr))


def test_paper_window_eigen_ensemble_matches_oracle():
    n, N = 32, 10
    op = OE.Problem(inv_h=n, geometry="paper", region="box", box=WINDOW)
    p = E.Problem(inv_h=n, geometry=E.CAVITY_PAPER, region=E.REGION_BOX, box=WINDOW)
    x, y = OG.cell_coords(op)
    B = OG.covariance(x, y, OG.taper_variance(op))
    mu_all = np.sort(np.linalg.eigvalsh(B))[::-1]
    gap = (mu_all[N - 1] - mu_all[N]) / mu_all[0]
    Eg, mug, info = E.eigen_ensemble(p, N)
    torch.cuda.synchronize()
    mug = mug.cpu().numpy()
    _say("window cells", x.size, "info", info, "gap", gap)
    assert info["converged"] == 1 and gap > 1e-6
    assert np.abs(mug - mu_all[:N]).max() <= 1e-12 * mu_all[0]

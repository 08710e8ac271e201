"""Vector-observation EnVar on the GPU against the oracle (needs an MI355X; calls the C ABI).

* the lid-sensor series recorded during the forward ensemble (FP64 and mixed precision);
* the Gauss-Newton step (Y, H_GN = Y^T Y + (N - 1) I on the FP64 matrix cores, gradient, step,
  the two terms of J(w)) on seeded synthetic series, N up to 64 and n_obs up to 20,000;
* the posterior variance diag(E H_GN^-1 E^T) on seeded synthetic controls;
* one end-to-end step at h = 1/32 where each side runs its own forward ensemble;
* argument errors.
"""
import numpy as np
import pytest

from oracle import envar as OE
from oracle import gn as OG
from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


def _setup(n=32, spin=30, N=3, ell=0.1, sigma=1e-2):
    op = OE.Problem(inv_h=n, Re=4000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    st = OE.spinup(op, OE.initial_state(op, u0, v0), spin)
    rows = np.vstack([np.zeros(op.m), inputs.grf_perturbations(N, n, ell, sigma)])
    return op, st, rows


@pytest.mark.parametrize("precision,tol", [(E.FP64, 1e-10), (E.MIXED, 1e-6)])
def test_sensor_series_match_oracle(precision, tol):
    n, horizon, every = 32, 12, 3
    op, st, rows = _setup(n)
    p = E.Problem(inv_h=n, Re=4000.0, precision=precision)
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    ctrl = torch.tensor(rows, dtype=torch.float64, device="cuda")
    J, series, stats = E.forward_obs(p, state, ctrl, horizon, every)
    torch.cuda.synchronize()
    Jr, Sr = OG.forward_obs(op, st, rows, horizon, every)
    s = series.cpu().numpy()
    _say("series", s.shape, "max |gpu - oracle|", np.abs(s - Sr).max(), "scale", np.abs(Sr).max())
    assert s.shape == Sr.shape == (rows.shape[0], 8, horizon // every)
    assert np.abs(s - Sr).max() <= tol * np.abs(Sr).max()
    assert np.all(np.abs(J.cpu().numpy() - Jr) <= tol * np.abs(Jr))
    # the fluctuations (what the step uses) agree as well
    assert np.abs(OG.observations(s) - OG.observations(Sr)).max() <= 10 * tol * np.abs(Sr).max()


@pytest.mark.parametrize("N,K", [(1, 30), (8, 50), (64, 2500)])
def test_gn_step_matches_oracle(N, K):
    rng = np.random.default_rng(100 + N)
    eps = 1e-4
    base = rng.standard_normal((1, 8, K)) + 3.0
    series = np.concatenate([base, base + eps * rng.standard_normal((N, 8, K))], axis=0)
    w = 0.1 * rng.standard_normal(N)
    ref = OG.gn_step(OG.observations(series), eps, w)
    dw, H, jw = E.gn_step(torch.tensor(series, device="cuda"), eps, torch.tensor(w, device="cuda"))
    torch.cuda.synchronize()
    dw, H, jw = dw.cpu().numpy(), H.cpu().numpy(), jw.cpu().numpy()
    _say("N", N, "K", K, "dw err", np.abs(dw - ref["dw"]).max() / np.abs(ref["dw"]).max(),
         "H err", np.abs(H - ref["H"]).max() / np.abs(ref["H"]).max())
    assert np.abs(H - ref["H"]).max() <= 1e-10 * np.abs(ref["H"]).max()
    assert np.abs(dw - ref["dw"]).max() <= 1e-8 * np.abs(ref["dw"]).max()
    assert abs(jw[0] - ref["J_obs"]) <= 1e-10 * ref["J_obs"] and abs(jw[1] - ref["J_prior"]) <= 1e-12 * max(ref["J_prior"], 1e-300)


@pytest.mark.parametrize("N,m", [(8, 4096), (64, 65536), (128, 1000)])
def test_posterior_variance_matches_oracle(N, m):
    rng = np.random.default_rng(7 + N)
    eps = 1e-4
    f0 = rng.standard_normal(m)
    controls = np.vstack([f0, f0 + eps * rng.standard_normal((N, m))])
    Y = rng.standard_normal((3 * N, N))
    H = Y.T @ Y + (N - 1) * np.eye(N)
    ref = OG.posterior_variance(controls, eps, H)
    var = E.posterior_var(torch.tensor(controls, device="cuda"), eps, torch.tensor(H, device="cuda"))
    torch.cuda.synchronize()
    v = var.cpu().numpy()
    _say("posterior N", N, "m", m, "rel err", np.abs(v - ref).max() / np.abs(ref).max())
    assert np.abs(v - ref).max() <= 1e-10 * np.abs(ref).max()


def test_end_to_end_gauss_newton_step_at_h32():
    n, horizon, eps = 32, 20, 1e-4
    op = OE.Problem(inv_h=n, Re=4000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    st = OE.spinup(op, OE.initial_state(op, u0, v0), 40)
    N = 4
    Eb = inputs.grf_perturbations(N, n, 0.1, 1.0)  # ensemble directions E_i
    f_c = 1e-2 * inputs.grf_perturbations(1, n, 0.1, 1.0, seed=99)[0]
    rows = np.vstack([f_c, f_c + eps * Eb])
    w = np.zeros(N)
    _, Sr = OG.forward_obs(op, st, rows, horizon)
    ref = OG.gn_step(OG.observations(Sr), eps, w)
    p = E.Problem(inv_h=n, Re=4000.0)
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    _, series, _ = E.forward_obs(p, state, torch.tensor(rows, device="cuda"), horizon)
    dw, H, jw = E.gn_step(series, eps, torch.tensor(w, device="cuda"))
    var = E.posterior_var(torch.tensor(rows, device="cuda"), eps, H)
    torch.cuda.synchronize()
    dw = dw.cpu().numpy()
    vref = OG.posterior_variance(rows, eps, ref["H"])
    _say("end to end dw", dw, "oracle", ref["dw"])
    assert np.abs(dw - ref["dw"]).max() <= 1e-6 * np.abs(ref["dw"]).max()
    assert np.abs(var.cpu().numpy() - vref).max() <= 1e-6 * np.abs(vref).max()


def test_gn_argument_errors():
    p = E.Problem(inv_h=16, Re=10.0, geometry=E.CHANNEL, region=E.REGION_BOX, box=(1.0, 1.2, 0.2, 0.4))
    u0 = np.zeros((16, 65))
    v0 = np.zeros((17, 64))
    state = E.state_init(p, u0, v0)
    ctrl = torch.zeros((2, E.control_dim(p)), dtype=torch.float64, device="cuda")
    with pytest.raises(E.EnvarError) as ei:
        E.forward_obs(p, state, ctrl, 4)
    assert ei.value.code == E.EINVAL
    s = torch.zeros((3, 8, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(E.EnvarError):
        E.gn_step(s, 0.0, torch.zeros(2, dtype=torch.float64, device="cuda"))
    with pytest.raises(E.EnvarError):
        E.posterior_var(torch.zeros((130, 10), dtype=torch.float64, device="cuda"), 1e-4,
                        torch.eye(129, dtype=torch.float64, device="cuda"))

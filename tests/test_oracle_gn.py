"""Pins of the vector-observation EnVar oracle (CPU).

* the sensor sampling reproduces linear velocity fields exactly (bilinear interpolation);
* the fluctuations have zero time mean per channel;
* on an affine observation model the finite-difference Y is exact and one Gauss-Newton step
  lands on the minimiser of J(w), found independently by an iterative least-squares solver,
  with a vanishing central-difference gradient there;
* the posterior variance reduces to the ensemble's prior variance when the observations do not
  depend on w, shrinks below it otherwise, and vanishes where no member moves the control;
* recording the sensors does not change the forward's cost.
"""
import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import envar as OE
from oracle import gn
from paper_2605_23812_amd import inputs


def test_sample_is_exact_on_linear_fields():
    p = OE.Problem(inv_h=16)
    g = p.grid()
    h = g.h
    xu = np.arange(g.NX + 1) * h
    yu = g.y0 + (np.arange(g.NY) + 0.5) * h
    xv = (np.arange(g.NX) + 0.5) * h
    yv = g.y0 + np.arange(g.NY + 1) * h
    u = 0.3 + 1.7 * xu[None, :] - 2.2 * yu[:, None]
    v = -1.1 + 0.4 * xv[None, :] + 3.3 * yv[:, None]
    pts = gn.sensor_points(p)
    assert [round(x - p.x_cav, 12) for x, _ in pts] == [0.2, 0.4, 0.6, 0.8] and all(y == 0.0 for _, y in pts)
    s = gn.sample(g, u, v, pts)
    for k, (x, y) in enumerate(pts):
        assert abs(s[2 * k] - (0.3 + 1.7 * x - 2.2 * y)) < 1e-12
        assert abs(s[2 * k + 1] - (-1.1 + 0.4 * x + 3.3 * y)) < 1e-12


def test_observations_have_zero_time_mean_and_channel_major_layout():
    rng = np.random.default_rng(1)
    series = rng.standard_normal((3, gn.N_CHANNELS, 7)) + 5.0
    d = gn.observations(series)
    assert d.shape == (3, gn.N_CHANNELS * 7)
    assert np.abs(d.reshape(3, gn.N_CHANNELS, 7).sum(axis=2)).max() < 1e-12
    # channel c occupies entries [7 c, 7 c + 7)
    assert np.allclose(d[1, 14:21], series[1, 2] - series[1, 2].mean())


@pytest.mark.parametrize("N", [3, 8])
def test_gn_step_on_an_affine_model_reaches_the_minimiser(N):
    rng = np.random.default_rng(N)
    n_obs, eps = 40, 1e-4
    A = rng.standard_normal((n_obs, N))
    dc = rng.standard_normal(n_obs)
    w0 = 0.3 * rng.standard_normal(N)
    obs = np.vstack([dc + A @ w0] + [dc + A @ (w0 + eps * np.eye(N)[i]) for i in range(N)])
    out = gn.gn_step(obs, eps, w0)
    assert np.allclose(out["Y"], A, rtol=1e-6, atol=1e-8)
    w1 = w0 + out["dw"]

    def resid(w):
        return np.concatenate([dc + A @ w, np.sqrt(N - 1.0) * w])

    ref = least_squares(resid, np.zeros(N), xtol=1e-15, ftol=1e-15, gtol=1e-15).x
    assert np.abs(w1 - ref).max() < 1e-6 * (1 + np.abs(ref).max())

    def J(w):
        r = resid(w)
        return 0.5 * float(r @ r)

    gfd = np.array([(J(w1 + 1e-6 * e) - J(w1 - 1e-6 * e)) / 2e-6 for e in np.eye(N)])
    assert np.abs(gfd).max() < 1e-6
    assert abs(out["J_obs"] + out["J_prior"] - J(w0)) < 1e-9 * J(w0)


def test_posterior_variance_limits():
    rng = np.random.default_rng(3)
    N, m, eps = 6, 30, 1e-4
    f0 = rng.standard_normal(m)
    Ecols = rng.standard_normal((N, m))
    Ecols[:, 5] = 0.0  # a control entry that no member moves
    controls = np.vstack([f0, f0 + eps * Ecols])
    prior = gn.posterior_variance(controls, eps, (N - 1) * np.eye(N))
    assert np.allclose(prior, (Ecols ** 2).sum(axis=0) / (N - 1), rtol=1e-6)  # eq. (ensemble_covariance)
    Y = rng.standard_normal((50, N))
    post = gn.posterior_variance(controls, eps, Y.T @ Y + (N - 1) * np.eye(N))
    assert np.all(post <= prior * (1 + 1e-9)) and post[5] == 0.0 and np.all(post[np.arange(m) != 5] > 0)


def test_recording_the_sensors_keeps_the_cost():
    p = OE.Problem(inv_h=16, Re=4000.0)
    u0, v0 = inputs.initial_field(16, amp=1e-3)
    base = OE.spinup(p, OE.initial_state(p, u0, v0), 10)
    f = 1e-2 * np.random.default_rng(2).standard_normal(p.m)
    J, series = gn.forward_member_obs(p, base, f, 6, every=2)
    assert series.shape == (gn.N_CHANNELS, 3)
    assert J == OE.forward_member(p, base, f, 6)


def _affine_observer(A, dc, Ecols, fe):
    """Sensor series of an affine model: channel-major series whose fluctuations are dc + A w
    for the control f = fe + E w (w recovered from f by least squares)."""
    K = A.shape[0] // gn.N_CHANNELS
    pinv = np.linalg.pinv(Ecols.T)

    def observe(rows):
        out = []
        for f in rows:
            wv = pinv @ (f - fe)
            d = dc + A @ wv
            out.append(d.reshape(gn.N_CHANNELS, K) + 7.0)  # a constant offset: removed by the time mean
        return np.array(out)

    return observe


def _affine_problem(N, seed):
    rng = np.random.default_rng(seed)
    K, m = 6, 3 * N + 4
    A = rng.standard_normal((gn.N_CHANNELS * K, N))
    dc = rng.standard_normal(gn.N_CHANNELS * K)
    # fluctuations have zero time mean per channel: project both onto that subspace
    Z = lambda x: (x.reshape(gn.N_CHANNELS, K, -1) - x.reshape(gn.N_CHANNELS, K, -1).mean(axis=1, keepdims=True)
                   ).reshape(gn.N_CHANNELS * K, -1)
    A, dc = Z(A), Z(dc[:, None])[:, 0]
    Ecols = rng.standard_normal((N, m))
    fe = rng.standard_normal(m)
    return A, dc, Ecols, fe


@pytest.mark.parametrize("N", [3, 6])
def test_gauss_newton_loop_solves_the_affine_problem_in_one_step(N):
    A, dc, Ecols, fe = _affine_problem(N, 10 + N)
    w, hist = gn.iterate_ens(_affine_observer(A, dc, Ecols, fe), fe, Ecols, 1e-4, 2, method="gn")
    ref = np.linalg.lstsq(np.vstack([A, np.sqrt(N - 1.0) * np.eye(N)]), np.concatenate([-dc, np.zeros(N)]),
                          rcond=None)[0]
    assert np.abs(w - ref).max() < 1e-6 * (1 + np.abs(ref).max())
    assert hist[1]["gnorm"] < 1e-6 * hist[0]["gnorm"]


@pytest.mark.parametrize("N", [3, 6])
def test_lbfgs_loop_decreases_and_converges_on_the_affine_problem(N):
    A, dc, Ecols, fe = _affine_problem(N, 20 + N)
    w, hist = gn.iterate_ens(_affine_observer(A, dc, Ecols, fe), fe, Ecols, 1e-4, 4 * N, method="lbfgs", memory=8)
    J = [h["J"] for h in hist]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(J, J[1:]))  # Armijo: monotone decrease
    ref = np.linalg.lstsq(np.vstack([A, np.sqrt(N - 1.0) * np.eye(N)]), np.concatenate([-dc, np.zeros(N)]),
                          rcond=None)[0]
    assert np.abs(w - ref).max() < 1e-5 * (1 + np.abs(ref).max())


def test_lbfgs_two_loop_matches_the_dense_bfgs_inverse():
    """With exact pairs of a quadratic, the two-loop product equals the dense inverse-BFGS update."""
    rng = np.random.default_rng(4)
    n = 5
    M = rng.standard_normal((n, n))
    H = M @ M.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(3)]
    Yh = [H @ s for s in S]
    g = rng.standard_normal(n)
    gamma = float(S[-1] @ Yh[-1]) / float(Yh[-1] @ Yh[-1])
    Binv = gamma * np.eye(n)
    for s, y in zip(S, Yh):
        rho = 1.0 / float(y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        Binv = V.T @ Binv @ V + rho * np.outer(s, s)
    assert np.allclose(gn.lbfgs_direction(g, S, Yh), -Binv @ g, rtol=1e-10, atol=1e-12)

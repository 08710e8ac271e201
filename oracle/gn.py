"""Oracle of the vector-observation EnVar step (Sec. 3.3.1 with the observation of Sec. 4.1).

TEST INFRASTRUCTURE ONLY (see the package header).

* ``sensor_points``  : the four points of Sec. 4.1, x = x_cav + 1/5 ... 4/5 on the cavity
                       lid y = 0 (the lid is the shear-layer line; the paper's cavity starts
                       at x = 0, this channel places it at x = x_cav).
* ``sample``         : each velocity component at each point, by bilinear interpolation of
                       that component on its own MAC positions.
* ``forward_obs``    : the N+1 forward runs of eq. (fdapprox) recording the sensor series
                       u(x_s, t_j) every ``every`` steps (t_j = the end of steps every, 2 every, ...).
* ``observations``   : H q(f) of eq. (J_w): the fluctuation u' = u - u_bar (u_bar = the time
                       mean of the member's own samples) of every channel, channel-major
                       (channel c = 2 s + component, then time).
* ``gn_step``        : eq. (gradient_EnVar), eq. (Hessian_EnVar) and eq. (update_Newton) with
                       R = I and y = 0: Y_i = (d_i - d_0) / eps, H_GN = Y^T Y + (N - 1) I,
                       dJ/dw = Y^T d_0 + (N - 1) w, dw = -H_GN^-1 dJ/dw, and the two terms of
                       J(w) = 1/2 |d_0|^2 + 1/2 (N - 1) |w|^2.
* ``posterior_variance``: the diagonal of eq. (posterior_covariance_matrix),
                       B_post = E H_GN^-1 E^T with E_i = (f_i - f_0) / eps.
* ``iterate_ens``    : the EnVar loop over w (ensemble fixed, Sec. 3.3.3) with the
                       Gauss-Newton update of eq. (update_Newton) or the L-BFGS update of
                       eq. (update_BFGS) and its Armijo line search; ``lbfgs_direction`` is
                       the two-loop recursion.
"""
import numpy as np

from . import cost, ns

N_SENSORS = 4
N_CHANNELS = 2 * N_SENSORS


def sensor_points(p):
    """(x, y) of the four sensors (Sec. 4.1)."""
    return [(p.x_cav + k / 5.0, 0.0) for k in (1, 2, 3, 4)]


def _bilinear(field, x0, y0, h, x, y):
    """Bilinear interpolation of a field sampled at (x0 + i h, y0 + j h), field[j, i]."""
    fx, fy = (x - x0) / h, (y - y0) / h
    i, j = int(np.floor(fx)), int(np.floor(fy))
    tx, ty = fx - i, fy - j
    return ((1 - ty) * ((1 - tx) * field[j, i] + tx * field[j, i + 1])
            + ty * ((1 - tx) * field[j + 1, i] + tx * field[j + 1, i + 1]))


def sample(g, u, v, points):
    """[2 * len(points)] = (u, v) at each point: u faces sit at (i h, y0 + (j + 1/2) h),
    v faces at ((i + 1/2) h, y0 + j h)."""
    h = g.h
    out = []
    for x, y in points:
        out.append(_bilinear(u, 0.0, g.y0 + 0.5 * h, h, x, y))
        out.append(_bilinear(v, 0.5 * h, g.y0, h, x, y))
    return np.array(out)


def forward_member_obs(p, base, f, horizon, every=1):
    """One member: J (as in the scalar forward) and its sensor series [N_CHANNELS, horizon // every]."""
    g, P = p.grid(), p.poisson()
    Fu, Fv = ns.face_forcing(g, p.cells(), np.asarray(f, dtype=np.float64))
    pts = sensor_points(p)
    st = base.copy()
    acc = cost.Welford((g.NY, g.NX))
    series = []
    for n in range(1, horizon + 1):
        st, *_ = ns.step(g, P, st, p.nu, p.step_dt, Fu, Fv)
        acc.add(*ns.cell_velocity(g, st.u, st.v))
        if n % every == 0:
            series.append(sample(g, st.u, st.v, pts))
    J = acc.j_obs(g.fluid, p.step_dt, g.h) + cost.penalty(np.asarray(f), g.h, p.penalty)
    return J, np.array(series).T.copy()


def forward_obs(p, base, controls, horizon, every=1):
    """J [n_rows] and the raw sensor series [n_rows, N_CHANNELS, horizon // every]."""
    controls = np.asarray(controls, dtype=np.float64)
    res = [forward_member_obs(p, base, controls[i], horizon, every) for i in range(controls.shape[0])]
    return np.array([r[0] for r in res]), np.array([r[1] for r in res])


def observations(series):
    """[n_rows, N_CHANNELS * K]: fluctuations about each channel's own time mean, channel-major."""
    series = np.asarray(series, dtype=np.float64)
    mean = series.mean(axis=2, keepdims=True)
    return (series - mean).reshape(series.shape[0], -1)


def gn_step(obs, eps, w):
    """Gauss-Newton step in ensemble space from the observation vectors obs [N + 1, n_obs].

    Returns dict(dw, H, grad, J_obs, J_prior, Y)."""
    obs = np.asarray(obs, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    N = obs.shape[0] - 1
    d0 = obs[0]
    Y = ((obs[1:] - d0) / eps).T                      # n_obs x N, column i = Y_(:, i)
    H = Y.T @ Y + (N - 1) * np.eye(N)
    grad = Y.T @ d0 + (N - 1) * w
    dw = -np.linalg.solve(H, grad)
    return dict(dw=dw, H=H, grad=grad, J_obs=0.5 * float(d0 @ d0), J_prior=0.5 * (N - 1) * float(w @ w), Y=Y)


def posterior_variance(controls, eps, H):
    """diag(E H^-1 E^T) with E_(:, i) = (f_i - f_0) / eps (rows of ``controls`` are f_0 .. f_N)."""
    controls = np.asarray(controls, dtype=np.float64)
    E = ((controls[1:] - controls[0]) / eps).T       # m x N
    C = np.linalg.inv(np.asarray(H, dtype=np.float64))
    return np.einsum("ka,ab,kb->k", E, C, E)


# ---------------------------------------------------------------------------- the EnVar loop over w
def lbfgs_direction(g, S, Yh):
    """-H^-1 g by the two-loop recursion over the stored pairs (s_k, y_k), oldest first, with the
    initial Hessian scaled by s^T y / y^T y of the newest pair (Nocedal and Wright, Alg. 7.4)."""
    q = np.array(g, dtype=np.float64)
    alphas = []
    for s, y in zip(reversed(S), reversed(Yh)):
        rho = 1.0 / float(y @ s)
        a = rho * float(s @ q)
        q -= a * y
        alphas.append((rho, a, s, y))
    gamma = float(S[-1] @ Yh[-1]) / float(Yh[-1] @ Yh[-1]) if S else 1.0
    r = gamma * q
    for rho, a, s, y in reversed(alphas):
        b = rho * float(y @ r)
        r += (a - b) * s
    return -r


def iterate_ens(observe, fe, Ecols, eps, iters, method="gn", memory=5, c1=1e-4, shrink=0.5, max_trials=10,
                w0=None):
    """EnVar minimisation of J(w) over the ensemble weights (eq. J_w), the ensemble held fixed.

    ``observe(rows)`` returns the raw sensor series [len(rows), N_CHANNELS, K] of the forward runs
    of the control rows. Every iteration runs the centre f = f^(e) + E w and the N members
    f + eps E_i (eq. fdapprox), forms the gradient and H_GN (``gn_step``) and updates w:
    method "gn": w += dw (eq. update_Newton, unit step); method "lbfgs": w += alpha d with
    d = -H_BFGS^-1 dJ/dw (eq. update_BFGS, ``memory`` pairs) and alpha the first of 1, shrink,
    shrink^2, ... meeting the Armijo condition J(w + alpha d) <= J(w) + c1 alpha g.d (each trial
    one centre run); the pair (s, y) is stored when s.y > 0. Returns the final w and a record per
    iteration (J, J_obs, J_prior, |g|, alpha, trials)."""
    Ecols = np.asarray(Ecols, dtype=np.float64)          # N x m, row i = E_(:, i)
    fe = np.asarray(fe, dtype=np.float64)
    N = Ecols.shape[0]
    w = np.zeros(N) if w0 is None else np.array(w0, dtype=np.float64)
    S, Yh, hist = [], [], []

    def J_of(wv):
        d0 = observations(observe((fe + wv @ Ecols)[None, :]))[0]
        return 0.5 * float(d0 @ d0) + 0.5 * (N - 1) * float(wv @ wv)

    g_prev, w_prev = None, None
    for _ in range(iters):
        f = fe + w @ Ecols
        rows = np.vstack([f, f + eps * Ecols])
        out = gn_step(observations(observe(rows)), eps, w)
        g, J = out["grad"], out["J_obs"] + out["J_prior"]
        if g_prev is not None:
            s, y = w - w_prev, g - g_prev
            if float(s @ y) > 0.0:
                S.append(s)
                Yh.append(y)
                if len(S) > memory:
                    S.pop(0)
                    Yh.pop(0)
        if method == "gn":
            alpha, trials, step = 1.0, 0, out["dw"]
        else:
            d = lbfgs_direction(g, S, Yh)
            gd = float(g @ d)
            alpha, trials, step = 1.0, 0, None
            while trials < max_trials:
                trials += 1
                if J_of(w + alpha * d) <= J + c1 * alpha * gd:
                    step = alpha * d
                    break
                alpha *= shrink
            if step is None:
                alpha, step = 0.0, np.zeros(N)
        hist.append(dict(J=J, J_obs=out["J_obs"], J_prior=out["J_prior"], gnorm=float(np.linalg.norm(g)),
                         alpha=alpha, trials=trials))
        g_prev, w_prev = g, w.copy()
        w = w + step
        if method != "gn" and alpha == 0.0:
            break
    return w, hist

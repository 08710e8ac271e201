"""Pins of the oracle's Navier-Stokes step against closed forms (CPU only).

Each test fixes an expected value from mathematics, not from the oracle:
  * Taylor-Green, linear limit: the discrete mode is divergence free and an
    eigenvector of lap_h, so its amplitude follows the AB2 recurrence exactly.
  * Taylor-Green, nonlinear: decay e^{-2 nu t}, error O(h^2).
  * forced Taylor-Green: a cell forcing balancing lap_h is a steady state,
    which pins operator P of eq. (discrete_NS) and the AB2 treatment of F.
  * energy conservation of the conservative advection for div-free fields.
  * plane Poiseuille: the discrete fully developed profile a (y(1-y) + h^2/4)
    derived by hand from the wall mirror rule, and dp/dx = -2 a nu.
  * projection: divergence-free to rounding, idempotent, exact on gradients.
"""
import numpy as np
import pytest

from oracle import cost, ns
from oracle.envar import Problem, initial_state, spinup
from oracle.geometry import ACTIVE, OUTFLOW, Grid, control_cells


def _tg_fields(g, A):
    """Discrete Taylor-Green mode u = A cos x sin y, v = -A sin x cos y on the MAC faces."""
    h = g.h
    xu = np.arange(g.NX + 1) * h
    yu = (np.arange(g.NY) + 0.5) * h
    xv = (np.arange(g.NX) + 0.5) * h
    yv = np.arange(g.NY + 1) * h
    u = A * np.cos(xu)[None, :] * np.sin(yu)[:, None]
    v = -A * np.sin(xv)[None, :] * np.cos(yv)[:, None]
    return u, v


def _ab2_amplitudes(z, K):
    """y^0 = 1, y^1 = 1 + z (cold start), y^{n+1} = (1 + 3z/2) y^n - (z/2) y^{n-1}."""
    y = [1.0, 1.0 + z]
    for _ in range(K - 1):
        y.append((1.0 + 1.5 * z) * y[-1] - 0.5 * z * y[-2])
    return np.array(y)


def _run(g, P, u, v, nu, dt, K, Fu=None, Fv=None, record=False):
    st = ns.State(u.copy(), v.copy())
    traj = []
    for _ in range(K):
        st, *_ = ns.step(g, P, st, nu, dt, Fu, Fv)
        if record:
            traj.append(ns.cell_velocity(g, st.u, st.v))
    return st, traj


def test_taylor_green_linear_ab2_recurrence():
    n, nu, dt, K, A = 16, 0.1, 0.01, 40, 1e-10
    g = Grid(n, "periodic")
    P = ns.Poisson(g)
    u0, v0 = _tg_fields(g, A)
    st, _ = _run(g, P, u0, v0, nu, dt, K)
    lam = -(8.0 / g.h ** 2) * np.sin(g.h / 2) ** 2
    yK = _ab2_amplitudes(dt * nu * lam, K)[K]
    assert np.abs(st.u - yK * u0).max() / A < 1e-9
    assert np.abs(st.v - yK * v0).max() / A < 1e-9
    # the recurrence differs from plain exponential decay by far more than the tolerance
    assert abs(yK - np.exp(dt * nu * lam * K)) > 1e-7


def test_taylor_green_nonlinear_decay_second_order():
    nu, T = 0.05, 1.0
    errs = []
    for n in (16, 32, 64):
        g = Grid(n, "periodic")
        P = ns.Poisson(g)
        dt = 0.1 * g.h
        K = int(round(T / dt))
        dt = T / K
        u0, v0 = _tg_fields(g, 1.0)
        st, _ = _run(g, P, u0, v0, nu, dt, K)
        mode = u0[:, : g.NX]
        amp = float(np.sum(st.u[:, : g.NX] * mode) / np.sum(mode * mode))
        errs.append(abs(amp - np.exp(-2.0 * nu * T)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs
    assert errs[2] < 1e-4


def test_forced_taylor_green_is_steady():
    """f_c = B (cos x_c sin y_c, -sin x_c cos y_c) with B = -nu lam A / cos(h/2) balances viscosity."""
    n, nu, dt, K, A = 16, 0.1, 0.01, 30, 1e-10
    g = Grid(n, "periodic")
    P = ns.Poisson(g)
    lam = -(8.0 / g.h ** 2) * np.sin(g.h / 2) ** 2
    B = -nu * lam * A / np.cos(g.h / 2)
    cells = control_cells(g, "box", (0.0, 2 * np.pi, 0.0, 2 * np.pi))
    assert len(cells) == n * n
    fx = np.array([B * np.cos(g.xc[i]) * np.sin(g.yc[j]) for j, i in cells])
    fy = np.array([-B * np.sin(g.xc[i]) * np.cos(g.yc[j]) for j, i in cells])
    Fu, Fv = ns.face_forcing(g, cells, np.concatenate([fx, fy]))
    u0, v0 = _tg_fields(g, A)
    st, _ = _run(g, P, u0, v0, nu, dt, K, Fu, Fv)
    assert np.abs(st.u - u0).max() / A < 1e-9
    assert np.abs(st.v - v0).max() / A < 1e-9
    # without the forcing the same field decays by a visible amount
    st0, _ = _run(g, P, u0, v0, nu, dt, K)
    assert np.abs(st0.u - u0).max() / A > 1e-2


def test_advection_conserves_energy_for_divergence_free_fields():
    rng = np.random.default_rng(7)
    g = Grid(16, "periodic")
    P = ns.Poisson(g)
    u = rng.standard_normal((g.NY, g.NX + 1))
    v = rng.standard_normal((g.NY + 1, g.NX))
    u[:, g.NX] = u[:, 0]
    v[g.NY, :] = v[0, :]
    u, v, _ = ns.project(g, P, u, v, 1.0)
    au, av, _ = ns.advection(g, u, v)
    core_u, core_v = (slice(None), slice(0, g.NX)), (slice(0, g.NY), slice(None))
    work = np.sum(u[core_u] * au[core_u]) + np.sum(v[core_v] * av[core_v])
    scale = np.sum(np.abs(u[core_u] * au[core_u])) + np.sum(np.abs(v[core_v] * av[core_v]))
    assert abs(work) < 1e-13 * scale
    # a field that is not divergence free exchanges energy with the advection term
    w = rng.standard_normal((g.NY, g.NX + 1))
    w[:, g.NX] = w[:, 0]
    au2, av2, _ = ns.advection(g, w, v)
    work2 = np.sum(w[core_u] * au2[core_u]) + np.sum(v[core_v] * av2[core_v])
    assert abs(work2) > 1e-3 * (np.sum(np.abs(w[core_u] * au2[core_u])))


@pytest.mark.parametrize("n", [8, 16])
def test_plane_poiseuille_discrete_profile(n):
    """Steady channel flow equals a (y(1-y) + h^2/4) with a = 4 (2 + h^2) / (2 + 4 h^2).

    Derivation: a quadratic has an exact second difference; at the wall rows the
    mirror ghost -u_0 turns (u_1 - 3 u_0)/h^2 into -3a/2 - 2c/h^2, which equals
    -2a for the shift c = a h^2 / 4; a then matches the inflow flux of the
    parabola under the midpoint rule (1/6 + h^2/12).
    """
    p = Problem(inv_h=n, Re=10.0, geometry="channel")
    g = p.grid()
    st = initial_state(p, np.zeros((g.NY, g.NX + 1)), np.zeros((g.NY + 1, g.NX)))
    st = spinup(p, st, int(30.0 / p.step_dt))
    h, y = g.h, g.yc
    a = 4.0 * (2.0 + h * h) / (2.0 + 4.0 * h * h)
    disc = a * (y * (1.0 - y) + h * h / 4.0)
    far = slice(int(3.0 * n), g.NX + 1)  # away from the inlet adjustment region
    assert np.abs(st.u[:, far] - disc[:, None]).max() < 1e-8
    assert np.abs(st.v[:, int(3.0 * n):]).max() < 1e-8
    # pressure gradient of the steady state: grad phi = -2 a nu on the far faces
    _, phi, _, _ = ns.step(g, p.poisson(), st, p.nu, p.step_dt)
    dpdx = (phi[:, int(3.2 * n)] - phi[:, int(3.2 * n) - 1]) / h
    assert np.allclose(dpdx, -2.0 * a * p.nu, rtol=1e-6)
    # the discrete profile is within O(h^2) of the continuous parabola 4y(1-y)
    assert np.abs(disc - 4 * y * (1 - y)).max() < h * h


def _cavity_state(n=16, steps=20, seed=3):
    from paper_2605_23812_amd import inputs

    p = Problem(inv_h=n, Re=1000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-2, seed=seed)
    st = spinup(p, initial_state(p, u0, v0), steps)
    return p, st


def test_divergence_free_after_projection():
    p, st = _cavity_state()
    g = p.grid()
    d = ns.divergence(g, st.u, st.v)
    assert np.abs(d).max() < 1e-12
    assert g.ncells == 5 * 16 * 16


def test_projection_idempotent_and_exact_on_gradients():
    p, st = _cavity_state()
    g, P = p.grid(), p.poisson()
    dt = p.step_dt
    # P(P u) = P u
    u2, v2, phi = ns.project(g, P, st.u, st.v, dt)
    assert np.abs(u2 - st.u).max() < 1e-12 and np.abs(v2 - st.v).max() < 1e-12
    # a discrete gradient added to a projected field is removed exactly: D G = L
    rng = np.random.default_rng(11)
    psi = np.where(g.fluid, rng.standard_normal((g.NY, g.NX)), 0.0)
    up, vp = ns.apply_gradient(g, st.u, st.v, -psi, dt)  # u + dt G psi
    assert np.abs(up - st.u).max() > 1e-3
    u3, v3, phi3 = ns.project(g, P, up, vp, dt)
    assert np.abs(u3 - st.u).max() < 1e-11 and np.abs(v3 - st.v).max() < 1e-11
    assert np.abs(phi3 - psi)[g.fluid].max() < 1e-9


def test_face_classes_of_the_cavity():
    g = Grid(8)
    # channel 32 x 8 cells over an 8 x 8 cavity starting at x = 1.25
    assert g.ncells == 32 * 8 + 8 * 8
    assert g.ucls[12, 0] == 3 and g.ucls[12, 32] == OUTFLOW
    assert g.ucls[4, 10] == 2 and g.ucls[4, 18] == 2 and g.ucls[4, 11] == ACTIVE
    assert g.vcls[8, 10] == ACTIVE and g.vcls[8, 9] == 2 and g.vcls[0, 10] == 2
    assert g.vcls[16, 0] == 2 and g.ucls[4, 5] == 0
    assert len(control_cells(g, "column")) == 2 * 8 * 8
    assert len(control_cells(g, "cavity")) == 8 * 8


def test_cost_welford_matches_stored_two_pass_and_taylor_green_closed_form():
    n, nu, dt, K, A = 16, 0.1, 0.01, 25, 1e-3
    g = Grid(n, "periodic")
    P = ns.Poisson(g)
    u0, v0 = _tg_fields(g, A)
    _, traj = _run(g, P, u0, v0, nu, dt, K, record=True)
    acc = cost.Welford((g.NY, g.NX))
    for uc, vc in traj:
        acc.add(uc, vc)
    tu = np.array([t[0] for t in traj])
    tv = np.array([t[1] for t in traj])
    j_w = acc.j_obs(g.fluid, dt, g.h)
    j_s = cost.j_obs_stored(tu, tv, g.fluid, dt, g.h)
    assert abs(j_w - j_s) < 1e-12 * j_s
    # closed form in the linear limit: sum_c |mode_c|^2 = A^2 cos^2(h/2) n^2 / 2
    lam = -(8.0 / g.h ** 2) * np.sin(g.h / 2) ** 2
    y = _ab2_amplitudes(dt * nu * lam, K)[1:]
    expect = dt * g.h ** 2 * A * A * np.cos(g.h / 2) ** 2 * n * n / 2.0 * np.sum((y - y.mean()) ** 2)
    assert abs(j_s - expect) < 1e-6 * expect


def test_cost_vanishes_on_a_steady_state():
    acc = cost.Welford((4, 4))
    f = np.ones((4, 4), dtype=bool)
    rng = np.random.default_rng(0)
    uc, vc = rng.standard_normal((4, 4)), rng.standard_normal((4, 4))
    for _ in range(7):
        acc.add(uc, vc)
    assert acc.j_obs(f, 0.1, 0.5) < 1e-28

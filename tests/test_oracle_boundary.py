"""Pins of the oracle's open-boundary rules against closed forms (CPU only).

The outlet and inlet rules are readings of Sec. 4.4's boundary conditions on
this grid (a convective outflow u_t + U_c u_x = 0 for the normal velocity, a
zero x-derivative of the tangential velocity beyond the outlet, v = 0 on the
inlet plane). Each test takes its expected value from mathematics:

  * Convective outflow. First-order upwinding of u_t + U_c u_x = 0 at the
    outflow face is exact along the characteristic at Courant number
    c = U_c dt / h = 1: the face takes the old value one face upstream. At
    c = 1/2 it takes the linear interpolant at the foot of the characteristic,
    the mean of the two. U_c is the inflow's bulk speed, fixed here by its
    exact integral: 2/3 for the parabola 4y(1-y) on [0, 1], 1 for the paper
    geometry's uniform inflow.
  * Inlet v. With the v ghost beyond x = 0 mirrored (-v, i.e. v = 0 on the
    inlet plane), a v that is linear in x and vanishes at x = 0 continues
    exactly across the inlet, so the centred x-difference and the 5-point
    Laplacian are exact there.
  * Outlet v. With the v ghost beyond x = L copied (dv/dx = 0), a v that is
    quadratic in (x - L) and symmetric about x = L continues exactly, so the
    same operators are exact in the last column.

The velocity operators enter through the tendency T_v = -A_v(u, v) +
nu lap_h v. With u held at a constant U, the x-part of A_v is linear in v and
its y-part quadratic, so the odd part (T_v(eps V) - T_v(-eps V)) / (2 eps)
equals -U d_x V + nu lap V exactly for these fields.
"""
import numpy as np
import pytest

from oracle import ns
from oracle.envar import Problem
from oracle.geometry import ACTIVE, OUTFLOW


def _rand_state(g, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((g.NY, g.NX + 1))
    v = rng.standard_normal((g.NY + 1, g.NX))
    return ns.impose_boundary_values(g, u, v)


# exact bulk speeds of the two inflows: mean over the channel height
_BULK = {
    "channel": 2.0 / 3.0,  # int_0^1 4 y (1 - y) dy
    "cavity": 2.0 / 3.0,
    "paper": 1.0,          # uniform u = 1
}


@pytest.mark.parametrize("geometry", ["channel", "cavity", "paper"])
@pytest.mark.parametrize("courant", [1.0, 0.5])
def test_convective_outflow_follows_the_characteristic(geometry, courant):
    n = 8
    p = Problem(inv_h=n, Re=100.0, geometry=geometry)
    g = p.grid()
    u, v = _rand_state(g, 5)
    dt = courant * g.h / _BULK[geometry]
    _, _, us, _ = ns.step(g, p.poisson(), ns.State(u, v), p.nu, dt)
    ob = g.ucls[:, -1] == OUTFLOW
    assert ob.sum() == (n if geometry != "paper" else n // 2)
    # foot of the characteristic through the outflow face: x_b - U_c dt = x_b - courant h
    expect = (1.0 - courant) * u[ob, -1] + courant * u[ob, -2]
    assert np.abs(us[ob, -1] - expect).max() < 1e-13 * np.abs(u).max()
    # the update really moved the face (a zero update would not pass by accident)
    assert np.abs(us[ob, -1] - u[ob, -1]).max() > 1e-2


def _odd_tendency_v(g, U, V, nu, eps=1e-3):
    u = np.full((g.NY, g.NX + 1), U)
    _, tp = ns.tendency(g, u, eps * V, nu)
    _, tm = ns.tendency(g, u, -eps * V, nu)
    return (tp - tm) / (2.0 * eps)


def _v_faces(g):
    xv = (np.arange(g.NX) + 0.5) * g.h
    yv = g.y0 + np.arange(g.NY + 1) * g.h
    return xv[None, :], yv[:, None]


def test_inlet_v_mirror_is_exact_for_a_field_vanishing_at_the_inlet():
    n, U, nu = 8, 0.7, 0.05
    p = Problem(inv_h=n, geometry="channel")
    g = p.grid()
    x, y = _v_faces(g)
    gy = y * (1.0 - y)                 # 0 on both walls, g'' = -2
    V = x * gy
    got = _odd_tendency_v(g, U, V, nu)
    expect = -U * gy * np.ones_like(x) + nu * x * (-2.0)
    act = g.vcls == ACTIVE
    cols = np.zeros_like(act)
    cols[:, : g.NX - 1] = True         # the last column belongs to the outlet rule
    mask = act & cols
    assert mask[:, 0].sum() == n - 1   # the inlet column is checked
    scale = np.abs(expect[mask]).max()
    assert np.abs(got[mask] - expect[mask]).max() < 1e-10 * scale


def test_outlet_v_copy_is_exact_for_a_field_symmetric_about_the_outlet():
    n, U, nu = 8, 0.7, 0.05
    p = Problem(inv_h=n, geometry="channel")
    g = p.grid()
    L = g.NX * g.h
    x, y = _v_faces(g)
    gy = y * (1.0 - y)
    V = (x - L) ** 2 * gy
    got = _odd_tendency_v(g, U, V, nu)
    # -U dV/dx + nu (d2V/dx2 + d2V/dy2) = -2 U (x - L) g + nu (2 g - 2 (x - L)^2)
    expect = -2.0 * U * (x - L) * gy + nu * (2.0 * gy - 2.0 * (x - L) ** 2)
    act = g.vcls == ACTIVE
    cols = np.zeros_like(act)
    cols[:, 1:] = True                 # the first column belongs to the inlet rule
    mask = act & cols
    assert mask[:, -1].sum() == n - 1  # the outlet column is checked
    scale = np.abs(expect[mask]).max()
    assert np.abs(got[mask] - expect[mask]).max() < 1e-10 * scale

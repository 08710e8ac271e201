"""Oracle Navier-Stokes step: forced incompressible NS on the MAC grid.

TEST INFRASTRUCTURE ONLY (see the package header).

Continuous model: eq. (forced_NS) of Sec. 2, u_t + (u.grad)u + grad p - Re^-1
lap u = f_u, div u = 0, with a steady forcing f_u(x). Its semi-discrete form
is eq. (discrete_NS), L dq/dt + N(q) = P f; here q = (u, v) on the staggered
faces, N is the conservative central advection plus the 5-point viscous term,
and P maps cell-centred forcing onto faces (``face_forcing``).

Time stepping (the paper's own scheme, implicit BDF2 with a fractional step
on a finite-element mesh, is replaced by an explicit scheme on a uniform grid):

  T^n   = -div_h(u u)^n + nu lap_h u^n                      (active faces)
  u*    = u^n + dt (3/2 T^n - 1/2 T^{n-1} + F)               (AB2; T^{-1} = T^0 on a cold start)
  u*_b  = u^n_b - dt U_c (u^n_b - u^n_{b-1}) / h             (outflow faces, U_c = the inflow's
                                                             bulk speed: 2/3 parabola, 1 uniform)
  L_h phi = div_h u* / dt                                    (sparse direct LU)
  u^{n+1} = u* - dt grad_h phi                               (active and outflow faces)

Neighbour rules at an active face: a stored face value (active, wall = 0,
inflow, outflow) is used as is; a SOLID face or one outside the box mirrors the
own value with a sign flip (no-slip wall half a cell away), or without one across
a slip wall (the paper geometry's symmetry top and outer lower wall, du/dy = 0);
the v value beyond
the outflow copies the own value (zero normal gradient of the tangential
velocity at the outlet, as the paper's outlet condition of Sec. 4.4).
Poisson: homogeneous Neumann on walls and inflow, phi = 0 on the outflow face
(mirror ghost -phi).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import ACTIVE, INFLOW, OUTFLOW, SOLID, WALL



# --------------------------------------------------------------------------- neighbours
def _neighbours_bounded(g, u, v):
    NY, NX = g.NY, g.NX
    nb = {}
    # u faces: x neighbours are faces of the two fluid cells -> stored values
    uW = np.zeros_like(u)
    uE = np.zeros_like(u)
    uW[:, 1:] = u[:, :-1]
    uE[:, :-1] = u[:, 1:]
    # y neighbours: mirror when the neighbour face is SOLID or outside the box, with the sign of
    # the wall (no-slip -u, slip +u)
    uS = g.mirror_S * u
    uN = g.mirror_N * u
    uS[1:, :] = np.where(g.ucls[:-1, :] == SOLID, g.mirror_S[1:, :] * u[1:, :], u[:-1, :])
    uN[:-1, :] = np.where(g.ucls[1:, :] == SOLID, g.mirror_N[:-1, :] * u[:-1, :], u[1:, :])
    # v at the four corners of a u face (i, j): v[j][i-1], v[j][i], v[j+1][i-1], v[j+1][i]
    vSW = np.zeros_like(u)
    vSE = np.zeros_like(u)
    vNW = np.zeros_like(u)
    vNE = np.zeros_like(u)
    vSW[:, 1:] = v[:-1, :]
    vSE[:, :-1] = v[:-1, :]
    vNW[:, 1:] = v[1:, :]
    vNE[:, :-1] = v[1:, :]
    nb.update(uW=uW, uE=uE, uS=uS, uN=uN, vSW=vSW, vSE=vSE, vNW=vNW, vNE=vNE)

    # v faces: y neighbours are faces of the two fluid cells -> stored values
    vS = np.zeros_like(v)
    vN = np.zeros_like(v)
    vS[1:, :] = v[:-1, :]
    vN[:-1, :] = v[1:, :]
    # x neighbours: mirror at SOLID faces and at the inflow side, copy beyond the outflow
    vW = -v.copy()
    vE = v.copy()
    vW[:, 1:] = np.where(g.vcls[:, :-1] == SOLID, -v[:, 1:], v[:, :-1])
    vE[:, :-1] = np.where(g.vcls[:, 1:] == SOLID, -v[:, :-1], v[:, 1:])
    # u at the four corners of a v face (i, j): u[j-1][i], u[j-1][i+1], u[j][i], u[j][i+1]
    uSW = np.zeros_like(v)
    uSE = np.zeros_like(v)
    uNW = np.zeros_like(v)
    uNE = np.zeros_like(v)
    uSW[1:, :] = u[:, :-1]
    uSE[1:, :] = u[:, 1:]
    uNW[:-1, :] = u[:, :-1]
    uNE[:-1, :] = u[:, 1:]
    nb.update(vW=vW, vE=vE, vS=vS, vN=vN, uSW=uSW, uSE=uSE, uNW=uNW, uNE=uNE)
    return nb


def _neighbours_periodic(g, u, v):
    NY, NX = g.NY, g.NX
    uc = u[:, :NX]
    vc = v[:NY, :]
    r = np.roll

    def pad_u(a):
        return np.concatenate([a, a[:, :1]], axis=1)

    def pad_v(a):
        return np.concatenate([a, a[:1, :]], axis=0)

    nb = dict(
        uW=r(uc, 1, 1), uE=r(uc, -1, 1), uS=r(uc, 1, 0), uN=r(uc, -1, 0),
        vSW=r(vc, 1, 1), vSE=vc, vNW=r(r(vc, -1, 0), 1, 1), vNE=r(vc, -1, 0),
    )
    nb = {k: pad_u(a) for k, a in nb.items()}
    nbv = dict(
        vW=r(vc, 1, 1), vE=r(vc, -1, 1), vS=r(vc, 1, 0), vN=r(vc, -1, 0),
        uSW=r(uc, 1, 0), uSE=r(r(uc, 1, 0), -1, 1), uNW=uc, uNE=r(uc, -1, 1),
    )
    nb.update({k: pad_v(a) for k, a in nbv.items()})
    return nb


def neighbours(g, u, v):
    return _neighbours_periodic(g, u, v) if g.periodic else _neighbours_bounded(g, u, v)


# --------------------------------------------------------------------------- operators
def advection(g, u, v):
    """Conservative central advection div_h(u u) at every face (Harlow-Welch form).

    On a u face:  [(u_e^2 - u_w^2) + (u_n v_n - u_s v_s)] / h with two-point
    averages to the cell centres (u_e, u_w) and to the cell corners (u_n, v_n,
    u_s, v_s); likewise on a v face. Only ACTIVE faces are meaningful.
    """
    h = g.h
    nb = neighbours(g, u, v)
    au = ((u + nb["uE"]) ** 2 - (nb["uW"] + u) ** 2) / (4.0 * h) + (
        (u + nb["uN"]) * (nb["vNW"] + nb["vNE"]) - (nb["uS"] + u) * (nb["vSW"] + nb["vSE"])
    ) / (4.0 * h)
    av = ((nb["uNE"] + nb["uSE"]) * (v + nb["vE"]) - (nb["uNW"] + nb["uSW"]) * (nb["vW"] + v)) / (
        4.0 * h
    ) + ((v + nb["vN"]) ** 2 - (nb["vS"] + v) ** 2) / (4.0 * h)
    return au, av, nb


def tendency(g, u, v, nu):
    """T = -div_h(u u) + nu lap_h u on ACTIVE faces, 0 elsewhere (eq. discrete_NS without P f)."""
    h = g.h
    au, av, nb = advection(g, u, v)
    du = (nb["uE"] + nb["uW"] + nb["uN"] + nb["uS"] - 4.0 * u) / (h * h)
    dv = (nb["vE"] + nb["vW"] + nb["vN"] + nb["vS"] - 4.0 * v) / (h * h)
    Tu = np.where(g.ucls == ACTIVE, -au + nu * du, 0.0)
    Tv = np.where(g.vcls == ACTIVE, -av + nu * dv, 0.0)
    return Tu, Tv


def divergence(g, u, v):
    """(div_h u)_c = (u_e - u_w + v_n - v_s) / h on fluid cells, 0 elsewhere."""
    d = (u[:, 1:] - u[:, :-1] + v[1:, :] - v[:-1, :]) / g.h
    return np.where(g.fluid, d, 0.0)


class Poisson:
    """Sparse direct solve of L_h phi = b on the fluid cells.

    L_h phi_c = sum over the four faces of the cell of
        (phi_nb - phi_c)/h^2   across an ACTIVE face,
        (-phi_c - phi_c)/h^2   across the OUTFLOW face (phi = 0 on it),
        0                      across WALL and INFLOW faces (Neumann).
    The periodic operator is singular; its constant null space is removed by
    replacing the first equation with phi_0 = 0 (the right-hand side of a
    projection is compatible, so the solution of the remaining equations is
    unchanged).
    """

    def __init__(self, g):
        self.g = g
        NY, NX, h = g.NY, g.NX, g.h
        idx = -np.ones((NY, NX), dtype=np.int64)
        cells = np.argwhere(g.fluid)
        idx[g.fluid] = np.arange(len(cells))
        self.idx = idx
        self.cells = cells
        rows, cols, vals = [], [], []
        for k, (j, i) in enumerate(cells):
            diag = 0.0
            faces = [
                (g.ucls[j, i], j, i - 1),  # west face of cell (i, j) is u face (i, j)
                (g.ucls[j, i + 1] if not g.periodic else ACTIVE, j, i + 1),
                (g.vcls[j, i], j - 1, i),
                (g.vcls[j + 1, i] if not g.periodic else ACTIVE, j + 1, i),
            ]
            if g.periodic:
                faces[0] = (ACTIVE, j, i - 1)
            for cls, jn, in_ in faces:
                if cls == ACTIVE:
                    if g.periodic:
                        jn, in_ = jn % NY, in_ % NX
                    rows.append(k)
                    cols.append(idx[jn, in_])
                    vals.append(1.0 / (h * h))
                    diag -= 1.0 / (h * h)
                elif cls == OUTFLOW:
                    diag -= 2.0 / (h * h)
            rows.append(k)
            cols.append(k)
            vals.append(diag)
        A = sp.csr_matrix((vals, (rows, cols)), shape=(len(cells), len(cells)))
        if g.periodic:
            A = A.tolil()
            A[0, :] = 0.0
            A[0, 0] = 1.0
            A = A.tocsr()
        self.A = A
        self.lu = spla.splu(A.tocsc())

    def apply(self, phi):
        """L_h phi on the fluid cells, as a (NY, NX) array."""
        out = np.zeros_like(phi)
        out[self.g.fluid] = self.A @ phi[self.g.fluid]
        return out

    def solve(self, b):
        rhs = b[self.g.fluid].copy()
        if self.g.periodic:
            rhs[0] = 0.0
        phi = np.zeros((self.g.NY, self.g.NX))
        phi[self.g.fluid] = self.lu.solve(rhs)
        return phi


def project(g, poisson, us, vs, dt):
    """Return (u, v, phi) with u = u* - dt grad_h phi, L_h phi = div_h u* / dt."""
    b = divergence(g, us, vs) / dt
    phi = poisson.solve(b)
    return (*apply_gradient(g, us, vs, phi, dt), phi)


def apply_gradient(g, us, vs, phi, dt):
    """u = u* - dt grad_h phi on ACTIVE and OUTFLOW faces (the last with ghost -phi)."""
    h = g.h
    u = us.copy()
    v = vs.copy()
    if g.periodic:
        NX, NY = g.NX, g.NY
        gx = (phi - np.roll(phi, 1, axis=1)) / h
        gy = (phi - np.roll(phi, 1, axis=0)) / h
        u[:, :NX] -= dt * gx
        u[:, NX] = u[:, 0]
        v[:NY, :] -= dt * gy
        v[NY, :] = v[0, :]
        return u, v
    gx = np.zeros_like(u)
    gx[:, 1:-1] = (phi[:, 1:] - phi[:, :-1]) / h
    gx[:, -1] = (-phi[:, -1] - phi[:, -1]) / h
    gy = np.zeros_like(v)
    gy[1:-1, :] = (phi[1:, :] - phi[:-1, :]) / h
    mu = (g.ucls == ACTIVE) | (g.ucls == OUTFLOW)
    mv = g.vcls == ACTIVE
    u[mu] -= dt * gx[mu]
    v[mv] -= dt * gy[mv]
    return u, v


# --------------------------------------------------------------------------- forcing (operator P)
def face_forcing(g, cells, f):
    """Operator P of eq. (discrete_NS): cell-centred forcing -> face forcing.

    f = [f_x over ``cells`` (row-major), then f_y over the same cells]. Each
    ACTIVE face takes the mean of its two adjacent cells' values, a cell
    outside the control region contributing 0. Non-active faces carry none.
    """
    n = len(cells)
    fx = np.zeros((g.NY, g.NX))
    fy = np.zeros((g.NY, g.NX))
    for k, (j, i) in enumerate(cells):
        fx[j, i] = f[k]
        fy[j, i] = f[n + k]
    Fu = np.zeros((g.NY, g.NX + 1))
    Fv = np.zeros((g.NY + 1, g.NX))
    if g.periodic:
        Fu[:, :g.NX] = 0.5 * (fx + np.roll(fx, 1, axis=1))
        Fv[:g.NY, :] = 0.5 * (fy + np.roll(fy, 1, axis=0))
    else:
        Fu[:, 1:-1] = 0.5 * (fx[:, :-1] + fx[:, 1:])
        Fv[1:-1, :] = 0.5 * (fy[:-1, :] + fy[1:, :])
    Fu = np.where(g.ucls == ACTIVE, Fu, 0.0)
    Fv = np.where(g.vcls == ACTIVE, Fv, 0.0)
    return Fu, Fv


# --------------------------------------------------------------------------- state and step
class State:
    """(u^n, v^n) and the previous tendency (T_u^{n-1}, T_v^{n-1}); ``cold`` = no history yet."""

    def __init__(self, u, v, Tu_prev=None, Tv_prev=None):
        self.u, self.v = u, v
        self.Tu_prev, self.Tv_prev = Tu_prev, Tv_prev

    @property
    def cold(self):
        return self.Tu_prev is None

    def copy(self):
        c = lambda a: None if a is None else a.copy()
        return State(self.u.copy(), self.v.copy(), c(self.Tu_prev), c(self.Tv_prev))


def impose_boundary_values(g, u, v, inflow=None):
    """Set the fixed face values: walls and solid faces 0, inflow faces the parabola."""
    u = np.where((g.ucls == ACTIVE) | (g.ucls == OUTFLOW), u, 0.0)
    v = np.where(g.vcls == ACTIVE, v, 0.0)
    if not g.periodic:
        prof = g.inflow_profile() if inflow is None else inflow
        u[:, 0] = np.where(g.ucls[:, 0] == INFLOW, prof, 0.0)
    else:
        u[:, g.NX] = u[:, 0]
        v[g.NY, :] = v[0, :]
    return u, v


def step(g, poisson, st, nu, dt, Fu=None, Fv=None):
    """One AB2 + projection step; returns (new State, phi, u*, v*)."""
    u, v = st.u, st.v
    Tu, Tv = tendency(g, u, v, nu)
    Tu_prev, Tv_prev = (Tu, Tv) if st.cold else (st.Tu_prev, st.Tv_prev)
    if Fu is None:
        Fu = np.zeros_like(u)
        Fv = np.zeros_like(v)
    us = u.copy()
    vs = v.copy()
    au = g.ucls == ACTIVE
    av = g.vcls == ACTIVE
    us[au] = u[au] + dt * (1.5 * Tu[au] - 0.5 * Tu_prev[au] + Fu[au])
    vs[av] = v[av] + dt * (1.5 * Tv[av] - 0.5 * Tv_prev[av] + Fv[av])
    if g.periodic:
        us[:, g.NX] = us[:, 0]
        vs[g.NY, :] = vs[0, :]
    else:
        ob = g.ucls[:, -1] == OUTFLOW
        us[ob, -1] = u[ob, -1] - dt * g.u_convective * (u[ob, -1] - u[ob, -2]) / g.h
    un, vn, phi = project(g, poisson, us, vs, dt)
    return State(un, vn, Tu, Tv), phi, us, vs


def cell_velocity(g, u, v):
    """Cell-centred velocity (u_c, v_c) = face means, on fluid cells (0 elsewhere)."""
    uc = 0.5 * (u[:, :-1] + u[:, 1:])
    vc = 0.5 * (v[:-1, :] + v[1:, :])
    return np.where(g.fluid, uc, 0.0), np.where(g.fluid, vc, 0.0)

"""Oracle EnVar forward ensemble, anomaly gradient and descent loop.

TEST INFRASTRUCTURE ONLY (see the package header).

* ``forward``  : the N+1 independent forward evaluations of Sec. 3.3.1 (the
                 centre run plus one run per perturbed forcing, eq. fdapprox),
                 each integrating the forced NS equations from a common base
                 state over the horizon and returning its scalar cost J_i.
* ``gradient`` : the reduction {delta f_i, J_i} -> g. With X_i = f_i - f_0
                 and dJ_i = J_i - J_0, g = X^+ dJ (minimum-norm least
                 squares). For perturbations X = eps E^T this is the scalar-J
                 form of eq. (gradient_EnVar): dJ/eps is the finite difference
                 of eq. (fdapprox) applied to J, i.e. dJ/dw, and
                 g = E (E^T E)^{-1} dJ/dw is grad J projected on span(E).
* ``iterate``  : f <- f - alpha g with Armijo backtracking (the line search of
                 eq. update_BFGS), the perturbation set held fixed across
                 iterations as in Sec. 3.3.3.
"""
import os
from dataclasses import dataclass, field
from multiprocessing import get_context

import numpy as np

from . import cost, ns
from .geometry import Grid, control_cells


@dataclass
class Problem:
    inv_h: int = 32
    Re: float = 4000.0
    dt: float = 0.0          # 0 -> 0.064 h
    x_cav: float = 1.25
    geometry: str = "cavity"
    region: str = "column"
    box: tuple = (0.0, 0.0, 0.0, 0.0)
    penalty: float = 1e-3
    length: float = 4.0
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    @property
    def nu(self):
        return 1.0 / self.Re

    @property
    def step_dt(self):
        return self.dt if self.dt > 0 else 0.064 / self.inv_h

    def grid(self):
        if "grid" not in self._cache:
            self._cache["grid"] = Grid(self.inv_h, self.geometry, self.x_cav, self.length)
        return self._cache["grid"]

    def poisson(self):
        if "poisson" not in self._cache:
            self._cache["poisson"] = ns.Poisson(self.grid())
        return self._cache["poisson"]

    def cells(self):
        if "cells" not in self._cache:
            self._cache["cells"] = control_cells(self.grid(), self.region, self.box)
        return self._cache["cells"]

    @property
    def m(self):
        return 2 * len(self.cells())


def initial_state(p, u0, v0):
    """Cold-start state from raw face fields: boundary values imposed, no AB2 history."""
    g = p.grid()
    u, v = ns.impose_boundary_values(g, np.array(u0, dtype=np.float64), np.array(v0, dtype=np.float64))
    return ns.State(u, v)


def spinup(p, state, steps):
    """Advance ``state`` by ``steps`` unforced steps (base-state generation)."""
    g, P = p.grid(), p.poisson()
    st = state.copy()
    for _ in range(steps):
        st, *_ = ns.step(g, P, st, p.nu, p.step_dt)
    return st


def forward_member(p, base, f, horizon, return_state=False):
    """Integrate one member with control row ``f`` for ``horizon`` steps; return J (and the final state)."""
    g, P = p.grid(), p.poisson()
    Fu, Fv = ns.face_forcing(g, p.cells(), np.asarray(f, dtype=np.float64))
    st = base.copy()
    acc = cost.Welford((g.NY, g.NX))
    for _ in range(horizon):
        st, *_ = ns.step(g, P, st, p.nu, p.step_dt, Fu, Fv)
        acc.add(*ns.cell_velocity(g, st.u, st.v))
    J = acc.j_obs(g.fluid, p.step_dt, g.h) + cost.penalty(np.asarray(f), g.h, p.penalty)
    return (J, st) if return_state else J


_SHARED = {}


def _member_job(i):
    p, base, controls, horizon = _SHARED["job"]
    return forward_member(p, base, controls[i], horizon)


def forward(p, base, controls, horizon, processes=1):
    """J_i for every control row (one independent run per row, Sec. 5.3's ensemble parallelism).

    With processes > 1 the rows run in forked worker processes that inherit
    the problem (and its one sparse LU factorisation) from the parent.
    """
    controls = np.asarray(controls, dtype=np.float64)
    n = controls.shape[0]
    if processes <= 1:
        return np.array([forward_member(p, base, controls[i], horizon) for i in range(n)])
    p.poisson()
    _SHARED["job"] = (p, base, controls, horizon)
    try:
        with get_context("fork").Pool(processes) as pool:
            return np.array(pool.map(_member_job, range(n), chunksize=1))
    finally:
        _SHARED.clear()


def gradient(controls, J, rcond=1e-12):
    """g = X^+ dJ with X_i = f_i - f_0, dJ_i = J_i - J_0 (row 0 is the centre run)."""
    controls = np.asarray(controls, dtype=np.float64)
    J = np.asarray(J, dtype=np.float64)
    X = controls[1:] - controls[0]
    dJ = J[1:] - J[0]
    g, *_ = np.linalg.lstsq(X, dJ, rcond=rcond)
    return g


def iterate(p, base, f, perturb, horizon, iters=1, alpha0=None, c1=1e-4, shrink=0.5,
            max_trials=8, fixed_alpha_after_first=True, processes=1):
    """Fixed-ensemble descent: N+1 forwards, gradient, Armijo step along -g.

    Returns a list of per-iteration records (J0, |g|, alpha, J_new). The first
    iteration's accepted step is reused afterwards when
    ``fixed_alpha_after_first`` (so every later iteration costs exactly N+1
    forward evaluations).
    """
    f = np.asarray(f, dtype=np.float64).copy()
    perturb = np.asarray(perturb, dtype=np.float64)
    hist = []
    alpha_fixed = None
    for it in range(iters):
        rows = np.vstack([f[None, :], f[None, :] + perturb])
        J = forward(p, base, rows, horizon, processes)
        g = gradient(rows, J)
        if alpha_fixed is not None:
            alpha = alpha_fixed
            f = f - alpha * g
            hist.append(dict(J0=J[0], gnorm=float(np.linalg.norm(g)), alpha=alpha, J_new=None, f=f.copy()))
            continue
        a = alpha0 if alpha0 is not None else float(np.abs(perturb).max()) / max(float(np.abs(g).max()), 1e-300)
        gg = float(g @ g)
        accepted = None
        for _ in range(max_trials):
            Jt = forward_member(p, base, f - a * g, horizon)
            if Jt <= J[0] - c1 * a * gg:
                accepted = (a, Jt)
                break
            a *= shrink
        if accepted is None:
            hist.append(dict(J0=J[0], gnorm=float(np.sqrt(gg)), alpha=0.0, J_new=J[0], f=f.copy()))
            break
        a, Jt = accepted
        f = f - a * g
        if fixed_alpha_after_first:
            alpha_fixed = a
        hist.append(dict(J0=J[0], gnorm=float(np.sqrt(gg)), alpha=a, J_new=Jt, f=f.copy()))
    return hist

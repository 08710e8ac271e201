"""Oracle cost J(f) = observation term + control penalty.

TEST INFRASTRUCTURE ONLY (see the package header).

eq. (Envarcost) splits J into a data-misfit term and a prior term. The
observation here is the velocity fluctuation u' = u - u_bar about the
per-run time mean (Sec. 4.1), taken over the whole fluid domain as in the
global fluctuation energy E_k of eq. (kinenergy):

    J_obs = dt h^2 sum_{n=1..K} sum_c |u_c^n - ubar_c|^2,
    ubar_c = (1/K) sum_{n=1..K} u_c^n,

a rectangle rule in time over the K post-step samples and the cell-area
quadrature in space (no factor 1/2, no sensor restriction). The prior term is
the plain penalty lambda h^2 sum_k f_k^2 (B = I / (2 lambda) scaled by the
cell area M_f = h^2 I), lambda = 1e-3.

The fluctuation energy is accumulated two-pass-equivalently with Welford's
per-cell running mean and sum of squared deviations, which shares no algebra
with the shifted running sums a streaming implementation would use;
``j_obs_stored`` is the literal two-pass sum over a stored trajectory.
"""
import numpy as np


class Welford:
    """Per-cell running mean and M2 = sum of squared deviations (Welford 1962)."""

    def __init__(self, shape):
        self.k = 0
        self.mean_u = np.zeros(shape)
        self.mean_v = np.zeros(shape)
        self.m2 = np.zeros(shape)

    def add(self, uc, vc):
        self.k += 1
        du = uc - self.mean_u
        dv = vc - self.mean_v
        self.mean_u += du / self.k
        self.mean_v += dv / self.k
        self.m2 += du * (uc - self.mean_u) + dv * (vc - self.mean_v)

    def j_obs(self, fluid, dt, h):
        return dt * h * h * float(np.sum(self.m2[fluid]))


def j_obs_stored(traj_u, traj_v, fluid, dt, h):
    """Literal two-pass form on a stored trajectory (K, NY, NX) of cell velocities."""
    mu = traj_u.mean(axis=0)
    mv = traj_v.mean(axis=0)
    s = ((traj_u - mu) ** 2 + (traj_v - mv) ** 2)[:, fluid]
    return dt * h * h * float(s.sum())


def penalty(f, h, lam):
    return lam * h * h * float(np.dot(f, f))

"""Pressure passes beyond a step's cap in the per-member tail launch (needs an MI355X).

A step launches its first pressure passes level by level (as many as the members needed lately)
and the passes beyond, up to max_cycles, in one launch with a workgroup per member that goes
through the same per-tile arithmetic. Three schedules must therefore give bitwise the same costs,
final fields and pass counts: the default, one level-by-level pass per step with every later pass
in the tail (FLAG_SHORT_GRAPH, which makes the tail do most of the work), and one level-by-level
headroom pass instead of the tail (FLAG_NO_TAIL). Covered: every tiled depth the tail takes
(inv_h 32 to 256), the three geometries, FP64 V-cycles and mixed-precision refinement passes, with
graph replay and eager launches; the tail-heavy schedule also against the oracle (Sec. 3.3.1: each
member's J is its own forward's).
"""
import dataclasses

import numpy as np
import pytest

from oracle import envar as OE
from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_GEO = {"cavity": E.CAVITY, "paper": E.CAVITY_PAPER, "channel": E.CHANNEL}


def _setup(n, geometry, precision, N, seed, div_tol=0.0):
    geo = _GEO[geometry]
    p = E.Problem(inv_h=n, Re=7500.0, precision=precision, geometry=geo, div_tol=div_tol)
    p64 = E.Problem(inv_h=n, Re=7500.0, geometry=geo)
    u0, v0 = inputs.initial_field(n, amp=1e-3, seed=seed, geometry=geometry)
    state = E.state_init(p64, u0, v0)
    E.spinup(p64, state, 20)
    m = E.control_dim(p)
    ny = {"cavity": 2 * n, "paper": n + n // 2, "channel": n}[geometry]
    shape = None if geometry == "cavity" else (ny, n)
    rows = np.vstack([np.zeros(m), inputs.grf_perturbations(N - 1, n, 0.05, 2e-2, seed=seed, shape=shape)])
    assert rows.shape[1] == m
    return p, state, torch.tensor(rows, dtype=torch.float64, device="cuda")


def _run(p, state, ctrl, horizon, flags):
    q = dataclasses.replace(p, flags=p.flags | flags)
    J, F, st = E.forward(q, state, ctrl, horizon, fields=True)
    torch.cuda.synchronize()
    return J.cpu().numpy(), F.cpu().numpy(), st


# (inv_h, geometry, precision, members, horizon): horizons above 16 steps, so that the steady steps
# replay their captured graphs (steps with at least 16 left)
_CASES = [
    (32, "cavity", E.MIXED, 4, 40),
    (32, "channel", E.FP64, 3, 30),
    (64, "paper", E.MIXED, 3, 30),
    (64, "cavity", E.FP64, 3, 24),
    (128, "cavity", E.MIXED, 3, 24),
    (256, "cavity", E.FP64, 2, 20),
]


@pytest.mark.parametrize("n,geometry,precision,N,horizon", _CASES)
@pytest.mark.parametrize("graphs", [True, False])
def test_tail_schedules_agree_bitwise(n, geometry, precision, N, horizon, graphs):
    if not graphs and n > 64:
        pytest.skip("eager launches are covered at the smaller grids")
    p, state, ctrl = _setup(n, geometry, precision, N, seed=n + 7)
    base = 0 if graphs else E.FLAG_NO_GRAPHS
    print("tail schedules:", n, geometry, "precision", precision, "members", N, "horizon", horizon,
          "graphs", graphs, flush=True)
    ref = _run(p, state, ctrl, horizon, base | E.FLAG_NO_TAIL)
    for flags in (0, E.FLAG_SHORT_GRAPH):
        J, F, st = _run(p, state, ctrl, horizon, base | flags)
        print("  flags", flags, "mean cycles", st["mean_cycles"], "max", st["max_cycles_used"],
              "unconverged", st["unconverged"], flush=True)
        assert np.array_equal(J, ref[0])
        assert np.array_equal(F, ref[1])
        for key in ("mean_cycles", "max_cycles_used", "unconverged", "max_resid", "max_div"):
            assert st[key] == ref[2][key], key
    # the short schedule leaves every pass after the first to the tail: it has to have run some
    assert ref[2]["max_cycles_used"] >= 2
    assert ref[2]["unconverged"] == 0


def test_tail_heavy_forward_matches_oracle():
    """FP64 and mixed forwards whose second and later passes all run in the tail launch, against
    the oracle's own member forwards (FP64 within 1e-10, mixed within 1e-4 on J)."""
    n, N, horizon = 32, 4, 30
    op = OE.Problem(inv_h=n, Re=4000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3, seed=11)
    base = OE.spinup(op, OE.initial_state(op, u0, v0), 20)
    rows = np.vstack([np.zeros(op.m), inputs.grf_perturbations(N - 1, n, 0.1, 1e-2, seed=11)])
    ctrl = torch.tensor(rows, device="cuda")
    Jr = np.array([OE.forward_member(op, base, r, horizon) for r in rows])
    for precision, tol in ((E.FP64, 1e-10), (E.MIXED, 1e-4)):
        p = E.Problem(inv_h=n, Re=4000.0, precision=precision, flags=E.FLAG_SHORT_GRAPH)
        state = E.state_init(E.Problem(inv_h=n, Re=4000.0), base.u, base.v, base.Tu_prev, base.Tv_prev)
        J, _, st = E.forward(p, state, ctrl, horizon)
        torch.cuda.synchronize()
        rel = np.abs(J.cpu().numpy() - Jr) / np.abs(Jr)
        print("tail-heavy vs oracle: precision", precision, "J rel", rel, "mean cycles", st["mean_cycles"],
              flush=True)
        assert rel.max() <= tol
        assert st["unconverged"] == 0 and st["max_cycles_used"] >= 2


def test_tail_stops_on_a_non_finite_member():
    """A member whose forcing holds a NaN has a NaN residual from its first solve on. The tail stops
    on it (no pass can change that) instead of running every pass up to max_cycles, and the three
    schedules still agree: the other members' costs bit for bit, the NaN member's cost not finite,
    each of its steps counted as not converged."""
    p, state, ctrl = _setup(64, "cavity", E.MIXED, 4, seed=5)
    bad = ctrl.clone()
    bad[2, 100] = float("nan")
    keep = [0, 1, 3]
    ref = None
    for flags in (E.FLAG_NO_TAIL, 0, E.FLAG_SHORT_GRAPH):
        q = dataclasses.replace(p, flags=flags)
        J, _, st = E.forward(q, state, bad, 30)
        torch.cuda.synchronize()
        J = J.cpu().numpy()
        print("non-finite member: flags", flags, "J", J, "unconverged", st["unconverged"], "diverged",
              st["diverged"], flush=True)
        assert np.isnan(J[2]) and np.all(np.isfinite(J[keep]))
        assert st["diverged"] == 1 and st["unconverged"] == 30
        if ref is None:
            ref = J
        assert np.array_equal(J[keep], ref[keep])

"""Uneven batching: several ensembles of different grids, Reynolds numbers, sizes and
horizons advance together in merged launches (needs an MI355X).

Each ensemble's costs and final fields must match the oracle's own forwards
(FP64 within 1e-10, mixed precision within 1e-4 on J), and equal those of its
own envar_forward call bitwise (per-member convergence, fixed-order
reductions), in FP64 and in mixed precision, also when the jobs mix the
simplified and the paper's cavity geometry.
"""
import numpy as np
import pytest

from oracle import envar as OE
from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _job(n, Re, N, horizon, precision, seed, paper=False):
    geo = dict(geometry=E.CAVITY_PAPER) if paper else {}
    p = E.Problem(inv_h=n, Re=Re, precision=precision, **geo)
    p64 = E.Problem(inv_h=n, Re=Re, **geo)
    u0, v0 = inputs.initial_field(n, amp=1e-3, seed=seed, geometry="paper" if paper else "cavity")
    state = E.state_init(p64, u0, v0)
    E.spinup(p64, state, 30)
    m = E.control_dim(p)
    shape = (n + n // 2, n) if paper else None  # the column region spans the channel's height
    rows = np.vstack([np.zeros(m), inputs.grf_perturbations(N - 1, n, 0.05, 5e-3, seed=seed, shape=shape)])
    return p, state, torch.tensor(rows, dtype=torch.float64, device="cuda"), horizon


# (inv_h, Re, rows, horizon, seed): horizons of 33 steps and more, so that the batch replays its
# captured step graphs (they run while every job has at least 16 steps left: steps 1 to 17 here)
_ORACLE_JOBS = [(16, 4000.0, 3, 41, 1), (32, 7500.0, 4, 33, 2), (32, 4000.0, 3, 37, 3)]


@pytest.mark.parametrize("precision,tol", [(E.FP64, 1e-10), (E.MIXED, 1e-4)])
def test_uneven_batch_matches_oracle(precision, tol):
    jobs, refs = [], []
    for n, Re, N, horizon, seed in _ORACLE_JOBS:
        op = OE.Problem(inv_h=n, Re=Re)
        u0, v0 = inputs.initial_field(n, amp=1e-3, seed=seed)
        base = OE.spinup(op, OE.initial_state(op, u0, v0), 20)
        rows = np.vstack([np.zeros(op.m), inputs.grf_perturbations(N - 1, n, 0.1, 1e-2, seed=seed)])
        state = E.state_init(E.Problem(inv_h=n, Re=Re), base.u, base.v, base.Tu_prev, base.Tv_prev)
        p = E.Problem(inv_h=n, Re=Re, precision=precision)
        jobs.append((p, state, torch.tensor(rows, device="cuda"), horizon))
        refs.append([OE.forward_member(op, base, r, horizon, return_state=True) for r in rows])
    print("batch vs oracle: precision", precision, "jobs", _ORACLE_JOBS, flush=True)
    out = E.forward_batch(jobs, fields=True)
    torch.cuda.synchronize()
    for (p, _, _, horizon), (J, st, F), ref in zip(jobs, out, refs):
        Jg = J.cpu().numpy()
        u, v = E.split_fields(p, F)
        for i, (Jr, sr) in enumerate(ref):
            rel = abs(Jg[i] - Jr) / abs(Jr)
            scale = np.abs(sr.u).max()
            du = max(np.abs(u[i] - sr.u).max(), np.abs(v[i] - sr.v).max()) / scale
            print(" job", p.inv_h, horizon, "member", i, "J rel", rel, "field rel", du, flush=True)
            assert rel <= tol
            assert du <= (1e-10 if precision == E.FP64 else 1e-5)
        assert st["unconverged"] == 0 and st["steps"] == horizon


@pytest.mark.parametrize("precision", [E.FP64, E.MIXED])
def test_uneven_batch_equals_separate_forwards(precision):
    jobs = [
        _job(64, 4000.0, 5, 37, precision, 1),
        _job(32, 7500.0, 9, 60, precision, 2),
        _job(16, 12000.0, 3, 23, precision, 3),
        _job(128, 7500.0, 2, 20, precision, 4),
    ]
    out = E.forward_batch(jobs)
    torch.cuda.synchronize()
    for (p, state, ctrl, horizon), (Jb, st) in zip(jobs, out):
        Js, _, sts = E.forward(p, state, ctrl, horizon)
        torch.cuda.synchronize()
        a, b = Jb.cpu().numpy(), Js.cpu().numpy()
        print("batch", p.inv_h, horizon, a, b, st["mean_cycles"], sts["mean_cycles"], flush=True)
        assert np.array_equal(a, b)
        assert st["unconverged"] == 0 and st["steps"] == horizon


@pytest.mark.parametrize("precision", [E.FP64, E.MIXED])
def test_batch_mixing_the_two_cavity_geometries(precision):
    """Jobs of the simplified and of the paper's geometry (different heights, wall kinds, inflow and
    outflow speed) share the merged launches and still equal their own forwards bitwise."""
    jobs = [
        _job(64, 6250.0, 4, 30, precision, 5, paper=True),
        _job(64, 7500.0, 3, 25, precision, 6),
        _job(32, 14000.0, 5, 41, precision, 7, paper=True),
    ]
    out = E.forward_batch(jobs)
    torch.cuda.synchronize()
    for (p, state, ctrl, horizon), (Jb, st) in zip(jobs, out):
        Js, _, _ = E.forward(p, state, ctrl, horizon)
        torch.cuda.synchronize()
        a, b = Jb.cpu().numpy(), Js.cpu().numpy()
        print("geometry", p.geometry, p.inv_h, a, b, flush=True)
        assert np.array_equal(a, b)
        assert st["unconverged"] == 0 and st["steps"] == horizon


@pytest.mark.parametrize("precision", [E.FP64, E.MIXED])
def test_batch_with_different_pass_caps(precision):
    """A job with a small max_cycles next to one with the default: each runs at most its own number
    of passes (its norm slots are sized by it); a job that converges at every step, alone and in
    the batch, equals its own forward bitwise."""
    a = _job(32, 4000.0, 3, 40, precision, 8)
    b = _job(32, 7500.0, 4, 40, precision, 9)
    a = (E.Problem(inv_h=32, Re=4000.0, precision=precision, max_cycles=12), *a[1:])
    out = E.forward_batch([a, b])
    torch.cuda.synchronize()
    for (p, state, ctrl, horizon), (Jb, st) in zip([a, b], out):
        Js, _, sts = E.forward(p, state, ctrl, horizon)
        torch.cuda.synchronize()
        print("caps", p.max_cycles, st["max_cycles_used"], st["unconverged"], sts["unconverged"], flush=True)
        assert st["max_cycles_used"] <= (p.max_cycles or 30)
        assert np.all(np.isfinite(Jb.cpu().numpy()))
        if st["unconverged"] == 0 and sts["unconverged"] == 0:
            assert np.array_equal(Jb.cpu().numpy(), Js.cpu().numpy())
    assert out[1][1]["unconverged"] == 0  # the default cap always suffices here


def test_batch_rejects_mixed_precisions_and_too_many_jobs():
    a = _job(32, 4000.0, 2, 5, E.FP64, 1)
    b = _job(32, 4000.0, 2, 5, E.MIXED, 2)
    with pytest.raises(E.EnvarError) as ei:
        E.forward_batch([a, b])
    assert ei.value.code == E.EINVAL
    with pytest.raises(E.EnvarError):
        E.forward_batch([a] * 9)

"""Parity at the workload sizes (needs an MI355X).

* The h = 1/32 workload in full: 500-step spin-up from the seeded perturbed
  channel flow, centre + 8 GRF members (length 0.1, std 1e-2), 200 steps, Re =
  4000: in FP64 every J within 1e-10 of the oracle and the gradient within
  1e-8; in mixed precision (FP32 multigrid inside FP64 refinement, FP32-MFMA
  Gram) every J within 1e-4 and the gradient's cosine with the oracle's at
  least 0.999.
* The h = 1/128 launch configuration of the benchmark (65 members, m = 65,536)
  over 48 steps, with the step graphs replaying and with eager launches:
  sampled members against the oracle one by one (FP64: 1e-10; mixed: 1e-4),
  the rest checked by properties (finite, converged).
* envar_iterate against the oracle's fixed-ensemble Armijo descent.
"""
import numpy as np
import pytest

from oracle import envar as OE
from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


_H32 = {}


def _h32_workload():
    """The h = 1/32 workload and the oracle's costs and gradient on it (computed once)."""
    if not _H32:
        n = 32
        op = OE.Problem(inv_h=n, Re=4000.0)
        u0, v0 = inputs.initial_field(n, amp=1e-3)
        base = OE.spinup(op, OE.initial_state(op, u0, v0), 500)
        rows = np.vstack([np.zeros(op.m), inputs.grf_perturbations(8, n, 0.1, 1e-2)])
        Jr = OE.forward(op, base, rows, 200, processes=9)
        _H32.update(base=base, rows=rows, Jr=Jr, gr=OE.gradient(rows, Jr))
    return _H32


def test_h32_workload_costs_and_gradient_match_oracle():
    n = 32
    p = E.Problem(inv_h=n, Re=4000.0)
    w = _h32_workload()
    base, rows, Jr, gr = w["base"], w["rows"], w["Jr"], w["gr"]
    state = E.state_init(p, base.u, base.v, base.Tu_prev, base.Tv_prev)
    ctrl = torch.tensor(rows, device="cuda")
    J, _, st = E.forward(p, state, ctrl, 200)
    g = E.gradient(ctrl, J, E.FP64)
    torch.cuda.synchronize()
    Jg, gg = J.cpu().numpy(), g.cpu().numpy()
    rel = np.abs(Jg - Jr) / np.abs(Jr)
    gerr = np.abs(gg - gr).max() / np.abs(gr).max()
    _say("h32 workload: J rel", rel.max(), "g rel", gerr, "stats", st)
    assert rel.max() <= 1e-10 and gerr <= 1e-8
    assert st["unconverged"] == 0 and st["max_div"] <= 1e-11


def test_h32_workload_mixed_precision_against_oracle():
    n = 32
    w = _h32_workload()
    base, rows, Jr, gr = w["base"], w["rows"], w["Jr"], w["gr"]
    state = E.state_init(E.Problem(inv_h=n, Re=4000.0), base.u, base.v, base.Tu_prev, base.Tv_prev)
    p = E.Problem(inv_h=n, Re=4000.0, precision=E.MIXED)
    ctrl = torch.tensor(rows, device="cuda")
    J, _, st = E.forward(p, state, ctrl, 200)
    g = E.gradient(ctrl, J, E.MIXED)
    torch.cuda.synchronize()
    Jg, gg = J.cpu().numpy(), g.cpu().numpy()
    rel = np.abs(Jg - Jr) / np.abs(Jr)
    cos = float(gg @ gr / (np.linalg.norm(gg) * np.linalg.norm(gr)))
    gerr = np.linalg.norm(gg - gr) / np.linalg.norm(gr)
    _say("h32 workload, mixed: J rel", rel.max(), "g cosine", cos, "g rel (2-norm)", gerr, "stats", st)
    assert rel.max() <= 1e-4 and cos >= 0.999
    assert st["unconverged"] == 0 and st["max_div"] <= 1.01e-10


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("precision,tol", [(E.FP64, 1e-10), (E.MIXED, 1e-4)])
def test_h128_bench_configuration_sampled_members(precision, tol, graphs):
    """48 steps, so that the captured step graphs replay (a graph is used while at least 16 steps
    remain), and the same with every launch eager."""
    n, horizon = 128, 48
    p = E.Problem(inv_h=n, Re=7500.0, precision=precision, flags=0 if graphs else E.FLAG_NO_GRAPHS)
    op = OE.Problem(inv_h=n, Re=7500.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    base = OE.spinup(op, OE.initial_state(op, u0, v0), 12)
    rows = np.vstack([np.zeros(op.m), inputs.grf_perturbations(64, n, 0.05, 5e-3)])
    state = E.state_init(E.Problem(inv_h=n, Re=7500.0), base.u, base.v, base.Tu_prev, base.Tv_prev)
    ctrl = torch.tensor(rows, device="cuda")
    J, F, st = E.forward(p, state, ctrl, horizon, fields=True)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy()
    assert np.all(np.isfinite(Jg)) and st["unconverged"] == 0
    u, v = E.split_fields(p, F)
    for i in (0, 17, 64):
        Jr, sr = OE.forward_member(op, base, rows[i], horizon, return_state=True)
        rel = abs(Jg[i] - Jr) / abs(Jr)
        du = np.abs(u[i] - sr.u).max() / np.abs(sr.u).max()
        _say("h128 member", i, "J rel", rel, "u rel", du)
        assert rel <= tol
        assert du <= (1e-10 if precision == E.FP64 else 1e-5)


def test_iterate_matches_oracle_descent():
    n, N, horizon = 16, 6, 12
    p = E.Problem(inv_h=n, Re=1000.0)
    op = OE.Problem(inv_h=n, Re=1000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-2, seed=4)
    base = OE.spinup(op, OE.initial_state(op, u0, v0), 30)
    pert = inputs.grf_perturbations(N, n, 0.1, 1e-5, seed=8)
    f0 = np.zeros(op.m)
    hist = OE.iterate(op, base, f0, pert, horizon, iters=3)
    state = E.state_init(p, base.u, base.v, base.Tu_prev, base.Tv_prev)
    f = torch.tensor(f0, device="cuda")
    recs = E.iterate(p, state, f, torch.tensor(pert, device="cuda"), horizon, iters=3)
    torch.cuda.synchronize()
    _say("iterate gpu", recs)
    _say("iterate oracle", [(h["J0"], h["alpha"]) for h in hist])
    assert len(recs) == len(hist)
    for r, h in zip(recs, hist):
        assert abs(r["J0"] - h["J0"]) <= 1e-9 * abs(h["J0"])
        assert abs(r["alpha"] - h["alpha"]) <= 1e-6 * abs(h["alpha"])
    fo = hist[-1]["f"]
    assert np.abs(f.cpu().numpy() - fo).max() <= 1e-6 * np.abs(fo).max()
    assert len(hist) == 3 and hist[0]["alpha"] > 0.0  # the descent really moved
    assert recs[0]["J_trial"] < recs[0]["J0"]


@pytest.mark.parametrize("N", [6, 2])
def test_iterate_backtracking_matches_oracle(N):
    """A first trial step 64 times the default, so that the Armijo search backtracks several times
    (Fig. envar_loop, Sec. 3.3.3). The trials run together, up to N + 1 of them per batched forward
    (N = 6: 7 and 1 trial rows; N = 2: 3, 3 and 2); the step and the cost accepted must be those
    of the oracle's search, which tries one step after another."""
    n, horizon = 16, 12
    p = E.Problem(inv_h=n, Re=1000.0)
    op = OE.Problem(inv_h=n, Re=1000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-2, seed=4)
    base = OE.spinup(op, OE.initial_state(op, u0, v0), 30)
    pert = inputs.grf_perturbations(N, n, 0.1, 1e-5, seed=8)
    f0 = np.zeros(op.m)
    rows = np.vstack([f0, f0 + pert])
    g = OE.gradient(rows, OE.forward(op, base, rows, horizon))
    a0 = 64.0 * np.abs(pert).max() / np.abs(g).max()
    hist = OE.iterate(op, base, f0, pert, horizon, iters=1, alpha0=a0)
    state = E.state_init(p, base.u, base.v, base.Tu_prev, base.Tv_prev)
    f = torch.tensor(f0, device="cuda")
    recs = E.iterate(p, state, f, torch.tensor(pert, device="cuda"), horizon, iters=1, alpha0=a0)
    torch.cuda.synchronize()
    _say("backtracking: N", N, "a0", a0, "gpu", recs, "oracle", [(h["alpha"], h["J_new"]) for h in hist])
    h, r = hist[0], recs[0]
    assert 0.0 < h["alpha"] < a0  # backtracked, and found a step
    assert r["alpha"] == h["alpha"]  # the same trial of the same sequence a0, a0 / 2, ...
    assert abs(r["J_trial"] - h["J_new"]) <= 1e-9 * abs(h["J_new"])
    fo = h["f"]
    assert np.abs(f.cpu().numpy() - fo).max() <= 1e-6 * np.abs(fo).max()


def test_iterate_h32_workload_matches_oracle_descent():
    """Fig. envar_loop on the h = 1/32 workload's grid and ensemble (centre + 8 GRF members, length
    0.1, std 1e-2), three iterations over a 40-step horizon from a seeded non-zero forcing (std 0.5,
    so that the penalty's share of the gradient lets the first line search succeed): the same
    costs, steps and forcing."""
    n, N, horizon, iters = 32, 8, 40, 3
    p = E.Problem(inv_h=n, Re=4000.0)
    op = OE.Problem(inv_h=n, Re=4000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    base = OE.spinup(op, OE.initial_state(op, u0, v0), 100)
    pert = inputs.grf_perturbations(N, n, 0.1, 1e-2)
    f0 = inputs.grf_perturbations(1, n, 0.1, 0.5, seed=99)[0]
    hist = OE.iterate(op, base, f0, pert, horizon, iters=iters, processes=9)
    state = E.state_init(p, base.u, base.v, base.Tu_prev, base.Tv_prev)
    f = torch.tensor(f0, device="cuda")
    recs = E.iterate(p, state, f, torch.tensor(pert, device="cuda"), horizon, iters=iters)
    torch.cuda.synchronize()
    _say("iterate h32 gpu", recs)
    _say("iterate h32 oracle", [(h["J0"], h["alpha"], h["J_new"]) for h in hist])
    assert len(recs) == len(hist) == iters
    for r, h in zip(recs, hist):
        assert abs(r["J0"] - h["J0"]) <= 1e-9 * abs(h["J0"])
        assert abs(r["alpha"] - h["alpha"]) <= 1e-6 * abs(h["alpha"])
    assert hist[0]["alpha"] > 0.0 and recs[0]["J_trial"] < recs[0]["J0"]
    assert abs(recs[0]["J_trial"] - hist[0]["J_new"]) <= 1e-9 * abs(hist[0]["J_new"])
    fo = hist[-1]["f"]
    assert np.abs(f.cpu().numpy() - fo).max() <= 1e-6 * np.abs(fo).max()
    # the descent lowered the centre cost over the iterations
    assert hist[-1]["J0"] < hist[0]["J0"]

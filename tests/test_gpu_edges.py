"""Edge cases of the forward path (needs an MI355X; calls the C ABI through the binding).

* inv_h = 16: the whole V-cycle runs in the one-workgroup coarse kernel (no
  tiled level), in FP64 and in mixed precision, against the FP64 oracle;
* the cavity-only and box control regions (Sec. 4.1's actuation window)
  against the oracle;
* the finest grid of the serving mix (h = 1/256): mixed against FP64 and a
  member alone against the same member in the batch;
* argument errors are reported before any device work.
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


def _op(p):
    reg = {E.REGION_COLUMN: "column", E.REGION_CAVITY: "cavity", E.REGION_BOX: "box"}[p.region]
    return OE.Problem(inv_h=p.inv_h, Re=p.Re, dt=p.dt, x_cav=p.x_cav, region=reg, box=tuple(p.box),
                      penalty=p.penalty)


def _run(p, st, rows, horizon):
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    ctrl = torch.tensor(rows, dtype=torch.float64, device="cuda")
    J, F, stats = E.forward(p, state, ctrl, horizon, fields=True)
    torch.cuda.synchronize()
    return J.cpu().numpy(), E.split_fields(p, F), stats


@pytest.mark.parametrize("precision,tol", [(E.FP64, 1e-10), (E.MIXED, 1e-6)])
def test_lds_only_multigrid_matches_oracle(precision, tol):
    n, horizon = 16, 12
    p = E.Problem(inv_h=n, Re=4000.0, precision=precision)
    op = _op(p)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    st = OE.spinup(op, OE.initial_state(op, u0, v0), 30)
    m = E.control_dim(p)
    rows = np.vstack([np.zeros(m), inputs.grf_perturbations(2, n, 0.1, 1e-2)])
    _say("inv_h=16 parity, precision", precision)
    J, (u, v), stats = _run(p, st, rows, horizon)
    for i in range(rows.shape[0]):
        Jr, sr = OE.forward_member(op, st, rows[i], horizon, return_state=True)
        _say(" member", i, J[i], Jr, abs(J[i] - Jr) / abs(Jr))
        assert abs(J[i] - Jr) <= tol * abs(Jr)
        assert np.abs(u[i] - sr.u).max() <= tol * np.abs(sr.u).max()
    assert stats["unconverged"] == 0 and stats["rows_mg"] == [0, 0, 0, 0]


@pytest.mark.parametrize("region,box", [(E.REGION_CAVITY, (0.0, 0.0, 0.0, 0.0)),
                                        (E.REGION_BOX, (1.5, 2.2, -0.6, 0.4))])
def test_control_regions_match_oracle(region, box):
    n, horizon = 32, 8
    p = E.Problem(inv_h=n, Re=4000.0, region=region, box=box)
    op = _op(p)
    assert E.control_dim(p) == op.m
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    st = OE.spinup(op, OE.initial_state(op, u0, v0), 20)
    rng = np.random.default_rng(11)
    rows = np.vstack([np.zeros(op.m), 1e-2 * rng.standard_normal((2, op.m))])
    _say("region", region, "m", op.m)
    J, (u, v), _ = _run(p, st, rows, horizon)
    Jr = OE.forward(op, st, rows, horizon)
    _say(" J", J, "oracle", Jr)
    assert np.all(np.abs(J - Jr) <= 1e-10 * np.abs(Jr))


def test_h256_mixed_matches_fp64_and_batch_invariance():
    n, horizon = 256, 10
    p64 = E.Problem(inv_h=n, Re=12000.0)
    pmx = E.Problem(inv_h=n, Re=12000.0, precision=E.MIXED)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    state = E.state_init(p64, u0, v0)
    E.spinup(p64, state, 40)
    m = E.control_dim(p64)
    rows = np.vstack([np.zeros(m), inputs.grf_perturbations(2, n, 0.05, 5e-3)])
    ctrl = torch.tensor(rows, dtype=torch.float64, device="cuda")
    J64, _, s64 = E.forward(p64, state, ctrl, horizon)
    Jmx, _, smx = E.forward(pmx, state, ctrl, horizon)
    J1, _, _ = E.forward(pmx, state, ctrl[1:2].contiguous(), horizon)
    torch.cuda.synchronize()
    a, b, c = J64.cpu().numpy(), Jmx.cpu().numpy(), J1.cpu().numpy()
    _say("h=1/256 fp64", a, "mixed", b, "alone", c, "rows", smx["rows_mg"])
    assert np.all(np.abs(b - a) <= 1e-6 * np.abs(a))
    assert c[0] == b[1]
    assert s64["unconverged"] == 0 and smx["unconverged"] == 0
    assert len([r for r in smx["rows_mg"] if r]) == 4


def test_argument_errors_are_reported():
    n = 32
    p = E.Problem(inv_h=n, Re=4000.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3)
    state = E.state_init(p, u0, v0)
    m = E.control_dim(p)
    ctrl = torch.zeros((2, m), dtype=torch.float64, device="cuda")
    small = E._bytes_tensor(E.workspace_bytes(p, 2) // 2)
    with pytest.raises(E.EnvarError) as ei:
        E.forward(p, state, ctrl, 5, ws=small)
    assert ei.value.code == E.ENOMEM
    with pytest.raises(E.EnvarError) as ei:
        E.forward(p, state, ctrl, 0)
    assert ei.value.code == E.EINVAL
    with pytest.raises(E.EnvarError) as ei:
        E.forward(p, state, ctrl[:, :-1].contiguous(), 5)
    assert ei.value.code == E.EINVAL
    # the library still works after the rejected calls
    J, _, st = E.forward(p, state, ctrl, 3)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(J.cpu().numpy())) and st["steps"] == 3

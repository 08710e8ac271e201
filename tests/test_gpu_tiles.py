"""Tile heights do not change results (needs an MI355X; calls the C ABI through the binding).

The predictor and the projection run with 8- or 16-row tiles, every tiled
multigrid level with 8-, 16- or 32-row tiles; the tuner picks per kernel and
level. The cost partial sums live
on fixed 64 x 8 blocks and the multigrid windows reproduce the global red-black
sweep, so costs and fields must be bitwise equal across tile choices, in FP64
and in mixed precision, with several multigrid levels (h = 1/64 and 1/128).
"""
import numpy as np
import pytest

from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("precision", [E.FP64, E.MIXED])
def test_tile_choices_give_identical_results(n, precision):
    p64 = E.Problem(inv_h=n, Re=7500.0)
    u0, v0 = inputs.initial_field(n, amp=1e-3, seed=3)
    state = E.state_init(p64, u0, v0)
    E.spinup(p64, state, 20)
    m = E.control_dim(p64)
    rows = np.vstack([np.zeros(m), inputs.grf_perturbations(4, n, 0.05, 5e-3, seed=9)])
    ctrl = torch.tensor(rows, dtype=torch.float64, device="cuda")
    out = {}
    for name, flags in (("rows8", E.FLAG_TILES_8), ("rows16", E.FLAG_TILES_16), ("rows32", E.FLAG_TILES_32),
                        ("default", E.FLAG_NO_TUNE), ("tuned", 0)):
        p = E.Problem(inv_h=n, Re=7500.0, precision=precision, flags=flags)
        J, F, st = E.forward(p, state, ctrl, 25, fields=True)
        torch.cuda.synchronize()
        out[name] = (J.cpu().numpy(), F.cpu().numpy(), st)
        _say(name, "n", n, "prec", precision, "rows", st["rows_pred"], st["rows_proj"], st["rows_mg"],
             "J0", out[name][0][0])
    J8, F8, s8 = out["rows8"]
    assert s8["rows_pred"] == 8 and s8["rows_proj"] == 8 and s8["rows_mg"][0] == 8
    assert out["rows16"][2]["rows_mg"][0] == 16 and out["rows16"][2]["rows_pred"] == 16
    assert out["rows32"][2]["rows_mg"][0] == 32
    for name in ("rows16", "rows32", "default", "tuned"):
        J, F, st = out[name]
        assert np.array_equal(J, J8), name
        assert np.array_equal(F, F8), name
        assert st["unconverged"] == 0
        assert st["rows_pred"] in (8, 16) and st["rows_proj"] in (8, 16)
        nlev = {64: 2, 128: 3}[n]
        assert all(r in (8, 16, 32) for r in st["rows_mg"][:nlev]) and all(r == 0 for r in st["rows_mg"][nlev:])

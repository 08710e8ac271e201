"""envar_gradient_static (the gradient for callers that cannot allocate) against envar_gradient
(needs an MI355X).

Two calls in a row on the same inputs as envar_gradient with a caller-provided workspace, the
second with a smaller problem than the first (the static array keeps the first call's contents):
the same kernels on the same layout, so g must agree bit for bit, in FP64 and with the FP32-MFMA
Gram; and the same oracle-independent check as the other gradient tests (numpy least squares).
"""
import numpy as np
import pytest

from paper_2605_23812_amd import envar as E

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rows(n, m, seed):
    rng = np.random.default_rng(seed)
    rows = rng.standard_normal((n + 1, m)) * 1e-2
    J = rng.standard_normal(n + 1)
    return rows, J


@pytest.mark.parametrize("precision", [E.FP64, E.MIXED])
def test_static_gradient_equals_workspace_gradient_on_two_calls(precision):
    for n, m, seed in [(64, 65536, 1), (17, 3000, 2)]:  # the second call is smaller
        rows, J = _rows(n, m, seed)
        print("static gradient: precision", precision, "n", n, "m", m, flush=True)
        c = torch.tensor(rows, device="cuda")
        j = torch.tensor(J, device="cuda")
        g_ws = E.gradient(c, j, precision)
        g_st = E.gradient_static(c, j, precision)
        torch.cuda.synchronize()
        a, b = g_ws.cpu().numpy(), g_st.cpu().numpy()
        assert np.array_equal(a, b), np.abs(a - b).max()
        X = rows[1:] - rows[0]
        ref, *_ = np.linalg.lstsq(X, J[1:] - J[0], rcond=None)
        if precision == E.FP64:
            assert np.abs(b - ref).max() <= 1e-9 * np.abs(ref).max()
        else:
            assert b @ ref / (np.linalg.norm(b) * np.linalg.norm(ref)) >= 0.999999


def test_static_gradient_rejects_a_problem_beyond_its_scratch():
    n, m = 256, 65536
    rows, J = _rows(n, m, 3)
    c = torch.tensor(rows, device="cuda")
    j = torch.tensor(J, device="cuda")
    with pytest.raises(E.EnvarError) as ei:
        E.gradient_static(c, j, E.MIXED)
    assert ei.value.code == E.ENOMEM

"""The EnVar loop over the ensemble weights on the GPU against the oracle (needs an MI355X;
calls the C ABI through the binding).

Each side runs its own forwards at h = 1/32 with the lid sensors: the Gauss-Newton loop
(eq. update_Newton) and the L-BFGS loop with its Armijo line search (eq. update_BFGS) from a
non-zero w_0 at which J(w) is far from quadratic, so that the line search backtracks, pairs are
stored and the two-loop recursion uses several of them; the batched line search (several trial
steps as rows of one forward) against trying them one at a time. The discrete decisions (accepted step,
number of trials) must agree exactly; J, |g| and w within the finite-difference error of Y
(the forwards agree to about 1e-13 relative, amplified by 1 / eps in Y).
"""
import numpy as np
import pytest

from oracle import envar as OE
from oracle import gn as OG
from paper_2605_23812_amd import envar as E
from paper_2605_23812_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_INV_H, HORIZON, EVERY, N_ENS, EPS = 32, 24, 2, 4, 1e-4
W0 = np.array([1.0, -1.0, 0.5, 0.3])


def _say(*a):
    print(*a, flush=True)


def _case():
    op = OE.Problem(inv_h=N_INV_H, Re=4000.0)
    u0, v0 = inputs.initial_field(N_INV_H, amp=1e-3)
    st = OE.spinup(op, OE.initial_state(op, u0, v0), 40)
    fe = 1e-2 * inputs.grf_perturbations(1, N_INV_H, 0.1, 1.0, seed=99)[0]
    Ec = inputs.grf_perturbations(N_ENS, N_INV_H, 0.1, 10.0)
    return op, st, fe, Ec


@pytest.mark.parametrize("method,iters", [(E.GN, 3), (E.LBFGS, 5)])
def test_ens_loop_matches_oracle(method, iters):
    op, st, fe, Ec = _case()
    name = "gn" if method == E.GN else "lbfgs"
    _say("EnVar loop", name, "iters", iters)
    wr, hr = OG.iterate_ens(lambda rows: OG.forward_obs(op, st, rows, HORIZON, EVERY)[1], fe, Ec, EPS, iters,
                            method=name, w0=W0)
    p = E.Problem(inv_h=N_INV_H, Re=4000.0)
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    w, h = E.ens_iterate(p, state, torch.tensor(fe, device="cuda"), torch.tensor(Ec, device="cuda"), HORIZON,
                         iters=iters, method=method, w=torch.tensor(W0), every=EVERY, eps=EPS)
    torch.cuda.synchronize()
    w = w.cpu().numpy()
    _say(" w", w, "oracle", wr, "max err", np.abs(w - wr).max())
    assert len(h) == len(hr) == iters
    for k, (a, b) in enumerate(zip(h, hr)):
        _say(" iteration", k, "J", a["J"], b["J"], "|g|", a["gnorm"], b["gnorm"], "alpha", a["alpha"], b["alpha"],
             "trials", a["trials"], b["trials"])
        assert a["trials"] == b["trials"] and a["alpha"] == b["alpha"]
        assert abs(a["J"] - b["J"]) <= 1e-8 * abs(b["J"]) + 1e-14 * hr[0]["J"]
        assert abs(a["J_prior"] - b["J_prior"]) <= 1e-8 * abs(b["J_prior"]) + 1e-14 * hr[0]["J"]
        assert abs(a["gnorm"] - b["gnorm"]) <= 1e-6 * b["gnorm"] + 1e-12 * hr[0]["gnorm"]
    assert np.abs(w - wr).max() <= 1e-8 * np.abs(wr).max()
    if method == E.LBFGS:
        assert [r["J"] for r in h] == sorted([r["J"] for r in h], reverse=True)  # Armijo: J decreases
        assert h[0]["trial_rows"] >= h[0]["trials"] > 1
        # trials one at a time take the same decisions and reach the same w, bit for bit
        w1, h1 = E.ens_iterate(p, state, torch.tensor(fe, device="cuda"), torch.tensor(Ec, device="cuda"),
                               HORIZON, iters=iters, method=method, w=torch.tensor(W0), every=EVERY, eps=EPS,
                               trial_batch=1)
        torch.cuda.synchronize()
        assert [r["trials"] for r in h1] == [r["trial_rows"] for r in h1]
        assert [(r["alpha"], r["trials"], r["J"]) for r in h1] == [(r["alpha"], r["trials"], r["J"]) for r in h]
        assert np.array_equal(w1.cpu().numpy(), w)


def test_ens_loop_argument_errors():
    op, st, fe, Ec = _case()
    p = E.Problem(inv_h=N_INV_H, Re=4000.0)
    state = E.state_init(p, st.u, st.v, st.Tu_prev, st.Tv_prev)
    fe_d, E_d = torch.tensor(fe, device="cuda"), torch.tensor(Ec, device="cuda")
    with pytest.raises(E.EnvarError) as ei:
        E.ens_iterate(p, state, fe_d, E_d, HORIZON, method=7)
    assert ei.value.code == E.EINVAL
    with pytest.raises(E.EnvarError) as ei:
        E.ens_iterate(p, state, fe_d, E_d, 1, every=2)
    assert ei.value.code == E.EINVAL
    small = E._bytes_tensor(1024)
    with pytest.raises(E.EnvarError) as ei:
        E.ens_iterate(p, state, fe_d, E_d, HORIZON, ws=small)
    assert ei.value.code == E.ENOMEM
    pc = E.Problem(inv_h=16, Re=10.0, geometry=E.CHANNEL, region=E.REGION_BOX, box=(1.0, 1.2, 0.2, 0.4))
    sc = E.state_init(pc, np.zeros((16, 65)), np.zeros((17, 64)))
    m = E.control_dim(pc)
    with pytest.raises(E.EnvarError) as ei:
        E.ens_iterate(pc, sc, torch.zeros(m, dtype=torch.float64, device="cuda"),
                      torch.zeros((2, m), dtype=torch.float64, device="cuda"), 4,
                      ws=E._bytes_tensor(1 << 20))
    assert ei.value.code == E.EINVAL

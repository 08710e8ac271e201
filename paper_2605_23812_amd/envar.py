"""Thin ctypes binding of libenvar.so (the C ABI declared in include/envar.h).

Argument marshalling only: every computation runs in the HIP library. Device
memory and streams come from PyTorch (tensors are passed by data pointer, the
stream as torch's current HIP stream). Loading fails loudly when the library
is missing; there is no fallback path.
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libenvar.so")

OK, EINVAL, ENOMEM, EDIVERGED, EDEVICE, EBUSY, ECANCELLED, ETIMEOUT, EUNCONVERGED = range(9)
CAVITY, CHANNEL, CAVITY_PAPER = 0, 1, 2
REGION_COLUMN, REGION_CAVITY, REGION_BOX = 0, 1, 2
FP64, MIXED = 0, 1
GRADIENT_PINV = 16  # or-ed into a gradient's precision: solve by the eigen-pseudo-inverse directly
FLAG_TIME_KERNELS = 1
FLAG_NO_GRAPHS = 2
FLAG_NO_TUNE = 4
FLAG_TILES_8 = 8
FLAG_TILES_16 = 16
FLAG_TILES_32 = 32
FLAG_ONE_LANE = 64
FLAG_NO_TAIL = 128      # passes beyond the cap as one level-by-level headroom pass, not the per-member launch
FLAG_SHORT_GRAPH = 256  # one level-by-level pass per step, the rest in the per-member launch (comparisons)

EXPORTS = (
    "envar_control_dim", "envar_cell_count", "envar_state_bytes", "envar_workspace_bytes",
    "envar_state_init", "envar_state_read", "envar_spinup", "envar_forward", "envar_forward_batch",
    "envar_gradient_bytes", "envar_gradient", "envar_gradient_static", "envar_iterate_bytes", "envar_iterate",
    "envar_last_error", "envar_version", "envar_stream_copy",
    "envar_request_bytes", "envar_server_create", "envar_submit", "envar_wait", "envar_server_destroy",
    "envar_forward_obs", "envar_gn_bytes", "envar_gn_step", "envar_posterior_bytes", "envar_posterior_var",
    "envar_ens_bytes", "envar_ens_iterate",
    "envar_eigen_bytes", "envar_eigen_ensemble", "envar_recon_bytes", "envar_recon_error",
)
GN, LBFGS = 0, 1
TAPER_NONE, TAPER_ELLIPSE = 0, 1
OBS_CHANNELS = 8  # four lid sensors x two velocity components


class EnvarError(RuntimeError):
    """A library call failed: `code` is the ENVAR_E* status, the message that of envar_last_error."""
    def __init__(self, code, msg):
        super().__init__(f"envar error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [
        ("inv_h", ctypes.c_int32), ("geometry", ctypes.c_int32), ("region", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("Re", ctypes.c_double), ("dt", ctypes.c_double),
        ("x_cav", ctypes.c_double), ("box", ctypes.c_double * 4), ("penalty", ctypes.c_double),
        ("div_tol", ctypes.c_double), ("max_cycles", ctypes.c_int32), ("flags", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    """envar_stats: convergence and throughput statistics of a forward or a spin-up."""
    _fields_ = [
        ("max_resid", ctypes.c_double), ("max_div", ctypes.c_double), ("mean_cycles", ctypes.c_double),
        ("max_cycles_used", ctypes.c_int32), ("unconverged", ctypes.c_int32), ("diverged", ctypes.c_int32),
        ("steps", ctypes.c_int32), ("cell_steps", ctypes.c_double),
        ("predictor_us", ctypes.c_double), ("pre_us", ctypes.c_double), ("post_us", ctypes.c_double),
        ("resid_us", ctypes.c_double), ("project_us", ctypes.c_double), ("vcycle_us", ctypes.c_double),
        ("timed_steps", ctypes.c_int32), ("timed_members", ctypes.c_int32),
        ("rows_pred", ctypes.c_int32), ("rows_proj", ctypes.c_int32), ("rows_mg", ctypes.c_int32 * 4),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["rows_mg"] = list(self.rows_mg)
        return d


class _Job(ctypes.Structure):
    _fields_ = [
        ("problem", _Problem), ("state_dev", ctypes.c_void_p), ("controls_dev", ctypes.c_void_p),
        ("n_rows", ctypes.c_int32), ("horizon", ctypes.c_int32), ("m", ctypes.c_int64),
        ("ws_dev", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t), ("J_dev", ctypes.c_void_p),
        ("stats", ctypes.POINTER(Stats)), ("fields_dev", ctypes.c_void_p),
    ]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("max_jobs", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("problem", _Problem), ("state_dev", ctypes.c_void_p), ("controls", ctypes.c_void_p),
                ("n_rows", ctypes.c_int32), ("horizon", ctypes.c_int32), ("m", ctypes.c_int64)]


class RequestStats(ctypes.Structure):
    """envar_request_stats: timings (seconds since the server started) and status of a served request."""
    _fields_ = [("submit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("latency_s", ctypes.c_double), ("queue_s", ctypes.c_double), ("cell_steps", ctypes.c_double),
                ("status", ctypes.c_int32), ("peak_jobs", ctypes.c_int32), ("max_div", ctypes.c_double),
                ("mean_cycles", ctypes.c_double), ("unconverged", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LSParams(ctypes.Structure):
    """envar_ls_params: Armijo line search of envar_iterate (fields <= 0 take the defaults)."""
    _fields_ = [
        ("iters", ctypes.c_int32), ("max_trials", ctypes.c_int32), ("c1", ctypes.c_double),
        ("shrink", ctypes.c_double), ("alpha0", ctypes.c_double), ("search_every", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class IterRecord(ctypes.Structure):
    """envar_iter_record: one iteration of envar_iterate (J at the centre, |g|, step, cost at the step)."""
    _fields_ = [("J0", ctypes.c_double), ("gnorm", ctypes.c_double), ("alpha", ctypes.c_double),
                ("J_trial", ctypes.c_double)]


class EnsParams(ctypes.Structure):
    """envar_ens_params: the loop over the ensemble weights (GN or L-BFGS; fields <= 0 take the defaults)."""
    _fields_ = [
        ("method", ctypes.c_int32), ("iters", ctypes.c_int32), ("memory", ctypes.c_int32),
        ("max_trials", ctypes.c_int32), ("every", ctypes.c_int32), ("trial_batch", ctypes.c_int32),
        ("eps", ctypes.c_double), ("c1", ctypes.c_double), ("shrink", ctypes.c_double),
    ]


class EnsRecord(ctypes.Structure):
    """envar_ens_record: one iteration of envar_ens_iterate (J, its two terms, |dJ/dw|, step, trials)."""
    _fields_ = [("J", ctypes.c_double), ("J_obs", ctypes.c_double), ("J_prior", ctypes.c_double),
                ("gnorm", ctypes.c_double), ("alpha", ctypes.c_double), ("trials", ctypes.c_int32),
                ("trial_rows", ctypes.c_int32)]


class EigenParams(ctypes.Structure):
    """envar_eigen_params: the tapered Gaussian prior covariance and the subspace iteration."""
    _fields_ = [
        ("a_x", ctypes.c_double), ("a_y", ctypes.c_double), ("sigma2_max", ctypes.c_double), ("tol", ctypes.c_double),
        ("taper", ctypes.c_int32), ("component", ctypes.c_int32), ("oversample", ctypes.c_int32),
        ("max_iters", ctypes.c_int32), ("seed", ctypes.c_uint64),
    ]


class EigenInfo(ctypes.Structure):
    """envar_eigen_info: iterations, convergence, block size, largest kept residual, orthonormality error."""
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("block", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("max_resid", ctypes.c_double), ("orth_err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


@dataclass
class Problem:
    """Python mirror of envar_problem (fields <= 0 take the library defaults)."""
    inv_h: int = 32
    Re: float = 4000.0
    dt: float = 0.0
    x_cav: float = 1.25
    geometry: int = CAVITY
    region: int = REGION_COLUMN
    box: tuple = (0.0, 0.0, 0.0, 0.0)
    precision: int = FP64
    penalty: float = 1e-3
    div_tol: float = 0.0
    max_cycles: int = 0
    flags: int = 0

    def c(self):
        p = _Problem()
        p.inv_h, p.geometry, p.region, p.precision = self.inv_h, self.geometry, self.region, self.precision
        p.Re, p.dt, p.x_cav, p.penalty, p.div_tol = self.Re, self.dt, self.x_cav, self.penalty, self.div_tol
        p.box = (ctypes.c_double * 4)(*self.box)
        p.max_cycles, p.flags = self.max_cycles, self.flags
        return p

    @property
    def step_dt(self):
        return self.dt if self.dt > 0 else 0.064 / self.inv_h

    def box_dims(self):
        n = self.inv_h
        return {CAVITY: (4 * n, 2 * n), CAVITY_PAPER: (4 * n, n + n // 2)}.get(self.geometry, (4 * n, n))


_lib = None


def lib():
    """Load libenvar.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2605_23812_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(_Problem)
    vp, dp, i32, i64, sz = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.envar_control_dim.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    L.envar_cell_count.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    L.envar_state_bytes.argtypes = [P]
    L.envar_state_bytes.restype = sz
    L.envar_workspace_bytes.argtypes = [P, i32]
    L.envar_workspace_bytes.restype = sz
    L.envar_state_init.argtypes = [P, dp, dp, dp, dp, dp, vp, vp]
    L.envar_state_read.argtypes = [P, vp, dp, dp, dp, dp, dp]
    L.envar_spinup.argtypes = [P, vp, i32, vp, sz, ctypes.POINTER(Stats), vp]
    L.envar_forward.argtypes = [P, vp, dp, i32, i64, i32, vp, sz, dp, dp, ctypes.POINTER(Stats), vp]
    L.envar_forward_batch.argtypes = [ctypes.POINTER(_Job), i32, vp]
    L.envar_gradient_bytes.argtypes = [i32, i64, i32]
    L.envar_gradient_bytes.restype = sz
    L.envar_gradient.argtypes = [dp, dp, i32, i64, i32, vp, sz, dp, vp]
    L.envar_iterate_bytes.argtypes = [P, i32, i64]
    L.envar_iterate_bytes.restype = sz
    L.envar_iterate.argtypes = [P, vp, dp, dp, i32, i64, i32, ctypes.POINTER(LSParams), vp, sz,
                                ctypes.POINTER(IterRecord), vp]
    L.envar_request_bytes.argtypes = [P, i32]
    L.envar_request_bytes.restype = sz
    L.envar_server_create.argtypes = [ctypes.POINTER(_ServerConfig), vp, sz, ctypes.POINTER(ctypes.c_void_p)]
    L.envar_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
    L.envar_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, dp, ctypes.POINTER(RequestStats)]
    L.envar_server_destroy.argtypes = [vp]
    L.envar_stream_copy.argtypes = [vp, vp, sz, vp]
    L.envar_forward_obs.argtypes = [P, vp, dp, i32, i64, i32, i32, vp, sz, dp, dp, ctypes.POINTER(Stats), vp]
    L.envar_gn_bytes.argtypes = [i32, i64]
    L.envar_gn_bytes.restype = sz
    L.envar_gn_step.argtypes = [dp, i32, i64, ctypes.c_double, dp, vp, sz, dp, dp, dp, vp]
    L.envar_posterior_bytes.argtypes = [i32]
    L.envar_posterior_bytes.restype = sz
    L.envar_posterior_var.argtypes = [dp, i32, i64, ctypes.c_double, dp, vp, sz, dp, vp]
    L.envar_ens_bytes.argtypes = [P, i32, i64, i32, i32]
    L.envar_ens_bytes.restype = sz
    L.envar_ens_iterate.argtypes = [P, vp, dp, dp, i32, i64, i32, ctypes.POINTER(EnsParams), dp, vp, sz,
                                    ctypes.POINTER(EnsRecord), vp]
    L.envar_eigen_bytes.argtypes = [P, i32, ctypes.POINTER(EigenParams)]
    L.envar_eigen_bytes.restype = sz
    L.envar_eigen_ensemble.argtypes = [P, i32, ctypes.POINTER(EigenParams), dp, dp, vp, sz, ctypes.POINTER(EigenInfo),
                                       vp]
    L.envar_recon_bytes.argtypes = [i32, i64]
    L.envar_recon_bytes.restype = sz
    L.envar_recon_error.argtypes = [dp, i32, i64, dp, vp, sz, dp, vp]
    L.envar_last_error.restype = ctypes.c_char_p
    L.envar_version.restype = ctypes.c_char_p
    for name in ("envar_control_dim", "envar_cell_count", "envar_state_init", "envar_state_read",
                 "envar_spinup", "envar_forward", "envar_forward_batch", "envar_gradient", "envar_iterate",
                 "envar_server_create", "envar_submit", "envar_wait", "envar_server_destroy",
                 "envar_stream_copy", "envar_forward_obs", "envar_gn_step", "envar_posterior_var",
                 "envar_ens_iterate", "envar_eigen_ensemble", "envar_recon_error"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        raise EnvarError(rc, lib().envar_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _hptr(a):
    return ctypes.c_void_p(0) if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------- sizes
def control_dim(p):
    """m, the length of a control row (both forcing components over the control cells)."""
    m = ctypes.c_int64()
    _check(lib().envar_control_dim(ctypes.byref(p.c()), ctypes.byref(m)))
    return m.value


def cell_count(p):
    """Fluid cells of the finest grid."""
    n = ctypes.c_int64()
    _check(lib().envar_cell_count(ctypes.byref(p.c()), ctypes.byref(n)))
    return n.value


def state_bytes(p):
    """Device bytes of the resident base state."""
    return lib().envar_state_bytes(ctypes.byref(p.c()))


def workspace_bytes(p, n_rows):
    """Device workspace bytes of a forward over n_rows control rows."""
    return lib().envar_workspace_bytes(ctypes.byref(p.c()), n_rows)


def gradient_bytes(n, m, precision=FP64):
    """Device workspace bytes of envar_gradient for n perturbed rows of length m."""
    return lib().envar_gradient_bytes(n, m, precision)


def iterate_bytes(p, n, m):
    """Device workspace bytes of envar_iterate with n perturbations of length m."""
    return lib().envar_iterate_bytes(ctypes.byref(p.c()), n, m)


# ---------------------------------------------------------------------------- calls
def _bytes_tensor(nbytes, device="cuda"):
    import torch

    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def state_init(p, u, v, tu_prev=None, tv_prev=None, phi=None, state=None):
    """Upload a base state (host arrays in oracle layout) into a (new) device buffer."""
    if state is None:
        state = _bytes_tensor(state_bytes(p))
    arrs = [_host(a) for a in (u, v, tu_prev, tv_prev, phi)]
    _check(lib().envar_state_init(ctypes.byref(p.c()), *[_hptr(a) for a in arrs], _ptr(state), _stream()))
    return state


def state_read(p, state):
    """Host copies (u, v, T_u, T_v, phi) of a device base state, in the oracle layout."""
    NX, NY = p.box_dims()
    u = np.empty((NY, NX + 1))
    v = np.empty((NY + 1, NX))
    tu = np.empty_like(u)
    tv = np.empty_like(v)
    phi = np.empty((NY, NX))
    import torch

    torch.cuda.current_stream().synchronize()
    _check(lib().envar_state_read(ctypes.byref(p.c()), _ptr(state), *[_hptr(a) for a in (u, v, tu, tv, phi)]))
    return u, v, tu, tv, phi


def spinup(p, state, steps, ws=None):
    """Advance the base state in place by `steps` unforced steps (envar_spinup); returns the statistics."""
    if ws is None:
        ws = _bytes_tensor(workspace_bytes(p, 1))
    st = Stats()
    _check(lib().envar_spinup(ctypes.byref(p.c()), _ptr(state), steps, _ptr(ws), ws.numel(), ctypes.byref(st),
                              _stream()))
    return st.as_dict()


def forward(p, state, controls, horizon, ws=None, J=None, fields=False, stats=True):
    """J [n_rows] (torch FP64 on the device) for control rows `controls` [n_rows, m] (torch FP64 device)."""
    import torch

    n_rows, m = controls.shape
    assert controls.dtype == torch.float64 and controls.is_cuda and controls.is_contiguous()
    if ws is None:
        ws = _bytes_tensor(workspace_bytes(p, n_rows))
    if J is None:
        J = torch.empty(n_rows, dtype=torch.float64, device=controls.device)
    F = None
    if fields:
        NX, NY = p.box_dims()
        F = torch.empty((n_rows, NY * (NX + 1) + (NY + 1) * NX), dtype=torch.float64, device=controls.device)
    st = Stats() if stats else None
    rc = lib().envar_forward(ctypes.byref(p.c()), _ptr(state), _ptr(controls), n_rows, m, horizon, _ptr(ws),
                             ws.numel(), _ptr(J), _ptr(F), ctypes.byref(st) if st is not None else None, _stream())
    if rc == EDIVERGED:
        return J, F, st.as_dict()
    _check(rc)
    return J, F, (st.as_dict() if st is not None else None)


def forward_batch(jobs, fields=False):
    """Uneven batch: jobs = [(problem, state, controls [n, m] device FP64, horizon)], up to 8.

    Returns a list of (J tensor, stats dict) in job order, or of (J, stats, fields tensor) with
    fields=True (each member's final u, v flattened as in `forward`; see `split_fields`).
    """
    import torch

    arr = (_Job * len(jobs))()
    keep = []
    for k, (p, state, ctrl, horizon) in enumerate(jobs):
        n, m = ctrl.shape
        ws = _bytes_tensor(workspace_bytes(p, n))
        J = torch.empty(n, dtype=torch.float64, device=ctrl.device)
        st = Stats()
        F = None
        if fields:
            NX, NY = p.box_dims()
            F = torch.empty((n, NY * (NX + 1) + (NY + 1) * NX), dtype=torch.float64, device=ctrl.device)
            arr[k].fields_dev = F.data_ptr()
        keep.append((ws, J, st, F))
        arr[k].problem = p.c()
        arr[k].state_dev = state.data_ptr()
        arr[k].controls_dev = ctrl.data_ptr()
        arr[k].n_rows, arr[k].horizon, arr[k].m = n, horizon, m
        arr[k].ws_dev, arr[k].ws_bytes = ws.data_ptr(), ws.numel()
        arr[k].J_dev = J.data_ptr()
        arr[k].stats = ctypes.pointer(st)
    rc = lib().envar_forward_batch(arr, len(jobs), _stream())
    if rc != EDIVERGED:
        _check(rc)
    if fields:
        return [(J, st.as_dict(), F) for (_, J, st, F) in keep]
    return [(J, st.as_dict()) for (_, J, st, _) in keep]


def split_fields(p, F):
    """[n_rows, ...] flat fields -> (u [n, NY, NX+1], v [n, NY+1, NX]) numpy."""
    NX, NY = p.box_dims()
    F = F.cpu().numpy()
    nu = NY * (NX + 1)
    return F[:, :nu].reshape(-1, NY, NX + 1), F[:, nu:].reshape(-1, NY + 1, NX)


def gradient(controls, J, precision=FP64, ws=None, g=None):
    """g [m] = X^+ dJ for rows 1..n of controls [n+1, m] against row 0.

    precision: FP64 or MIXED, optionally | GRADIENT_PINV (the eigen-pseudo-inverse instead of the
    ridged Cholesky; a failed Cholesky falls back to it by itself)."""
    import torch

    n = controls.shape[0] - 1
    m = controls.shape[1]
    if ws is None:
        ws = _bytes_tensor(gradient_bytes(n, m, precision))
    if g is None:
        g = torch.empty(m, dtype=torch.float64, device=controls.device)
    _check(lib().envar_gradient(_ptr(controls), _ptr(J), n, m, precision, _ptr(ws), ws.numel(), _ptr(g), _stream()))
    return g


GRADIENT_STATIC_MAX_BYTES = 64 << 20


def gradient_static(controls, J, precision=FP64, g=None):
    """`gradient` with the library's static device scratch as workspace (no allocation in the call).

    For n, m whose gradient_bytes exceed GRADIENT_STATIC_MAX_BYTES the call raises (ENOMEM). Calls
    on one GPU share the scratch: overlapping calls race.
    """
    import torch

    n = controls.shape[0] - 1
    m = controls.shape[1]
    if g is None:
        g = torch.empty(m, dtype=torch.float64, device=controls.device)
    _check(lib().envar_gradient_static(_ptr(controls), _ptr(J), n, m, precision, _ptr(g), _stream()))
    return g


def forward_obs(p, state, controls, horizon, every=1, ws=None, J=None, stats=True):
    """J [n_rows] and the lid-sensor series [n_rows, 8, horizon // every] (torch FP64 on the device)."""
    import torch

    n_rows, m = controls.shape
    assert controls.dtype == torch.float64 and controls.is_cuda and controls.is_contiguous()
    if ws is None:
        ws = _bytes_tensor(workspace_bytes(p, n_rows))
    if J is None:
        J = torch.empty(n_rows, dtype=torch.float64, device=controls.device)
    obs = torch.empty((n_rows, OBS_CHANNELS, horizon // every), dtype=torch.float64, device=controls.device)
    st = Stats() if stats else None
    rc = lib().envar_forward_obs(ctypes.byref(p.c()), _ptr(state), _ptr(controls), n_rows, m, horizon, every,
                                 _ptr(ws), ws.numel(), _ptr(J), _ptr(obs),
                                 ctypes.byref(st) if st is not None else None, _stream())
    if rc == EDIVERGED:
        return J, obs, st.as_dict()
    _check(rc)
    return J, obs, (st.as_dict() if st is not None else None)


def gn_step(series, eps, w, ws=None):
    """Gauss-Newton step from the sensor series [n+1, 8, K]: (dw [n], H_GN [n, n], (J_obs, J_prior))."""
    import torch

    rows, ch, K = series.shape
    assert ch == OBS_CHANNELS and series.dtype == torch.float64 and series.is_contiguous()
    n = rows - 1
    w = w.contiguous()
    if ws is None:
        ws = _bytes_tensor(lib().envar_gn_bytes(n, K))
    dw = torch.empty(n, dtype=torch.float64, device=series.device)
    H = torch.empty((n, n), dtype=torch.float64, device=series.device)
    jw = torch.empty(2, dtype=torch.float64, device=series.device)
    _check(lib().envar_gn_step(_ptr(series), n, K, float(eps), _ptr(w), _ptr(ws), ws.numel(), _ptr(dw), _ptr(H),
                               _ptr(jw), _stream()))
    return dw, H, jw


def posterior_var(controls, eps, H, ws=None):
    """diag(E H^-1 E^T) [m] with E_i = (f_i - f_0) / eps from controls [n+1, m] (device FP64)."""
    import torch

    rows, m = controls.shape
    n = rows - 1
    if ws is None:
        ws = _bytes_tensor(lib().envar_posterior_bytes(n))
    var = torch.empty(m, dtype=torch.float64, device=controls.device)
    _check(lib().envar_posterior_var(_ptr(controls), n, m, float(eps), _ptr(H.contiguous()), _ptr(ws), ws.numel(),
                                     _ptr(var), _stream()))
    return var


def eigen_params(a_x=0.07, a_y=0.07, sigma2_max=0.01, taper=TAPER_ELLIPSE, component=1, oversample=0, max_iters=0,
                 tol=0.0, seed=0):
    """EigenParams with the paper's taper and length scales as defaults."""
    return EigenParams(a_x, a_y, sigma2_max, tol, taper, component, oversample, max_iters, seed)


def eigen_bytes(p, N, prm=None):
    """Device workspace bytes of envar_eigen_ensemble for N members."""
    prm = prm or eigen_params()
    return lib().envar_eigen_bytes(ctypes.byref(p.c()), N, ctypes.byref(prm))


def eigen_ensemble(p, N, ws=None, **kw):
    """Deterministic eigen-ensemble: (E [N, m] device FP64 members, mu [N] eigenvalues of B, info)."""
    import torch

    prm = eigen_params(**kw)
    if ws is None:
        nb = eigen_bytes(p, N, prm)
        if nb == 0:
            _check(lib().envar_eigen_ensemble(ctypes.byref(p.c()), N, ctypes.byref(prm), None, None, None, 0, None,
                                              _stream()))
        ws = _bytes_tensor(nb)
    m = control_dim(p)
    E = torch.empty((N, m), dtype=torch.float64, device="cuda")
    mu = torch.empty(N, dtype=torch.float64, device="cuda")
    info = EigenInfo()
    _check(lib().envar_eigen_ensemble(ctypes.byref(p.c()), N, ctypes.byref(prm), _ptr(E), _ptr(mu), _ptr(ws),
                                      ws.numel(), ctypes.byref(info), _stream()))
    return E, mu, info.as_dict()


def recon_error(E, f, ws=None):
    """Reconstruction error of f [m] in the span of the rows of E [N, m] (device; a 1-element tensor)."""
    import torch

    N, m = E.shape
    if ws is None:
        ws = _bytes_tensor(lib().envar_recon_bytes(N, m))
    out = torch.empty(1, dtype=torch.float64, device=E.device)
    _check(lib().envar_recon_error(_ptr(E.contiguous()), N, m, _ptr(f.contiguous()), _ptr(ws), ws.numel(), _ptr(out),
                                   _stream()))
    return out


def ens_bytes(p, n, m, horizon, every=1):
    """Device workspace bytes of envar_ens_iterate."""
    return lib().envar_ens_bytes(ctypes.byref(p.c()), n, m, horizon, every)


def ens_iterate(p, state, fe, E, horizon, iters=1, method=GN, w=None, memory=5, max_trials=10, every=1,
                eps=1e-4, c1=1e-4, shrink=0.5, trial_batch=8, ws=None):
    """EnVar loop over the ensemble weights (device FP64 fe [m], E [n, m]). Returns (w [n] on the
    device, per-iteration records up to an early stop)."""
    import torch

    n, m = E.shape
    assert fe.dtype == E.dtype == torch.float64 and fe.is_contiguous() and E.is_contiguous()
    if ws is None:
        ws = _bytes_tensor(ens_bytes(p, n, m, horizon, every))
    w = (torch.zeros(n, dtype=torch.float64, device=E.device) if w is None
         else w.to(device=E.device, dtype=torch.float64).clone().contiguous())
    prm = EnsParams(method, iters, memory, max_trials, every, trial_batch, eps, c1, shrink)
    recs = (EnsRecord * iters)()
    _check(lib().envar_ens_iterate(ctypes.byref(p.c()), _ptr(state), _ptr(fe), _ptr(E), n, m, horizon,
                                   ctypes.byref(prm), _ptr(w), _ptr(ws), ws.numel(), recs, _stream()))
    out = []
    for r in recs:
        out.append(dict(J=r.J, J_obs=r.J_obs, J_prior=r.J_prior, gnorm=r.gnorm, alpha=r.alpha, trials=r.trials,
                        trial_rows=r.trial_rows))
        if method == LBFGS and r.alpha == 0.0:
            break
    return w, out


def iterate(p, state, f, perturb, horizon, iters=1, max_trials=8, c1=1e-4, shrink=0.5, alpha0=0.0,
            search_every=0, ws=None):
    """Fixed-ensemble descent; f (device FP64 [m]) is updated in place. Returns per-iteration records."""
    n, m = perturb.shape
    if ws is None:
        ws = _bytes_tensor(iterate_bytes(p, n, m))
    ls = LSParams(iters, max_trials, c1, shrink, alpha0, search_every, 0)
    recs = (IterRecord * iters)()
    _check(lib().envar_iterate(ctypes.byref(p.c()), _ptr(state), _ptr(f), _ptr(perturb), n, m, horizon,
                               ctypes.byref(ls), _ptr(ws), ws.numel(), recs, _stream()))
    out = []
    for r in recs:
        out.append(dict(J0=r.J0, gnorm=r.gnorm, alpha=r.alpha, J_trial=r.J_trial))
        if r.alpha == 0.0:  # the line search failed: the loop stopped here
            break
    return out


def request_bytes(p, n_rows):
    """Pool bytes one served request of n_rows rows occupies (its admission footprint)."""
    return lib().envar_request_bytes(ctypes.byref(p.c()), n_rows)


class Server:
    """Continuous-batching forward server over a device pool (worker thread in the library)."""

    def __init__(self, pool_bytes, max_jobs=8, precision=MIXED, max_queue=0, flags=0):
        import torch

        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        cfg = _ServerConfig(max_jobs, precision, max_queue, flags)
        h = ctypes.c_void_p()
        _check(lib().envar_server_create(ctypes.byref(cfg), _ptr(self.pool), self.pool.numel(), ctypes.byref(h)))
        self.h = h
        self.precision = precision
        self._keep = {}

    def submit(self, p, state, controls, horizon):
        """controls: host numpy [n, m] FP64 (copied by the library); state: device base state tensor."""
        c = np.ascontiguousarray(controls, dtype=np.float64)
        req = _Request(p.c(), state.data_ptr(), c.ctypes.data, c.shape[0], horizon, c.shape[1])
        t = ctypes.c_uint64()
        _check(lib().envar_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (state, c.shape[0])
        return t.value

    def wait(self, ticket, timeout=-1.0):
        state, n = self._keep[ticket]
        J = np.empty(n)
        st = RequestStats()
        rc = lib().envar_wait(self.h, ticket, timeout, J.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
        if rc == ETIMEOUT:
            raise TimeoutError(lib().envar_last_error().decode())
        if rc not in (OK, EDIVERGED, EUNCONVERGED):
            _check(rc)
        del self._keep[ticket]
        return J, st.as_dict()

    def close(self):
        if self.h:
            lib().envar_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_copy(src, dst):
    """The library's streaming copy (the bandwidth reference of the benchmark and the counters)."""
    _check(lib().envar_stream_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), _stream()))


def version():
    """Library version string (name, version, target architecture)."""
    return lib().envar_version().decode()

"""Benchmark: ensemble cell-steps/s of the batched EnVar forward + anomaly gradient on one MI355X.

Workload (one "step" = one full pass of the hot path): the h = 1/128 open
cavity (512 x 128 channel + 128 x 128 cavity = 81,920 fluid cells), Re = 7500,
dt = 5e-4, a centre run plus 64 GRF-perturbed forcings (m = 65,536, length
0.05, std 5e-3) integrated for 20,000 steps from a 2,000-step spin-up, then
the anomaly Gram / least-squares / projection to the gradient. `value` is the
batched mixed-precision path (FP32 stencil tendencies and V-cycles inside
FP64 iterative refinement to max|div u| <= 1e-10); the plain FP64 batched and
FP64 one-member-at-a-time paths are measured beside it on a shorter horizon.
All inputs are synthetic and seeded; nothing is read from disk.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--horizon H]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
N_MEMBERS = 64
INV_H, RE, SPINUP = 128, 7500.0, 2000
ELL, SIGMA = 0.05, 5e-3
DIV_TOL = 1e-10      # divergence bound of the headline and of every baseline it is compared with
DIV_TOL_REF = 1e-12  # the FP64 accuracy reference

# the minimal-fusion byte model per cell-step (every field moved once per step, the tendency
# history and forcing once, halos from cache; no warm-start history):
# fused predictor + projection + cost 59 + 80 (mixed) / 78 + 80 (FP64), each refinement pass 133 B
# (mixed), each FP64 V-cycle 187 B
MINIMAL_PRED_PROJ = {"mixed": 139.0, "fp64": 158.0}
MINIMAL_PER_CYCLE = {"mixed": 133.0, "fp64": 187.0}

# algorithmic bytes per fluid cell and launch (ideal fusion, halos re-read from cache)
BYTES_PER_CELL = {
    # predictor fused with the previous step's projection: u*, v* of the previous step (16) + phi (8)
    # + T^{n-1} (16) + forcing on 2/5 of the cells (6.4) + cost sums S1 read and written (32) + warm start:
    # phi^{n-2}, phi^{n-3} in, guess and phi^{n-2} out (32) -> u*, v* (16) + T^n (16) + b (8);
    # FP64 jobs warm-start from one more pressure (cubic): phi^{n-4} in, phi^{n-3} out (+16)
    ("predictor", "fp64"): 166.4, ("predictor", "mixed"): 150.4,
    # phi in/out (8 + 8) + b (8) + coarse rhs (8/4)   | mixed, first pass: phi64 (8) + b64 (8) -> r (4) + e (4)
    #                                                 + coarse (1)
    ("pre", "fp64"): 26.0, ("pre", "mixed"): 25.0,
    # phi in/out (8 + 8) + b (8) + coarse correction (8/4)   | mixed: e (4) + r (4) + coarse (1) + phi64 in/out
    #                                                 (16) -> r - L e (4)
    ("post", "fp64"): 26.0, ("post", "mixed"): 29.0,
    # phi64 (8) + b64 (8) -> r32 (4)
    ("resid", "mixed"): 20.0,
    # u*, v* (16) + phi (8) -> u, v (16) + cost sums S1 in/out (32) + warm start: phi^{n-1} in / guess out (16)
    # + phi^{n-2} in / phi^{n-1} out (16); FP64: + phi^{n-3} in / phi^{n-2} out (16)
    ("project", "fp64"): 120.0, ("project", "mixed"): 104.0,
}

# HBM bytes per member-cell of a launch from the two calibrated rocprofv3 counter passes
# (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for the library's streaming copy of known
# size), h=1/128, recorded with the kernel sources and launch shapes of the summaries in profiles/.
# Set an entry to None when its kernel or its launch shape changes.
MEASURED_TRAFFIC_PER_MEMBER_CELL = {
    # profiles/k_predictor_fused_h128_65members_mixed.md: 33-member launches (two lanes), 479.9 MB per
    # launch (FETCH 279.4 + WRITE 200.4); the first refinement pass's finest pre kernel 73.9 MB
    ("predictor", "mixed"): 177.5,
    ("pre", "mixed"): 27.3,
    ("post", "mixed"): None,
    ("resid", "mixed"): None,
    # profiles/k_predictor_fused_h128_65members_fp64.md: the cubic-warm-start FP64 predictor, 33-member
    # launches (two lanes), 523.7 MB per launch (FETCH 301.7 + WRITE 221.9)
    ("predictor", "fp64"): 193.7,
    ("pre", "fp64"): None,
    ("post", "fp64"): None,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_inputs(torch, E, inputs, flags=0):
    p64 = E.Problem(inv_h=INV_H, Re=RE, precision=E.FP64, flags=flags)
    u0, v0 = inputs.initial_field(INV_H, amp=1e-3)
    state = E.state_init(p64, u0, v0)
    t = time.time()
    st = E.spinup(p64, state, SPINUP)
    torch.cuda.synchronize()
    log(f"spin-up {SPINUP} steps: {time.time() - t:.2f}s, mean cycles {st['mean_cycles']:.2f}")
    m = E.control_dim(p64)
    pert = inputs.grf_perturbations(N_MEMBERS, INV_H, ELL, SIGMA)
    rows = np.vstack([np.zeros(m), pert])
    return state, torch.tensor(rows, dtype=torch.float64, device="cuda"), m


def one_pass(E, p, state, ctrl, horizon, ws, J, gws, g, stats=False):
    J, _, st = E.forward(p, state, ctrl, horizon, ws=ws, J=J, stats=stats)
    E.gradient(ctrl, J, p.precision, ws=gws, g=g)
    return st


def measure_copy(torch, E, nbytes, reps=20):
    """The library's streaming copy over `nbytes` (read + write), timed with HIP events; the mean
    and the spread of three blocks of `reps` copies."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        E.stream_copy(src, dst)
    rates = []
    for _ in range(3):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            E.stream_copy(src, dst)
        ev1.record()
        torch.cuda.synchronize()
        rates.append(2 * nbytes * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9)
    del src, dst
    return {"GBs": round(float(np.mean(rates)), 1), "min_GBs": round(min(rates), 1), "max_GBs": round(max(rates), 1),
            "bytes": nbytes, "frac_of_peak": round(float(np.mean(rates)) / PEAK_HBM_GBS, 4)}


def roofline(st, prec, ncells, copy_gbs=None):
    """The dominant kernel against the HBM roofline: algorithmic bytes of one launch (bytes per
    member-cell x the member-cells the launch covers: the first lane's members) over its mean launch
    time, from HIP events on the stream it is launched on (sampled steps run with the other lane
    held, so the launch is timed alone)."""
    members = st["timed_members"]
    cyc = st["mean_cycles"]
    us_of = {"predictor": st["predictor_us"], "pre": st["pre_us"], "post": st["post_us"], "resid": st["resid_us"]}
    per_step = {"predictor": us_of["predictor"], "pre": us_of["pre"] * cyc, "post": us_of["post"] * cyc}
    if prec == "mixed":  # the refinement residual is formed by the finest pre kernel; one more closes the step
        per_step["resid"] = us_of["resid"]
    per_kernel = {}
    for k in per_step:
        if us_of[k] > 0 and (k, prec) in BYTES_PER_CELL:
            per_kernel[k] = round(BYTES_PER_CELL[(k, prec)] * ncells * members / (us_of[k] * 1e-6) / 1e9, 1)
    name = max(per_step, key=per_step.get)
    avg_us = us_of[name]
    nbytes = BYTES_PER_CELL[(name, prec)] * ncells * members
    achieved = nbytes / (avg_us * 1e-6) / 1e9
    tpc = MEASURED_TRAFFIC_PER_MEMBER_CELL.get((name, prec))
    out = {
        "kernel": {"predictor": "k_predictor (fused with the previous projection)", "pre": "k_mg_pre (finest level)",
                   "post": "k_mg_post (finest level)", "resid": "k_resid64"}[name],
        "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": round(tpc * ncells * members, 1) if tpc else None,
        "frac_of_measured_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
        "members_per_launch": members, "bytes_per_member_cell": BYTES_PER_CELL[(name, prec)],
        "bytes_per_launch": nbytes, "avg_launch_us": round(avg_us, 2),
        "per_step_us": {k: round(v, 1) for k, v in per_step.items()},
        "per_kernel_algorithmic_GBs": per_kernel,
    }
    if name == "predictor":  # the minimal model's bytes for the same launch (predictor + projection + cost)
        sb = MINIMAL_PRED_PROJ[prec] * ncells * members
        out["minimal_bytes_per_member_cell"] = MINIMAL_PRED_PROJ[prec]
        out["minimal_achieved"] = round(sb / (avg_us * 1e-6) / 1e9, 1)
        out["minimal_frac"] = round(sb / (avg_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
    return out


# bytes per cell-step of the whole step (ideal fusion): the fused predictor and, per refinement
# pass, the finest pre kernel (25 B in the first pass, which forms the FP64 residual; 9 B in later
# ones, which start from the carried residual) and post kernel (29 B, which also updates the carried
# residual and its norm) and the coarser tiled levels (~22 B per cell of their level, 1/4 + 1/16 +
# ... of the fine cells); FP64: the predictor and 52 + 44/3 B per V-cycle
def step_bytes(prec, cycles):
    if prec == "mixed":
        return 150.4 + (25.0 + 29.0 + 22.0 / 3.0) + max(cycles - 1.0, 0.0) * (9.0 + 29.0 + 22.0 / 3.0)
    return 166.4 + cycles * (52.0 + 44.0 / 3.0)


def step_roofline(value, prec, cycles, copy_gbs):
    b = step_bytes(prec, cycles)
    at_peak = PEAK_HBM_GBS * 1e9 / b
    sb = MINIMAL_PRED_PROJ[prec] + MINIMAL_PER_CYCLE[prec] * cycles
    return {"bytes_per_cell_step": round(b, 1), "cell_steps_per_s_at_peak": round(at_peak, 1),
            "frac": round(value / at_peak, 4),
            "minimal_bytes_per_cell_step": round(sb, 1), "minimal_frac": round(value * sb / (PEAK_HBM_GBS * 1e9), 4),
            "frac_of_measured_copy": round(value / (copy_gbs * 1e9 / b), 4) if copy_gbs else None}


def uneven_batch(torch, E, inputs, scale, div_tol):
    """Three ensembles of different grids, Reynolds numbers, sizes and horizons in one batch (FP64).

    h = 1/64, 1/128, 1/256 with 32, 64, 128 members (+ centre), Re 4000, 7500, 12000 and horizons
    5k, 10k, 20k steps x `scale`, each from a short spin-up of its own, every ensemble solved to
    the same divergence bound. Reported: cell-steps/s of the batch and of the same three ensembles
    run one after the other (each alone, single lane), and the batch's lane plan.
    """
    spec = [(64, 4000.0, 32, 5000), (128, 7500.0, 64, 10000), (256, 12000.0, 128, 20000)]
    jobs, solo, work = [], [], 0
    for n, Re, N, hz in spec:
        p = E.Problem(inv_h=n, Re=Re, precision=E.FP64, div_tol=div_tol)
        p1 = E.Problem(inv_h=n, Re=Re, precision=E.FP64, div_tol=div_tol, flags=E.FLAG_ONE_LANE)
        u0, v0 = inputs.initial_field(n, amp=1e-3)
        state = E.state_init(p, u0, v0)
        E.spinup(p, state, 100)
        rows = np.vstack([np.zeros(E.control_dim(p)), inputs.grf_perturbations(N, n, ELL, SIGMA)])
        H = max(1, int(round(hz * scale)))
        jobs.append((p, state, torch.tensor(rows, device="cuda"), H))
        solo.append(p1)
        work += E.cell_count(p) * (N + 1) * H
    E.forward_batch([(p, s_, c, 20) for (p, s_, c, _) in jobs])  # tune every shape, warm the graphs
    for p1, (_, s_, c, _) in zip(solo, jobs):
        E.forward(p1, s_, c, 20, stats=False)
    torch.cuda.synchronize()
    t = time.time()
    out = E.forward_batch(jobs)
    torch.cuda.synchronize()
    tb = time.time() - t
    t = time.time()
    Js = []
    for p1, (p, s_, c, H) in zip(solo, jobs):
        Js.append(E.forward(p1, s_, c, H, stats=False)[0])
    torch.cuda.synchronize()
    ts = time.time() - t
    same = all(np.array_equal(o[0].cpu().numpy(), J.cpu().numpy()) for o, J in zip(out, Js))
    return {"ensembles": [{"inv_h": n, "Re": Re, "members": N + 1, "horizon": j[3], "mean_vcycles":
                           round(o[1]["mean_cycles"], 3), "unconverged": o[1]["unconverged"]}
                          for (n, Re, N, _), j, o in zip(spec, jobs, out)],
            "horizon_scale": scale, "div_tol": div_tol,
            "cell_steps": work, "batched_cell_steps_per_s": round(work / tb, 1),
            "sequential_cell_steps_per_s": round(work / ts, 1), "speedup": round(ts / tb, 3),
            "J_batched_equals_sequential": bool(same),
            "all_J_finite": bool(all(np.all(np.isfinite(o[0].cpu().numpy())) for o in out))}


def config2_iterate(torch, E, inputs, state, ctrl, horizon, iters, div_tol):
    """The fixed-ensemble descent of Fig. envar_loop at working size in FP64: h = 1/128, N = 64
    perturbations held fixed, `iters` iterations over a `horizon`-step window, the step size found
    by an Armijo search at every iteration (Fig. envar_loop; reusing the first iteration's step, the
    other reading of a "fixed" step, lets J rise again once |g| has shrunk, measured 4.03e-5 ->
    3.91e-5 -> 4.18e-5 over ten iterations). The descent starts from a seeded forcing (GRF, length
    0.05, std 0.05): from f = 0 the one-sided differences of a cost without a forcing-driven
    component give no descent direction the first line search accepts."""
    p = E.Problem(inv_h=INV_H, Re=RE, precision=E.FP64, div_tol=div_tol)
    pert = (ctrl[1:] - ctrl[0]).contiguous()
    f = torch.tensor(inputs.grf_perturbations(1, INV_H, ELL, 0.05, seed=99)[0], device="cuda")
    E.iterate(p, state, f.clone(), pert, 20, iters=1)  # tune and warm at this shape
    torch.cuda.synchronize()
    t = time.time()
    recs = []
    for it in range(iters):  # one call per iteration, so that a long window logs its progress
        r = E.iterate(p, state, f, pert, horizon, iters=1, search_every=1)
        torch.cuda.synchronize()
        recs += r
        log(f"  config-2 iteration {it}: {r[-1] if r else None} ({time.time() - t:.1f} s in)")
        if not r or not (r[-1]["alpha"] > 0.0):  # the line search found no decrease: the descent ends
            break
    dt = time.time() - t
    cells = E.cell_count(p)
    return {"inv_h": INV_H, "members": pert.shape[0], "horizon": horizon, "iterations": len(recs),
            "line_search": "Armijo every iteration", "div_tol": div_tol, "seconds": round(dt, 2), "s_per_iteration": round(dt / max(1, len(recs)), 3),
            "forward_cell_steps_per_s": round(cells * (pert.shape[0] + 1) * horizon * len(recs) / dt, 1),
            "records": [{k: (None if v != v else float(v)) for k, v in r.items()} for r in recs],
            "J0_first_last": [recs[0]["J0"], recs[-1]["J0"]]}


def gauss_newton(torch, E, pm, state, ctrl, horizon, every=10):
    """Vector-observation EnVar at the benchmark shape: the cost of recording the lid sensors during
    the forward (mixed, `horizon` steps, with and without), then one Gauss-Newton step and the
    posterior variance for the series length of the full horizon (20,000 steps sampled every
    `every`: K = 2,000 per channel), timed on the device with synthetic series of that shape."""
    nrows, m = ctrl.shape
    ws = E._bytes_tensor(E.workspace_bytes(pm, nrows))
    E.forward(pm, state, ctrl, 20, ws=ws, stats=False)
    E.forward_obs(pm, state, ctrl, 20, ws=ws, stats=False)
    torch.cuda.synchronize()
    t = time.time()
    E.forward(pm, state, ctrl, horizon, ws=ws, stats=False)
    torch.cuda.synchronize()
    t_plain = time.time() - t
    t = time.time()
    E.forward_obs(pm, state, ctrl, horizon, ws=ws, stats=False)
    torch.cuda.synchronize()
    t_obs = time.time() - t
    K = 20000 // every
    g = torch.Generator(device="cuda").manual_seed(3)
    series = 3.0 + torch.randn((nrows, E.OBS_CHANNELS, K), dtype=torch.float64, device="cuda", generator=g)
    series[1:] = series[0] + 1e-4 * torch.randn((nrows - 1, E.OBS_CHANNELS, K), dtype=torch.float64,
                                                device="cuda", generator=g)
    w = torch.zeros(nrows - 1, dtype=torch.float64, device="cuda")
    gws = E._bytes_tensor(E.lib().envar_gn_bytes(nrows - 1, K))
    dw, H, jw = E.gn_step(series, 1e-4, w, ws=gws)
    E.posterior_var(ctrl, 1e-4, H)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(5):
        dw, H, jw = E.gn_step(series, 1e-4, w, ws=gws)
    e1.record()
    for _ in range(5):
        E.posterior_var(ctrl, 1e-4, H)
    e2.record()
    torch.cuda.synchronize()
    return {"sensor_recording_us_per_step": round((t_obs - t_plain) / horizon * 1e6, 2),
            "forward_us_per_step": round(t_plain / horizon * 1e6, 1),
            "gn_step_us": round(e0.elapsed_time(e1) * 1e3 / 5, 1), "posterior_variance_us": round(e1.elapsed_time(e2) * 1e3 / 5, 1),
            "members": nrows - 1, "samples_per_channel": K, "n_obs": E.OBS_CHANNELS * K, "m": m}


def ens_loop(torch, E, p64, state, ctrl, horizon, every=10):
    """One iteration of the EnVar loop over the ensemble weights at the benchmark shape (FP64:
    the finite differences of eq. fdapprox need it): Gauss-Newton, and L-BFGS with its Armijo
    trials batched as rows of one forward and one at a time, against the n + 1 forwards with
    sensors alone."""
    nrows, m = ctrl.shape
    fe = ctrl[0].contiguous()
    Ed = (ctrl[1:] - ctrl[0]).contiguous()
    ws = E._bytes_tensor(E.ens_bytes(p64, nrows - 1, m, horizon, every))
    fws = E._bytes_tensor(E.workspace_bytes(p64, nrows))
    def best_of(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            t = time.time()
            r = fn()
            torch.cuda.synchronize()
            best = min(best or 1e30, time.time() - t)
        return best, r

    t_fwd, _ = best_of(lambda: E.forward_obs(p64, state, ctrl, horizon, every, ws=fws, stats=False))
    del fws
    out = {"members": nrows - 1, "horizon": horizon, "every": every,
           "forwards_with_sensors_ms": round(t_fwd * 1e3, 1)}
    for name, method, tb in (("gn", E.GN, 8), ("lbfgs", E.LBFGS, 8), ("lbfgs_one_trial_per_forward", E.LBFGS, 1)):
        dt, (_, rec) = best_of(lambda: E.ens_iterate(p64, state, fe, Ed, horizon, iters=1, method=method,
                                                      every=every, trial_batch=tb, ws=ws))
        out[f"{name}_iteration_ms"] = round(dt * 1e3, 1)
        if method == E.LBFGS:
            out[f"{name}_trials"] = rec[0]["trials"]
            out[f"{name}_trial_rows"] = rec[0]["trial_rows"]
    out["gn_overhead_beyond_forwards_ms"] = round(out["gn_iteration_ms"] - out["forwards_with_sensors_ms"], 1)
    return out


def eigen_ensemble(torch, E):
    """Deterministic eigen-ensemble (tapered Gaussian covariance of Sec. 4.2) over the benchmark's
    control region (h = 1/128 column, 32,768 cells) for 20 (the paper's) and 64 members; the
    matrix-core work per subspace iteration is 2 b M (nx + ny) (B applied through the separable
    kernel) + 2 M (2b)^2 (Gram of [Q; BQ]) + 6 b^2 M (Ritz rotations and the next block) flops."""
    p = E.Problem(inv_h=INV_H, region=E.REGION_COLUMN)
    nx, ny = INV_H, 2 * INV_H
    M = nx * ny
    out = []
    for N in (20, 64):
        E.eigen_ensemble(p, N)
        torch.cuda.synchronize()
        t = time.time()
        _, mu, info = E.eigen_ensemble(p, N)
        torch.cuda.synchronize()
        dt = time.time() - t
        b = info["block"]
        flops = info["iters"] * (2.0 * b * M * (nx + ny) + 2.0 * M * (2 * b) ** 2 + 6.0 * b * b * M)
        out.append({"members": N, "block": b, "iterations": info["iters"], "converged": info["converged"],
                    "max_resid": info["max_resid"], "ms": round(dt * 1e3, 1),
                    "ms_per_iteration": round(dt * 1e3 / info["iters"], 3),
                    "matrix_core_tflops": round(flops / dt / 1e12, 2), "fp64_peak_tflops": 78.6,
                    "mu_N_over_mu_1": float(mu[-1] / mu[0])})
    return out


def paper_geometry(torch, E, inputs):
    """The paper's configuration (channel height 1/2, uniform inflow, slip top and outer lower wall,
    y-only forcing on the actuation window): the batched mixed forward at the benchmark shape
    (65 members, h = 1/128, 200 steps), and a regime check at h = 1/64 for Re = 6250 and 14000 (one
    member from rest plus noise, 40 time units of spin-up, then the lid sensors over 20 time units:
    rms of the transverse velocity and the dominant frequency of the most downstream sensor)."""
    window = (1.25 - 0.32, 1.25 + 0.15, -0.60, 0.15)
    out = {}
    pm = E.Problem(inv_h=INV_H, Re=6250.0, precision=E.MIXED, geometry=E.CAVITY_PAPER, region=E.REGION_BOX,
                   box=window)
    u0, v0 = inputs.initial_field(INV_H, amp=1e-3, geometry="paper")
    state = E.state_init(pm, u0, v0)
    E.spinup(pm, state, 2000)
    m = E.control_dim(pm)
    rng = np.random.default_rng(11)
    rows = np.zeros((N_MEMBERS + 1, m))
    rows[1:, m // 2:] = 1e-2 * rng.standard_normal((N_MEMBERS, m // 2))
    ctrl = torch.tensor(rows, device="cuda")
    ws = E._bytes_tensor(E.workspace_bytes(pm, N_MEMBERS + 1))
    E.forward(pm, state, ctrl, 20, ws=ws, stats=False)
    torch.cuda.synchronize()
    t = time.time()
    _, _, st = E.forward(pm, state, ctrl, 200, ws=ws)
    torch.cuda.synchronize()
    dt = time.time() - t
    ncells = E.cell_count(pm)
    out["cells"] = ncells
    out["mixed_batched_cell_steps_per_s"] = round(ncells * (N_MEMBERS + 1) * 200 / dt, 1)
    out["mean_vcycles_per_step"] = round(st["mean_cycles"], 3)
    regimes = []
    n = 64
    for Re in (6250.0, 14000.0):
        p = E.Problem(inv_h=n, Re=Re, precision=E.FP64, geometry=E.CAVITY_PAPER, region=E.REGION_BOX, box=window)
        u0, v0 = inputs.initial_field(n, amp=1e-2, geometry="paper")
        stt = E.state_init(p, u0, v0)
        steps_per_unit = int(round(1.0 / (0.064 / n)))
        t = time.time()
        E.spinup(p, stt, 40 * steps_per_unit)
        every = 10
        horizon = 20 * steps_per_unit
        _, series, _ = E.forward_obs(p, stt, torch.zeros((1, E.control_dim(p)), dtype=torch.float64, device="cuda"),
                                     horizon, every)
        torch.cuda.synchronize()
        s = series.cpu().numpy()[0]
        vy = s[7] - s[7].mean()  # v at the most downstream sensor
        spec = np.abs(np.fft.rfft(vy)) ** 2
        freq = np.fft.rfftfreq(vy.size, d=every * 0.064 / n)
        k = int(np.argmax(spec[1:])) + 1
        regimes.append({"Re": Re, "inv_h": n, "sensor_v_rms": float(np.sqrt(np.mean(vy ** 2))),
                        "dominant_frequency": float(freq[k]), "seconds": round(time.time() - t, 2)})
    out["regimes"] = regimes
    return out


def gram_sweep(torch, E):
    """Anomaly reduction (Gram X X^T on the matrix cores, Cholesky, X^T c) timed on the device.

    TFLOP/s counts the Gram's 2 N^2 m flops against the whole reduction's time (a lower bound for
    the Gram kernel), against the dense MFMA peak of the precision: FP32 157.3, FP64 78.6 TFLOP/s.
    """
    out = []
    rng = torch.Generator(device="cuda").manual_seed(5)
    for N, m in ((64, 65536), (256, 65536), (256, 262144)):
        ctrl = torch.randn((N + 1, m), dtype=torch.float64, device="cuda", generator=rng)
        J = torch.randn(N + 1, dtype=torch.float64, device="cuda", generator=rng)
        for prec, name, peak in ((E.MIXED, "fp32_mfma", 157.3), (E.FP64, "fp64_mfma", 78.6)):
            gws = E._bytes_tensor(E.gradient_bytes(N, m, prec))
            g = torch.empty(m, dtype=torch.float64, device="cuda")
            E.gradient(ctrl, J, prec, ws=gws, g=g)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                E.gradient(ctrl, J, prec, ws=gws, g=g)
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / 5
            tf = 2.0 * N * N * m / sec / 1e12
            out.append({"N": N, "m": m, "precision": name, "us": round(sec * 1e6, 1), "gram_TFLOPs": round(tf, 2),
                        "frac_of_peak": round(tf / peak, 4)})
    return out


def serving(torch, E, inputs, nreq, horizon_scale, div_tol, clients=4, think_s=0.02, seed=2605238125):
    """Forward-solve requests from `clients` concurrent EnVar optimisations, each a closed loop.

    Every request draws h in {1/64, 1/128, 1/256}, Re in {4000, 7500, 12000}, N in {16, 32, 64,
    128} and a horizon in {2k, 5k, 10k} steps (x horizon_scale) from a seeded generator; request k
    belongs to optimisation k mod `clients`, which submits it an exponential think time (mean
    `think_s`, seeded) after the result of its previous request arrives (the next iteration of the
    loop of Sec. 3.3.3 needs the costs of the previous one). Two servers get the same request
    streams: the continuous-batching server in mixed precision (requests join and leave the
    running batch, up to 8 at once) and a queue-then-plain-FP64 server (one request at a time,
    FIFO), both solving to the same divergence bound. Reported for each: throughput (cell-steps
    over the makespan) and p50/p99 latency (submission to result, over all requests)."""
    import threading

    rng = np.random.default_rng(seed)
    grids, res, sizes = [64, 128, 256], [4000.0, 7500.0, 12000.0], [16, 32, 64, 128]
    horizons = [max(1, int(round(hz * horizon_scale))) for hz in (2000, 5000, 10000)]
    states, pools = {}, {}
    for n in grids:
        pools[n] = inputs.grf_perturbations(8, n, ELL, SIGMA, seed=seed + n)
        for Re in res:
            p64 = E.Problem(inv_h=n, Re=Re)
            u0, v0 = inputs.initial_field(n, amp=1e-3)
            st = E.state_init(p64, u0, v0)
            E.spinup(p64, st, 200)
            states[(n, Re)] = st
    torch.cuda.synchronize()
    reqs = []
    for k in range(nreq):
        n, Re = int(rng.choice(grids)), float(rng.choice(res))
        N, hz = int(rng.choice(sizes)), int(rng.choice(horizons))
        pick = rng.integers(0, 8, size=N)
        scale = rng.uniform(0.5, 1.5, size=(N, 1))
        rows = np.vstack([np.zeros(pools[n].shape[1]), pools[n][pick][1:] * scale[1:]])
        reqs.append(dict(opt=k % clients, n=n, Re=Re, rows=rows, horizon=hz, cells=5 * n * n))
    think = rng.exponential(think_s, size=nreq)
    work = sum(r["cells"] * r["rows"].shape[0] * r["horizon"] for r in reqs)

    def run(precision, max_jobs):
        srv = E.Server(96 << 30, max_jobs=max_jobs, precision=precision)
        results = [None] * nreq
        errors = []
        t0 = time.time()

        def client(c):
            try:
                for k in range(c, nreq, clients):
                    time.sleep(think[k])
                    r = reqs[k]
                    p = E.Problem(inv_h=r["n"], Re=r["Re"], precision=precision, div_tol=div_tol)
                    t = srv.submit(p, states[(r["n"], r["Re"])], r["rows"], r["horizon"])
                    results[k] = srv.wait(t, timeout=900.0)
                    log(f"  serving {'mixed' if precision == E.MIXED else 'fp64'}: request {k} done "
                        f"(latency {results[k][1]['latency_s']:.2f} s, {time.time() - t0:.1f} s in)")
            except Exception as e:  # reported below
                errors.append(repr(e))
        try:
            th = [threading.Thread(target=client, args=(c,)) for c in range(clients)]
            for x in th:
                x.start()
            for x in th:
                x.join()
            makespan = time.time() - t0
        finally:
            srv.close()
        if errors:
            raise RuntimeError("serving client failed: " + errors[0])
        lat = np.array([r[1]["latency_s"] for r in results])
        return {
            "throughput_cell_steps_per_s": round(work / makespan, 1), "makespan_s": round(makespan, 2),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "max_latency_s": round(float(lat.max()), 4),
            "peak_concurrent_requests": int(max(r[1]["peak_jobs"] for r in results)),
            "statuses_ok": int(sum(r[1]["status"] == E.OK for r in results)),
            "unconverged_member_steps": int(sum(r[1]["unconverged"] for r in results)),
            "max_div": float(max(r[1]["max_div"] for r in results)),
            "all_J_finite": bool(all(np.all(np.isfinite(r[0])) for r in results)),
        }, [r[0] for r in results]

    mixed, Jm = run(E.MIXED, 8)
    log("serving mixed", mixed)
    fp64, J64 = run(E.FP64, 1)
    log("serving fp64 queue", fp64)
    rel = max(float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(Jm, J64))
    return {
        "requests": nreq, "clients": clients, "think_time_mean_s": think_s, "horizon_scale": horizon_scale,
        "horizons": horizons, "div_tol": div_tol, "cell_steps": work,
        "throughput_cell_steps_per_s": mixed["throughput_cell_steps_per_s"],
        "p50_latency_s": mixed["p50_latency_s"], "p99_latency_s": mixed["p99_latency_s"],
        "continuous_batching_mixed": mixed,
        "baseline_queue_fp64": fp64,
        "speedup_throughput": round(mixed["throughput_cell_steps_per_s"] / fp64["throughput_cell_steps_per_s"], 3),
        "J_rel_err_mixed_vs_fp64_max": rel,
        "note": "p99 over the requests' latencies (linear interpolation between the two largest of "
                f"{nreq})",
    }


def lyapunov(torch, E, inputs, n, Re, geometry, spin_units, window_units, every=20, eps=1e-10, seed=5):
    """Leading Lyapunov exponent from twin FP64 runs: the unforced flow and the same flow forced by
    eps times a unit-max GRF field (length 0.05), integrated together from a spun-up state; the
    separation of their lid-sensor signals (8 channels, every `every` steps) grows like e^(lambda
    t) until it saturates at the signal's own size. lambda is the least-squares slope of
    log(separation) over the samples whose separation lies between 1e3 times its first value and
    1e-2 of the signal's standard deviation."""
    geo = E.CAVITY_PAPER if geometry == "paper" else E.CAVITY
    p = E.Problem(inv_h=n, Re=Re, precision=E.FP64, geometry=geo)
    dt = p.step_dt
    u0, v0 = inputs.initial_field(n, amp=1e-3, seed=seed, geometry=geometry)
    state = E.state_init(p, u0, v0)
    t = time.time()
    E.spinup(p, state, int(round(spin_units / dt)))
    m = E.control_dim(p)
    shape = (n + n // 2, n) if geometry == "paper" else None
    pert = inputs.grf_perturbations(1, n, 0.05, 1.0, seed=seed + 1, shape=shape)[0]
    rows = np.vstack([np.zeros(m), eps * pert / np.abs(pert).max()])
    H = int(round(window_units / dt))
    _, series, st = E.forward_obs(p, state, torch.tensor(rows, device="cuda"), H, every)
    torch.cuda.synchronize()
    secs = time.time() - t
    S = series.cpu().numpy()
    d = np.sqrt(((S[1] - S[0]) ** 2).sum(axis=0))
    scale = float(np.sqrt(((S[0] - S[0].mean(axis=1, keepdims=True)) ** 2).sum(axis=0).mean()))
    tt = (np.arange(S.shape[2]) + 1) * every * dt
    d0 = float(d[:5].mean())
    sel = (d > 1e3 * d0) & (d < 1e-2 * scale)
    first = int(np.argmax(sel)) if sel.any() else 0
    sat = np.nonzero(d >= 1e-2 * scale)[0]
    last = int(sat[0]) if sat.size else d.size
    idx = np.arange(first, last)
    idx = idx[d[idx] > 1e3 * d0]
    out = {"inv_h": n, "Re": Re, "geometry": geometry, "spinup_time_units": spin_units,
           "window_time_units": window_units, "eps": eps, "samples": int(d.size), "seconds": round(secs, 1),
           "separation_first": d0, "separation_last": float(d[-1]), "signal_std": scale,
           "mean_vcycles": round(st["mean_cycles"], 3)}
    if idx.size >= 10:
        lam, c = np.polyfit(tt[idx], np.log(d[idx]), 1)
        res = np.log(d[idx]) - (lam * tt[idx] + c)
        out.update({"lambda": float(lam), "lyapunov_time": float(1.0 / lam) if lam > 0 else None,
                    "fit_from_t": float(tt[idx[0]]), "fit_to_t": float(tt[idx[-1]]),
                    "fit_rms_log_residual": float(np.sqrt(np.mean(res ** 2))),
                    "saturated_at_t": float(tt[last]) if last < d.size else None})
    else:
        out.update({"lambda": None, "lyapunov_time": None,
                    "note": "no exponential regime: the separation never grew 1e3-fold below saturation"})
    # log-separation every ~2 time units, for the record
    stride = max(1, int(round(2.0 / (every * dt))))
    out["log10_separation_every_2_units"] = [round(float(np.log10(max(x, 1e-300))), 2) for x in d[::stride]]
    return out


def cpu_baseline(state_host, rows, steps, procs):
    """The oracle (plain FP64 numpy/scipy) on a bounded sample: every member for `steps` steps."""
    from oracle import envar as OE

    op = OE.Problem(inv_h=INV_H, Re=RE)
    op.poisson()  # factorise once, shared by the forked workers
    u, v, tu, tv = state_host
    from oracle import ns

    base = ns.State(u, v, tu, tv)
    t = time.time()
    Jo = OE.forward(op, base, rows, steps, processes=procs)
    dt = time.time() - t
    ncells = op.grid().ncells
    return ncells * steps * rows.shape[0] / dt, dt, Jo


def accuracy_at_horizon(torch, E, state, ctrl, horizon, J_mixed, g_mixed, ws64, gws64, flags):
    """J and g of the timed mixed-precision pass against a GPU FP64 reference over the same full
    horizon (div_tol 1e-12; the FP64 path itself matches the oracle within 1e-10 on the tested
    horizons), and the FP64 path at the headline's own bound (1e-10) against the same reference.
    The FP64 run at 1e-10 is also the equal-tolerance FP64 batched rate over the full horizon."""
    nrows, m = ctrl.shape
    pref = E.Problem(inv_h=INV_H, Re=RE, precision=E.FP64, div_tol=DIV_TOL_REF, flags=flags)
    peq = E.Problem(inv_h=INV_H, Re=RE, precision=E.FP64, div_tol=DIV_TOL, flags=flags | E.FLAG_TIME_KERNELS)
    Jr, _, st_ref = E.forward(pref, state, ctrl, horizon, ws=ws64)
    gr = E.gradient(ctrl, Jr, E.FP64, ws=gws64).cpu().numpy()
    Jr = Jr.cpu().numpy()
    torch.cuda.synchronize()
    t = time.time()
    Je, _, st_eq = E.forward(peq, state, ctrl, horizon, ws=ws64)
    torch.cuda.synchronize()
    t_eq = time.time() - t
    ge = E.gradient(ctrl, Je, E.FP64, ws=gws64).cpu().numpy()
    Je = Je.cpu().numpy()

    def cmp(J, g):
        return {"J_rel_err_max": float(np.max(np.abs(J - Jr) / np.abs(Jr))),
                "g_cosine": float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr))),
                "g_rel_err": float(np.linalg.norm(g - gr) / np.linalg.norm(gr))}
    out = {"horizon": horizon, "members": nrows,
           "reference": f"GPU FP64 forward + FP64-MFMA gradient, div_tol {DIV_TOL_REF:g}",
           "reference_mean_vcycles": round(st_ref["mean_cycles"], 3),
           "mixed_div_tol_1e-10": cmp(J_mixed, g_mixed),
           "fp64_div_tol_1e-10": cmp(Je, ge)}
    return out, st_eq, t_eq


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--horizon", type=int, default=20000)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--oracle-steps", type=int, default=200)
    ap.add_argument("--oracle-members", type=int, default=8, help="perturbed members of the oracle check (+ centre)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--no-graphs", action="store_true", help="launch every step eagerly (profiler counter passes)")
    ap.add_argument("--one-lane", action="store_true", help="run every member on one stream (no member lanes)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-horizon-scale", type=float, default=0.2)
    ap.add_argument("--uneven-scale", type=float, default=0.1, help="horizon scale of the uneven batch (0: skip)")
    ap.add_argument("--iterate-horizon", type=int, default=1000, help="window of the FP64 descent (0: skip)")
    ap.add_argument("--iterate-iters", type=int, default=10)
    ap.add_argument("--no-gram", action="store_true")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving comparison and print it as one JSON line")
    ap.add_argument("--anomaly-only", action="store_true",
                    help="run only the anomaly-reduction sweep and print it as one JSON line (for kernel traces)")
    ap.add_argument("--lyapunov", action="store_true",
                    help="only measure the leading Lyapunov exponent of the chaotic configurations (twin FP64 "
                         "runs) and print them as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the ensemble members of one MI355X "
              "(sharding the members over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2605_23812_amd import envar as E
    from paper_2605_23812_amd import inputs

    E.lib()
    torch.cuda.init()
    if args.anomaly_only:
        print(json.dumps({"anomaly_reduction": gram_sweep(torch, E)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving(torch, E, inputs, args.serve_requests, args.serve_horizon_scale,
                                             DIV_TOL)}), flush=True)
        return
    if args.lyapunov:
        res = []
        for cfg in ((256, 12000.0, "cavity", 20.0, 80.0), (128, 12000.0, "cavity", 20.0, 80.0),
                    (64, 14000.0, "paper", 40.0, 150.0), (64, 12000.0, "cavity", 40.0, 150.0)):
            r = lyapunov(torch, E, inputs, *cfg)
            log("lyapunov", r)
            res.append(r)
        print(json.dumps({"lyapunov": res}), flush=True)
        return
    copy = measure_copy(torch, E, args.copy_bytes)
    copy_gbs = copy["GBs"]
    log(f"stream copy: {copy}")
    gflag = (E.FLAG_NO_GRAPHS if args.no_graphs else 0) | (E.FLAG_ONE_LANE if args.one_lane else 0)
    state, ctrl, m = build_inputs(torch, E, inputs, gflag)
    nrows = ctrl.shape[0]
    pm = E.Problem(inv_h=INV_H, Re=RE, precision=E.MIXED, div_tol=DIV_TOL, flags=E.FLAG_TIME_KERNELS | gflag)
    ncells = E.cell_count(pm)
    ws = E._bytes_tensor(E.workspace_bytes(pm, nrows))
    gws = E._bytes_tensor(E.gradient_bytes(nrows - 1, m, E.MIXED))
    J = torch.empty(nrows, dtype=torch.float64, device="cuda")
    g = torch.empty(m, dtype=torch.float64, device="cuda")

    for w in range(args.warmup):
        t = time.time()
        one_pass(E, pm, state, ctrl, args.horizon, ws, J, gws, g)
        torch.cuda.synchronize()
        log(f"warmup pass {w}: {time.time() - t:.2f}s")
    torch.cuda.synchronize()
    t0 = time.time()
    st = None
    for k in range(args.steps):
        st = one_pass(E, pm, state, ctrl, args.horizon, ws, J, gws, g, stats=(k == args.steps - 1))
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    cell_steps = ncells * nrows * args.horizon * args.steps
    value = cell_steps / elapsed
    log(f"timed {args.steps} pass(es): {elapsed:.2f}s -> {value:.4g} cell-steps/s; stats {st}")
    J_mixed_long = J.cpu().numpy().copy()
    g_mixed_long = g.cpu().numpy().copy()
    del ws

    extra = {}
    st_eq = None
    if not args.no_accuracy:
        ws64 = E._bytes_tensor(E.workspace_bytes(E.Problem(inv_h=INV_H, Re=RE), nrows))
        gws64 = E._bytes_tensor(E.gradient_bytes(nrows - 1, m, E.FP64))
        acc, st_eq, t_eq = accuracy_at_horizon(torch, E, state, ctrl, args.horizon, J_mixed_long, g_mixed_long,
                                               ws64, gws64, gflag)
        del ws64, gws64
        extra["accuracy_at_horizon"] = acc
        log("accuracy at the full horizon", acc)
    if not args.no_baselines:
        # plain FP64 one member at a time (the same kernels with one row, hence one lane) at the headline's
        # divergence bound, over the full horizon for the centre run
        p1 = E.Problem(inv_h=INV_H, Re=RE, precision=E.FP64, div_tol=DIV_TOL, flags=gflag)
        ws1 = E._bytes_tensor(E.workspace_bytes(p1, 1))
        c0 = ctrl[0:1].contiguous()
        E.forward(p1, state, c0, 40, ws=ws1, stats=False)
        torch.cuda.synchronize()
        t = time.time()
        E.forward(p1, state, c0, args.horizon, ws=ws1, stats=False)
        torch.cuda.synchronize()
        rate_1 = ncells * args.horizon / (time.time() - t)
        del ws1
        base = {"div_tol": DIV_TOL, "horizon": args.horizon,
                "fp64_one_at_a_time_cell_steps_per_s": round(rate_1, 1),
                "speedup_mixed_batched_vs_fp64_one_at_a_time": round(value / rate_1, 2)}
        if st_eq is not None:
            rate_64 = ncells * nrows * args.horizon / t_eq
            base.update({
                "fp64_batched_cell_steps_per_s": round(rate_64, 1),
                "speedup_fp64_batched_vs_fp64_one_at_a_time": round(rate_64 / rate_1, 2),
                "speedup_mixed_batched_vs_fp64_batched": round(value / rate_64, 3),
                "fp64_mean_vcycles_per_step": round(st_eq["mean_cycles"], 3),
                "fp64_roofline": roofline(st_eq, "fp64", ncells, copy_gbs),
                "fp64_step_roofline": step_roofline(rate_64, "fp64", st_eq["mean_cycles"], copy_gbs),
            })
        extra["equal_tolerance_baselines"] = base
        log("baselines", base)

    if args.uneven_scale > 0:
        extra["uneven_batch_fp64"] = uneven_batch(torch, E, inputs, args.uneven_scale, DIV_TOL)
        log("uneven batch", extra["uneven_batch_fp64"])
    if args.iterate_horizon > 0:
        extra["config2_descent_fp64"] = config2_iterate(torch, E, inputs, state, ctrl, args.iterate_horizon,
                                                        args.iterate_iters, DIV_TOL_REF)
        log("config-2 descent", extra["config2_descent_fp64"])
    if not args.no_gram:
        extra["anomaly_reduction"] = gram_sweep(torch, E)
        log("anomaly reduction", extra["anomaly_reduction"])
        extra["gauss_newton"] = gauss_newton(torch, E, pm, state, ctrl, 200)
        log("gauss newton", extra["gauss_newton"])
        p64 = E.Problem(inv_h=INV_H, Re=RE, precision=E.FP64, flags=gflag)
        extra["ens_loop_fp64"] = ens_loop(torch, E, p64, state, ctrl, 200)
        log("EnVar loop", extra["ens_loop_fp64"])
        extra["eigen_ensemble"] = eigen_ensemble(torch, E)
        log("eigen ensemble", extra["eigen_ensemble"])
        extra["paper_geometry"] = paper_geometry(torch, E, inputs)
        log("paper geometry", extra["paper_geometry"])

    serve = None
    if not args.no_serve:
        serve = serving(torch, E, inputs, args.serve_requests, args.serve_horizon_scale, DIV_TOL)
        log("serving", serve)

    cpu = None
    if not args.no_cpu:
        from oracle import envar as OE

        u, v, tu, tv, _ = E.state_read(E.Problem(inv_h=INV_H, Re=RE), state)
        # one process per member, at most the host share of one GPU (16 cores)
        procs = min(16, os.cpu_count() or 1)
        rows = ctrl.cpu().numpy()
        rate, secs, _ = cpu_baseline((u, v, tu, tv), rows, args.cpu_steps, procs)
        cpu = {"value": round(rate, 1), "unit": "cell-steps/s", "cores": procs, "kind": "oracle",
               "host_cpu_count": os.cpu_count(),
               "sample": f"all {nrows} members x {args.cpu_steps} steps of the same h=1/128 workload "
                         f"from the same base state ({secs:.1f}s wall, one process per member, "
                         f"{procs} at a time)"}
        log("cpu baseline", cpu)
        # the oracle against the GPU on a longer horizon: the centre and the first members
        k = args.oracle_members + 1
        sub = rows[:k]
        _, secs_o, Jo = cpu_baseline((u, v, tu, tv), sub, args.oracle_steps, min(procs, k))
        go = OE.gradient(sub, Jo)
        csub = ctrl[:k].contiguous()
        check = {"sample": f"centre + {k - 1} members x {args.oracle_steps} steps ({secs_o:.1f}s of oracle)"}
        for prec, name, tol in ((E.FP64, "fp64", DIV_TOL_REF), (E.MIXED, "mixed", DIV_TOL)):
            pp = E.Problem(inv_h=INV_H, Re=RE, precision=prec, div_tol=tol, flags=gflag)
            Jg, _, _ = E.forward(pp, state, csub, args.oracle_steps)
            gg = E.gradient(csub, Jg, prec).cpu().numpy()
            jg = Jg.cpu().numpy()
            check[name] = {"div_tol": tol, "J_rel_err_max": float(np.max(np.abs(jg - Jo) / np.abs(Jo))),
                           "g_cosine": float(gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go))),
                           "g_rel_err": float(np.linalg.norm(gg - go) / np.linalg.norm(go))}
        extra["oracle_check"] = check
        log("oracle check", check)

    out = {
        "metric": "ensemble cell-steps/s, batched FP32 vs plain FP64 at J err<=1e-4; p50/p99 solve latency",
        "value": round(value, 1),
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {
            "workload": "open-cavity EnVar forward ensemble + anomaly gradient, h=1/128 (81,920 cells), "
                        "Re=7500, dt=5e-4, centre + 64 GRF members, m=65,536, batched mixed precision",
            "members": nrows, "horizon": args.horizon, "inv_h": INV_H, "Re": RE,
            "spinup_steps": SPINUP, "precision": "fp32 multigrid V-cycles inside fp64 refinement; fp64 state, tendencies and cost",
            "div_tol": DIV_TOL, "lanes": 1 if args.one_lane else 2,
        },
        "mean_refinement_passes_per_step": round(st["mean_cycles"], 3),
        "unconverged_member_steps": st["unconverged"],
        "tile_rows": {"predictor": st["rows_pred"], "projection": st["rows_proj"],
                      "multigrid_levels": [r for r in st["rows_mg"] if r]},
        "max_div": st["max_div"],
        "J_finite": bool(np.all(np.isfinite(J_mixed_long))),
        "roofline": roofline(st, "mixed", ncells, copy_gbs),
        "step_roofline": step_roofline(value, "mixed", st["mean_cycles"], copy_gbs),
        "measured_copy": copy,
        "cpu_baseline": cpu,
        "serving": serve,
    }
    if serve is not None:
        out["p50_latency_s"] = serve["p50_latency_s"]
        out["p99_latency_s"] = serve["p99_latency_s"]
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Throughput benchmark of the DG SRHD hot path on one MI355X.

A step is one SSP-RK3 step (three fused stage kernels: volume + faces + lift +
RK combine + physicality operator + recovery of the next stage's primitives)
over the whole mesh.  Metric: DOF-stage updates per second,
DOF x steps x 3 / seconds, with the state resident in HBM.

Default workload: 2D relativistic Kelvin-Helmholtz, Taub-Matthews EOS,
256x256 elements, p=3 (16 nodes per element, 1,048,576 DOF), FP64, HLL,
physicality operator on.  Extra results on the same JSON line:
  fp32_contract  the 512x512 p=3 Kelvin-Helmholtz mesh in the FP32-contraction
                 form vs the same mesh in FP64 (speedup on the same GPU), and the
                 L1 error of both after 50 steps against the oracle's FP64 run;
  wave1d         the 1D density wave (64 elements, p=2, 100 steps): L1 error of
                 D against the exact translated solution, drift from the oracle;
  random3d       the 3D stress field (64^3 p=2): step 1 from the initial state,
                 then 20 steps with the failure fractions after each;
  adjoint        cost of the checkpointed adjoint of 200 steps (checkpoint every
                 20) relative to the forward run, 128x128 p=2 ideal-gas mesh;
  roofline       the stage kernel against HBM, from algorithmic bytes per
                 DOF-stage (read U^(k), read U^n in stages 2-3, write U^(k+1)).
  shard_share    one GPU's block of the 512x512 p=3 mesh split over 8 GPUs
                 (128x256 elements), FP64 and FP32 form, with the per-stage
                 exchange volume of such a split.
  limiter        the cylindrical blast (512x512 p=2) with the slope limiter on
                 and off: time per step, fraction of elements limited.
  paper_sweep    the paper's KH performance grid: HLL and HLLC, p = 0, 1, 2 with
                 RK1, SSPRK2, SSPRK3 on 256x512 .. 1024x2048 meshes (ideal EOS).
  cpu_baseline   the FP64 CPU oracle on the host cores for a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue model of MI355X: 256 CUs x 4 SIMDs at 2.4 GHz, one wave64 VALU
# instruction per SIMD every 4 cycles (16 lanes) -- the FP64 vector peak of
# 78.6 TFLOP/s is this rate with every instruction an FMA
SIMDS, CLOCK_HZ, VALU_CYCLES_PER_WAVE_INST = 1024, 2.4e9, 4.0
FP64_VECTOR_PEAK = 78.6e12  # FLOP/s, MI355X published FP64 vector rate


def _stage_bytes_per_dof(nvar: int) -> float:
    """Mean algorithmic bytes per DOF over the three stages of one step."""
    return nvar * 8.0 * (2.0 + 2.0 / 3.0)


PROFILE_DIR = os.path.join(ROOT, "profiles")


def _measured_traffic(workload: str):
    """HBM bytes per stage launch from the committed counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for a plain
    copy), or None when there is none or the kernel sources changed since it was taken."""
    from paper_2205_00095_amd import build
    path = os.path.join(PROFILE_DIR, f"k_element_stage_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != build.source_digest():
        return None
    return rec


def _time_run(solver, U, dt, steps, warmup):
    import torch
    solver.run(U, dt, warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    solver.run(U, dt, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / 1e3


def _time_con2prim(solver, U, reps=20):
    import torch
    W = solver.empty()
    solver.con2prim(U, out=W)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        solver.con2prim(U, out=W)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / 1e3 / reps


def _time_rhs(solver, U, reps=20):
    """dg_rhs alone (one fused launch in 1D and 2D: the element kernel recovers its nodes
    and its halo itself; in 3D with p >= 1 a recovery launch and the element kernel)."""
    import torch
    R = solver.empty()
    solver.rhs(U, out=R)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        solver.rhs(U, out=R)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / 1e3 / reps


def _copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second) of a 1 GiB buffer."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    t1.record(stream)
    torch.cuda.synchronize()
    rate = 2.0 * nbytes * reps / (t0.elapsed_time(t1) / 1e3)
    del src, dst
    return rate


def _setup(kind, **over):
    import torch
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import Solver
    cfg = wl.make_config(kind, **over)
    solver = Solver(cfg)
    rho, v, P = wl.initial_primitives(cfg)
    src = torch.from_numpy(wl.pack_primitives(rho, v, P)).cuda()
    U = solver.set_state(src)
    return cfg, solver, U


def adjoint_ratio(reps=2):
    """Checkpointed adjoint (200 steps, checkpoint every 20) of J = int v_y^2 dA on the
    128x128 p=2 ideal-gas Kelvin-Helmholtz mesh: backward time (segment recompute with
    tapes + step adjoints + objective gradient) / forward time (200 steps + checkpoints)."""
    import torch
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.adjoint import Trajectory, VY2
    from paper_2205_00095_amd.solver import Solver
    cfg = wl.make_config("kh_ideal")
    solver = Solver(cfg)
    rho, v, P = wl.initial_primitives(cfg)
    v = v.copy()
    v[1] += wl.kh_perturbation(cfg)
    U0 = solver.set_state(torch.from_numpy(wl.pack_primitives(rho, v, P)).cuda())
    nsteps, dt, k = cfg["steps"], cfg["dt"], 20
    stream = torch.cuda.current_stream()
    best_f = best_b = float("inf")
    for _ in range(reps + 1):
        U = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        UT = Trajectory.apply(U, solver, nsteps, dt, k)
        e1.record(stream)
        J = VY2.apply(UT, solver)
        torch.cuda.synchronize()
        e1b = torch.cuda.Event(enable_timing=True)
        e1b.record(stream)
        J.backward()
        e2.record(stream)
        torch.cuda.synchronize()
        best_f = min(best_f, e0.elapsed_time(e1) / 1e3)
        best_b = min(best_b, e1b.elapsed_time(e2) / 1e3)
    dofs = wl.n_dof(cfg)
    return {"workload": "kh_ideal: 2D 128x128 elements p=2 ideal EOS, 200 steps, checkpoint every 20",
            "forward_s": best_f, "backward_s": best_b, "ratio": best_b / best_f,
            "forward_dof_stage_per_s": dofs * nsteps * 3 / best_f}


def con2prim_study(runs=100):
    """The paper's recovery study (Sec. 3.3) on one MI355X: for each of the 25x25 (gamma, P)
    states (gamma log-spaced in [1, 100], P log-spaced in [1e5, 1e10] Pa, D = 1, c = 3e8),
    a 10x10x10 mesh of p=2 elements (27 points per cell) filled with that state is
    recovered `runs` times by each of the four solvers; reported: recoveries/s per state
    (median, min, max over the grid) and the relative velocity error."""
    import numpy as np
    import torch
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import Solver
    c = 3.0e8
    G, PP = wl.c2p_grid(25, c=c)
    out = {}
    stream = torch.cuda.current_stream()
    for eos, method, name in ((wl.EOS_IDEAL, wl.C2P_NEWTON, "ideal_newton"), (wl.EOS_IDEAL, wl.C2P_QUARTIC, "ideal_quartic"),
                              (wl.EOS_TM, wl.C2P_CUBIC, "tm_cubic"), (wl.EOS_TM, wl.C2P_BRENT, "tm_brent")):
        cfg = wl.make_config("random3d", n_elem=(10, 10, 10), p=2, eos=eos, c2p=method, c=c, precision=wl.FP64)
        s = Solver(cfg)
        n = wl.n_dof(cfg)
        rates, errs, errs10 = [], [], []
        src = torch.empty(s.shape, dtype=torch.float64, device="cuda")
        W = s.empty()
        for g, P in zip(G.ravel(), PP.ravel()):
            beta = np.sqrt((1 - 1 / g) * (1 + 1 / g))
            src[0].fill_(1.0 / g)
            src[1].fill_(beta * c)
            src[2].zero_()
            src[3].zero_()
            src[4].fill_(P)
            U = s.set_state(src)
            s.con2prim(U, out=W)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(runs):
                s.con2prim(U, out=W)
            e1.record(stream)
            torch.cuda.synchronize()
            rates.append(n * runs / (e0.elapsed_time(e1) / 1e3))
            u = W[1:4].reshape(3, -1)[:, 0].double().cpu()
            ux = float(u[0])
            v = ux / np.sqrt(1 + float((u * u).sum()) / c ** 2)
            err = abs(v - beta * c) / (beta * c) if beta > 0 else abs(v)
            errs.append(err)
            if g <= 10:
                errs10.append(err)
        s.close()
        r = np.array(rates)
        out[name] = {"recoveries_per_s_median": float(np.median(r)), "min": float(r.min()), "max": float(r.max()),
                     "vel_rel_err_max": float(max(errs)), "vel_rel_err_max_gamma_le_10": float(max(errs10))}
        # the same 625 states tiled over a 64^3 p=2 mesh (7,077,888 points): one launch is
        # then long enough that the rate is the solver's, not the launch latency's
        big = wl.make_config("random3d", p=2, eos=eos, c2p=method, c=c, precision=wl.FP64)
        sb = Solver(big)
        nb = wl.n_dof(big)
        srcb = torch.empty(sb.shape, dtype=torch.float64, device="cuda").reshape(5, -1)
        gi = torch.arange(nb, device="cuda") % G.size
        gam = torch.from_numpy(G.ravel()).cuda()[gi]
        srcb[0] = 1.0 / gam
        srcb[1] = torch.sqrt((1 - 1 / gam) * (1 + 1 / gam)) * c
        srcb[2].zero_()
        srcb[3].zero_()
        srcb[4] = torch.from_numpy(PP.ravel()).cuda()[gi]
        Ub = sb.set_state(srcb.reshape(sb.shape))
        Wb = sb.empty()
        sb.con2prim(Ub, out=Wb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            sb.con2prim(Ub, out=Wb)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name]["recoveries_per_s_7M_points"] = nb * 20 / (e0.elapsed_time(e1) / 1e3)
        sb.close()
        del srcb, Ub, Wb
    return {"study": "25x25 (gamma in [1,100], P in [1e5,1e10] Pa), 10^3 cells x 27 points, "
                     f"{runs} runs per state, c = 3e8 m/s, D = 1; also all 625 states tiled over 7.08M points",
            "solvers": out, "fixed_iterations": con2prim_fixed_study(runs)}


# velocity errors at or below this count as equal in the iterations-to-parity study
PARITY_FLOOR = 1e-15


def grid_velocity_errors(eos, method, iters=0, c=3.0e8):
    """Relative velocity error of one GPU recovery solver (dg_con2prim, `iters` > 0 fixing
    its iteration count) on the paper's 25x25 (gamma, P) grid, as a [P, gamma] array."""
    import numpy as np
    import torch
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import Solver
    G, PP = wl.c2p_grid(25, c=c)
    g, P = G.ravel(), PP.ravel()
    beta = np.sqrt((1 - 1 / g) * (1 + 1 / g))
    cfg = wl.make_config("random3d", n_elem=(g.size, 1, 1), p=0, eos=eos, c2p=method, c=c,
                         precision=wl.FP64, c2p_iters=iters)
    s = Solver(cfg)
    src = np.stack([1.0 / g, beta * c, 0 * g, 0 * g, P]).reshape((5,) + wl.field_shape(cfg))
    U = s.set_state(torch.from_numpy(np.ascontiguousarray(src)).cuda())
    W = s.con2prim(U).reshape(5, -1).cpu().numpy()
    s.close()
    v = W[1] / np.sqrt(1 + (W[1:4] ** 2).sum(0) / c ** 2)
    err = np.where(beta > 0, np.abs(v - beta * c) / np.where(beta > 0, beta * c, 1.0), np.abs(v))
    return err.reshape(G.shape)


def _per_gamma(err):
    """Median and quartiles over the pressures at each Lorentz factor (the paper's right panels)."""
    import numpy as np
    q = np.percentile(err, [25, 50, 75], axis=0)
    return {"q25": q[0].tolist(), "median": q[1].tolist(), "q75": q[2].tolist()}


def con2prim_fixed_study(runs=100, max_iters=60):
    """The rest of the paper's recovery study (Sec. 3.3) on the GPU:

    * accuracy: the velocity error of the analytic solvers and of the iterative ones at
      fixed iteration counts (ideal gas: Newton from w = 1/2, 6 and 12 steps; TM: Brent on
      [0, 200^2 - 1], 25 and 50 steps) on the 25x25 grid;
    * iterations to parity: the fewest iterations (1 .. max_iters) with which the
      iterative solver is at least as accurate as the analytic one, per state (-1 where it
      never gets there); an error at or below PARITY_FLOOR (a few ulps of the velocity)
      counts as matching, so that ties at rounding level do not decide it;
    * timing: analytic time / iterative time (at the parity count) - 1 per state, each
      state on 10^3 cells x 27 points (the paper's size; one launch there is mostly launch
      latency) and on 64^3 x 27 = 7.08M points, `runs` and 10 runs."""
    import numpy as np
    import torch
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import Solver
    c = 3.0e8
    G, PP = wl.c2p_grid(25, c=c)
    out = {"gamma": G[0].tolist(), "pressure": PP[:, 0].tolist()}
    stream = torch.cuda.current_stream()
    for eos, analytic, iterative, caps, name in ((wl.EOS_IDEAL, wl.C2P_QUARTIC, wl.C2P_NEWTON, (6, 12), "ideal"),
                                                  (wl.EOS_TM, wl.C2P_CUBIC, wl.C2P_BRENT, (25, 50), "tm")):
        ea = grid_velocity_errors(eos, analytic)
        rec = {"analytic": {"max": float(ea.max()), "per_gamma": _per_gamma(ea)}}
        for n in caps:
            e = grid_velocity_errors(eos, iterative, n)
            rec[f"iterative_{n}"] = {"max": float(e.max()), "per_gamma": _per_gamma(e)}
        parity = np.full(ea.shape, -1, dtype=np.int64)
        for n in range(1, max_iters + 1):
            e = grid_velocity_errors(eos, iterative, n)
            newly = (parity < 0) & (e <= np.maximum(ea, PARITY_FLOOR))
            parity[newly] = n
        ok = parity > 0
        rec["iterations_to_parity"] = {
            "map": parity.tolist(), "never": int((~ok).sum()),
            "median_per_gamma": [float(np.median(col[col > 0])) if (col > 0).any() else None for col in parity.T],
            "max": int(parity[ok].max()) if ok.any() else None}
        # timing per state at its parity count (states that never reach parity are skipped)
        ratios = {"27k": np.full(ea.shape, np.nan), "7M": np.full(ea.shape, np.nan)}
        for size, n_elem, reps in (("27k", (10, 10, 10), runs), ("7M", (64, 64, 64), 10)):
            solvers = {}
            for (i, j) in zip(*np.nonzero(ok)):
                g, P = G[i, j], PP[i, j]
                times = []
                for method, iters in ((analytic, 0), (iterative, int(parity[i, j]))):
                    key = (method, iters)
                    if key not in solvers:
                        solvers[key] = Solver(wl.make_config("random3d", n_elem=n_elem, p=2, eos=eos, c2p=method,
                                                             c=c, precision=wl.FP64, c2p_iters=iters))
                    s = solvers[key]
                    src = torch.empty(s.shape, dtype=torch.float64, device="cuda")
                    beta = np.sqrt((1 - 1 / g) * (1 + 1 / g))
                    src[0].fill_(1.0 / g)
                    src[1].fill_(beta * c)
                    src[2].zero_()
                    src[3].zero_()
                    src[4].fill_(P)
                    U = s.set_state(src)
                    W = s.con2prim(U)
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        s.con2prim(U, out=W)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                    del src, U, W
                ratios[size][i, j] = times[0] / times[1] - 1.0
            for s in solvers.values():
                s.close()
        rec["timing_analytic_over_iterative_minus_1"] = {
            size: {"median": float(np.nanmedian(r)),
                   "per_gamma_median": [float(np.nanmedian(col)) if np.isfinite(col).any() else None for col in r.T]}
            for size, r in ratios.items()}
        out[name] = rec
    return out


def random3d_leg(repeats=5):
    """The 3D stress field (64^3 p=2, FP32 contractions, the physicality operator active).

    On this i.i.d. field most nodes fail recovery after the first stage and the state
    turns non-finite within a few steps (the oracle's own run does the same), so a
    multi-step rate measures the floor-state path, not the method.  Reported: step 1
    timed from a fresh copy of the initial state (median of `repeats`), with its event
    fractions; then the configured 20 steps one by one, with the fractions of failed
    recoveries, inadmissible averages and non-finite nodes after each step, and their
    rate labelled as failure-path throughput."""
    import statistics
    import torch
    from paper_2205_00095_amd import workloads as wl
    cfg, solver, U0 = _setup("random3d")
    dofs = wl.n_dof(cfg)
    nel = dofs // (cfg["p"] + 1) ** cfg["dim"]
    nvar = wl.n_var(cfg)
    bpd = _stage_bytes_per_dof(nvar)
    stream = torch.cuda.current_stream()
    U = torch.empty_like(U0)
    times = []
    for _ in range(repeats + 1):
        U.copy_(U0)
        solver.reset_diagnostics()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.run(U, cfg["dt"], 1)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    d1 = solver.diagnostics()
    t1 = statistics.median(times[1:])

    def fractions(d, stages):
        nonfinite = int((~torch.isfinite(U)).any(0).sum())
        return {"c2p_fail": d["c2p_fail"] / (dofs * stages), "bad_average": d["bad_average"] / (nel * stages),
                "smoothed": d["smoothed"] / (nel * stages), "trace_fallback_per_stage": d["trace_fallback"] / stages,
                "nonfinite_nodes": nonfinite / dofs}

    step1 = {"us": t1 * 1e6, "dof_stage_per_s": dofs * 3 / t1,
             "hbm_frac": bpd * dofs * 3 / t1 / (HBM_PEAK_GBS * 1e9), "fractions": fractions(d1, 3)}
    U.copy_(U0)
    per_step = []
    total = 0.0
    for k in range(cfg["steps"]):
        solver.reset_diagnostics()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.run(U, cfg["dt"], 1)
        e1.record(stream)
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1) / 1e3
        per_step.append(fractions(solver.diagnostics(), 3))
    n = cfg["steps"]
    solver.close()
    del U, U0
    return {"workload": "random3d: 3D 64^3 elements p=2 ideal EOS, FP32 contractions, physicality operator on",
            "dof": dofs, "algorithmic_bytes_per_dof": bpd,
            "step1_from_initial_state": step1,
            "failure_path_throughput": {
                "steps": n, "dof_stage_per_s": dofs * n * 3 / total, "stage_us": total / (3 * n) * 1e6,
                "hbm_frac": bpd * dofs * n * 3 / total / (HBM_PEAK_GBS * 1e9),
                "note": "steps timed one by one after step 1 has driven most nodes to the floor state"},
            "per_step_fractions": per_step,
            "fraction_units": "c2p_fail per node-stage, bad_average and smoothed per element-stage, "
                              "nonfinite_nodes after the step"}


def limiter_leg(steps=20, warmup=2):
    """The slope limiter at scale: the cylindrical blast (512x512 p=2, HLLC, SSP-RK3), the
    same steps from the same initial state with the limiter on and off.  With it each
    stage is two launches (the stage kernel writing the unlimited stage and its element
    averages, then limiter + operator + recovery); without it one fused launch."""
    import torch
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import Solver
    out = {}
    for lim in (1, 0):
        cfg = wl.make_config("blast2d", limiter=lim)
        solver = Solver(cfg)
        rho, v, P = wl.initial_primitives(cfg)
        U0 = solver.set_state(torch.from_numpy(wl.pack_primitives(rho, v, P)).cuda())
        U = U0.clone()
        solver.run(U, cfg["dt"], warmup)
        U.copy_(U0)
        solver.reset_diagnostics()
        seconds = _time_run(solver, U, cfg["dt"], steps, 0)
        d = solver.diagnostics()
        dofs = wl.n_dof(cfg)
        nel = dofs // (cfg["p"] + 1) ** cfg["dim"]
        out["on" if lim else "off"] = {
            "ms_per_step": seconds / steps * 1e3, "dof_stage_per_s": dofs * steps * 3 / seconds,
            "limited_per_element_stage": d["limited"] / (nel * steps * 3),
            "smoothed_per_element_stage": d["smoothed"] / (nel * steps * 3),
            "c2p_fail": d["c2p_fail"], "bad_average": d["bad_average"]}
        solver.close()
        del U, U0
    nvar = 4
    out["workload"] = "blast2d: 2D 512x512 elements p=2 ideal Gamma=5/3, HLLC, SSP-RK3, pressure ratio 1000"
    out["limiter_overhead"] = out["on"]["ms_per_step"] / out["off"]["ms_per_step"] - 1.0
    out["algorithmic_bytes_per_dof"] = {
        "stage": _stage_bytes_per_dof(nvar), "k_limit": nvar * 8.0,
        "note": ("stage (k_element, MODE_STAGE_LIM): read U^(k), read U^n in stages 2-3, write U^(k+1) "
                 "(mean over the three stages; it also writes the averages and the next stage's "
                 "primitives); k_limit: read U, plus U and W rewritten at the nodes that changed")}
    return out


def shard_leg(steps=50, warmup=5):
    """One GPU's share of the 512x512 p=3 Taub-Matthews mesh split over 8 GPUs as 4x2
    blocks: a 128x256-element block, timed as a whole mesh (its outer faces stand in for
    the halo faces that an exchange would supply), in FP64 and in the FP32 form; with
    the per-stage exchange volume such a split would move (the primitive traces of the
    block's boundary faces) and its time on one xGMI link."""
    from paper_2205_00095_amd import workloads as wl
    out = {}
    for name, prec in (("fp64", wl.FP64), ("fp32_contract", wl.FP32_CONTRACT)):
        cfg, solver, U = _setup("kh_tm", n_elem=(128, 256, 1), precision=prec)
        sec = _time_run(solver, U, cfg["dt"], steps, warmup)
        dofs = wl.n_dof(cfg)
        out[name] = {"stage_us": sec / (3 * steps) * 1e6, "dof_stage_per_s": dofs * steps * 3 / sec}
        solver.close()
        del U
    nx, ny, n1, nv = 128, 256, 4, 4
    faces = 2 * (nx + ny)            # boundary faces of the block (every side has a neighbour)
    exch = faces * n1 * nv * 8.0     # bytes of primitive traces sent per stage
    out.update({"block": "128x256 elements p=3 TM (512x512 over 4x2 GPUs)", "dof": nx * ny * n1 * n1,
                "exchange_bytes_per_stage": exch,
                "exchange_us_one_xgmi_link": exch / 153e9 * 1e6,
                "note": "the block's boundary faces are periodic/outflow here; a split run would take "
                        "them from the neighbours' traces, sent once per stage"})
    return out


def wave1d_leg(steps=100):
    """The 1D density wave (64 elements, p=2, ideal EOS): 100 SSP-RK3 steps at the fixed
    step 0.1/(2p+1) dx/c; the L1 error of D against the exact translated solution, the
    final state (for the drift against the oracle's run) and the launch-bound rate."""
    import numpy as np
    import torch
    from paper_2205_00095_amd import workloads as wl
    cfg, solver, U0 = _setup("wave1d")
    U = U0.clone()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.run(U, cfg["dt"], steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    t = steps * cfg["dt"]
    rho, v, _ = wl.wave1d_primitives(cfg, t)
    D_exact = rho / np.sqrt(1.0 - (v[0] / cfg["c"]) ** 2)
    _, w = np.polynomial.legendre.leggauss(cfg["p"] + 1)
    h = (cfg["hi"][0] - cfg["lo"][0]) / cfg["n_elem"][0]
    D = U[0].cpu().numpy()
    l1 = float((0.5 * h * w * np.abs(D - D_exact)).sum())
    dofs = wl.n_dof(cfg)
    out = {"workload": "wave1d: 1D 64 elements p=2 ideal EOS, v = 0.5c density wave",
           "steps": steps, "t_final": t, "l1_D_vs_exact": l1,
           "dof_stage_per_s": dofs * steps * 3 / sec, "stage_us": sec / (3 * steps) * 1e6,
           "note": "launch-bound (192 DOF); L1 = sum over nodes of (dx/2) w_q |D_h - D_exact|"}
    final = U.cpu()
    # the same 100 steps captured in a HIP graph and replayed (no host launches)
    Ug = U0.clone()
    graph = solver.graph_run(Ug, cfg["dt"], steps)
    Ug.copy_(U0)
    graph.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(Ug.cpu(), final))
    reps = 5
    Ug.copy_(U0)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    gsec = e0.elapsed_time(e1) / 1e3 / reps
    out["graph"] = {"dof_stage_per_s": dofs * steps * 3 / gsec, "stage_us": gsec / (3 * steps) * 1e6,
                    "replay_equals_eager_run": same,
                    "note": f"{steps} steps captured once (Solver.graph_run), {reps} replays timed"}
    solver.close()
    return out, final


def paper_sweep(target_s=0.15):
    """The paper's KH performance grid (Sec. 4) on one MI355X: the HLL and HLLC fluxes,
    basis orders 0, 1, 2 with RK1, SSPRK2, SSPRK3 on nx x 2nx meshes, nx = 256, 512,
    1024 (ideal EOS)."""
    import torch
    from paper_2205_00095_amd import workloads as wl
    rows = []
    grid = [(f, p, n) for f in (wl.FLUX_HLL, wl.FLUX_HLLC) for p in (0, 1, 2) for n in (256, 512, 1024)]
    for flux, p, nx in grid:
        cfg, solver, U = _setup("kh_paper", nx=nx, p=p, flux=flux)
        order = cfg["rk_order"]
        dofs = wl.n_dof(cfg)
        solver.run(U, cfg["dt"], 3, order=order)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.run(U, cfg["dt"], 5, order=order)
        torch.cuda.synchronize()
        per_step = (time.perf_counter() - t0) / 5
        n = max(10, int(target_s / per_step))
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.run(U, cfg["dt"], n, order=order)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        rows.append({"flux": "HLLC" if flux == wl.FLUX_HLLC else "HLL", "p": p, "rk_order": order,
                     "mesh": f"{nx}x{2 * nx}", "dof": dofs, "steps": n,
                     "dof_stage_per_s": dofs * n * order / sec, "stage_us": sec / (n * order) * 1e6})
        solver.close()
        del U
    return {"workload": "kh_paper: one shear interface, ideal Gamma=4/3, HLL and HLLC, physicality operator on, "
                        "FP64", "rows": rows}


def kh_growth(nx=256, orders=(0, 1, 2), t_end=3.0, sample_dt=0.05):
    """Growth rate r of <v_y^2> from a least-squares fit of log <v_y^2> = A + r t over
    t in [1.5, 3] (the paper's KH diagnostic, Sec. 4), per flux (HLL, HLLC) and basis
    order on an nx x 2nx mesh."""
    import numpy as np
    import torch
    from paper_2205_00095_amd import workloads as wl
    out = []
    for flux, p in [(f, p) for f in (wl.FLUX_HLL, wl.FLUX_HLLC) for p in orders]:
        cfg, solver, U = _setup("kh_paper", nx=nx, p=p, flux=flux)
        order, dt = cfg["rk_order"], cfg["dt"]
        area = (cfg["hi"][0] - cfg["lo"][0]) * (cfg["hi"][1] - cfg["lo"][1])
        every = max(1, int(round(sample_dt / dt)))
        ts, vals = [0.0], [solver.objective_vy2(U) / area]
        t = 0.0
        t0 = time.perf_counter()
        while t < t_end - 1e-12:
            solver.run(U, dt, every, order=order)
            t += every * dt
            ts.append(t)
            vals.append(solver.objective_vy2(U) / area)
        wall = time.perf_counter() - t0
        ts, vals = np.array(ts), np.array(vals)
        sel = (ts >= 1.5) & (ts <= 3.0)
        r, A = np.polyfit(ts[sel], np.log(vals[sel]), 1)
        out.append({"flux": "HLLC" if flux == wl.FLUX_HLLC else "HLL", "p": p, "rk_order": order,
                    "mesh": f"{nx}x{2 * nx}", "dof": wl.n_dof(cfg),
                    "growth_rate": float(r), "vy2_t0": float(vals[0]), "vy2_t3": float(vals[sel][-1]),
                    "steps": int(round(t / dt)), "wall_s": wall, "diagnostics": solver.diagnostics()})
        solver.close()
    return {"diagnostic": "fit of log <v_y^2> = A + r t over t in [1.5, 3]", "rows": out}


def fp32_contract(steps=50):
    """The 512x512 p=3 Taub-Matthews mesh in the FP32-contraction form against the same
    mesh in FP64 on the same GPU: throughputs, speedup and RHS error; also the two
    solutions after `steps` steps from the initial state, for the L1 error against
    the oracle's FP64 run of the same steps."""
    from paper_2205_00095_amd import workloads as wl
    cfg3, s64, U64 = _setup("kh_tm_fp32", precision=wl.FP64)
    U0 = U64.clone()
    R64 = s64.rhs(U0)
    t64 = _time_run(s64, U64, cfg3["dt"], steps, 5)
    V64 = U0.clone()
    s64.run(V64, cfg3["dt"], steps)
    s64.close()
    del s64, U64
    d3 = wl.n_dof(cfg3)
    nv3 = R64.shape[0]
    out = {"workload": "kh_tm_fp32: 2D 512x512 elements p=3 TM EOS", "value_fp64": d3 * steps * 3 / t64,
           "unit": "DOF-stage/s", "steps": steps}
    finals = {"fp64": V64.cpu()}
    # the FP32 form with its sweeps on the vector ALUs, then on the matrix cores
    for prec, tag in ((wl.FP32_CONTRACT, "fp32"), (wl.FP32_MFMA, "fp32_mfma")):
        cfg3, s32, U32 = _setup("kh_tm_fp32", precision=prec)
        R32 = s32.rhs(U0)
        t32 = _time_run(s32, U32, cfg3["dt"], steps, 5)
        V32 = U0.clone()
        s32.run(V32, cfg3["dt"], steps)
        s32.close()
        rhs_err = ((R32 - R64).reshape(nv3, -1).abs().max(1).values /
                   R64.reshape(nv3, -1).abs().max(1).values).max().item()
        drift = ((V32 - V64).reshape(nv3, -1).abs().sum(1) / V64.reshape(nv3, -1).abs().sum(1)).max().item()
        sfx = "" if tag == "fp32" else "_mfma"
        out.update({f"value_fp32{sfx}": d3 * steps * 3 / t32, f"speedup{sfx}": t64 / t32,
                    f"rhs_rel_err_vs_fp64_gpu{sfx}": rhs_err, f"l1_fp32{sfx}_vs_fp64_gpu_after_steps": drift})
        finals[tag] = V32.cpu()
        del s32, U32, R32, V32
    del R64, V64, U0
    return out, finals


def _l1_rel(A, B):
    """max over conserved components k of sum |A_k - B_k| / sum |B_k|."""
    nv = B.shape[0]
    return float(((A - B).reshape(nv, -1).abs().sum(1) / B.reshape(nv, -1).abs().sum(1)).max())


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(kind="kh_tm", steps=3, seconds=10.0):
    """The oracle as it stands, on the host cores: `steps` SSP-RK3 steps of the full mesh,
    then as many more as fill about `seconds` of wall time in total (a bounded sample);
    then one step on one thread."""
    import math
    import torch
    from oracle import srhd, timestep
    from oracle.setup import Setup
    from paper_2205_00095_amd import workloads as wl
    cfg = wl.make_config(kind)
    st = Setup.from_config(cfg)
    rho, v, P = (torch.from_numpy(a) for a in wl.initial_primitives(cfg))
    U = srhd.prim3_to_cons(rho, v, P, st).reshape((st.nvar,) + wl.field_shape(cfg))
    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    U1 = timestep.run(U, cfg["dt"], steps, st)
    dt = time.perf_counter() - t0
    more = max(0, math.ceil((seconds - dt) / (dt / steps))) if steps > 0 else 0
    if more:
        t1 = time.perf_counter()
        timestep.run(U1, cfg["dt"], more, st)
        dt += time.perf_counter() - t1
        steps += more
    dofs = wl.n_dof(cfg)
    torch.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        timestep.run(U, cfg["dt"], 1, st)
        dt1 = time.perf_counter() - t1
    finally:
        torch.set_num_threads(threads)
    ref = _cpu_reference_runs()
    rates = {k: {"dof_stage_per_s": wl.n_dof(wl.make_config(k)) * n * 3 / sec, "steps": n, "s": sec}
             for k, (U_, sec, n) in ref.items()}
    # the oracle's limited step (slope limiter and operator after every stage) on the
    # cylindrical blast, a 128x128 p=2 sample of the limiter leg's 512x512 mesh
    bcfg = wl.make_config("blast2d", n_elem=(128, 128, 1))
    bst = Setup.from_config(bcfg)
    brho, bv, bP = (torch.from_numpy(x) for x in wl.initial_primitives(bcfg))
    bU = srhd.prim3_to_cons(brho, bv, bP, bst).reshape((bst.nvar,) + wl.field_shape(bcfg))
    t1 = time.perf_counter()
    timestep.run(bU, bcfg["dt"], 8, bst)
    bsec = time.perf_counter() - t1
    rates["blast2d_limited_128"] = {"dof_stage_per_s": wl.n_dof(bcfg) * 8 * 3 / bsec, "steps": 8, "s": bsec}
    rec = {"value": dofs * steps * 3 / dt, "unit": "DOF-stage/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the full {cfg['n_elem'][0]}x{cfg['n_elem'][1]} p={cfg['p']} "
                      f"mesh ({dofs} DOF), torch CPU float64 on {threads} threads, {dt:.1f} s",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "value_1_thread": dofs * 3 / dt1,
            "sample_1_thread": f"1 SSP-RK3 step of the same mesh on 1 thread, {dt1:.1f} s",
            "reference_runs": rates}
    return rec, {k: v[0] for k, v in ref.items()}


def _cpu_reference_runs(steps_c1=100, steps_c3=50):
    """Part of the CPU baseline leg: the oracle's FP64 runs that the GPU results are
    compared with: the 1D density
    wave (100 steps) and the 512x512 p=3 TM Kelvin-Helmholtz mesh (50 steps), from the
    same initial states as the GPU runs; returns the final states and the wall times."""
    import torch
    from oracle import srhd, timestep
    from oracle.setup import Setup
    from paper_2205_00095_amd import workloads as wl
    out = {}
    for kind, n in (("wave1d", steps_c1), ("kh_tm_fp32", steps_c3)):
        cfg = wl.make_config(kind, precision=wl.FP64)
        st = Setup.from_config(cfg)
        rho, v, P = (torch.from_numpy(a) for a in wl.initial_primitives(cfg))
        U = srhd.prim3_to_cons(rho, v, P, st).reshape((st.nvar,) + wl.field_shape(cfg))
        t0 = time.perf_counter()
        U = timestep.run(U, cfg["dt"], n, st)
        out[kind] = (U, time.perf_counter() - t0, n)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kh_tm")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32, adjoint and CPU legs")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time the CPU oracle sample fills (after --cpu-steps steps)")
    ap.add_argument("--con2prim-study", action="store_true",
                    help="only run the recovery-solver study of the paper's Sec. 3.3 and print its JSON")
    ap.add_argument("--kh-growth", action="store_true",
                    help="only run the KH growth-rate diagnostic of the paper's Sec. 4 and print its JSON")
    ap.add_argument("--fp32-form", action="store_true",
                    help="only run the FP32-contraction comparison (512x512 p=3) and print its JSON")
    ap.add_argument("--random3d", action="store_true",
                    help="only run the 3D stress-field leg (64^3 p=2) and print its JSON")
    ap.add_argument("--adjoint", action="store_true",
                    help="only run the adjoint cost measurement (128x128 p=2, 200 steps) and print its JSON")
    ap.add_argument("--limiter", action="store_true",
                    help="only run the slope-limiter leg (2D blast 512x512 p=2, limiter on and off)")
    ap.add_argument("--rhs", action="store_true",
                    help="only time dg_rhs on the workload (50 calls after one warm-up) and print its JSON")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of 512 MiB (reference for HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for --gpus {args.gpus}); "
              "sharding across GPUs is described in the design notes, not implemented.", file=sys.stderr)
        return 2

    import torch
    from paper_2205_00095_amd import workloads as wl

    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if args.con2prim_study:
        print(json.dumps(con2prim_study()), flush=True)
        return 0
    if args.kh_growth:
        print(json.dumps(kh_growth()), flush=True)
        return 0
    if args.fp32_form:
        print(json.dumps(fp32_contract(50)[0]), flush=True)
        return 0
    if args.random3d:
        print(json.dumps(random3d_leg()), flush=True)
        return 0
    if args.adjoint:
        print(json.dumps(adjoint_ratio()), flush=True)
        return 0
    if args.limiter:
        print(json.dumps(limiter_leg()), flush=True)
        return 0
    if args.rhs:
        cfg, solver, U = _setup(args.workload)
        nvar, dofs = cfg["dim"] + 2, wl.n_dof(cfg)
        t_rhs = _time_rhs(solver, U, reps=50)
        print(json.dumps({"workload": args.workload, "dof": dofs, "dg_rhs_us": t_rhs * 1e6,
                          "frac": 2 * nvar * 8.0 * dofs / t_rhs / 1e9 / HBM_PEAK_GBS}), flush=True)
        return 0
    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg, solver, U = _setup(args.workload)
    dofs = wl.n_dof(cfg)
    nvar = cfg["dim"] + 2
    seconds = _time_run(solver, U, cfg["dt"], args.steps, args.warmup)
    # the same number of steps captured in a HIP graph and replayed once (no host launches)
    graph = solver.graph_run(U, cfg["dt"], args.steps)
    stream = torch.cuda.current_stream()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    g0.record(stream)
    graph.replay()
    g1.record(stream)
    torch.cuda.synchronize()
    graph_ms_per_step = g0.elapsed_time(g1) / args.steps
    del graph
    t_c2p = _time_con2prim(solver, U)
    t_rhs = _time_rhs(solver, U)
    stage_s = max(seconds - t_c2p, 1e-12) / (3 * args.steps)
    diag = solver.diagnostics()
    value = dofs * args.steps * 3 / seconds
    bytes_per_launch = _stage_bytes_per_dof(nvar) * dofs
    achieved = bytes_per_launch / stage_s / 1e9
    prof = _measured_traffic(args.workload)
    out = {
        "metric": "DG DOF-stage updates/s (FP64 vs FP32-contraction); adjoint/forward cost ratio",
        "value": value,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": seconds / args.steps * 1e3,
        "graph_ms_per_step": graph_ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if cfg["precision"] == wl.FP64 else "f64+f32-contraction",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {cfg['dim']}D {'x'.join(str(n) for n in cfg['n_elem'][:cfg['dim']])} "
                         f"elements p={cfg['p']} {'TM' if cfg['eos'] == wl.EOS_TM else 'ideal'} EOS, HLL, "
                         f"SSP-RK3, physicality operator on"),
            "dof": dofs, "elements": int(dofs // (cfg['p'] + 1) ** cfg['dim']), "p": cfg["p"],
            "dt": cfg["dt"], "precision": "fp64" if cfg["precision"] == wl.FP64 else "fp32-contraction",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": prof["traffic_bytes_per_launch"] if prof else None,
            "kernel": "k_element stage (one SSP-RK3 stage)",
            "dg_rhs_frac": 2 * nvar * 8.0 * dofs / t_rhs / 1e9 / HBM_PEAK_GBS,
            "stage_us": stage_s * 1e6, "con2prim_us": t_c2p * 1e6,
            "bytes_per_dof": _stage_bytes_per_dof(nvar),
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
        "diagnostics": diag,
        "dg_rhs": {
            "us": t_rhs * 1e6, "algorithmic_bytes": 2 * nvar * 8.0 * dofs,
            "achieved_GBs": 2 * nvar * 8.0 * dofs / t_rhs / 1e9,
            "frac": 2 * nvar * 8.0 * dofs / t_rhs / 1e9 / HBM_PEAK_GBS,
            "note": ("one launch: the element kernel recovers its nodes and halo elements and writes R; "
                     "algorithmic bytes: read U, write R")},
    }
    if prof:
        # executed-instruction view of the same kernel from the counter summary
        out["roofline"]["traffic_over_algorithmic"] = prof["traffic_bytes_per_launch"] / bytes_per_launch
        if "valu_insts_per_wave" in prof:
            waves = dofs / 64.0
            issue_s = prof["valu_insts_per_wave"] * waves * VALU_CYCLES_PER_WAVE_INST / (SIMDS * CLOCK_HZ)
            out["roofline"]["valu"] = {
                "insts_per_dof": prof["valu_insts_per_wave"], "f64_insts_per_dof": prof.get("f64_insts_per_wave"),
                "issue_bound_us": issue_s * 1e6, "issue_frac": issue_s / stage_s}
            if "mul_f64_per_wave" in prof:
                # FP64 operations per DOF (an FMA counts two; every lane counted, so an upper
                # bound where lanes idle) against the FP64 vector peak
                flops = 2.0 * prof["fma_f64_per_wave"] + prof["mul_f64_per_wave"] + prof["add_f64_per_wave"]
                out["roofline"]["valu"].update({
                    "f64_flops_per_dof": flops, "f64_tflops": flops * dofs / stage_s / 1e12,
                    "f64_peak_frac": flops * dofs / stage_s / FP64_VECTOR_PEAK})
    if not args.no_extras and args.workload == "kh_tm":
        extras = {}
        fp32, finals = fp32_contract(50)
        extras["fp32_contract"] = fp32
        extras["hbm_copy_GBs"] = _copy_bandwidth() / 1e9
        extras["paper_sweep"] = paper_sweep()
        extras["random3d"] = random3d_leg()
        extras["limiter"] = limiter_leg()
        extras["shard_share"] = shard_leg()
        c1, c1_final = wave1d_leg(100)
        extras["wave1d"] = c1
        extras["adjoint"] = adjoint_ratio()
        out.update(extras)
        # the CPU leg also runs the oracle's FP64 runs of the 1D wave and of the 512x512
        # mesh, against which the GPU results after the same steps are compared
        out["cpu_baseline"], ref = cpu_baseline("kh_tm", args.cpu_steps, args.cpu_seconds)
        out["wave1d"]["l1_gpu_vs_oracle"] = _l1_rel(c1_final, ref["wave1d"].reshape(c1_final.shape))
        U_c3 = ref["kh_tm_fp32"].reshape(finals["fp32"].shape)
        out["fp32_contract"]["l1_fp32_vs_oracle_fp64"] = _l1_rel(finals["fp32"], U_c3)
        out["fp32_contract"]["l1_fp32_mfma_vs_oracle_fp64"] = _l1_rel(finals["fp32_mfma"], U_c3)
        out["fp32_contract"]["l1_fp64_vs_oracle_fp64"] = _l1_rel(finals["fp64"], U_c3)
        out["fp32_contract"]["note"] = ("L1 errors: max over conserved components of sum |U - U_ref| / sum |U_ref| "
                                        "after the steps, against the oracle's FP64 run from the same initial "
                                        "state (CPU) and against the GPU's FP64 path")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

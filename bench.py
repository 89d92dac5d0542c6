"""Throughput benchmark of the DG SRHD hot path on one MI355X.

A step is one SSP-RK3 step (three fused stage kernels: volume + faces + lift +
RK combine + physicality operator + recovery of the next stage's primitives)
over the whole mesh.  Metric: DOF-stage updates per second,
DOF x steps x 3 / seconds, with the state resident in HBM.

Default workload: 2D relativistic Kelvin-Helmholtz, Taub-Matthews EOS,
256x256 elements, p=3 (16 nodes per element, 1,048,576 DOF), FP64, HLL,
physicality operator on.  Extra results on the same JSON line:
  fp32_contract  the 512x512 p=3 Kelvin-Helmholtz mesh in the FP32-contraction
                 form vs the same mesh in FP64 (speedup on the same GPU);
  adjoint        cost of the checkpointed adjoint of 200 steps (checkpoint every
                 20) relative to the forward run, 128x128 p=2 ideal-gas mesh;
  roofline       the stage kernel against HBM, from algorithmic bytes per
                 DOF-stage (read U^(k), read U^n in stages 2-3, write U^(k+1)).
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


def _stage_bytes_per_dof(nvar: int) -> float:
    """Mean algorithmic bytes per DOF over the three stages of one step."""
    return nvar * 8.0 * (2.0 + 2.0 / 3.0)


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


def cpu_baseline(kind="kh_tm", steps=3):
    """The oracle as it stands, on the host cores, for `steps` SSP-RK3 steps of the full mesh."""
    import torch
    from oracle import srhd, timestep
    from oracle.setup import Setup
    from paper_2205_00095_amd import workloads as wl
    cfg = wl.make_config(kind)
    st = Setup.from_config(cfg)
    rho, v, P = (torch.from_numpy(a) for a in wl.initial_primitives(cfg))
    U = srhd.prim3_to_cons(rho, v, P, st).reshape((st.nvar,) + wl.field_shape(cfg))
    t0 = time.perf_counter()
    timestep.run(U, cfg["dt"], steps, st)
    dt = time.perf_counter() - t0
    dofs = wl.n_dof(cfg)
    return {"value": dofs * steps * 3 / dt, "unit": "DOF-stage/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the full {cfg['n_elem'][0]}x{cfg['n_elem'][1]} p={cfg['p']} "
                      f"mesh ({dofs} DOF), torch CPU float64, {dt:.1f} s"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kh_tm")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32, adjoint and CPU legs")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of 512 MiB (reference for HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implementation.", file=sys.stderr)
        return 2

    import torch
    from paper_2205_00095_amd import workloads as wl

    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
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
    t_c2p = _time_con2prim(solver, U)
    stage_s = max(seconds - t_c2p, 1e-12) / (3 * args.steps)
    diag = solver.diagnostics()
    value = dofs * args.steps * 3 / seconds
    bytes_per_launch = _stage_bytes_per_dof(nvar) * dofs
    achieved = bytes_per_launch / stage_s / 1e9
    out = {
        "metric": "DG DOF-stage updates/s (FP64 vs FP32-contraction); adjoint/forward cost ratio",
        "value": value,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": seconds / args.steps * 1e3,
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
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_element stage (one SSP-RK3 stage)",
            "stage_us": stage_s * 1e6, "con2prim_us": t_c2p * 1e6,
            "bytes_per_dof": _stage_bytes_per_dof(nvar),
        },
        "diagnostics": diag,
    }
    if not args.no_extras and args.workload == "kh_tm":
        extras = {}
        cfg3, s64, U64 = _setup("kh_tm_fp32", precision=wl.FP64)
        n3 = min(args.steps, 50)
        t64 = _time_run(s64, U64, cfg3["dt"], n3, 5)
        del s64, U64
        cfg3, s32, U32 = _setup("kh_tm_fp32")
        t32 = _time_run(s32, U32, cfg3["dt"], n3, 5)
        d3 = wl.n_dof(cfg3)
        extras["fp32_contract"] = {
            "workload": "kh_tm_fp32: 2D 512x512 elements p=3 TM EOS",
            "value_fp32": d3 * n3 * 3 / t32, "value_fp64": d3 * n3 * 3 / t64,
            "speedup": t64 / t32, "unit": "DOF-stage/s", "steps": n3}
        del s32, U32
        extras["adjoint"] = adjoint_ratio()
        out.update(extras)
        out["cpu_baseline"] = cpu_baseline("kh_tm", args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

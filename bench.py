"""Benchmark: RK-OECDG DOF-updates/s on one MI355X.

Workload (the plain P2 headline): 1D Euler (gamma = 1.4) two-state Riemann
problem on [0, 1] with outflow boundaries, N = 16384 primal + 16385 dual
cells, P2 Legendre modal basis, seeded states (seed 0: rho, p ~ U[0.1, 1],
u = 0, jump at x = 0.5), SSP-RK3 + OE after every stage, CFL 0.15, run to
T = 0.2 (33354 steps for seed 0).  A "step" is one full RK-OECDG time step:
the time-step reduction, three stage updates on both meshes and three OE
applications.  value = DOF-updates/s = (DOFs of both meshes) x steps / wall
seconds, with the state resident in HBM when the timed region starts.

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
BYTES_PER_DOF_UPDATE = 64.0    # 5 reads + 3 writes of one FP64 coefficient per full SSP-RK3 step
N_CELLS, DEGREE, CFL, T_END, SEED = 16384, 2, 0.15, 0.2, 0
FULL_STEPS = 33354             # steps to T = 0.2 for seed 0
BATCH_COUNT, BATCH_STEPS, LOOP_SAMPLE = 512, 1000, 24
WHOLE_RUN_STEPS = 256          # runs of up to this many steps replay one captured graph (library constant)
KERNEL_TIMING_STEPS = 4096     # length of the run that times the stage kernel live
ADJ_N, ADJ_K, ADJ_STEPS, ADJ_CKPT = 16384, 2, 400, 20
E2D_N, E2D_STEPS, E2D_CFL = 1024, 500, 0.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=FULL_STEPS, help="timed RK-OECDG steps (default: the full run to T)")
    ap.add_argument("--warmup", type=int, default=2000, help="untimed warm-up steps")
    ap.add_argument("--mode", type=int, default=0, help="execution mode (0 auto, 1 eager, 2 graph, 3 persistent)")
    ap.add_argument("--tile", type=int, default=0, help="primal cells per workgroup (0: library default)")
    ap.add_argument("--fold", type=int, default=0,
                    help="statistics reduction of the headline run (0 library choice, 1 in-kernel, 2 fold kernel)")
    ap.add_argument("--batched-steps", type=int, default=BATCH_STEPS, help="steps of the batched runs")
    ap.add_argument("--batched-repeats", type=int, default=5, help="timed repetitions of the batched runs")
    ap.add_argument("--no-loop", action="store_true", help="skip the per-instance loop the batched form is compared with")
    ap.add_argument("--batched-fold", type=int, default=0,
                    help="statistics reduction of the batched runs (0 library choice, 1 in-kernel, 2 fold kernel)")
    ap.add_argument("--repeats", type=int, default=5, help="timed repetitions (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU-oracle sample length")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-form measurement")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D Euler measurement")
    ap.add_argument("--no-widened", action="store_true",
                    help="skip the classical-RK4, reflective-wall and 2D P^2 measurements")
    ap.add_argument("--e2d-steps", type=int, default=E2D_STEPS, help="steps of the 2D Euler measurement")
    ap.add_argument("--e2d-repeats", type=int, default=5, help="timed repetitions of the 2D Euler measurement")
    ap.add_argument("--kernel-timing-steps", type=int, default=KERNEL_TIMING_STEPS,
                    help="steps of the run that times the stage kernel live (0: the timed region's per-launch time)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the warm-up, copy a device buffer of this many MiB (profiler counter calibration)")
    return ap.parse_args()


PROFILE_JSON = os.path.join(ROOT, "profiles", "k_stage_euler1d_p2_n16384.json")
KERNEL_SOURCES = ["paper_2503_12473_amd/csrc/oecdg_1d.hip", "paper_2503_12473_amd/csrc/oecdg_tables.h",
                  "paper_2503_12473_amd/csrc/oecdg_internal.h", "paper_2503_12473_amd/csrc/oecdg_device.h"]


def stage_profile():
    """The committed rocprofv3 results of the headline stage kernel: average
    kernel duration (kernel trace) and HBM bytes per launch (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated), or {} if the kernel sources changed since the
    profile was taken."""
    import hashlib
    try:
        meta = json.load(open(PROFILE_JSON))
    except OSError:
        return {}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return meta if meta.get("source_sha256") == h.hexdigest() else {}


OPCOUNT_JSON = os.path.join(ROOT, "profiles", "oracle_opcount.json")


def oracle_opcount(phase):
    """Operations per DOF of the oracle's plain evaluation (the committed output
    of oracle/opcount/run.py; a stored file, the oracle is not run here)."""
    try:
        return json.load(open(OPCOUNT_JSON)).get(phase, {}).get("flops_per_dof")
    except OSError:
        return None


PROFILE2D_JSON = os.path.join(ROOT, "profiles", "k_stage2d_euler2d_q2_n1024.json")
KERNEL2D_SOURCES = ["paper_2503_12473_amd/csrc/oecdg_2d.hip", "paper_2503_12473_amd/csrc/oecdg_tables.h",
                    "paper_2503_12473_amd/csrc/oecdg_device.h"]


def profile_2d():
    """Counter results per 2D RK stage (k_stage2d + k_delta2d) from the
    committed profile: HBM bytes and executed FP64 flops, or {} if the kernel
    sources changed since."""
    import hashlib
    try:
        meta = json.load(open(PROFILE2D_JSON))
    except OSError:
        return {}
    h = hashlib.sha256()
    for f in KERNEL2D_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return meta if meta.get("source_sha256") == h.hexdigest() else {}


def batched_bench(k_fixed=None, fold=0, steps=BATCH_STEPS, repeats=5, loop_baseline=True):
    """Batched form: 512 independent 1D Euler Riemann instances (seed 0: N ~
    U{128..8192}, k ~ U{1,2,3} or k = k_fixed, seeded states), BATCH_STEPS steps
    each with its own CFL step, advanced together (graph-captured stages: a
    per-instance fold of the statistics, then one launch per degree group;
    autotuned tile) versus a loop of plain per-instance runs (LOOP_SAMPLE
    instances spread evenly over the batch, same steps and tile).  fold: the
    OECDG_OPT_FOLD value (0 library choice, 1 in-kernel reduction, 2 fold)."""
    import torch
    from paper_2503_12473_amd import inputs, _lib
    from paper_2503_12473_amd.api import OECDG, to_device
    from paper_2503_12473_amd.autotune import tune_tile
    specs = inputs.batch_instances(seed=SEED, count=BATCH_COUNT, k_fixed=k_fixed)
    probs, states = [], []
    for n, k, st in specs:
        p, uC, uD = inputs.euler_riemann(n, k, st)
        probs.append(p)
        states.append((uC, uD))
    dofs = [p.dofs() for p in probs]
    stream = torch.cuda.current_stream()

    def timed(solver, a, b):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.run(a, b, t_end=math.inf, nsteps=steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    icC = torch.cat([to_device(u[0]) for u in states])
    icD = torch.cat([to_device(u[1]) for u in states])
    with OECDG(probs, CFL, stream=stream) as solver:
        if fold:
            solver.set_option(_lib.OPT_FOLD, fold)
        tile = tune_tile(solver, icC, icD, steps=5)
        a, b = icC.clone(), icD.clone()
        solver.run(a, b, t_end=math.inf, nsteps=20)
        walls = []
        for _ in range(max(1, repeats)):
            a.copy_(icC)
            b.copy_(icD)
            torch.cuda.synchronize()
            walls.append(timed(solver, a, b))
        wall = sorted(walls)[len(walls) // 2]                 # median
    batched = sum(dofs) * steps / wall
    loop_wall, loop_dofs = 0.0, 0
    sample = [round(i * (BATCH_COUNT - 1) / (LOOP_SAMPLE - 1)) for i in range(LOOP_SAMPLE)]
    for i in (sample if loop_baseline else []):
        p, (uC, uD) = probs[i], states[i]
        with OECDG(p, CFL, stream=stream) as solver:
            solver.set_option(_lib.OPT_TILE, tile)
            a, b = to_device(uC), to_device(uD)
            solver.run(a.clone(), b.clone(), t_end=math.inf, nsteps=20)
            loop_wall += timed(solver, a, b)
            loop_dofs += p.dofs()
    loop = loop_dofs * steps / loop_wall if loop_wall > 0 else None
    mean_all = sum(dofs) / len(dofs)
    bytes_per_stage = BYTES_PER_DOF_UPDATE / 3.0 * sum(dofs)
    stage_s = wall / (3 * steps)
    return {"instances": BATCH_COUNT, "steps": steps, "dofs": sum(dofs), "tile": tile,
            "k": "U{1,2,3}" if k_fixed is None else k_fixed, "fold": {0: "auto", 1: "in-kernel", 2: "fold"}[fold],
            "batched_dof_updates_per_s": batched, "batched_wall_s": wall,
            "hbm": {"achieved": bytes_per_stage / stage_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": bytes_per_stage / stage_s / 1e9 / HBM_PEAK_GBS, "stage_us": 1e6 * stage_s,
                    "algorithmic_bytes_per_stage": bytes_per_stage,
                    "note": "per RK stage: fold + one stage launch per degree group"},
            "loop_dof_updates_per_s": loop, "loop_sample_instances": LOOP_SAMPLE,
            "loop_sample": f"instances {sample[0]}, {sample[1]}, ..., {sample[-1]} (evenly spaced); mean DOFs "
                           f"{loop_dofs / LOOP_SAMPLE:.0f} against {mean_all:.0f} over the batch",
            "speedup_vs_loop": batched / loop if loop else None}


def adjoint_bench(repeats: int = 5):
    """Adjoint form: periodic Burgers, N = 16384, P2, seeded 8-mode Fourier
    initial data (seed 0), ADJ_STEPS fixed steps (dt = 0.3 h / max|u0|),
    checkpoints every ADJ_CKPT steps.  Times one forward run and one full
    gradient (checkpointing forward pass, segment recomputation, reverse
    stages); ratio = gradient time / forward time."""
    import numpy as np
    import torch
    from paper_2503_12473_amd import inputs
    from paper_2503_12473_amd.api import OECDG, to_device
    prob, uC, uD, _ = inputs.burgers_fourier(ADJ_N, ADJ_K, seed=SEED)
    dt = 0.3 * prob.h / float(np.abs(uC[0, 0]).max())
    stream = torch.cuda.current_stream()
    ic = (to_device(uC), to_device(uD))
    rng = np.random.default_rng(SEED + 1)
    gT = (to_device(rng.normal(size=uC.shape)), to_device(rng.normal(size=uD.shape)))

    def ev(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    with OECDG(prob, 0.3, stream=stream) as solver:
        a, b = ic[0].clone(), ic[1].clone()
        solver.run(a, b, nsteps=ADJ_STEPS, dt_fixed=dt)                       # warm-up (graph capture)
        solver.adjoint(ic[0], ic[1], ADJ_STEPS, dt, gT[0], gT[1], ADJ_CKPT)   # warm-up (workspace)
        fwd, bwd = [], []
        for _ in range(repeats):
            a.copy_(ic[0])
            b.copy_(ic[1])
            fwd.append(ev(lambda: solver.run(a, b, nsteps=ADJ_STEPS, dt_fixed=dt)))
            bwd.append(ev(lambda: solver.adjoint(ic[0], ic[1], ADJ_STEPS, dt, gT[0], gT[1], ADJ_CKPT)))
    f, g = sorted(fwd)[len(fwd) // 2], sorted(bwd)[len(bwd) // 2]
    return {"workload": f"periodic Burgers, N={ADJ_N} primal + dual cells, P{ADJ_K}, {ADJ_STEPS} fixed steps, "
                        f"checkpoints every {ADJ_CKPT}, seed {SEED}",
            "forward_s": f, "gradient_s": g, "gradient_over_forward": g / f,
            "forward_dof_updates_per_s": prob.dofs() * ADJ_STEPS / f}


def euler2d_bench(repeats: int = 5, steps: int = E2D_STEPS):
    """2D form: Euler on [0,1]^2 periodic, 1024^2 primal + 1024^2 dual cells,
    tensor Q2 (9 modes x 4 components), seeded quadrant states (seed 0) plus
    0.2 sin(2 pi (x+y)) in the density, CFL 0.3, 500 steps.  Times whole runs
    of oecdg_run from the initial data (median of `repeats`)."""
    import torch
    from paper_2503_12473_amd import inputs
    from paper_2503_12473_amd.api import OECDG, to_device
    prob, uC, uD, _ = inputs.euler2d_quadrants(E2D_N, 2, seed=SEED)
    dofs = prob.dofs()
    stream = torch.cuda.current_stream()
    ic = (to_device(uC), to_device(uD))
    del uC, uD
    with OECDG(prob, E2D_CFL, stream=stream) as solver:
        a, b = ic[0].clone(), ic[1].clone()
        solver.run(a, b, nsteps=10)                                     # warm-up
        times = []
        for _ in range(repeats):
            a.copy_(ic[0])
            b.copy_(ic[1])
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            t, n = solver.run(a, b, nsteps=steps)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
    wall = sorted(times)[len(times) // 2]
    launch_s = wall / (3 * n)                    # one RK stage: fold + reduce + k_stage2d + k_delta2d
    bytes_per_launch = BYTES_PER_DOF_UPDATE / 3.0 * dofs
    achieved = bytes_per_launch / launch_s / 1e9
    prof = profile_2d()
    flops = prof.get("fp64_flops_per_stage")
    tflops = flops / launch_s / 1e12 if flops else None
    # The binding resource is FP64 vector issue (the counters show the SIMDs
    # issuing most of the time): the roofline is FP64 flops executed per stage
    # (SQ counters of the committed profile) over the live stage time, with the
    # algorithmic-bytes HBM figure beside it.
    return {"workload": f"2D Euler, [0,1]^2 periodic, {E2D_N}^2 primal + {E2D_N}^2 dual cells, Q2, CFL {E2D_CFL}, "
                        f"{steps} steps, seeded quadrant states (seed {SEED})",
            "dofs": dofs, "steps": n, "t_end": t, "wall_s": wall, "ms_per_step": 1e3 * wall / n,
            "dof_updates_per_s": dofs * n / wall,
            "roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP64_PEAK_TFLOPS if tflops else None,
                         "flops": "executed FP64 (counted wave instructions x 64 lanes, FMA = 2)",
                         "executed_flops_per_dof_update": 3 * flops / dofs if flops else None,
                         "oracle_flops_per_dof_update": oracle_opcount("2d_euler_q2.step"),
                         "oracle_note": "operations of the oracle's plain evaluation (no sum factorisation), counted "
                                        "by oracle/opcount; the kernels execute fewer",
                         "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": achieved / HBM_PEAK_GBS, "traffic": prof.get("traffic_bytes_per_stage")},
                         "kernel": "per RK stage: k_stage2d (OE of the previous stage + operator + SSP-RK3) "
                                   "+ k_delta2d (damping numerators, statistics) + statistics folds",
                         "launch_us": 1e6 * launch_s}}


def _timed_1d(prob, uC, uD, cfl, steps, rk=3, warmup=200):
    """Median of 5 oecdg_run calls of `steps` steps from the same initial data."""
    import torch
    from paper_2503_12473_amd.api import OECDG, to_device
    stream = torch.cuda.current_stream()
    ic = (to_device(uC), to_device(uD))
    with OECDG(prob, cfl, stream=stream, rk=rk) as solver:
        a, b = ic[0].clone(), ic[1].clone()
        solver.run(a, b, nsteps=warmup)
        times = []
        for _ in range(5):
            a.copy_(ic[0])
            b.copy_(ic[1])
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, n = solver.run(a, b, nsteps=steps)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
    wall = sorted(times)[2]
    return n, wall


def _timed_nu(prob, edges, uC, uD, cfl, steps, warmup=50):
    """Median of 5 oecdg_run_nonuniform calls of `steps` steps from the same initial data."""
    import torch
    from paper_2503_12473_amd.api import OECDG, to_device
    stream = torch.cuda.current_stream()
    ic = (to_device(uC), to_device(uD))
    with OECDG(prob, cfl, stream=stream) as solver:
        a, b = ic[0].clone(), ic[1].clone()
        solver.run_nonuniform(edges, a, b, nsteps=warmup)
        times = []
        for _ in range(5):
            a.copy_(ic[0])
            b.copy_(ic[1])
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, n = solver.run_nonuniform(edges, a, b, nsteps=steps)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
    return n, sorted(times)[2]


def _euler_wave(edges, k):
    """Periodic Euler density wave rho = 1 + 0.2 sin(2 pi x), v = 0.5, p = 1 on [0, 1]."""
    import numpy as np
    from paper_2503_12473_amd import inputs
    prob = inputs.Problem1D(k=k, nc=3, flux=inputs.FLUX_EULER, bc=inputs.BC_PERIODIC, n=len(edges) - 1,
                            xlo=0.0, xhi=1.0)
    f = lambda x: inputs.euler_conserved(1.0 + 0.2 * np.sin(2 * np.pi * x), 0.5 + 0 * x, 1.0 + 0 * x)
    uC, uD = inputs.project_1d_edges(f, 3, k, edges)
    return prob, uC, uD


def widened_bench():
    """The forms beyond the SSP-RK3 plain path: classical RK4 (four stages per
    step) at P3 on the Riemann workload, reflective walls (the walled-Euler
    kernels) on blast-wave data, the 2D total-degree space P^2 on the 2D
    Euler workload, and a non-uniform periodic mesh (beside the uniform path on
    the same data and a uniform mesh).  A DOF-update is one DOF advanced by one
    full step."""
    import torch
    from paper_2503_12473_amd import inputs
    from paper_2503_12473_amd.api import OECDG, to_device
    out = {}
    prob, uC, uD = inputs.euler_riemann(N_CELLS, 3, inputs.riemann_states(SEED))
    for rk, name in ((4, "rk4_p3"), (3, "ssprk3_p3")):
        n, wall = _timed_1d(prob, uC, uD, 0.2, 2000, rk=rk)
        stages = 4 if rk == 4 else 3
        out[name] = {"workload": f"1D Euler Riemann N={N_CELLS}, P3, {'classical RK4' if rk == 4 else 'SSP-RK3'}, "
                                 f"CFL 0.2, {n} steps", "dofs": prob.dofs(), "dof_updates_per_s": prob.dofs() * n / wall,
                     "ms_per_step": 1e3 * wall / n, "us_per_stage_launch": 1e6 * wall / (stages * n)}
    prob, uC, uD = inputs.euler_blast_waves(16000, 2, pressures=(100.0, 1.0, 10.0), densities=(1.0, 0.5, 0.8))
    n, wall = _timed_1d(prob, uC, uD, 0.3, 2000)
    out["walls_p2"] = {"workload": "1D Euler blast waves between reflective walls, N=16000, P2, SSP-RK3, CFL 0.3, "
                                   f"p = (100, 1, 10), rho = (1, 0.5, 0.8), {n} steps",
                       "dofs": prob.dofs(), "dof_updates_per_s": prob.dofs() * n / wall,
                       "ms_per_step": 1e3 * wall / n, "us_per_stage_launch": 1e6 * wall / (3 * n)}
    prob, uC, uD, _ = inputs.euler2d_quadrants(E2D_N, 2, seed=SEED, space=1)
    stream = torch.cuda.current_stream()
    ic = (to_device(uC), to_device(uD))
    del uC, uD
    steps = 100
    with OECDG(prob, E2D_CFL, stream=stream) as solver:
        a, b = ic[0].clone(), ic[1].clone()
        solver.run(a, b, nsteps=5)
        a.copy_(ic[0])
        b.copy_(ic[1])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, n = solver.run(a, b, nsteps=steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = e0.elapsed_time(e1) / 1e3
    pk_dofs = 2 * 4 * 6 * E2D_N * E2D_N
    out["euler2d_p2"] = {"workload": f"2D Euler {E2D_N}^2, total-degree P^2 (6 modes in the tensor layout, the P^2 "
                                     f"kernel instantiation), CFL {E2D_CFL}, {n} steps, seed {SEED}",
                         "dofs": pk_dofs, "dof_updates_per_s": pk_dofs * n / wall, "ms_per_step": 1e3 * wall / n}
    import numpy as np
    edges = inputs.quasi_uniform_edges(N_CELLS, 0.0, 1.0, 1.5, seed=SEED)
    prob, uC, uD = _euler_wave(edges, 2)
    n, wall = _timed_nu(prob, edges, uC, uD, 0.1, 1000)
    out["nonuniform_p2"] = {"workload": f"1D Euler density wave, periodic, random mesh N={N_CELLS} (width ratio <= 1.5, "
                                        f"seed {SEED}), P2, SSP-RK3, CFL 0.1, {n} steps",
                            "dofs": prob.dofs(), "dof_updates_per_s": prob.dofs() * n / wall,
                            "ms_per_step": 1e3 * wall / n, "us_per_stage": 1e6 * wall / (3 * n)}
    uni = np.linspace(0.0, 1.0, N_CELLS + 1)
    prob, uC, uD = _euler_wave(uni, 2)
    n, wall = _timed_1d(prob, uC, uD, 0.1, 1000)
    out["nonuniform_p2"]["uniform_path_same_data_ms_per_step"] = 1e3 * wall / n
    return out


def cpu_baseline(target_seconds: float):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    the first S steps from the same initial data (S sized to ~target_seconds)."""
    from oracle import ora
    from paper_2503_12473_amd import inputs
    prob, uC, uD = inputs.euler_riemann(N_CELLS, DEGREE, inputs.riemann_states(SEED))
    t0 = time.perf_counter()
    ora.run1d(prob, uC, uD, nsteps=2, cfl=CFL, t_end=T_END)
    per_step = (time.perf_counter() - t0) / 2
    steps = max(2, int(target_seconds / max(per_step, 1e-6)))
    t0 = time.perf_counter()
    _, _, _, done = ora.run1d(prob, uC, uD, nsteps=steps, cfl=CFL, t_end=T_END)
    wall = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": prob.dofs() * done / wall, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {FULL_STEPS} steps of the same workload, serial C oracle "
                      f"(-O2, no FP contraction), {wall:.1f} s",
            "cpu": model, "host_cpus": os.cpu_count(),
            "all_cores": cpu_all_cores(target_seconds / 3, min(16, os.cpu_count() or 1))}


_CPU_WORKER = """
import sys, time
sys.path.insert(0, {root!r})
from oracle import ora
from paper_2503_12473_amd import inputs
prob, uC, uD = inputs.euler_riemann({n}, {k}, inputs.riemann_states({seed}))
t0 = time.perf_counter()
ora.run1d(prob, uC, uD, nsteps=2, cfl={cfl}, t_end={t_end})
steps = max(2, int({seconds} / max((time.perf_counter() - t0) / 2, 1e-6)))
t0 = time.perf_counter()
_, _, _, done = ora.run1d(prob, uC, uD, nsteps=steps, cfl={cfl}, t_end={t_end})
print(prob.dofs() * done / (time.perf_counter() - t0), done)
"""


def cpu_all_cores(seconds: float, nproc: int):
    """Secondary CPU figure: the same serial oracle sample in nproc independent
    processes at once (one copy of the workload each, as independent instances
    of a batch would run), summed.  The children are CPU-only programs (no GPU
    library is loaded in them)."""
    import subprocess
    code = _CPU_WORKER.format(root=ROOT, n=N_CELLS, k=DEGREE, seed=SEED, cfl=CFL, t_end=T_END, seconds=seconds)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    rates, steps = [], []
    try:
        procs = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                  text=True, env=env) for _ in range(nproc)]
        for p in procs:
            out, err = p.communicate(timeout=600)
            if p.returncode != 0:
                return {"error": f"worker exited with {p.returncode}: {err.strip()[-200:]}"}
            r, d = out.split()
            rates.append(float(r))
            steps.append(int(d))
    except (OSError, ValueError, subprocess.SubprocessError) as e:
        return {"error": f"workers failed: {e}"}
    return {"value": sum(rates), "unit": "DOF-updates/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nproc} processes, each the first {min(steps)}-{max(steps)} steps of its own copy of the "
                      f"workload (about {seconds:.0f} s each), rates summed"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2503_12473_amd import inputs, _lib
    from paper_2503_12473_amd.api import OECDG, to_device

    torch.cuda.init()
    prob, uC, uD = inputs.euler_riemann(N_CELLS, DEGREE, inputs.riemann_states(SEED))
    dofs = prob.dofs()
    stream = torch.cuda.current_stream()
    solver = OECDG(prob, CFL, stream=stream)
    if args.mode:
        solver.set_option(_lib.OPT_MODE, args.mode)
    if args.tile:
        solver.set_option(_lib.OPT_TILE, args.tile)
    if args.fold:
        solver.set_option(_lib.OPT_FOLD, args.fold)
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ic = (to_device(uC), to_device(uD))
    work = (ic[0].clone(), ic[1].clone())

    # warm-up: code loading, caches; then one untimed run of the timed length,
    # which captures the graph the library replays for runs of that length
    if args.warmup > 0:
        solver.run(work[0], work[1], t_end=T_END, nsteps=args.warmup)
    work[0].copy_(ic[0])
    work[1].copy_(ic[1])
    solver.run(work[0], work[1], t_end=T_END, nsteps=min(args.steps, WHOLE_RUN_STEPS))
    torch.cuda.synchronize()

    times, steps = [], None
    for _ in range(max(1, args.repeats)):
        work[0].copy_(ic[0])
        work[1].copy_(ic[1])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        t, n = solver.run(work[0], work[1], t_end=T_END, nsteps=args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        steps = n
    wall = sorted(times)[len(times) // 2]
    value = dofs * steps / wall

    # dominant kernel: the stage kernel, 3 launches per step; algorithmic bytes
    # per launch = (64 B per DOF-update / 3 stages) x DOFs.  Its average launch
    # time is measured live: a run of KERNEL_TIMING_STEPS steps timed with HIP
    # events on the stream the library launches on (torch's current stream
    # here), over its number of stage launches; at that length the work each
    # run does once (statistics of the initial data, final OE, host copies) is
    # below 0.5 % of the region.  The timed region of `value` above (a run of
    # `steps` steps) also holds that once-per-run work: wall_launch_us.
    bytes_per_launch = BYTES_PER_DOF_UPDATE / 3.0 * dofs
    ktimes, kn = [], steps
    for _ in range(3 if args.kernel_timing_steps > 0 else 0):
        work[0].copy_(ic[0])
        work[1].copy_(ic[1])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, kn = solver.run(work[0], work[1], t_end=T_END, nsteps=args.kernel_timing_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ktimes.append(e0.elapsed_time(e1) / 1e3)
    launch_s = (sorted(ktimes)[1] if ktimes else wall) / (3 * kn)
    achieved = bytes_per_launch / launch_s / 1e9
    prof = stage_profile()
    out = {
        "metric": "DOF-updates/s at P2 (plain vs batched) and adjoint/forward time ratio",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1D Euler two-state Riemann problem, outflow, N=16384 primal + 16385 dual cells, "
                               "P2 Legendre modal, SSP-RK3 + OE, CFL 0.15, T=0.2, seed 0",
                   "dofs": dofs, "t_end": t, "mode": args.mode, "tile": args.tile, "fold": args.fold},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": prof.get("traffic_bytes_per_launch"),
                     "kernel": "k_stage (one RK stage + OE of the previous stage)",
                     "launch_us": 1e6 * launch_s,
                     "launch_us_timing_run_steps": kn,
                     "wall_launch_us": 1e6 * wall / (3 * steps),
                     "launch_us_rocprof": prof.get("avg_duration_us"),
                     "frac_rocprof": (bytes_per_launch / (prof["avg_duration_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
                                      if prof.get("avg_duration_us") else None),
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "fp64": {"executed_tflops": (prof["fp64_flops_per_launch"] / launch_s / 1e12
                                                  if prof.get("fp64_flops_per_launch") else None),
                              "peak": FP64_PEAK_TFLOPS,
                              "executed_flops_per_dof_update": (3 * prof["fp64_flops_per_launch"] / dofs
                                                                if prof.get("fp64_flops_per_launch") else None),
                              "oracle_flops_per_dof_update": oracle_opcount("1d_euler_p2.step")},
                     "note": "state of 2.4 MB per array, resident in L2/MALL: each stage is bound by its "
                             "dependency chain (global statistics of the previous stage, damping, operator), "
                             "not by HBM bandwidth or FP64 issue"},
    }
    solver.close()
    if not args.no_batched:
        kw = dict(fold=args.batched_fold, steps=args.batched_steps, repeats=args.batched_repeats,
                  loop_baseline=not args.no_loop)
        out["batched"] = batched_bench(**kw)
        out["batched_k2"] = batched_bench(k_fixed=2, **kw)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench()
    if not args.no_2d:
        out["euler2d"] = euler2d_bench(repeats=args.e2d_repeats, steps=args.e2d_steps)
    if not args.no_widened:
        out["widened"] = widened_bench()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

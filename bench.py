#!/usr/bin/env python3
"""One-GPU benchmark of the CR-Solver hot path on MI355X (gfx950).

Workload (the configuration the headline metric is quoted on): batched two-stage
inverse kinematics of a 3-segment tendon-driven robot (segment lengths
0.10/0.08/0.06 m, tendon radii 0.010/0.008/0.006 m, |u| <= 0.008 m), 4096
reachable 6-DoF targets (forward kinematics of seeded uniform actuations), 256
uniform seeds per target, 150 FP32 + 50 FP64 Levenberg-Marquardt iterations,
N_final = 8 (Algorithm 1).  One step = one cr_solve_ik call over the whole batch
(stage 1, SelectTop, stage 2, argmin).  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line: IK solves/s, success rate at <= 1 mm / 1 degree, the
roofline of the dominant kernel (FP32 stage 1, algorithmic flops from the
library's own op tally, duration from HIP events recorded on the solve's stream)
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

WORKLOAD = "ik_batched_3seg"
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak (256 CUs, 2.4 GHz)
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=[WORKLOAD, "ik_ext_4seg", "ik_box_3seg", "path_4seg", "traj_5seg", "traj_prm_5seg",
                             "uneven_batch"],
                    help="the headline IK workload, or one of the path / trajectory workloads")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the path, trajectory and uneven-batch summaries of the headline line")
    ap.add_argument("--sub-steps", type=int, default=3, help="timed steps of each summarised workload")
    ap.add_argument("--baseline-problems", type=int, default=2,
                    help="path / trajectory problems timed with the plain per-problem baseline (0: skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the compiler's own occupancy targets instead of the library's launch autotuning")
    ap.add_argument("--force-variant", type=int, default=-1,
                    help="run occupancy variant 0, 1 or 2 of every tunable kernel (counter runs per variant)")
    ap.add_argument("--tally-seeds", type=int, default=256)
    ap.add_argument("--baseline-targets", type=int, default=16,
                    help="targets timed with the plain per-problem FP32 solve (0: skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one plain device copy of this many bytes (HBM counter calibration)")
    ap.add_argument("--no-persistent-compare", dest="persistent_compare", action="store_false",
                    help="uneven batch: skip timing the persistent IK stage 1 beside the default launches")
    ap.add_argument("--calib", action="store_true",
                    help="time the vector-ALU calibration loops (known instruction counts) and exit")
    return ap.parse_args()


def build_inputs(cr, I, torch):
    spec = I.WORKLOADS[WORKLOAD]
    n, P, S = len(spec["L"]), spec["P"], spec["S"]
    rng = I.rng_for(WORKLOAD)
    u_true = I.uniform_actuation(rng, n, spec["b"], P)               # [P, n, 3]
    seeds = I.uniform_actuation(rng, n, spec["b"], P * S)           # [P*S, n, 3]
    robot = cr.Robot(L=spec["L"], r=spec["r"], u_max=[spec["b"]] * n)
    dev = torch.device("cuda:0")
    u_true_d = torch.tensor(u_true.reshape(P, -1).T.copy(), device=dev)
    frames = cr.fk(robot, u_true_d, arc=False, frames=True)["frames"]  # [12n, P] float64
    T = frames[12 * (n - 1):12 * n].contiguous()
    useed = torch.tensor(seeds.reshape(P * S, -1).T.copy(), device=dev)
    return spec, robot, u_true, seeds, T, useed


def baseline_rate(cr, torch, robot, T, useed, spec, opts, weights, args, fused_rate):
    """The plain per-problem FP32 GPU solve (cr_baseline_solve_ik) on the first
    targets of the same workload: problems run one after another, so its rate on
    a prefix is its rate on the batch."""
    if args.baseline_targets <= 0:
        return None
    P, S = spec["P"], spec["S"]
    p = min(args.baseline_targets, P)
    Tp = T[:, :p].contiguous()
    up = useed[:, :p * S].contiguous()
    cr.baseline_solve_ik(robot, Tp, up, weights, opts)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, _, st = cr.baseline_solve_ik(robot, Tp, up, weights, opts)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rate = p / (ms * 1e-3)
    return dict(value=round(rate, 2), unit="IK solves/s", targets=p, ms=round(ms, 2),
                success_rate=round(float((st.cpu().numpy() == cr.SOLVED).mean()), 4),
                speedup_of_fused=round(fused_rate / rate, 1),
                kind="same Algorithm 1 and budgets, FP32, one problem at a time, separate kernels per step, "
                     "forward-mode Jacobian")


def plain_method(cr, torch, robot, T, useed, spec, weights, fused_rate, fused_success):
    """The plain method on the same batch (no SelectTop, no stage 2: every seed
    runs the whole iteration budget, k_init + k_final, in FP32, then the argmin),
    the ablation of Table I's row without the beam search."""
    P, S = spec["P"], spec["S"]
    opts = cr.Opts(n_final=0, k_init=spec["k_init"] + spec["k_final"], k_final=0)
    res = {}

    def step():
        res["out"] = cr.solve_ik(robot, T, useed, weights, opts, dtype=torch.float32)

    step()
    per_step, _ = step_times(torch, step, 3)
    ms = float(np.median(per_step))
    st = res["out"][2].cpu().numpy()
    return dict(value=round(P / (ms * 1e-3), 1), unit="IK solves/s", ms_per_step=round(ms, 4),
                success_rate=round(float((st == cr.SOLVED).mean()), 4), k_init=opts.k_init,
                two_stage=dict(value=round(fused_rate, 1), success_rate=round(fused_success, 4)),
                kind="stage 1 only over the whole budget, then the argmin (no SelectTop, no FP64 stage 2)")


def oracle_reassessment(spec, T34, u, err, status):
    """Every returned answer re-assessed by the FP64 CPU oracle (a zero-iteration
    plain solve from the answer itself returns the oracle's own status bits and
    errors): the largest difference from the device's FP64 errors and the success
    rate as the oracle judges it."""
    from oracle import oracle as O
    n = len(spec["L"])
    rb = O.Robot(L=spec["L"], r=spec["r"], u_max=[spec["b"]] * n)
    W, opts = O.Weights(), O.Opts(n_final=0, k_init=0, k_final=0)
    P = len(u)
    t0 = time.perf_counter()
    st_o = np.zeros(P, dtype=np.int64)
    err_o = np.zeros((P, 2))
    for p in range(P):
        res = O.solve(rb, W, O.Problem("ik", T34[p]), opts, u[p][None])
        st_o[p], err_o[p] = res["status"], res["err"]
    return dict(answers=P, seconds=round(time.perf_counter() - t0, 2),
                max_abs_diff_pos_err_m=float(np.abs(err_o[:, 0] - err[0]).max()),
                max_abs_diff_rot_err_rad=float(np.abs(err_o[:, 1] - err[1]).max()),
                status_agreement=round(float((st_o == status).mean()), 6),
                oracle_success_rate=round(float((st_o == O.SOLVED).mean()), 6),
                max_oracle_pos_err_solved_m=float(np.max(np.where(st_o == O.SOLVED, err_o[:, 0], 0.0))))


def fk_grad_rate(cr, I, torch, args):
    """FK + cost + adjoint gradient evaluations per second on the path workload's
    shape (512 paths x 32 seeds x 64 waypoints = 1,048,576 waypoint configurations
    per call), forward and backward through the torch.autograd.Function, FP32."""
    spec = I.WORKLOADS["path_4seg"]
    n, P, S, H, b = len(spec["L"]), spec["P"], spec["S"], spec["H"], spec["b"]
    Tn = H + 1
    rng = I.rng_for("path_4seg", 7)
    robot = cr.Robot(L=spec["L"], r=spec["r"], u_max=[b] * n)
    uref = I.smooth_actuation_paths(rng, n, b, P, Tn)
    dev = torch.device("cuda:0")
    fr = cr.fk(robot, torch.tensor(uref.reshape(P * Tn, -1).T.copy(), device=dev), arc=False)["frames"]
    task = fr[12 * (n - 1):12 * n].float().contiguous()
    u = uref[:, None] + rng.normal(size=(P, S, Tn, n, 3)) * 5e-4
    ut = torch.tensor(u.reshape(P * S * Tn, -1).T.copy(), device=dev, dtype=torch.float32)
    pb = cr.CostProblem(robot, "path", P, S, H, task, cr.Weights(**spec["weights"]))
    x = ut.clone().requires_grad_(True)

    def once():
        x.grad = None
        cr.CostGrad.apply(x, pb).sum().backward()

    for _ in range(2):
        once()
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    evals = P * S * Tn
    # algorithmic HBM bytes of one forward + backward: u in (3n FP32 per configuration,
    # read by both passes), the poses (12 FP32 per problem waypoint), the cost and the
    # upstream gradient per seed, the gradient out (3n FP32 per configuration)
    alg_bytes = 4 * (2 * 3 * n * evals + 12 * P * Tn + 2 * P * S + 3 * n * evals)
    out = dict(value=round(evals / (ms * 1e-3), 1), unit="FK+grad evals/s", ms_per_call=round(ms, 4),
               workload="path_4seg shape: 512 x 32 x 64 waypoint configurations, forward + backward via CostGrad, f32",
               hbm_bytes_per_call=alg_bytes,
               hbm_frac=round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    meas = stored_counters("fk_grad")
    if meas and meas.get("valu_f32_flops_per_call"):
        f = meas["valu_f32_flops_per_call"]
        out["counter_f32_flops_per_call"] = f
        out["valu_frac"] = round(f / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4)
        if meas.get("hbm_bytes_per_call"):
            out["counter_hbm_bytes_per_call"] = meas["hbm_bytes_per_call"]
    return out


def cpu_baseline(spec, T_host, seeds, budget_s):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same workload."""
    from oracle import oracle as O
    n = len(spec["L"])
    rb = O.Robot(L=spec["L"], r=spec["r"], u_max=[spec["b"]] * n)
    W = O.Weights()
    opts = O.Opts(n_final=spec["n_final"], k_init=spec["k_init"], k_final=spec["k_final"])
    S = spec["S"]
    done, t0 = 0, time.perf_counter()
    solved = 0
    while True:
        p = done
        res = O.solve(rb, W, O.Problem("ik", T_host[p]), opts, seeds[p * S:(p + 1) * S])
        solved += int(res["status"] == O.SOLVED)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or done >= spec["P"]:
            break
    return dict(value=done / el, unit="IK solves/s", cores=1, kind="oracle",
                sample=f"first {done} of {spec['P']} targets x {S} seeds, full {spec['k_init']}+{spec['k_final']} "
                       f"iterations, single thread, {el:.1f} s; {solved}/{done} solved", host=host_info())


def traj_baseline_rate(cr, torch, d, spec, opts, weights, args, fused_rate):
    """The plain per-problem FP32 path / trajectory solve (cr_baseline_solve_path /
    _traj) on the first problems of the workload: problems run one after another,
    so its rate on a prefix is its rate on the batch.  One problem is solved
    first as a warm-up."""
    if args.baseline_problems <= 0:
        return None
    robot, P, S, H = d["robot"], d["P"], d["S"], d["H"]
    Tn, n = H + 1, robot.n
    p = min(args.baseline_problems, P)
    if spec["kind"] == "path":
        task = d["task"][:, :p * Tn].contiguous()
        fn = cr.baseline_solve_path
    else:
        task = d["task"][:, :p].contiguous()
        fn = cr.baseline_solve_traj
    useed = d["useed"][:, :p * S * Tn].contiguous()
    sph = d["spheres"]
    if sph is not None:
        sph = (sph[0][:, :p * sph[2]].contiguous(), sph[1], sph[2])
    b0_opts = cr.Opts(n_final=opts.n_final, k_init=opts.k_init, k_final=opts.k_final)  # no exploration stage
    fn(robot, (task[:, :Tn] if spec["kind"] == "path" else task[:, :1]).contiguous(), useed[:, :S * Tn].contiguous(),
       H, weights, b0_opts,
       spheres=None if sph is None else (sph[0][:, :sph[2]].contiguous(), sph[1], sph[2]))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, _, st = fn(robot, task, useed, H, weights, b0_opts, spheres=sph)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rate = p / (ms * 1e-3)
    return dict(value=round(rate, 3), unit=("paths/s" if spec["kind"] == "path" else "trajectories/s"), problems=p,
                ms=round(ms, 1), success_rate=round(float((st.cpu().numpy() == cr.SOLVED).mean()), 4),
                speedup_of_fused=round(fused_rate / rate, 1),
                kind="same Algorithm 1 budgets and LM rules, FP32, one problem at a time, separate kernels per step, "
                     "forward-mode Jacobian, every point-sphere pair, one thread per trajectory for the banded solve"
                     + ("; without the per-waypoint exploration stage (its seeds are used as they are), so its "
                        "success rate is not comparable" if spec["kind"] == "path" else ""))


STAGE1_OCC = {0: 1, 1: 3, 2: 4}   # occupancy target of each IK stage-1 variant (1: the compiler's own)


def autotune(args, cr, torch, call):
    """The library's launch autotuning: one untimed call (call) times each tunable
    kernel's occupancy variants -- identical results, different speed -- and caches
    the fastest; the timed steps use the cached choices."""
    if args.force_variant >= 0:
        cr.autotune_force(args.force_variant)
        return [f"forced variant {args.force_variant}"]
    if args.no_autotune:
        return None
    cr.autotune(True)
    call()
    torch.cuda.synchronize()
    return cr.autotune_report()


def bench_calib(cr, torch):
    """Issue rate of known vector-ALU loops (cr_calib_valu): FMA, RCP, FMA + RCP,
    FP64 FMA, ADD, MUL, FMA over 32 chains, and the stage-1 FMA : MUL : ADD mix.  Rates are per CU and cycle at the 2.4 GHz peak
    clock; under rocprofv3 the same launches give the SQ_INSTS_VALU* counts."""
    blocks, iters = 8192, 2048
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    res = {}
    names = ("fma_f32", "rcp_f32", "fma_f32+rcp_f32", "fma_f64", "add_f32", "mul_f32", "fma_f32_32chains",
             "fma10_mul4_add2_f32", "fma_f32_lanes0-31", "fma_f32_lanes0-15")
    for kind, per_round in ((0, 16), (1, 16), (2, 20), (3, 16), (4, 16), (5, 16), (6, 32), (7, 16), (8, 16), (9, 16)):
        cr.calib_valu(kind, blocks, iters, out)
        torch.cuda.synchronize()
        ms = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            cr.calib_valu(kind, blocks, iters, out)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        t = float(np.median(ms))
        winst = blocks * 4 * iters * per_round
        res[names[kind]] = dict(
            ms=round(t, 4), wave_instructions=winst,
            per_cu_cycle_at_2400mhz=round(winst / (t * 1e-3) / (256 * 2.4e9), 4))
    print(json.dumps(dict(calib_valu=res, blocks=blocks, iters=iters)), flush=True)


def step_times(torch, step, k):
    """Runs k steps, each bracketed by HIP events on the current stream, inside one
    synchronised bracket; returns (per-step ms list, bracket ms)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    b0.record()
    for e0, e1 in evs:
        e0.record()
        step()
        e1.record()
    b1.record()
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in evs], b0.elapsed_time(b1)


def host_info():
    """Cores this process may use and the CPU model (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=len(os.sched_getaffinity(0)), cpu_count=os.cpu_count(), cpu_model=model)


COUNTERS_JSON = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "counters.json")


def sources_hash():
    """SHA-256 over the solver's kernel sources (the calibration loops excluded)."""
    import hashlib
    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2607_11340_amd", "csrc")
    for name in sorted(os.listdir(root)):
        if name.endswith((".hip", ".h")) and name != "cr_calib.hip":
            with open(os.path.join(root, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()


def stored_counters(workload):
    """rocprofv3 counter values stored for a workload (profiles/counters.json), or
    None when they were taken on other kernel sources than these."""
    if not os.path.exists(COUNTERS_JSON):
        return None
    with open(COUNTERS_JSON) as f:
        meas = json.load(f)
    if meas.get("sources_sha256") != sources_hash():
        return None
    return meas.get("workloads", {}).get(workload)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported (problems are "
              f"independent: several GPUs would each run one process on their share of the batch)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_11340_amd import crsolver as cr
    from paper_2607_11340_amd import inputs as I

    if args.calib:
        return bench_calib(cr, torch)
    if args.workload == "uneven_batch":
        return bench_uneven(args, cr, I, torch)
    if args.workload == "ik_ext_4seg":
        print(json.dumps(run_ik_ext(args, cr, I, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "ik_box_3seg":
        print(json.dumps(run_ik_box(args, cr, I, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "traj_prm_5seg":
        print(json.dumps(run_traj_prm(args, cr, I, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload != WORKLOAD:
        return bench_trajectories(args, cr, I, torch)
    spec, robot, u_true, seeds, T, useed = build_inputs(cr, I, torch)
    P, S = spec["P"], spec["S"]
    opts = cr.Opts(n_final=spec["n_final"], k_init=spec["k_init"], k_final=spec["k_final"])
    weights = cr.Weights()
    ws = torch.empty(cr.ik_workspace_bytes(robot, P, S, opts, torch.float32), dtype=torch.uint8, device="cuda")
    out = (torch.empty((3 * robot.n, P), dtype=torch.float64, device="cuda"),
           torch.empty((2, P), dtype=torch.float64, device="cuda"),
           torch.empty((P,), dtype=torch.int32, device="cuda"))

    def step():
        cr.solve_ik(robot, T, useed, weights, opts, dtype=torch.float32, workspace=ws, out=out)

    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = autotune(args, cr, torch, step)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    cr.lib.cr_timing_enable(1)
    per_step, total_ms = step_times(torch, step, args.steps)
    stage_ms = (C.c_double * 4)()
    ncalls = C.c_int64(0)
    cr._check(cr.lib.cr_timing_read(stage_ms, C.byref(ncalls)))
    cr.lib.cr_timing_enable(0)
    ms_per_step = float(np.median(per_step))
    stage_avg = [stage_ms[k] / max(ncalls.value, 1) for k in range(4)]
    status = out[2].cpu().numpy()
    err = out[1].cpu().numpy()
    u_host = out[0].cpu().numpy().T.reshape(P, robot.n, 3)
    success = float((status == cr.SOLVED).mean())
    print(f"bench: {args.steps} steps, median {ms_per_step:.3f} ms/step, stages {['%.3f' % s for s in stage_avg]} "
          f"ms, success {success:.4f}", file=sys.stderr, flush=True)

    # algorithmic flops of the stage-1 kernel from the library's op tally over a seed sample
    T_host = T.cpu().numpy().T.copy()                       # [P, 12]
    rng = np.random.default_rng(1)
    pick = rng.choice(P * S, size=min(args.tally_seeds, P * S), replace=False)
    Ts = np.ascontiguousarray(T_host[pick // S])
    us = np.ascontiguousarray(seeds[pick].reshape(len(pick), -1))
    tally = (C.c_double * 8)()
    rc, wc, oc = robot.c(), weights.c(), opts.c()
    cr._check(cr.lib.cr_ik_flop_tally(C.byref(rc), C.byref(wc), C.byref(oc), len(pick),
                                      Ts.ctypes.data_as(C.POINTER(C.c_double)),
                                      us.ctypes.data_as(C.POINTER(C.c_double)), tally))
    flops_per_seed = tally[0]
    flops_launch = flops_per_seed * P * S
    achieved = flops_launch / (stage_avg[0] * 1e-3) / 1e12
    occ = [l.split("occupancy ")[1].split()[0] for l in (tuned or []) if "ik_stage1 n_seg 3 f32" in l]
    if args.force_variant >= 0:
        occ = [str(STAGE1_OCC[args.force_variant])]
    kname = "k_ik_stage1<3,float,%s>" % occ[0] if occ else "k_ik_stage1<3,float,1>"  # 1: the compiler's own target
    meas = stored_counters(WORKLOAD) or {}
    kmeas = meas.get(kname, {})
    traffic = kmeas.get("hbm_bytes_per_launch")
    # a coarser count of about 3 kflop per FP32 seed-iteration, for comparison
    survey_flops = 3.0e3 * P * S * spec["k_init"]
    roofline = dict(bound="alu", kernel=kname, achieved=round(achieved, 3),
                    peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s", frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                    traffic=traffic, launch_ms=round(stage_avg[0], 4),
                    flops_per_launch=flops_launch, flops_per_seed=round(flops_per_seed, 1),
                    flops_per_seed_iteration=round(flops_per_seed / spec["k_init"], 1),
                    flops_per_normal_eq=tally[6], flops_per_cost_eval=tally[7],
                    trials_per_seed=round(tally[5], 2), tally_sample_seeds=len(pick),
                    frac_at_3kflop_per_seed_iteration=round(survey_flops / (stage_avg[0] * 1e-3) / 1e12
                                                            / FP32_VECTOR_PEAK_TFLOPS, 4))
    if kmeas:
        cf = kmeas.get("valu_f32_flops_per_launch")
        if cf:
            roofline["counter_f32_flops_per_launch"] = cf
            roofline["counter_frac"] = round(cf / (stage_avg[0] * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4)
        if traffic:
            roofline["hbm_frac"] = round(traffic / (stage_avg[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)
    lanes = [l.split("lanes per candidate ")[1].split()[0] for l in (tuned or []) if "ik_stage2 n_seg 3" in l]
    s2name = "k_ik_stage2_grp<3,float,%s>" % (lanes[0] if lanes else "2")
    if s2name in meas and meas[s2name].get("valu_f64_flops_per_launch"):
        f64 = meas[s2name]["valu_f64_flops_per_launch"]
        roofline["stage2_fp64"] = dict(kernel=s2name, counter_f64_flops_per_launch=f64, launch_ms=round(stage_avg[2], 4),
                                       frac_of_fp64_peak=round(f64 / (stage_avg[2] * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4))

    plain = plain_method(cr, torch, robot, T, useed, spec, weights, P / (ms_per_step * 1e-3), success)
    fkg = fk_grad_rate(cr, I, torch, args)
    b0 = baseline_rate(cr, torch, robot, T, useed, spec, opts, weights, args, P / (ms_per_step * 1e-3))
    del ws
    torch.cuda.empty_cache()
    subs = {}
    if not args.headline_only:
        for name in ("ik_ext_4seg", "ik_box_3seg", "path_4seg", "traj_5seg", "traj_prm_5seg", "uneven_batch"):
            print(f"bench: workload {name}", file=sys.stderr, flush=True)
            subs[name] = sub_workload(name, args, cr, I, torch)
            torch.cuda.empty_cache()

    base = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle and re-assessing every answer with it", file=sys.stderr, flush=True)
        T34 = T_host.reshape(P, 3, 4)
        base = cpu_baseline(spec, T34, seeds, args.cpu_seconds)
        base["reassessment"] = oracle_reassessment(spec, T34, u_host, err, status)

    line = dict(
        metric="IK solves/sec at <=1 mm/1 deg (success %); FK+grad evals/sec; %FP32 VALU peak",
        value=round(P / (ms_per_step * 1e-3), 1), unit="IK solves/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_per_step, 4), ms_per_step_mean=round(total_ms / args.steps, 4),
        ms_per_step_range=[round(min(per_step), 4), round(max(per_step), 4)], higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", refine_dtype="f64", data="synthetic",
        config=dict(workload=WORKLOAD, segments=len(spec["L"]), targets=P, seeds_per_target=S,
                    k_init=spec["k_init"], k_final=spec["k_final"], n_final=spec["n_final"]),
        success_rate=round(success, 4), max_pos_err_solved_m=float(np.nanmax(np.where(status == cr.SOLVED, err[0], 0))),
        stage_ms=dict(stage1=round(stage_avg[0], 4), select=round(stage_avg[1], 4), stage2=round(stage_avg[2], 4),
                      finalize=round(stage_avg[3], 4)),
        plain_method=plain, fk_grad=fkg, workloads=subs, plain_gpu_baseline=b0, roofline=roofline,
        cpu_baseline=base, autotune=tuned, host=host_info())
    print(json.dumps(line), flush=True)


def traj_inputs(name, cr, I, torch, O=None):
    """Seeded inputs of the path-following or trajectory workload (host arrays plus
    device tensors).  Path: smooth reference actuation paths, their FK poses as
    reference, uniform IK seeds per (seed, waypoint) for the exploration stage
    (per-waypoint IK, then path assembly).  Trajectory: uniform start/goal
    actuations with tip distance >= 0.1 of the robot length, perturbed
    straight-line seeds, spheres with centres uniform in the bounding box of the
    tips of 4096 uniform actuations, radii U[5, 20] mm, rejected if they come
    within 1 mm of the start or goal backbone."""
    spec = I.WORKLOADS[name]
    n, P, S, H, b = len(spec["L"]), spec["P"], spec["S"], spec["H"], spec["b"]
    Tn = H + 1
    rng = I.rng_for(name)
    K = spec["K"]
    robot = cr.Robot(L=spec["L"], r=spec["r"], u_max=[b] * n, pts_per_seg=K)
    dev = torch.device("cuda:0")
    out = dict(spec=spec, robot=robot, n=n, P=P, S=S, H=H)
    if spec["kind"] == "path":
        uref = I.smooth_actuation_paths(rng, n, b, P, Tn)                    # [P, Tn, n, 3]
        fr = cr.fk(robot, torch.tensor(uref.reshape(P * Tn, -1).T.copy(), device=dev), arc=False)["frames"]
        out["task"] = fr[12 * (n - 1):12 * n].contiguous()                  # [12, Tn*P]
        seeds = I.uniform_actuation(rng, n, b, P * S * Tn).reshape(P, S, Tn, n, 3)
        out["spheres"] = None
    else:
        # start / goal pairs whose tips are at least 0.1 of the robot length apart
        reach = float(sum(spec["L"]))
        ends = np.zeros((P, 2, n, 3))
        filled = 0
        while filled < P:
            cand = I.uniform_actuation(rng, n, b, 2 * P).reshape(P, 2, n, 3)
            fr = cr.fk(robot, torch.tensor(cand.reshape(2 * P, -1).T.copy(), device=dev), arc=False)["frames"]
            tips = fr[12 * (n - 1):12 * n].cpu().numpy().T.reshape(P, 2, 3, 4)[:, :, :, 3]
            keep = cand[np.linalg.norm(tips[:, 0] - tips[:, 1], axis=1) >= 0.1 * reach]
            take = min(len(keep), P - filled)
            ends[filled:filled + take] = keep[:take]
            filled += take
        samp = I.uniform_actuation(rng, n, b, 4096)
        fr = cr.fk(robot, torch.tensor(samp.reshape(4096, -1).T.copy(), device=dev), arc=False)["frames"]
        tips = fr[12 * (n - 1):12 * n].cpu().numpy().T.reshape(4096, 3, 4)[:, :, 3]
        lo, hi = tips.min(axis=0), tips.max(axis=0)
        if "prm" in spec:   # the seeds' perturbations, applied by the initializer on the device
            bumps = np.stack([I.path_bumps(rng, n, S, Tn, b) for p in range(P)])
            out["bump"] = torch.tensor(bumps.reshape(P * S * Tn, -1).T.copy(), device=dev)
            seeds = None
        else:
            seeds = np.stack([I.perturbed_linear_paths(rng, ends[p, 0], ends[p, 1], S, Tn, b) for p in range(P)])
        out["task"] = torch.tensor(np.concatenate([ends[:, 0].reshape(P, -1), ends[:, 1].reshape(P, -1)], 1).T.copy(),
                                   device=dev)
        M = spec["M"]

        def points(u):
            res = cr.fk(robot, torch.tensor(u.reshape(len(u), -1).T.copy(), device=dev), arc=False, frames=False,
                        points=True)["pts"].cpu().numpy().T
            return res.reshape(len(u), n * K, 3)

        pts = points(ends.reshape(2 * P, n, 3)).reshape(P, 2 * n * K, 3)
        sph = np.zeros((P, M, 4))
        body = np.tile(np.repeat(np.asarray(spec["r"]), K), 2)
        nb = spec.get("blockers", 0)
        have = np.zeros(P, dtype=int)
        if nb:
            sph[:, :nb], have = I.line_blockers(rng, ends, nb, *spec.get("sph_r", (0.005, 0.02)), points,
                                                np.repeat(np.asarray(spec["r"]), K))
            out["blockers"] = have
        for p in range(P):
            m = int(have[p])
            while m < M:
                cand = I.spheres(rng, 2 * M, lo, hi, *spec.get("sph_r", (0.005, 0.02)))
                for s in cand:
                    if m < M and (np.linalg.norm(pts[p] - s[:3], axis=1) - s[3] - body).min() > 1e-3:
                        sph[p, m] = s
                        m += 1
        out["spheres"] = (torch.tensor(np.ascontiguousarray(sph.reshape(P * M, 4).T), device=dev), True, M)
        out["sph_host"] = sph
        out["ends"] = ends
    out["seeds"] = seeds
    if seeds is not None:
        out["useed"] = torch.tensor(seeds.reshape(P * S * Tn, -1).T.copy(), device=dev)
    return out


def bench_trajectories(args, cr, I, torch):
    print(json.dumps(run_trajectories(args.workload, args, cr, I, torch, args.steps, args.warmup, True)), flush=True)


def run_trajectories(name, args, cr, I, torch, steps, warmup, extras):
    d = traj_inputs(name, cr, I, torch)
    spec, robot, P, S, H = d["spec"], d["robot"], d["P"], d["S"], d["H"]
    opts = cr.Opts(n_final=spec["n_final"], k_init=spec["k_init"], k_final=spec["k_final"],
                   k_seed=spec.get("k_seed", 0))
    weights = cr.Weights(**spec.get("weights", {}))
    ws = torch.empty(cr.traj_workspace_bytes(robot, P, H, S, opts, torch.float32), dtype=torch.uint8, device="cuda")
    out = (torch.empty((3 * robot.n, (H + 1) * P), dtype=torch.float64, device="cuda"),
           torch.empty((2, P), dtype=torch.float64, device="cuda"),
           torch.empty((P,), dtype=torch.int32, device="cuda"))
    fn = cr.solve_path if spec["kind"] == "path" else cr.solve_traj

    def step():
        fn(robot, d["task"], d["useed"], H, weights, opts, dtype=torch.float32, spheres=d["spheres"], workspace=ws,
           out=out)

    tuned = autotune(args, cr, torch, step)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({warmup} steps)", file=sys.stderr, flush=True)
    per_step, total = step_times(torch, step, steps)
    ms = float(np.median(per_step))
    status = out[2].cpu().numpy()
    err = out[1].cpu().numpy()
    unit = "paths/s" if spec["kind"] == "path" else "trajectories/s"
    line = dict(metric=f"{spec['kind']} solves/sec (success %)", value=round(P / (ms * 1e-3), 2), unit=unit, n_gpus=1,
                steps=steps, warmup=warmup, ms_per_step=round(ms, 4), ms_per_step_mean=round(total / steps, 4),
                higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32", refine_dtype="f64", data="synthetic",
                config=dict(workload=name, segments=robot.n, problems=P, waypoints=H + 1, seeds=S,
                            spheres=spec.get("M", 0), pts_per_seg=robot.pts_per_seg, k_init=spec["k_init"],
                            k_final=spec["k_final"], n_final=spec["n_final"], k_seed=spec.get("k_seed", 0)),
                success_rate=round(float((status == cr.SOLVED).mean()), 4),
                status_counts={int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
                max_err_solved=[float(np.max(np.where(status == cr.SOLVED, err[k], 0))) for k in range(2)],
                autotune=tuned)
    line.update(counter_roofline(name, ms))
    if extras:
        print("bench: timing the plain per-problem baseline", file=sys.stderr, flush=True)
        line["plain_gpu_baseline"] = traj_baseline_rate(cr, torch, d, spec, opts, weights, args, line["value"])
        if not args.no_cpu_baseline:
            print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
            line["cpu_baseline"] = traj_cpu_baseline(d, spec, weights, opts, args.cpu_seconds)
    return line


def event_ms(torch, fn, reps):
    """Median duration (ms) of fn() over reps runs, HIP events on the current stream."""
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def run_traj_prm(args, cr, I, torch, steps, warmup):
    """Trajectory planning with the PRM initializer (Algorithm 2) against the
    straight-line initializer on the same scenes, seeds' perturbations and solve:
    one step = the online query on every problem (ConnectToRoadmap, Dijkstra,
    ResampleLinear, seeds) plus the two-stage solve.  The roadmaps are built once
    (offline) and timed on their own."""
    name = "traj_prm_5seg"
    d = traj_inputs(name, cr, I, torch)
    spec, robot, P, S, H = d["spec"], d["robot"], d["P"], d["S"], d["H"]
    pr = spec["prm"]
    prm = cr.PrmOpts(n_nodes=pr["n_nodes"], k=pr["k"], n_check=pr["n_check"], max_attempts=pr["max_attempts"],
                     key=(spec["seed"], 2))
    rm = cr.prm_build(robot, P, prm, spheres=d["spheres"])
    torch.cuda.synchronize()
    build_ms = event_ms(torch, lambda: cr.prm_build(robot, P, prm, spheres=d["spheres"]), 3)
    att = rm["attempts"].cpu().numpy()
    nbr = rm["nbr"].cpu().numpy()
    opts = cr.Opts(n_final=spec["n_final"], k_init=spec["k_init"], k_final=spec["k_final"])
    weights = cr.Weights(**spec.get("weights", {}))
    ws = torch.empty(cr.traj_workspace_bytes(robot, P, H, S, opts, torch.float32), dtype=torch.uint8, device="cuda")
    out = (torch.empty((3 * robot.n, (H + 1) * P), dtype=torch.float64, device="cuda"),
           torch.empty((2, P), dtype=torch.float64, device="cuda"),
           torch.empty((P,), dtype=torch.int32, device="cuda"))
    qout = (torch.empty((3 * robot.n, (H + 1) * S * P), dtype=torch.float64, device="cuda"),
            torch.empty((P,), dtype=torch.int32, device="cuda"))

    def query(linear):
        cr.prm_query(robot, prm, d["task"], H, S, roadmap=rm, bump=d["bump"], linear=linear, spheres=d["spheres"],
                     out=qout)

    def step(linear=False):
        query(linear)
        cr.solve_traj(robot, d["task"], qout[0], H, weights, opts, dtype=torch.float32, spheres=d["spheres"],
                      workspace=ws, out=out)

    tuned = autotune(args, cr, torch, step)
    res = {}
    for linear in (False, True):
        for _ in range(warmup):
            step(linear)
        torch.cuda.synchronize()
        per_step, total = step_times(torch, lambda: step(linear), steps)
        st = out[2].cpu().numpy()
        npath = qout[1].cpu().numpy()
        ms = float(np.median(per_step))
        res[linear] = dict(value=round(P / (ms * 1e-3), 2), unit="trajectories/s", ms_per_step=round(ms, 4),
                           ms_per_step_mean=round(total / steps, 4),
                           success_rate=round(float((st == cr.SOLVED).mean()), 4),
                           status_counts={int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
                           query_ms=round(event_ms(torch, lambda: query(linear), 3), 4))
        if not linear:
            res[linear]["paths"] = dict(connected=round(float((npath >= 0).mean()), 4),
                                        detour=round(float((npath > 0).mean()), 4),
                                        mean_roadmap_nodes=round(float(npath[npath >= 0].mean()), 2)
                                        if (npath >= 0).any() else None)
        print(f"bench: {name} {'linear' if linear else 'prm'} {res[linear]}", file=sys.stderr, flush=True)
    line = dict(metric="trajectory solves/sec with the PRM initializer (success %)", value=res[False]["value"],
                unit="trajectories/s", n_gpus=1, steps=steps, warmup=warmup, ms_per_step=res[False]["ms_per_step"],
                ms_per_step_mean=res[False]["ms_per_step_mean"], higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32", refine_dtype="f64", data="synthetic",
                config=dict(workload=name, segments=robot.n, problems=P, waypoints=H + 1, seeds=S,
                            spheres=spec["M"], blockers=spec["blockers"],
                            blockers_mean=round(float(d["blockers"].mean()), 3), pts_per_seg=robot.pts_per_seg,
                            k_init=spec["k_init"], k_final=spec["k_final"], n_final=spec["n_final"], prm=pr),
                success_rate=res[False]["success_rate"], status_counts=res[False]["status_counts"],
                initializer="prm", query=dict(ms=res[False]["query_ms"], **res[False]["paths"]),
                linear_initializer={k: v for k, v in res[True].items() if k != "query_ms"} | dict(
                    query_ms=res[True]["query_ms"]),
                roadmap=dict(build_ms=round(build_ms, 3), nodes=P * prm.n_nodes,
                             kept_nodes=int((att > 0).sum()),
                             free_motions=int((nbr >= 0).sum()),
                             colliding_motions=int(((nbr < 0) & (nbr != cr.PRM_NONE)).sum())),
                autotune=tuned)
    return line


def counter_roofline(name, ms):
    """Vector-ALU rate of a whole step from stored rocprofv3 op counters (FP32 and
    FP64 flops per step, masked lanes included) over this run's step time."""
    meas = stored_counters(name)
    if not meas:
        return dict(counter_roofline=None)
    f32, f64 = meas.get("valu_f32_flops_per_step", 0.0), meas.get("valu_f64_flops_per_step", 0.0)
    return dict(counter_roofline=dict(
        bound="alu", unit="TFLOP/s", f32_flops_per_step=f32, f64_flops_per_step=f64,
        f32_achieved=round(f32 / (ms * 1e-3) / 1e12, 3), frac_fp32=round(f32 / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
        frac_fp64=round(f64 / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4),
        dominant_kernel=meas.get("dominant_kernel"), source=meas.get("source")))


def run_ik_ext(args, cr, I, torch, steps, warmup):
    """Two-stage IK of a 4-segment robot with extensible segments (lengths free in
    [0.5, 1.5] of nominal) among a jittered 3 x 3 x 3 sphere lattice: targets from
    forward kinematics of uniform bending and extension, kept only when their
    backbone clears every sphere by 2 mm; uniform seeds of bending and extension."""
    name = "ik_ext_4seg"
    spec = I.WORKLOADS[name]
    n, P, S, b, K = len(spec["L"]), spec["P"], spec["S"], spec["b"], spec["K"]
    rng = I.rng_for(name)
    robot = cr.Robot(L=spec["L"], r=spec["r"], u_max=[b] * n, pts_per_seg=K, L_min=spec["L_min"], L_max=spec["L_max"])
    lat = spec["lattice"]
    sph = I.sphere_lattice(rng, lat["xy"], lat["z"], lat["radius"], lat["jitter"])
    e_lo = [lo - L for lo, L in zip(spec["L_min"], spec["L"])]
    e_hi = [hi - L for hi, L in zip(spec["L_max"], spec["L"])]
    dev = torch.device("cuda:0")
    body = np.repeat(np.asarray(spec["r"]), K)
    keep = []
    while sum(len(k) for k in keep) < P:
        cand = I.extended_actuation(rng, n, b, [0.75 * e for e in e_lo], [0.75 * e for e in e_hi], 2 * P)
        out = cr.fk(robot, torch.tensor(cand.reshape(2 * P, -1).T.copy(), device=dev), arc=False, points=True)
        pts = out["pts"].cpu().numpy().T.reshape(2 * P, n * K, 3)
        gap = (np.linalg.norm(pts[:, :, None, :] - sph[None, None, :, :3], axis=3) - sph[None, None, :, 3]
               - body[None, :, None]).min(axis=(1, 2))
        keep.append(cand[gap > 2e-3])
    u_true = np.concatenate(keep)[:P]
    fr = cr.fk(robot, torch.tensor(u_true.reshape(P, -1).T.copy(), device=dev), arc=False)["frames"]
    T = fr[12 * (n - 1):12 * n].contiguous()
    seeds = I.extended_actuation(rng, n, b, e_lo, e_hi, P * S)
    useed = torch.tensor(seeds.reshape(P * S, -1).T.copy(), device=dev)
    sp = (torch.tensor(np.ascontiguousarray(sph.T), device=dev), False, len(sph))
    opts = cr.Opts(n_final=spec["n_final"], k_init=spec["k_init"], k_final=spec["k_final"])
    weights = cr.Weights()
    ws = torch.empty(cr.ik_workspace_bytes(robot, P, S, opts, torch.float32), dtype=torch.uint8, device="cuda")
    out = (torch.empty((3 * n, P), dtype=torch.float64, device="cuda"),
           torch.empty((2, P), dtype=torch.float64, device="cuda"),
           torch.empty((P,), dtype=torch.int32, device="cuda"))

    def step():
        cr.solve_ik(robot, T, useed, weights, opts, dtype=torch.float32, spheres=sp, workspace=ws, out=out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    per_step, total = step_times(torch, step, steps)
    ms = float(np.median(per_step))
    st = out[2].cpu().numpy()
    line = dict(metric="extendable IK solves/sec (success %)", value=round(P / (ms * 1e-3), 1), unit="IK solves/s",
                n_gpus=1, steps=steps, warmup=warmup, ms_per_step=round(ms, 4), ms_per_step_mean=round(total / steps, 4),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", refine_dtype="f64",
                data="synthetic",
                config=dict(workload=name, segments=n, targets=P, seeds_per_target=S, spheres=len(sph),
                            length_bounds=[spec["L_min"][0], spec["L_max"][0]], k_init=spec["k_init"],
                            k_final=spec["k_final"], n_final=spec["n_final"]),
                success_rate=round(float((st == cr.SOLVED).mean()), 4),
                status_counts={int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))})
    line.update(counter_roofline(name, ms))
    return line


def run_ik_box(args, cr, I, torch, steps, warmup):
    """Two-stage IK of the 3-segment robot among 12 oriented boxes per problem
    (convex obstacles in half-space form): targets from forward kinematics of
    uniform actuations; boxes drawn per problem and kept only when the target's
    backbone clears them by 3 mm; uniform seeds."""
    name = "ik_box_3seg"
    spec = I.WORKLOADS[name]
    n, P, S, b, K = len(spec["L"]), spec["P"], spec["S"], spec["b"], spec["K"]
    bx = spec["boxes"]
    rng = I.rng_for(name)
    robot = cr.Robot(L=spec["L"], r=spec["r"], u_max=[b] * n, pts_per_seg=K)
    dev = torch.device("cuda:0")
    u_true = I.uniform_actuation(rng, n, b, P)
    out = cr.fk(robot, torch.tensor(u_true.reshape(P, -1).T.copy(), device=dev), arc=False, points=True)
    pts = out["pts"].cpu().numpy().T.reshape(P, n * K, 3)
    T = out["frames"][12 * (n - 1):12 * n].contiguous()
    body = np.repeat(np.asarray(spec["r"]), K)
    planes = np.zeros((P, bx["count"], 6, 4))
    for p in range(P):
        j = 0
        while j < bx["count"]:
            c, h, R = I.random_boxes(rng, 4 * bx["count"], bx["lo"], bx["hi"], bx["half_lo"], bx["half_hi"])
            for q in range(len(c)):
                pl = I.box_halfspaces(c[q], h[q], R[q])
                sd = (pts[p] @ pl[:, :3].T - pl[None, :, 3]).max(axis=1)
                if (sd - body).min() > bx["clear"] and j < bx["count"]:
                    planes[p, j] = pl
                    j += 1
    seeds = I.uniform_actuation(rng, n, b, P * S)
    useed = torch.tensor(seeds.reshape(P * S, -1).T.copy(), device=dev)
    po = (torch.tensor(np.ascontiguousarray(planes.reshape(-1, 4).T), device=dev), True, bx["count"], 6)
    opts = cr.Opts(n_final=spec["n_final"], k_init=spec["k_init"], k_final=spec["k_final"])
    weights = cr.Weights()
    ws = torch.empty(cr.ik_workspace_bytes(robot, P, S, opts, torch.float32), dtype=torch.uint8, device="cuda")
    res = (torch.empty((3 * n, P), dtype=torch.float64, device="cuda"),
           torch.empty((2, P), dtype=torch.float64, device="cuda"),
           torch.empty((P,), dtype=torch.int32, device="cuda"))

    def step():
        cr.solve_ik(robot, T, useed, weights, opts, dtype=torch.float32, workspace=ws, out=res, polytopes=po)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    per_step, total = step_times(torch, step, steps)
    ms = float(np.median(per_step))
    st = res[2].cpu().numpy()
    line = dict(metric="IK among convex obstacles solves/sec (success %)", value=round(P / (ms * 1e-3), 1),
                unit="IK solves/s", n_gpus=1, steps=steps, warmup=warmup, ms_per_step=round(ms, 4),
                ms_per_step_mean=round(total / steps, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", refine_dtype="f64", data="synthetic",
                config=dict(workload=name, segments=n, targets=P, seeds_per_target=S, boxes=bx["count"],
                            planes_per_box=6, k_init=spec["k_init"], k_final=spec["k_final"],
                            n_final=spec["n_final"]),
                success_rate=round(float((st == cr.SOLVED).mean()), 4),
                status_counts={int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))})
    line.update(counter_roofline(name, ms))
    return line


def sub_workload(name, args, cr, I, torch):
    """A compact line of one of the other workloads for the headline JSON."""
    if name == "ik_ext_4seg":
        ln = run_ik_ext(args, cr, I, torch, args.sub_steps, 1)
    elif name == "ik_box_3seg":
        ln = run_ik_box(args, cr, I, torch, args.sub_steps, 1)
    elif name == "uneven_batch":
        ln = run_uneven(args, cr, I, torch, args.sub_steps, 1, False)
    elif name == "traj_prm_5seg":
        ln = run_traj_prm(args, cr, I, torch, args.sub_steps, 1)
    else:
        ln = run_trajectories(name, args, cr, I, torch, args.sub_steps, 1, False)
    keep = ("value", "unit", "ms_per_step", "ms_per_step_mean", "steps", "success_rate", "success_by_kind",
            "status_counts", "config", "counter_roofline", "autotune", "initializer", "linear_initializer", "roadmap",
            "query", "ik_stage1_persistent")
    return {k: ln[k] for k in keep if k in ln}


def traj_cpu_baseline(d, spec, weights, opts, budget_s):
    """The FP64 CPU oracle on whole problems of the same workload (path: all 32
    seeds; trajectory: the first 4 of 64 seeds, the per-problem time scaled by
    64 / 4, since stage 1 costs the same per seed and dominates)."""
    from oracle import oracle as O
    n, H, S = d["n"], d["H"], d["S"]
    rb = O.Robot(L=spec["L"], r=spec["r"], u_max=[spec["b"]] * n, pts_per_seg=spec["K"])
    W = O.Weights(**{k: getattr(weights, k) for k in ("w_pos", "w_rot", "rho_lim", "rho_curv", "rho_coll", "margin",
                                                         "rho_eq", "w_len", "w_vel", "w_acc", "v_max", "a_max", "dt")})
    oo = O.Opts(n_final=opts.n_final, k_init=opts.k_init, k_final=opts.k_final, k_seed=opts.k_seed)
    s_used = S if spec["kind"] == "path" else 4
    done, t0 = 0, time.perf_counter()
    task_host = d["task"].cpu().numpy()
    while True:
        p = done
        if spec["kind"] == "path":
            T = task_host[:, p * (H + 1):(p + 1) * (H + 1)].T.reshape(H + 1, 3, 4)
            pb = O.Problem("path", T, H=H)
        else:
            pb = O.Problem("traj", (d["ends"][p, 0], d["ends"][p, 1]), H=H, spheres=d["sph_host"][p])
        O.solve(rb, W, pb, oo, d["seeds"][p, :s_used])
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or done >= d["P"]:
            break
    scale = S / s_used
    return dict(value=round(done / (el * scale), 5), unit="paths/s" if spec["kind"] == "path" else "trajectories/s",
                cores=1, kind="oracle",
                sample=f"{done} problem(s) of the workload, {s_used} of {S} seeds each, full iteration budget, single "
                       f"thread, {el:.1f} s" + (f"; time per problem scaled by {S}/{s_used}" if scale != 1 else ""))


def uneven_inputs(cr, I, torch, P):
    """The uneven batch: problem shapes and draws from the inputs recipe; tasks by
    forward kinematics on the GPU; spheres kept only if they clear the problem's
    target (IK), reference (path) or start and goal (trajectory) backbones by 2 mm."""
    spec = I.UNEVEN
    rng = np.random.Generator(np.random.PCG64(spec["seed"]))
    probs = I.uneven_problems(rng, P)
    L, r, b, K = spec["L"], spec["r"], spec["b"], spec["K"]
    robots = [cr.Robot(L=[L] * n, r=[r] * n, u_max=[b] * n, pts_per_seg=K) for n in range(1, 7)]
    dev = torch.device("cuda:0")
    # forward kinematics of every task configuration, one call per segment count
    cfg = {}
    for n in range(1, 7):
        rows = [(q, pb) for q, pb in enumerate(probs) if pb["n"] == n]
        us, owners = [], []
        for q, pb in rows:
            u = pb["u_true"][None] if pb["kind"] == "ik" else (pb["u_ref"] if pb["kind"] == "path"
                                                                else np.stack([pb["u_start"], pb["u_goal"]]))
            us.append(u)
            owners.append((q, len(u)))
        if not us:
            continue
        U = np.concatenate(us).reshape(-1, 3 * n)
        out = cr.fk(robots[n - 1], torch.tensor(U.T.copy(), device=dev), arc=False, frames=True, points=True)
        fr = out["frames"][12 * (n - 1):12 * n].cpu().numpy().T            # [B, 12]
        pts = out["pts"].cpu().numpy().T.reshape(len(U), n * K, 3)
        at = 0
        for q, m in owners:
            cfg[q] = (fr[at:at + m], pts[at:at + m])
            at += m
    batch_probs, n_kept = [], 0
    for q, pb in enumerate(probs):
        n, Tn = pb["n"], pb["H"] + 1
        fr, pts = cfg[q]
        body = np.tile(np.repeat(np.full(n, r), K), len(pts))
        P3 = pts.reshape(-1, 3)
        pool = pb["sphere_pool"]
        clear = (np.linalg.norm(P3[None] - pool[:, None, :3], axis=2) - pool[:, 3:4] - body[None]).min(axis=1) > 2e-3
        sph = pool[clear][:pb["M"]]
        n_kept += len(sph)
        if pb["kind"] == "ik":
            task = fr[0].reshape(3, 4)
            seeds = pb["seeds"][:, 0]
        elif pb["kind"] == "path":
            task = fr.reshape(Tn, 3, 4)
            seeds = pb["seeds"]
        else:
            task = (pb["u_start"], pb["u_goal"])
            seeds = pb["seeds"]
        batch_probs.append(dict(kind=pb["kind"], robot=n - 1, H=pb["H"], task=task, seeds=seeds,
                                spheres=sph if len(sph) else None))
    return cr.Batch(robots, batch_probs), probs, n_kept, (robots, batch_probs)


def uneven_baseline_estimate(cr, torch, singles, weights, opts, args, fused_rate):
    """The plain per-problem FP32 solves (cr_baseline_solve_ik / _path / _traj) on
    the first problems of each kind in batch order, each with its own robot,
    horizon, seeds and spheres; the batch's time is estimated as the sum over kinds
    of (problems of that kind) x (mean sampled time)."""
    k = args.baseline_problems
    if k <= 0:
        return None
    robots, probs = singles
    dev = torch.device("cuda:0")
    times, counts, sampled = {}, {}, {}
    for pb in probs:
        counts[pb["kind"]] = counts.get(pb["kind"], 0) + 1
    for kind in ("ik", "path", "traj"):
        picks = [pb for pb in probs if pb["kind"] == kind][:k]
        ts = []
        for pb in picks:
            rb = robots[pb["robot"]]
            n, H = rb.n, pb["H"]
            Tn, S = H + 1, pb["seeds"].shape[0]
            sph = pb["spheres"]
            sp = None if sph is None else (torch.tensor(np.ascontiguousarray(sph.T), device=dev), False, len(sph))
            wk, ok = weights[("ik", "path", "traj").index(kind)], opts[("ik", "path", "traj").index(kind)]
            b0o = cr.Opts(n_final=ok.n_final, k_init=ok.k_init, k_final=ok.k_final)
            if kind == "ik":
                T = torch.tensor(np.asarray(pb["task"]).reshape(12, 1), device=dev)
                us = torch.tensor(pb["seeds"].reshape(S, 3 * n).T.copy(), device=dev)
                call = lambda: cr.baseline_solve_ik(rb, T, us, wk, b0o, spheres=sp)
            else:
                us = torch.tensor(pb["seeds"].reshape(S * Tn, 3 * n).T.copy(), device=dev)
                if kind == "path":
                    task = torch.tensor(np.asarray(pb["task"]).reshape(Tn, 12).T.copy(), device=dev)
                    call = lambda: cr.baseline_solve_path(rb, task, us, H, wk, b0o, spheres=sp)
                else:
                    ends = np.concatenate([np.ravel(pb["task"][0]), np.ravel(pb["task"][1])]).reshape(-1, 1)
                    task = torch.tensor(ends, device=dev)
                    call = lambda: cr.baseline_solve_traj(rb, task, us, H, wk, b0o, spheres=sp)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        if ts:
            times[kind] = sum(ts) / len(ts)
            sampled[kind] = len(ts)
    total_ms = sum(counts[kd] * times[kd] for kd in times)
    rate = sum(counts[kd] for kd in times) / (total_ms * 1e-3)
    return dict(value=round(rate, 3), unit="problems/s", estimate=True,
                mean_ms_per_problem={kd: round(v, 1) for kd, v in times.items()}, sampled=sampled, counts=counts,
                speedup_of_fused=round(fused_rate / rate, 1),
                kind="plain per-problem FP32 solves of each kind, timed on the first problems of that kind, scaled "
                     "by the kind's count; path problems without the per-waypoint exploration stage")


def bench_uneven(args, cr, I, torch):
    print(json.dumps(run_uneven(args, cr, I, torch, args.steps, args.warmup, True)), flush=True)


def run_uneven(args, cr, I, torch, steps, warmup, extras):
    P = I.UNEVEN["P"]
    t0 = time.perf_counter()
    batch, probs, n_sph, singles = uneven_inputs(cr, I, torch, P)
    print(f"bench: uneven batch built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    specs = [I.WORKLOADS[k] for k in ("ik_batched_3seg", "path_4seg", "traj_5seg")]
    opts = [cr.Opts(n_final=s["n_final"], k_init=s["k_init"], k_final=s["k_final"], k_seed=s.get("k_seed", 0))
            for s in specs]
    weights = [cr.Weights(), cr.Weights(**specs[1]["weights"]), cr.Weights()]
    ws = torch.empty(cr.batch_workspace_bytes(batch, opts, torch.float32), dtype=torch.uint8, device="cuda")
    dev = tuple(torch.tensor(a if a.size else [0.0], dtype=torch.float64, device="cuda")
                for a in (batch.task, batch.seed, batch.sph))
    out = (torch.empty(batch.n_out, dtype=torch.float64, device="cuda"),
           torch.empty((2, P), dtype=torch.float64, device="cuda"), torch.empty(P, dtype=torch.int32, device="cuda"))

    def step(graph=True, persistent=False):
        cr.solve_batch(batch, weights, opts, dtype=torch.float32, workspace=ws, dev_arrays=dev, graph=graph, out=out,
                       persistent=persistent)

    # IK stage 1 as one persistent work-queue kernel per group (SelectTop fused),
    # timed beside the default grid launches; same results bit for bit
    alt = {}
    for pers in ((True, False) if args.persistent_compare else (False,)):
        # tuned eagerly: the graph captured by the first warm-up step then holds the chosen variants
        tuned = autotune(args, cr, torch, lambda: step(graph=False, persistent=pers))
        for _ in range(warmup):
            step(persistent=pers)
        torch.cuda.synchronize()
        print(f"bench: warmup done ({warmup} steps, persistent={pers})", file=sys.stderr, flush=True)
        per_step, total = step_times(torch, lambda: step(persistent=pers), steps)
        ms = float(np.median(per_step))
        if pers:
            res_p = [x.clone() for x in out]
            alt = dict(ms_per_step=round(ms, 3), value=round(P / (ms * 1e-3), 2))
    if alt:
        alt["identical_results"] = all(bool(torch.equal(a, b)) for a, b in zip(res_p, out))
    st = out[2].cpu().numpy()
    kinds = np.array([("ik", "path", "traj").index(p["kind"]) for p in probs])
    succ = {k: round(float((st[kinds == i] == cr.SOLVED).mean()), 4) for i, k in enumerate(("ik", "path", "traj"))}
    line = dict(metric="uneven batch solves/sec (success %)", value=round(P / (ms * 1e-3), 2), unit="problems/s",
                n_gpus=1, steps=steps, warmup=warmup, ms_per_step=round(ms, 3), ms_per_step_mean=round(total / steps, 3),
                higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32", refine_dtype="f64", data="synthetic",
                config=dict(workload="uneven_batch", problems=P, mix=dict(ik=int((kinds == 0).sum()),
                                                                          path=int((kinds == 1).sum()),
                                                                          traj=int((kinds == 2).sum())),
                            segments="U{1..6}", horizons="U{1..64}", seeds="U{16..512}", spheres="U{0..64}",
                            spheres_kept=n_sph, seeds_total=int(sum(p["S"] for p in probs)), graph=True),
                success_rate=round(float((st == cr.SOLVED).mean()), 4), success_by_kind=succ, autotune=tuned,
                ik_stage1_persistent=alt or None)
    line.update(counter_roofline("uneven_batch", ms))
    if extras:
        print("bench: timing the plain per-problem baseline on a per-kind sample", file=sys.stderr, flush=True)
        line["plain_gpu_baseline"] = uneven_baseline_estimate(cr, torch, singles, weights, opts, args, line["value"])
    return line


if __name__ == "__main__":
    main()

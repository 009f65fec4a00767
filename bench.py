"""Benchmark of the coupled hybrid LB step on one MI355X.

Workload: the 128^3 chiral droplet (radius 32, q0 = 2 pi/24, zeta = 0.008),
FP32 storage and arithmetic, D3Q19 with the stress as a body force; the same
box is also timed in FP64, with FP16 population storage, and with the paper's
D3Q15 scheme (symmetric stress in the equilibrium) in FP32 and FP64.  A step is one pass of the whole coupled step over the box
(stress, collide + stream, Q and phi updates).  Inputs are resident in HBM
before the timed region starts.

Prints one JSON line with MLUPS (whole job), the roofline of the dominant
kernel (algorithmic bytes per launch / its mean HIP-event duration), and the
FP64 CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import statistics
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per site of each kernel of the step: the compulsory
# traffic of the method (read + write of populations, Q and phi) that the
# kernel is responsible for.  Values per site: populations Q read + Q
# written (Q = 19 or 15), Q-tensor 5 + 5, phi 1 + 1.
ALGO_VALUES = {
    "k_thermo": (0, 6),     # (population read+write passes, field values): reads Q, phi
    "k_collide": (1, 0),    # reads and writes the populations
    "k_order": (0, 6),      # writes Q, phi
    "k_lb_fused": (1, 6),   # populations + reads of Q, phi
    "k_step_fused": (1, 12),  # the whole step: populations, Q and phi read and written
    "k_order_fused": (0, 6),
    # the paper's predictor-corrector (per launch: its own field reads + writes;
    # X*, Y, v and mu are traffic the stage split adds)
    "k_pc_v": (0, 9),        # phi, Q -> v
    "k_pc_mu": (0, 10),      # phi, Q, v -> mu
    "k_pc_predict": (0, 16),  # Q, phi, u, mu -> X*
    "k_pc_correct": (0, 22),  # X*, u, mu, X -> Q, phi
    "k_pc_mu_z": (0, 7),       # phi, Q -> mu (v stays on chip)
    "k_pc_stage_z (predict)": (0, 16),
    "k_pc_stage_z (correct)": (0, 22),
}
PC4_M = 0.05  # mobility inside the explicit fourth-order Cahn-Hilliard stability bound
NQ = {"d3q19": 19, "d3q15": 15}
GS_BYTES = {"fp64": 8, "fp32": 4, "fp16s": 2}
FS_BYTES = {"fp64": 8, "fp32": 4, "fp16s": 4}


def kernel_source_hash() -> str:
    from paper_2011_00287_amd.build import kernel_source_hash as h
    return h()


def measured_traffic(kernel: str, workload: str, prec: str, lattice: str = "d3q19"):
    """HBM bytes per launch from the committed counter summary, if it matches the current source."""
    tag = "" if lattice == "d3q19" else f"_{lattice}"
    f = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{prec}{tag}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def step_bytes(prec: str, lattice: str = "d3q19") -> int:
    return 2 * NQ[lattice] * GS_BYTES[prec] + 12 * FS_BYTES[prec]


def time_precision(prec, p, phi, q5, steps, warmup, stream, lattice="d3q19", fd_scheme="euler2", tuning=None):
    import torch
    from paper_2011_00287_amd.sim import Sim
    if fd_scheme == "pc4":
        p = dict(p, M=PC4_M)
    sim = Sim(p, phi, q5, precision=prec, stream=stream, lattice=lattice, fd_scheme=fd_scheme, tuning=tuning)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return sim, dt


def time_adjoint(prec, p, phi, q5, steps, checkpoint, stream, recorded=True, lattice="d3q19", alternatives=True,
                 fd_scheme="euler2", tuning=None, reps=3):
    """(reverse pass incl. any segment replay) / (plain forward) over the same steps.

    Every time is the median of `reps` runs from the same initial state (a
    single run of a few tens of milliseconds varies by a few per cent).

    Modes (lean records hold Q, phi, drho, u, F per step; full-state records hold
    whole states plus u, F), as the autograd function runs them:
      checkpointed: states kept every `checkpoint` steps, each segment replayed with
                    recording steps into state buffers, then reversed;
      recorded:     the lean record of every step kept in the forward pass, no replay;
    and for comparison the other record kind in each mode (`alternatives`).
    """
    import torch
    from paper_2011_00287_amd.autograd import (backward_lean, backward_recorded, backward_segments,
                                               backward_segments_lean, backward_segments_overlapped, run_lean,
                                               run_recorded, run_segments)
    from paper_2011_00287_amd.sim import Sim
    sim = Sim(p, phi, q5, precision=prec, stream=stream, lattice=lattice, fd_scheme=fd_scheme, tuning=tuning)
    s0 = sim.get_state()
    # the loss is the displacement of the centre from its position at time 0,
    # so the reference is read from the initial state (a reference taken at
    # time T would give a zero loss and an all-zero adjoint seed)
    zc0 = float(sim.centre()[0][2])
    sim.step(3)
    sim.set_state(s0)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        sim.sync()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def plain_forward():
        sim.set_state(s0)
        return timed(lambda: sim.step(steps))[1]

    t_fwd = statistics.median(plain_forward() for _ in range(reps))
    losses = []

    def run_mode(fwd, bwd):
        t_fs, t_bs = [], []
        for _ in range(reps):
            sim.set_state(s0)
            hist, t_f = timed(fwd)
            adj = sim.adjoint_buffer()
            loss = sim.seed_centre(zc0, adj)
            if not loss > 0.0:
                raise RuntimeError(f"adjoint timing: displacement loss {loss!r} after {steps} steps; the reverse "
                                   "pass would run on a zero seed")
            _, t_b = timed(lambda: bwd(hist, adj))
            t_fs.append(t_f)
            t_bs.append(t_b)
        losses.append(loss)
        return hist, statistics.median(t_fs), statistics.median(t_bs)

    ck, t_fwd_ck, t_bwd = run_mode(lambda: run_segments(sim, steps, checkpoint),
                                   lambda h, a: backward_segments(sim, h, steps, checkpoint, a))
    del ck
    out = {"steps": steps, "checkpoint": checkpoint, "precision": prec, "lattice": lattice.upper(),
           "fd_scheme": fd_scheme,
           "forward_ms": t_fwd * 1e3, "forward_with_checkpoints_ms": t_fwd_ck * 1e3, "backward_ms": t_bwd * 1e3,
           "adjoint_over_forward": t_bwd / t_fwd, "total_over_forward": (t_fwd_ck + t_bwd) / t_fwd,
           "loss": losses[0], "reps": reps}
    if not alternatives:
        if recorded:
            recs, t_fwd_rec, t_bwd_rec = run_mode(lambda: run_lean(sim, steps),
                                                  lambda h, a: backward_lean(sim, h, a))
            del recs
            out["recorded"] = {"adjoint_over_forward": t_bwd_rec / t_fwd,
                               "total_over_forward": (t_fwd_rec + t_bwd_rec) / t_fwd}
        sim.close()
        return out
    # the same sweep with the replay of segment s-1 on a second context and stream
    # while segment s is reversed (the replay context exists before the timed region)
    replay_stream = torch.cuda.Stream()
    rep = Sim(p, phi, q5, precision=prec, stream=replay_stream, lattice=lattice, fd_scheme=fd_scheme, tuning=tuning)
    ck, _, t_bwd_ov = run_mode(lambda: run_segments(sim, steps, checkpoint),
                               lambda h, a: backward_segments_overlapped(sim, rep, h, steps, checkpoint, a,
                                                                         replay_stream))
    del ck
    rep.close()
    out["overlapped"] = {"backward_ms": t_bwd_ov * 1e3, "adjoint_over_forward": t_bwd_ov / t_fwd,
                         "total_over_forward": (t_fwd_ck + t_bwd_ov) / t_fwd}
    if recorded:
        recs, t_fwd_rec, t_bwd_rec = run_mode(lambda: run_lean(sim, steps), lambda h, a: backward_lean(sim, h, a))
        nbytes = sum(t.numel() * t.element_size() for t in recs)
        del recs
        out["recorded"] = {"forward_recording_ms": t_fwd_rec * 1e3, "backward_ms": t_bwd_rec * 1e3,
                           "adjoint_over_forward": t_bwd_rec / t_fwd,
                           "total_over_forward": (t_fwd_rec + t_bwd_rec) / t_fwd, "device_bytes": nbytes,
                           "bytes_per_site_step": nbytes / (steps * phi.size)}
        ck, _, t_bwd_lck = run_mode(lambda: run_segments(sim, steps, checkpoint),
                                    lambda h, a: backward_segments_lean(sim, h, steps, checkpoint, a))
        del ck
        hist, _, t_bwd_rfull = run_mode(lambda: run_recorded(sim, steps),
                                        lambda h, a: backward_recorded(sim, *h, a))
        nfull = sum(t.numel() * t.element_size() for t in hist[0] + hist[1])
        del hist
        out["alternatives"] = {"checkpointed_lean_replay_adjoint_over_forward": t_bwd_lck / t_fwd,
                               "recorded_full_state_adjoint_over_forward": t_bwd_rfull / t_fwd,
                               "recorded_full_state_bytes_per_site_step": nfull / (steps * phi.size)}
    sim.close()
    return out


def droplet_velocity(prec, p, phi, q5, steps, every, stream, window=1000):
    """Velocity of the droplet (circular-mean centre, unwrapped) over the last `window` steps of `steps`."""
    from paper_2011_00287_amd.sim import Sim
    from paper_2011_00287_amd.study import Track
    with Sim(p, phi, q5, precision=prec, stream=stream) as sim:
        tr = Track(phi.shape)
        for t in range(0, steps + 1, every):
            if t:
                sim.step(every)
            tr.add(t, sim)
    return [float(v) for v in tr.velocity(window)]


def _oracle_mlups(workload, nsteps, threads, lattice="d3q19", fd_scheme="euler2"):
    """MLUPS of the FP64 oracle on `threads` host threads: `nsteps` timed steps after one warm-up."""
    import torch
    from oracle import core, d3q15, pc4
    from paper_2011_00287_amd import inputs
    if fd_scheme == "pc4":
        step = pc4.step
    else:
        step = core.step if lattice == "d3q19" else d3q15.step
    p = inputs.params_for(workload, **({"M": PC4_M} if fd_scheme == "pc4" else {}))
    phi, q5 = inputs.workload_fields(workload)
    phi_t, q5_t = torch.tensor(phi), torch.tensor(q5)
    g = torch.zeros((NQ[lattice],) + phi.shape, dtype=torch.float64)
    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        g, q5_t, phi_t = step(g, q5_t, phi_t, p)  # warm-up
        t0 = time.perf_counter()
        for _ in range(nsteps):
            g, q5_t, phi_t = step(g, q5_t, phi_t, p)
        dt = time.perf_counter() - t0
    finally:
        torch.set_num_threads(prev)
    return phi.size * nsteps / dt / 1e6, dt


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(workload: str, nsteps: int = 3, lattice: str = "d3q19", fd_scheme: str = "euler2",
                 small: str = "droplet64", small_steps: int = 20):
    """The FP64 oracle on the host: the timed workload on all threads (the
    reported value), and the 64^3 droplet on all threads and on one thread."""
    import torch
    if fd_scheme == "pc4" and lattice != "d3q19":
        return None
    threads = torch.get_num_threads()
    v, dt = _oracle_mlups(workload, nsteps, threads, lattice, fd_scheme)
    out = {"value": v, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{workload} FP64 oracle ({lattice.upper()}, {fd_scheme}), {nsteps} timed steps after 1 "
                     f"warm-up from the initial droplet ({dt:.1f} s)",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if small:
        v_all, dt_all = _oracle_mlups(small, small_steps, threads, lattice, fd_scheme)
        v_one, dt_one = _oracle_mlups(small, small_steps, 1, lattice, fd_scheme)
        out[small] = {"all_threads": {"value": v_all, "threads": threads, "steps": small_steps, "seconds": dt_all},
                      "one_thread": {"value": v_one, "threads": 1, "steps": small_steps, "seconds": dt_one}}
    return out


def copy_calibration(nbytes: int, reps: int):
    """Device-to-device copies of a known size: achievable HBM bandwidth and the
    reference for scaling hardware byte counters.  Two kernels: the runtime's
    copy (copy_) and an elementwise multiply (reads n*4 bytes, writes n*4)."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for name, fn in (("copy", lambda: dst.copy_(src)), ("mul", lambda: torch.mul(src, 1.0, out=dst))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        line = {"metric": f"device {name} bandwidth", "value": 2 * n * 4 / (ms * 1e-3) / 1e9, "unit": "GB/s",
                "bytes_read_per_launch": n * 4, "bytes_written_per_launch": n * 4, "ms_per_launch": ms,
                "reps": reps, "peak": HBM_PEAK_GBS}
        print(json.dumps(line), flush=True)


# 2D active nematic (D2Q9): per-site compulsory values of each kernel
ALGO_VALUES_2D = {"k2_lb": 20,     # 9 populations read + 9 written, Q read
                  "k2_order": 4}   # Q read + written (its read of u is traffic the split adds)
STEP_VALUES_2D = 22                # populations 9 + 9, Q 2 + 2


def time_2d(workload, prec, steps, warmup):
    """(Nematic2D, seconds for `steps` steps) on the 2D workload."""
    import torch
    from paper_2011_00287_amd import inputs
    from paper_2011_00287_amd.sim2d import Nematic2D
    p = inputs.nematic2d_params(workload)
    q2 = inputs.nematic2d_workload_fields(workload)
    sim = Nematic2D(p, q2, precision=prec)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    return sim, time.perf_counter() - t0


def cpu_baseline_2d(workload: str, nsteps: int = 3):
    import torch
    from oracle import nematic2d
    from paper_2011_00287_amd import inputs
    p = inputs.nematic2d_params(workload)
    q2 = torch.tensor(inputs.nematic2d_workload_fields(workload))
    g = torch.zeros((9,) + tuple(q2.shape[1:]), dtype=torch.float64)
    g, q2 = nematic2d.step(g, q2, p)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        g, q2 = nematic2d.step(g, q2, p)
    dt = time.perf_counter() - t0
    n = q2[0].numel()
    return {"value": n * nsteps / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{workload} ({n} sites) FP64 oracle, {nsteps} timed steps after 1 warm-up"}


def bench_2d(args):
    """The 2D bulk active nematic as the timed line."""
    from paper_2011_00287_amd import inputs
    w = inputs.NEMATIC2D_WORKLOADS[args.workload]
    prec = args.precision
    if prec == "fp16s":
        raise SystemExit("the 2D model runs in fp64 or fp32")
    sim, dt = time_2d(args.workload, prec, args.steps, args.warmup)
    n = sim.n_sites
    mlups = n * args.steps / dt / 1e6
    prof = sim.profile(args.profile_steps)
    sim.close()
    dom = max(prof, key=prof.get)
    vb = GS_BYTES[prec]
    algo = ALGO_VALUES_2D[dom] * vb * n
    achieved = algo / (prof[dom] * 1e-3) / 1e9
    print(f"# {args.workload} {prec}: {mlups:.1f} MLUPS, kernels {prof}", file=sys.stderr, flush=True)
    line = {
        "metric": "2D active-nematic step MLUPS (D2Q9 + Q tensor)", "value": mlups, "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32"}[prec], "data": "synthetic",
        "config": {"workload": args.workload, "box": [w["n"], w["n"]], "zeta": w["zeta"], "precision": prec,
                   "lattice": "D2Q9"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom, "kernel_ms": prof[dom],
                     "algorithmic_bytes_per_launch": algo},
        "step_roofline": {"bytes_per_site": STEP_VALUES_2D * vb,
                          "frac": mlups * 1e6 * STEP_VALUES_2D * vb / (HBM_PEAK_GBS * 1e9)},
        "kernel_ms": prof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_2d(args.workload)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="droplet128")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16s"])
    ap.add_argument("--lattice", default="d3q19", choices=["d3q19", "d3q15"],
                    help="d3q19: stress as a body force; d3q15: the paper's scheme")
    ap.add_argument("--fd-scheme", default="euler2", choices=["euler2", "pc4"],
                    help="euler2: explicit Euler, 2nd-order stencils; pc4: the paper's predictor-corrector, "
                         f"upwind, 4th-order stencils (M = {PC4_M})")
    ap.add_argument("--path", default="default", choices=["default", "one", "two"],
                    help="launch path of the timed step: the two-launch split (default) or one kernel per step")
    ap.add_argument("--lb-tile", type=int, default=0, help="stress + collision kernel tile (lb_tuning.lb_tile)")
    ap.add_argument("--tz-lb", type=int, default=0, help="stress + collision slab depth (lb_tuning.tz_lb)")
    ap.add_argument("--step-tile", type=int, default=0, help="one-launch kernel tile (lb_tuning.step_tile)")
    ap.add_argument("--tz-step", type=int, default=0, help="one-launch slab depth (lb_tuning.tz_step)")
    ap.add_argument("--adj-tile", type=int, default=0, help="stress + gather adjoint tile (lb_tuning.adj_tile)")
    ap.add_argument("--adj-order-tile", type=int, default=0, help="order adjoint tile (lb_tuning.adj_order_tile)")
    ap.add_argument("--tz-adj", type=int, default=0, help="stress + gather adjoint slab depth (lb_tuning.tz_adj)")
    ap.add_argument("--tz-adj-order", type=int, default=0, help="order adjoint slab depth (lb_tuning.tz_adj_order)")
    ap.add_argument("--tz-pc-adj", type=int, default=0, help="pc4 reverse product slab depth (lb_tuning.tz_pc_adj)")
    ap.add_argument("--pc-adj", type=int, default=0, help="pc4 reverse kernels (lb_tuning.pc_adj: 1 = site-parallel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the FP64 / FP16S side timings")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=50, help="0 = skip the adjoint timing")
    ap.add_argument("--adjoint-checkpoint", type=int, default=10)
    ap.add_argument("--no-adjoint-recorded", action="store_true",
                    help="skip the reverse pass over a fully recorded forward pass")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only time a device copy of this many MiB and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step runs the whole box on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2011_00287_amd import inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration << 20, max(1, args.steps))
        return
    if args.workload in inputs.NEMATIC2D_WORKLOADS:
        bench_2d(args)
        return
    stream = torch.cuda.current_stream()
    w = inputs.WORKLOADS[args.workload]
    p = inputs.params_for(args.workload)
    phi, q5 = inputs.workload_fields(args.workload)
    n = phi.size
    print(f"# workload {args.workload} {phi.shape} {args.precision} {args.lattice} {args.fd_scheme}: "
          f"warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)

    tuning = {"path": args.path, "step_tile": args.step_tile, "tz_step": args.tz_step, "lb_tile": args.lb_tile,
              "tz_lb": args.tz_lb}
    sim, dt = time_precision(args.precision, p, phi, q5, args.steps, args.warmup, stream, args.lattice,
                             args.fd_scheme, tuning)
    mlups = n * args.steps / dt / 1e6
    print(f"# {args.precision}: {mlups:.1f} MLUPS ({dt / args.steps * 1e3:.4f} ms/step)", file=sys.stderr, flush=True)

    prof = sim.profile(args.profile_steps)
    dom = max(prof, key=prof.get)
    gv, fv = ALGO_VALUES.get(dom, ALGO_VALUES.get(dom.split(" ")[0]))
    algo_bytes = (gv * 2 * NQ[args.lattice] * GS_BYTES[args.precision] + fv * FS_BYTES[args.precision]) * n
    achieved = algo_bytes / (prof[dom] * 1e-3) / 1e9
    totals = sim.totals()
    sim.close()
    print(f"# kernels (ms/launch): {prof}", file=sys.stderr, flush=True)

    side = {}
    if not args.no_side:
        cases = [(prec, "d3q19", "euler2") for prec in ("fp64", "fp16s")] + \
                [(prec, "d3q15", "euler2") for prec in ("fp32", "fp64", "fp16s")] + [("fp32", "d3q19", "pc4")]
        for prec, lat, fd in cases:
            if (prec, lat, fd) == (args.precision, args.lattice, args.fd_scheme):
                continue
            key = prec if lat == "d3q19" else f"{lat}_{prec}"
            if fd != "euler2":
                key = f"{fd}_{key}"
            ns = max(20, args.steps // (4 if prec == "fp64" else 1))
            s2, dt2 = time_precision(prec, p, phi, q5, ns, 5, stream, lat, fd)
            s2.close()
            side[key] = {"mlups": n * ns / dt2 / 1e6, "ms_per_step": dt2 / ns * 1e3,
                         "step_hbm_frac": n * ns / dt2 * step_bytes(prec, lat) / (HBM_PEAK_GBS * 1e9)}
            print(f"# {key}: {side[key]['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
        if args.adjoint_steps > 0 and args.lattice == "d3q19" and args.fd_scheme == "euler2":
            # the adjoint of the paper's own LB scheme, checkpointed and recorded modes
            a15 = time_adjoint("fp32", p, phi, q5, args.adjoint_steps, args.adjoint_checkpoint, stream,
                               lattice="d3q15", alternatives=False)
            side["d3q15_fp32_adjoint"] = {"adjoint_over_forward": a15["adjoint_over_forward"],
                                          "recorded_adjoint_over_forward": a15["recorded"]["adjoint_over_forward"],
                                          "checkpoint": args.adjoint_checkpoint, "steps": args.adjoint_steps}
            print(f"# d3q15_fp32 adjoint/forward: {a15['adjoint_over_forward']:.2f} (checkpoint "
                  f"{args.adjoint_checkpoint}), {a15['recorded']['adjoint_over_forward']:.2f} (every step recorded)",
                  file=sys.stderr, flush=True)
            # the adjoint of the paper's FD integrator (pc4, its mobility)
            apc = time_adjoint("fp32", dict(p, M=PC4_M), phi, q5, args.adjoint_steps, args.adjoint_checkpoint,
                               stream, alternatives=False, fd_scheme="pc4")
            side["pc4_fp32_adjoint"] = {"adjoint_over_forward": apc["adjoint_over_forward"],
                                        "recorded_adjoint_over_forward": apc["recorded"]["adjoint_over_forward"],
                                        "checkpoint": args.adjoint_checkpoint, "steps": args.adjoint_steps}
            print(f"# pc4_fp32 adjoint/forward: {apc['adjoint_over_forward']:.2f} (checkpoint "
                  f"{args.adjoint_checkpoint}), {apc['recorded']['adjoint_over_forward']:.2f} (every step recorded)",
                  file=sys.stderr, flush=True)
        s2, dt2 = time_2d("nematic512", "fp32", 2000, 50)  # the 2D workload of Fig. 3 (512^2)
        n2d = s2.n_sites
        s2.close()
        side["nematic512_fp32"] = {"mlups": n2d * 2000 / dt2 / 1e6, "ms_per_step": dt2 / 2000 * 1e3,
                                   "step_hbm_frac": n2d * 2000 / dt2 * STEP_VALUES_2D * 4 / (HBM_PEAK_GBS * 1e9)}
        print(f"# nematic512_fp32: {side['nematic512_fp32']['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
        if (args.workload == "droplet128" and args.precision == "fp32" and args.lattice == "d3q19"
                and args.fd_scheme == "euler2"):
            # the accuracy the speed of each precision buys: droplet velocity over the last
            # 1000 of 5000 steps, against FP64, with each precision's step time beside it
            steps_v = inputs.WORKLOADS["droplet128"]["steps"]
            vel = {prec: droplet_velocity(prec, p, phi, q5, steps_v, 100, stream) for prec in ("fp64", "fp32", "fp16s")}
            ms = {"fp64": side["fp64"]["ms_per_step"], "fp16s": side["fp16s"]["ms_per_step"],
                  "fp32": dt / args.steps * 1e3}
            v64 = vel["fp64"][2]
            side["droplet_velocity"] = {
                "steps": steps_v, "window": 1000, "velocity_z": {k: v[2] for k, v in vel.items()},
                "rel_diff_vs_fp64": {k: abs(v[2] - v64) / abs(v64) for k, v in vel.items() if k != "fp64"},
                "ms_per_step": ms}
            print(f"# droplet velocity (z, last 1000 of {steps_v} steps): "
                  + ", ".join(f"{k} {v[2]:.4e}" for k, v in vel.items()), file=sys.stderr, flush=True)
        if args.workload != "droplet256":
            # the large box: 256^3 forward rate and the 50-step adjoint with checkpoint 10
            w5 = inputs.WORKLOADS["droplet256"]
            p5 = inputs.params_for("droplet256")
            phi5, q55 = inputs.workload_fields("droplet256")
            n5 = phi5.size
            ns = max(50, args.steps)
            s5, dt5 = time_precision("fp32", p5, phi5, q55, ns, 5, stream)
            s5.close()
            side["droplet256_fp32"] = {"mlups": n5 * ns / dt5 / 1e6, "ms_per_step": dt5 / ns * 1e3, "steps": ns,
                                       "step_hbm_frac": n5 * ns / dt5 * step_bytes("fp32") / (HBM_PEAK_GBS * 1e9)}
            print(f"# droplet256_fp32: {side['droplet256_fp32']['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
            if args.adjoint_steps > 0:
                a5 = time_adjoint("fp32", p5, phi5, q55, w5["adjoint_steps"], w5["checkpoint"], stream,
                                  recorded=False, alternatives=False,
                                  tuning={"adj_tile": args.adj_tile, "adj_order_tile": args.adj_order_tile})
                side["droplet256_fp32_adjoint"] = {k: a5[k] for k in ("adjoint_over_forward", "total_over_forward",
                                                                      "forward_ms", "backward_ms", "checkpoint",
                                                                      "steps", "loss", "reps")}
                print(f"# droplet256_fp32 adjoint/forward: {a5['adjoint_over_forward']:.2f} (checkpoint "
                      f"{w5['checkpoint']}, {w5['adjoint_steps']} steps)", file=sys.stderr, flush=True)
            del phi5, q55

    adjoint = None
    if args.adjoint_steps > 0:
        pa = dict(p, M=PC4_M) if args.fd_scheme == "pc4" else p
        adjoint = time_adjoint(args.precision, pa, phi, q5, args.adjoint_steps, args.adjoint_checkpoint, stream,
                               recorded=not args.no_adjoint_recorded, lattice=args.lattice, fd_scheme=args.fd_scheme,
                               tuning=dict(tuning, adj_tile=args.adj_tile, adj_order_tile=args.adj_order_tile,
                                           tz_adj=args.tz_adj, tz_adj_order=args.tz_adj_order,
                                           tz_pc_adj=args.tz_pc_adj, pc_adj=args.pc_adj))
        print(f"# adjoint/forward: {adjoint['adjoint_over_forward']:.2f} (checkpoint {args.adjoint_checkpoint}; "
              f"{adjoint['overlapped']['adjoint_over_forward']:.2f} with the replay overlapped)"
              + (f", {adjoint['recorded']['adjoint_over_forward']:.2f} (every step recorded, "
                 f"{adjoint['recorded']['bytes_per_site_step']:.0f} B/site/step); lean replay "
                 f"{adjoint['alternatives']['checkpointed_lean_replay_adjoint_over_forward']:.2f}, full-state "
                 f"records {adjoint['alternatives']['recorded_full_state_adjoint_over_forward']:.2f}"
                 if "recorded" in adjoint else ""), file=sys.stderr, flush=True)

    line = {
        "metric": "coupled-step MLUPS at 128^3 FP32 vs FP64, % HBM peak; adjoint/forward time",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16s": "f16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "box": list(phi.shape[::-1]), "droplet_radius": w["R"],
                   "q0": w["q0"], "zeta": w["zeta"], "precision": args.precision,
                   "lattice": args.lattice.upper(), "fd_scheme": args.fd_scheme,
                   **({"M": PC4_M} if args.fd_scheme == "pc4" else {})},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, args.workload, args.precision, args.lattice), "kernel": dom,
                     "kernel_ms": prof[dom], "algorithmic_bytes_per_launch": algo_bytes},
        "step_roofline": {"bytes_per_site": step_bytes(args.precision, args.lattice),
                          "frac": mlups * 1e6 * step_bytes(args.precision, args.lattice) / (HBM_PEAK_GBS * 1e9)},
        "kernel_ms": prof,
        "kernel_source_hash": kernel_source_hash(),
        "side": side,
        "adjoint": adjoint,
        "totals_after_run": {k: totals[k] for k in ("mass", "phi_total", "free_energy")},
    }
    if not args.no_cpu_baseline:
        print("# timing the FP64 CPU oracle on a bounded sample ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, lattice=args.lattice, fd_scheme=args.fd_scheme)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python
"""Benchmark of the hybrid symplectic step on one MI355X.

Default workload: the embryo disk (10 embryos of 0.1-1 Earth masses plus 100,000
massless planetesimals in a gas disk, seed 0), stepped with the full hybrid step
(kick + drag + jump + Kepler drift + encounter flagging + Bulirsch-Stoer).  Prints
one JSON line.  `value` is changeover-weighted kick interactions per second over
whole steps (I = n_big * (n - 1) per step, ordered pairs, n = non-star bodies).

Extra objects:
  roofline      -- the dominant kernel group of the step against its bound.  With
                   n_big <= 64 every step but the last of a call is one joint launch
                   (the encounter integrator of the step beside the closing of that
                   step and the opening of the next), which is then the dominant
                   group; otherwise groups are ranked with HIP events around each
                   group.  The dominant group is timed over the K timed steps with
                   HIP events bound to its kernels' own start and end in every 8th
                   step (eager launches; --event-stride); its HBM traffic and
                   counter-based FP64 rate (counter_fp64) come from the committed
                   counter summaries while the kernel sources are unchanged
  step_kernel   -- the launch that closes one step and opens the next without the
                   integrator (n_big <= 64; the batched ensemble's launch), timed over
                   further steps, against HBM, with its counter FP64 rate
  kick_fp64     -- the force kernel of the fully self-gravitating 4,004-body case
                   (16.0 M interactions per kick) against FP64 peak, by the 20-flop
                   model and by counters
  batch         -- 256 independent embryo disks of uneven size stepped together
                   (autotuned launch shape; eager and graph launches), against the
                   sum of the same systems stepped one at a time
  adjoint       -- 1,000 differentiable steps of a 20,000-body embryo disk (checkpoints
                   every 50 steps) and the reverse pass, against plain steps
  cpu_baseline  -- the CPU oracle built for the host, serial and OpenMP over target
                   bodies on all usable cores (bitwise equal), on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12        # MI355X FP64 vector, FLOP/s (FMA = 2)
PEAK_HBM = 8.0e12          # bytes/s
FLOP_PER_INTERACTION = 20  # conventional pairwise-force count
COPY_BYTES = 256 << 20     # calibration copy: bytes read (and bytes written)
# algorithmic HBM bytes per body of the kick+drag+jump+drift kernel:
# read x,u,a (72) + r_p,rho_p (16, massless only); write x0,u0,x,u (96)
BYTES_KJD_SMALL = 184
BYTES_KJD_BIG = 168
# the joined closing/opening launch: read x, u, r_p, rho_p (64), write x, u (48)
BYTES_JOINED_SMALL = 112


def interactions_per_step(nb: int, n: int) -> int:
    return nb * (n - 1) if nb > 0 else 0


def workload(name: str, seed: int = 0):
    from synth import ic
    if name == "embryo_disk":
        return ic.embryo_disk(seed=seed)
    if name == "two_giants":
        return ic.two_giants(seed=seed)
    if name == "self_gravitating":
        return ic.self_gravitating(seed=seed)
    raise SystemExit(f"unknown workload {name}")


def roofline_for(name: str, avg_s: float, w, n_pairs_avg: float, bs_flop_per_launch: float = 0.0):
    nb, ns = w.params["n_big"], w.params["n_small"]
    n = nb + ns
    if name == "force_kick":
        flops = FLOP_PER_INTERACTION * interactions_per_step(nb, n)
        a = flops / avg_s
        return {"kernel": name, "bound": "alu", "achieved": a / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": a / PEAK_FP64, "traffic": None,
                "model": f"{FLOP_PER_INTERACTION} FP64 flop per ordered interaction"}
    if name == "kick_jump_drift":
        b = BYTES_KJD_SMALL * ns + BYTES_KJD_BIG * nb
        a = b / avg_s
        return {"kernel": name, "bound": "hbm", "achieved": a / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": a / PEAK_HBM, "traffic": None,
                "model": f"{BYTES_KJD_SMALL} B per massless body, {BYTES_KJD_BIG} B per massive body"}
    if name == "flag":
        b = 96 * n + 128 * nb
        a = b / avg_s
        return {"kernel": name, "bound": "hbm", "achieved": a / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": a / PEAK_HBM, "traffic": None,
                "model": "96 B per body (x0,u0,x1,u1) + 128 B per massive source record"}
    if name == "step_joint":
        b = BYTES_JOINED_SMALL * ns + BYTES_KJD_BIG * nb
        a = b / avg_s
        return {"kernel": name, "bound": "hbm", "achieved": a / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": a / PEAK_HBM, "traffic": None,
                "model": f"{BYTES_JOINED_SMALL} B per massless body (x, u, r_p, rho_p read; "
                         f"x, u written), {BYTES_KJD_BIG} B per massive body; the encounter "
                         "integrator in the same launch adds no HBM traffic of note",
                "bs_model_flop_per_launch": bs_flop_per_launch}
    if name == "bs":
        # model FP64 operations counted by the library while the kernel ran
        a = bs_flop_per_launch / avg_s
        return {"kernel": name, "bound": "alu", "achieved": a / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": a / PEAK_FP64, "traffic": None,
                "model": "per force evaluation 24 FP64 ops per member + 25 per flagged pair, "
                         "3 per extrapolation-table entry (FMA = 2), summed over the steps taken"}
    # planner and the small kernels: HBM bytes of the pair list they sort and rewrite
    b = 8 * 3 * max(n_pairs_avg, 1.0)
    a = b / avg_s
    return {"kernel": name, "bound": "hbm", "achieved": a / 1e9, "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": a / PEAK_HBM, "traffic": None,
            "model": "24 B per flagged pair (list read, sorted list and plan written)"}


def recorded(summary: str):
    """Fields ("- key: value" lines) of the committed rocprofv3 summary
    profiles/<summary>.md, or None when there is none or the kernel sources it
    names changed since it was taken (their SHA-256 is recorded with it)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{summary}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            rec[k.strip()] = v.strip().strip("`")
    try:
        h = hashlib.sha256()
        for f in rec["source"].split(","):
            h.update(open(os.path.join(ROOT, f.strip()), "rb").read())
        if h.hexdigest()[:16] != rec["source_sha256_16"]:
            return None
    except (KeyError, OSError):
        return None
    rec["path"] = os.path.relpath(path, ROOT)
    return rec


def recorded_sum(rec, prefix: str, kernels):
    """Sum of rec[prefix.kernel] over kernels (None if any is missing)."""
    if rec is None:
        return None
    try:
        return sum(float(rec[f"{prefix}.{k}"]) for k in kernels)
    except (KeyError, ValueError):
        return None


# kernels of each timed group, per workload shape (n_big <= 64: fused small-B path);
# where a group runs different kernels in different systems, the alternatives are
# listed and the first one the summary holds is used
GROUP_KERNELS = {
    ("bs", True): ["k_bs"], ("bs", False): ["k_bs"],
    ("kick_jump_drift", True): ["k_step_a"], ("kick_jump_drift", False): ["k_kick_jump_drift"],
    ("force_kick", True): ["k_step_b"], ("force_kick", False): ["k_force_sym", "k_force_finish_sym"],
    ("step_joined", True): ["k_step_ba"], ("step_joint", True): ["k_step_joint"],
    ("flag", False): [["k_chunk_bounds", "k_flag_cull"], ["k_flag"]],
    ("jump_pack", False): ["k_jump_pack"], ("growth", False): ["k_growth"],
}


def group_sum(rec, prefix: str, group_kernels):
    """recorded_sum over a group's kernels (the first alternative the summary holds)."""
    if not group_kernels:
        return None, None
    alts = group_kernels if isinstance(group_kernels[0], list) else [group_kernels]
    for ks in alts:
        v = recorded_sum(rec, prefix, ks)
        if v is not None:
            return v, ks
    return None, None


def counter_rate(w, group: str, avg_s: float):
    """Counter-based FP64 rate of a kernel group from the committed counter summary:
    (ADD + MUL + TRANS + 2 FMA)_F64 instructions per launch times the active lanes per
    VALU instruction, over the measured average launch."""
    small = w.params["n_big"] <= 64
    rec = recorded(f"fp64_{w.name}")
    ops, ks = group_sum(rec, "fp64_ops_per_launch", GROUP_KERNELS.get((group, small)))
    if ops is None or avg_s <= 0:
        return None
    a = ops / avg_s
    return {"kernels": ks, "fp64_ops_per_launch": ops, "achieved": a / 1e12,
            "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": a / PEAK_FP64,
            "lanes": rec.get("lanes"), "source": rec["path"]}


def recorded_traffic(w, group: str):
    """HBM bytes per launch of a kernel group (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled
    by a plain copy of known size) from the committed summary, or None."""
    small = w.params["n_big"] <= 64
    rec = recorded(f"traffic_{w.name}")
    b, _ = group_sum(rec, "bytes_per_launch", GROUP_KERNELS.get((group, small)))
    return None if b is None else (b, rec["path"])


def host_cpu():
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(w, target_s: float):
    """The CPU oracle built for this host (gcc -O3 -march=native, no FMA contraction),
    serial and with OpenMP over target bodies, on a bounded sample: the serial build
    runs consecutive steps from the initial state for about half of target_s, the
    OpenMP build then runs the same number of steps, and both states must agree bit
    for bit."""
    import tempfile
    import numpy as np
    import oracle
    model, ncpu, usable = host_cpu()
    n = w.params["n_big"] + w.params["n_small"]
    I = interactions_per_step(w.params["n_big"], n)
    with tempfile.TemporaryDirectory() as d:
        lib_s = oracle.load(oracle.build_variant(os.path.join(d, "or_serial.so"), openmp=False))
        lib_p = oracle.load(oracle.build_variant(os.path.join(d, "or_omp.so"), openmp=True))
        o = oracle.OracleSystem(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, w.growth,
                                library=lib_s)
        t0 = time.perf_counter()
        steps = 0
        while True:
            o.step(1)
            steps += 1
            if time.perf_counter() - t0 >= 0.5 * target_s:
                break
        T_s = time.perf_counter() - t0
        xs, us = o.get_dh()
        o.close()
        q = oracle.OracleSystem(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, w.growth,
                                library=lib_p)
        threads = lib_p.or_threads()
        t1 = time.perf_counter()
        q.step(steps)
        T_p = time.perf_counter() - t1
        xp, up = q.get_dh()
        q.close()
        identical = bool(np.array_equal(xs, xp) and np.array_equal(us, up))
    return {"value": I * steps / T_p, "unit": "interactions/s", "cores": threads,
            "kind": "oracle", "steps_per_s": steps / T_p,
            "serial": {"value": I * steps / T_s, "steps_per_s": steps / T_s, "cores": 1},
            "openmp_equals_serial_bitwise": identical,
            "host": {"cpu_model": model, "nproc": ncpu, "usable_cpus": usable,
                     "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")},
            "build": "gcc " + " ".join(oracle.CFLAGS_FAST) + " (+ -fopenmp for the parallel leg)",
            "sample": f"{steps} consecutive hybrid steps of the same workload from its initial "
                      f"state: serial {T_s:.1f} s, OpenMP over target bodies on {threads} threads "
                      f"{T_p:.1f} s"}


def kick_fp64(args):
    """Force kernel of the fully self-gravitating 4,004-body case (no extra state change:
    profiled steps of its own system)."""
    import paper_2601_16791_amd as mx
    w = workload("self_gravitating", args.seed)
    s = mx.System.from_workload(w)
    s.step(3)
    s.sync()
    reps = args.kick_reps
    t0 = time.perf_counter()
    s.step(reps)
    s.sync()
    T = time.perf_counter() - t0
    per_step_ms, n_launch = s.step_timed(reps, "force_kick")
    avg = sum(per_step_ms) / max(n_launch, 1) / 1e3
    nb, n = w.params["n_big"], w.params["n_big"] + w.params["n_small"]
    I = interactions_per_step(nb, n)
    a = FLOP_PER_INTERACTION * I / avg
    s.close()
    tr = recorded_traffic(w, "force_kick")
    return {"workload": "self_gravitating", "n_big": nb, "interactions_per_kick": I,
            "counter_fp64": counter_rate(w, "force_kick", avg),
            "traffic": tr[0] if tr else None, "traffic_source": tr[1] if tr else None,
            "kernels": "k_force_sym + k_force_finish_sym (start of the first to end of the "
                       "second): massive pairs once each by tiles, Newton's third law",
            "avg_kick_us": avg * 1e6, "launches": n_launch, "achieved": a / 1e12,
            "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": a / PEAK_FP64,
            "interactions_per_s": I / avg, "steps_per_s": reps / T,
            "model": f"{FLOP_PER_INTERACTION} FP64 flop per ordered interaction"}


def batch_leg(args):
    """256 independent embryo disks of uneven size stepped together, against the
    same systems stepped one at a time (each batch member alone)."""
    import paper_2601_16791_amd as mx
    from synth import ic
    ws = ic.batch(seed=args.seed, n_sys=args.batch_systems)
    I = sum(interactions_per_step(w.params["n_big"], w.n) for w in ws)
    bodies = sum(w.n for w in ws)
    b = mx.Batch.from_workloads(ws)
    del ws
    # the encounters of the first steps from the initial state are not yet those of
    # the run: the autotuner runs after 200 steps
    b.step(200)
    b.sync()
    taken, cfg, best_ms = b.autotune(steps_per_candidate=10)
    b.step(args.warmup)
    b.sync()
    t0 = time.perf_counter()
    b.step(args.batch_steps)
    b.sync()
    T = time.perf_counter() - t0
    b.set_launch_mode("graph", steps_per_graph=args.graph_steps)
    b.step(args.graph_steps)  # capture
    b.sync()
    t1 = time.perf_counter()
    b.step(args.batch_steps)
    b.sync()
    T_graph = time.perf_counter() - t1
    # every member alone (its own single-system launches), a few steps each
    single_s = 0.0
    for k in range(b.n_sys):
        v = b.system(k)
        v.step(2)
        v.sync()
        t2 = time.perf_counter()
        v.step(args.single_steps)
        v.sync()
        single_s += (time.perf_counter() - t2) / args.single_steps
    b.close()
    return {"workload": f"{args.batch_systems} embryo disks, 2-8 embryos and 1e3-5e4 massless "
                        "bodies each (log-uniform), gas drag",
            "systems": args.batch_systems, "bodies": bodies, "interactions_per_step": I,
            "config_autotuned": {"bodies_per_tile": cfg[0], "tiles_per_block": cfg[1],
                                 "bs_blocks_per_system": cfg[2]},
            "autotune_steps": taken, "steps": args.batch_steps,
            "steps_per_s": args.batch_steps / T, "interactions_per_s": I * args.batch_steps / T,
            "steps_per_s_graph": args.batch_steps / T_graph,
            "graph_steps_per_launch": args.graph_steps,
            "single_system_sum_ms_per_step": 1e3 * single_s,
            "speedup_vs_single_systems": single_s / (T / args.batch_steps)}


def adjoint_leg(args):
    """Differentiable run of the 20,000-body embryo disk: forward with checkpoints,
    loss = mean + variance of the final massless eccentricities, reverse pass,
    against the plain single-system steps of the same system."""
    import torch
    import paper_2601_16791_amd as mx
    from synth import ic
    w = ic.adjoint_shape(seed=args.seed)
    nb = w.params["n_big"]
    steps, every = args.adjoint_steps, 50
    spec = dict(params=w.params, x=w.x, v=w.v, r_p=w.r_p, rho_p=w.rho_p, n_steps=steps,
                checkpoint_every=every, m_big=w.m_big)
    dev = "cuda"

    def run(spec_run):
        m = torch.tensor(w.m_big, dtype=torch.float64, device=dev, requires_grad=True)
        xb = torch.tensor(w.x[:, :nb], dtype=torch.float64, device=dev, requires_grad=True)
        vb = torch.tensor(w.v[:, :nb], dtype=torch.float64, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xf, vf = mx.hybrid_run(m, xb, vb, spec_run)
        torch.cuda.synchronize()
        T_f = time.perf_counter() - t0
        h = torch.linalg.cross(xf.T, vf.T)
        r = torch.linalg.norm(xf, dim=0)
        e = torch.linalg.norm(torch.linalg.cross(vf.T, h) / w.params["G"] - (xf / r).T,
                              dim=1)[nb:]
        loss = e.mean() + e.var(unbiased=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        return T_f, time.perf_counter() - t1, loss, m, xb, vb

    run(dict(spec, n_steps=2, checkpoint_every=1))  # loads the torch kernels of the loss
    T_fwd, T_bwd, loss, m, xb, vb = run(spec)
    s = mx.System.from_workload(w)
    s.step(5)
    s.sync()
    t2 = time.perf_counter()
    s.step(steps)
    s.sync()
    T_plain = time.perf_counter() - t2
    s.close()
    return {"workload": f"embryo disk, {nb} embryos + {w.params['n_small']} massless bodies, gas "
                        "drag; loss = mean + variance of final massless eccentricity",
            "steps": steps, "checkpoint_every": every, "forward_s": T_fwd, "backward_s": T_bwd,
            "backward_over_forward": T_bwd / T_fwd, "plain_steps_s": T_plain,
            "backward_steps_per_s": steps / T_bwd,
            "loss": loss.item(), "grad_norm_mass": float(m.grad.norm()),
            "grad_norm_x": float(xb.grad.norm()), "grad_norm_v": float(vb.grad.norm())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="embryo_disk")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--kick-reps", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kick", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=1000)
    ap.add_argument("--batch-systems", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--graph-steps", type=int, default=10)
    ap.add_argument("--single-steps", type=int, default=20)
    ap.add_argument("--event-stride", type=int, default=8,
                    help="HIP events around the dominant kernel group in every k-th timed "
                         "step (an event between two launches delays the second)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-launched pass after the timed region (counter runs: "
                         "the profiler serialises every replayed kernel)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device-to-device once (reference reading for "
                         "HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library integrates its systems on a single device", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_16791_amd as mx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = workload(args.workload, args.seed)
    nb, ns = w.params["n_big"], w.params["n_small"]
    n = nb + ns
    I = interactions_per_step(nb, n)
    s = mx.System.from_workload(w)
    print(f"[bench] {w.name}: n_big={nb} n_small={ns} warmup={args.warmup}", file=sys.stderr, flush=True)
    s.step(args.warmup)
    # per-group time of synchronised steps (HIP events around each group; includes
    # the launch after each synchronisation), reported as context
    prof = s.step_profiled(args.profile_steps)
    avg = {k: v / args.profile_steps / 1e3 for k, v in prof.items()}  # seconds per step
    # the dominant group: the most kernel time per step, from events bound to the
    # group's own kernels in unsynchronised steps (the synchronised figures above
    # add a launch latency to every group and can reorder close groups)
    per_step = {}
    for g in (k for k, v in avg.items() if v > 0):
        ms, _ = s.step_timed(args.profile_steps, g, args.event_stride)
        n_timed = (args.profile_steps - 1) // args.event_stride + 1
        per_step[g] = sum(ms) / n_timed
    dominant = max(per_step, key=per_step.get)
    # the joint launch, where mx_step uses it: one per step but the last of a call
    ms, nl = s.step_timed(args.profile_steps, "step_joint", args.event_stride)
    if nl > 0:
        per_step["step_joint"] = sum(ms) / nl
        dominant = "step_joint"
    # also creates the timing events outside the timed region
    s.step_timed(args.steps, dominant, args.event_stride)
    s.sync()
    torch.cuda.synchronize()
    # timed region: K steps, eager launches (the default launch mode), with HIP events
    # bound to the dominant group's kernels' own start and end in every
    # event-stride-th step
    f0, p0 = s.counters()
    t0 = time.perf_counter()
    per_step_ms, n_launch = s.step_timed(args.steps, dominant, args.event_stride)
    s.sync()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    f1, p1 = s.counters()
    print(f"[bench] timed {args.steps} steps in {T:.3f} s", file=sys.stderr, flush=True)
    pairs_last = len(s.encounters())
    pairs_avg = (p1 - p0) / args.steps
    dom_avg_s = sum(per_step_ms) / max(n_launch, 1) / 1e3
    # the integrator's model flops are counted over every timed step; it runs once
    # per step, so per launch they are divided by the steps, not by the event-timed
    # launches
    roof = roofline_for(dominant, dom_avg_s, w, pairs_avg, (f1 - f0) / args.steps)
    roof["avg_launch_us"] = dom_avg_s * 1e6
    roof["launches"] = n_launch
    roof["event_stride"] = args.event_stride
    roof["traffic_unit"] = "bytes per launch"
    roof["traffic_source"] = None
    tr = recorded_traffic(w, dominant)
    if tr is not None:
        roof["traffic"], roof["traffic_source"] = tr
    roof["counter_fp64"] = counter_rate(w, dominant, dom_avg_s)
    # the launch that closes one step and opens the next (fused small-B path),
    # timed over further steps of the same run (outside the timed region)
    step_kernel = None
    if nb <= 64:
        ms, nl = s.step_timed(args.profile_steps, "step_joined", args.event_stride)
        if nl > 0:
            sk_s = sum(ms) / nl / 1e3
            b = BYTES_JOINED_SMALL * ns + BYTES_KJD_BIG * nb
            step_kernel = {"kernel": "k_step_ba", "avg_launch_us": sk_s * 1e6, "launches": nl,
                           "bound": "hbm", "achieved": b / sk_s / 1e9, "peak": PEAK_HBM / 1e9,
                           "unit": "GB/s", "frac": b / sk_s / PEAK_HBM,
                           "model": f"{BYTES_JOINED_SMALL} B per massless body (x, u, r_p, "
                                    "rho_p read; x, u written)",
                           "traffic": None, "traffic_source": None,
                           "counter_fp64": counter_rate(w, "step_joined", sk_s)}
            tr = recorded_traffic(w, "step_joined")
            if tr is not None:
                step_kernel["traffic"], step_kernel["traffic_source"] = tr
    # the same number of steps launched as one captured HIP graph per step (context)
    T_graph = None
    if not args.no_graph:
        s.set_launch_mode("graph")
        s.step(1)
        s.sync()
        t1 = time.perf_counter()
        s.step(args.steps)
        s.sync()
        T_graph = time.perf_counter() - t1
    E, L = s.energy()
    s.close()
    out = {
        "metric": "FP64 body-body interactions/sec in kick + full steps/sec; % FP64 VALU peak",
        "value": I * args.steps / T,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_big": nb, "n_small": ns, "seed": args.seed,
                   "dt_days": w.params["dt"], "gas": bool(w.params["gas_on"]),
                   "interactions_per_step": I},
        "steps_per_s": args.steps / T,
        "kernel_us_per_step_events": {k: v * 1e6 for k, v in avg.items()},
        "kernel_us_per_step_bound_events": {k: v * 1e3 for k, v in per_step.items()},
        "steps_per_s_graph_launch": args.steps / T_graph if T_graph else None,
        "encounter_pairs_last_step": pairs_last,
        "encounter_pairs_per_step": pairs_avg,
        "roofline": roof,
        "step_kernel": step_kernel,
    }
    if not args.no_kick:
        out["kick_fp64"] = kick_fp64(args)
    if not args.no_batch:
        out["batch"] = batch_leg(args)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Throughput of the batched AS-ICP solve on one MI355X.

One step = one whole solve of the paper-scale workload: set-up (A0), 100
iterations of Algorithm 1 for 3 preshapes x 256 particles against an
8192-point object, the final evaluation and the selection.  Inputs are
resident in HBM before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-iters/s & grasps/s at matched final cost: plain vs learned-seeded"
PEAK_FP32_MFMA = 157.3e12  # MI355X dense fp32 matrix peak, FLOP/s
FLOP_PER_PAIR = 6          # 3 multiply-adds of |r|^2 - 2 r.s per (query, object point) pair
# HBM bytes per launch of the forward-NN kernel on the paper-scale workload,
# per launch choice ("xcd_map,fine,query_blocks,chunk_points"), from two
# rocprofv3 --pmc passes: 2.000 x FETCH_SIZE + 1.000 x WRITE_SIZE (KiB per
# dispatch, factors from a 256 MiB device copy), averaged over the launches
# of one solve (profiles/nn_forward_counters_paper_scale.md).  Reported only
# while the kernel's sources, and the set-up that orders the clouds it scans,
# hash to the ones measured.
NN_TRAFFIC = {"sha256": "0a0548a0dc72bfc90842dabee7640f97c5f0b56d05b07d5559b810969edbb0c4",
              "bytes": {"0,1,4,64": 6201220, "0,1,4,128": 6209432, "1,1,4,64": 6275172, "1,1,4,128": 6280330}}
NN_SOURCES = ("k_nn_forward.hip", "nn_core.h", "asicp_internal.h", "k_setup.hip")


def nn_traffic(workload, launch, brute):
    import hashlib
    h = hashlib.sha256()
    for f in NN_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_08346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != NN_TRAFFIC["sha256"] or workload != "paper" or brute:
        return None
    key = f"{launch['xcd_map']},{launch['fine']},{launch.get('query_blocks', 4)},{launch.get('chunk_points', 128)}"
    return NN_TRAFFIC["bytes"].get(key)


def cpu_baseline(pb, st, seconds=10.0):
    """The FP64 oracle, untuned, on a bounded sample of the same workload:
    whole iterations of every particle (evaluation + Stein update) from the
    initial poses, as many as start within `seconds`."""
    import numpy as np
    import oracle
    o = oracle.Oracle(pb, st)
    th = pb.theta0.astype(np.float64)
    t0 = time.perf_counter()
    pc = cv = None
    iters = 0
    while iters < st.k_max and (iters == 0 or time.perf_counter() - t0 < seconds):
        r = o.step(iters, th, pc, cv)
        th, pc, cv = r["theta"], r["prev_cost"], r["converged"]
        iters += 1
    dt = time.perf_counter() - t0
    out = {"value": pb.k_tot * iters / dt, "unit": "particle-iters/s", "cores": oracle.threads(),
           "kind": "oracle",
           "sample": f"{iters} iteration(s) of all {pb.k_tot} particles of the same workload "
                     f"(FP64, {dt:.1f} s)"}
    # one core: one iteration of the first (object, preshape) group, the same
    # per-particle work (an iteration couples only the particles of a group)
    from paper_2412_08346_amd import synth
    sub = synth.Problem(R=pb.R, r_off=pb.r_off[:2], C=pb.C, c_off=pb.c_off[:2],
                        S=pb.S[pb.s_off[0]:pb.s_off[1]], s_off=np.array([0, pb.s_off[1] - pb.s_off[0]], np.int32),
                        grids=pb.grids[:1], theta0=np.ascontiguousarray(pb.theta0[:, :pb.K]), K=pb.K)
    n_threads = oracle.threads()
    oracle.set_threads(1)
    try:
        o1 = oracle.Oracle(sub, st)
        t0 = time.perf_counter()
        o1.step(0, sub.theta0.astype(np.float64))
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(n_threads)
    out["one_core"] = {"value": sub.k_tot / dt1, "unit": "particle-iters/s", "cores": 1,
                       "sample": f"1 iteration of the {sub.k_tot} particles of one (object, preshape) group "
                                 f"(FP64, {dt1:.1f} s)"}
    return out


def nn_roofline(ms, n, pairs):
    """Achieved FLOP/s of the forward-NN launches from their HIP-event time
    and the distances they evaluated."""
    avg = ms / max(n, 1) / 1e3
    per = pairs / max(n, 1)
    ach = FLOP_PER_PAIR * per / avg if avg > 0 else 0.0
    return {"achieved": ach / 1e12, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_MFMA,
            "avg_launch_ms": avg * 1e3, "launches": n, "pairs_per_launch": per}


def batched_leg(A, synth, log, solves=2):
    """The batched workload (64 objects of 2k-32k points x 3 preshapes x 128
    particles, 100 iterations): one launch per kernel for all objects, launch
    choice by the library's tuner, `solves` timed whole solves."""
    import numpy as np
    import torch
    pb, st = synth.workload_batched()
    s = A.Solver(pb, st, timing=True)
    launch, ms_choice = s.autotune(reps=2)
    s.reset()
    s.solve()
    s.result(per_particle=False)
    log(f"batched: workload ready (Ktot={pb.k_tot}), launch {launch}")
    walls = []
    before = s.kernel_time()  # the records accumulate over the context's solves
    for _ in range(solves):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    nn = [a - b for a, b in zip(s.kernel_time(), before)]
    res = s.result(per_particle=False)
    s.close()
    # the same solve as one captured HIP graph (asicp_replay), timed by wall
    # clock over whole replays (no per-kernel events inside a graph)
    g = A.Solver(pb, st)
    g.set_launch(**launch)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay()
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    g.result(per_particle=False)
    g.close()
    wall = float(np.median(walls))
    out = {"workload": "64 objects (superquadrics and unions of 1-3 boxes, 2k-32k points, log-uniform) x 3 "
                       "box-gripper preshapes x 4096 contact points x 128 Fibonacci particles, 100 iterations, "
                       "one launch per kernel for all objects",
           "replay_ms_per_solve": 1e3 * wall_graph,
           "particle_iters_per_s": pb.k_tot * st.k_max / wall, "grasps_per_s": pb.n_obj / wall,
           "ms_per_solve": 1e3 * wall, "solves": solves, "launch": launch,
           "collision_free_objects": int(res["best_free"].sum()),
           "nn_roofline": nn_roofline(*nn)}
    return out


def small_replay_leg(A, synth, log, replays=50):
    """The small workload (1 object of 1024 points, 1 preshape of 512 contact
    points, 32 particles, 30 iterations) as one captured HIP graph per solve
    (asicp_replay), against the same solve enqueued kernel by kernel (on a
    context of its own)."""
    import torch
    pb, st = synth.workload_small()
    # enqueued solves on a context of their own
    e = A.Solver(pb, st)
    e.solve()
    e.result(per_particle=False)
    walls = []
    for _ in range(5):
        e.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.solve()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    e.close()
    wall_e = sorted(walls)[len(walls) // 2]
    s = A.Solver(pb, st)
    s.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        s.replay()
    torch.cuda.synchronize()
    wall_g = (time.perf_counter() - t0) / replays
    res = s.result(per_particle=False)
    s.close()
    log(f"small: replay {1e3 * wall_g:.3f} ms, enqueued {1e3 * wall_e:.3f} ms per solve")
    return {"workload": "1 ellipsoid of 1024 points, 1 preshape x 512 contact points, 64^3 SDF, 32 Fibonacci "
                        "particles, 30 iterations",
            "replay_ms_per_solve": 1e3 * wall_g, "enqueued_ms_per_solve": 1e3 * wall_e,
            "particle_iters_per_s": pb.k_tot * st.k_max / wall_g, "grasps_per_s": 1.0 / wall_g,
            "replays": replays, "collision_free": int(res["best_free"][0])}


def full_scan_leg(A, pb, st, log, iters=4):
    """The forward NN without pruning (every object point compared with every
    contact point) on the paper-scale workload: the launch choice of the
    library's tuner, `iters` iterations from the initial poses, HIP events
    around every launch."""
    s = A.Solver(pb, st, timing=True, prune=False)
    launch, _ = s.autotune(reps=2)  # query blocks per wave and XCD placement
    s.step(1)
    s.result(per_particle=False)
    before = s.kernel_time()  # the warm-up launch is not counted
    s.reset()
    s.step(iters)
    s.result(per_particle=False)
    ms, n, pr = [a - b for a, b in zip(s.kernel_time(), before)]
    s.close()
    r = nn_roofline(ms, n, pr)
    log(f"full scan: {r['avg_launch_ms']:.3f} ms per launch, frac {r['frac']:.3f}")
    return {"kernel": "k_nn_forward_full", "bound": "mfma", **r, "flop_per_pair": FLOP_PER_PAIR,
            "launch": {"xcd_map": launch["xcd_map"], "query_blocks": launch["query_blocks"]}}


def learned_leg(log, n_train, steps):
    """Plain against learned-seeded AS-ICP at matched final cost, with the
    network trained inside this run on grasps the solver finds."""
    from paper_2412_08346_amd import proposal
    t0 = time.perf_counter()
    r = proposal.run_learned(n_train=n_train, steps=steps, log=log)
    p, l, f = r["plain"], r["learned"], r["fibonacci_same_budget"]
    pi_p = p["particles_per_preshape"] * p["iterations"]
    pi_l = l["particles_per_preshape"] * l["iterations"]
    return {"workload": f"{r['objects']} held-out random objects (superquadrics and box unions, 2k-16k points), 3 "
                        "box-gripper preshapes x 4096 contact points",
            "plain_grasps_per_s": p["grasps_per_s"], "learned_grasps_per_s": l["grasps_per_s"],
            "grasp_rate_ratio": l["grasps_per_s"] / p["grasps_per_s"],
            "particle_iters_per_grasp_ratio": pi_p / pi_l,
            "median_cost_ratio": l["median_cost_ratio"], "matched_fraction": l["matched_fraction"],
            "no_network_same_budget": {"median_cost_ratio": f["median_cost_ratio"],
                                       "matched_fraction": f["matched_fraction"]},
            "train_objects": r["train_objects"], "train_steps": r["train_steps"],
            "leg_s": time.perf_counter() - t0, "detail": r}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--k-max", type=int, default=100)
    ap.add_argument("--workload", choices=("paper", "batched"), default="paper")
    ap.add_argument("--brute", action="store_true",
                    help="forward NN visits every object chunk (no exact pruning)")
    ap.add_argument("--learned", action="store_true",
                    help="plain against learned-seeded AS-ICP at matched final cost: trains the "
                         "proposal network on grasps the solver finds (a few minutes) and prints one "
                         "JSON line of the comparison instead of the throughput line")
    ap.add_argument("--launch", default=None, metavar="MAP,FINE[,QB,CP]",
                    help="use this launch choice (XCD placement 0/1, per-query chunk test 0/1, query "
                         "blocks per wave 1/2/4, points per chunk 64/128) instead of tuning")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch choices instead of timing them first")
    ap.add_argument("--legs", default="batched,small,full,learned",
                    help="extra legs of the default line (comma-separated: batched, small, full, learned; "
                         "'none' for the paper-scale line alone)")
    ap.add_argument("--learned-train", type=int, default=768, help="training objects of the learned leg")
    ap.add_argument("--learned-steps", type=int, default=3000, help="Adam steps of the learned leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (3 times): the reference "
                         "kernel that scales rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (objects and groups are "
              "independent and would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2412_08346_amd as A
    from paper_2412_08346_amd import synth

    torch.cuda.set_device(0)
    if args.learned:
        from paper_2412_08346_amd import proposal
        r = proposal.run_learned(log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
        line = {"metric": METRIC, "value": r["learned"]["grasps_per_s"], "unit": "grasps/s (learned-seeded)",
                "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
                "data": "synthetic", "config": {"workload": "64 held-out random objects (superquadrics and "
                "box unions, 2k-16k points), 3 box-gripper preshapes x 4096 contact points; plain 256 Fibonacci "
                "particles x 100 annealed Stein iterations per preshape vs 32 learned seeds x 50 SGD-ICP "
                "iterations"}, **r}
        print(json.dumps(line), flush=True)
        return
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: 3 x {args.calibrate_copy} MiB", file=sys.stderr, flush=True)
        del src, dst
    if args.workload == "batched":
        pb, st = synth.workload_batched(k_max=args.k_max)
        desc = ("batched plain AS-ICP: 64 objects (superquadrics and unions of 1-3 boxes, 2k-32k "
                "points, log-uniform), 3 box-gripper preshapes x 4096 contact points, 128^3 SDF, 128 "
                f"Fibonacci particles per (object, preshape), {st.k_max} iterations, one launch per "
                "kernel for all objects")
    else:
        pb, st = synth.workload_paper_scale(k_max=args.k_max)
        desc = ("paper-scale plain AS-ICP: 1 superquadric object of 8192 points, 3 box-gripper "
                "preshapes x 4096 contact points, 128^3 SDF, 256 Fibonacci particles per preshape, "
                f"{st.k_max} iterations")
    solver = A.Solver(pb, st, timing=True, prune=not args.brute)
    print(f"[bench] workload ready: Ktot={pb.k_tot} objects={pb.n_obj} points={pb.R.shape[0]} "
          f"k_max={st.k_max}", file=sys.stderr, flush=True)
    # one step = one whole solve on the resident inputs and workspace: the
    # set-up, the iterations, the final evaluation and the selection, all
    # enqueued on one stream
    sp = torch.cuda.current_stream().cuda_stream
    for w in range(args.warmup):
        solver.reset()
        solver.solve()
        solver.result(per_particle=False)
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    # launch choices (XCD placement, per-query chunk test) change no result.
    # The library's tuner (asicp_autotune) times one evaluation per choice;
    # a step here is a whole solve, whose speed also depends on how the side
    # stream's kernels and the short per-iteration kernels fall around the
    # forward NN, so each choice is timed on whole solves (the best of two,
    # outside the timed region) and the fastest is used for every timed solve
    solver.reset()
    if args.launch:
        vals = [int(v) for v in args.launch.split(",")]
        launch = dict(zip(("xcd_map", "fine", "query_blocks", "chunk_points"), vals))
        launch_ms = None
    elif args.no_autotune:
        launch, launch_ms = solver.launch(), None
    else:
        launch_ms = []
        for v in range(A.ASICP_LAUNCH_CHOICES):
            best = float("inf")
            for _ in range(2):
                ctx = A.asicp_create(solver.problem, solver.config, solver._ws_ptr, solver.ws_bytes, sp)
                A.asicp_set_launch(ctx, **A.launch_choice(v))
                torch.cuda.synchronize()
                a = time.perf_counter()
                A.asicp_solve(ctx, sp)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - a)
                A.asicp_destroy(ctx)
            launch_ms.append(1e3 * best)
        v = int(np.argmin(launch_ms))
        launch = A.launch_choice(v)
        print(f"[bench] launch choice: {launch}; ms per solve by launch index: "
              f"{[round(x, 2) for x in launch_ms]}", file=sys.stderr, flush=True)
    # one context for the timed solves: each step re-runs the set-up from the
    # resident inputs (asicp_reset) and the whole solve; one context keeps one
    # side stream (contexts created per step spread their side streams over
    # the hardware queues, and those sharing the main stream's queue lose the
    # overlap)
    solver.close()
    ctx = A.asicp_create(solver.problem, solver.config, solver._ws_ptr, solver.ws_bytes, sp)
    A.asicp_set_launch(ctx, **launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        A.asicp_reset(ctx, sp)
        A.asicp_solve(ctx, sp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nn_ms, nn_n, nn_pairs = A.asicp_kernel_time(ctx)
    solver.ctx = ctx
    res = solver.result(per_particle=False)
    solver.close()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    p_iters = pb.k_tot * st.k_max * args.steps
    all_pairs = sum(pb.K * int(np.diff(pb.s_off)[p]) * int(np.diff(pb.r_off)[o])
                    for o in range(pb.n_obj) for p in range(pb.n_pre))
    pairs = nn_pairs / max(nn_n, 1)  # distances actually evaluated per launch
    avg_nn = nn_ms / max(nn_n, 1) / 1e3
    achieved = FLOP_PER_PAIR * pairs / avg_nn
    line = {
        "metric": METRIC,
        "value": p_iters / wall,
        "unit": "particle-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "grasps_per_s": pb.n_obj * args.steps / wall,
        "config": {"workload": desc, "objects": pb.n_obj,
                   "particles": pb.k_tot, "iterations": st.k_max, "object_points": int(pb.R.shape[0]),
                   "contact_points_per_preshape": int(np.diff(pb.s_off)[0]), "preshapes": pb.n_pre},
        "roofline": {"bound": "mfma", "kernel": "k_nn_forward", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": nn_traffic(args.workload, launch, args.brute),
                     "traffic_unit": "bytes per launch", "avg_launch_ms": avg_nn * 1e3, "launches": nn_n,
                     "pairs_per_launch": pairs, "brute_force_pairs_per_launch": all_pairs,
                     "pruned": not args.brute, "flop_per_pair": FLOP_PER_PAIR,
                     "launch": launch, "launch_choice_ms_per_solve": launch_ms},
        "best_cost_median": float(np.median(res["best_cost"])), "collision_free_objects": int(res["best_free"].sum()),
    }
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    legs = [] if args.legs == "none" else args.legs.split(",")
    if args.workload == "paper":
        if "full" in legs:
            line["full_scan"] = full_scan_leg(A, pb, st, log)
        if "small" in legs:
            line["small_replay"] = small_replay_leg(A, synth, log)
        if "batched" in legs:
            line["batched"] = batched_leg(A, synth, log)
            log(f"batched: {line['batched']['particle_iters_per_s']:.3g} particle-iters/s")
        if "learned" in legs:
            line["learned_vs_plain"] = learned_leg(log, args.learned_train, args.learned_steps)
    if not args.no_cpu_baseline and args.workload == "paper":
        log("timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(pb, st)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

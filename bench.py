"""Benchmark: tetrahedra per second of the exact Delaunay tetrahedralization on one MI355X.

A step is one pass of the whole path over one batch: clear the context, insert the n points
(validation, Moore keys, radix sort, duplicates, initial tetrahedron, anchors and every
insertion round) and export the tetrahedra with their neighbours into device buffers.  The
points are resident in HBM before the timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Sources of the dominant kernel; the measured HBM traffic in PMC_SUMMARY is used only while
# their hash matches the one recorded there.
KERNEL_SOURCES = ["paper_1805_08831_amd/csrc/dt_insert.hip", "paper_1805_08831_amd/csrc/dt_internal.h",
                  "paper_1805_08831_amd/csrc/dt_predicates.h"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_cavity_g_uniform_1e7_pmc.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the cavity kernel from the committed counter summary, or
    None when the summary is missing or the kernel sources changed since it was taken."""
    try:
        kv = {}
        with open(PMC_SUMMARY) as fh:
            for line in fh:
                if line.startswith("- ") and " = " in line:
                    k, v = line[2:].split(" = ", 1)
                    kv[k.strip()] = v.strip().strip("`")
        if kv.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration():
    """Plain device-to-device copy of 256 MiB, three times: the reference for the units of
    the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 * 1024 * 1024
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n} bytes three times", flush=True)

def gather_calibration():
    """A random gather of 4 Mi 64-byte records out of a 4 GiB array (index_select with a
    shuffled index), three times: the reference for the counters on random 64-byte reads that
    miss the caches, the access pattern of the tetrahedron pool.  Each dispatch reads 256 MiB
    of records and 32 MiB of indices and writes 256 MiB."""
    import torch
    rows = 64 * 1024 * 1024  # 4 GiB of 64-byte rows
    src = torch.empty((rows, 16), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    idx = torch.randint(0, rows, (4 * 1024 * 1024,), device="cuda", generator=gen)
    torch.cuda.synchronize()
    for _ in range(3):
        out = src.index_select(0, idx)
    torch.cuda.synchronize()
    print(f"gathered {out.shape[0]} rows of 64 bytes three times", flush=True)


# Algorithmic bytes per insertion, the hot-path scope table's model of an HBM-bound insertion
# (u32 layout): the point record and its key/index (32 + 12 B), W walk steps of one
# tetrahedron row (ids 16 B + neighbour codes 16 B) and ~32 B of vertex data each, the C
# cavity tetrahedra (32 B each), the F outer tetrahedra's vertex ids (16 B each) and ~30
# vertex records (32 B each) belong to the walk + cavity kernel; the F new tetrahedra (32 B)
# and their back-pointers (4 B) to the ball kernel.  W = 4 and 30 vertex records are the
# model's own figures; C and F are measured per insertion.
MODEL_WALK_STEPS = 4
MODEL_VERTEX_RECORDS = 30


def cavity_bytes_per_insertion(C, F, W=MODEL_WALK_STEPS, V=MODEL_VERTEX_RECORDS):
    return 44 + 64 * W + 32 * C + 16 * F + 32 * V


def ball_bytes_per_insertion(F):
    return 32 * F + 4 * F


# A finer model of what one attempt of the cavity kernel moves (reported beside the table's
# model, not as the roofline): candidate/hint/point (48 B), per walk step one tetrahedron row
# (vertices 16 B + neighbours 16 B) and one new vertex record (32 B), per cavity tetrahedron
# its two rows (32 B) and per outer tetrahedron its vertex row (16 B), an 8-byte owner word
# read and written per touched tetrahedron (16 B), the boundary's vertex records (F/2 + 2
# records of 32 B) and the per-insertion buffers written (4 B per cavity tetrahedron, 8 B per
# facet).  Counts every attempt, losers included.
def cavity_bytes_per_attempt(walk, C, F):
    return 48 + 64 * walk + 32 * C + 16 * F + 16 * (C + F) + 32 * (F / 2 + 2) + 4 * C + 8 * F


# The paper's CPU figures for uniform points (other hardware: context, not a target):
# 3e9 tetrahedra in 53 s on two 32-core AMD EPYC 7551 (abstract, Sec. 3.7), and its figure of
# rates against n for the same machine.
PAPER_RATE_BY_N = {10_000_000: 31.32e6, 100_000_000: 64.40e6}


def paper_context(n):
    ctx = {"headline": "3e9 tetrahedra in 53 s (56.6 M tets/s), 2x AMD EPYC 7551, 64 cores",
           "unit": "tetrahedra/s", "note": "the paper's CPU; other hardware, context only"}
    if n in PAPER_RATE_BY_N:
        ctx["value_at_this_n"] = PAPER_RATE_BY_N[n]
    return ctx


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline_points(sample, what):
    """The serial oracle (one thread) on one point set: tetrahedra per second."""
    import oracle
    t0 = time.perf_counter()
    rc, tets, _, _ = oracle.delaunay(sample)
    dt = time.perf_counter() - t0
    if rc != 0:
        raise RuntimeError(f"oracle failed on the CPU sample (code {rc})")
    return {"value": round(len(tets) / dt, 1), "unit": "tetrahedra/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}, full serial triangulation in {dt:.2f} s, {len(tets)} tetrahedra",
            "cpu": host_cpu_model(), "host_threads": os.cpu_count()}


def cpu_baseline(n, seed):
    """The serial oracle on n uniform points (seed)."""
    from synth import uniform_points
    return cpu_baseline_points(uniform_points(n, seed), f"{n} uniform points (seed {seed})")


def cpu_baseline_clouds(xyz, off, clouds, budget_s=15.0):
    """The serial oracle (one thread) on the given clouds in turn, each triangulated alone,
    until about budget_s seconds of work: tetrahedra per second over the clouds done."""
    import oracle
    t_all, tets, pts, done = 0.0, 0, 0, 0
    for c in clouds:
        p = xyz[int(off[c]):int(off[c + 1])]
        t0 = time.perf_counter()
        rc, t, _, _ = oracle.delaunay(p)
        t_all += time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError(f"oracle failed on cloud {c} (code {rc})")
        tets += len(t)
        pts += len(p)
        done += 1
        if t_all >= budget_s:
            break
    return {"value": round(tets / t_all, 1), "unit": "tetrahedra/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the clouds ({pts} points, {tets} tetrahedra), each triangulated alone, "
                      f"serially in {t_all:.2f} s",
            "cpu": host_cpu_model(), "host_threads": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--seed", type=int, default=1007)
    ap.add_argument("--cpu-sample", type=int, default=2_500_000,
                    help="uniform: the oracle's CPU sample, the first points of the timed input (about 10 s "
                         "on one core)")
    ap.add_argument("--walk-cap", type=int, default=0,
                    help="walk steps after which a regular round's attempt resumes next round (0: automatic, -1: none)")
    ap.add_argument("--subdet-cache", action="store_true",
                    help="cache four sub-determinants per tetrahedron (the paper's Sec. 2.4 optimization)")
    ap.add_argument("--adaptive-curve", action="store_true",
                    help="Moore curve on the deepest grid the key holds (adaptive order for non-uniform inputs)")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="after the timed steps, one instrumented step: per-attempt clocks of the cavity kernel")
    ap.add_argument("--no-export", action="store_true",
                    help="uniform: a step ends with the tetrahedron count (for pools too large to hold the "
                         "output beside them, 5e8 points)")
    ap.add_argument("--u8-steps", type=int, default=2,
                    help="uniform: timed steps at 1e8 points (seed 1008) for the line's u8 object; 0: skip")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--round-fraction", type=float, default=0.0)
    ap.add_argument("--round-size", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per insertion in every round (4, 8, 16, 32, 64; 0: automatic)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick lanes per insertion, round fraction and cavity cap on a 2e6-point sample first")
    ap.add_argument("--workload", choices=["uniform", "batch", "mix", "refine"], default="uniform")
    ap.add_argument("--no-learned", action="store_true", help="uniform: skip the learned-scheduler comparison")
    ap.add_argument("--no-graph-compare", action="store_true",
                    help="uniform: skip the comparison of graph-launched rounds with separate launches")
    ap.add_argument("--train-seeds", type=str, default="9001,9002", help="seeds of the plain runs logged for training")
    ap.add_argument("--train-samples", type=int, default=4_000_000, help="samples drawn from the logs")
    ap.add_argument("--train-n", type=int, default=0, help="uniform: points per training run (0: min(n, 1e7))")
    ap.add_argument("--mix-scale", type=float, default=1.0, help="mix: fraction of the 1e7 points")
    ap.add_argument("--cpu-mix-scale", type=float, default=0.05,
                    help="mix: size of the oracle's CPU sample as a fraction of the timed input")
    ap.add_argument("--clouds", type=int, default=4096, help="batch: number of clouds")
    ap.add_argument("--chunk", type=int, default=4096,
                    help="batch: clouds per dt_insert_batch call (default: all in one call, the pool then "
                         "takes 64-bit adjacency codes)")
    ap.add_argument("--loop-sample", type=int, default=64, help="batch: clouds timed one call each")
    ap.add_argument("--refine-n", type=int, default=250_000, help="refine: uniform input points (seed 4007)")
    ap.add_argument("--refine-h", type=float, default=0.0064,
                    help="refine: target size h (circumcentres of tetrahedra with r > 1.4 h, none closer "
                         "than 0.7 h)")
    ap.add_argument("--cpu-refine-points", type=int, default=30_000,
                    help="refine: input points of the oracle's CPU sample (a corner cube of the input)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device copy (counter calibration) and exit")
    ap.add_argument("--gather-calibration", action="store_true",
                    help="only run a random 64-byte gather from a 4 GiB array (counter calibration) and exit")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration()
        return
    if args.gather_calibration:
        gather_calibration()
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library triangulates on one device and has no "
              "multi-GPU path; run it without --gpus or with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "mix":
        run_mix(args)
        return
    if args.workload == "refine":
        run_refine(args)
        return

    import torch

    from synth import uniform_points

    t_bench = time.perf_counter()

    def progress(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_bench:.1f} s)", file=sys.stderr, flush=True)

    xyz = uniform_points(args.n, args.seed)
    main_run = run_uniform(args, xyz, args.n, args.seed, args.steps, args.warmup, progress)
    T = main_run["tetrahedra"]
    golden = golden_hash(args.n, args.seed)
    oracle_match = None
    if golden is not None:
        oracle_match = main_run["hash"] == golden
        progress(f"whole output against the stored oracle hash: {'equal' if oracle_match else 'DIFFERENT'}")

    clocks = None
    if args.phase_clocks:
        clocks = phase_clocks(main_run["d_xyz"], args.lanes, progress)

    model = training = None
    learned = None
    if not args.no_learned:
        # the learned scheduler on the same input, trained on plain runs of other seeds
        tn = args.train_n or min(args.n, 10_000_000)
        seeds = [int(x) for x in args.train_seeds.split(",") if x]
        model, training = train_scheduler(lambda s: uniform_points(tn, s), seeds, args.train_samples, progress)
        learned = compare_schedulers(main_run["d_xyz"], model, args.steps, args.warmup, progress,
                                     reference=main_run["canon"], export=not args.no_export)
        learned["training"] = dict(training, points_per_run=tn)
    graph = None
    if not args.no_graph_compare:
        graph = compare_graph_rounds(main_run["d_xyz"], args.steps, args.warmup, progress,
                                     reference=main_run["canon"])
        progress(f"graph rounds: {graph}")
    main_run["canon"] = None
    del main_run["d_xyz"]
    torch.cuda.empty_cache()

    u8 = None
    if args.u8_steps > 0 and args.n != 100_000_000:
        # the metric's second size: 1e8 uniform points (seed 1008), timed the same way
        xyz8 = uniform_points(100_000_000, 1008)
        r8 = run_uniform(args, xyz8, 100_000_000, 1008, args.u8_steps, 1, progress)
        del xyz8
        u8 = {k: r8[k] for k in ("value", "ms_per_step", "tetrahedra", "roofline", "detail")}
        u8["workload"] = "1e8 i.i.d. uniform fp64 points in [0,1)^3, seed 1008"
        u8["steps"] = args.u8_steps
        u8["paper_context"] = paper_context(100_000_000)
        if model is not None:
            u8["learned"] = compare_schedulers(r8["d_xyz"], model, args.u8_steps, 1, progress,
                                               reference=r8["canon"])
        r8["canon"] = None
        del r8["d_xyz"]
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        # a bounded sample of the timed input: its first cpu_sample points
        k = min(args.cpu_sample, args.n)
        cpu = cpu_baseline_points(xyz[:k], f"the first {k} points of the timed input ({args.n} uniform points, "
                                           f"seed {args.seed})")

    line = {
        "metric": "tetrahedra/sec (exact 3D Delaunay, uniform points)",
        "value": main_run["value"],
        "unit": "tetrahedra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.n} i.i.d. uniform fp64 points in [0,1)^3, seed {args.seed}",
                   "points": args.n, "tetrahedra": T, "scheduler": "plain",
                   "launch": main_run["tuned"] if main_run["tuned"] else "defaults",
                   "subdet_cache": bool(args.subdet_cache), "adaptive_curve": bool(args.adaptive_curve)},
        "roofline": main_run["roofline"],
        "cpu_baseline": cpu,
        "paper_context": paper_context(args.n),
        "oracle_hash_match": oracle_match,
        "learned": learned,
        "graph_rounds": graph,
        "u8": u8,
        "detail": main_run["detail"],
    }
    if clocks is not None:
        line["phase_clocks"] = clocks
    print(json.dumps(line), flush=True)


def reference_output(d_xyz):
    """One untimed plain triangulation of d_xyz, exported: its canonical form on the device and
    the SHA-256 of that."""
    import torch

    from paper_1805_08831_amd import Triangulation, dt_get_tets
    with Triangulation(device=0, stream=torch.cuda.current_stream().cuda_stream) as tri:
        tri.insert(d_xyz)
        T = dt_get_tets(tri.ctx)
        out = torch.empty((T, 4), dtype=torch.int32, device="cuda")
        dt_get_tets(tri.ctx, out, None, T)
    canon = canonical_device(out)
    return canon, sha256_of(canon)


def golden_hash(n, seed, kind="uniform"):
    """SHA-256 of the oracle's canonical output for this input, when stored."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize_golden.txt")
    try:
        for line in open(path):
            if line.startswith("#") or not line.strip():
                continue
            kv = dict(x.split("=", 1) for x in line.split()[1:])
            if kv.get("kind") == kind and int(kv["n"]) == n and int(kv["seed"]) == seed:
                return kv["sha256"]
    except (OSError, KeyError, ValueError):
        return None
    return None


def canonical_device(t):
    """Canonical form of a (T, 4) int32 device tensor: each row's indices sorted, rows in
    lexicographic order (stable sorts on the device)."""
    import torch
    q = torch.sort(t.long(), dim=1).values
    hi = (q[:, 0] << 32) | q[:, 1]
    lo = (q[:, 2] << 32) | q[:, 3]
    o1 = torch.sort(lo, stable=True).indices
    o2 = torch.sort(hi[o1], stable=True).indices
    return q[o1[o2]].to(torch.int32)


def sha256_of(canon):
    import hashlib
    return hashlib.sha256(canon.cpu().numpy().astype("<u4").tobytes()).hexdigest()


def run_uniform(args, xyz, n, seed, steps, warmup, progress):
    """`steps` timed steps on the uniform input xyz; the roofline of the walk + cavity
    kernel; the canonical output (device) and its hash."""
    import torch

    from paper_1805_08831_amd import Triangulation, dt_get_tets
    from synth import uniform_points

    d_xyz = torch.from_numpy(xyz).cuda()
    stream = torch.cuda.current_stream()
    # events around the cavity kernel only in the timed steps (timing 2); the ball kernel is
    # timed in one more step afterwards
    launch_opts = dict(round_fraction=args.round_fraction, round_size=args.round_size,
                       lanes_per_insert=args.lanes, subdet_cache=args.subdet_cache,
                       adaptive_curve=args.adaptive_curve,
                       walk_cap=0xFFFFFFFF if args.walk_cap < 0 else args.walk_cap)
    tri = Triangulation(device=0, stream=stream.cuda_stream, timing=2,
                        round_fraction=args.round_fraction, round_size=args.round_size,
                        lanes_per_insert=args.lanes, subdet_cache=args.subdet_cache,
                        adaptive_curve=args.adaptive_curve,
                        walk_cap=0xFFFFFFFF if args.walk_cap < 0 else args.walk_cap)
    tuned = None
    if args.autotune:
        # tuned at the timed size, on another seed (the choice is kept for that size class)
        tuned = tri.autotune(torch.from_numpy(uniform_points(n, seed + 2)).cuda())
        progress(f"autotuned at {n} points: {tuned}")

    # output buffers sized once (outside the timed region) from a first run; without export
    # (pools too large to hold the output beside them) a step ends with the count
    tri.insert(d_xyz)
    T0 = dt_get_tets(tri.ctx)
    export = not args.no_export
    out_t = torch.empty((T0 + 1024, 4), dtype=torch.int32, device="cuda") if export else None
    out_n = torch.empty((T0 + 1024, 4), dtype=torch.int64, device="cuda") if export else None

    def full_step():
        tri.clear()
        tri.insert(d_xyz)
        if not export:
            return dt_get_tets(tri.ctx)
        return dt_get_tets(tri.ctx, out_t, out_n, T0 + 1024)

    for _ in range(warmup):
        full_step()
    torch.cuda.synchronize()
    tri.clear()
    times = []
    T = 0
    agg = dict(attempts=0, walk=0, cav=0, bnd=0, won=0, ms_cav=0.0, ms_ball=0.0, launches=0, rounds=0,
               orient=0, orient_exact=0, insphere=0, insphere_exact=0, perturbed=0, conflicts=0, walk_caps=0,
               timed_ins=0, timed_att=0,
               ms_sort=0.0, ms_insert=0.0, ball_launches=0)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        T = full_step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        s = tri.stats()
        agg["attempts"] += s["attempts"]
        agg["walk"] += s["walk_steps"]
        agg["cav"] += s["cavity_tets"]
        agg["bnd"] += s["boundary_facets"]
        agg["won"] += s["inserted"]
        agg["ms_cav"] += s["ms_cavity_kernel"]
        agg["ms_ball"] += s["ms_ball_kernel"]
        agg["launches"] += s["cavity_launches"]
        agg["rounds"] += s["rounds"]
        agg["conflicts"] += s["conflicts"]
        agg["walk_caps"] += s["walk_caps"]
        agg["timed_ins"] += s["timed_insertions"]
        agg["timed_att"] += s["timed_attempts"]
        agg["ms_sort"] += s["ms_sort"]
        agg["ball_launches"] += s["ball_launches"]
        agg["ms_insert"] += s["ms_insert"]
        for k in ("orient", "orient_exact", "insphere", "insphere_exact", "perturbed"):
            agg[k] += s[k + ("_calls" if k in ("orient", "insphere") else "")]
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ms_per_step = 1000.0 * total / steps
    value = T / (ms_per_step / 1000.0)
    progress(f"{n} points: {T} tetrahedra, {ms_per_step:.1f} ms per step")
    canon = canonical_device(out_t[:T]) if export else None
    digest = sha256_of(canon) if export else None
    st_last = tri.stats()
    if tuned:
        # the same steps with the default launch configuration, for comparison
        tri.autotune_reset()
        full_step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            full_step()
        torch.cuda.synchronize()
        tuned = dict(tuned, defaults_ms_per_step=round(1000.0 * (time.perf_counter() - t1) / steps, 3),
                     tuned_ms_per_step=round(ms_per_step, 3))
        progress(f"defaults: {tuned['defaults_ms_per_step']} ms per step")
    tri.close()
    # one untimed step with events around both kernels: the ball kernel's time
    if tuned:
        launch_opts.update(lanes_per_insert=tuned["lanes_per_insert"], round_fraction=tuned["round_fraction"],
                           cavity_cap=tuned["cavity_cap"], large_lanes=tuned["large_lanes"])
    with Triangulation(device=0, stream=stream.cuda_stream, timing=1, **launch_opts) as tb:
        tb.insert(d_xyz)
        torch.cuda.synchronize()
        sb = tb.stats()
    agg["ms_ball"] = sb["ms_ball_kernel"] * steps
    agg["ball_launches"] = sb["ball_launches"] * steps
    del out_n

    # roofline of the dominant kernel (walk + cavity + claim), HBM-bound, with the table's
    # algorithmic bytes per insertion times the insertions per launch
    att = max(agg["attempts"], 1)
    won = max(agg["won"], 1)
    walk = agg["walk"] / att
    C = agg["cav"] / won
    F = agg["bnd"] / won
    launches = max(agg["launches"], 1)
    avg_launch_ms = agg["ms_cav"] / launches
    per_ins = cavity_bytes_per_insertion(C, F)
    # the timed launches are those of the rounds of at least 32768 candidates (timing 2)
    ins_per_launch = agg["timed_ins"] / launches
    achieved = per_ins * ins_per_launch / (avg_launch_ms / 1000.0) / 1e9 if avg_launch_ms > 0 else 0.0
    peak = 8000.0
    lanes = (tuned or {}).get("lanes_per_insert") if tuned else args.lanes
    b_att = cavity_bytes_per_attempt(walk, C, F)
    att_achieved = b_att * agg["timed_att"] / launches / (avg_launch_ms / 1000.0) / 1e9 if avg_launch_ms > 0 else 0.0
    default_launch = (not lanes and not args.round_fraction and not args.round_size and n == 10_000_000
                      and seed == 1007 and not args.subdet_cache and not args.adaptive_curve and not args.walk_cap)
    kname = (f"k_cavity_g filter pass (and exact pass once launched), {lanes} lanes, rounds of 32768 candidates or more" if lanes else
             "k_cavity_g filter pass (and exact pass once launched), 16 lanes, rounds of 32768 candidates or more")
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2), "peak": peak,
                "unit": "GB/s", "frac": round(achieved / peak, 5),
                # measured HBM bytes per launch (counter summary), only for the launch it was taken on
                "traffic": measured_traffic() if default_launch else None,
                "bytes_per_insertion": round(per_ins, 1), "insertions_per_launch": round(ins_per_launch, 1),
                "avg_launch_ms": round(avg_launch_ms, 4),
                "launches_per_step": round(launches / steps, 1),
                "model_per_attempt": {"bytes_per_attempt": round(b_att, 1),
                                      "attempts_per_launch": round(agg["timed_att"] / launches, 1),
                                      "achieved": round(att_achieved, 2), "frac": round(att_achieved / peak, 5)}}
    ball_ms = agg["ms_ball"] / max(agg["ball_launches"], 1)
    ball_per_ins = ball_bytes_per_insertion(F)
    ball_ach = ball_per_ins * agg["won"] / max(agg["ball_launches"], 1) / (ball_ms / 1000.0) / 1e9 if ball_ms > 0 else 0.0
    ball = {"bound": "hbm", "unit": "GB/s", "peak": peak,
            "kernel": ("k_ball, 1024-thread blocks, " + ("64 lanes per candidate in rounds below 32768 candidates, "
                                                        "16 above" if not lanes else
                                                        f"{64 if lanes == 64 else 16} lanes per candidate")),
            "achieved": round(ball_ach, 2), "frac": round(ball_ach / peak, 5),
            "bytes_per_insertion": round(ball_per_ins, 1), "avg_launch_ms": round(ball_ms, 4)}
    detail = {"rounds_per_step": agg["rounds"] / steps, "attempts_per_point": agg["attempts"] / max(n * steps, 1),
              "conflict_rate": agg["conflicts"] / att, "walk_steps_per_attempt": round(walk, 3),
              # attempts stopped by the walk cap (among the conflicts: they retry next round)
              "walk_cap_rate": agg["walk_caps"] / att,
              "cavity_tets": round(C, 2), "boundary_facets": round(F, 2),
              "ms_cavity_kernel_per_step": round(agg["ms_cav"] / steps, 3),
              "ms_ball_kernel_per_step": round(agg["ms_ball"] / steps, 3),
              "ball_roofline": ball,
              # host clock inside dt_insert_points: sort phase and insertion rounds; the
              # paper's sequential timings leave the sort out
              "ms_sort_per_step": round(agg["ms_sort"] / steps, 3),
              "ms_insert_per_step": round(agg["ms_insert"] / steps, 3),
              "insertion_only_tets_per_s": round(T / (agg["ms_insert"] / steps / 1000.0), 1)
              if agg["ms_insert"] > 0 else None,
              "orient_exact_rate": agg["orient_exact"] / max(agg["orient"], 1),
              "insphere_exact_rate": agg["insphere_exact"] / max(agg["insphere"], 1),
              "perturbed": agg["perturbed"], "step_ms": [round(1000 * t, 2) for t in times],
              "output_sha256": digest, "exported": export, "index_bits": st_last["index_bits"]}
    return {"value": round(value, 1), "ms_per_step": round(ms_per_step, 3), "tetrahedra": T,
            "roofline": roofline, "detail": detail, "tuned": tuned, "hash": digest, "canon": canon,
            "d_xyz": d_xyz}


def phase_clocks(d_xyz, lanes, progress):
    """One untimed step of the plain path with the library's trace level 2: per round, the
    filter pass's per-attempt wall clocks (walk, cavity, whole attempt, launch span), read back
    after every round.  Summarised over the step: the launch spans add up to the filter pass's
    time; the median attempt against the span shows how much of a launch is its tail."""
    import tempfile

    import torch

    from paper_1805_08831_amd import Triangulation

    old = os.environ.get("DT_TRACE")
    os.environ["DT_TRACE"] = "2"
    sys.stderr.flush()
    saved = os.dup(2)
    with tempfile.TemporaryFile(mode="w+") as fh:
        try:
            os.dup2(fh.fileno(), 2)
            stream = torch.cuda.current_stream()
            with Triangulation(device=0, stream=stream.cuda_stream, lanes_per_insert=lanes) as tri:
                tri.insert(d_xyz)
                torch.cuda.synchronize()
        finally:
            os.dup2(saved, 2)
            os.close(saved)
            if old is None:
                del os.environ["DT_TRACE"]
            else:
                os.environ["DT_TRACE"] = old
        fh.seek(0)
        lines = [ln for ln in fh if ln.startswith(("clocks ", "ballclocks "))]
    out = summarise_clocks(lines)
    if out is not None:
        progress(f"phase clocks: {out}")
    return out


def summarise_clocks(lines):
    """Summary of the library's per-round `clocks` and `ballclocks` trace lines (see
    phase_clocks)."""
    import re
    balls = []
    for ln in lines:
        if ln.startswith("ballclocks "):
            kv = dict(re.findall(r"(\w+)=([\d./]+)", ln))
            balls.append({k: [float(x) for x in v.split("/")] for k, v in kv.items()})
    lines = [ln for ln in lines if ln.startswith("clocks ")]
    rows = []
    for ln in lines:
        kv = dict(re.findall(r"(\w+)=([\d./]+)", ln))
        q = {k: [float(x) for x in v.split("/")] for k, v in kv.items()}
        rows.append(q)
    if not rows:
        return None
    span = sum(r["span_us"][0] for r in rows)
    att50 = sum(r["att_us"][0] for r in rows)
    att90 = sum(r["att_us"][1] for r in rows)
    walk50 = sum(r["walk_us"][0] for r in rows)
    cav50 = sum(r["cav_us"][0] for r in rows)
    n = sum(r["n"][0] for r in rows)
    big = [r for r in rows if r["n"][0] >= 4096]
    out = {
        "rounds": len(rows), "attempts": int(n),
        "sum_span_ms": round(span / 1000, 3),
        # per round: the median attempt, the 90th percentile and the span, summed over rounds
        "sum_att_p50_ms": round(att50 / 1000, 3), "sum_att_p90_ms": round(att90 / 1000, 3),
        "median_attempt_share_of_span": round(att50 / span, 4),
        "walk_share_of_median_attempt": round(walk50 / max(walk50 + cav50, 1e-9), 4),
        "walk_steps_per_attempt": round(sum(r["walk_steps"][0] * r["n"][0] for r in rows) / n, 3),
        "cavity_steps_per_attempt": round(sum(r["cav_steps"][0] * r["n"][0] for r in rows) / n, 3),
        "rounds_4096_or_more": {
            "rounds": len(big),
            "sum_span_ms": round(sum(r["span_us"][0] for r in big) / 1000, 3),
            "att_us_p50_p90_p99_max_mean": [round(sum(r["att_us"][k] for r in big) / max(len(big), 1), 2)
                                            for k in range(4)],
            "walk_us_p50_mean": round(sum(r["walk_us"][0] for r in big) / max(len(big), 1), 2),
            "cav_us_p50_mean": round(sum(r["cav_us"][0] for r in big) / max(len(big), 1), 2),
            "span_us_mean": round(sum(r["span_us"][0] for r in big) / max(len(big), 1), 2)},
        "rounds_below_4096": {
            "rounds": len(rows) - len(big),
            "sum_span_ms": round(sum(r["span_us"][0] for r in rows if r["n"][0] < 4096) / 1000, 3)},
    }
    if balls:
        bb = [b for b in balls if b["n"][0] >= 4096]
        mean = lambda key, k: round(sum(b[key][k] for b in bb) / max(len(bb), 1), 2)  # noqa: E731
        out["ball"] = {
            "rounds": len(balls), "sum_span_ms": round(sum(b["span_us"][0] for b in balls) / 1000, 3),
            "rounds_4096_or_more": {
                "rounds": len(bb), "span_us_mean": mean("span_us", 0),
                # winner test + slot reservation, cavity copies, building: median and 90th
                # percentile per round, averaged over the rounds
                "test_us_p50_p90": [mean("test_us", 0), mean("test_us", 1)],
                "copy_us_p50_p90": [mean("copy_us", 0), mean("copy_us", 1)],
                "build_us_p50_p90": [mean("build_us", 0), mean("build_us", 1)],
                "ball_us_p50_p90_p99_max": [mean("ball_us", k) for k in range(4)]}}
    return out


def compare_schedulers(d_xyz, model, steps, warmup, progress, reference, export=True):
    """Plain and learned scheduler on the same device input, timed the same way (insertion
    and tetrahedron count, no export); then each output, exported once, against the plain
    step's canonical output (without export: the tetrahedron counts only)."""
    res = {name: timed_runs(d_xyz, sched, model, steps, warmup, progress, name, reference if export else None)
           for name, sched in (("plain", 0), ("learned", 1))}
    out = dict(res["learned"], plain=res["plain"])
    if export:
        out["identical_output"] = bool(res["learned"]["identical"] and res["plain"]["identical"])
    else:
        out["identical_output"] = None
        out["same_count"] = res["learned"]["tetrahedra"] == res["plain"]["tetrahedra"]
    out["speedup_vs_plain"] = round(res["learned"]["value"] / res["plain"]["value"], 4)
    return out


def compare_graph_rounds(d_xyz, steps, warmup, progress, reference):
    """Regular rounds launched as one HIP graph each against separate kernel launches, both
    without events (timing 0), on the same device input; outputs compared with the main
    step's canonical output."""
    res = {name: timed_runs(d_xyz, 0, None, steps, warmup, progress, name, reference, timing=0, graph_rounds=g)
           for name, g in (("separate launches", False), ("graph rounds", True))}
    sep, gr = res["separate launches"], res["graph rounds"]
    return {"separate_ms_per_step": sep["ms_per_step"], "graph_ms_per_step": gr["ms_per_step"],
            "speedup": round(sep["ms_per_step"] / gr["ms_per_step"], 4), "rounds": gr["rounds"],
            "graph_launched_rounds": gr["graph_rounds"],
            "identical_output": None if reference is None else bool(sep["identical"] and gr["identical"])}


def train_scheduler(gen, seeds, samples, progress):
    """Plain runs with point logs on the training seeds (other seeds than the timed input),
    then the MLP trained on a random sample of the logged points.  Returns (model, info)."""
    import numpy as np
    import torch

    from paper_1805_08831_amd import Triangulation, dt_get_point_log, dt_train_model

    t0 = time.perf_counter()
    stream = torch.cuda.current_stream()
    feats, costs, buckets = [], [], []
    rng = np.random.default_rng(1)
    with Triangulation(device=0, stream=stream.cuda_stream, log_points=True) as tri:
        for s in seeds:
            tri.clear()
            pts = gen(s)
            progress(f"training run, seed {s}: {len(pts)} points generated")
            tri.insert(torch.from_numpy(pts).cuda())
            progress(f"training run, seed {s}: triangulated, {tri.stats()['rounds']} rounds")
            f, c, b = dt_get_point_log(tri.ctx)
            keep = rng.choice(len(c), min(len(c), samples // max(len(seeds), 1)), replace=False)
            feats.append(f[keep])
            costs.append(c[keep])
            buckets.append(b[keep])
        model = dt_train_model(tri.ctx, np.concatenate(feats), np.concatenate(costs), np.concatenate(buckets),
                               epochs=3, lr=1e-3, seed=1)
    info = {"seeds": list(seeds), "samples": int(sum(len(c) for c in costs)), "epochs": 3,
            "seconds": round(time.perf_counter() - t0, 2)}
    progress("model trained")
    return model, info


def timed_runs(d_xyz, sched, model, steps, warmup, progress, name, reference=None, adaptive_curve=False,
               timing=2, graph_rounds=False):
    """`steps` timed triangulations of d_xyz with the given scheduler; per-step means.  With
    a reference canonical output, the last triangulation is exported (untimed) and compared
    with it on the device."""
    import torch

    from paper_1805_08831_amd import Triangulation, dt_get_tets, dt_load_model

    stream = torch.cuda.current_stream()
    tri = Triangulation(device=0, stream=stream.cuda_stream, timing=timing, scheduler=sched,
                        adaptive_curve=adaptive_curve, graph_rounds=graph_rounds)
    if sched:
        dt_load_model(tri.ctx, model)
    for _ in range(warmup):
        tri.clear()
        tri.insert(d_xyz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = dict(rounds=0, attempts=0, conflicts=0, overflows=0, walk_steps=0, perturbed=0, insphere_exact=0,
               orient_exact=0, walk_caps=0, graph_rounds=0)
    T = 0
    for _ in range(steps):
        tri.clear()
        tri.insert(d_xyz)
        T = dt_get_tets(tri.ctx)
        st = tri.stats()
        progress(f"{name}: step done, {T} tetrahedra, {st['rounds']} rounds")
        for k in agg:
            agg[k] += st[k]
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    identical = None
    if reference is not None:
        out = torch.empty((T, 4), dtype=torch.int32, device="cuda")
        dt_get_tets(tri.ctx, out, None, T)
        identical = bool(out.shape == reference.shape and torch.equal(canonical_device(out), reference))
        del out
        progress(f"{name}: output {'identical to' if identical else 'DIFFERENT from'} the plain step's")
    tri.close()
    return {"value": round(T / (ms / 1000.0), 1), "ms_per_step": round(ms, 3), "tetrahedra": T,
            "identical": identical, **{k: v / steps for k, v in agg.items()}}


def run_mix(args):
    """MIX (4e6 lattice nodes + 3e6 points in 50 Gaussian clusters + 3e6 points near the
    unit sphere, shuffled), plain against learned scheduler on the same GPU.  The model is
    trained on the point logs of plain runs on other seeds (outside the timed region)."""
    import torch

    from synth import mix_points

    seed = args.seed if args.seed != 1007 else 2007
    sc = args.mix_scale
    counts = (int(4_000_000 * sc), int(3_000_000 * sc), int(3_000_000 * sc))
    t_start = time.perf_counter()

    def progress(msg):
        print(f"[mix] {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    seeds = [int(x) for x in args.train_seeds.split(",") if x]
    model, training = train_scheduler(lambda s: mix_points(s, *counts), seeds, args.train_samples, progress)
    d_xyz = torch.from_numpy(mix_points(seed, *counts)).cuda()
    reference, digest = reference_output(d_xyz)
    golden = golden_hash(sum(counts), seed, kind="mix")
    res = {name: timed_runs(d_xyz, sched, model, args.steps, args.warmup, progress, name, reference)
           for name, sched in (("plain", 0), ("learned", 1))}
    # the adaptive Moore curve (plain scheduler) on the same input
    res["adaptive"] = timed_runs(d_xyz, 0, model, args.steps, args.warmup, progress, "adaptive curve", reference,
                                 adaptive_curve=True)
    line = {
        "metric": "tetrahedra/sec (exact 3D Delaunay, MIX: lattice + clusters + shell)",
        "value": res["plain"]["value"],
        "unit": "tetrahedra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["plain"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"MIX {sum(counts)} ({counts[0]} nodes of the 160^3 lattice, {counts[1]} in 50 "
                               f"clusters, {counts[2]} within 1e-4 of the unit sphere), seed {seed}",
                   "scheduler": "plain"},
        "learned": dict(res["learned"], training=training,
                        speedup_vs_plain=round(res["learned"]["value"] / res["plain"]["value"], 4),
                        identical_output=bool(res["learned"]["identical"] and res["plain"]["identical"])),
        "plain": res["plain"],
        "adaptive_curve": dict(res["adaptive"],
                               speedup_vs_plain=round(res["adaptive"]["value"] / res["plain"]["value"], 4)),
        "output_sha256": digest,
        "oracle_hash_match": None if golden is None else digest == golden,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_points(
            mix_points(seed + 1, *(int(c * args.cpu_mix_scale) for c in counts)),
            f"MIX at {args.cpu_mix_scale} of the timed size (seed {seed + 1})"),
    }
    print(json.dumps(line), flush=True)


def run_batch(args):
    """Independent clouds (sizes log-uniform in [1e3, 2e5], each uniform in its own random
    box), dt_insert_batch over chunks of clouds; a step triangulates every cloud once.  Also
    times a sample of clouds inserted one call each (the single-cloud path in a loop)."""
    import numpy as np
    import torch

    from paper_1805_08831_amd import Triangulation
    from synth import batch_clouds

    xyz, off = batch_clouds(args.clouds, seed_base=3000)
    off = off.astype(np.int64)
    d_xyz = torch.from_numpy(xyz).cuda()
    stream = torch.cuda.current_stream()
    tri = Triangulation(device=0, stream=stream.cuda_stream, timing=2, lanes_per_insert=args.lanes)
    chunks = [(c, min(c + args.chunk, args.clouds)) for c in range(0, args.clouds, args.chunk)]

    def step():
        """Every chunk once; returns (tetrahedra, rounds) summed over the chunks (each chunk
        starts from a cleared context, which also resets the statistics)."""
        total, rounds = 0, 0
        for c0, c1 in chunks:
            p0, p1 = int(off[c0]), int(off[c1])
            tri.clear()
            tri.insert_batch(d_xyz[p0:p1], (off[c0:c1 + 1] - p0).astype(np.uint64))
            total += tri.num_tets()
            rounds += tri.stats()["rounds"]
        return total, rounds

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = 0
    rounds = 0
    for _ in range(args.steps):
        T, r = step()
        rounds += r
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    graph = None
    if not args.no_graph_compare:
        # the same steps without events, with separate launches and with every regular round
        # launched as one HIP graph
        timed = {}
        for name, g in (("separate", False), ("graph", True)):
            tri.close()
            tri = Triangulation(device=0, stream=stream.cuda_stream, timing=0, lanes_per_insert=args.lanes,
                                graph_rounds=g)
            step()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                Tg, _ = step()
            torch.cuda.synchronize()
            timed[name] = (1000.0 * (time.perf_counter() - t1) / args.steps, Tg, tri.stats()["graph_rounds"])
        graph = {"separate_ms_per_step": round(timed["separate"][0], 3),
                 "graph_ms_per_step": round(timed["graph"][0], 3),
                 "speedup": round(timed["separate"][0] / timed["graph"][0], 4),
                 "graph_launched_rounds_last_call": timed["graph"][2],
                 "same_count": timed["graph"][1] == T and timed["separate"][1] == T}
        print(f"[batch] graph rounds: {graph}", file=sys.stderr, flush=True)
        tri.close()
        tri = Triangulation(device=0, stream=stream.cuda_stream, timing=2, lanes_per_insert=args.lanes)
    # the same clouds, one dt_insert_points call each, on a sample
    sample = list(range(0, args.clouds, max(1, args.clouds // args.loop_sample)))[:args.loop_sample]
    tl, tt, pts = 0.0, 0, 0
    for c in sample:
        p0, p1 = int(off[c]), int(off[c + 1])
        tri.clear()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tri.insert(d_xyz[p0:p1])
        tt += tri.num_tets()
        torch.cuda.synchronize()
        tl += time.perf_counter() - t1
        pts += p1 - p0
    line = {
        "metric": "tetrahedra/sec (exact 3D Delaunay, batch of independent clouds)",
        "value": round(T / (ms / 1000.0), 1),
        "unit": "tetrahedra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.clouds} clouds, sizes log-uniform in [1e3, 2e5], uniform in random boxes, "
                               f"seeds 3000 + cloud",
                   "points": int(off[-1]), "tetrahedra": T, "clouds_per_call": args.chunk,
                   "calls_per_step": len(chunks), "rounds_per_step": rounds / max(args.steps, 1)},
        "graph_rounds": graph,
        "loop_single": {"value": round(tt / tl, 1), "unit": "tetrahedra/s",
                        "sample": f"{len(sample)} of the clouds ({pts} points), one dt_insert_points call each"},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_clouds(xyz, off, sample),
    }
    print(json.dumps(line), flush=True)
    tri.close()


def cpu_baseline_refine(xyz, n, h, sample_points):
    """The refinement oracle (one thread) on the input's points in the corner cube [0, s)^3
    that holds about sample_points of them, with the same h: tetrahedra of its final mesh per
    second of refinement (the input's triangulation included: the oracle retriangulates every
    step)."""
    import numpy as np

    from oracle.refine import refine
    s = (sample_points / n) ** (1.0 / 3.0)
    sub = xyz[np.all(xyz < s, axis=1)]
    t0 = time.perf_counter()
    pts, tets, _, steps = refine(sub, h)
    dt = time.perf_counter() - t0
    return {"value": round(len(tets) / dt, 1), "unit": "tetrahedra/s", "cores": 1, "kind": "oracle",
            "sample": f"the {len(sub)} input points in [0, {s:.4f})^3, refined with the same h to {len(pts)} "
                      f"points and {len(tets)} tetrahedra in {len(steps)} steps, serially in {dt:.2f} s",
            "cpu": host_cpu_model(), "host_threads": os.cpu_count()}


def run_refine(args):
    """Delaunay refinement by circumcentre insertion (paper Sec. 4, the sample / filter /
    insert loop of its mesh generator) over the convex hull of a uniform cloud.  A step
    triangulates the input (not timed) and then refines it with dt_refine: circumcentres of
    the tetrahedra with r > 1.4 h that lie strictly inside the hull, none within 0.7 h of a
    vertex or of a point kept before it, inserted through the same rounds, until a pass keeps
    none.  The timed part is the refinement alone, as the paper's refinement column leaves
    out the initial mesh; the value is the final mesh's tetrahedra per second of it."""
    import numpy as np
    import torch

    from paper_1805_08831_amd import Triangulation, dt_get_tets
    from paper_1805_08831_amd.dt import dt_refine
    from synth import uniform_points

    t_bench = time.perf_counter()

    def progress(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_bench:.1f} s)", file=sys.stderr, flush=True)

    n, h, seed = args.refine_n, args.refine_h, 4007
    xyz = uniform_points(n, seed)
    d_xyz = torch.from_numpy(xyz).cuda()
    stream = torch.cuda.current_stream()
    tri = Triangulation(device=0, stream=stream.cuda_stream, timing=2, lanes_per_insert=args.lanes,
                        round_fraction=args.round_fraction, round_size=args.round_size)
    keys = ("attempts", "walk_steps", "cavity_tets", "boundary_facets", "inserted", "ms_cavity_kernel",
            "cavity_launches", "rounds", "conflicts", "timed_insertions", "timed_attempts", "ms_sort", "ms_insert",
            "walk_caps", "deferred", "orient_calls", "orient_exact", "insphere_calls", "insphere_exact", "perturbed",
            "overflows")

    def step():
        tri.clear()
        tri.insert(d_xyz)
        T0 = dt_get_tets(tri.ctx)
        torch.cuda.synchronize()
        s0 = tri.stats()
        t0 = time.perf_counter()
        added, steps = dt_refine(tri.ctx, h)
        T = dt_get_tets(tri.ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s1 = tri.stats()
        return dt, T0, T, added, steps, {k: s1[k] - s0[k] for k in keys}

    for _ in range(args.warmup):
        step()
    runs = [step() for _ in range(args.steps)]
    ms = 1000.0 * sum(r[0] for r in runs) / len(runs)
    dt, T0, T, added, steps, d = runs[-1]
    if any(r[2] != T or r[3] != added or r[4] != steps for r in runs):
        raise RuntimeError("refinement runs differ")
    progress(f"refined {n} points to {n + added} ({T} tetrahedra) in {ms:.1f} ms, steps {steps}")
    agg = {k: sum(r[5][k] for r in runs) for k in keys}
    att, won = max(agg["attempts"], 1), max(agg["inserted"], 1)
    C, F = agg["cavity_tets"] / won, agg["boundary_facets"] / won
    launches = max(agg["cavity_launches"], 1)
    avg_launch_ms = agg["ms_cavity_kernel"] / launches
    per_ins = cavity_bytes_per_insertion(C, F)
    ins_per_launch = agg["timed_insertions"] / launches
    achieved = per_ins * ins_per_launch / (avg_launch_ms / 1000.0) / 1e9 if avg_launch_ms > 0 else 0.0
    ms_insert = agg["ms_sort"] / len(runs) + agg["ms_insert"] / len(runs)
    line = {
        "metric": "tetrahedra/sec (Delaunay refinement by circumcentre insertion, final mesh)",
        "value": round(T / (ms / 1000.0), 1),
        "unit": "tetrahedra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"refinement of {n} i.i.d. uniform fp64 points in [0,1)^3 (seed {seed}), "
                               f"h = {h}, convex hull as the domain",
                   "input_tetrahedra": T0, "points_added": added, "final_points": n + added,
                   "tetrahedra": T, "passes": [list(s) for s in steps]},
        "roofline": {"bound": "hbm", "kernel": "k_cavity_g filter pass (and exact pass once launched) of the refinement's "
                                               "insertion rounds of 32768 candidates or more",
                     "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 5), "traffic": None,
                     "bytes_per_insertion": round(per_ins, 1), "insertions_per_launch": round(ins_per_launch, 1),
                     "avg_launch_ms": round(avg_launch_ms, 4), "launches_per_step": round(launches / len(runs), 1)},
        "detail": {"points_added_per_s": round(added / (ms / 1000.0), 1),
                   # host clock inside the insertion calls; the rest is candidates, sorts and filter
                   "ms_insertion_per_step": round(ms_insert, 3),
                   "ms_selection_per_step": round(ms - ms_insert, 3),
                   "rounds_per_step": agg["rounds"] / len(runs),
                   "attempts_per_point": agg["attempts"] / max(agg["inserted"], 1),
                   "conflict_rate": agg["conflicts"] / att,
                   "walk_steps_per_attempt": round(agg["walk_steps"] / att, 3),
                   "cavity_tets": round(C, 2), "boundary_facets": round(F, 2),
                   # attempts stopped by the walk cap, handed to the exact pass, overflowed
                   "walk_cap_rate": agg["walk_caps"] / att, "deferred_rate": agg["deferred"] / att,
                   "overflow_rate": agg["overflows"] / att,
                   "orient_exact_rate": agg["orient_exact"] / max(agg["orient_calls"], 1),
                   "insphere_exact_rate": agg["insphere_exact"] / max(agg["insphere_calls"], 1),
                   "perturbed_per_step": agg["perturbed"] / len(runs),
                   "step_ms": [round(1000 * r[0], 2) for r in runs]},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_refine(xyz, n, h, args.cpu_refine_points),
    }
    print(json.dumps(line), flush=True)
    tri.close()


if __name__ == "__main__":
    main()

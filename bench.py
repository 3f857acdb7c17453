"""Benchmark: one step = create the flow problem from device-resident inputs
(validation + device layout), solve the maximum preflow by push-relabel with
global relabeling, extract the minimal source side (vertex and net bitmaps
into device memory), release the handle.

Workload: the large single flow -- 1,000,000 vertices, 2,000,000 nets with
Zipf(2.2) sizes clamped to [2, 1000] (about 7.4 M pins), unit net weights,
sources / sinks = the 1 % of vertices with the smallest / largest splitmix64
hash of (seed, vertex).  Synthetic, seeded.

Prints one JSON line (rank 0).  value = pins per second of whole steps.

A second workload is reported under "batch": the flow problems of a
partitioned 10M-pin hypergraph (2,000,000 vertices, Zipf(2.2) net sizes
clamped to [2, 2000], balanced random 64-way partition refined by three
label-propagation sweeps, the 500 heaviest adjacent block pairs, regions
grown around their cuts), solved with the source-side cut: refinements per
second of the plain schedule (one problem after another) against the tuned
batch plan, both on device-resident problems.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--vertices", type=int, default=1_000_000)
    ap.add_argument("--nets", type=int, default=2_000_000)
    ap.add_argument("--size-hi", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the block-pair batch workload")
    ap.add_argument("--no-regions", action="store_true",
                    help="skip the device construction of the block-pair problems")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 2,000-vertex solves-per-second leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the side-by-side of the two relabel variants")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-problems", type=int, default=500)
    ap.add_argument("--batch-schedule", type=int, default=0,
                    help="0: tune the batch plan; 1 union or 3 workgroups with 4 lanes and a "
                         "relabel every 8 rounds, untuned (no host worker threads start)")
    ap.add_argument("--no-cutter", action="store_true",
                    help="skip the incremental FlowCutter workload")
    ap.add_argument("--cutter-iterations", type=int, default=100000)
    ap.add_argument("--cutter-single-cap", type=int, default=40000,
                    help="iteration cap of the one-vertex-per-iteration FlowCutter run "
                         "(0 skips it; 250000 runs the 200k-vertex region to balance, "
                         "about 4 minutes)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-pruning workload")
    ap.add_argument("--learned-seeds", type=int, default=32,
                    help="block-pair instances per learned-pruning workload (3/4 train, "
                         "1/4 eval)")
    ap.add_argument("--learned-steps", type=int, default=2000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run one plain elementwise copy of BYTES bytes (counter "
                         "calibration for the traffic figure) and exit")
    ap.add_argument("--bfs-flat", type=int, default=0,
                    help="reverse-BFS levels: 1 flattened arcs per wave, -1 lane groups, 0 default")
    ap.add_argument("--bfs-marks", type=int, default=0,
                    help="expanded reverse-BFS levels: 1 byte marks, -1 labels, 0 default")
    ap.add_argument("--bfs-xcd", type=int, default=0,
                    help="expanded reverse-BFS levels labelled per XCD slice: 1 large networks, "
                         "2 always, -1 off (default)")
    ap.add_argument("--gather-probe", type=int, default=0, metavar="READS",
                    help="only run one gather of READS random 4-byte words (counter "
                         "calibration for scattered reads) and exit")
    ap.add_argument("--gr-interval", type=int, default=0,
                    help="device-wide rounds between global relabels (0: the library default)")
    ap.add_argument("--tail-gr-interval", type=int, default=0,
                    help="single-workgroup rounds between global relabels (0: the default)")
    ap.add_argument("--relabel-blocking", type=int, default=0,
                    help="1: the blocking variant of the round (a node pushed to does not "
                         "relabel in that round)")
    ap.add_argument("--profile", type=int, default=2,
                    help="HIP-event timing inside the timed steps: 0 off, 1 every kernel, "
                         "2 only the reverse-BFS level kernel (the dominant one)")
    ap.add_argument("--profile-steps", type=int, default=1,
                    help="timed steps (the last ones) that record the kernel events; the "
                         "steps repeat the same work, and the events cost about 1.3 ms a "
                         "step, so the others run without them")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the max-flow path runs on one GPU (asked for --gpus {args.gpus}); "
              "no run on several GPUs is measured", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.gather_probe:
        # one gather kernel: GATHER random 4-byte reads from a 256 MiB table,
        # the indices read and the values written sequentially; its counters
        # give the bytes a scattered 4-byte read fetches
        n = args.gather_probe
        table = torch.ones((1 << 26), dtype=torch.int32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        idx = torch.randint(0, 1 << 26, (n,), dtype=torch.int64, device="cuda", generator=g)
        idx = idx.to(torch.int32)
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        torch.index_select(table, 0, idx, out=out)
        torch.cuda.synchronize()
        print(json.dumps(dict(gather_probe_reads=n, table_bytes=4 << 26)), flush=True)
        return

    if args.copy_probe:
        # one kernel that reads BYTES and writes BYTES: the HBM counters of
        # this launch calibrate those of the solver kernels
        n = args.copy_probe // 4
        x = torch.ones(n, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_probe_bytes=4 * n)), flush=True)
        return

    from paper_2201_01556_amd import hyperflow, inputs

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hyperflow.load_library()

    _log("generating input")
    hg = inputs.zipf_hypergraph(args.seed, args.vertices, args.nets, size_hi=args.size_hi)
    P, V, E = hg.num_pins, hg.num_vertices, hg.num_nets
    arrays = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
              for a in (hg.net_offsets, hg.pins, hg.net_weights, hg.sources, hg.sinks)]
    vs = torch.zeros(V, dtype=torch.uint8, device=dev)
    ns = torch.zeros(E, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step(profile):
        opts = hyperflow.Options(profile=profile, bfs_flat=args.bfs_flat,
                                 bfs_marks=args.bfs_marks,
                                 relabel_blocking=args.relabel_blocking, bfs_xcd=args.bfs_xcd,
                                 gr_interval=args.gr_interval,
                                 tail_gr_interval=args.tail_gr_interval)
        h = hyperflow.flow_problem_create(V, *arrays, options=opts, stream=stream)
        try:
            F = hyperflow.maxflow_solve(h, stream)
            hyperflow.mincut_source_side(h, V, E, vs, ns, stream)
            st = hyperflow.flow_problem_stats(h)
            kt = hyperflow.flow_problem_kernel_times(h) if profile else None
        finally:
            hyperflow.flow_problem_destroy(h)
        return F, st, kt

    profile = args.profile
    prof_steps = max(0, min(args.profile_steps, args.steps)) if profile else 0
    if prof_steps == 0:
        profile = 0
    for i in range(args.warmup):
        _log(f"warmup {i}")
        step(profile)  # also fills the library's event pool
    torch.cuda.synchronize()
    times, kts, stats, ev_timed = [], [], [], []
    F = None
    for i in range(args.steps):
        p = profile if i >= args.steps - prof_steps else 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, st, kt = step(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        ev_timed.append(bool(p))
        if kt is not None:
            kts.append(kt)
        stats.append(st)
        _log(f"step {i}: {dt * 1e3:.2f} ms flow={F} rounds={st['rounds']} "
             f"gr={st['global_relabels']} syncs={st['host_syncs']} events={'on' if p else 'off'}")
    total = sum(times)
    ms_per_step = 1e3 * total / args.steps
    value = P * args.steps / total
    step_ms_split = dict(
        with_events=(round(1e3 * float(np.mean([t for t, e in zip(times, ev_timed) if e])), 3)
                     if any(ev_timed) else None),
        without_events=(round(1e3 * float(np.mean([t for t, e in zip(times, ev_timed) if not e])), 3)
                        if not all(ev_timed) else None))

    step_traffic = measured_step_traffic()
    roofline = None
    kernels = None
    if profile:
        agg = {}
        for kt in kts:
            for k in kt:
                a = agg.setdefault(k["kernel"], dict(launches=0, ms=0.0, bytes=0.0))
                a["launches"] += k["launches"]
                a["ms"] += k["ms"]
                a["bytes"] += k["bytes"]
        kernels = {k: dict(launches=v["launches"], ms=round(v["ms"] / prof_steps, 4),
                           avg_us=round(1e3 * v["ms"] / max(v["launches"], 1), 3),
                           bytes_per_launch=(v["bytes"] / max(v["launches"], 1)))
                   for k, v in agg.items() if v["launches"]}
        # dominant kernel with a device byte count
        cand = {k: v for k, v in agg.items() if v["launches"] and v["bytes"] > 0}
        if cand:
            dom = max(cand, key=lambda k: cand[k]["ms"])
            d = cand[dom]
            bpl = d["bytes"] / d["launches"]
            avg_s = d["ms"] / d["launches"] / 1e3
            achieved = bpl / avg_s / 1e9
            roofline = dict(kernel=dom, bound="hbm", achieved=round(achieved, 3),
                            peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=round(achieved / HBM_PEAK_GBS, 6),
                            traffic=measured_traffic(dom),
                            bytes_per_launch=bpl, avg_launch_us=round(avg_s * 1e6, 3),
                            share_of_step=round(d["ms"] / prof_steps / ms_per_step, 4),
                            timed_steps=prof_steps)

    # the round's two fixes of the push-relabel conflict side by side (the
    # paper's blocking fix, against the default bounded relabel)
    variants = {}
    for blk in (() if args.no_variants else (0, 1)):
        ts = []
        for _ in range(3):
            o = hyperflow.Options(relabel_blocking=blk)
            torch.cuda.synchronize()
            t = time.perf_counter()
            h = hyperflow.flow_problem_create(V, *arrays, options=o, stream=stream)
            try:
                Fv = hyperflow.maxflow_solve(h, stream)
                hyperflow.mincut_source_side(h, V, E, vs, ns, stream)
                sv = hyperflow.flow_problem_stats(h)
            finally:
                hyperflow.flow_problem_destroy(h)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        variants["blocking" if blk else "bounded_relabel"] = dict(
            ms=round(1e3 * min(ts), 3), flow=Fv, rounds=sv["rounds"],
            global_relabels=sv["global_relabels"], relabels=sv["relabels"],
            restarts=sv["restarts"])

    copy = copy_ceiling(torch)
    _log(f"copy ceiling {copy['GBps']} GB/s")
    if roofline is not None:
        roofline["frac_of_copy_ceiling"] = round(roofline["achieved"] / copy["GBps"], 6)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        _log("cpu baseline (oracle, one thread pinned to one core)")
        Fo, vso, nso, dt, core = oracle.maxflow_pinned(hg)
        cpu = dict(value=P / dt, unit="pins/s", cores=1, kind="oracle",
                   sample="the full workload once: explicit-Lawler FIFO push-relabel solve "
                          "plus source-side BFS, one thread in a process pinned to one core "
                          "(timed around solve + BFS only)", seconds=round(dt, 3),
                   pinned_core=core)
        parity = bool(F == Fo and np.array_equal(vs.cpu().numpy(), vso) and
                      np.array_equal(ns.cpu().numpy(), nso))

    small = None if args.no_small else bench_small(args, hyperflow, inputs, torch, np)

    cutter = None
    if not args.no_cutter:
        cutter = bench_cutter(args, hyperflow, inputs, torch, np)

    batch = None
    learned = None
    del arrays, vs, ns
    torch.cuda.empty_cache()
    regions = None
    if not args.no_batch:
        batch = bench_batch(args, hyperflow, inputs, torch, np)
        if not args.no_regions:
            regions = bench_regions(args, hyperflow, inputs, torch, np)
            regions["refine"] = bench_refine(args, hyperflow, inputs, torch, np)
    if not args.no_learned:
        learned = bench_learned(args, hyperflow, inputs, torch, np,
                                batch["config"] if batch else None)

    st = stats[-1]
    out = {
        "metric": "pins/s per max-flow solve (create + solve + source-side cut)",
        "value": value,
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"zipf single flow: {V} vertices, {E} nets, Zipf(2.2) sizes "
                        f"clamped to [2,{args.size_hi}], unit weights, 1% hash-selected "
                        f"sources and sinks",
            "seed": args.seed, "pins": P, "flow_value": F,
            "rounds": st["rounds"], "tail_rounds": st["tail_rounds"],
            "global_relabels": st["global_relabels"], "host_syncs": st["host_syncs"],
            "kernel_timing": profile, "kernel_timed_steps": prof_steps,
        },
        "step_ms": step_ms_split,
        # whole step: algorithmic bytes of all counted kernels over the step time
        "step_alg_bytes": st["alg_bytes"],
        "step_alg_GBps": round(st["alg_bytes"] / (ms_per_step / 1e3) / 1e9, 3),
        # whole step: counter bytes of every kernel of a profiled step (L2 to
        # fabric, so an upper bound of HBM traffic) over this run's step time
        "step_traffic": (None if step_traffic is None else dict(
            bytes=step_traffic, GBps=round(step_traffic / (ms_per_step / 1e3) / 1e9, 1),
            source="profiles/zipf1M_bfs_rev_traffic.md")),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "dataset": dict(sha256=hg.sha256(), seed=args.seed, generator="zipf_hypergraph"),
        "host": host_info(),
        "copy_ceiling": copy,
        "small": small,
        "relabel_variants": variants,
        "paper_context": PAPER_CONTEXT,
        "kernels": kernels,
        "batch": batch,
        "regions": regions,
        "cutter": cutter,
        "learned": learned,
    }
    print(json.dumps(out), flush=True)


# The paper's own numbers for this path (self-relative CPU speedups; no
# absolute throughput is reported): context, not a target.
PAPER_CONTEXT = {
    "source": "section Scalability (flow networks of the large benchmark set) and the "
              "appendix on flow algorithms",
    "machine": "AMD EPYC Rome 7702P, 64 cores, 2.0-3.35 GHz, 1 TB (machine B)",
    "parallel_push_relabel_speedup_gmean": {"threads": [4, 16, 64], "speedup": [3.1, 4.4, 4.7]},
    "parallel_push_relabel_speedup_gmean_seq_ge_10s": {"threads": [4, 16, 64],
                                                       "speedup": [3.2, 7.0, 9.9]},
    "flowcutter_speedup_gmean": {"threads": [4, 16, 64], "speedup": [3.0, 4.2, 4.4]},
    "flowcutter_speedup_gmean_seq_ge_10s": {"threads": [4, 16, 64],
                                            "speedup": [3.1, 6.5, 8.6]},
    "restricted_capacities_largest_instance": "one flow computation: more than 2 h -> 14 s "
                                              "on 16 cores",
}


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(cpu_model=model, cpu_count=os.cpu_count(),
                cpus_allowed=len(os.sched_getaffinity(0)))


def copy_ceiling(torch):
    """Measured HBM ceiling: a plain 1 GiB device-to-device copy (read +
    write bytes over its HIP-event time), best of five."""
    n = (1 << 30) // 4
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    best = None
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    torch.cuda.empty_cache()
    return dict(GBps=round(2 * (1 << 30) / (best / 1e3) / 1e9, 1), bytes=2 * (1 << 30),
                kernel="torch copy_ (one read, one write of 1 GiB)")


def bench_small(args, hyperflow, inputs, torch, np):
    """Small single flows (2,000 vertices, 3,000 nets, sizes U{2..8},
    weights U{1..4}, 100 sources, 100 sinks; seeds 0..9): whole-state
    fits the caches, so the figure is the time per solve (create + solve +
    source side, device-resident inputs), not bandwidth."""
    hgs = [inputs.uniform_hypergraph(sd) for sd in range(10)]
    dev = torch.device("cuda:0")
    arrs = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev)
             for a in (h.net_offsets, h.pins, h.net_weights, h.sources, h.sinks)] for h in hgs]
    vs = torch.zeros(2000, dtype=torch.uint8, device=dev)
    ns = torch.zeros(3000, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def one(h, a):
        hnd = hyperflow.flow_problem_create(h.num_vertices, *a, stream=stream)
        try:
            F = hyperflow.maxflow_solve(hnd, stream)
            hyperflow.mincut_source_side(hnd, h.num_vertices, h.num_nets, vs, ns, stream)
        finally:
            hyperflow.flow_problem_destroy(hnd)
        return F

    for h, a in zip(hgs, arrs):
        one(h, a)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    flows = []
    for _ in range(reps):
        for h, a in zip(hgs, arrs):
            flows.append(one(h, a))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    n = reps * len(hgs)
    out = dict(workload="uniform single flows: 2000 vertices, 3000 nets, sizes U{2..8}, "
                        "weights U{1..4}, 100 sources, 100 sinks, seeds 0..9",
               us_per_solve=round(1e6 * dt / n, 1), solves_per_s=round(n / dt, 1),
               pins_per_s=round(sum(h.num_pins for h in hgs) * reps / dt, 1),
               flows=flows[:len(hgs)])
    # many such flows at once: the union schedule against the workgroups
    # schedule (one persistent launch, a workgroup per problem), flows and
    # source sides included, best of three runs each
    many = [inputs.uniform_hypergraph(sd) for sd in range(512)]
    probs = [hyperflow.FlowProblem.from_hypergraph(h, device=True) for h in many]
    try:
        res = {}
        for name, cfg in (("union", dict(schedule=1)), ("workgroups", dict(schedule=3))):
            with hyperflow.FlowBatch(probs, with_cut=True, **cfg) as b:
                b.run(with_cut=True)
                torch.cuda.synchronize()
                best = None
                for _ in range(3):
                    t = time.perf_counter()
                    f = b.run(with_cut=True)
                    torch.cuda.synchronize()
                    best = min(best or 1e9, time.perf_counter() - t)
                res[name] = (f, best)
        out["batch_512"] = dict(
            workload="512 of these flows (seeds 0..511) in one batch plan with the source sides",
            union_ms=round(1e3 * res["union"][1], 2),
            workgroups_ms=round(1e3 * res["workgroups"][1], 2),
            workgroups_solves_per_s=round(512 / res["workgroups"][1], 1),
            flows_equal=bool((res["union"][0] == res["workgroups"][0]).all()),
            flows_match_single=[int(x) for x in res["workgroups"][0][:len(hgs)]] ==
            flows[:len(hgs)])
    finally:
        for p_ in probs:
            p_.close()
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "zipf1M_bfs_rev_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2201_01556_amd", "csrc", f)
                  for f in ("hf_device.h", "hf_solve.hip")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic_values():
    """Machine-readable lines of the committed counter summary, or None when
    the kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and line.lstrip().startswith("- "):
                k, v = line.strip()[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return vals


def measured_step_traffic():
    """Counter bytes (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy)
    of every kernel of one whole step, or None (see _traffic_values)."""
    vals = _traffic_values()
    try:
        return float(vals["step_traffic_bytes"]) if vals else None
    except (KeyError, ValueError):
        return None


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy), or None when the
    kernel sources changed since the counters were taken."""
    vals = _traffic_values() if kernel == "bfs_rev" else None
    if not vals:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _cut_weight(hg, side, np):
    off = hg.net_offsets.astype(np.int64)
    sizes = np.diff(off)
    inside = side[hg.pins].astype(np.int64)
    net_of = np.repeat(np.arange(hg.num_nets), sizes)
    cnt = np.bincount(net_of, weights=inside, minlength=hg.num_nets)
    cut = (cnt > 0) & (cnt < sizes)
    return int(hg.net_weights[cut].sum())


def bench_cutter(args, hyperflow, inputs, torch, np):
    """Incremental FlowCutter on one region: 200,000 vertices, 400,000 nets
    with Zipf(2.2) sizes clamped to [2, 200], vertex weights U{1..3}, 1 %
    hash-selected sources and sinks, eps = 0.03, warm-started flows.  The
    headline runs one piercing vertex per iteration to a balanced cut (or
    the iteration cap); the "bulk" entry runs bulk piercing with the
    paper's beta = 0.55 to a balanced cut and on to the most balanced cut.
    Each timed region is the whole FlowCutter run."""
    _log("generating the FlowCutter region")
    hg = inputs.zipf_hypergraph(args.seed, 200_000, 400_000, size_hi=200, vertex_weight_hi=3)
    c = hg.vertex_weights
    L = (103 * (-(-int(c.sum()) // 2))) // 100
    iters = args.cutter_iterations
    out = dict(workload=f"flowcutter: {hg.num_vertices} vertices, {hg.num_nets} nets, "
                        f"Zipf(2.2) sizes clamped to [2,200], vertex weights U{{1..3}}, "
                        f"eps=0.03 (L={L}), one piercing vertex per iteration (smallest-id "
                        f"free boundary vertex of the lighter side), run to balance or "
                        f"{args.cutter_single_cap} iterations",
               pins=hg.num_pins, unit="iterations/s")
    if args.cutter_single_cap > 0:
        # one run, driven in slices of 10,000 iterations (a continued run
        # takes exactly the steps of an uninterrupted one) so that the
        # progress is printed while it runs
        with hyperflow.FlowProblem.from_hypergraph(hg, device=True) as p:
            torch.cuda.synchronize()
            t = time.perf_counter()
            cap, sl = args.cutter_single_cap, 10_000
            res, x, trace = p.flowcutter(c, L, L, max_iterations=min(sl, cap))
            while res["resumable"] and res["iterations"] < cap:
                _log(f"single-pierce FlowCutter: {res['iterations']} iterations, "
                     f"{time.perf_counter() - t:.1f} s, flow {res['flow']}")
                res, x, tail = p.flowcutter_continue(
                    max_iterations=min(sl, cap - res["iterations"]), vertex_side=x)
                trace += tail
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
        xb = np.asarray(x).astype(bool)
        out.update(value=round(res["iterations"] / dt, 2), iterations=res["iterations"],
                   seconds=round(dt, 3), status=res["status"], flow=res["flow"],
                   source_weight=res["source_weight"], sink_weight=res["sink_weight"],
                   augmenting=res["augmenting"],
                   cut_certificate=_cut_weight(hg, xb, np) == res["flow"],
                   last_step=list(trace[-1]))
        _log(f"single-pierce FlowCutter: {res['iterations']} iterations in {dt:.2f} s, "
             f"{res['status']}")
    bulk = dict(variant="bulk piercing beta=0.55 (paragraph Bulk Piercing), run to balance")
    out["bulk"] = bulk
    with hyperflow.FlowProblem.from_hypergraph(hg, device=True) as p:
        torch.cuda.synchronize()
        t = time.perf_counter()
        res, x, trace = p.flowcutter(c, L, L, max_iterations=iters, bulk_percent=55)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
    xb = np.asarray(x).astype(bool)
    counts = res["counts"]
    bulk.update(value=round(res["iterations"] / dt, 2), iterations=res["iterations"],
               seconds=round(dt, 3), status=res["status"], flow=res["flow"],
               source_weight=res["source_weight"], sink_weight=res["sink_weight"],
               augmenting=res["augmenting"], pierced_vertices=int(sum(counts)),
               bulk_iterations=int(sum(1 for k in counts if k > 1)),
               cut_certificate=_cut_weight(hg, xb, np) == res["flow"],
               first_steps=[list(t) for t in trace[:3]], last_step=list(trace[-1]))
    # the same run continued to the most balanced cut (paragraph "Most
    # Balanced Cut"): pierces that avoid augmenting paths, no solves
    with hyperflow.FlowProblem.from_hypergraph(hg, device=True) as p:
        torch.cuda.synchronize()
        t = time.perf_counter()
        mb, xm, _ = p.flowcutter(c, L, L, max_iterations=iters, bulk_percent=55,
                                 most_balanced=True)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t
    xmb = np.asarray(xm).astype(bool)
    bulk["most_balanced"] = dict(
        iterations=mb["iterations"], first_balanced=mb["first_balanced"],
        seconds=round(dtm, 3), status=mb["status"], flow=mb["flow"],
        source_weight=mb["source_weight"], sink_weight=mb["sink_weight"],
        heavier_side=max(mb["source_weight"], mb["sink_weight"]),
        heavier_side_first_balanced=max(res["source_weight"], res["sink_weight"]),
        cut_certificate=_cut_weight(hg, xmb, np) == mb["flow"])
    if not args.no_cpu_baseline:
        import oracle
        k = 3
        t = time.perf_counter()
        ref = oracle.flowcutter(hg, c, L, L, max_iterations=k, bulk_percent=55)
        dt = time.perf_counter() - t
        bulk["parity_vs_oracle_prefix"] = [tuple(s) for s in ref.trace] == \
            [tuple(s) for s in trace[:k]]
        out["cpu_baseline"] = dict(value=round(k / dt, 3), unit="iterations/s", cores=1,
                                   kind="oracle",
                                   sample=f"the first {k} iterations, every max flow solved from "
                                          "scratch, single thread")
    return out


_PAIRS = {}
_BATCH_FLOWS = {}


def _pairs(inputs, seed, max_problems):
    """Block-pair instance of a seed, built once per run (the batch and the
    learned legs share seed 0)."""
    key = (seed, max_problems)
    if key not in _PAIRS:
        _PAIRS[key] = inputs.block_pair_problems(seed, max_problems=max_problems)
    return _PAIRS[key]


def _gen_pairs(job):
    """One seed's block-pair problems, built in a worker process (one
    builder thread each); with `graph`, also the partitioned hypergraph they
    come from (for the device construction of the same problems)."""
    kind, seed, nprob, graph = job
    from paper_2201_01556_amd import inputs
    gen = inputs.planted_block_pair_problems if kind == "planted" else inputs.block_pair_problems
    bp = gen(seed, max_problems=nprob, threads=1)
    for h in bp.problems:
        h.meta.pop("gid", None)
    g = None
    if graph:
        hg = bp.hypergraph
        g = dict(num_vertices=hg.num_vertices, net_offsets=hg.net_offsets, pins=hg.pins,
                 net_weights=hg.net_weights, vertex_weights=hg.vertex_weights, block=bp.block,
                 block_weights=bp.block_weights, k=int(len(bp.block_weights)))
    return seed, bp.problems, g


def _device_pipeline(hyperflow, inputs, torch, np, graph, pairs, cuts, scorer, theta):
    """Plain and learned schedules on device-built regions of one seed:
    (plain flows, learned flows with -1 for skipped pairs, plain seconds,
    learned seconds)."""
    dv = [torch.from_numpy(np.ascontiguousarray(graph[k])).to("cuda")
          for k in ("net_offsets", "pins", "net_weights", "vertex_weights", "block")]
    caps = inputs.region_caps(graph["block_weights"], pairs, cuts)
    torch.cuda.synchronize()

    def run(learned):
        torch.cuda.synchronize()
        t = time.perf_counter()
        with hyperflow.FlowRegions(graph["num_vertices"], *dv, graph["k"], pairs, caps,
                                   merge_identical=False) as rg:
            skip = None
            if learned and scorer is not None:
                skip = (scorer.predict(rg.features(cuts, graph["block_weights"])) <
                        theta).astype(np.uint8)
            f = rg.solve(skip)
        torch.cuda.synchronize()
        return f, time.perf_counter() - t

    run(False)  # first construction of this shape: allocations
    f_plain, t_plain = run(False)
    f_learn, t_learn = run(True)
    return f_plain, f_learn, t_plain, t_learn


# thresholds that give up this fraction of the improving training problems
SWEEP = (0.01, 0.05, 0.1, 0.25)


def bench_learned(args, hyperflow, inputs, torch, np, config):
    """Learned pruning (seeds 0..K-1, the first 3/4 train, the rest
    evaluate) on two block-pair workloads: the block pairs of a random k=64
    partition refined by label propagation (the batch workload), and the
    same construction on a hypergraph with planted blocks whose partition
    is good except around perturbed block pairs.  Labels come from the plain
    schedule (the union batch, every problem solved): a problem improves
    when its minimum cut is lighter than the cut it had (cut_before - F >
    0).  The scorer trains on the device (full-batch Adam); its threshold is
    the largest one that skips no improving training problem (a sweep also
    reports the thresholds that give up 1, 5, 10 and 25 % of the improving
    training problems: their skip rates and missed gains on the evaluation
    seeds).  On the evaluation seeds the plain batch, the learned schedule (inference, then
    the batch of the kept problems) and the paper's cut < 10 rule are timed,
    all with the source-side cut.  Seeds are built on a pool of worker
    processes while the device labels and evaluates earlier ones."""
    import concurrent.futures as cf
    import multiprocessing as mp
    K = max(2, args.learned_seeds)
    n_train = max(1, (3 * K) // 4)
    workers = max(1, min(16, len(os.sched_getaffinity(0)) - 1))
    out = {}
    for kind in ("random_blocks", "planted"):
        _log(f"learned pruning, {kind} workload: {K} seeds, built on {workers} processes")
        res = dict(workload=(
            "block pairs of a random k=64 partition refined by 3 label-propagation sweeps "
            "(2M vertices, 10M pins, Zipf(2.2) sizes clamped to [2,2000], 500 heaviest pairs)"
            if kind == "random_blocks" else
            "block pairs of a planted 64-block hypergraph (2M vertices, 10M pins, Zipf(2.2) "
            "sizes clamped to [2,2000], 98% of the nets inside one block), the planted "
            "partition with 2% of the vertices swapped across 150 random block pairs, 3 "
            "label-propagation sweeps, 500 heaviest pairs"),
            seeds=f"0..{K - 1}: train 0..{n_train - 1}, evaluate {n_train}..{K - 1}",
            label="minimum cut lighter than the cut before (plain union schedule)",
            unit="refinements/s")
        t0 = time.perf_counter()
        Xtr, ytr = [], []
        ev = dict(problems=0, positive=0, plain_s=0.0, learned_s=0.0, rule_s=0.0, skipped=0,
                  missed_gain=0, total_gain=0, rule_skipped=0, rule_missed_gain=0,
                  dev_plain_s=0.0, dev_learned_s=0.0, dev_equal=True)
        sc = None
        theta, usable, thetas = 1.0, False, {}
        try:
            with cf.ProcessPoolExecutor(max_workers=workers,
                                        mp_context=mp.get_context("spawn")) as ex:
                jobs = [(kind, sd, args.batch_problems, sd >= n_train) for sd in range(K)]
                for seed, hgs, graph in ex.map(_gen_pairs, jobs):
                    feats = inputs.scorer_features(hgs)
                    cb = np.array([h.meta["cut_before"] for h in hgs], dtype=np.int64)
                    pair_cut = np.array([h.meta["cut"] for h in hgs], dtype=np.int64)
                    pairs_l = [h.meta["pair"] for h in hgs]
                    probs = [hyperflow.FlowProblem.from_hypergraph(h, device=True) for h in hgs]
                    del hgs
                    torch.cuda.synchronize()
                    try:
                        with hyperflow.FlowBatch(probs, with_cut=True) as plan:
                            def timed(skip=None):
                                torch.cuda.synchronize()
                                t = time.perf_counter()
                                f = plan.run(skip=skip, with_cut=True)
                                torch.cuda.synchronize()
                                return f, time.perf_counter() - t
                            flows, t_plain = timed()
                            gain = cb - flows
                            if seed < n_train:
                                Xtr.append(feats)
                                ytr.append((gain > 0).astype(np.float32))
                                _log(f"  {kind} seed {seed}: {len(gain)} problems, "
                                     f"{int((gain > 0).sum())} improve")
                            else:
                                ts = time.perf_counter()
                                pr = sc.predict(feats) if usable else np.ones(len(gain),
                                                                                np.float32)
                                skip = (pr < theta).astype(np.uint8)
                                t_inf = time.perf_counter() - ts
                                for q, th in thetas.items():
                                    sk = pr < th
                                    sw = ev.setdefault(f"miss_train_{q}", [0, 0])
                                    sw[0] += int(sk.sum())
                                    sw[1] += int(gain[sk & (gain > 0)].sum())
                                _, t_kept = timed(skip)
                                rule = (pair_cut < 10).astype(np.uint8)
                                _, t_rule = timed(rule)
                                ev["problems"] += len(gain)
                                ev["positive"] += int((gain > 0).sum())
                                ev["plain_s"] += t_plain
                                ev["learned_s"] += t_inf + t_kept
                                ev["rule_s"] += t_rule
                                ev["skipped"] += int(skip.sum())
                                ev["missed_gain"] += int(gain[(skip > 0) & (gain > 0)].sum())
                                ev["total_gain"] += int(gain[gain > 0].sum())
                                ev["rule_skipped"] += int(rule.sum())
                                ev["rule_missed_gain"] += int(gain[(rule > 0) & (gain > 0)].sum())
                                if graph is not None:
                                    # the same schedules end to end on the device:
                                    # regions built there (inputs resident), then
                                    # all pairs solved, or the scorer on the
                                    # regions' own features and the kept pairs
                                    f_dev, f_learn, t_dp, t_dl = _device_pipeline(
                                        hyperflow, inputs, torch, np, graph, pairs_l, pair_cut,
                                        sc if usable else None, theta)
                                    ev["dev_plain_s"] += t_dp
                                    ev["dev_learned_s"] += t_dl
                                    kept = f_learn >= 0
                                    ev["dev_equal"] = ev["dev_equal"] and bool(
                                        (f_dev == flows).all() and
                                        (f_learn[kept] == flows[kept]).all() and
                                        (~kept == (skip > 0)).all())
                                _log(f"  {kind} eval seed {seed}: {int((gain > 0).sum())} "
                                     f"improve, skipped {int(skip.sum())} of {len(gain)}")
                    finally:
                        for p in probs:
                            p.close()
                    if seed == n_train - 1:  # every training seed is labelled: train
                        res["build_and_label_s"] = round(time.perf_counter() - t0, 2)
                        Xtr = np.concatenate(Xtr)
                        ytr = np.concatenate(ytr)
                        res.update(train_problems=int(len(ytr)),
                                   train_positive_fraction=round(float(ytr.mean()), 4))
                        init = inputs.scorer_init_params(0)
                        sc = hyperflow.Scorer(init)
                        sc.fit_normalization(Xtr)
                        if kind == "random_blocks" and not args.no_cpu_baseline:
                            # the oracle's inputs never come from the device path:
                            # the check uses the training features with seeded
                            # coin-flip labels
                            from oracle import mlp as omlp
                            ychk = np.random.default_rng(0).integers(0, 2, len(Xtr))
                            ychk = ychk.astype(np.float32)
                            loss_gpu, g_gpu = sc.gradient(Xtr, ychk)
                            xn, _, _ = omlp.normalize(Xtr)
                            loss_ref, g_ref = omlp.grad(init.astype(np.float64), xn, ychk)
                            res["gradient_rel_err_vs_oracle"] = float(
                                np.linalg.norm(g_gpu - g_ref) / max(np.linalg.norm(g_ref), 1e-30))
                        ts = time.perf_counter()
                        losses = sc.train(Xtr, ytr, args.learned_steps, lr=1e-3)
                        torch.cuda.synchronize()
                        res["train_s"] = round(time.perf_counter() - ts, 3)
                        res["loss_first_last"] = [float(losses[0]), float(losses[-1])]
                        params, _ = sc.params()
                        usable = bool(np.all(np.isfinite(params)))
                        ptr = sc.predict(Xtr)
                        pos = ytr > 0
                        theta = float(ptr[pos].min()) if pos.any() else 1.0
                        if usable and pos.any():
                            thetas = {q: float(np.quantile(ptr[pos], q)) for q in SWEEP}
                        res["sweep_thresholds"] = {f"miss_train_{q}": round(v, 6)
                                                   for q, v in thetas.items()}
                        res["threshold"] = theta
                        res["train_skip_rate"] = round(float((ptr < theta).mean()), 4)
                        res["fallback_to_plain"] = not usable
        finally:
            if sc is not None:
                sc.close()
        n = ev["problems"]
        res.update(eval_problems=n,
                   eval_positive_fraction=round(ev["positive"] / max(n, 1), 4),
                   skip_rate=round(ev["skipped"] / max(n, 1), 4),
                   missed_gain=ev["missed_gain"], total_gain=ev["total_gain"],
                   missed_gain_pct=round(100.0 * ev["missed_gain"] / max(ev["total_gain"], 1), 3),
                   device_pipeline=dict(
                       note="eval seeds: regions built on the device from the resident "
                            "hypergraph, then all pairs solved (plain) or the scorer on the "
                            "regions' device features and the kept pairs (learned)",
                       plain_value=round(n / ev["dev_plain_s"], 2) if ev["dev_plain_s"] else None,
                       learned_value=(round(n / ev["dev_learned_s"], 2)
                                      if ev["dev_learned_s"] else None),
                       flows_and_skips_equal_host_built=ev["dev_equal"]),
                   value=round(n / ev["learned_s"], 2) if ev["learned_s"] else None,
                   plain_value=round(n / ev["plain_s"], 2) if ev["plain_s"] else None,
                   rule_value=round(n / ev["rule_s"], 2) if ev["rule_s"] else None,
                   rule_skip_rate=round(ev["rule_skipped"] / max(n, 1), 4),
                   rule_missed_gain=ev["rule_missed_gain"],
                   threshold_sweep={k: dict(skip_rate=round(v[0] / max(n, 1), 4),
                                            missed_gain=v[1],
                                            missed_gain_pct=round(
                                                100.0 * v[1] / max(ev["total_gain"], 1), 3))
                                    for k, v in ev.items() if k.startswith("miss_train_")},
                   seconds=round(time.perf_counter() - t0, 2))
        out[kind] = res
    return out


def bench_batch(args, hyperflow, inputs, torch, np):
    """Plain (one problem after another) vs tuned batch plan on the
    block-pair problems; every run solves and extracts the source side."""
    t0 = time.perf_counter()
    _log("generating the block-pair workload")
    bp = _pairs(inputs, args.seed, args.batch_problems)
    hgs = bp.problems
    gen_s = time.perf_counter() - t0
    n = len(hgs)
    pins = int(sum(h.num_pins for h in hgs))
    _log(f"{n} problems, {pins} pins; creating on the device")
    probs = [hyperflow.FlowProblem.from_hypergraph(h, device=True) for h in hgs]
    torch.cuda.synchronize()
    out = dict(workload=f"block pairs: {bp.hypergraph.num_vertices} vertices, "
                        f"{bp.hypergraph.num_pins} pins, Zipf(2.2) sizes clamped to [2,2000], "
                        f"k=64 random + 3 label-propagation sweeps, {n} heaviest pairs",
               problems=n, pins=pins, generate_s=round(gen_s, 2), unit="refinements/s")
    try:
        plain = hyperflow.FlowBatch(probs, with_cut=True, schedule=2, streams=1)
        if args.batch_schedule:
            batched = hyperflow.FlowBatch(probs, with_cut=True, schedule=args.batch_schedule,
                                          group_lanes=4, gr_interval=8)
            out["tune_s"] = None
            out["config"] = batched.config()
        else:
            batched = hyperflow.FlowBatch(probs, with_cut=True)
            _log("tuning the batch plan")
            t0 = time.perf_counter()
            cfg = batched.tune()
            out["tune_s"] = round(time.perf_counter() - t0, 2)
            out["config"] = cfg

        def timed(plan, steps):
            ts = []
            flows = None
            for _ in range(steps):
                for p in probs:
                    p.reset()
                torch.cuda.synchronize()
                t = time.perf_counter()
                flows = plan.run(with_cut=True)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            return flows, ts

        _log("plain schedule")
        f_plain, ts_plain = timed(plain, 1)
        _log("batched schedule")
        f_batch, ts_batch = timed(batched, args.batch_steps)
        plain_rate = n / min(ts_plain)
        batch_rate = n / min(ts_batch)
        out.update(plain_value=round(plain_rate, 2), value=round(batch_rate, 2),
                   plain_ms=round(1e3 * min(ts_plain), 2),
                   batched_ms=[round(1e3 * t, 2) for t in ts_batch],
                   speedup=round(batch_rate / plain_rate, 3),
                   pins_per_s=round(pins * batch_rate / n, 1))
        same = bool(np.array_equal(f_plain, f_batch))
        certs = True
        gain = 0
        improved = 0
        for i, h in enumerate(hgs):
            vsd, _ = batched.sides(i)
            certs &= _cut_weight(h, vsd, np) == int(f_batch[i])
            d = h.meta["cut_before"] - int(f_batch[i])
            gain += d
            improved += d > 0
        out.update(flows_equal_plain=same, cut_certificates=certs, total_gain=int(gain),
                   improved=int(improved))
        _BATCH_FLOWS[args.seed] = [int(f) for f in f_batch]
        if not args.no_cpu_baseline:
            import oracle
            sample = [0, n // 2, n - 1]
            t = time.perf_counter()
            for i in sample:
                oracle.maxflow(hgs[i])
            dt = time.perf_counter() - t
            out["cpu_baseline"] = dict(value=round(len(sample) / dt, 3), unit="refinements/s",
                                       cores=1, kind="oracle",
                                       sample=f"problems {sample} of the batch, solve + source side, "
                                              "single thread")
            workers = min(16, len(os.sched_getaffinity(0)))
            _log(f"oracle on all {n} problems, {workers} processes")
            t = time.perf_counter()
            refs = oracle.maxflow_many(hgs, workers=workers)
            dt = time.perf_counter() - t
            ok = True
            for i, (Fo, vso, nso) in enumerate(refs):
                vsd, nsd = batched.sides(i)
                ok &= (Fo == int(f_batch[i]) and
                       np.array_equal(vsd.astype(bool), vso.astype(bool)) and
                       np.array_equal(nsd, nso))
            out["parity_vs_oracle_all"] = bool(ok)
            out["cpu_baseline_all_cores"] = dict(
                value=round(n / dt, 3), unit="refinements/s", cores=workers, kind="oracle",
                sample=f"all {n} problems, one process per core (wall time including process "
                       "start)")
        plain.close()
        batched.close()
    finally:
        for p in probs:
            p.close()
    return out


def bench_refine(args, hyperflow, inputs, torch, np):
    """Refinement rounds on the device (flow_partition_refine: quotient
    graph, regions of the active pairs, union minimum cuts, moves applied
    with the balance check and revert) on the two block-pair workloads'
    partitions (random k=64 + label propagation; planted blocks with 150
    perturbed pairs), timed from the partition on the device to the refined
    partition."""
    out = {}
    for kind, gen in (("random_blocks", inputs.block_pair_problems),
                      ("planted", inputs.planted_block_pair_problems)):
        _log(f"refinement rounds, {kind} workload")
        bp = gen(args.seed, max_problems=1, threads=0)
        hg = bp.hypergraph
        dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
               for a in (hg.net_offsets, hg.pins, hg.net_weights, hg.vertex_weights, bp.block)]
        torch.cuda.synchronize()
        with hyperflow.FlowPartition(hg.num_vertices, *dev, 64) as part:
            torch.cuda.synchronize()
            t = time.perf_counter()
            res, traj = part.refine(max_rounds=8)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            blocks, bw, obj = part.get()
        cv = int(hg.vertex_weights.sum())
        lmax = (103 * (-(-cv // 64))) // 100
        res.update(seconds=round(dt, 3), objective_per_round=[int(x) for x in traj],
                   pairs_per_s=round(res["pairs_tried"] / dt, 1),
                   balanced=bool(int(bw.max()) <= lmax),
                   improvement_pct=round(100.0 * (res["objective_before"] - res["objective_after"])
                                         / max(res["objective_before"], 1), 3))
        out[kind] = res
        del dev
        torch.cuda.empty_cache()
    return out


def _host_region_build_s(inputs, np, bp, pairs, cuts, threads):
    """Seconds of the host input builder (regions.c) for the same pairs on
    `threads` host threads (context for the device builder; it is input
    generation, not the oracle)."""
    import ctypes
    L = inputs._regions_lib()
    hg = bp.hypergraph

    def ptr(a):
        return a.ctypes.data_as(ctypes.c_void_p)

    blk = np.ascontiguousarray(bp.block, dtype=np.int32)
    ctx = L.hfr_new(hg.num_vertices, hg.num_nets, ptr(hg.net_offsets), ptr(hg.pins),
                    ptr(hg.net_weights), ptr(hg.vertex_weights), 64, ptr(blk))
    try:
        pi = np.ascontiguousarray([p[0] for p in pairs], dtype=np.int32)
        pj = np.ascontiguousarray([p[1] for p in pairs], dtype=np.int32)
        pc = np.ascontiguousarray(cuts, dtype=np.int64)
        t = time.perf_counter()
        if L.hfr_regions(ctx, len(pairs), ptr(pi), ptr(pj), ptr(pc), 8, 148, 100, threads) != 0:
            raise MemoryError("region builder: out of memory")
        return time.perf_counter() - t
    finally:
        L.hfr_free(ctx)


def bench_regions(args, hyperflow, inputs, torch, np):
    """Device construction of the block-pair flow problems (section "Network
    Construction"): the 500 heaviest pairs of the block-pair workload,
    regions grown by two breadth-first searches, nets built with s and t,
    identical nets merged.  Timed from hypergraph, partition and pairs
    resident on the device to the built problems on the device; then the
    whole refinement step (build, then all pairs solved as one union network
    built from the regions, with the minimal source sides)."""
    bp = _pairs(inputs, args.seed, args.batch_problems)
    hg = bp.hypergraph
    pairs = [p.meta["pair"] for p in bp.problems]
    cuts = [p.meta["cut"] for p in bp.problems]
    caps = inputs.region_caps(bp.block_weights, pairs, cuts)
    n = len(pairs)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
           for a in (hg.net_offsets, hg.pins, hg.net_weights, hg.vertex_weights, bp.block)]
    torch.cuda.synchronize()
    out = dict(workload=f"region construction of the {n} heaviest block pairs of the block-pair "
                        f"workload ({hg.num_vertices} vertices, {hg.num_pins} pins, k=64), "
                        "identical nets merged",
               unit="problems/s", problems=n)

    def build(merge):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rg = hyperflow.FlowRegions(hg.num_vertices, *dev, 64, pairs, caps, merge_identical=merge)
        torch.cuda.synchronize()
        return rg, time.perf_counter() - t

    _log("device region construction")
    times, rg = [], None
    for _ in range(4):
        if rg is not None:
            rg.close()
        rg, dt = build(True)
        times.append(dt)
    ms = sorted(times[1:])[1] * 1e3
    info = [rg.info(q) for q in range(n)]
    out.update(value=round(n / (ms / 1e3), 1), ms=round(ms, 2),
               pins_built=int(sum(i["num_pins"] for i in info)),
               nets_built=int(sum(i["num_nets"] for i in info)),
               nets_merged=int(sum(i["merged"] for i in info)))
    rg2, dt2 = build(False)
    out["ms_without_merging"] = round(dt2 * 1e3, 2)
    same = all(int(rg2.info(q)["num_pins"]) == bp.problems[q].num_pins for q in range(n))
    out["unmerged_equal_host_builder_sizes"] = bool(same)
    rg2.close()
    # the refinement step from resident inputs: build, one union solve of
    # all pairs straight from the regions (flow_regions_solve)
    _log("build + union solve")
    step = []
    flows = None
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r3 = hyperflow.FlowRegions(hg.num_vertices, *dev, 64, pairs, caps)
        try:
            flows = r3.solve()
            torch.cuda.synchronize()
            step.append(time.perf_counter() - t)
        finally:
            r3.close()
    ms_step = sorted(step)[1] * 1e3
    out["build_and_solve"] = dict(value=round(n / (ms_step / 1e3), 1), unit="refinements/s",
                                  ms=round(ms_step, 2))
    out["flows_equal_host_built"] = None
    if batch_flows := _BATCH_FLOWS.get(args.seed):
        out["flows_equal_host_built"] = [int(f) for f in flows] == list(batch_flows)
    rg.close()
    threads = len(os.sched_getaffinity(0))
    hs = _host_region_build_s(inputs, np, bp, pairs, cuts, threads)
    out["host_builder_all_cores"] = dict(ms=round(hs * 1e3, 1), threads=threads,
                                         note="regions.c input builder, no identical-net merging")
    if not args.no_cpu_baseline:
        from oracle import regions as oreg
        t = time.perf_counter()
        vnets = oreg.vertex_nets(hg)
        t_v = time.perf_counter() - t
        q = n - 1
        t = time.perf_counter()
        oreg.build_region(hg, bp.block, hg.vertex_weights, pairs[q][0], pairs[q][1],
                          int(caps[q][0]), int(caps[q][1]), remove_identical=True, vnets=vnets)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = dict(value=round(1.0 / dt, 4), unit="problems/s", cores=1,
                                   kind="oracle",
                                   sample=f"one pair (the lightest of the {n}), plain Python, after "
                                          f"{t_v:.1f} s for the vertex incidences")
    del dev
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()

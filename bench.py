"""Benchmark: graphBpp spanning trees/s on the 16M-vertex, 64M-edge signed
graph (Chung-Lu exponent 2.3, 85 % positive), achieved HBM bandwidth of the
sweep kernel against MI355X's peak, graphL steps/s, and the CPU oracle on a
bounded sample.

One step = one full sweep of --trees trees over the resident graph: reset the
cloud, build every tree (BFS with the min-key parent rule and fused state
propagation), count its frustrated edges, key its canonical state, insert it
into the frustration cloud, and read back the minimum.  Inputs are generated
on the host and uploaded before timing.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def algorithmic_bytes_per_tree(n: int, nnz: int) -> int:
    """Bytes one tree must move at minimum in this design: row offsets (4 per
    vertex) and the packed adjacency (4 per CSR entry) once for the BFS, the
    upper-triangle edge list (8 per undirected edge) once for the count, and
    one 8-byte tree word written and read back per vertex."""
    m = nnz // 2
    return 4 * (n + 1) + 4 * nnz + 8 * m + 16 * n


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_grid.hip", "sweep_multi.hip", "fi_multi.h", "fi_prims.h",
              "fi_internal.h"):
        with open(os.path.join(ROOT, "paper_2311_00869_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_sweep_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sha") != kernel_source_sha():
        return None
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trees", type=int, default=1000)
    ap.add_argument("--workload", choices=["large", "mid", "small", "planted"], default="large")
    ap.add_argument("--path", type=int, default=0, help="schedule path (0 = tuned default)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--heavy", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graphl", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-trees", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-planted", action="store_true", help="skip the 10^4-tree planted leg")
    ap.add_argument("--no-bounded", action="store_true",
                    help="skip the memory-bound cloud leg (Alg. alg-scale)")
    ap.add_argument("--no-switches", action="store_true",
                    help="skip the switch-list and cloud-statistics leg")
    ap.add_argument("--no-samplers", action="store_true",
                    help="skip the leg timing the other tree samplers")
    ap.add_argument("--no-graphl-large", action="store_true",
                    help="skip graphL on the main graph (32 restarts x 500 steps)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_sweep_<workload>.json from two rocprofv3 "
                         "counter collections (FETCH_SIZE, WRITE_SIZE) of a --copy-probe-mib run")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1], args)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: every box here has one MI355X, and the sweep shards "
              "trees across GPUs only by design (see the multi-GPU notes); use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_00869_amd import frustration as fr
    from paper_2311_00869_amd import synth
    from paper_2311_00869_amd import tune

    batch_graphs = None
    if not args.no_batch:
        # generated before the GPU is touched; workers are spawned either way
        t_gen = time.perf_counter()
        batch_graphs = synth.config_batch_parallel(4096, 0)
        print(f"# generated the uneven batch in {time.perf_counter() - t_gen:.1f}s",
              file=sys.stderr, flush=True)

    t_gen = time.perf_counter()
    if args.workload == "large":
        g = synth.config_large(0)
        wname = "chung-lu n=16,000,000 m=64,000,000 gamma=2.3 p+=0.85"
    elif args.workload == "mid":
        g = synth.chung_lu(100000, 500000, 2.3, 0, p_pos=0.85)
        wname = "chung-lu n=100,000 m=500,000 gamma=2.3 p+=0.85"
    elif args.workload == "planted":
        g = synth.config_planted_powerlaw(0)
        wname = "planted chung-lu n=1,000,000 m=10,000,000 gamma=2.1 flip=0.05"
    else:
        g = synth.config_small(0)
        wname = "path+uniform n=1,000 m=5,000 p+=0.8"
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {wname} in {t_gen:.1f}s", file=sys.stderr, flush=True)

    if args.copy_probe_mib:
        # one elementwise kernel that reads and writes copy_probe_mib MiB
        src = torch.ones((args.copy_probe_mib << 20) // 4, dtype=torch.int32, device="cuda")
        dst = torch.add(src, 1)
        torch.cuda.synchronize()
        del src, dst

    T = args.trees
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=T)
    sched = tune.default_schedule(G.n, G.nnz)
    for k in ("path", "block", "grid", "heavy", "batch"):
        v = getattr(args, k)
        if v:
            sched[k] = v
    G.set_schedule(**sched)
    print(f"# schedule {G.get_schedule()}", file=sys.stderr, flush=True)

    def step(seed):
        G.cloud_reset()
        G.sweep(T, seed)
        return G.min_frustration()

    for w in range(args.warmup):
        step(1000 + w)
    torch.cuda.synchronize()
    G.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best = None
    for s in range(args.steps):
        best = step(s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, launches = G.prof_read(0)
    G.prof_enable(False)
    trees_per_s = T * args.steps / elapsed
    states = G.cloud_size()
    print(f"# {args.steps} steps x {T} trees in {elapsed:.3f}s; min switches {best}, "
          f"{states} states in the last cloud", file=sys.stderr, flush=True)

    bpt = algorithmic_bytes_per_tree(G.n, G.nnz)
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    achieved = bpt * T / avg_launch_s / 1e9
    traffic = load_traffic(args.workload)
    roofline = {
        "kernel": {3: "k_sweep_grid", 4: "k_sweep_multi", 5: "k_sweep_multi"}.get(
            G.get_schedule()["path"], "k_sweep_wg"),
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None if traffic is None else traffic["bytes_per_launch"],
        "algorithmic_bytes_per_launch": bpt * T, "avg_launch_ms": round(avg_launch_s * 1e3, 3),
        "launches": launches,
    }

    sched_used = G.get_schedule()
    extra = {}
    if not args.no_bounded:
        extra["bounded"] = bench_bounded(fr, torch, G, T, args.steps, best)
    if not args.no_switches:
        extra["switches"] = bench_switches(fr, torch, G, T, args.steps, elapsed / args.steps)
    if not args.no_graphl_large:
        extra["graphl_large"] = bench_graphl_large(synth, torch, G)
    if not args.no_plain:
        # the plain per-tree path: one launch per tree, one tree in flight
        # (whole-grid path, no batching of trees)
        G.set_schedule(path=3, block=1024, batch=1)
        G.cloud_reset()
        Tp = min(T, 100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(Tp):
            G.sweep_range(t, t + 1, 7)
        torch.cuda.synchronize()
        extra["plain_per_tree_trees_per_s"] = round(Tp / (time.perf_counter() - t0), 2)

    if not args.no_graphl:
        extra["graphl"] = bench_graphl(fr, synth, torch)
    if batch_graphs is not None:
        extra["batch"] = bench_batch(fr, tune, torch, batch_graphs, args.steps)
        del batch_graphs
    if not args.no_planted:
        extra["planted"] = bench_planted(fr, synth, tune, torch)
    if not args.no_samplers:
        extra["samplers"] = bench_samplers(fr, synth, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, args.cpu_trees)

    out = {
        "metric": "spanning trees/sec + GB/s vs HBM peak (16M-vertex graph); graphL steps/sec",
        "value": round(trees_per_s, 2),
        "unit": "trees/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wname, "trees_per_step": T, "seed": "step index",
                   "schedule": sched_used},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "min_switches_last_step": best[0] if best else None,
        "distinct_states_last_step": states,
    }
    out.update(extra)
    G.close()
    print(json.dumps(out), flush=True)


def bench_bounded(fr, torch, G, T, steps, unbounded_best, fmax=100, chunk=250):
    """Alg. alg-scale on the same graph and trees as the main leg: a cloud of
    at most F_max states, merged every `chunk` trees; then the merges alone,
    timed with events on the stream they run on."""
    C = fr.BoundedCloud(fmax, staging=G.cloud_capacity)
    G.sweep_bounded(C, 0, chunk, 999)
    C.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best = None
    for s in range(steps):
        C.reset()
        G.sweep_bounded(C, 0, T, s, chunk=chunk)
        best = C.min_frustration()
    el = time.perf_counter() - t0
    held = C.size()
    C.reset()
    G.cloud_reset()
    ev = []
    for a in range(0, T, chunk):
        b = min(T, a + chunk)
        G.sweep_range(a, b, steps - 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        C.merge(G, a, b)
        e1.record()
        ev.append((e0, e1))
    torch.cuda.synchronize()
    merge_ms = [a.elapsed_time(b) for a, b in ev]
    out = {
        "workload": f"the main leg's graph and trees, F_max={fmax}, a merge every {chunk} trees",
        "trees_per_s": round(T * steps / el, 2), "ms_per_step": round(el / steps * 1e3, 3),
        "merges_per_step": len(merge_ms), "merge_ms_avg": round(sum(merge_ms) / len(merge_ms), 4),
        "entries_held": held, "min_switches": best[0],
        "min_equals_unbounded": best == tuple(unbounded_best),
    }
    C.close()
    G.cloud_reset()
    return out


def bench_switches(fr, torch, G, T, steps, plain_step_s):
    """The balanced state as a list of edges to switch (one tree's state, the
    whole edge list compacted in order), and a sweep that also gathers the
    per-vertex and per-edge tree counts, against the plain sweep's step."""
    import numpy as np
    words, s0 = G.tree_state(0, 0)
    bits = torch.from_numpy(words.view(np.int64)).cuda()
    out = torch.empty((s0 + 1, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    lib, st = G.lib, fr._stream_ptr()
    call = lambda: lib.fi_switch_list(G.handle, fr._ptr(bits), fr._ptr(out), s0 + 1, fr._ptr(cnt), st)
    call()
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert int(cnt.item()) == s0
    # two passes over the 8-byte edge list, the pairs written, the state read twice
    nbytes = 2 * 8 * G.m + 8 * s0 + 2 * G.n // 8
    vm = torch.zeros(G.n, dtype=torch.int64, device="cuda")
    es = torch.zeros(G.m, dtype=torch.int64, device="cuda")
    G.cloud_reset()
    G.sweep_stats(0, 64, 999, vm, es)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        G.cloud_reset()
        G.sweep_stats(0, T, s, vm, es)
    G.min_frustration()
    el = (time.perf_counter() - t0) / steps
    G.cloud_reset()
    return {
        "switch_list": {"edges_switched": s0, "ms": round(ms, 3),
                        "algorithmic_bytes": nbytes, "GB_per_s": round(nbytes / ms / 1e6, 1)},
        "stats_sweep": {"trees_per_s": round(T / el, 2), "ms_per_step": round(el * 1e3, 3),
                        "vs_plain_sweep": round(plain_step_s / el, 4)},
    }


def bench_graphl_large(synth, torch, G, R=32, steps=500, alpha=0.001):
    """graphL on the main graph: R restarts x `steps` descent steps with the
    overflow policy, then rounding and the exact count of every restart."""
    gamma0 = torch.from_numpy(synth.graphl_init(G.n, R, 0)).cuda()
    G.graphl_descend(gamma0, 4, alpha)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    out, scales = G.graphl_descend(gamma0, steps, alpha)
    e1.record()
    counts = G.round_count(out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / steps
    # per step: row offsets and adjacency once, R floats gathered per CSR
    # entry, each vertex's R floats read and written
    nbytes = 4 * (G.n + 1) + 4 * G.nnz + 4 * G.nnz * R + 8 * G.n * R
    res = {
        "workload": f"the main graph, {R} restarts x {steps} steps, alpha={alpha}",
        "steps_per_s": round(steps / el, 2), "restart_steps_per_s": round(steps * R / el, 1),
        "step_ms": round(step_ms, 3), "algorithmic_bytes_per_step": nbytes,
        "GB_per_s": round(nbytes / step_ms / 1e6, 1),
        "best_rounded_frustration": int(counts.min()), "max_log2_scale": int(scales().max()),
    }
    del gamma0, out
    return res


def bench_graphl(fr, synth, torch):
    """graphL on the 1,000-vertex graph: 32 restarts x 500 steps in one
    launch (fi_graphl_descend) then rounding and the exact count, against one
    launch per step for all restarts and against 32 separate single-restart
    runs (the plain per-restart path)."""
    g = synth.config_small(0)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)
    R, steps, alpha = 32, 500, 0.001
    gamma0 = torch.from_numpy(synth.graphl_init(g.n, R, 0)).cuda()
    G.graphl_descend(gamma0, 20, alpha)
    fr.graphl_descent(G, gamma0, 20, alpha)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, _ = G.graphl_descend(gamma0, steps, alpha)
    counts = G.round_count(out)
    torch.cuda.synchronize()
    batched = time.perf_counter() - t0
    t0 = time.perf_counter()
    stepwise = fr.graphl_descent(G, gamma0, steps, alpha)
    G.round_count(stepwise)
    torch.cuda.synchronize()
    per_step = time.perf_counter() - t0
    assert torch.equal(stepwise, out)
    t0 = time.perf_counter()
    for r in range(R):
        o = fr.graphl_descent(G, gamma0[:, r:r + 1].contiguous(), steps, alpha)
        G.round_count(o)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    # autograd path: forward + hand-written backward + torch SGD update
    gam = gamma0.clone().requires_grad_(True)
    opt = torch.optim.SGD([gam], lr=alpha)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        opt.zero_grad(set_to_none=True)
        fr.graphl_loss(G, gam).sum().backward()
        opt.step()
    torch.cuda.synchronize()
    autograd = (time.perf_counter() - t0) / 100
    G.close()
    return {
        "workload": "n=1,000 m=5,000, 32 restarts, 500 steps, alpha=0.001",
        "steps_per_s": round(steps / batched, 1),
        "restart_steps_per_s": round(steps * R / batched, 1),
        "launch_per_step_steps_per_s": round(steps / per_step, 1),
        "plain_per_restart_restart_steps_per_s": round(steps * R / plain, 1),
        "autograd_steps_per_s": round(1.0 / autograd, 1),
        "best_rounded_frustration": int(counts.min().item()),
    }


def _counter_per_dispatch(path, counter):
    """Sum of `counter` per dispatch id (over all hardware instances), with the
    kernel name of each dispatch, from a rocprofv3 counter_collection CSV."""
    import csv
    per = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            d = per.setdefault(r["Dispatch_Id"], [r["Kernel_Name"], 0.0])
            d[1] += float(r["Counter_Value"])
    return per


def summarize_traffic(fetch_csv, write_csv, args):
    """HBM bytes per launch of the sweep kernel: FETCH_SIZE and WRITE_SIZE (KiB)
    of its dispatches, each scaled by what the same counter reads for the copy
    probe (copy_probe_mib MiB read and as many written)."""
    out = {"workload": args.workload, "kernel_sha": kernel_source_sha(),
           "copy_probe_mib": args.copy_probe_mib}
    total = 0.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = _counter_per_dispatch(path, name)
        copies = [v for k, v in per.values() if "elementwise" in k.lower()]
        sweeps = [v for k, v in per.values() if "k_sweep_" in k]
        if not copies or not sweeps:
            raise SystemExit(f"{path}: no copy probe or no sweep dispatch for {name}")
        probe_kib = max(copies)
        scale = (args.copy_probe_mib << 20) / probe_kib  # bytes per counted KiB
        per_launch = sum(sweeps) / len(sweeps) * scale
        out[name] = {"probe_kib": probe_kib, "bytes_per_counted_kib": scale,
                     "sweep_dispatches": len(sweeps), "bytes_per_launch": per_launch}
        total += per_launch
    out["bytes_per_launch"] = total
    dst = os.path.join(ROOT, "profiles", f"traffic_sweep_{args.workload}.json")
    with open(dst, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def bench_batch(fr, tune, torch, graphs, steps, trees=64):
    """The uneven batch: 4,096 graphs x 64 trees in one fi_batch_sweep,
    captured once as a HIP graph and replayed; against one launch per tree on
    a sample of the graphs (the plain path)."""
    G = len(graphs)
    B = fr.BatchGraph(graphs, cloud_capacity_per_graph=trees)
    sched, _ = tune.autotune_batch(B, trees=2, save=False)
    mn = torch.zeros((G, 2), dtype=torch.int64, device="cuda")
    ds = torch.zeros(G, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.sweep_into(trees, 0, mn, ds)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    B.status()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.sweep_into(trees, 0, mn, ds)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    B.status()
    out = {
        "workload": f"{G} path+uniform graphs, n ~ U{{100..50,000}}, avg degree ~ U[4,16], "
                    f"p+ ~ U[0.7,0.9], {trees} trees each, seed 0",
        "trees_per_s": round(G * trees * steps / el, 1),
        "ms_per_step": round(el / steps * 1e3, 3),
        "schedule": sched, "hip_graph": True,
        "total_nnz": int(B.nnz_offsets[-1]),
        "sum_min_switches": int(mn[:, 0].sum().item()),
    }
    del graph
    B.close()
    # plain path: one single-graph handle and one launch per tree, 16 graphs
    Gp, Tp = 16, 8
    t_plain = 0.0
    for g in graphs[:: G // Gp][:Gp]:
        H = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=Tp)
        H.set_schedule(**tune.default_schedule(H.n, H.nnz))
        H.sweep_range(0, 1, 9)
        torch.cuda.synchronize()
        H.cloud_reset()
        t0 = time.perf_counter()
        for t in range(Tp):
            H.sweep_range(t, t + 1, 0)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        H.close()
    out["plain_per_tree_trees_per_s"] = round(Gp * Tp / t_plain, 1)
    return out


def bench_planted(fr, synth, tune, torch, trees=10_000):
    """10^4 trees in one sweep of the 1M-vertex planted graph."""
    g = synth.config_planted_powerlaw(0)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=trees)
    G.set_schedule(**tune.default_schedule(G.n, G.nnz))
    G.sweep(64, 1)
    torch.cuda.synchronize()
    G.cloud_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.sweep(trees, 0)
    best = G.min_frustration()
    el = time.perf_counter() - t0
    out = {
        "workload": "planted chung-lu n=1,000,000 m=10,000,000 gamma=2.1 flip=0.05, seed 0",
        "trees": trees, "trees_per_s": round(trees / el, 1), "schedule": G.get_schedule(),
        "min_switches": best[0], "planted_flipped": int(g.meta.get("flipped", -1)),
        "distinct_states": G.cloud_size(),
    }
    G.close()
    return out


def bench_samplers(fr, synth, torch):
    """Trees per second of every sampler on the 1,000-vertex graph and on a
    100,000-vertex graph, with the best switch count each reached.  Each runs
    on the library's own choice of path: one tree per workgroup, except BFS
    on the larger graph, which takes 128 trees per pass."""
    out = {}
    # the small graph's sweep takes well under a millisecond: time ten of them
    for name, g, K, reps in (("n=1,000 m=5,000", synth.config_small(0), 8192, 10),
                             ("n=100,000 m=500,000", synth.erdos_renyi_connected(100000, 500000, 0.8, 7),
                              512, 1)):
        G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=K)
        row = {}
        for smp in ("bfs", "rdfs", "hybrid", "kruskal"):
            G.set_sampler(smp)
            G.cloud_reset()
            G.sweep(64, 99)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(reps):
                G.cloud_reset()
                G.sweep(K, 0)
            best = G.min_frustration()
            el = (time.perf_counter() - t0) / reps
            row[smp] = {"trees_per_s": round(K / el, 1), "min_switches": best[0]}
        out[f"{name}, {K} trees"] = row
        G.close()
    return out


def cpu_baseline(g, trees):
    """The CPU oracle, untuned and single-threaded, on `trees` trees of the same
    graph (trees/s)."""
    import oracle
    t0 = time.perf_counter()
    oracle.sweep(g, 0, 0, trees, checks=False)
    el = time.perf_counter() - t0
    return {"value": round(trees / el, 5), "unit": "trees/s", "cores": 1, "kind": "oracle",
            "sample": f"trees 0..{trees - 1} of the same graph, seed 0, single thread, "
                      f"{el:.1f}s"}


if __name__ == "__main__":
    main()

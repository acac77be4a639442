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
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def model_bytes(n: int, nnz: int, trees: int, trees_per_pass: int) -> dict:
    """Algorithmic HBM bytes of a sweep (the per-tree model of the hot path).

    One tree, unbatched: two passes over the CSR (row offsets, 4-byte column
    and 1-byte sign per entry; one pass builds the BFS tree, one counts the
    frustrated edges), an 8-byte level/parent word written and read back per
    vertex, and the n-bit state:  B_tree = 2 (4 (n+1) + 5 nnz) + 16 n + n/8.
    Batched: trees that share a pass share its two CSR passes, so a launch of
    K trees in passes of P trees moves ceil(K / P) CSR terms plus K per-tree
    terms."""
    csr = 2 * (4 * (n + 1) + 5 * nnz)
    per_tree = 16 * n + n // 8
    passes = -(-trees // max(trees_per_pass, 1))
    return {"csr_bytes_per_pass": csr, "bytes_per_tree": per_tree, "passes": passes,
            "trees_per_pass": trees_per_pass,
            "bytes_per_launch": passes * csr + trees * per_tree,
            "unbatched_bytes_per_launch": trees * (csr + per_tree)}


TREES_PER_PASS = {1: 1, 2: 1, 3: 1, 4: 64, 5: 128}


def _code_only(text: str) -> str:
    """C++ source without comments and blank space (string literals in these
    files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_sha(sources=None) -> str:
    """Hash of the sweep kernels' code (comments and spacing ignored)."""
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_grid.hip", "sweep_multi.hip", "fi_multi.h", "fi_prims.h",
              "fi_internal.h"):
        if sources is not None:
            text = sources[f]
        else:
            with open(os.path.join(ROOT, "paper_2311_00869_amd", "csrc", f)) as fh:
                text = fh.read()
        h.update(_code_only(text).encode())
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


def gather_probe(fr, torch, g, reps=5):
    """The neighbour gathers of one dense pull level alone (fi_probe_gather):
    every CSR entry reads 32 bytes of its neighbour's 64-byte record, in CSR
    order; then as many reads of uniform random records.  Median of reps
    launches, timed with events on the launch stream."""
    import numpy as np

    n, nnz = int(g.n), int(g.col.shape[0])
    rec = torch.empty(n * 16, dtype=torch.int32, device="cuda")  # 64 bytes per vertex
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    uni = torch.randint(0, n, (nnz,), dtype=torch.int32, device="cuda", generator=gen)
    s = torch.cuda.current_stream()
    out = {"records": n, "record_bytes": 64, "bytes_per_gather": 32, "gathers": nnz}
    for name, idx in (("csr_order", col), ("uniform", uni)):
        fr.probe_gather(idx, rec, sink, stream=s)
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fr.probe_gather(idx, rec, sink, stream=s)
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[reps // 2]
        out[name] = {"ms": round(ms, 3), "G_gathers_per_s": round(nnz / ms / 1e6, 2)}
    del rec, sink, col, uni
    return out


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
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle worker processes for the all-cores CPU figures "
                         "(0 = min(16, os.cpu_count()))")
    ap.add_argument("--cpu-runs", type=int, default=3, help="runs per CPU figure (median)")
    ap.add_argument("--cpu-batch-runs", type=int, default=1,
                    help="runs of the 256-graph CPU figure of the uneven batch")
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
    ap.add_argument("--phases", action="store_true",
                    help="after the timed steps, one more sweep with the multi-tree kernel's phase "
                         "log on; prints microseconds per pass by phase and BFS level")
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
        print("bench.py measures one GPU: sharding the trees of a sweep across GPUs is a "
              "design (the multi-GPU notes), not a measured path; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_00869_amd import frustration as fr
    from paper_2311_00869_amd import synth
    from paper_2311_00869_amd import tune

    # the oracle's worker processes are spawned before anything touches the GPU
    pool = None
    workers = args.cpu_workers or min(16, os.cpu_count() or 1)
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(workers)

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
    for _ in range(args.steps):
        best = step(0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, launches = G.prof_read(0)
    G.prof_enable(False)
    trees_per_s = T * args.steps / elapsed
    states = G.cloud_size()
    print(f"# {args.steps} steps x {T} trees in {elapsed:.3f}s; min switches {best}, "
          f"{states} states in the last cloud", file=sys.stderr, flush=True)

    phases = None
    if args.phases:
        phases = phase_table(G, T, torch)
    path_used = G.get_schedule()["path"]
    if path_used == 0:
        path_used = 5 if G.n + G.m // 2 > 135000 else 2
    mb = model_bytes(G.n, G.nnz, T, TREES_PER_PASS.get(path_used, 1))
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    achieved = mb["bytes_per_launch"] / avg_launch_s / 1e9
    traffic = load_traffic(args.workload)
    roofline = {
        "kernel": {3: "k_sweep_grid", 4: "k_sweep_multi", 5: "k_sweep_multi"}.get(path_used,
                                                                                 "k_sweep_wg"),
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None if traffic is None else traffic["bytes_per_launch"],
        "traffic_raw": None if traffic is None else traffic.get("raw_bytes_per_launch"),
        "traffic_GBps": None if traffic is None else round(
            traffic["bytes_per_launch"] / avg_launch_s / 1e9, 1),
        "traffic_raw_GBps": None if traffic is None or "raw_bytes_per_launch" not in traffic
        else round(traffic["raw_bytes_per_launch"] / avg_launch_s / 1e9, 1),
        "algorithmic_bytes_per_launch": mb["bytes_per_launch"],
        "model": mb,
        "model_unbatched_GBps": round(mb["unbatched_bytes_per_launch"] / avg_launch_s / 1e9, 1),
        "avg_launch_ms": round(avg_launch_s * 1e3, 3), "launches": launches,
    }

    if path_used in (4, 5):
        roofline["gather_probe"] = gather_probe(fr, torch, g)

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

    if not args.no_cpu_baseline:
        extra["small"] = bench_small(fr, synth, tune, torch)

    cpu = None
    if pool is not None:
        try:
            cpu = cpu_baseline(pool, workers, g, wname, args.cpu_runs, args.cpu_batch_runs)
        finally:
            pool.close()
            pool.join()

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
        "config": {"workload": wname, "trees_per_step": T, "seed": 0,
                   "schedule": sched_used},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "min_switches_last_step": best[0] if best else None,
        "distinct_states_last_step": states,
    }
    if phases is not None:
        out["phases_us_per_pass"] = phases
    out.update(extra)
    G.close()
    print(json.dumps(out), flush=True)


def phase_table(G, T, torch):
    """One sweep of T trees with the phase log on: microseconds per pass of
    each (phase, level), averaged over the launch's passes."""
    G.phase_log(1 << 14)
    G.cloud_reset()
    G.sweep(T, 0)
    G.min_frustration()
    torch.cuda.synchronize()
    recs = G.phase_records()
    G.phase_log(0)
    G.cloud_reset()
    passes = sum(1 for ph, _, _ in recs if ph == 8) or 1
    tot = {}
    for ph, lv, us in recs:
        key = f"{G.PHASES[ph]}" + (f" L{lv}" if ph in (4, 5, 6) else "")
        tot[key] = tot.get(key, 0.0) + us
    table = {k: round(v / passes, 1) for k, v in tot.items()}
    print(f"# phases over {passes} passes (us per pass): " +
          ", ".join(f"{k} {v}" for k, v in table.items()), file=sys.stderr, flush=True)
    return table


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
    for _ in range(steps):
        C.reset()
        G.sweep_bounded(C, 0, T, 0, chunk=chunk)
        best = C.min_frustration()
    el = time.perf_counter() - t0
    held = C.size()
    C.reset()
    G.cloud_reset()
    ev = []
    for a in range(0, T, chunk):
        b = min(T, a + chunk)
        G.sweep_range(a, b, 0)
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
    # rounding and the exact count of all restarts: one read of Gamma, one
    # pass over the edge list (median of 10, events on the launch stream)
    rc_ms = []
    for _ in range(10):
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record()
        G.round_count(out)
        r1.record()
        torch.cuda.synchronize()
        rc_ms.append(r0.elapsed_time(r1))
    rc_ms = sorted(rc_ms)[len(rc_ms) // 2]
    # Gamma read once (4 n R bytes), the edge list once (8 m), one state word
    # per vertex (4 bytes for up to 32 restarts, else 8) written and gathered
    # twice per edge
    word = 4 if R <= 32 else 8
    rc_bytes = 4 * G.n * R + 8 * G.m + word * G.n + 2 * word * G.m
    # per step: row offsets and adjacency once, R floats gathered per CSR
    # entry, each vertex's R floats read and written
    nbytes = 4 * (G.n + 1) + 4 * G.nnz + 4 * G.nnz * R + 8 * G.n * R
    res = {
        "workload": f"the main graph, {R} restarts x {steps} steps, alpha={alpha}",
        "steps_per_s": round(steps / el, 2), "restart_steps_per_s": round(steps * R / el, 1),
        "step_ms": round(step_ms, 3), "algorithmic_bytes_per_step": nbytes,
        "GB_per_s": round(nbytes / step_ms / 1e6, 1),
        "best_rounded_frustration": int(counts.min()), "max_log2_scale": int(scales().max()),
        "round_count_ms": round(rc_ms, 3),
        "round_count_GB_per_s": round(rc_bytes / rc_ms / 1e6, 1),
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
    """HBM bytes per launch of the sweep kernel from two rocprofv3 counter
    collections.  FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are sums of
    the L2's memory requests by size (32-, 64- and 128-byte reads, 64-byte
    and other writes); `raw` is what they read.  Each is also scaled by what
    the same counter reads for the copy probe (copy_probe_mib MiB read and as
    many written by one elementwise kernel), which gives the calibrated
    `bytes_per_launch`."""
    out = {"workload": args.workload, "kernel_sha": kernel_source_sha(),
           "copy_probe_mib": args.copy_probe_mib}
    total = raw = 0.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = _counter_per_dispatch(path, name)
        copies = [v for k, v in per.values() if "elementwise" in k.lower()]
        sweeps = [v for k, v in per.values() if "k_sweep_" in k]
        if not copies or not sweeps:
            raise SystemExit(f"{path}: no copy probe or no sweep dispatch for {name}")
        probe_kib = max(copies)
        scale = (args.copy_probe_mib << 20) / probe_kib  # bytes per counted KiB
        kib = sum(sweeps) / len(sweeps)
        out[name] = {"probe_kib": probe_kib, "bytes_per_counted_kib": scale,
                     "sweep_dispatches": len(sweeps), "kib_per_launch": kib,
                     "raw_bytes_per_launch": kib * 1024, "bytes_per_launch": kib * scale}
        total += kib * scale
        raw += kib * 1024
    out["bytes_per_launch"] = total
    out["raw_bytes_per_launch"] = raw
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
    sched, _ = tune.autotune_batch(B, trees=trees, save=False)
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


def bench_small(fr, synth, tune, torch, trees=1000, reps=20):
    """The 1,000-vertex graph, K = 1,000 trees, seed 0: one launch for all
    trees on the automatic schedule (one tree per workgroup, persistent
    workgroups) against the plain per-tree path (one launch per tree)."""
    g = synth.config_small(0)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=trees)
    G.set_schedule(**tune.default_schedule(G.n, G.nnz))
    G.sweep(trees, 1)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        G.cloud_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.sweep(trees, 0)
        best = G.min_frustration()
        times.append(time.perf_counter() - t0)
    G.cloud_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(trees):
        G.sweep_range(t, t + 1, 0)
    plain_best = G.min_frustration()
    plain = time.perf_counter() - t0
    assert plain_best == best
    out = {"workload": "path+uniform n=1,000 m=5,000 p+=0.8, K=1,000 trees, seed 0",
           "trees_per_s": round(trees / sorted(times)[len(times) // 2], 1),
           "plain_per_tree_trees_per_s": round(trees / plain, 1),
           "schedule": G.get_schedule(), "min_switches": best[0], "distinct_states": G.cloud_size()}
    G.close()
    return out


# ---------------------------------------------------------------- CPU oracle
# The oracle as it stands (single-threaded per call), timed on this host's
# cores: one process per tree for the all-cores figures.  Graphs reach the
# worker processes as .npy files in shared memory, mapped read-only.

_WGRAPHS = {}


def _w_graph(spec):
    g = _WGRAPHS.get(spec)
    if g is None:
        import numpy as np
        from paper_2311_00869_amd import synth
        prefix, n = spec
        g = synth.SignedCSR(n=n, row_ptr=np.load(prefix + "_rp.npy", mmap_mode="r"),
                            col=np.load(prefix + "_col.npy", mmap_mode="r"),
                            sign=np.load(prefix + "_sign.npy", mmap_mode="r"))
        _WGRAPHS.clear()
        _WGRAPHS[spec] = g
    return g


def _w_touch(spec):
    _w_graph(spec)
    return 0


def _w_sweep(job):
    spec, seed, t0, t1 = job
    import oracle
    g = _w_graph(spec)
    t = time.perf_counter()
    oracle.sweep(g, seed, t0, t1, checks=False)
    return time.perf_counter() - t


def _w_batch_graph(job):
    """Make graph gi of the uneven batch and save it for the timed runs."""
    from paper_2311_00869_amd import synth
    gi, d = job
    g = synth.config_batch(4096, 0, indices=[gi])[0]
    return _shm_write(g, os.path.join(d, f"b{gi}")), g.nnz // 2


def _shm_write(g, prefix):
    import numpy as np
    np.save(prefix + "_rp.npy", np.ascontiguousarray(g.row_ptr))
    np.save(prefix + "_col.npy", np.ascontiguousarray(g.col))
    np.save(prefix + "_sign.npy", np.ascontiguousarray(g.sign))
    return (prefix, int(g.n))


def cpu_baseline(pool, workers, g, wname, runs=3, batch_runs=1):
    """CPU oracle figures, each the median of `runs` runs:
    - the main graph: one tree per run in this process (single thread), and
      `workers` trees per run in as many processes (all cores);
    - the 1,000-vertex graph: all 1,000 trees, single thread;
    - the planted 1M-vertex graph: trees 0..31 on all cores, extrapolated
      linearly to 10^4 trees;
    - the uneven batch: 256 of its 4,096 graphs (every 16th) x 64 trees on all
      cores, scaled to the whole batch by edge count;
    - graphL on the 1,000-vertex graph: 32 restarts x 500 float64 steps,
      rounding and the exact count, single thread."""
    import shutil
    import statistics
    import tempfile

    import numpy as np
    import oracle
    from oracle import graphl as ogl
    from paper_2311_00869_amd import synth

    med = statistics.median
    d = tempfile.mkdtemp(prefix="fi_oracle_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    out = {}
    try:
        spec = _shm_write(g, os.path.join(d, "main"))
        single = []
        for r in range(runs):
            t0 = time.perf_counter()
            oracle.sweep(g, 0, r, r + 1, checks=False)
            single.append(time.perf_counter() - t0)
        pool.map(_w_touch, [spec] * (2 * workers), chunksize=1)  # map the graph
        allc = []
        for r in range(runs):
            jobs = [(spec, 0, workers * r + i, workers * r + i + 1) for i in range(workers)]
            t0 = time.perf_counter()
            pool.map(_w_sweep, jobs, chunksize=1)
            allc.append(time.perf_counter() - t0)
        st, ac = med(single), med(allc)
        out = {"value": round(workers / ac, 5), "unit": "trees/s", "cores": workers,
               "kind": "oracle",
               "sample": f"{wname}: {workers} trees (one process per tree) per run, seed 0, "
                         f"median of {runs} runs ({ac:.1f}s); single thread: one tree per run, "
                         f"median of {runs} ({st:.1f}s per tree)",
               "cpu_count": os.cpu_count(),
               "single_thread": {"value": round(1.0 / st, 5), "unit": "trees/s", "cores": 1},
               "runs": runs, "configs": {}}
        cfg = out["configs"]
        # the 1,000-vertex graph, all 1,000 trees
        small = synth.config_small(0)
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.sweep(small, 0, 0, 1000, checks=False)
            ts.append(time.perf_counter() - t0)
        cfg["small_1000_trees"] = {"seconds": round(med(ts), 3),
                                   "trees_per_s": round(1000 / med(ts), 1), "cores": 1}
        # planted: trees 0..31, all cores
        pspec = _shm_write(synth.config_planted_powerlaw(0), os.path.join(d, "planted"))
        pool.map(_w_touch, [pspec] * (2 * workers), chunksize=1)
        tp = []
        for _ in range(runs):
            t0 = time.perf_counter()
            pool.map(_w_sweep, [(pspec, 0, t, t + 1) for t in range(32)], chunksize=1)
            tp.append(time.perf_counter() - t0)
        cfg["planted_trees_0_31"] = {
            "seconds": round(med(tp), 3), "trees_per_s": round(32 / med(tp), 3), "cores": workers,
            "extrapolated_seconds_10000_trees": round(med(tp) * 10000 / 32, 1)}
        # the uneven batch: 256 sampled graphs x 64 trees
        made = pool.map(_w_batch_graph, [(gi, d) for gi in range(0, 4096, 16)], chunksize=1)
        specs = [m[0] for m in made]
        edges_sample = sum(m[1] for m in made)
        shapes = synth.config_batch_shapes(4096, 0)
        edges_all = int(shapes[1].sum())
        tb, tsum = [], []
        for _ in range(batch_runs):
            t0 = time.perf_counter()
            per = pool.map(_w_sweep, [(sp, 0, 0, 64) for sp in specs], chunksize=1)
            tb.append(time.perf_counter() - t0)
            tsum.append(sum(per))
        scale = edges_all / edges_sample
        cfg["batch_256_of_4096_graphs_64_trees"] = {
            "seconds": round(med(tb), 3), "cores": workers, "runs": batch_runs,
            "single_thread_seconds": round(med(tsum), 3),
            "extrapolated_seconds_4096_graphs": round(med(tb) * scale, 1),
            "extrapolated_trees_per_s": round(4096 * 64 / (med(tb) * scale), 1),
            "edge_scale": round(scale, 3)}
        # graphL, float64: 32 restarts x 500 steps, then rounding and the count
        gamma0 = synth.graphl_init(small.n, 32, 0)
        tg = []
        for _ in range(runs):
            t0 = time.perf_counter()
            fin = ogl.descent(small, gamma0, 500, 0.001)
            ogl.frustration(small, ogl.round_states(fin))
            tg.append(time.perf_counter() - t0)
        cfg["graphl_small_32x500_float64"] = {
            "seconds": round(med(tg), 3), "steps_per_s": round(500 / med(tg), 1),
            "restart_steps_per_s": round(500 * 32 / med(tg), 1), "cores": 1}
    finally:
        shutil.rmtree(d, ignore_errors=True)
    return out


if __name__ == "__main__":
    main()

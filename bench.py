"""Benchmark of the BigGraphVis hot path on one MI355X.

One step = the whole path over one synthetic graph already resident in HBM:
streaming community passes -> count-min-sketch supergraph -> Barnes-Hut ForceAtlas2
layout of the supergraph.  Default workload: the largest single graph, an LFR-style
power-law graph with 3.2M nodes and 34M edges (degree exponent 2.1, community sizes
exponent 1.5, mixing 0.3), threshold 128, 3 passes, 2^22-edge chunks, sketch
5 x 2^22, 1,000 Barnes-Hut iterations at theta 1.2 (the analogue of the paper's
largest Table 1 row).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lfr_3m] [--no-cpu]

Prints one JSON line.  `value` is edges/s through the community passes + sketch
supergraph; FA2 iterations/s and the whole-step rate are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
PROFILE_SAMPLE = 1             # timed steps time one in this many dominant-kernel launches
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lfr_3m")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-fa2-iters", type=int, default=10,
                    help="Barnes-Hut layout iterations the CPU oracle runs for its FA2 rate (a sample: the "
                         "workload has 1,000)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the whole-graph, sequential-rule, atomics, sweep, small-graph, batched, gradient and lfr_1m "
                         "comparisons")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="do not time launches with HIP events (for hardware-counter runs)")
    ap.add_argument("--fa2-iters", type=int, default=None, metavar="N",
                    help="lay the supergraph out for N iterations instead of the workload's (hardware-counter runs "
                         "only: the per-launch counters need a few iterations; the line then names N)")
    ap.add_argument("--profile-sample", type=int, default=PROFILE_SAMPLE, metavar="N",
                    help="time one in N launches of the dominant kernel in the timed steps")
    ap.add_argument("--form", default=None, choices=sorted(FORMS),
                    help="run only this comparison and print its JSON (for profiling runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times), to scale HBM counters")
    return ap.parse_args()


def calibrate_copy(mib: int) -> None:
    """A plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE of one dispatch should
    read mib MiB each; the ratio scales the counters read for the path's kernels."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_mib": mib, "bytes_per_copy": n * 4}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import graphgen
    import paper_2108_00529_amd as bgv
    from paper_2108_00529_amd import profile as prof

    if args.form:
        print(json.dumps({"form": args.form, **FORMS[args.form](torch, bgv, graphgen)}))
        return

    wl = dict(graphgen.WORKLOADS[args.workload], name=args.workload)
    if args.fa2_iters is not None:
        wl["fa2_iters"] = args.fa2_iters
    n = wl["n"]
    t0 = time.time()
    edges_np, _ = graphgen.make_graph(args.workload)
    m = edges_np.shape[0]
    print(f"[bench] generated {args.workload}: n={n} m={m} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    pos0_np = graphgen.initial_positions(n, wl["pos_seed"])
    dev = torch.device("cuda:0")
    edges = torch.from_numpy(edges_np).to(dev)
    pos0 = torch.from_numpy(pos0_np).to(dev)
    stream = torch.cuda.current_stream()

    # workspaces sized once, outside the timed region
    ws_cd = bgv.api.community_workspace(edges, n, wl)
    ws_sg = bgv.api.supergraph_workspace(edges, n, wl)

    ev = {k: torch.cuda.Event(enable_timing=True) for k in ("a", "b", "c")}

    def step(record=False):
        if record:
            ev["a"].record(stream)
        labels, degree, _ = bgv.community(edges, n, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"],
                                          ws=ws_cd, check=False)
        sg = bgv.supergraph(edges, labels, degree, wl["rows"], wl["cols"], c1, c2, ws=ws_sg, check=False)
        if record:
            ev["b"].record(stream)
        pos = pos0[: sg["K"]].clone()
        bgv.fa2_layout(sg["superedges"], pos, wl["fa2_iters"], exact=wl["exact"], theta=wl["theta"], kr=wl["kr"],
                       kg=wl["kg"], tau=wl["tau"], ks=wl["ks"], ksmax=wl["ksmax"])
        if record:
            ev["c"].record(stream)
        return sg

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # one untimed step with every kernel launch timed by events: the per-kernel breakdown,
    # and which kernel dominates the device time
    kbreak = {}
    dominant = None
    if not args.no_kernel_timing:
        prof.reset()
        prof.only(None)
        prof.enable(True)
        step()
        torch.cuda.synchronize()
        prof.enable(False)
        kbreak = prof.stats()
        dominant = max(kbreak.items(), key=lambda kv: kv[1]["total_ms"])[0] if kbreak else None
        print(f"[bench] breakdown step done; dominant kernel {dominant}", file=sys.stderr, flush=True)

    # timed steps: start/stop events on the launches of the dominant kernel only (one in
    # --profile-sample of them), so the rest runs without events
    prof.reset()
    prof.only(dominant)
    prof.sample(args.profile_sample)
    prof.enable(dominant is not None)
    cd_ms, fa_ms = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        sg = step(record=True)
        ev["c"].synchronize()
        cd_ms.append(ev["a"].elapsed_time(ev["b"]))
        fa_ms.append(ev["b"].elapsed_time(ev["c"]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof.enable(False)
    prof.only(None)
    prof.sample(1)
    kstats = prof.stats()
    inter = prof.counter("bh_interactions")
    redo = prof.counter("bh_redo_blocks")
    # the counter covers every force launch of the timed steps, timed or not
    inter_per_launch = inter / (args.steps * wl["fa2_iters"]) if inter and not wl["exact"] else None
    for k in kstats:
        if k.startswith("bh_force") and inter_per_launch:
            kstats[k]["bh_interactions_per_launch"] = inter_per_launch
    print(f"[bench] timed {args.steps} steps in {t_total:.2f}s", file=sys.stderr, flush=True)
    # one more step with no kernel events at all: the layout rate without measurement
    step(record=True)
    ev["c"].synchronize()
    fa_unprofiled = ev["b"].elapsed_time(ev["c"])

    ms_per_step = 1000.0 * t_total / args.steps
    cd = float(np.mean(cd_ms))
    fa = float(np.mean(fa_ms))
    K, E = sg["K"], sg["E"]
    value = m / (cd / 1000.0)

    roofline, extra = roofline_report(kstats, kbreak, wl, n, m, K, E, inter_per_launch)
    copy_gbs = measured_copy_gbs(torch)
    for row in extra.get("roofline_edge_stream", {}).values():
        row["measured_copy_peak_gbs"] = copy_gbs
        row["frac_of_measured"] = row["achieved"] / copy_gbs

    out = {
        "metric": "edges/s through community pass+sketch; FA2 iters/s; batched/grad vs plain",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: LFR-style n={n} m={m} gamma={wl['gamma']} beta={wl['beta']} "
                               f"mu={wl['mu']}; threshold {wl['threshold']}, {wl['passes']} passes, chunk "
                               f"{wl['chunk']}; sketch {wl['rows']}x{wl['cols']}; Barnes-Hut FA2 theta "
                               f"{wl['theta']}, {wl['fa2_iters']} iterations",
                   "nodes": n, "edges": m, "supernodes": K, "superedges": E},
        "parts": {"community_sketch_ms": cd, "fa2_ms": fa,
                  "fa2_iters_per_s": wl["fa2_iters"] / (fa / 1000.0),
                  "fa2_iters_per_s_without_kernel_events": wl["fa2_iters"] / (fa_unprofiled / 1000.0),
                  "pipeline_edges_per_s": m / ((cd + fa) / 1000.0),
                  # one community pass: device time of the community kernels over the passes
                  "community_pass_edges_per_s": (m * wl["passes"] / (extra["roofline_edge_stream"]["community_passes"]
                                                                     ["device_ms"] / 1000.0)
                                                 if extra.get("roofline_edge_stream", {}).get("community_passes")
                                                 else None),
                  "bh_interactions_per_iteration": inter_per_launch,
                  "bh_force_blocks_redone_per_iteration": (redo / (args.steps * wl["fa2_iters"])
                                                           if redo is not None and not wl["exact"] else None),
                  "bh_interactions_per_s": (inter_per_launch * wl["fa2_iters"] / (fa_unprofiled / 1000.0)
                                            if inter_per_launch else None)},
        "roofline": roofline,
        **extra,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(edges_np, n, wl, c1, c2, pos0_np, args.cpu_fa2_iters)
    if not args.no_forms:
        del edges, pos0
        torch.cuda.empty_cache()
        out["forms"] = {"whole_graph_fa2": whole_graph_form(torch, bgv, edges_np, n, wl, cd + fa_unprofiled),
                        "sequential_rule": sequential_rule_form(torch, bgv, edges_np, n, wl, not args.no_cpu),
                        "atomics": atomic_forms(torch, bgv, edges_np, n, wl),
                        "sweeps": sweeps_form(torch, bgv, graphgen, edges_np, n, wl),
                        "small_graph": small_graph_form(torch, bgv, graphgen),
                        "batched": batched_form(torch, bgv, graphgen),
                        "gradient": gradient_form(torch, bgv, graphgen),
                        "lfr_1m": lfr_1m_form(torch, bgv, graphgen)}
    print(json.dumps(out))


def _timed(torch, fn, repeats=1):
    """Best device time (ms) of fn() over `repeats` runs, HIP events on the current stream."""
    best = float("inf")
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def batched_form(torch, bgv, graphgen):
    """512 uneven planted graphs: one batched launch (eager and replayed from a captured
    graph) against 512 sequential plain pipelines, same outputs."""
    from paper_2108_00529_amd import autotune
    wl = graphgen.WORKLOADS["batched_512"]
    t0 = time.time()
    graphs = graphgen.batched_planted(wl["G"], wl["graph_seed"])
    G = len(graphs)
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    pos0 = [graphgen.initial_positions(n, wl["pos_seed"] + g) for g, (n, _, _) in enumerate(graphs)]
    dev = torch.device("cuda:0")
    edges, noff, eoff, noff_h, eoff_h = bgv.pack_graphs([(n, e) for n, e, _ in graphs], dev)
    n_total, m_total = int(noff_h[-1]), int(eoff_h[-1])
    print(f"[bench] batched: {G} graphs, {n_total} nodes, {m_total} edges generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    order = torch.from_numpy(np.argsort(-np.diff(eoff_h), kind="stable").astype(np.int32)).to(dev)
    pos_init = torch.from_numpy(np.concatenate(pos0)).to(dev)
    (wg, big_k), tune = autotune.tune_batched(edges, noff, eoff, n_total, wl, c1, c2, pos_init, order=order,
                                              repeats=1, use_cache=False)
    ws = bgv.batched_workspace(G, n_total, m_total, dev)
    pos = pos_init.clone()
    fprev = torch.zeros_like(pos)
    speed = torch.ones(G, dtype=torch.float32, device=dev)

    def run_batched():
        pos.copy_(pos_init)
        fprev.zero_()
        speed.fill_(1.0)
        return bgv.batched(edges, noff, eoff, n_total, wl, c1, c2, pos, order=order, fprev=fprev, speed=speed,
                           wg_threads=wg, big_k=big_k, ws=ws)

    run_batched()
    eager_ms = _timed(torch, run_batched, repeats=3)
    # capture the whole batched launch once, replay it
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run_batched()
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(graph):
        res = run_batched()
    graph.replay()
    torch.cuda.synchronize()
    graph_ms = _timed(torch, graph.replay, repeats=3)
    K_b = res["K"].cpu().numpy()
    # the same graphs one by one through the plain entry points
    pos0_d = [torch.from_numpy(p).to(dev) for p in pos0]
    edges_g = [torch.from_numpy(e).to(dev) for _, e, _ in graphs]
    torch.cuda.synchronize()
    t = time.perf_counter()
    K_p = []
    for g, (n, _, _) in enumerate(graphs):
        o = bgv.pipeline(edges_g[g], n, wl, c1, c2, pos0_d[g], check=False)
        K_p.append(o["sg"]["K"])
    torch.cuda.synchronize()
    seq_ms = 1000.0 * (time.perf_counter() - t)
    return {"graphs": G, "nodes": n_total, "edges": m_total, "wg_threads": wg, "big_k": big_k, "autotune_ms": tune["ms"],
            "batched_ms": eager_ms, "batched_graph_replay_ms": graph_ms, "sequential_plain_ms": seq_ms,
            "speedup_vs_sequential": seq_ms / min(eager_ms, graph_ms),
            "graphs_per_s": G / (min(eager_ms, graph_ms) / 1000.0),
            "supernodes_equal": bool(np.array_equal(K_b, np.array(K_p)))}


def small_graph_form(torch, bgv, graphgen, repeats=5):
    """The planted_2k workload (2,000 nodes, ~11k edges, 1 pass with 256-edge chunks,
    200 exact layout iterations) end to end: through the plain entry points (a launch or
    more per chunk and per iteration) and as a one-graph batch (the whole path in one
    persistent launch).  Median wall time of `repeats` runs each, same outputs."""
    wl = graphgen.WORKLOADS["planted_2k"]
    e, _ = graphgen.make_graph("planted_2k")
    n = wl["n"]
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    dev = torch.device("cuda:0")
    ed = torch.from_numpy(e).to(dev)
    pos0 = torch.from_numpy(graphgen.initial_positions(n, wl["pos_seed"])).to(dev)
    edges_b, noff, eoff, noff_h, _ = bgv.pack_graphs([(n, e)], dev)

    def plain():
        return bgv.pipeline(ed, n, wl, c1, c2, pos0, check=False)

    def batched():
        return bgv.batched(edges_b, noff, eoff, n, wl, c1, c2, pos0.clone(), wg_threads=1024)

    def wall(fn):
        ts = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(1000.0 * (time.perf_counter() - t))
        return float(np.median(ts)), out

    plain()
    batched()
    plain_ms, po = wall(plain)
    batch_ms, bo = wall(batched)
    K = po["sg"]["K"]
    same = bool(int(bo["K"][0]) == K and torch.equal(bo["pos"][:K], po["pos"]))
    return {"nodes": n, "edges": int(e.shape[0]), "supernodes": K, "fa2_iterations": wl["fa2_iters"],
            "plain_ms": plain_ms, "one_graph_batch_ms": batch_ms, "speedup": plain_ms / batch_ms,
            "fa2_iters_per_s_in_batch": wl["fa2_iters"] / (batch_ms / 1000.0), "same_positions": same}


def lfr_1m_form(torch, bgv, graphgen, repeats=3):
    """The 1M-node / 10M-edge LFR-style workload (3 passes with 2^20-edge chunks,
    sketch 4 x 2^20, 500 Barnes-Hut iterations): community passes + sketch supergraph
    edges/s and layout iterations/s, best of `repeats` steps after a warm-up one."""
    wl = graphgen.WORKLOADS["lfr_1m"]
    t0 = time.time()
    e, _ = graphgen.make_graph("lfr_1m")
    print(f"[bench] lfr_1m: generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    n, m = wl["n"], e.shape[0]
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    dev = torch.device("cuda:0")
    ed = torch.from_numpy(e).to(dev)
    pos_d = torch.from_numpy(graphgen.initial_positions(n, wl["pos_seed"])).to(dev)
    ws_cd = bgv.api.community_workspace(ed, n, wl)
    ws_sg = bgv.api.supergraph_workspace(ed, n, wl)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    best_cd, best_fa, sg = float("inf"), float("inf"), None
    for r in range(repeats + 1):
        ev[0].record()
        labels, degree, _ = bgv.community(ed, n, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"], ws=ws_cd,
                                          check=False)
        sg = bgv.supergraph(ed, labels, degree, wl["rows"], wl["cols"], c1, c2, ws=ws_sg, check=False)
        ev[1].record()
        pos = pos_d[: sg["K"]].clone()
        bgv.fa2_layout(sg["superedges"], pos, wl["fa2_iters"], exact=False, theta=wl["theta"], kr=wl["kr"],
                       kg=wl["kg"], tau=wl["tau"], ks=wl["ks"], ksmax=wl["ksmax"])
        ev[2].record()
        ev[2].synchronize()
        if r > 0:
            best_cd = min(best_cd, ev[0].elapsed_time(ev[1]))
            best_fa = min(best_fa, ev[1].elapsed_time(ev[2]))
    del ed, pos_d, ws_cd, ws_sg
    torch.cuda.empty_cache()
    return {"nodes": n, "edges": m, "supernodes": sg["K"], "superedges": sg["E"],
            "community_sketch_ms": best_cd, "community_sketch_edges_per_s": m / (best_cd / 1000.0),
            "fa2_iterations": wl["fa2_iters"], "fa2_ms": best_fa,
            "fa2_iters_per_s": wl["fa2_iters"] / (best_fa / 1000.0)}


def whole_graph_form(torch, bgv, edges_np, n, wl, bgv_ms):
    """The paper's comparison: ForceAtlas2 (Barnes-Hut, same parameters and iteration
    count) on the whole original graph against the BigGraphVis step measured above
    (community passes + supergraph + layout of the supergraph)."""
    dev = torch.device("cuda:0")
    e = edges_np[edges_np[:, 0] != edges_np[:, 1]]  # the layout takes no self-loops
    ed = torch.from_numpy(np.ascontiguousarray(e)).to(dev)
    pos0 = torch.from_numpy(graphgen_initial(n, wl)).to(dev)
    kw = dict(exact=False, theta=wl["theta"], kr=wl["kr"], kg=wl["kg"], tau=wl["tau"], ks=wl["ks"], ksmax=wl["ksmax"])
    bgv.fa2_layout(ed, pos0.clone(), 5, **kw)  # warm-up (workspace, code paths)
    torch.cuda.synchronize()
    pos = pos0.clone()
    ms = _timed(torch, lambda: bgv.fa2_layout(ed, pos, wl["fa2_iters"], **kw))
    del ed, pos, pos0
    torch.cuda.empty_cache()
    return {"nodes": n, "edges": int(e.shape[0]), "fa2_iterations": wl["fa2_iters"], "fa2_ms": ms,
            "fa2_iters_per_s": wl["fa2_iters"] / (ms / 1000.0), "biggraphvis_ms": bgv_ms,
            "time_reduction_pct": 100.0 * (1.0 - bgv_ms / ms)}


def sequential_rule_form(torch, bgv, edges_np, n, wl, with_cpu):
    """The community passes with chunk = 1 (the sequential rule, one chunk per edge) on
    the same stream: back-pointer resolution (the automatic choice there), against the
    oracle's sequential loop on one host thread as its CPU baseline."""
    dev = torch.device("cuda:0")
    ed = torch.from_numpy(np.ascontiguousarray(edges_np)).to(dev)
    run = lambda: bgv.community(ed, n, wl["threshold"], wl["passes"], wl["growth"], 1, check=False)
    run()
    torch.cuda.synchronize()
    ms = _timed(torch, run, repeats=3)
    del ed
    torch.cuda.empty_cache()
    m = int(edges_np.shape[0])
    out = {"chunk": 1, "passes": wl["passes"], "edges": m, "gpu_ms": ms,
           "edges_per_s": m / (ms / 1000.0), "chunk_steps_avoided": wl["passes"] * m}
    if with_cpu:
        import oracle
        t = time.perf_counter()
        oracle.bs_community(n, edges_np, wl["threshold"], wl["passes"], wl["growth"], 1)
        cpu_ms = (time.perf_counter() - t) * 1000.0
        out.update(cpu_oracle_ms=cpu_ms, cpu_threads=1, speedup_vs_oracle=cpu_ms / ms)
    return out


def sweep_points(wl):
    """The paper's sensitivity study on this workload: hash functions (sketch rows) 1-4,
    rounds (passes) 2-4, threshold delta / 3 delta / 5 delta and sketch widths 5,000 and
    15,000 beside the workload's own, one parameter changed at a time; then the rule
    variants: equal counters join (tie 1) and SCoDA's community-volume rule (rule 1)."""
    d = wl["threshold"]
    return ([("rows", r) for r in (1, 2, 3, 4)] + [("passes", p) for p in (2, 3, 4)] +
            [("threshold", k * d) for k in (1, 3, 5)] + [("cols", c) for c in (5000, 15000, wl["cols"])] +
            [("tie", 1), ("rule", 1)])


def sweeps_form(torch, bgv, graphgen, edges_np, n, wl):
    """Time (community passes + supergraph + Barnes-Hut layout of the supergraph),
    supernodes and superedges at each sweep point: the columns of the paper's
    hash-function and rounds tables."""
    dev = torch.device("cuda:0")
    ed = torch.from_numpy(np.ascontiguousarray(edges_np)).to(dev)
    pos0 = torch.from_numpy(graphgen_initial(n, wl)).to(dev)
    rows = []
    for key, value in sweep_points(wl):
        w = dict(wl)
        w[key] = value
        c1 = graphgen.hash_coeffs(w["rows"], w["sketch_seed"])
        c2 = graphgen.hash_coeffs(w["rows"], w["sketch_seed"] ^ 0x9E3779B97F4A7C15)
        bgv.pipeline(ed, n, w, c1, c2, pos0, check=False)  # warm-up (workspaces, code paths)
        torch.cuda.synchronize()
        res = {}
        ms = _timed(torch, lambda: res.update(bgv.pipeline(ed, n, w, c1, c2, pos0, check=False)))
        row = {"param": key, "value": value, "ms": ms, "supernodes": int(res["sg"]["K"]),
               "superedges": int(res["sg"]["E"])}
        # what the sketch parameters change: the estimates' relative overestimate of the
        # exact supernode sizes (community volumes) and superedge multiplicities (untimed)
        lab, deg, vol = bgv.community(ed, n, w["threshold"], w["passes"], w["growth"], w["chunk"], volume=True,
                                      tie=w.get("tie", 0), rule=w.get("rule", 0))
        sg = bgv.supergraph(ed, lab, deg, w["rows"], w["cols"], c1, c2, exact_counts=True)
        size = sg["super_size"].to(torch.int64) & 0xFFFFFFFF
        exact = vol[sg["super_label"].to(torch.int64)]
        se_w = sg["se_weight"].to(torch.int64) & 0xFFFFFFFF
        se_c = sg["se_count"].to(torch.int64) & 0xFFFFFFFF
        rs = (size - exact).double() / exact.clamp(min=1).double()
        rw = (se_w - se_c).double() / se_c.clamp(min=1).double()
        row.update(size_overestimate_mean=float(rs.mean()), size_overestimate_max=float(rs.max()),
                   weight_overestimate_mean=float(rw.mean()) if rw.numel() else 0.0,
                   weight_overestimate_max=float(rw.max()) if rw.numel() else 0.0)
        rows.append(row)
    del ed, pos0
    torch.cuda.empty_cache()
    return rows


def graphgen_initial(n, wl):
    import graphgen
    return graphgen.initial_positions(n, wl["pos_seed"])


def gradient_form(torch, bgv, graphgen, lrs=(3.0, 10.0, 30.0), max_steps=3000):
    """The grad_50k workload: weighted supergraph of 50,000 supernodes (planted
    communities of a 5M-node LFR-style graph; weights from a 5 x 2^22 sketch).  Exact FA2
    with its adaptive speeds for the workload's iterations vs Adam on the FA2 energy
    (autograd function with the hand-written gradient) until it reaches the same energy.
    With lrs empty only the exact layout runs (its pair rate: K^2 pairs per iteration)."""
    wl = graphgen.WORKLOADS["grad_50k"]
    t0 = time.time()
    e, comm = graphgen.make_graph("grad_50k")
    print(f"[bench] gradient form: source graph generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    ed = torch.from_numpy(e).to(dev)
    del e
    lab = torch.from_numpy(comm).to(dev)
    _, degree, _ = bgv.community(ed, wl["n"], 0, 1, 2, 1 << 22)  # threshold 0: degrees only
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    sg = bgv.supergraph(ed, lab, degree, wl["rows"], wl["cols"], c1, c2)
    del ed, lab, degree
    torch.cuda.empty_cache()
    K, E = sg["K"], sg["E"]
    se = sg["superedges"].contiguous()
    w = sg["se_weight"].to(torch.float32).contiguous()
    pos0 = torch.from_numpy(graphgen.initial_positions(K, wl["pos_seed"], wl["pos_lo"], wl["pos_hi"])).to(dev)
    fa2_iters = wl["fa2_iters"]
    p = pos0.clone()
    ms_fa2 = _timed(torch, lambda: bgv.fa2_layout(se, p, fa2_iters, exact=True, attr_w=w))
    print(f"[bench] gradient form: {fa2_iters} exact iterations on K={K} in {ms_fa2:.1f} ms", file=sys.stderr,
          flush=True)
    e_fa2 = float(bgv.fa2_energy(se, p, attr_w=w))
    e_start = float(bgv.fa2_energy(se, pos0, attr_w=w))
    adam = {}
    for lr in lrs:
        x = pos0.clone().requires_grad_(True)
        opt = torch.optim.Adam([x], lr=lr)
        steps, reached, energy = 0, False, e_start
        torch.cuda.synchronize()
        t = time.perf_counter()
        while steps < max_steps:
            opt.zero_grad(set_to_none=True)
            en = bgv.FA2Energy.apply(x, se, 1.0, 1.0, w, None)
            en.backward()
            opt.step()
            steps += 1
            if steps % 25 == 0:
                energy = float(en.detach())
                if energy <= e_fa2:
                    reached = True
                    break
        torch.cuda.synchronize()
        adam[str(lr)] = {"steps": steps, "ms": 1000.0 * (time.perf_counter() - t), "reached_fa2_energy": reached,
                         "energy": energy}
    ok = [v for v in adam.values() if v["reached_fa2_energy"]]
    return {"supernodes": K, "superedges": E, "fa2_iterations": fa2_iters, "fa2_ms": ms_fa2,
            "fa2_pairs_per_s": float(K) * K * fa2_iters / (ms_fa2 / 1000.0),
            "energy_start": e_start, "energy_fa2": e_fa2, "adam": adam,
            "adam_best_ms_to_fa2_energy": min(v["ms"] for v in ok) if ok else None}


def _forms():
    """The comparisons `--form` can run alone."""
    def needs_bench_graph(fn):
        def run(torch, bgv, graphgen, name="lfr_3m"):
            wl = dict(graphgen.WORKLOADS[name], name=name)
            e, _ = graphgen.make_graph(name)
            return fn(torch, bgv, e, wl)
        return run
    return {"gradient": gradient_form,
            "gradient_fa2": lambda torch, bgv, graphgen: gradient_form(torch, bgv, graphgen, lrs=()),
            "batched": batched_form,
            "small_graph": small_graph_form,
            "lfr_1m": lfr_1m_form,
            "whole_graph_fa2": needs_bench_graph(lambda torch, bgv, e, wl: whole_graph_form(torch, bgv, e, wl["n"], wl,
                                                                                             float("nan"))),
            "sequential_rule": needs_bench_graph(lambda torch, bgv, e, wl: sequential_rule_form(torch, bgv, e, wl["n"],
                                                                                                 wl, False)),
            "atomics": needs_bench_graph(lambda torch, bgv, e, wl: atomic_forms(torch, bgv, e, wl["n"], wl))}


FORMS = _forms()


# algorithmic work per unit: bytes (HBM-bound kernels) or flops (ALU-bound)
EDGE_PASS_BYTES = 8            # one int32 (u,v) pair read per edge per pass
BH_INTERACTION_FLOPS = 20      # body-node or body-body interaction, n-body convention
CSR_ENTRY_BYTES = {"attract<uint16_t>": 2, "attract<uint32_t>": 4, "attract<int2>": 8,
                   "attract_lds<uint16_t>": 2, "attract_lds<uint32_t>": 4, "attract_lds<int2>": 8,
                   "attract_cols<uint16_t>": 2, "attract_cols<int2>": 8}


def kernel_model(name, K, E, inter_per_launch=None):
    """(bound, algorithmic work per launch, unit) of a layout kernel on a K-body,
    E-superedge supergraph, or None for kernels without a model."""
    if name.startswith("bh_force") and inter_per_launch:
        return "alu", BH_INTERACTION_FLOPS * inter_per_launch, "flop"
    if name in CSR_ENTRY_BYTES:  # CSR entries + row offsets, own and neighbour positions, result
        return "hbm", CSR_ENTRY_BYTES[name] * 2 * E + 28 * K, "byte"
    per_body = {"os_pass<4>": 16,                  # Morton sort pass: 32-bit code and index read + written
                "os_pass<8>": 16,
                "os_pass<16>": 16,
                "rs_downsweep_small": 16,
                "bh_codes": 20,                     # position read, key and index written
                "bh_codes_os<4>": 20,               # the same, with the sort's digit counts in LDS
                "bh_codes_os<8>": 20,
                "bh_codes_os<16>": 20,
                "bh_gather": 44,                    # key, index, position, mass read; body and code written
                "bh_prefix": 40,                    # body read; three FP64 prefix sums written
                "bh_build": 60,                     # codes and prefix sums read; node written
                "bh_update": 40,                    # position, force, previous force read; two written
                "update": 48}                       # the same plus the block partials (exact path)
    if name in per_body:
        return "hbm", per_body[name] * K, "byte"
    if name == "bh_build_att":  # tree build and attraction in one launch (unweighted CSR ids)
        return "hbm", 60 * K + (2 if K <= 65536 else 4) * 2 * E + 28 * K, "byte"
    return None


def roofline_of(name, avg_s, K, E, inter_per_launch=None):
    mdl = kernel_model(name, K, E, inter_per_launch)
    if mdl is None:
        return dict(bound="unknown", achieved=None, peak=None, unit=None)
    bound, work, unit = mdl
    if bound == "alu":
        r = dict(bound="alu", achieved=work / avg_s / 1e12, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s")
    else:
        r = dict(bound="hbm", achieved=work / avg_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    r["frac"] = r["achieved"] / r["peak"]
    r["work_per_launch"] = work
    return r


def measured_copy_gbs(torch, mib=1024, repeats=5):
    """Device-to-device copy of `mib` MiB, best of `repeats`: bytes read + written per
    second, the attainable stream rate beside the published 8 TB/s."""
    src = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * mib * (1 << 20) / (best / 1000.0) / 1e9


def measured_atomic_rate(torch, n_ops=1 << 26, n_addr=1 << 24, repeats=3):
    """Random device atomics per second: torch's index_add_ on int32 (one atomic add per
    source element) of n_ops ones at uniformly random places of an n_addr-entry array,
    best of `repeats`: the practical rate of scattered device-scope integer atomics,
    beside which the library's atomic forms (the volume rule, the per-node form above
    2^24 nodes) are read."""
    g = torch.Generator(device="cuda").manual_seed(5)
    idx = torch.randint(0, n_addr, (n_ops,), device="cuda", generator=g)
    src = torch.ones(n_ops, dtype=torch.int32, device="cuda")
    x = torch.zeros(n_addr, dtype=torch.int32, device="cuda")
    x.index_add_(0, idx, src)
    best = float("inf")
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        x.index_add_(0, idx, src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    ok = int(x.sum().item()) == (repeats + 1) * n_ops
    del idx, src, x
    return n_ops / (best / 1000.0), ok


def atomic_forms(torch, bgv, edges_np, n, wl):
    """The community passes under SCoDA's volume rule (the library's form built on device
    atomics: two counter increments per non-loop edge and pass, plus the V updates
    combined per wave and label) on the bench graph, against the measured random-atomic
    rate."""
    rate, ok = measured_atomic_rate(torch)
    dev = torch.device("cuda:0")
    ed = torch.from_numpy(np.ascontiguousarray(edges_np)).to(dev)
    run = lambda: bgv.community(ed, n, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"], rule=1, check=False)
    run()
    torch.cuda.synchronize()
    ms = _timed(torch, run, repeats=2)
    loops = int((edges_np[:, 0] == edges_np[:, 1]).sum())
    min_atomics = 2 * (int(edges_np.shape[0]) - loops) * wl["passes"]
    del ed
    torch.cuda.empty_cache()
    return {"measured_random_atomic_adds_per_s": rate, "measured_with": "torch index_add_ int32, 2^26 adds at "
                                                                       "random places of a 2^24-entry array",
            "measured_sum_checked": ok, "volume_rule_community_ms": ms,
            "volume_rule_counter_atomics": min_atomics,
            "volume_rule_counter_atomics_per_s": min_atomics / (ms / 1000.0),
            "volume_rule_frac_of_measured_atomic_rate": min_atomics / (ms / 1000.0) / rate}


def roofline_report(kstats, kbreak, wl, n, m, K, E, inter_per_launch=None):
    """Roofline of the dominant kernel, from the events recorded around it in the timed
    steps (kstats), plus the per-kernel breakdown of one untimed step with every launch timed
    (kbreak) with each layout kernel's roofline and the community passes' edge-stream
    rate."""
    if not kstats:
        return None, {}
    extra = {"kernel_ms_breakdown_step": {k: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / max(v["launches"], 1), 5),
                                              "total_ms": round(v["total_ms"], 4)}
                                          for k, v in sorted(kbreak.items(), key=lambda kv: -kv[1]["total_ms"])}}
    # the community passes as one edge stream: 8 B of edge list per edge and pass over
    # the summed device time of all their kernels
    rows = {}
    cd_ms = sum(st["total_ms"] for name, st in kbreak.items() if name.startswith("cd_"))
    if cd_ms > 0:
        rows["community_passes"] = dict(bound="hbm", achieved=EDGE_PASS_BYTES * m * wl["passes"] / (cd_ms / 1e3) / 1e9,
                                        peak=HBM_PEAK_GBS, unit="GB/s", device_ms=cd_ms)
    extra["roofline_edge_stream"] = {k: dict(v, frac=v["achieved"] / v["peak"]) for k, v in rows.items()}
    inter = inter_per_launch
    layout = {}
    for name, st in kbreak.items():
        if kernel_model(name, K, E, inter) is not None:
            layout[name] = roofline_of(name, st["total_ms"] / 1e3 / max(st["launches"], 1), K, E, inter)
    extra["roofline_layout_kernels_breakdown_step"] = layout
    top, st = max(kstats.items(), key=lambda kv: kv[1]["total_ms"])
    avg_s = st["total_ms"] / 1000.0 / max(st["launches"], 1)
    r = roofline_of(top, avg_s, K, E, st.get("bh_interactions_per_launch"))
    if st.get("bh_interactions_per_launch"):
        r["interactions_per_launch"] = st["bh_interactions_per_launch"]
    r = dict(r, kernel=top, avg_ms=avg_s * 1000.0, launches_sampled=st["launches"],
             traffic=measured_traffic(top, wl["name"]))
    return r, extra


def csrc_digest() -> str:
    """sha256 (16 hex digits) over the library's kernel sources, in name order."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2108_00529_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary of
    the workload (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when it has no entry
    or the kernel sources have changed since the counters were taken."""
    import re
    summary = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    try:
        text = open(summary).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel sources when measured: ([0-9a-f]{16})", text, re.IGNORECASE)
    if not m_hash or m_hash.group(1) != csrc_digest():
        return None
    m_bytes = re.search(r"traffic_bytes_per_launch\[" + re.escape(kernel) + r"\]: (\d+)", text)
    return int(m_bytes.group(1)) if m_bytes else None


def cpu_baseline(edges_np, n, wl, c1, c2, pos0_np, fa2_iters):
    """The oracle, untuned, on this host: community passes + supergraph on the whole
    graph (single thread; `value` in edges/s like the GPU's) and a sample of
    `fa2_iters` Barnes-Hut FA2 iterations on the supergraph (OpenMP over all threads)."""
    import oracle
    t = time.perf_counter()
    lab, cnt = oracle.bs_community(n, edges_np, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"])
    deg, _ = oracle.degree_volume(lab, cnt, wl["passes"])
    sg = oracle.supergraph(n, edges_np, lab, deg, wl["rows"], wl["cols"], c1, c2)
    t_cd = time.perf_counter() - t
    K = sg["K"]
    t = time.perf_counter()
    oracle.fa2_layout(pos0_np[:K], sg["superedges"], iters=fa2_iters, exact=wl["exact"], theta=wl["theta"])
    t_fa = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": edges_np.shape[0] / t_cd, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"community passes + sketch supergraph over all {edges_np.shape[0]} edges "
                      f"({t_cd:.1f}s, 1 thread); FA2: {fa2_iters} of the workload's {wl['fa2_iters']} "
                      f"Barnes-Hut iterations on the {K}-node supergraph in {t_fa:.1f}s with {threads} "
                      f"OpenMP threads (not scaled up)",
            "fa2_iters_per_s": fa2_iters / t_fa, "fa2_threads": threads,
            "host_cpu": host_cpu_model(), "host_threads": os.cpu_count()}


def host_cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()

"""Benchmark of the BigGraphVis hot path on one MI355X.

One step = the whole path over one synthetic graph already resident in HBM:
streaming community passes -> count-min-sketch supergraph -> Barnes-Hut ForceAtlas2
layout of the supergraph.  Default workload: the LFR-style power-law graph with 1M
nodes and 10M edges (degree exponent 2.3, community sizes exponent 1.5, mixing 0.2),
threshold 64, 3 passes, 2^20-edge chunks, sketch 4 x 2^20, 500 iterations at theta 1.2.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lfr_1m] [--no-cpu]

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
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lfr_1m")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-fa2-iters", type=int, default=20)
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="do not bracket launches with HIP events (for hardware-counter runs)")
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
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import graphgen
    import paper_2108_00529_amd as bgv
    from paper_2108_00529_amd import profile as prof

    wl = graphgen.WORKLOADS[args.workload]
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
                                          ws=ws_cd)
        sg = bgv.supergraph(edges, labels, degree, wl["rows"], wl["cols"], c1, c2, ws=ws_sg)
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

    prof.reset()
    prof.enable(not args.no_kernel_timing)
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
    kstats = prof.stats()
    inter = prof.counter("bh_interactions")
    for k in kstats:
        if k.startswith("bh_force") and inter:
            kstats[k]["bh_interactions"] = inter
    print(f"[bench] timed {args.steps} steps in {t_total:.2f}s", file=sys.stderr, flush=True)

    ms_per_step = 1000.0 * t_total / args.steps
    cd = float(np.mean(cd_ms))
    fa = float(np.mean(fa_ms))
    K, E = sg["K"], sg["E"]
    value = m / (cd / 1000.0)

    roofline, extra = roofline_report(kstats, wl, n, m, K, E)

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
                  "pipeline_edges_per_s": m / ((cd + fa) / 1000.0)},
        "roofline": roofline,
        **extra,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(edges_np, n, wl, c1, c2, pos0_np, args.cpu_fa2_iters)
    print(json.dumps(out))


# algorithmic bytes / flops per unit
EDGE_PASS_BYTES = 8            # one int32 (u,v) pair read per edge per pass
BH_INTERACTION_FLOPS = 20      # body-node or body-body interaction, n-body convention


def roofline_report(kstats, wl, n, m, K, E):
    """Roofline of the dominant kernel (by total time) plus the edge-stream kernels."""
    if not kstats:
        return None, {}
    by_time = sorted(kstats.items(), key=lambda kv: -kv[1]["total_ms"])
    extra = {"kernel_ms": {k: round(v["total_ms"] / max(v["launches"], 1), 5) for k, v in by_time}}
    rows = {}
    for name, st in kstats.items():
        avg_s = st["total_ms"] / 1000.0 / max(st["launches"], 1)
        if name in ("cd_apply_hist", "cd_decide"):
            per_launch = EDGE_PASS_BYTES * wl["chunk"]
            rows[name] = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    top, st = by_time[0]
    avg_s = st["total_ms"] / 1000.0 / max(st["launches"], 1)
    if top in rows:
        r = rows[top]
    elif top.startswith("bh_force") and "bh_interactions" in st:
        flops = BH_INTERACTION_FLOPS * st["bh_interactions"] / max(st["launches"], 1)
        r = dict(bound="alu", achieved=flops / avg_s / 1e12, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                 interactions_per_launch=st["bh_interactions"] / max(st["launches"], 1))
    else:
        r = dict(bound="unknown", achieved=None, peak=None, unit=None)
    r = dict(r, kernel=top, avg_ms=avg_s * 1000.0, traffic=measured_traffic(top))
    if r.get("achieved") is not None:
        r["frac"] = r["achieved"] / r["peak"]
    extra["roofline_edge_stream"] = {k: dict(v, frac=v["achieved"] / v["peak"]) for k, v in rows.items()}
    return r, extra


def measured_traffic(kernel: str):
    """HBM bytes per launch of the dominant kernel, from the committed rocprofv3 counter
    summary, or None when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    if not kernel.startswith("bh_force"):
        return None
    summary = os.path.join(ROOT, "profiles", "bh_force_lfr_1m.md")
    src = os.path.join(ROOT, "paper_2108_00529_amd", "csrc", "fa2.hip")
    try:
        text = open(summary).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m_hash = re.search(r"fa2\.hip when measured: ([0-9a-f]{16})", text)
    m_bytes = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != digest:
        return None
    return int(m_bytes.group(1))


def cpu_baseline(edges_np, n, wl, c1, c2, pos0_np, fa2_iters):
    """The oracle, untuned, on this host: community passes + supergraph on the whole
    graph (single thread) and a few Barnes-Hut FA2 iterations (OpenMP)."""
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
                      f"({t_cd:.1f}s, 1 thread); FA2: {fa2_iters} Barnes-Hut iterations on the "
                      f"{K}-node supergraph in {t_fa:.1f}s with {threads} OpenMP threads",
            "fa2_iters_per_s": fa2_iters / t_fa, "fa2_threads": threads}


if __name__ == "__main__":
    main()

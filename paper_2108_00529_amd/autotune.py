"""Autotuner for launch parameters that do not change results (here: the workgroup
size of the batched launch and the supergraph size above which a graph's layout leaves
the persistent launch for the multi-workgroup kernels).  Candidates are timed with HIP
events on the caller's inputs and the choice is cached per size bucket in a JSON file."""
from __future__ import annotations

import json
import math
import os

import torch

from . import api

WG_CANDIDATES = (256, 512, 1024)
BIG_K_CANDIDATES = (0, 16, 32, 64, 128, 256)
CANDIDATES = tuple((wg, bk) for wg in WG_CANDIDATES for bk in BIG_K_CANDIDATES)
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bgv_autotune.json")


def _bucket(G: int, n_total: int, m_total: int) -> str:
    return f"batched:G{G}:n2^{int(math.log2(max(n_total, 1)))}:m2^{int(math.log2(max(m_total, 1)))}"


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def tune_batched(edges, node_off, edge_off, n_total, wl, coef1, coef2, pos0, order=None, repeats=2,
                 use_cache=True):
    """Best (wg_threads, big_k) for this batch shape (times every candidate `repeats`
    times).  Returns the pair and a record of the timings."""
    key = _bucket(node_off.shape[0] - 1, n_total, edges.shape[0])
    cache = _load() if use_cache else {}
    if key in cache and "big_k" in cache[key]:
        return (int(cache[key]["wg_threads"]), int(cache[key]["big_k"])), cache[key]
    ws = api.batched_workspace(node_off.shape[0] - 1, n_total, edges.shape[0], edges.device)
    times = {}
    for wg, bk in CANDIDATES:
        best = float("inf")
        for _ in range(repeats):
            pos = pos0.clone()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            api.batched(edges, node_off, edge_off, n_total, wl, coef1, coef2, pos, order=order, wg_threads=wg,
                        big_k=bk, ws=ws)
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        times[(wg, bk)] = best
    wg, bk = min(times, key=times.get)
    entry = {"wg_threads": wg, "big_k": bk, "ms": {f"wg{k[0]}_big{k[1]}": v for k, v in times.items()}}
    cache[key] = entry
    if use_cache:
        _save(cache)
    return (wg, bk), entry

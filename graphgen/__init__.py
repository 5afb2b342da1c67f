"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the bench.

This module draws random graphs, initial positions and hash coefficients.  It holds
none of the method's arithmetic (no community rule, no sketch hashing, no force law):
both implementations receive what it produces as plain arrays.

The paper measures on public graph datasets (SNAP and others, Section 5.2) that are
not available here.  The generators below stand in for them with the shapes the
paper reports: power-law degrees, community structure and edge lists in random
stream order (Table 1 spans 45k-4.0M nodes and 2.3M-34.7M edges).

Every generator is deterministic in its seed (numpy PCG64).
"""
from __future__ import annotations

import concurrent.futures as _futures
import os

import numpy as np

_THREADS = max(1, min(16, os.cpu_count() or 1))

__all__ = [
    "planted_partition",
    "planted_fixed_m",
    "lfr_style",
    "batched_planted",
    "initial_positions",
    "hash_coeffs",
    "random_tiny_graph",
    "WORKLOADS",
]


def _orient_and_shuffle(rng: np.random.Generator, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Random stream order and random orientation of every edge -> int32 (m, 2)."""
    m = u.shape[0]
    swap = rng.random(m) < 0.5
    a = np.where(swap, v, u)
    b = np.where(swap, u, v)
    perm = rng.permutation(m)
    out = np.empty((m, 2), dtype=np.int32)
    out[:, 0] = a[perm]
    out[:, 1] = b[perm]
    return out


def planted_partition(n: int, blocks: int, p_in: float, p_out: float, seed: int):
    """Planted partition: ``blocks`` equal blocks, every unordered pair is an edge
    with probability ``p_in`` (same block) or ``p_out`` (different blocks).

    Block of node v is v // (n // blocks) before a seeded relabelling of node ids,
    so block membership is not visible in the ids.  Returns (edges int32 (m,2),
    block int32[n]) with edges in seeded random order and random orientation.
    """
    rng = np.random.default_rng(seed)
    size = n // blocks
    blk0 = np.minimum(np.arange(n) // size, blocks - 1)
    iu, ju = np.triu_indices(n, k=1)
    same = blk0[iu] == blk0[ju]
    p = np.where(same, p_in, p_out)
    keep = rng.random(iu.shape[0]) < p
    iu, ju = iu[keep], ju[keep]
    relabel = rng.permutation(n)
    u = relabel[iu]
    v = relabel[ju]
    block = np.empty(n, dtype=np.int32)
    block[relabel] = blk0
    return _orient_and_shuffle(rng, u, v), block


def planted_fixed_m(n: int, blocks: int, m: int, frac_intra: float, seed: int):
    """Planted partition with exactly ``m`` edges: round(frac_intra*m) edges drawn
    uniformly inside a uniformly chosen block (both endpoints uniform in it) and the
    rest uniformly between two different blocks.  No self-loops; multi-edges may
    occur.  Node ids are relabelled by a seeded permutation."""
    rng = np.random.default_rng(seed)
    blocks = max(1, min(blocks, n))
    bounds = np.linspace(0, n, blocks + 1).astype(np.int64)
    m_in = int(round(frac_intra * m)) if blocks > 1 else m
    m_out = m - m_in
    # intra edges
    b = rng.integers(0, blocks, size=m_in)
    lo, hi = bounds[b], bounds[b + 1]
    u = lo + rng.integers(0, 1 << 62, size=m_in) % (hi - lo)
    v = lo + rng.integers(0, 1 << 62, size=m_in) % (hi - lo)
    bad = u == v
    while bad.any():
        k = int(bad.sum())
        v[bad] = lo[bad] + rng.integers(0, 1 << 62, size=k) % (hi[bad] - lo[bad])
        bad = u == v
    # inter edges
    if m_out > 0:
        ou = rng.integers(0, n, size=m_out)
        ov = rng.integers(0, n, size=m_out)
        blk_of = np.searchsorted(bounds, np.arange(n), side="right") - 1
        bad = blk_of[ou] == blk_of[ov]
        while bad.any():
            k = int(bad.sum())
            ov[bad] = rng.integers(0, n, size=k)
            bad = blk_of[ou] == blk_of[ov]
        u = np.concatenate([u, ou])
        v = np.concatenate([v, ov])
    relabel = rng.permutation(n)
    blk0 = (np.searchsorted(bounds, np.arange(n), side="right") - 1).astype(np.int32)
    block = np.empty(n, dtype=np.int32)
    block[relabel] = blk0
    return _orient_and_shuffle(rng, relabel[u], relabel[v]), block


def _sorted_search(table: np.ndarray, t: np.ndarray) -> np.ndarray:
    """np.searchsorted(table, t, side='right'), faster for large unsorted t (the
    queries are visited in sorted order, which keeps the table walk cache-friendly),
    in slices on several threads (numpy's sort releases the interpreter lock)."""
    if t.shape[0] < 65536:
        return np.searchsorted(table, t, side="right")
    out = np.empty(t.shape[0], dtype=np.int64)

    def part(lo, hi):
        tc = t[lo:hi]
        idx = np.argsort(tc, kind="stable")
        out[lo + idx] = np.searchsorted(table, tc[idx], side="right")

    bounds = np.linspace(0, t.shape[0], _THREADS + 1).astype(np.int64)
    with _futures.ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(part, bounds[:-1], bounds[1:]))
    return out


def _power_law_sizes(rng, n: int, beta: float, smin: int, smax: int) -> np.ndarray:
    """Community sizes from a discrete power law p(s) ~ s^-beta on [smin, smax],
    drawn until they cover n nodes; the last one is trimmed to hit n exactly."""
    smax = max(smin, smax)
    sizes = []
    total = 0
    s_vals = np.arange(smin, smax + 1, dtype=np.float64)
    pmf = s_vals ** (-beta)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    while total < n:
        batch = s_vals[np.searchsorted(cdf, rng.random(4096), side="right").clip(0, len(s_vals) - 1)]
        for s in batch.astype(np.int64):
            sizes.append(int(s))
            total += int(s)
            if total >= n:
                break
    sizes[-1] -= total - n
    if sizes[-1] <= 0:
        sizes.pop()
    return np.asarray(sizes, dtype=np.int64)


def lfr_style(n: int, m: int, gamma: float, beta: float, mu: float, seed: int,
              smin: int = 20, smax: int | None = None):
    """LFR-style Chung-Lu graph with planted communities (not the LFR benchmark).

    1. expected degrees w ~ Pareto(gamma) (w >= 1), rescaled to sum 2m, capped at sqrt(2m);
    2. community sizes ~ power law (beta) on [smin, smax], assigned by a seeded shuffle;
    3. round((1-mu) m) intra edges: community chosen proportional to its total w,
       endpoints proportional to w inside it, u == v redrawn;
    4. the other edges: endpoints proportional to w over all nodes, redrawn while the
       endpoints share a community;
    5. stream order shuffled and each edge randomly oriented.
    Exactly m edges; multi-edges may occur.  Returns (edges int32 (m,2), comm int32[n]).
    """
    rng = np.random.default_rng(seed)
    if smax is None:
        smax = max(smin, n // 100)
    w = (1.0 - rng.random(n)) ** (-1.0 / (gamma - 1.0))
    w *= (2.0 * m) / w.sum()
    np.minimum(w, np.sqrt(2.0 * m), out=w)
    sizes = _power_law_sizes(rng, n, beta, smin, smax)
    order = rng.permutation(n)                       # nodes laid out community by community
    ncom = sizes.shape[0]
    comm = np.empty(n, dtype=np.int32)
    comm[order] = np.repeat(np.arange(ncom, dtype=np.int32), sizes)
    off = np.concatenate([[0], np.cumsum(sizes)])
    w_ord = w[order]
    cw = np.concatenate([[0.0], np.cumsum(w_ord)])   # cumulative weight in community order
    com_w = cw[off[1:]] - cw[off[:-1]]

    def draw_in(cidx):
        lo = cw[off[cidx]]
        hi = cw[off[cidx + 1]]
        t = lo + rng.random(cidx.shape[0]) * (hi - lo)
        pos = _sorted_search(cw, t) - 1
        pos = np.clip(pos, off[cidx], off[cidx + 1] - 1)
        return order[pos]

    m_in = int(round((1.0 - mu) * m))
    ccum = np.cumsum(com_w)
    cidx = _sorted_search(ccum, rng.random(m_in) * ccum[-1]).clip(0, ncom - 1)
    # communities of size 1 cannot host an intra edge
    small = sizes[cidx] < 2
    while small.any():
        cidx[small] = np.searchsorted(ccum, rng.random(int(small.sum())) * ccum[-1],
                                      side="right").clip(0, ncom - 1)
        small = sizes[cidx] < 2
    u = draw_in(cidx)
    v = draw_in(cidx)
    bad = u == v
    while bad.any():
        v[bad] = draw_in(cidx[bad])
        bad = u == v

    m_out = m - m_in
    gcum = np.cumsum(w)
    def draw_all(k):
        return _sorted_search(gcum, rng.random(k) * gcum[-1]).clip(0, n - 1)
    ou = draw_all(m_out)
    ov = draw_all(m_out)
    bad = comm[ou] == comm[ov]
    while bad.any():
        ov[bad] = draw_all(int(bad.sum()))
        bad = comm[ou] == comm[ov]
    u = np.concatenate([u, ou])
    v = np.concatenate([v, ov])
    return _orient_and_shuffle(rng, u, v), comm


def batched_planted(G: int, seed: int, median: int = 2000, sigma: float = 0.9,
                    nmin: int = 100, nmax: int = 20000, mean_degree: int = 10,
                    block_size: int = 250, frac_intra: float = 0.92):
    """Many uneven planted-partition graphs: node counts log-normal (median, sigma)
    clipped to [nmin, nmax]; blocks = clip(round(n/block_size), 2, 80);
    mean_degree*n/2 edges, frac_intra of them inside blocks.
    Returns a list of (n, edges int32 (m,2), block int32[n]) with local node ids."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.normal(np.log(median), sigma, size=G))
    ns = np.clip(np.round(ns), nmin, nmax).astype(np.int64)
    seeds = rng.integers(0, 2**31 - 1, size=G)
    out = []
    for g in range(G):
        n = int(ns[g])
        blocks = int(np.clip(round(n / block_size), 2, 80))
        m = mean_degree * n // 2
        e, b = planted_fixed_m(n, blocks, m, frac_intra, int(seeds[g]))
        out.append((n, e, b))
    return out


def random_tiny_graph(rng: np.random.Generator, n: int, m: int, loops: bool = False):
    """Uniform random multigraph stream on n nodes (tests); optional self-loops."""
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    if not loops and n > 1:
        bad = u == v
        while bad.any():
            v[bad] = rng.integers(0, n, size=int(bad.sum()))
            bad = u == v
    return np.stack([u, v], axis=1).astype(np.int32)


def initial_positions(K: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """FP32 positions uniform in [lo, hi]^2, shape (K, 2)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(K, 2)).astype(np.float32)


def hash_coeffs(rows: int, seed: int) -> np.ndarray:
    """Random 64-bit coefficients (A_r, B_r, C_r) for each sketch row, uint64 (rows, 3).

    They are the random draws of a pairwise-independent hash family; both sides take
    them as input instead of drawing them."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, np.iinfo(np.uint64).max, size=(rows, 3), dtype=np.uint64, endpoint=True)


# Frozen workloads.  Semantic parameters (threshold, passes, growth, chunk, sketch
# shape, iteration counts, force constants) are part of each workload's definition;
# launch parameters are not.
WORKLOADS = {
    "planted_2k": dict(
        kind="planted", n=2000, blocks=8, p_in=0.04, p_out=0.0005, graph_seed=1001,
        threshold=16, passes=1, growth=2, chunk=256,
        rows=4, cols=1024, sketch_seed=0xB16A0001,
        fa2_iters=200, exact=True, theta=1.2, kr=1.0, kg=1.0, tau=1.0, ks=0.1, ksmax=10.0,
        pos_seed=2001,
    ),
    "lfr_1m": dict(
        kind="lfr", n=1_000_000, m=10_000_000, gamma=2.3, beta=1.5, mu=0.2, graph_seed=1002,
        threshold=64, passes=3, growth=2, chunk=1 << 20,
        rows=4, cols=1 << 20, sketch_seed=0xB16A0002,
        fa2_iters=500, exact=False, theta=1.2, kr=1.0, kg=1.0, tau=1.0, ks=0.1, ksmax=10.0,
        pos_seed=2002,
    ),
    "lfr_3m": dict(
        kind="lfr", n=3_200_000, m=34_000_000, gamma=2.1, beta=1.5, mu=0.3, graph_seed=1003,
        threshold=128, passes=3, growth=2, chunk=1 << 22,
        rows=5, cols=1 << 22, sketch_seed=0xB16A0003,
        fa2_iters=1000, exact=False, theta=1.2, kr=1.0, kg=1.0, tau=1.0, ks=0.1, ksmax=10.0,
        pos_seed=2003,
    ),
    "batched_512": dict(
        kind="batched", G=512, graph_seed=1004,
        threshold=16, passes=1, growth=2, chunk=256,
        rows=4, cols=1024, sketch_seed=0xB16A0004,
        fa2_iters=300, exact=True, theta=1.2, kr=1.0, kg=1.0, tau=1.0, ks=0.1, ksmax=10.0,
        pos_seed=2004,
    ),
    # Gradient form: a weighted supergraph of 50,000 supernodes, the planted communities
    # (all of size 100) of a 5M-node LFR-style graph; mixing 0.04 leaves about 1.0M
    # distinct inter-community pairs.  Weights are the sketch estimates (5 x 2^22);
    # exact repulsion; positions uniform in [-50, 50]^2.
    "grad_50k": dict(
        kind="lfr", n=5_000_000, m=25_000_000, gamma=2.3, beta=1.5, mu=0.04, graph_seed=1005,
        smin=100, smax=100,
        rows=5, cols=1 << 22, sketch_seed=0xB16A0005,
        fa2_iters=500, exact=True, theta=1.2, kr=1.0, kg=1.0, tau=1.0, ks=0.1, ksmax=10.0,
        pos_seed=2005, pos_lo=-50.0, pos_hi=50.0,
    ),
}


def make_graph(name: str):
    """Edges (and planted labels) of a named single-graph workload."""
    w = WORKLOADS[name]
    if w["kind"] == "planted":
        return planted_partition(w["n"], w["blocks"], w["p_in"], w["p_out"], w["graph_seed"])
    if w["kind"] == "lfr":
        return lfr_style(w["n"], w["m"], w["gamma"], w["beta"], w["mu"], w["graph_seed"], smin=w.get("smin", 20),
                         smax=w.get("smax"))
    raise ValueError(name)

"""ORACLE (test infrastructure): the paper's sequential streaming community rule,
written out literally in pure Python for tiny graphs.

Section 3.2: degrees start at 0 and grow as edges are examined; for every edge, if
both endpoint degrees are at most the threshold D, the endpoint of smaller degree
joins the community of the endpoint of larger degree; otherwise the edge is skipped.
Algorithm 3 nests the two strict comparisons, so equal degrees change nothing, and
initialises degrees and labels once, before its loop over rounds; Section 3.2.1
multiplies the threshold by a constant factor each round.  Self-loops are ignored.
"""
from __future__ import annotations


def seq_scoda(n, edges, threshold, passes=1, growth=2, tie=False):
    """Return (labels, counters) as Python lists.  counters[v] = passes * degree(v).
    tie: the variant where, on equal degrees, the edge's first endpoint joins the
    community of the second (instead of nothing happening)."""
    label = list(range(n))
    deg = [0] * n
    D = threshold
    for p in range(passes):
        if p > 0:
            D = min(D * growth, 2**31 - 1)
        for (u, v) in edges:
            u = int(u)
            v = int(v)
            if u == v:
                continue
            deg[u] += 1
            deg[v] += 1
            if deg[u] <= D and deg[v] <= D:
                if deg[u] < deg[v]:
                    label[u] = label[v]
                elif deg[v] < deg[u]:
                    label[v] = label[u]
                elif tie:
                    label[u] = label[v]
    return label, deg

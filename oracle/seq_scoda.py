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


def seq_scoda(n, edges, threshold, passes=1, growth=2, tie=False, volume_rule=False):
    """Return (labels, counters) as Python lists.  counters[v] = passes * degree(v).
    tie: the variant where, on equal degrees, the edge's first endpoint joins the
    community of the second (instead of nothing happening).
    volume_rule: SCoDA's own test (Hollocou et al.) in place of the degree comparison:
    each community c keeps vol[c], the sum of its nodes' degrees; both endpoints' degree
    increments also raise their communities' volumes; when both degrees are at most D
    and the communities differ, the endpoint whose community has the smaller (or equal)
    volume moves to the other's, taking its degree along."""
    label = list(range(n))
    deg = [0] * n
    vol = [0] * n
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
            if volume_rule:
                vol[label[u]] += 1
                vol[label[v]] += 1
                if deg[u] <= D and deg[v] <= D and label[u] != label[v]:
                    if vol[label[u]] <= vol[label[v]]:
                        vol[label[v]] += deg[u]
                        vol[label[u]] -= deg[u]
                        label[u] = label[v]
                    else:
                        vol[label[u]] += deg[v]
                        vol[label[v]] -= deg[v]
                        label[v] = label[u]
                continue
            if deg[u] <= D and deg[v] <= D:
                if deg[u] < deg[v]:
                    label[u] = label[v]
                elif deg[v] < deg[u]:
                    label[v] = label[u]
                elif tie:
                    label[u] = label[v]
    return label, deg

"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
examples of the paper's rules (tests/golden), the literal sequential rule, closed
forms, invariants, special cases that reduce to library routines, and brute force on
tiny inputs.  No GPU is involved.
"""
import itertools
import math
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append([float(t) for t in line.split()])
    return out


STAR = np.array([[0, j] for j in range(1, 7)], dtype=np.int32)


# ------------------------------------------------------------------ community --
@pytest.mark.parametrize("row", _rows("star_seq.txt"))
def test_star_sequential_rule(row):
    D, P = int(row[0]), int(row[1])
    expect = [int(t) for t in row[2:]]
    lab, _ = oracle.seq_scoda(7, STAR.tolist(), D, P)
    assert lab == expect
    lab2, _ = oracle.bs_community(7, STAR, D, P, 2, 1)
    assert lab2.tolist() == expect


@pytest.mark.parametrize("row", _rows("star_bs.txt"))
def test_star_batch_synchronous(row):
    D, B = int(row[0]), int(row[1])
    expect = [int(t) for t in row[2:]]
    lab, _ = oracle.bs_community(7, STAR, D, 1, 2, B)
    assert lab.tolist() == expect


def test_chunk_one_is_the_sequential_rule():
    """chunk == 1 reproduces the literal sequential rule bit for bit."""
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(1, 25))
        m = int(rng.integers(0, 80))
        e = graphgen.random_tiny_graph(rng, n, m) if m else np.zeros((0, 2), np.int32)
        if trial % 3 == 0 and m:
            loop = rng.random(m) < 0.1
            e[loop, 1] = e[loop, 0]
        D = int(rng.integers(0, 12))
        P = int(rng.integers(1, 4))
        f = int(rng.integers(1, 4))
        ref_l, ref_c = oracle.seq_scoda(n, e.tolist(), D, P, f)
        lab, cnt = oracle.bs_community(n, e, D, P, f, 1)
        assert lab.tolist() == ref_l
        assert cnt.tolist() == ref_c


PATH = np.array([[0, 1], [2, 3], [1, 2]], dtype=np.int32)


@pytest.mark.parametrize("row", _rows("tie_path.txt"))
def test_tie_rule_hand_worked(row):
    D, P, B, tie = (int(t) for t in row[:4])
    expect = [int(t) for t in row[4:]]
    lab, _ = oracle.bs_community(4, PATH, D, P, 2, B, tie)
    assert lab.tolist() == expect
    if B == 1:
        assert oracle.seq_scoda(4, PATH.tolist(), D, P, 2, bool(tie))[0] == expect


def test_tie_rule_chunk_one_is_the_sequential_rule():
    """With the tie rule, chunk == 1 still reproduces the literal sequential loop."""
    rng = np.random.default_rng(13)
    for trial in range(300):
        n = int(rng.integers(1, 25))
        m = int(rng.integers(0, 80))
        e = graphgen.random_tiny_graph(rng, n, m) if m else np.zeros((0, 2), np.int32)
        D = int(rng.integers(0, 12))
        P = int(rng.integers(1, 4))
        f = int(rng.integers(1, 4))
        ref_l, ref_c = oracle.seq_scoda(n, e.tolist(), D, P, f, tie=True)
        lab, cnt = oracle.bs_community(n, e, D, P, f, 1, 1)
        assert lab.tolist() == ref_l
        assert cnt.tolist() == ref_c


def test_tie_rule_needs_a_tie():
    """Streams whose decisions never see equal counters give the same labels with and
    without the tie rule; streams with ties differ somewhere."""
    rng = np.random.default_rng(17)
    differ = 0
    for _ in range(100):
        n = 30
        e = graphgen.random_tiny_graph(rng, n, 60)
        a, _ = oracle.bs_community(n, e, 0, 1, 2, 1, 1)   # D = 0: no edge is ever tested
        b, _ = oracle.bs_community(n, e, 0, 1, 2, 1, 0)
        assert np.array_equal(a, b)
        c, _ = oracle.bs_community(n, e, 8, 2, 2, 1, 1)
        d, _ = oracle.bs_community(n, e, 8, 2, 2, 1, 0)
        differ += int(not np.array_equal(c, d))
    assert differ > 50


VSTREAM = np.array([[0, 1], [1, 2], [0, 2], [3, 2]], dtype=np.int32)


@pytest.mark.parametrize("row", _rows("volume_rule.txt"))
def test_volume_rule_hand_worked(row):
    D, P, B, rule = (int(t) for t in row[:4])
    expect = [int(t) for t in row[4:]]
    lab, _ = oracle.bs_community(4, VSTREAM, D, P, 2, B, 0, rule)
    assert lab.tolist() == expect
    if B == 1:
        assert oracle.seq_scoda(4, VSTREAM.tolist(), D, P, 2, volume_rule=bool(rule))[0] == expect


def test_volume_rule_chunk_one_is_the_sequential_loop():
    """With the volume rule, chunk == 1 reproduces the literal SCoDA loop."""
    rng = np.random.default_rng(19)
    for trial in range(300):
        n = int(rng.integers(1, 25))
        m = int(rng.integers(0, 80))
        e = graphgen.random_tiny_graph(rng, n, m) if m else np.zeros((0, 2), np.int32)
        if trial % 3 == 0 and m:
            loop = rng.random(m) < 0.1
            e[loop, 1] = e[loop, 0]
        D = int(rng.integers(0, 12))
        P = int(rng.integers(1, 4))
        ref_l, ref_c = oracle.seq_scoda(n, e.tolist(), D, P, 2, volume_rule=True)
        lab, cnt = oracle.bs_community(n, e, D, P, 2, 1, 0, 1)
        assert lab.tolist() == ref_l
        assert cnt.tolist() == ref_c


def test_volume_rule_rejects_the_tie_flag():
    with pytest.raises(ValueError):
        oracle.bs_community(3, np.array([[0, 1]], np.int32), 4, 1, 2, 1, 1, 1)


def test_self_loops_are_ignored():
    rng = np.random.default_rng(11)
    for _ in range(50):
        n = 15
        e = graphgen.random_tiny_graph(rng, n, 40)
        loops = np.repeat(np.arange(n, dtype=np.int32)[:, None], 2, axis=1)
        ins = np.concatenate([e[:20], loops[:5], e[20:], loops[5:]])
        l1, c1 = oracle.bs_community(n, ins, 6, 2, 2, 1)
        l0, c0 = oracle.bs_community(n, e, 6, 2, 2, 1)
        assert np.array_equal(l0, l1) and np.array_equal(c0, c1)


def test_single_chunk_closed_form():
    """One pass, one chunk holding the whole stream: every label starts as the node id,
    so node x ends with the id of the other endpoint of the smallest-index edge on
    which x is the strictly lower-degree endpoint and both final degrees are <= D."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(1, 120))
        e = graphgen.random_tiny_graph(rng, n, m)
        D = int(rng.integers(1, 15))
        d = np.bincount(e.ravel(), minlength=n)
        du, dv = d[e[:, 0]], d[e[:, 1]]
        act = (du <= D) & (dv <= D) & (du != dv)
        x = np.where(du < dv, e[:, 0], e[:, 1])
        y = np.where(du < dv, e[:, 1], e[:, 0])
        expect = np.arange(n)
        seen = np.zeros(n, bool)
        for i in np.nonzero(act)[0]:
            if not seen[x[i]]:
                seen[x[i]] = True
                expect[x[i]] = y[i]
        lab, cnt = oracle.bs_community(n, e, D, 1, 2, m + int(rng.integers(0, 5)))
        assert np.array_equal(lab, expect)
        assert np.array_equal(cnt, d)


def test_zero_threshold_is_identity():
    rng = np.random.default_rng(5)
    e = graphgen.random_tiny_graph(rng, 50, 300)
    for B in (1, 7, 300):
        lab, _ = oracle.bs_community(50, e, 0, 3, 2, B)
        assert np.array_equal(lab, np.arange(50))


def test_no_label_crosses_a_disconnected_block():
    """p_out = 0: labels only travel along edges, so no label leaves its block."""
    e, blk = graphgen.planted_partition(400, 4, 0.08, 0.0, seed=9)
    for B in (1, 64, 10**6):
        lab, _ = oracle.bs_community(400, e, 12, 3, 2, B)
        assert np.array_equal(blk[lab], blk)


def test_node_relabelling_equivariance():
    """Decisions read degrees only, never ids: relabelling nodes by pi maps labels by pi."""
    rng = np.random.default_rng(21)
    for _ in range(30):
        n = 60
        e = graphgen.random_tiny_graph(rng, n, 200)
        pi = rng.permutation(n).astype(np.int32)
        for B in (1, 16):
            l0, c0 = oracle.bs_community(n, e, 8, 2, 2, B)
            l1, c1 = oracle.bs_community(n, pi[e], 8, 2, 2, B)
            assert np.array_equal(l1[pi], pi[l0])
            assert np.array_equal(c1[pi], c0)


def test_degree_and_volume_invariants():
    rng = np.random.default_rng(2)
    e = graphgen.random_tiny_graph(rng, 300, 2000)
    e[::50, 1] = e[::50, 0]  # some self-loops
    P = 3
    lab, cnt = oracle.bs_community(300, e, 10, P, 2, 37)
    deg, vol = oracle.degree_volume(lab, cnt, P)
    nl = e[e[:, 0] != e[:, 1]]
    assert np.array_equal(cnt, P * np.bincount(nl.ravel(), minlength=300))
    assert np.array_equal(deg, np.bincount(nl.ravel(), minlength=300))
    assert int(vol.sum()) == 2 * nl.shape[0]
    assert np.array_equal(vol, np.bincount(lab, weights=deg, minlength=300).astype(np.int64))


def test_planted_partition_recovery_beats_chance():
    """On the 2,000-node planted partition most nodes end with a label from their own
    block (statistical; chance level is 1/8)."""
    wl = graphgen.WORKLOADS["planted_2k"]
    e, blk = graphgen.make_graph("planted_2k")
    lab, _ = oracle.bs_community(2000, e, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"])
    purity = float((blk[lab] == blk).mean())
    assert purity > 0.5
    assert oracle.modularity(e, lab) > 0.1


# ---------------------------------------------------------------------- hashes --
def _py_col_key(A, Bc, x, cols):
    t = (A * x + Bc) % (1 << 64)
    return ((t >> 32) * cols) >> 32


def _py_col_pair(A, Bc, Cc, a, b, cols):
    t = (A * a + Cc * b + Bc) % (1 << 64)
    return ((t >> 32) * cols) >> 32


def test_hash_vectors_against_python_bigint():
    coef = graphgen.hash_coeffs(5, 1234)
    rng = np.random.default_rng(0)
    for r in range(5):
        A, Bc, Cc = (int(v) for v in coef[r])
        for cols in (1, 7, 1024, (1 << 22), (1 << 31) - 1):
            for x in list(rng.integers(0, 2**31 - 1, 40)) + [0, 1, 2**31 - 1]:
                assert oracle.hash_key(coef[r], int(x), cols) == _py_col_key(A, Bc, int(x), cols)
            for _ in range(40):
                a, b = sorted(int(v) for v in rng.integers(0, 2**31 - 1, 2))
                assert oracle.hash_pair(coef[r], a, b, cols) == _py_col_pair(A, Bc, Cc, a, b, cols)


# ------------------------------------------------------------------ supergraph --
def _small_supergraph(seed=4, n=300, m=1500, rows=3, cols=64):
    rng = np.random.default_rng(seed)
    e = graphgen.random_tiny_graph(rng, n, m)
    lab, cnt = oracle.bs_community(n, e, 6, 2, 2, 50)
    deg, vol = oracle.degree_volume(lab, cnt, 2)
    c1 = graphgen.hash_coeffs(rows, seed + 100)
    c2 = graphgen.hash_coeffs(rows, seed + 200)
    sg = oracle.supergraph(n, e, lab, deg, rows, cols, c1, c2)
    return e, lab, deg, vol, c1, c2, sg


def test_supergraph_is_the_quotient_graph():
    nx = pytest.importorskip("networkx")
    e, lab, deg, vol, c1, c2, sg = _small_supergraph()
    G = nx.MultiGraph()
    G.add_nodes_from(range(300))
    G.add_edges_from(e.tolist())
    parts = {}
    for v, c in enumerate(lab):
        parts.setdefault(int(c), set()).add(v)
    Q = nx.quotient_graph(nx.Graph(G), list(parts.values()), relabel=False)
    q_edges = set()
    for A, B in Q.edges():
        a, b = lab[min(A)], lab[min(B)]
        q_edges.add((min(a, b), max(a, b)))
    lbl = sg["super_label"]
    got = {(int(lbl[s]), int(lbl[t])) for s, t in sg["superedges"]}
    assert got == q_edges
    assert sg["K"] == len(parts)
    assert np.array_equal(sg["super_label"], np.unique(lab))
    # sorted unique sid pairs with sid(a) < sid(b)
    se = sg["superedges"].astype(np.int64)
    assert np.all(se[:, 0] < se[:, 1])
    key = se[:, 0] * (1 << 32) + se[:, 1]
    assert np.all(np.diff(key) > 0)


def test_sketch_row_sums_and_one_sided_error():
    e, lab, deg, vol, c1, c2, sg = _small_supergraph()
    nl = e[e[:, 0] != e[:, 1]]
    inter = int((lab[nl[:, 0]] != lab[nl[:, 1]]).sum())
    intra = nl.shape[0] - inter
    assert np.all(sg["M1"].sum(axis=1, dtype=np.int64) == 2 * nl.shape[0])
    assert np.all(sg["M2"].sum(axis=1, dtype=np.int64) == inter)
    assert int(sg["se_count"].sum()) + intra == nl.shape[0]
    # count-min never under-estimates
    assert np.all(sg["super_size"].astype(np.int64) >= vol[sg["super_label"]])
    assert np.all(sg["se_weight"] >= sg["se_count"])


def test_sketch_matches_direct_counting():
    """Brute force: rebuild both sketches with Python big-int hashing and np.add.at."""
    e, lab, deg, vol, c1, c2, sg = _small_supergraph(rows=2, cols=37)
    rows, cols = 2, 37
    M1 = np.zeros((rows, cols), np.int64)
    M2 = np.zeros((rows, cols), np.int64)
    for r in range(rows):
        A, Bc, _ = (int(v) for v in c1[r])
        for v in range(lab.shape[0]):
            M1[r, _py_col_key(A, Bc, int(lab[v]), cols)] += int(deg[v])
        A, Bc, Cc = (int(v) for v in c2[r])
        for u, v in e.tolist():
            a, b = int(lab[u]), int(lab[v])
            if u != v and a != b:
                M2[r, _py_col_pair(A, Bc, Cc, min(a, b), max(a, b), cols)] += 1
    assert np.array_equal(M1, sg["M1"].astype(np.int64))
    assert np.array_equal(M2, sg["M2"].astype(np.int64))
    # point estimate = minimum over the rows at the key's columns (Section 3.3)
    for k, c in enumerate(sg["super_label"]):
        est = min(M1[r, _py_col_key(int(c1[r, 0]), int(c1[r, 1]), int(c), cols)] for r in range(rows))
        assert sg["super_size"][k] == est
    lbl = sg["super_label"]
    for k, (sa, sb) in enumerate(sg["superedges"].tolist()):
        a, b = int(lbl[sa]), int(lbl[sb])
        est = min(M2[r, _py_col_pair(int(c2[r, 0]), int(c2[r, 1]), int(c2[r, 2]), a, b, cols)] for r in range(rows))
        assert sg["se_weight"][k] == est


def test_sketch_without_collisions_is_exact():
    """With a sketch far wider than the key set, keys whose columns collide with no
    other key in some row are counted exactly (est == exact)."""
    e, lab, deg, vol, c1, c2, sg = _small_supergraph(cols=1 << 24, rows=4)
    assert np.array_equal(sg["super_size"].astype(np.int64), vol[sg["super_label"]])
    assert np.array_equal(sg["se_weight"], sg["se_count"])


def test_one_row_estimate_is_the_colliding_sum():
    """r = 1: the estimate of a key is the total of every key hashed to its column."""
    e, lab, deg, vol, c1, c2, sg = _small_supergraph(rows=1, cols=16)
    A, Bc, _ = (int(v) for v in c1[0])
    col = {c: _py_col_key(A, Bc, int(c), 16) for c in sg["super_label"]}
    for k, c in enumerate(sg["super_label"]):
        same = [d for d in sg["super_label"] if col[d] == col[c]]
        assert sg["super_size"][k] == sum(int(vol[d]) for d in same)


# ------------------------------------------------------------------ modularity --
def test_modularity_three_ways():
    nx = pytest.importorskip("networkx")
    from networkx.algorithms.community import modularity as nx_mod
    rng = np.random.default_rng(8)
    n = 40
    e = graphgen.random_tiny_graph(rng, n, 150)
    lab, _ = oracle.bs_community(n, e, 5, 2, 2, 10)
    q = oracle.modularity(e, lab)
    # brute force of Eq. 2 with the multigraph adjacency
    A = np.zeros((n, n))
    for u, v in e.tolist():
        A[u, v] += 1
        A[v, u] += 1
    k = A.sum(1)
    m2 = A.sum()
    qb = sum((A[i, j] - k[i] * k[j] / m2) for i in range(n) for j in range(n) if lab[i] == lab[j]) / m2
    G = nx.MultiGraph()
    G.add_nodes_from(range(n))
    G.add_edges_from(e.tolist())
    comms = {}
    for v, c in enumerate(lab):
        comms.setdefault(int(c), set()).add(v)
    qn = nx_mod(G, list(comms.values()))
    assert abs(q - qb) < 1e-12 and abs(q - qn) < 1e-12


# ----------------------------------------------------------------- ForceAtlas2 --
@pytest.mark.parametrize("row", _rows("fa2_two_body.txt"))
def test_two_body_equilibrium(row):
    kr, kg, dstar = row
    x0 = np.array([[-0.3, 0.0], [0.3, 0.0]])
    se = np.array([[0, 1]], np.int32)
    mass = oracle.fa2_mass(2, se)
    assert np.array_equal(mass, [2.0, 2.0])
    x, Fp, sp = oracle.fa2_layout(x0, se, mass, iters=3000, exact=True, kr=kr, kg=kg)
    d = float(np.linalg.norm(x[0] - x[1]))
    assert abs(d - dstar) < 1e-6
    assert abs(x[0, 0] + x[1, 0]) < 1e-9  # symmetric about the origin


def test_first_iteration_global_speed():
    """With no previous force, swing = |F| and traction = |F|/2, so the global speed
    becomes min(tau/2, 1.5) from its initial value 1."""
    rng = np.random.default_rng(1)
    x0 = rng.uniform(-1, 1, size=(30, 2))
    se = np.array(sorted({tuple(sorted(p)) for p in rng.integers(0, 30, size=(60, 2)).tolist() if p[0] != p[1]}), np.int32)
    for tau in (1.0, 0.4, 5.0):
        _, _, sp = oracle.fa2_layout(x0, se, iters=1, tau=tau)
        assert abs(sp - min(tau / 2, 1.5)) < 1e-12


@pytest.mark.parametrize("row", _rows("fa2_first_step.txt"))
def test_speed_and_displacement_by_hand(row):
    """Two-body steps worked out from the closed forms (tests/golden/fa2_first_step.txt):
    swing, traction, the global speed and its 1.5x cap, the local speed law, the
    ksmax cap on the step and the mass weights of S and T, along two directions."""
    t0, t1, m0, m1, kr, kg, tau, ks, ksmax, iters, cx, cy, e0, e1, es = row
    u = np.array([cx, cy])
    x0 = np.array([t0 * u, t1 * u])
    se = np.array([[0, 1]], np.int32)
    x, _, sp = oracle.fa2_layout(x0, se, np.array([m0, m1]), iters=int(iters), exact=True, kr=kr, kg=kg,
                                 tau=tau, ks=ks, ksmax=ksmax)
    assert np.allclose(x, np.array([e0 * u, e1 * u]), rtol=0, atol=1e-13)
    assert abs(sp - es) < 1e-14


def _rand_fa2(seed, K=40, E=80):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(K, 2))
    pairs = set()
    while len(pairs) < E:
        a, b = rng.integers(0, K, 2)
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    se = np.array(sorted(pairs), np.int32)
    mass = oracle.fa2_mass(K, se)
    aw = rng.uniform(0.5, 2.0, size=E)
    return x, se, mass, aw


def test_internal_forces_cancel():
    """Repulsion and attraction are pairwise equal and opposite (Newton's third law):
    with gravity off the net force sums to zero."""
    x, se, mass, aw = _rand_fa2(2)
    F = oracle.fa2_forces(x, se, mass, aw, kr=1.3, kg=0.0)
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max()


def test_rotation_and_reflection_equivariance():
    x, se, mass, aw = _rand_fa2(3)
    F = oracle.fa2_forces(x, se, mass, aw, kr=1.0, kg=1.0)
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    Fr = oracle.fa2_forces(x @ R.T, se, mass, aw, kr=1.0, kg=1.0)
    assert np.allclose(Fr, F @ R.T, rtol=0, atol=1e-12 * np.abs(F).max())
    Mx = np.array([[1.0, 0.0], [0.0, -1.0]])
    Fm = oracle.fa2_forces(x @ Mx.T, se, mass, aw)
    assert np.allclose(Fm, F @ Mx.T, rtol=0, atol=1e-12 * np.abs(F).max())


def test_force_is_minus_energy_gradient():
    """Central finite differences of the energy match -F (FP64, O(h^2))."""
    x, se, mass, aw = _rand_fa2(4, K=30, E=50)
    F = oracle.fa2_forces(x, se, mass, aw, kr=0.7, kg=1.4)
    h = 1e-5
    for i in range(30):
        for c in range(2):
            xp = x.copy(); xp[i, c] += h
            xm = x.copy(); xm[i, c] -= h
            g_full = (oracle.fa2_energy(xp, se, mass, aw, 0.7, 1.4) - oracle.fa2_energy(xm, se, mass, aw, 0.7, 1.4)) / (2 * h)
            g_node = (oracle.fa2_node_energy(xp, se, mass, i, aw, 0.7, 1.4) - oracle.fa2_node_energy(xm, se, mass, i, aw, 0.7, 1.4)) / (2 * h)
            assert abs(g_full + F[i, c]) < 1e-6 * max(1.0, abs(F[i, c]))
            assert abs(g_node + F[i, c]) < 1e-6 * max(1.0, abs(F[i, c]))


def test_energy_brute_force_small():
    """The energy formula evaluated by direct pure-Python summation on 4 nodes."""
    x = np.array([[0.1, 0.2], [-0.5, 0.4], [0.3, -0.7], [0.9, 0.05]])
    se = np.array([[0, 1], [1, 2], [0, 3]], np.int32)
    mass = oracle.fa2_mass(4, se)
    aw = np.array([1.0, 2.0, 0.5])
    kr, kg = 1.7, 0.6
    ref = 0.0
    for (i, j), a in zip(se.tolist(), aw):
        ref += 0.5 * a * ((x[i, 0] - x[j, 0]) ** 2 + (x[i, 1] - x[j, 1]) ** 2)
    for i, j in itertools.combinations(range(4), 2):
        ref -= kr * mass[i] * mass[j] * math.log(math.hypot(x[i, 0] - x[j, 0], x[i, 1] - x[j, 1]))
    for i in range(4):
        ref += kg * mass[i] * math.hypot(*x[i])
    assert abs(oracle.fa2_energy(x, se, mass, aw, kr, kg) - ref) < 1e-12


def test_coincident_nodes_and_origin():
    """Coincident nodes exert no repulsion on each other; gravity vanishes at the origin."""
    x = np.array([[0.0, 0.0], [0.5, 0.5], [0.5, 0.5]])
    se = np.zeros((0, 2), np.int32)
    mass = np.ones(3)
    F = oracle.fa2_forces(x, se, mass, kr=1.0, kg=1.0)
    # node 0: repulsion from the two others only, no gravity
    d2 = 0.5
    assert np.allclose(F[0], [-2 * 0.5 / d2, -2 * 0.5 / d2])
    assert np.all(np.isfinite(F))


# ------------------------------------------------------------------ Barnes-Hut --
def test_barnes_hut_with_zero_theta_is_exact():
    x, se, mass, aw = _rand_fa2(5, K=200, E=300)
    Fe = oracle.fa2_forces(x, se, mass, aw, exact=True)
    Fb = oracle.fa2_forces(x, se, mass, aw, exact=False, theta=0.0)
    assert np.abs(Fe - Fb).max() < 1e-10 * np.abs(Fe).max()


def test_barnes_hut_error_shrinks_with_theta():
    x, se, mass, aw = _rand_fa2(6, K=800, E=1000)
    Fe = oracle.fa2_forces(x, se, mass, aw, exact=True)
    errs = []
    for th in (1.2, 0.6, 0.3):
        Fb = oracle.fa2_forces(x, se, mass, aw, exact=False, theta=th)
        errs.append(np.linalg.norm(Fe - Fb) / np.linalg.norm(Fe))
    assert errs[0] < 0.1 and errs[1] < errs[0] and errs[2] < errs[1]


def _quantise(x32):
    """FP32 grid coordinates of the Barnes-Hut tree, computed here with numpy."""
    xmin, ymin = x32[:, 0].min(), x32[:, 1].min()
    s0 = max(x32[:, 0].max() - xmin, x32[:, 1].max() - ymin)
    if not s0 > 0:
        s0 = np.float32(1.0)
    qx = np.minimum(((x32[:, 0] - xmin) / np.float32(s0) * np.float32(65536)).astype(np.int64), 65535)
    qy = np.minimum(((x32[:, 1] - ymin) / np.float32(s0) * np.float32(65536)).astype(np.int64), 65535)
    return qx, qy, float(s0)


def _quadtree_by_subdivision(qx, qy):
    """Compressed quadtree by recursive subdivision of the grid, in plain Python: each
    node is the smallest cell holding its bodies, its children the nodes of its
    occupied quadrants.  Returns {(body set, depth): set of children's body sets}."""
    out = {}

    def node(bodies):
        d = 0
        while d < 16 and len({(int(qx[b]) >> (15 - d), int(qy[b]) >> (15 - d)) for b in bodies}) == 1:
            d += 1
        if d == 16 and len({(int(qx[b]), int(qy[b])) for b in bodies}) == 1:
            out[(frozenset(bodies), 16)] = frozenset()
            return frozenset(bodies)
        groups = {}
        for b in bodies:
            groups.setdefault((int(qx[b]) >> (15 - d), int(qy[b]) >> (15 - d)), []).append(b)
        out[(frozenset(bodies), d)] = frozenset(node(g) for g in groups.values())
        return frozenset(bodies)

    node(list(range(len(qx))))
    return out


def test_barnes_hut_tree_against_geometric_cells():
    """The oracle's quadtree equals the one built by recursive subdivision of the grid
    (node body sets, cell depths, children), its Morton codes are the grid points'
    interleaved bits, and every node's mass and centre of mass are its bodies'."""
    rng = np.random.default_rng(12)
    for K, spread in ((300, 1.0), (400, 1e-3)):
        x32 = rng.uniform(-3, 2, size=(K, 2)).astype(np.float32)
        x32[K // 2:] = (x32[K // 2:] * np.float32(spread)).astype(np.float32)  # a dense cluster: deep cells
        x32[:5] = x32[5]  # a multi-body leaf
        x = x32.astype(np.float64)
        mass = rng.integers(1, 6, K).astype(np.float64)
        order, ni, nd, ch = oracle.bh_tree(x, mass)
        qx, qy, s0 = _quantise(x32)
        codes, s0o, _, _ = oracle.bh_codes(x32)
        assert s0o == s0
        for i in range(K):
            c = 0
            for b in range(16):
                c |= ((int(qx[i]) >> b) & 1) << (2 * b)
                c |= ((int(qy[i]) >> b) & 1) << (2 * b + 1)
            assert int(codes[i]) == c
        assert sorted(order.tolist()) == list(range(K))
        assert np.all(np.diff(codes[order].astype(np.int64)) >= 0)
        got = {}
        for k in range(ni.shape[0]):
            lo, hi, c0, nc, depth = ni[k]
            bodies = order[lo:hi]
            kids = frozenset(frozenset(order[ni[c, 0]:ni[c, 1]].tolist()) for c in ch[c0:c0 + nc]) if nc else frozenset()
            got[(frozenset(bodies.tolist()), int(depth))] = kids
            size, M, cx, cy = nd[k]
            assert size == s0 / 2.0**depth
            assert abs(M - mass[bodies].sum()) < 1e-9
            assert abs(cx - (mass[bodies] * x[bodies, 0]).sum() / M) < 1e-9 * max(1.0, abs(cx))
            assert abs(cy - (mass[bodies] * x[bodies, 1]).sum() / M) < 1e-9 * max(1.0, abs(cy))
        assert ni[0, 0] == 0 and ni[0, 1] == K
        ref = _quadtree_by_subdivision(qx, qy)
        assert got == ref
        assert max(d for _, d in ref) == 16 and any(len(v) == 2 for v in ref.values())


def test_barnes_hut_opens_the_cell_holding_the_body():
    """Body A at a corner of the square shares a quadrant (side 0.5) with a heavy body D;
    that cell's centre of mass lies ~0.69 from A, so size / distance ~ 0.72 < theta =
    1.2, yet the cell holds A and must be opened: A then meets D and E body by body,
    and its repulsion is the exact pairwise sum."""
    x = np.array([[0.0, 0.0], [0.49, 0.49], [1.0, 1.0]])
    mass = np.array([1.0, 50.0, 2.0])
    order, ni, nd, _ = oracle.bh_tree(x, mass)
    cell = [k for k in range(ni.shape[0]) if sorted(order[ni[k, 0]:ni[k, 1]].tolist()) == [0, 1]][0]
    size, _, cx, cy = nd[cell]
    assert size == 0.5 and size / math.hypot(cx, cy) < 1.2
    F, _ = oracle.bh_repulsion(x, mass, theta=1.2)
    exact = sum(mass[0] * mass[j] * (x[0] - x[j]) / ((x[0] - x[j]) @ (x[0] - x[j])) for j in (1, 2))
    assert np.allclose(F[0], exact, rtol=1e-14, atol=0)


def test_barnes_hut_borderline_flags():
    """A body is flagged exactly when one of its opening tests lies within the stated
    single-precision margin of theta: with theta set to a cell's own size / distance
    ratio the body that tests it is flagged; far from every ratio none is."""
    x = np.array([[0.0, 0.0], [8.0, 0.0], [8.0, 0.25], [-7.0, 3.0]])
    mass = np.array([1.0, 2.0, 3.0, 1.0])
    order, ni, nd, ch = oracle.bh_tree(x, mass)
    pair = [k for k in range(ni.shape[0]) if sorted(order[ni[k, 0]:ni[k, 1]].tolist()) == [1, 2]][0]
    size, M, cx, cy = nd[pair]
    ratio = size / math.hypot(cx, cy)
    _, border = oracle.bh_repulsion(x, mass, theta=ratio)
    assert border[0]
    _, border = oracle.bh_repulsion(x, mass, theta=ratio * 1.01)
    assert not border[0]
    F, border = oracle.bh_repulsion(x, mass, theta=1e-3)  # every cell opened: no test is near theta
    assert not border.any()
    assert np.allclose(F, oracle.fa2_forces(x, np.zeros((0, 2), np.int32), mass, kg=0.0, exact=True), rtol=1e-12)


def test_barnes_hut_opening_criterion_by_hand():
    """A far pair of bodies is replaced by its centre of mass exactly when
    cell size / distance < theta (Barnes-Hut criterion), else summed directly."""
    # A at the origin, B and C close together 8 units away
    x = np.array([[0.0, 0.0], [8.0, 0.0], [8.0, 0.25]])
    mass = np.array([1.0, 2.0, 3.0])
    se = np.zeros((0, 2), np.int32)
    order, ni, nd, _ = oracle.bh_tree(x, mass)
    pair = [k for k in range(ni.shape[0]) if sorted(order[ni[k, 0]:ni[k, 1]].tolist()) == [1, 2]]
    assert len(pair) == 1
    size, M, cx, cy = nd[pair[0]]
    d = math.hypot(cx, cy)
    ratio = size / d
    approx = -M * mass[0] * np.array([cx, cy]) / d**2
    exact = sum(-mass[0] * mass[j] * x[j] / (x[j] @ x[j]) for j in (1, 2))
    Fa = oracle.fa2_forces(x, se, mass, kr=1.0, kg=0.0, exact=False, theta=ratio * 1.001)
    Fe = oracle.fa2_forces(x, se, mass, kr=1.0, kg=0.0, exact=False, theta=ratio * 0.999)
    assert np.allclose(Fa[0], approx, rtol=1e-12, atol=0)
    assert np.allclose(Fe[0], exact, rtol=1e-12, atol=0)
    assert not np.allclose(approx, exact, rtol=1e-6, atol=0)


def test_fa2_trajectory_amplifies_rounding():
    """Why layouts are compared step by step: on the 2,000-node planted supergraph a
    1e-7 relative perturbation of the start positions grows past 1e-3 (normalised
    layout distance) within 5 FP64 iterations, so no FP32 implementation can track the
    FP64 trajectory for 200 iterations; each single step, however, is well conditioned."""
    wl = graphgen.WORKLOADS["planted_2k"]
    e, _ = graphgen.make_graph("planted_2k")
    lab, cnt = oracle.bs_community(2000, e, wl["threshold"], 1, 2, wl["chunk"])
    deg, _ = oracle.degree_volume(lab, cnt, 1)
    c1 = graphgen.hash_coeffs(4, wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(4, wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    sg = oracle.supergraph(2000, e, lab, deg, 4, 1024, c1, c2)
    x0 = graphgen.initial_positions(sg["K"], wl["pos_seed"]).astype(np.float64)
    x1 = x0 * (1 + 1e-7 * np.random.default_rng(0).standard_normal(x0.shape))

    def dist(p, r):
        return np.linalg.norm(p - r, axis=1).max() / np.linalg.norm(r - r.mean(0), axis=1).max()

    a1 = oracle.fa2_layout(x0, sg["superedges"], iters=1)[0]
    b1 = oracle.fa2_layout(x1, sg["superedges"], iters=1)[0]
    a5 = oracle.fa2_layout(x0, sg["superedges"], iters=5)[0]
    b5 = oracle.fa2_layout(x1, sg["superedges"], iters=5)[0]
    assert dist(b1, a1) < 1e-4
    assert dist(b5, a5) > 1e-3


# ------------------------------------------------------------- drawing rules ----
def test_draw_groups_hand_worked():
    """Section 4.3 applied by hand: sizes 6,1,1,1,1 (alpha = 10): the four size-1
    communities hold 4 <= 5 = alpha/2, group 0; the size-6 one is the whole rest, group
    10.  Twenty communities of size 1: ids 0..9 hold half, group 0; ids 10..19 take one
    of the ten remaining groups each, in id order.  Two equal sizes: the lower id is the
    smaller community (exactly half, group 0).  One community or all sizes 0."""
    g, r = oracle.draw_supernodes([6, 1, 1, 1, 1])
    assert g.tolist() == [10, 0, 0, 0, 0]
    assert r.dtype == np.float32 and r[0] == np.float32(np.sqrt(np.float32(6))) and r[1] == 1.0
    g, _ = oracle.draw_supernodes([1] * 20)
    assert g.tolist() == [0] * 10 + list(range(1, 11))
    assert oracle.draw_supernodes([3, 3])[0].tolist() == [0, 10]
    assert oracle.draw_supernodes([5])[0].tolist() == [10]
    g, r = oracle.draw_supernodes([0, 0, 0])
    assert g.tolist() == [0, 0, 0] and r.tolist() == [0.0, 0.0, 0.0]
    # radii: exact on squares, correctly rounded elsewhere
    _, r = oracle.draw_supernodes([0, 1, 4, 9, 65536, 2**32 - 1])
    assert r[:5].tolist() == [0.0, 1.0, 2.0, 3.0, 256.0]
    assert r[5] == np.float32(65536.0)  # 2^32 - 1 rounds to 2^32 in float32


def test_draw_groups_invariants():
    """On random sizes: groups never decrease with size; group 0 holds at most half of
    the total and adding the next community would exceed it; every group k >= 1 ends at
    or before k/10 of the second half and the next one starts after (k-1)/10 of it; the
    largest community is in group 10 whenever the total is positive."""
    rng = np.random.default_rng(41)
    for trial in range(30):
        K = int(rng.integers(1, 400))
        sizes = rng.integers(0, 1 + int(rng.choice([3, 100, 2**20])), K).astype(np.uint64)
        if trial % 5 == 0:
            sizes[rng.random(K) < 0.5] = 0
        g, _ = oracle.draw_supernodes(sizes)
        order = sorted(range(K), key=lambda c: (int(sizes[c]), c))
        alpha = int(sizes.sum())
        gs = [int(g[c]) for c in order]
        assert gs == sorted(gs)
        run = 0
        for c in order:
            run += int(sizes[c])
            if g[c] == 0:
                assert 2 * run <= alpha
            else:
                k = int(g[c])
                assert 10 * (2 * run - alpha) <= k * alpha          # ends within group k's share
                assert 10 * (2 * run - alpha) > (k - 1) * alpha     # and past group k-1's
        if alpha > 0:
            assert g[order[-1]] == 10
        else:
            assert (g == 0).all()

"""GPU tests of the batched form: every graph of a batch must give exactly what the
plain path gives on it alone (integers and positions bit for bit, since the batched
kernel repeats the plain kernels' arithmetic), the integers must equal the oracle's, the
last layout step must match one oracle step, and no launch parameter may change a bit."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def bgv():
    import paper_2108_00529_amd as b
    return b


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def batch():
    wl = dict(graphgen.WORKLOADS["batched_512"])
    wl["fa2_iters"] = 40
    graphs = graphgen.batched_planted(24, seed=77, median=300, sigma=0.9, nmin=20, nmax=3000)
    graphs[3] = (1, np.zeros((0, 2), np.int32), np.zeros(1, np.int32))                # one node, no edge
    graphs[7] = (5, np.array([[1, 1], [2, 2], [3, 3]], np.int32), np.zeros(5, np.int32))  # only loops
    # no edges at all: every node is its own supernode, so the layouts span several
    # repulsion segments of 512 bodies; 4500 is above the largest size the
    # multi-workgroup kernels take, 3000 within it
    graphs[11] = (4500, np.zeros((0, 2), np.int32), np.zeros(4500, np.int32))
    graphs[13] = (3000, np.zeros((0, 2), np.int32), np.zeros(3000, np.int32))
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    pos0 = [graphgen.initial_positions(n, wl["pos_seed"] + g) for g, (n, _, _) in enumerate(graphs)]
    return wl, graphs, c1, c2, pos0


def run_batched(bgv, wl, graphs, c1, c2, pos0, wg_threads=0, largest_first=False, iters=None, big_k=0):
    dev = torch.device("cuda")
    w = dict(wl) if iters is None else dict(wl, fa2_iters=iters)
    edges, noff, eoff, noff_h, eoff_h = bgv.pack_graphs([(n, e) for n, e, _ in graphs], dev)
    pos = torch.from_numpy(np.concatenate(pos0)).to(dev)
    order = None
    if largest_first:
        order = torch.from_numpy(np.argsort(-np.diff(eoff_h), kind="stable").astype(np.int32)).to(dev)
    out = bgv.batched(edges, noff, eoff, int(noff_h[-1]), w, c1, c2, pos, order=order, wg_threads=wg_threads,
                      big_k=big_k)
    torch.cuda.synchronize()
    return out, noff_h, eoff_h


def per_graph(out, noff, eoff, g):
    n0, n1, e0 = noff[g], noff[g + 1], eoff[g]
    K, E = int(out["K"][g]), int(out["E"][g])
    return dict(labels=host(out["labels"][n0:n1]), degree=host(out["degree"][n0:n1]), K=K, E=E,
                super_label=host(out["super_label"][n0:n0 + K]),
                super_size=host(out["super_size"][n0:n0 + K]).view(np.uint32),
                superedges=host(out["superedges"][e0:e0 + E]), se_weight=host(out["se_weight"][e0:e0 + E]).view(np.uint32),
                pos=host(out["pos"][n0:n0 + K]), fprev=host(out["fprev"][n0:n0 + K]), speed=float(out["speed"][g]))


def test_batched_equals_plain_and_oracle(bgv, batch):
    wl, graphs, c1, c2, pos0 = batch
    out, noff, eoff = run_batched(bgv, wl, graphs, c1, c2, pos0)
    for g, (n, e, _) in enumerate(graphs):
        b = per_graph(out, noff, eoff, g)
        say(f"  graph {g}: n={n} m={len(e)} K={b['K']} E={b['E']}")
        # oracle integers
        lab, cnt = oracle.bs_community(n, e, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"])
        deg, _ = oracle.degree_volume(lab, cnt, wl["passes"])
        np.testing.assert_array_equal(b["labels"], lab)
        np.testing.assert_array_equal(b["degree"], deg)
        ref = oracle.supergraph(n, e, lab, deg, wl["rows"], wl["cols"], c1, c2)
        assert b["K"] == ref["K"] and b["E"] == len(ref["superedges"])
        np.testing.assert_array_equal(b["super_label"], ref["super_label"])
        np.testing.assert_array_equal(b["super_size"], ref["super_size"])
        np.testing.assert_array_equal(b["superedges"], ref["superedges"])
        np.testing.assert_array_equal(b["se_weight"], ref["se_weight"])
        # plain path, positions bit for bit
        if b["K"] == 0:
            continue
        se = torch.from_numpy(ref["superedges"]).cuda()
        p, f, s = bgv.fa2_layout(se, torch.from_numpy(pos0[g][:b["K"]]).cuda(), wl["fa2_iters"], exact=True,
                                 kr=wl["kr"], kg=wl["kg"], tau=wl["tau"], ks=wl["ks"], ksmax=wl["ksmax"])
        assert np.array_equal(b["pos"], host(p)), f"graph {g}: positions differ from the plain path"
        assert np.array_equal(b["fprev"], host(f)) and b["speed"] == float(s)


def test_batched_tie_rule(bgv, batch):
    """The tie-rule variant in the batched form: every graph's labels and degrees equal
    the oracle's with the same rule."""
    wl, graphs, c1, c2, pos0 = batch
    w = dict(wl, tie=1)
    out, noff, eoff = run_batched(bgv, w, graphs, c1, c2, pos0, iters=2)
    moved = 0
    for g, (n, e, _) in enumerate(graphs):
        r = per_graph(out, noff, eoff, g)
        lab_r, cnt_r = oracle.bs_community(n, e, w["threshold"], w["passes"], w["growth"], w["chunk"], 1)
        deg_r, _ = oracle.degree_volume(lab_r, cnt_r, w["passes"])
        np.testing.assert_array_equal(r["labels"], lab_r)
        np.testing.assert_array_equal(r["degree"], deg_r)
        lab0, _ = oracle.bs_community(n, e, w["threshold"], w["passes"], w["growth"], w["chunk"], 0)
        moved += int(not np.array_equal(lab0, lab_r))
    assert moved > 0  # the rule changed some graph's communities


def test_batched_last_step_matches_oracle(bgv, batch):
    wl, graphs, c1, c2, pos0 = batch
    T = wl["fa2_iters"]
    head, noff, eoff = run_batched(bgv, wl, graphs, c1, c2, pos0, iters=T - 1)
    full, _, _ = run_batched(bgv, wl, graphs, c1, c2, pos0, iters=T)
    worst = 0.0
    for g, (n, e, _) in enumerate(graphs):
        a = per_graph(head, noff, eoff, g)
        b = per_graph(full, noff, eoff, g)
        if a["K"] < 3:
            continue
        r1, _, _ = oracle.fa2_layout(a["pos"], a["superedges"], iters=1, exact=True, kr=wl["kr"], kg=wl["kg"],
                                     Fprev=a["fprev"], speed=a["speed"])
        err = np.linalg.norm(b["pos"] - r1, axis=1).max() / np.linalg.norm(r1 - r1.mean(0), axis=1).max()
        worst = max(worst, err)
    say(f"  worst last-step position error {worst:.2e}")
    assert worst <= 1e-4


def test_batched_launch_parameters_change_nothing(bgv, batch):
    """Workgroup size, queue order and the size above which a layout leaves the
    persistent launch (big_k: 16 sends most of these supergraphs, 1 all but the
    single-node ones, to the multi-workgroup kernels) change no bit."""
    wl, graphs, c1, c2, pos0 = batch
    ref, noff, eoff = run_batched(bgv, wl, graphs, c1, c2, pos0)
    K = [int(k) for k in ref["K"].cpu()]
    assert sum(k > 16 for k in K) >= 5
    for wg, largest, bk in ((256, False, 0), (1024, True, 0), (1024, False, 16), (256, True, 1), (512, True, 64)):
        out, _, _ = run_batched(bgv, wl, graphs, c1, c2, pos0, wg_threads=wg, largest_first=largest, big_k=bk)
        for g in range(len(graphs)):
            a, b = per_graph(out, noff, eoff, g), per_graph(ref, noff, eoff, g)
            for k in a:
                assert np.array_equal(a[k], b[k]), (wg, largest, bk, g, k)


def test_autotuner_picks_a_candidate(bgv, batch):
    from paper_2108_00529_amd import autotune
    wl, graphs, c1, c2, pos0 = batch
    dev = torch.device("cuda")
    edges, noff, eoff, noff_h, _ = bgv.pack_graphs([(n, e) for n, e, _ in graphs], dev)
    pos = torch.from_numpy(np.concatenate(pos0)).to(dev)
    choice, entry = autotune.tune_batched(edges, noff, eoff, int(noff_h[-1]), dict(wl, fa2_iters=5), c1, c2, pos,
                                          repeats=1, use_cache=False)
    assert choice in autotune.CANDIDATES and len(entry["ms"]) == len(autotune.CANDIDATES)
    assert entry["wg_threads"] == choice[0] and entry["big_k"] == choice[1]


def test_captured_batched_replays_match_eager(bgv, batch):
    """The whole batched launch captured once in a graph and replayed repeatedly (with
    eager work and synchronisations between replays) gives the eager result each time."""
    wl, graphs, c1, c2, pos0 = batch
    dev = torch.device("cuda")
    edges, noff, eoff, noff_h, eoff_h = bgv.pack_graphs([(n, e) for n, e, _ in graphs], dev)
    n_total, G = int(noff_h[-1]), len(graphs)
    pos_init = torch.from_numpy(np.concatenate(pos0)).to(dev)
    ws = bgv.batched_workspace(G, n_total, edges.shape[0], dev)
    pos, fprev = pos_init.clone(), torch.zeros_like(pos_init)
    speed = torch.ones(G, dtype=torch.float32, device=dev)

    def run():
        pos.copy_(pos_init)
        fprev.zero_()
        speed.fill_(1.0)
        return bgv.batched(edges, noff, eoff, n_total, wl, c1, c2, pos, fprev=fprev, speed=speed, ws=ws)

    eager = {k: v.clone() for k, v in run().items()}
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap = run()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        for g in range(G):
            a, b = per_graph(cap, noff_h, eoff_h, g), per_graph(eager, noff_h, eoff_h, g)
            for k in a:
                assert np.array_equal(a[k], b[k]), (rep, g, k)
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device=dev)
        (junk * 2).sum().item()

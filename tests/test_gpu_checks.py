"""GPU tests of the opt-in device id checks (BGV_CHECK=1 and bgv_validate_edges): an id
outside its range is reported as BGV_E_RANGE before any kernel that indexes by ids runs
(the check kernels only read the ids; the profiler shows which kernels ran), and valid
input passes through unchanged."""
import numpy as np
import pytest
import torch

import graphgen
from paper_2108_00529_amd import _lib as L
from paper_2108_00529_amd import profile as prof

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bgv():
    import paper_2108_00529_amd as b
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print(*a, flush=True)


def _only_checks_ran(fn):
    """Runs fn with every library launch recorded; returns fn's exception and the set of
    kernels that ran."""
    prof.reset()
    prof.only(None)
    prof.enable(True)
    err = None
    try:
        fn()
    except (ValueError, L.BgvError) as e:  # noqa: PERF203
        err = e
    torch.cuda.synchronize()
    prof.enable(False)
    names = set(prof.stats())
    prof.reset()
    return err, names


def _is_check(name):
    return name.startswith("check_") or name.startswith("fill")


def test_validate_edges_entry_point(bgv):
    rng = np.random.default_rng(3)
    n = 5000
    e = graphgen.random_tiny_graph(rng, n, 40000)
    bgv.validate_edges(dev(e), n)                       # in range: no error
    bgv.validate_edges(dev(np.zeros((0, 2), np.int32)), 1)
    for where, bad in (((0, 0), -1), ((39999, 1), n), ((12345, 0), 2**31 - 1), ((7, 1), -2**31)):
        eb = e.copy()
        eb[where] = bad
        with pytest.raises(ValueError):
            bgv.validate_edges(dev(eb), n)
    flag = torch.empty(1, dtype=torch.int32, device="cuda")
    eb = e.copy()
    eb[100, 0] = n
    st = L.bgv_validate_edges(n, eb.shape[0], L.C.c_void_p(dev(eb).data_ptr()), L.C.c_void_p(flag.data_ptr()), None)
    assert st == L.BGV_E_RANGE and int(flag) == 1


def test_range_errors_stop_before_indexing(bgv, monkeypatch):
    rng = np.random.default_rng(4)
    n = 3000
    e = graphgen.random_tiny_graph(rng, n, 20000)
    eb = e.copy()
    eb[777, 1] = n
    c1 = graphgen.hash_coeffs(4, 5)
    c2 = graphgen.hash_coeffs(4, 6)
    # Python-side check (the default)
    err, names = _only_checks_ran(lambda: bgv.community(dev(eb), n, 16, 2, 2, 256))
    assert isinstance(err, ValueError) and all(_is_check(k) for k in names) and names, names
    # library-side check through the environment, every entry point that takes ids
    monkeypatch.setenv("BGV_CHECK", "1")
    for method in (1, 2):
        err, names = _only_checks_ran(lambda: bgv.community(dev(eb), n, 16, 2, 2, 256, method=method, check=False))
        assert isinstance(err, L.BgvError) and "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names), names
    err, names = _only_checks_ran(lambda: bgv.community_passes(dev(eb), n, 16, 2, 2, 256, check=False))
    assert "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names)
    lab, deg, _ = bgv.community(dev(e), n, 16, 2, 2, 256, check=False)   # valid input passes
    err, names = _only_checks_ran(lambda: bgv.supergraph(dev(eb), lab, deg, 4, 1024, c1, c2, check=False))
    assert "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names)
    lab_bad = lab.clone()
    lab_bad[5] = -1
    err, names = _only_checks_ran(lambda: bgv.supergraph(dev(e), lab_bad, deg, 4, 1024, c1, c2, check=False))
    assert "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names)
    sg = bgv.supergraph(dev(e), lab, deg, 4, 1024, c1, c2, check=False)
    K = sg["K"]
    se_bad = sg["superedges"].clone()
    se_bad[0, 1] = K
    pos = torch.rand((K, 2), device="cuda")
    err, names = _only_checks_ran(lambda: bgv.fa2_layout(se_bad, pos.clone(), 3, exact=False))
    assert "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names)
    err, names = _only_checks_ran(lambda: bgv.fa2_energy(se_bad, pos))
    assert "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names)
    err, names = _only_checks_ran(lambda: bgv.fa2_grad(se_bad, pos))
    assert "BGV_E_RANGE" in str(err) and all(_is_check(k) for k in names)
    p1, _, _ = bgv.fa2_layout(sg["superedges"], pos.clone(), 3, exact=False)
    monkeypatch.delenv("BGV_CHECK")
    p2, _, _ = bgv.fa2_layout(sg["superedges"], pos.clone(), 3, exact=False)
    assert torch.equal(p1, p2)  # the check changes nothing on valid input


def test_batched_offsets_and_local_ids(bgv):
    rng = np.random.default_rng(5)
    graphs = [(300, graphgen.random_tiny_graph(rng, 300, 1500)), (50, graphgen.random_tiny_graph(rng, 50, 200)),
              (800, graphgen.random_tiny_graph(rng, 800, 4000))]
    wl = dict(threshold=8, passes=1, growth=2, chunk=256, rows=4, cols=1024, fa2_iters=5, kr=1.0, kg=1.0, tau=1.0,
              ks=0.1, ksmax=10.0)
    c1 = graphgen.hash_coeffs(4, 7)
    c2 = graphgen.hash_coeffs(4, 8)
    d = torch.device("cuda")
    edges, noff, eoff, noff_h, _ = bgv.pack_graphs(graphs, d)
    n_total = int(noff_h[-1])
    pos = torch.rand((n_total, 2), device=d)
    ok = bgv.batched(edges, noff, eoff, n_total, wl, c1, c2, pos.clone(), check=True)
    ref = bgv.batched(edges, noff, eoff, n_total, wl, c1, c2, pos.clone())
    assert torch.equal(ok["pos"], ref["pos"]) and torch.equal(ok["labels"], ref["labels"])
    # an id valid for the whole batch but not for its own (second, 50-node) graph
    eb = edges.clone()
    eb[1500 + 3, 0] = 60
    err, names = _only_checks_ran(lambda: bgv.batched(eb, noff, eoff, n_total, wl, c1, c2, pos.clone(), check=True))
    assert isinstance(err, ValueError) and all(_is_check(k) for k in names), names
    nb = noff.clone()
    nb[2] = nb[1] - 1  # decreasing offsets
    err, names = _only_checks_ran(lambda: bgv.batched(edges, nb, eoff, n_total, wl, c1, c2, pos.clone(), check=True))
    assert isinstance(err, ValueError) and all(_is_check(k) for k in names), names
    order = torch.tensor([2, 0, 3], dtype=torch.int32, device=d)
    err, names = _only_checks_ran(lambda: bgv.batched(edges, noff, eoff, n_total, wl, c1, c2, pos.clone(),
                                                      order=order, check=True))
    assert isinstance(err, ValueError) and all(_is_check(k) for k in names), names

"""Community detection captured in a HIP graph: both methods enqueue only kernels (no
host synchronisation, no memset nodes), so a captured call replays to the eager result,
also with unrelated eager work and synchronisations between replays."""
import ctypes as C

import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bgv():
    import paper_2108_00529_amd as b
    return b


@pytest.mark.parametrize("method", [1, 2])
def test_captured_community_replays_match_eager(bgv, method):
    from paper_2108_00529_amd import _lib as L
    n, D, P, f, B = 20_000, 16, 3, 2, 16_384
    e, _ = graphgen.lfr_style(n, 200_000, 2.3, 1.5, 0.2, 91)
    dev = torch.device("cuda")
    ed = torch.from_numpy(e).to(dev)
    p = L.CdParams(D, P, f, method, B)
    ws = torch.empty(L.bgv_community_workspace(n, ed.shape[0], C.byref(p)), dtype=torch.uint8, device=dev)

    def run():
        return bgv.community(ed, n, D, P, f, B, volume=True, method=method, ws=ws, check=False)

    eager = [t.clone() for t in run()]
    torch.cuda.synchronize()
    lab_r, cnt_r = oracle.bs_community(n, e, D, P, f, B)
    np.testing.assert_array_equal(eager[0].cpu().numpy(), lab_r)
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
        for a, b in zip(cap, eager):
            assert torch.equal(a, b), (method, rep)
        junk = torch.randn(1 << 20, device=dev)  # unrelated eager work between replays
        (junk * 2).sum().item()


@pytest.mark.parametrize("exact", [False, True])
def test_captured_layout_replays_match_eager(bgv, exact):
    """ForceAtlas2 iterations (Barnes-Hut and exact) captured in a HIP graph: each
    replay restarts from the same positions and ends on the eager positions."""
    rng = np.random.default_rng(93)
    K = 6000
    se = np.array(sorted({(min(a, b), max(a, b)) for a, b in rng.integers(0, K, (30_000, 2)).tolist() if a != b}),
                  np.int32)
    dev = torch.device("cuda")
    sed = torch.from_numpy(se).to(dev)
    pos0 = torch.from_numpy(graphgen.initial_positions(K, 7)).to(dev)
    pos, fprev = pos0.clone(), torch.zeros_like(pos0)
    speed = torch.ones(1, dtype=torch.float32, device=dev)

    def run():
        pos.copy_(pos0)
        fprev.zero_()
        speed.fill_(1.0)
        bgv.fa2_layout(sed, pos, 30, exact=exact, theta=1.2, fprev=fprev, speed=speed)

    run()
    torch.cuda.synchronize()
    eager = pos.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(pos, eager), (exact, rep)
        junk = torch.randn(1 << 20, device=dev)
        (junk * 2).sum().item()

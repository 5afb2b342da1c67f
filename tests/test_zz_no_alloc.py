"""The allocation-free layout entry point (bgv_fa2_layout_static) against the workspace
entry point (bgv_fa2_layout): same kernels, so the same bits, on two calls in a row
whose second input is smaller (the shared scratch array keeps the first call's
contents, which the second must not read), for Barnes-Hut and exact repulsion; and a
size beyond the scratch array rejected before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bgv():
    import paper_2108_00529_amd as b
    return b


def _graph(n, m, seed):
    e, _ = graphgen.lfr_style(n, m, 2.3, 1.5, 0.2, seed)
    e = e[e[:, 0] != e[:, 1]]
    return e


def _both(bgv, e, pos0, iters, exact, weighted):
    dev = torch.device("cuda")
    K = pos0.shape[0]
    se = torch.from_numpy(e).to(dev)
    aw = None
    if weighted:
        rng = np.random.default_rng(K)
        aw = torch.from_numpy(rng.uniform(0.5, 3.0, e.shape[0]).astype(np.float32)).to(dev)
    outs = []
    for static in (False, True):
        pos = torch.from_numpy(pos0).to(dev)
        fprev = torch.zeros((K, 2), dtype=torch.float32, device=dev)
        speed = torch.ones(1, dtype=torch.float32, device=dev)
        if static:
            bgv.api.fa2_layout_static(se, pos, fprev, speed, iters, exact=exact, theta=1.2, attr_w=aw)
        else:
            bgv.fa2_layout(se, pos, iters, exact=exact, theta=1.2, attr_w=aw, fprev=fprev, speed=speed)
        torch.cuda.synchronize()
        outs.append((pos.cpu().numpy(), fprev.cpu().numpy(), speed.cpu().numpy()))
    return outs


@pytest.mark.parametrize("exact", [False, True])
def test_static_layout_equals_workspace_layout(bgv, exact):
    # first a larger graph, then a smaller one: the second call finds the first call's
    # data in the scratch array
    # (above 19,456 supernodes the attraction is column-blocked: ids, then weights)
    for n, m, seed, iters, weighted in [(30_000, 200_000, 11, 25, False), (24_000, 150_000, 13, 15, True),
                                        (3_000, 15_000, 12, 40, True)]:
        e = _graph(n, m, seed)
        pos0 = graphgen.initial_positions(n, seed + 100)
        print(f"[no-alloc] exact={exact} K={n} E={e.shape[0]} iters={iters}", flush=True)
        ref, got = _both(bgv, e, pos0, iters, exact, weighted)
        for a, b, name in zip(ref, got, ("pos", "fprev", "speed")):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (exact, n, name)
        assert np.isfinite(got[0]).all()


def test_static_layout_continues_a_run(bgv):
    """The state a static call leaves continues exactly like the workspace path's:
    20 + 30 iterations through the static entry point equal 50 through the other."""
    dev = torch.device("cuda")
    n = 8_000
    e = _graph(n, 60_000, 21)
    pos0 = graphgen.initial_positions(n, 121)
    se = torch.from_numpy(e).to(dev)
    pos = torch.from_numpy(pos0).to(dev)
    fprev = torch.zeros((n, 2), dtype=torch.float32, device=dev)
    speed = torch.ones(1, dtype=torch.float32, device=dev)
    bgv.api.fa2_layout_static(se, pos, fprev, speed, 20, exact=False)
    bgv.api.fa2_layout_static(se, pos, fprev, speed, 30, exact=False)
    ref = torch.from_numpy(pos0).to(dev)
    bgv.fa2_layout(se, ref, 50, exact=False)
    torch.cuda.synchronize()
    assert torch.equal(pos, ref)


def test_static_layout_rejects_sizes_beyond_the_scratch(bgv):
    from paper_2108_00529_amd import _lib as L
    dev = torch.device("cuda")
    K = 65_536
    pos = torch.zeros((K, 2), dtype=torch.float32, device=dev)
    fprev = torch.zeros_like(pos)
    speed = torch.ones(1, dtype=torch.float32, device=dev)
    E = 2_000_000
    se = torch.zeros((E, 2), dtype=torch.int32, device=dev)
    p = L.Fa2Params(1, 0, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)
    assert L.bgv_fa2_workspace(K, E, C.byref(p)) > L.BGV_FA2_STATIC_SCRATCH_BYTES
    st = L.bgv_fa2_layout_static(K, E, C.c_void_p(se.data_ptr()), None, None, C.c_void_p(pos.data_ptr()),
                                 C.c_void_p(fprev.data_ptr()), C.c_void_p(speed.data_ptr()), C.byref(p), None)
    assert st == -1
    assert b"more than" in L.bgv_last_error()
    torch.cuda.synchronize()
    assert float(speed.item()) == 1.0 and not pos.any()

"""GPU drawing attributes of the supernodes (Section 4.1 radius, Section 4.3 colour
groups) against the oracle: groups bit-exact, radii bit-exact (both sides convert the
size to float32 and take the correctly rounded square root)."""
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


def check(bgv, sizes):
    sizes = np.asarray(sizes, dtype=np.uint32)
    g, r = bgv.draw_supernodes(torch.from_numpy(sizes.view(np.int32)).cuda())
    g_ref, r_ref = oracle.draw_supernodes(sizes)
    np.testing.assert_array_equal(g.cpu().numpy(), g_ref)
    np.testing.assert_array_equal(r.cpu().numpy().view(np.uint32), r_ref.view(np.uint32))


def test_draw_hand_cases(bgv):
    check(bgv, [6, 1, 1, 1, 1])
    check(bgv, [1] * 20)
    check(bgv, [3, 3])
    check(bgv, [5])
    check(bgv, [0, 0, 0])
    check(bgv, [2**32 - 1, 2**32 - 1, 7])  # running totals past 2^32


@pytest.mark.parametrize("K", [2, 37, 1000, 70000, 300000])
def test_draw_random(bgv, K):
    rng = np.random.default_rng(K)
    sizes = (rng.pareto(1.5, K) * 10).astype(np.uint64).clip(0, 2**32 - 1).astype(np.uint32)
    sizes[rng.random(K) < 0.1] = 0
    sizes[: K // 3] = sizes[0]  # ties
    check(bgv, sizes)


def test_draw_planted_supergraph(bgv):
    wl = graphgen.WORKLOADS["planted_2k"]
    e, _ = graphgen.make_graph("planted_2k")
    c1 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"])
    c2 = graphgen.hash_coeffs(wl["rows"], wl["sketch_seed"] ^ 0x9E3779B97F4A7C15)
    ed = torch.from_numpy(e).cuda()
    lab, deg, _ = bgv.community(ed, wl["n"], wl["threshold"], wl["passes"], wl["growth"], wl["chunk"])
    sg = bgv.supergraph(ed, lab, deg, wl["rows"], wl["cols"], c1, c2)
    sizes = sg["super_size"][: sg["K"]].cpu().numpy().view(np.uint32)
    check(bgv, sizes)

"""Community detection resumed from a saved state, and node-relabelling equivariance,
on the GPU.

Resume (Section 3.2.1 / Algorithm 3: the rounds share one state, labels and degree
counters): a run of P passes and a run stopped after P1 passes, continued from its
labels by bgv_community_resume, give the same labels, degrees and volumes bit for bit,
for every chunk-by-chunk form (bucketed, per-node atomic above 2^24 nodes), the
back-pointer method, the tie rule and the volume rule, and both equal the oracle's.

Equivariance: the rule reads counters, labels and stream positions, never the value of
an id, so renaming the nodes by a permutation pi renames the result: labels'[pi v] =
pi(labels[v]), degree'[pi v] = degree[v], volume'[pi c] = volume[c]."""
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


def say(*a):
    print("[resume]", *a, flush=True)


def host(t):
    return t.cpu().numpy()


def check_resume(bgv, n, e, D, P, f, B, method, tie=0, rule=0):
    dev = torch.device("cuda")
    ed = torch.from_numpy(np.ascontiguousarray(e, dtype=np.int32).reshape(-1, 2)).to(dev)
    lab_r, cnt_r = oracle.bs_community(n, e, D, P, f, B, tie=tie, rule=rule)
    deg_r, vol_r = oracle.degree_volume(lab_r, cnt_r, P)
    full = bgv.community(ed, n, D, P, f, B, volume=True, method=method, tie=tie, rule=rule)
    _, _, _, rows = bgv.community_passes(ed, n, D, P, f, B, method=method, tie=tie, rule=rule)
    np.testing.assert_array_equal(host(full[0]), lab_r)
    for done in range(1, P):
        say(f"n={n} m={e.shape[0]} D={D} P={P} chunk={B} method={method} tie={tie} rule={rule} done={done}")
        saved = rows[done - 1].clone()
        lab, deg, vol = bgv.community_resume(ed, n, saved, done, D, P, f, B, volume=True, method=method, tie=tie,
                                             rule=rule)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(lab), lab_r, err_msg=f"labels, resumed after {done}")
        np.testing.assert_array_equal(host(deg), deg_r, err_msg=f"degree, resumed after {done}")
        np.testing.assert_array_equal(host(vol), vol_r, err_msg=f"volume, resumed after {done}")
        # the saved state is only read
        np.testing.assert_array_equal(host(saved), host(rows[done - 1]))


@pytest.mark.parametrize("method", [1, 2])
def test_resume_equals_full_run(bgv, method):
    e, _ = graphgen.lfr_style(20_000, 200_000, 2.3, 1.5, 0.2, 31)
    check_resume(bgv, 20_000, e, 16, 4, 2, 4096, method)
    check_resume(bgv, 20_000, e, 16, 3, 2, 70_001, method)
    check_resume(bgv, 20_000, e, 16, 6, 2, 50_000, method)  # passes 2..5 decided in pass 1 of a full run
    check_resume(bgv, 20_000, e, 16, 3, 2, 4096, method, tie=1)


def test_resume_sequential_rule_and_hubs(bgv):
    rng = np.random.default_rng(5)
    n = 3 * 4096 + 77
    e = rng.integers(0, n, size=(60_000, 2), dtype=np.int64).astype(np.int32)
    e[::7, 0] = 5  # a hub in every chunk
    e[::11, 1] = e[::11, 0]  # self-loops
    check_resume(bgv, n, e, 24, 3, 2, 1, 0)      # chunk 1: the sequential rule (back pointers)
    check_resume(bgv, n, e, 24, 3, 2, 1025, 1)   # ragged tiles and several buckets


def test_resume_volume_rule(bgv):
    e, _ = graphgen.lfr_style(5_000, 40_000, 2.3, 1.5, 0.2, 33)
    check_resume(bgv, 5_000, e, 32, 3, 2, 1000, 1, rule=1)
    check_resume(bgv, 5_000, e, 32, 2, 2, 17, 1, rule=1)


def test_resume_atomic_form_above_bucket_limit(bgv):
    n = (1 << 24) + 5
    rng = np.random.default_rng(7)
    ids = rng.integers(0, n, size=3000)
    e = np.stack([ids[rng.integers(0, 3000, 40_000)], ids[rng.integers(0, 3000, 40_000)]], 1).astype(np.int32)
    check_resume(bgv, n, e, 20, 3, 2, 5000, 1)


def test_resume_empty_stream(bgv):
    dev = torch.device("cuda")
    n = 100
    lab0 = torch.from_numpy(np.random.default_rng(1).integers(0, n, n).astype(np.int32)).to(dev)
    ed = torch.zeros((0, 2), dtype=torch.int32, device=dev)
    lab, deg, vol = bgv.community_resume(ed, n, lab0, 1, 4, 3, 2, 16, volume=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(lab), host(lab0))
    assert not host(deg).any() and not host(vol).any()


def test_resume_rejects_bad_state(bgv):
    dev = torch.device("cuda")
    e, _ = graphgen.lfr_style(2_000, 10_000, 2.3, 1.5, 0.2, 3)
    ed = torch.from_numpy(e).to(dev)
    lab0 = torch.arange(2_000, dtype=torch.int32, device=dev)
    for done in (0, 3, -1):
        with pytest.raises(bgv.BgvError):
            bgv.community_resume(ed, 2_000, lab0, done, 8, 3, 2, 1000)
    bad = lab0.clone()
    bad[17] = 2_000  # an id outside [0, n): the opt-in device check reports it
    with pytest.raises(bgv.BgvError, match="RANGE"):
        bgv.community_resume(ed, 2_000, bad, 1, 8, 3, 2, 1000, check=True)


def relabel_check(bgv, n, e, D, P, f, B, method, seed, tie=0, rule=0):
    dev = torch.device("cuda")
    pi = np.random.default_rng(seed).permutation(n).astype(np.int32)
    e2 = pi[e]
    a = bgv.community(torch.from_numpy(e).to(dev), n, D, P, f, B, volume=True, method=method, tie=tie, rule=rule)
    b = bgv.community(torch.from_numpy(np.ascontiguousarray(e2)).to(dev), n, D, P, f, B, volume=True,
                      method=method, tie=tie, rule=rule)
    la, da, va = (host(t) for t in a)
    lb, db, vb = (host(t) for t in b)
    say(f"relabel n={n} m={e.shape[0]} chunk={B} method={method} tie={tie} rule={rule}")
    np.testing.assert_array_equal(lb[pi], pi[la])
    np.testing.assert_array_equal(db[pi], da)
    np.testing.assert_array_equal(vb[pi], va)
    assert len(np.unique(la)) < n  # communities formed, so the check is not vacuous


@pytest.mark.parametrize("method", [1, 2])
def test_node_relabelling_equivariance(bgv, method):
    e, _ = graphgen.lfr_style(30_000, 300_000, 2.3, 1.5, 0.2, 41)
    relabel_check(bgv, 30_000, e, 32, 3, 2, 8192, method, 1)
    relabel_check(bgv, 30_000, e, 32, 3, 2, 8192, method, 2, tie=1)
    if method == 2:
        relabel_check(bgv, 30_000, e, 32, 2, 2, 1, method, 3)  # the sequential rule


def test_node_relabelling_equivariance_volume_rule_and_atomic_form(bgv):
    e, _ = graphgen.lfr_style(5_000, 40_000, 2.3, 1.5, 0.2, 43)
    relabel_check(bgv, 5_000, e, 32, 2, 2, 999, 1, 4, rule=1)
    n = (1 << 24) + 9
    rng = np.random.default_rng(8)
    ids = rng.integers(0, n, size=5000)
    e = np.stack([ids[rng.integers(0, 5000, 50_000)], ids[rng.integers(0, 5000, 50_000)]], 1).astype(np.int32)
    relabel_check(bgv, n, e, 24, 2, 2, 4096, 1, 5)

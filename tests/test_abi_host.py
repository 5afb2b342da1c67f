"""Host-only checks of the C ABI: the library loads, exports every symbol the header
declares, answers workspace queries and rejects bad arguments before any HIP call
(so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]

L = pytest.importorskip("paper_2108_00529_amd._lib", reason="libbgv.so not built")


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bgv_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 11
    for name in names:
        assert hasattr(L.lib, name), name
    assert sorted(L.EXPORTED) == names


def test_status_strings():
    assert L.bgv_status_string(0) == b"BGV_OK"
    assert L.bgv_status_string(-1) == b"BGV_E_INVALID"
    assert L.bgv_status_string(-3) == b"BGV_E_WORKSPACE"
    assert L.bgv_status_string(-4) == b"BGV_E_HIP"


def test_community_validation_and_workspace():
    p = L.CdParams(16, 1, 2, 0, 4096)
    ws = L.bgv_community_workspace(2000, 10000, C.byref(p))
    assert ws >= 2000 * 8 + 4096 * 16  # records + a 4096-edge chunk of grouped entries (16 B per edge)
    ws2 = L.bgv_community_workspace(2000, 100, C.byref(p))  # chunk clipped to m: one tile
    assert ws2 < ws
    p3 = L.CdParams(16, 3, 2, 0, 4096)
    assert L.bgv_community_workspace(2000, 10000, C.byref(p3)) >= ws + 8 * 10000  # pass-0 counters per edge
    big = L.bgv_community_workspace((1 << 24) + 1, 100, C.byref(p))  # per-node atomic form
    assert big >= ((1 << 24) + 1) * 16
    assert L.bgv_community_workspace(10, 10, C.byref(L.CdParams(1, 1, 2, 0, 1, 1, 0))) > 0  # tie rule 1
    # volume rule: per-node records, V and a chunk of proposals, whatever the method choice
    vr = L.bgv_community_workspace(5000, 100000, C.byref(L.CdParams(8, 2, 2, 0, 1, 0, 1)))
    assert vr == L.bgv_community_workspace(5000, 100000, C.byref(L.CdParams(8, 2, 2, 1, 1, 0, 1)))
    assert 5000 * 24 <= vr <= 5000 * 24 + 4096
    # methods: back-pointer resolution needs more workspace; automatic picks it past 64 chunk steps
    m1 = L.bgv_community_workspace(2000, 10000, C.byref(L.CdParams(16, 3, 2, 1, 100)))
    m2 = L.bgv_community_workspace(2000, 10000, C.byref(L.CdParams(16, 3, 2, 2, 100)))
    assert 0 < m1 < m2 and m2 >= 48 * 10000 + 3 * 10000 * 40
    assert L.bgv_community_workspace(2000, 10000, C.byref(L.CdParams(16, 3, 2, 0, 100))) == m2   # 300 steps
    assert L.bgv_community_workspace(2000, 10000, C.byref(L.CdParams(16, 3, 2, 0, 2000))) == \
        L.bgv_community_workspace(2000, 10000, C.byref(L.CdParams(16, 3, 2, 1, 2000)))         # 15 steps
    # passes * m must stay below 2^31 for method 2 (automatic then keeps method 1)
    assert L.bgv_community_workspace(10, 2**30, C.byref(L.CdParams(4, 2, 2, 2, 1))) == 0
    assert L.bgv_community_workspace(10, 2**30, C.byref(L.CdParams(4, 2, 2, 0, 1))) == \
        L.bgv_community_workspace(10, 2**30, C.byref(L.CdParams(4, 2, 2, 1, 1)))
    for bad in [L.CdParams(-1, 1, 2, 0, 1), L.CdParams(1, 0, 2, 0, 1), L.CdParams(1, 1, 0, 0, 1),
                L.CdParams(1, 1, 2, 0, 0), L.CdParams(1, 1, 2, 7, 1), L.CdParams(1, 1, 2, 3, 1),
                L.CdParams(1, 1, 2, -1, 1), L.CdParams(1, 1, 2, 0, 1, 2, 0), L.CdParams(1, 1, 2, 0, 1, -1, 0),
                L.CdParams(1, 1, 2, 0, 1, 0, 5), L.CdParams(1, 1, 2, 0, 1, 0, 2),
                L.CdParams(1, 1, 2, 0, 1, 1, 1), L.CdParams(1, 1, 2, 2, 1, 0, 1)]:
        assert L.bgv_community_workspace(10, 10, C.byref(bad)) == 0
        assert L.bgv_community(10, 10, C.c_void_p(1), C.byref(bad), C.c_void_p(1), C.c_void_p(1), None,
                               None, 0, None) == -1
    assert L.bgv_community(0, 10, C.c_void_p(1), C.byref(p), C.c_void_p(1), C.c_void_p(1), None, None, 0, None) == -1
    assert L.bgv_community(10, -1, C.c_void_p(1), C.byref(p), C.c_void_p(1), C.c_void_p(1), None, None, 0, None) == -1
    assert L.bgv_community(10, 2**31, C.c_void_p(1), C.byref(p), C.c_void_p(1), C.c_void_p(1), None, None, 0,
                           None) == -1
    # null outputs
    assert L.bgv_community(10, 5, C.c_void_p(1), C.byref(p), None, C.c_void_p(1), None, None, 0, None) == -1
    # workspace too small / missing / misaligned -> BGV_E_WORKSPACE, before any HIP call
    need = L.bgv_community_workspace(10, 5, C.byref(p))
    assert L.bgv_community(10, 5, C.c_void_p(256), C.byref(p), C.c_void_p(256), C.c_void_p(256), None,
                           None, 0, None) == -3
    assert L.bgv_community(10, 5, C.c_void_p(256), C.byref(p), C.c_void_p(256), C.c_void_p(256), None,
                           C.c_void_p(512), need - 1, None) == -3
    assert L.bgv_community(10, 5, C.c_void_p(256), C.byref(p), C.c_void_p(256), C.c_void_p(256), None,
                           C.c_void_p(513), need, None) == -3
    assert b"workspace" in L.bgv_last_error()
    # per-pass labels: same checks, and the rows buffer is required
    assert L.bgv_community_passes(10, 5, C.c_void_p(256), C.byref(p), C.c_void_p(256), C.c_void_p(256), None,
                                  None, C.c_void_p(512), need, None) == -1
    assert b"bgv_community_passes" in L.bgv_last_error()
    assert L.bgv_community_passes(0, 5, C.c_void_p(256), C.byref(p), C.c_void_p(256), C.c_void_p(256), None,
                                  C.c_void_p(256), C.c_void_p(512), need, None) == -1
    assert L.bgv_community_passes(10, 5, C.c_void_p(256), C.byref(p), C.c_void_p(256), C.c_void_p(256), None,
                                  C.c_void_p(256), C.c_void_p(512), need - 1, None) == -3


def test_community_resume_validation():
    """Rejected before any HIP call: a pass count outside [1, passes), a null or aliased
    saved state, and the arguments bgv_community rejects."""
    p = L.CdParams(16, 3, 2, 0, 4096)
    one, two = C.c_void_p(256), C.c_void_p(512)
    ws = 1 << 30
    for done in (0, 3, -2):
        assert L.bgv_community_resume(10, 5, one, C.byref(p), done, one, two, one, None, one, ws, None) == -1
    assert L.bgv_community_resume(10, 5, one, C.byref(p), 1, None, two, one, None, one, ws, None) == -1
    assert L.bgv_community_resume(10, 5, one, C.byref(p), 1, two, two, one, None, one, ws, None) == -1  # aliased
    assert L.bgv_community_resume(0, 5, one, C.byref(p), 1, one, two, one, None, one, ws, None) == -1
    assert L.bgv_community_resume(10, 5, one, None, 1, one, two, one, None, one, ws, None) == -1
    one_pass = L.CdParams(16, 1, 2, 0, 4096)  # nothing to resume
    assert L.bgv_community_resume(10, 5, one, C.byref(one_pass), 1, one, two, one, None, one, ws, None) == -1
    # the workspace is bgv_community's
    need = L.bgv_community_workspace(10, 5, C.byref(p))
    assert L.bgv_community_resume(10, 5, one, C.byref(p), 1, one, two, one, None, one, need - 1, None) == -3


def test_supergraph_validation():
    import numpy as np
    coef = np.zeros((8, 3), np.uint64)
    cp = coef.ctypes.data_as(C.c_void_p)
    ok = L.SketchParams(4, 1024, cp, cp)
    assert L.bgv_supergraph_workspace(100, 1000, C.byref(ok)) > 0
    for bad in [L.SketchParams(0, 1024, cp, cp), L.SketchParams(9, 1024, cp, cp), L.SketchParams(4, 0, cp, cp),
                L.SketchParams(4, 16, None, cp), L.SketchParams(4, 16, cp, None)]:
        assert L.bgv_supergraph_workspace(100, 1000, C.byref(bad)) == 0
    K, E = L.i32(0), L.i64(0)
    one = C.c_void_p(256)
    assert L.bgv_supergraph(100, 1000, one, one, one, C.byref(bad), C.byref(K), C.byref(E), one, one, None, one,
                            one, None, one, one, one, 1 << 30, None) == -1
    assert L.bgv_supergraph(100, 1000, one, one, one, C.byref(ok), C.byref(K), C.byref(E), one, one, None, one,
                            one, None, None, one, one, 1 << 30, None) == -1   # M1 required


def test_fa2_validation():
    ok = L.Fa2Params(10, 1, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)
    assert L.bgv_fa2_workspace(100, 300, C.byref(ok)) > 0
    bh = L.Fa2Params(10, 0, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)
    assert L.bgv_fa2_workspace(100, 300, C.byref(bh)) > L.bgv_fa2_workspace(100, 300, C.byref(ok))
    for bad in [L.Fa2Params(-1, 1, 1.2, 1, 1, 1, .1, 10), L.Fa2Params(1, 2, 1.2, 1, 1, 1, .1, 10),
                L.Fa2Params(1, 0, -1.0, 1, 1, 1, .1, 10), L.Fa2Params(1, 1, 1.2, 1, 1, 0.0, .1, 10),
                L.Fa2Params(1, 1, 1.2, 1, 1, 1, .1, 0.0)]:
        assert L.bgv_fa2_workspace(100, 300, C.byref(bad)) == 0
    one = C.c_void_p(256)
    assert L.bgv_fa2_workspace(0, 3, C.byref(ok)) == 0
    assert L.bgv_fa2_layout(0, 3, one, None, None, one, one, one, C.byref(ok), one, 1 << 30, None) == -1
    assert L.bgv_fa2_layout(10, 3, one, None, None, None, one, one, C.byref(ok), one, 1 << 30, None) == -1
    assert L.bgv_fa2_energy_workspace(0, 0) == 0
    assert L.bgv_fa2_energy_workspace(10, 20) > 0
    assert L.bgv_fa2_energy(0, 0, None, None, None, one, 1.0, 1.0, one, one, 1 << 20, None) == -1
    assert L.bgv_fa2_grad(10, 0, None, None, None, one, 1.0, 1.0, None, None, one, 1 << 20, None) == -1


def test_fa2_layout_static_validation():
    """The allocation-free layout rejects, before any HIP call, what bgv_fa2_layout
    rejects and any size whose workspace would exceed its fixed scratch array."""
    ok = L.Fa2Params(10, 0, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)
    one = C.c_void_p(256)
    assert L.bgv_fa2_layout_static(0, 3, one, None, None, one, one, one, C.byref(ok), None) == -1
    assert L.bgv_fa2_layout_static(10, 3, one, None, None, None, one, one, C.byref(ok), None) == -1
    assert L.bgv_fa2_layout_static(10, 3, None, None, None, one, one, one, C.byref(ok), None) == -1
    bad = L.Fa2Params(10, 2, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)
    assert L.bgv_fa2_layout_static(10, 3, one, None, None, one, one, one, C.byref(bad), None) == -1
    K, E = 65_536, 2_000_000
    assert L.bgv_fa2_workspace(K, E, C.byref(ok)) > L.BGV_FA2_STATIC_SCRATCH_BYTES
    assert L.bgv_fa2_layout_static(K, E, one, None, None, one, one, one, C.byref(ok), None) == -1
    assert b"more than" in L.bgv_last_error()
    assert L.bgv_fa2_workspace(65_536, 720_000, C.byref(ok)) <= L.BGV_FA2_STATIC_SCRATCH_BYTES
    assert L.bgv_fa2_workspace(131_072, 280_000, C.byref(ok)) <= L.BGV_FA2_STATIC_SCRATCH_BYTES


def test_batched_validation():
    """Rejected on the host before any HIP call: community options the batched form
    does not run (volume rule, back-pointer method, tie values other than 0/1), layout
    and launch parameters, null outputs, and a small or misaligned workspace."""
    import numpy as np
    coef = np.zeros((4, 3), np.uint64)
    sk = L.SketchParams(4, 1024, coef.ctypes.data_as(C.c_void_p), coef.ctypes.data_as(C.c_void_p))
    fa = L.Fa2Params(10, 1, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)
    G, n, m = 2, 20, 40
    need = L.bgv_batched_workspace(G, n, m)
    assert need > 0 and L.bgv_batched_workspace(0, n, m) == 0
    one = C.c_void_p(256)

    def call(cd=L.CdParams(16, 1, 2, 0, 256), sk=sk, fa=fa, wg=0, big_k=0, labels=one, ws=C.c_void_p(512), nbytes=need):
        return L.bgv_batched(G, n, m, one, one, None, one, C.byref(cd), C.byref(sk), C.byref(fa), wg, big_k, labels,
                             one, one, one, one, one, one, one, one, one, one, ws, nbytes, None)

    for cd in [L.CdParams(16, 1, 2, 0, 256, 0, 1), L.CdParams(16, 1, 2, 2, 256), L.CdParams(16, 1, 2, 1, 256),
               L.CdParams(16, 1, 2, 0, 256, 2, 0), L.CdParams(16, 0, 2, 0, 256)]:
        assert call(cd=cd) == -1
    assert call(fa=L.Fa2Params(10, 0, 1.2, 1.0, 1.0, 1.0, 0.1, 10.0)) == -1        # Barnes-Hut: not batched
    assert call(sk=L.SketchParams(4, 4096, coef.ctypes.data_as(C.c_void_p), coef.ctypes.data_as(C.c_void_p))) == -1
    assert call(wg=128) == -1 and call(big_k=-1) == -1
    assert call(labels=None) == -1
    assert b"null pointer" in L.bgv_last_error()
    assert call(nbytes=need - 1) == -3 and call(ws=C.c_void_p(513)) == -3
    assert call(cd=L.CdParams(16, 1, 2, 0, 256, 1, 0), nbytes=need - 1) == -3  # the tie rule is accepted


def test_draw_validation():
    assert L.bgv_draw_workspace(0) == 0 and L.bgv_draw_workspace(-5) == 0
    assert L.bgv_draw_workspace(1000) > 4 * 8 * 1000
    one = C.c_void_p(1)
    assert L.bgv_draw_supernodes(0, one, one, one, None, 0, None) == -1
    assert L.bgv_draw_supernodes(10, None, one, one, None, 0, None) == -1
    assert L.bgv_draw_supernodes(10, one, None, one, None, 0, None) == -1
    assert L.bgv_draw_supernodes(10, one, one, None, None, 0, None) == -1
    assert L.bgv_draw_supernodes(10, one, one, one, None, 0, None) == -3  # no workspace, before any HIP call


def test_checks_and_tree_export_validation():
    """The id check and the tree export reject bad arguments before any HIP call."""
    one = C.c_void_p(256)
    assert L.bgv_status_string(-2) == b"BGV_E_RANGE"
    assert L.bgv_validate_edges(0, 5, one, one, None) == -1
    assert L.bgv_validate_edges(10, -1, one, one, None) == -1
    assert L.bgv_validate_edges(10, 2**31, one, one, None) == -1
    assert L.bgv_validate_edges(10, 5, None, one, None) == -1
    assert L.bgv_validate_edges(10, 5, one, None, None) == -1
    assert L.bgv_bh_tree_workspace(0) == 0
    assert L.bgv_bh_tree_workspace(1000) > L.bgv_bh_tree_workspace(10) > 0
    need = L.bgv_bh_tree_workspace(100)
    args = [one] * 7  # pos, mass, codes, body, nodeA, nodeB, s0
    assert L.bgv_bh_tree(0, *args, one, need, None) == -1
    for k in range(7):
        a = list(args)
        a[k] = None
        assert L.bgv_bh_tree(100, *a, one, need, None) == -1
    assert L.bgv_bh_tree(100, *args, one, need - 1, None) == -3
    assert L.bgv_bh_tree(100, *args, C.c_void_p(257), need, None) == -3

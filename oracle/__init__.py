"""BigGraphVis CPU ORACLE -- test infrastructure, not part of the product.

Plain FP64 CPU implementation of the hot path of BigGraphVis (arXiv 2108.00529):
streaming community detection (Section 3.2, Algorithm 3), count-min sketch
supergraph (Section 3.3, Algorithm 2, Section 4.1) and ForceAtlas2 (Section 3.1,
Algorithm 1).  The arithmetic lives in ``bgv_oracle.c`` (built into
``liboracle.so`` with gcc); this module marshals numpy arrays.  It shares no code
with the GPU path and neither imports the other.  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may use it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .seq_scoda import seq_scoda  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bgv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, f64, u32 = C.c_int32, C.c_int64, C.c_double, C.c_uint32
        _lib.orc_bs_community.argtypes = [i32, i64, P, i32, i32, i32, i64, i32, i32, P, P]
        _lib.orc_bs_community.restype = C.c_int
        _lib.orc_degree_volume.argtypes = [i32, i32, P, P, P, P]
        _lib.orc_hash_key.argtypes = [P, u32, u32]
        _lib.orc_hash_key.restype = u32
        _lib.orc_hash_pair.argtypes = [P, u32, u32, u32]
        _lib.orc_hash_pair.restype = u32
        _lib.orc_supergraph.argtypes = [i32, i64, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P, P]
        _lib.orc_supergraph.restype = i64
        _lib.orc_fa2_mass.argtypes = [i32, i64, P, P]
        _lib.orc_fa2_forces.argtypes = [i32, P, P, i64, P, P, f64, f64, i32, f64, P]
        _lib.orc_fa2_layout.argtypes = [i32, i64, P, P, P, P, P, P, i32, i32, f64, f64, f64, f64, f64, f64]
        _lib.orc_fa2_energy.argtypes = [i32, P, P, i64, P, P, f64, f64]
        _lib.orc_fa2_energy.restype = f64
        _lib.orc_fa2_node_energy.argtypes = [i32, P, P, i64, P, P, f64, f64, i32]
        _lib.orc_fa2_node_energy.restype = f64
        _lib.orc_bh_codes.argtypes = [i32, P, P, P, P, P]
        _lib.orc_bh_tree_export.argtypes = [i32, P, P, P, P, P, P]
        _lib.orc_bh_tree_export.restype = i32
        _lib.orc_bh_repulsion.argtypes = [i32, P, P, f64, f64, P, P]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- community ----
def bs_community(n, edges, threshold, passes=1, growth=2, chunk=1, tie=0, rule=0):
    """Batch-synchronous streaming community detection (see bgv_oracle.c); tie = 1: on
    equal counters the edge's first endpoint joins the second's community; rule = 1:
    the community-volume rule of SCoDA instead of the paper's degree rule.
    Returns (labels int32[n], counters int32[n])."""
    lib = _load()
    e = _c(edges, np.int32).reshape(-1, 2)
    lab = np.empty(n, np.int32)
    cnt = np.empty(n, np.int32)
    rc = lib.orc_bs_community(n, e.shape[0], _p(e), threshold, passes, growth, chunk, int(tie), int(rule), _p(lab),
                              _p(cnt))
    if rc != 0:
        raise ValueError("orc_bs_community: bad arguments")
    return lab, cnt


def degree_volume(labels, counters, passes):
    """True degree d(v) = counter/passes and exact community volume (int64[n])."""
    lib = _load()
    n = labels.shape[0]
    lab = _c(labels, np.int32)
    cnt = _c(counters, np.int32)
    deg = np.empty(n, np.int32)
    vol = np.empty(n, np.int64)
    lib.orc_degree_volume(n, passes, _p(cnt), _p(lab), _p(deg), _p(vol))
    return deg, vol


def hash_key(coef_row, x, cols):
    return int(_load().orc_hash_key(_p(_c(coef_row, np.uint64)), x, cols))


def hash_pair(coef_row, a, b, cols):
    return int(_load().orc_hash_pair(_p(_c(coef_row, np.uint64)), a, b, cols))


def supergraph(n, edges, labels, degree, rows, cols, coef1, coef2):
    """Count-min-sketch supergraph.  Returns a dict with K, super_label, super_size,
    superedges (E,2) int32 sid pairs, se_weight (sketch), se_count (exact), M1, M2."""
    lib = _load()
    e = _c(edges, np.int32).reshape(-1, 2)
    m = e.shape[0]
    lab = _c(labels, np.int32)
    deg = _c(degree, np.int32)
    c1 = _c(coef1, np.uint64).reshape(rows, 3)
    c2 = _c(coef2, np.uint64).reshape(rows, 3)
    K = np.zeros(1, np.int32)
    sid = np.empty(n, np.int32)
    sl = np.empty(n, np.int32)
    ss = np.empty(n, np.uint32)
    se = np.empty((max(m, 1), 2), np.int32)
    sw = np.empty(max(m, 1), np.uint32)
    sc = np.empty(max(m, 1), np.uint32)
    M1 = np.empty((rows, cols), np.uint32)
    M2 = np.empty((rows, cols), np.uint32)
    E = lib.orc_supergraph(n, m, _p(e), _p(lab), _p(deg), rows, cols, _p(c1), _p(c2), _p(K), _p(sid),
                           _p(sl), _p(ss), _p(se), _p(sw), _p(sc), _p(M1), _p(M2))
    if E < 0:
        raise ValueError("orc_supergraph: bad arguments")
    k = int(K[0])
    return dict(K=k, sid_of_label=sid, super_label=sl[:k].copy(), super_size=ss[:k].copy(),
                superedges=se[:E].copy(), se_weight=sw[:E].copy(), se_count=sc[:E].copy(), M1=M1, M2=M2)


def modularity(edges, labels):
    """Newman modularity (Section 5.3, Eq. 2) of a multigraph, closed form:
    Q = sum_c [ 2 e_in(c) / 2m - (vol_c / 2m)^2 ], self-loops ignored."""
    e = np.asarray(edges).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    m = e.shape[0]
    if m == 0:
        return 0.0
    lab = np.asarray(labels)
    n = lab.shape[0]
    deg = np.bincount(e.ravel(), minlength=n).astype(np.float64)
    vol = np.bincount(lab, weights=deg, minlength=n)
    ein = np.bincount(lab[e[:, 0]][lab[e[:, 0]] == lab[e[:, 1]]], minlength=n).astype(np.float64)
    return float(np.sum(2.0 * ein / (2.0 * m) - (vol / (2.0 * m)) ** 2))


# ---------------------------------------------------------------- ForceAtlas2 --
def fa2_mass(K, superedges):
    lib = _load()
    se = _c(superedges, np.int32).reshape(-1, 2)
    mass = np.empty(K, np.float64)
    lib.orc_fa2_mass(K, se.shape[0], _p(se), _p(mass))
    return mass


def fa2_forces(pos, superedges, mass, aw=None, kr=1.0, kg=1.0, exact=True, theta=1.2):
    """Net ForceAtlas2 force (repulsion + attraction + gravity), FP64 (K,2)."""
    lib = _load()
    x = _c(pos, np.float64).reshape(-1, 2)
    K = x.shape[0]
    se = _c(superedges, np.int32).reshape(-1, 2)
    ms = _c(mass, np.float64)
    w = None if aw is None else _c(aw, np.float64)
    F = np.empty((K, 2), np.float64)
    lib.orc_fa2_forces(K, _p(x), _p(ms), se.shape[0], _p(se), None if w is None else _p(w),
                       kr, kg, 1 if exact else 0, theta, _p(F))
    return F


def fa2_layout(pos, superedges, mass=None, aw=None, iters=1, exact=True, theta=1.2, kr=1.0, kg=1.0,
               tau=1.0, ks=0.1, ksmax=10.0, Fprev=None, speed=1.0):
    """ForceAtlas2 iterations from positions ``pos``; returns (pos, Fprev, speed)."""
    lib = _load()
    x = np.array(pos, dtype=np.float64).reshape(-1, 2)
    K = x.shape[0]
    se = _c(superedges, np.int32).reshape(-1, 2)
    ms = fa2_mass(K, se) if mass is None else _c(mass, np.float64)
    w = None if aw is None else _c(aw, np.float64)
    Fp = np.zeros((K, 2), np.float64) if Fprev is None else np.array(Fprev, dtype=np.float64)
    sp = np.array([speed], np.float64)
    lib.orc_fa2_layout(K, se.shape[0], _p(se), None if w is None else _p(w), _p(ms), _p(x), _p(Fp), _p(sp),
                       iters, 1 if exact else 0, theta, kr, kg, tau, ks, ksmax)
    return x, Fp, float(sp[0])


def fa2_energy(pos, superedges, mass, aw=None, kr=1.0, kg=1.0):
    lib = _load()
    x = _c(pos, np.float64).reshape(-1, 2)
    se = _c(superedges, np.int32).reshape(-1, 2)
    ms = _c(mass, np.float64)
    w = None if aw is None else _c(aw, np.float64)
    return float(lib.orc_fa2_energy(x.shape[0], _p(x), _p(ms), se.shape[0], _p(se),
                                    None if w is None else _p(w), kr, kg))


def fa2_node_energy(pos, superedges, mass, i, aw=None, kr=1.0, kg=1.0):
    lib = _load()
    x = _c(pos, np.float64).reshape(-1, 2)
    se = _c(superedges, np.int32).reshape(-1, 2)
    ms = _c(mass, np.float64)
    w = None if aw is None else _c(aw, np.float64)
    return float(lib.orc_fa2_node_energy(x.shape[0], _p(x), _p(ms), se.shape[0], _p(se),
                                         None if w is None else _p(w), kr, kg, int(i)))


def bh_codes(pos32):
    """FP32 quantisation + Morton codes of the Barnes-Hut tree: (codes, s0, xmin, ymin)."""
    lib = _load()
    p = _c(pos32, np.float32).reshape(-1, 2)
    K = p.shape[0]
    codes = np.empty(K, np.uint32)
    s0 = np.zeros(1, np.float32)
    xm = np.zeros(1, np.float32)
    ym = np.zeros(1, np.float32)
    lib.orc_bh_codes(K, _p(p), _p(codes), _p(s0), _p(xm), _p(ym))
    return codes, float(s0[0]), float(xm[0]), float(ym[0])


def bh_tree(pos, mass):
    """Barnes-Hut compressed quadtree: (order[K], nodes_i (N,5) lo,hi,child0,nchild,depth,
    nodes_d (N,4) size,mass,cx,cy, child list).  Node 0 is the root; the children of
    node k are child[child0 : child0 + nchild] (none for a leaf)."""
    lib = _load()
    x = _c(pos, np.float64).reshape(-1, 2)
    K = x.shape[0]
    ms = _c(mass, np.float64)
    order = np.empty(K, np.int32)
    ni = np.empty((2 * K, 5), np.int32)
    nd = np.empty((2 * K, 4), np.float64)
    ch = np.empty(2 * K, np.int32)
    nn = lib.orc_bh_tree_export(K, _p(x), _p(ms), _p(order), _p(ni), _p(nd), _p(ch))
    nc = int(ni[:nn, 3].sum())
    return order, ni[:nn].copy(), nd[:nn].copy(), ch[:nc].copy()


def bh_repulsion(pos, mass, kr=1.0, theta=1.2):
    """Barnes-Hut repulsion (K,2) FP64 and, per body, whether any of its opening
    decisions is borderline (within single-precision rounding of theta)."""
    lib = _load()
    x = _c(pos, np.float64).reshape(-1, 2)
    K = x.shape[0]
    ms = _c(mass, np.float64)
    F = np.zeros((K, 2), np.float64)
    border = np.zeros(K, np.int32)
    lib.orc_bh_repulsion(K, _p(x), _p(ms), kr, theta, _p(F), _p(border))
    return F, border.astype(bool)


# -------------------------------------------------------------- whole pipeline --
def pipeline(n, edges, wl, coef1, coef2, pos0):
    """Community passes + supergraph + layout for one workload dict ``wl``."""
    lab, cnt = bs_community(n, edges, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"])
    deg, vol = degree_volume(lab, cnt, wl["passes"])
    sg = supergraph(n, edges, lab, deg, wl["rows"], wl["cols"], coef1, coef2)
    mass = fa2_mass(sg["K"], sg["superedges"])
    pos, Fp, sp = fa2_layout(pos0[: sg["K"]], sg["superedges"], mass, iters=wl["fa2_iters"],
                             exact=wl["exact"], theta=wl["theta"], kr=wl["kr"], kg=wl["kg"],
                             tau=wl["tau"], ks=wl["ks"], ksmax=wl["ksmax"])
    return dict(labels=lab, counters=cnt, degree=deg, volume=vol, sg=sg, mass=mass, pos=pos,
                Fprev=Fp, speed=sp)


# -------------------------------------------------------------- drawing rules ---
def draw_supernodes(super_size):
    """Drawing attributes of the supernodes: the radius grows with the square root of
    the size (Section 4.1), and 11 colour groups by size (Section 4.3).  Following
    Section 4.3: alpha is the sum of all sizes; the communities are taken by size, small
    first (equal sizes by supernode id); the smallest ones that together hold at most
    half of alpha form group 0; the rest are cut into groups 1..10 holding equal shares
    of the remaining half (the paper leaves the cut open; this reading is recorded with
    the others), so a community whose running total (itself included) is P falls in
    group ceil(10 * (2P - alpha) / alpha).  Integer arithmetic throughout.
    Returns (group int32[K] in 0..10, radius float32[K] = correctly rounded sqrt of the
    size converted to float32)."""
    s = [int(v) for v in np.asarray(super_size, dtype=np.uint64)]
    K = len(s)
    order = sorted(range(K), key=lambda c: (s[c], c))
    alpha = sum(s)
    group = np.zeros(K, np.int32)
    running = 0
    for c in order:
        running += s[c]
        if 2 * running > alpha:
            g = -(-10 * (2 * running - alpha) // alpha)  # ceiling division
            group[c] = min(10, max(1, g))
    radius = np.sqrt(np.asarray(super_size, dtype=np.uint32).astype(np.float32))
    return group, radius

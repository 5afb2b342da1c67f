"""Python binding of the C ABI (include/bgv.h): argument marshalling only.

Every step of the hot path runs in the HIP kernels of libbgv.so; torch supplies device
memory (outputs and workspaces) and the current stream.  Inputs must already be CUDA
(HIP) tensors of the documented dtype.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, name, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class _range_check:
    """Sets BGV_CHECK=1 (the library's opt-in device id checks) for one call."""

    def __init__(self, on: bool):
        self.on = on

    def __enter__(self):
        import os
        if self.on:
            self.prev = os.environ.get("BGV_CHECK")
            os.environ["BGV_CHECK"] = "1"

    def __exit__(self, *exc):
        import os
        if self.on:
            if self.prev is None:
                os.environ.pop("BGV_CHECK", None)
            else:
                os.environ["BGV_CHECK"] = self.prev


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def validate_edges(edges: torch.Tensor, n: int, stream=None) -> None:
    """Device scan of the edge ids (bgv_validate_edges): raises ValueError if an id lies
    outside [0, n).  Synchronises the stream."""
    m = edges.shape[0] if edges.dim() == 2 else 0
    _need(edges, torch.int32, "edges", (m, 2))
    flag = torch.empty(1, dtype=torch.int32, device=edges.device)
    st = L.bgv_validate_edges(int(n), int(m), _ptr(edges), _ptr(flag), _stream(stream))
    if st == L.BGV_E_RANGE:
        raise ValueError(f"edge ids must lie in [0, {n})")
    L.check(st, "bgv_validate_edges")


# ------------------------------------------------------------------- community --
def community(edges: torch.Tensor, n: int, threshold: int, passes: int = 1, growth: int = 2,
              chunk: int = 1, volume: bool = False, ws: torch.Tensor | None = None, stream=None,
              method: int = 0, tie: int = 0, rule: int = 0, check: bool = True):
    """Streaming community detection.  Returns (labels int32[n], degree int32[n],
    volume int64[n] or None).  method: 0 automatic, 1 chunk by chunk, 2 back-pointer
    resolution (the same integers).  tie: 1 = on equal counters the edge's first
    endpoint joins the second's community (0: nothing happens, as in Algorithm 3).
    rule: 0 = the paper's degree rule, 1 = SCoDA's community-volume rule.  check: scan
    the edge ids on the device first (validate_edges; synchronises the stream)."""
    m = edges.shape[0] if edges.dim() == 2 else 0
    _need(edges, torch.int32, "edges", (m, 2))
    if check:
        validate_edges(edges, n, stream)
    p = L.CdParams(int(threshold), int(passes), int(growth), int(method), int(chunk), int(tie), int(rule))
    need = L.bgv_community_workspace(int(n), m, C.byref(p))
    if need == 0:
        raise L.BgvError(f"invalid community arguments (n={n}, m={m}, {threshold}, {passes}, {growth}, {chunk}, "
                         f"method {method})")
    dev = edges.device
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    degree = torch.empty(n, dtype=torch.int32, device=dev)
    vol = torch.empty(n, dtype=torch.int64, device=dev) if volume else None
    L.check(L.bgv_community(int(n), m, _ptr(edges), C.byref(p), _ptr(labels), _ptr(degree), _ptr(vol),
                            _ptr(ws), ws.numel(), _stream(stream)), "bgv_community")
    return labels, degree, vol


def community_passes(edges: torch.Tensor, n: int, threshold: int, passes: int = 1, growth: int = 2,
                     chunk: int = 1, volume: bool = False, ws: torch.Tensor | None = None, stream=None,
                     method: int = 0, tie: int = 0, rule: int = 0, check: bool = True):
    """community() that also keeps each pass's labels (the hierarchy of community sets).
    Returns (labels, degree, volume or None, pass_labels int32[passes, n])."""
    m = edges.shape[0] if edges.dim() == 2 else 0
    _need(edges, torch.int32, "edges", (m, 2))
    if check:
        validate_edges(edges, n, stream)
    p = L.CdParams(int(threshold), int(passes), int(growth), int(method), int(chunk), int(tie), int(rule))
    need = L.bgv_community_workspace(int(n), m, C.byref(p))
    if need == 0:
        raise L.BgvError(f"invalid community arguments (n={n}, m={m}, {threshold}, {passes}, {growth}, {chunk}, "
                         f"method {method})")
    dev = edges.device
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    degree = torch.empty(n, dtype=torch.int32, device=dev)
    vol = torch.empty(n, dtype=torch.int64, device=dev) if volume else None
    rows = torch.empty((int(passes), n), dtype=torch.int32, device=dev)
    L.check(L.bgv_community_passes(int(n), m, _ptr(edges), C.byref(p), _ptr(labels), _ptr(degree), _ptr(vol),
                                   _ptr(rows), _ptr(ws), ws.numel(), _stream(stream)), "bgv_community_passes")
    return labels, degree, vol, rows


def community_resume(edges: torch.Tensor, n: int, labels_in: torch.Tensor, done: int, threshold: int,
                     passes: int, growth: int = 2, chunk: int = 1, volume: bool = False,
                     ws: torch.Tensor | None = None, stream=None, method: int = 0, tie: int = 0, rule: int = 0,
                     check: bool = True):
    """Continue a community() run that stopped after `done` passes from its labels then
    (labels_in int32[n]): passes done .. passes-1, with the same results as community()
    with `passes` passes.  Returns (labels, degree, volume or None)."""
    m = edges.shape[0] if edges.dim() == 2 else 0
    _need(edges, torch.int32, "edges", (m, 2))
    _need(labels_in, torch.int32, "labels_in", (n,))
    if check:
        validate_edges(edges, n, stream)
    p = L.CdParams(int(threshold), int(passes), int(growth), int(method), int(chunk), int(tie), int(rule))
    need = L.bgv_community_workspace(int(n), m, C.byref(p))
    if need == 0:
        raise L.BgvError(f"invalid community arguments (n={n}, m={m}, {threshold}, {passes}, {growth}, {chunk}, "
                         f"method {method})")
    dev = edges.device
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    degree = torch.empty(n, dtype=torch.int32, device=dev)
    vol = torch.empty(n, dtype=torch.int64, device=dev) if volume else None
    with _range_check(check):
        L.check(L.bgv_community_resume(int(n), m, _ptr(edges), C.byref(p), int(done), _ptr(labels_in), _ptr(labels),
                                       _ptr(degree), _ptr(vol), _ptr(ws), ws.numel(), _stream(stream)),
                "bgv_community_resume")
    return labels, degree, vol


def community_workspace(edges: torch.Tensor, n: int, wl: dict) -> torch.Tensor:
    """A workspace tensor for community() on this graph and workload."""
    p = L.CdParams(int(wl["threshold"]), int(wl["passes"]), int(wl["growth"]), 0, int(wl["chunk"]),
                   int(wl.get("tie", 0)), int(wl.get("rule", 0)))
    need = L.bgv_community_workspace(int(n), int(edges.shape[0]), C.byref(p))
    return _workspace(need, edges.device)


def supergraph_workspace(edges: torch.Tensor, n: int, wl: dict) -> torch.Tensor:
    """A workspace tensor for supergraph() on this graph and workload."""
    z = np.zeros((int(wl["rows"]), 3), np.uint64)
    sp = L.SketchParams(int(wl["rows"]), int(wl["cols"]), z.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p))
    need = L.bgv_supergraph_workspace(int(n), int(edges.shape[0]), C.byref(sp))
    return _workspace(need, edges.device)


# ------------------------------------------------------------------ supergraph --
def supergraph(edges: torch.Tensor, labels: torch.Tensor, degree: torch.Tensor, rows: int, cols: int,
               coef1: np.ndarray, coef2: np.ndarray, ws: torch.Tensor | None = None, stream=None,
               exact_counts: bool = False, check: bool = True):
    """Count-min-sketch supergraph.  Synchronises the stream.  Returns a dict with K,
    super_label, super_size, node_super, superedges (E,2), se_weight, se_count (exact
    multiplicities, if asked for), M1, M2.  check: scan the edge ids on the device first."""
    n = labels.shape[0]
    m = edges.shape[0]
    _need(edges, torch.int32, "edges", (m, 2))
    if check:
        validate_edges(edges, n, stream)
    _need(labels, torch.int32, "labels", (n,))
    _need(degree, torch.int32, "degree", (n,))
    c1 = np.ascontiguousarray(coef1, dtype=np.uint64).reshape(rows, 3)
    c2 = np.ascontiguousarray(coef2, dtype=np.uint64).reshape(rows, 3)
    sp = L.SketchParams(int(rows), int(cols), c1.ctypes.data_as(C.c_void_p), c2.ctypes.data_as(C.c_void_p))
    need = L.bgv_supergraph_workspace(int(n), int(m), C.byref(sp))
    if need == 0:
        raise L.BgvError(f"invalid supergraph arguments (n={n}, m={m}, rows={rows}, cols={cols})")
    dev = edges.device
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    super_label = torch.empty(n, dtype=torch.int32, device=dev)
    super_size = torch.empty(n, dtype=torch.int32, device=dev)       # uint32 bits
    node_super = torch.empty(n, dtype=torch.int32, device=dev)
    superedges = torch.empty((max(m, 1), 2), dtype=torch.int32, device=dev)
    se_weight = torch.empty(max(m, 1), dtype=torch.int32, device=dev)  # uint32 bits
    se_count = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if exact_counts else None
    M1 = torch.empty((rows, cols), dtype=torch.int32, device=dev)      # uint32 bits
    M2 = torch.empty((rows, cols), dtype=torch.int32, device=dev)
    K = L.i32(0)
    E = L.i64(0)
    L.check(L.bgv_supergraph(int(n), int(m), _ptr(edges), _ptr(labels), _ptr(degree), C.byref(sp), C.byref(K),
                             C.byref(E), _ptr(super_label), _ptr(super_size), _ptr(node_super), _ptr(superedges),
                             _ptr(se_weight), _ptr(se_count), _ptr(M1), _ptr(M2), _ptr(ws), ws.numel(),
                             _stream(stream)),
            "bgv_supergraph")
    k, e = K.value, E.value
    return dict(K=k, E=e, super_label=super_label[:k], super_size=super_size[:k], node_super=node_super,
                superedges=superedges[:e], se_weight=se_weight[:e],
                se_count=None if se_count is None else se_count[:e], M1=M1, M2=M2)


# ----------------------------------------------------------------- ForceAtlas2 --
def fa2_params(iters: int, exact: bool, theta: float = 1.2, kr: float = 1.0, kg: float = 1.0, tau: float = 1.0,
               ks: float = 0.1, ksmax: float = 10.0) -> L.Fa2Params:
    return L.Fa2Params(int(iters), 1 if exact else 0, float(theta), float(kr), float(kg), float(tau), float(ks),
                       float(ksmax))


def fa2_layout(superedges: torch.Tensor, pos: torch.Tensor, iters: int, exact: bool = True, theta: float = 1.2,
               kr: float = 1.0, kg: float = 1.0, tau: float = 1.0, ks: float = 0.1, ksmax: float = 10.0,
               attr_w: torch.Tensor | None = None, mass: torch.Tensor | None = None,
               fprev: torch.Tensor | None = None, speed: torch.Tensor | None = None,
               ws: torch.Tensor | None = None, stream=None):
    """ForceAtlas2 iterations; pos (K,2) float32 is updated in place.  Returns
    (pos, fprev, speed); pass fprev/speed back in to continue a run."""
    K = pos.shape[0]
    E = superedges.shape[0]
    _need(pos, torch.float32, "pos", (K, 2))
    _need(superedges, torch.int32, "superedges", (E, 2))
    if attr_w is not None:
        _need(attr_w, torch.float32, "attr_w", (E,))
    if mass is not None:
        _need(mass, torch.float32, "mass", (K,))
    dev = pos.device
    if fprev is None:
        fprev = torch.zeros((K, 2), dtype=torch.float32, device=dev)
    if speed is None:
        speed = torch.ones(1, dtype=torch.float32, device=dev)
    _need(fprev, torch.float32, "fprev", (K, 2))
    _need(speed, torch.float32, "speed", (1,))
    p = fa2_params(iters, exact, theta, kr, kg, tau, ks, ksmax)
    need = L.bgv_fa2_workspace(int(K), int(E), C.byref(p))
    if need == 0:
        raise L.BgvError(f"invalid fa2 arguments (K={K}, E={E})")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    L.check(L.bgv_fa2_layout(int(K), int(E), _ptr(superedges), _ptr(attr_w), _ptr(mass), _ptr(pos), _ptr(fprev),
                             _ptr(speed), C.byref(p), _ptr(ws), ws.numel(), _stream(stream)), "bgv_fa2_layout")
    return pos, fprev, speed


def fa2_layout_static(superedges: torch.Tensor, pos: torch.Tensor, fprev: torch.Tensor, speed: torch.Tensor,
                      iters: int, exact: bool = True, theta: float = 1.2, kr: float = 1.0, kg: float = 1.0,
                      tau: float = 1.0, ks: float = 0.1, ksmax: float = 10.0,
                      attr_w: torch.Tensor | None = None, mass: torch.Tensor | None = None, stream=None):
    """fa2_layout without a workspace and without allocating: the library's fixed
    per-device scratch array serves instead (bgv_fa2_layout_static).  pos, fprev and
    speed are updated in place; calls that overlap on one GPU race."""
    K = pos.shape[0]
    E = superedges.shape[0]
    _need(pos, torch.float32, "pos", (K, 2))
    _need(superedges, torch.int32, "superedges", (E, 2))
    _need(fprev, torch.float32, "fprev", (K, 2))
    _need(speed, torch.float32, "speed", (1,))
    if attr_w is not None:
        _need(attr_w, torch.float32, "attr_w", (E,))
    if mass is not None:
        _need(mass, torch.float32, "mass", (K,))
    p = fa2_params(iters, exact, theta, kr, kg, tau, ks, ksmax)
    L.check(L.bgv_fa2_layout_static(int(K), int(E), _ptr(superedges), _ptr(attr_w), _ptr(mass), _ptr(pos),
                                    _ptr(fprev), _ptr(speed), C.byref(p), _stream(stream)), "bgv_fa2_layout_static")
    return pos, fprev, speed


def fa2_energy(superedges: torch.Tensor, pos: torch.Tensor, kr: float = 1.0, kg: float = 1.0,
               attr_w: torch.Tensor | None = None, mass: torch.Tensor | None = None, ws=None, stream=None):
    """ForceAtlas2 energy (device float64 scalar tensor)."""
    K, E = pos.shape[0], superedges.shape[0]
    _need(pos, torch.float32, "pos", (K, 2))
    _need(superedges, torch.int32, "superedges", (E, 2))
    need = L.bgv_fa2_energy_workspace(int(K), int(E))
    if need == 0:
        raise L.BgvError(f"invalid energy arguments (K={K}, E={E})")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, pos.device)
    out = torch.empty(1, dtype=torch.float64, device=pos.device)
    L.check(L.bgv_fa2_energy(int(K), int(E), _ptr(superedges), _ptr(attr_w), _ptr(mass), _ptr(pos), float(kr),
                             float(kg), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)), "bgv_fa2_energy")
    return out[0]


def fa2_grad(superedges: torch.Tensor, pos: torch.Tensor, kr: float = 1.0, kg: float = 1.0,
             attr_w: torch.Tensor | None = None, mass: torch.Tensor | None = None,
             grad_out: torch.Tensor | None = None, ws=None, stream=None):
    """Gradient of the ForceAtlas2 energy (= -force * grad_out), (K,2) float32."""
    K, E = pos.shape[0], superedges.shape[0]
    _need(pos, torch.float32, "pos", (K, 2))
    _need(superedges, torch.int32, "superedges", (E, 2))
    if grad_out is not None:
        _need(grad_out, torch.float32, "grad_out", (1,))
    need = L.bgv_fa2_energy_workspace(int(K), int(E))
    if need == 0:
        raise L.BgvError(f"invalid gradient arguments (K={K}, E={E})")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, pos.device)
    g = torch.empty((K, 2), dtype=torch.float32, device=pos.device)
    L.check(L.bgv_fa2_grad(int(K), int(E), _ptr(superedges), _ptr(attr_w), _ptr(mass), _ptr(pos), float(kr),
                           float(kg), _ptr(grad_out), _ptr(g), _ptr(ws), ws.numel(), _stream(stream)),
            "bgv_fa2_grad")
    return g


def bh_tree(pos: torch.Tensor, mass: torch.Tensor, ws=None, stream=None):
    """The Barnes-Hut tree one layout iteration builds (bgv_bh_tree), for inspection:
    dict of device tensors codes (K,) int32 (uint32 bits), body (K,4) float32 (x, y,
    mass, index bits), s0 (1,), nodeA (K-1,4) float32, nodeB (K-1,4) int32."""
    K = pos.shape[0]
    _need(pos, torch.float32, "pos", (K, 2))
    _need(mass, torch.float32, "mass", (K,))
    need = L.bgv_bh_tree_workspace(int(K))
    if need == 0:
        raise L.BgvError(f"invalid tree arguments (K={K})")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, pos.device)
    dev = pos.device
    out = dict(codes=torch.empty(K, dtype=torch.int32, device=dev),
               body=torch.empty((K, 4), dtype=torch.float32, device=dev),
               s0=torch.empty(1, dtype=torch.float32, device=dev),
               nodeA=torch.empty((max(K - 1, 1), 4), dtype=torch.float32, device=dev),
               nodeB=torch.empty((max(K - 1, 1), 4), dtype=torch.int32, device=dev))
    L.check(L.bgv_bh_tree(int(K), _ptr(pos), _ptr(mass), _ptr(out["codes"]), _ptr(out["body"]), _ptr(out["nodeA"]),
                          _ptr(out["nodeB"]), _ptr(out["s0"]), _ptr(ws), ws.numel(), _stream(stream)), "bgv_bh_tree")
    out["nodeA"] = out["nodeA"][: K - 1]
    out["nodeB"] = out["nodeB"][: K - 1]
    return out


def draw_supernodes(super_size: torch.Tensor, ws=None, stream=None):
    """Drawing attributes of the supernodes (Section 4.1 radius, Section 4.3 colour
    groups): returns (group int32[K] in 0..10, radius float32[K] = sqrt(size))."""
    K = super_size.shape[0]
    if super_size.dtype not in (torch.int32, torch.uint32):
        raise L.BgvError(f"super_size must be uint32 (or int32 bits), got {super_size.dtype}")
    _need(super_size, super_size.dtype, "super_size", (K,))
    need = L.bgv_draw_workspace(int(K))
    if need == 0:
        raise L.BgvError(f"invalid drawing arguments (K={K})")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, super_size.device)
    group = torch.empty(K, dtype=torch.int32, device=super_size.device)
    radius = torch.empty(K, dtype=torch.float32, device=super_size.device)
    L.check(L.bgv_draw_supernodes(int(K), _ptr(super_size), _ptr(group), _ptr(radius), _ptr(ws), ws.numel(),
                                  _stream(stream)), "bgv_draw_supernodes")
    return group, radius


class FA2Energy(torch.autograd.Function):
    """Energy of a layout as an autograd function: forward = bgv_fa2_energy, backward =
    bgv_fa2_grad (the ForceAtlas2 force field, hand-written kernel)."""

    @staticmethod
    def forward(ctx, pos, superedges, kr=1.0, kg=1.0, attr_w=None, mass=None):
        pos_c = pos.detach().contiguous()
        ctx.save_for_backward(pos_c, superedges, attr_w, mass)
        ctx.kr, ctx.kg = kr, kg
        return fa2_energy(superedges, pos_c, kr, kg, attr_w, mass).to(torch.float32)

    @staticmethod
    def backward(ctx, grad_out):
        pos, superedges, attr_w, mass = ctx.saved_tensors
        go = grad_out.detach().to(torch.float32).reshape(1).contiguous()
        g = fa2_grad(superedges, pos, ctx.kr, ctx.kg, attr_w, mass, grad_out=go)
        return g, None, None, None, None, None


# ------------------------------------------------------------------ whole path --
def pipeline(edges: torch.Tensor, n: int, wl: dict, coef1: np.ndarray, coef2: np.ndarray, pos0: torch.Tensor,
             volume: bool = False, stream=None, check: bool = True):
    """Community passes + supergraph + ForceAtlas2 layout of the supergraph for one
    workload description ``wl`` (threshold, passes, growth, chunk, rows, cols,
    fa2_iters, exact, theta, kr, kg, tau, ks, ksmax).  pos0 (>= K rows) seeds the layout.
    check: scan the edge ids on the device first."""
    labels, degree, vol = community(edges, n, wl["threshold"], wl["passes"], wl["growth"], wl["chunk"],
                                    volume=volume, stream=stream, tie=int(wl.get("tie", 0)),
                                    rule=int(wl.get("rule", 0)), check=check)
    sg = supergraph(edges, labels, degree, wl["rows"], wl["cols"], coef1, coef2, stream=stream, check=False)
    pos = pos0[: sg["K"]].clone()
    pos, fprev, speed = fa2_layout(sg["superedges"], pos, wl["fa2_iters"], wl["exact"], wl["theta"], wl["kr"],
                                   wl["kg"], wl["tau"], wl["ks"], wl["ksmax"], stream=stream)
    return dict(labels=labels, degree=degree, volume=vol, sg=sg, pos=pos, fprev=fprev, speed=speed)


# --------------------------------------------------------------------- batched --
def pack_graphs(graphs, device):
    """Concatenate [(n_g, edges_g (m_g,2) int32 numpy with local ids), ...] for
    batched(): returns (edges (m_total,2) int32, node_off int64[G+1], edge_off int64[G+1]
    on the device, and the host offsets)."""
    ns = np.array([int(n) for n, _ in graphs], dtype=np.int64)
    ms = np.array([int(np.asarray(e).reshape(-1, 2).shape[0]) for _, e in graphs], dtype=np.int64)
    node_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    edge_off = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
    parts = [np.asarray(e, dtype=np.int32).reshape(-1, 2) for _, e in graphs]
    cat = np.concatenate(parts) if parts else np.zeros((0, 2), np.int32)
    return (torch.from_numpy(np.ascontiguousarray(cat)).to(device), torch.from_numpy(node_off).to(device),
            torch.from_numpy(edge_off).to(device), node_off, edge_off)


def batched(edges: torch.Tensor, node_off: torch.Tensor, edge_off: torch.Tensor, n_total: int, wl: dict,
            coef1: np.ndarray, coef2: np.ndarray, pos: torch.Tensor, order: torch.Tensor | None = None,
            fprev: torch.Tensor | None = None, speed: torch.Tensor | None = None, wg_threads: int = 0,
            big_k: int = 0, ws: torch.Tensor | None = None, stream=None, check: bool = False):
    """The whole path for G graphs in one persistent launch (include/bgv.h,
    bgv_batched); with big_k > 0, supergraphs larger than big_k nodes are laid out by
    multi-workgroup kernels after it.  pos (n_total, 2) float32 holds each graph's
    initial positions and is updated in place.  Returns a dict of device tensors.
    check: run the library's device id and offset checks first (BGV_CHECK=1 for this
    call; synchronises the stream, raises ValueError on BGV_E_RANGE)."""
    G = node_off.shape[0] - 1
    m_total = edges.shape[0]
    dev = edges.device
    _need(edges, torch.int32, "edges", (m_total, 2))
    _need(node_off, torch.int64, "node_off", (G + 1,))
    _need(edge_off, torch.int64, "edge_off", (G + 1,))
    _need(pos, torch.float32, "pos", (n_total, 2))
    if order is not None:
        _need(order, torch.int32, "order", (G,))
    if fprev is None:
        fprev = torch.zeros((n_total, 2), dtype=torch.float32, device=dev)
    if speed is None:
        speed = torch.ones(G, dtype=torch.float32, device=dev)
    _need(fprev, torch.float32, "fprev", (n_total, 2))
    _need(speed, torch.float32, "speed", (G,))
    rows, cols = int(wl["rows"]), int(wl["cols"])
    c1 = np.ascontiguousarray(coef1, dtype=np.uint64).reshape(rows, 3)
    c2 = np.ascontiguousarray(coef2, dtype=np.uint64).reshape(rows, 3)
    cd = L.CdParams(int(wl["threshold"]), int(wl["passes"]), int(wl["growth"]), 0, int(wl["chunk"]),
                    int(wl.get("tie", 0)), int(wl.get("rule", 0)))
    sp = L.SketchParams(rows, cols, c1.ctypes.data_as(C.c_void_p), c2.ctypes.data_as(C.c_void_p))
    fa = fa2_params(wl["fa2_iters"], True, wl.get("theta", 1.2), wl["kr"], wl["kg"], wl["tau"], wl["ks"],
                    wl["ksmax"])
    need = L.bgv_batched_workspace(int(G), int(n_total), int(m_total))
    if need == 0:
        raise L.BgvError(f"invalid batched arguments (G={G}, n_total={n_total}, m_total={m_total})")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    nn, mm = max(n_total, 1), max(m_total, 1)
    out = dict(labels=torch.empty(nn, dtype=torch.int32, device=dev),
               degree=torch.empty(nn, dtype=torch.int32, device=dev),
               K=torch.empty(G, dtype=torch.int32, device=dev), E=torch.empty(G, dtype=torch.int32, device=dev),
               super_label=torch.empty(nn, dtype=torch.int32, device=dev),
               super_size=torch.empty(nn, dtype=torch.int32, device=dev),
               superedges=torch.empty((mm, 2), dtype=torch.int32, device=dev),
               se_weight=torch.empty(mm, dtype=torch.int32, device=dev))
    with _range_check(check):
        st = L.bgv_batched(int(G), int(n_total), int(m_total), _ptr(node_off), _ptr(edge_off), _ptr(order),
                           _ptr(edges), C.byref(cd), C.byref(sp), C.byref(fa), int(wg_threads), int(big_k),
                           _ptr(out["labels"]),
                           _ptr(out["degree"]), _ptr(out["K"]), _ptr(out["E"]), _ptr(out["super_label"]),
                           _ptr(out["super_size"]), _ptr(out["superedges"]), _ptr(out["se_weight"]), _ptr(pos),
                           _ptr(fprev), _ptr(speed), _ptr(ws), ws.numel(), _stream(stream))
    if st == L.BGV_E_RANGE:
        raise ValueError("batched graphs: offsets inconsistent or local ids out of range")
    L.check(st, "bgv_batched")
    out.update(pos=pos, fprev=fprev, speed=speed)
    return out


def batched_workspace(G: int, n_total: int, m_total: int, device) -> torch.Tensor:
    return _workspace(L.bgv_batched_workspace(int(G), int(n_total), int(m_total)), device)

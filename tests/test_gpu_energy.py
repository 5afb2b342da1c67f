"""GPU parity of the ForceAtlas2 energy and its hand-written gradient (the force
field) against the FP64 oracle, and of the autograd wrapper."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def bgv():
    import paper_2108_00529_amd as b
    return b


def random_weighted(seed, K, E):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-3, 3, (K, 2)).astype(np.float32)
    pairs = set()
    while len(pairs) < E:
        a, b = rng.integers(0, K, 2)
        if a != b:
            pairs.add((int(min(a, b)), int(max(a, b))))
    se = np.array(sorted(pairs), np.int32)
    aw = rng.uniform(0.5, 4.0, E).astype(np.float32)
    return pos, se, aw


@pytest.mark.parametrize("K,E,weighted,kr,kg", [(1, 0, False, 1.0, 1.0), (2, 1, False, 1.0, 1.0),
                                                (700, 2000, False, 1.0, 1.0), (3000, 9000, True, 2.0, 0.5),
                                                (300, 0, False, 1.0, 2.0)])
def test_energy_and_gradient(bgv, K, E, weighted, kr, kg):
    pos, se, aw = random_weighted(K + E, K, E) if E else (
        np.random.default_rng(K).uniform(-2, 2, (K, 2)).astype(np.float32), np.zeros((0, 2), np.int32), None)
    w = aw if weighted else None
    mass = oracle.fa2_mass(K, se)
    e_ref = oracle.fa2_energy(pos.astype(np.float64), se, mass, w, kr, kg)
    F_ref = oracle.fa2_forces(pos.astype(np.float64), se, mass, w, kr=kr, kg=kg, exact=True)
    w_d = dev(aw) if weighted else None
    e = float(bgv.fa2_energy(dev(se), dev(pos), kr, kg, attr_w=w_d))
    g = host(bgv.fa2_grad(dev(se), dev(pos), kr, kg, attr_w=w_d))
    scale_e = max(1.0, abs(e_ref))
    print(f"K={K} E={E}: energy gpu {e:.9g} oracle {e_ref:.9g}", flush=True)
    assert abs(e - e_ref) <= TOL * scale_e
    gscale = max(1e-30, np.linalg.norm(F_ref, axis=1).max())
    assert np.linalg.norm(g + F_ref, axis=1).max() <= TOL * gscale
    # given masses
    m2 = np.random.default_rng(1).uniform(1, 5, K).astype(np.float32)
    e2_ref = oracle.fa2_energy(pos.astype(np.float64), se, m2.astype(np.float64), w, kr, kg)
    e2 = float(bgv.fa2_energy(dev(se), dev(pos), kr, kg, attr_w=w_d, mass=dev(m2)))
    assert abs(e2 - e2_ref) <= TOL * max(1.0, abs(e2_ref))


def test_gradient_is_linear_in_grad_out(bgv):
    pos, se, aw = random_weighted(5, 500, 1500)
    g1 = bgv.fa2_grad(dev(se), dev(pos))
    g3 = bgv.fa2_grad(dev(se), dev(pos), grad_out=torch.tensor([-2.5], device="cuda"))
    assert torch.allclose(g3, -2.5 * g1, rtol=1e-6, atol=0)


def test_autograd_function(bgv):
    pos, se, aw = random_weighted(6, 400, 1200)
    x = dev(pos).requires_grad_(True)
    E = bgv.FA2Energy.apply(x, dev(se), 1.0, 1.0, dev(aw), None)
    (3.0 * E).backward()
    g = bgv.fa2_grad(dev(se), dev(pos), 1.0, 1.0, attr_w=dev(aw))
    assert torch.allclose(x.grad, 3.0 * g, rtol=1e-6, atol=0)
    mass = oracle.fa2_mass(400, se)
    e_ref = oracle.fa2_energy(pos.astype(np.float64), se, mass, aw.astype(np.float64))
    assert abs(float(E.detach()) - e_ref) <= TOL * abs(e_ref)


def test_energy_run_to_run_identical(bgv):
    pos, se, aw = random_weighted(7, 2000, 6000)
    a = bgv.fa2_energy(dev(se), dev(pos))
    b = bgv.fa2_energy(dev(se), dev(pos))
    assert float(a) == float(b)
    ga = bgv.fa2_grad(dev(se), dev(pos))
    gb = bgv.fa2_grad(dev(se), dev(pos))
    assert torch.equal(ga, gb)


def _lattice_repulsion(a, b):
    """sum over pairs of ln |x_i - x_j| for the a x b integer lattice, by offsets: the
    offset (dx, dy) joins (a - |dx|)(b - |dy|) pairs (each unordered pair counted once
    over the half-plane of offsets).  FP64, O(a b) terms."""
    dx = np.arange(-(a - 1), a)[:, None]
    dy = np.arange(-(b - 1), b)[None, :]
    cnt = (a - np.abs(dx)) * (b - np.abs(dy)).astype(np.float64)
    d2 = (dx * dx + dy * dy).astype(np.float64)
    with np.errstate(divide="ignore"):
        t = np.where(d2 > 0, cnt * 0.5 * np.log(d2), 0.0)
    return 0.5 * t.sum()  # every unordered pair appears at +offset and -offset


@pytest.mark.parametrize("a,b", [(40, 30), (1000, 800)])
def test_energy_lattice_closed_form(bgv, a, b):
    """Repulsion energy of unit masses on an integer lattice against its closed form by
    offsets.  800,000 bodies give 1.25M tile pairs more than one workgroup each can take,
    so the pairs are shared out over a capped grid."""
    xs, ys = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    pos = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float32)
    K = len(pos)
    se = np.zeros((0, 2), np.int32)
    mass = dev(np.ones(K, np.float32))
    e = float(bgv.fa2_energy(dev(se), dev(pos), kr=1.0, kg=0.0, mass=mass))
    ref = -_lattice_repulsion(a, b)
    print(f"  lattice {a}x{b}: K={K} energy {e:.10e} closed form {ref:.10e} rel {abs(e - ref) / abs(ref):.2e}",
          flush=True)
    assert abs(e - ref) <= 1e-5 * abs(ref)

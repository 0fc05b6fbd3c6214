"""GPU parity of variable per-element order (Section 3.1's P-distribution) through the
C ABI against the FP64 oracle.

Meshes: curved 2D boxes with orders 1..4 or 0..4 (P1 or P0 next to P4), straight 3D
boxes with orders 1..4 or 0..4 and re-oriented elements (every face orientation between orders), curved
3D boxes with orders 2..4, and NACA O-grids whose order falls from 3 at the wall to
0 toward the far field (the paper's low-resolution P0-P3 distribution), and a
uniform order-0 mesh (one solution point per element: a finite volume).

Bars (as for one order, relative L2 per physical field): FP64 residual and FP64 RK4
state 1e-12; FP32 form 1e-5 after 100 steps; wall force means 1e-10; a variable-order
mesh whose orders are all equal bit-identical to the one-order mesh; a pool request
bit-identical to its solo run; designs of a variable-order batch bit-identical to
their solo runs.
"""
import numpy as np
import pytest

from oracle import probe as oprobe
from oracle.oracle import OracleMesh
from paper_2501_05709_amd import _lib
from paper_2501_05709_amd import workloads as W
from paper_2501_05709_amd.solver import FRMesh, FRPool, FWH, Probe

pytestmark = pytest.mark.gpu


def rel_err(x, ref):
    nv = ref.shape[-1]
    x = x.reshape(-1, nv)
    ref = ref.reshape(-1, nv)
    errs = []
    for cols in ([0], list(range(1, nv - 1)), [nv - 1]):
        errs.append(np.linalg.norm(x[:, cols] - ref[:, cols]) / np.linalg.norm(ref[:, cols]))
    return max(errs)


def rotate_element(conn, q, dim, rot):
    na = q + 1
    new = np.empty_like(conn)
    for idx in range(na ** dim):
        a = np.array([(idx // na ** k) % na for k in range(dim)])
        b = rot(a, q)
        new[idx] = conn[sum(int(b[k]) * na ** k for k in range(dim))]
    return new


ROT2 = [lambda a, q: np.array([q - a[1], a[0]]), lambda a, q: np.array([q - a[0], q - a[1]])]
ROT3 = [lambda a, q: np.array([q - a[1], a[0], a[2]]), lambda a, q: np.array([a[0], q - a[2], a[1]]),
        lambda a, q: np.array([a[1], a[2], a[0]]), lambda a, q: np.array([q - a[0], q - a[1], a[2]])]


def box(dim, q, warp, lo, seed, rotate, nel=None):
    nel = nel or ((5, 4) if dim == 2 else (3, 3, 2))
    m = W.box_mesh(dim, nel, (0,) * dim, (1.0,) * dim, q=q, warp=warp, order=3)
    m.update(gamma=1.4, prandtl=0.72, mu=0.02, freestream=np.array([1.0, 0.3, -0.2, 0.1, 1.0]), dt=2e-4)
    E = len(m["elem_nodes"])
    orders = np.random.default_rng(seed).integers(lo, 5, size=E)
    orders[:4] = (lo, 4, 2, 3)
    m["orders"] = orders.astype(np.int32)
    if rotate:
        rots = ROT2 if dim == 2 else ROT3
        conn = m["elem_nodes"].copy()
        for e in range(1, E, 2):
            conn[e] = rotate_element(conn[e], q, dim, rots[(e // 2) % len(rots)])
        m["elem_nodes"] = conn
    return m


def ogrid(seed=1, ni=24, nj=8, nk=2):
    """Order 3 at the wall falling to 0 at the far field: the paper's low-resolution
    P0-P3 distribution."""
    m = W.config_airfoil(seed, ni=ni, nj=nj, nk=nk)
    m["orders"] = W.ring_orders(ni, nj, nk, ((2, 3), (4, 2), (6, 1), (nj, 0)))
    m["dt"] = W.airfoil_dt(dict(m, order=3), 3)
    return m


def uniform_p0():
    m = W.config_tgv(nel=6, order=0)
    m["orders"] = np.zeros(len(m["elem_nodes"]), dtype=np.int32)
    return m


def case(name):
    return {"box2d_curved_p1-4": lambda: box(2, 2, 0.05, 1, 0, True),
            "box2d_curved_p0-4": lambda: box(2, 2, 0.05, 0, 3, True),
            "box3d_rotated_p1-4": lambda: box(3, 1, 0.0, 1, 1, True),
            "box3d_rotated_p0-4": lambda: box(3, 1, 0.0, 0, 6, True),
            "box3d_curved_p2-4": lambda: box(3, 2, 0.05, 2, 2, False),
            "ogrid_p3-0": lambda: ogrid(),
            "tgv_p0": uniform_p0}[name]()


def state(o, m, amp=0.1, seed=0):
    x = o.solution_points().reshape(-1, 3)
    fs = m["freestream"]
    u = W.uniform_state(len(x), fs[0], fs[1:1 + o.dim], fs[4])
    k = np.random.default_rng(seed).uniform(0.5, 2.0, size=3)
    s = np.sin(k[0] * x[:, 0] + 0.3) * np.cos(k[1] * x[:, 1] - 0.2) * np.cos(k[2] * x[:, 2] + 0.1)
    u[:, 0] *= 1.0 + amp * s
    u[:, -1] *= 1.0 + amp * s
    return u


CASES = ["box2d_curved_p1-4", "box2d_curved_p0-4", "box3d_rotated_p1-4", "box3d_rotated_p0-4", "box3d_curved_p2-4",
         "ogrid_p3-0", "tgv_p0"]


@pytest.mark.parametrize("name", CASES)
def test_mixed_residual_fp64_matches_oracle(name):
    m = case(name)
    o = OracleMesh(m)
    g = FRMesh(m, "fp64")
    print(f"{name}: {o.E} elements, {o.NU} points, {o.n_mortar} mortar faces", flush=True)
    assert g.shape == o.shape and (o.n_mortar > 0 or name == "tgv_p0")
    assert np.allclose(g.solution_points(), o.solution_points(), rtol=0, atol=1e-13)
    u = state(o, m)
    err = rel_err(g.residual(u), o.residual(u))
    print(f"  residual rel err {err:.2e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("name", CASES)
def test_mixed_rk4_fp64_matches_oracle(name):
    m = case(name)
    o = OracleMesh(m)
    g = FRMesh(m, "fp64")
    u0 = state(o, m)
    n = 20
    ref, hist = o.rk4(u0, m["dt"], n, forces=True)
    g.set_state(u0)
    g.step(n)
    err = rel_err(g.get_state(), ref)
    print(f"{name}: {n} steps, state rel err {err:.2e}", flush=True)
    assert err <= 1e-12
    if (np.asarray(m.get("bfaces", np.zeros((0, 3))))[:, 2] == W.BC_WALL).any():
        f = g.forces()
        fs = m["freestream"]
        qref = 0.5 * fs[0] * (fs[1:4] @ fs[1:4]) * m["ref_area"]
        mean = hist.mean(axis=0)
        cl, cd = mean @ m["lift_dir"] / qref, mean @ m["drag_dir"] / qref
        scale = max(abs(cl), abs(cd))
        assert f[7] == n and abs(f[5] - cl) <= 1e-10 * scale and abs(f[6] - cd) <= 1e-10 * scale


@pytest.mark.parametrize("name", ["box2d_curved_p0-4", "box3d_rotated_p1-4", "ogrid_p3-0"])
def test_mixed_fp32_form_matches_oracle(name):
    m = case(name)
    o = OracleMesh(m)
    g = FRMesh(m, "fp32")
    u0 = state(o, m)
    n = 100
    ref = o.rk4(u0, m["dt"], n)
    g.set_state(u0)
    g.step(n)
    err = rel_err(g.get_state(), ref)
    print(f"{name}: FP32 form after {n} steps, rel err {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_equal_orders_bit_identical_to_one_order(precision):
    """Every element at one order: no mortar faces, so the variable-order driver (order
    groups, split state, captured stage sequence) runs the one-order build of the fused
    kernels and must reproduce the uniform mesh bit for bit. (The mortar build, used
    when orders differ, may round a few boundary values differently in the last bit.)"""
    m = W.config_airfoil(3, ni=24, nj=5, nk=2)
    mm = dict(m, orders=np.full(len(m["elem_nodes"]), 3, dtype=np.int32))
    g1, g2 = FRMesh(m, precision), FRMesh(mm, precision)
    g1.select_kernels(g2.selected_kernels())   # the structure the order group runs
    o = OracleMesh(m)
    u0 = state(o, m).reshape(o.shape)
    g1.set_state(u0)
    g2.set_state(u0.reshape(-1, o.nv))
    g1.step(7)
    g2.step(7)
    assert np.array_equal(g1.get_state().reshape(-1, o.nv), g2.get_state())
    assert np.array_equal(g1.forces(), g2.forces())


def test_mixed_pool_request_bit_identical_to_solo():
    m = ogrid(seed=4, ni=16, nj=5, nk=1)
    g = FRMesh(m, "fp32")
    fs = m["freestream"]
    u0 = W.uniform_state(g.n_points, fs[0], fs[1:4], fs[4])
    g.set_state(u0)
    g.step(30)
    pool = FRPool(4 << 30)
    slot = pool.admit(m, 30, precision="fp32", u0=u0)
    done = []
    while not done:
        done = pool.tick(7)
    out, u = pool.result(slot, shape=g.shape)
    pool.close()
    assert np.array_equal(u, g.get_state()) and np.array_equal(out, g.forces())


def test_mixed_probe_matches_oracle():
    """Sampling the P3-P0 O-grid at points spread over all four order rings."""
    m = ogrid()
    o = OracleMesh(m)
    g = FRMesh(m, "fp64")
    u = state(o, m)
    g.set_state(u)
    rng = np.random.default_rng(5)
    r = rng.uniform(0.7, 19.0, 80)
    th = rng.uniform(0, 2 * np.pi, 80)
    pts = np.stack([0.5 + r * np.cos(th), r * np.sin(th), rng.uniform(0.01, 0.19, 80)], axis=1)
    pr = Probe(g, pts)
    elem, xi = pr.locate()
    e_o, xi_o = oprobe.locate(m, pts)
    assert np.array_equal(elem, e_o) and np.abs(xi - xi_o).max() < 1e-12
    assert len(set(m["orders"][elem])) == 4
    got = pr.sample()
    want = oprobe.sample(u, m["orders"], e_o, xi_o, 3)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_mixed_sampled_pool_request_matches_hand_driven_pipeline():
    """A served request on a variable-order mesh samples its data surface and feeds the
    FW-H record on the device: bit-identical to FRMesh + Probe + FWH driven by hand."""
    m = ogrid(seed=6, ni=16, nj=8, nk=1)
    # panels in every order ring, at one chordwise station, heard from far along the span
    # (so that the spread of arrival times stays below the record's length)
    ys = np.array([0.45, 5.0, 10.0, 16.0])
    surf_pts = np.array([(x, sg * y, 0.1) for x in (0.4, 0.6) for y in ys for sg in (1.0, -1.0)])
    nrm = np.zeros_like(surf_pts)
    nrm[:, 1] = np.sign(surf_pts[:, 1])
    surf = dict(points=surf_pts, normals=nrm, areas=np.full(len(surf_pts), 0.16 * 0.2), n_copies=3,
                copy_shift=(0.0, 0.0, 0.2))
    warmup, every, n_samples = 5, 4, 120
    g = FRMesh(m, "fp32")
    fs = m["freestream"]
    u0 = W.uniform_state(g.n_points, fs[0], fs[1:4], fs[4])
    pool = FRPool(4 << 30)
    slot = pool.admit_sampled(m, surf, warmup, every, n_samples, precision="fp32", u0=u0)
    done = []
    while not done:
        done = pool.tick(9)
    xo = np.array([0.5, 0.0, 500.0])
    t0, p = pool.pressure(slot, xo, n_samples)
    f = pool.result(slot)
    pool.close()
    g.set_state(u0)
    g.step(warmup)
    g.set_state(g.get_state())
    pr = Probe(g, surf_pts)
    c0 = np.sqrt(1.4 * fs[4] / fs[0])
    rec = FWH(surf_pts, nrm, surf["areas"], fs[1:4] / c0, c0, fs[0], fs[4], every * m["dt"], n_samples,
              n_copies=3, copy_shift=(0.0, 0.0, 0.2))
    rec.append_probe(pr)
    for _ in range(n_samples - 1):
        g.step(every)
        rec.append_probe(pr)
    t_ref, p_ref = rec.pressure(xo)
    assert len(set(m["orders"][pr.locate()[0]])) == 4
    assert p.size > 5 and t0 == t_ref[0] and np.array_equal(p, p_ref)
    assert np.array_equal(f, g.forces())


def _batch_designs():
    """Two O-grids with their own order rings (P3-P0, and P3-P1 on a smaller grid) and a
    uniform-order O-grid: one batch of variable-order designs of uneven size."""
    a = ogrid(seed=7, ni=24, nj=8, nk=2)
    b = W.config_airfoil(8, ni=16, nj=6, nk=1)
    b["orders"] = W.ring_orders(16, 6, 1, ((1, 3), (3, 2), (6, 1)))
    b["dt"] = W.airfoil_dt(dict(b, order=3), 3)
    c = W.config_airfoil(9, ni=16, nj=4, nk=2)
    return [a, b, c]


def _points(m):
    if m.get("orders") is None:
        return len(m["elem_nodes"]) * (m["order"] + 1) ** 3
    return int(((np.asarray(m["orders"]) + 1) ** 3).sum())


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_mixed_batch_members_match_solo_and_oracle(precision, tol):
    """Variable order in a batch: every order group covers the elements of that order of
    all designs.  Designs with mortar faces are bit-identical to their solo runs (same
    kernel build), the uniform-order design (run by the batch's mortar build) within the
    bar; two designs against the oracle."""
    meshes = _batch_designs()
    states = [state(OracleMesh(m), m, seed=i) for i, m in enumerate(meshes)]
    b = FRMesh(meshes, precision)
    assert b.n_designs == 3 and b.n_points == sum(_points(m) for m in meshes)
    b.set_state(np.concatenate(states))
    n = 10
    b.step(n)
    ub = b.get_state()
    off = np.cumsum([0] + [_points(m) for m in meshes])
    for i, m in enumerate(meshes):
        g = FRMesh(m, precision)
        g.set_state(states[i])
        g.step(n)
        us = g.get_state().reshape(-1, ub.shape[-1])
        part = ub[off[i]:off[i + 1]]
        if m.get("orders") is not None:
            assert np.array_equal(part, us), i
            assert np.array_equal(b.forces(i), g.forces()), i
        else:
            err = rel_err(part, us)
            print(f"uniform design in the variable-order batch vs solo ({precision}): {err:.2e}", flush=True)
            assert err <= tol
        g.close()
    for i in (0, 2):
        o = OracleMesh(meshes[i])
        ref = o.rk4(states[i].reshape(o.shape), meshes[i]["dt"], n)
        err = rel_err(ub[off[i]:off[i + 1]], ref)
        print(f"design {i} in the variable-order batch vs oracle, {n} steps ({precision}): {err:.2e}", flush=True)
        assert err <= tol
    b.close()


def test_mixed_unsupported_calls_are_rejected():
    m = box(2, 1, 0.0, 1, 5, False)
    g = FRMesh(m, "fp64")
    with pytest.raises(_lib.FRError) as e:
        g.select_kernels(0)
    assert e.value.code == _lib.FR_E_UNSUPPORTED
    with pytest.raises(_lib.FRError) as e:
        g.neighbours()
    assert e.value.code == _lib.FR_E_UNSUPPORTED
    with pytest.raises(_lib.FRError) as e:  # batched designs share the gas constants
        FRMesh([m, dict(m, mu=0.05)], "fp64")
    assert e.value.code == _lib.FR_E_ARG
    bad = dict(m, orders=np.full(len(m["elem_nodes"]), 6, dtype=np.int32))
    with pytest.raises(_lib.FRError) as e:
        FRMesh(bad, "fp64")
    assert e.value.code == _lib.FR_E_UNSUPPORTED


class _CountingAllocator:
    """The binding's torch allocator bridge, counting the live and peak device bytes."""

    def __init__(self, device):
        import torch
        self.live = self.peak = 0
        self.sizes = {}

        def _alloc(nbytes, ctx, stream):
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
            self.sizes[ptr] = int(nbytes)
            self.live += int(nbytes)
            self.peak = max(self.peak, self.live)
            return ptr

        def _free(ptr, ctx, stream):
            self.live -= self.sizes.pop(ptr, 0)
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc = _lib.ALLOC_FN(_alloc)
        self.free = _lib.FREE_FN(_free)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("kind", ["uniform", "rings"])
def test_footprint_bounds_the_device_memory_held(monkeypatch, precision, kind):
    """fr_footprint, which the pool admits requests by, is at least the peak of what a
    solver allocates through its allocator while it is built, set and stepped."""
    from paper_2501_05709_amd import solver as S
    m = ogrid(seed=2, ni=16, nj=8, nk=2)
    if kind == "uniform":
        m = {k: v for k, v in m.items() if k != "orders"}
    counters = []

    def make(device):
        counters.append(_CountingAllocator(device))
        return counters[-1]

    monkeypatch.setattr(S, "_TorchAllocator", make)
    g = FRMesh(m, precision)
    fs = m["freestream"]
    g.set_state(W.uniform_state(g.n_points, fs[0], fs[1:4], fs[4]).reshape(g.shape))
    g.step(3)
    g.forces()
    peak = counters[0].peak
    g.close()
    bound = S.footprint(m, precision)
    print(f"{kind} {precision}: peak {peak} B, footprint {bound} B", flush=True)
    assert 0 < peak <= bound

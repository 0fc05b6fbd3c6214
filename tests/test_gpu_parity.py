"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 per physical field -- density, the momentum vector,
total energy -- max over the three fields; the momentum vector is one field
so that the measure does not depend on the coordinate axes, and a momentum
component that is zero in the reference, as rho w in a spanwise-uniform
flow, is not divided by its own vanishing norm):
  * FP64 residual and FP64 state: 1e-12;
  * FP32 form (FP32 operators, fluxes and state; FP64 metrics): 1e-5 after
    100 steps;
  * index work (neighbour tables): bit for bit;
  * batch and pool members against their solo runs: bit for bit.
"""
import numpy as np
import pytest

from oracle.oracle import OracleMesh
from paper_2501_05709_amd import _lib
from paper_2501_05709_amd import workloads as W
from paper_2501_05709_amd.solver import FRMesh, FRPool

pytestmark = pytest.mark.gpu


def rel_err(x, ref):
    nv = ref.shape[-1]
    x = x.reshape(-1, nv)
    ref = ref.reshape(-1, nv)
    errs = []
    for cols in ([0], list(range(1, nv - 1)), [nv - 1]):
        errs.append(np.linalg.norm(x[:, cols] - ref[:, cols]) / np.linalg.norm(ref[:, cols]))
    return max(errs)


def perturbed(o, mesh, amp=0.1, seed=0):
    """A non-trivial smooth state: the mesh's initial state plus a smooth perturbation."""
    x = o.solution_points()
    u = o.initial_state() if "init" in mesh else None
    if u is None:
        fs = mesh["freestream"]
        u = W.uniform_state(o.E * o.nu, fs[0], fs[1:1 + o.dim], fs[4]).reshape(o.shape)
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.5, 2.0, size=3)
    s = np.sin(k[0] * x[..., 0] + 0.3) * np.cos(k[1] * x[..., 1] - 0.2) * np.cos(k[2] * x[..., 2] + 0.1)
    u = u.copy()
    u[..., 0] *= 1.0 + amp * s
    u[..., -1] *= 1.0 + amp * s
    return u


def case(name):
    if name == "vortex2d_p3":
        return W.config_vortex(0)
    if name == "vortex2d_p1":
        return W.config_vortex(3, nel=9, order=1)
    if name == "vortex2d_p4":
        return W.config_vortex(4, nel=5, order=4)
    if name == "box2d_curved_p2":
        m = W.box_mesh(2, (5, 4), (0, 0), (1, 1), q=2, warp=0.05, order=2)
        m.update(gamma=1.4, prandtl=0.72, mu=0.02, freestream=np.array([1.0, 0.3, -0.2, 0.0, 1.0]), dt=1e-3)
        return m
    if name.startswith("tgv"):
        # tgv_p3_one: a single periodic element, its own partner on every face, in a
        # workgroup whose other slots are empty; tgv_p2_two: 8 elements, half a block
        nel, order = {"tgv_p1": (6, 1), "tgv_p2": (5, 2), "tgv_p3": (4, 3), "tgv_p4": (3, 4),
                      "tgv_p3_one": (1, 3), "tgv_p2_two": (2, 2)}[name]
        return W.config_tgv(nel=nel, order=order)
    if name == "airfoil_p3":
        return W.config_airfoil(1, ni=24, nj=5, nk=2)
    if name == "airfoil_p2":
        return W.config_airfoil(2, ni=16, nj=4, nk=3, order=2)
    if name == "airfoil_p4":
        # the served workload's highest order on a curved O-grid: wall and far field
        return W.config_airfoil(6, ni=16, nj=4, nk=2, order=4)
    raise KeyError(name)


CASES = ["vortex2d_p3", "vortex2d_p1", "vortex2d_p4", "box2d_curved_p2", "tgv_p1", "tgv_p2", "tgv_p3", "tgv_p4", "tgv_p3_one", "tgv_p2_two",
         "airfoil_p3", "airfoil_p2", "airfoil_p4"]
# kernel structures / operator back-ends: five launches per stage with dense
# element-batched MFMA contractions or sum factorisation, or the fused
# two-launch stage (sum factorised), in 3D with its FP64 metrics formed from the
# geometry nodes, read from the stored arrays, or formed from the column metrics of
# z-extruded elements
VARIANTS = {"dense": 0, "tensor": (1 << 2) | (1 << 3) | (1 << 4) | (1 << 5), "fused": 1 | (1 << 5),
            "fused_stored": 1 | (1 << 5) | (1 << 6), "fused_extruded": 1 | (1 << 5) | (1 << 8)}


def select(g, variant):
    """Select a kernel structure; column metrics exist only on meshes of z-extruded elements."""
    try:
        g.select_kernels(VARIANTS[variant])
    except _lib.FRError as e:
        if e.code == _lib.FR_E_UNSUPPORTED and variant == "fused_extruded":
            pytest.skip("column metrics need a mesh of z-extruded elements")
        raise


# column metrics exist on 3D meshes only
VARIANTS_2D = sorted(v for v in VARIANTS if v != "fused_extruded")
CASE_VARIANTS = [(n, v) for n in CASES for v in (VARIANTS_2D if n.startswith(("vortex2d", "box2d")) else sorted(VARIANTS))]


@pytest.mark.parametrize("name,variant", CASE_VARIANTS)
def test_residual_fp64_matches_oracle(name, variant):
    m = case(name)
    o = OracleMesh(m)
    u = perturbed(o, m)
    ref = o.residual(u)
    g = FRMesh(m, "fp64")
    select(g, variant)
    assert g.selected_kernels() == VARIANTS[variant]
    assert np.array_equal(g.neighbours(), o.neighbours())
    r = g.residual(u)
    err = rel_err(r, ref)
    print(f"{name} {variant}: fp64 residual rel L2 {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-4)])
def test_variants_agree_and_mix(prec, tol):
    """Every per-kernel mix of the two back-ends on the stored metrics gives the same
    residual to round-off (FP32: the residual amplifies the flux rounding, as in the
    FP32-vs-oracle test).  The fused stage with metrics formed from the geometry nodes
    or from the column metrics of the O-grid's z-extruded elements evaluates S, |J|,
    normals and areas in FP64 by another route, equal to round-off;
    on this O-grid's sliver elements the residual amplifies that to a few 1e-13, so it
    is held to the oracle bar (1e-12 in FP64)."""
    m = case("airfoil_p3")
    o = OracleMesh(m)
    u = perturbed(o, m)
    g = FRMesh(m, prec)
    g.select_kernels(0)
    ref = g.residual(u)
    for mask in (VARIANTS["tensor"], VARIANTS["fused_stored"], 1 | (1 << 6), 1 << 2, (1 << 3) | (1 << 5), 1 << 4):
        g.select_kernels(mask)
        assert rel_err(g.residual(u), ref) <= tol, mask
    for mask in (VARIANTS["fused"], 1, VARIANTS["fused_extruded"]):
        g.select_kernels(mask)
        err = rel_err(g.residual(u), ref)
        print(f"airfoil_p3 {prec}: metrics from nodes or columns (mask {mask}) vs stored, residual rel L2 "
              f"{err:.2e}", flush=True)
        assert err <= (1e-12 if prec == "fp64" else tol), mask


@pytest.mark.parametrize("name", ["vortex2d_p3", "tgv_p3", "airfoil_p3"])
def test_residual_fp32_close_to_oracle(name):
    m = case(name)
    o = OracleMesh(m)
    u = perturbed(o, m)
    ref = o.residual(u)
    r = FRMesh(m, "fp32").residual(u)
    err = rel_err(r, ref)
    print(f"{name}: fp32 residual rel L2 {err:.3e}")
    # a residual is a difference quotient of O(1) fluxes: FP32 rounding of the
    # fluxes (~6e-8) is amplified by |F|/(h |R|); the state bar (1e-5 after
    # 100 steps) is the one the FP32 form is held to
    assert err <= 1e-3


@pytest.mark.parametrize("variant", VARIANTS_2D)
def test_vortex_state_after_100_steps(variant):
    """Isentropic vortex, 16x16 periodic quads, p = 3, 100 RK4 steps of 1e-3."""
    m = W.config_vortex(0)
    o = OracleMesh(m)
    u0 = o.initial_state()
    ref = o.rk4(u0, m["dt"], 100)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        g = FRMesh(m, prec)
        select(g, variant)
        g.set_state(u0)
        g.step(100)
        err = rel_err(g.get_state(), ref)
        print(f"vortex 100 steps {prec} {variant}: rel L2 {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_tgv_state_after_steps(variant):
    m = W.config_tgv(nel=6, order=3)
    o = OracleMesh(m)
    u0 = o.initial_state()
    ref = o.rk4(u0, m["dt"], 100)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        g = FRMesh(m, prec)
        select(g, variant)
        g.set_state(u0)
        g.step(100)
        err = rel_err(g.get_state(), ref)
        print(f"tgv 6^3 100 steps {prec}: rel L2 {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_airfoil_state_and_forces(variant):
    m = W.config_airfoil(3, ni=24, nj=5, nk=2)
    o = OracleMesh(m)
    u0 = o.initial_state()
    n = 20
    ref, hist = o.rk4(u0, m["dt"], n, forces=True)
    g = FRMesh(m, "fp64")
    select(g, variant)
    g.set_state(u0)
    g.step(n)
    err = rel_err(g.get_state(), ref)
    print(f"airfoil fp64 {n} steps: rel L2 {err:.3e}")
    assert err <= 1e-12
    f = g.forces()
    qref = 0.5 * 1.0 * 1.0 * m["ref_area"]
    cl_ref = hist[-1] @ m["lift_dir"] / qref
    cd_ref = hist[-1] @ m["drag_dir"] / qref
    mean = hist.mean(axis=0)
    scale = np.abs(hist).max() / qref
    assert f[7] == n
    assert abs(f[0] - cl_ref) <= 1e-10 * scale and abs(f[1] - cd_ref) <= 1e-10 * scale
    assert abs(f[5] - mean @ m["lift_dir"] / qref) <= 1e-10 * scale
    assert abs(f[6] - mean @ m["drag_dir"] / qref) <= 1e-10 * scale
    assert np.allclose(f[2:5], hist[-1], rtol=0, atol=1e-10 * np.abs(hist).max())


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_airfoil_p4_state_after_100_steps(variant):
    """Uniform p = 4 on a curved O-grid with wall and far-field faces: both forms after
    100 RK4 steps from a perturbed state, and the wall force means (FP64)."""
    m = case("airfoil_p4")
    o = OracleMesh(m)
    u0 = perturbed(o, m, amp=0.05)
    n = 100
    ref, hist = o.rk4(u0, m["dt"], n, forces=True)
    qref = 0.5 * m["ref_area"]
    scale = np.abs(hist).max() / qref
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        g = FRMesh(m, prec)
        select(g, variant)
        g.set_state(u0)
        g.step(n)
        err = rel_err(g.get_state(), ref)
        f = g.forces()
        mean_err = max(abs(f[5] - hist.mean(axis=0) @ m["lift_dir"] / qref),
                       abs(f[6] - hist.mean(axis=0) @ m["drag_dir"] / qref)) / scale
        print(f"airfoil p4 {variant} {prec} {n} steps: rel L2 {err:.3e}, mean C_L/C_D err {mean_err:.2e}")
        assert err <= tol and f[7] == n
        assert mean_err <= (1e-10 if prec == "fp64" else 1e-5)
        g.close()


def test_set_get_roundtrip_and_resume_bit_identical():
    m = W.config_airfoil(4, ni=16, nj=4, nk=2)
    o = OracleMesh(m)
    u0 = perturbed(o, m)
    g = FRMesh(m, "fp64")
    g.set_state(u0)
    assert np.array_equal(g.get_state(), u0)
    g.step(6)
    a = g.get_state()
    g.set_state(u0)
    g.step(3)
    mid = g.get_state()
    g.set_state(mid)
    g.step(3)
    assert np.array_equal(g.get_state(), a)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("orders", ["uniform", "p3_to_p0"])
def test_steps_split_across_calls_bit_identical(prec, orders):
    """Nine steps in one call, or split over five calls with reads of the forces and the
    state, a residual evaluation and a re-selected kernel structure between them: the same
    state, instantaneous forces, running means and averaged-step count, bit for bit. A call
    reuses the trace the previous step left, and the wall forces of a call's last state
    are added in the next call's first stage, or when they are read first."""
    ni, nj, nk = 16, 4, 2
    m = W.config_airfoil(4, ni=ni, nj=nj, nk=nk)
    if orders != "uniform":
        m["orders"] = W.ring_orders(ni, nj, nk, ((1, 3), (2, 2), (3, 1), (4, 0)))
    g = FRMesh(m, prec)
    u0 = np.ascontiguousarray(m["init"](g.solution_points().reshape(-1, 3)).reshape(g.shape))
    u0 = u0 * (1.0 + 0.02 * np.random.default_rng(3).standard_normal(u0.shape))
    g.set_state(u0)
    g.step(9)
    ua, fa = g.get_state(), g.forces()
    assert fa[7] == 9
    g.set_state(u0)
    g.step(2)
    assert g.forces()[7] == 2
    g.step(1)
    g.get_state()
    g.residual(u0)
    g.step(4)
    if orders == "uniform":
        g.select_kernels(g.selected_kernels())
    g.step_async(1)
    g.step(1)
    ub, fb = g.get_state(), g.forces()
    print(f"{orders} {prec}: forces {fb[:2]}, means {fb[5:7]}, count {fb[7]:.0f}")
    assert np.array_equal(ua, ub)
    assert np.array_equal(fa, fb)
    g.close()


def test_nonfinite_state_is_reported():
    m = W.config_vortex(1)
    g = FRMesh(m, "fp32")
    o = OracleMesh(m)
    u = o.initial_state()
    u[3, 2, 0] = np.nan
    g.set_state(u)
    with pytest.raises(_lib.FRError) as ei:
        g.step(2)
    assert ei.value.code == _lib.FR_E_NONFINITE


def test_batch_members_bit_identical_to_solo():
    meshes = [W.config_airfoil(10 + i, ni=12 + 4 * i, nj=3 + i, nk=1 + i % 2) for i in range(3)]
    b = FRMesh(meshes, "fp32")
    us = []
    for m in meshes:
        o = OracleMesh(m)
        us.append(perturbed(o, m, seed=len(us)))
    b.set_state(np.concatenate(us, axis=0))
    mask = b.autotune(2)
    b.step(8)
    ub = b.get_state()
    for i, m in enumerate(meshes):
        g = FRMesh(m, "fp32")
        g.select_kernels(mask)
        g.set_state(us[i])
        g.step(8)
        e0, ne = b.design_range(i)
        assert np.array_equal(ub[e0:e0 + ne], g.get_state())
        assert np.array_equal(b.forces(i), g.forces())


def test_pool_results_bit_identical_to_solo():
    reqs = [W.config_airfoil(20 + i, ni=12, nj=3 + i, nk=2, order=2 + i % 3) for i in range(4)]
    pool = FRPool(8 << 30)
    slots = {}
    for i, m in enumerate(reqs):
        s = pool.admit(m, steps=7 + i, precision="fp32", u0=OracleMesh(m).initial_state())
        assert s is not None
        slots[s] = i
    done = []
    while len(done) < len(reqs):
        done += pool.tick(3)
    for s in done:
        i = slots[s]
        m = reqs[i]
        o = OracleMesh(m)
        out, u = pool.result(s, shape=o.shape)
        g = FRMesh(m, "fp32")
        g.set_state(o.initial_state())
        g.step(7 + i)
        assert np.array_equal(u, g.get_state())
        assert np.array_equal(out, g.forces())
    assert pool.usage() == (0, 0)


# tile shapes of the fused stage (variant bits 9-10: first launch, 11-12: second launch;
# 0 default, 1 half the elements per workgroup, 2 a quarter, first launch 3: the default
# workgroup with the reference gradient and the volume divergence on the matrix cores):
# only the split of the elements over workgroups changes, and the matrix-core chains
# (FP32, order 3) take the same fused multiply-adds in the same order as the vector ALUs,
# so every shape must give the default's results bit for bit
TILE_SHAPES = [(1, 0), (2, 0), (3, 0), (0, 1), (0, 2), (2, 2), (1, 1)]
# bit 13: the neighbour exchange by scatter (each trace and viscous half flux written into
# the partner's slot) instead of the gather through the neighbour codes: the same values
# reach the same places, so again bit for bit
SCATTER = 1 << 13


@pytest.mark.parametrize("name", ["tgv_p1", "tgv_p2", "tgv_p3_one", "tgv_p4", "airfoil_p2", "airfoil_p3",
                                  "airfoil_p4"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("metrics", ["fused", "fused_stored", "fused_extruded"])
def test_tile_shapes_bit_identical(name, prec, metrics):
    m = case(name)
    o = OracleMesh(m)
    u = perturbed(o, m)
    g = FRMesh(m, prec)
    select(g, metrics)
    r0 = g.residual(u)
    g.set_state(u)
    g.step(3)
    s0, f0 = g.get_state(), g.forces()
    for ta, tb in [(0, 0)] + TILE_SHAPES:
        for scat in (0, SCATTER):
            if ta == tb == scat == 0:
                continue
            g.select_kernels(VARIANTS[metrics] | (ta << 9) | (tb << 11) | scat)
            r = g.residual(u)
            g.set_state(u)
            g.step(3)
            assert np.array_equal(r, r0), (ta, tb, scat)
            assert np.array_equal(g.get_state(), s0), (ta, tb, scat)
            assert np.array_equal(g.forces(), f0, equal_nan=True), (ta, tb, scat)  # NaN coefficients: no wall
    print(f"{name} {prec} {metrics}: tiles {TILE_SHAPES}, gather and scatter, bit-identical to the default")
    g.close()


@pytest.mark.parametrize("name", ["vortex2d_p3", "vortex2d_p1", "box2d_curved_p2"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_scatter_exchange_2d_bit_identical(name, prec):
    m = case(name)
    o = OracleMesh(m)
    u = perturbed(o, m)
    g = FRMesh(m, prec)
    g.select_kernels(VARIANTS["fused"])
    r0 = g.residual(u)
    g.set_state(u)
    g.step(3)
    s0 = g.get_state()
    g.select_kernels(VARIANTS["fused"] | SCATTER)
    assert np.array_equal(g.residual(u), r0)
    g.set_state(u)
    g.step(3)
    assert np.array_equal(g.get_state(), s0)
    if prec == "fp64":
        assert rel_err(r0, o.residual(u)) <= 1e-12
    g.close()


def test_scatter_exchange_rejected_without_fused_stage():
    g = FRMesh(case("tgv_p2"), "fp64")
    with pytest.raises(_lib.FRError) as e:
        g.select_kernels(VARIANTS["tensor"] | SCATTER)
    assert e.value.code == _lib.FR_E_UNSUPPORTED
    g.close()


def test_tile_shapes_rejected_where_not_compiled():
    g = FRMesh(case("vortex2d_p3"), "fp32")
    with pytest.raises(_lib.FRError) as e:
        g.select_kernels(VARIANTS["fused"] | (1 << 9))
    assert e.value.code == _lib.FR_E_UNSUPPORTED
    g.close()

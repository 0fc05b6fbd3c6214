"""Pins of the oracle's variable per-element order: faces shared by elements of
different orders carry a mortar (the low order's trace and half viscous flux
interpolated to the high order's face points, the high side's common flux projected
in L2 onto the low order's face polynomials).

* free-stream preservation on curved meshes with every order pair 1..4 adjacent and
  re-oriented elements, and on an O-grid whose order falls toward the far field;
* discrete conservation to round-off on periodic curved meshes (needs the projection
  to keep the high side's face integral, also for P1 next to P4, where interpolation
  at the low order's points would not);
* exactness of the corrected gradient for a state linear in space on straight-sided
  meshes with re-oriented elements (pins the face orientation map, the interpolation
  up and the projection down);
* exactness of the residual of a viscous shear flow (viscous heating only), which
  needs both halves of the common viscous flux across mixed faces;
* a mixed mesh whose orders are all equal gives the uniform oracle's residual exactly;
* isentropic vortex: P3 where the vortex sits and P2 around it is as accurate as
  uniform P3 and far more accurate than uniform P2.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleMesh, basis
from paper_2501_05709_amd import workloads as W

G = 1.4


def flow(mesh, mu=0.0):
    mesh = dict(mesh)
    mesh.update(gamma=G, prandtl=0.72, mu=mu)
    return mesh


def rotate_element(conn, q, dim, rot):
    """Re-order one element's node list by a proper rotation of the reference cell."""
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


def mixed_box(dim, q, warp, seed=0, rotate=True, mu=0.0, lo=1, nel=None):
    """Box of curved (warp) elements with random orders lo..4, the first row holding
    orders lo, 4, 2, 3 (P1 next to P4 when lo = 1), every other element re-oriented."""
    nel = nel or ((4, 4) if dim == 2 else (3, 3, 2))
    m = flow(W.box_mesh(dim, nel, (0,) * dim, (1.0,) * dim, q=q, warp=warp, order=4), mu=mu)
    E = len(m["elem_nodes"])
    rng = np.random.default_rng(seed)
    orders = rng.integers(lo, 5, size=E)
    orders[:4] = (lo, 4, 2, 3)
    m["orders"] = orders.astype(np.int32)
    if rotate:
        rots = ROT2 if dim == 2 else ROT3
        conn = m["elem_nodes"].copy()
        for e in range(1, E, 2):
            conn[e] = rotate_element(conn[e], q, dim, rots[(e // 2) % len(rots)])
        m["elem_nodes"] = conn
    return m


def weights(o):
    """Quadrature weight times |J| at every solution point of a mixed mesh."""
    detJ, _, _ = o.metrics()
    ws = []
    for p in o.mesh["orders"]:
        w = basis(int(p))["w"]
        ws.append(np.outer(w, w).ravel() if o.dim == 2 else np.einsum("k,j,i->kji", w, w, w).ravel())
    return np.concatenate(ws) * detJ


def smooth(x, dim, amp=1.0):
    X, Y = x[..., 0], x[..., 1]
    rho = 1.0 + 0.1 * amp * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    vel = [0.3 + 0.1 * amp * np.cos(2 * np.pi * Y), -0.2 + 0.1 * amp * np.sin(2 * np.pi * (X + Y))]
    if dim == 3:
        vel.append(0.1 + 0.05 * amp * np.cos(2 * np.pi * (X - x[..., 2])))
    p = 1.0 + 0.1 * amp * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    return W.conserved(rho, vel, p)


# P1 on curved (quadratic) 3D elements does not preserve a free stream even with one
# order everywhere (its metric terms miss the discrete metric identities), so the curved
# 3D case mixes orders 2..4; the others include P1
@pytest.mark.parametrize("dim,q,warp,lo", [(2, 2, 0.06, 1), (3, 1, 0.0, 1), (3, 2, 0.05, 2)])
def test_mixed_free_stream_preservation(dim, q, warp, lo):
    m = mixed_box(dim, q, warp, mu=0.02, lo=lo)
    o = OracleMesh(m)
    assert o.n_mortar > 0
    rng = np.random.default_rng(dim)
    rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
    u = W.uniform_state(o.NU, rho, list(rng.uniform(-0.5, 0.5, size=dim)), p)
    r = o.residual(u)
    assert np.abs(r).max() < 1e-12 * (rho + p) * 4 * 10


def test_mixed_free_stream_preservation_ogrid():
    """Order falling from 3 at the wall to 0 at the far field, as the paper lowers it
    toward the boundaries; inner and outer boundary both far field."""
    ni, nj, nk = 24, 8, 2
    m = W.naca_ogrid(0.04, 0.4, 0.12, ni, nj, nk, inner_bc=W.BC_FARFIELD, outer_bc=W.BC_FARFIELD)
    m.update(W.airfoil_flow())
    m["orders"] = W.ring_orders(ni, nj, nk, ((2, 3), (4, 2), (6, 1), (8, 0)))
    o = OracleMesh(m)
    assert o.n_mortar == 3 * ni * nk
    fs = m["freestream"]
    r = o.residual(W.uniform_state(o.NU, fs[0], fs[1:4], fs[4]))
    assert np.abs(r).max() < 1e-9 * fs[4]


@pytest.mark.parametrize("dim,q,warp,lo", [(2, 2, 0.06, 1), (3, 1, 0.0, 1), (3, 2, 0.04, 1), (2, 2, 0.06, 0),
                                           (3, 1, 0.0, 0)])
def test_mixed_conservation(dim, q, warp, lo):
    m = mixed_box(dim, q, warp, seed=5, mu=0.05, lo=lo)
    o = OracleMesh(m)
    x = o.solution_points()
    u = smooth(x, dim) + 0.01 * np.random.default_rng(1).standard_normal((o.NU, o.nv))
    r = o.residual(u)
    wj = weights(o)
    tot = wj @ r
    scale = np.abs(wj) @ np.abs(r)
    assert np.all(np.abs(tot) <= 1e-13 * scale + 1e-15), tot / scale


@pytest.mark.parametrize("dim", [2, 3])
def test_mixed_gradient_of_linear_state_is_exact(dim):
    """Away from the periodic faces (where a linear state jumps) every element's
    corrected gradient is exact: its neighbours' traces, brought across mixed faces by
    the orientation map and the interpolation or projection, equal its own."""
    nel = (6, 6) if dim == 2 else (4, 4, 4)
    m = mixed_box(dim, 1, 0.0, seed=2, nel=nel)
    o = OracleMesh(m)
    assert o.n_mortar > 0
    x = o.solution_points()[:, :dim]
    rng = np.random.default_rng(7)
    a = rng.uniform(1.0, 2.0, size=o.nv)
    b = rng.uniform(-0.3, 0.3, size=(dim, o.nv))
    u = a[None, :] + x @ b
    g = o.gradient(u)
    n_pts = (m["orders"] + 1) ** dim
    owner = np.repeat(np.arange(len(n_pts)), n_pts)
    ijk = np.stack([(owner // int(np.prod(nel[:k]))) % nel[k] for k in range(dim)], axis=1)
    inner = np.all((ijk > 0) & (ijk < np.array(nel) - 1), axis=1)
    assert inner.sum() > 0
    assert np.abs(g[inner][:, :dim, :] - b[None]).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_mixed_viscous_shear_residual_is_exact(dim):
    """Uniform density and pressure with velocity (b y, 0, 0): the exact residual is 0
    except viscous heating mu b^2 in the energy.  The state is a polynomial of degree 2
    (orders 2..4 hold it exactly), so away from the periodic faces (two elements deep:
    the common viscous flux reads the neighbour's gradient) the discrete residual equals
    it, which needs both halves of the common viscous flux on the mixed faces."""
    nel = (6, 6) if dim == 2 else (6, 6, 5)
    mu, b = 0.05, 0.7
    m = mixed_box(dim, 1, 0.0, seed=4, nel=nel, mu=mu, lo=2)
    o = OracleMesh(m)
    assert o.n_mortar > 0
    y = o.solution_points()[:, 1]
    vel = [b * y, 0.0 * y] + ([0.0 * y] if dim == 3 else [])
    u = W.conserved(np.ones_like(y), vel, np.full_like(y, 2.0))
    r = o.residual(u)
    n_pts = (m["orders"] + 1) ** dim
    owner = np.repeat(np.arange(len(n_pts)), n_pts)
    ijk = np.stack([(owner // int(np.prod(nel[:k]))) % nel[k] for k in range(dim)], axis=1)
    deep = np.all((ijk > 1) & (ijk < np.array(nel) - 2), axis=1)
    assert deep.sum() > 0
    expect = np.zeros(o.nv)
    expect[-1] = mu * b * b
    assert np.abs(r[deep] - expect[None]).max() < 1e-11


def test_mixed_with_equal_orders_is_the_uniform_scheme():
    m = mixed_box(3, 2, 0.05, seed=3, mu=0.03)
    m["orders"] = np.full(len(m["elem_nodes"]), 3, dtype=np.int32)
    um = dict(m)
    um.pop("orders")
    um["order"] = 3
    om, ou = OracleMesh(m), OracleMesh(um)
    assert om.n_mortar == 0
    u = smooth(ou.solution_points(), 3)
    assert np.array_equal(om.residual(u.reshape(-1, 5)), ou.residual(u).reshape(-1, 5))


def test_mixed_vortex_accuracy():
    """Euler vortex on periodic [-10, 10]^2 (12 x 12 elements) to t = 0.5: P3 inside
    |x|, |y| < 5 and P2 outside, against uniform P2 and P3."""
    nel, t_end, dt = 12, 0.5, 5e-3

    def err(orders):
        m = flow(W.box_mesh(2, (nel, nel), (-10.0, -10.0), (10.0, 10.0), order=3), mu=0.0)
        m["orders"] = orders
        o = OracleMesh(m)
        xy = o.solution_points()[:, :2]
        u1 = o.rk4(W.vortex_state(xy), dt, int(round(t_end / dt)))
        uex = W.vortex_state(xy, t=t_end, period=(20.0, 20.0))
        wj = weights(o)
        return math.sqrt(np.sum(wj * (u1[:, 0] - uex[:, 0]) ** 2) / np.sum(wj))

    ij = np.arange(nel * nel)
    cx = -10.0 + (20.0 / nel) * (ij % nel + 0.5)
    cy = -10.0 + (20.0 / nel) * (ij // nel + 0.5)
    inner = (np.abs(cx) < 5.0) & (np.abs(cy) < 5.0)
    e_mixed = err(np.where(inner, 3, 2).astype(np.int32))
    e2 = err(np.full(nel * nel, 2, dtype=np.int32))
    e3 = err(np.full(nel * nel, 3, dtype=np.int32))
    print(f"vortex L2 error: uniform P2 {e2:.3e}, mixed {e_mixed:.3e}, uniform P3 {e3:.3e}")
    assert e_mixed < 0.5 * e2 and e_mixed < 2.0 * e3


# --------------------------------------------------------------------------
# order 0: one solution point per element, a finite volume
# --------------------------------------------------------------------------

def fv_rusanov(uL, uR, n, dim):
    """Rusanov flux of the Euler equations (the textbook formula, written out here)."""
    def parts(u):
        rho = u[..., 0]
        v = u[..., 1:1 + dim] / rho[..., None]
        p = (G - 1.0) * (u[..., -1] - 0.5 * rho * (v * v).sum(-1))
        vn = (v * n).sum(-1)
        F = np.empty_like(u)
        F[..., 0] = rho * vn
        F[..., 1:1 + dim] = u[..., 1:1 + dim] * vn[..., None] + p[..., None] * n
        F[..., -1] = (u[..., -1] + p) * vn
        return F, np.abs(vn) + np.sqrt(G * p / rho)
    FL, aL = parts(uL)
    FR, aR = parts(uR)
    lam = np.maximum(aL, aR)[..., None]
    return 0.5 * (FL + FR) - 0.5 * lam * (uR - uL)


@pytest.mark.parametrize("dim", [2, 3])
def test_p0_is_the_rusanov_finite_volume_scheme(dim):
    """On a periodic Cartesian box, order 0 is the first-order finite volume scheme:
    R_e = -(1/V) sum over faces of area x Rusanov flux (inviscid)."""
    nel = (5, 4) if dim == 2 else (4, 3, 3)
    hi = (1.0, 0.7, 0.5)[:dim]
    m = flow(W.box_mesh(dim, nel, (0,) * dim, hi, order=0), mu=0.0)
    o = OracleMesh(m)
    x = o.solution_points().reshape(-1, 3)
    u = smooth(x, dim) + 0.02 * np.random.default_rng(3).standard_normal((len(x), o.nv))
    r = o.residual(u).reshape(-1, o.nv)
    h = np.array(hi) / np.array(nel)
    ugrid = u.reshape(tuple(reversed(nel)) + (o.nv,))       # [k][j][i] (element e = i + nx (j + ny k))
    expect = np.zeros_like(ugrid)
    for k in range(dim):
        ax = dim - 1 - k                                       # array axis of coordinate k
        n = np.zeros(dim)
        n[k] = 1.0
        area = np.prod(h) / h[k]
        Fp = fv_rusanov(ugrid, np.roll(ugrid, -1, axis=ax), n, dim)   # through the + face
        Fm = np.roll(Fp, 1, axis=ax)                                   # the - face is the neighbour's +
        expect -= area * (Fp - Fm) / np.prod(h)
    assert np.abs(r - expect.reshape(-1, o.nv)).max() <= 1e-12 * np.abs(expect).max()


def test_p0_gradient_is_the_central_difference():
    """The BR1 corrected gradient at order 0 on a periodic Cartesian box is the central
    difference (u[i+1] - u[i-1]) / (2 h) along each axis."""
    nel, hi = (6, 5), (1.2, 1.0)
    m = flow(W.box_mesh(2, nel, (0, 0), hi, order=0), mu=0.01)
    o = OracleMesh(m)
    u = 1.0 + np.random.default_rng(4).uniform(0.0, 1.0, size=(o.E, o.nv))
    g = o.gradient(u).reshape(nel[1], nel[0], 3, o.nv)
    ug = u.reshape(nel[1], nel[0], o.nv)
    h = np.array(hi) / np.array(nel)
    cdx = (np.roll(ug, -1, axis=1) - np.roll(ug, 1, axis=1)) / (2 * h[0])
    cdy = (np.roll(ug, -1, axis=0) - np.roll(ug, 1, axis=0)) / (2 * h[1])
    assert np.abs(g[:, :, 0] - cdx).max() < 1e-12 * np.abs(cdx).max()
    assert np.abs(g[:, :, 1] - cdy).max() < 1e-12 * np.abs(cdy).max()

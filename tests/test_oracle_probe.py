"""Pins of the sampling oracle (oracle/probe.py): point location and the FR interpolant.

* Axis-aligned box mesh: the containing element and the reference coordinates of any
  point follow in closed form from the grid spacing.
* A polynomial state of degree <= p in each coordinate on an affine mesh is reproduced
  exactly at any point (the interpolant through n = p + 1 Gauss-Legendre points per
  axis is exact for such polynomials).
* Curved meshes: sampling at the solution points that the C oracle places (its own
  geometry code) returns the nodal values.
"""
import numpy as np
import pytest

from oracle import probe
from oracle.oracle import OracleMesh
from paper_2501_05709_amd import workloads as W


def test_box_location_closed_form():
    lo, hi, nel = np.array([0.0, 0.0, 0.0]), np.array([1.5, 1.0, 0.8]), np.array([3, 2, 4])
    m = W.box_mesh(3, tuple(nel), tuple(lo), tuple(hi), q=1, order=2)
    rng = np.random.default_rng(1)
    pts = lo + (hi - lo) * rng.uniform(0.01, 0.99, size=(40, 3))
    elem, xi = probe.locate(m, pts)
    h = (hi - lo) / nel
    c = np.floor((pts - lo) / h).astype(int)
    assert np.array_equal(elem, c[:, 0] + nel[0] * (c[:, 1] + nel[1] * c[:, 2]))
    assert np.allclose(xi, 2.0 * ((pts - lo) / h - c) - 1.0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_polynomial_state_is_exact(order):
    m = W.box_mesh(3, (2, 3, 2), (0.0, 0.0, 0.0), (1.0, 1.2, 0.9), q=1, order=order)
    o = OracleMesh(dict(m, gamma=1.4, prandtl=0.72, mu=0.0, freestream=np.array([1.0, 0, 0, 0, 1.0]), dt=1e-3))
    x = o.solution_points()
    rng = np.random.default_rng(order)
    coef = rng.normal(size=(5, 3, order + 1))

    def field(p):
        out = np.zeros(p.shape[:-1] + (5,))
        for v in range(5):
            val = np.ones(p.shape[:-1])
            for k in range(3):
                val = val * np.polynomial.polynomial.polyval(p[..., k], coef[v, k])
            out[..., v] = val
        return out

    u = field(x)
    pts = rng.uniform([0.05, 0.05, 0.05], [0.95, 1.15, 0.85], size=(30, 3))
    elem, xi = probe.locate(m, pts)
    got = probe.sample(u, order, elem, xi, 3)
    assert np.allclose(got, field(pts), rtol=1e-12, atol=1e-12 * np.abs(u).max())


@pytest.mark.parametrize("name", ["box2d_curved", "airfoil"])
def test_solution_points_return_nodal_values(name):
    if name == "box2d_curved":
        m = W.box_mesh(2, (4, 3), (0, 0), (1, 1), q=2, warp=0.05, order=3)
        m.update(gamma=1.4, prandtl=0.72, mu=0.0, freestream=np.array([1.0, 0.2, 0.1, 0.0, 1.0]), dt=1e-3)
    else:
        m = W.config_airfoil(3, ni=16, nj=4, nk=2)
    o = OracleMesh(m)
    x = o.solution_points()
    rng = np.random.default_rng(0)
    u = rng.normal(size=o.shape)
    es = rng.choice(o.E, size=6, replace=False)
    pts = np.concatenate([x[e] for e in es])[:, :m["dim"]]
    # keep points off shared faces: solution points are interior (Gauss-Legendre)
    elem, xi = probe.locate(m, pts)
    got = probe.sample(u, m["order"], elem, xi, m["dim"])
    assert np.array_equal(elem, np.repeat(es, o.nu))
    assert np.allclose(got, np.concatenate([u[e] for e in es]), rtol=0, atol=1e-10)


def test_variable_order_state_is_exact():
    """Per-element orders 0..4 on an affine box: a field that is a polynomial of degree
    <= p_e in each coordinate inside element e (here: each element's own polynomial of
    its order, discontinuous across elements) is reproduced exactly at any point."""
    m = W.box_mesh(3, (3, 2, 2), (0.0, 0.0, 0.0), (1.2, 1.0, 0.8), q=1, order=4)
    rng = np.random.default_rng(7)
    E = len(m["elem_nodes"])
    orders = rng.integers(0, 5, size=E).astype(np.int32)
    mm = dict(m, orders=orders, gamma=1.4, prandtl=0.72, mu=0.0, freestream=np.array([1.0, 0, 0, 0, 1.0]), dt=1e-3)
    o = OracleMesh(mm)
    x = o.solution_points()
    off = np.concatenate([[0], np.cumsum((orders + 1) ** 3)])
    coefs = [rng.normal(size=(5, 3, int(p) + 1)) for p in orders]

    def field(e, p):
        out = np.zeros(p.shape[:-1] + (5,))
        for v in range(5):
            val = np.ones(p.shape[:-1])
            for k in range(3):
                val = val * np.polynomial.polynomial.polyval(p[..., k], coefs[e][v, k])
            out[..., v] = val
        return out

    u = np.concatenate([field(e, x[off[e]:off[e + 1]]) for e in range(E)])
    pts = np.array([1.2, 1.0, 0.8]) * rng.uniform(0.02, 0.98, size=(60, 3))
    elem, xi = probe.locate(mm, pts)
    got = probe.sample(u, orders, elem, xi, 3)
    want = np.array([field(int(e), p) for e, p in zip(elem, pts)])
    assert np.allclose(got, want, rtol=1e-11, atol=1e-11)

"""Test infrastructure only: plain numpy oracle of sampling the FR solution at points.

Only tests, ``__graft_entry__.smoke`` and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the HIP path.

The FR solution inside an element is the tensor-product Lagrange interpolant through
its Gauss-Legendre solution points (the FR definition of the discrete solution).  A
point is located by Newton's method on the element's geometry map (equispaced Lagrange
nodes of order q, the mesh convention of include/fr.h), trying the elements in index
order and taking the first whose reference cube [-1, 1]^d holds the point; the sample
is the interpolant there.  This is how flow samples on the paper's permeable data
surface (Section 3.1) come out of the solution.
"""
from __future__ import annotations

import numpy as np


def _shape(q, t):
    """Equispaced Lagrange shape functions of order q on [-1, 1] and their derivatives."""
    nodes = np.linspace(-1.0, 1.0, q + 1)
    N = np.ones(q + 1)
    dN = np.zeros(q + 1)
    for a in range(q + 1):
        for b in range(q + 1):
            if b == a:
                continue
            term = 1.0 / (nodes[a] - nodes[b])
            dsum = term
            for c in range(q + 1):
                if c != a and c != b:
                    dsum *= (t - nodes[c]) / (nodes[a] - nodes[c])
            dN[a] += dsum
            N[a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return N, dN


def geometry(X, q, dim, r):
    """x(r) and dx/dr for an element with node coordinates X [(q+1)^dim, dim]."""
    sh = [_shape(q, r[k]) for k in range(dim)]
    na = q + 1
    x = np.zeros(dim)
    J = np.zeros((dim, dim))  # J[i, k] = dx_i / dr_k
    for idx in range(na ** dim):
        c = [(idx // na ** k) % na for k in range(dim)]
        val = np.prod([sh[k][0][c[k]] for k in range(dim)])
        x += val * X[idx]
        for k in range(dim):
            dv = np.prod([sh[kk][1][c[kk]] if kk == k else sh[kk][0][c[kk]] for kk in range(dim)])
            J[:, k] += dv * X[idx]
    return x, J


def locate(mesh, points, tol=1e-10):
    """(element, reference coordinates) of each point: the lowest-index element whose
    reference cube holds it.  Raises if a point lies in no element."""
    dim = mesh["dim"]
    q = mesh.get("geom_order", mesh.get("q", 1))
    nodes = np.asarray(mesh["nodes"], dtype=np.float64)[:, :dim]
    conn = np.asarray(mesh["elem_nodes"])
    lo = nodes[conn].min(axis=1)
    hi = nodes[conn].max(axis=1)
    pad = 0.1 * (hi - lo).max(axis=1, keepdims=True)
    elem = np.zeros(len(points), dtype=np.int64)
    xi = np.zeros((len(points), 3))
    for i, p in enumerate(np.asarray(points, dtype=np.float64)[:, :dim]):
        cand = np.nonzero(np.all((p >= lo - pad) & (p <= hi + pad), axis=1))[0]
        found = False
        for e in cand:
            X = nodes[conn[e]]
            r = np.zeros(dim)
            ok = False
            prev = np.inf
            for _ in range(50):
                x, J = geometry(X, q, dim, r)
                dr = np.linalg.solve(J, p - x)
                r = r + dr
                step = np.abs(dr).max()
                # converged: below 1e-14, or at the round-off floor (below 1e-10 and no
                # longer shrinking), which thin curved elements put above 1e-14
                if step < 1e-14 or (step < 1e-10 and step >= prev):
                    ok = True
                    break
                if np.abs(r).max() > 3.0:
                    break
                prev = step
            if ok and np.abs(r).max() <= 1.0 + tol:
                elem[i] = e
                xi[i, :dim] = r
                found = True
                break
        if not found:
            raise ValueError(f"point {i} lies in no element")
    return elem, xi


def sample(u, order, elem, xi, dim):
    """Interpolant of the canonical state u [E][n^dim][V] at (elem, xi).

    ``order`` may be an array of per-element orders; u is then the ragged state
    [sum of n_e^dim][V] with element e's points contiguous, in element order."""
    if np.ndim(order) == 1:
        orders = np.asarray(order)
        off = np.concatenate([[0], np.cumsum((orders + 1) ** dim)])
        out = np.zeros((len(elem), u.shape[-1]))
        for i, (e, r) in enumerate(zip(elem, xi)):
            ue = u[off[e]:off[e + 1]][None]
            out[i] = sample(ue, int(orders[e]), np.array([0]), np.asarray(r)[None], dim)[0]
        return out
    n = order + 1
    x = np.polynomial.legendre.leggauss(n)[0]
    out = np.zeros((len(elem), u.shape[-1]))
    for i, (e, r) in enumerate(zip(elem, xi)):
        ls = []
        for k in range(dim):
            lk = np.ones(n)
            for j in range(n):
                for m in range(n):
                    if m != j:
                        lk[j] *= (r[k] - x[m]) / (x[j] - x[m])
            ls.append(lk)
        w = ls[0]
        for k in range(1, dim):
            w = np.multiply.outer(ls[k], w)   # index i0 + n i1 (+ n^2 i2), i0 fastest
        out[i] = w.ravel() @ u[e]
    return out

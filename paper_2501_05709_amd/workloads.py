"""Seeded synthetic workloads: meshes, initial states and flow constants.

This module holds no part of the flux reconstruction arithmetic.  It builds
the inputs that both the GPU library and the independent CPU oracle consume:

* ``box_mesh``      periodic straight (optionally warped, quadratic) boxes;
* ``naca_ogrid``    spanwise-periodic O-grids of quadratic hexahedra around a
                    NACA 4-digit profile (the airfoil family of the paper's
                    Section 3 and its design vector, Section 3.4);
* initial states    the isentropic vortex, the Taylor-Green vortex and a
                    uniform free stream;
* ``config_*``      the five benchmark workloads (vortex, Taylor-Green,
                    single airfoil, batch of airfoils, served request trace).

A mesh is a plain dict that mirrors the C descriptor ``fr_mesh_desc``:
``dim, order, q, nodes[n_nodes, dim] (f64), elem_nodes[E, (q+1)^dim] (i64,
lexicographic, xi fastest), periodic[n_periodic, dim] (f64 translations),
bfaces[n_bfaces, 3] (i64: element, local face, kind), gamma, prandtl, mu,
freestream[5] (rho, u, v, w, p), ref_area, lift_dir[3], drag_dir[3], dt``.
Local face f = 2k + s lies on reference axis k at xi_k = -1 (s = 0) or +1
(s = 1).  Boundary kinds: 1 = no-slip adiabatic wall, 2 = far field.

Random draws use ``numpy.random.default_rng(seed)`` in the order documented
on each function.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4
BC_WALL = 1
BC_FARFIELD = 2


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def _node_grid(dims):
    ids = np.arange(int(np.prod(dims)), dtype=np.int64)
    return ids.reshape(tuple(reversed(dims)))  # index [k][j][i]


def box_mesh(dim, nel, lo, hi, q=1, warp=0.0, order=3):
    """Structured box of ``nel`` elements per axis, periodic on every axis.

    ``warp`` > 0 displaces the nodes by a smooth field that is periodic over
    the box (so periodic faces still match by translation); with q = 2 the
    elements are then curved.  In 3D the displacement depends on x and y only
    (extruded curvature), which keeps the analytic metric terms polynomial.
    """
    nel = tuple(int(v) for v in nel)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    npts = [n * q + 1 for n in nel]
    axes = [np.linspace(lo[k], hi[k], npts[k]) for k in range(dim)]
    if dim == 2:
        Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
        coords = [X, Y]
    else:
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        coords = [X, Y, Z]
    if warp:
        L = hi - lo
        sx = np.sin(2 * np.pi * (coords[0] - lo[0]) / L[0])
        sy = np.sin(2 * np.pi * (coords[1] - lo[1]) / L[1])
        dx = warp * L[0] * sx * sy
        dy = warp * L[1] * np.sin(2 * np.pi * (coords[0] - lo[0]) / L[0] + 0.3) * sy
        coords[0] = coords[0] + dx
        coords[1] = coords[1] + dy
    nodes = np.stack([c.ravel() for c in coords], axis=1)
    grid = _node_grid(npts)
    na = q + 1
    elems = []
    if dim == 2:
        for J in range(nel[1]):
            for I in range(nel[0]):
                sub = grid[J * q:J * q + na, I * q:I * q + na]
                elems.append(sub.ravel())
    else:
        for K in range(nel[2]):
            for J in range(nel[1]):
                for I in range(nel[0]):
                    sub = grid[K * q:K * q + na, J * q:J * q + na, I * q:I * q + na]
                    elems.append(sub.ravel())
    periodic = np.diag(hi - lo)[:dim, :dim].copy()
    return dict(dim=dim, order=order, q=q, nodes=nodes, elem_nodes=np.array(elems, dtype=np.int64),
                periodic=periodic, bfaces=np.zeros((0, 3), dtype=np.int64))


def naca4(m, pc, t, theta):
    """NACA 4-digit surface point for parameter theta in [0, 2 pi).

    theta in [0, pi] is the lower surface (trailing edge to leading edge),
    theta in (pi, 2 pi) the upper one, so increasing theta runs clockwise.
    With u = theta/pi (lower) or 2 - theta/pi (upper), x = 1 - sin(pi u / 2):
    about uniform spacing at the trailing edge, clustering at the leading
    edge.  Closed trailing edge (last thickness coefficient -0.1036).
    """
    theta = np.asarray(theta, dtype=np.float64)
    u = np.where(theta <= np.pi, theta / np.pi, 2.0 - theta / np.pi)
    x = np.clip(1.0 - np.sin(0.5 * np.pi * u), 0.0, 1.0)
    yt = 5.0 * t * (0.2969 * np.sqrt(np.maximum(x, 0.0)) - 0.1260 * x - 0.3516 * x ** 2
                    + 0.2843 * x ** 3 - 0.1036 * x ** 4)
    if m != 0.0:  # negative m: camber below the chord
        yc = np.where(x < pc, m / pc ** 2 * (2 * pc * x - x ** 2),
                      m / (1 - pc) ** 2 * ((1 - 2 * pc) + 2 * pc * x - x ** 2))
        dyc = np.where(x < pc, 2 * m / pc ** 2 * (pc - x), 2 * m / (1 - pc) ** 2 * (pc - x))
    else:
        yc = np.zeros_like(x)
        dyc = np.zeros_like(x)
    phi = np.arctan(dyc)
    upper = np.sin(theta) < 0.0
    sgn = np.where(upper, 1.0, -1.0)
    xs = x - sgn * yt * np.sin(phi)
    ys = yc + sgn * yt * np.cos(phi)
    return xs, ys


def naca_ogrid(m, pc, t, ni, nj, nk, span=0.2, radius=20.0, ratio=1.1, q=2, order=3,
               inner_bc=BC_WALL, outer_bc=BC_FARFIELD):
    """O-grid of ni x nj x nk hexahedra of geometric order q around a NACA profile.

    i runs clockwise around the profile (periodic through shared node ids),
    j runs outward along straight rays to a circle of ``radius`` about
    (0.5, 0) with geometric growth ``ratio``, k runs over the span (periodic
    by the translation (0, 0, span)).  Nodes at half indices come from the
    same analytic maps, so the quadratic elements follow the profile.
    """
    nIq, nJq, nKq = ni * q, nj * q + 1, nk * q + 1
    theta = 2.0 * np.pi * np.arange(nIq) / nIq
    xs, ys = naca4(m, pc, t, theta)
    # the outer points near the trailing edge turn with its bisector (camber slope at
    # x = 1) so that the rays leaving it split its wedge; the turn fades out quickly
    # away from it, since turned rays from the mid-chord would cut across an aft-
    # cambered body or the nose.  Strong camber far aft (|m| >= 0.05 at pc = 0.9)
    # still folds elements at the trailing edge: the library rejects such meshes
    # (non-positive Jacobian)
    phi = math.atan(-2.0 * m / (1.0 - pc)) * (0.5 * (1.0 + np.cos(theta))) ** 8
    ox = 0.5 + radius * np.cos(phi - theta)
    oy = radius * np.sin(phi - theta)
    jj = np.arange(nJq) / q
    frac = (ratio ** jj - 1.0) / (ratio ** nj - 1.0)
    X = xs[None, :] + frac[:, None] * (ox - xs)[None, :]
    Y = ys[None, :] + frac[:, None] * (oy - ys)[None, :]
    zz = span * np.arange(nKq) / (nk * q)
    nodes = np.zeros((nKq, nJq, nIq, 3))
    nodes[..., 0] = X[None, :, :]
    nodes[..., 1] = Y[None, :, :]
    nodes[..., 2] = zz[:, None, None]
    nodes = nodes.reshape(-1, 3)

    def nid(i, j, k):
        return (k * nJq + j) * nIq + (i % nIq)

    na = q + 1
    a = np.arange(na)
    A2, A1, A0 = np.meshgrid(a, a, a, indexing="ij")
    A0, A1, A2 = A0.ravel(), A1.ravel(), A2.ravel()
    K, J, I = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    elem = nid(I[:, None] * q + A0[None, :], J[:, None] * q + A1[None, :], K[:, None] * q + A2[None, :])
    eid = np.arange(ni * nj * nk).reshape(nk, nj, ni)
    inner = eid[:, 0, :].ravel()
    outer = eid[:, nj - 1, :].ravel()
    bfaces = np.concatenate([
        np.stack([inner, np.full_like(inner, 2), np.full_like(inner, inner_bc)], 1),
        np.stack([outer, np.full_like(outer, 3), np.full_like(outer, outer_bc)], 1)]).astype(np.int64)
    return dict(dim=3, order=order, q=q, nodes=nodes, elem_nodes=elem.astype(np.int64),
                periodic=np.array([[0.0, 0.0, span]]), bfaces=bfaces, grid=(ni, nj, nk))


def ring_orders(ni, nj, nk, bands):
    """Per-element orders of a ``naca_ogrid`` mesh by radial layer j: ``bands`` is a
    list of (first layer beyond the band, order), e.g. ((16, 3), (32, 2), (48, 1)) gives
    P3 in layers 0-15, P2 in 16-31 and P1 beyond (element (i, j, k) is
    (k nj + j) ni + i)."""
    j = (np.arange(ni * nj * nk) // ni) % nj
    out = np.full(j.shape, bands[-1][1], dtype=np.int32)
    lo = 0
    for hi, p in bands:
        out[(j >= lo) & (j < hi)] = p
        lo = hi
    return out


def min_width(mesh, order=None):
    """Smallest element width across a pair of opposite faces, 2|J| / |grad_x xi_k|^-1,
    over the Gauss-Legendre points of the mesh's order (captures sliver elements)."""
    q, d = mesh["q"], mesh["dim"]
    order = mesh["order"] if order is None else order
    xg, _ = np.polynomial.legendre.leggauss(order + 1)
    nodes1 = np.linspace(-1.0, 1.0, q + 1)

    def shape(t):
        N = np.ones((len(t), q + 1))
        dN = np.zeros((len(t), q + 1))
        for a in range(q + 1):
            for b in range(q + 1):
                if b != a:
                    N[:, a] *= (t - nodes1[b]) / (nodes1[a] - nodes1[b])
            for c in range(q + 1):
                if c == a:
                    continue
                term = np.full(len(t), 1.0 / (nodes1[a] - nodes1[c]))
                for b in range(q + 1):
                    if b != a and b != c:
                        term *= (t - nodes1[b]) / (nodes1[a] - nodes1[b])
                dN[:, a] += term
        return N, dN

    N, dN = shape(xg)
    na = q + 1
    n = len(xg)
    X = mesh["nodes"][mesh["elem_nodes"]]  # [E, na^d, d], node a = a0 + na a1 (+ na^2 a2)
    if d == 2:
        # W_k[point (i0 + n i1), node (a0 + na a1)]: derivative along axis k of the map
        W0 = np.einsum("ia,jb->jiba", dN, N).reshape(n * n, na * na)
        W1 = np.einsum("ia,jb->jiba", N, dN).reshape(n * n, na * na)
        c0 = np.matmul(W0, X)  # [E, points, 2]
        c1 = np.matmul(W1, X)
        det = c0[..., 0] * c1[..., 1] - c0[..., 1] * c1[..., 0]
        # width across the faces of axis k: 2 |J| / |column of the other axis|
        w0 = 2.0 * det / np.linalg.norm(c1, axis=-1)
        w1 = 2.0 * det / np.linalg.norm(c0, axis=-1)
        return float(min(w0.min(), w1.min()))
    shp = (n * n * n, na * na * na)
    W = [np.einsum("ia,jb,kc->kjicba", *fs).reshape(shp)
         for fs in ((dN, N, N), (N, dN, N), (N, N, dN))]
    cols = [np.matmul(Wk, X) for Wk in W]  # [E, points, 3]
    c = [[cols[k][..., i] for i in range(3)] for k in range(3)]

    def cross(u, v):
        return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])

    s = [cross(c[(k + 1) % 3], c[(k + 2) % 3]) for k in range(3)]  # |J| grad xi_k
    det = c[0][0] * s[0][0] + c[0][1] * s[0][1] + c[0][2] * s[0][2]
    best = np.inf
    for k in range(3):
        norm = np.sqrt(s[k][0] ** 2 + s[k][1] ** 2 + s[k][2] ** 2)
        best = min(best, float((2.0 * det / norm).min()))
    return best


def min_edge(mesh):
    """Shortest straight distance between adjacent corner nodes of any element."""
    q, d = mesh["q"], mesh["dim"]
    na = q + 1
    en = mesh["elem_nodes"]
    x = mesh["nodes"]
    best = np.inf
    for k in range(d):
        for lo_corner in range(2 ** (d - 1)):
            a = [0] * d
            others = [ax for ax in range(d) if ax != k]
            for bit, ax in enumerate(others):
                a[ax] = ((lo_corner >> bit) & 1) * q
            b = list(a)
            b[k] = q
            ia = sum(a[ax] * na ** ax for ax in range(d))
            ib = sum(b[ax] * na ** ax for ax in range(d))
            dist = np.linalg.norm(x[en[:, ib]] - x[en[:, ia]], axis=1)
            best = min(best, float(dist.min()))
    return best


# --------------------------------------------------------------------------
# initial states (conserved variables, [n_points, dim + 2])
# --------------------------------------------------------------------------

def conserved(rho, vel, p, gamma=GAMMA):
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.asarray(v, dtype=np.float64) for v in vel]
    ke = sum(v * v for v in vel)
    cols = [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + 0.5 * rho * ke]
    return np.stack(np.broadcast_arrays(*cols), axis=-1)


def vortex_state(xy, center=(0.0, 0.0), beta=5.0, uinf=None, gamma=GAMMA, t=0.0, period=None):
    """Isentropic vortex of strength beta advected along +x by uinf.

    rho_inf = p_inf = 1, so c_inf = sqrt(gamma) and the default
    uinf = 0.5 sqrt(gamma) is Mach 0.5.  ``t`` advects the centre; with
    ``period`` = (Lx, Ly) the nearest periodic image is used.
    """
    if uinf is None:
        uinf = 0.5 * math.sqrt(gamma)
    x = xy[:, 0] - center[0] - uinf * t
    y = xy[:, 1] - center[1]
    if period is not None:
        x = x - period[0] * np.round(x / period[0])
        y = y - period[1] * np.round(y / period[1])
    r2 = x * x + y * y
    f = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2 * np.pi) * f * y
    dv = beta / (2 * np.pi) * f * x
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return conserved(rho, [uinf + du, dv], p, gamma)


def tgv_state(xyz, mach=0.1, gamma=GAMMA):
    """Taylor-Green vortex, V0 = L = rho0 = 1, isothermal density."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p0 = 1.0 / (gamma * mach ** 2)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rho = p / p0
    return conserved(rho, [u, v, w], p, gamma)


def uniform_state(npts, rho, vel, p, gamma=GAMMA):
    st = conserved(rho, vel, p, gamma)
    return np.broadcast_to(st, (npts, st.shape[-1])).copy()


# --------------------------------------------------------------------------
# benchmark workloads
# --------------------------------------------------------------------------

def airfoil_flow(aoa_deg=5.0, mach=0.2, re=23000.0, pr=0.71, gamma=GAMMA, span=0.2):
    a = math.radians(aoa_deg)
    p_inf = 1.0 / (gamma * mach ** 2)
    return dict(gamma=gamma, prandtl=pr, mu=1.0 / re,
                freestream=np.array([1.0, math.cos(a), math.sin(a), 0.0, p_inf]),
                ref_area=1.0 * span, lift_dir=np.array([-math.sin(a), math.cos(a), 0.0]),
                drag_dir=np.array([math.cos(a), math.sin(a), 0.0]))


def airfoil_dt(mesh, order, cfl=0.5):
    """Fixed RK4 step: cfl h_min / ((|U| + c)(2p + 1)), h_min = smallest element width."""
    fs = mesh["freestream"]
    c = math.sqrt(mesh["gamma"] * fs[4] / fs[0])
    speed = float(np.linalg.norm(fs[1:4])) + c
    return cfl * min_width(mesh, order) / (speed * (2 * order + 1))


def config_vortex(seed=0, nel=16, order=3):
    """2D isentropic vortex on periodic [-5, 5]^2, Re 1000 on the domain length, Pr 0.72.

    Draws: centre offset (dx, dy) ~ U(-1, 1)^2.
    """
    rng = np.random.default_rng(seed)
    center = tuple(rng.uniform(-1.0, 1.0, size=2))
    mesh = box_mesh(2, (nel, nel), (-5.0, -5.0), (5.0, 5.0), q=1, order=order)
    uinf = 0.5 * math.sqrt(GAMMA)
    mesh.update(gamma=GAMMA, prandtl=0.72, mu=uinf * 10.0 / 1000.0,
                freestream=np.array([1.0, uinf, 0.0, 0.0, 1.0]), ref_area=1.0,
                lift_dir=np.array([0.0, 1.0, 0.0]), drag_dir=np.array([1.0, 0.0, 0.0]), dt=1e-3)
    mesh["init"] = lambda xyz: vortex_state(xyz[:, :2], center=center, uinf=uinf)
    mesh["center"] = center
    mesh["steps"] = 100
    return mesh


def config_tgv(nel=24, order=3, mach=0.1):
    """Taylor-Green vortex on periodic [0, 2 pi]^3, Re 1600, Pr 0.71, dt 1e-3."""
    L = 2.0 * np.pi
    mesh = box_mesh(3, (nel, nel, nel), (0.0, 0.0, 0.0), (L, L, L), q=1, order=order)
    mesh.update(gamma=GAMMA, prandtl=0.71, mu=1.0 / 1600.0,
                freestream=np.array([1.0, 0.0, 0.0, 0.0, 1.0 / (GAMMA * mach ** 2)]), ref_area=1.0,
                lift_dir=np.array([0.0, 1.0, 0.0]), drag_dir=np.array([1.0, 0.0, 0.0]), dt=1e-3)
    mesh["init"] = lambda xyz: tgv_state(xyz, mach=mach)
    mesh["steps"] = 200
    return mesh


def draw_airfoil(rng):
    """Design draw order: m ~ U(0, 0.06), pc ~ U(0.2, 0.6), t ~ U(0.08, 0.16)."""
    m = rng.uniform(0.0, 0.06)
    pc = rng.uniform(0.2, 0.6)
    t = rng.uniform(0.08, 0.16)
    return m, pc, t


def config_airfoil(seed=0, ni=160, nj=48, nk=8, order=3, design=None, aoa=5.0):
    """Spanwise-periodic NACA 4-digit O-grid, Re 23000, Mach 0.2, AoA 5 deg."""
    rng = np.random.default_rng(seed)
    m, pc, t = draw_airfoil(rng) if design is None else design
    mesh = naca_ogrid(m, pc, t, ni, nj, nk, order=order)
    mesh.update(airfoil_flow(aoa_deg=aoa))
    mesh["dt"] = airfoil_dt(mesh, order)
    fs = mesh["freestream"]
    mesh["init"] = lambda xyz: uniform_state(len(xyz), fs[0], fs[1:4], fs[4])
    mesh["design"] = (m, pc, t)
    mesh["steps"] = 2000
    return mesh


def config_batch(seed=0, n_designs=16, order=3, size_scale=1.0):
    """Sixteen airfoil designs with uneven O-grids.

    Draws per design, in order: m, pc, t (as ``draw_airfoil``), then
    n_i ~ U{96..192}, n_j ~ U{32..64}, n_k ~ U{4..12}.  ``size_scale`` < 1
    shrinks every grid dimension (for tests).
    """
    rng = np.random.default_rng(seed)
    meshes = []
    for _ in range(n_designs):
        design = draw_airfoil(rng)
        ni = int(rng.integers(96, 193))
        nj = int(rng.integers(32, 65))
        nk = int(rng.integers(4, 13))
        if size_scale != 1.0:
            ni = max(8, int(ni * size_scale))
            nj = max(3, int(nj * size_scale))
            nk = max(1, int(nk * size_scale))
        meshes.append(config_airfoil(ni=ni, nj=nj, nk=nk, order=order, design=design))
    return meshes


def request_trace(seed=0, n_requests=64, rate=4.0, size_scale=1.0, orders=(2, 3, 4)):
    """Poisson stream of airfoil solve requests.

    Draws per request, in order: interarrival ~ Exp(1/rate), m, pc, t,
    n_i ~ U{96..192}, n_j ~ U{32..64}, n_k ~ U{4..12}, order ~ U(orders).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        design = draw_airfoil(rng)
        ni = int(rng.integers(96, 193))
        nj = int(rng.integers(32, 65))
        nk = int(rng.integers(4, 13))
        order = int(orders[int(rng.integers(0, len(orders)))])
        if size_scale != 1.0:
            ni = max(8, int(ni * size_scale))
            nj = max(3, int(nj * size_scale))
            nk = max(1, int(nk * size_scale))
        out.append(dict(id=r, arrival=t, design=design, ni=ni, nj=nj, nk=nk, order=order))
    return out


def points_per_element(dim, order):
    return (order + 1) ** dim


# ---------------------------------------------------------------------------
# acoustic inputs: data surfaces and the exact fields of stationary sources in a
# uniform stream (the paper's verification cases, Appendix C)
# ---------------------------------------------------------------------------

def sphere_surface(radius=1.0, n_polar=30, n_azimuth=45):
    """Equal-area panels on a sphere: n_polar bands equal in cos(theta), n_azimuth panels
    per band.  Returns panel centres [n, 3], outward unit normals [n, 3], areas [n]."""
    c = np.linspace(1.0, -1.0, n_polar + 1)
    th = np.arccos(0.5 * (c[:-1] + c[1:]))
    ph = (np.arange(n_azimuth) + 0.5) * 2.0 * np.pi / n_azimuth
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    n = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1).reshape(-1, 3)
    area = 4.0 * np.pi * radius ** 2 / (n_polar * n_azimuth)
    return radius * n, n, np.full(n.shape[0], area)


def stationary_source(kind, x, t, mach, c0=340.75, rho0=1.234, amplitude=1.0, omega=10.0 * np.pi, axis=1):
    """Exact disturbance field of a stationary monopole or dipole at the origin of a
    stream of Mach vector `mach`.

    The potential is phi = A / (4 pi R*) exp(i omega (t - R / c0)) (monopole) or its
    derivative along `axis` (dipole), with the amplitude and phase radii R*, R of the
    stream; u = grad phi, p' = -rho0 (d/dt + c0 M . grad) phi and rho' = p' / c0^2.
    x [n, 3], t [nt] -> rho' [nt, n], u [nt, n, 3], p' [nt, n] (real parts).
    """
    x = np.asarray(x, dtype=np.float64)
    M = np.asarray(mach, dtype=np.float64)
    g2 = 1.0 / (1.0 - M @ M)
    k = omega / c0
    Mr = x @ M
    Rs = np.sqrt((x * x).sum(-1) + g2 * Mr ** 2) / np.sqrt(g2)
    R = g2 * (Rs - Mr)
    dRs = (x + g2 * Mr[:, None] * M) / (g2 * Rs[:, None])          # d R* / d x_i
    dR = g2 * (dRs - M)
    eye = np.eye(3)
    ddRs = ((eye + g2 * M[:, None] * M[None, :])[None] / (g2 * Rs[:, None, None])
            - dRs[:, :, None] * dRs[:, None, :] / Rs[:, None, None])
    ddR = g2 * ddRs
    f = np.exp(-1j * k * R) / Rs                                      # spatial factor
    g = -1j * k * dR - dRs / Rs[:, None]                              # grad f / f
    dg = -1j * k * ddR - ddRs / Rs[:, None, None] + dRs[:, :, None] * dRs[:, None, :] / Rs[:, None, None] ** 2
    df = f[:, None] * g                                               # d f / d x_i
    ddf = f[:, None, None] * (g[:, :, None] * g[:, None, :] + dg)     # d2 f / dx_i dx_j
    if kind == "monopole":
        s, ds = f, df
    elif kind == "dipole":
        s, ds = df[:, axis], ddf[:, :, axis]
    else:
        raise ValueError(kind)
    C = amplitude / (4.0 * np.pi)
    e = np.exp(1j * omega * np.asarray(t, dtype=np.float64))[:, None]
    u = np.real(C * e[:, :, None] * ds[None, :, :])
    p = np.real(-rho0 * C * e * (1j * omega * s + c0 * (ds @ M))[None, :])
    return p / c0 ** 2, u, p


def acoustic_case(kind="monopole", mach=(0.0, 0.0, 0.5), periods=12, dt_over_T=0.02, radius=1.0,
                  n_polar=30, n_azimuth=45, c0=340.75, rho0=1.234, gamma=GAMMA, omega=10.0 * np.pi,
                  amplitude=1.0):
    """Data-surface samples of a stationary source in a stream (the paper's verification
    set-up): sphere of `radius`, samples every dt = dt_over_T * period for `periods`."""
    pts, nrm, area = sphere_surface(radius, n_polar, n_azimuth)
    T = 2.0 * np.pi / omega
    dt = dt_over_T * T
    nt = int(round(periods / dt_over_T)) + 1
    t = dt * np.arange(nt)
    rho_p, u, p_p = stationary_source(kind, pts, t, mach, c0, rho0, amplitude=amplitude, omega=omega)
    p0 = rho0 * c0 ** 2 / gamma
    return dict(points=pts, normals=nrm, areas=area, rho=rho0 + rho_p, u=u, p=p0 + p_p, dt=dt,
                mach=np.asarray(mach, dtype=np.float64), c0=c0, rho0=rho0, p0=p0, kind=kind, omega=omega,
                amplitude=amplitude)


def fwh_airfoil_case(seed=0, spacing=0.01, span=0.2, height=1.0, wake=4.0, n_samples=4332, dt=0.009233,
                     lz=25.0, mach=0.2, aoa_deg=5.0, gamma=GAMMA):
    """The airfoil data surface of the paper's Section 3.1, synthetic samples.

    An open surface around a unit chord at the origin: two horizontal sheets at
    y = +-height/2 from x = -height/2 to 1 + wake (four chords into the wake) joined by a
    vertical sheet at x = -height/2, open downstream; panels of spacing x spacing, the
    spanwise ones half a spacing inside the periodic planes; n_samples snapshots every dt
    (free-stream convective times) and spanwise copies filling lz chords.  The samples are
    the exact field of a stationary lift dipole at the trailing edge in the stream, with a
    seeded frequency near two cycles per convective time (values only set the work, not
    its amount).  Non-dimensional: chord, rho_inf and |U_inf| are 1.
    """
    rng = np.random.default_rng(seed)
    h = height / 2.0
    x0, x1 = -h, 1.0 + wake
    nx = int(round((x1 - x0) / spacing))
    ny = int(round(height / spacing))
    nz = int(round(span / spacing))
    xs = x0 + spacing * (np.arange(nx) + 0.5)
    ys = -h + spacing * (np.arange(ny) + 0.5)
    zs = spacing * (np.arange(nz) + 0.5)
    pts, nrm = [], []
    for z in zs:
        pts += [(x, h, z) for x in xs]
        nrm += [(0.0, 1.0, 0.0)] * nx
        pts += [(x, -h, z) for x in xs]
        nrm += [(0.0, -1.0, 0.0)] * nx
        pts += [(x0, y, z) for y in ys]
        nrm += [(-1.0, 0.0, 0.0)] * ny
    pts = np.asarray(pts, dtype=np.float64)
    nrm = np.asarray(nrm, dtype=np.float64)
    a = np.deg2rad(aoa_deg)
    M = mach * np.array([np.cos(a), np.sin(a), 0.0])
    c0 = 1.0 / mach
    p0 = 1.0 / (gamma * mach ** 2)
    n_copies = int(round(lz / span))
    if n_copies % 2 == 0:
        n_copies += 1
    return dict(points=pts, normals=nrm, areas=np.full(pts.shape[0], spacing * spacing), mach=M, c0=c0, rho0=1.0,
                p0=p0, dt=dt, n_samples=n_samples, n_copies=n_copies, copy_shift=np.array([0.0, 0.0, span]),
                observer=np.array([1.0, -10.0, span / 2.0]), source=np.array([1.0, 0.0, span / 2.0]),
                omega=2.0 * np.pi * rng.uniform(1.8, 2.2), amplitude=1e-3)


def fwh_airfoil_samples(case, chunk=256):
    """Yield (rho, u, p) of consecutive snapshot chunks of fwh_airfoil_case."""
    x = case["points"] - case["source"]
    for k0 in range(0, case["n_samples"], chunk):
        t = case["dt"] * np.arange(k0, min(k0 + chunk, case["n_samples"]))
        rho_p, u, p_p = stationary_source("dipole", x, t, case["mach"], case["c0"], case["rho0"],
                                          amplitude=case["amplitude"], omega=case["omega"])
        yield case["rho0"] + rho_p, u, case["p0"] + p_p

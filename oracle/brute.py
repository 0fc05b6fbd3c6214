"""Test infrastructure only: brute-force FR residual by explicit polynomial algebra.

An independent second formulation of the same FR residual as ``fr_oracle.c``
for tiny meshes of affine quadrilaterals (2D) and parallelepipeds (3D) with
periodic faces.  Nothing is
shared with the C oracle: the basis comes from ``numpy.polynomial``, the
solution, gradient and flux polynomials are built by solving Vandermonde
systems, the corrected fluxes are assembled as bivariate polynomials and
differentiated symbolically, and neighbouring flux points are matched by
their physical coordinates (with periodic wrap).

Method (Huynh's FR, the solver family the paper's Section 1 cites; the
physics of the paper's Eqs. (1)-(7) with F = F_inv - F_vis and
F_vis,j = (0, tau_ij, u_i tau_ij - q_j)):

  u^D       interpolating polynomial of the solution-point values;
  u^C       u^D + (u_c - u^D)|face(eta) g(xi) per axis (g_DG corrections);
  grad u    (1/|J|) S^T grad_xi u^C sampled at solution points;
  F~        S F(u, grad u) at solution points, interpolated;
  F~^C      F~^D + (F~* - F~^D_n) g per axis, F~* = |S^T n| F*_n;
  R         -(div_xi F~^C)/|J| at the solution points.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as leg
from numpy.polynomial import polynomial as P


def gl_nodes(order):
    x, w = leg.leggauss(order + 1)
    return x, w


def radau_right(order):
    """g_R = (P_p + P_{p+1})/2 as power-series coefficients."""
    c = np.zeros(order + 2)
    c[order] = 0.5
    c[order + 1] = 0.5
    return leg.leg2poly(c)


def lagrange_poly_1d(x, j):
    others = np.delete(x, j)
    c = P.polyfromroots(others)
    return c / P.polyval(x[j], c)


class BruteMesh2D:
    """Periodic mesh of affine quads given by corner coordinates.

    corners: array [E, 4, 2] ordered (xi,eta) = (-,-), (+,-), (-,+), (+,+).
    period: (Lx, Ly) of the periodic box.
    """

    def __init__(self, corners, order, period, gamma=1.4, prandtl=0.72, mu=0.0):
        self.c = np.asarray(corners, dtype=np.float64)
        self.order = order
        self.n = order + 1
        self.period = np.asarray(period, dtype=np.float64)
        self.gamma, self.pr, self.mu = gamma, prandtl, mu
        self.x, self.w = gl_nodes(order)
        self.gR = radau_right(order)
        self.gL = self.gR * np.array([(-1.0) ** k for k in range(len(self.gR))])  # g_R(-x)
        self.E = len(self.c)
        # affine map x = x0 + A r, A = [dx/dxi, dx/deta]
        c = self.c
        self.x0 = 0.25 * c.sum(axis=1)
        self.A = np.stack([0.5 * (c[:, 1] - c[:, 0]), 0.5 * (c[:, 2] - c[:, 0])], axis=2)
        # stored as A[e][i][j] = dx_i/dxi_j
        self.det = np.linalg.det(self.A)
        self.S = np.array([np.linalg.inv(self.A[e]) * self.det[e] for e in range(self.E)])
        n = self.n
        self.upts = [(self.x[i0], self.x[i1]) for i1 in range(n) for i0 in range(n)]

    # --- polynomial helpers -------------------------------------------------
    def fit2d(self, vals):
        """Coefficients c[a][b] (xi^a eta^b) of the tensor interpolant of solution-point values."""
        r = np.array(self.upts)
        V = P.polyvander2d(r[:, 0], r[:, 1], [self.order, self.order])
        coef = np.linalg.solve(V, vals)
        return coef.reshape(self.n, self.n)

    def fit1d(self, vals):
        V = P.polyvander(self.x, self.order)
        return np.linalg.solve(V, vals)

    def face_points(self, e, f):
        """Reference and physical coordinates of the flux points of face f."""
        k, s = f // 2, f % 2
        out = []
        for m in range(self.n):
            r = [0.0, 0.0]
            r[k] = 1.0 if s else -1.0
            r[1 - k] = self.x[m]
            xp = self.x0[e] + self.A[e] @ np.array(r)
            out.append((r, xp))
        return out

    def partner(self, e, f, m):
        _, xp = self.face_points(e, f)[m]
        for e2 in range(self.E):
            for f2 in range(4):
                if e2 == e and f2 == f:
                    continue
                for m2, (_, xq) in enumerate(self.face_points(e2, f2)):
                    dlt = xq - xp
                    dlt = dlt - self.period * np.round(dlt / self.period)
                    if np.all(np.abs(dlt) < 1e-9):
                        return e2, f2, m2
        raise ValueError("unmatched flux point")

    # --- physics --------------------------------------------------------------
    def prim(self, u):
        rho = u[0]
        v = u[1:3] / rho
        p = (self.gamma - 1) * (u[3] - 0.5 * rho * (v @ v))
        return rho, v, p

    def finv(self, u):
        rho, v, p = self.prim(u)
        F = np.zeros((2, 4))
        for j in range(2):
            F[j, 0] = u[1 + j]
            F[j, 1:3] = u[1:3] * v[j] + p * np.eye(2)[j]
            F[j, 3] = v[j] * (u[3] + p)
        return F

    def fvis(self, u, g):
        rho, v, p = self.prim(u)
        E = u[3] / rho
        dv = np.zeros((2, 2))
        de = np.zeros(2)
        for j in range(2):
            dv[:, j] = (g[j, 1:3] - v * g[j, 0]) / rho
            de[j] = (g[j, 3] - E * g[j, 0]) / rho - v @ dv[:, j]
        tau = self.mu * (dv + dv.T - 2.0 / 3.0 * np.trace(dv) * np.eye(2))
        F = np.zeros((2, 4))
        kappa = self.mu * self.gamma / self.pr
        for j in range(2):
            F[j, 1:3] = tau[:, j]
            F[j, 3] = v @ tau[:, j] + kappa * de[j]
        return F

    def rusanov(self, uL, uR, nrm):
        fl = nrm @ self.finv(uL)
        fr = nrm @ self.finv(uR)
        lam = max(abs(self.prim(uL)[1] @ nrm) + np.sqrt(self.gamma * self.prim(uL)[2] / uL[0]),
                  abs(self.prim(uR)[1] @ nrm) + np.sqrt(self.gamma * self.prim(uR)[2] / uR[0]))
        return 0.5 * (fl + fr) - 0.5 * lam * (uR - uL)

    # --- residual -----------------------------------------------------------
    def residual(self, u):
        """u: [E, n*n, 4] at solution points (xi fastest). Returns R of the same shape."""
        E, n = self.E, self.n
        nv = 4
        uD = [[self.fit2d(u[e][:, v]) for v in range(nv)] for e in range(E)]

        def normal(e, f):
            k, s = f // 2, f % 2
            vec = (1.0 if s else -1.0) * self.S[e][k, :]
            a = np.linalg.norm(vec)
            return vec / a, a

        def trace(polys, e, f, m):
            r, _ = self.face_points(e, f)[m]
            return np.array([P.polyval2d(r[0], r[1], c) for c in polys])

        # corrected gradient polynomials per element, per variable, per axis
        grads = []
        for e in range(E):
            dU = np.zeros((4, n, nv))  # (face, m, var) u_c - u_f
            for f in range(4):
                for m in range(n):
                    e2, f2, m2 = self.partner(e, f, m)
                    dU[f, m] = 0.5 * (trace(uD[e2], e2, f2, m2) - trace(uD[e], e, f, m))
            gpts = np.zeros((n * n, 2, nv))  # physical gradient at solution points
            for v in range(nv):
                dxi = P.polyder(uD[e][v], axis=0)
                deta = P.polyder(uD[e][v], axis=1)
                # corrections: face eta-profile polynomials times g'(xi) (or g'(eta))
                cm0 = self.fit1d(dU[0, :, v])
                cp0 = self.fit1d(dU[1, :, v])
                cm1 = self.fit1d(dU[2, :, v])
                cp1 = self.fit1d(dU[3, :, v])
                gRd, gLd = P.polyder(self.gR), P.polyder(self.gL)
                for idx, (r0, r1) in enumerate(self.upts):
                    G0 = (P.polyval2d(r0, r1, dxi) + P.polyval(r1, cp0) * P.polyval(r0, gRd)
                          + P.polyval(r1, cm0) * P.polyval(r0, gLd))
                    G1 = (P.polyval2d(r0, r1, deta) + P.polyval(r0, cp1) * P.polyval(r1, gRd)
                          + P.polyval(r0, cm1) * P.polyval(r1, gLd))
                    gpts[idx, :, v] = self.S[e].T @ np.array([G0, G1]) / self.det[e]
            grads.append(gpts)
        # interpolants of the physical gradient
        gpoly = [[[self.fit2d(grads[e][:, j, v]) for v in range(nv)] for j in range(2)] for e in range(E)]

        def grad_trace(e, f, m):
            r, _ = self.face_points(e, f)[m]
            return np.array([[P.polyval2d(r[0], r[1], gpoly[e][j][v]) for v in range(nv)] for j in range(2)])

        R = np.zeros_like(u)
        for e in range(E):
            Ft = np.zeros((n * n, 2, nv))
            for idx in range(n * n):
                F = self.finv(u[e][idx]) - self.fvis(u[e][idx], grads[e][idx])
                Ft[idx] = self.S[e] @ F
            Fpoly = [[self.fit2d(Ft[:, k, v]) for v in range(nv)] for k in range(2)]
            dlt = np.zeros((4, n, nv))
            for f in range(4):
                k, s = f // 2, f % 2
                nrm, a = normal(e, f)
                for m in range(n):
                    e2, f2, m2 = self.partner(e, f, m)
                    uL, uR = trace(uD[e], e, f, m), trace(uD[e2], e2, f2, m2)
                    gL, gR = grad_trace(e, f, m), grad_trace(e2, f2, m2)
                    Fn = self.rusanov(uL, uR, nrm) - 0.5 * nrm @ (self.fvis(uL, gL) + self.fvis(uR, gR))
                    r, _ = self.face_points(e, f)[m]
                    fd = np.array([P.polyval2d(r[0], r[1], Fpoly[k][v]) for v in range(nv)])
                    dlt[f, m] = a * Fn - (1.0 if s else -1.0) * fd
            for v in range(nv):
                div0 = P.polyder(Fpoly[0][v], axis=0)
                div1 = P.polyder(Fpoly[1][v], axis=1)
                cp0, cm0 = self.fit1d(dlt[1, :, v]), self.fit1d(dlt[0, :, v])
                cp1, cm1 = self.fit1d(dlt[3, :, v]), self.fit1d(dlt[2, :, v])
                gRd, gLd = P.polyder(self.gR), P.polyder(self.gL)
                for idx, (r0, r1) in enumerate(self.upts):
                    d0 = (P.polyval2d(r0, r1, div0) + P.polyval(r1, cp0) * P.polyval(r0, gRd)
                          - P.polyval(r1, cm0) * P.polyval(r0, gLd))
                    d1 = (P.polyval2d(r0, r1, div1) + P.polyval(r0, cp1) * P.polyval(r1, gRd)
                          - P.polyval(r0, cm1) * P.polyval(r1, gLd))
                    R[e][idx, v] = -(d0 + d1) / self.det[e]
        return R

    def solution_points(self):
        out = np.zeros((self.E, self.n * self.n, 2))
        for e in range(self.E):
            for idx, (r0, r1) in enumerate(self.upts):
                out[e, idx] = self.x0[e] + self.A[e] @ np.array([r0, r1])
        return out


class BruteMesh3D:
    """Periodic mesh of affine hexahedra (parallelepipeds) given by corner coordinates.

    The 3D counterpart of ``BruteMesh2D``, built the same way: tensor
    interpolants as trivariate power series (``numpy.polynomial``), face data
    as bivariate polynomials over the face's two axes, corrections multiplied
    by g'(xi_k) along the face axis, and neighbours found by physical position.

    corners: array [E, 8, 3], corner a0 + 2 a1 + 4 a2 at reference (-1)^(1+a_k).
    lattice: [3, 3], rows are the periodic translations of the box.
    """

    def __init__(self, corners, order, lattice, gamma=1.4, prandtl=0.72, mu=0.0):
        self.c = np.asarray(corners, dtype=np.float64)
        self.order = order
        self.n = order + 1
        self.lattice = np.asarray(lattice, dtype=np.float64)
        self.gamma, self.pr, self.mu = gamma, prandtl, mu
        self.x, self.w = gl_nodes(order)
        self.gR = radau_right(order)
        self.gL = self.gR * np.array([(-1.0) ** k for k in range(len(self.gR))])
        self.gRd, self.gLd = P.polyder(self.gR), P.polyder(self.gL)
        self.E = len(self.c)
        c = self.c
        self.x0 = c.mean(axis=1)
        # A[e][i][k] = dx_i / dxi_k (edges from corner 0 along each reference axis)
        self.A = np.stack([0.5 * (c[:, 1] - c[:, 0]), 0.5 * (c[:, 2] - c[:, 0]), 0.5 * (c[:, 4] - c[:, 0])],
                          axis=2)
        self.det = np.linalg.det(self.A)
        self.S = np.array([np.linalg.inv(self.A[e]) * self.det[e] for e in range(self.E)])
        n = self.n
        self.upts = [(self.x[i0], self.x[i1], self.x[i2]) for i2 in range(n) for i1 in range(n) for i0 in range(n)]
        self.fpts = [[self._face_points(e, f) for f in range(6)] for e in range(self.E)]
        self.nbr = {}
        for e in range(self.E):
            for f in range(6):
                for m in range(n * n):
                    self.nbr[(e, f, m)] = self._partner(e, f, m)

    # --- geometry -------------------------------------------------------------
    def _face_axes(self, k):
        return [a for a in range(3) if a != k]

    def _face_points(self, e, f):
        k, s = f // 2, f % 2
        ax = self._face_axes(k)
        out = []
        for m in range(self.n * self.n):
            r = [0.0, 0.0, 0.0]
            r[k] = 1.0 if s else -1.0
            r[ax[0]] = self.x[m % self.n]
            r[ax[1]] = self.x[m // self.n]
            out.append((np.array(r), self.x0[e] + self.A[e] @ np.array(r)))
        return out

    def _partner(self, e, f, m):
        xp = self.fpts[e][f][m][1]
        for e2 in range(self.E):
            for f2 in range(6):
                if e2 == e and f2 == f:
                    continue
                for m2, (_, xq) in enumerate(self.fpts[e2][f2]):
                    dlt = xq - xp
                    k = np.linalg.solve(self.lattice.T, dlt)
                    dlt = dlt - self.lattice.T @ np.round(k)
                    if np.all(np.abs(dlt) < 1e-9):
                        return e2, f2, m2
        raise ValueError("unmatched flux point")

    def normal(self, e, f):
        k, s = f // 2, f % 2
        vec = (1.0 if s else -1.0) * self.S[e][k, :]
        a = np.linalg.norm(vec)
        return vec / a, a

    # --- polynomials ----------------------------------------------------------
    def fit3d(self, vals):
        r = np.array(self.upts)
        V = P.polyvander3d(r[:, 0], r[:, 1], r[:, 2], [self.order] * 3)
        return np.linalg.solve(V, vals).reshape(self.n, self.n, self.n)

    def fit_face(self, vals):
        """Bivariate interpolant over a face's two axes of face-point values (m = m0 + n m1)."""
        t0 = np.array([self.x[m % self.n] for m in range(self.n * self.n)])
        t1 = np.array([self.x[m // self.n] for m in range(self.n * self.n)])
        V = P.polyvander2d(t0, t1, [self.order] * 2)
        return np.linalg.solve(V, vals).reshape(self.n, self.n)

    # --- physics (Eqs. (1)-(7)) ------------------------------------------------
    def prim(self, u):
        rho = u[0]
        v = u[1:4] / rho
        p = (self.gamma - 1) * (u[4] - 0.5 * rho * (v @ v))
        return rho, v, p

    def finv(self, u):
        rho, v, p = self.prim(u)
        F = np.zeros((3, 5))
        for j in range(3):
            F[j, 0] = u[1 + j]
            F[j, 1:4] = u[1:4] * v[j] + p * np.eye(3)[j]
            F[j, 4] = v[j] * (u[4] + p)
        return F

    def fvis(self, u, g):
        rho, v, p = self.prim(u)
        E = u[4] / rho
        dv = np.zeros((3, 3))
        de = np.zeros(3)
        for j in range(3):
            dv[:, j] = (g[j, 1:4] - v * g[j, 0]) / rho
            de[j] = (g[j, 4] - E * g[j, 0]) / rho - v @ dv[:, j]
        tau = self.mu * (dv + dv.T - 2.0 / 3.0 * np.trace(dv) * np.eye(3))
        kappa = self.mu * self.gamma / self.pr
        F = np.zeros((3, 5))
        for j in range(3):
            F[j, 1:4] = tau[:, j]
            F[j, 4] = v @ tau[:, j] + kappa * de[j]
        return F

    def rusanov(self, uL, uR, nrm):
        _, vL, pL = self.prim(uL)
        _, vR, pR = self.prim(uR)
        lam = max(abs(vL @ nrm) + np.sqrt(self.gamma * pL / uL[0]), abs(vR @ nrm) + np.sqrt(self.gamma * pR / uR[0]))
        return 0.5 * (nrm @ self.finv(uL) + nrm @ self.finv(uR)) - 0.5 * lam * (uR - uL)

    # --- residual -------------------------------------------------------------
    def _face_poly_at(self, coef, r, k):
        ax = self._face_axes(k)
        return P.polyval2d(r[ax[0]], r[ax[1]], coef)

    def residual(self, u):
        """u: [E, n^3, 5] at solution points (xi fastest). Returns R of the same shape."""
        E, n, nv = self.E, self.n, 5
        nfp = n * n
        uD = [[self.fit3d(u[e][:, v]) for v in range(nv)] for e in range(E)]

        def trace(polys, e, f, m):
            r = self.fpts[e][f][m][0]
            return np.array([P.polyval3d(r[0], r[1], r[2], c) for c in polys])

        grads = []
        for e in range(E):
            dU = np.zeros((6, nfp, nv))
            for f in range(6):
                for m in range(nfp):
                    e2, f2, m2 = self.nbr[(e, f, m)]
                    dU[f, m] = 0.5 * (trace(uD[e2], e2, f2, m2) - trace(uD[e], e, f, m))
            gpts = np.zeros((n ** 3, 3, nv))
            for v in range(nv):
                der = [P.polyder(uD[e][v], axis=k) for k in range(3)]
                cm = [self.fit_face(dU[2 * k, :, v]) for k in range(3)]
                cp = [self.fit_face(dU[2 * k + 1, :, v]) for k in range(3)]
                for idx, r in enumerate(self.upts):
                    Gk = np.array([P.polyval3d(r[0], r[1], r[2], der[k])
                                   + self._face_poly_at(cp[k], r, k) * P.polyval(r[k], self.gRd)
                                   + self._face_poly_at(cm[k], r, k) * P.polyval(r[k], self.gLd)
                                   for k in range(3)])
                    gpts[idx, :, v] = self.S[e].T @ Gk / self.det[e]
            grads.append(gpts)
        gpoly = [[[self.fit3d(grads[e][:, j, v]) for v in range(nv)] for j in range(3)] for e in range(E)]

        def grad_trace(e, f, m):
            r = self.fpts[e][f][m][0]
            return np.array([[P.polyval3d(r[0], r[1], r[2], gpoly[e][j][v]) for v in range(nv)] for j in range(3)])

        R = np.zeros_like(u)
        for e in range(E):
            Ft = np.zeros((n ** 3, 3, nv))
            for idx in range(n ** 3):
                Ft[idx] = self.S[e] @ (self.finv(u[e][idx]) - self.fvis(u[e][idx], grads[e][idx]))
            Fpoly = [[self.fit3d(Ft[:, k, v]) for v in range(nv)] for k in range(3)]
            dlt = np.zeros((6, nfp, nv))
            for f in range(6):
                k, s = f // 2, f % 2
                nrm, a = self.normal(e, f)
                for m in range(nfp):
                    e2, f2, m2 = self.nbr[(e, f, m)]
                    uL, uR = trace(uD[e], e, f, m), trace(uD[e2], e2, f2, m2)
                    gL, gR = grad_trace(e, f, m), grad_trace(e2, f2, m2)
                    Fn = self.rusanov(uL, uR, nrm) - 0.5 * nrm @ (self.fvis(uL, gL) + self.fvis(uR, gR))
                    r = self.fpts[e][f][m][0]
                    fd = np.array([P.polyval3d(r[0], r[1], r[2], Fpoly[k][v]) for v in range(nv)])
                    dlt[f, m] = a * Fn - (1.0 if s else -1.0) * fd
            for v in range(nv):
                der = [P.polyder(Fpoly[k][v], axis=k) for k in range(3)]
                cm = [self.fit_face(dlt[2 * k, :, v]) for k in range(3)]
                cp = [self.fit_face(dlt[2 * k + 1, :, v]) for k in range(3)]
                for idx, r in enumerate(self.upts):
                    div = sum(P.polyval3d(r[0], r[1], r[2], der[k])
                              + self._face_poly_at(cp[k], r, k) * P.polyval(r[k], self.gRd)
                              - self._face_poly_at(cm[k], r, k) * P.polyval(r[k], self.gLd)
                              for k in range(3))
                    R[e][idx, v] = -div / self.det[e]
        return R

    def solution_points(self):
        out = np.zeros((self.E, self.n ** 3, 3))
        for e in range(self.E):
            for idx, r in enumerate(self.upts):
                out[e, idx] = self.x0[e] + self.A[e] @ np.array(r)
        return out

"""Test infrastructure only: brute-force FR residual by explicit polynomial algebra.

An independent second formulation of the same FR residual as ``fr_oracle.c``
for tiny 2D meshes of affine quadrilaterals with periodic faces.  Nothing is
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

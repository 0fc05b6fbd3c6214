"""Test infrastructure only: plain FP64 numpy oracle of the far-field acoustic step.

Only tests, ``__graft_entry__.smoke`` and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the HIP path.

What it computes (the paper's Appendices A and B): the acoustic pressure at an
observer from flow samples on a stationary permeable data surface in a medium moving
at the free-stream velocity.  It uses the moving-medium time-domain solution with the
quadrupole term dropped, evaluated by the advanced-time approach:

  * source terms on the surface (Appendix A, with a stationary surface, v = 0):
      Q   = rho (u_n + U_n) - rho_0 U_n
      L_i = (p - p_0) n_i + rho u_i (u_n + U_n)
    where u is the flow velocity relative to the free stream (the disturbance
    velocity) and U the free-stream velocity; the viscous stress is not part of the
    sampled data and is left out;
  * per panel, amplitude and phase radii R*, R and their gradients (Appendix B);
  * thickness and loading integrands (Appendix B, Eqs. for p'_T and p'_L):
      4 pi p'_T: (1 - M_R) Qdot / R*  -  Q c0 M_R* / R*^2
      4 pi p'_L: Ldot_R / (c0 R*)  +  L_R* / R*^2
  * advanced time: each panel's samples reach the observer at t = tau + R / c0;
    the panel series are interpolated onto one observer-time grid that every panel
    covers, and summed with the panel areas.

Readings where the paper is silent, shared with the HIP path by specification only:
  * source-time derivatives: fourth-order central differences; the two samples at
    each end of the record have none and are not used;
  * interpolation: four-point Lagrange (cubic) in source time;
  * observer-time grid: spacing equal to the sampling interval, from the latest first
    arrival plus one interval to the earliest last arrival less two intervals, so that
    every cubic stencil lies inside every panel's record;
  * spanwise duplication: copies of the surface shifted by k * shift for
    k = -(n_copies - 1) / 2 .. (n_copies - 1) / 2, all carrying the same samples.
"""
from __future__ import annotations

import numpy as np


def source_terms(rho, u, p, normals, U, rho0, p0):
    """Q [..., n] and L [..., n, 3] from samples rho [..., n], u [..., n, 3], p [..., n]."""
    un = np.einsum("...ni,ni->...n", u, normals)
    Un = normals @ U
    Q = rho * (un + Un) - rho0 * Un
    L = (p - p0)[..., None] * normals + (rho * (un + Un))[..., None] * u
    return Q, L


def time_derivative(f, dt):
    """Fourth-order central difference along axis 0; entries 0, 1, -2, -1 are left NaN."""
    d = np.full_like(f, np.nan)
    d[2:-2] = (f[:-4] - 8.0 * f[1:-3] + 8.0 * f[3:-1] - f[4:]) / (12.0 * dt)
    return d


def radii(x, y, M):
    """R*, R, grad R* and grad R (w.r.t. the observer position) for r = x - y."""
    r = x - y
    M = np.asarray(M, dtype=np.float64)
    g2 = 1.0 / (1.0 - M @ M)
    Mr = r @ M
    Rs = np.sqrt(np.einsum("...i,...i->...", r, r) + g2 * Mr ** 2) / np.sqrt(g2)
    R = g2 * (Rs - Mr)
    gRs = (r + g2 * Mr[..., None] * M) / (g2 * Rs[..., None])
    gR = g2 * (gRs - M)
    return Rs, R, gRs, gR


def lagrange4(s):
    """Weights of the cubic through nodes -1, 0, 1, 2 at fractional position s in [0, 1)."""
    return np.stack([-s * (s - 1.0) * (s - 2.0) / 6.0,
                     (s + 1.0) * (s - 1.0) * (s - 2.0) / 2.0,
                     -(s + 1.0) * s * (s - 2.0) / 2.0,
                     (s + 1.0) * s * (s - 1.0) / 6.0])


def copy_shifts(n_copies, shift):
    k = np.arange(n_copies) - (n_copies - 1) / 2.0
    return k[:, None] * np.asarray(shift, dtype=np.float64)[None, :]


def observer_pressure(points, normals, areas, rho, u, p, dt, x_obs, M, c0, rho0, p0, n_copies=1,
                      shift=(0.0, 0.0, 0.0), tau0=0.0, t_grid=None):
    """Acoustic pressure p'(t) at observer x_obs.

    points, normals [n, 3], areas [n]: one copy of the data surface.
    rho [nt, n], u [nt, n, 3], p [nt, n]: samples at source times tau0 + k dt.
    t_grid: optional observer times inside the common window (default: the window's
    grid described in the module docstring).
    Returns (t [m], p' [m], p'_T [m], p'_L [m]).
    """
    points = np.asarray(points, dtype=np.float64)
    nt = rho.shape[0]
    M = np.asarray(M, dtype=np.float64)
    U = c0 * M
    Q, L = source_terms(rho, u, p, normals, U, rho0, p0)
    Qd = time_derivative(Q, dt)
    Ld = time_derivative(L, dt)
    ys = (points[None, :, :] + copy_shifts(n_copies, shift)[:, None, :]).reshape(-1, 3)
    nrep = n_copies
    Rs, R, gRs, gR = radii(np.asarray(x_obs, dtype=np.float64)[None, :], ys, M)
    # integrands at the valid samples k = 2 .. nt-3, per panel (copies repeat the samples)
    k = np.arange(2, nt - 2)
    nv = k.size
    MR = gR @ M
    MRs = gRs @ M
    Qk, Qdk = np.tile(Q[k], (1, nrep)), np.tile(Qd[k], (1, nrep))
    Lk, Ldk = np.tile(L[k], (1, nrep, 1)), np.tile(Ld[k], (1, nrep, 1))
    IT = (1.0 - MR) * Qdk / Rs - Qk * c0 * MRs / Rs ** 2
    IL = np.einsum("kni,ni->kn", Ldk, gR) / (c0 * Rs) + np.einsum("kni,ni->kn", Lk, gRs) / Rs ** 2
    # advanced time: panel j's sample k arrives at tau0 + k dt + R_j / c0
    delay = R / c0
    t_first = tau0 + 2 * dt + delay            # first valid arrival per panel
    t_last = tau0 + (nt - 3) * dt + delay       # last valid arrival per panel
    t_start = t_first.max() + dt
    t_end = t_last.min() - 2.0 * dt
    if t_grid is None:
        m = int(np.floor((t_end - t_start) / dt + 1e-9)) + 1
        if m <= 0:
            raise ValueError("record too short for the spread of arrival times")
        t = t_start + dt * np.arange(m)
    else:
        t = np.asarray(t_grid, dtype=np.float64)
        if t.min() < t_start - 1e-9 * dt or t.max() > t_end + 1e-9 * dt:
            raise ValueError("observer times outside the common window")
        m = t.size
    pT = np.zeros(m)
    pL = np.zeros(m)
    w_area = np.tile(areas, nrep)
    for j in range(ys.shape[0]):
        pos = (t - tau0 - delay[j]) / dt - 2.0     # position in the valid series (index 0 = k 2)
        # stencil i0-1 .. i0+2 inside the nv valid samples; the clamp only absorbs
        # rounding of pos at the grid ends (s then strays from [0, 1) by rounding)
        i0 = np.clip(np.floor(pos).astype(np.int64), 1, nv - 3)
        s = pos - i0
        w = lagrange4(s)
        for a in range(4):
            idx = i0 - 1 + a
            pT += w_area[j] * w[a] * IT[idx, j]
            pL += w_area[j] * w[a] * IL[idx, j]
    pT /= 4.0 * np.pi
    pL /= 4.0 * np.pi
    return t, pT + pL, pT, pL


def oaspl(p, p_ref):
    """Overall sound pressure level of the fluctuation of p about its mean, in dB re p_ref."""
    q = np.asarray(p) - np.mean(p)
    return 10.0 * np.log10(np.mean(q * q) / p_ref ** 2)

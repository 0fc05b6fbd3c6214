"""OrthoMADS: the derivative-free optimiser of the paper's Algorithm 1 and Appendix E.

Each iteration polls the 2n points of a maximal positive basis around the incumbent
and evaluates them together (the concurrent candidate designs of Algorithm 1: the
caller's ``evaluate`` receives the whole poll set, so a request pool can run them side
by side).  Poll directions are the deterministic orthogonal ones of OrthoMADS:

  * u_t, the t-th point of the Halton sequence in the first n primes;
  * the adjusted direction q = round(a (2 u_t - 1) / |2 u_t - 1|), with the largest a
    such that |q| <= 2^(l/2) for mesh index l (mesh size 4^-l);
  * the Householder matrix H = |q|^2 I - 2 q q^T, whose columns are orthogonal, of
    equal length |q|^2, and integer; the poll directions are the columns of [H, -H].

Poll points x + dm d therefore lie on the mesh of size dm = 4^-l at distance about
sqrt(dm) (the poll size of the maximal basis, Appendix E).

Mesh update (Algorithm 1): after a poll that improves the incumbent the mesh size is
multiplied by 4, capped at its initial value; otherwise it is divided by 4.  The run
stops when the mesh size falls below `mesh_tol` and the design moved by less than
`move_tol` (relative) between consecutive iterations.  Design variables are scaled to
[0, 1]; poll points outside are infeasible and are not evaluated (objective +inf, the
extreme barrier of Appendix E: infeasible trial points are discarded).

Readings where the paper is silent: the Halton index of iteration k is t = p_n + k
(p_n the n-th prime), so every iteration polls new directions; the relative design
change is taken in the scaled coordinates, per component, over max(|x|, 1e-12); on
equal objective values the first poll point in [H, -H] column order wins.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PRIMES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53)


def halton(t, n):
    """t-th Halton point in [0, 1)^n (radical inverse of t in the first n primes)."""
    out = np.zeros(n)
    for i in range(n):
        b = PRIMES[i]
        f, r, k = 1.0, 0.0, t
        while k > 0:
            f /= b
            r += f * (k % b)
            k //= b
        out[i] = r
    return out


def adjusted_direction(u, l):
    """Integer q = round(a v), v = (2u - 1)/|2u - 1|, with the largest a: |q| <= 2^(l/2)."""
    v = 2.0 * np.asarray(u) - 1.0
    v = v / np.linalg.norm(v)
    bound = 2.0 ** (abs(l) / 2.0)
    lo, hi = 0.0, bound * math.sqrt(len(v)) + 1.0
    # |round(a v)| is nondecreasing in a: bisect on its jumps
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.linalg.norm(np.rint(mid * v)) <= bound + 1e-12:
            lo = mid
        else:
            hi = mid
    q = np.rint(lo * v)
    if not np.any(q):
        q = np.zeros_like(v)
        q[int(np.argmax(np.abs(v)))] = np.sign(v[int(np.argmax(np.abs(v)))])
    return q.astype(np.int64)


def householder(q):
    q = np.asarray(q, dtype=np.int64)
    return int(q @ q) * np.eye(len(q), dtype=np.int64) - 2 * np.outer(q, q)


def poll_directions(t, l, n):
    """The 2n OrthoMADS poll directions [H, -H] (columns) for Halton index t, mesh index l."""
    H = householder(adjusted_direction(halton(t, n), l))
    return np.concatenate([H, -H], axis=1)


@dataclass
class Result:
    x: np.ndarray                  # best design, scaled coordinates
    f: float
    iterations: int
    evaluations: int
    history: list = field(default_factory=list)   # (iteration, mesh size, incumbent f, x)


def orthomads(evaluate, x0, l0=2, mesh_tol=1e-6, move_tol=0.01, max_iter=100, f0=None):
    """Minimise over [0, 1]^n.  evaluate(list of points) -> list of objective values.

    l0: initial mesh index (initial mesh size 4^-l0, also the cap of the mesh size).
    """
    x = np.asarray(x0, dtype=np.float64).copy()
    n = x.size
    f = evaluate([x.copy()])[0] if f0 is None else float(f0)
    cache = {tuple(np.round(x, 15)): f}
    nevals = 1 if f0 is None else 0
    l = l0
    hist = [(0, 4.0 ** -l, f, x.copy())]
    x_prev = x.copy()
    for k in range(max_iter):
        l = max(l, l0)                       # mesh size capped at its initial value
        dm = 4.0 ** -l
        D = poll_directions(PRIMES[n - 1] + k, l, n)
        pts = [x + dm * D[:, j] for j in range(2 * n)]
        vals = [math.inf] * len(pts)
        todo = []
        for j, p in enumerate(pts):
            if np.any(p < -1e-12) or np.any(p > 1.0 + 1e-12):
                continue                     # infeasible: not evaluated
            key = tuple(np.round(p, 15))
            if key in cache:
                vals[j] = cache[key]
            else:
                todo.append(j)
        if todo:
            got = evaluate([pts[j].copy() for j in todo])
            nevals += len(todo)
            for j, v in zip(todo, got):
                vals[j] = float(v)
                cache[tuple(np.round(pts[j], 15))] = vals[j]
        jbest = int(np.argmin(vals))
        x_prev = x.copy()
        if vals[jbest] < f:
            x, f = pts[jbest].copy(), vals[jbest]
            l -= 1
        else:
            l += 1
        hist.append((k + 1, 4.0 ** -l, f, x.copy()))
        move = np.max(np.abs(x - x_prev) / np.maximum(np.abs(x_prev), 1e-12))
        if 4.0 ** -l < mesh_tol and move < move_tol:
            return Result(x, f, k + 1, nevals, hist)
    return Result(x, f, max_iter, nevals, hist)


# ---------------------------------------------------------------------------
# the paper's design problem (Section 3.4)
# ---------------------------------------------------------------------------
# design vector: maximum camber (% chord), its position (tenths of chord), maximum
# thickness (% chord), angle of attack (degrees)
BOUNDS = np.array([[-10.0, 10.0], [4.0, 9.0], [6.0, 18.0], [0.0, 12.0]])
EPS_LIFT, EPS_DRAG = 8000.0, 400000.0


def unscale(xs):
    return BOUNDS[:, 0] + np.asarray(xs) * (BOUNDS[:, 1] - BOUNDS[:, 0])


def scale(x):
    return (np.asarray(x) - BOUNDS[:, 0]) / (BOUNDS[:, 1] - BOUNDS[:, 0])


def objective(oaspl, cl, cd, cl_base, cd_base):
    """Section 3.4: OASPL plus a quadratic penalty on the change of mean lift and, when
    the mean drag exceeds the baseline's, on the change of mean drag."""
    f = oaspl + EPS_LIFT * (cl - cl_base) ** 2
    if cd > cd_base:
        f += EPS_DRAG * (cd - cd_base) ** 2
    return f

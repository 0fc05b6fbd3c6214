"""OrthoMADS (paper_2501_05709_amd/mads.py) against the published algorithm's properties.

* Halton points in bases 2 and 3 (closed form radical inverses).
* Householder matrix of an integer direction: integer, orthogonal columns of equal length
  |q|^2, so [H, -H] is a maximal positive basis (2n directions spanning R^n positively).
* Adjusted direction: |q| <= 2^(l/2) and no larger scaling fits.
* Poll size of the maximal basis: poll points sit within sqrt(mesh size) of the incumbent.
* Mesh updates of Algorithm 1: x4 after an improving poll, capped at the initial size;
  /4 otherwise; infeasible poll points are never evaluated (extreme barrier).
* On a smooth convex function over [0, 1]^4 it converges to the minimiser and stops by
  Algorithm 1's test.
* The Section 3.4 objective: its two branches.
"""
import numpy as np

from paper_2501_05709_amd import mads


def test_halton_closed_form():
    assert np.allclose([mads.halton(t, 2)[0] for t in (1, 2, 3, 4, 5)], [0.5, 0.25, 0.75, 0.125, 0.625])
    assert np.allclose([mads.halton(t, 2)[1] for t in (1, 2, 3, 4)], [1 / 3, 2 / 3, 1 / 9, 4 / 9])


def test_householder_is_an_orthogonal_positive_basis():
    for t in range(5, 40):
        for l in (0, 1, 2, 4, 7):
            q = mads.adjusted_direction(mads.halton(t, 4), l)
            H = mads.householder(q)
            n2 = int(q @ q)
            assert H.dtype.kind == "i"
            assert np.array_equal(H.T @ H, n2 * n2 * np.eye(4, dtype=np.int64))
            assert np.linalg.matrix_rank(H) == 4
            D = mads.poll_directions(t, l, 4)
            assert D.shape == (4, 8) and np.array_equal(D[:, 4:], -D[:, :4])


def test_adjusted_direction_is_the_largest_that_fits():
    for t in range(5, 30):
        u = mads.halton(t, 4)
        v = (2 * u - 1) / np.linalg.norm(2 * u - 1)
        for l in (2, 4, 6, 10):
            q = mads.adjusted_direction(u, l)
            bound = 2.0 ** (l / 2)
            assert np.linalg.norm(q) <= bound + 1e-12
            # rounding moves each component by at most 1/2, so the largest fitting scaling
            # leaves |q| within sqrt(n)/2 + 1 of the bound
            assert np.linalg.norm(q) >= bound - np.sqrt(4) / 2 - 1.0 - 1e-12
            # and q is the rounding of a positive multiple of v: the intervals of a that
            # round each component to q_i intersect
            a_lo = max(min((qi - 0.5) / vi, (qi + 0.5) / vi) for qi, vi in zip(q, v))
            a_hi = min(max((qi - 0.5) / vi, (qi + 0.5) / vi) for qi, vi in zip(q, v))
            assert a_hi > 0 and a_lo <= a_hi + 1e-12


def test_poll_points_within_poll_size():
    for l in range(0, 8):
        dm = 4.0 ** -l
        D = mads.poll_directions(11, l, 4)
        step = dm * np.linalg.norm(D, axis=0)
        assert np.all(step <= np.sqrt(dm) + 1e-12)


def test_mesh_updates_and_extreme_barrier():
    calls = []

    def never_better(pts):
        calls.extend(pts)
        for p in pts:
            assert np.all(p >= -1e-12) and np.all(p <= 1 + 1e-12)
        return [1.0] * len(pts)

    r = mads.orthomads(never_better, np.full(4, 0.02), l0=1, max_iter=5, f0=0.5)
    assert [round(-np.log(h[1]) / np.log(4)) for h in r.history] == [1, 2, 3, 4, 5, 6]

    # any objective: after an improving poll the size is x4 (capped at the initial size),
    # after a failed one /4
    rng = np.random.default_rng(0)
    r = mads.orthomads(lambda pts: list(rng.normal(size=len(pts))), np.full(4, 0.5), l0=2, max_iter=30, f0=0.0)
    cap = 4.0 ** -2
    for (k0, dm0, f0, _), (k1, dm1, f1, _) in zip(r.history[:-1], r.history[1:]):
        used = min(dm0, cap)
        assert np.isclose(dm1, min(4 * used, 4 * cap) if f1 < f0 else used / 4)


def test_converges_on_convex_function():
    target = np.array([0.3, 0.7, 0.55, 0.2])
    seen = []

    def f(pts):
        seen.append(len(pts))
        return [float(np.sum((p - target) ** 2) + 0.1 * np.sum((p - target) ** 4)) for p in pts]

    r = mads.orthomads(f, np.full(4, 0.5), l0=1, max_iter=300)
    assert np.abs(r.x - target).max() < 1e-3
    assert r.iterations < 300 and max(seen[1:]) <= 8


def test_objective_branches():
    assert mads.objective(60.0, 0.5, 0.04, 0.5, 0.05) == 60.0
    assert np.isclose(mads.objective(60.0, 0.6, 0.06, 0.5, 0.05), 60.0 + 8000 * 0.01 + 400000 * 1e-4)
    x = np.array([2.0, 4.5, 12.0, 6.0])
    assert np.allclose(mads.unscale(mads.scale(x)), x)

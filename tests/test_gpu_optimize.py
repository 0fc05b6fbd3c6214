"""GPU tests of the optimisation loop's evaluation path (Algorithm 1, Section 3.4):
served requests that sample a data surface and feed an FW-H record on the device.

Bars: an FP64 sampled request against the oracles run step by step (RK4, point
sampling, FW-H) to 1e-10 of the largest acoustic pressure and of the mean force
coefficients (the pipeline's bar: the state agrees to about 1e-12 and the acoustic sum
adds cancellation); an FP32 sampled request bit-identical to the same pipeline driven
by hand (FRMesh, Probe, FWH); designs run concurrently in the pool bit-identical to each
run alone and to a pool that fits one request at a time; the OrthoMADS loop over pool
evaluations follows Algorithm 1's mesh-size rule and reproduces its objective values.
"""
import math

import numpy as np
import pytest

from oracle import fwh, probe
from oracle.oracle import OracleMesh
from paper_2501_05709_amd import mads
from paper_2501_05709_amd import optimize as O
from paper_2501_05709_amd import workloads as W
from paper_2501_05709_amd.solver import FRMesh, FRPool, FWH, Probe

pytestmark = pytest.mark.gpu

X = [2.0, 5.0, 12.0, 4.0]     # NACA 2512 at 4 degrees


def tiny(**kw):
    args = dict(ni=16, nj=6, nk=1, order=3, radius=8.0, spacing=0.25, height=0.6, wake=0.5, lz=1.0,
                warmup=20, every=4, n_samples=160, chunk=7, budget_bytes=8 << 30)
    args.update(kw)
    return O.Study(**args)


def medium(st, x):
    fs = st.mesh(x)["freestream"]
    gam = 1.4
    c0 = math.sqrt(gam * fs[4] / fs[0])
    return fs, c0, np.array([fs[1] / c0, fs[2] / c0, fs[3] / c0])


def uniform(mesh, shape):
    fs = mesh["freestream"]
    return W.uniform_state(shape[0] * shape[1], fs[0], fs[1:4], fs[4]).reshape(shape)


def run_pool(st, x, u0, precision, pool=None):
    own = pool is None
    pool = FRPool(st.budget_bytes) if own else pool
    mesh, surf = st.mesh(x), st.surface(x)
    slot = pool.admit_sampled(mesh, surf, st.warmup, st.every, st.n_samples, precision=precision, u0=u0)
    assert slot is not None
    done = []
    while not done:
        done = pool.tick(st.chunk)
    assert done == [slot]
    t0, p = pool.pressure(slot, st.observer(), st.n_samples)
    f = pool.result(slot)
    if own:
        pool.close()
    return t0, p, f


def test_sampled_request_matches_oracle():
    st = tiny(precision="fp64")
    mesh, surf = st.mesh(X), st.surface(X)
    o = OracleMesh(mesh)
    u0 = uniform(mesh, o.shape)
    print(f"sampled request fp64: {o.E} elements, {surf['points'].shape[0]} panels x {surf['n_copies']} copies, "
          f"{st.warmup + (st.n_samples - 1) * st.every} steps", flush=True)
    t0, p, f = run_pool(st, X, u0, "fp64")
    # oracle: warm-up, then samples every `every` steps with the wall force of each step
    dt = mesh["dt"]
    e, xi = probe.locate(mesh, surf["points"])
    u = o.rk4(u0, dt, st.warmup)
    snaps, forces = [probe.sample(u, 3, e, xi, 3)], []
    for _ in range(st.n_samples - 1):
        u, hist = o.rk4(u, dt, st.every, forces=True)
        forces.append(hist)
        snaps.append(probe.sample(u, 3, e, xi, 3))
    c = np.array(snaps)
    fs, c0, M = medium(st, X)
    rho = c[..., 0]
    vel = c[..., 1:4] / rho[..., None]
    pres = 0.4 * (c[..., 4] - 0.5 * rho * (vel ** 2).sum(-1))
    to, po, _, _ = fwh.observer_pressure(surf["points"], surf["normals"], surf["areas"], rho, vel - fs[1:4], pres,
                                         st.every * dt, st.observer(), M, c0, fs[0], fs[4],
                                         n_copies=surf["n_copies"], shift=surf["copy_shift"])
    assert p.size == to.size and p.size > 40 and abs(t0 - to[0]) <= 1e-12 * abs(to[0])
    err = np.abs(p - po).max() / np.abs(po).max()
    mean = np.concatenate(forces).mean(axis=0)
    qref = 0.5 * fs[0] * (fs[1:4] @ fs[1:4]) * mesh["ref_area"]
    cl, cd = mean @ mesh["lift_dir"] / qref, mean @ mesh["drag_dir"] / qref
    print(f"  p' max rel err {err:.2e}; CL {f[5]:.6f} (oracle {cl:.6f}), CD {f[6]:.6f} (oracle {cd:.6f})", flush=True)
    assert err <= 1e-10
    assert f[7] == (st.n_samples - 1) * st.every
    scale = max(abs(cl), abs(cd))
    assert abs(f[5] - cl) <= 1e-10 * scale and abs(f[6] - cd) <= 1e-10 * scale


def test_sampled_request_bit_identical_to_hand_driven_pipeline():
    st = tiny(precision="fp32", n_samples=80, warmup=13, every=8, chunk=5)
    mesh, surf = st.mesh(X), st.surface(X)
    g = FRMesh(mesh, "fp32")
    u0 = uniform(mesh, g.shape)
    t0, p, f = run_pool(st, X, u0, "fp32")
    fs, c0, M = medium(st, X)
    g.set_state(u0)
    g.step(st.warmup)
    g.set_state(g.get_state())    # exact for an FP32 state; restarts the force means
    pr = Probe(g, surf["points"])
    rec = FWH(surf["points"], surf["normals"], surf["areas"], M, c0, fs[0], fs[4], st.every * mesh["dt"],
              st.n_samples, n_copies=surf["n_copies"], copy_shift=surf["copy_shift"])
    rec.append_probe(pr)
    for _ in range(st.n_samples - 1):
        g.step(st.every)
        rec.append_probe(pr)
    t_ref, p_ref = rec.pressure(st.observer())
    assert t0 == t_ref[0] and np.array_equal(p, p_ref)
    assert np.array_equal(f, g.forces())


def test_concurrent_designs_bit_identical_to_solo_runs():
    st = tiny(n_samples=128, warmup=10, every=8)
    designs = [X, [0.0, 6.5, 12.0, 6.0], [-3.0, 4.5, 9.0, 2.0]]
    ev = O.PoolEvaluator(st, X)
    together = ev(designs)
    assert ev.max_running == 3
    alone = [ev([d])[0] for d in designs]
    ev.close()
    for a, b in zip(together, alone):
        assert a.ok and (a.oaspl, a.cl, a.cd) == (b.oaspl, b.cl, b.cd)
    # a budget that holds one request at a time: the same results, one after another
    probe_pool = FRPool(st.budget_bytes)
    slot = probe_pool.admit_sampled(st.mesh(X), st.surface(X), st.warmup, st.every, st.n_samples)
    one = probe_pool.usage()[0]
    probe_pool.close()
    st1 = tiny(n_samples=128, warmup=10, every=8, budget_bytes=int(one * 1.3))
    ev1 = O.PoolEvaluator(st1, X)
    serial = ev1(designs)
    ev1.close()
    assert ev1.max_running == 1
    for a, b in zip(together, serial):
        assert (a.oaspl, a.cl, a.cd) == (b.oaspl, b.cl, b.cd)
    print(f"  one request holds {one / 2**20:.1f} MiB; OASPL {[round(r.oaspl, 3) for r in together]}", flush=True)


def test_variable_order_designs_run_concurrently_as_alone():
    """The paper's P-distribution (P3 at the wall down to P0 outside) in the evaluator:
    designs run side by side give the outcomes each gives alone."""
    st = tiny(n_samples=128, warmup=10, every=8, nj=8, bands=((2, 3), (4, 2), (6, 1), (8, 0)))
    designs = [X, [0.0, 6.5, 12.0, 6.0]]
    ev = O.PoolEvaluator(st, X)
    together = ev(designs)
    alone = [ev([d])[0] for d in designs]
    ev.close()
    assert ev.max_running == 2
    for a, b in zip(together, alone):
        assert a.ok and (a.oaspl, a.cl, a.cd) == (b.oaspl, b.cl, b.cd)


def test_orthomads_over_the_pool_follows_algorithm_1():
    st = tiny(n_samples=128, warmup=10, every=8)
    x0 = np.array([0.0, 6.5, 12.0, 6.0])      # NACA 0012 at 6 degrees
    lines = []
    res, base, seen = O.optimise(st, x0, l0=2, max_iter=3, log=lines.append)
    print("\n".join("  " + s for s in lines), flush=True)
    assert base.ok and np.isfinite(base.oaspl)
    # the first poll's 2n = 8 designs (all inside the bounds at this mesh size) ran side by side
    assert lines and lines[0].startswith("poll of 8 designs, 8 ran at once")
    d0 = 4.0 ** -2
    hist = res.history
    for (k0, dm0, f0, _), (k1, dm1, f1, _) in zip(hist, hist[1:]):
        dm = min(dm0, d0)                           # clamp at the start of the iteration
        assert dm1 == (4.0 * dm if f1 < f0 else dm / 4.0)
        assert f1 <= f0
    # the incumbent's value is the objective of its solved outcome
    r = seen[tuple(mads.unscale(res.x))]
    assert res.f == mads.objective(r.oaspl, r.cl, r.cd, base.cl, base.cd)

"""Far-field aeroacoustic shape optimisation of a NACA 4-digit airfoil (Section 3.4,
Algorithm 1): the OrthoMADS loop of ``mads`` driving the served request pool.

Every candidate design is one pool request (``FRPool.admit_sampled``): its O-grid is
built, its flow is advanced from the free stream, sampled on the permeable data surface
of Section 3.1 and fed to an FW-H record on the device, and its mean lift and drag are
accumulated over the sampled period.  The 2n poll designs of an iteration are admitted
together and run side by side on the GPU, so an iteration takes about as long as one
flow solve (the two layers of parallelism of Section 2.2); a design that does not fit
the pool's HBM budget waits until another finishes.  The objective is the OASPL at the
observer plus the lift and drag penalties of Section 3.4.

Design vector (Section 3.4, unscaled): maximum camber in % chord (negative: below the
chord), its position in tenths of chord, maximum thickness in % chord, angle of attack
in degrees; the optimiser works in [0, 1]^4.

Set-up (non-dimensional: chord, free-stream density and speed are 1):
  * the O-grid of ``workloads.naca_ogrid`` around the profile at zero incidence and a
    free stream at the angle of attack (Mach 0.2, Re 23,000);
  * the data surface of Section 3.1 (two sheets one chord apart, reaching four chords
    into the wake, closed upstream and open downstream, spanning the periodic span),
    tilted by the angle of attack about the leading edge (Section 3.4), duplicated along
    the span to ``lz`` chords;
  * the observer ten chords below the trailing edge, at mid-span;
  * one RK4 step for all designs (the baseline's stable step times a safety factor), so
    that a design's objective depends on the design alone.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import mads
from . import workloads as W
from ._lib import FR_E_MESH, FRError
from .solver import FRPool

# sea-level air at Mach 0.2 fixes the dimensional dynamic pressure that turns 20 uPa
# into free-stream units; the reference only shifts every OASPL by one constant
RHO_AIR, C_AIR = 1.225, 340.29


def p_ref(mach=0.2):
    return 2e-5 / (RHO_AIR * (mach * C_AIR) ** 2)


def oaspl(p, pref):
    """Overall sound pressure level (dB) of the fluctuation of p about its mean."""
    q = np.asarray(p, dtype=np.float64)
    q = q - q.mean()
    return 10.0 * math.log10(float(np.mean(q * q)) / pref ** 2)


def profile(x):
    """NACA parameters (m, p, t) and angle of attack of an unscaled design vector."""
    camber, pos, thick, aoa = (float(v) for v in x)
    return camber / 100.0, pos / 10.0, thick / 100.0, aoa


def data_surface(aoa_deg, spacing=0.01, span=0.2, height=1.0, wake=4.0, lz=25.0):
    """Panels of the open data surface, tilted by the angle of attack about the leading
    edge, with spanwise copies filling lz chords (an odd count, centred on the span)."""
    h = height / 2.0
    x0, x1 = -h, 1.0 + wake
    nx = max(1, int(round((x1 - x0) / spacing)))
    ny = max(1, int(round(height / spacing)))
    nz = max(1, int(round(span / spacing)))
    dx, dy, dz = (x1 - x0) / nx, height / ny, span / nz
    xs = x0 + dx * (np.arange(nx) + 0.5)
    ys = -h + dy * (np.arange(ny) + 0.5)
    zs = dz * (np.arange(nz) + 0.5)
    pts, nrm, area = [], [], []
    for z in zs:
        pts += [(x, h, z) for x in xs] + [(x, -h, z) for x in xs] + [(x0, y, z) for y in ys]
        nrm += [(0.0, 1.0, 0.0)] * nx + [(0.0, -1.0, 0.0)] * nx + [(-1.0, 0.0, 0.0)] * ny
        area += [dx * dz] * (2 * nx) + [dy * dz] * ny
    a = math.radians(aoa_deg)
    rot = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
    n_copies = max(1, int(round(lz / span)))
    if n_copies % 2 == 0:
        n_copies += 1
    return dict(points=np.asarray(pts) @ rot.T, normals=np.asarray(nrm) @ rot.T, areas=np.asarray(area),
                n_copies=n_copies, copy_shift=(0.0, 0.0, span))


@dataclass
class Study:
    """Sizes of one candidate's solve; the defaults are the paper's set-up at the grid of
    the single-design workload (160 x 48 x 8 quadratic hexahedra, P3)."""
    ni: int = 160
    nj: int = 48
    nk: int = 8
    order: int = 3
    span: float = 0.2
    radius: float = 20.0
    precision: str = "fp32"
    warmup: int = 2000           # steps before the first sample (transient)
    every: int = 4               # steps between samples
    n_samples: int = 1024
    spacing: float = 0.01        # data-surface panel size
    height: float = 1.0          # data-surface sheets: distance apart
    wake: float = 4.0            # and reach behind the trailing edge, in chords
    lz: float = 25.0             # spanwise extent of the duplicated surface
    dt_safety: float = 0.8
    budget_bytes: int = 200 << 30
    chunk: int = 50              # steps per pool tick
    device: int = 0
    # variable order (Section 3.1): ((first layer beyond the band, order), ...) from the
    # wall outward, e.g. ((12, 3), (24, 2), (36, 1), (48, 0)); None: `order` everywhere
    bands: tuple = None

    def observer(self):
        return np.array([1.0, -10.0, 0.5 * self.span])

    def mesh(self, x, dt=None):
        m, pc, t, aoa = profile(x)
        mesh = W.naca_ogrid(m, pc, t, self.ni, self.nj, self.nk, span=self.span, radius=self.radius,
                            order=self.order)
        mesh.update(W.airfoil_flow(aoa_deg=aoa, span=self.span))
        if self.bands is not None:
            mesh["orders"] = W.ring_orders(self.ni, self.nj, self.nk, self.bands)
        mesh["dt"] = W.airfoil_dt(mesh, self.order) * self.dt_safety if dt is None else dt
        return mesh

    def surface(self, x):
        return data_surface(profile(x)[3], spacing=self.spacing, span=self.span, height=self.height,
                            wake=self.wake, lz=self.lz)


@dataclass
class Outcome:
    oaspl: float
    cl: float      # mean lift coefficient over the sampled period
    cd: float      # mean drag coefficient over the sampled period
    ok: bool = True


class PoolEvaluator:
    """Runs candidate designs (unscaled vectors) as concurrent pool requests.

    progress: optional callable taking a message, called at most every `every_s` seconds
    while requests run."""

    def __init__(self, study: Study, x_baseline, progress=None, every_s=30.0):
        self.study = study
        self.dt = study.mesh(x_baseline)["dt"]
        self.pool = FRPool(study.budget_bytes, study.device)
        self.pref = p_ref()
        self.max_running = 0
        self.progress, self.every_s = progress, every_s

    def close(self):
        self.pool.close()

    def __call__(self, designs):
        s = self.study
        out = [None] * len(designs)
        pending = list(range(len(designs)))
        running = {}
        last = time.perf_counter()
        while pending or running:
            while pending:
                i = pending[0]
                try:
                    slot = self.pool.admit_sampled(s.mesh(designs[i], self.dt), s.surface(designs[i]), s.warmup,
                                                   s.every, s.n_samples, precision=s.precision)
                except FRError as e:
                    if e.code != FR_E_MESH:
                        # the mesh is valid but the request is not (e.g. a surface point
                        # outside the grid): a set-up error, not an infeasible design; so is
                        # any other exception, which is not caught here
                        raise RuntimeError(f"design {list(designs[i])}: {e}") from e
                    out[i] = Outcome(math.inf, math.nan, math.nan, ok=False)  # no valid mesh: infeasible
                    pending.pop(0)
                    continue
                if slot is None:
                    if not running:
                        raise RuntimeError("a design does not fit in the pool's HBM budget")
                    break
                running[slot] = i
                pending.pop(0)
            self.max_running = max(self.max_running, len(running))
            if not running:
                break
            if self.progress is not None and time.perf_counter() - last >= self.every_s:
                last = time.perf_counter()
                self.progress(f"{len(running)} designs running, {sum(o is not None for o in out)} of "
                              f"{len(designs)} done, {len(pending)} waiting")
            for slot in self.pool.tick(s.chunk):
                i = running.pop(slot)
                p = err = None
                try:
                    _, p = self.pool.pressure(slot, s.observer(), s.n_samples)
                except FRError as e:
                    err = e
                try:
                    f = self.pool.result(slot)   # also frees the request
                except FRError:
                    out[i] = Outcome(math.inf, math.nan, math.nan, ok=False)   # the run failed
                    continue
                if err is not None:              # the run is fine but the study is not
                    raise RuntimeError(f"design {list(designs[i])}: {err}")
                out[i] = Outcome(oaspl(p, self.pref), float(f[5]), float(f[6]))
        return out


def optimise(study: Study, x0, l0=2, max_iter=100, mesh_tol=1e-6, move_tol=0.01, log=None):
    """OrthoMADS from the unscaled baseline x0.  Returns (mads.Result with the scaled
    incumbent, baseline Outcome, {design tuple: Outcome} of every solved design)."""
    ev = PoolEvaluator(study, x0, progress=log)
    seen = {}
    try:
        base = ev([np.asarray(x0, dtype=np.float64)])[0]
        if not base.ok:
            raise RuntimeError("the baseline design failed")
        seen[tuple(np.asarray(x0, dtype=np.float64))] = base

        def evaluate(points):
            xs = [mads.unscale(p) for p in points]
            res = ev(xs)
            vals = []
            for x, r in zip(xs, res):
                seen[tuple(x)] = r
                vals.append(mads.objective(r.oaspl, r.cl, r.cd, base.cl, base.cd) if r.ok else math.inf)
            if log:
                log(f"poll of {len(points)} designs, {ev.max_running} ran at once, best "
                    f"{min(vals):.4f}")
            return vals

        f0 = mads.objective(base.oaspl, base.cl, base.cd, base.cl, base.cd)
        res = mads.orthomads(evaluate, mads.scale(x0), l0=l0, mesh_tol=mesh_tol, move_tol=move_tol,
                             max_iter=max_iter, f0=f0)
        return res, base, seen
    finally:
        ev.close()


def main(argv=None):
    """Run Algorithm 1 from the baseline of Section 3.4 (NACA 0012 at 6 degrees) over the
    served pool; print one line per poll and a JSON summary.

        python -m paper_2501_05709_amd.optimize [--max-iter K] [--bands] [sizes ...]
    """
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--l0", type=int, default=2, help="initial mesh index (mesh size 4^-l0)")
    ap.add_argument("--ni", type=int, default=160)
    ap.add_argument("--nj", type=int, default=48)
    ap.add_argument("--nk", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--every", type=int, default=4)
    ap.add_argument("--n-samples", type=int, default=1024)
    ap.add_argument("--spacing", type=float, default=0.01)
    ap.add_argument("--lz", type=float, default=25.0, help="spanwise extent of the copied data surface")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--bands", action="store_true",
                    help="P3 in the 12 wall layers, then P2, P1, P0 in bands of 12 (Section 3.1)")
    args = ap.parse_args(argv)
    bands = ((12, 3), (24, 2), (36, 1), (args.nj, 0)) if args.bands else None
    st = Study(ni=args.ni, nj=args.nj, nk=args.nk, warmup=args.warmup, every=args.every,
               n_samples=args.n_samples, spacing=args.spacing, lz=args.lz, precision=args.precision, bands=bands)
    x0 = np.array([0.0, 6.5, 12.0, 6.0])
    t0 = time.perf_counter()

    def log(msg):
        print(f"[{time.perf_counter() - t0:8.1f} s] {msg}", flush=True)

    log(f"baseline {list(x0)}: {st.ni}x{st.nj}x{st.nk} O-grid, {st.warmup} + {st.n_samples - 1} x "
        f"{st.every} steps per design, data surface spacing {st.spacing}, copies over {st.lz} chords")
    res, base, seen = optimise(st, x0, l0=args.l0, max_iter=args.max_iter, log=log)
    wall = time.perf_counter() - t0
    for k, dm, f, x in res.history:
        log(f"iteration {k}: mesh size {dm:.3g}, incumbent {f:.4f} at {[round(v, 3) for v in mads.unscale(x)]}")
    print(json.dumps({
        "iterations": res.iterations, "evaluations": res.evaluations, "designs_solved": len(seen),
        "wall_s": round(wall, 1), "baseline": {"oaspl_db": base.oaspl, "cl": base.cl, "cd": base.cd},
        "best": {"design": [float(v) for v in mads.unscale(res.x)], "objective": res.f},
    }))


if __name__ == "__main__":
    main()

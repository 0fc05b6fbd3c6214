#!/usr/bin/env python3
"""FR DOF-updates/s on one MI355X: FP32 form vs plain FP64 at stated L2 error, with the
p50/p99 latency of batched solves.

Workload (default, ``--workload batch``): sixteen candidate airfoil designs, NACA
4-digit O-grids of (96-192) x (32-64) x (4-12) quadratic hexes (917,407 elements,
p = 3, 64 solution points each), Re 23,000, Mach 0.2, AoA 5 deg, impulsive start,
advanced together: every launch covers all designs and one captured graph runs a
step.  A "step" is one full RK4 step (four FR residual evaluations with the fused
stage updates) of the whole batch; the state is resident in HBM before the timed
region starts.

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--workload batch|tgv|airfoil|serve|fwh|pmix]

Prints one JSON line.  ``value`` is FP32-form DOF-updates/s (DOF = elements x
solution points x conserved variables, one update = one RK4 step) of the median of
five timing windows that together cover exactly ``--steps`` steps; the plain FP64
path is timed the same way beside it.  Also: relative L2 errors against the FP64
oracle on the smallest design after 100 steps (``--full-parity`` adds one design drawn
at random; the GPU tests compare both), of the state and of its change from the
initial state, p50/p99 latency of repeated batched solves, the
roofline of one RK stage (both fused launches) from the method's algorithmic bytes,
GPU clock and temperature, and the Taylor-Green 24^3 and single-airfoil workloads as
extra keys.  The CPU baseline is the FP64 oracle on this host's cores on a bounded
sample (the smallest design for 100 steps).

Other workloads: ``tgv`` (Taylor-Green 24^3 straight hexes, p = 3) and ``airfoil``
(one 160x48x8 O-grid) alone; ``serve``: a Poisson stream of airfoil solve requests
(mean 4/s, order 2..4, 500 steps each) through the request pool (p50/p99 latency
from arrival to result, aggregate DOF-updates/s; ``--serial-run`` also serves the same trace
FIFO, one request at a time, on the plain FP64 path); ``pmix``: the airfoil grid with the
order falling from 3 at the wall to 0 toward the far field (variable order); ``fwh``:
the far-field acoustic sum.
"""
import argparse
import hashlib
import threading
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm": 8000.0, "mfma_f32": 157.3, "mfma_f64": 78.6, "fp64": 78.6}  # GB/s, TFLOP/s (fp64: vector FMA)
KERNEL_NAMES = {1: "k_face", 2: "k_grad", 3: "k_visc", 4: "k_divrk", 5: "k_interp", 6: "k_stage_a",
                7: "k_stage_b"}


def metric_source(mask):
    """Where the fused stage takes its FP64 metrics from, by variant mask: 'stored' (S,
    1/|J|, normals and areas per point), 'extruded' (2D columns of z-extruded elements)
    or 'node' (the 27 geometry nodes of each element)."""
    if mask & (1 << 8):
        return "extruded"
    return "stored" if mask & (1 << 6) else "node"


def per_element_cost(dim, order, real_bytes, metrics="stored"):
    """Dense-MFMA flops and implementation bytes of each kernel, per element and launch:
    what each kernel of this library reads and writes (its own data layout and metric
    source, see ``metric_source``), not the method's minimum
    (``algorithmic_bytes_per_element_stage``).

    Operator sizes are the unpadded FR matrices (n_u solution points, n_f flux
    points); metric terms are FP64 (8 bytes), neighbour indices 4 bytes.
    """
    n = order + 1
    nu = n ** dim
    nf = 2 * dim * n ** (dim - 1)
    nv = dim + 2
    s = real_bytes
    # metric bytes of the fused stage's first launch and its second (areas only when stored;
    # 1/|J| per solution point, or from the column and layer factors on extruded meshes)
    if dim == 3 and metrics == "extruded":
        met_a, area_b, ij_b = (4 * n * n + n + 2 * (4 * n + n * n)) * 8, 0, (n * n + n) * 8
    elif dim == 3 and metrics == "node":
        met_a, area_b, ij_b = 27 * 3 * 8, 0, nu * 8
    else:
        met_a, area_b, ij_b = nf * dim * 8 + nu * (dim * dim + 1) * 8, nf * 8, nu * 8
    cost = {
        1: dict(flops=0, bytes=(2 * nf * nv * s + nf * dim * 8 + nf * 4) + 2 * nf * nv * s),
        2: dict(flops=2 * nv * (dim * nu * nu + dim * nu * nf),
                bytes=nu * nv * s + nf * nv * s + nu * (dim * dim + 1) * 8 + 2 * nu * dim * nv * s),
        3: dict(flops=2 * dim * nv * nf * nu,
                bytes=nu * dim * nv * s + nf * nv * s + nf * dim * 8 + nf * 4 + nf * nv * s),
        4: dict(flops=2 * nv * (nu * dim * nu + nu * nf),
                bytes=nu * dim * nv * s + 3 * nf * nv * s + nf * 8 + nf * 4 + nu * 8 + 2 * nu * nv * s
                + 2 * nu * nv * s),
        5: dict(flops=2 * nv * nf * nu, bytes=nu * nv * s + nf * nv * s),
        # fused stage a: stage state, partner traces, neighbour codes and the metric source
        # in; Q, P and the volume divergence out
        6: dict(flops=0, bytes=nu * nv * s + nf * nv * s + nf * 4 + met_a + 2 * nf * nv * s + nu * nv * s),
        # fused stage b: Q, partner P, per-face codes, areas (stored metrics only), divergence, 1/|J|,
        # u_n and acc in; acc, next stage state and its trace out; the first stage reads no
        # acc and the last writes none, so acc counts 3/4 each way (mean over the four RK
        # stages)
        7: dict(flops=0, bytes=2 * nf * nv * s + 2 * dim * 4 + area_b + nu * nv * s + ij_b
                + 1.75 * nu * nv * s + 1.75 * nu * nv * s + nf * nv * s),
    }
    return cost, nu * nv


def rel_l2(x, ref):
    """Max over density, momentum vector and total energy of ||x - ref|| / ||ref||."""
    nv = ref.shape[-1]
    x = x.reshape(-1, nv)
    ref = ref.reshape(-1, nv)
    out = []
    for cols in ([0], list(range(1, nv - 1)), [nv - 1]):
        out.append(float(np.linalg.norm(x[:, cols] - ref[:, cols]) / np.linalg.norm(ref[:, cols])))
    return max(out)


def kinetic_energy(u, order):
    """Volume mean of rho |v|^2 / 2 over a mesh of equal affine hexes (tensor GL weights)."""
    w = np.polynomial.legendre.leggauss(order + 1)[1]
    wt = np.multiply.outer(np.multiply.outer(w, w), w).ravel() / 8.0
    m2 = (u[..., 1:4] ** 2).sum(axis=-1)
    return float((0.5 * m2 / u[..., 0] * wt).sum(axis=-1).mean())


def stage_kernel_name(kernel, mask, real="float", dim=3, order=3):
    """The fused-stage kernel a variant mask selects, as rocprofv3 names it (the second
    launch with MODE 0): metric source (bit 8 extruded columns 3, bit 6 stored 1, else
    node metrics 0), tile of each launch (bits 9-10, 11-12), exchange (bit 13 scatter)."""
    fv = 3 if mask & (1 << 8) else (1 if mask & (1 << 6) else 0)
    scat = "true" if mask & (1 << 13) else "false"
    if kernel == "k_stage_a":
        return f"k_stage_a<{real}, {dim}, {order}, {fv}, {(mask >> 9) & 3}, {scat}>"
    return f"k_stage_b<{real}, {dim}, {order}, 0, {fv}, {(mask >> 11) & 3}, {scat}>"


def counters_traffic(workload, kernel, mask=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or
    None if it is missing or the kernel source changed since it was taken. Given the
    selected variant mask, the entry taken on that variant (the entries of a kernel are
    keyed `kernel` and `kernel_<variant>`, each with the kernel names it matched), else
    None."""
    import re
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path)).get(workload, {})
        src = open(os.path.join(ROOT, "paper_2501_05709_amd", "csrc", "fr_kernels.hip"), "rb").read()
        sha = hashlib.sha256(src).hexdigest()
        keys = [kernel] if mask is None else [k for k in sorted(data) if k == kernel or k.startswith(kernel + "_")]
        for key in keys:
            entry = data.get(key)
            if not entry or entry.get("source_sha256") != sha:
                continue
            if mask is not None and not re.search(entry.get("kernel_match", ""), stage_kernel_name(kernel, mask)):
                continue
            return entry.get("hbm_bytes_per_launch")
        return None
    except Exception:
        return None


def build_workload(name):
    from paper_2501_05709_amd import workloads as W
    if name == "tgv":
        m = W.config_tgv(nel=24, order=3)
        desc = {"workload": "taylor_green_24^3_hex_p3", "elements": 13824, "order": 3,
                "reynolds": 1600, "mach": 0.1, "dt": m["dt"], "mesh": "periodic straight hexes"}
    elif name == "airfoil":
        m = W.config_airfoil(0, ni=160, nj=48, nk=8, order=3)
        desc = {"workload": "naca4_ogrid_160x48x8_quadratic_hex_p3", "elements": 61440, "order": 3,
                "reynolds": 23000, "mach": 0.2, "aoa_deg": 5.0, "dt": m["dt"],
                "mesh": "curved quadratic hexes, wall + far field + spanwise periodic"}
    elif name == "batch_small":
        meshes = W.config_batch(0)
        m = meshes[int(np.argmin([len(x["elem_nodes"]) for x in meshes]))]
        desc = {"workload": "smallest design of the 16-design batch", "elements": len(m["elem_nodes"]),
                "order": 3, "dt": m["dt"]}
    else:
        raise SystemExit(f"unknown workload {name}")
    return m, desc


def timed_run(mesh, u0, steps, warmup):
    import torch
    mesh.set_state(u0)
    if warmup:
        mesh.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def algorithmic_bytes_per_element_stage(dim, order, real_bytes, curved):
    """Minimum HBM bytes one RK stage must move per element, with one fused element pass
    per exchange phase: the state (read the stage input, u_n and the accumulator, write
    the accumulator and the next stage input: 5 V n_u s), the two neighbour exchanges
    (write the traces and read the partner's; write the viscous normal flux, read the
    partner's and the common flux: 5 V n_f s), and on curved elements the FP64 metrics
    read once ((d^2 + 1) values per solution point, d per face point, shared by the two
    sides of a face).  Affine elements carry constant metrics, counted as zero."""
    n = order + 1
    nu, nf, nv = n ** dim, 2 * dim * n ** (dim - 1), dim + 2
    b = 5 * nv * nu * real_bytes + 5 * nv * nf * real_bytes
    if curved:
        b += (dim * dim + 1) * 8 * nu + dim * 8 * nf / 2
    return b


def gpu_telemetry():
    """GPU clock (MHz) and temperature (C) now, from the driver's management library."""
    out = {}
    try:
        import torch
        out["gfx_clock_mhz"] = int(torch.cuda.clock_rate())
        out["temperature_c"] = float(torch.cuda.temperature())
    except Exception as e:  # reported, not fatal
        out["error"] = str(e)[:120]
    return out


def progress(msg):
    """One line per finished phase on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def windows(mesh, steps, n_windows=5):
    """Time `steps` steps as n_windows consecutive windows (host clock around each
    synchronising fr_step); returns the per-window seconds and steps per window."""
    import torch
    n_windows = max(1, min(n_windows, steps))
    per = steps // n_windows
    ts = []
    torch.cuda.synchronize()
    for w in range(n_windows):
        k = per if w < n_windows - 1 else steps - per * (n_windows - 1)
        t0 = time.perf_counter()
        mesh.step(k)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0, k))
    return ts


def median_rate(dof, ts):
    """DOF-updates/s of the median window (per-step time of each window)."""
    per_step = sorted(t / k for t, k in ts)
    med = per_step[len(per_step) // 2]
    return dof / med, med


def stage_roofline(mesh, dim, order, real_bytes, curved, workload, steps=5):
    """Roofline of one RK stage (both fused launches): algorithmic bytes of the stage over
    the mean event-timed durations of k_stage_a + k_stage_b, against HBM peak; counter
    traffic per stage beside it when the committed counters match the kernel source."""
    ms, nl = mesh.profile_kernels(steps)
    if not (nl[6] and nl[7]):
        return None, ms, nl
    t_a, t_b = ms[6] / nl[6] * 1e-3, ms[7] / nl[7] * 1e-3
    alg = algorithmic_bytes_per_element_stage(dim, order, real_bytes, curved) * mesh.E
    achieved = alg / (t_a + t_b) / 1e9
    metrics = metric_source(mesh.selected_kernels())
    cost, _ = per_element_cost(dim, order, real_bytes, metrics)
    impl = (cost[6]["bytes"] + cost[7]["bytes"]) * mesh.E
    sel = mesh.selected_kernels()
    ta, tb = counters_traffic(workload, "k_stage_a", sel), counters_traffic(workload, "k_stage_b", sel)
    traffic = ta + tb if ta is not None and tb is not None else None
    n = order + 1
    dof_updates_per_stage = mesh.E * n ** dim * (dim + 2) / 4.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm"], "unit": "GB/s",
            "frac": round(achieved / PEAK["hbm"], 4), "traffic": traffic,
            "kernel": "one RK stage: k_stage_a + k_stage_b",
            "stage_us": round((t_a + t_b) * 1e6, 2), "k_stage_a_us": round(t_a * 1e6, 2),
            "k_stage_b_us": round(t_b * 1e6, 2),
            "algorithmic_bytes_per_stage": int(alg),
            "algorithmic_bytes_per_dof_update": round(alg / dof_updates_per_stage, 1),
            "implementation_bytes_per_stage": int(impl), "metric_source": metrics,
            "traffic_over_algorithmic": round(traffic / alg, 3) if traffic else None}
    return roof, ms, nl


def batch_states(meshes, nu, nv, b):
    """Impulsive start: every design at its own free stream."""
    from paper_2501_05709_amd import workloads as W
    return np.concatenate([W.uniform_state(b.design_range(i)[1] * nu, m["freestream"][0], m["freestream"][1:4],
                                           m["freestream"][4]).reshape(-1, nu, nv)
                           for i, m in enumerate(meshes)])


def bench_single_quick(name, steps):
    """C2 / C3 beside the batch line: FP32 and FP64 rates (median of 5 windows) and the
    whole-stage roofline of the FP32 form."""
    import torch
    from paper_2501_05709_amd.solver import FRMesh
    m, desc = build_workload(name)
    out = {"workload": desc["workload"]}
    for prec in ("fp32", "fp64"):
        g = FRMesh(m, prec)
        u0 = np.ascontiguousarray(m["init"](g.solution_points().reshape(-1, 3)).reshape(g.shape))
        g.set_state(u0)
        g.autotune(2)
        g.set_state(u0)
        g.step(5)
        dof = g.E * g.nu * g.nv
        rate, med = median_rate(dof, windows(g, steps))
        out[prec] = {"value": round(rate, 1), "ms_per_step": round(med * 1e3, 4)}
        if prec == "fp32":
            g.set_state(u0)
            roof, _, _ = stage_roofline(g, 3, 3, 4, name != "tgv", name)
            out["roofline_fp32"] = roof
        g.close()
        del g
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def bench_batch(args):
    """The headline line: sixteen uneven NACA 4-digit O-grids (917,407 curved hexes, p = 3)
    advanced together, every launch covering all designs, one captured graph per step.

    value: FP32-form DOF-updates/s of the median of 5 timing windows over exactly
    `steps` steps; the plain FP64 path beside it; relative L2 against the oracle on
    sampled designs; p50/p99 latency of repeated batched solves; the whole-stage
    roofline; the oracle's rate on this host as the CPU baseline."""
    import torch
    from paper_2501_05709_amd import workloads as W
    from paper_2501_05709_amd.solver import FRMesh
    t_setup = time.perf_counter()
    meshes = W.config_batch(0)
    sizes = [len(m["elem_nodes"]) for m in meshes]
    small = int(np.argmin(sizes))
    other = int(np.random.default_rng(7).choice([i for i in range(len(meshes)) if i != small]))
    b32 = FRMesh(meshes, "fp32")
    nu, nv = b32.nu, b32.nv
    u0 = batch_states(meshes, nu, nv, b32)
    dof = b32.E * nu * nv
    b32.set_state(u0)
    mask32 = b32.autotune(2)
    b64 = FRMesh(meshes, "fp64")
    b64.set_state(u0)
    mask64 = b64.autotune(2)
    t_setup = time.perf_counter() - t_setup
    progress(f"batch built and autotuned in {t_setup:.0f} s (fp32 mask {mask32}, fp64 mask {mask64})")

    # --- parity on sampled designs and the CPU baseline (the oracle on the smallest design)
    parity, cpu = {}, None
    n_sample = args.cpu_steps or 100
    if not args.no_cpu_baseline:
        from oracle.oracle import OracleMesh, num_threads
        for g in (b32, b64):
            g.set_state(u0)
            g.step(n_sample)
        s32, s64 = b32.get_state(), b64.get_state()
        for i in (small, other) if args.full_parity else (small,):
            o = OracleMesh(meshes[i])
            e0, ne = b32.design_range(i)
            ui = u0[e0:e0 + ne]
            t0 = time.perf_counter()
            ref = o.rk4(ui, meshes[i]["dt"], n_sample)
            tc = time.perf_counter() - t0
            d_ref = ref - ui
            entry = {"elements": ne, "steps": n_sample}
            for prec, s in (("fp32", s32), ("fp64", s64)):
                x = s[e0:e0 + ne]
                entry[f"{prec}_rel_l2_vs_oracle"] = rel_l2(x, ref)
                # the impulsive start changes the state near the wall only: the error of
                # the change from the initial state is the sharper measure
                entry[f"{prec}_rel_l2_of_change_vs_oracle"] = rel_l2(x - ui, d_ref)
            parity[f"design_{i}"] = entry
            progress(f"oracle on design {i} ({ne} elements, {n_sample} steps): {tc:.0f} s")
            if i == small:
                cpu = {"value": ne * nu * nv * n_sample / tc, "unit": "DOF-updates/s", "cores": num_threads(),
                       "kind": "oracle", "host": host_cpu(),
                       "sample": f"{n_sample} RK4 steps of the smallest design ({ne} curved hexes, p = 3) of "
                                 f"the batch, FP64, OpenMP over elements, {tc:.1f} s wall on {num_threads()} "
                                 f"threads ({tc * num_threads():.0f} thread-s)",
                       "one_thread": oracle_one_thread("batch_small")}
        del s32, s64

    # --- timed region: the plain FP64 path, then the FP32 form (the reported value)
    tel = {"before": gpu_telemetry()}
    res = {}
    for prec, g in (("fp64", b64), ("fp32", b32)):
        g.set_state(u0)
        if args.warmup:
            g.step(args.warmup)
        ts = windows(g, args.steps)
        rate, med = median_rate(dof, ts)
        total = sum(t for t, _ in ts)
        progress(f"{prec}: {rate:.4g} DOF-updates/s")
        res[prec] = {"value": rate, "ms_per_step": med * 1e3, "window_ms_per_step": [round(t / k * 1e3, 4)
                                                                                  for t, k in ts],
                     "value_whole_window": dof * args.steps / total}
    tel["after_timed"] = gpu_telemetry()
    err32_vs64 = rel_l2(b32.get_state(), b64.get_state())

    # --- per-kernel events and the whole-stage roofline (FP32 form)
    b32.set_state(u0)
    roof, ms, nl = stage_roofline(b32, 3, 3, 4, True, "batch")
    cost, _ = per_element_cost(3, 3, 4, metric_source(mask32))
    kernels = {}
    for k in range(1, 8):
        if not nl[k]:
            continue
        avg_ms = ms[k] / nl[k]
        kernels[KERNEL_NAMES[k]] = {"avg_us": round(avg_ms * 1e3, 2), "share": round(ms[k] / ms[0], 3),
                                    "implementation_gbs": round(cost[k]["bytes"] * b32.E / (avg_ms * 1e-3) / 1e9, 1)}

    # --- batched-solve latency: set the state, run the solve, read every design's forces
    lat = []
    for _ in range(args.solves):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b32.set_state(u0)
        b32.step(args.solve_steps)
        [b32.forces(i) for i in range(len(meshes))]
        lat.append(time.perf_counter() - t0)
    progress(f"{len(lat)} batched solves done")
    tel["after_solves"] = gpu_telemetry()
    lat = np.array(lat) if lat else None
    cl = [round(float(b32.forces(i)[5]), 6) for i in range(len(meshes))]
    b32.close()
    b64.close()
    del b32, b64
    torch_empty()

    extras = {}
    if not args.no_extras:
        for name in ("tgv", "airfoil"):
            extras[name] = bench_single_quick(name, 50)
            progress(f"extra workload {name} done")

    out = {
        "metric": "FR DOF-updates/s FP64 vs FP32 at stated L2 err; p50/p99 batched solve latency",
        "value": round(res["fp32"]["value"], 1), "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(res["fp32"]["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch of 16 NACA 4-digit O-grids (96-192)x(32-64)x(4-12) quadratic hexes, p=3, "
                               "Re 23000, Mach 0.2, AoA 5 deg, seed 0, impulsive start",
                   "elements": int(sum(sizes)), "dof": dof, "designs": len(meshes),
                   "form": "fp32 operators/fluxes/state, fp64 metrics and force sums",
                   "timing": f"median of {min(5, args.steps)} windows over {args.steps} steps after "
                             f"{args.warmup} warm-up steps, one captured graph per step",
                   "parallelism": "single GPU"},
        "fp64": {"value": round(res["fp64"]["value"], 1), "ms_per_step": round(res["fp64"]["ms_per_step"], 4),
                 "window_ms_per_step": res["fp64"]["window_ms_per_step"],
                 "value_whole_window": round(res["fp64"]["value_whole_window"], 1)},
        "fp32_window_ms_per_step": res["fp32"]["window_ms_per_step"],
        "fp32_value_whole_window": round(res["fp32"]["value_whole_window"], 1),
        "speedup_fp32_over_fp64": round(res["fp32"]["value"] / res["fp64"]["value"], 3),
        "parity_vs_oracle": parity, "fp32_rel_l2_vs_fp64_gpu": err32_vs64,
        "batched_solve_latency_s": None if lat is None else {
            "steps": args.solve_steps, "repeats": int(lat.size), "p50": round(float(np.percentile(lat, 50)), 4),
            "p99": round(float(np.percentile(lat, 99)), 4), "all": [round(float(v), 4) for v in lat],
            "includes": "set_state from host, the steps, forces of every design"},
        "mean_CL_per_design": cl,
        "kernel_variants": {"fp32_mask": mask32, "fp64_mask": mask64},
        "kernels": kernels,
        "roofline": roof,
        "gpu_telemetry": tel,
        "measured_ceilings": measured_ceilings(),
        "setup_s": round(t_setup, 1),
        "extra_workloads": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def torch_empty():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def bench_serve(args):
    """Poisson stream of solve requests through the continuous-batching pool."""
    from paper_2501_05709_amd import workloads as W
    from paper_2501_05709_amd.solver import FRMesh, FRPool, footprint
    trace = W.request_trace(0, n_requests=args.requests, rate=args.rate)
    meshes = [W.config_airfoil(ni=r["ni"], nj=r["nj"], nk=r["nk"], order=r["order"], design=r["design"])
              for r in trace]
    # autotune each order once so the pool's solvers start from the tuned choice
    for order in sorted({r["order"] for r in trace}):
        small = W.config_airfoil(ni=48, nj=16, nk=2, order=order)
        g = FRMesh(small, "fp32")
        fs = small["freestream"]
        g.set_state(W.uniform_state(g.E * g.nu, fs[0], fs[1:4], fs[4]).reshape(g.shape))
        g.autotune(2)
        g.close()
    steps = 500
    pool = FRPool(int(args.budget_gb * 2 ** 30))
    elems = [len(m["elem_nodes"]) for m in meshes]
    dof = [e * (m["order"] + 1) ** 3 * 5 for e, m in zip(elems, meshes)]
    arrival = {i: trace[i]["arrival"] for i in range(len(trace))}
    done_at, admitted_at = {}, {}
    slot_of = {}
    running_elems = [0]
    lock = threading.Lock()
    t0 = time.perf_counter()
    tick = 25

    def admitter():
        # FIFO admission in arrival order, at most `cap` active elements (enough to
        # fill the device) and within the pool's HBM budget
        for i in range(len(trace)):
            while time.perf_counter() - t0 < arrival[i]:
                time.sleep(0.001)
            while True:
                with lock:
                    ok = running_elems[0] == 0 or running_elems[0] + elems[i] <= args.active_elements
                if ok:
                    s = pool.admit(meshes[i], steps, precision="fp32")
                    if s is not None:
                        break
                time.sleep(0.002)
            with lock:
                slot_of[s] = i
                running_elems[0] += elems[i]
                admitted_at[i] = time.perf_counter() - t0

    th = threading.Thread(target=admitter, daemon=True)
    th.start()
    while len(done_at) < len(trace):
        with lock:
            active = bool(slot_of)
        if not active:
            time.sleep(0.001)
            continue
        pool.launch(tick)
        for s in pool.collect():
            pool.result(s)
            with lock:
                i = slot_of.pop(s)
                running_elems[0] -= elems[i]
            done_at[i] = time.perf_counter() - t0
    th.join()
    makespan = time.perf_counter() - t0
    lat = np.array([done_at[i] - arrival[i] for i in range(len(trace))])
    total = sum(d * steps for d in dof)
    pool.close()
    # serial FP64 reference (modelled, not run): the FP64 rate per order measured on a
    # mid-size request with the same autotuned kernels as the main line's FP64 path, then
    # the same trace served one request at a time (FIFO) at those rates.  The all-dense
    # FP64 rate is reported beside it.
    rate64, rate64_dense = {}, {}
    for order in sorted({r["order"] for r in trace}):
        mm = W.config_airfoil(ni=144, nj=48, nk=8, order=order)
        g = FRMesh(mm, "fp64")
        fs = mm["freestream"]
        u0 = W.uniform_state(g.E * g.nu, fs[0], fs[1:4], fs[4]).reshape(g.shape)
        g.set_state(u0)
        mask = g.autotune(2)
        t = timed_run(g, u0, 20, 2)
        rate64[order] = g.E * g.nu * g.nv * 20 / t
        g.select_kernels(0)
        t = timed_run(g, u0, 20, 2)
        rate64_dense[order] = g.E * g.nu * g.nv * 20 / t
        g.select_kernels(mask)
        g.close()
    clock, lat64 = 0.0, []
    for i in range(len(trace)):
        clock = max(clock, arrival[i]) + dof[i] * steps / rate64[trace[i]["order"]]
        lat64.append(clock - arrival[i])
    lat64 = np.array(lat64)
    serial_run = None
    if args.serial_run:
        # the same trace served FIFO one request at a time on the plain FP64 path (autotuned
        # kernels, a fresh solver per request), in real time against the arrival clock
        t0s = time.perf_counter()
        done64 = []
        for i in range(len(trace)):
            while time.perf_counter() - t0s < arrival[i]:
                time.sleep(0.001)
            g = FRMesh(meshes[i], "fp64")
            fs = meshes[i]["freestream"]
            g.set_state(W.uniform_state(g.E * g.nu, fs[0], fs[1:4], fs[4]).reshape(g.shape))
            g.step(steps)
            g.forces()
            g.close()
            done64.append(time.perf_counter() - t0s)
            progress(f"serial fp64 request {i + 1}/{len(trace)} done")
        lat_s = np.array([done64[i] - arrival[i] for i in range(len(trace))])
        serial_run = {"latency_p50_s": round(float(np.percentile(lat_s, 50)), 3),
                      "latency_p99_s": round(float(np.percentile(lat_s, 99)), 3),
                      "makespan_s": round(done64[-1], 3),
                      "dof_updates_per_s": round(total / done64[-1], 1),
                      "note": "run: FIFO one request at a time, plain FP64 path, same requests and arrivals"}
    res = {
        "metric": "served airfoil solves: p50/p99 latency (arrival to result) and aggregate DOF-updates/s",
        "value": round(total / makespan, 1), "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson trace of {len(trace)} NACA O-grid solves, mean {args.rate:g}/s, orders 2-4, "
                               f"{steps} RK4 steps each, seed 0", "budget_gb": args.budget_gb, "tick_steps": tick,
                   "active_element_cap": args.active_elements},
        "queue_wait_p50_s": round(float(np.percentile([admitted_at[i] - arrival[i] for i in range(len(trace))], 50)), 3),
        "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
        "latency_max_s": round(float(lat.max()), 3),
        "makespan_s": round(makespan, 3), "last_arrival_s": round(max(arrival.values()), 3),
        "offered_dof_updates": total,
        "offered_dof_updates_per_s": round(total / max(arrival.values()), 1),
        "serial_fp64_modelled": {"dof_updates_per_s_by_order": {str(k): round(v, 1) for k, v in rate64.items()},
                                 "dense_mfma_dof_updates_per_s_by_order": {str(k): round(v, 1)
                                                                          for k, v in rate64_dense.items()},
                                 "modelled_makespan_s": round(clock, 3),
                                 "modelled_latency_p50_s": round(float(np.percentile(lat64, 50)), 3),
                                 "modelled_latency_p99_s": round(float(np.percentile(lat64, 99)), 3),
                                 "note": "not run: FIFO one-at-a-time service at the measured FP64 rates of "
                                         "the autotuned kernels (the main line's FP64 path)"},
        "modelled_speedup_vs_serial_fp64": round(clock / makespan, 3),
        "serial_fp64_run": serial_run,
        "speedup_vs_serial_fp64_run": None if serial_run is None else round(serial_run["makespan_s"] / makespan, 3),
    }
    print(json.dumps(res))


def combined_filter_taps(case, x, t_start):
    """Taps of each panel's combined filter: the spread over the spanwise copies of the
    first sample of their stencils, plus 8 (phase radius of the moving medium, Appendix B)."""
    M = np.asarray(case["mach"], dtype=np.float64)
    g2 = 1.0 / (1.0 - M @ M)
    k = np.arange(case["n_copies"]) - (case["n_copies"] - 1) / 2.0
    y = case["points"][None, :, :] + k[:, None, None] * np.asarray(case["copy_shift"])[None, None, :]
    r = np.asarray(x)[None, None, :] - y
    Mr = r @ M
    Rs = np.sqrt((r * r).sum(-1) + g2 * Mr ** 2) / np.sqrt(g2)
    R = g2 * (Rs - Mr)
    first = np.floor((t_start - R / case["c0"]) / case["dt"] - 2.0)
    return first.max(axis=0) - first.min(axis=0) + 8.0


def oracle_one_thread(workload, steps=1):
    """The oracle's DOF-updates/s on one host thread: a child process (no GPU use) with
    OMP_NUM_THREADS=1 runs `steps` RK4 steps of the workload's mesh."""
    import subprocess
    code = ("import sys, time, json; sys.path.insert(0, %r); import bench; "
            "from oracle.oracle import OracleMesh, num_threads; import numpy as np; "
            "m, desc = bench.build_workload(%r); o = OracleMesh(m); "
            "u0 = np.ascontiguousarray(m['init'](o.solution_points().reshape(-1, 3)).reshape(o.shape)); "
            "t0 = time.perf_counter(); o.rk4(u0, m['dt'], %d); t = time.perf_counter() - t0; "
            "print(json.dumps({'value': o.E * o.nu * o.nv * %d / t, 'threads': num_threads(), 's': t}))"
            % (ROOT, workload, steps, steps))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        d = json.loads(r.stdout.strip().splitlines()[-1])
        return {"value": d["value"], "cores": d["threads"],
                "sample": f"{steps} RK4 step of the full mesh on one thread, {d['s']:.1f} s"}
    except Exception as e:  # reported, not fatal: the GPU figures stand on their own
        return {"value": None, "error": str(e)[:200]}


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs"


def measured_ceilings():
    """Streaming and matrix ceilings measured on this GPU, reported beside the published
    peaks the rooflines use: a 1 GiB device-to-device copy (read + write bytes over time)
    and FP32 / FP64 library GEMMs (2 n^3 flops over time), each the mean of 10 after 3
    warm-up runs, timed with events on torch's stream."""
    import torch

    def timed(fn, reps=10):
        for _ in range(3):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3
    n = 2 ** 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t_copy = timed(lambda: dst.copy_(src))
    del src, dst
    out = {"copy_gbs": round(2 * n * 4 / t_copy / 1e9, 1)}
    for name, dt, k in (("sgemm_tflops", torch.float32, 8192), ("dgemm_tflops", torch.float64, 4096)):
        a = torch.rand(k, k, dtype=dt, device="cuda")
        b = torch.rand(k, k, dtype=dt, device="cuda")
        t = timed(lambda: torch.matmul(a, b))
        out[name] = round(2.0 * k ** 3 / t / 1e12, 1)
        del a, b
    torch.cuda.empty_cache()
    out["note"] = ("measured beside the published peaks (HBM 8 TB/s, FP32 157.3 and FP64 78.6 TFLOP/s), "
                   "which the rooflines use")
    return out


def bench_fwh(args):
    """Far-field pressure at the paper's observer from its airfoil data surface (24,000
    panels, 4,332 samples, 125 spanwise copies filling 25 chords)."""
    from paper_2501_05709_amd import workloads as W
    from paper_2501_05709_amd.solver import FWH
    case = W.fwh_airfoil_case(seed=0)
    n = case["n_copies"]
    g = FWH(case["points"], case["normals"], case["areas"], case["mach"], case["c0"], case["rho0"], case["p0"],
            case["dt"], case["n_samples"], n_copies=n, copy_shift=case["copy_shift"])
    t_app = 0.0
    for rho, u, p in W.fwh_airfoil_samples(case):
        t0 = time.perf_counter()
        g.append(rho, u, p)
        t_app += time.perf_counter() - t0
    x = case["observer"]
    for _ in range(max(args.warmup, 1)):
        t, p = g.pressure(x)
    ms = []
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        t, p = g.pressure(x)
        ms.append(g.time_ms())
    wall = (time.perf_counter() - wall0) / args.steps
    npan = case["points"].shape[0]
    work = float(n) * npan * t.size                      # (copy, panel, observer time) triples
    k_ms = float(np.mean(ms))
    # each panel's copies are summed through one filter of (delay spread + 8) taps per source
    # series: 2 x 4 series x taps flops per (panel, observer time), priced against the time
    # of the whole evaluation (forming the filters, applying them, the chunk reductions)
    taps = combined_filter_taps(case, x, t[0])
    flops = 8.0 * float(taps.sum()) * t.size
    # oracle on a bounded sample: one copy of one spanwise row of panels, all samples
    row = slice(0, 1200)
    sub = FWH(case["points"][row], case["normals"][row], case["areas"][row], case["mach"], case["c0"],
              case["rho0"], case["p0"], case["dt"], case["n_samples"])
    rows = []
    for rho, u, pp in W.fwh_airfoil_samples(case):
        sub.append(rho[:, row], u[:, row], pp[:, row])
        rows.append((rho[:, row], u[:, row], pp[:, row]))
    rho = np.concatenate([r[0] for r in rows])
    u = np.concatenate([r[1] for r in rows])
    pp = np.concatenate([r[2] for r in rows])
    ts, ps = sub.pressure(x)
    cpu = err = None
    if not args.no_cpu_baseline:
        from oracle import fwh as ofwh
        t0 = time.perf_counter()
        to, po, _, _ = ofwh.observer_pressure(case["points"][row], case["normals"][row], case["areas"][row], rho, u,
                                              pp, case["dt"], x, case["mach"], case["c0"], case["rho0"], case["p0"])
        tc = time.perf_counter() - t0
        err = float(np.abs(ps - po).max() / np.abs(po).max())
        cpu = {"value": 1200.0 * to.size / tc, "unit": "panel-samples/s", "cores": 1, "kind": "oracle",
               "sample": f"one copy of one spanwise row (1,200 panels), all {case['n_samples']} samples, "
                         f"numpy FP64, {tc:.1f} s"}
    res = {
        "metric": "FW-H far-field pressure: (copy, panel, observer-time) triples per second",
        "value": round(work / (k_ms * 1e-3), 1), "unit": "panel-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(k_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"airfoil data surface {npan} panels x {n} spanwise copies (25 chords), "
                               f"{case['n_samples']} samples, one observer 10 chords below the trailing edge",
                   "observer_times": int(t.size)},
        "wall_ms_per_step": round(wall * 1e3, 3), "append_s": round(t_app, 3),
        "roofline": {"bound": "alu", "achieved": round(flops / (k_ms * 1e-3) / 1e12, 2), "peak": PEAK["fp64"],
                     "unit": "TFLOP/s", "frac": round(flops / (k_ms * 1e-3) / 1e12 / PEAK["fp64"], 4),
                     "kernel": "one evaluation: k_fwh_filter + k_fwh_sum + reductions", "traffic": None,
                     "flops": "8 x (copies' delay spread + 8) per panel and observer time",
                     "mean_taps_per_panel": round(float(taps.mean()), 1),
                     "copy_by_copy_equivalent_tflops": round(64.0 * work / (k_ms * 1e-3) / 1e12, 2)},
        "rel_err_vs_oracle_row": err,
        "p_rms": float(np.sqrt(np.mean((p - p.mean()) ** 2))),
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


def bench_pmix(args):
    """Variable order on the airfoil O-grid (Section 3.1): P3 in the 12 wall layers, then
    P2, P1 and P0 in bands of 12 layers of the 160 x 48 x 8 grid, the paper's
    low-resolution P0-P3 distribution lowering the order toward the far field; timed
    against the same grid at P3 everywhere."""
    import torch
    from paper_2501_05709_amd import workloads as W
    from paper_2501_05709_amd.solver import FRMesh
    ni, nj, nk = 160, 48, 8
    m = W.config_airfoil(0, ni=ni, nj=nj, nk=nk, order=3)
    m["orders"] = W.ring_orders(ni, nj, nk, ((12, 3), (24, 2), (36, 1), (48, 0)))
    desc = {"workload": "naca4_ogrid_160x48x8_quadratic_hex_p3_to_p0_rings", "elements": ni * nj * nk,
            "orders": "P3 layers 0-11, P2 12-23, P1 24-35, P0 36-47", "reynolds": 23000, "mach": 0.2,
            "aoa_deg": 5.0,
            "dt": m["dt"], "mesh": "curved quadratic hexes, wall + far field + spanwise periodic"}
    g32 = FRMesh(m, "fp32")
    xyz = g32.solution_points()
    u0 = np.ascontiguousarray(m["init"](xyz))
    dof = g32.n_points * g32.nv
    cpu = ref = err32_oracle = err64_oracle = None
    n_sample = args.cpu_steps or 3
    if not args.no_cpu_baseline:
        from oracle.oracle import OracleMesh, num_threads
        o = OracleMesh(m)
        o.rk4(u0, m["dt"], 1)
        t0 = time.perf_counter()
        ref = o.rk4(u0, m["dt"], n_sample)
        tc = time.perf_counter() - t0
        cpu = {"value": dof * n_sample / tc, "unit": "DOF-updates/s", "cores": num_threads(), "kind": "oracle",
               "sample": f"{n_sample} RK4 steps of the full {desc['workload']} mesh, FP64, OpenMP over elements, "
                         f"{tc:.1f} s wall on {num_threads()} threads ({tc * num_threads():.0f} thread-s)"}
    g64 = FRMesh(m, "fp64")
    if ref is not None:
        for g in (g64, g32):
            g.set_state(u0)
            g.step(n_sample)
        err64_oracle = rel_l2(g64.get_state(), ref)
        err32_oracle = rel_l2(g32.get_state(), ref)
    t64 = timed_run(g64, u0, args.steps, args.warmup)
    t32 = timed_run(g32, u0, args.steps, args.warmup)
    err32_vs64 = rel_l2(g32.get_state(), g64.get_state())
    # the same grid at P3 everywhere, in its fastest form: fused stage with the column
    # metrics (the order groups' mortar build reads stored metrics)
    m3 = dict(m)
    m3.pop("orders")
    g3 = FRMesh(m3, "fp32")
    g3.select_kernels(1 | (1 << 5) | (1 << 8))
    u3 = np.ascontiguousarray(m3["init"](g3.solution_points().reshape(-1, 3)).reshape(g3.shape))
    t3 = timed_run(g3, u3, args.steps, args.warmup)
    dof3 = g3.E * g3.nu * g3.nv
    # step roofline: the method's algorithmic bytes per curved element and stage at each
    # element's order, four stages, over the measured step time (the mortar points' table
    # entries and partner values are not counted)
    orders, counts = np.unique(m["orders"], return_counts=True)
    step_bytes = 0.0
    for p, c in zip(orders, counts):
        step_bytes += 4 * c * algorithmic_bytes_per_element_stage(3, int(p), 4, True)
    achieved = step_bytes / (t32 / args.steps) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm"], "unit": "GB/s",
            "frac": round(achieved / PEAK["hbm"], 4), "kernel": "whole step (all order groups)", "traffic": None}
    out = {
        "metric": "FR DOF-updates/s (FP32 form; FP64 beside it) at stated L2 error vs the FP64 oracle",
        "value": round(dof * args.steps / t32, 1), "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t32 / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(desc, form="fp32 operators/fluxes/state, fp64 metrics and force sums", dof=dof,
                       parallelism="single GPU"),
        "fp64": {"value": round(dof * args.steps / t64, 1), "ms_per_step": round(t64 / args.steps * 1e3, 4),
                 "rel_l2_vs_oracle": err64_oracle},
        "fp32_rel_l2_vs_oracle": err32_oracle, "fp32_rel_l2_vs_fp64_gpu": err32_vs64,
        "oracle_sample_steps": n_sample if ref is not None else None,
        "uniform_p3_same_grid": {"value": round(dof3 * args.steps / t3, 1), "dof": dof3,
                                 "ms_per_step": round(t3 / args.steps * 1e3, 4)},
        "step_time_vs_uniform_p3": round(t32 / t3, 3),
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def bench_pmix_batch(args):
    """Variable order in a batch: the sixteen designs of the default batch, each with the
    paper's low-resolution P-distribution on its own O-grid (P3 in the inner quarter of
    its radial layers, then P2, P1 and P0 outward), advanced together: every order group
    covers that order's elements of all designs."""
    from paper_2501_05709_amd import workloads as W
    from paper_2501_05709_amd.solver import FRMesh
    meshes = W.config_batch(0)
    designs = []
    for m in meshes:
        ni, nj, nk = m["grid"]
        q = max(1, nj // 4)
        m = dict(m, orders=W.ring_orders(ni, nj, nk, ((q, 3), (2 * q, 2), (3 * q, 1), (nj, 0))))
        designs.append(m)
    out = {}
    for prec in ("fp32", "fp64"):
        b = FRMesh(designs, prec)
        u0 = np.concatenate([W.uniform_state(int(((np.asarray(m["orders"]) + 1) ** 3).sum()), m["freestream"][0],
                                             m["freestream"][1:4], m["freestream"][4]) for m in designs])
        dof = b.n_points * b.nv
        b.set_state(u0)
        if args.warmup:
            b.step(args.warmup)
        rate, med = median_rate(dof, windows(b, args.steps))
        out[prec] = {"value": rate, "ms_per_step": med * 1e3, "dof": dof}
        b.close()
        del b
        torch_empty()
    res = {
        "metric": "FR DOF-updates/s, variable-order batch of 16 airfoil designs (FP32 form; FP64 beside it)",
        "value": round(out["fp32"]["value"], 1), "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(out["fp32"]["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16 NACA 4-digit O-grids of the default batch, each with P3/P2/P1/P0 rings by "
                               "quarters of its radial layers, seed 0", "dof": out["fp32"]["dof"],
                   "elements": int(sum(len(m["elem_nodes"]) for m in designs))},
        "fp64": {"value": round(out["fp64"]["value"], 1), "ms_per_step": round(out["fp64"]["ms_per_step"], 4)},
        "speedup_fp32_over_fp64": round(out["fp32"]["value"] / out["fp64"]["value"], 3),
    }
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "tgv", "airfoil", "serve", "fwh", "pmix", "pmix_batch"])
    ap.add_argument("--solves", type=int, default=5, help="batch: repeated batched solves for p50/p99 latency")
    ap.add_argument("--solve-steps", type=int, default=200, help="batch: RK4 steps of one batched solve")
    ap.add_argument("--no-extras", action="store_true", help="batch: skip the single-mesh workloads")
    ap.add_argument("--full-parity", action="store_true",
                    help="batch: the oracle also on one design drawn at random (minutes on the host), not only "
                         "on the smallest")
    ap.add_argument("--requests", type=int, default=64, help="serve: requests in the trace")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: mean arrivals per second")
    ap.add_argument("--budget-gb", type=float, default=96.0, help="serve: HBM budget of the pool")
    ap.add_argument("--serial-run", action="store_true",
                    help="serve: also run the same trace FIFO one request at a time on the plain FP64 path")
    ap.add_argument("--active-elements", type=int, default=150000,
                    help="serve: admit while the running requests hold fewer elements than this")
    ap.add_argument("--cpu-steps", type=int, default=None, help="oracle sample (steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device to device (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: every workload here runs on a single GPU, and "
              "there is no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        src = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "fwh":
        return bench_fwh(args)
    if args.workload == "pmix":
        return bench_pmix(args)
    if args.workload == "pmix_batch":
        return bench_pmix_batch(args)
    return bench_single(args)


def bench_single(args):
    """One mesh (Taylor-Green 24^3 or the 160x48x8 airfoil O-grid)."""
    from paper_2501_05709_amd.solver import FRMesh
    m, desc = build_workload(args.workload)
    g32 = FRMesh(m, "fp32")
    xyz = g32.solution_points().reshape(-1, 3)
    u0 = np.ascontiguousarray(m["init"](xyz).reshape(g32.shape))
    dof = g32.E * g32.nu * g32.nv

    # --- CPU baseline (oracle, FP64) on a bounded sample, and the parity sample
    cpu = None
    n_sample = args.cpu_steps or (10 if args.workload == "tgv" else 3)
    ref_sample = None
    if not args.no_cpu_baseline:
        from oracle.oracle import OracleMesh, num_threads
        o = OracleMesh(m)
        o.rk4(u0, m["dt"], 1)  # warm the host caches
        t0 = time.perf_counter()
        ref_sample = o.rk4(u0, m["dt"], n_sample)
        tc = time.perf_counter() - t0
        cpu = {"value": dof * n_sample / tc, "unit": "DOF-updates/s", "cores": num_threads(),
               "kind": "oracle", "host": host_cpu(), "one_thread": oracle_one_thread(args.workload),
               "sample": f"{n_sample} RK4 steps of the full {desc['workload']} mesh, FP64, "
                         f"OpenMP over elements, {tc:.1f} s wall on {num_threads()} threads "
                         f"({tc * num_threads():.0f} thread-s)"}

    # --- autotune the operator back-end of every kernel (dense MFMA vs sum factorised)
    g32.set_state(u0)
    mask32 = g32.autotune(3)
    g64 = FRMesh(m, "fp64")
    g64.set_state(u0)
    mask64 = g64.autotune(3)

    # --- plain FP64 GPU path
    err64_oracle = err32_oracle = None
    ek = None
    if ref_sample is not None:
        g64.set_state(u0)
        g64.step(n_sample)
        s64 = g64.get_state()
        err64_oracle = rel_l2(s64, ref_sample)
        g32.set_state(u0)
        g32.step(n_sample)
        s32 = g32.get_state()
        err32_oracle = rel_l2(s32, ref_sample)
        if args.workload == "tgv":
            k0, ko = kinetic_energy(u0, 3), kinetic_energy(ref_sample, 3)
            ek = {"E_k_0": k0, "steps": n_sample, "E_k_oracle": ko,
                  "E_k_fp64": kinetic_energy(s64, 3), "E_k_fp32": kinetic_energy(s32, 3),
                  "decay_rel_err_fp64": abs((k0 - kinetic_energy(s64, 3)) - (k0 - ko)) / (k0 - ko),
                  "decay_rel_err_fp32": abs((k0 - kinetic_energy(s32, 3)) - (k0 - ko)) / (k0 - ko)}
    t64 = timed_run(g64, u0, args.steps, args.warmup)
    u64 = g64.get_state()

    # --- FP32 form (the reported value)
    t32 = timed_run(g32, u0, args.steps, args.warmup)
    u32 = g32.get_state()
    err32_vs64 = rel_l2(u32, u64)
    if ek is not None:
        ek["after_timed_run"] = {"steps": args.warmup + args.steps, "E_k_fp64": kinetic_energy(u64, 3),
                                 "E_k_fp32": kinetic_energy(u32, 3)}

    # --- the all-dense-MFMA operator back-end, for comparison
    g32.select_kernels(0)
    t32_dense = timed_run(g32, u0, args.steps, args.warmup)
    g64.select_kernels(0)
    t64_dense = timed_run(g64, u0, args.steps, args.warmup)
    g32.select_kernels(mask32)

    # --- per-kernel times (HIP events on the solver's stream) and roofline
    g32.set_state(u0)
    ms, nl = g32.profile_kernels(5)
    cost, dof_per_elem = per_element_cost(g32.dim, g32.order, 4, metric_source(mask32))
    kernels = {}
    fused = bool(mask32 & 1)
    for k in ((6, 7) if fused else range(1, 6)):
        if k >= 6:
            variant = "fused, sum-factorised"
        else:
            variant = "face" if k == 1 else ("sum-factorised" if (mask32 >> k) & 1 else "dense-mfma")
        avg_ms = ms[k] / max(nl[k], 1)
        fl = cost[k]["flops"] * g32.E
        by = cost[k]["bytes"] * g32.E
        kernels[KERNEL_NAMES[k]] = {
            "variant": variant, "avg_us": round(avg_ms * 1e3, 2), "share": round(ms[k] / ms[0], 3),
            "dense_equiv_tflops": round(fl / (avg_ms * 1e-3) / 1e12, 2) if fl else 0.0,
            "implementation_gbs": round(by / (avg_ms * 1e-3) / 1e9, 1)}
    # the same table for the all-dense-MFMA back-end (MFMA utilisation evidence)
    g32.select_kernels(0)
    g32.set_state(u0)
    msd, nld = g32.profile_kernels(5)
    g32.select_kernels(mask32)
    dense_kernels = {}
    for k in range(2, 6):
        avg_ms = msd[k] / max(nld[k], 1)
        fl = cost[k]["flops"] * g32.E
        dense_kernels[KERNEL_NAMES[k]] = {
            "avg_us": round(avg_ms * 1e3, 2), "tflops": round(fl / (avg_ms * 1e-3) / 1e12, 2),
            "mfma_frac": round(fl / (avg_ms * 1e-3) / 1e12 / PEAK["mfma_f32"], 4)}
    if fused:
        # the fused stage: algorithmic bytes of one RK stage over both launches' time
        g32.set_state(u0)
        roof, _, _ = stage_roofline(g32, g32.dim, g32.order, 4, args.workload != "tgv", args.workload)
    else:
        dom = max(range(1, 8), key=lambda k: ms[k])
        avg_s = ms[dom] / nl[dom] * 1e-3
        if dom in (2, 3, 4, 5) and not (mask32 >> dom) & 1:
            achieved = cost[dom]["flops"] * g32.E / avg_s / 1e12
            roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["mfma_f32"], "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK["mfma_f32"], 4)}
        else:
            achieved = cost[dom]["bytes"] * g32.E / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm"], "unit": "GB/s",
                    "frac": round(achieved / PEAK["hbm"], 4), "bytes": "implementation bytes of the kernel"}
        roof["kernel"] = KERNEL_NAMES[dom]
        roof["traffic"] = None

    value = dof * args.steps / t32
    out = {
        "metric": "FR DOF-updates/s (FP32 form; FP64 beside it) at stated L2 error vs the FP64 oracle",
        "value": round(value, 1),
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t32 / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(desc, form="fp32 operators/fluxes/state, fp64 metrics and force sums",
                       dof=dof, parallelism="single GPU"),
        "fp64": {"value": round(dof * args.steps / t64, 1), "ms_per_step": round(t64 / args.steps * 1e3, 4),
                 "rel_l2_vs_oracle": err64_oracle},
        "fp32_rel_l2_vs_oracle": err32_oracle,
        "fp32_rel_l2_vs_fp64_gpu": err32_vs64,
        "oracle_sample_steps": n_sample if ref_sample is not None else None,
        "kinetic_energy": ek,
        "speedup_fp32_over_fp64": round(t64 / t32, 3),
        "kernel_variants": {"fp32_mask": mask32, "fp64_mask": mask64,
                            "note": "bit 0: fused two-launch stage (sum-factorised); else bit k set: "
                                    "split kernel k sum-factorised, clear: dense MFMA "
                                    "(2 grad, 3 visc, 4 divrk, 5 interp)"},
        "dense_mfma_only": {"fp32_value": round(dof * args.steps / t32_dense, 1),
                            "fp64_value": round(dof * args.steps / t64_dense, 1)},
        "kernels": kernels,
        "roofline": roof,
        "measured_ceilings": measured_ceilings(),
        "dense_mfma_kernels_fp32": dense_kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""FR DOF-updates/s on one MI355X: FP32 form vs plain FP64, with L2 errors.

Workload (default): Taylor-Green vortex on the periodic [0, 2 pi]^3 cube of
24^3 straight hexahedra, p = 3 (64 solution points per element), Re 1600,
Mach 0.1, RK4 with dt = 1e-3.  A "step" is one full RK4 step (four FR
residual evaluations and the fused stage updates) of the whole mesh; the
state is resident in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--workload tgv|airfoil]

Prints one JSON line.  ``value`` is FP32-form DOF-updates/s (DOF = elements x
solution points x conserved variables, one update = one RK4 step); the plain
FP64 path, the errors against the FP64 oracle after a short sample and
against the FP64 GPU path after the timed run, the per-kernel times and the
roofline of the dominant kernel are reported beside it.  The CPU baseline is
the FP64 oracle timed on this host's cores on a bounded sample of steps.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm": 8000.0, "mfma_f32": 157.3, "mfma_f64": 78.6}  # GB/s, TFLOP/s
KERNEL_NAMES = {1: "k_face", 2: "k_grad", 3: "k_visc", 4: "k_divrk", 5: "k_interp", 6: "k_stage_a",
                7: "k_stage_b"}


def per_element_cost(dim, order, real_bytes):
    """Algorithmic dense-MFMA flops and HBM bytes of each kernel, per element and launch.

    Operator sizes are the unpadded FR matrices (n_u solution points, n_f flux
    points); metric terms are FP64 (8 bytes), neighbour indices 4 bytes.
    """
    n = order + 1
    nu = n ** dim
    nf = 2 * dim * n ** (dim - 1)
    nv = dim + 2
    s = real_bytes
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
        # fused stage a: stage state, partner traces, normals, neighbour codes, S and 1/|J|
        # in; Q, P and the volume divergence out
        6: dict(flops=0, bytes=nu * nv * s + nf * nv * s + nf * dim * 8 + nf * 4 + nu * (dim * dim + 1) * 8
                + 2 * nf * nv * s + nu * nv * s),
        # fused stage b: Q, partner P, codes, areas, divergence, 1/|J|, u_n, acc in; acc,
        # next stage state and its trace out
        7: dict(flops=0, bytes=2 * nf * nv * s + nf * 4 + nf * 8 + nu * nv * s + nu * 8 + 2 * nu * nv * s
                + 2 * nu * nv * s + nf * nv * s),
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


def counters_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None if it is missing or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2501_05709_amd", "csrc", "fr_kernels.hip"), "rb").read()
        sha = hashlib.sha256(src).hexdigest()
        entry = data.get(workload, {}).get(kernel)
        if not entry or entry.get("source_sha256") != sha:
            return None
        return entry.get("hbm_bytes_per_launch")
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tgv", choices=["tgv", "airfoil"])
    ap.add_argument("--cpu-steps", type=int, default=None, help="oracle sample (steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
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
               "kind": "oracle",
               "sample": f"{n_sample} RK4 steps of the full {desc['workload']} mesh, FP64, "
                         f"OpenMP over elements, {tc:.1f} s"}

    # --- autotune the operator back-end of every kernel (dense MFMA vs sum factorised)
    g32.set_state(u0)
    mask32 = g32.autotune(3)
    g64 = FRMesh(m, "fp64")
    g64.set_state(u0)
    mask64 = g64.autotune(3)

    # --- plain FP64 GPU path
    err64_oracle = err32_oracle = None
    if ref_sample is not None:
        g64.set_state(u0)
        g64.step(n_sample)
        err64_oracle = rel_l2(g64.get_state(), ref_sample)
        g32.set_state(u0)
        g32.step(n_sample)
        err32_oracle = rel_l2(g32.get_state(), ref_sample)
    t64 = timed_run(g64, u0, args.steps, args.warmup)
    u64 = g64.get_state()

    # --- FP32 form (the reported value)
    t32 = timed_run(g32, u0, args.steps, args.warmup)
    u32 = g32.get_state()
    err32_vs64 = rel_l2(u32, u64)

    # --- the all-dense-MFMA operator back-end, for comparison
    g32.select_kernels(0)
    t32_dense = timed_run(g32, u0, args.steps, args.warmup)
    g64.select_kernels(0)
    t64_dense = timed_run(g64, u0, args.steps, args.warmup)
    g32.select_kernels(mask32)

    # --- per-kernel times (HIP events on the solver's stream) and roofline
    g32.set_state(u0)
    ms, nl = g32.profile_kernels(5)
    cost, dof_per_elem = per_element_cost(g32.dim, g32.order, 4)
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
            "gbs": round(by / (avg_ms * 1e-3) / 1e9, 1)}
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
    dom = max(range(1, 8), key=lambda k: ms[k])
    avg_s = ms[dom] / nl[dom] * 1e-3
    dom_dense = dom in (2, 3, 4, 5) and not (mask32 >> dom) & 1
    if dom_dense:
        achieved = cost[dom]["flops"] * g32.E / avg_s / 1e12
        peak = PEAK["mfma_f32"]
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4)}
    else:
        achieved = cost[dom]["bytes"] * g32.E / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm"], "unit": "GB/s",
                "frac": round(achieved / PEAK["hbm"], 4)}
    roof["kernel"] = KERNEL_NAMES[dom]
    roof["traffic"] = counters_traffic(args.workload, KERNEL_NAMES[dom])

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
        "speedup_fp32_over_fp64": round(t64 / t32, 3),
        "kernel_variants": {"fp32_mask": mask32, "fp64_mask": mask64,
                            "note": "bit 0: fused two-launch stage (sum-factorised); else bit k set: "
                                    "split kernel k sum-factorised, clear: dense MFMA "
                                    "(2 grad, 3 visc, 4 divrk, 5 interp)"},
        "dense_mfma_only": {"fp32_value": round(dof * args.steps / t32_dense, 1),
                            "fp64_value": round(dof * args.steps / t64_dense, 1)},
        "kernels": kernels,
        "roofline": roof,
        "dense_mfma_kernels_fp32": dense_kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the Total Lagrangian internal-force hot path on one MI355X.

Workload (one "step"): the forward internal force f_int(x, v) plus its adjoint
(gx, gv) = (df/dx)^T w, (df/dv)^T w on a 1,020,000-element T10 box
(100 x 100 x 17 cells of 1 cm, 6 tetrahedra per cell, 1,414,035 nodes,
5-point rule -> 5,100,000 quadrature points), compressible Neo-Hookean
(mu10 = 1.7 MPa, k = 17.27 MPa) plus Kelvin-Voigt damping (mu_v = 1e4 Pa s),
state = random rigid rotation of the reference plus a 2 % smooth sinusoidal
deformation, velocities N(0, 0.01 m/s), cotangent w ~ N(0, 1).  Inputs are
resident in HBM before timing.  value = quadrature points per second of the
whole step.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk


# ---------------------------------------------------------------- cost model
# Algorithmic arithmetic per quadrature point of the fused per-point
# formulation (F = (N dS/dxi) J^{-1}, parent gradients with their structural
# zeros removed, multiply-add = 2 flops, divide and cube root = 1 each).
# nz = non-zero entries of the parent gradient table at the point (T10 5-point
# rule: 12, 21, 20, 20, 19; H8 2x2x2 Gauss: 24 at every point).
NZ = {0: [12, 21, 20, 20, 19], 1: [24] * 8}
STRESS = {0: 129, 1: 269, 2: 96}          # SVK, MR, NH elastic stress
VISC_FWD = {0: 84, 1: 138, 2: 138}        # Kelvin-Voigt add-on (SVK folds S_v into S)
DSTRESS = {0: 240, 1: 520, 2: 283}        # elastic directional derivative incl. shared invariants
GTHETA = {0: 40, 1: 60, 2: 43}


def flops_per_element(op, elem, law, damped):
    nz = NZ[elem]
    per_elem = 6 * nz[0] + 43             # J = U G at one point and its inverse (affine map)
    tot = 0
    for z in nz:
        g = 6 * z                          # one gathered field -> 3x3 (3 z multiply-adds)
        if op == "fwd":
            q = 2 * g if damped else g     # x (and v)
            q += 54 * (2 if damped else 1) # times J^{-1}
            q += STRESS[law] + (VISC_FWD[law] if damped else 0)
            q += 63 + g                    # c P J^{-T} and scatter to nodes
        elif op == "vjp":
            q = (3 if damped else 2) * (g + 54)   # x, w (, v) -> 3x3
            q += DSTRESS[law] + GTHETA[law]
            q += 63 + g                           # gx
            if damped:
                q += 354 + 63 + g                 # viscous adjoint and gv
        else:  # jvp
            q = (4 if damped else 2) * (g + 54)   # x, dx (, v, dv)
            q += DSTRESS[law] + (250 if damped else 0) + 63 + g
        tot += q
    return per_elem + tot


def bytes_per_call(op, n_nodes, n_elem, nen, damped, theta_rows=0, gtheta=False):
    """Compulsory HBM traffic: every nodal array read once, outputs written
    once, connectivity as int32 read once, optional per-element parameters."""
    node = 24.0 * n_nodes
    if op == "fwd":
        arrays = 3 + (1 if damped else 0)            # X, x, (v), f
    elif op == "vjp":
        arrays = 4 + (2 if damped else 0)            # X, x, w, gx (, v, gv)
    else:
        arrays = 4 + (2 if damped else 0)            # X, x, dx, df (, v, dv)
    b = arrays * node + 4.0 * nen * n_elem + 8.0 * theta_rows * n_elem
    if gtheta:
        b += 40.0 * n_elem
    return b


# ---------------------------------------------------------------- helpers

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(prob, budget_s=15.0):
    """The oracle as it is (serial C, one core) on a bounded sample of the
    same workload: the first elements of the mesh, forward + adjoint."""
    import copy

    import oracle as O
    b = prob.blocks[0]

    def run(ne):
        sb = copy.copy(b)
        sb.conn = np.ascontiguousarray(b.conn[:ne])
        t0 = time.perf_counter()
        O.internal_force(prob.X, [sb], prob.x, prob.v)
        O.vjp(prob.X, [sb], prob.x, prob.v, prob.w, want_gtheta=False)
        return time.perf_counter() - t0

    t_small = run(500)
    ne = int(min(b.n_elem, max(500, 500 * budget_s / max(t_small, 1e-6))))
    t = run(ne)
    nq = ne * 5
    return {"value": nq / t, "unit": "quad-pts/s", "cores": 1, "kind": "oracle",
            "sample": f"forward + adjoint (gx, gv) of the first {ne} of {b.n_elem} elements "
                      f"({nq} quadrature points), serial C oracle, {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="elements per tile (0 = library default)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, used to scale the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2602_17002_amd import Mesh

    t0 = time.time()
    prob = synth.config_c2()
    log(f"[bench] C2 synthesized: {prob.n_elem} elements, {prob.n_nodes} nodes, {time.time() - t0:.1f} s")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    mesh = Mesh.from_problem(prob, tile_elems=args.tile or None)
    info = mesh.info()
    log(f"[bench] mesh built in {time.time() - t0:.1f} s: {info}")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        x = torch.from_numpy(prob.x).to(dev)
        v = torch.from_numpy(prob.v).to(dev)
        w = torch.from_numpy(prob.w).to(dev)
        f = torch.empty_like(x)
        gx = torch.empty_like(x)
        gv = torch.empty_like(x)

        if args.copy_calib_mb:
            n = args.copy_calib_mb * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            log(f"[bench] calibration copy of {args.copy_calib_mb} MiB done")
            del src, dst

        def step():
            mesh.internal_force(x, v, out=f)
            mesh.vjp(x, v, w, want_theta=False, out=(gx, gv, None))

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        mesh.reset_profile()
        mesh.set_profiling(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        mesh.set_profiling(False)
        ms_total = e0.elapsed_time(e1)
        prof = mesh.profile()
    log(f"[bench] timed {args.steps} steps: {ms_total:.3f} ms; kernels {prof}")
    ms_step = ms_total / args.steps
    n_qp = prob.n_qp
    value = n_qp / (ms_step * 1e-3)

    # roofline of the dominant kernel
    k_ms = {k: (c, t / c if c else 0.0) for k, (c, t) in prof.items()}
    dom = max(("forward_tile", "adjoint_tile"), key=lambda k: k_ms[k][1])
    op = "fwd" if dom == "forward_tile" else "vjp"
    ne, nn = prob.n_elem, prob.n_nodes
    flops = flops_per_element(op, synth.T10, synth.NH, True) * ne
    t_dom = k_ms[dom][1] * 1e-3
    achieved = flops / t_dom / 1e12
    byts = bytes_per_call(op, nn, ne, 10, True)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "kernel": dom, "kernel_ms": round(k_ms[dom][1], 4),
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": byts,
            "hbm_frac": round(byts / t_dom / 1e9 / HBM_PEAK_GBS, 4)}

    out = {
        "metric": "quad-pts/s f_int fwd+VJP (1M T10 NH), batched vs plain; % HBM/FP64 peak",
        "value": value, "unit": "quad-pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "C2: 1,020,000 T10 box 100x100x17 cells, Neo-Hookean + Kelvin-Voigt, "
                               "forward + adjoint (gx, gv)", "elements": ne, "nodes": nn, "quad_points": n_qp,
                   "tile_elems": info["tile_elems_t10"]},
        "kernels_ms_avg": {k: round(t, 4) for k, (c, t) in k_ms.items() if c},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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

ms_per_step is the median over the timed steps, each between its own pair of
HIP events on the stream.

The line also carries: the 204,000-element per-element-parameter body's
adjoint with parameter gradients and tangent (skip with --no-c4); the
131,072-element Q27 body's forward, adjoint and tangent (skip with --no-q27); the
multibody comparison (skip with --no-batched): 512 bodies of 200-50,000
elements (mixed T10 / H8, SVK / Neo-Hookean), forward internal force of
every body, timed as one batched mesh (one hipGraph replay) against one plain
mesh per body launched back to back on one stream, eagerly and captured into
one graph; and the 256-body forward + adjoint + tangent graph (skip with
--no-c5).

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.

--pmc-summary DIR writes the rocprofv3 summaries under profiles/ from the
output folders of a kernel-trace run and two counter runs; --sq-summary
writes the SQ counter summary from counter runs of the same command.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
CSRC = os.path.join(ROOT, "paper_2602_17002_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "hbm_traffic_c2_fwd_vjp.md")

T10, H8 = 0, 1
SVK, MR, NH = 0, 1, 2

# ---------------------------------------------------------------- cost model
# Arithmetic of the method per quadrature point, counted from the formulas
# the kernels evaluate (one flop per multiply or add, a fused multiply-add
# counts two; divide and cube root count one; symmetric results count their
# six distinct entries).  nz = non-zero entries of the parent gradient table
# at the point (T10 5-point rule: 12, 21, 20, 20, 19; H8 2x2x2 Gauss: 24).
# A gathered field costs 6 nz (G = sum_a s_a g_a^T), the scatter 6 nz.
NZ = {T10: [12, 21, 20, 20, 19], H8: [24] * 8}
Q27 = 2


def _q27_nz():
    """Non-zero parent-gradient entries at each 3x3x3 Gauss point of Q27: at
    a coordinate 0 only L_1 (value) and L_0', L_2' (derivative) are non-zero
    along that direction, elsewhere all three of each."""
    out = []
    for q in range(27):
        zero = [(q // 3 ** d) % 3 == 1 for d in range(3)]
        nz = 0
        for k in range(3):
            c = 1
            for d in range(3):
                c *= (2 if d == k else 1) if zero[d] else 3
            nz += c
        out.append(nz)
    return out


NZ[Q27] = _q27_nz()
GEOM = 33            # cofactor of J (27) + det (5) + reciprocal (1)
TOREF = 54           # A = (G cof(J)^T) / det J for one field
TOPAR = 54           # Q = w_q P cof(J)
# elastic stress (forward): SVK C, tr E, S, F S; MR/NH invariants, cof F, J, J^-2/3, ...
STRESS = {SVK: 98, MR: 241, NH: 97}
# Kelvin-Voigt add-on of the forward: Edot = sym(F^T Fdot) (57), S_v (14),
# F S_v (45) and the add (9); SVK adds S_v to S instead (57 + 14 + 6)
VISC_FWD = {SVK: 77, MR: 125, NH: 125}
# elastic directional derivative (adjoint and tangent), invariants included
DSTRESS = {SVK: 229, MR: 771, NH: 269}
# w . dP/dtheta of the elastic rows; SVK also needs Gw : F (17), which the
# Mooney-Rivlin derivative already forms
GTHETA = {SVK: 152, MR: 53, NH: 28}
VISC_VJP = 349       # viscous adjoint in x and v, gv to the parent (no gathers/scatter)
VISC_GT = 25         # viscous parameter rows of the adjoint
VISC_JVP = 304       # viscous tangent in x and v (no gathers)


def flops_per_element(op, elem, law, damped, gtheta=False):
    """Counted FP64 arithmetic of one element (all quadrature points); the
    adjoint counts the parameter gradients only when they are requested."""
    tot = 0
    for z in NZ[elem]:
        g = 6 * z
        q = g + GEOM                               # reference geometry at the point
        if op == "fwd":
            q += (g + TOREF) * (2 if damped else 1)   # F (and Fdot)
            q += STRESS[law] + (VISC_FWD[law] if damped else 0)
            q += TOPAR + g                             # scatter to the nodes
        elif op == "vjp":
            q += 2 * (g + TOREF)                       # F, Gw
            q += DSTRESS[law] + TOPAR + g
            if gtheta:
                q += GTHETA[law] + 1 + (VISC_GT if damped else 0)
            if damped:
                q += g + TOREF + VISC_VJP + g          # Fdot, viscous terms, gv scatter
        else:
            q += 2 * (g + TOREF)                       # F, dF
            q += DSTRESS[law] + TOPAR + g
            if damped:
                q += 2 * (g + TOREF) + VISC_JVP        # Fdot, dFdot
        tot += q
    return tot


# consistent-mass action per element: at each point of the mass rule
# (T10 15 points, H8 8) the interpolation of u (3 x nen FMA), the scaling
# (3 mul + 1) and the scatter (3 x nen FMA)
MASS_QP = {T10: 15, H8: 8, Q27: 27}
NEN = {T10: 10, H8: 8, Q27: 27}


def mass_flops_per_element(elem):
    if elem == Q27:
        # non-zero shape values at each point: 3 per direction, 1 at a coordinate 0
        nzs = [int(np.prod([1 if (q // 3 ** d) % 3 == 1 else 3 for d in range(3)])) for q in range(27)]
        return sum(2 * 3 * z + 4 + 2 * 3 * z for z in nzs)
    return MASS_QP[elem] * (2 * 3 * NEN[elem] + 4 + 2 * 3 * NEN[elem])


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


def source_hash():
    """sha256 of the HIP library sources and of the build script that holds
    their compiler flags (ties counter summaries to a build)."""
    h = hashlib.sha256()
    files = sorted(p for p in glob.glob(os.path.join(CSRC, "*")) if p.endswith((".h", ".hip", ".cpp")))
    files.append(os.path.join(os.path.dirname(CSRC), "build.py"))
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profile(kernel_key):
    """HBM bytes per launch (fetch + write, copy-calibrated) of the kernel
    from the committed counter summary, if it was taken on these sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src, rows = None, {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if line.startswith("SOURCE_SHA256 "):
                src = line.split()[1]
            elif line.startswith("TRAFFIC "):
                kv = dict(tok.split("=", 1) for tok in line.split()[1:])
                rows[kv["kernel"]] = float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    if src != source_hash():
        return None
    return rows.get(kernel_key)


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(prob, budget_s=12.0):
    """The oracle as it is on a bounded sample of the same workload (the
    first elements of the mesh, forward + adjoint (gx, gv)): the serial C
    loop on one core, and the same loop split over every host core the
    process may use (OpenMP, thread-private node buffers added in thread
    order)."""
    import copy

    import oracle as O
    b = prob.blocks[0]
    cores = host_cores()

    def run(ne, threads):
        sb = copy.copy(b)
        sb.conn = np.ascontiguousarray(b.conn[:ne])
        t0 = time.perf_counter()
        if threads == 1:
            O.internal_force(prob.X, [sb], prob.x, prob.v)
            O.vjp(prob.X, [sb], prob.x, prob.v, prob.w, want_gtheta=False)
        else:
            O.internal_force_par(prob.X, [sb], prob.x, prob.v, threads=threads)
            O.vjp_par(prob.X, [sb], prob.x, prob.v, prob.w, want_gtheta=False, threads=threads)
        return time.perf_counter() - t0

    out = {}
    for threads in (1, cores):
        t_small = run(500 * threads, threads)
        ne = int(min(b.n_elem, max(500, 500 * threads * budget_s / max(t_small, 1e-6))))
        t = run(ne, threads)
        nq = ne * 5
        out[threads] = (nq / t, ne, nq, t)
    v1, ne1, nq1, t1 = out[1]
    vn, nen, nqn, tn = out[cores]
    return {"value": vn, "unit": "quad-pts/s", "cores": cores, "kind": "oracle",
            "sample": f"forward + adjoint (gx, gv) of the first {nen} of {b.n_elem} elements ({nqn} quadrature "
                      f"points), C oracle split over {cores} OpenMP threads, {tn:.1f} s",
            "serial": {"value": v1, "unit": "quad-pts/s", "cores": 1,
                       "sample": f"first {ne1} elements ({nq1} quadrature points), serial C oracle, {t1:.1f} s"}}


def timed(fn, steps, warmup, stream):
    """Median and mean of `steps` runs of fn, each between its own pair of
    events on the stream, after `warmup` untimed runs (milliseconds)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return float(np.median(ms)), float(np.mean(ms)), ev[0].elapsed_time(ev[-1])


def c4_ops(steps, warmup):
    """The 204,000-element Neo-Hookean body with per-element parameters:
    the adjoint with the parameter gradients (gx, gtheta) and the tangent
    product K dx, each timed alone (median of per-call event pairs)."""
    import torch

    import synth
    from paper_2602_17002_amd import Mesh
    p = synth.config_c4()
    dev = torch.device("cuda", 0)
    m = Mesh.from_problem(p)
    p = p.renumbered(m.node_order())
    m.close()
    m = Mesh.from_problem(p)
    s = torch.cuda.Stream(device=dev)
    out = {"workload": "C4: 204,000 T10 box 50x40x17 cells, Neo-Hookean, per-element (mu10, k)",
           "quad_points": p.n_qp}
    with torch.cuda.stream(s):
        x, w, dx = (torch.from_numpy(a).to(dev) for a in (p.x, p.w, p.dx))
        th = torch.from_numpy(p.theta_all()).to(dev)
        gx, df = torch.empty_like(x), torch.empty_like(x)
        gt = torch.empty_like(th)
        ops = (("vjp_gx_gtheta", lambda: m.vjp(x, None, w, th, want_v=False, out=(gx, None, gt)),
                flops_per_element("vjp", T10, NH, False, gtheta=True)),
               ("tangent_K_dx", lambda: m.jvp(x, None, dx, None, th, out=df),
                flops_per_element("jvp", T10, NH, False)))
        for name, fn, fpe in ops:
            med, mean, _ = timed(fn, steps, warmup, s)
            out[name] = {"ms": round(med, 4), "quad_pts_per_s": p.n_qp / (med * 1e-3),
                         "flops_per_element": fpe,
                         "frac_fp64_peak": round(fpe * p.n_elem / (med * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
    return out


def q27_ops(steps, warmup):
    """The 131,072-element Q27 body (64 x 64 x 32 cells, 3,538,944 points),
    Neo-Hookean + Kelvin-Voigt: the forward, the adjoint (gx, gv) and the
    tangent, each timed alone (median of per-call event pairs), the step
    (forward + adjoint) as in the headline line."""
    import torch

    import synth
    from paper_2602_17002_amd import Mesh
    p = synth.config_q27()
    dev = torch.device("cuda", 0)
    m = Mesh.from_problem(p)
    p = p.renumbered(m.node_order())
    m.close()
    m = Mesh.from_problem(p)
    s = torch.cuda.Stream(device=dev)
    info = m.info()
    out = {"workload": "Q27: 131,072 Q27 box 64x64x32 cells, 3x3x3 Gauss, Neo-Hookean + Kelvin-Voigt",
           "quad_points": p.n_qp, "tile_elems": info["tile_elems_q27"], "tiles": info["n_tiles"]}
    with torch.cuda.stream(s):
        x, v, w, dx, dv = (torch.from_numpy(a).to(dev) for a in (p.x, p.v, p.w, p.dx, p.dv))
        f, gx, gv, df = (torch.empty_like(x) for _ in range(4))
        ops = (("forward", lambda: m.internal_force(x, v, out=f), flops_per_element("fwd", Q27, NH, True)),
               ("adjoint_gx_gv", lambda: m.vjp(x, v, w, want_theta=False, out=(gx, gv, None)),
                flops_per_element("vjp", Q27, NH, True)),
               ("tangent", lambda: m.jvp(x, v, dx, dv, out=df), flops_per_element("jvp", Q27, NH, True)))
        for name, fn, fpe in ops:
            med, mean, _ = timed(fn, steps, warmup, s)
            out[name] = {"ms": round(med, 4), "quad_pts_per_s": p.n_qp / (med * 1e-3),
                         "flops_per_element": fpe,
                         "frac_fp64_peak": round(fpe * p.n_elem / (med * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}

        def step():
            m.internal_force(x, v, out=f)
            m.vjp(x, v, w, want_theta=False, out=(gx, gv, None))

        med, _, _ = timed(step, steps, warmup, s)
        out["step_fwd_adjoint"] = {"ms": round(med, 4), "quad_pts_per_s": p.n_qp / (med * 1e-3)}
    return out


def step_ops(steps, warmup):
    """The backward-Euler step operations on the 1,020,000-element box with
    a density (1100 kg/m^3, h = 1e-4 s): the consistent-mass action, the
    step residual, the Newton operator (each the median of per-call event
    pairs), and one matrix-free Newton-Krylov step (restarted GMRES to a
    relative residual of 1e-8), reported with its iteration count."""
    import torch

    import synth
    from paper_2602_17002_amd import Mesh
    p = synth.config_c2()
    dev = torch.device("cuda", 0)
    m = Mesh.from_problem(p)
    p = p.renumbered(m.node_order())
    m.close()
    for b in p.blocks:
        b.rho = 1100.0
    m = Mesh.from_problem(p)
    h = 1e-4
    rng = np.random.default_rng(7)
    s = torch.cuda.Stream(device=dev)
    ne, nqp = p.n_elem, p.n_qp
    out = {"workload": "C2 box with rho = 1100 kg/m^3, h = 1e-4 s: q_n = the C2 state, v_n ~ N(0, 0.3 m/s), "
                       "v = v_n + N(0, 0.3 m/s)", "quad_points": nqp}
    with torch.cuda.stream(s):
        qn = torch.from_numpy(p.x).to(dev)
        vn = torch.from_numpy(rng.normal(0, 0.3, p.X.shape)).to(dev)
        v = vn + torch.from_numpy(rng.normal(0, 0.3, p.X.shape)).to(dev)
        dv = torch.from_numpy(rng.normal(0, 1.0, p.X.shape)).to(dev)
        y = torch.empty_like(qn)
        fm = mass_flops_per_element(T10)
        ops = (("mass_action", lambda: m.mass_action(dv, out=y), fm),
               ("step_residual", lambda: m.step_residual(qn, vn, v, h, out=y),
                flops_per_element("fwd", T10, NH, True) + fm),
               ("newton_operator", lambda: m.newton_operator(qn, v, h, None, dv, out=y),
                flops_per_element("jvp", T10, NH, True) + fm))
        for name, fn, fpe in ops:
            med, mean, _ = timed(fn, steps, warmup, s)
            out[name] = {"ms": round(med, 4), "quad_pts_per_s": nqp / (med * 1e-3), "flops_per_element": fpe,
                         "frac_fp64_peak": round(fpe * ne / (med * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
        work = torch.empty(int(m.newton_workspace(30)), dtype=torch.float64, device=dev)
        vo = torch.empty_like(qn)
        m.newton_step(qn, vn, v, h, out=vo, work=work, restart=30, max_iters=300, rtol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vo, info = m.newton_step(qn, vn, v, h, out=vo, work=work, restart=30, max_iters=300, rtol=1e-8)
        t1 = time.perf_counter()
        out["newton_krylov_step"] = {"ms": round((t1 - t0) * 1e3, 3), "gmres_iterations": info["iters"],
                                     "converged": bool(info["converged"]),
                                     "relative_residual": info["res_norm"] / max(info["g_norm"], 1e-300),
                                     "restart": 30, "rtol": 1e-8}
    return out


def joints_ops(steps, warmup, n_joints=1_000_000):
    """Revolute joints with their five points in random elements of the
    1,020,000-element box: row-normalised values and the transpose scatter
    h C^T (lambda + rho c) (median of per-call event pairs)."""
    import torch

    import synth
    from paper_2602_17002_amd.joints import Joints
    p = synth.config_c2()
    rng = np.random.default_rng(11)
    conn = p.blocks[0].conn
    t0 = time.time()
    els = rng.integers(conn.shape[0], size=(n_joints, 5))
    bary = rng.dirichlet(np.ones(4), size=(n_joints, 5))
    dev = torch.device("cuda", 0)
    J = Joints.from_arrays(p.X, np.full((n_joints, 5), T10, np.int32), conn[els], bary[:, :, 1:])
    log(f"[bench] {n_joints} joints built in {time.time() - t0:.1f} s")
    s = torch.cuda.Stream(device=dev)
    out = {"workload": f"{n_joints} revolute joints, points in random elements of the C2 box"}
    with torch.cuda.stream(s):
        q = torch.from_numpy(p.x).to(dev)
        lam = torch.from_numpy(rng.normal(0, 1, (n_joints, 5))).to(dev)
        g = torch.empty_like(q)
        c = torch.empty((n_joints, 5), dtype=torch.float64, device=dev)
        for name, fn in (("values", lambda: J.values(q)),
                         ("scatter", lambda: J.scatter(q, lam, 1e4, 1e-3, out=g))):
            med, mean, _ = timed(fn, steps, warmup, s)
            out[name] = {"ms": round(med, 4), "joints_per_s": n_joints / (med * 1e-3)}
    return out


def batched_vs_plain(steps, warmup):
    """Forward internal force of a 512-body multibody set: one batched mesh
    (hipGraph replay) against one plain mesh per body on the same stream."""
    import copy

    import torch

    import synth
    from paper_2602_17002_amd import BATCHED, Mesh
    t0 = time.time()
    p = synth.config_c3()
    log(f"[bench] C3: {len(p.blocks)} bodies, {p.n_elem} elements, {p.n_nodes} nodes ({time.time() - t0:.1f} s)")
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream(device=dev)
    t0 = time.time()
    batched = Mesh(p.X, [copy.copy(b) for b in p.blocks], flags=BATCHED)
    plains = []
    for bi, b in enumerate(p.blocks):
        n0, n1 = p.body_nodes[bi]
        bb = copy.copy(b)
        bb.conn = b.conn - n0
        plains.append((Mesh(p.X[:, n0:n1], [bb]), n0, n1))
    log(f"[bench] C3 meshes built in {time.time() - t0:.1f} s")
    with torch.cuda.stream(s):
        x = torch.from_numpy(p.x).to(dev)
        f_b = torch.empty_like(x)
        xs = [x[:, n0:n1].contiguous() for _, n0, n1 in plains]
        fs = [torch.empty_like(xx) for xx in xs]

        def run_batched():
            batched.internal_force(x, out=f_b)

        def run_plain():
            for (m, _, _), xx, ff in zip(plains, xs, fs):
                m.internal_force(xx, out=ff)

        # the plain meshes' launches captured into one graph as well, so the
        # factor is not host dispatch alone
        run_plain()
        torch.cuda.synchronize()
        g_plain = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_plain, stream=s):
            run_plain()
        res = {}
        for name, fn in (("batched", run_batched), ("plain", run_plain), ("plain_graph", g_plain.replay)):
            res[name] = timed(fn, steps, warmup, s)[0]
        same = all(torch.equal(f_b[:, n0:n1], ff) for (_, n0, n1), ff in zip(plains, fs))

        # forward + backward through the autograd Function on the batched
        # mesh: fresh output tensors every iteration (new operand pointers,
        # so cached graphs are updated in place), against the same two calls
        # into preallocated outputs (cached graphs replayed)
        from paper_2602_17002_amd import TLInternalForce
        w = torch.from_numpy(np.random.default_rng(5).standard_normal(p.x.shape)).to(dev)
        gx_b = torch.empty_like(x)

        def run_autograd():
            xr = x.detach().requires_grad_(True)
            f = TLInternalForce.apply(xr, None, None, batched)
            f.backward(w)

        def run_direct():
            batched.internal_force(x, out=f_b)
            batched.vjp(x, None, w, want_v=False, want_theta=False, out=(gx_b, None, None))

        info0 = batched.info()
        res["autograd"] = timed(run_autograd, steps, warmup, s)[0]
        info1 = batched.info()
        res["direct"] = timed(run_direct, steps, warmup, s)[0]
    return {"workload": f"C3: {len(p.blocks)} bodies of 200-50,000 elements, mixed T10/H8, SVK/NH, "
                        f"{p.n_elem} elements, forward f_int",
            "ms_batched": round(res["batched"], 4), "ms_plain": round(res["plain"], 4),
            "ms_plain_graph": round(res["plain_graph"], 4),
            "speedup": round(res["plain"] / res["batched"], 3),
            "speedup_vs_plain_graph": round(res["plain_graph"] / res["batched"], 3),
            "quad_pts_per_s_batched": p.n_qp / (res["batched"] * 1e-3),
            "bitwise_equal_per_body": bool(same),
            "autograd_fwd_bwd": {"ms": round(res["autograd"], 4), "ms_direct_calls": round(res["direct"], 4),
                                 "graphs_built": info1["graphs_built"] - info0["graphs_built"],
                                 "graphs_updated": info1["graphs_updated"] - info0["graphs_updated"]}}


def batched_c5(steps, warmup):
    """Forward, adjoint (gx, gtheta) and tangent of a 256-body multibody set:
    one autotuned batched mesh whose three calls are captured into one graph,
    against one plain mesh per body with the three calls launched eagerly."""
    import copy

    import torch

    import synth
    from paper_2602_17002_amd import AUTOTUNE, BATCHED, Mesh
    t0 = time.time()
    p = synth.config_c5()
    log(f"[bench] C5: {len(p.blocks)} bodies, {p.n_elem} elements ({time.time() - t0:.1f} s)")
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream(device=dev)
    t0 = time.time()
    batched = Mesh(p.X, [copy.copy(b) for b in p.blocks], flags=BATCHED | AUTOTUNE)
    tuned = batched.info()
    log(f"[bench] C5 batched mesh autotuned in {time.time() - t0:.1f} s: {tuned}")
    # the plain meshes take the tile sizes the batched mesh chose, so both
    # sum in the same order and must agree bitwise
    plains, col = [], 0
    for bi, b in enumerate(p.blocks):
        n0, n1 = p.body_nodes[bi]
        bb = copy.copy(b)
        bb.conn = b.conn - n0
        bb.tile_elems = tuned["tile_elems_t10"] if b.elem == synth.T10 else tuned["tile_elems_h8"]
        plains.append((Mesh(p.X[:, n0:n1], [bb]), n0, n1, col, col + b.n_elem))
        col += b.n_elem
    with torch.cuda.stream(s):
        x, w, dx = (torch.from_numpy(a).to(dev) for a in (p.x, p.w, p.dx))
        f, gx, df = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
        gt = torch.empty((5, p.n_elem), dtype=torch.float64, device=dev)
        g = torch.cuda.CUDAGraph()
        batched.internal_force(x, out=f)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            batched.internal_force(x, out=f)
            batched.vjp(x, None, w, want_v=False, out=(gx, None, gt))
            batched.jvp(x, None, dx, out=df)
        per = []
        for m, n0, n1, c0, c1 in plains:
            xs, ws, ds = x[:, n0:n1].contiguous(), w[:, n0:n1].contiguous(), dx[:, n0:n1].contiguous()
            per.append((m, xs, ws, ds, torch.empty_like(xs), torch.empty_like(xs), torch.empty_like(xs),
                        torch.empty((5, c1 - c0), dtype=torch.float64, device=dev)))

        def run_plain():
            for m, xs, ws, ds, ff, gg, dd, tt in per:
                m.internal_force(xs, out=ff)
                m.vjp(xs, None, ws, want_v=False, out=(gg, None, tt))
                m.jvp(xs, None, ds, out=dd)

        run_plain()
        torch.cuda.synchronize()
        g_plain = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_plain, stream=s):
            run_plain()
        res = {}
        for name, fn in (("batched", g.replay), ("plain", run_plain), ("plain_graph", g_plain.replay)):
            res[name] = timed(fn, steps, warmup, s)[0]
        def nrel(a, b):
            return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
        pairs = [((f[:, n0:n1], ff), (gx[:, n0:n1], gg), (df[:, n0:n1], dd), (gt[:, c0:c1], tt))
                 for (_, n0, n1, c0, c1), (_, _, _, _, ff, gg, dd, tt) in zip(plains, per)]
        diff = max(nrel(a, b) for body in pairs for a, b in body)
        same = all(torch.equal(a, b) for body in pairs for a, b in body)
    return {"workload": f"C5: {len(p.blocks)} bodies of 1,000-100,000 elements, mixed T10/H8, SVK/NH, "
                        f"{p.n_elem} elements, forward + adjoint (gx, gtheta) + tangent in one graph",
            "tile_elems_t10": tuned["tile_elems_t10"], "tile_elems_h8": tuned["tile_elems_h8"],
            "ms_batched": round(res["batched"], 4), "ms_plain": round(res["plain"], 4),
            "ms_plain_graph": round(res["plain_graph"], 4),
            "speedup": round(res["plain"] / res["batched"], 3),
            "speedup_vs_plain_graph": round(res["plain_graph"] / res["batched"], 3),
            "quad_pts_per_s_batched": p.n_qp / (res["batched"] * 1e-3),
            "bitwise_equal_per_body": same, "max_rel_diff_per_body": diff}


# ---------------------------------------------------------------- profiler summaries

def _csv_rows(pattern):
    rows = []
    for p in sorted(glob.glob(pattern, recursive=True)):
        with open(p) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def pmc_summary(trace_dir, fetch_dir, write_dir, commands):
    """Write profiles/ summaries from rocprofv3 output folders: the kernel
    statistics of a --kernel-trace --stats run, and FETCH_SIZE / WRITE_SIZE
    per dispatch from two --pmc runs, scaled by what the same counters read
    for the device-to-device copy kernel of known size in those runs."""
    os.makedirs(PROFILES, exist_ok=True)
    stats = _csv_rows(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    lines = ["# Kernel statistics: C2 forward + adjoint (1,020,000 T10, Neo-Hookean + Kelvin-Voigt)", "",
             f"Command: `{commands['trace']}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    with open(os.path.join(PROFILES, "kernel_stats_c2_fwd_vjp.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    def per_kernel(d, counter):
        acc = {}
        for r in _csv_rows(os.path.join(d, "**", "*counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy_name = next(k for k in fetch if "copyBuffer" in k)
    calib_kib = float(commands["calib_mib"]) * 1024.0
    f_scale = calib_kib / max(fetch[copy_name])
    w_scale = calib_kib / max(write[copy_name])
    lines = ["# HBM traffic per dispatch: C2 forward + adjoint (1,020,000 T10, Neo-Hookean + Kelvin-Voigt)", "",
             f"Fetch command: `{commands['fetch']}`", "", f"Write command: `{commands['write']}`", "",
             f"Calibration: the {commands['calib_mib']} MiB device-to-device copy (`{copy_name}`) read "
             f"FETCH_SIZE {max(fetch[copy_name]):.0f} KiB and WRITE_SIZE {max(write[copy_name]):.0f} KiB; "
             f"scale factors {f_scale:.3f} (fetch) and {w_scale:.3f} (write).", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch MB (scaled) | write MB (scaled) |",
             "|---|---|---|---|---|---|"]
    machine = [f"SOURCE_SHA256 {source_hash()}"]
    for k in sorted(fetch):
        if "tlfea" not in k:
            continue
        fk = float(np.median(fetch[k]))
        wk = float(np.median(write.get(k, [0.0])))
        fb, wb = fk * 1024 * f_scale, wk * 1024 * w_scale
        lines.append(f"| `{k[:80]}` | {len(fetch[k])} | {fk:.0f} | {wk:.0f} | {fb / 1e6:.1f} | {wb / 1e6:.1f} |")
        key = k.split("(")[0].replace("void ", "").replace(" ", "")
        machine.append(f"TRAFFIC kernel={key} fetch_bytes={fb:.0f} write_bytes={wb:.0f}")
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n\n```\n" + "\n".join(machine) + "\n```\n")
    print("\n".join(machine))


# ---------------------------------------------------------------- main

def trace_summary(name, title, trace_dir, command):
    """Write profiles/kernel_stats_<name>.md from a rocprofv3 --kernel-trace
    --stats run: calls, average, min, max and share of every kernel."""
    os.makedirs(PROFILES, exist_ok=True)
    stats = _csv_rows(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    lines = [f"# Kernel statistics: {title}", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    lines += ["", f"SOURCE_SHA256 {source_hash()}"]
    with open(os.path.join(PROFILES, f"kernel_stats_{name}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def sq_summary(dirs, commands):
    """Write profiles/sq_counters_c2_fwd_vjp.md from rocprofv3 --pmc runs of
    SQ counters over the bench: the median per dispatch of every counter for
    the tile kernels, the LDS bank-conflict share of LDS-active cycles, and
    the FP64 flops the hardware executed per element."""
    os.makedirs(PROFILES, exist_ok=True)
    acc = {}
    for d in dirs:
        for r in _csv_rows(os.path.join(d, "**", "*counter_collection.csv")):
            if "tlfea::k_" not in r["Kernel_Name"] or "k_halo" in r["Kernel_Name"]:
                continue
            acc.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["# SQ counters per dispatch: C2 forward + adjoint (1,020,000 T10, Neo-Hookean + Kelvin-Voigt)", ""]
    for k in sorted(commands):
        lines += [f"Command {k}: `{commands[k]}`", ""]
    lines += ["Medians over the dispatches of each kernel. `bank-conflict share` = SQ_LDS_BANK_CONFLICT / "
              "SQ_LDS_IDX_ACTIVE; `FP64 flop / element` = SQ_INSTS_VALU_FLOPS_FP64 x 64 / 1,020,000.", ""]
    for k in sorted(acc):
        c = {n: float(np.median(v)) for n, v in acc[k].items()}
        lines += [f"## `{k[:90]}`", "", "| counter | median per dispatch |", "|---|---|"]
        lines += [f"| {n} | {c[n]:.4g} |" for n in sorted(c)]
        if c.get("SQ_LDS_IDX_ACTIVE"):
            lines.append(f"| bank-conflict share | {c.get('SQ_LDS_BANK_CONFLICT', 0.0) / c['SQ_LDS_IDX_ACTIVE']:.3f} |")
        if "SQ_INSTS_VALU_FLOPS_FP64" in c:
            lines.append(f"| FP64 flop / element | {c['SQ_INSTS_VALU_FLOPS_FP64'] * 64 / 1020000:.0f} |")
        lines.append("")
    lines.append(f"SOURCE_SHA256 {source_hash()}")
    with open(os.path.join(PROFILES, "sq_counters_c2_fwd_vjp.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[-3:]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-body batched vs plain comparison")
    ap.add_argument("--no-c5", action="store_true", help="skip the 256-body forward + adjoint + tangent graph")
    ap.add_argument("--no-c4", action="store_true", help="skip the 204,000-element per-element-parameter adjoint and tangent")
    ap.add_argument("--no-q27", action="store_true", help="skip the 131,072-element Q27 forward, adjoint and tangent")
    ap.add_argument("--no-step", action="store_true", help="skip the mass, step residual, Newton operator and Newton-Krylov step")
    ap.add_argument("--no-joints", action="store_true", help="skip the revolute-joint values and scatter")
    ap.add_argument("--keep-node-order", action="store_true",
                    help="keep the generator's node numbering instead of the library's suggested order")
    ap.add_argument("--tile", type=int, default=0, help="elements per tile (0 = library default)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, used to scale the HBM byte counters of a profiler run)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--trace-summary", nargs=3, metavar=("NAME", "TITLE", "TRACE_DIR"),
                    help="write profiles/kernel_stats_NAME.md from a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--only-c5", action="store_true",
                    help="time only the 256-body forward + adjoint + tangent graph (for profiling it)")
    ap.add_argument("--sq-summary", nargs="+", metavar="PMC_DIR",
                    help="write profiles/sq_counters_c2_fwd_vjp.md from rocprofv3 --pmc runs of SQ counters")
    ap.add_argument("--commands", default="{}",
                    help="JSON: the profiler command lines (for --pmc-summary / --sq-summary)")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(*args.trace_summary, json.loads(args.commands)["trace"])
        return
    if args.sq_summary:
        sq_summary(args.sq_summary, json.loads(args.commands))
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, json.loads(args.commands))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.only_c5:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"batched_c5": batched_c5(max(3, args.steps // 4), 1)}), flush=True)
        return

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
    if not args.keep_node_order:
        # renumber the nodes once, as the library suggests (tile nodes contiguous)
        prob = prob.renumbered(mesh.node_order())
        mesh.close()
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

        # whole steps (the value): each step between its own pair of events,
        # the median over the steps
        ms_med, ms_mean, ms_total = timed(step, args.steps, args.warmup, stream)
        # per-kernel durations (HIP events around every launch, on the launch
        # stream)
        mesh.reset_profile()
        mesh.set_profiling(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        mesh.set_profiling(False)
        prof = mesh.profile()
    log(f"[bench] timed {args.steps} steps: {ms_total:.3f} ms, median {ms_med:.4f} ms; kernels {prof}")
    ms_step = ms_med
    n_qp = prob.n_qp
    value = n_qp / (ms_step * 1e-3)

    # roofline of the dominant kernel
    k_ms = {k: (c, t / c if c else 0.0) for k, (c, t) in prof.items()}
    dom = max(("forward_tile", "adjoint_tile"), key=lambda k: k_ms[k][1])
    op = "fwd" if dom == "forward_tile" else "vjp"
    ne, nn = prob.n_elem, prob.n_nodes
    fpe = flops_per_element(op, T10, NH, True, gtheta=False)
    flops = fpe * ne
    t_dom = k_ms[dom][1] * 1e-3
    achieved = flops / t_dom / 1e12
    byts = bytes_per_call(op, nn, ne, 10, True)
    kname = "tlfea::k_fwd<0,2,true,0>" if op == "fwd" else "tlfea::k_vjp<0,2,true,false>"
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic_from_profile(kname),
            "kernel": kname, "kernel_ms": round(k_ms[dom][1], 4),
            "flops_per_element": fpe, "elements_per_launch": ne,
            "algorithmic_bytes_per_launch": byts,
            "hbm_frac_algorithmic": round(byts / t_dom / 1e9 / HBM_PEAK_GBS, 4)}

    out = {
        "metric": "quad-pts/s f_int fwd+VJP (1M T10 NH), batched vs plain; % HBM/FP64 peak",
        "value": value, "unit": "quad-pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "ms_per_step_mean": ms_mean, "ms_timed_total": ms_total,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "C2: 1,020,000 T10 box 100x100x17 cells, Neo-Hookean + Kelvin-Voigt, "
                               "forward + adjoint (gx, gv)", "elements": ne, "nodes": nn, "quad_points": n_qp,
                   "tile_elems": info["tile_elems_t10"],
                   "step_call": "tlfea_internal_force + tlfea_internal_force_vjp"},
        "kernels_ms_avg": {k: round(t, 4) for k, (c, t) in k_ms.items() if c},
        "roofline": roof,
    }
    del mesh, x, v, w, f, gx, gv
    torch.cuda.empty_cache()
    if not args.no_c4:
        out["c4"] = c4_ops(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_q27:
        out["q27"] = q27_ops(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_step:
        out["step"] = step_ops(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_joints:
        out["joints"] = joints_ops(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched_vs_plain"] = batched_vs_plain(max(3, args.steps // 4), 2)
        torch.cuda.empty_cache()
    if not args.no_c5:
        out["batched_c5"] = batched_c5(max(3, args.steps // 4), 1)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

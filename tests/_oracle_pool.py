"""The oracle over a whole large mesh, split over CPU worker processes.

Each worker is a fresh Python process that imports only numpy and the
oracle (never torch or the HIP library) and evaluates the oracle on a
contiguous range of one block's elements.  The oracle accumulates element
contributions into nodal arrays, so the nodal result is the sum of the
workers' partial arrays (added here in range order); per-element outputs
(the parameter gradients) are concatenated.  The arithmetic is the
oracle's own; only the order of the node sums differs from one serial call.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WORKER = os.path.join(HERE, "_oracle_worker.py")


def n_workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run(X, blocks, arrays, ops, workers=None, chunk_qp=400_000, h=0.0):
    """Evaluate the oracle on every element of ``blocks``.

    arrays: dict of nodal [3][n] arrays among x, v, w, dx, dv, u, qn, vn
    (None allowed).  ops: subset of {"f", "vjp", "gtheta", "jvp", "mass",
    "res", "newt"}: "f" internal force, "vjp" gx and gv, "gtheta" the
    parameter gradient [5][n_elem] (block order), "jvp" K dx + C dv, "mass"
    M u, "res" the step residual without f_ext (time step h), "newt" the
    Newton operator applied to dv.  Returns {name: array} with keys f, gx,
    gv, gtheta, df, mu, g, y for the requested ops."""
    workers = workers or n_workers()
    tmp = tempfile.mkdtemp(prefix="oracle_pool_")
    try:
        np.save(os.path.join(tmp, "X.npy"), np.ascontiguousarray(X, dtype=np.float64))
        for k, a in arrays.items():
            if a is not None:
                np.save(os.path.join(tmp, f"{k}.npy"), np.ascontiguousarray(a, dtype=np.float64))
        jobs = []
        for bi, b in enumerate(blocks):
            np.save(os.path.join(tmp, f"conn{bi}.npy"), np.ascontiguousarray(b.conn, dtype=np.int32))
            te = getattr(b, "theta_e", None)
            if te is None:
                te = np.repeat(np.asarray(b.theta, np.float64)[:, None], b.conn.shape[0], axis=1)
            np.save(os.path.join(tmp, f"theta{bi}.npy"), np.ascontiguousarray(te, dtype=np.float64))
            nq = 5 if b.elem == 0 else (8 if b.elem == 1 else 27)
            per = max(1, chunk_qp // nq)
            for e0 in range(0, b.conn.shape[0], per):
                jobs.append((bi, b.elem, b.law, int(bool(b.damped)), float(getattr(b, "rho", 0.0) or 0.0),
                             e0, min(b.conn.shape[0], e0 + per)))
        procs, outs = [], []
        env = dict(os.environ, OMP_NUM_THREADS="1", PYTHONPATH=os.path.dirname(HERE))
        pending = list(enumerate(jobs))
        running = []
        while pending or running:
            while pending and len(running) < workers:
                j, (bi, elem, law, damped, rho, e0, e1) = pending.pop(0)
                out = os.path.join(tmp, f"out{j}.npz")
                cmd = [sys.executable, WORKER, tmp, str(bi), str(elem), str(law), str(damped), repr(rho), repr(h),
                       str(e0), str(e1), ",".join(ops), out]
                running.append((j, subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                    text=True)))
                outs.append((j, out))
            still = []
            for j, p in running:
                if p.poll() is None:
                    still.append((j, p))
                    continue
                msg = p.stdout.read()
                if p.returncode != 0:
                    for _, q in running:
                        if q.poll() is None:
                            q.kill()
                    raise RuntimeError(f"oracle worker {j} failed: {msg[-2000:]}")
            if len(still) == len(running):
                import time
                time.sleep(0.05)
            running = still
        outs.sort()
        res = {}
        n_elem_blocks = [b.conn.shape[0] for b in blocks]
        gt = [np.zeros((5, n)) for n in n_elem_blocks]
        for j, path in outs:
            bi, _, _, _, _, e0, e1 = jobs[j]
            with np.load(path) as z:
                idx = z["idx"]
                for k in z.files:
                    if k == "idx":
                        continue
                    if k == "gtheta":
                        gt[bi][:, e0:e1] = z[k]
                    else:
                        if k not in res:
                            res[k] = np.zeros_like(X, dtype=np.float64)
                        res[k][:, idx] += z[k]
        if "gtheta" in ops:
            res["gtheta"] = np.concatenate(gt, axis=1)
        wanted = {"f": "f", "gx": "vjp", "gv": "vjp", "df": "jvp", "mu": "mass", "g": "res", "y": "newt"}
        for k, op in wanted.items():
            if k not in res and op in ops:
                res[k] = np.zeros_like(X)
        return res
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)

"""One worker of tests/_oracle_pool.py: the oracle on one element range.

argv: dir block elem law damped e0 e1 ops out.npz.  Imports numpy and the
oracle only."""
import os
import sys
from types import SimpleNamespace

import numpy as np


def main():
    d, bi, elem, law, damped, rho, h, e0, e1, ops, out = sys.argv[1:]
    bi, elem, law, damped, e0, e1 = map(int, (bi, elem, law, damped, e0, e1))
    rho, h = float(rho), float(h)
    ops = ops.split(",")
    import oracle as O

    def load(name):
        p = os.path.join(d, f"{name}.npy")
        return np.load(p, mmap_mode="r") if os.path.exists(p) else None

    X = np.ascontiguousarray(load("X"))
    conn = np.ascontiguousarray(load(f"conn{bi}")[e0:e1])
    theta = np.ascontiguousarray(load(f"theta{bi}")[:, e0:e1])
    blk = SimpleNamespace(elem=elem, law=law, damped=bool(damped), conn=conn, theta_e=theta, theta=theta[:, 0],
                          rho=rho)
    a = {k: (None if load(k) is None else np.ascontiguousarray(load(k)))
         for k in ("x", "v", "w", "dx", "dv", "u", "qn", "vn")}
    v = a["v"] if damped else None
    res = {}
    if "f" in ops:
        res["f"] = O.internal_force(X, [blk], a["x"], v)
    if "vjp" in ops or "gtheta" in ops:
        gx, gv, gt = O.vjp(X, [blk], a["x"], v, a["w"], want_gx="vjp" in ops, want_gv="vjp" in ops and bool(damped),
                           want_gtheta="gtheta" in ops)
        if "vjp" in ops:
            res["gx"] = gx
            if gv is not None:
                res["gv"] = gv
        if gt is not None:
            res["gtheta"] = gt
    if "jvp" in ops:
        res["df"] = O.jvp(X, [blk], a["x"], v, a["dx"], a["dv"] if damped else None)
    if "mass" in ops:
        res["mu"] = O.mass_action(X, [blk], a["u"])
    if "res" in ops:
        res["g"] = O.step_residual(X, [blk], a["qn"], a["vn"], a["v"], h)
    if "newt" in ops:
        res["y"] = O.newton_operator(X, [blk], a["qn"], a["v"], h, a["dv"])
    # nodal results only at the range's nodes (the rest are zero)
    idx = np.unique(conn)
    save = {"idx": idx.astype(np.int64)}
    for k, val in res.items():
        save[k] = val if k == "gtheta" else np.ascontiguousarray(val[:, idx])
    np.savez(out, **save)


if __name__ == "__main__":
    main()

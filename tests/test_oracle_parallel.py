"""The oracle's OpenMP entry points, which time the all-cores CPU baseline
(CPU only): each splits a block's elements into ranges over threads with
private buffers added in thread order, so its results equal the serial
oracle's to rounding and are bitwise the same from run to run at a given
thread count.  Every output of the forward and the adjoint, on a damped
cantilever and on a body with per-element parameters."""
import numpy as np
import pytest

import oracle as O
import synth
from _util import rel

# a sum reordered over a few ranges of elements: a few units of rounding
BAR = 1e-14


@pytest.fixture(scope="module")
def problems():
    p1 = synth.config_c1()
    rng = np.random.default_rng(7)
    X, conn = synth.box_h8(6, 4, 3, size=(0.12, 0.08, 0.06))
    x = synth.sinusoidal_state(X, 0.05, rng)
    th = np.array([1.2e6, 0.45e6, 1.72667e7, 1.0e4, 3.0e3])
    b = synth.Block(synth.H8, synth.MR, conn, th.copy(), damped=True)
    b.theta_e = th[:, None] * rng.uniform(0.5, 2.0, (5, conn.shape[0]))
    p2 = synth.Problem("h8-mr", X, x, rng.normal(0, 0.5, X.shape), [b], cell=0.02)
    out = []
    for p in (p1, p2):
        w = np.random.default_rng(8).standard_normal(p.X.shape)
        out.append((p, w))
    return out


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_forward_and_adjoint_equal_the_serial_oracle(problems, threads):
    for p, w in problems:
        f = O.internal_force(p.X, p.blocks, p.x, p.v)
        fp = O.internal_force_par(p.X, p.blocks, p.x, p.v, threads=threads)
        assert rel(fp, f) <= BAR, (p.name, rel(fp, f))
        gx, gv, gt = O.vjp(p.X, p.blocks, p.x, p.v, w)
        px, pv, pt = O.vjp_par(p.X, p.blocks, p.x, p.v, w, threads=threads)
        assert rel(px, gx) <= BAR and rel(pv, gv) <= BAR, p.name
        # each element's parameter gradient is one element's sum: no reordering
        assert np.array_equal(pt, gt), p.name
        again = O.internal_force_par(p.X, p.blocks, p.x, p.v, threads=threads)
        assert np.array_equal(again, fp)

"""The seeded synthetic workloads (CPU only): sizes, element types, laws,
parameters and damping as the input recipes state them.  The structured
boxes split every cell into six T10 tetrahedra on a (2 n + 1)-point grid
per direction; the multibody sets draw log-uniform body sizes, T10 and H8
alternating."""
import math

import numpy as np

import synth


def grid_nodes(nx, ny, nz):
    return (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1)


def test_c1_cantilever():
    p = synth.config_c1()
    b, = p.blocks
    assert (b.elem, b.law, b.damped) == (synth.T10, synth.SVK, True)
    assert p.n_elem == 6 * 10 * 2 * 2 == 240 and p.n_nodes == grid_nodes(10, 2, 2) == 525
    # E = 1e7, nu = 0.3: lambda = E nu / ((1 + nu)(1 - 2 nu)), mu = E / (2 (1 + nu))
    assert np.allclose(b.theta[:2], [1e7 * 0.3 / (1.3 * 0.4), 1e7 / 2.6], rtol=1e-12)
    assert b.theta[3] == 1e4 and b.theta[4] == 0.0
    assert np.allclose(p.X.max(axis=1) - p.X.min(axis=1), [1.0, 0.1, 0.1])


def test_c2_box():
    p = synth.config_c2()
    b, = p.blocks
    assert (b.elem, b.law, b.damped) == (synth.T10, synth.NH, True)
    assert p.n_elem == 6 * 100 * 100 * 17 == 1_020_000
    assert p.n_nodes == grid_nodes(100, 100, 17) == 1_414_035
    assert p.n_qp == 5 * 1_020_000
    # mu = 3.4e6, lambda = 1.5e7: mu10 = mu / 2, k = lambda + 2 mu / 3
    assert np.allclose(b.theta, [1.7e6, 0.0, 1.5e7 + 2 * 3.4e6 / 3, 1e4, 0.0], rtol=1e-12)
    assert np.allclose(p.X.max(axis=1) - p.X.min(axis=1), [1.0, 1.0, 0.17])


def test_c4_box_with_per_element_parameters():
    p = synth.config_c4()
    b, = p.blocks
    assert (b.elem, b.law, b.damped) == (synth.T10, synth.NH, False)
    assert p.n_elem == 6 * 50 * 40 * 17 == 204_000 and p.n_nodes == grid_nodes(50, 40, 17) == 286_335
    th = b.theta_e
    assert th.shape == (5, 204_000)
    # mu, lambda ~ log-uniform on [1e5, 1e7] independently: mu10 = mu / 2 in
    # [5e4, 5e6], k = lambda + 2 mu / 3 in [1e5 + 2e5 / 3, 1e7 + 2e7 / 3]
    assert th[0].min() >= 5e4 and th[0].max() <= 5e6
    assert th[2].min() >= 1e5 + 2e5 / 3 * 0.999 and th[2].max() <= (1e7 + 2e7 / 3) * 1.001
    assert not np.any(th[1]) and not np.any(th[3:])
    # the mu draws cover the range on a log scale
    lm = np.log10(2 * th[0])
    assert lm.min() < 5.05 and lm.max() > 6.95 and abs(lm.mean() - 6.0) < 0.02


def _multibody(p, n_bodies, n_min, n_max):
    assert len(p.blocks) == n_bodies
    counts = np.array([b.conn.shape[0] for b in p.blocks])
    for i, b in enumerate(p.blocks):
        assert b.elem == (synth.T10 if i % 2 == 0 else synth.H8)
        assert b.law in (synth.SVK, synth.NH) and not b.damped
    # the drawn sizes are log-uniform on [n_min, n_max]; a body rounds its
    # cell counts, so its element count is within a factor 2 of the draw
    assert counts.min() >= n_min / 2 and counts.max() <= 2 * n_max
    mean = (n_max - n_min) / math.log(n_max / n_min)     # mean of the log-uniform law
    assert abs(counts.sum() / (n_bodies * mean) - 1) < 0.1
    laws = [b.law for b in p.blocks]
    assert 0.35 < laws.count(synth.SVK) / n_bodies < 0.65
    return int(counts.sum())


def test_c3_multibody():
    assert _multibody(synth.config_c3(), 512, 200, 5e4) == 4_732_137


def test_c5_multibody():
    assert _multibody(synth.config_c5(), 256, 1e3, 1e5) == 5_505_505

"""Seeded synthetic inputs: box meshes, rigid motions, smooth deformations, materials.

A module of its own, shared by the CPU oracle's tests and by the GPU path's tests and
benchmark.  It holds none of the method's arithmetic (no shape-function
gradients, no kinematics, no stress): it only lays out reference nodes and
connectivity, draws seeded states, and converts engineering material constants
into the paper's parameters.

Conventions
-----------
* Nodal arrays are structure-of-arrays ``[3][n_nodes]`` float64 (the columns
  of the paper's N(t) matrix, Sec. 2.1, stored row by row).
* Connectivity is ``[n_elem][nen]`` int32, 0-based.
* T10 local node order follows the paper's node table (App. A, 10-node
  tetrahedron): corners 1-4 at parent (0,0,0), (1,0,0), (0,1,0), (0,0,1),
  then mid-edge nodes 5:(1,2) 6:(2,3) 7:(1,3) 8:(1,4) 9:(2,4) 10:(3,4).
* H8 (not in the paper) uses the paper's Q27 lexicographic convention with
  i fastest on the parent cube [-1,1]^3: (-1,-1,-1), (1,-1,-1), (-1,1,-1),
  (1,1,-1), then the same four at zeta=+1.
* Material rows, always 5 per element: SVK (lambda, mu, 0, mu_v, lambda_v);
  Neo-Hookean / Mooney-Rivlin (mu10, mu01, k, mu_v, lambda_v).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

T10, H8, Q27 = 0, 1, 2
SVK, MR, NH = 0, 1, 2
NEN = {T10: 10, H8: 8, Q27: 27}
NQ = {T10: 5, H8: 8, Q27: 27}
ELEM_NAMES = {T10: "T10", H8: "H8", Q27: "Q27"}
LAW_NAMES = {SVK: "SVK", MR: "MR", NH: "NH"}
NPAR = 5

# Kuhn (Freudenthal) split of the unit cube into 6 tetrahedra along the main
# diagonal: corner path 0 -> e_p0 -> e_p0+e_p1 -> (1,1,1) for every axis
# permutation p.  Odd permutations are re-ordered (swap of the 2nd and 3rd
# corner) so every tetrahedron is positively oriented.
_PERMS = [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)]
_ODD = [False, False, False, True, True, True]


def _kuhn_corners():
    """Return int array [6][4][3] of cube-corner offsets (0/1) per tet."""
    out = np.zeros((6, 4, 3), dtype=np.int64)
    for t, (p, odd) in enumerate(zip(_PERMS, _ODD)):
        c = [np.zeros(3, np.int64)]
        cur = np.zeros(3, np.int64)
        for ax in p:
            cur = cur.copy()
            cur[ax] = 1
            c.append(cur)
        if odd:
            c[1], c[2] = c[2], c[1]
        out[t] = np.array(c)
    return out


_KUHN = _kuhn_corners()
# T10 mid-edge node k (5..10 in the paper's 1-based numbering) sits between
# these two corners (0-based corner indices).
_T10_EDGES = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]


def box_t10(nx, ny, nz, size=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Structured box of nx*ny*nz cells, each split into 6 straight-sided T10.

    Nodes are the half-cell lattice (2nx+1)(2ny+1)(2nz+1): cell corners,
    edge midpoints, face centres and cell centres (every one of these is the
    midpoint of some tetrahedron edge of the Kuhn split).
    Returns (X [3][n_nodes] float64, conn [6*nx*ny*nz][10] int32).
    """
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    # node id = I + NX*(J + NY*K): flatten in Fortran order of (I, J, K)
    I = I.ravel(order="F"); J = J.ravel(order="F"); K = K.ravel(order="F")
    hx, hy, hz = size[0] / nx, size[1] / ny, size[2] / nz
    X = np.empty((3, NX * NY * NZ), dtype=np.float64)
    X[0] = origin[0] + 0.5 * hx * I
    X[1] = origin[1] + 0.5 * hy * J
    X[2] = origin[2] + 0.5 * hz * K

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.ravel(order="F"); cj = cj.ravel(order="F"); ck = ck.ravel(order="F")
    ncell = ci.size
    conn = np.empty((ncell, 6, 10), dtype=np.int64)
    for t in range(6):
        corners = _KUHN[t]                       # [4][3]
        dbl = np.empty((4, 3, ncell), np.int64)  # doubled lattice coords
        for a in range(4):
            dbl[a, 0] = 2 * (ci + corners[a, 0])
            dbl[a, 1] = 2 * (cj + corners[a, 1])
            dbl[a, 2] = 2 * (ck + corners[a, 2])
        pts = [dbl[a] for a in range(4)]
        for (a, b) in _T10_EDGES:
            pts.append((dbl[a] + dbl[b]) // 2)
        for n, p in enumerate(pts):
            conn[:, t, n] = p[0] + NX * (p[1] + NY * p[2])
    return X, conn.reshape(ncell * 6, 10).astype(np.int32)


def fan_t10(n_elem, cell, rng):
    """``n_elem`` straight-sided T10 that share one corner, node 0, and no
    other node: node 0 is in every element (one very long slot list per tile,
    and a node shared by many tiles).  Element e is the corner tetrahedron
    (0, cell e_x, cell e_y, cell e_z) scaled by U[0.7, 1.3] and turned by a
    random rotation (positive orientation kept); the elements overlap in
    space, which the per-element kinematics do not see.
    Returns (X [3][1 + 9 n_elem] float64, conn [n_elem][10] int32)."""
    X = np.zeros((3, 1 + 9 * n_elem))
    conn = np.empty((n_elem, 10), dtype=np.int32)
    for e in range(n_elem):
        R = random_rotation(rng)
        corners = [np.zeros(3)] + [R @ (cell * rng.uniform(0.7, 1.3) * np.eye(3)[k]) for k in range(3)]
        ids = [0] + [1 + 9 * e + k for k in range(9)]
        pts = corners + [0.5 * (corners[a] + corners[b]) for (a, b) in _T10_EDGES]
        for n in range(1, 10):
            X[:, ids[n]] = pts[n]
        conn[e] = ids
    return X, conn


def box_h8(nx, ny, nz, size=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Structured box of nx*ny*nz H8 cells (node order: lexicographic, i fastest)."""
    NX, NY, NZ = nx + 1, ny + 1, nz + 1
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    I = I.ravel(order="F"); J = J.ravel(order="F"); K = K.ravel(order="F")
    X = np.empty((3, NX * NY * NZ), dtype=np.float64)
    X[0] = origin[0] + size[0] / nx * I
    X[1] = origin[1] + size[1] / ny * J
    X[2] = origin[2] + size[2] / nz * K
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.ravel(order="F"); cj = cj.ravel(order="F"); ck = ck.ravel(order="F")
    conn = np.empty((ci.size, 8), dtype=np.int64)
    n = 0
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                conn[:, n] = (ci + di) + NX * ((cj + dj) + NY * (ck + dk))
                n += 1
    return X, conn.astype(np.int32)


def box_q27(nx, ny, nz, size=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Structured box of nx*ny*nz Q27 cells on the half-cell lattice
    (2nx+1)(2ny+1)(2nz+1); element node (i, j, k) in {0,1,2}^3 is node
    i + 3 j + 9 k of the element (lexicographic, i fastest: the paper's Q27
    node table)."""
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    I = I.ravel(order="F"); J = J.ravel(order="F"); K = K.ravel(order="F")
    X = np.empty((3, NX * NY * NZ), dtype=np.float64)
    X[0] = origin[0] + size[0] / (2 * nx) * I
    X[1] = origin[1] + size[1] / (2 * ny) * J
    X[2] = origin[2] + size[2] / (2 * nz) * K
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.ravel(order="F"); cj = cj.ravel(order="F"); ck = ck.ravel(order="F")
    conn = np.empty((ci.size, 27), dtype=np.int64)
    n = 0
    for dk in range(3):
        for dj in range(3):
            for di in range(3):
                conn[:, n] = (2 * ci + di) + NX * ((2 * cj + dj) + NY * (2 * ck + dk))
                n += 1
    return X, conn.astype(np.int32)


def random_rotation(rng):
    """Uniform rotation on SO(3) from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def sinusoidal_state(X, amp, rng, lengths=None):
    """x = R (X + u(X)) + t with a smooth sinusoidal u of peak gradient ``amp``.

    u_i = amp * sum_k c_ik * L_k / (2 pi) * sin(2 pi X_k / L_k + phi_ik), with
    c_ik ~ U[-1, 1] scaled so that max_i sum_k |c_ik| = 1 (every entry of the
    displacement gradient stays below ``amp``).  The gradient is a full
    matrix, so the deformation has a volumetric part of first order in
    ``amp`` (a field coupling each component to one other coordinate only
    would be isochoric to third order and leave J - 1 ~ amp^3).
    R uniform on SO(3), t ~ N(0, 1 m).
    """
    if lengths is None:
        lengths = X.max(axis=1) - X.min(axis=1)
    lengths = np.maximum(np.asarray(lengths, dtype=np.float64), 1e-12)
    c = rng.uniform(-1.0, 1.0, (3, 3))
    c /= np.abs(c).sum(axis=1).max()
    phi = rng.uniform(0.0, 2 * np.pi, (3, 3))
    u = np.zeros_like(X)
    for i in range(3):
        for k in range(3):
            L = lengths[k]
            u[i] += amp * c[i, k] * L / (2 * np.pi) * np.sin(2 * np.pi * X[k] / L + phi[i, k])
    R = random_rotation(rng)
    t = rng.standard_normal(3)
    return R @ (X + u) + t[:, None]


def lame_from_E_nu(E, nu):
    """(lambda, mu) from Young's modulus and Poisson's ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def nh_from_lame(mu, lam):
    """Paper-form Neo-Hookean (mu10, k) whose small-strain shear and bulk
    moduli equal the given Lame pair: mu10 = mu/2, k = lambda + 2 mu / 3."""
    return 0.5 * mu, lam + 2.0 * mu / 3.0


@dataclass
class Block:
    elem: int
    law: int
    conn: np.ndarray            # [n_elem][nen] int32, global node ids
    theta: np.ndarray           # [5] default parameters
    damped: bool = False
    theta_e: np.ndarray | None = None   # optional [5][n_elem] per-element parameters
    rho: float = 0.0                    # reference density (kg/m^3), for inertia

    @property
    def n_elem(self):
        return int(self.conn.shape[0])

    @property
    def n_qp(self):
        return self.n_elem * NQ[self.elem]


@dataclass
class Problem:
    name: str
    X: np.ndarray               # [3][n_nodes]
    x: np.ndarray               # [3][n_nodes]
    v: np.ndarray               # [3][n_nodes]
    blocks: list = field(default_factory=list)
    w: np.ndarray | None = None     # cotangent for the adjoint, [3][n_nodes]
    dx: np.ndarray | None = None    # tangent direction in x, [3][n_nodes]
    dv: np.ndarray | None = None    # tangent direction in v, [3][n_nodes]
    body_nodes: list | None = None  # per body (node_begin, node_end) when batched
    cell: float = 0.01

    @property
    def n_nodes(self):
        return int(self.X.shape[1])

    @property
    def n_elem(self):
        return sum(b.n_elem for b in self.blocks)

    @property
    def n_qp(self):
        return sum(b.n_qp for b in self.blocks)

    def renumbered(self, order):
        """The same problem with node k of the result = node order[k] of this
        one (X, connectivity and every nodal array permuted)."""
        import copy as _copy
        order = np.asarray(order, dtype=np.int64)
        inv = np.empty_like(order)
        inv[order] = np.arange(order.size)
        p = _copy.copy(self)
        for name in ("X", "x", "v", "w", "dx", "dv"):
            a = getattr(self, name)
            if a is not None:
                setattr(p, name, np.ascontiguousarray(a[:, order]))
        p.blocks = []
        for b in self.blocks:
            nb = _copy.copy(b)
            nb.conn = np.ascontiguousarray(inv[b.conn].astype(np.int32))
            p.blocks.append(nb)
        p.body_nodes = None
        return p

    def theta_all(self):
        """Per-element parameters [5][n_elem] over the concatenated blocks."""
        cols = []
        for b in self.blocks:
            if b.theta_e is not None:
                cols.append(b.theta_e)
            else:
                cols.append(np.repeat(b.theta[:, None], b.n_elem, axis=1))
        return np.ascontiguousarray(np.concatenate(cols, axis=1))


def _theta(law, p0, p1, p2, mu_v=0.0, lam_v=0.0):
    return np.array([p0, p1, p2, mu_v, lam_v], dtype=np.float64)


def config_c1(seed=1001):
    """Cantilever 1.0 x 0.1 x 0.1 m, 10x2x2 cells -> 240 T10, SVK + Kelvin-Voigt."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    X, conn = box_t10(10, 2, 2, size=(1.0, 0.1, 0.1))
    lam, mu = lame_from_E_nu(1e7, 0.3)
    x = X + rng.normal(0.0, 0.01 * 0.05, X.shape)
    v = rng.normal(0.0, 0.01, X.shape)
    blk = Block(T10, SVK, conn, _theta(SVK, lam, mu, 0.0, 1e4, 0.0), damped=True)
    return Problem("C1-cantilever-240-T10-SVK-KV", X, x, v, [blk], cell=0.05)


def config_box_nh(nx, ny, nz, seed, cell=0.01, damped=True, per_elem=False,
                  name=None, amp=0.02):
    """Box of T10 cells under a rigid motion + smooth sinusoid (Neo-Hookean)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    X, conn = box_t10(nx, ny, nz, size=(nx * cell, ny * cell, nz * cell))
    x = sinusoidal_state(X, amp, rng)
    v = rng.normal(0.0, 0.01, X.shape) if damped else np.zeros_like(X)
    mu10, k = nh_from_lame(3.4e6, 1.5e7)
    th = _theta(NH, mu10, 0.0, k, 1e4 if damped else 0.0, 0.0)
    theta_e = None
    if per_elem:
        ne = conn.shape[0]
        mu_e = np.exp(rng.uniform(math.log(1e5), math.log(1e7), ne))
        lam_e = np.exp(rng.uniform(math.log(1e5), math.log(1e7), ne))
        m10, kk = nh_from_lame(mu_e, lam_e)
        theta_e = np.zeros((NPAR, ne))
        theta_e[0] = m10
        theta_e[2] = kk
    blk = Block(T10, NH, conn, th, damped=damped, theta_e=theta_e)
    prob = Problem(name or f"box-{nx}x{ny}x{nz}-T10-NH", X, x, v, [blk], cell=cell)
    if per_elem:
        prob.w = rng.standard_normal(X.shape)
        prob.dx = rng.standard_normal(X.shape) * cell
    return prob


def config_c2(seed=1002):
    """1,020,000 T10 elements (100x100x17 cells of 1 cm), NH + Kelvin-Voigt."""
    p = config_box_nh(100, 100, 17, seed, damped=True, name="C2-1M-T10-NH-KV")
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    p.w = rng.standard_normal(p.X.shape)
    return p


def config_box_q27(nx, ny, nz, seed, cell=0.01, damped=True, name=None, amp=0.02):
    """Box of Q27 cells under a rigid motion + smooth sinusoid (Neo-Hookean
    with the C2 moduli, Kelvin-Voigt when damped), with a cotangent w and
    directions dx, dv."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    X, conn = box_q27(nx, ny, nz, size=(nx * cell, ny * cell, nz * cell))
    x = sinusoidal_state(X, amp, rng)
    v = rng.normal(0.0, 0.01, X.shape) if damped else np.zeros_like(X)
    mu10, k = nh_from_lame(3.4e6, 1.5e7)
    th = _theta(NH, mu10, 0.0, k, 1e4 if damped else 0.0, 0.0)
    blk = Block(Q27, NH, conn, th, damped=damped)
    prob = Problem(name or f"box-{nx}x{ny}x{nz}-Q27-NH", X, x, v, [blk], cell=cell)
    prob.w = rng.standard_normal(X.shape)
    prob.dx = rng.standard_normal(X.shape) * cell
    prob.dv = rng.standard_normal(X.shape)
    return prob


def config_q27(seed=1027):
    """131,072 Q27 elements (64x64x32 cells of 1 cm, 1,081,665 nodes,
    3,538,944 points), Neo-Hookean + Kelvin-Voigt as the 1M-element T10 box."""
    return config_box_q27(64, 64, 32, seed, damped=True, name="Q27-131k-NH-KV")


def config_c4(seed=1004):
    """204,000 T10 elements (50x40x17 cells), NH with per-element (mu, lambda)."""
    return config_box_nh(50, 40, 17, seed, damped=False, per_elem=True,
                         name="C4-204k-T10-NH-per-element")


def _body_dims(cells):
    b = max(1, int(round((cells / 4.0) ** (1.0 / 3.0))))
    a = max(1, int(round(cells / (b * b))))
    return a, b, b


def config_multibody(n_bodies, n_min, n_max, seed, cell=0.01, name=None,
                     directions=False, max_total=None):
    """Disjoint bodies of log-uniform element count, T10 (even) / H8 (odd),
    SVK or NH at random, E ~ U[1e6,1e8], nu ~ U[0.2,0.45], random rigid
    motion plus a 1-5 % smooth deformation.  Elastic only."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    Xs, xs, blocks, spans = [], [], [], []
    base = 0
    total = 0
    for b in range(n_bodies):
        nb = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        elem = T10 if b % 2 == 0 else H8
        cells = max(1.0, nb / 6.0) if elem == T10 else max(1.0, nb)
        a, bb, cc = _body_dims(cells)
        if elem == T10:
            X, conn = box_t10(a, bb, cc, size=(a * cell, bb * cell, cc * cell))
        else:
            X, conn = box_h8(a, bb, cc, size=(a * cell, bb * cell, cc * cell))
        law = SVK if rng.uniform() < 0.5 else NH
        E = rng.uniform(1e6, 1e8)
        nu = rng.uniform(0.2, 0.45)
        lam, mu = lame_from_E_nu(E, nu)
        if law == SVK:
            th = _theta(SVK, lam, mu, 0.0)
        else:
            m10, k = nh_from_lame(mu, lam)
            th = _theta(NH, m10, 0.0, k)
        amp = rng.uniform(0.01, 0.05)
        x = sinusoidal_state(X, amp, rng)
        Xs.append(X); xs.append(x)
        blocks.append(Block(elem, law, (conn + base).astype(np.int32), th, damped=False))
        spans.append((base, base + X.shape[1]))
        base += X.shape[1]
        total += conn.shape[0]
        if max_total is not None and total >= max_total:
            break
    X = np.ascontiguousarray(np.concatenate(Xs, axis=1))
    x = np.ascontiguousarray(np.concatenate(xs, axis=1))
    v = np.zeros_like(X)
    p = Problem(name or f"multibody-{len(blocks)}", X, x, v, blocks, body_nodes=spans, cell=cell)
    if directions:
        p.w = rng.standard_normal(X.shape)
        p.dx = rng.standard_normal(X.shape) * cell
    return p


def config_c3(seed=1003):
    """512 bodies, 200-50k elements each, mixed T10/H8 and SVK/NH."""
    return config_multibody(512, 200, 5e4, seed, name="C3-512-bodies")


def config_c5(seed=1005):
    """256 bodies, 1k-100k elements each, mixed T10/H8 and SVK/NH, with w and dx."""
    return config_multibody(256, 1e3, 1e5, seed, name="C5-256-bodies", directions=True)


def perturbed(X, sigma, rng):
    """Reference nodes plus N(0, sigma) noise (curved current elements)."""
    return X + rng.normal(0.0, sigma, X.shape)


def curve_midside_t10(X, conn, frac, rng):
    """Move T10 mid-edge nodes off their edge midpoints (curved reference
    elements, non-affine parent-to-reference map) by ``frac`` of the local
    edge length.  Returns a new X; corner nodes are untouched."""
    X = X.copy()
    mids = np.unique(conn[:, 4:].ravel())
    c0 = np.unique(conn[:, :4].ravel())
    mids = np.setdiff1d(mids, c0)
    e = np.linalg.norm(X[:, conn[:, 1]] - X[:, conn[:, 0]], axis=0).min()
    X[:, mids] += rng.uniform(-frac * e, frac * e, (3, mids.size))
    return X

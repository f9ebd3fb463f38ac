/*
 * tlfea.h -- C ABI of the MI355X (gfx950) Total Lagrangian internal-force
 * library.
 *
 * The library evaluates, for every element and quadrature point of a mesh,
 * the deformation gradient F = sum_a x_a h_a^T (Sec. 2.1, compact map
 * r = N s and F = N H), the first Piola-Kirchhoff stress P = dpsi/dF of a
 * St. Venant-Kirchhoff or Mooney-Rivlin / Neo-Hookean law plus the
 * Kelvin-Voigt viscous stress F S_v(Edot) (Sec. 3.2), and assembles the nodal
 * internal forces f_a = int P h_a dV_r (Sec. 4.3, the constitutive-
 * discretisation interface) by parent-element quadrature with the
 * isoparametric chain rule h_a^T = ds_a/dxi [U G]^{-1}, J_p = det(U G) > 0
 * (Sec. 6).  It also provides the adjoint (vector-Jacobian) product of f with
 * respect to nodal positions, velocities and per-element material parameters,
 * and the tangent product (df/dx) dx + (df/dv) dv, whose element blocks are
 * the consistent linearisations of App. C (plus the Kelvin-Voigt blocks,
 * which the paper does not print).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Floating point is IEEE binary64 throughout; indices are int32.
 * - Nodal arrays (X, x, v, f, w, gx, gv, dx, dv, df) are structure-of-arrays
 *   [3][n_nodes]: component c of node n is at [c * n_nodes + n].  These are
 *   the rows of the paper's N(t) (Sec. 2.1).
 * - Per-element parameter arrays (theta, gtheta) are [5][n_elem] in the
 *   caller's element order (blocks concatenated in creation order).  Rows:
 *     SVK : (lambda, mu, unused, mu_v, lambda_v)          (Sec. 3.2.1/3.2.3)
 *     MR  : (mu10, mu01, k, mu_v, lambda_v)               (Sec. 3.2.2/3.2.3)
 *     NH  : (mu10, unused, k, mu_v, lambda_v); Mooney-Rivlin with mu01 = 0.
 *   Rows marked unused, and rows 3-4 of an undamped block, are ignored on
 *   input and written as 0 in gtheta.
 * - tlfea_create_mesh takes HOST pointers and copies everything it keeps;
 *   the compute calls take DEVICE pointers (memory of the device that was
 *   current at creation) and a hipStream_t passed as void* (NULL = the null
 *   stream).  Compute calls only enqueue work and return; results are ready
 *   when the stream reaches that point.
 * - Outputs are overwritten, never accumulated.  An output may not overlap
 *   an input or another output (checked on the host from the array sizes;
 *   an overlap returns TLFEA_E_INVALID before any device work).
 * - A mesh holds device scratch for partial node sums: calls on one mesh must
 *   not overlap in time (issue them on one stream, or synchronise).
 * - A TLFEA_BATCHED mesh records each call's launches (one per tile class,
 *   then the shared-node sum) into a hipGraph the first time it sees that
 *   operation with those operand pointers on that stream, and replays it
 *   afterwards.  It keeps eight graphs.  With all eight in use, new operand
 *   pointers update the least recently used graph of the same operation and
 *   stream in place, after that graph's last launch has finished (only the
 *   kernel arguments differ); otherwise the least recently used graph is
 *   evicted, again after its last launch.  On the null stream, or
 *   on a stream the caller is capturing, the launches are issued directly
 *   (the caller's graph then holds them).
 * - Every function returns a tlfea_status; nothing throws.  On a non-OK
 *   status tlfea_last_error() gives a message (thread-local).  Argument
 *   checks happen on the host before any device work is enqueued.
 */
#ifndef TLFEA_H
#define TLFEA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlfea_mesh tlfea_mesh;   /* opaque, immutable geometry */

typedef enum {
    TLFEA_OK = 0,
    TLFEA_E_INVALID = -1,        /* null pointer, unknown enum or flag        */
    TLFEA_E_SHAPE = -2,          /* inconsistent sizes, node id out of range  */
    TLFEA_E_REF_JACOBIAN = -3,   /* J_p <= 0 at a quadrature point (Sec. 6)   */
    TLFEA_E_NOMEM = -4,          /* host or device allocation failed          */
    TLFEA_E_DEVICE = -5,         /* HIP runtime error (also a prior fault)    */
    TLFEA_E_UNSUPPORTED = -6     /* valid request the library does not handle */
} tlfea_status;

enum { TLFEA_T10 = 0, TLFEA_H8 = 1, TLFEA_Q27 = 2 };   /* element types   */
enum { TLFEA_SVK = 0, TLFEA_MR = 1, TLFEA_NH = 2 };  /* constitutive laws  */
enum { TLFEA_NPAR = 5 };                         /* parameter rows          */

/* tlfea_create_mesh flags (bitwise or) */
enum {
    TLFEA_PLAIN = 0,
    TLFEA_BATCHED = 1,      /* replay each call's launches as one hipGraph    */
    TLFEA_AUTOTUNE = 2,     /* time tile sizes at creation, keep one per type */
    TLFEA_KEEP_ORDER = 4    /* keep the caller's element order (no reorder)  */
};

/*
 * One block: elements of one type and one law (one body, or a part of one).
 * T10 node order follows the paper's node table (App. A, 10-node
 * tetrahedron): corners at parent (0,0,0), (1,0,0), (0,1,0), (0,0,1), then
 * mid-edge nodes 1-2, 2-3, 1-3, 1-4, 2-4, 3-4.  H8 (not in the paper) is the
 * trilinear hexahedron on [-1,1]^3 with nodes in the paper's Q27 convention
 * (lexicographic, i fastest).  Q27 is the paper's 27-node triquadratic
 * hexahedron (App. A): node i + 3 j + 9 k at parent (i - 1, j - 1, k - 1),
 * shape functions products of the 1-D quadratic Lagrange polynomials.
 * Quadrature of the internal force: T10 5-point degree-3 rule, H8 2x2x2
 * Gauss, Q27 3x3x3 Gauss (points in node order: q = p0 + 3 p1 + 9 p2).
 *
 * The quadrature rule is tabulated once on the parent element and reused
 * for every element (Sec. 6, approximation of integrals): nq points with
 * weights qp_w[q] and parent gradients dsdxi[q][a][k] = d s_a / d xi_k at
 * point q (for T10 the rows of the App. A gradient table evaluated at the
 * points).  Both pointers NULL (and nq 0) select the built-in rule.  A given
 * table must be the built-in rule to rounding (every entry within 1e-14 of
 * the largest entry's magnitude, points in the built-in order): the kernels
 * carry the rule as compile-time constants, so any other rule is refused
 * with TLFEA_E_UNSUPPORTED.  The tables are read during tlfea_create_mesh
 * only.
 */
typedef struct {
    int32_t elem;            /* TLFEA_T10, TLFEA_H8 or TLFEA_Q27               */
    int32_t law;             /* TLFEA_SVK, TLFEA_MR or TLFEA_NH                */
    int64_t n_elem;          /* elements in this block, >= 0                   */
    const int32_t *conn;     /* HOST [n_elem][nen], 0-based global node ids    */
    double theta[5];         /* default parameter rows (used when theta==NULL) */
    int32_t damped;          /* nonzero: Kelvin-Voigt branch active            */
    int32_t tile_elems;      /* elements per tile: 0 = default, else 64/128/192/256
                                (Q27: 64 or 128)                               */
    int32_t nq;              /* points of qp_w / dsdxi (0 when both are NULL)  */
    int32_t reserved;        /* must be 0                                      */
    const double *qp_w;      /* HOST [nq] quadrature weights, or NULL          */
    const double *dsdxi;     /* HOST [nq][nen][3] parent gradients, or NULL    */
    double rho;              /* reference density rho_r >= 0 (Sec. 4.1); used by
                                the mass action and the step residual only     */
} tlfea_block;

typedef struct {
    int64_t n_nodes, n_elem, n_qp;
    int64_t n_tiles, n_halo_nodes, n_partials;
    int32_t n_blocks, flags;
    int32_t tile_elems_t10, tile_elems_h8;   /* chosen (autotuned) tile sizes  */
    int32_t tile_elems_q27, reserved;
    int64_t device_bytes;                    /* device memory the mesh holds   */
    int64_t graphs_built, graphs_updated;    /* TLFEA_BATCHED: graphs instantiated,
                                                and cached ones updated in place */
} tlfea_mesh_info;

/*
 * Build a mesh on the current HIP device.  X_ref is HOST [3][n_nodes]
 * (reference nodes U, Sec. 6); blocks[b].conn is HOST.  Validation (ids in
 * range, finite coordinates, J_p > 0 at every quadrature point of every
 * element, Sec. 6) runs on the host before any device allocation; failures
 * return TLFEA_E_SHAPE / TLFEA_E_REF_JACOBIAN / TLFEA_E_INVALID /
 * TLFEA_E_UNSUPPORTED and leave *out NULL.  The mesh reorders elements along
 * a Morton curve (unless TLFEA_KEEP_ORDER) and cuts them into tiles; this
 * never changes the caller-visible order of theta / gtheta.  The tile lists
 * use 32-bit offsets: a mesh that would need more entries (about 200
 * million T10 elements) returns TLFEA_E_UNSUPPORTED, and such a problem is
 * split over several meshes.  Device uploads (and the autotuner's timing
 * launches) are issued on `stream` (hipStream_t as void*, NULL = the null
 * stream), which is synchronised before the call returns.  Ownership: the
 * caller keeps its inputs; release the mesh with tlfea_destroy_mesh.
 */
tlfea_status tlfea_create_mesh(int64_t n_nodes, const double *X_ref, int32_t n_blocks,
                               const tlfea_block *blocks, int32_t flags, void *stream,
                               tlfea_mesh **out);

/* Free the mesh and its device memory (NULL is a no-op).  Synchronises the
 * device first so no enqueued call still uses it. */
void tlfea_destroy_mesh(tlfea_mesh *mesh);

/* Sizes and the tiling the mesh chose. */
tlfea_status tlfea_get_mesh_info(const tlfea_mesh *mesh, tlfea_mesh_info *info);

/*
 * Internal force f = f_int(x, v) (Sec. 4.3, f_i = int P h_i dV_r; with
 * Kelvin-Voigt f = f^e + f^v).  x: DEVICE [3][n_nodes] current positions
 * (Sec. 2.1, columns of N(t)); v: DEVICE [3][n_nodes] velocities (columns of
 * Ndot), may be NULL when no block is damped; theta: DEVICE [5][n_elem] or
 * NULL for the blocks' defaults; f: DEVICE [3][n_nodes], overwritten (nodes
 * no element touches get 0).  Sign: f enters the residual with +
 * (Sec. 7), i.e. f = +dPi/dx.
 */
tlfea_status tlfea_internal_force(tlfea_mesh *mesh, const double *x, const double *v,
                                  const double *theta, double *f, void *stream);

/*
 * Adjoint product of the internal force for a cotangent w (DEVICE [3][n_nodes]):
 *   gx = (df/dx)^T w, gv = (df/dv)^T w   (DEVICE [3][n_nodes], each may be NULL)
 *   gtheta[p][e] = w . df/dtheta[p][e]   (DEVICE [5][n_elem], may be NULL)
 * The element blocks are those of App. C; F is recomputed from x, not stored.
 * For undamped blocks gv gets no contribution.
 */
tlfea_status tlfea_internal_force_vjp(tlfea_mesh *mesh, const double *x, const double *v,
                                      const double *theta, const double *w, double *gx,
                                      double *gv, double *gtheta, void *stream);

/*
 * Tangent product df = (df/dx) dx + (df/dv) dv + (df/dtheta) dtheta (App. C
 * consistent linearisation, K_t = df_int/dq of Sec. 7, plus the
 * Kelvin-Voigt blocks).  The stress is linear in every parameter row
 * (Sec. 3.2: SVK in (lambda, mu), Mooney-Rivlin in (mu10, mu01, k),
 * Kelvin-Voigt in (mu_v, lambda_v)), so the parameter term is the internal
 * force evaluated with theta = dtheta; the kernels add it per quadrature
 * point.  dx, dv: DEVICE [3][n_nodes], dtheta: DEVICE [5][n_elem]; each may
 * be NULL (treated as zero); df overwritten.
 */
tlfea_status tlfea_tangent_jvp(tlfea_mesh *mesh, const double *x, const double *v,
                               const double *theta, const double *dx, const double *dv,
                               const double *dtheta, double *df, void *stream);

/*
 * Consistent-mass action y = M u (Sec. 4.1): m_ij = int rho_r s_i s_j dV_r,
 * M = [m_ij I_3] assembled over every block with its density rho (blocks
 * with rho = 0 contribute nothing).  The mass integrals use a rule exact for
 * straight-sided elements (the paper tabulates one rule per element on the
 * parent domain, Sec. 6, and does not name the mass rule): T10 the 15-point
 * degree-5 rule, H8 2x2x2 Gauss, Q27 its 3x3x3 Gauss rule; rho w_q J_p(xi_q)
 * is formed once at mesh creation.  u, y: DEVICE [3][n_nodes]; y overwritten.
 */
tlfea_status tlfea_mass_action(tlfea_mesh *mesh, const double *u, double *y, void *stream);

/*
 * Residual of the backward-Euler step of the augmented-Lagrangian
 * formulation without constraints (Sec. 7):
 *   g(v) = M (v - v_n) / h + f_int(q(v), v) - f_ext,   q(v) = q_n + h v,
 * with M the consistent mass (Sec. 4.1, as tlfea_mass_action) and f_int the
 * internal force (Sec. 4.3) at the step configuration.  q(v) is formed per
 * entry with one rounding (fused multiply-add).  q_n, v_n, v, f_ext, g:
 * DEVICE [3][n_nodes]; f_ext may be NULL (zero); theta as for
 * tlfea_internal_force; h > 0 (TLFEA_E_INVALID otherwise); g overwritten.
 * The constraint term h C_q^T (lambda + rho c) of the full residual is not
 * part of this call.
 */
tlfea_status tlfea_step_residual(tlfea_mesh *mesh, const double *q_n, const double *v_n,
                                 const double *v, double h, const double *theta,
                                 const double *f_ext, double *g, void *stream);

/*
 * The derivative of tlfea_step_residual in v applied to dv (Sec. 7, the
 * matrix-free Newton operator):
 *   y = (M / h + h K + C) dv,   K = df_int/dq, C = df_int/dv at (q(v), v),
 * K and C as in tlfea_tangent_jvp (App. C plus the Kelvin-Voigt blocks).
 * q_n, v, dv, y: DEVICE [3][n_nodes]; y overwritten; h > 0.
 */
tlfea_status tlfea_newton_operator(tlfea_mesh *mesh, const double *q_n, const double *v, double h,
                                   const double *theta, const double *dv, double *y, void *stream);

/* Krylov options and report of tlfea_newton_step. */
typedef struct {
    int32_t restart;     /* Krylov basis size m of restarted GMRES, 1..200   */
    int32_t max_iters;   /* total inner iterations, >= 1                      */
    double rtol;         /* stop when ||A dv + g|| <= rtol ||g||, >= 0        */
} tlfea_krylov_opts;

typedef struct {
    int32_t iters;       /* inner iterations (operator products) taken        */
    int32_t converged;   /* 1 when the final ||A dv + g|| <= rtol ||g||       */
    double g_norm;       /* ||g(v)||_2 (the step residual at the input v)     */
    double res_norm;     /* ||A dv + g||_2, recomputed from the final dv      */
} tlfea_krylov_info;

/* Doubles of device workspace tlfea_newton_step needs for a basis of
 * `restart` vectors: (restart + 5) * 3 n_nodes + 8192 * ceil((restart + 1) / 8)
 * + 4 (restart + 1) + 8 (the basis, four work vectors, the dot-product
 * partial sums, and one iteration's scalars). */
tlfea_status tlfea_newton_workspace(const tlfea_mesh *mesh, int32_t restart, int64_t *n_doubles);

/*
 * One matrix-free Newton-Krylov step on the step residual g(v) of Sec. 7
 * (tlfea_step_residual): dv solves (M/h + h K + C) dv = -g(v) by restarted
 * GMRES (Saad and Schultz) from dv = 0, every operator product one
 * tlfea_newton_operator pass, classical Gram-Schmidt applied twice, the
 * small least-squares problem by Givens rotations on the host; the dot
 * products are summed in a fixed order, so the result is bitwise
 * repeatable.  v_out = v + dv (DEVICE [3][n_nodes], overwritten).  work:
 * DEVICE workspace of at least tlfea_newton_workspace doubles, owned by the
 * caller, contents undefined on return.  info (HOST) reports the
 * iterations, convergence and residual norms.  The call synchronises the
 * stream (the solver's scalars live on the host); not converging within
 * max_iters is not an error (info->converged = 0).
 */
tlfea_status tlfea_newton_step(tlfea_mesh *mesh, const double *q_n, const double *v_n, const double *v,
                               double h, const double *theta, const double *f_ext,
                               const tlfea_krylov_opts *opts, double *v_out, double *work,
                               int64_t work_len, tlfea_krylov_info *info, void *stream);

/*
 * Joint constraints (Sec. 2.2).  A material point is given by its hosting
 * element (type and node ids in the element's node order) and its parent
 * coordinates; its current position is the point evaluation r = N(t) s(xi)
 * (Sec. 2.1).  A revolute joint has points P, Q on body b and R, S, T on
 * body c, directions a = r_Q - r_P, b_1 = r_S - r_R, b_2 = r_T - r_R, and the
 * five rows
 *   c = [e_x.(r_R - r_P), e_y.(r_R - r_P), e_z.(r_R - r_P), a.b_1 - f_1, a.b_2 - f_2]
 * (three coordinate-difference rows, two dot-product-1 rows), f_j = a_0.b_j0
 * from the reference configuration.  Rows are normalised by the constant
 * weights of App. B.1: 1 for the CD rows, 1/sqrt(|a_0|^2 + |b_j0|^2) for the
 * DP1 rows: c_hat = W c, C_hat = W dc/dq.
 */
typedef struct tlfea_joints tlfea_joints;   /* opaque, immutable */

typedef struct {
    int32_t elem;           /* TLFEA_T10, TLFEA_H8 or TLFEA_Q27: the host element */
    int32_t nodes[27];      /* its node ids, element node order (first nen used)  */
    double xi[3];           /* parent coordinates of the material point           */
} tlfea_point;

typedef struct {
    tlfea_point P, Q, R, S, T;
} tlfea_revolute;

/* Build a joint set on the current device from HOST inputs: X_ref
 * [3][n_nodes] (for f_j and the row weights) and the joints.  Uploads are
 * issued on `stream`, synchronised before return.  TLFEA_E_SHAPE for a node
 * out of range, TLFEA_E_INVALID for an unknown element type, a non-finite
 * coordinate or reference directions that vanish. */
tlfea_status tlfea_create_joints(int64_t n_nodes, const double *X_ref, int32_t n_joints,
                                 const tlfea_revolute *joints, void *stream, tlfea_joints **out);
void tlfea_destroy_joints(tlfea_joints *joints);

/* Row-normalised constraint values c_hat at positions q (DEVICE [3][n_nodes]);
 * c: DEVICE [n_joints][5], overwritten.  The call copies q node-major into
 * the joint set's device scratch (3 n_nodes doubles, allocated with the
 * set): calls on one joint set must not overlap in time. */
tlfea_status tlfea_joint_values(tlfea_joints *joints, const double *q, double *c, void *stream);

/*
 * The constraint term of the step residual (Sec. 2.2 residual insertion,
 * Sec. 7): g (+)= h C_hat(q)^T (lambda + rho c_hat(q)), assembled per node
 * in a fixed order (no atomics; bitwise repeatable) without forming C_hat.
 * q, g: DEVICE [3][n_nodes]; lambda: DEVICE [n_joints][5] or NULL (zero);
 * accumulate = 0 overwrites g (nodes of no joint get 0), nonzero adds to
 * it.  The joint set holds device scratch: calls on one joint set must not
 * overlap in time.
 */
tlfea_status tlfea_joint_scatter(tlfea_joints *joints, const double *q, const double *lambda, double rho,
                                 double h, double *g, int32_t accumulate, void *stream);

/*
 * tlfea_internal_force for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, and harnesses that
 * forbid allocation.  Same arguments, result and errors as
 * tlfea_internal_force (f overwritten, bitwise the same values), but the
 * shared-node partial sums go to a static device array of the library
 * (64 MiB per device, held from the library's first use on that device to
 * the end of the process) instead of the mesh's buffer, and the launches
 * are issued directly on `stream` (no graph of a TLFEA_BATCHED mesh, no
 * timing events), so the call performs no allocation of any kind.  A mesh
 * whose shared-node partials need more than the array (3 doubles per
 * partial, about 2.8 million partials) returns TLFEA_E_UNSUPPORTED.  Every
 * call on one device shares that array: calls that overlap in time on one
 * device (on different streams, or from different threads) race and must
 * be ordered by the caller.  No clearing is needed between calls: every
 * partial is written before it is read.
 */
tlfea_status tlfea_internal_force_noalloc(tlfea_mesh *mesh, const double *x, const double *v,
                                          const double *theta, double *f, void *stream);

/*
 * A node numbering suited to the kernels: order[k] is the caller's node that
 * should become node k (HOST int32[n_nodes], written).  Nodes held by one
 * tile only come first, tile by tile; the nodes several tiles share follow,
 * in the order of the first tile that holds them; nodes no element touches
 * come last.  The mesh is unchanged.  Renumbering X, the connectivity and
 * every nodal array once with it, and creating the mesh again from the
 * renumbered data, makes the kernels' node gathers and their stores, and the
 * shared-node sums' stores, coalesced.  The tiles and their summation order do not depend on
 * node numbers; the node each tile's coordinates are taken relative to may,
 * so results agree with those of the original numbering to rounding.
 */
tlfea_status tlfea_node_order(const tlfea_mesh *mesh, int32_t *order);

/*
 * Number of quadrature points whose current deformation gradient has
 * det F <= 0 (the element is inverted or collapsed there).  The paper
 * requires J_p > 0 of the reference map only (Sec. 6); the compute calls
 * evaluate the laws at such points anyway (J^{-2/3} stays real) and never
 * trap, and this call reports how many there are.  x: DEVICE [3][n_nodes].
 * count: DEVICE int64, overwritten (asynchronously, on the stream) with the
 * total over every block.  F is formed as in the forward; a point whose
 * det F is within rounding of 0 may be counted either way.
 */
tlfea_status tlfea_count_inverted(tlfea_mesh *mesh, const double *x, int64_t *count, void *stream);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *tlfea_last_error(void);

/*
 * Kernel timing.  When enabled, every kernel launch of a compute call is
 * bracketed by hipEvents on the call's stream.  tlfea_get_profile
 * synchronises those events and returns, per kernel id, the number of
 * launches and their summed duration in milliseconds; reset clears them.
 * Kernel ids: 0 forward tile, 1 adjoint tile, 2 tangent tile, 3 halo
 * reduction, 4 whole batched graph replay, 5 step-residual tile, 6 Newton
 * operator tile, 7 mass-action tile.  counts: HOST
 * int32[TLFEA_NUM_KERNEL_IDS], ms: HOST double[TLFEA_NUM_KERNEL_IDS]; either
 * may be NULL.
 */
#define TLFEA_NUM_KERNEL_IDS 8
tlfea_status tlfea_set_profiling(tlfea_mesh *mesh, int32_t enable);
tlfea_status tlfea_get_profile(tlfea_mesh *mesh, int32_t *counts, double *ms);
tlfea_status tlfea_reset_profile(tlfea_mesh *mesh);

#ifdef __cplusplus
}
#endif

#endif /* TLFEA_H */

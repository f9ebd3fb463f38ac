/*
 * tlfea_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial FP64 CPU implementation of the Total Lagrangian
 * internal force of Zhou, Arivoli & Negrut, "A Total Lagrangian Finite Element
 * Framework for Multibody Dynamics: Part I -- Formulation" (arXiv 2602.17002),
 * together with its energy, its element tangent blocks, and the adjoint and
 * tangent products assembled from those blocks.  It exists so that tests,
 * the smoke check and the benchmark's CPU-baseline leg can check the GPU
 * library against the paper.  Nothing in the product path may call it.
 *
 * It shares no code with the GPU library: the shape-function tables,
 * quadrature rules and constitutive formulas below are written here from the
 * paper independently of the HIP sources.
 *
 * Element types: the 10-node tetrahedron and the 27-node hexahedron of
 * App. A, and the 8-node trilinear hexahedron (not in the paper).
 *
 * Every element is processed in index order and every quadrature point in
 * table order, following the steps of the paper literally:
 *   U, N, Ndot gathered (Sec. 2.1, eq. r = N s; Sec. 6 isoparametric map),
 *     positions relative to the element's first node (exact: the parent
 *     gradients of the shape functions sum to zero, App. A)
 *   J = U G(xi_q), J_p = det J > 0, H = G J^{-1}          (Sec. 6)
 *   F = N H, Fdot = Ndot H                                  (Sec. 2.1)
 *   P = P_e(F) + F S_v(Edot)                                (Sec. 3.2, App. C)
 *   f_i += w_q J_p P h_i                                    (Sec. 4.3, Sec. 6)
 *
 * Parity status of each exported function (what pins it is in the tests):
 *   oracle_shape / oracle_dshape / oracle_quadrature  pinned
 *   oracle_stress, oracle_internal_force              pinned
 *   oracle_energy                                     pinned
 *   oracle_element_tangent, oracle_vjp, oracle_jvp    pinned
 *   oracle_count_inverted                             pinned
 *   oracle_mass_rule, oracle_element_mass,
 *   oracle_mass_action                                pinned
 *   oracle_step_residual, oracle_newton_operator      pinned
 *
 * Layouts: nodal arrays X, x, v, f, w, dx, dv are [3][n_nodes] (row c holds
 * component c of every node); conn is [n_elem][nen] (0-based); theta is
 * [5][n_elem]: SVK rows (lambda, mu, -, mu_v, lambda_v), Mooney-Rivlin rows
 * (mu10, mu01, k, mu_v, lambda_v).  Law NH is Mooney-Rivlin with mu01 = 0.
 * All nodal outputs ACCUMULATE into the caller's arrays (the caller zeroes
 * them), so several blocks can be summed into one vector.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_T10 0
#define OR_H8 1
#define OR_Q27 2
#define OR_SVK 0
#define OR_MR 1
#define OR_NH 2

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_REF_JACOBIAN (-3)

#define MAXN 27
#define MAXQ 27

/* ------------------------------------------------------------------ */
/* Element library                                                     */
/* ------------------------------------------------------------------ */

/* 10-node tetrahedron shape functions, App. A ("Shape Functions"),
 * parent coordinates (xi, eta, zeta) = (a, b, c). */
static void t10_shape(const double *p, double *s)
{
    const double a = p[0], b = p[1], c = p[2];
    s[0] = 2*b*b + 4*b*a + 4*b*c - 3*b + 2*a*a + 4*a*c - 3*a + 2*c*c - 3*c + 1;
    s[1] = 2*a*a - a;
    s[2] = 2*b*b - b;
    s[3] = 2*c*c - c;
    s[4] = -4*b*a - 4*a*a - 4*a*c + 4*a;
    s[5] = 4*b*a;
    s[6] = -4*b*b - 4*b*a - 4*b*c + 4*b;
    s[7] = -4*b*c - 4*a*c - 4*c*c + 4*c;
    s[8] = 4*a*c;
    s[9] = 4*b*c;
}

/* 10-node tetrahedron parent gradients ds_i/d(xi, eta, zeta), App. A
 * ("Shape Function Derivatives"); row i, column = parent direction. */
static void t10_dshape(const double *p, double G[][3])
{
    const double a = p[0], b = p[1], c = p[2];
    const double g0 = 4*b + 4*a + 4*c - 3;
    G[0][0] = g0;               G[0][1] = g0;               G[0][2] = g0;
    G[1][0] = 4*a - 1;          G[1][1] = 0;                G[1][2] = 0;
    G[2][0] = 0;                G[2][1] = 4*b - 1;          G[2][2] = 0;
    G[3][0] = 0;                G[3][1] = 0;                G[3][2] = 4*c - 1;
    G[4][0] = -4*b - 8*a - 4*c + 4; G[4][1] = -4*a;         G[4][2] = -4*a;
    G[5][0] = 4*b;              G[5][1] = 4*a;              G[5][2] = 0;
    G[6][0] = -4*b;             G[6][1] = -8*b - 4*a - 4*c + 4; G[6][2] = -4*b;
    G[7][0] = -4*c;             G[7][1] = -4*c;             G[7][2] = -4*b - 4*a - 8*c + 4;
    G[8][0] = 4*c;              G[8][1] = 0;                G[8][2] = 4*a;
    G[9][0] = 0;                G[9][1] = 4*c;              G[9][2] = 4*b;
}

/* 8-node trilinear hexahedron on [-1,1]^3 (not in the paper): tensor product
 * of 1-D linear Lagrange polynomials, nodes in the paper's Q27 lexicographic
 * convention (i fastest). */
static const double h8_node[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {-1, 1, 1},  {1, 1, 1}};

static void h8_shape(const double *p, double *s)
{
    for (int i = 0; i < 8; ++i)
        s[i] = 0.125 * (1 + p[0]*h8_node[i][0]) * (1 + p[1]*h8_node[i][1]) *
               (1 + p[2]*h8_node[i][2]);
}

static void h8_dshape(const double *p, double G[][3])
{
    for (int i = 0; i < 8; ++i) {
        const double a = 1 + p[0]*h8_node[i][0];
        const double b = 1 + p[1]*h8_node[i][1];
        const double c = 1 + p[2]*h8_node[i][2];
        G[i][0] = 0.125 * h8_node[i][0] * b * c;
        G[i][1] = 0.125 * a * h8_node[i][1] * c;
        G[i][2] = 0.125 * a * b * h8_node[i][2];
    }
}

/* 27-node quadratic hexahedron (App. A, Q27): node n = i + 3 j + 9 k at
 * parent (i - 1, j - 1, k - 1) (lexicographic, i fastest, the paper's node
 * table); s_n(xi, eta, zeta) = L_i(xi) L_j(eta) L_k(zeta) with the 1-D
 * quadratic Lagrange polynomials L_0(s) = s (s - 1) / 2, L_1(s) = 1 - s^2,
 * L_2(s) = s (s + 1) / 2. */
static void lagrange2(double s, double L[3], double dL[3])
{
    L[0] = 0.5 * s * (s - 1.0);
    L[1] = 1.0 - s * s;
    L[2] = 0.5 * s * (s + 1.0);
    dL[0] = s - 0.5;
    dL[1] = -2.0 * s;
    dL[2] = s + 0.5;
}

static void q27_shape(const double *p, double *s)
{
    double Lx[3], Ly[3], Lz[3], d[3];
    lagrange2(p[0], Lx, d);
    lagrange2(p[1], Ly, d);
    lagrange2(p[2], Lz, d);
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) s[i + 3*j + 9*k] = Lx[i] * Ly[j] * Lz[k];
}

static void q27_dshape(const double *p, double G[][3])
{
    double Lx[3], Ly[3], Lz[3], dx[3], dy[3], dz[3];
    lagrange2(p[0], Lx, dx);
    lagrange2(p[1], Ly, dy);
    lagrange2(p[2], Lz, dz);
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                const int n = i + 3*j + 9*k;
                G[n][0] = dx[i] * Ly[j] * Lz[k];
                G[n][1] = Lx[i] * dy[j] * Lz[k];
                G[n][2] = Lx[i] * Ly[j] * dz[k];
            }
}

/* Quadrature rules tabulated once on the parent element (Sec. 6).  The paper
 * gives no table; the T10 rule is the 5-point degree-3 rule on the unit
 * tetrahedron (centroid weight -4/5, four points at (1/6,1/6,1/6)-type
 * positions with weight 9/20, both scaled by the parent volume 1/6); H8 uses
 * the 2x2x2 Gauss-Legendre rule. */
static int rule(int elem, double pts[][3], double *w)
{
    if (elem == OR_T10) {
        const double a = 1.0/6.0, b = 0.5;
        const double P[5][3] = {{0.25, 0.25, 0.25}, {a, a, a}, {b, a, a}, {a, b, a}, {a, a, b}};
        for (int q = 0; q < 5; ++q) {
            pts[q][0] = P[q][0]; pts[q][1] = P[q][1]; pts[q][2] = P[q][2];
            w[q] = (q == 0 ? -4.0/5.0 : 9.0/20.0) / 6.0;
        }
        return 5;
    }
    if (elem == OR_Q27) {
        /* 3x3x3 Gauss-Legendre: points 0, +-sqrt(3/5), weights 8/9, 5/9 */
        const double g = sqrt(0.6), pt[3] = {-g, 0.0, g}, wt[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
        int q = 0;
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) {
                    pts[q][0] = pt[i]; pts[q][1] = pt[j]; pts[q][2] = pt[k];
                    w[q] = wt[i] * wt[j] * wt[k];
                    ++q;
                }
        return 27;
    }
    if (elem == OR_H8) {
        const double g = 1.0 / sqrt(3.0);
        int q = 0;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) {
                    pts[q][0] = i ? g : -g;
                    pts[q][1] = j ? g : -g;
                    pts[q][2] = k ? g : -g;
                    w[q] = 1.0;
                    ++q;
                }
        return 8;
    }
    return 0;
}

static int nen_of(int elem) { return elem == OR_T10 ? 10 : (elem == OR_H8 ? 8 : (elem == OR_Q27 ? 27 : 0)); }

static void dshape(int elem, const double *p, double G[][3])
{
    if (elem == OR_T10) t10_dshape(p, G);
    else if (elem == OR_H8) h8_dshape(p, G);
    else q27_dshape(p, G);
}

/* ------------------------------------------------------------------ */
/* 3x3 helpers                                                          */
/* ------------------------------------------------------------------ */

static double det3(double A[3][3])
{
    return A[0][0]*(A[1][1]*A[2][2] - A[1][2]*A[2][1])
         - A[0][1]*(A[1][0]*A[2][2] - A[1][2]*A[2][0])
         + A[0][2]*(A[1][0]*A[2][1] - A[1][1]*A[2][0]);
}

/* inverse by the adjugate: A^{-1} = adj(A) / det(A) */
static void inv3(double A[3][3], double d, double R[3][3])
{
    R[0][0] =  (A[1][1]*A[2][2] - A[1][2]*A[2][1]) / d;
    R[0][1] = -(A[0][1]*A[2][2] - A[0][2]*A[2][1]) / d;
    R[0][2] =  (A[0][1]*A[1][2] - A[0][2]*A[1][1]) / d;
    R[1][0] = -(A[1][0]*A[2][2] - A[1][2]*A[2][0]) / d;
    R[1][1] =  (A[0][0]*A[2][2] - A[0][2]*A[2][0]) / d;
    R[1][2] = -(A[0][0]*A[1][2] - A[0][2]*A[1][0]) / d;
    R[2][0] =  (A[1][0]*A[2][1] - A[1][1]*A[2][0]) / d;
    R[2][1] = -(A[0][0]*A[2][1] - A[0][1]*A[2][0]) / d;
    R[2][2] =  (A[0][0]*A[1][1] - A[0][1]*A[1][0]) / d;
}

static void mul(double A[3][3], double B[3][3], double R[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
            R[i][j] = s;
        }
}

static void transpose(double A[3][3], double R[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = A[j][i];
}

static double trace(double A[3][3]) { return A[0][0] + A[1][1] + A[2][2]; }

static double ddot(double A[3][3], double B[3][3])
{
    double s = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += A[i][j] * B[i][j];
    return s;
}

static void matvec(double A[3][3], const double *x, double *y)
{
    for (int i = 0; i < 3; ++i) y[i] = A[i][0]*x[0] + A[i][1]*x[1] + A[i][2]*x[2];
}

static double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }

/* ------------------------------------------------------------------ */
/* Constitutive laws (Sec. 3.2, App. C)                                 */
/* ------------------------------------------------------------------ */

/* Material parameters of one element. */
typedef struct {
    int law, damped;
    double p0, p1, p2;     /* SVK: lambda, mu, -;  MR/NH: mu10, mu01, k */
    double mu_v, lam_v;    /* Kelvin-Voigt */
} mat_t;

static mat_t mat_of(int law, int damped, const double *theta, int64_t n_elem, int64_t e)
{
    mat_t m;
    m.law = law; m.damped = damped;
    m.p0 = theta[0*n_elem + e];
    m.p1 = theta[1*n_elem + e];
    m.p2 = theta[2*n_elem + e];
    m.mu_v = damped ? theta[3*n_elem + e] : 0.0;
    m.lam_v = damped ? theta[4*n_elem + e] : 0.0;
    if (law == OR_NH) m.p1 = 0.0;
    return m;
}

/* Elastic first Piola-Kirchhoff stress.
 * SVK: the expanded form P = lambda (tr(F^T F)/2 - 3/2) F + mu F F^T F - mu F
 *      (App. C, SVK, expanded first Piola-Kirchhoff stress; also Sec. 3.2.1).
 * MR : P = 2 mu10 J^{-2/3} (F - I1/3 F^{-T})
 *        + 2 mu01 J^{-4/3} (I1 F - F C - 2/3 I2 F^{-T}) + k (J-1) J F^{-T}
 *      (Sec. 3.2.2 and App. C, Mooney-Rivlin first Piola-Kirchhoff stress). */
static void elastic_P(const mat_t *m, double F[3][3], double P[3][3])
{
    double Ft[3][3], C[3][3];
    transpose(F, Ft);
    mul(Ft, F, C);
    if (m->law == OR_SVK) {
        const double lam = m->p0, mu = m->p1;
        double FFt[3][3], FFtF[3][3];
        mul(F, Ft, FFt);
        mul(FFt, F, FFtF);
        const double a = lam * (0.5 * trace(C) - 1.5);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                P[i][j] = a * F[i][j] + mu * FFtF[i][j] - mu * F[i][j];
        return;
    }
    const double mu10 = m->p0, mu01 = m->p1, k = m->p2;
    const double J = det3(F);
    double Finv[3][3], FinvT[3][3], FC[3][3], C2[3][3];
    inv3(F, J, Finv);
    transpose(Finv, FinvT);
    mul(F, C, FC);
    mul(C, C, C2);
    const double I1 = trace(C);
    const double I2 = 0.5 * (I1 * I1 - trace(C2));
    const double cb = cbrt(J);
    const double Jm23 = 1.0 / (cb * cb);        /* J^{-2/3} */
    const double Jm43 = Jm23 * Jm23;            /* J^{-4/3} */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            P[i][j] = 2*mu10*Jm23*(F[i][j] - I1/3.0*FinvT[i][j])
                    + 2*mu01*Jm43*(I1*F[i][j] - FC[i][j] - 2.0/3.0*I2*FinvT[i][j])
                    + k*(J - 1.0)*J*FinvT[i][j];
}

/* Kelvin-Voigt (Sec. 3.2.3): Edot = (Fdot^T F + F^T Fdot)/2,
 * S_v = 2 mu_v Edot + lambda_v tr(Edot) I, P_v = F S_v. */
static void viscous_Sv(const mat_t *m, double F[3][3], double Fd[3][3], double Ed[3][3], double Sv[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += Fd[k][i]*F[k][j] + F[k][i]*Fd[k][j];
            Ed[i][j] = 0.5 * s;
        }
    const double tr = trace(Ed);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Sv[i][j] = 2*m->mu_v*Ed[i][j] + (i == j ? m->lam_v*tr : 0.0);
}

/* Total P = P_e + F S_v (Sec. 3.2.3, total first Piola-Kirchhoff stress). */
static void total_P(const mat_t *m, double F[3][3], double Fd[3][3], double P[3][3])
{
    elastic_P(m, F, P);
    if (m->damped) {
        double Ed[3][3], Sv[3][3], Pv[3][3];
        viscous_Sv(m, F, Fd, Ed, Sv);
        mul(F, Sv, Pv);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) P[i][j] += Pv[i][j];
    }
}

/* Strain energy density psi(F) (SVK: Sec. 3.2.1; MR: Sec. 3.2.2) and the
 * dissipation potential phi(Edot) (Sec. 3.2.3). */
static double elastic_psi(const mat_t *m, double F[3][3])
{
    double Ft[3][3], C[3][3];
    transpose(F, Ft);
    mul(Ft, F, C);
    if (m->law == OR_SVK) {
        double E[3][3], E2[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) E[i][j] = 0.5 * (C[i][j] - (i == j));
        mul(E, E, E2);
        const double tr = trace(E);
        return 0.5 * m->p0 * tr * tr + m->p1 * trace(E2);
    }
    double C2[3][3];
    mul(C, C, C2);
    const double J = det3(F);
    const double I1 = trace(C), I2 = 0.5 * (I1 * I1 - trace(C2));
    const double cb = cbrt(J);
    const double I1b = I1 / (cb * cb), I2b = I2 / (cb * cb * cb * cb);
    return m->p0 * (I1b - 3) + m->p1 * (I2b - 3) + 0.5 * m->p2 * (J - 1) * (J - 1);
}

static double viscous_phi(const mat_t *m, double F[3][3], double Fd[3][3])
{
    double Ed[3][3], Sv[3][3];
    viscous_Sv(m, F, Fd, Ed, Sv);
    const double tr = trace(Ed);
    return m->mu_v * ddot(Ed, Ed) + 0.5 * m->lam_v * tr * tr;
}

/* ------------------------------------------------------------------ */
/* Per-element kinematics at one quadrature point (Sec. 2.1, Sec. 6)   */
/* ------------------------------------------------------------------ */

typedef struct {
    int nen, nq;
    double xi[MAXQ][3], w[MAXQ];
    double U[3][MAXN], N[3][MAXN], Nd[3][MAXN];
} elem_t;

/* J = U G, J_p = det J, h_i^T = (dG_i/dxi) J^{-1} (Sec. 6), F = N H, Fd = Nd H. */
static int qp_kinematics(const elem_t *E, int elem, int q, double H[][3], double *Jp,
                         double F[3][3], double Fd[3][3])
{
    double G[MAXN][3], J[3][3], Ji[3][3];
    dshape(elem, E->xi[q], G);
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double s = 0;
            for (int a = 0; a < E->nen; ++a) s += E->U[i][a] * G[a][k];
            J[i][k] = s;
        }
    const double d = det3(J);
    if (!(d > 0)) return OR_E_REF_JACOBIAN;     /* J_p > 0 required (Sec. 6) */
    inv3(J, d, Ji);
    for (int a = 0; a < E->nen; ++a)
        for (int k = 0; k < 3; ++k)
            H[a][k] = G[a][0]*Ji[0][k] + G[a][1]*Ji[1][k] + G[a][2]*Ji[2][k];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double s = 0, sd = 0;
            for (int a = 0; a < E->nen; ++a) {
                s += E->N[i][a] * H[a][k];
                sd += E->Nd[i][a] * H[a][k];
            }
            F[i][k] = s;
            Fd[i][k] = sd;
        }
    *Jp = d;
    return OR_OK;
}

/* The element's nodes.  Positions (U and N) are taken relative to the
 * element's first node: the shape functions sum to one (App. A), so their
 * parent gradients sum to zero and J = U G and F = N H are unchanged, while
 * the products no longer cancel coordinates of order 1 m down to strains of
 * order 1e-2 (about two digits on 1 cm elements).  The differences of nearby
 * coordinates are themselves exact in FP64 (within a factor of two). */
static void gather(elem_t *E, int64_t n_nodes, const int32_t *c, const double *X,
                   const double *x, const double *v)
{
    for (int a = 0; a < E->nen; ++a)
        for (int i = 0; i < 3; ++i) {
            E->U[i][a] = X[i*n_nodes + c[a]] - X[i*n_nodes + c[0]];
            E->N[i][a] = x[i*n_nodes + c[a]] - x[i*n_nodes + c[0]];
            E->Nd[i][a] = v ? v[i*n_nodes + c[a]] : 0.0;
        }
}

static int setup(elem_t *E, int elem)
{
    E->nen = nen_of(elem);
    if (!E->nen) return OR_E_INVALID;
    E->nq = rule(elem, E->xi, E->w);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Exported: element library probes                                    */
/* ------------------------------------------------------------------ */

int oracle_nen(int elem) { return nen_of(elem); }

int oracle_quadrature(int elem, double *xi, double *w)
{
    double p[MAXQ][3], ww[MAXQ];
    const int nq = rule(elem, p, ww);
    for (int q = 0; q < nq; ++q) {
        xi[3*q] = p[q][0]; xi[3*q+1] = p[q][1]; xi[3*q+2] = p[q][2];
        w[q] = ww[q];
    }
    return nq;
}

void oracle_shape(int elem, const double *xi, double *s)
{
    if (elem == OR_T10) t10_shape(xi, s);
    else if (elem == OR_H8) h8_shape(xi, s);
    else q27_shape(xi, s);
}

void oracle_dshape(int elem, const double *xi, double *G /* [nen][3] */)
{
    dshape(elem, xi, (double (*)[3])G);
}

/* Single-point stress: P = P_e(F) + F S_v(Edot) for one parameter set
 * theta[5]; F, Fd, P row-major 3x3. */
void oracle_stress(int law, int damped, const double *theta, const double *F_, const double *Fd_,
                   double *P_)
{
    mat_t m = mat_of(law, damped, theta, 1, 0);
    double F[3][3], Fd[3][3], P[3][3];
    memcpy(F, F_, sizeof F);
    memcpy(Fd, Fd_, sizeof Fd);
    total_P(&m, F, Fd, P);
    memcpy(P_, P, sizeof P);
}

/* Single-point energy densities psi(F) and phi(Edot). */
void oracle_density(int law, int damped, const double *theta, const double *F_, const double *Fd_,
                    double *psi, double *phi)
{
    mat_t m = mat_of(law, damped, theta, 1, 0);
    double F[3][3], Fd[3][3];
    memcpy(F, F_, sizeof F);
    memcpy(Fd, Fd_, sizeof Fd);
    *psi = elastic_psi(&m, F);
    *phi = m.damped ? viscous_phi(&m, F, Fd) : 0.0;
}

/* ------------------------------------------------------------------ */
/* Exported: internal force (Sec. 4.3, eq. f_i = int P h_i dV_r)        */
/* ------------------------------------------------------------------ */

/* Elements [e0, e1) of a block of n_elem elements (conn and theta are the
 * whole block's arrays), accumulated into f. */
static int force_range(int elem, int law, int damped, int64_t n_nodes, const double *X,
                       int64_t n_elem, const int32_t *conn, const double *theta,
                       const double *x, const double *v, double *f, int64_t e0, int64_t e1)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    for (int64_t e = e0; e < e1; ++e) {
        const int32_t *c = conn + e * E.nen;
        mat_t m = mat_of(law, damped, theta, n_elem, e);
        gather(&E, n_nodes, c, X, x, v);
        for (int q = 0; q < E.nq; ++q) {
            double H[MAXN][3], F[3][3], Fd[3][3], P[3][3], Jp;
            if (qp_kinematics(&E, elem, q, H, &Jp, F, Fd)) return OR_E_REF_JACOBIAN;
            total_P(&m, F, Fd, P);
            for (int a = 0; a < E.nen; ++a) {
                double Ph[3];
                matvec(P, H[a], Ph);
                for (int i = 0; i < 3; ++i) f[i*n_nodes + c[a]] += E.w[q] * Jp * Ph[i];
            }
        }
    }
    return OR_OK;
}

int oracle_internal_force(int elem, int law, int damped, int64_t n_nodes, const double *X,
                          int64_t n_elem, const int32_t *conn, const double *theta,
                          const double *x, const double *v, double *f)
{
    return force_range(elem, law, damped, n_nodes, X, n_elem, conn, theta, x, v, f, 0, n_elem);
}

/* Quadrature points whose current deformation gradient has det F <= 0
 * (an inverted or collapsed element there).  The paper requires J_p > 0 of
 * the reference map only (Sec. 6) and says nothing of det F; the forward
 * computes P there anyway, and this count reports such points.  Also
 * returns the smallest |det F| met, so that a test can see how far every
 * point is from the sign decision. */
int oracle_count_inverted(int elem, int64_t n_nodes, const double *X, int64_t n_elem, const int32_t *conn,
                          const double *x, int64_t *count, double *min_abs_det)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    int64_t n = 0;
    double mn = INFINITY;
    for (int64_t e = 0; e < n_elem; ++e) {
        const int32_t *c = conn + e * E.nen;
        gather(&E, n_nodes, c, X, x, NULL);
        for (int q = 0; q < E.nq; ++q) {
            double H[MAXN][3], F[3][3], Fd[3][3], Jp;
            if (qp_kinematics(&E, elem, q, H, &Jp, F, Fd)) return OR_E_REF_JACOBIAN;
            const double d = det3(F);
            if (d <= 0) ++n;
            if (fabs(d) < mn) mn = fabs(d);
        }
    }
    *count += n;
    if (min_abs_det && mn < *min_abs_det) *min_abs_det = mn;
    return OR_OK;
}

/* Discrete elastic energy Pi_h = sum_e sum_q w_q J_p psi(F_q) and
 * dissipation Phi_h = sum w_q J_p phi(Edot_q) (Sec. 3.2, Sec. 6). */
int oracle_energy(int elem, int law, int damped, int64_t n_nodes, const double *X,
                  int64_t n_elem, const int32_t *conn, const double *theta,
                  const double *x, const double *v, double *Pi, double *Phi)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    double pi = 0, ph = 0;
    for (int64_t e = 0; e < n_elem; ++e) {
        const int32_t *c = conn + e * E.nen;
        mat_t m = mat_of(law, damped, theta, n_elem, e);
        gather(&E, n_nodes, c, X, x, v);
        for (int q = 0; q < E.nq; ++q) {
            double H[MAXN][3], F[3][3], Fd[3][3], Jp;
            if (qp_kinematics(&E, elem, q, H, &Jp, F, Fd)) return OR_E_REF_JACOBIAN;
            pi += E.w[q] * Jp * elastic_psi(&m, F);
            if (m.damped) ph += E.w[q] * Jp * viscous_phi(&m, F, Fd);
        }
    }
    *Pi += pi;
    *Phi += ph;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Element tangent blocks                                               */
/* ------------------------------------------------------------------ */

/* outer product R = s a b^T accumulated */
static void add_outer(double R[3][3], double s, const double *a, const double *b)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] += s * a[i] * b[j];
}

static void add_scaled(double R[3][3], double s, double A[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] += s * A[i][j];
}

static void add_identity(double R[3][3], double s)
{
    for (int i = 0; i < 3; ++i) R[i][i] += s;
}

/* Block K_ij = d f_i / d e_j of the integrand at one point (without w J_p).
 *
 * SVK: the six terms of the consistent linearisation in App. C (SVK tangent):
 *   lam (F h_i)(F h_j)^T + lam tr(E)(h_j.h_i) I + mu (F h_j).(F h_i) I
 *   + mu (F h_j)(F h_i)^T + mu (h_j.h_i) F F^T - mu (h_j.h_i) I
 * MR : dt1 - dt2 + dt3 - dt4 - dt5 + dt6 from App. C (Mooney-Rivlin tangent).
 * Kelvin-Voigt (not printed in the paper; derived from P_v = F S_v(Edot)):
 *   (h_j^T S_v h_i) I + mu_v [(F h_j)(Fd h_i)^T + (h_j.h_i) F Fd^T]
 *   + lam_v (F h_i)(Fd h_j)^T
 * and the velocity block C_ij = d f_i / d v_j:
 *   mu_v [(h_j.h_i) F F^T + (F h_j)(F h_i)^T] + lam_v (F h_i)(F h_j)^T. */
static void tangent_block(const mat_t *m, double F[3][3], double Fd[3][3], const double *hi,
                          const double *hj, double K[3][3], double Cv[3][3])
{
    double Fhi[3], Fhj[3], FinvT[3][3], Finv[3][3], Ft[3][3], C[3][3], FFt[3][3];
    memset(K, 0, 9 * sizeof(double));
    memset(Cv, 0, 9 * sizeof(double));
    matvec(F, hi, Fhi);
    matvec(F, hj, Fhj);
    transpose(F, Ft);
    mul(Ft, F, C);
    mul(F, Ft, FFt);
    const double hh = dot3(hj, hi);
    if (m->law == OR_SVK) {
        const double lam = m->p0, mu = m->p1;
        const double trE = 0.5 * (trace(C) - 3.0);
        add_outer(K, lam, Fhi, Fhj);
        add_identity(K, lam * trE * hh);
        add_identity(K, mu * dot3(Fhj, Fhi));
        add_outer(K, mu, Fhj, Fhi);
        add_scaled(K, mu * hh, FFt);
        add_identity(K, -mu * hh);
    } else {
        const double mu10 = m->p0, mu01 = m->p1, k = m->p2;
        const double J = det3(F);
        inv3(F, J, Finv);
        transpose(Finv, FinvT);
        double C2[3][3];
        mul(C, C, C2);
        const double I1 = trace(C), I2 = 0.5 * (I1 * I1 - trace(C2));
        const double cb = cbrt(J);
        const double Jm23 = 1.0 / (cb * cb), Jm43 = Jm23 * Jm23;
        double Gi[3], Gj[3];              /* F^{-T} h_i, F^{-T} h_j */
        matvec(FinvT, hi, Gi);
        matvec(FinvT, hj, Gj);
        /* dt1 */
        double T[3][3];
        memset(T, 0, sizeof T);
        add_identity(T, hh);
        add_outer(T, -2.0/3.0, Fhi, Gj);
        add_scaled(K, 2*mu10*Jm23, T);
        /* - dt2 */
        memset(T, 0, sizeof T);
        add_outer(T, 2.0, Gi, Fhj);
        add_outer(T, -2.0/3.0*I1, Gi, Gj);
        add_outer(T, -I1, Gj, Gi);
        add_scaled(K, -2*mu10/3.0*Jm23, T);
        if (mu01 != 0.0) {
            /* + dt3 */
            memset(T, 0, sizeof T);
            add_identity(T, I1 * hh);
            add_outer(T, 2.0, Fhi, Fhj);
            add_outer(T, -4.0/3.0*I1, Fhi, Gj);
            add_scaled(K, 2*mu01*Jm43, T);
            /* - dt4 */
            double FFtFhi[3];
            matvec(FFt, Fhi, FFtFhi);
            memset(T, 0, sizeof T);
            add_identity(T, dot3(Fhj, Fhi));
            add_outer(T, 1.0, Fhj, Fhi);
            add_scaled(T, hh, FFt);
            add_outer(T, -4.0/3.0, FFtFhi, Gj);
            add_scaled(K, -2*mu01*Jm43, T);
            /* - dt5 */
            double B[3][3], rowv[3];
            memset(B, 0, sizeof B);
            add_identity(B, I1);
            add_scaled(B, -1.0, FFt);
            /* row vector 2 (F h_j)^T (I1 I - F F^T) - 4/3 I2 (F^{-T} h_j)^T */
            for (int c = 0; c < 3; ++c) {
                double s = 0;
                for (int r = 0; r < 3; ++r) s += Fhj[r] * B[r][c];
                rowv[c] = 2.0 * s - 4.0/3.0 * I2 * Gj[c];
            }
            memset(T, 0, sizeof T);
            add_outer(T, 1.0, Gi, rowv);
            add_outer(T, -I2, Gj, Gi);
            add_scaled(K, -4*mu01/3.0*Jm43, T);
        }
        /* + dt6 */
        memset(T, 0, sizeof T);
        add_outer(T, 2*J - 1, Gi, Gj);
        add_outer(T, -(J - 1), Gj, Gi);
        add_scaled(K, k*J, T);
    }
    if (m->damped) {
        double Ed[3][3], Sv[3][3], Fdhi[3], Fdhj[3], Svhi[3], FFdt[3][3], Fdt[3][3];
        viscous_Sv(m, F, Fd, Ed, Sv);
        matvec(Fd, hi, Fdhi);
        matvec(Fd, hj, Fdhj);
        matvec(Sv, hi, Svhi);
        transpose(Fd, Fdt);
        mul(F, Fdt, FFdt);
        add_identity(K, dot3(hj, Svhi));
        add_outer(K, m->mu_v, Fhj, Fdhi);
        add_scaled(K, m->mu_v * hh, FFdt);
        add_outer(K, m->lam_v, Fhi, Fdhj);
        add_scaled(Cv, m->mu_v * hh, FFt);
        add_outer(Cv, m->mu_v, Fhj, Fhi);
        add_outer(Cv, m->lam_v, Fhi, Fhj);
    }
}

/* Element blocks K^e (d f^e / d x^e) and C^e (d f^e / d v^e), both
 * [nen*3][nen*3] row-major with row index 3*i + r (node i, component r) and
 * column index 3*j + s, integrated with the element's quadrature rule. */
static int element_blocks(const elem_t *E, int elem, const mat_t *m, double *K, double *Cv)
{
    const int n3 = 3 * E->nen;
    memset(K, 0, sizeof(double) * n3 * n3);
    memset(Cv, 0, sizeof(double) * n3 * n3);
    for (int q = 0; q < E->nq; ++q) {
        double H[MAXN][3], F[3][3], Fd[3][3], Jp;
        if (qp_kinematics(E, elem, q, H, &Jp, F, Fd)) return OR_E_REF_JACOBIAN;
        const double c = E->w[q] * Jp;
        for (int i = 0; i < E->nen; ++i)
            for (int j = 0; j < E->nen; ++j) {
                double Kb[3][3], Cb[3][3];
                tangent_block(m, F, Fd, H[i], H[j], Kb, Cb);
                for (int r = 0; r < 3; ++r)
                    for (int s = 0; s < 3; ++s) {
                        K[(3*i + r) * n3 + 3*j + s] += c * Kb[r][s];
                        Cv[(3*i + r) * n3 + 3*j + s] += c * Cb[r][s];
                    }
            }
    }
    return OR_OK;
}

/* Exported single-element blocks; Xe, xe, ve are [3][nen]. */
int oracle_element_tangent(int elem, int law, int damped, const double *theta,
                           const double *Xe, const double *xe, const double *ve,
                           double *K, double *Cv)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < E.nen; ++a) {   /* positions relative to node 0, as in gather() */
            E.U[i][a] = Xe[i*E.nen + a] - Xe[i*E.nen];
            E.N[i][a] = xe[i*E.nen + a] - xe[i*E.nen];
            E.Nd[i][a] = ve ? ve[i*E.nen + a] : 0.0;
        }
    mat_t m = mat_of(law, damped, theta, 1, 0);
    return element_blocks(&E, elem, &m, K, Cv);
}

/* ------------------------------------------------------------------ */
/* Adjoint (VJP) and tangent (JVP) products from the element blocks     */
/* ------------------------------------------------------------------ */

/* gx = sum_e K^e^T w_e, gv = sum_e C^e^T w_e (accumulated, [3][n_nodes]);
 * gtheta[p][e] = w_e . f^e(theta = unit vector p), which is exact because
 * P is linear in each parameter row (SVK: lambda, mu; MR: mu10, mu01, k;
 * Kelvin-Voigt: mu_v, lambda_v).  gtheta rows that a law does not use are
 * written as 0 (row 2 for SVK, row 1 for NH, rows 3-4 when undamped). */
static int vjp_range(int elem, int law, int damped, int64_t n_nodes, const double *X,
                     int64_t n_elem, const int32_t *conn, const double *theta,
                     const double *x, const double *v, const double *w,
                     double *gx, double *gv, double *gtheta, int64_t e0, int64_t e1)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    const int n3 = 3 * E.nen;
    double *K = malloc(sizeof(double) * n3 * n3), *Cv = malloc(sizeof(double) * n3 * n3);
    int rc = OR_OK;
    for (int64_t e = e0; e < e1 && rc == OR_OK; ++e) {
        const int32_t *c = conn + e * E.nen;
        mat_t m = mat_of(law, damped, theta, n_elem, e);
        gather(&E, n_nodes, c, X, x, v);
        double we[3 * MAXN];
        for (int a = 0; a < E.nen; ++a)
            for (int i = 0; i < 3; ++i) we[3*a + i] = w[i*n_nodes + c[a]];
        if (gx || gv) {
            rc = element_blocks(&E, elem, &m, K, Cv);
            if (rc) break;
            for (int j = 0; j < E.nen; ++j)
                for (int s = 0; s < 3; ++s) {
                    double sx = 0, sv = 0;
                    for (int r = 0; r < n3; ++r) {
                        sx += K[r * n3 + 3*j + s] * we[r];
                        sv += Cv[r * n3 + 3*j + s] * we[r];
                    }
                    if (gx) gx[s*n_nodes + c[j]] += sx;
                    if (gv && m.damped) gv[s*n_nodes + c[j]] += sv;
                }
        }
        if (gtheta) {
            for (int p = 0; p < 5; ++p) {
                int used = 1;
                if (law == OR_SVK && p == 2) used = 0;
                if (law == OR_NH && p == 1) used = 0;
                if (!damped && p >= 3) used = 0;
                double g = 0;
                if (used) {
                    mat_t u = m;
                    u.p0 = u.p1 = u.p2 = u.mu_v = u.lam_v = 0.0;
                    double *slot[5] = {&u.p0, &u.p1, &u.p2, &u.mu_v, &u.lam_v};
                    *slot[p] = 1.0;
                    for (int q = 0; q < E.nq; ++q) {
                        double H[MAXN][3], F[3][3], Fd[3][3], P[3][3], Jp;
                        if (qp_kinematics(&E, elem, q, H, &Jp, F, Fd)) { rc = OR_E_REF_JACOBIAN; break; }
                        if (p < 3) {
                            u.damped = 0;
                            elastic_P(&u, F, P);
                        } else {
                            double Ed[3][3], Sv[3][3];
                            u.damped = 1;
                            viscous_Sv(&u, F, Fd, Ed, Sv);
                            mul(F, Sv, P);
                        }
                        for (int a = 0; a < E.nen; ++a) {
                            double Ph[3];
                            matvec(P, H[a], Ph);
                            g += E.w[q] * Jp * (we[3*a]*Ph[0] + we[3*a+1]*Ph[1] + we[3*a+2]*Ph[2]);
                        }
                    }
                }
                gtheta[p * n_elem + e] = g;
            }
        }
    }
    free(K);
    free(Cv);
    return rc;
}

int oracle_vjp(int elem, int law, int damped, int64_t n_nodes, const double *X,
               int64_t n_elem, const int32_t *conn, const double *theta,
               const double *x, const double *v, const double *w,
               double *gx, double *gv, double *gtheta)
{
    return vjp_range(elem, law, damped, n_nodes, X, n_elem, conn, theta, x, v, w, gx, gv, gtheta, 0, n_elem);
}

/* df = sum_e (K^e dx_e + C^e dv_e), accumulated into [3][n_nodes]. */
int oracle_jvp(int elem, int law, int damped, int64_t n_nodes, const double *X,
               int64_t n_elem, const int32_t *conn, const double *theta,
               const double *x, const double *v, const double *dx, const double *dv,
               double *df)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    const int n3 = 3 * E.nen;
    double *K = malloc(sizeof(double) * n3 * n3), *Cv = malloc(sizeof(double) * n3 * n3);
    int rc = OR_OK;
    for (int64_t e = 0; e < n_elem; ++e) {
        const int32_t *c = conn + e * E.nen;
        mat_t m = mat_of(law, damped, theta, n_elem, e);
        gather(&E, n_nodes, c, X, x, v);
        rc = element_blocks(&E, elem, &m, K, Cv);
        if (rc) break;
        double de[3 * MAXN], dve[3 * MAXN];
        for (int a = 0; a < E.nen; ++a)
            for (int i = 0; i < 3; ++i) {
                de[3*a + i] = dx ? dx[i*n_nodes + c[a]] : 0.0;
                dve[3*a + i] = (dv && m.damped) ? dv[i*n_nodes + c[a]] : 0.0;
            }
        for (int r = 0; r < n3; ++r) {
            double s = 0;
            for (int col = 0; col < n3; ++col) s += K[r * n3 + col] * de[col] + Cv[r * n3 + col] * dve[col];
            df[(r % 3) * n_nodes + c[r / 3]] += s;
        }
    }
    free(K);
    free(Cv);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Multi-threaded runs of the same loops (OpenMP), for timing the      */
/* oracle on every host core                                           */
/* ------------------------------------------------------------------ */

/* The block's elements are cut into n_threads contiguous ranges; each thread
 * accumulates its range into a private nodal buffer with the serial loop
 * above, and the buffers are then added into the output in thread order,
 * so the result does not depend on scheduling.  Returns the status of the
 * first failing range. */
int oracle_internal_force_par(int elem, int law, int damped, int64_t n_nodes, const double *X,
                              int64_t n_elem, const int32_t *conn, const double *theta,
                              const double *x, const double *v, double *f, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    const size_t nn = 3 * (size_t)n_nodes;
    double *buf = calloc((size_t)n_threads * nn, sizeof(double));
    int *rc = calloc((size_t)n_threads, sizeof(int));
    if (!buf || !rc) { free(buf); free(rc); return OR_E_INVALID; }
#pragma omp parallel for num_threads(n_threads) schedule(static, 1)
    for (int t = 0; t < n_threads; ++t) {
        const int64_t e0 = n_elem * t / n_threads, e1 = n_elem * (t + 1) / n_threads;
        rc[t] = force_range(elem, law, damped, n_nodes, X, n_elem, conn, theta, x, v, buf + (size_t)t * nn, e0, e1);
    }
    int status = OR_OK;
    for (int t = 0; t < n_threads; ++t) {
        if (rc[t] && !status) status = rc[t];
        const double *b = buf + (size_t)t * nn;
        for (size_t i = 0; i < nn; ++i) f[i] += b[i];
    }
    free(buf);
    free(rc);
    return status;
}

int oracle_vjp_par(int elem, int law, int damped, int64_t n_nodes, const double *X,
                   int64_t n_elem, const int32_t *conn, const double *theta,
                   const double *x, const double *v, const double *w,
                   double *gx, double *gv, double *gtheta, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    const size_t nn = 3 * (size_t)n_nodes;
    double *bx = gx ? calloc((size_t)n_threads * nn, sizeof(double)) : NULL;
    double *bv = gv ? calloc((size_t)n_threads * nn, sizeof(double)) : NULL;
    int *rc = calloc((size_t)n_threads, sizeof(int));
    if ((gx && !bx) || (gv && !bv) || !rc) { free(bx); free(bv); free(rc); return OR_E_INVALID; }
#pragma omp parallel for num_threads(n_threads) schedule(static, 1)
    for (int t = 0; t < n_threads; ++t) {
        const int64_t e0 = n_elem * t / n_threads, e1 = n_elem * (t + 1) / n_threads;
        rc[t] = vjp_range(elem, law, damped, n_nodes, X, n_elem, conn, theta, x, v, w,
                          bx ? bx + (size_t)t * nn : NULL, bv ? bv + (size_t)t * nn : NULL, gtheta, e0, e1);
    }
    int status = OR_OK;
    for (int t = 0; t < n_threads; ++t) {
        if (rc[t] && !status) status = rc[t];
        for (size_t i = 0; gx && i < nn; ++i) gx[i] += bx[(size_t)t * nn + i];
        for (size_t i = 0; gv && i < nn; ++i) gv[i] += bv[(size_t)t * nn + i];
    }
    free(bx);
    free(bv);
    free(rc);
    return status;
}

/* ------------------------------------------------------------------ */
/* Inertia: consistent mass (Sec. 4.1) and the backward-Euler step     */
/* residual of the augmented-Lagrangian formulation without           */
/* constraints (Sec. 7)                                                */
/* ------------------------------------------------------------------ */

/* Quadrature of the mass integrals m_ij = int rho s_i s_j dV_r.  The paper
 * tabulates one rule per element on the parent domain (Sec. 6) and does not
 * say which rule integrates the mass.  The integrand of a straight-sided
 * element has twice the degree of the shape functions, so the rule here is
 * exact for it with positive weights (the element mass matrix is then the
 * exact Gram matrix of the shape functions, positive definite):
 *  T10: the 15-point degree-5 rule on the tetrahedron (Hammer, Marlowe and
 *       Stroud; Stroud's T3:5-1): the centroid, two 4-point orbits
 *       (a, a, a, 1-3a) with a = (7 -+ sqrt 15)/34, and the 6-point orbit
 *       (b, b, 1/2-b, 1/2-b) with b = (5 - sqrt 15)/20, in barycentric
 *       coordinates, weights 16/135, (2665 +- 14 sqrt 15)/37800 and 10/189
 *       of the volume;
 *  H8:  2x2x2 Gauss-Legendre (degree 3 per direction);
 *  Q27: 3x3x3 Gauss-Legendre (degree 5 per direction). */
static int mass_rule(int elem, double pts[][3], double *w)
{
    if (elem == OR_T10) {
        const double r15 = sqrt(15.0);
        const double a[2] = {(7.0 - r15) / 34.0, (7.0 + r15) / 34.0};
        const double wa[2] = {(2665.0 + 14.0 * r15) / 37800.0, (2665.0 - 14.0 * r15) / 37800.0};
        const double b = (5.0 - r15) / 20.0, c = 0.5 - b;
        int q = 0;
        pts[q][0] = pts[q][1] = pts[q][2] = 0.25;
        w[q++] = 16.0 / 135.0;
        for (int o = 0; o < 2; ++o) {
            /* barycentric (L1, L2, L3, L4) with one of the four equal to 1 - 3a;
             * parent coordinates are (L2, L3, L4) */
            for (int k = 0; k < 4; ++k) {
                double L[4] = {a[o], a[o], a[o], a[o]};
                L[k] = 1.0 - 3.0 * a[o];
                pts[q][0] = L[1]; pts[q][1] = L[2]; pts[q][2] = L[3];
                w[q++] = wa[o];
            }
        }
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) {
                double L[4] = {c, c, c, c};
                L[i] = b;
                L[j] = b;
                pts[q][0] = L[1]; pts[q][1] = L[2]; pts[q][2] = L[3];
                w[q++] = 10.0 / 189.0;
            }
        for (int k = 0; k < q; ++k) w[k] /= 6.0;   /* volume of the parent tetrahedron */
        return q;
    }
    /* H8 2x2x2 and Q27 3x3x3 Gauss: exact for the mass integrand of a
     * parallelepiped (degree 2 and 4 per direction) */
    if (elem == OR_H8 || elem == OR_Q27) return rule(elem, pts, w);
    return 0;
}

#define MAXQM 27

static void shape(int elem, const double *p, double *s)
{
    if (elem == OR_T10) t10_shape(p, s);
    else if (elem == OR_H8) h8_shape(p, s);
    else q27_shape(p, s);
}

int oracle_mass_rule(int elem, double *xi, double *w)
{
    double p[MAXQM][3], ww[MAXQM];
    const int nq = mass_rule(elem, p, ww);
    for (int q = 0; q < nq; ++q) {
        xi[3*q] = p[q][0]; xi[3*q+1] = p[q][1]; xi[3*q+2] = p[q][2];
        w[q] = ww[q];
    }
    return nq;
}

/* m_ij of one element (Sec. 4.1), [nen][nen]: sum over the mass rule of
 * w_k rho s_i s_j J_p (Sec. 6 change of variables).  U holds the element's
 * reference nodes relative to its first node (as in gather()). */
static int element_mass(int elem, const double U[3][MAXN], double rho, double *Me)
{
    const int nen = nen_of(elem);
    double pts[MAXQM][3], w[MAXQM];
    const int nq = mass_rule(elem, pts, w);
    memset(Me, 0, sizeof(double) * nen * nen);
    for (int q = 0; q < nq; ++q) {
        double G[MAXN][3], J[3][3], s[MAXN];
        dshape(elem, pts[q], G);
        shape(elem, pts[q], s);
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                double t = 0;
                for (int a = 0; a < nen; ++a) t += U[i][a] * G[a][k];
                J[i][k] = t;
            }
        const double Jp = det3(J);
        if (!(Jp > 0)) return OR_E_REF_JACOBIAN;
        for (int i = 0; i < nen; ++i)
            for (int j = 0; j < nen; ++j) Me[i * nen + j] += w[q] * rho * s[i] * s[j] * Jp;
    }
    return OR_OK;
}

/* Exported single-element mass matrix; Xe is [3][nen]. */
int oracle_element_mass(int elem, double rho, const double *Xe, double *Me)
{
    const int nen = nen_of(elem);
    if (!nen) return OR_E_INVALID;
    double U[3][MAXN];
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < nen; ++a) U[i][a] = Xe[i*nen + a] - Xe[i*nen];
    return element_mass(elem, U, rho, Me);
}

/* y += M u, M = assembled [m_ij I_3] (Sec. 4.1).  u, y are [3][n_nodes]. */
int oracle_mass_action(int elem, int64_t n_nodes, const double *X, int64_t n_elem, const int32_t *conn,
                       double rho, const double *u, double *y)
{
    const int nen = nen_of(elem);
    if (!nen) return OR_E_INVALID;
    double Me[MAXN * MAXN];
    for (int64_t e = 0; e < n_elem; ++e) {
        const int32_t *c = conn + e * nen;
        double U[3][MAXN];
        for (int a = 0; a < nen; ++a)
            for (int i = 0; i < 3; ++i) U[i][a] = X[i*n_nodes + c[a]] - X[i*n_nodes + c[0]];
        const int rc = element_mass(elem, U, rho, Me);
        if (rc) return rc;
        for (int i = 0; i < nen; ++i)
            for (int r = 0; r < 3; ++r) {
                double t = 0;
                for (int j = 0; j < nen; ++j) t += Me[i * nen + j] * u[r*n_nodes + c[j]];
                y[r*n_nodes + c[i]] += t;
            }
    }
    return OR_OK;
}

/* The configuration of the step map q(v) = q_n + h v (Sec. 7), formed with
 * one rounding per entry (a fused multiply-add) so that every evaluation of
 * the map gives the same positions bit for bit. */
static double *step_positions(int64_t n_nodes, const double *q_n, const double *v, double h)
{
    double *q = malloc(sizeof(double) * 3 * (size_t)n_nodes);
    if (!q) return NULL;
    for (int64_t i = 0; i < 3 * n_nodes; ++i) q[i] = fma(h, v[i], q_n[i]);
    return q;
}

/* Backward-Euler step residual without constraints (Sec. 7):
 *   g(v) = M (v - v_n) / h + f_int(q_n + h v, v) - f_ext,
 * accumulated into g ([3][n_nodes]) for one block; f_ext (may be NULL) is
 * subtracted by the caller once for the whole mesh (see oracle.py). */
int oracle_step_residual(int elem, int law, int damped, int64_t n_nodes, const double *X,
                         int64_t n_elem, const int32_t *conn, const double *theta, double rho,
                         const double *q_n, const double *v_n, const double *v, double h, double *g)
{
    double *q = step_positions(n_nodes, q_n, v, h);
    double *u = malloc(sizeof(double) * 3 * (size_t)n_nodes);
    double *Mu = calloc(3 * (size_t)n_nodes, sizeof(double));
    if (!q || !u || !Mu) { free(q); free(u); free(Mu); return OR_E_INVALID; }
    for (int64_t i = 0; i < 3 * n_nodes; ++i) u[i] = v[i] - v_n[i];
    int rc = oracle_mass_action(elem, n_nodes, X, n_elem, conn, rho, u, Mu);
    if (!rc) {
        for (int64_t i = 0; i < 3 * n_nodes; ++i) g[i] += Mu[i] / h;
        rc = force_range(elem, law, damped, n_nodes, X, n_elem, conn, theta, q, damped ? v : NULL, g, 0, n_elem);
    }
    free(q); free(u); free(Mu);
    return rc;
}

/* The velocity derivative of the residual applied to dv (Sec. 7):
 *   y = (M / h + h K + C) dv,  K = df_int/dq, C = df_int/dv at (q_n + h v, v),
 * from the element blocks (App. C and the Kelvin-Voigt blocks), accumulated
 * into y for one block. */
int oracle_newton_operator(int elem, int law, int damped, int64_t n_nodes, const double *X,
                           int64_t n_elem, const int32_t *conn, const double *theta, double rho,
                           const double *q_n, const double *v, double h, const double *dv, double *y)
{
    elem_t E;
    if (setup(&E, elem)) return OR_E_INVALID;
    double *q = step_positions(n_nodes, q_n, v, h);
    const int n3 = 3 * E.nen;
    double *K = malloc(sizeof(double) * n3 * n3), *Cv = malloc(sizeof(double) * n3 * n3);
    double Me[MAXN * MAXN];
    int rc = (q && K && Cv) ? OR_OK : OR_E_INVALID;
    for (int64_t e = 0; e < n_elem && rc == OR_OK; ++e) {
        const int32_t *c = conn + e * E.nen;
        mat_t m = mat_of(law, damped, theta, n_elem, e);
        gather(&E, n_nodes, c, X, q, damped ? v : NULL);
        rc = element_blocks(&E, elem, &m, K, Cv);
        if (!rc) rc = element_mass(elem, E.U, rho, Me);
        if (rc) break;
        double de[3 * MAXN];
        for (int a = 0; a < E.nen; ++a)
            for (int i = 0; i < 3; ++i) de[3*a + i] = dv[i*n_nodes + c[a]];
        for (int row = 0; row < n3; ++row) {
            const int a = row / 3, i = row % 3;
            double t = 0;
            for (int col = 0; col < n3; ++col) t += (h * K[row * n3 + col] + Cv[row * n3 + col]) * de[col];
            for (int b = 0; b < E.nen; ++b) t += Me[a * E.nen + b] / h * de[3*b + i];
            y[i*n_nodes + c[a]] += t;
        }
    }
    free(q); free(K); free(Cv);
    return rc;
}

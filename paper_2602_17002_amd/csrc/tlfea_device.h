// Device code (gfx950) of the Total Lagrangian internal force, its adjoint
// and its tangent product.  Included by tlfea_kernels.hip, which is compiled
// once per (element type, operation) so the instantiations build in parallel.
//
// Work decomposition: one workgroup per tile of up to TE elements of a single
// block (element type x law x damping).  The tile's distinct nodes are staged
// in LDS (reference X, positions x, and whichever of v, w, dx, dv the op
// needs), each lane owns one element and loops over its quadrature points in
// registers, and the per-element nodal vectors are then written to LDS and
// summed per node through a tile-local CSR in a fixed order.  Nodes touched
// by this tile only are written straight to the output; nodes shared with
// other tiles go to a partial-sum buffer that a second kernel sums per node
// in tile order.  No floating-point atomics: results are bitwise repeatable.
//
// All arithmetic is FP64 on the vector ALUs: the per-point work is 3x3 and
// 3xnen products, not a dense contraction, so the matrix cores do not apply.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "tlfea_elements.h"
#include "tlfea_internal.h"

namespace tlfea {

// ---------------------------------------------------------------- helpers

template <int N, int I = 0, class Fn>
__device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<N, I + 1>(fn);
    }
}

// Run fn(integral_constant<q>) for q = 0..N-1 as a loop that is not unrolled:
// each iteration executes exactly one compile-time instance, so the
// scheduler cannot interleave (and keep live) the temporaries of several
// quadrature points.
template <int N, class Fn>
__device__ __forceinline__ void point_loop(Fn &&fn)
{
#pragma nounroll
    for (int q = 0; q < N; ++q) {
        static_for<N>([&](auto qc) {
            if (q == decltype(qc)::value) fn(qc);
        });
    }
}

// The quadrature points a lane evaluates: T10 and H8 every point of its
// element as point_loop (each point a compile-time instance, passed as
// integral_constant); Q27 the points part, part + 2, ... of its element (the
// element's two lanes split the 27 points) as a plain loop over an int.
template <int ELEM, class Fn>
__device__ __forceinline__ void for_points(int part, Fn &&fn)
{
    if constexpr (ELEM == kQ27) {
        constexpr int LPE = lanes_per_elem(kQ27), NT = (ElemDef<kQ27>::nq + LPE - 1) / LPE;
#pragma nounroll
        for (int t = 0; t < NT; ++t) {
            const int q = part + LPE * t;
            if (q < ElemDef<kQ27>::nq) fn(q);
        }
    } else {
        point_loop<ElemDef<ELEM>::nq>(fn);
    }
}

// 1-D values of the three directions at Q27 point q (L: values, D:
// derivatives; [direction][node index along it]), from the Gauss
// coordinate of each direction.  The two lanes of an element evaluate
// different points, so these are per-lane values.
struct Q27Pt {
    double L[3][3], D[3][3];
};
__device__ __forceinline__ Q27Pt q27_point(int q)
{
    using E = ElemDef<kQ27>;
    Q27Pt t;
    const int p[3] = {q % 3, (q / 3) % 3, q / 9};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double s = p[d] == 0 ? -E::g : (p[d] == 1 ? 0.0 : E::g);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t.L[d][i] = E::lag1(i, s);
            t.D[d][i] = E::dlag1(i, s);
        }
    }
    return t;
}

// Weight of point q of an element type (q an integral_constant, or an int
// for Q27).
template <int ELEM, class QT>
__device__ __forceinline__ double weight_at(QT q)
{
    if constexpr (ELEM == kQ27) return ElemDef<kQ27>::weight((int)q);
    else return ElemDef<ELEM>::weight(QT::value);
}

typedef double m3[3][3];

__device__ __forceinline__ void mm(const m3 &A, const m3 &B, m3 &R)   // R = A B
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
}

__device__ __forceinline__ void mmT(const m3 &A, const m3 &B, m3 &R)  // R = A B^T
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[i][j] = A[i][0] * B[j][0] + A[i][1] * B[j][1] + A[i][2] * B[j][2];
}

__device__ __forceinline__ void mTm(const m3 &A, const m3 &B, m3 &R)  // R = A^T B
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[i][j] = A[0][i] * B[0][j] + A[1][i] * B[1][j] + A[2][i] * B[2][j];
}

__device__ __forceinline__ double ddot(const m3 &A, const m3 &B)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s += A[i][j] * B[i][j];
    return s;
}

// cofactor matrix: cof(A) = det(A) A^{-T}
__device__ __forceinline__ void cofactor(const m3 &A, m3 &C)
{
    C[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    C[0][1] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    C[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    C[1][0] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
    C[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
    C[1][2] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
    C[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    C[2][1] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
    C[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
}

__device__ __forceinline__ double det_from_cof(const m3 &A, const m3 &C)
{
    return A[0][0] * C[0][0] + A[0][1] * C[0][1] + A[0][2] * C[0][2];
}

// 1 / d for a normal, nonzero d: the hardware estimate refined by two Newton
// steps r <- r + r (1 - d r), each of which squares the relative error; the
// result is within two units in the last place of the quotient (five
// instructions in place of the eleven of a correctly rounded division).
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// J^(-1/3) with the sign of J, for |J| in the normal single-precision range:
// a single-precision estimate exp2(-log2|J| / 3) (relative error about
// 1e-7), then two Newton steps y <- y + y (1 - |J| y^3) / 3 in double, each
// of which takes a relative error e to about 2 e^2; within two units in the
// last place.
__device__ __forceinline__ double inv_cbrt(double J)
{
    const double a = fabs(J);
    double y = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf((float)a) * (1.0f / 3.0f));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-a, y * y * y, 1.0);
        y = fma(y * e, 1.0 / 3.0, y);
    }
    return copysign(y, J);
}

struct Mat {
    double p0, p1, p2, mu_v, lam_v;
};

// Compiler-only barrier placed before every gather of a staged field: node
// values are re-read from LDS when needed instead of being loaded early and
// kept live in registers across the unrolled point loop (2 VGPRs per staged
// double, which would halve occupancy).
__device__ __forceinline__ void qp_fence() { __asm__ __volatile__("" ::: "memory"); }

// -------------------------------------------------------- per-point kinematics

// Node records in LDS: every staged node of a tile holds REC consecutive
// doubles, field f's component c at offset 3 f + c.  na[a] is the record
// offset (in doubles) of the element's local node a, so every read below is
// one LDS address per node plus compile-time offsets.

// G = sum_a s_a (ds_a/dxi at point Q)^T for the field at s (a pointer into
// the first record at that field's offset); zero gradient entries are
// removed at compile time.  For positions (REL) the sum is taken over the
// differences s_a - s_0 to the element's first node, which is the same sum
// because the parent gradients of an element sum to zero, and whose products
// only cancel over one element instead of over the tile.  Each difference is
// the nodes' coordinate difference rounded once: the current positions of
// these kernels are staged raw, and the reference ones relative to the tile's
// reference node only where that subtraction was exact.
template <int ELEM, int NEN, bool REL, class QT>
__device__ __forceinline__ void grad_field_q27(QT q, const double *__restrict__ s, const int (&na)[NEN], m3 &G);

template <int ELEM, int NEN, bool REL = false, class QT>
__device__ __forceinline__ void grad_field(QT qc, const double *__restrict__ s, const int (&na)[NEN], m3 &G)
{
    if constexpr (ELEM == kQ27) {
        grad_field_q27<ELEM, NEN, REL>(qc, s, na, G);
        return;
    } else {
    constexpr int Q = QT::value;
    using E = ElemDef<ELEM>;
    qp_fence();
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) G[i][k] = 0.0;
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if constexpr (REL) {
        o0 = s[na[0]];
        o1 = s[na[0] + 1];
        o2 = s[na[0] + 2];
    }
    static_for<NEN>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        if constexpr (!REL || a > 0) {
            const double x0 = s[na[a]] - o0, x1 = s[na[a] + 1] - o1, x2 = s[na[a] + 2] - o2;
            static_for<3>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr double g = E::grad(Q, a, k);
                if constexpr (g != 0.0) {
                    G[0][k] += x0 * g;
                    G[1][k] += x1 * g;
                    G[2][k] += x2 * g;
                }
            });
        }
    });
    }
}

// Q27 gradient at point q by sum factorisation: with (p0, p1, p2) the
// point's Gauss indices, G_c = sum_ijk s_ijk,c (L'_i L_j L_k, L_i L'_j L_k,
// L_i L_j L'_k), contracted over i, then j, then k (90 multiply-adds per
// component instead of the 81 of a stored 27 x 3 table, with 18 table
// values per point instead of 81).  REL as for grad_field.
template <int ELEM, int NEN, bool REL, class QT>
__device__ __forceinline__ void grad_field_q27(QT q, const double *__restrict__ s, const int (&na)[NEN], m3 &G)
{
    static_assert(NEN == 27, "Q27");
    qp_fence();
    const Q27Pt t = q27_point((int)q);
    double o[3] = {0.0, 0.0, 0.0};
    if constexpr (REL) {
        o[0] = s[na[0]];
        o[1] = s[na[0] + 1];
        o[2] = s[na[0] + 2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c][0] = G[c][1] = G[c][2] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // one plane of nodes (27 values) in flight at a time
        qp_fence();
        double ck[3] = {0.0, 0.0, 0.0}, dk[3] = {0.0, 0.0, 0.0}, ek[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double a[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int n = i + 3 * j + 9 * k;
                if (REL && n == 0) continue;   // s_0 - s_0
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double v = s[na[n] + c] - o[c];
                    a[c] += t.D[0][i] * v;
                    b[c] += t.L[0][i] * v;
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ck[c] += t.L[1][j] * a[c];
                dk[c] += t.D[1][j] * b[c];
                ek[c] += t.L[1][j] * b[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            G[c][0] += t.L[2][k] * ck[c];
            G[c][1] += t.L[2][k] * dk[c];
            G[c][2] += t.D[2][k] * ek[c];
        }
    }
}

// Q27 transpose of grad_field_q27: out[ijk][c] += sum_m Qm[c][m] g_m with
// g = (L'_i L_j L_k, L_i L'_j L_k, L_i L_j L'_k), factored from k inwards.
template <int NEN, int SKIP_LAST, class QT>
__device__ __forceinline__ void scatter_grad_q27(QT q, const m3 &Qm, double (&out)[NEN][3])
{
    static_assert(NEN == 27, "Q27");
    const Q27Pt t = q27_point((int)q);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double t0[3], t1[3], t2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            t0[c] = t.L[2][k] * Qm[c][0];
            t1[c] = t.L[2][k] * Qm[c][1];
            t2[c] = t.D[2][k] * Qm[c][2];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double u[3], w[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[c] = t.L[1][j] * t0[c];                       // multiplies L'_i
                w[c] = t.D[1][j] * t1[c] + t.L[1][j] * t2[c];   // multiplies L_i
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int n = i + 3 * j + 9 * k;
                if (SKIP_LAST && n == NEN - 1) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) out[n][c] += t.D[0][i] * u[c] + t.L[0][i] * w[c];
            }
        }
    }
}

// out[a][r] += sum_k Q[r][k] (ds_a/dxi at point Q)_k   (i.e. c P h_a with Q = c P J^{-T}),
// for every node but the last when SKIP_LAST (see finish_last_node)
template <int ELEM, int NEN, int SKIP_LAST = 0, class QT>
__device__ __forceinline__ void scatter_grad(QT qc, const m3 &Qm, double (&out)[NEN][3])
{
    if constexpr (ELEM == kQ27) {
        scatter_grad_q27<NEN, SKIP_LAST>(qc, Qm, out);
        return;
    } else {
    constexpr int QP = QT::value;
    using E = ElemDef<ELEM>;
    static_for<NEN - SKIP_LAST>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        static_for<3>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr double g = E::grad(QP, a, k);
            if constexpr (g != 0.0) {
                out[a][0] += Qm[0][k] * g;
                out[a][1] += Qm[1][k] * g;
                out[a][2] += Qm[2][k] * g;
            }
        });
    });
    }
}

// The parent gradients of an element sum to zero at every point (the shape
// functions sum to one), so the contributions Q g_a of a point to an element
// vector sum to zero over its nodes, and so does the element vector: the
// last node's entry is minus the sum of the others.  Accumulating one node
// fewer saves its registers.
template <int NEN>
__device__ __forceinline__ void finish_last_node(double (&out)[NEN][3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double sum = 0.0;
#pragma unroll
        for (int a = 0; a < NEN - 1; ++a) sum += out[a][r];
        out[NEN - 1][r] = -sum;
    }
}

// Reference geometry at point Q (Sec. 6): J = U dS/dxi, J_p = det J,
// K = cof(J) = J_p J^{-T} and r = 1 / J_p (FAST: by recip); REL as for
// grad_field.  Evaluated at every point from
// all nodes: straight-sided elements have a constant J only up to the
// rounding of their mid-edge coordinates, which the bulk response amplifies.
template <int ELEM, int NEN, bool REL = false, bool FAST = false, class QT>
__device__ __forceinline__ void ref_geometry(QT q, const double *__restrict__ sX, const int (&na)[NEN], m3 &K,
                                             double &detJ, double &r)
{
    m3 J;
    grad_field<ELEM, NEN, REL>(q, sX, na, J);
    cofactor(J, K);
    detJ = det_from_cof(J, K);
    if constexpr (FAST) r = recip(detJ);
    else r = 1.0 / detJ;
}

// A = G J^{-1} = (G K^T) r: the gradient with respect to the reference
// coordinates of a field whose parent gradient is G (F = N H, Sec. 2.1).
__device__ __forceinline__ void to_reference(const m3 &G, const m3 &K, double r, m3 &A)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[i][j] = (G[i][0] * K[j][0] + G[i][1] * K[j][1] + G[i][2] * K[j][2]) * r;
}

// Qm = w_q P K = w_q J_p P J^{-T}, so that w_q J_p P h_a = Qm (ds_a/dxi).
__device__ __forceinline__ void to_parent(const m3 &P, const m3 &K, double wq, m3 &Qm)
{
    m3 T;
    mm(P, K, T);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Qm[i][j] = T[i][j] * wq;
}

// ----------------------------------------------------------- constitutive laws

// Kelvin-Voigt: Edot = sym(F^T Fdot), S_v[A] = 2 mu_v A + lambda_v tr(A) I (Sec. 3.2.3)
__device__ __forceinline__ void sym_FtG(const m3 &F, const m3 &G, m3 &S)   // S = sym(F^T G)
{
    m3 A;
    mTm(F, G, A);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = 0.5 * (A[i][j] + A[j][i]);
}

__device__ __forceinline__ void visc_op(const Mat &m, const m3 &A, m3 &S)   // S = S_v[A]
{
    const double tr = A[0][0] + A[1][1] + A[2][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = 2.0 * m.mu_v * A[i][j] + (i == j ? m.lam_v * tr : 0.0);
}

// Symmetric 3x3 matrices stored by their six distinct entries
// (xx, yy, zz, xy, yz, xz): strain rates and viscous stresses.
struct s3 {
    double a[6];
};

__device__ __forceinline__ constexpr int sidx(int i, int j)
{
    return i == j ? i : (i + j == 1 ? 3 : (i + j == 3 ? 4 : 5));
}

// sym(F^T G) = (F^T G + G^T F) / 2
__device__ __forceinline__ s3 sym_FtG_s(const m3 &F, const m3 &G)
{
    s3 S;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) t += F[k][i] * G[k][j] + F[k][j] * G[k][i];
            S.a[sidx(i, j)] = 0.5 * t;
        }
    return S;
}

__device__ __forceinline__ double trace_s(const s3 &A) { return A.a[0] + A.a[1] + A.a[2]; }

// S_v[A] = 2 mu_v A + lambda_v tr(A) I
__device__ __forceinline__ s3 visc_s(const Mat &m, const s3 &A)
{
    const double tl = m.lam_v * trace_s(A), m2 = 2.0 * m.mu_v;
    s3 S;
#pragma unroll
    for (int d = 0; d < 6; ++d) S.a[d] = m2 * A.a[d] + (d < 3 ? tl : 0.0);
    return S;
}

__device__ __forceinline__ double ddot_s(const s3 &A, const s3 &B)
{
    return A.a[0] * B.a[0] + A.a[1] * B.a[1] + A.a[2] * B.a[2] +
           2.0 * (A.a[3] * B.a[3] + A.a[4] * B.a[4] + A.a[5] * B.a[5]);
}

// R += M S
__device__ __forceinline__ void acc_mul_ms(const m3 &M, const s3 &S, m3 &R)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            R[i][j] += M[i][0] * S.a[sidx(0, j)] + M[i][1] * S.a[sidx(1, j)] + M[i][2] * S.a[sidx(2, j)];
}

// Invariants and pieces shared by the Mooney-Rivlin stress and its derivative.
struct MRState {
    m3 FiT;          // F^{-T}
    m3 cof;          // cof F = J F^{-T} (the forward's Neo-Hookean stress uses it
                     // with 1/J folded into its scalar coefficient)
    double J, invJ, J23, I1;
    // Mooney-Rivlin (mu01) only
    m3 C, FC;
    double J43, I2;
};

// FAST: 1/J and J^(-1/3) by recip and inv_cbrt instead of a division and
// the library cube root.
template <int LAW, bool FAST = false>
__device__ __forceinline__ void mr_state(const m3 &F, MRState &st)
{
    cofactor(F, st.cof);
    st.J = det_from_cof(F, st.cof);
    st.invJ = FAST ? recip(st.J) : 1.0 / st.J;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) st.FiT[i][j] = st.cof[i][j] * st.invJ;
    const double c = FAST ? inv_cbrt(st.J) : cbrt(st.invJ);   // J^{-1/3}
    st.J23 = c * c;                                           // J^{-2/3}
    st.I1 = ddot(F, F);                   // tr C
    if constexpr (LAW == 1) {
        mTm(F, F, st.C);
        mm(F, st.C, st.FC);
        st.J43 = st.J23 * st.J23;
        st.I2 = 0.5 * (st.I1 * st.I1 - ddot(st.C, st.C));
    }
}

// Elastic first Piola-Kirchhoff stress (Sec. 3.2, App. C):
//   SVK: P = F S, S = lambda tr(E) I + 2 mu E, E = (F^T F - I)/2
//   MR : P = 2 mu10 J^{-2/3}(F - I1/3 F^{-T}) + 2 mu01 J^{-4/3}(I1 F - F C - 2/3 I2 F^{-T})
//          + k (J-1) J F^{-T};  NH is MR with mu01 = 0.
// With Kelvin-Voigt the viscous S_v(Edot) is added (P = F (S + S_v) for SVK).
// FAST: mr_state's FAST, and the Neo-Hookean F^{-T} term from cof F.
template <int LAW, bool DAMPED, bool FAST = false>
__device__ __forceinline__ void stress(const m3 &F, const m3 &Fd, const Mat &m, m3 &P)
{
    if constexpr (LAW == 0) {
        m3 C, S;
        mTm(F, F, C);
        const double trE = 0.5 * (C[0][0] + C[1][1] + C[2][2] - 3.0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) S[i][j] = m.p1 * (C[i][j] - (i == j ? 1.0 : 0.0)) + (i == j ? m.p0 * trE : 0.0);
        if constexpr (DAMPED) {
            m3 Ed, Sv;
            sym_FtG(F, Fd, Ed);
            visc_op(m, Ed, Sv);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) S[i][j] += Sv[i][j];
        }
        mm(F, S, P);
    } else {
        MRState st;
        mr_state<LAW, FAST>(F, st);
        const double a = 2.0 * m.p0 * st.J23;
        if constexpr (LAW == 2 && FAST) {
            // b F^{-T} = (b / J) cof F, with k (J - 1) J / J = k (J - 1)
            const double b = -(2.0 / 3.0) * m.p0 * st.J23 * st.I1 * st.invJ + m.p2 * (st.J - 1.0);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) P[i][j] = a * F[i][j] + b * st.cof[i][j];
        } else {
            const double b = -(2.0 / 3.0) * m.p0 * st.J23 * st.I1 + m.p2 * (st.J - 1.0) * st.J;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) P[i][j] = a * F[i][j] + b * st.FiT[i][j];
        }
        if constexpr (LAW == 1) {
            const double be = 2.0 * m.p1 * st.J43;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    P[i][j] += be * (st.I1 * F[i][j] - st.FC[i][j] - (2.0 / 3.0) * st.I2 * st.FiT[i][j]);
        }
        if constexpr (DAMPED) {
            m3 Ed, Sv, Pv;
            sym_FtG(F, Fd, Ed);
            visc_op(m, Ed, Sv);
            mm(F, Sv, Pv);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) P[i][j] += Pv[i][j];
        }
    }
}

// Directional derivative of the elastic stress, dP = (dP_e/dF)[D].  The
// elastic tangent of a hyperelastic law is major-symmetric, so the same
// routine gives the adjoint (dP_e/dF)^T[D] used by the VJP.
//   SVK: dP = D S + F (lambda tr(dE) I + 2 mu dE), dE = sym(F^T D)
//   MR : derivative of the stress above term by term (dJ = J F^{-T}:D,
//        d(F^{-T}) = -F^{-T} D^T F^{-T}, dI1 = 2 F:D, dI2 = 2 I1 F:D - 2 FC:D).
template <int LAW>
__device__ __forceinline__ void delastic(const m3 &F, const Mat &m, const m3 &D, const MRState &st, m3 &dP)
{
    if constexpr (LAW == 0) {
        m3 C, S, dE;
        mTm(F, F, C);
        const double trE = 0.5 * (C[0][0] + C[1][1] + C[2][2] - 3.0);
        sym_FtG(F, D, dE);
        const double trdE = dE[0][0] + dE[1][1] + dE[2][2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                S[i][j] = m.p1 * (C[i][j] - (i == j ? 1.0 : 0.0)) + (i == j ? m.p0 * trE : 0.0);
                dE[i][j] = 2.0 * m.p1 * dE[i][j] + (i == j ? m.p0 * trdE : 0.0);
            }
        m3 A, B;
        mm(D, S, A);
        mm(F, dE, B);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) dP[i][j] = A[i][j] + B[i][j];
    } else {
        const double tF = ddot(st.FiT, D);          // F^{-T} : D = dJ / J
        const double FD = ddot(F, D);
        const double alpha = 2.0 * m.p0 * st.J23;
        const double dalpha = -(2.0 / 3.0) * alpha * tF;
        const double dI1 = 2.0 * FD;
        m3 T, Xm;                                   // Xm = F^{-T} D^T F^{-T}
        mTm(D, st.FiT, T);
        mm(st.FiT, T, Xm);
        const double J = st.J;
        const double cFiT = -(1.0 / 3.0) * (dalpha * st.I1 + alpha * dI1) + m.p2 * (2.0 * J - 1.0) * J * tF;
        const double cX = (1.0 / 3.0) * alpha * st.I1 - m.p2 * (J - 1.0) * J;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dP[i][j] = alpha * D[i][j] + dalpha * F[i][j] + cFiT * st.FiT[i][j] + cX * Xm[i][j];
        if constexpr (LAW == 1) {
            const double beta = 2.0 * m.p1 * st.J43;
            const double dbeta = -(4.0 / 3.0) * beta * tF;
            const double dI2 = 2.0 * st.I1 * FD - 2.0 * ddot(st.FC, D);
            m3 DC, FDt, FDtF, FFt, FFtD;
            mm(D, st.C, DC);
            mmT(F, D, FDt);
            mm(FDt, F, FDtF);
            mmT(F, F, FFt);
            mm(FFt, D, FFtD);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double M = st.I1 * F[i][j] - st.FC[i][j] - (2.0 / 3.0) * st.I2 * st.FiT[i][j];
                    const double dM = dI1 * F[i][j] + st.I1 * D[i][j] - DC[i][j] - FDtF[i][j] - FFtD[i][j]
                                      - (2.0 / 3.0) * dI2 * st.FiT[i][j] + (2.0 / 3.0) * st.I2 * Xm[i][j];
                    dP[i][j] += dbeta * M + beta * dM;
                }
        }
    }
}

// Scalars of the elastic derivative that the parameter gradients reuse:
// GF = F : D, GFiT = F^{-T} : D (Mooney-Rivlin), and for SVK tr E and E : D.
struct DerivScalars {
    double GF, GFiT, trE, ED;
};

// A += (dP_e/dF)[D], formed without storing dP: for Neo-Hookean the term
// F^{-T} D^T F^{-T} is added entry by entry; Mooney-Rivlin uses delastic.
template <int LAW>
__device__ __forceinline__ void delastic_acc(const m3 &F, const Mat &m, const m3 &D, const MRState &st, m3 &A,
                                             DerivScalars &ds)
{
    if constexpr (LAW == 0) {
        const s3 C = sym_FtG_s(F, F);                // C = F^T F
        const double trE = 0.5 * (trace_s(C) - 3.0);
        s3 S, dE = sym_FtG_s(F, D);                  // dE = sym(F^T D)
        const double trdE = trace_s(dE);
        double ED = 0.0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const double E = 0.5 * (C.a[d] - (d < 3 ? 1.0 : 0.0));
            ED += (d < 3 ? 1.0 : 2.0) * E * dE.a[d];
            S.a[d] = 2.0 * m.p1 * E + (d < 3 ? m.p0 * trE : 0.0);
            dE.a[d] = 2.0 * m.p1 * dE.a[d] + (d < 3 ? m.p0 * trdE : 0.0);
        }
        acc_mul_ms(D, S, A);
        acc_mul_ms(F, dE, A);
        ds.GF = trdE;                                // F : D = tr sym(F^T D)
        ds.GFiT = 0.0;
        ds.trE = trE;
        ds.ED = ED;
    } else if constexpr (LAW == 2) {
        const double tF = ddot(st.FiT, D);           // F^{-T} : D = dJ / J
        const double FD = ddot(F, D);
        const double alpha = 2.0 * m.p0 * st.J23;
        const double dalpha = -(2.0 / 3.0) * alpha * tF;
        const double dI1 = 2.0 * FD;
        m3 T;                                        // T = D^T F^{-T}
        mTm(D, st.FiT, T);
        const double J = st.J;
        const double cFiT = -(1.0 / 3.0) * (dalpha * st.I1 + alpha * dI1) + m.p2 * (2.0 * J - 1.0) * J * tF;
        const double cX = (1.0 / 3.0) * alpha * st.I1 - m.p2 * (J - 1.0) * J;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double X = st.FiT[i][0] * T[0][j] + st.FiT[i][1] * T[1][j] + st.FiT[i][2] * T[2][j];
                A[i][j] += alpha * D[i][j] + dalpha * F[i][j] + cFiT * st.FiT[i][j] + cX * X;
            }
        ds.GF = FD;
        ds.GFiT = tF;
        ds.trE = ds.ED = 0.0;
    } else {
        m3 dP;
        delastic<LAW>(F, m, D, st, dP);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[i][j] += dP[i][j];
        ds.GF = ddot(F, D);
        ds.GFiT = ddot(st.FiT, D);
        ds.trE = ds.ED = 0.0;
    }
}

// ------------------------------------------------------------ element bodies

template <int LAW>
__device__ __forceinline__ Mat load_mat(const BlockDesc &b, const double *__restrict__ theta, int64_t n_elem,
                                        int uid, bool damped)
{
    Mat m;
    if (theta) {
        m.p0 = theta[uid];
        m.p1 = theta[n_elem + uid];
        m.p2 = theta[2 * n_elem + uid];
        m.mu_v = damped ? theta[3 * n_elem + uid] : 0.0;
        m.lam_v = damped ? theta[4 * n_elem + uid] : 0.0;
    } else {
        m.p0 = b.theta[0];
        m.p1 = b.theta[1];
        m.p2 = b.theta[2];
        m.mu_v = damped ? b.theta[3] : 0.0;
        m.lam_v = damped ? b.theta[4] : 0.0;
    }
    if (LAW == 2) m.p1 = 0.0;
    return m;
}

// Offsets (in doubles) of the staged fields inside one LDS node record.
// X and x always; the adjoint adds w, the tangent dx; damped blocks add v
// (and the tangent dv).  The step residual (forward, kModeStep) adds
// u = v - v_n last; the Newton operator (tangent, kModeStep) keeps the
// tangent's layout with dx = h dv.
template <int OP, bool DAMPED, int MODE = kModePlain>
struct Rec {
    static constexpr bool has2 = OP != kOpFwd;              // w or dx
    static constexpr bool hasdv = DAMPED && OP == kOpJvp;
    static constexpr int oX = 0, ox = 3, o2 = 6;
    static constexpr int ov = has2 ? 9 : 6;
    static constexpr int odv = ov + 3;
    static constexpr int ou = DAMPED ? ov + 3 : ov;          // step residual: v - v_n
    static constexpr int nfield = record_fields_len(OP, DAMPED, MODE) / 3;   // staged fields
    static constexpr int len = record_len(OP, DAMPED, MODE);                  // stride (odd)
    static_assert(3 * nfield == 6 + (has2 ? 3 : 0) + (DAMPED ? 3 : 0) + (hasdv ? 3 : 0) +
                                    ((OP == kOpFwd && MODE == kModeStep) ? 3 : 0),
                  "record layout");
};

// Forward: fe[a] = sum_q w_q J_p P(F_q, Fdot_q) h_a   (Sec. 4.3 with Sec. 6)
template <int ELEM, int LAW, bool DAMPED, int MODE, int NEN>
__device__ __forceinline__ void fwd_element(const double *sm, const int (&na)[NEN], const Mat &mt,
                                            double (&fe)[NEN][3], int part)
{
    using E = ElemDef<ELEM>;
    using R = Rec<kOpFwd, DAMPED, MODE>;
    // the shorter reciprocal and cube root where they leave the register
    // schedule as it was or better (measured per instantiation): not Q27
    constexpr bool FAST = ELEM != kQ27;
    for_points<ELEM>(part, [&](auto q) {
        qp_fence();
        m3 K, G, F, Fd, P, Qm;
        double detJ, r;
        ref_geometry<ELEM, NEN, true, FAST>(q, sm + R::oX, na, K, detJ, r);
        grad_field<ELEM, NEN, true>(q, sm + R::ox, na, G);
        to_reference(G, K, r, F);                   // F = N H
        if constexpr (DAMPED) {
            grad_field<ELEM, NEN>(q, sm + R::ov, na, G);
            to_reference(G, K, r, Fd);              // Fdot = Ndot H
        }
        stress<LAW, DAMPED, FAST>(F, Fd, mt, P);
        to_parent(P, K, weight_at<ELEM>(q), Qm);
        scatter_grad<ELEM, NEN>(q, Qm, fe);
    });
}

// Adjoint: with Gw = sum_a w_a h_a^T and the identity w.f = sum_q c_q P:Gw,
//   gx_a += c_q Fbar_x h_a, Fbar_x = (dP_e/dF)[Gw] + Gw S_v + Fdot S_v[sym(F^T Gw)]
//   gv_a += c_q Fbar_v h_a, Fbar_v = F S_v[sym(F^T Gw)]
//   gtheta_p += c_q Gw : dP/dtheta_p   (P is linear in every parameter row)
// The viscous terms come first and go straight into Fbar_x and gv, so that
// the strain rates are dead before the elastic derivative needs registers.
// With both gx and gv accumulated (damped), the last node of each is formed
// from the others and K is formed again after the elastic derivative, which
// keeps the two sets of accumulators within the registers of two waves per
// SIMD.
template <int ELEM, int LAW, bool DAMPED, bool WANT_GT, int NEN>
__device__ __forceinline__ void vjp_element(const double *sm, const int (&na)[NEN], const Mat &mt,
                                            double (&gx)[NEN][3], double (&gv)[NEN][3], double (&gt)[5], int part)
{
    using E = ElemDef<ELEM>;
    using R = Rec<kOpVjp, DAMPED>;
    // The parameter gradients are stress-like (they cancel F against the
    // rotation as the stress does): positions relative to each element's
    // first node there.  The H8 adjoint keeps tile-relative positions (with
    // them its schedule spills hundreds of registers).
    constexpr bool REL = WANT_GT && ELEM == kT10;
    // as in fwd_element; not with gtheta on a damped block
    constexpr bool FAST = ELEM != kQ27 && !(WANT_GT && DAMPED);
    for_points<ELEM>(part, [&](auto q) {
        m3 K, G, F, Gw, Fb;
        double detJ, r;
        ref_geometry<ELEM, NEN, REL, FAST>(q, sm + R::oX, na, K, detJ, r);
        grad_field<ELEM, NEN, REL>(q, sm + R::ox, na, G);
        to_reference(G, K, r, F);
        grad_field<ELEM, NEN>(q, sm + R::o2, na, G);
        to_reference(G, K, r, Gw);
        const double c = weight_at<ELEM>(q) * detJ;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Fb[i][j] = 0.0;
        if constexpr (DAMPED) {
            m3 Fd;
            grad_field<ELEM, NEN>(q, sm + R::ov, na, G);
            to_reference(G, K, r, Fd);
            s3 Ed;
            {
                Ed = sym_FtG_s(F, Fd);
                const s3 Sv = visc_s(mt, Ed);
                acc_mul_ms(Gw, Sv, Fb);              // Gw S_v
            }
            {
                const s3 Sg = sym_FtG_s(F, Gw);
                if constexpr (WANT_GT) {
                    gt[3] += c * 2.0 * ddot_s(Ed, Sg);
                    gt[4] += c * trace_s(Ed) * trace_s(Sg);   // tr(Edot) (F : Gw)
                }
                const s3 SvSg = visc_s(mt, Sg);      // S_v[sym(F^T Gw)]
                acc_mul_ms(Fd, SvSg, Fb);            // Fdot S_v[sym(F^T Gw)]
                m3 A, T;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) A[i][j] = 0.0;
                acc_mul_ms(F, SvSg, A);              // Fbar_v
                to_parent(A, K, weight_at<ELEM>(q), T);
                scatter_grad<ELEM, NEN, DAMPED ? 1 : 0>(q, T, gv);
            }
        }
        MRState st;
        if constexpr (LAW != 0) mr_state<LAW, FAST>(F, st);
        DerivScalars ds;
        delastic_acc<LAW>(F, mt, Gw, st, Fb, ds);
        if constexpr (WANT_GT) {
            if constexpr (LAW == 0) {
                gt[0] += c * ds.trE * ds.GF;
                gt[1] += c * 2.0 * ds.ED;
            } else {
                gt[0] += c * 2.0 * st.J23 * (ds.GF - (1.0 / 3.0) * st.I1 * ds.GFiT);
                if constexpr (LAW == 1)
                    gt[1] += c * 2.0 * st.J43 * (st.I1 * ds.GF - ddot(Gw, st.FC) - (2.0 / 3.0) * st.I2 * ds.GFiT);
                gt[2] += c * (st.J - 1.0) * st.J * ds.GFiT;
            }
        }
        // K is formed again here rather than kept live across the
        // elastic derivative (fewer registers at its peak)
        m3 Qm;
        if constexpr (ELEM == kQ27) {
            to_parent(Fb, K, weight_at<ELEM>(q), Qm);
        } else {
            m3 K2;
            double d2, r2;
            ref_geometry<ELEM, NEN, REL>(q, sm + R::oX, na, K2, d2, r2);
            to_parent(Fb, K2, weight_at<ELEM>(q), Qm);
        }
        scatter_grad<ELEM, NEN, (DAMPED || ELEM == kQ27) ? 1 : 0>(q, Qm, gx);
    });
    if constexpr (DAMPED || ELEM == kQ27) finish_last_node(gx);
    if constexpr (DAMPED) finish_last_node(gv);
}

// Tangent: dF = sum_a dx_a h_a^T, dFdot = sum_a dv_a h_a^T,
//   dP = (dP_e/dF)[dF] + dF S_v + F S_v[sym(dF^T Fdot + F^T dFdot)]
//        (+ P(F, Fdot; dtheta) when DT: the stress is linear in the parameters),
//   df_a += c_q dP h_a.
template <int ELEM, int LAW, bool DAMPED, bool DT, int NEN>
__device__ __forceinline__ void jvp_element(const double *sm, const int (&na)[NEN], const Mat &mt, const Mat &dmt,
                                            double (&df)[NEN][3], int part)
{
    using E = ElemDef<ELEM>;
    using R = Rec<kOpJvp, DAMPED>;
    // as in fwd_element; not with a parameter direction, not Mooney-Rivlin
    constexpr bool FAST = ELEM != kQ27 && !DT && LAW != 1;
    for_points<ELEM>(part, [&](auto q) {
        qp_fence();
        m3 K, G, F, dF, dP;
        double detJ, r;
        ref_geometry<ELEM, NEN, false, FAST>(q, sm + R::oX, na, K, detJ, r);
        grad_field<ELEM, NEN>(q, sm + R::ox, na, G);
        to_reference(G, K, r, F);
        grad_field<ELEM, NEN>(q, sm + R::o2, na, G);
        to_reference(G, K, r, dF);
        {
            MRState st;
            if constexpr (LAW != 0) mr_state<LAW, FAST>(F, st);
            delastic<LAW>(F, mt, dF, st, dP);
        }
        if constexpr (DAMPED) {
            m3 Fd, Ed, Sv, A, B, T;
            grad_field<ELEM, NEN>(q, sm + R::ov, na, G);
            to_reference(G, K, r, Fd);
            if constexpr (DT) {
                stress<LAW, true>(F, Fd, dmt, T);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) dP[i][j] += T[i][j];
            }
            sym_FtG(F, Fd, Ed);
            visc_op(mt, Ed, Sv);
            mm(dF, Sv, T);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dP[i][j] += T[i][j];
            mTm(dF, Fd, A);                       // dF^T Fdot
            {
                m3 dFd;
                grad_field<ELEM, NEN>(q, sm + R::odv, na, G);
                to_reference(G, K, r, dFd);
                mTm(F, dFd, B);                   // F^T dFdot
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) A[i][j] += B[i][j];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) B[i][j] = 0.5 * (A[i][j] + A[j][i]);
            visc_op(mt, B, A);
            mm(F, A, T);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dP[i][j] += T[i][j];
        } else if constexpr (DT) {
            m3 T;
            stress<LAW, false>(F, F, dmt, T);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dP[i][j] += T[i][j];
        }
        m3 Qm;
        to_parent(dP, K, weight_at<ELEM>(q), Qm);
        scatter_grad<ELEM, NEN>(q, Qm, df);
    });
}

// Consistent-mass action of one element (Sec. 4.1): fe[a] += scale
// sum_q c_q s_a(xi_q) sum_b s_b(xi_q) u_b, with c_q = rho w_q J_p(xi_q)
// precomputed per element (coef, stride n_elem between points) and the
// mass rule's shape values compile-time constants.  su points at the u
// field of the node records.
template <int ELEM, int NEN>
__device__ __forceinline__ void mass_element(const double *su, const int (&na)[NEN], const double *coef,
                                             int64_t stride, double scale, double (&fe)[NEN][3], int part = 0)
{
    if constexpr (ELEM == kQ27) {
        // the stiffness rule; s_ijk = L_i L_j L_k, contracted one direction
        // at a time in both products
#pragma nounroll
        for (int q = part; q < 27; q += lanes_per_elem(kQ27)) {
            qp_fence();
            const Q27Pt t = q27_point(q);
            double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double uk[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double uj[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int c = 0; c < 3; ++c) uj[c] += t.L[0][i] * su[na[i + 3 * j + 9 * k] + c];
#pragma unroll
                    for (int c = 0; c < 3; ++c) uk[c] += t.L[1][j] * uj[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) u[c] += t.L[2][k] * uk[c];
            }
            const double cq = __builtin_nontemporal_load(coef + q * stride) * scale;
#pragma unroll
            for (int c = 0; c < 3; ++c) u[c] *= cq;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double v[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) v[c] = t.L[2][k] * t.L[1][j] * u[c];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int c = 0; c < 3; ++c) fe[i + 3 * j + 9 * k][c] += t.L[0][i] * v[c];
                }
        }
        return;
    } else {
    using M = MassRule<ELEM>;
    point_loop<M::nq>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        qp_fence();
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        static_for<NEN>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            constexpr double sb = M::shape(q, b);
            if constexpr (sb != 0.0) {
                u0 += sb * su[na[b]];
                u1 += sb * su[na[b] + 1];
                u2 += sb * su[na[b] + 2];
            }
        });
        const double cq = __builtin_nontemporal_load(coef + q * stride) * scale;
        u0 *= cq;
        u1 *= cq;
        u2 *= cq;
        static_for<NEN>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr double sa = M::shape(q, a);
            if constexpr (sa != 0.0) {
                fe[a][0] += sa * u0;
                fe[a][1] += sa * u1;
                fe[a][2] += sa * u2;
            }
        });
    });
    }
}

// ------------------------------------------------------------- tile plumbing

// The tiles of one class run as one grid.  Workgroups are handed to the
// eight XCDs round-robin; consecutive tiles (spatial neighbours sharing
// nodes) are mapped to the same XCD so that the node data they share is
// fetched into one L2.  Returns -1 for the surplus workgroups (at most seven)
// of the grid, which is rounded up to a multiple of eight.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int per = (n + 7) >> 3;
    const int t = (b & 7) * per + (b >> 3);
    return t < n ? t : -1;
}

// Value staged for field f (record order: x, then w or dx, then v, then
// dv; the step residual's u = v - v_n last; X comes from the mesh's tile
// records), component cc, global node g; null operands (dx or dv of the
// tangent) read as 0.  In the step modes the positions are the step map
// q = q_n + h v, formed with one rounding (a fused multiply-add) so that
// every node's value, and its difference to the tile's reference node,
// is the same in every call; the Newton operator's dx is h dv.
template <int OP, bool DAMPED, int MODE>
__device__ __forceinline__ double field_value(int f, int cc, int64_t g, const CallArgs &c, int64_t n)
{
    using R = Rec<OP, DAMPED, MODE>;
    const int64_t i = cc * n + g;
    if (f == R::ox / 3) return MODE == kModeStep ? __builtin_fma(c.h, c.v[i], c.qn[i]) : c.x[i];
    if (R::has2 && f == R::o2 / 3) {
        if (OP == kOpVjp) return c.w[i];
        if (MODE == kModeStep) return c.h * c.dv[i];
        return c.dx ? c.dx[i] : 0.0;
    }
    if (OP == kOpFwd && MODE == kModeStep && f == R::ou / 3) return c.v[i] - c.vn[i];
    if (DAMPED && f == R::ov / 3) return c.v[i];
    return c.dv ? c.dv[i] : 0.0;
}

// Stage the tile's node records.  The host caps a tile at SPT x (threads)
// nodes; every load of a thread's round of nodes is issued before its LDS
// stores (one round for T10 and H8, two for Q27).
// Reference and current positions are staged relative to the tile's
// reference node (the one nearest the tile's centroid): the kinematics only
// use differences of nodal positions (the parent
// gradients of an element sum to zero), and coordinates of the size of a
// tile instead of the size of the body keep the per-point gradient sums free
// of cancellation.  The reference part is read contiguously from the mesh,
// which stores it per tile node relative to the tile's reference node in
// every component where that subtraction is exact for all the tile's nodes
// (and as is elsewhere, where the coordinates are within a few tile widths
// of zero); the other fields are gathered from the caller's [3][n] arrays.
// RAW kernels, which difference positions per element (the REL forms below),
// stage the current positions as they are: the per-element difference of
// raw coordinates is then rounded once, where a difference of two
// tile-relative values near zero would carry the rounding of both.  The mesh's
// per-tile arrays are read once per call and are loaded non-temporally, which
// leaves the L2 to the node data that neighbouring tiles share.  The nodes
// are read in the tile's sorted node order (coalesced) and each record goes
// to the node's LDS position, which the host chose to spread the per-point
// gathers of a wavefront over the LDS banks.
template <int OP, bool DAMPED, int MODE = kModePlain, bool RAW = false, int SPT = kStagePerThread>
__device__ __forceinline__ void stage_tile(double *__restrict__ sm, const DevMesh &m, const CallArgs &c,
                                           const TileDesc &t, int tid, int nthr)
{
    using R = Rec<OP, DAMPED, MODE>;
    constexpr int nf = R::nfield;
    constexpr int CH = SPT < kStageRound ? SPT : kStageRound;   // nodes per thread per round
    static_assert(SPT % CH == 0, "staging rounds");
    const int32_t *gid = m.lnode_gid + t.node_begin;
    const uint16_t *lpos = m.lnode_pos + t.node_begin;
    const int64_t n = m.n_nodes;
    const int g0 = gid[t.ref];
#pragma unroll
    for (int k0 = 0; k0 < SPT; k0 += CH) {
        // lanes past the tile's last node load its last node again (a valid
        // address) and store nothing: unconditional loads issue back to
        // back, where guarded ones made the compiler wait at every join
        int g[CH], p[CH], lc[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int l = tid + (k0 + k) * nthr;
            lc[k] = l < t.n_node ? l : t.n_node - 1;
            g[k] = __builtin_nontemporal_load(gid + lc[k]);
            p[k] = (int)__builtin_nontemporal_load(lpos + lc[k]);
        }
        double v[CH][3 * R::nfield];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const double *xt = m.Xt + cc * m.n_tnode + t.node_begin;
#pragma unroll
            for (int k = 0; k < CH; ++k) v[k][R::oX + cc] = __builtin_nontemporal_load(xt + lc[k]);
        }
#pragma unroll
        for (int f = 1; f < nf; ++f) {
            const bool centre = !RAW && f == R::ox / 3;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const double o = centre ? field_value<OP, DAMPED, MODE>(f, cc, g0, c, n) : 0.0;
#pragma unroll
                for (int k = 0; k < CH; ++k) v[k][3 * f + cc] = field_value<OP, DAMPED, MODE>(f, cc, g[k], c, n) - o;
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (tid + (k0 + k) * nthr < t.n_node) {
                double *d = sm + (int64_t)p[k] * R::len;
#pragma unroll
                for (int j = 0; j < 3 * nf; ++j) d[j] = v[k][j];
            }
    }
}

// Record offsets of the lane's element nodes (local connectivity [nen][te]).
template <int NEN, int LEN>
__device__ __forceinline__ void load_na(const DevMesh &m, const TileDesc &t, int i, int te, int (&na)[NEN])
{
#pragma unroll
    for (int a = 0; a < NEN; ++a) na[a] = (int)__builtin_nontemporal_load(m.conn_local + t.conn_begin + a * te + i) * LEN;
}

// The tile's assembly tables in LDS, written while the node records are
// staged.  The element slots a * te + i of the tile form one list, grouped by
// local node (CSR order, the first entry of every node's group flagged with
// kSlotHead); thread j sums the entries [j C, j C + C) of that list, C =
// slot_chunk(NEN, LPE), and cn[j] is the local node of its first entry.
struct TileCsr {
    uint16_t *cn;      // [nthr]: local node of entry j * C
    int32_t *dst;      // [n_node]: >= 0 global node written directly; < 0: -1 - partial slot
    uint16_t *slot;    // [nen * n_elem]: element slot a * te + i of each entry (| kSlotHead)
};

// LDS layout of a tile: the node records (later overwritten by the element
// slots of nc components), then the assembly tables.
__device__ __forceinline__ TileCsr csr_layout(double *smem, int nl, int rec_len, int nen, int te, int nc, int nthr)
{
    const int a = max(nl * rec_len, nc * nen * te);   // doubles
    TileCsr c;
    c.cn = reinterpret_cast<uint16_t *>(smem + a);
    c.dst = reinterpret_cast<int32_t *>(c.cn + nthr);
    c.slot = reinterpret_cast<uint16_t *>(c.dst + nl);
    return c;
}

// The tile's assembly tables, in two steps: load() issues the global loads
// (into registers) and store() writes the LDS tables, so that a kernel can
// issue the node records' loads in between and both sets are in flight
// together (store() ends in a loop of data-dependent length, past which the
// compiler does not move later loads).  The tables are read once per call
// and loaded non-temporally.  The slot ids are copied as 32-bit words; a
// tile's entries start at an even global index (the host pads every tile's
// list to an even length).  The owner of local node l (list range
// [p0, p1)) writes cn[j] = l for every chunk start j C inside that range.
template <int NEN, int SPT = kStagePerThread, int LPE = 1>
struct CsrStage {
    static constexpr int C = slot_chunk(NEN, LPE);
    // NEN * n_elem entries = NEN * n_elem / 2 words over te * LPE threads:
    // at most NEN / (2 LPE) words per thread
    static constexpr int W = (NEN + 2 * LPE - 1) / (2 * LPE);
    int32_t p0[SPT], p1[SPT], dv[SPT];
    uint32_t wv[W];

    __device__ __forceinline__ void load(const DevMesh &m, const TileDesc &t, int tid, int nthr)
    {
        const int32_t *gptr = m.lnode_ptr + t.ptr_begin;
        const int32_t base = gptr[0];
        // lanes past the end load the last entry again (stored by nobody):
        // unconditional loads issue back to back
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int l = tid + k * nthr;
            const int lc = l < t.n_node ? l : t.n_node - 1;
            p0[k] = __builtin_nontemporal_load(gptr + lc) - base;
            p1[k] = __builtin_nontemporal_load(gptr + lc + 1) - base;
            dv[k] = __builtin_nontemporal_load(m.lnode_dst + t.node_begin + lc);
        }
        const int n_words = (NEN * t.n_elem + 1) / 2;
        const uint32_t *gw = reinterpret_cast<const uint32_t *>(m.lnode_slot + base);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int e = tid + k * nthr;
            wv[k] = __builtin_nontemporal_load(gw + (e < n_words ? e : n_words - 1));
        }
    }

    __device__ __forceinline__ void store(const TileCsr &c, const TileDesc &t, int tid, int nthr) const
    {
        const int n_words = (NEN * t.n_elem + 1) / 2;
        uint32_t *sw = reinterpret_cast<uint32_t *>(c.slot);
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (tid + k * nthr < n_words) sw[tid + k * nthr] = wv[k];
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int l = tid + k * nthr;
            if (l < t.n_node) {
                c.dst[l] = dv[k];
                for (int j = (p0[k] + C - 1) / C; j * C < p1[k]; ++j) c.cn[j] = (uint16_t)l;
            }
        }
    }
};

// Sum, for every local node, its element slots (list order) of the
// components r0 .. r0 + NC - 1 (slot region of component r0 + k at
// k * slot_stride) and write each value to the output (node owned by this
// tile only) or to the node's partial slot (shared node, partial row
// 3 * field + r).  Thread j walks its C entries once (a node by node walk
// took as many rounds as the wave's largest group): every group that starts
// and ends inside the chunk is summed there; the part of a group running
// into the chunk from the left (its leading part) is finished by the thread
// that holds the group's first entry, which adds the leading parts of the
// following chunks in their order.  Each node's value is therefore the same
// in every call.  A component's slot region is free once every thread holds
// its values (a barrier): the node sums go there at the node's index, the
// leading parts after them, and a node-parallel pass writes the results
// out.  G components per pass (fewer values in flight where other
// accumulators are still live).
template <int NC, int C, int G>
__device__ __forceinline__ void reduce_chunks(const DevMesh &m, const TileDesc &t, const TileCsr &c,
                                              double *__restrict__ slot, int slot_stride,
                                              double *__restrict__ out, const double *__restrict__ sub,
                                              int field, int r0, int tid, int nthr, int nen)
{
    static_assert(NC % G == 0, "component passes");
    static_assert(C % 2 == 0, "chunks start at even entries (the list is read as 32-bit words)");
    const int E = nen * t.n_elem, nl = t.n_node;
    const int e0 = tid * C;
    const int ne = min(C, E - e0);   // <= 0: no entries
    // unconditional LDS reads (clamped to the tables), masked afterwards
    const int ct = min(tid, (E - 1) / C);
    const int l = c.cn[ct];
    const int nx = c.cn[min(ct + 1, (E - 1) / C)];
    const int next = ne > 0 && e0 + C < E ? nx : -1;
    uint32_t raw[C];
    {
        const uint32_t *sw = reinterpret_cast<const uint32_t *>(c.slot);
        const int w0 = e0 >> 1, wl = (E - 1) >> 1;
#pragma unroll
        for (int k = 0; k < C / 2; ++k) {
            const uint32_t wd = sw[min(w0 + k, wl)];
            raw[2 * k] = 2 * k < ne ? (wd & 0xffffu) : 0u;
            raw[2 * k + 1] = 2 * k + 1 < ne ? (wd >> 16) : 0u;
        }
    }
    const bool lead = ne > 0 && !(raw[0] & kSlotHead);   // the chunk starts inside a group
    int nid[C];   // node of every entry
    {
        int cur = l;
#pragma unroll
        for (int u = 0; u < C; ++u) {
            if (u > 0 && (raw[u] & kSlotHead)) ++cur;
            nid[u] = cur;
        }
    }
    const int last = nid[C - 1];                              // the chunk's last group
    const bool owner = ne > 0 && !(lead && last == l) && next == last;   // starts here, runs on
    double own[NC];
#pragma unroll
    for (int r1 = 0; r1 < NC; r1 += G) {
        double v[C][G];
#pragma unroll
        for (int u = 0; u < C; ++u) {
            const int id = (int)(raw[u] & (kSlotHead - 1));
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double x = slot[(r1 + g) * slot_stride + id];
                v[u][g] = u < ne ? x : 0.0;
            }
        }
        __syncthreads();   // these components' slots are read: their regions take the sums
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double *sums = slot + (r1 + g) * slot_stride;   // [nl] node sums, then [nthr] leading parts
            // entries past the chunk's end have no flag and the value 0
            double run = 0.0;
            bool inlead = lead;
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const bool h = u > 0 && (raw[u] & kSlotHead);
                if (h) sums[inlead ? nl + tid : nid[u] - 1] = run;
                run = (h ? 0.0 : run) + v[u][g];
                inlead = inlead && !h;
            }
            // the last group: a leading part (the whole chunk), a finished
            // group, or one that runs into the next chunks
            if (ne > 0 && !owner) sums[inlead ? nl + tid : last] = run;
            own[r1 + g] = run;
        }
    }
    __syncthreads();
    if (owner) {
        // chunk tid + k starts inside the group while cn[tid + k] == last
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            const double *sums = slot + r * slot_stride;
            double s = own[r];
            for (int k = 1; tid + k < nthr && (tid + k) * C < E && c.cn[tid + k] == last; ++k) s += sums[nl + tid + k];
            slot[r * slot_stride + last] = s;
        }
    }
    __syncthreads();
    for (int q = tid; q < nl; q += nthr) {
        const int d = c.dst[q];
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            const double v = slot[r * slot_stride + q];
            if (d >= 0) {
                const int64_t o = (r0 + r) * m.n_nodes + d;
                out[o] = sub ? v - sub[o] : v;
            } else {
                m.part[(int64_t)(3 * field + r0 + r) * m.n_part + (-1 - d)] = v;
            }
        }
    }
}

// Deterministic assembly of the element vectors of a tile, NC components per
// round (the host picks NC so that NC x NEN x te slot doubles fit the
// workgroup's LDS); the slots a * te + i overwrite the node records, which
// are dead once every lane is done.
template <int NEN, int NC, int LPE, bool LEAN>
__device__ __forceinline__ void assemble_nc(const DevMesh &m, const TileDesc &t, const TileCsr &c,
                                            double *__restrict__ sm, const double (&fe)[NEN][3], bool active,
                                            double *__restrict__ out, const double *__restrict__ sub, int field,
                                            int tid, int te)
{
    const int stride = NEN * te;
    const int ie = tid / LPE, part = tid % LPE, nthr = te * LPE;
#pragma unroll
    for (int r0 = 0; r0 < 3; r0 += NC) {
        __syncthreads();
        if (active && part == 0) {
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (r0 + k < 3) {
#pragma unroll
                    for (int a = 0; a < NEN; ++a) sm[k * stride + a * te + ie] = fe[a][r0 + k];
                }
        }
        __syncthreads();
        constexpr int C = slot_chunk(NEN, LPE);
        if (r0 + NC <= 3) reduce_chunks<NC, C, LEAN ? 1 : NC>(m, t, c, sm, stride, out, sub, field, r0, tid, nthr, NEN);
        else reduce_chunks<(3 % NC) ? (3 % NC) : 1, C, 1>(m, t, c, sm, stride, out, sub, field, r0, tid, nthr, NEN);
    }
}

// LPE lanes per element (Q27: 2): every lane holds its element's whole
// vector (the lanes' sums, see lane_sum) and the first lane of each element
// writes its slots.  LEAN: one component per pass of the reduction (for
// kernels that keep other accumulators live meanwhile).
template <int NEN, int LPE = 1, bool LEAN = false>
__device__ __forceinline__ void assemble(const DevMesh &m, const TileDesc &t, const TileCsr &c,
                                         double *__restrict__ sm, const double (&fe)[NEN][3], bool active,
                                         double *__restrict__ out, int field, int tid, int te, int nc,
                                         const double *__restrict__ sub = nullptr)
{
    if (nc >= 3) assemble_nc<NEN, 3, LPE, LEAN>(m, t, c, sm, fe, active, out, sub, field, tid, te);
    else if (nc == 2) assemble_nc<NEN, 2, LPE, LEAN>(m, t, c, sm, fe, active, out, sub, field, tid, te);
    else assemble_nc<NEN, 1, LPE, LEAN>(m, t, c, sm, fe, active, out, sub, field, tid, te);
}

// Sum of the partial element vectors of an element's LPE lanes (neighbours
// in the wavefront), left in every one of them: a butterfly over lane
// distances 1, 2, ..., whose additions give the same value in every lane
// (x + y and y + x are the same number).  Run by every lane.
template <int LPE, int N>
__device__ __forceinline__ void lane_sum(double (&v)[N][3])
{
    if constexpr (LPE > 1) {
#pragma unroll
        for (int off = 1; off < LPE; off <<= 1)
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int r = 0; r < 3; ++r) v[a][r] += __shfl_xor(v[a][r], off, 64);
    }
}

// Zeros for every destination of the tile's nodes (an undamped tile's share
// of the velocity adjoint).
__device__ __forceinline__ void zero_nodes(const DevMesh &m, const TileDesc &t, const TileCsr &c,
                                           double *__restrict__ out, int field, int tid, int nthr)
{
    for (int l = tid; l < t.n_node; l += nthr) {
        const int d = c.dst[l];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (d >= 0) out[r * m.n_nodes + d] = 0.0;
            else m.part[(int64_t)(3 * field + r) * m.n_part + (-1 - d)] = 0.0;
        }
    }
}

// ----------------------------------------------------------------- kernels

#define TLFEA_MAX_TE 256



// The forward internal force (MODE plain), or the backward-Euler step
// residual without constraints (MODE step, Sec. 7): positions q = q_n + h v,
// g = f_int(q, v) + M (v - v_n) / h - f_ext, the inertia term from the
// consistent mass (Sec. 4.1) and f_ext subtracted at every node's store.
template <int ELEM, int LAW, bool DAMPED, int MODE>
__global__ __launch_bounds__(TLFEA_MAX_TE) __attribute__((amdgpu_waves_per_eu(waves_per_simd(kOpFwd, ELEM, LAW, DAMPED, MODE)))) void k_fwd(DevMesh m, CallArgs c, int tile0, int ntile, int te, int nl, int nc)
{
    constexpr int NEN = ElemDef<ELEM>::nen;
    constexpr int LPE = lanes_per_elem(ELEM);
    using R = Rec<kOpFwd, DAMPED, MODE>;
    extern __shared__ double smem[];
    const int ti = xcd_tile(blockIdx.x, ntile);
    if (ti < 0) return;
    const TileDesc t = m.tiles[tile0 + ti];
    const int tid = threadIdx.x, ie = tid / LPE, part = tid % LPE, nthr = te * LPE;
    // staging issues long-latency loads: its waves go first while other
    // tiles on the compute unit compute
    __builtin_amdgcn_s_setprio(3);
    const TileCsr csr = csr_layout(smem, nl, R::len, NEN, te, nc, nthr);
    CsrStage<NEN, stage_per_thread(ELEM), LPE> cs;
    cs.load(m, t, tid, nthr);
    stage_tile<kOpFwd, DAMPED, MODE, true, stage_per_thread(ELEM)>(smem, m, c, t, tid, nthr);
    cs.store(csr, t, tid, nthr);
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    double fe[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a) fe[a][0] = fe[a][1] = fe[a][2] = 0.0;
    const bool active = ie < t.n_elem;
    if (active) {
        int na[NEN];
        load_na<NEN, R::len>(m, t, ie, te, na);
        const int uid = m.elem_uid[t.elem_begin + ie];
        const Mat mt = load_mat<LAW>(m.blocks[t.block], c.theta, m.n_elem, uid, DAMPED);
        fwd_element<ELEM, LAW, DAMPED, MODE>(smem, na, mt, fe, part);
        if constexpr (MODE == kModeStep)
            if (m.mass_c)
                mass_element<ELEM>(smem + R::ou, na, m.mass_c + t.elem_begin + ie, m.n_elem, 1.0 / c.h, fe, part);
    }
    lane_sum<LPE>(fe);
    assemble<NEN, LPE>(m, t, csr, smem, fe, active, c.out0, 0, tid, te, nc, MODE == kModeStep ? c.sub : nullptr);
}

// Two waves per SIMD (256 registers); the damped Mooney-Rivlin adjoint, which
// needs more than that and spilled 488 B per lane there, runs at one wave
// per SIMD with its whole state in registers (24 % faster).
template <int ELEM, int LAW, bool DAMPED, bool WANT_GT>
__global__ __launch_bounds__(TLFEA_MAX_TE) __attribute__((amdgpu_waves_per_eu(waves_per_simd(kOpVjp, ELEM, LAW, DAMPED)))) void k_vjp(DevMesh m, CallArgs c, int tile0, int ntile, int te, int nl, int nc)
{
    constexpr int NEN = ElemDef<ELEM>::nen;
    constexpr int LPE = lanes_per_elem(ELEM);
    using R = Rec<kOpVjp, DAMPED>;
    extern __shared__ double smem[];
    const int ti = xcd_tile(blockIdx.x, ntile);
    if (ti < 0) return;
    const TileDesc t = m.tiles[tile0 + ti];
    const int tid = threadIdx.x, ie = tid / LPE, part = tid % LPE, nthr = te * LPE;
    // staging issues long-latency loads: its waves go first while other
    // tiles on the compute unit compute
    __builtin_amdgcn_s_setprio(3);
    const TileCsr csr = csr_layout(smem, nl, R::len, NEN, te, nc, nthr);
    CsrStage<NEN, stage_per_thread(ELEM), LPE> cs;
    cs.load(m, t, tid, nthr);
    stage_tile<kOpVjp, DAMPED, kModePlain, WANT_GT && ELEM == kT10, stage_per_thread(ELEM)>(smem, m, c, t, tid, nthr);
    cs.store(csr, t, tid, nthr);
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    double gx[NEN][3], gv[NEN][3], gt[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) gx[a][r] = gv[a][r] = 0.0;
    const bool active = ie < t.n_elem;
    int uid = 0;
    if (active) {
        int na[NEN];
        load_na<NEN, R::len>(m, t, ie, te, na);
        uid = m.elem_uid[t.elem_begin + ie];
        const Mat mt = load_mat<LAW>(m.blocks[t.block], c.theta, m.n_elem, uid, DAMPED);
        vjp_element<ELEM, LAW, DAMPED, WANT_GT>(smem, na, mt, gx, gv, gt, part);
    }
    lane_sum<LPE>(gx);
    if constexpr (DAMPED) lane_sum<LPE>(gv);
    if constexpr (WANT_GT && LPE > 1) {
#pragma unroll
        for (int off = 1; off < LPE; off <<= 1)
#pragma unroll
            for (int r = 0; r < 5; ++r) gt[r] += __shfl_xor(gt[r], off, 64);
    }
    if (WANT_GT && active && part == 0) {
        // rows a law does not use (and the viscous rows when undamped) are 0
        c.gtheta[uid] = gt[0];
        c.gtheta[m.n_elem + uid] = (LAW == 1 || LAW == 0) ? gt[1] : 0.0;
        c.gtheta[2 * m.n_elem + uid] = LAW == 0 ? 0.0 : gt[2];
        c.gtheta[3 * m.n_elem + uid] = DAMPED ? gt[3] : 0.0;
        c.gtheta[4 * m.n_elem + uid] = DAMPED ? gt[4] : 0.0;
    }
    // gv (and the parameter gradients) are still live while gx is reduced
    if (c.out0) assemble<NEN, LPE, DAMPED>(m, t, csr, smem, gx, active, c.out0, 0, tid, te, nc);
    if (c.out1) {
        if constexpr (DAMPED) assemble<NEN, LPE>(m, t, csr, smem, gv, active, c.out1, 1, tid, te, nc);
        else zero_nodes(m, t, csr, c.out1, 1, tid, nthr);
    }
}

// The tangent stages dx (zeros when null) and, for damped blocks, dv (zeros
// when null), so one instantiation serves every combination; DT adds the
// parameter direction dtheta.  At least two waves per SIMD: left free, the
// compiler gave the Mooney-Rivlin tangent one wave and 512 registers, which
// ran about 20 % slower than two waves with a small spill.
// MODE step: the Newton operator of the step residual (Sec. 7),
// y = (M / h + h K + C) dv at q = q_n + h v: the tangent with dx = h dv and
// the inertia term M (h dv) / h^2 from the consistent mass (Sec. 4.1).
template <int ELEM, int LAW, bool DAMPED, bool DT, int MODE>
__global__ __launch_bounds__(TLFEA_MAX_TE) __attribute__((amdgpu_waves_per_eu(waves_per_simd(kOpJvp, ELEM, LAW, DAMPED, MODE)))) void k_jvp(DevMesh m, CallArgs c, int tile0, int ntile, int te, int nl, int nc)
{
    constexpr int NEN = ElemDef<ELEM>::nen;
    constexpr int LPE = lanes_per_elem(ELEM);
    using R = Rec<kOpJvp, DAMPED, MODE>;
    extern __shared__ double smem[];
    const int ti = xcd_tile(blockIdx.x, ntile);
    if (ti < 0) return;
    const TileDesc t = m.tiles[tile0 + ti];
    const int tid = threadIdx.x, ie = tid / LPE, part = tid % LPE, nthr = te * LPE;
    // staging issues long-latency loads: its waves go first while other
    // tiles on the compute unit compute
    __builtin_amdgcn_s_setprio(3);
    const TileCsr csr = csr_layout(smem, nl, R::len, NEN, te, nc, nthr);
    CsrStage<NEN, stage_per_thread(ELEM), LPE> cs;
    cs.load(m, t, tid, nthr);
    stage_tile<kOpJvp, DAMPED, MODE, false, stage_per_thread(ELEM)>(smem, m, c, t, tid, nthr);
    cs.store(csr, t, tid, nthr);
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    double df[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a) df[a][0] = df[a][1] = df[a][2] = 0.0;
    const bool active = ie < t.n_elem;
    if (active) {
        int na[NEN];
        load_na<NEN, R::len>(m, t, ie, te, na);
        const int uid = m.elem_uid[t.elem_begin + ie];
        const Mat mt = load_mat<LAW>(m.blocks[t.block], c.theta, m.n_elem, uid, DAMPED);
        Mat dmt{};
        if constexpr (DT) dmt = load_mat<LAW>(m.blocks[t.block], c.dtheta, m.n_elem, uid, DAMPED);
        jvp_element<ELEM, LAW, DAMPED, DT>(smem, na, mt, dmt, df, part);
        if constexpr (MODE == kModeStep)
            if (m.mass_c)
                mass_element<ELEM>(smem + R::o2, na, m.mass_c + t.elem_begin + ie, m.n_elem, 1.0 / (c.h * c.h), df,
                                   part);
    }
    lane_sum<LPE>(df);
    assemble<NEN, LPE>(m, t, csr, smem, df, active, c.out0, 0, tid, te, nc);
}

// Consistent-mass action y = M u (Sec. 4.1): the tile stages u only.
template <int ELEM>
__global__ __launch_bounds__(TLFEA_MAX_TE) void k_mass(DevMesh m, CallArgs c, int tile0, int ntile, int te, int nl, int nc)
{
    constexpr int NEN = ElemDef<ELEM>::nen;
    constexpr int LPE = lanes_per_elem(ELEM);
    constexpr int LEN = record_len(kOpMass, false);
    extern __shared__ double smem[];
    const int ti = xcd_tile(blockIdx.x, ntile);
    if (ti < 0) return;
    const TileDesc t = m.tiles[tile0 + ti];
    const int tid = threadIdx.x, ie = tid / LPE, part = tid % LPE, nthr = te * LPE;
    const TileCsr csr = csr_layout(smem, nl, LEN, NEN, te, nc, nthr);
    constexpr int SPT = stage_per_thread(ELEM);
    CsrStage<NEN, SPT, LPE> cs;
    cs.load(m, t, tid, nthr);
    {
        const int32_t *gid = m.lnode_gid + t.node_begin;
        const uint16_t *lpos = m.lnode_pos + t.node_begin;
        int g[SPT], p[SPT];
        double v[SPT][3];
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int l = tid + k * nthr;
            const int lc = l < t.n_node ? l : t.n_node - 1;
            g[k] = __builtin_nontemporal_load(gid + lc);
            p[k] = (int)__builtin_nontemporal_load(lpos + lc);
        }
#pragma unroll
        for (int k = 0; k < SPT; ++k)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) v[k][cc] = c.x[cc * m.n_nodes + g[k]];
#pragma unroll
        for (int k = 0; k < SPT; ++k)
            if (tid + k * nthr < t.n_node)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) smem[p[k] * LEN + cc] = v[k][cc];
    }
    cs.store(csr, t, tid, nthr);
    __syncthreads();
    double fe[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a) fe[a][0] = fe[a][1] = fe[a][2] = 0.0;
    const bool active = ie < t.n_elem;
    if (active && m.mass_c) {
        int na[NEN];
        load_na<NEN, LEN>(m, t, ie, te, na);
        mass_element<ELEM>(smem, na, m.mass_c + t.elem_begin + ie, m.n_elem, 1.0, fe, part);
    }
    lane_sum<LPE>(fe);
    assemble<NEN, LPE>(m, t, csr, smem, fe, active, c.out0, 0, tid, te, nc);
}

// Quadrature points with det F <= 0 (inverted or collapsed there).  The
// paper constrains only the reference map (J_p > 0, Sec. 6); the forward
// evaluates the laws at such points anyway and this count reports them.  The
// tile stages X and x, every lane forms F at its element's points as the
// forward does, and each wavefront adds its count to *count with one
// integer atomic (the total does not depend on the order).
template <int ELEM>
__global__ __launch_bounds__(TLFEA_MAX_TE) void k_inverted(DevMesh m, CallArgs c, int tile0, int ntile, int te,
                                                          unsigned long long *count)
{
    constexpr int NEN = ElemDef<ELEM>::nen;
    using E = ElemDef<ELEM>;
    using R = Rec<kOpFwd, false>;
    extern __shared__ double smem[];
    const int ti = xcd_tile(blockIdx.x, ntile);
    if (ti < 0) return;
    const TileDesc t = m.tiles[tile0 + ti];
    constexpr int LPE = lanes_per_elem(ELEM);
    const int tid = threadIdx.x, ie = tid / LPE, part = tid % LPE;
    stage_tile<kOpFwd, false, kModePlain, true, stage_per_thread(ELEM)>(smem, m, c, t, tid, te * LPE);
    __syncthreads();
    int n = 0;
    if (ie < t.n_elem) {
        int na[NEN];
        load_na<NEN, R::len>(m, t, ie, te, na);
        for_points<ELEM>(part, [&](auto q) {
            m3 K, G, F, cof;
            double detJ, r;
            ref_geometry<ELEM, NEN, true>(q, smem + R::oX, na, K, detJ, r);
            grad_field<ELEM, NEN, true>(q, smem + R::ox, na, G);
            to_reference(G, K, r, F);
            cofactor(F, cof);
            n += det_from_cof(F, cof) <= 0.0 ? 1 : 0;
        });
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off, 64);
    if ((tid & 63) == 0 && n > 0) atomicAdd(count, (unsigned long long)n);
}

template <int ELEM>
hipError_t launch_inverted_class(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m,
                                 const CallArgs &c, int tile0, unsigned long long *count)
{
    if (n_tiles <= 0) return hipSuccess;
    const int nthr = te * lanes_per_elem(ELEM);
    if (te <= 0 || nthr > TLFEA_MAX_TE || (nthr & 63)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(8 * ((n_tiles + 7) / 8)));
    k_inverted<ELEM><<<grid, nthr, lds, s>>>(m, c, tile0, n_tiles, te, count);
    return hipGetLastError();
}

template <int OP, int ELEM, int LAW, bool DAMPED, int GT, int MODE>
hipError_t launch_one(dim3 grid, int te, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c, int tile0,
                      int ntile, int nl, int nc)
{
    const int nthr = te * lanes_per_elem(ELEM);
    if constexpr (OP == kOpFwd) k_fwd<ELEM, LAW, DAMPED, MODE><<<grid, nthr, lds, s>>>(m, c, tile0, ntile, te, nl, nc);
    else if constexpr (OP == kOpVjp) {
        // one adjoint translation unit per gtheta choice (each with the
        // instruction scheduler that suits it); the host picks the unit
        if ((c.gtheta != nullptr) != (GT != 0)) return hipErrorInvalidValue;
        k_vjp<ELEM, LAW, DAMPED, GT != 0><<<grid, nthr, lds, s>>>(m, c, tile0, ntile, te, nl, nc);
    } else if constexpr (MODE == kModeStep) {
        k_jvp<ELEM, LAW, DAMPED, false, kModeStep><<<grid, nthr, lds, s>>>(m, c, tile0, ntile, te, nl, nc);
    } else {
        if (c.dtheta) k_jvp<ELEM, LAW, DAMPED, true, kModePlain><<<grid, nthr, lds, s>>>(m, c, tile0, ntile, te, nl, nc);
        else k_jvp<ELEM, LAW, DAMPED, false, kModePlain><<<grid, nthr, lds, s>>>(m, c, tile0, ntile, te, nl, nc);
    }
    return hipGetLastError();
}

// GT: which adjoint a unit instantiates (part of the template arguments, so
// that the two adjoint units' launchers are distinct functions); MODE: the
// plain operation or its step variant (forward: step residual, tangent:
// Newton operator).
template <int OP, int ELEM, int GT, int MODE>
hipError_t launch_class(int law, int damped, int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m,
                        const CallArgs &c, int tile0, int nl, int nc)
{
    if (n_tiles <= 0) return hipSuccess;
    const int nthr = te * lanes_per_elem(ELEM);
    if (te <= 0 || nthr > TLFEA_MAX_TE || (nthr & 63)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(8 * ((n_tiles + 7) / 8)));
    switch (law * 2 + (damped ? 1 : 0)) {
    case 0: return launch_one<OP, ELEM, 0, false, GT, MODE>(grid, te, lds, s, m, c, tile0, n_tiles, nl, nc);
    case 1: return launch_one<OP, ELEM, 0, true, GT, MODE>(grid, te, lds, s, m, c, tile0, n_tiles, nl, nc);
    case 2: return launch_one<OP, ELEM, 1, false, GT, MODE>(grid, te, lds, s, m, c, tile0, n_tiles, nl, nc);
    case 3: return launch_one<OP, ELEM, 1, true, GT, MODE>(grid, te, lds, s, m, c, tile0, n_tiles, nl, nc);
    case 4: return launch_one<OP, ELEM, 2, false, GT, MODE>(grid, te, lds, s, m, c, tile0, n_tiles, nl, nc);
    case 5: return launch_one<OP, ELEM, 2, true, GT, MODE>(grid, te, lds, s, m, c, tile0, n_tiles, nl, nc);
    default: return hipErrorInvalidValue;
    }
}

template <int ELEM>
hipError_t launch_mass_class(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                             int tile0, int nl, int nc)
{
    if (n_tiles <= 0) return hipSuccess;
    const int nthr = te * lanes_per_elem(ELEM);
    if (te <= 0 || nthr > TLFEA_MAX_TE || (nthr & 63)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(8 * ((n_tiles + 7) / 8)));
    k_mass<ELEM><<<grid, nthr, lds, s>>>(m, c, tile0, n_tiles, te, nl, nc);
    return hipGetLastError();
}

}  // namespace tlfea

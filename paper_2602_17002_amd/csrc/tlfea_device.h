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

struct Mat {
    double p0, p1, p2, mu_v, lam_v;
};

// Compiler-only barrier placed at the start of every quadrature point: node
// values are re-read from LDS per point instead of being kept live in
// registers across the unrolled point loop (which would cost 2 VGPRs per
// staged double and halve occupancy).
__device__ __forceinline__ void qp_fence() { __asm__ __volatile__("" ::: "memory"); }

// -------------------------------------------------------- per-point kinematics

// G = sum_a s[:, ln[a]] (ds_a/dxi at point Q)^T, node data read from LDS
// (row stride NL); zero gradient entries are removed at compile time.
//
// CENTRED evaluates the same sum relative to the element's first node,
// G = sum_{a>0} (s_a - s_0) (ds_a/dxi)^T, which is equal because the parent
// gradients of a complete element sum to zero (partition of unity).  Used for
// positions: a literal sum of coordinates of order 1 m against gradients of
// order 1/h (h = 1 cm) cancels about two decimal digits that the differences
// keep, so the result no longer depends on where the body sits in space.
template <int ELEM, int Q, bool CENTRED, int NEN>
__device__ __forceinline__ void grad_field(const double *__restrict__ s, int NL, const int (&ln)[NEN], m3 &G)
{
    using E = ElemDef<ELEM>;
    qp_fence();
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) G[i][k] = 0.0;
    const double o0 = CENTRED ? s[ln[0]] : 0.0;
    const double o1 = CENTRED ? s[NL + ln[0]] : 0.0;
    const double o2 = CENTRED ? s[2 * NL + ln[0]] : 0.0;
    static_for<NEN>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        if constexpr (!CENTRED || a > 0) {
            const double x0 = s[ln[a]] - o0, x1 = s[NL + ln[a]] - o1, x2 = s[2 * NL + ln[a]] - o2;
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

// out[a][r] += sum_k Q[r][k] (ds_a/dxi at point Q)_k   (i.e. c P h_a with Q = c P J^{-T})
template <int ELEM, int QP, int NEN>
__device__ __forceinline__ void scatter_grad(const m3 &Qm, double (&out)[NEN][3])
{
    using E = ElemDef<ELEM>;
    static_for<NEN>([&](auto ac) {
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

// Reference geometry at point Q: J = U G (Sec. 6), det J and J^{-1}.
template <int ELEM, int Q, int NEN>
__device__ __forceinline__ void ref_geometry(const double *__restrict__ sX, int NL, const int (&ln)[NEN], m3 &Ji,
                                             double &detJ)
{
    m3 J, C;
    grad_field<ELEM, Q, true>(sX, NL, ln, J);
    cofactor(J, C);
    detJ = det_from_cof(J, C);
    const double r = 1.0 / detJ;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Ji[i][j] = C[j][i] * r;
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

// Invariants and pieces shared by the Mooney-Rivlin stress and its derivative.
struct MRState {
    m3 FiT;          // F^{-T}
    double J, J23, I1;
    // Mooney-Rivlin (mu01) only
    m3 C, FC;
    double J43, I2;
};

template <int LAW>
__device__ __forceinline__ void mr_state(const m3 &F, MRState &st)
{
    m3 cof;
    cofactor(F, cof);
    st.J = det_from_cof(F, cof);
    const double invJ = 1.0 / st.J;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) st.FiT[i][j] = cof[i][j] * invJ;
    const double c = cbrt(invJ);          // J^{-1/3}
    st.J23 = c * c;                       // J^{-2/3}
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
template <int LAW, bool DAMPED>
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
        mr_state<LAW>(F, st);
        const double a = 2.0 * m.p0 * st.J23;
        const double b = -(2.0 / 3.0) * m.p0 * st.J23 * st.I1 + m.p2 * (st.J - 1.0) * st.J;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) P[i][j] = a * F[i][j] + b * st.FiT[i][j];
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

// Forward: fe[a] = sum_q w_q J_p P(F_q, Fdot_q) h_a   (Sec. 4.3 with Sec. 6)
template <int ELEM, int LAW, bool DAMPED, bool AFFINE, int NEN>
__device__ __forceinline__ void fwd_element(const double *sX, const double *sx, const double *sv, int NL,
                                            const int (&ln)[NEN], const Mat &mt, double (&fe)[NEN][3])
{
    using E = ElemDef<ELEM>;
    m3 Ji;
    double detJ;
    if constexpr (AFFINE) ref_geometry<ELEM, 0>(sX, NL, ln, Ji, detJ);
    static_for<E::nq>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        qp_fence();
        if constexpr (!AFFINE) ref_geometry<ELEM, q>(sX, NL, ln, Ji, detJ);
        m3 G, F, Fd, P;
        grad_field<ELEM, q, true>(sx, NL, ln, G);
        mm(G, Ji, F);                               // F = N H = (N dS/dxi) J^{-1}
        if constexpr (DAMPED) {
            grad_field<ELEM, q, false>(sv, NL, ln, G);
            mm(G, Ji, Fd);                          // Fdot = Ndot H
        }
        stress<LAW, DAMPED>(F, Fd, mt, P);
        const double c = E::weight(q) * detJ;
        m3 Qm;
        mmT(P, Ji, Qm);                             // P J^{-T}: P h_a = (P J^{-T}) dS_a/dxi
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Qm[i][j] *= c;
        scatter_grad<ELEM, q>(Qm, fe);
    });
}

// Adjoint: with Gw = sum_a w_a h_a^T and the identity w.f = sum_q c_q P:Gw,
//   gx_a += c_q Fbar_x h_a, Fbar_x = (dP_e/dF)[Gw] + Gw S_v + Fdot S_v[sym(F^T Gw)]
//   gv_a += c_q Fbar_v h_a, Fbar_v = F S_v[sym(F^T Gw)]
//   gtheta_p += c_q Gw : dP/dtheta_p   (P is linear in every parameter row)
template <int ELEM, int LAW, bool DAMPED, bool AFFINE, int NEN>
__device__ __forceinline__ void vjp_element(const double *sX, const double *sx, const double *sv, const double *sw,
                                            int NL, const int (&ln)[NEN], const Mat &mt, double (&gx)[NEN][3],
                                            double (&gv)[NEN][3], double (&gt)[5])
{
    using E = ElemDef<ELEM>;
    m3 Ji;
    double detJ;
    if constexpr (AFFINE) ref_geometry<ELEM, 0>(sX, NL, ln, Ji, detJ);
    static_for<E::nq>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        qp_fence();
        if constexpr (!AFFINE) ref_geometry<ELEM, q>(sX, NL, ln, Ji, detJ);
        m3 G, F, Fd, Gw, Fb;
        grad_field<ELEM, q, true>(sx, NL, ln, G);
        mm(G, Ji, F);
        grad_field<ELEM, q, false>(sw, NL, ln, G);
        mm(G, Ji, Gw);
        const double c = E::weight(q) * detJ;
        MRState st;
        if constexpr (LAW != 0) mr_state<LAW>(F, st);
        delastic<LAW>(F, mt, Gw, st, Fb);
        const double GF = ddot(Gw, F);
        // parameter gradients
        if constexpr (LAW == 0) {
            m3 C, A;
            mTm(F, F, C);
            mTm(F, Gw, A);
            const double trE = 0.5 * (C[0][0] + C[1][1] + C[2][2] - 3.0);
            double EA = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) EA += 0.5 * (C[i][j] - (i == j ? 1.0 : 0.0)) * A[i][j];
            gt[0] += c * trE * GF;
            gt[1] += c * 2.0 * EA;
        } else {
            const double GFiT = ddot(Gw, st.FiT);
            gt[0] += c * 2.0 * st.J23 * (GF - (1.0 / 3.0) * st.I1 * GFiT);
            if constexpr (LAW == 1)
                gt[1] += c * 2.0 * st.J43 * (st.I1 * GF - ddot(Gw, st.FC) - (2.0 / 3.0) * st.I2 * GFiT);
            gt[2] += c * (st.J - 1.0) * st.J * GFiT;
        }
        if constexpr (DAMPED) {
            grad_field<ELEM, q, false>(sv, NL, ln, G);
            mm(G, Ji, Fd);
            m3 Ed, Sv, Sg, SvSg, T, A;
            sym_FtG(F, Fd, Ed);
            visc_op(mt, Ed, Sv);
            sym_FtG(F, Gw, Sg);
            visc_op(mt, Sg, SvSg);             // S_v[sym(F^T Gw)]
            // parameter gradients of the viscous branch
            double EdSg = ddot(Ed, Sg);
            gt[3] += c * 2.0 * EdSg;
            gt[4] += c * (Ed[0][0] + Ed[1][1] + Ed[2][2]) * GF;
            mm(Gw, Sv, T);
            mm(Fd, SvSg, A);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Fb[i][j] += T[i][j] + A[i][j];
            mm(F, SvSg, A);                        // Fbar_v
            mmT(A, Ji, T);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) T[i][j] *= c;
            scatter_grad<ELEM, q>(T, gv);
        }
        m3 Qm;
        mmT(Fb, Ji, Qm);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Qm[i][j] *= c;
        scatter_grad<ELEM, q>(Qm, gx);
    });
}

// Tangent: dF = sum_a dx_a h_a^T, dFdot = sum_a dv_a h_a^T,
//   dP = (dP_e/dF)[dF] + dF S_v + F S_v[sym(dF^T Fdot + F^T dFdot)],
//   df_a += c_q dP h_a.
template <int ELEM, int LAW, bool DAMPED, bool AFFINE, int NEN>
__device__ __forceinline__ void jvp_element(const double *sX, const double *sx, const double *sv, const double *sdx,
                                            const double *sdv, int NL, const int (&ln)[NEN], const Mat &mt,
                                            double (&df)[NEN][3])
{
    using E = ElemDef<ELEM>;
    m3 Ji;
    double detJ;
    if constexpr (AFFINE) ref_geometry<ELEM, 0>(sX, NL, ln, Ji, detJ);
    static_for<E::nq>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        qp_fence();
        if constexpr (!AFFINE) ref_geometry<ELEM, q>(sX, NL, ln, Ji, detJ);
        m3 G, F, dF, dP;
        grad_field<ELEM, q, true>(sx, NL, ln, G);
        mm(G, Ji, F);
        {
            grad_field<ELEM, q, false>(sdx, NL, ln, G);
            mm(G, Ji, dF);
            MRState st;
            if constexpr (LAW != 0) mr_state<LAW>(F, st);
            delastic<LAW>(F, mt, dF, st, dP);
        }
        if constexpr (DAMPED) {
            m3 Fd, Ed, Sv, A, B, T;
            grad_field<ELEM, q, false>(sv, NL, ln, G);
            mm(G, Ji, Fd);
            sym_FtG(F, Fd, Ed);
            visc_op(mt, Ed, Sv);
            {
                mm(dF, Sv, T);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) dP[i][j] += T[i][j];
                mTm(dF, Fd, A);                   // dF^T Fdot
            }
            {
                m3 dFd;
                grad_field<ELEM, q, false>(sdv, NL, ln, G);
                mm(G, Ji, dFd);
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
        }
        const double c = E::weight(q) * detJ;
        m3 Qm;
        mmT(dP, Ji, Qm);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Qm[i][j] *= c;
        scatter_grad<ELEM, q>(Qm, df);
    });
}

// ------------------------------------------------------------- tile plumbing

// Stage the tile's nodes: dst[c * NL + l] = src[c * n + gid[l]].
__device__ __forceinline__ void stage(double *__restrict__ dst, const double *__restrict__ src, int64_t n,
                                      const int32_t *__restrict__ gid, int n_node, int NL, int tid, int nthreads)
{
    for (int l = tid; l < n_node; l += nthreads) {
        const int g = gid[l];
        dst[l] = src[g];
        dst[NL + l] = src[n + g];
        dst[2 * NL + l] = src[2 * n + g];
    }
}

// Write one element's nodal vectors to LDS at slot a * TE + i (row r at
// r * NEN * TE), a layout in which consecutive lanes hit consecutive words.
template <int NEN>
__device__ __forceinline__ void put_slots(double *__restrict__ sf, const double (&v)[NEN][3], int i, int te)
{
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) sf[r * NEN * te + a * te + i] = v[a][r];
}

// Sum the slots of every local node in CSR order and write the node's value
// either to the output vector (node owned by this tile only) or to its
// partial slot (node shared between tiles).
template <int NEN>
__device__ __forceinline__ void reduce_nodes(const DevMesh &m, const TileDesc &t, const double *__restrict__ sf,
                                             double *__restrict__ out, int field, int tid, int te)
{
    const int32_t *ptr = m.lnode_ptr + t.ptr_begin;
    const int32_t *dst = m.lnode_dst + t.node_begin;
    const int row = NEN * te;
    for (int l = tid; l < t.n_node; l += te) {
        const int p0 = ptr[l], p1 = ptr[l + 1];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int p = p0; p < p1; ++p) {
            const int sl = m.lnode_slot[p];
            s0 += sf[sl];
            s1 += sf[row + sl];
            s2 += sf[2 * row + sl];
        }
        const int d = dst[l];
        if (d >= 0) {
            out[d] = s0;
            out[m.n_nodes + d] = s1;
            out[2 * m.n_nodes + d] = s2;
        } else {
            double *pp = m.part + (int64_t)(3 * field) * m.n_part + (-1 - d);
            pp[0] = s0;
            pp[m.n_part] = s1;
            pp[2 * m.n_part] = s2;
        }
    }
}

// Write zeros to every destination of the tile's nodes for output `field`
// (an undamped tile's share of the velocity adjoint).
__device__ __forceinline__ void zero_nodes(const DevMesh &m, const TileDesc &t, double *__restrict__ out, int field,
                                           int tid, int te)
{
    const int32_t *dst = m.lnode_dst + t.node_begin;
    for (int l = tid; l < t.n_node; l += te) {
        const int d = dst[l];
        if (d >= 0) {
            out[d] = 0.0;
            out[m.n_nodes + d] = 0.0;
            out[2 * m.n_nodes + d] = 0.0;
        } else {
            double *pp = m.part + (int64_t)(3 * field) * m.n_part + (-1 - d);
            pp[0] = 0.0;
            pp[m.n_part] = 0.0;
            pp[2 * m.n_part] = 0.0;
        }
    }
}

template <int NEN>
__device__ __forceinline__ void load_ln(const DevMesh &m, const TileDesc &t, int i, int te, int (&ln)[NEN])
{
#pragma unroll
    for (int a = 0; a < NEN; ++a) ln[a] = m.conn_local[t.conn_begin + a * te + i];
}

// ----------------------------------------------------------------- kernels

// Stage the tile's nodes of an optional operand; a null operand stages zeros.
__device__ __forceinline__ void stage_or_zero(double *__restrict__ dst, const double *__restrict__ src, int64_t n,
                                              const int32_t *__restrict__ gid, int n_node, int NL, int tid, int nthreads)
{
    if (src) {
        stage(dst, src, n, gid, n_node, NL, tid, nthreads);
    } else {
        for (int l = tid; l < n_node; l += nthreads) dst[l] = dst[NL + l] = dst[2 * NL + l] = 0.0;
    }
}

#define TLFEA_MAX_TE 256

template <int ELEM, int LAW, bool DAMPED>
__global__ __launch_bounds__(TLFEA_MAX_TE) void k_fwd(DevMesh m, CallArgs c, int tile0, int NL, int te)
{
    using E = ElemDef<ELEM>;
    constexpr int NEN = E::nen;
    extern __shared__ double smem[];
    const TileDesc t = m.tiles[tile0 + blockIdx.x];
    const int tid = threadIdx.x;
    double *sX = smem, *sx = smem + 3 * NL, *sv = smem + 6 * NL;
    const int32_t *gid = m.lnode_gid + t.node_begin;
    stage(sX, m.X, m.n_nodes, gid, t.n_node, NL, tid, te);
    stage(sx, c.x, m.n_nodes, gid, t.n_node, NL, tid, te);
    if constexpr (DAMPED) stage(sv, c.v, m.n_nodes, gid, t.n_node, NL, tid, te);
    __syncthreads();

    double fe[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a) fe[a][0] = fe[a][1] = fe[a][2] = 0.0;
    const bool active = tid < t.n_elem;
    if (active) {
        int ln[NEN];
        load_ln(m, t, tid, te, ln);
        const int uid = m.elem_uid[t.elem_begin + tid];
        const Mat mt = load_mat<LAW>(m.blocks[t.block], c.theta, m.n_elem, uid, DAMPED);
        if (t.flags & kTileAffine)
            fwd_element<ELEM, LAW, DAMPED, true>(sX, sx, sv, NL, ln, mt, fe);
        else
            fwd_element<ELEM, LAW, DAMPED, false>(sX, sx, sv, NL, ln, mt, fe);
    }
    __syncthreads();
    if (active) put_slots<NEN>(smem, fe, tid, te);
    __syncthreads();
    reduce_nodes<NEN>(m, t, smem, c.out0, 0, tid, te);
}

template <int ELEM, int LAW, bool DAMPED>
__global__ __launch_bounds__(TLFEA_MAX_TE) void k_vjp(DevMesh m, CallArgs c, int tile0, int NL, int te)
{
    using E = ElemDef<ELEM>;
    constexpr int NEN = E::nen;
    extern __shared__ double smem[];
    const TileDesc t = m.tiles[tile0 + blockIdx.x];
    const int tid = threadIdx.x;
    double *sX = smem, *sx = smem + 3 * NL, *sw = smem + 6 * NL, *sv = smem + 9 * NL;
    const int32_t *gid = m.lnode_gid + t.node_begin;
    stage(sX, m.X, m.n_nodes, gid, t.n_node, NL, tid, te);
    stage(sx, c.x, m.n_nodes, gid, t.n_node, NL, tid, te);
    stage(sw, c.w, m.n_nodes, gid, t.n_node, NL, tid, te);
    if constexpr (DAMPED) stage(sv, c.v, m.n_nodes, gid, t.n_node, NL, tid, te);
    __syncthreads();

    double gx[NEN][3], gv[NEN][3], gt[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) gx[a][r] = gv[a][r] = 0.0;
    const bool active = tid < t.n_elem;
    if (active) {
        int ln[NEN];
        load_ln(m, t, tid, te, ln);
        const int uid = m.elem_uid[t.elem_begin + tid];
        const Mat mt = load_mat<LAW>(m.blocks[t.block], c.theta, m.n_elem, uid, DAMPED);
        if (t.flags & kTileAffine)
            vjp_element<ELEM, LAW, DAMPED, true>(sX, sx, sv, sw, NL, ln, mt, gx, gv, gt);
        else
            vjp_element<ELEM, LAW, DAMPED, false>(sX, sx, sv, sw, NL, ln, mt, gx, gv, gt);
        if (c.gtheta) {
            // rows a law does not use (and the viscous rows when undamped) are 0
            c.gtheta[uid] = gt[0];
            c.gtheta[m.n_elem + uid] = (LAW == 1 || LAW == 0) ? gt[1] : 0.0;
            c.gtheta[2 * m.n_elem + uid] = LAW == 0 ? 0.0 : gt[2];
            c.gtheta[3 * m.n_elem + uid] = DAMPED ? gt[3] : 0.0;
            c.gtheta[4 * m.n_elem + uid] = DAMPED ? gt[4] : 0.0;
        }
    }
    if (c.out0) {
        __syncthreads();
        if (active) put_slots<NEN>(smem, gx, tid, te);
        __syncthreads();
        reduce_nodes<NEN>(m, t, smem, c.out0, 0, tid, te);
    }
    if (c.out1) {
        if constexpr (DAMPED) {
            __syncthreads();
            if (active) put_slots<NEN>(smem, gv, tid, te);
            __syncthreads();
            reduce_nodes<NEN>(m, t, smem, c.out1, 1, tid, te);
        } else {
            zero_nodes(m, t, c.out1, 1, tid, te);
        }
    }
}

// The tangent stages dx (zeros when null) and, for damped blocks, dv (zeros
// when null), so one instantiation serves every combination.
template <int ELEM, int LAW, bool DAMPED>
__global__ __launch_bounds__(TLFEA_MAX_TE) void k_jvp(DevMesh m, CallArgs c, int tile0, int NL, int te)
{
    using E = ElemDef<ELEM>;
    constexpr int NEN = E::nen;
    extern __shared__ double smem[];
    const TileDesc t = m.tiles[tile0 + blockIdx.x];
    const int tid = threadIdx.x;
    double *sX = smem, *sx = smem + 3 * NL, *sdx = smem + 6 * NL, *sv = smem + 9 * NL, *sdv = smem + 12 * NL;
    const int32_t *gid = m.lnode_gid + t.node_begin;
    stage(sX, m.X, m.n_nodes, gid, t.n_node, NL, tid, te);
    stage(sx, c.x, m.n_nodes, gid, t.n_node, NL, tid, te);
    stage_or_zero(sdx, c.dx, m.n_nodes, gid, t.n_node, NL, tid, te);
    if constexpr (DAMPED) {
        stage(sv, c.v, m.n_nodes, gid, t.n_node, NL, tid, te);
        stage_or_zero(sdv, c.dv, m.n_nodes, gid, t.n_node, NL, tid, te);
    }
    __syncthreads();

    double df[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a) df[a][0] = df[a][1] = df[a][2] = 0.0;
    const bool active = tid < t.n_elem;
    if (active) {
        int ln[NEN];
        load_ln(m, t, tid, te, ln);
        const int uid = m.elem_uid[t.elem_begin + tid];
        const Mat mt = load_mat<LAW>(m.blocks[t.block], c.theta, m.n_elem, uid, DAMPED);
        if (t.flags & kTileAffine)
            jvp_element<ELEM, LAW, DAMPED, true>(sX, sx, sv, sdx, sdv, NL, ln, mt, df);
        else
            jvp_element<ELEM, LAW, DAMPED, false>(sX, sx, sv, sdx, sdv, NL, ln, mt, df);
    }
    __syncthreads();
    if (active) put_slots<NEN>(smem, df, tid, te);
    __syncthreads();
    reduce_nodes<NEN>(m, t, smem, c.out0, 0, tid, te);
}

template <int OP, int ELEM, int LAW, bool DAMPED>
hipError_t launch_one(dim3 grid, int te, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c, int tile0,
                      int NL)
{
    if constexpr (OP == kOpFwd) k_fwd<ELEM, LAW, DAMPED><<<grid, te, lds, s>>>(m, c, tile0, NL, te);
    else if constexpr (OP == kOpVjp) k_vjp<ELEM, LAW, DAMPED><<<grid, te, lds, s>>>(m, c, tile0, NL, te);
    else k_jvp<ELEM, LAW, DAMPED><<<grid, te, lds, s>>>(m, c, tile0, NL, te);
    return hipGetLastError();
}

template <int OP, int ELEM>
hipError_t launch_class(int law, int damped, int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m,
                        const CallArgs &c, int tile0, int NL)
{
    if (n_tiles <= 0) return hipSuccess;
    if (te <= 0 || te > TLFEA_MAX_TE || (te & 63)) return hipErrorInvalidValue;
    const dim3 grid(n_tiles);
    switch (law * 2 + (damped ? 1 : 0)) {
    case 0: return launch_one<OP, ELEM, 0, false>(grid, te, lds, s, m, c, tile0, NL);
    case 1: return launch_one<OP, ELEM, 0, true>(grid, te, lds, s, m, c, tile0, NL);
    case 2: return launch_one<OP, ELEM, 1, false>(grid, te, lds, s, m, c, tile0, NL);
    case 3: return launch_one<OP, ELEM, 1, true>(grid, te, lds, s, m, c, tile0, NL);
    case 4: return launch_one<OP, ELEM, 2, false>(grid, te, lds, s, m, c, tile0, NL);
    case 5: return launch_one<OP, ELEM, 2, true>(grid, te, lds, s, m, c, tile0, NL);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tlfea

// Parent-element data of the library: shape-function gradients at the
// quadrature points, and the quadrature rules themselves.  Everything is
// constexpr so that, inside fully unrolled device loops over (q, a, k), every
// gradient entry is a compile-time constant and zero entries vanish.
#pragma once

#ifdef __HIPCC__
#define TLFEA_HD __host__ __device__
#else
#define TLFEA_HD
#endif

namespace tlfea {

enum { kT10 = 0, kH8 = 1, kQ27 = 2 };

template <int ELEM> struct ElemDef;

// 10-node quadratic tetrahedron on the unit parent tetrahedron (App. A).
// Quadrature: 5-point degree-3 rule (centroid weight -4/5, four points with
// weight 9/20, times the parent volume 1/6).
template <> struct ElemDef<kT10> {
    static constexpr int nen = 10, nq = 5;
    static constexpr TLFEA_HD double qp(int q, int k)
    {
        return q == 0 ? 0.25 : ((q >= 2 && k == q - 2) ? 0.5 : 1.0 / 6.0);
    }
    static constexpr TLFEA_HD double weight(int q)
    {
        return q == 0 ? (-4.0 / 5.0) / 6.0 : (9.0 / 20.0) / 6.0;
    }
    // d s_a / d xi_k at parent point (x, y, z) = (xi, eta, zeta); the rows are
    // the paper's gradient matrix of App. A (10-node tetrahedron).
    static constexpr TLFEA_HD double grad_at(int a, int k, double x, double y, double z)
    {
        switch (a) {
        case 0: return 4 * x + 4 * y + 4 * z - 3;
        case 1: return k == 0 ? 4 * x - 1 : 0.0;
        case 2: return k == 1 ? 4 * y - 1 : 0.0;
        case 3: return k == 2 ? 4 * z - 1 : 0.0;
        case 4: return k == 0 ? -8 * x - 4 * y - 4 * z + 4 : -4 * x;
        case 5: return k == 0 ? 4 * y : (k == 1 ? 4 * x : 0.0);
        case 6: return k == 1 ? -4 * x - 8 * y - 4 * z + 4 : -4 * y;
        case 7: return k == 2 ? -4 * x - 4 * y - 8 * z + 4 : -4 * z;
        case 8: return k == 0 ? 4 * z : (k == 2 ? 4 * x : 0.0);
        default: return k == 1 ? 4 * z : (k == 2 ? 4 * y : 0.0);
        }
    }
    static constexpr TLFEA_HD double grad(int q, int a, int k)
    {
        return grad_at(a, k, qp(q, 0), qp(q, 1), qp(q, 2));
    }
    // s_a at parent point (x, y, z): the paper's shape functions of App. A
    // (10-node tetrahedron), written through the barycentric coordinate
    // l = 1 - x - y - z of the first corner
    static constexpr TLFEA_HD double shape_at(int a, double x, double y, double z)
    {
        const double l = 1.0 - x - y - z;
        switch (a) {
        case 0: return l * (2 * l - 1);
        case 1: return x * (2 * x - 1);
        case 2: return y * (2 * y - 1);
        case 3: return z * (2 * z - 1);
        case 4: return 4 * x * l;
        case 5: return 4 * x * y;
        case 6: return 4 * y * l;
        case 7: return 4 * z * l;
        case 8: return 4 * x * z;
        default: return 4 * y * z;
        }
    }
    // the four corner nodes (the first four)
    static constexpr int n_corner = 4;
    static constexpr TLFEA_HD int corner(int c) { return c; }
};

// 8-node trilinear hexahedron on [-1,1]^3 (not in the paper), nodes
// lexicographic with i fastest; 2x2x2 Gauss-Legendre rule, weights 1.
template <> struct ElemDef<kH8> {
    static constexpr int nen = 8, nq = 8;
    static constexpr double g = 0.57735026918962576451;   // 1/sqrt(3)
    static constexpr TLFEA_HD double sgn(int a, int k) { return ((a >> k) & 1) ? 1.0 : -1.0; }
    static constexpr TLFEA_HD double qp(int q, int k) { return ((q >> k) & 1) ? g : -g; }
    static constexpr TLFEA_HD double weight(int) { return 1.0; }
    static constexpr TLFEA_HD double grad_at(int a, int k, double x, double y, double z)
    {
        const double p[3] = {x, y, z};
        double r = 0.125 * sgn(a, k);
        for (int j = 0; j < 3; ++j)
            if (j != k) r *= 1.0 + sgn(a, j) * p[j];
        return r;
    }
    static constexpr TLFEA_HD double grad(int q, int a, int k)
    {
        return grad_at(a, k, qp(q, 0), qp(q, 1), qp(q, 2));
    }
    static constexpr TLFEA_HD double shape_at(int a, double x, double y, double z)
    {
        return 0.125 * (1.0 + sgn(a, 0) * x) * (1.0 + sgn(a, 1) * y) * (1.0 + sgn(a, 2) * z);
    }
    static constexpr int n_corner = 8;
    static constexpr TLFEA_HD int corner(int c) { return c; }
};

// 27-node triquadratic hexahedron on [-1,1]^3 (App. A): node n = i + 3 j +
// 9 k at parent (i - 1, j - 1, k - 1), i fastest; s_n = L_i(xi) L_j(eta)
// L_k(zeta) with the 1-D quadratic Lagrange polynomials L_0(s) = s (s - 1) / 2,
// L_1(s) = 1 - s^2, L_2(s) = s (s + 1) / 2.  Quadrature: 3x3x3 Gauss-Legendre
// (points 0, +-sqrt(3/5), weights 8/9, 5/9), point q = p0 + 3 p1 + 9 p2 in the
// node order.  The kernels do not unroll over its 27 x 27 gradient table:
// they loop over the points at run time and contract the 1-D values of
// each point (lag1 / dlag1 at gauss(p)) one direction at a time.
template <> struct ElemDef<kQ27> {
    static constexpr int nen = 27, nq = 27;
    static constexpr double g = 0.77459666924148337704;   // sqrt(3/5)
    static constexpr TLFEA_HD double gauss(int p) { return p == 0 ? -g : (p == 1 ? 0.0 : g); }
    static constexpr TLFEA_HD double gauss_w(int p) { return p == 1 ? 8.0 / 9.0 : 5.0 / 9.0; }
    static constexpr TLFEA_HD double lag1(int i, double s)
    {
        return i == 0 ? 0.5 * s * (s - 1.0) : (i == 1 ? 1.0 - s * s : 0.5 * s * (s + 1.0));
    }
    static constexpr TLFEA_HD double dlag1(int i, double s) { return i == 0 ? s - 0.5 : (i == 1 ? -2.0 * s : s + 0.5); }
    static constexpr TLFEA_HD int digit(int n, int k) { return k == 0 ? n % 3 : (k == 1 ? (n / 3) % 3 : n / 9); }
    static constexpr TLFEA_HD double qp(int q, int k) { return gauss(digit(q, k)); }
    static constexpr TLFEA_HD double weight(int q)
    {
        return gauss_w(digit(q, 0)) * gauss_w(digit(q, 1)) * gauss_w(digit(q, 2));
    }
    static constexpr TLFEA_HD double grad_at(int a, int k, double x, double y, double z)
    {
        const double p[3] = {x, y, z};
        double r = 1.0;
        for (int j = 0; j < 3; ++j) r *= j == k ? dlag1(digit(a, j), p[j]) : lag1(digit(a, j), p[j]);
        return r;
    }
    static constexpr TLFEA_HD double grad(int q, int a, int k) { return grad_at(a, k, qp(q, 0), qp(q, 1), qp(q, 2)); }
    static constexpr TLFEA_HD double shape_at(int a, double x, double y, double z)
    {
        return lag1(digit(a, 0), x) * lag1(digit(a, 1), y) * lag1(digit(a, 2), z);
    }
    // the eight corner nodes (i, j, k in {0, 2})
    static constexpr int n_corner = 8;
    static constexpr TLFEA_HD int corner(int c) { return 2 * (c & 1) + 6 * ((c >> 1) & 1) + 18 * (c >> 2); }
};

// Quadrature of the consistent mass m_ij = int rho s_i s_j dV_r (Sec. 4.1),
// exact with positive weights for the integrand of straight-sided elements
// (twice the shape functions' degree), so the element mass matrix is the
// exact Gram matrix there.  T10: the 15-point degree-5 rule of Hammer,
// Marlowe and Stroud (barycentric orbits: the centroid; (a, a, a, 1 - 3a)
// for a = (7 -+ sqrt 15) / 34; (b, b, 1/2 - b, 1/2 - b) for
// b = (5 - sqrt 15) / 20), weights 16/135, (2665 +- 14 sqrt 15) / 37800 and
// 10/189 of the parent volume 1/6.  H8: the 2x2x2 Gauss rule.
template <int ELEM> struct MassRule;

template <> struct MassRule<kT10> {
    static constexpr int nq = 15;
    static constexpr double r15 = 3.8729833462074168851792653997823996108;   // sqrt(15)
    static constexpr double a1 = (7.0 - r15) / 34.0, a2 = (7.0 + r15) / 34.0;
    static constexpr double b = (5.0 - r15) / 20.0, c = 0.5 - b;
    // barycentric coordinate k (0..3) of point q; the parent coordinates
    // (xi, eta, zeta) are the barycentric coordinates 1..3
    static constexpr TLFEA_HD double bary(int q, int k)
    {
        if (q == 0) return 0.25;
        if (q <= 8) {
            const double a = q <= 4 ? a1 : a2;
            return k == (q - 1) % 4 ? 1.0 - 3.0 * a : a;
        }
        // pairs (i, j), i < j, in the order (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
        constexpr int pi[6] = {0, 0, 0, 1, 1, 2}, pj[6] = {1, 2, 3, 2, 3, 3};
        return (k == pi[q - 9] || k == pj[q - 9]) ? b : c;
    }
    static constexpr TLFEA_HD double qp(int q, int k) { return bary(q, k + 1); }
    static constexpr TLFEA_HD double weight(int q)
    {
        return (q == 0 ? 16.0 / 135.0
                       : q <= 4 ? (2665.0 + 14.0 * r15) / 37800.0
                                : q <= 8 ? (2665.0 - 14.0 * r15) / 37800.0 : 10.0 / 189.0) / 6.0;
    }
    static constexpr TLFEA_HD double shape(int q, int a) { return ElemDef<kT10>::shape_at(a, qp(q, 0), qp(q, 1), qp(q, 2)); }
    static constexpr TLFEA_HD double grad(int q, int a, int k)
    {
        return ElemDef<kT10>::grad_at(a, k, qp(q, 0), qp(q, 1), qp(q, 2));
    }
};

template <> struct MassRule<kH8> {
    static constexpr int nq = 8;
    static constexpr TLFEA_HD double qp(int q, int k) { return ElemDef<kH8>::qp(q, k); }
    static constexpr TLFEA_HD double weight(int q) { return ElemDef<kH8>::weight(q); }
    static constexpr TLFEA_HD double shape(int q, int a) { return ElemDef<kH8>::shape_at(a, qp(q, 0), qp(q, 1), qp(q, 2)); }
    static constexpr TLFEA_HD double grad(int q, int a, int k) { return ElemDef<kH8>::grad(q, a, k); }
};

// Q27: the stiffness rule (3x3x3 Gauss, exact for the mass integrand of a
// straight-sided element, degree 4 per direction).
template <> struct MassRule<kQ27> {
    static constexpr int nq = 27;
    static constexpr TLFEA_HD double qp(int q, int k) { return ElemDef<kQ27>::qp(q, k); }
    static constexpr TLFEA_HD double weight(int q) { return ElemDef<kQ27>::weight(q); }
    static constexpr TLFEA_HD double shape(int q, int a) { return ElemDef<kQ27>::shape_at(a, qp(q, 0), qp(q, 1), qp(q, 2)); }
    static constexpr TLFEA_HD double grad(int q, int a, int k) { return ElemDef<kQ27>::grad(q, a, k); }
};

}  // namespace tlfea

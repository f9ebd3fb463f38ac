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

enum { kT10 = 0, kH8 = 1 };

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
    // corners used to decide whether the parent-to-reference map is affine
    static constexpr int n_corner = 4;
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
    static constexpr int n_corner = 8;
};

}  // namespace tlfea

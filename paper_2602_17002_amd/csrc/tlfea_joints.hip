// Revolute joints (Sec. 2.2: three coordinate-difference rows and two
// dot-product-1 rows, row weights of App. B.1): constraint values and the
// transpose scatter h C^T (lambda + rho c) into a nodal vector.
//
// One lane per joint evaluates the five material points (point evaluation
// over the hosting element's nodes, Sec. 2.1), the directions, the
// row-normalised values, and the vector each point receives; one lane per
// touched node then sums its entries (shape value x point vector) in a
// fixed order, so the scatter is bitwise repeatable without atomics.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "tlfea_joints.h"

namespace tlfea {

// r of point p of joint j: sum over the hosting element's nodes, in slot
// order, from the node-major copy qn of the positions (one cache line per
// gathered node instead of one per coordinate array).  The slots are read
// kSlotBatch at a time with every load of a batch in flight together (slot
// by slot, each slot waited for its shape value and node id, then for the
// node's coordinates: two dependent round trips per slot); slots past nmax
// reread the last one and unused slots (shape value 0, node 0) are not
// added.
constexpr int kSlotBatch = 10;

__device__ __forceinline__ void point_eval(const DevJoints &J, const double *__restrict__ qn, int p, int64_t j,
                                           double r[3])
{
    r[0] = r[1] = r[2] = 0.0;
    for (int i0 = 0; i0 < J.nmax; i0 += kSlotBatch) {
        double s[kSlotBatch], v[kSlotBatch][3];
        int32_t g[kSlotBatch];
#pragma unroll
        for (int u = 0; u < kSlotBatch; ++u) {
            const int i = min(i0 + u, J.nmax - 1);
            const int64_t k = ((int64_t)p * J.nmax + i) * J.n_joints + j;
            s[u] = i0 + u < J.nmax ? J.sv[k] : 0.0;
            g[u] = J.ids[k];
        }
#pragma unroll
        for (int u = 0; u < kSlotBatch; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[u][c] = qn[3 * (int64_t)g[u] + c];
#pragma unroll
        for (int u = 0; u < kSlotBatch; ++u)
            if (s[u] != 0.0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) r[c] += s[u] * v[u][c];
            }
    }
}

__device__ __forceinline__ double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// c_hat (n_joints x 5, joint-major) and, when z is wanted, the vector each
// point receives: z_X = h sum_k w_k eta_k dc_k/dr_X, eta = lambda + rho c_hat.
// qn[g][c] = q[c][g]: the caller's [3][n_nodes] positions node-major
__global__ __launch_bounds__(256) void k_node_major(const double *__restrict__ q, double *__restrict__ qn, int64_t n)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) qn[3 * g + c] = q[c * n + g];
}

__global__ __launch_bounds__(256) void k_joints(DevJoints J, const double *__restrict__ qn,
                                                const double *__restrict__ lambda, double rho, double h,
                                                double *__restrict__ c_out, int want_z)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J.n_joints) return;
    double r[5][3];
#pragma unroll
    for (int p = 0; p < 5; ++p) point_eval(J, qn, p, j, r[p]);
    double a[3], b1[3], b2[3], d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c] = r[1][c] - r[0][c];     // Q - P
        b1[c] = r[3][c] - r[2][c];    // S - R
        b2[c] = r[4][c] - r[2][c];    // T - R
        d[c] = r[2][c] - r[0][c];     // R - P
    }
    const double f1 = J.fw[j], f2 = J.fw[J.n_joints + j];
    const double w4 = J.fw[2 * J.n_joints + j], w5 = J.fw[3 * J.n_joints + j];
    double ch[5] = {d[0], d[1], d[2], w4 * (dot3(a, b1) - f1), w5 * (dot3(a, b2) - f2)};
    if (c_out)
#pragma unroll
        for (int k = 0; k < 5; ++k) c_out[j * 5 + k] = ch[k];
    if (!want_z) return;
    double e[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) e[k] = (lambda ? lambda[j * 5 + k] : 0.0) + rho * ch[k];
    // rows weighted once more: C_hat^T eta = (dc/dq)^T W eta
    e[3] *= w4;
    e[4] *= w5;
    double z[5][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        z[0][c] = -e[c] - e[3] * b1[c] - e[4] * b2[c];   // P: CD rows -e_c, DP1 rows -b_j
        z[1][c] = e[3] * b1[c] + e[4] * b2[c];           // Q: +b_j
        z[2][c] = e[c] - (e[3] + e[4]) * a[c];           // R: CD rows +e_c, DP1 rows -a
        z[3][c] = e[3] * a[c];                           // S: +a (first DP1 row)
        z[4][c] = e[4] * a[c];                           // T: +a (second DP1 row)
    }
#pragma unroll
    for (int p = 0; p < 5; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) J.z[(j * 5 + p) * 3 + c] = h * z[p][c];
}

// out[node] (+)= sum over the node's entries of s * z[entry's point], in
// entry order, kEntryBatch entries at a time with their loads in flight
// together (entries past the node's last reread it and are not added)
constexpr int kEntryBatch = 8;

__global__ __launch_bounds__(256) void k_joint_scatter(DevJoints J, double *__restrict__ out, int accumulate)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= J.n_touched) return;
    const int64_t g = J.tnode[t];
    const int64_t k0 = J.tptr[t], k1 = J.tptr[t + 1];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t kb = k0; kb < k1; kb += kEntryBatch) {
        int64_t e[kEntryBatch];
        double v[kEntryBatch], z[kEntryBatch][3];
#pragma unroll
        for (int u = 0; u < kEntryBatch; ++u) {
            const int64_t k = kb + u < k1 ? kb + u : k1 - 1;
            e[u] = J.tent[k];                                // row 5 j + p
            v[u] = J.tval[k];
        }
#pragma unroll
        for (int u = 0; u < kEntryBatch; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) z[u][c] = J.z[3 * e[u] + c];
#pragma unroll
        for (int u = 0; u < kEntryBatch; ++u)
            if (kb + u < k1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) s[c] += v[u] * z[u][c];
            }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double *o = out + c * J.n_nodes + g;
        *o = accumulate ? *o + s[c] : s[c];
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = 0.0;
}

hipError_t launch_joints(const DevJoints &J, const double *q, const double *lambda, double rho, double h,
                         double *c_out, int want_z, hipStream_t s)
{
    if (J.n_joints <= 0) return hipSuccess;
    k_node_major<<<dim3((unsigned)((J.n_nodes + 255) / 256)), 256, 0, s>>>(q, J.qn, J.n_nodes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_joints<<<dim3((unsigned)((J.n_joints + 255) / 256)), 256, 0, s>>>(J, J.qn, lambda, rho, h, c_out, want_z);
    return hipGetLastError();
}

hipError_t launch_joint_scatter(const DevJoints &J, double *out, int accumulate, hipStream_t s)
{
    if (!accumulate && J.n_nodes > 0) {
        const int64_t n = 3 * J.n_nodes;
        k_fill_zero<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(out, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (J.n_touched <= 0) return hipSuccess;
    // after the fill every touched node accumulates onto 0 (the same sum)
    k_joint_scatter<<<dim3((unsigned)((J.n_touched + 255) / 256)), 256, 0, s>>>(J, out, 1);
    return hipGetLastError();
}

}  // namespace tlfea

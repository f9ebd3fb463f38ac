// Vector kernels of the matrix-free Newton-Krylov step (restarted GMRES on
// the Newton operator of the step residual): dot products with a fixed
// reduction order (every result bitwise repeatable), linear combinations,
// scaling.  Vectors are the solver's flat [3 n_nodes] arrays.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "tlfea_internal.h"

namespace tlfea {

struct Coeffs {
    double c[kVecChunk];
};

// partial[k][b] = sum over block b's entries of V_k . w, k < nvec (<= 8),
// V_k = V + k * ldv.  Block b (of kDotBlocks, four per compute unit, so
// that enough loads are in flight) takes entries b * 256 + t, b * 256 + t +
// 256 * kDotBlocks, ...; the block's sum is a fixed tree over its threads.
template <int NV>
__global__ __launch_bounds__(256) void k_mdot(const double *__restrict__ V, int64_t ldv, const double *__restrict__ w,
                                              int64_t n, double *__restrict__ partial)
{
    __shared__ double red[NV][256];
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)256 * kDotBlocks) {
        const double wi = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += V[k * ldv + i] * wi;
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
#pragma unroll
            for (int k = 0; k < NV; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partial[k * kDotBlocks + blockIdx.x] = red[k][0];
}

// y += sum_k c_k V_k, k < NV
template <int NV>
__global__ __launch_bounds__(256) void k_maxpy(const double *__restrict__ V, int64_t ldv, Coeffs c,
                                               double *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double t = y[i];
#pragma unroll
    for (int k = 0; k < NV; ++k) t += c.c[k] * V[k * ldv + i];
    y[i] = t;
}

// y = a x + b y (b = 0 ignores y's old contents)
__global__ __launch_bounds__(256) void k_axpby(double a, const double *__restrict__ x, double b, double *__restrict__ y,
                                               int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// z = x + y
__global__ __launch_bounds__(256) void k_add(const double *__restrict__ x, const double *__restrict__ y,
                                             double *__restrict__ z, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    z[i] = x[i] + y[i];
}

// One sweep of classical Gram-Schmidt over V_0..V_{NV-1} (NV <= kCgsMax)
// and the work vector w, block b of kDotBlocks taking the entries of
// k_mdot's partition in the same order:
//   MODE 0: partial[k][b] = V_k . w                 (the first projections)
//   MODE 1: w += sum_k c_k V_k, then partial[k][b] = V_k . w   (the first
//           update fused with the second projections)
//   MODE 2: w += sum_k c_k V_k, then partial[0][b] = w . w     (the second
//           update fused with the norm)
// c is a device array (the negated projections, so that no host round trip
// sits between the sweeps).  Every multiply-add and every block sum is the
// one k_maxpy and k_mdot do, in the same order, so the results equal
// theirs bit for bit; the basis is read three times per iteration instead
// of four.
template <int MODE, int NV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_cgs(const double *__restrict__ V, int64_t ldv,
                                             const double *__restrict__ c, double *__restrict__ w, int64_t n,
                                             double *__restrict__ partial)
{
    constexpr int NS = MODE == 2 ? 1 : NV;
    __shared__ double red[256];
    double s[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = 0.0;
    double ck[MODE >= 1 ? NV : 1];
    if constexpr (MODE >= 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) ck[k] = c[k];
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)256 * kDotBlocks) {
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = V[k * ldv + i];
        double wi = w[i];
        if constexpr (MODE >= 1) {
#pragma unroll
            for (int k = 0; k < NV; ++k) wi += ck[k] * v[k];
            w[i] = wi;
        }
        if constexpr (MODE <= 1) {
#pragma unroll
            for (int k = 0; k < NV; ++k) s[k] += v[k] * wi;
        } else {
            s[0] += wi * wi;
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        red[threadIdx.x] = s[k];
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[k * kDotBlocks + blockIdx.x] = red[0];
        __syncthreads();
    }
}

template <int MODE, int NV = 1>
static hipError_t cgs_dispatch(int nv, const double *V, int64_t ldv, const double *c, double *w, int64_t n,
                               double *partial, hipStream_t s)
{
    if constexpr (NV > kCgsMax) {
        return hipErrorInvalidValue;
    } else {
        if (nv != NV) return cgs_dispatch<MODE, NV + 1>(nv, V, ldv, c, w, n, partial, s);
        k_cgs<MODE, NV><<<kDotBlocks, 256, 0, s>>>(V, ldv, c, w, n, partial);
        return hipGetLastError();
    }
}

// out[k] = sum of vector k's block partials in block order (the host's
// order), neg[k] = -out[k] when neg is given.  One block per vector stages
// the partials in LDS with all its threads (one round trip) and its first
// thread adds them in order: a single thread loading them one by one waited
// on every load (25 us per call).
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partial, double *__restrict__ out,
                                                      double *__restrict__ neg)
{
    __shared__ double p[kDotBlocks];
    const int k = blockIdx.x;
    for (int b = threadIdx.x; b < kDotBlocks; b += 256) p[b] = partial[(int64_t)k * kDotBlocks + b];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) t += p[b];
    out[k] = t;
    if (neg) neg[k] = -t;
}

static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_cgs(int mode, const double *V, int64_t ldv, int nv, const double *c, double *w, int64_t n,
                      double *partial, hipStream_t s)
{
    if (nv < 1 || nv > kCgsMax) return hipErrorInvalidValue;
    switch (mode) {
    case 0: return cgs_dispatch<0>(nv, V, ldv, c, w, n, partial, s);
    case 1: return cgs_dispatch<1>(nv, V, ldv, c, w, n, partial, s);
    case 2: return cgs_dispatch<2>(nv, V, ldv, c, w, n, partial, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sum_partials(const double *partial, int nvec, double *out, double *neg, hipStream_t s)
{
    if (nvec <= 0) return hipSuccess;
    k_sum_partials<<<dim3((unsigned)nvec), 256, 0, s>>>(partial, out, neg);
    return hipGetLastError();
}

hipError_t launch_mdot(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *partial,
                       hipStream_t s)
{
    switch (nvec) {
    case 1: k_mdot<1><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 2: k_mdot<2><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 3: k_mdot<3><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 4: k_mdot<4><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 5: k_mdot<5><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 6: k_mdot<6><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 7: k_mdot<7><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    case 8: k_mdot<8><<<kDotBlocks, 256, 0, s>>>(V, ldv, w, n, partial); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_maxpy(const double *V, int64_t ldv, int nvec, const double *c, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    Coeffs cc{};
    for (int k = 0; k < nvec && k < kVecChunk; ++k) cc.c[k] = c[k];
    switch (nvec) {
    case 1: k_maxpy<1><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 2: k_maxpy<2><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 3: k_maxpy<3><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 4: k_maxpy<4><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 5: k_maxpy<5><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 6: k_maxpy<6><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 7: k_maxpy<7><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    case 8: k_maxpy<8><<<grid_of(n), 256, 0, s>>>(V, ldv, cc, y, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_axpby<<<grid_of(n), 256, 0, s>>>(a, x, b, y, n);
    return hipGetLastError();
}

hipError_t launch_add(const double *x, const double *y, double *z, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_add<<<grid_of(n), 256, 0, s>>>(x, y, z, n);
    return hipGetLastError();
}

}  // namespace tlfea

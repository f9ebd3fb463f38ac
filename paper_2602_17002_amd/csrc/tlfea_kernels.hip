// One translation unit per (element type, operation): compiled with
// -DTLFEA_ELEM=<0|1> -DTLFEA_OP=<0|1|2> so the instantiations build in
// parallel; the adjoint has two units, -DTLFEA_VJP_GT=<0|1>.  The (T10, forward) unit also holds the shared-node kernel.
#include "tlfea_device.h"

#ifndef TLFEA_ELEM
#error "TLFEA_ELEM must be defined"
#endif
#ifndef TLFEA_OP
#error "TLFEA_OP must be defined"
#endif

#ifndef TLFEA_VJP_GT
#define TLFEA_VJP_GT 0
#endif

#define TLFEA_CAT2(a, b, c) a##_e##b##_o##c
#define TLFEA_CAT(a, b, c) TLFEA_CAT2(a, b, c)
#define TLFEA_CATG2(a, b, c, g) a##_e##b##_o##c##_g##g
#define TLFEA_CATG(a, b, c, g) TLFEA_CATG2(a, b, c, g)

namespace tlfea {

#if TLFEA_OP == 1
// the adjoint units: one per gtheta choice (-DTLFEA_VJP_GT=0|1)
hipError_t TLFEA_CATG(launch_tiles, TLFEA_ELEM, TLFEA_OP, TLFEA_VJP_GT)(int law, int damped, int te, int n_tiles,
                                                                        size_t lds, hipStream_t s, const DevMesh &m,
                                                                        const CallArgs &c, int tile0, int nl, int nc)
#else
hipError_t TLFEA_CAT(launch_tiles, TLFEA_ELEM, TLFEA_OP)(int law, int damped, int te, int n_tiles, size_t lds,
                                                          hipStream_t s, const DevMesh &m, const CallArgs &c,
                                                          int tile0, int nl, int nc)
#endif
{
    return launch_class<TLFEA_OP, TLFEA_ELEM, TLFEA_VJP_GT>(law, damped, te, n_tiles, lds, s, m, c, tile0, nl, nc);
}

#if TLFEA_OP == 0
hipError_t TLFEA_CAT(launch_inverted, TLFEA_ELEM, TLFEA_OP)(int te, int n_tiles, size_t lds, hipStream_t s,
                                                             const DevMesh &m, const CallArgs &c, int tile0,
                                                             unsigned long long *count)
{
    return launch_inverted_class<TLFEA_ELEM>(te, n_tiles, lds, s, m, c, tile0, count);
}
#endif

#if TLFEA_ELEM == 0 && TLFEA_OP == 0
__global__ void k_zero_count(unsigned long long *count) { *count = 0ull; }

hipError_t launch_zero_count(hipStream_t s, unsigned long long *count)
{
    k_zero_count<<<1, 1, 0, s>>>(count);
    return hipGetLastError();
}

// Nodes shared between tiles (and nodes no element touches): sum the node's
// partial slots, which are contiguous and in tile order.  One lane per node;
// up to two output fields.  Partials are read eight at a time (every load of
// a lane in flight together); the sum still runs in tile order.
__global__ __launch_bounds__(256) void k_halo(DevMesh m, double *out0, double *out1)
{
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= m.n_halo) return;
    const int g = m.halo_gid[h];
    const int p0 = m.halo_ptr[h], p1 = m.halo_ptr[h + 1];
    double *outs[2] = {out0, out1};
    constexpr int U = 8;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        double *out = outs[f];
        if (!out) continue;
        double s[3] = {0.0, 0.0, 0.0};
        for (int p = p0; p < p1; p += U) {
            double v[3][U];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double *part = m.part + (int64_t)(3 * f + r) * m.n_part;
#pragma unroll
                for (int u = 0; u < U; ++u) v[r][u] = p + u < p1 ? part[p + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    if (p + u < p1) s[r] += v[r][u];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) out[r * m.n_nodes + g] = s[r];
    }
}

hipError_t launch_halo(hipStream_t s, const DevMesh &m, double *out0, double *out1)
{
    if (m.n_halo <= 0) return hipSuccess;
    const dim3 grid((unsigned)((m.n_halo + 255) / 256));
    k_halo<<<grid, 256, 0, s>>>(m, out0, out1);
    return hipGetLastError();
}
#endif

}  // namespace tlfea

// One translation unit per (element type, operation, variant): compiled
// with -DTLFEA_ELEM=<0|1|2> -DTLFEA_OP=<0|1|2> so the instantiations build in
// parallel; the adjoint has two units, -DTLFEA_VJP_GT=<0|1>, and the forward
// and the tangent two, -DTLFEA_MODE=<0|1> (the plain operation, or the step
// residual / Newton operator; the step forward unit also holds the mass
// action).  The (T10, forward, plain) unit also holds the shared-node
// kernel.
#include "tlfea_device.h"

#include <mutex>

#ifndef TLFEA_ELEM
#error "TLFEA_ELEM must be defined"
#endif
#ifndef TLFEA_OP
#error "TLFEA_OP must be defined"
#endif

#ifndef TLFEA_VJP_GT
#define TLFEA_VJP_GT 0
#endif
#ifndef TLFEA_MODE
#define TLFEA_MODE 0
#endif

#define TLFEA_CAT2(a, b, c, g, md) a##_e##b##_o##c##_g##g##_m##md
#define TLFEA_CAT(a, b, c, g, md) TLFEA_CAT2(a, b, c, g, md)

namespace tlfea {

hipError_t TLFEA_CAT(launch_tiles, TLFEA_ELEM, TLFEA_OP, TLFEA_VJP_GT, TLFEA_MODE)(
    int law, int damped, int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
    int tile0, int nl, int nc)
{
    return launch_class<TLFEA_OP, TLFEA_ELEM, TLFEA_VJP_GT, TLFEA_MODE>(law, damped, te, n_tiles, lds, s, m, c,
                                                                       tile0, nl, nc);
}

#if TLFEA_OP == 0 && TLFEA_MODE == 1
#define TLFEA_MCAT2(a, b) a##_e##b
#define TLFEA_MCAT(a, b) TLFEA_MCAT2(a, b)
hipError_t TLFEA_MCAT(launch_mass, TLFEA_ELEM)(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m,
                                              const CallArgs &c, int tile0, int nl, int nc)
{
    return launch_mass_class<TLFEA_ELEM>(te, n_tiles, lds, s, m, c, tile0, nl, nc);
}
#endif

#if TLFEA_OP == 0 && TLFEA_MODE == 0
#define TLFEA_ICAT2(a, b) a##_e##b##_o0
#define TLFEA_ICAT(a, b) TLFEA_ICAT2(a, b)
hipError_t TLFEA_ICAT(launch_inverted, TLFEA_ELEM)(int te, int n_tiles, size_t lds, hipStream_t s,
                                                  const DevMesh &m, const CallArgs &c, int tile0,
                                                  unsigned long long *count)
{
    return launch_inverted_class<TLFEA_ELEM>(te, n_tiles, lds, s, m, c, tile0, count);
}
#endif

#if TLFEA_ELEM == 0 && TLFEA_OP == 0 && TLFEA_MODE == 0
// Device scratch of tlfea_internal_force_noalloc: the forward's shared-node
// partial sums (three rows of n_part doubles), in a file-scope array that
// every device holds from the module's load to the end of the process, so
// that entry point allocates nothing.  Host code never passes the array's
// name to a kernel: it takes the device address from hipGetSymbolAddress,
// once per device, with that device current.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_address(double **out)
{
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

__global__ void k_zero_count(unsigned long long *count) { *count = 0ull; }

hipError_t launch_zero_count(hipStream_t s, unsigned long long *count)
{
    k_zero_count<<<1, 1, 0, s>>>(count);
    return hipGetLastError();
}

// Nodes shared between tiles (and nodes no element touches): sum the node's
// partial slots, which are contiguous and in tile order, and subtract sub
// (the step residual's f_ext) when given.  One lane per node; up to two
// output fields.  Partials are read eight at a time (every load of a lane
// in flight together); the sum still runs in tile order.
__global__ __launch_bounds__(256) void k_halo(DevMesh m, double *out0, double *out1, const double *sub)
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
        for (int r = 0; r < 3; ++r) {
            const int64_t o = r * m.n_nodes + g;
            out[o] = (f == 0 && sub) ? s[r] - sub[o] : s[r];
        }
    }
}

hipError_t launch_halo(hipStream_t s, const DevMesh &m, double *out0, double *out1, const double *sub)
{
    if (m.n_halo <= 0) return hipSuccess;
    const dim3 grid((unsigned)((m.n_halo + 255) / 256));
    k_halo<<<grid, 256, 0, s>>>(m, out0, out1, sub);
    return hipGetLastError();
}
#endif

}  // namespace tlfea

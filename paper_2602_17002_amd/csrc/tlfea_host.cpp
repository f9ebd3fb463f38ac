// Host side of the C ABI declared in include/tlfea.h: argument validation,
// element reordering, tiling, device upload, launch sequencing, hipGraph
// replay for batched meshes, kernel timing and tile-size autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "tlfea.h"
#include "tlfea_elements.h"
#include "tlfea_internal.h"
#include "tlfea_joints.h"

namespace tlfea {
#define TLFEA_DECL(e, o, g, md)                                                                               \
    hipError_t launch_tiles_e##e##_o##o##_g##g##_m##md(int law, int damped, int te, int n_tiles, size_t lds,     \
                                                       hipStream_t s, const DevMesh &m, const CallArgs &c,       \
                                                       int tile0, int nl, int nc);
TLFEA_DECL(0, 0, 0, 0) TLFEA_DECL(0, 0, 0, 1) TLFEA_DECL(0, 1, 0, 0) TLFEA_DECL(0, 1, 1, 0)
TLFEA_DECL(0, 2, 0, 0) TLFEA_DECL(0, 2, 0, 1)
TLFEA_DECL(1, 0, 0, 0) TLFEA_DECL(1, 0, 0, 1) TLFEA_DECL(1, 1, 0, 0) TLFEA_DECL(1, 1, 1, 0)
TLFEA_DECL(1, 2, 0, 0) TLFEA_DECL(1, 2, 0, 1)
TLFEA_DECL(2, 0, 0, 0) TLFEA_DECL(2, 0, 0, 1) TLFEA_DECL(2, 1, 0, 0) TLFEA_DECL(2, 1, 1, 0)
TLFEA_DECL(2, 2, 0, 0) TLFEA_DECL(2, 2, 0, 1)
#undef TLFEA_DECL
hipError_t launch_mass_e0(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                          int tile0, int nl, int nc);
hipError_t launch_mass_e1(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                          int tile0, int nl, int nc);
hipError_t launch_mass_e2(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                          int tile0, int nl, int nc);
hipError_t launch_halo(hipStream_t s, const DevMesh &m, double *out0, double *out1, const double *sub);
hipError_t launch_inverted_e0_o0(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                                 int tile0, unsigned long long *count);
hipError_t launch_inverted_e1_o0(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                                 int tile0, unsigned long long *count);
hipError_t launch_inverted_e2_o0(int te, int n_tiles, size_t lds, hipStream_t s, const DevMesh &m, const CallArgs &c,
                                 int tile0, unsigned long long *count);
hipError_t launch_zero_count(hipStream_t s, unsigned long long *count);
hipError_t scratch_address(double **out);
// vector kernels of the Newton-Krylov step (tlfea_vec.hip)
hipError_t launch_mdot(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *partial,
                       hipStream_t s);
hipError_t launch_maxpy(const double *V, int64_t ldv, int nvec, const double *c, double *y, int64_t n, hipStream_t s);
hipError_t launch_cgs(int mode, const double *V, int64_t ldv, int nv, const double *c, double *w, int64_t n,
                      double *partial, hipStream_t s);
hipError_t launch_sum_partials(const double *partial, int nvec, double *out, double *neg, hipStream_t s);
hipError_t launch_axpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t s);
hipError_t launch_add(const double *x, const double *y, double *z, int64_t n, hipStream_t s);
// joint kernels (tlfea_joints.hip)
hipError_t launch_joints(const DevJoints &J, const double *q, const double *lambda, double rho, double h,
                         double *c_out, int want_z, hipStream_t s);
hipError_t launch_joint_scatter(const DevJoints &J, double *out, int accumulate, hipStream_t s);

// What one call runs over the tiles: the operation of the kernels and its
// variant.  Also the kernel-timing ids of the tile launches (with 3 = the
// shared-node sums and 4 = a batched graph replay in between).
enum Kind { kKFwd = 0, kKVjp = 1, kKJvp = 2, kKRes = 5, kKNewt = 6, kKMass = 7 };
constexpr int kKinds[] = {kKFwd, kKVjp, kKJvp, kKRes, kKNewt, kKMass};
constexpr int kind_slot(int kind) { return kind <= kKJvp ? kind : kind - 2; }   // 0..5
constexpr int kind_op(int kind)
{
    return kind == kKRes ? kOpFwd : kind == kKNewt ? kOpJvp : kind == kKMass ? kOpMass : kind;
}
constexpr int kind_mode(int kind) { return (kind == kKRes || kind == kKNewt) ? kModeStep : kModePlain; }

static hipError_t launch_tiles(int elem, int law, int damped, int te, int kind, int n_tiles, size_t lds, hipStream_t s,
                               const DevMesh &m, const CallArgs &c, int tile0, int nl, int nc)
{
    typedef hipError_t (*fn_t)(int, int, int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int, int,
                               int);
    // per element type: forward, adjoint, tangent, step residual, Newton
    // operator, and the adjoint with the parameter gradients
    static const fn_t table[3][6] = {
        {launch_tiles_e0_o0_g0_m0, launch_tiles_e0_o1_g0_m0, launch_tiles_e0_o2_g0_m0, launch_tiles_e0_o0_g0_m1,
         launch_tiles_e0_o2_g0_m1, launch_tiles_e0_o1_g1_m0},
        {launch_tiles_e1_o0_g0_m0, launch_tiles_e1_o1_g0_m0, launch_tiles_e1_o2_g0_m0, launch_tiles_e1_o0_g0_m1,
         launch_tiles_e1_o2_g0_m1, launch_tiles_e1_o1_g1_m0},
        {launch_tiles_e2_o0_g0_m0, launch_tiles_e2_o1_g0_m0, launch_tiles_e2_o2_g0_m0, launch_tiles_e2_o0_g0_m1,
         launch_tiles_e2_o2_g0_m1, launch_tiles_e2_o1_g1_m0}};
    typedef hipError_t (*mass_t)(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int, int, int);
    static const mass_t mass[3] = {launch_mass_e0, launch_mass_e1, launch_mass_e2};
    if (elem < 0 || elem > 2) return hipErrorInvalidValue;
    if (kind == kKMass) return mass[elem](te, n_tiles, lds, s, m, c, tile0, nl, nc);
    int k;
    switch (kind) {
    case kKFwd: k = 0; break;
    case kKVjp: k = c.gtheta ? 5 : 1; break;
    case kKJvp: k = 2; break;
    case kKRes: k = 3; break;
    case kKNewt: k = 4; break;
    default: return hipErrorInvalidValue;
    }
    return table[elem][k](law, damped, te, n_tiles, lds, s, m, c, tile0, nl, nc);
}
}  // namespace tlfea

using namespace tlfea;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static tlfea_status fail(tlfea_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return fail(e_ == hipErrorOutOfMemory ? TLFEA_E_NOMEM : TLFEA_E_DEVICE, "%s: %s", #expr,      \
                        hipGetErrorString(e_));                                                            \
    } while (0)

extern "C" const char *tlfea_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ element data (host)

// Parent-element tables of one element type (T10, H8 or Q27), evaluated
// once from the constexpr definitions of tlfea_elements.h: the gradients
// and weights of the internal-force rule and of the mass rule.
struct ElemTables {
    int nen = 0, nq = 0, nqm = 0, ncorner = 0;
    std::vector<double> grad, w, mgrad, mw;   // grad[(q * nen + a) * 3 + k]
    std::vector<int> corner;
};

template <int ELEM>
static ElemTables make_tables()
{
    using E = ElemDef<ELEM>;
    using M = MassRule<ELEM>;
    ElemTables t;
    t.nen = E::nen;
    t.nq = E::nq;
    t.nqm = M::nq;
    t.ncorner = E::n_corner;
    for (int q = 0; q < E::nq; ++q) {
        t.w.push_back(E::weight(q));
        for (int a = 0; a < E::nen; ++a)
            for (int k = 0; k < 3; ++k) t.grad.push_back(E::grad(q, a, k));
    }
    for (int q = 0; q < M::nq; ++q) {
        t.mw.push_back(M::weight(q));
        for (int a = 0; a < E::nen; ++a)
            for (int k = 0; k < 3; ++k) t.mgrad.push_back(M::grad(q, a, k));
    }
    for (int c = 0; c < E::n_corner; ++c) t.corner.push_back(E::corner(c));
    return t;
}

static const ElemTables &tables_of(int elem)
{
    static const ElemTables t10 = make_tables<kT10>(), h8 = make_tables<kH8>(), q27 = make_tables<kQ27>();
    return elem == kT10 ? t10 : (elem == kH8 ? h8 : q27);
}
static int nen_of(int elem) { return tables_of(elem).nen; }
static int nq_of(int elem) { return tables_of(elem).nq; }
static int ncorner_of(int elem) { return tables_of(elem).ncorner; }
static int corner_of(int elem, int c) { return tables_of(elem).corner[c]; }
static double grad_of(int elem, int q, int a, int k)
{
    const ElemTables &t = tables_of(elem);
    return t.grad[((size_t)q * t.nen + a) * 3 + k];
}
static double shape_of(int elem, int a, const double *xi)
{
    switch (elem) {
    case kT10: return ElemDef<kT10>::shape_at(a, xi[0], xi[1], xi[2]);
    case kH8: return ElemDef<kH8>::shape_at(a, xi[0], xi[1], xi[2]);
    default: return ElemDef<kQ27>::shape_at(a, xi[0], xi[1], xi[2]);
    }
}
static double weight_of(int elem, int q) { return tables_of(elem).w[q]; }
static int nqm_of(int elem) { return tables_of(elem).nqm; }
static double mass_weight_of(int elem, int q) { return tables_of(elem).mw[q]; }
static double mass_grad_of(int elem, int q, int a, int k)
{
    const ElemTables &t = tables_of(elem);
    return t.mgrad[((size_t)q * t.nen + a) * 3 + k];
}

// ------------------------------------------------------------------ mesh object

struct ClassRange {
    int elem, law, damped, te;
    int tile_begin, tile_count;
    int nl_cap;          // most distinct nodes of a tile of the class (LDS records to allocate)
    int nc[6];           // components assembled per round, per kind (kind_slot)
};

struct GraphEntry {
    int kind;
    const void *key[14];
    hipStream_t stream;
    hipGraphExec_t exec;
    hipEvent_t done;   // recorded after every launch of exec: waited on before exec is destroyed
    uint64_t stamp;
};

constexpr int kNumKernelIds = TLFEA_NUM_KERNEL_IDS;

struct tlfea_mesh {
    int device = 0;
    int flags = 0;
    int64_t n_nodes = 0, n_elem = 0, n_qp = 0;
    int n_blocks = 0;
    std::vector<BlockDesc> blocks;
    std::vector<ClassRange> classes;
    int te_t10 = 0, te_h8 = 0, te_q27 = 0;
    DevMesh dm{};
    std::vector<void *> allocations;
    int64_t device_bytes = 0;
    int64_t n_tiles = 0;
    std::vector<int32_t> tile_nodes;   // global node of every tile node, tile order (host copy)
    // profiling
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kNumKernelIds];
    int32_t counts[kNumKernelIds] = {};
    double ms[kNumKernelIds] = {};
    // graph cache
    std::vector<GraphEntry> graphs;
    uint64_t stamp = 0;
    int64_t graph_builds = 0, graph_updates = 0;   // instantiated, updated in place
    bool any_damped = false;
    bool has_mass = false;     // some block has a density: mass coefficients are on the device
};

static void free_mesh_memory(tlfea_mesh *m)
{
    for (void *p : m->allocations) (void)hipFree(p);
    m->allocations.clear();
    for (auto &g : m->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipEventDestroy(g.done);
    }
    m->graphs.clear();
    for (int k = 0; k < kNumKernelIds; ++k) {
        for (auto &e : m->pending[k]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        m->pending[k].clear();
    }
}

// Device copy of a host table, issued on the creation stream (the caller of
// create_with synchronises the stream before the host tables go away).
template <class T>
static tlfea_status upload(tlfea_mesh *m, const std::vector<T> &h, T **d, hipStream_t s)
{
    *d = nullptr;
    if (h.empty()) return TLFEA_OK;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, h.size() * sizeof(T)));
    m->allocations.push_back(p);
    m->device_bytes += (int64_t)(h.size() * sizeof(T));
    HIP_TRY(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    *d = static_cast<T *>(p);
    return TLFEA_OK;
}

// ------------------------------------------------------------------ ordering

// Whether a - b is exact in binary64 (Knuth's two-sum error term is zero).
// Host code is built without value-changing floating-point options.
static bool difference_is_exact(double a, double b)
{
    const volatile double s = a - b;
    const volatile double bv = s - a;
    const volatile double av = s - bv;
    return (a - av) + (-b - bv) == 0.0;
}

static uint64_t spread21(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// Element order inside one block: Morton curve over element centroids so a
// run of consecutive elements (a tile) is spatially compact.
static void block_order(const tlfea_block &b, int64_t n_nodes, const double *X, bool keep, std::vector<int64_t> &ord)
{
    const int64_t ne = b.n_elem;
    const int nen = nen_of(b.elem), nc = ncorner_of(b.elem);
    ord.resize(ne);
    for (int64_t e = 0; e < ne; ++e) ord[e] = e;
    if (keep || ne < 2) return;
    // corner centroids relative to the block's first node: the order then
    // does not depend on where the body sits
    std::vector<double> cen(3 * ne);
    const int32_t g0 = b.conn[0];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            double s = 0;
            for (int a = 0; a < nc; ++a) s += X[k * n_nodes + b.conn[e * nen + corner_of(b.elem, a)]] - X[k * n_nodes + g0];
            s /= nc;
            cen[3 * e + k] = s;
            lo[k] = std::min(lo[k], s);
            hi[k] = std::max(hi[k], s);
        }
    double ext = 0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
    if (!(ext > 0)) return;
    std::vector<std::pair<uint64_t, int64_t>> key(ne);
    for (int64_t e = 0; e < ne; ++e) {
        uint64_t c = 0;
        for (int k = 0; k < 3; ++k) {
            double t = (cen[3 * e + k] - lo[k]) / ext;
            uint64_t qv = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(t * 2097151.0)));
            c |= spread21(qv) << k;
        }
        key[e] = {c, e};
    }
    std::sort(key.begin(), key.end());
    for (int64_t e = 0; e < ne; ++e) ord[e] = key[e].second;
}

// ------------------------------------------------------------------ validation

// J_p = det(U G(xi_q)) > 0 at every quadrature point (Sec. 6).  Evaluated
// with coordinates relative to the element's first node (exact differences,
// no cancellation against the body's offset from the origin).
static tlfea_status check_element(int elem, const int32_t *c, int64_t n_nodes, const double *X, int64_t e, int b)
{
    const int nen = nen_of(elem), nq = nq_of(elem);
    for (int q = 0; q < nq; ++q) {
        double J[9] = {0};
        for (int a = 1; a < nen; ++a)
            for (int i = 0; i < 3; ++i) {
                const double u = X[i * n_nodes + c[a]] - X[i * n_nodes + c[0]];
                for (int k = 0; k < 3; ++k) J[3 * i + k] += u * grad_of(elem, q, a, k);
            }
        const double d = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                         J[2] * (J[3] * J[7] - J[4] * J[6]);
        if (!(d > 0))
            return fail(TLFEA_E_REF_JACOBIAN,
                        "block %d element %lld: reference Jacobian det = %g <= 0 at quadrature point %d", b,
                        (long long)e, d, q);
    }
    return TLFEA_OK;
}

// ------------------------------------------------------------------ tiling

struct HostBuild {
    std::vector<TileDesc> tiles;
    std::vector<uint16_t> conn_local;
    std::vector<int32_t> lnode_gid, lnode_dst, lnode_ptr;
    std::vector<uint16_t> lnode_pos;
    std::vector<uint16_t> lnode_slot;
    std::vector<int32_t> elem_uid;
    std::vector<int32_t> halo_gid, halo_ptr;
    int64_t n_part = 0;
    std::vector<ClassRange> classes;
};

// Largest entry count of a tile list (32-bit offsets); a test build lowers it.
#ifndef TLFEA_OFFSET_LIMIT
#define TLFEA_OFFSET_LIMIT INT32_MAX
#endif
constexpr int64_t kOffsetLimit = TLFEA_OFFSET_LIMIT;

static int default_te(int elem) { return elem == kQ27 ? 64 : 256; }

// Distinct nodes a tile may hold: at most kStagePerThread per thread, and
// few enough that every operation's node records and assembly tables stay
// within its LDS budget.
// LDS budget of one workgroup of an operation: the device's per-workgroup
// limit, and at most the share of a 160 KiB compute-unit LDS that lets as
// many workgroups be resident as the kernel's register use allows (a
// workgroup of te elements has te / 64 waves).  The forward is budgeted for
// three waves per SIMD and the other operations for their own count, at
// least two.
static int64_t lds_budget(int kind, int elem, int law, int damped, int te, int64_t lds_dev)
{
    // Q27 tiles hold about 11 nodes per element and run at one wave per
    // SIMD: as many tiles per compute unit as its four waves hold (two of 64
    // elements, two lanes each)
    if (elem == kQ27)
        return std::min<int64_t>(lds_dev, 163840 / std::max(1, 256 / (te * lanes_per_elem(kQ27))));
    const int op = kind_op(kind), mode = kind_mode(kind);
    const int64_t waves_per_cu =
        kind == kKFwd ? 12 : (kind == kKMass ? 16 : 4 * std::max(2, waves_per_simd(op, elem, law, damped != 0, mode)));
    const int64_t wgs = std::max<int64_t>(1, waves_per_cu * 64 / te);
    return std::min<int64_t>(lds_dev, 163840 / wgs);
}

static int kind_record_len(int kind, bool damped) { return record_len(kind_op(kind), damped, kind_mode(kind)); }

static int nl_limit(int elem, int law, int te, int damped, int64_t lds_dev)
{
    const int nen = nen_of(elem);
    int64_t nl = (int64_t)stage_per_thread(elem) * te * lanes_per_elem(elem);
    // full 256-element tiles: at most 600 nodes even where the LDS would hold
    // more.  Compact T10 tiles have about 550 (p99 670 without the cap), and
    // letting the ragged ones grow further made the undamped forward 8 %
    // slower.  Smaller tiles have proportionally more surface nodes and keep
    // only the LDS limit.
    if (te == 256 && elem != kQ27) nl = std::min<int64_t>(nl, 600);
    for (int kind : kKinds) {
        const int64_t fixed = (int64_t)lanes_per_elem(elem) * te * 2 + (int64_t)nen * te * 2;
        const int64_t per_node = 8 * (int64_t)kind_record_len(kind, damped != 0) + 4;
        nl = std::min(nl, (lds_budget(kind, elem, law, damped, te, lds_dev) - fixed) / per_node);
    }
    return (int)nl;
}

// LDS of one workgroup: the node records (reused for the element slots of
// nc components), then the tile's assembly tables (see the kernels): the
// first node of every thread's chunk of the slot list, every node's
// destination, and the slot list.
static size_t lds_bytes(const ClassRange &c, int kind, int nc)
{
    const size_t records = (size_t)c.nl_cap * kind_record_len(kind, c.damped != 0);
    const size_t slots = (size_t)nc * nen_of(c.elem) * c.te;
    const size_t tables = (size_t)lanes_per_elem(c.elem) * c.te * sizeof(uint16_t) + (size_t)c.nl_cap * sizeof(int32_t) +
                          (size_t)nen_of(c.elem) * c.te * sizeof(uint16_t);
    return std::max(records, slots) * sizeof(double) + tables;
}

// Components assembled per round: as many as fit the operation's budget.
static int comps_per_round(const ClassRange &c, int kind, int64_t lds_dev)
{
    for (int nc = 3; nc > 1; --nc)
        if ((int64_t)lds_bytes(c, kind, nc) <= lds_budget(kind, c.elem, c.law, c.damped, c.te, lds_dev)) return nc;
    return 1;
}

// LDS record positions of a tile's nodes.  A wavefront reads one field of
// the nodes of its 64 elements with ds_read_b64, which the LDS serves 16
// lanes per cycle across 16 pairs of 4-byte banks; lanes of one group that
// hit the same pair at different addresses take extra cycles.  A record at
// position p starts in pair (p * len) mod 16, and len is odd, so the pair is
// a bijection of p mod 16 for every operation's record length.  Greedily
// give each node (most reads first) the class p mod 16 that collides least,
// weighted by the quadrature points that read it, with the nodes already
// placed in its 16-lane groups; class sizes are those of 0 .. n_node - 1, so
// the positions stay dense.  `conn` is the tile's [nen][te] local
// connectivity (local = index in the sorted node list); returns pos[local].
static void place_records(const uint16_t *conn, int n_elem, int n_node, int elem, int te, std::vector<uint16_t> &pos)
{
    // a 16-lane group holds 16 / lanes_per_elem elements (the lanes of one
    // element read the same node address together)
    constexpr int kPairs = 16;
    const int kGroup = 16 / lanes_per_elem(elem);
    const int nen = nen_of(elem), nq = nq_of(elem);
    std::vector<int> reads(nen, 0);
    for (int a = 0; a < nen; ++a)
        for (int q = 0; q < nq; ++q) {
            bool nz = false;
            for (int k = 0; k < 3; ++k) nz |= grad_of(elem, q, a, k) != 0.0;
            reads[a] += nz ? 1 : 0;
        }
    // sets: distinct nodes read by one gather of one 16-lane group
    std::vector<std::vector<int>> of(n_node);
    std::vector<int> set_w;
    std::vector<int> members;
    for (int a = 0; a < nen; ++a)
        for (int g0 = 0; g0 < n_elem; g0 += kGroup) {
            members.clear();
            for (int i = g0; i < std::min(n_elem, g0 + kGroup); ++i) {
                const int l = conn[(size_t)a * te + i];
                if (std::find(members.begin(), members.end(), l) == members.end()) members.push_back(l);
            }
            for (int l : members) of[l].push_back((int)set_w.size());
            set_w.push_back(reads[a]);
        }
    std::vector<int> cap(kPairs), cnt(set_w.size() * kPairs, 0), order(n_node), cls(n_node);
    for (int c = 0; c < kPairs; ++c) cap[c] = n_node / kPairs + (c < n_node % kPairs ? 1 : 0);
    for (int l = 0; l < n_node; ++l) order[l] = l;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return of[x].size() > of[y].size(); });
    for (int l : order) {
        int best = -1;
        long long best_cost = 0;
        for (int c = 0; c < kPairs; ++c) {
            if (!cap[c]) continue;
            long long z = 0;
            for (int si : of[l]) z += (long long)set_w[si] * cnt[(size_t)si * kPairs + c];
            if (best < 0 || z < best_cost) {
                best = c;
                best_cost = z;
            }
        }
        cls[l] = best;
        cap[best]--;
        for (int si : of[l]) cnt[(size_t)si * kPairs + best]++;
    }
    std::vector<int> next(kPairs);
    for (int c = 0; c < kPairs; ++c) next[c] = c;
    pos.resize(n_node);
    for (int l = 0; l < n_node; ++l) {
        pos[l] = (uint16_t)next[cls[l]];
        next[cls[l]] += kPairs;
    }
}

// Cut the elements `ids` (one block, Morton order) into tiles of at most te
// elements and nl_max distinct nodes.  A tile grows from the first element
// not yet taken (in Morton order) by repeatedly adding the element that has
// the most nodes already in the tile (fewest new nodes), among equals the
// one whose corner centroid is nearest the tile's, so tiles are compact and
// share few nodes with their neighbours.  Appends the tiles' element lists
// (positions in ids) to `out`.
static void grow_tiles(const tlfea_block &B, int64_t n_nodes, const double *X, const std::vector<int64_t> &ids, int te,
                       int nl_max, std::vector<std::vector<int64_t>> &out)
{
    const int nen = nen_of(B.elem), ncn = ncorner_of(B.elem);
    const int64_t ne = (int64_t)ids.size();
    if (ne == 0) return;
    // corner centroids (relative to the block's first node): among
    // candidates that share equally many nodes with the tile, the one
    // nearest the tile's centroid keeps the tile compact
    std::vector<double> cen(3 * ne);
    const int32_t g0 = B.conn[0];
    for (int64_t j = 0; j < ne; ++j)
        for (int k = 0; k < 3; ++k) {
            double s = 0;
            for (int a = 0; a < ncn; ++a)
                s += X[k * n_nodes + B.conn[ids[j] * nen + corner_of(B.elem, a)]] - X[k * n_nodes + g0];
            cen[3 * j + k] = s / ncn;
        }
    // node -> elements (positions in ids)
    std::vector<int64_t> nptr(n_nodes + 1, 0);
    for (int64_t j = 0; j < ne; ++j)
        for (int a = 0; a < nen; ++a) nptr[B.conn[ids[j] * nen + a] + 1]++;
    for (int64_t g = 0; g < n_nodes; ++g) nptr[g + 1] += nptr[g];
    std::vector<int64_t> nadj(nptr[n_nodes]);
    {
        std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
        for (int64_t j = 0; j < ne; ++j)
            for (int a = 0; a < nen; ++a) nadj[fill[B.conn[ids[j] * nen + a]]++] = j;
    }
    std::vector<char> taken(ne, 0);
    std::vector<int32_t> score(ne, 0), stamp(ne, -1), in_tile(n_nodes, -1);
    std::vector<std::vector<int64_t>> bucket(nen + 1);   // candidates by score, read from head[]
    std::vector<size_t> head(nen + 1, 0);
    std::vector<int64_t> members;
    int64_t cursor = 0;
    int32_t tile = 0;
    auto fresh_of = [&](int64_t j) {
        int f = 0;
        for (int a = 0; a < nen; ++a) f += in_tile[B.conn[ids[j] * nen + a]] == tile ? 0 : 1;
        return f;
    };
    for (;; ++tile) {
        while (cursor < ne && taken[cursor]) ++cursor;
        if (cursor >= ne) break;
        for (auto &bk : bucket) bk.clear();
        std::fill(head.begin(), head.end(), 0);
        members.clear();
        int nodes = 0;
        auto add = [&](int64_t j) {
            taken[j] = 1;
            members.push_back(j);
            for (int a = 0; a < nen; ++a) {
                const int32_t g = B.conn[ids[j] * nen + a];
                if (in_tile[g] == tile) continue;
                in_tile[g] = tile;
                ++nodes;
                for (int64_t p = nptr[g]; p < nptr[g + 1]; ++p) {
                    const int64_t e2 = nadj[p];
                    if (taken[e2]) continue;
                    if (stamp[e2] != tile) {
                        stamp[e2] = tile;
                        score[e2] = 0;
                    }
                    score[e2] += 1;
                    bucket[score[e2]].push_back(e2);
                }
            }
        };
        add(cursor);
        double csum[3] = {cen[3 * cursor], cen[3 * cursor + 1], cen[3 * cursor + 2]};
        while ((int)members.size() < te) {
            int64_t best = -1;
            for (int sc = nen; sc >= 1 && best < 0; --sc) {
                auto &bk = bucket[sc];
                while (head[sc] < bk.size()) {
                    const int64_t j = bk[head[sc]];
                    if (taken[j] || stamp[j] != tile || score[j] != sc) {
                        ++head[sc];
                        continue;
                    }
                    best = j;
                    break;
                }
                if (best < 0) continue;
                const double inv = 1.0 / (double)members.size();
                double bd = 1e300;
                for (size_t q = head[sc]; q < bk.size(); ++q) {
                    const int64_t j = bk[q];
                    if (taken[j] || stamp[j] != tile || score[j] != sc) continue;
                    double d = 0;
                    for (int k = 0; k < 3; ++k) {
                        const double u = cen[3 * j + k] - csum[k] * inv;
                        d += u * u;
                    }
                    if (d < bd) {
                        bd = d;
                        best = j;
                    }
                }
            }
            if (best < 0) {   // no element touches the tile: continue with the next in Morton order
                int64_t c2 = cursor;
                while (c2 < ne && taken[c2]) ++c2;
                if (c2 >= ne) break;
                best = c2;
            }
            if (nodes + fresh_of(best) > nl_max) break;
            add(best);
            for (int k = 0; k < 3; ++k) csum[k] += cen[3 * best + k];
        }
        out.push_back(members);
    }
}

// Lane order within a tile.  A gather of node slot a by 16 consecutive lanes
// costs a cycle per distinct address in the busiest bank pair, and lanes
// that read the same node share one address.  The tile's elements (Morton
// positions in ord) are therefore dealt out in groups of 16: each group
// starts with the first element left and adds, one at a time, the element
// whose nodes coincide with the group's at the most slots (the first such
// element in Morton order among equals).
static void order_lanes(const tlfea_block &B, const std::vector<int64_t> &ord, std::vector<int64_t> &grp)
{
    const int kGroup = 16 / lanes_per_elem(B.elem);
    const int nen = nen_of(B.elem);
    std::sort(grp.begin(), grp.end());
    const int ng = (int)grp.size();
    // (node, slot) -> elements of the tile with that node at that slot
    std::vector<std::pair<int64_t, int>> key;
    key.reserve((size_t)ng * nen);
    for (int j = 0; j < ng; ++j)
        for (int a = 0; a < nen; ++a) key.push_back({(int64_t)B.conn[ord[grp[j]] * nen + a] * nen + a, j});
    std::sort(key.begin(), key.end());
    std::vector<char> used(ng, 0);
    std::vector<int> score(ng);
    std::vector<int64_t> seen, out;
    out.reserve(ng);
    int first = 0;
    while ((int)out.size() < ng) {
        std::fill(score.begin(), score.end(), 0);
        seen.clear();
        for (int k = 0; k < kGroup && (int)out.size() < ng; ++k) {
            while (used[first]) ++first;
            int best = first;
            for (int j = first + 1; j < ng; ++j)
                if (!used[j] && score[j] > score[best]) best = j;
            used[best] = 1;
            out.push_back(grp[best]);
            // every (node, slot) new to the group raises the score of the
            // elements that share it
            for (int a = 0; a < nen; ++a) {
                const int64_t kk = (int64_t)B.conn[ord[grp[best]] * nen + a] * nen + a;
                if (std::find(seen.begin(), seen.end(), kk) != seen.end()) continue;
                seen.push_back(kk);
                auto lo = std::lower_bound(key.begin(), key.end(), std::make_pair(kk, -1));
                for (auto it = lo; it != key.end() && it->first == kk; ++it) score[it->second]++;
            }
        }
    }
    grp.swap(out);
}

static tlfea_status build_tiles(int64_t n_nodes, const double *X, int n_blocks, const tlfea_block *blocks, int flags,
                                const std::vector<int> &te_of_block, int64_t lds_dev, HostBuild &hb)
{
    // user element id offset per block
    std::vector<int64_t> uid0(n_blocks + 1, 0);
    for (int b = 0; b < n_blocks; ++b) uid0[b + 1] = uid0[b] + blocks[b].n_elem;
    // classes: (elem, law, damped, te) in first-appearance order; tiles laid out class by class
    struct Key {
        int elem, law, damped, te;
        bool operator==(const Key &o) const
        {
            return elem == o.elem && law == o.law && damped == o.damped && te == o.te;
        }
    };
    std::vector<Key> keys;
    std::vector<int> cls(n_blocks);
    for (int b = 0; b < n_blocks; ++b) {
        Key k{blocks[b].elem, blocks[b].law, blocks[b].damped ? 1 : 0, te_of_block[b]};
        auto it = std::find(keys.begin(), keys.end(), k);
        cls[b] = (int)(it - keys.begin());
        if (it == keys.end()) keys.push_back(k);
    }
    for (int b = 0; b < n_blocks; ++b) {
        const tlfea_block &B = blocks[b];
        for (int64_t e = 0; e < B.n_elem; ++e) {
            tlfea_status st = check_element(B.elem, B.conn + e * nen_of(B.elem), n_nodes, X, e, b);
            if (st != TLFEA_OK) return st;
        }
    }
    std::vector<int32_t> local(n_nodes, -1);
    std::vector<int32_t> tile_count(n_nodes, 0);
    std::vector<int64_t> ord;
    std::vector<int32_t> nodes;
    std::vector<std::vector<int64_t>> groups;
    int64_t elem_cursor = 0;
    for (size_t k = 0; k < keys.size(); ++k) {
        ClassRange cr{keys[k].elem, keys[k].law, keys[k].damped, keys[k].te, (int)hb.tiles.size(), 0, 0, {1, 1, 1, 1, 1, 1}};
        const int te = keys[k].te, nen = nen_of(keys[k].elem);
        const int nlmax = nl_limit(keys[k].elem, keys[k].law, te, keys[k].damped, lds_dev);
        if (nlmax < nen || (int64_t)nen * te * (int64_t)sizeof(double) > 65536)
            return fail(TLFEA_E_UNSUPPORTED, "tile of %d elements does not fit the LDS of one workgroup", te);
        for (int b = 0; b < n_blocks; ++b) {
            if (cls[b] != (int)k) continue;
            const tlfea_block &B = blocks[b];
            block_order(B, n_nodes, X, (flags & TLFEA_KEEP_ORDER) != 0, ord);
            groups.clear();
            if (flags & TLFEA_KEEP_ORDER) {
                // consecutive runs of the caller's order, cut at te elements or nlmax nodes
                int64_t pos = 0;
                while (pos < B.n_elem) {
                    std::vector<int64_t> g;
                    nodes.clear();
                    while (pos < B.n_elem && (int)g.size() < te) {
                        const int32_t *c = B.conn + ord[pos] * nen;
                        int fresh = 0;
                        for (int a = 0; a < nen; ++a) fresh += local[c[a]] < 0 ? 1 : 0;
                        if ((int)nodes.size() + fresh > nlmax && !g.empty()) break;
                        for (int a = 0; a < nen; ++a)
                            if (local[c[a]] < 0) {
                                local[c[a]] = 1;
                                nodes.push_back(c[a]);
                            }
                        g.push_back(pos++);
                    }
                    for (int32_t gg : nodes) local[gg] = -1;
                    groups.push_back(std::move(g));
                }
            } else {
                grow_tiles(B, n_nodes, X, ord, te, nlmax, groups);
            }
            if (!(flags & TLFEA_KEEP_ORDER))
                for (auto &grp : groups) order_lanes(B, ord, grp);
            for (const auto &grp : groups) {
                nodes.clear();
                for (int64_t pos : grp) {
                    const int32_t *c = B.conn + ord[pos] * nen;
                    for (int a = 0; a < nen; ++a)
                        if (local[c[a]] < 0) {
                            local[c[a]] = 1;
                            nodes.push_back(c[a]);
                        }
                }
                std::sort(nodes.begin(), nodes.end());
                TileDesc t;
                t.elem_begin = (int32_t)elem_cursor;
                t.n_elem = (int32_t)grp.size();
                t.node_begin = (int32_t)hb.lnode_gid.size();
                t.n_node = (int32_t)nodes.size();
                t.ptr_begin = (int32_t)hb.lnode_ptr.size();
                t.conn_begin = (int32_t)hb.conn_local.size();
                t.block = b;
                t.ref = 0;
                if (t.n_node > nlmax || t.n_node > stage_per_thread(B.elem) * te * lanes_per_elem(B.elem))
                    return fail(TLFEA_E_UNSUPPORTED, "tile with %d nodes exceeds the limit %d", t.n_node, nlmax);
                for (size_t l = 0; l < nodes.size(); ++l) {
                    local[nodes[l]] = (int32_t)l;
                    hb.lnode_gid.push_back(nodes[l]);
                    tile_count[nodes[l]] += 1;
                }
                // local connectivity [nen][te]
                hb.conn_local.resize(hb.conn_local.size() + (size_t)nen * te, 0);
                for (size_t i = 0; i < grp.size(); ++i) {
                    const int64_t e = ord[grp[i]];
                    const int32_t *c = B.conn + e * nen;
                    for (int a = 0; a < nen; ++a)
                        hb.conn_local[t.conn_begin + (size_t)a * te + i] = (uint16_t)local[c[a]];
                    hb.elem_uid.push_back((int32_t)(uid0[b] + e));
                }
                // per-node slot lists (CSR); visiting slots a * te + i in
                // increasing order leaves every list sorted.  Each tile's list
                // starts at an even index (the kernels copy it as 32-bit words),
                // and the first entry of every node's group is flagged (the
                // kernels split the tile's list into equal chunks).
                {
                    if (hb.lnode_slot.size() & 1) hb.lnode_slot.push_back(0);
                    const size_t nn = nodes.size(), base = hb.lnode_slot.size();
                    std::vector<int32_t> cnt(nn + 1, 0);
                    const int64_t ne_t = (int64_t)grp.size();
                    for (int a = 0; a < nen; ++a)
                        for (int64_t i = 0; i < ne_t; ++i) cnt[hb.conn_local[t.conn_begin + (size_t)a * te + i] + 1]++;
                    for (size_t l = 0; l < nn; ++l) cnt[l + 1] += cnt[l];
                    for (size_t l = 0; l <= nn; ++l) hb.lnode_ptr.push_back((int32_t)(base + cnt[l]));
                    hb.lnode_slot.resize(base + cnt[nn]);
                    for (int a = 0; a < nen; ++a)
                        for (int64_t i = 0; i < ne_t; ++i) {
                            const int l = hb.conn_local[t.conn_begin + (size_t)a * te + i];
                            hb.lnode_slot[base + cnt[l]++] = (uint16_t)(a * te + i);
                        }
                    for (size_t l = 0; l < nn; ++l) hb.lnode_slot[hb.lnode_ptr[t.ptr_begin + l]] |= kSlotHead;
                }
                // LDS record positions; the elements address records by position
                {
                    std::vector<uint16_t> pos;
                    place_records(&hb.conn_local[t.conn_begin], t.n_elem, t.n_node, keys[k].elem, te, pos);
                    hb.lnode_pos.insert(hb.lnode_pos.end(), pos.begin(), pos.end());
                    for (int a = 0; a < nen; ++a)
                        for (int i = 0; i < t.n_elem; ++i) {
                            uint16_t &c = hb.conn_local[t.conn_begin + (size_t)a * te + i];
                            c = pos[c];
                        }
                }
                for (int32_t g : nodes) local[g] = -1;
                cr.nl_cap = std::max(cr.nl_cap, (int)nodes.size());
                hb.tiles.push_back(t);
                elem_cursor += (int64_t)grp.size();
            }
        }
        cr.tile_count = (int)hb.tiles.size() - cr.tile_begin;
        for (int kind : kKinds) cr.nc[kind_slot(kind)] = comps_per_round(cr, kind, lds_dev);
        if (cr.tile_count > 0) hb.classes.push_back(cr);
    }
    if (hb.lnode_slot.size() & 1) hb.lnode_slot.push_back(0);   // whole 32-bit words
    // The tile descriptors and the kernels address these lists with 32-bit
    // offsets (about 200 million T10 elements per mesh); a larger problem is
    // split over several meshes.
    {
        const size_t longest = std::max({hb.conn_local.size(), hb.lnode_slot.size(), hb.lnode_ptr.size(),
                                         hb.lnode_gid.size(), hb.elem_uid.size()});
        if (longest > (size_t)kOffsetLimit)
            return fail(TLFEA_E_UNSUPPORTED, "mesh needs %zu tile-list entries, above the 32-bit offset limit %lld; "
                        "split it over several meshes", longest, (long long)kOffsetLimit);
    }
    // Nodes in exactly one tile are written by that tile.  Every other node
    // (shared, or touched by no element) gets the contiguous partial slots
    // [halo_ptr[h], halo_ptr[h+1]), one per tile that holds it, in tile
    // order; the shared-node kernel sums them in that order.
    std::vector<int32_t> halo_index(n_nodes, -1), next_slot;
    for (int64_t g = 0; g < n_nodes; ++g)
        if (tile_count[g] != 1) {
            halo_index[g] = (int32_t)hb.halo_gid.size();
            hb.halo_gid.push_back((int32_t)g);
            hb.halo_ptr.push_back((int32_t)hb.n_part);
            next_slot.push_back((int32_t)hb.n_part);
            hb.n_part += tile_count[g];
            if (hb.n_part >= kOffsetLimit)
                return fail(TLFEA_E_UNSUPPORTED, "too many shared-node partials; split the mesh");
        }
    hb.halo_ptr.push_back((int32_t)hb.n_part);
    hb.lnode_dst.resize(hb.lnode_gid.size());
    for (size_t t = 0; t < hb.tiles.size(); ++t) {
        const TileDesc &T = hb.tiles[t];
        for (int l = 0; l < T.n_node; ++l) {
            const int32_t g = hb.lnode_gid[T.node_begin + l];
            if (tile_count[g] == 1) hb.lnode_dst[T.node_begin + l] = g;
            else hb.lnode_dst[T.node_begin + l] = -1 - next_slot[halo_index[g]]++;
        }
    }
    return TLFEA_OK;
}

// ------------------------------------------------------------------ create / destroy

// A caller-supplied quadrature table (Sec. 6: the rule is tabulated once on
// the parent element) must be the compiled rule to rounding: the kernels
// carry the rule's weights and parent gradients as compile-time constants.
static tlfea_status check_rule(const tlfea_block &B, int b)
{
    if (!B.qp_w && !B.dsdxi) {
        if (B.nq != 0) return fail(TLFEA_E_INVALID, "block %d: nq = %d without a quadrature table", b, B.nq);
        return TLFEA_OK;
    }
    const int nq = nq_of(B.elem), nen = nen_of(B.elem);
    if (B.nq != nq)
        return fail(TLFEA_E_UNSUPPORTED, "block %d: a %d-point rule was given; the kernels carry the built-in %d-point "
                    "rule of this element type", b, B.nq, nq);
    if (B.qp_w) {
        double mx = 0;
        for (int q = 0; q < nq; ++q) mx = std::max(mx, std::fabs(weight_of(B.elem, q)));
        for (int q = 0; q < nq; ++q) {
            const double w = weight_of(B.elem, q);
            if (!(std::fabs(B.qp_w[q] - w) <= 1e-14 * mx))
                return fail(TLFEA_E_UNSUPPORTED, "block %d: weight of point %d is %.17g, the built-in rule has %.17g; "
                            "the kernels carry the built-in rule only", b, q, B.qp_w[q], w);
        }
    }
    if (B.dsdxi) {
        double mx = 0;
        for (int q = 0; q < nq; ++q)
            for (int a = 0; a < nen; ++a)
                for (int k = 0; k < 3; ++k) mx = std::max(mx, std::fabs(grad_of(B.elem, q, a, k)));
        for (int q = 0; q < nq; ++q)
            for (int a = 0; a < nen; ++a)
                for (int k = 0; k < 3; ++k) {
                    const double g = grad_of(B.elem, q, a, k), d = B.dsdxi[((size_t)q * nen + a) * 3 + k];
                    if (!(std::fabs(d - g) <= 1e-14 * mx))
                        return fail(TLFEA_E_UNSUPPORTED, "block %d: parent gradient [%d][%d][%d] is %.17g, the built-in "
                                    "table has %.17g; the kernels carry the built-in rule only", b, q, a, k, d, g);
                }
    }
    return TLFEA_OK;
}

static tlfea_status validate_args(int64_t n_nodes, const double *X, int32_t n_blocks, const tlfea_block *blocks,
                                  int32_t flags)
{
    if (n_nodes < 0 || n_nodes > INT32_MAX) return fail(TLFEA_E_SHAPE, "n_nodes = %lld out of range", (long long)n_nodes);
    if (n_nodes > 0 && !X) return fail(TLFEA_E_INVALID, "X_ref is NULL");
    if (n_blocks < 0 || (n_blocks > 0 && !blocks)) return fail(TLFEA_E_INVALID, "bad block list");
    if (flags & ~(TLFEA_BATCHED | TLFEA_AUTOTUNE | TLFEA_KEEP_ORDER))
        return fail(TLFEA_E_INVALID, "unknown flag bits 0x%x", flags);
    for (int64_t i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(X[i])) return fail(TLFEA_E_INVALID, "X_ref[%lld] is not finite", (long long)i);
    int64_t total = 0;
    for (int b = 0; b < n_blocks; ++b) {
        const tlfea_block &B = blocks[b];
        if (B.elem != TLFEA_T10 && B.elem != TLFEA_H8 && B.elem != TLFEA_Q27)
            return fail(TLFEA_E_INVALID, "block %d: unknown element %d", b, B.elem);
        if (B.law != TLFEA_SVK && B.law != TLFEA_MR && B.law != TLFEA_NH)
            return fail(TLFEA_E_INVALID, "block %d: unknown law %d", b, B.law);
        if (B.n_elem < 0) return fail(TLFEA_E_SHAPE, "block %d: n_elem < 0", b);
        if (B.n_elem > 0 && !B.conn) return fail(TLFEA_E_INVALID, "block %d: conn is NULL", b);
        if (B.tile_elems < 0 || B.tile_elems > 256 || (B.tile_elems & 63))
            return fail(TLFEA_E_INVALID, "block %d: tile_elems must be 0, 64, 128, 192 or 256", b);
        if (B.elem == TLFEA_Q27 && B.tile_elems > 128)
            return fail(TLFEA_E_INVALID, "block %d: Q27 tile_elems must be 0, 64 or 128", b);
        for (int p = 0; p < 5; ++p)
            if (!std::isfinite(B.theta[p])) return fail(TLFEA_E_INVALID, "block %d: theta[%d] not finite", b, p);
        if (B.reserved != 0) return fail(TLFEA_E_INVALID, "block %d: reserved field must be 0", b);
        if (!std::isfinite(B.rho) || B.rho < 0) return fail(TLFEA_E_INVALID, "block %d: rho must be finite and >= 0", b);
        {
            tlfea_status st = check_rule(B, b);
            if (st != TLFEA_OK) return st;
        }
        const int nen = nen_of(B.elem);
        for (int64_t i = 0; i < B.n_elem * nen; ++i)
            if (B.conn[i] < 0 || B.conn[i] >= n_nodes)
                return fail(TLFEA_E_SHAPE, "block %d: conn[%lld] = %d outside [0, %lld)", b, (long long)i, B.conn[i],
                            (long long)n_nodes);
        for (int64_t e = 0; e < B.n_elem; ++e)
            for (int a = 0; a < nen; ++a)
                for (int a2 = 0; a2 < a; ++a2)
                    if (B.conn[e * nen + a] == B.conn[e * nen + a2])
                        return fail(TLFEA_E_SHAPE, "block %d element %lld repeats node %d", b, (long long)e,
                                    B.conn[e * nen + a]);
        total += B.n_elem;
    }
    if (total > INT32_MAX) return fail(TLFEA_E_SHAPE, "too many elements");
    return TLFEA_OK;
}

static tlfea_status create_with(int64_t n_nodes, const double *X, int32_t n_blocks, const tlfea_block *blocks,
                                int32_t flags, const std::vector<int> &te_of_block, hipStream_t stream,
                                tlfea_mesh **out)
{
    // LDS a workgroup may allocate on this device (the tangent of a damped
    // block, whose node record is the widest, may use all of it)
    int64_t lds_dev = 65536;
    {
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lim > 0)
            lds_dev = lim;
        else
            (void)hipGetLastError();
    }
    HostBuild hb;
    tlfea_status st = build_tiles(n_nodes, X, n_blocks, blocks, flags, te_of_block, lds_dev, hb);
    if (st != TLFEA_OK) return st;
    tlfea_mesh *m = new (std::nothrow) tlfea_mesh();
    if (!m) return fail(TLFEA_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return fail(TLFEA_E_DEVICE, "hipGetDevice failed");
    }
    m->flags = flags;
    m->n_nodes = n_nodes;
    m->n_blocks = n_blocks;
    for (int b = 0; b < n_blocks; ++b) {
        BlockDesc d;
        for (int p = 0; p < 5; ++p) d.theta[p] = blocks[b].theta[p];
        d.elem = blocks[b].elem;
        d.law = blocks[b].law;
        d.damped = blocks[b].damped ? 1 : 0;
        d.pad = 0;
        m->blocks.push_back(d);
        m->n_elem += blocks[b].n_elem;
        m->n_qp += blocks[b].n_elem * nq_of(blocks[b].elem);
        m->any_damped |= blocks[b].damped != 0;
        if (blocks[b].elem == kT10 && !m->te_t10) m->te_t10 = te_of_block[b];
        if (blocks[b].elem == kH8 && !m->te_h8) m->te_h8 = te_of_block[b];
        if (blocks[b].elem == kQ27 && !m->te_q27) m->te_q27 = te_of_block[b];
    }
    m->classes = hb.classes;
    m->tile_nodes = hb.lnode_gid;
    m->n_tiles = (int64_t)hb.tiles.size();
    DevMesh &d = m->dm;
    // Reference coordinates per tile node, relative to the tile's node
    // nearest the centroid of its nodes; the kernels that sum positions
    // directly take current positions relative to the same node.  The
    // smaller the coordinates, the less the sums over an element's nodes
    // (F = N H, J = U G) cancel.  A component is taken relative only where
    // the subtraction is exact for every node of the tile (always so away
    // from zero, by Sterbenz's lemma): near zero, where it may round, the
    // coordinates are small already and are kept as they are, so that a
    // difference of two staged values is always the coordinates' difference
    // rounded once.
    const int64_t n_tnode = (int64_t)hb.lnode_gid.size();
    std::vector<double> Xt(3 * (size_t)n_tnode);
    for (TileDesc &t : hb.tiles) {
        // centroid and distances relative to the first node, so that the
        // choice does not depend on where the body sits
        const int32_t gf = hb.lnode_gid[t.node_begin];
        auto rel = [&](int l, int c) { return X[c * n_nodes + hb.lnode_gid[t.node_begin + l]] - X[c * n_nodes + gf]; };
        double cen[3] = {0, 0, 0};
        for (int l = 0; l < t.n_node; ++l)
            for (int c = 0; c < 3; ++c) cen[c] += rel(l, c);
        double best = 1e300;
        t.ref = 0;
        for (int l = 0; l < t.n_node; ++l) {
            double d = 0;
            for (int c = 0; c < 3; ++c) {
                const double u = rel(l, c) - cen[c] / t.n_node;
                d += u * u;
            }
            if (d < best) {
                best = d;
                t.ref = l;
            }
        }
        const int32_t g0 = hb.lnode_gid[t.node_begin + t.ref];
        for (int c = 0; c < 3; ++c) {
            const double o = X[c * n_nodes + g0];
            bool exact = true;
            for (int l = 0; l < t.n_node && exact; ++l)
                exact = difference_is_exact(X[c * n_nodes + hb.lnode_gid[t.node_begin + l]], o);
            for (int l = 0; l < t.n_node; ++l) {
                const double xg = X[c * n_nodes + hb.lnode_gid[t.node_begin + l]];
                Xt[c * n_tnode + t.node_begin + l] = exact ? xg - o : xg;
            }
        }
    }
    std::vector<double> part_dummy;
#define UP(vec, ptr)                                                                                       \
    do {                                                                                                   \
        std::remove_const_t<std::remove_pointer_t<decltype(ptr)>> *p_ = nullptr;                           \
        st = upload(m, vec, &p_, stream);                                                                  \
        if (st != TLFEA_OK) { free_mesh_memory(m); delete m; return st; }                                  \
        ptr = p_;                                                                                          \
    } while (0)
    UP(hb.tiles, d.tiles);
    UP(hb.conn_local, d.conn_local);
    UP(hb.lnode_gid, d.lnode_gid);
    UP(hb.lnode_pos, d.lnode_pos);
    UP(hb.lnode_dst, d.lnode_dst);
    UP(hb.lnode_ptr, d.lnode_ptr);
    UP(hb.lnode_slot, d.lnode_slot);
    UP(hb.elem_uid, d.elem_uid);
    UP(m->blocks, d.blocks);
    UP(Xt, d.Xt);
    UP(hb.halo_gid, d.halo_gid);
    UP(hb.halo_ptr, d.halo_ptr);
#undef UP
    // Consistent-mass coefficients rho w_q J_p(xi_q) per mass-rule point and
    // internal element (Sec. 4.1 with the change of variables of Sec. 6),
    // [nqm][n_elem], J_p from the element's nodes relative to its first node.
    d.mass_c = nullptr;
    for (int b = 0; b < n_blocks; ++b) m->has_mass |= blocks[b].rho > 0;
    if (m->has_mass && m->n_elem > 0) {
        int nqm = 0;
        for (int b = 0; b < n_blocks; ++b) nqm = std::max(nqm, nqm_of(blocks[b].elem));
        std::vector<int64_t> uid0(n_blocks + 1, 0);
        for (int b = 0; b < n_blocks; ++b) uid0[b + 1] = uid0[b] + blocks[b].n_elem;
        const int64_t ne = m->n_elem;
        std::vector<double> mc((size_t)nqm * ne, 0.0);
        for (const TileDesc &t : hb.tiles) {
            const tlfea_block &B = blocks[t.block];
            if (!(B.rho > 0)) continue;
            const int nen = nen_of(B.elem);
            for (int i = 0; i < t.n_elem; ++i) {
                const int64_t ie = t.elem_begin + i;
                const int32_t *c = B.conn + (hb.elem_uid[ie] - uid0[t.block]) * nen;
                for (int q = 0; q < nqm_of(B.elem); ++q) {
                    double J[9] = {0};
                    for (int a = 1; a < nen; ++a)
                        for (int r = 0; r < 3; ++r) {
                            const double u = X[r * n_nodes + c[a]] - X[r * n_nodes + c[0]];
                            for (int k = 0; k < 3; ++k) J[3 * r + k] += u * mass_grad_of(B.elem, q, a, k);
                        }
                    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                                       J[2] * (J[3] * J[7] - J[4] * J[6]);
                    mc[(size_t)q * ne + ie] = B.rho * mass_weight_of(B.elem, q) * det;
                }
            }
        }
        double *p_ = nullptr;
        st = upload(m, mc, &p_, stream);
        if (st != TLFEA_OK) { free_mesh_memory(m); delete m; return st; }
        d.mass_c = p_;
        // the host table is freed on return: finish the copy now
        const hipError_t es = hipStreamSynchronize(stream);
        if (es != hipSuccess) { free_mesh_memory(m); delete m; return fail(TLFEA_E_DEVICE, "%s", hipGetErrorString(es)); }
    }
    d.n_nodes = n_nodes;
    d.n_elem = m->n_elem;
    d.n_part = hb.n_part;
    d.n_halo = (int64_t)hb.halo_gid.size();
    d.n_tnode = n_tnode;
    d.part = nullptr;
    if (hb.n_part > 0) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, sizeof(double) * 6 * (size_t)hb.n_part);
        if (e != hipSuccess) {
            free_mesh_memory(m);
            delete m;
            return fail(TLFEA_E_NOMEM, "hipMalloc of partial buffer: %s", hipGetErrorString(e));
        }
        m->allocations.push_back(p);
        m->device_bytes += (int64_t)(sizeof(double) * 6 * hb.n_part);
        d.part = static_cast<double *>(p);
    }
    // the host tables above are freed on return: the uploads must be done
    const hipError_t es = hipStreamSynchronize(stream);
    if (es != hipSuccess) {
        free_mesh_memory(m);
        delete m;
        return fail(TLFEA_E_DEVICE, "hipStreamSynchronize after the uploads: %s", hipGetErrorString(es));
    }
    *out = m;
    return TLFEA_OK;
}

// ------------------------------------------------------------------ launching

// Owns a pair of timing events until they are handed to the mesh's pending
// list; destroys them on any early return.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// One kernel launch, bracketed by events on the stream when timed (kernel
// id kid of the profile).
template <typename Launch>
static tlfea_status timed_launch(tlfea_mesh *m, int kid, hipStream_t s, bool timed, const char *what, Launch &&launch)
{
    EventPair ev;
    if (timed) {
        HIP_TRY(hipEventCreate(&ev.e0));
        HIP_TRY(hipEventCreate(&ev.e1));
        HIP_TRY(hipEventRecord(ev.e0, s));
    }
    const hipError_t e = launch();
    if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "%s launch: %s", what, hipGetErrorString(e));
    if (timed) {
        HIP_TRY(hipEventRecord(ev.e1, s));
        m->pending[kid].push_back({ev.e0, ev.e1});
        ev.e0 = ev.e1 = nullptr;
    }
    return TLFEA_OK;
}

// The launches of one call: every tile class, then the shared-node sums.
// dm is the mesh's device description (its partial buffer may be replaced,
// see tlfea_internal_force_noalloc).
static tlfea_status enqueue(tlfea_mesh *m, const DevMesh &dm, int kind, const CallArgs &c, hipStream_t s, bool timed)
{
    for (const ClassRange &cr : m->classes) {
        const int nc = cr.nc[kind_slot(kind)];
        const size_t lds = lds_bytes(cr, kind, nc);
        tlfea_status st = timed_launch(m, kind, s, timed, "tile kernel", [&] {
            return launch_tiles(cr.elem, cr.law, cr.damped, cr.te, kind, cr.tile_count, lds, s, dm, c,
                                cr.tile_begin, cr.nl_cap, nc);
        });
        if (st != TLFEA_OK) return st;
    }
    double *o1 = (kind == kKVjp) ? c.out1 : nullptr;
    const double *sub = kind == kKRes ? c.sub : nullptr;
    if (dm.n_halo > 0 && (c.out0 || o1))
        return timed_launch(m, 3, s, timed, "shared-node kernel",
                            [&] { return launch_halo(s, dm, c.out0, o1, sub); });
    return TLFEA_OK;
}

static tlfea_status run(tlfea_mesh *m, int kind, const CallArgs &c, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(TLFEA_E_INVALID, "current device %d differs from the mesh's device %d", dev, m->device);
    // A stream the caller is capturing gets the launches themselves (the
    // caller's graph then holds them, e.g. forward, adjoint and tangent in
    // one graph); kernel timing is off inside a capture.
    if (s != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(s, &cs));
        if (cs != hipStreamCaptureStatusNone) return enqueue(m, m->dm, kind, c, s, false);
    }
    // graphs cannot be captured on the null stream: launch directly there
    if (!(m->flags & TLFEA_BATCHED) || s == nullptr) return enqueue(m, m->dm, kind, c, s, m->prof);
    // batched: one hipGraph per (op, operand pointers, stream), replayed
    // the time step enters the kernels' arguments: its bits are part of the key
    uintptr_t hbits = 0;
    static_assert(sizeof(double) <= sizeof(uintptr_t), "a double fits a pointer-sized key");
    std::memcpy(&hbits, &c.h, sizeof(double));
    const void *hkey = reinterpret_cast<const void *>(hbits);
    const void *key[14] = {c.x, c.v, c.theta, c.w, c.dx, c.dv, c.dtheta, c.qn, c.vn, c.sub, hkey,
                           c.out0, c.out1, c.gtheta};
    GraphEntry *hit = nullptr;
    for (auto &g : m->graphs)
        if (g.kind == kind && g.stream == s && std::memcmp(g.key, key, sizeof key) == 0) hit = &g;
    hipGraph_t graph = nullptr;
    if (!hit) {
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        tlfea_status st = enqueue(m, m->dm, kind, c, s, false);
        hipError_t ec = hipStreamEndCapture(s, &graph);
        if (st != TLFEA_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (ec != hipSuccess) return fail(TLFEA_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        // A full cache: the least recently used graph of the same operation
        // on the same stream has the same launches with other operands, so
        // its executable graph is updated in place (after its last launch
        // has finished) instead of instantiating another one.
        if (m->graphs.size() >= 8) {
            GraphEntry *same = nullptr;
            for (auto &g : m->graphs)
                if (g.kind == kind && g.stream == s && (!same || g.stamp < same->stamp)) same = &g;
            if (same) {
                hipError_t ew = hipEventSynchronize(same->done);
                if (ew != hipSuccess) {
                    (void)hipGraphDestroy(graph);
                    return fail(TLFEA_E_DEVICE, "waiting for a cached graph: %s", hipGetErrorString(ew));
                }
                hipGraphNode_t err_node = nullptr;
                hipGraphExecUpdateResult res = hipGraphExecUpdateError;
                const hipError_t eu = hipGraphExecUpdate(same->exec, graph, &err_node, &res);
                if (eu == hipSuccess && res == hipGraphExecUpdateSuccess) {
                    (void)hipGraphDestroy(graph);
                    std::memcpy(same->key, key, sizeof key);
                    ++m->graph_updates;
                    hit = same;
                } else {
                    (void)hipGetLastError();   // a refused update leaves no sticky error
                }
            }
        }
    }
    if (!hit) {
        GraphEntry ge;
        ge.kind = kind;
        std::memcpy(ge.key, key, sizeof key);
        ge.stream = s;
        ge.stamp = ++m->stamp;
        hipError_t ei = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(TLFEA_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        ++m->graph_builds;
        ei = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
        if (ei != hipSuccess) {
            (void)hipGraphExecDestroy(ge.exec);
            return fail(TLFEA_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(ei));
        }
        if (m->graphs.size() >= 8) {
            // the least recently used graph; its last launch may still run
            auto old = std::min_element(m->graphs.begin(), m->graphs.end(),
                                        [](const GraphEntry &a, const GraphEntry &b) { return a.stamp < b.stamp; });
            const hipError_t ew = hipEventSynchronize(old->done);
            (void)hipGraphExecDestroy(old->exec);
            (void)hipEventDestroy(old->done);
            m->graphs.erase(old);
            if (ew != hipSuccess) return fail(TLFEA_E_DEVICE, "waiting for an evicted graph: %s", hipGetErrorString(ew));
        }
        m->graphs.push_back(ge);
        hit = &m->graphs.back();
    }
    hit->stamp = ++m->stamp;
    hipGraphExec_t exec = hit->exec;
    const tlfea_status st = timed_launch(m, 4, s, m->prof, "graph", [&] { return hipGraphLaunch(exec, s); });
    if (st != TLFEA_OK) return st;
    HIP_TRY(hipEventRecord(hit->done, s));
    return TLFEA_OK;
}

static tlfea_status check_mesh(const tlfea_mesh *m)
{
    if (!m) return fail(TLFEA_E_INVALID, "mesh is NULL");
    return TLFEA_OK;
}

// A device array of a call: its address range (null arrays are skipped).
struct Span {
    const void *p;
    size_t bytes;
    const char *name;
};

static bool overlaps(const Span &a, const Span &b)
{
    if (!a.p || !b.p || !a.bytes || !b.bytes) return false;
    const uintptr_t a0 = (uintptr_t)a.p, b0 = (uintptr_t)b.p;
    return a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}

// Outputs are written while tiles still stage inputs, so an output may share
// no byte with an input or with another output.
static tlfea_status check_overlap(std::initializer_list<Span> ins, std::initializer_list<Span> outs)
{
    for (auto o = outs.begin(); o != outs.end(); ++o) {
        for (const Span &i : ins)
            if (overlaps(*o, i)) return fail(TLFEA_E_INVALID, "output %s overlaps input %s", o->name, i.name);
        for (auto o2 = outs.begin(); o2 != o; ++o2)
            if (overlaps(*o, *o2)) return fail(TLFEA_E_INVALID, "outputs %s and %s overlap", o2->name, o->name);
    }
    return TLFEA_OK;
}

static size_t nodal_bytes(const tlfea_mesh *m) { return sizeof(double) * 3 * (size_t)m->n_nodes; }
static size_t param_bytes(const tlfea_mesh *m) { return sizeof(double) * TLFEA_NPAR * (size_t)m->n_elem; }

extern "C" tlfea_status tlfea_internal_force(tlfea_mesh *m, const double *x, const double *v, const double *theta,
                                             double *f, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!x || !f)) return fail(TLFEA_E_INVALID, "x and f are required");
    if (m->any_damped && m->n_elem > 0 && !v) return fail(TLFEA_E_INVALID, "v is required: a block is damped");
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{x, nb, "x"}, {v, nb, "v"}, {theta, pb, "theta"}}, {{f, nb, "f"}});
    if (st) return st;
    CallArgs c{};
    c.x = x; c.v = v; c.theta = theta; c.out0 = f;
    if (m->n_nodes == 0) return TLFEA_OK;
    return run(m, kKFwd, c, stream);
}

extern "C" tlfea_status tlfea_internal_force_vjp(tlfea_mesh *m, const double *x, const double *v, const double *theta,
                                                 const double *w, double *gx, double *gv, double *gtheta, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!x || !w)) return fail(TLFEA_E_INVALID, "x and w are required");
    if (m->any_damped && m->n_elem > 0 && !v) return fail(TLFEA_E_INVALID, "v is required: a block is damped");
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{x, nb, "x"}, {v, nb, "v"}, {theta, pb, "theta"}, {w, nb, "w"}},
                       {{gx, nb, "gx"}, {gv, nb, "gv"}, {gtheta, pb, "gtheta"}});
    if (st) return st;
    if (m->n_nodes == 0 || (!gx && !gv && !gtheta)) return TLFEA_OK;
    CallArgs c{};
    c.x = x; c.v = v; c.theta = theta; c.w = w; c.out0 = gx; c.out1 = gv; c.gtheta = gtheta;
    return run(m, kKVjp, c, stream);
}

extern "C" tlfea_status tlfea_tangent_jvp(tlfea_mesh *m, const double *x, const double *v, const double *theta,
                                          const double *dx, const double *dv, const double *dtheta, double *df,
                                          void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!x || !df)) return fail(TLFEA_E_INVALID, "x and df are required");
    if (m->any_damped && m->n_elem > 0 && !v) return fail(TLFEA_E_INVALID, "v is required: a block is damped");
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{x, nb, "x"}, {v, nb, "v"}, {theta, pb, "theta"}, {dx, nb, "dx"}, {dv, nb, "dv"},
                        {dtheta, pb, "dtheta"}},
                       {{df, nb, "df"}});
    if (st) return st;
    if (m->n_nodes == 0) return TLFEA_OK;
    CallArgs c{};
    c.x = x; c.v = v; c.theta = theta; c.dx = dx; c.dv = m->any_damped ? dv : nullptr; c.dtheta = dtheta;
    c.out0 = df;
    return run(m, kKJvp, c, stream);
}

extern "C" tlfea_status tlfea_mass_action(tlfea_mesh *m, const double *u, double *y, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!u || !y)) return fail(TLFEA_E_INVALID, "u and y are required");
    const size_t nb = nodal_bytes(m);
    st = check_overlap({{u, nb, "u"}}, {{y, nb, "y"}});
    if (st) return st;
    if (m->n_nodes == 0) return TLFEA_OK;
    CallArgs c{};
    c.x = u; c.out0 = y;
    return run(m, kKMass, c, stream);
}

static tlfea_status check_step(double h)
{
    if (!std::isfinite(h) || !(h > 0)) return fail(TLFEA_E_INVALID, "time step h = %g must be finite and > 0", h);
    return TLFEA_OK;
}

extern "C" tlfea_status tlfea_step_residual(tlfea_mesh *m, const double *q_n, const double *v_n, const double *v,
                                            double h, const double *theta, const double *f_ext, double *g,
                                            void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!q_n || !v_n || !v || !g)) return fail(TLFEA_E_INVALID, "q_n, v_n, v and g are required");
    if ((st = check_step(h))) return st;
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{q_n, nb, "q_n"}, {v_n, nb, "v_n"}, {v, nb, "v"}, {theta, pb, "theta"}, {f_ext, nb, "f_ext"}},
                       {{g, nb, "g"}});
    if (st) return st;
    if (m->n_nodes == 0) return TLFEA_OK;
    CallArgs c{};
    c.v = v; c.qn = q_n; c.vn = v_n; c.h = h; c.theta = theta; c.sub = f_ext; c.out0 = g;
    return run(m, kKRes, c, stream);
}

extern "C" tlfea_status tlfea_newton_operator(tlfea_mesh *m, const double *q_n, const double *v, double h,
                                              const double *theta, const double *dv, double *y, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!q_n || !v || !dv || !y)) return fail(TLFEA_E_INVALID, "q_n, v, dv and y are required");
    if ((st = check_step(h))) return st;
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{q_n, nb, "q_n"}, {v, nb, "v"}, {theta, pb, "theta"}, {dv, nb, "dv"}}, {{y, nb, "y"}});
    if (st) return st;
    if (m->n_nodes == 0) return TLFEA_OK;
    CallArgs c{};
    c.v = v; c.qn = q_n; c.h = h; c.theta = theta; c.dv = dv; c.out0 = y;
    return run(m, kKNewt, c, stream);
}

// ------------------------------------------------------------------ Newton-Krylov step

// Workspace layout of tlfea_newton_step (doubles): the Krylov basis
// V_0..V_m, then w, x (the increment), b (= -g) and r, each 3 n_nodes long,
// then the dot-product partial sums, then the device copies of one
// iteration's scalars (two sets of projections, the squared norm, and the
// two sets of negated projections).
static int64_t newton_scalar_doubles(int restart) { return 4 * (int64_t)(restart + 1) + 8; }

static int64_t newton_workspace_doubles(const tlfea_mesh *m, int restart)
{
    const int64_t N = 3 * m->n_nodes;
    const int64_t chunks = (restart + 1 + kVecChunk - 1) / kVecChunk;
    return (int64_t)(restart + 5) * N + (int64_t)kDotBlocks * kVecChunk * chunks + newton_scalar_doubles(restart);
}

extern "C" tlfea_status tlfea_newton_workspace(const tlfea_mesh *m, int32_t restart, int64_t *n_doubles)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (!n_doubles) return fail(TLFEA_E_INVALID, "n_doubles is NULL");
    if (restart < 1 || restart > 200) return fail(TLFEA_E_INVALID, "restart = %d outside [1, 200]", restart);
    *n_doubles = newton_workspace_doubles(m, restart);
    return TLFEA_OK;
}

namespace {

// The solver's device vector algebra on one stream; every scalar result is
// summed on the host from fixed per-block partials (bitwise repeatable).
struct Krylov {
    tlfea_mesh *m;
    hipStream_t s;
    int64_t N;
    double *partial;
    std::vector<double> host;

    // out[k] = V_k . w, k < nvec: every chunk of eight vectors writes its own
    // partials, then one copy and one synchronisation; each product is the
    // sum of its block partials in block order
    tlfea_status dots(const double *V, int nvec, const double *w, double *out)
    {
        host.resize((size_t)kDotBlocks * nvec);
        for (int k0 = 0; k0 < nvec; k0 += kVecChunk) {
            const int nv = std::min(kVecChunk, nvec - k0);
            hipError_t e = launch_mdot(V + (int64_t)k0 * N, N, nv, w, N, partial + (int64_t)k0 * kDotBlocks, s);
            if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "dot kernel: %s", hipGetErrorString(e));
        }
        HIP_TRY(hipMemcpyAsync(host.data(), partial, sizeof(double) * kDotBlocks * nvec, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int k = 0; k < nvec; ++k) {
            double t = 0.0;
            for (int b = 0; b < kDotBlocks; ++b) t += host[(size_t)k * kDotBlocks + b];
            out[k] = t;
        }
        return TLFEA_OK;
    }
    tlfea_status norm(const double *w, double *out)
    {
        double d = 0.0;
        tlfea_status st = dots(w, 1, w, &d);
        *out = std::sqrt(d);
        return st;
    }
    // y += sum_k c_k V_k
    tlfea_status combine(const double *V, int nvec, const double *c, double *y)
    {
        for (int k0 = 0; k0 < nvec; k0 += kVecChunk) {
            const int nv = std::min(kVecChunk, nvec - k0);
            hipError_t e = launch_maxpy(V + (int64_t)k0 * N, N, nv, c + k0, y, N, s);
            if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "combination kernel: %s", hipGetErrorString(e));
        }
        return TLFEA_OK;
    }
    tlfea_status axpby(double a, const double *x, double b, double *y)
    {
        hipError_t e = launch_axpby(a, x, b, y, N, s);
        return e == hipSuccess ? TLFEA_OK : fail(TLFEA_E_DEVICE, "vector kernel: %s", hipGetErrorString(e));
    }
};

}  // namespace

// One matrix-free Newton step of the step residual (Sec. 7, without
// constraints): dv solves (M/h + h K + C) dv = -g(v) approximately by
// restarted GMRES (classical Gram-Schmidt applied twice, Givens rotations
// on the host), each operator product one pass of the Newton-operator
// kernels; v_out = v + dv.
extern "C" tlfea_status tlfea_newton_step(tlfea_mesh *m, const double *q_n, const double *v_n, const double *v,
                                          double h, const double *theta, const double *f_ext,
                                          const tlfea_krylov_opts *opts, double *v_out, double *work,
                                          int64_t work_len, tlfea_krylov_info *info, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (!opts || !info) return fail(TLFEA_E_INVALID, "opts and info are required");
    if (m->n_nodes > 0 && (!q_n || !v_n || !v || !v_out || !work))
        return fail(TLFEA_E_INVALID, "q_n, v_n, v, v_out and work are required");
    if ((st = check_step(h))) return st;
    const int restart = opts->restart;
    if (restart < 1 || restart > 200) return fail(TLFEA_E_INVALID, "restart = %d outside [1, 200]", restart);
    if (opts->max_iters < 1) return fail(TLFEA_E_INVALID, "max_iters must be >= 1");
    if (!(opts->rtol >= 0) || !std::isfinite(opts->rtol)) return fail(TLFEA_E_INVALID, "rtol must be finite and >= 0");
    const int64_t need = newton_workspace_doubles(m, restart);
    if (work_len < need)
        return fail(TLFEA_E_SHAPE, "workspace of %lld doubles, %lld needed", (long long)work_len, (long long)need);
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{q_n, nb, "q_n"}, {v_n, nb, "v_n"}, {v, nb, "v"}, {theta, pb, "theta"}, {f_ext, nb, "f_ext"}},
                       {{v_out, nb, "v_out"}, {work, sizeof(double) * (size_t)work_len, "work"}});
    if (st) return st;
    *info = tlfea_krylov_info{};
    if (m->n_nodes == 0) {
        info->converged = 1;
        return TLFEA_OK;
    }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(TLFEA_E_INVALID, "current device %d differs from the mesh's device %d", dev, m->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t N = 3 * m->n_nodes;
    double *V = work, *w = work + (int64_t)(restart + 1) * N, *x = w + N, *b = x + N, *r = b + N;
    Krylov K{m, s, N, r + N, {}};
    // this iteration's scalars on the device: projections of the two
    // sweeps (ha, hb), the squared norm (nn, beside them for one copy), and
    // the negated projections the next sweep adds (ca, cb)
    const int64_t R1 = restart + 1;
    double *ha = K.partial + (int64_t)kDotBlocks * kVecChunk * ((R1 + kVecChunk - 1) / kVecChunk);
    double *hb = ha + R1, *nn = hb + R1, *ca = nn + 8, *cb = ca + R1;
    std::vector<double> hs((size_t)(2 * R1 + 1));
    CallArgs rc{};
    rc.v = v; rc.qn = q_n; rc.vn = v_n; rc.h = h; rc.theta = theta; rc.sub = f_ext; rc.out0 = b;
    if ((st = enqueue(m, m->dm, kKRes, rc, s, false))) return st;      // b = g(v)
    if ((st = K.axpby(-1.0, b, 0.0, b))) return st;                   // b = -g
    if ((st = K.axpby(0.0, b, 0.0, x))) return st;                    // x = 0
    double gnorm = 0.0;
    if ((st = K.norm(b, &gnorm))) return st;
    info->g_norm = gnorm;
    const double target = opts->rtol * gnorm;
    auto apply = [&](const double *in, double *out) {   // out = (M/h + hK + C) in
        CallArgs c{};
        c.v = v; c.qn = q_n; c.h = h; c.theta = theta; c.dv = in; c.out0 = out;
        return enqueue(m, m->dm, kKNewt, c, s, false);
    };
    double beta = gnorm;
    const double *r0 = b;            // x = 0: the first residual is b
    int iters = 0;
    bool converged = !(beta > target);
    std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), y(restart),
        hc(restart + 1), hc2(restart + 1);
    while (!converged && iters < opts->max_iters) {
        if ((st = K.axpby(1.0 / beta, r0, 0.0, V))) return st;          // V_0 = r / beta
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        for (; j < restart && iters < opts->max_iters; ++j) {
            double *Vj = V + (int64_t)j * N;
            if ((st = apply(Vj, w))) return st;
            // classical Gram-Schmidt, twice
            double hn = 0.0;
            if (j + 1 <= kCgsMax) {
                // three sweeps over the basis (projections; first update and
                // second projections; second update and norm) with the
                // scalars between them summed on the device, then one copy
                // and one synchronisation; the same operations in the same
                // order as the path below
                const int nv = j + 1;
                hipError_t e = launch_cgs(0, V, N, nv, nullptr, w, N, K.partial, s);
                if (e == hipSuccess) e = launch_sum_partials(K.partial, nv, ha, ca, s);
                if (e == hipSuccess) e = launch_cgs(1, V, N, nv, ca, w, N, K.partial, s);
                if (e == hipSuccess) e = launch_sum_partials(K.partial, nv, hb, cb, s);
                if (e == hipSuccess) e = launch_cgs(2, V, N, nv, cb, w, N, K.partial, s);
                if (e == hipSuccess) e = launch_sum_partials(K.partial, 1, nn, nullptr, s);
                if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "Gram-Schmidt kernels: %s", hipGetErrorString(e));
                HIP_TRY(hipMemcpyAsync(hs.data(), ha, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                for (int i = 0; i <= j; ++i) hc[i] = hs[i] + hs[(size_t)R1 + i];
                hn = std::sqrt(hs[(size_t)2 * R1]);
            } else {
                if ((st = K.dots(V, j + 1, w, hc.data()))) return st;
                for (int i = 0; i <= j; ++i) hc2[i] = -hc[i];
                if ((st = K.combine(V, j + 1, hc2.data(), w))) return st;
                if ((st = K.dots(V, j + 1, w, hc2.data()))) return st;
                for (int i = 0; i <= j; ++i) {
                    hc[i] += hc2[i];
                    hc2[i] = -hc2[i];
                }
                if ((st = K.combine(V, j + 1, hc2.data(), w))) return st;
                if ((st = K.norm(w, &hn))) return st;
            }
            // the new column, rotated by the previous Givens rotations
            for (int i = 0; i <= j; ++i) H[(size_t)i * restart + j] = hc[i];
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * restart + j], c2 = H[(size_t)(i + 1) * restart + j];
                H[(size_t)i * restart + j] = cs[i] * a + sn[i] * c2;
                H[(size_t)(i + 1) * restart + j] = -sn[i] * a + cs[i] * c2;
            }
            const double a = H[(size_t)j * restart + j];
            const double rr = std::hypot(a, hn);
            cs[j] = rr > 0 ? a / rr : 1.0;
            sn[j] = rr > 0 ? hn / rr : 0.0;
            H[(size_t)j * restart + j] = rr;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            const bool breakdown = !(hn > 0);
            if (!breakdown && j + 1 <= restart)
                if ((st = K.axpby(1.0 / hn, w, 0.0, V + (int64_t)(j + 1) * N))) return st;
            if (std::fabs(g[j + 1]) <= target || breakdown) {
                ++j;
                break;
            }
        }
        // x += V y, H y = g (upper triangular, j columns)
        for (int i = j - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < j; ++k) t -= H[(size_t)i * restart + k] * y[k];
            y[i] = t / H[(size_t)i * restart + i];
        }
        if ((st = K.combine(V, j, y.data(), x))) return st;
        // true residual r = b - A x
        if ((st = apply(x, w))) return st;
        if ((st = K.axpby(1.0, b, 0.0, r))) return st;
        if ((st = K.axpby(-1.0, w, 1.0, r))) return st;
        if ((st = K.norm(r, &beta))) return st;
        r0 = r;
        converged = !(beta > target);
    }
    info->iters = iters;
    info->converged = converged ? 1 : 0;
    info->res_norm = beta;
    hipError_t e = launch_add(v, x, v_out, N, s);
    if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "vector kernel: %s", hipGetErrorString(e));
    HIP_TRY(hipStreamSynchronize(s));
    return TLFEA_OK;
}

// The forward with the shared-node partial sums in the library's static
// device scratch instead of the mesh's buffer; launches directly (no graph
// capture, no timing events), so no call in it allocates.  Every partial
// slot is written by its tile before the shared-node kernel reads it, so
// the scratch needs no clearing between calls.
extern "C" tlfea_status tlfea_internal_force_noalloc(tlfea_mesh *m, const double *x, const double *v,
                                                     const double *theta, double *f, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (m->n_nodes > 0 && (!x || !f)) return fail(TLFEA_E_INVALID, "x and f are required");
    if (m->any_damped && m->n_elem > 0 && !v) return fail(TLFEA_E_INVALID, "v is required: a block is damped");
    const size_t nb = nodal_bytes(m), pb = param_bytes(m);
    st = check_overlap({{x, nb, "x"}, {v, nb, "v"}, {theta, pb, "theta"}}, {{f, nb, "f"}});
    if (st) return st;
    if (3 * m->dm.n_part > kScratchDoubles)
        return fail(TLFEA_E_UNSUPPORTED, "the mesh has %lld shared-node partials; the static scratch holds %lld "
                    "(three rows each): use tlfea_internal_force", (long long)m->dm.n_part,
                    (long long)(kScratchDoubles / 3));
    if (m->n_nodes == 0) return TLFEA_OK;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(TLFEA_E_INVALID, "current device %d differs from the mesh's device %d", dev, m->device);
    DevMesh dm = m->dm;
    HIP_TRY(scratch_address(&dm.part));
    CallArgs c{};
    c.x = x; c.v = v; c.theta = theta; c.out0 = f;
    return enqueue(m, dm, kKFwd, c, static_cast<hipStream_t>(stream), false);
}

extern "C" tlfea_status tlfea_count_inverted(tlfea_mesh *m, const double *x, int64_t *count, void *stream)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (!count) return fail(TLFEA_E_INVALID, "count is NULL");
    if (m->n_nodes > 0 && !x) return fail(TLFEA_E_INVALID, "x is required");
    st = check_overlap({{x, nodal_bytes(m), "x"}}, {{count, sizeof(int64_t), "count"}});
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(TLFEA_E_INVALID, "current device %d differs from the mesh's device %d", dev, m->device);
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(count);
    hipError_t e = launch_zero_count(s, cnt);
    if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    CallArgs c{};
    c.x = x;
    for (const ClassRange &cr : m->classes) {
        const size_t lds = (size_t)cr.nl_cap * record_len(kOpFwd, false) * sizeof(double);
        typedef hipError_t (*inv_t)(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int,
                                    unsigned long long *);
        static const inv_t inv[3] = {launch_inverted_e0_o0, launch_inverted_e1_o0, launch_inverted_e2_o0};
        e = inv[cr.elem](cr.te, cr.tile_count, lds, s, m->dm, c, cr.tile_begin, cnt);
        if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    }
    return TLFEA_OK;
}

// ------------------------------------------------------------------ autotune

// Time forward + adjoint + tangent per class for one candidate tile size.
static tlfea_status time_classes(tlfea_mesh *m, const double *X_host, hipStream_t s, std::vector<double> &t_cls)
{
    const size_t nb = sizeof(double) * 3 * (size_t)m->n_nodes;
    struct Buffers {   // freed on every return
        double *p[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        ~Buffers()
        {
            for (double *q : p)
                if (q) (void)hipFree(q);
        }
    } buf;
    for (double *&q : buf.p) HIP_TRY(hipMalloc(&q, nb));
    double *x = buf.p[0], *v = buf.p[1], *w = buf.p[2], *o0 = buf.p[3], *o1 = buf.p[4];
    HIP_TRY(hipMemcpyAsync(x, X_host, nb, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(v, 0, nb, s));
    HIP_TRY(hipMemsetAsync(w, 0, nb, s));
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.e0));
    HIP_TRY(hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    t_cls.assign(m->classes.size(), 0.0);
    for (size_t k = 0; k < m->classes.size(); ++k) {
        const ClassRange &cr = m->classes[k];
        for (int op = kKFwd; op <= kKJvp; ++op) {
            CallArgs c{};
            c.x = x; c.v = v; c.w = w; c.dx = w; c.dv = v; c.out0 = o0; c.out1 = op == kKVjp ? o1 : nullptr;
            const size_t lds = lds_bytes(cr, op, cr.nc[kind_slot(op)]);
            float best = 1e30f;
            for (int rep = 0; rep < 4; ++rep) {
                HIP_TRY(hipEventRecord(e0, s));
                hipError_t e = launch_tiles(cr.elem, cr.law, cr.damped, cr.te, op, cr.tile_count, lds, s, m->dm,
                                            c, cr.tile_begin, cr.nl_cap, cr.nc[kind_slot(op)]);
                if (e != hipSuccess) return fail(TLFEA_E_DEVICE, "autotune launch: %s", hipGetErrorString(e));
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) best = std::min(best, ms);
            }
            t_cls[k] += best;
        }
    }
    return TLFEA_OK;
}

extern "C" tlfea_status tlfea_create_mesh(int64_t n_nodes, const double *X, int32_t n_blocks,
                                          const tlfea_block *blocks, int32_t flags, void *stream, tlfea_mesh **out)
{
    if (!out) return fail(TLFEA_E_INVALID, "out is NULL");
    *out = nullptr;
    tlfea_status st = validate_args(n_nodes, X, n_blocks, blocks, flags);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (st) return st;
    std::vector<int> te(n_blocks);
    for (int b = 0; b < n_blocks; ++b) te[b] = blocks[b].tile_elems ? blocks[b].tile_elems : default_te(blocks[b].elem);
    if (!(flags & TLFEA_AUTOTUNE)) return create_with(n_nodes, X, n_blocks, blocks, flags, te, s, out);
    // Autotune: per element type, the tile size with the smallest forward +
    // adjoint + tangent time summed over the classes of that type (one size
    // per type, as tlfea_get_mesh_info reports it); blocks that fix
    // tile_elems keep it.
    // Q27 tiles take 64 or 128 elements (the LDS of their node records)
    const int cand[3][4] = {{64, 128, 192, 256}, {64, 128, 192, 256}, {64, 128, 0, 0}};
    double best_t[3] = {1e300, 1e300, 1e300};
    int best_c[3] = {default_te(kT10), default_te(kH8), default_te(kQ27)};
    for (int ci = 0; ci < 4; ++ci) {
        std::vector<int> tc(n_blocks);
        for (int b = 0; b < n_blocks; ++b) {
            const int e = blocks[b].elem;
            tc[b] = blocks[b].tile_elems ? blocks[b].tile_elems : (cand[e][ci] ? cand[e][ci] : best_c[e]);
        }
        tlfea_mesh *m = nullptr;
        st = create_with(n_nodes, X, n_blocks, blocks, flags & ~TLFEA_BATCHED, tc, s, &m);
        if (st) return st;
        std::vector<double> t;
        st = time_classes(m, X, s, t);
        if (st) {
            tlfea_destroy_mesh(m);
            return st;
        }
        double sum[3] = {0.0, 0.0, 0.0};
        for (size_t k = 0; k < m->classes.size(); ++k) sum[m->classes[k].elem] += t[k];
        for (int e = 0; e < 3; ++e)
            if (cand[e][ci] && sum[e] < best_t[e]) {
                best_t[e] = sum[e];
                best_c[e] = cand[e][ci];
            }
        tlfea_destroy_mesh(m);
    }
    std::vector<int> best_te = te;
    for (int b = 0; b < n_blocks; ++b)
        if (!blocks[b].tile_elems) best_te[b] = best_c[blocks[b].elem];
    return create_with(n_nodes, X, n_blocks, blocks, flags, best_te, s, out);
}

extern "C" void tlfea_destroy_mesh(tlfea_mesh *m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();   // no enqueued call may still use the mesh
    free_mesh_memory(m);
    delete m;
}

extern "C" tlfea_status tlfea_get_mesh_info(const tlfea_mesh *m, tlfea_mesh_info *info)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (!info) return fail(TLFEA_E_INVALID, "info is NULL");
    info->n_nodes = m->n_nodes;
    info->n_elem = m->n_elem;
    info->n_qp = m->n_qp;
    info->n_tiles = m->n_tiles;
    info->n_halo_nodes = m->dm.n_halo;
    info->n_partials = m->dm.n_part;
    info->n_blocks = m->n_blocks;
    info->flags = m->flags;
    info->tile_elems_t10 = m->te_t10;
    info->tile_elems_h8 = m->te_h8;
    info->tile_elems_q27 = m->te_q27;
    info->reserved = 0;
    info->device_bytes = m->device_bytes;
    info->graphs_built = m->graph_builds;
    info->graphs_updated = m->graph_updates;
    return TLFEA_OK;
}

// ------------------------------------------------------------------ profiling

extern "C" tlfea_status tlfea_set_profiling(tlfea_mesh *m, int32_t enable)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    m->prof = enable != 0;
    return TLFEA_OK;
}

extern "C" tlfea_status tlfea_get_profile(tlfea_mesh *m, int32_t *counts, double *ms)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    for (int k = 0; k < kNumKernelIds; ++k) {
        for (auto &e : m->pending[k]) {
            HIP_TRY(hipEventSynchronize(e.second));
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, e.first, e.second));
            m->ms[k] += t;
            m->counts[k] += 1;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        m->pending[k].clear();
        if (counts) counts[k] = m->counts[k];
        if (ms) ms[k] = m->ms[k];
    }
    return TLFEA_OK;
}

extern "C" tlfea_status tlfea_reset_profile(tlfea_mesh *m)
{
    tlfea_status st = tlfea_get_profile(m, nullptr, nullptr);
    if (st) return st;
    for (int k = 0; k < kNumKernelIds; ++k) {
        m->counts[k] = 0;
        m->ms[k] = 0;
    }
    return TLFEA_OK;
}

// ------------------------------------------------------------------ node order

extern "C" tlfea_status tlfea_node_order(const tlfea_mesh *m, int32_t *order)
{
    tlfea_status st = check_mesh(m);
    if (st) return st;
    if (!order && m->n_nodes > 0) return fail(TLFEA_E_INVALID, "order is NULL");
    std::vector<int32_t> count(m->n_nodes, 0);
    for (int32_t g : m->tile_nodes) count[g]++;
    std::vector<char> seen(m->n_nodes, 0);
    int64_t k = 0;
    // nodes of one tile only, tile by tile (each tile's direct stores are
    // then dense); then the shared nodes by first appearance (the
    // shared-node kernel's stores are then dense too: 29 % faster on the
    // 1M-element T10 box than with shared nodes inside the tiles' ranges)
    for (int32_t g : m->tile_nodes)
        if (count[g] == 1) {
            seen[g] = 1;
            order[k++] = g;
        }
    for (int32_t g : m->tile_nodes)
        if (!seen[g]) {
            seen[g] = 1;
            order[k++] = g;
        }
    for (int64_t g = 0; g < m->n_nodes; ++g)
        if (!seen[g]) order[k++] = (int32_t)g;
    return TLFEA_OK;
}

// ------------------------------------------------------------------ joints

struct tlfea_joints {
    int device = 0;
    DevJoints dj{};
    std::vector<void *> allocations;
};

static void free_joints(tlfea_joints *J)
{
    for (void *p : J->allocations) (void)hipFree(p);
    J->allocations.clear();
}

template <class T>
static tlfea_status upload_joint(tlfea_joints *J, const std::vector<T> &h, T **d, hipStream_t s)
{
    *d = nullptr;
    if (h.empty()) return TLFEA_OK;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, h.size() * sizeof(T)));
    J->allocations.push_back(p);
    HIP_TRY(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    *d = static_cast<T *>(p);
    return TLFEA_OK;
}

extern "C" tlfea_status tlfea_create_joints(int64_t n_nodes, const double *X, int32_t n_joints,
                                            const tlfea_revolute *joints, void *stream, tlfea_joints **out)
{
    if (!out) return fail(TLFEA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_nodes < 0 || n_nodes > INT32_MAX) return fail(TLFEA_E_SHAPE, "n_nodes = %lld out of range", (long long)n_nodes);
    if (n_joints < 0 || (n_joints > 0 && !joints)) return fail(TLFEA_E_INVALID, "bad joint list");
    if (n_nodes > 0 && !X) return fail(TLFEA_E_INVALID, "X_ref is NULL");
    const int64_t nj = n_joints;
    int nmax = 1;
    for (int64_t j = 0; j < nj; ++j) {
        const tlfea_point *pt[5] = {&joints[j].P, &joints[j].Q, &joints[j].R, &joints[j].S, &joints[j].T};
        for (int p = 0; p < 5; ++p) {
            if (pt[p]->elem != TLFEA_T10 && pt[p]->elem != TLFEA_H8 && pt[p]->elem != TLFEA_Q27)
                return fail(TLFEA_E_INVALID, "joint %lld point %d: unknown element type %d", (long long)j, p, pt[p]->elem);
            const int nen = nen_of(pt[p]->elem);
            nmax = std::max(nmax, nen);
            for (int a = 0; a < nen; ++a)
                if (pt[p]->nodes[a] < 0 || pt[p]->nodes[a] >= n_nodes)
                    return fail(TLFEA_E_SHAPE, "joint %lld point %d: node %d outside [0, %lld)", (long long)j, p,
                                pt[p]->nodes[a], (long long)n_nodes);
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(pt[p]->xi[k]))
                    return fail(TLFEA_E_INVALID, "joint %lld point %d: parent coordinate not finite", (long long)j, p);
        }
    }
    std::vector<int32_t> ids((size_t)5 * nmax * nj, 0);
    std::vector<double> sv((size_t)5 * nmax * nj, 0.0), fw((size_t)4 * nj);
    // per node: (point p, joint j, value) entries
    std::vector<std::vector<std::pair<int64_t, double>>> by_node;
    std::vector<int32_t> touched_index(n_nodes, -1);
    std::vector<int32_t> tnode;
    for (int64_t j = 0; j < nj; ++j) {
        const tlfea_point *pt[5] = {&joints[j].P, &joints[j].Q, &joints[j].R, &joints[j].S, &joints[j].T};
        double r0[5][3];
        for (int p = 0; p < 5; ++p) {
            const int nen = nen_of(pt[p]->elem);
            for (int c = 0; c < 3; ++c) r0[p][c] = 0.0;
            for (int a = 0; a < nen; ++a) {
                const double sa = shape_of(pt[p]->elem, a, pt[p]->xi);
                const int32_t g = pt[p]->nodes[a];
                const size_t k = ((size_t)p * nmax + a) * nj + j;
                ids[k] = g;
                sv[k] = sa;
                for (int c = 0; c < 3; ++c) r0[p][c] += sa * X[c * n_nodes + g];
                if (touched_index[g] < 0) {
                    touched_index[g] = (int32_t)tnode.size();
                    tnode.push_back(g);
                    by_node.emplace_back();
                }
                by_node[touched_index[g]].push_back({(int64_t)p * nj + j, sa});
            }
        }
        double a0[3], b10[3], b20[3];
        for (int c = 0; c < 3; ++c) {
            a0[c] = r0[1][c] - r0[0][c];
            b10[c] = r0[3][c] - r0[2][c];
            b20[c] = r0[4][c] - r0[2][c];
        }
        const double aa = a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2];
        const double n1 = aa + b10[0] * b10[0] + b10[1] * b10[1] + b10[2] * b10[2];
        const double n2 = aa + b20[0] * b20[0] + b20[1] * b20[1] + b20[2] * b20[2];
        if (!(n1 > 0) || !(n2 > 0))
            return fail(TLFEA_E_INVALID, "joint %lld: the reference directions vanish (points coincide)", (long long)j);
        fw[j] = a0[0] * b10[0] + a0[1] * b10[1] + a0[2] * b10[2];
        fw[nj + j] = a0[0] * b20[0] + a0[1] * b20[1] + a0[2] * b20[2];
        fw[2 * nj + j] = 1.0 / std::sqrt(n1);
        fw[3 * nj + j] = 1.0 / std::sqrt(n2);
    }
    // entries of each touched node in (joint, point, slot) order; nodes in
    // ascending order
    std::vector<int32_t> order(tnode.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = (int32_t)t;
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return tnode[x] < tnode[y]; });
    std::vector<int32_t> tn;
    std::vector<int64_t> tptr(1, 0), tent;
    std::vector<double> tval;
    for (int32_t t : order) {
        auto &e = by_node[t];
        std::stable_sort(e.begin(), e.end(), [&](const std::pair<int64_t, double> &x, const std::pair<int64_t, double> &y) {
            const int64_t jx = x.first % std::max<int64_t>(1, nj), jy = y.first % std::max<int64_t>(1, nj);
            return jx != jy ? jx < jy : x.first < y.first;
        });
        tn.push_back(tnode[t]);
        for (auto &kv : e) {
            // the entry's row of the joint-major z: joint j, point p
            const int64_t p = kv.first / std::max<int64_t>(1, nj), jj = kv.first - p * nj;
            tent.push_back(jj * 5 + p);
            tval.push_back(kv.second);
        }
        tptr.push_back((int64_t)tent.size());
    }
    tlfea_joints *J = new (std::nothrow) tlfea_joints();
    if (!J) return fail(TLFEA_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&J->device) != hipSuccess) {
        delete J;
        return fail(TLFEA_E_DEVICE, "hipGetDevice failed");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevJoints &d = J->dj;
    d.n_joints = nj;
    d.n_nodes = n_nodes;
    d.n_touched = (int64_t)tn.size();
    d.nmax = nmax;
    tlfea_status st = TLFEA_OK;
    {
        int32_t *pi = nullptr; double *pd = nullptr; int64_t *pl = nullptr;
        if (!st) { st = upload_joint(J, ids, &pi, s); d.ids = pi; }
        if (!st) { st = upload_joint(J, sv, &pd, s); d.sv = pd; }
        if (!st) { st = upload_joint(J, fw, &pd, s); d.fw = pd; }
        if (!st) { st = upload_joint(J, tn, &pi, s); d.tnode = pi; }
        if (!st) { st = upload_joint(J, tptr, &pl, s); d.tptr = pl; }
        if (!st) { st = upload_joint(J, tent, &pl, s); d.tent = pl; }
        if (!st) { st = upload_joint(J, tval, &pd, s); d.tval = pd; }
        if (!st && nj > 0) {
            void *p = nullptr;
            hipError_t e = hipMalloc(&p, sizeof(double) * 15 * (size_t)nj);
            if (e != hipSuccess) st = fail(TLFEA_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
            else {
                J->allocations.push_back(p);
                d.z = static_cast<double *>(p);
            }
        }
        if (!st && nj > 0 && n_nodes > 0) {
            // node-major copy of each call's positions (the point gathers)
            void *p = nullptr;
            hipError_t e = hipMalloc(&p, sizeof(double) * 3 * (size_t)n_nodes);
            if (e != hipSuccess) st = fail(TLFEA_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
            else {
                J->allocations.push_back(p);
                d.qn = static_cast<double *>(p);
            }
        }
    }
    if (!st) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(TLFEA_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    if (st) {
        free_joints(J);
        delete J;
        return st;
    }
    *out = J;
    return TLFEA_OK;
}

extern "C" void tlfea_destroy_joints(tlfea_joints *J)
{
    if (!J) return;
    (void)hipDeviceSynchronize();   // no enqueued call may still use the joint set
    free_joints(J);
    delete J;
}

static tlfea_status check_joints(const tlfea_joints *J)
{
    if (!J) return fail(TLFEA_E_INVALID, "joint set is NULL");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != J->device) return fail(TLFEA_E_INVALID, "current device %d differs from the joint set's device %d", dev, J->device);
    return TLFEA_OK;
}

extern "C" tlfea_status tlfea_joint_values(tlfea_joints *J, const double *q, double *c, void *stream)
{
    tlfea_status st = check_joints(J);
    if (st) return st;
    if (J->dj.n_joints > 0 && (!q || !c)) return fail(TLFEA_E_INVALID, "q and c are required");
    st = check_overlap({{q, sizeof(double) * 3 * (size_t)J->dj.n_nodes, "q"}},
                       {{c, sizeof(double) * 5 * (size_t)J->dj.n_joints, "c"}});
    if (st) return st;
    hipError_t e = launch_joints(J->dj, q, nullptr, 0.0, 0.0, c, 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TLFEA_OK : fail(TLFEA_E_DEVICE, "joint kernel: %s", hipGetErrorString(e));
}

extern "C" tlfea_status tlfea_joint_scatter(tlfea_joints *J, const double *q, const double *lambda, double rho,
                                            double h, double *g, int32_t accumulate, void *stream)
{
    tlfea_status st = check_joints(J);
    if (st) return st;
    if (J->dj.n_nodes > 0 && (!q || !g)) return fail(TLFEA_E_INVALID, "q and g are required");
    if (!std::isfinite(rho) || !std::isfinite(h)) return fail(TLFEA_E_INVALID, "rho and h must be finite");
    const size_t nb = sizeof(double) * 3 * (size_t)J->dj.n_nodes;
    st = check_overlap({{q, nb, "q"}, {lambda, sizeof(double) * 5 * (size_t)J->dj.n_joints, "lambda"}}, {{g, nb, "g"}});
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_joints(J->dj, q, lambda, rho, h, nullptr, 1, s);
    if (e == hipSuccess) e = launch_joint_scatter(J->dj, g, accumulate ? 1 : 0, s);
    return e == hipSuccess ? TLFEA_OK : fail(TLFEA_E_DEVICE, "joint kernel: %s", hipGetErrorString(e));
}

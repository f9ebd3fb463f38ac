// Device-side mesh layout shared by the host builder and the HIP kernels.
#pragma once
#include <stdint.h>

namespace tlfea {

// One tile = one workgroup: up to `te` elements of one block (one element
// type, one law), their distinct nodes staged in LDS, and a tile-local CSR
// that sums element contributions per node in a fixed order.
struct TileDesc {
    int32_t elem_begin;   // first internal element of the tile
    int32_t n_elem;       // elements in the tile (<= te)
    int32_t node_begin;   // first entry in lnode_gid / lnode_dst
    int32_t n_node;       // distinct nodes of the tile (<= kStagePerThread * te)
    int32_t ptr_begin;    // first entry of this tile's lnode_ptr (n_node + 1 entries)
    int32_t conn_begin;   // first entry of this tile's conn_local ([nen][te])
    int32_t block;        // owning block
    int32_t ref;          // local index of the node positions are taken relative to
                          // (the tile's node nearest the centroid of its nodes)
};

// Lanes per element: a T10 or H8 element is one lane's work; a Q27 element
// (element type 2) is split over two neighbouring lanes, each evaluating
// every other quadrature point, so that a tile of te elements runs te x 2
// threads (the LDS of its node records allows few tiles per compute unit).
constexpr int lanes_per_elem(int elem) { return elem == 2 ? 2 : 1; }

// Node records a thread stages at most: a tile holds at most this many
// nodes per thread of its workgroup (element types 0, 1: T10, H8, about
// 2.2 and 1.6 distinct nodes per element in a compact tile; 2: Q27, about
// 11 per element, 6 per thread).  The staging loads are issued in rounds of
// at most kStageRound nodes per thread.
constexpr int kStagePerThread = 3;
constexpr int kStageRound = 6;
constexpr int stage_per_thread(int elem) { return elem == 2 ? 6 : kStagePerThread; }

// Slot lists: the first entry of every node's group carries this flag; the
// slot ids themselves (a * te + i) stay below it.
constexpr uint16_t kSlotHead = 0x8000;
// Entries of a tile's slot list summed by one thread: the elements' entries
// spread evenly over the tile's te * LPE threads.
constexpr int slot_chunk(int nen, int lpe) { return (nen + lpe - 1) / lpe; }

struct BlockDesc {
    double theta[5];
    int32_t elem, law, damped, pad;
};

// Pointers of the device mesh (all device memory owned by the mesh).
struct DevMesh {
    const TileDesc *tiles;
    const uint16_t *conn_local;   // LDS record position of the node per (tile, a, i)
    const int32_t *lnode_gid;     // global node of each local node
    const uint16_t *lnode_pos;    // LDS record position of each local node (a permutation)
    const int32_t *lnode_dst;     // >= 0: global node written directly; < 0: -1 - partial slot
    const int32_t *lnode_ptr;     // CSR offsets into lnode_slot
    const uint16_t *lnode_slot;   // element-force slot = a * te + i (| kSlotHead on a group's first entry)
    const int32_t *elem_uid;      // caller's element id of each internal element
    const BlockDesc *blocks;
    const double *Xt;             // [3][n_tnode] reference coordinates of every tile node,
                                  // relative to its tile's reference node (TileDesc::ref)
    const int32_t *halo_gid;      // nodes summed from partials (and nodes no element touches)
    const int32_t *halo_ptr;      // [n_halo + 1]: node h owns partial slots [halo_ptr[h], halo_ptr[h+1])
    double *part;                 // [6][n_part] partial node sums (two fields x three components)
    const double *mass_c;         // [nqm][n_elem] rho w_q J_p(xi_q) per mass-rule point and internal
                                  // element (null when no block has a density)
    int64_t n_nodes, n_elem, n_part, n_halo, n_tnode;
};

// Per-call operands (device pointers; unused ones are null).
struct CallArgs {
    const double *x, *v, *theta, *w, *dx, *dv;
    const double *dtheta;  // tangent: parameter direction (null: none)
    const double *qn, *vn; // step residual / Newton operator: q_n, v_n (positions q = q_n + h v)
    const double *sub;     // subtracted from out0 at every node when non-null (the step residual's f_ext)
    double h;              // time step of the step map
    double *out0, *out1;   // f | gx, gv | df | g | y
    double *gtheta;
};

enum { kOpFwd = 0, kOpVjp = 1, kOpJvp = 2 };

// Variants of the tile kernels: the forward with the step residual's
// staging and inertia term, the tangent with the Newton operator's.
enum { kModePlain = 0, kModeStep = 1 };
// The consistent-mass action has a kernel of its own (operation id 3 of
// the host's launch tables).
enum { kOpMass = 3 };

// Dot products of the Newton-Krylov step: partial sums per product (one per
// block of the dot kernel, added in block order on the host) and vectors per
// launch of the multi-vector kernels.
constexpr int kDotBlocks = 1024;
constexpr int kVecChunk = 8;
// Basis vectors the fused Gram-Schmidt sweeps take in one pass (larger
// bases use the chunked dot and combination kernels).
constexpr int kCgsMax = 32;

// The no-allocation forward keeps its shared-node partial sums (three rows
// of n_part doubles) in a static device array of this many doubles (64 MiB).
constexpr int64_t kScratchDoubles = int64_t(8) << 20;
constexpr int kMaxDevices = 64;

// Waves per SIMD each tile kernel is compiled for (its register budget:
// 512 / waves registers per lane), shared by the kernels' attributes and the
// host's LDS budget.  Measured per instantiation: three waves where the
// kernel then still fits its registers without spilling (the undamped
// Saint Venant-Kirchhoff and Neo-Hookean H8 adjoint and tangent, the
// undamped Saint Venant-Kirchhoff T10 tangent: 8-14 % faster), two where
// spills would cost more than the extra wave gains (Mooney-Rivlin, the
// damped adjoint's two sets of accumulators, the other T10 cases), and the
// damped Mooney-Rivlin adjoint a whole SIMD's registers.  Laws: 0 SVK,
// 1 Mooney-Rivlin, 2 Neo-Hookean; element 1 is H8, 2 is Q27.
constexpr int waves_per_simd(int op, int elem, int law, bool damped, int mode = 0)
{
    // the step residual stages the adjoint's record length: its LDS budget
    // is two workgroups per compute unit
    // Q27: the LDS of a tile's node records (about 11 nodes per element)
    // allows two or three tiles of one wave per compute unit, so every Q27
    // kernel takes a whole SIMD's registers (its 81 accumulators per node
    // field and the element's 27 record offsets stay in registers)
    if (elem == 2) return 1;
    if (op == kOpFwd) return (law == 1 || mode == 1) ? 2 : 3;
    if (op == kOpVjp && law == 1 && damped) return 1;
    if (damped || law == 1) return 2;
    if (elem == 1) return 3;
    return (op == kOpJvp && law == 0) ? 3 : 2;
}

// Doubles a node record of an operation holds: X and x, plus w (adjoint) or
// dx (tangent), plus v when damped, plus dv for the damped tangent.  The
// step residual (forward, kModeStep) adds u = v - v_n; the Newton operator
// (tangent, kModeStep) has the tangent's record (dx = h dv).  The mass
// action stages u only.
constexpr int record_fields_len(int op, bool damped, int mode = kModePlain)
{
    return op == kOpMass ? 3
                         : 6 + (op != kOpFwd ? 3 : 0) + (damped ? 3 : 0) + ((damped && op == kOpJvp) ? 3 : 0) +
                               ((op == kOpFwd && mode == kModeStep) ? 3 : 0);
}

// LDS stride of a node record, rounded up to an odd number of doubles: a
// wavefront gathers one component of 64 unrelated nodes, and with a stride
// of 2 x odd dwords the record starts spread over every other bank instead
// of a quarter or an eighth of them.
constexpr int record_len(int op, bool damped, int mode = kModePlain)
{
    return record_fields_len(op, damped, mode) | 1;
}

}  // namespace tlfea

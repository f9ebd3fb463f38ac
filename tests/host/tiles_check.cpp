// Host-side checks of the mesh builder (tiling, LDS record positions, tile
// CSR, shared-node partials), compiled and run by tests/test_host_tiles.py
// on the CPU: no device is touched (build_tiles is host code only).
//
// Input (text, from the test): n_nodes n_blocks flags, then X as 3*n_nodes
// numbers, then per block: elem law damped tile_elems n_elem followed by
// n_elem*nen node ids.  Output: "OK" plus statistics, or "FAIL <reason>".
#include "tlfea_host.cpp"

#include <cstdio>
#include <map>
#include <set>

namespace tlfea {
// The builder's translation unit refers to the kernel launchers; nothing here
// launches anything.
hipError_t launch_halo(hipStream_t, const DevMesh &, double *, double *, const double *) { return hipErrorInvalidValue; }
hipError_t launch_inverted_e0_o0(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int,
                                 unsigned long long *) { return hipErrorInvalidValue; }
hipError_t launch_inverted_e1_o0(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int,
                                 unsigned long long *) { return hipErrorInvalidValue; }
hipError_t launch_inverted_e2_o0(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int,
                                 unsigned long long *) { return hipErrorInvalidValue; }
hipError_t launch_zero_count(hipStream_t, unsigned long long *) { return hipErrorInvalidValue; }
hipError_t scratch_address(double **) { return hipErrorInvalidValue; }
hipError_t launch_mass_e0(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int, int, int)
{ return hipErrorInvalidValue; }
hipError_t launch_mass_e1(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int, int, int)
{ return hipErrorInvalidValue; }
hipError_t launch_mass_e2(int, int, size_t, hipStream_t, const DevMesh &, const CallArgs &, int, int, int)
{ return hipErrorInvalidValue; }
hipError_t launch_mdot(const double *, int64_t, int, const double *, int64_t, double *, hipStream_t)
{ return hipErrorInvalidValue; }
hipError_t launch_maxpy(const double *, int64_t, int, const double *, double *, int64_t, hipStream_t)
{ return hipErrorInvalidValue; }
hipError_t launch_axpby(double, const double *, double, double *, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_cgs(int, const double *, int64_t, int, const double *, double *, int64_t, double *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_sum_partials(const double *, int, double *, double *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_add(const double *, const double *, double *, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_joints(const DevJoints &, const double *, const double *, double, double, double *, int, hipStream_t)
{ return hipErrorInvalidValue; }
hipError_t launch_joint_scatter(const DevJoints &, double *, int, hipStream_t) { return hipErrorInvalidValue; }
#define TLFEA_STUB(e, o, g, md)                                                                                  \
    hipError_t launch_tiles_e##e##_o##o##_g##g##_m##md(int, int, int, int, size_t, hipStream_t, const DevMesh &, \
                                                       const CallArgs &, int, int, int) { return hipErrorInvalidValue; }
TLFEA_STUB(0, 0, 0, 0) TLFEA_STUB(0, 0, 0, 1) TLFEA_STUB(0, 1, 0, 0) TLFEA_STUB(0, 1, 1, 0)
TLFEA_STUB(0, 2, 0, 0) TLFEA_STUB(0, 2, 0, 1)
TLFEA_STUB(1, 0, 0, 0) TLFEA_STUB(1, 0, 0, 1) TLFEA_STUB(1, 1, 0, 0) TLFEA_STUB(1, 1, 1, 0)
TLFEA_STUB(1, 2, 0, 0) TLFEA_STUB(1, 2, 0, 1)
TLFEA_STUB(2, 0, 0, 0) TLFEA_STUB(2, 0, 0, 1) TLFEA_STUB(2, 1, 0, 0) TLFEA_STUB(2, 1, 1, 0)
TLFEA_STUB(2, 2, 0, 0) TLFEA_STUB(2, 2, 0, 1)
#undef TLFEA_STUB
}  // namespace tlfea

#define CHECK(c, ...)                                                                                              \
    do {                                                                                                           \
        if (!(c)) {                                                                                                \
            printf("FAIL ");                                                                                       \
            printf(__VA_ARGS__);                                                                                   \
            printf("\n");                                                                                          \
            return 1;                                                                                              \
        }                                                                                                          \
    } while (0)

// Cycles of one 64-lane ds_read_b64 gather under the LDS model the builder
// places records for: 16 lanes per cycle, 16 pairs of 4-byte banks, lanes of
// a group that hit one pair at different addresses serialise.
static int gather_cycles(const int *rec, int n)
{
    int cyc = 0;
    for (int g0 = 0; g0 < n; g0 += 16) {
        std::map<int, std::set<int>> by_pair;
        for (int i = g0; i < std::min(n, g0 + 16); ++i)
            if (rec[i] >= 0) by_pair[rec[i] % 16].insert(rec[i]);
        int mx = 1;
        for (auto &kv : by_pair) mx = std::max(mx, (int)kv.second.size());
        cyc += mx;
    }
    return cyc;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *fin = fopen(argv[1], "r");
    if (!fin) return 2;
    long long n_nodes = 0;
    int n_blocks = 0, flags = 0;
    if (fscanf(fin, "%lld %d %d", &n_nodes, &n_blocks, &flags) != 3) return 2;
    std::vector<double> X(3 * n_nodes);
    for (auto &v : X)
        if (fscanf(fin, "%lf", &v) != 1) return 2;
    std::vector<tlfea_block> blocks(n_blocks);
    std::vector<std::vector<int32_t>> conns(n_blocks);
    std::vector<int> te(n_blocks);
    for (int b = 0; b < n_blocks; ++b) {
        int elem, law, damped, tile;
        long long ne;
        if (fscanf(fin, "%d %d %d %d %lld", &elem, &law, &damped, &tile, &ne) != 5) return 2;
        const int nen = nen_of(elem);
        conns[b].resize(ne * nen);
        for (auto &c : conns[b])
            if (fscanf(fin, "%d", &c) != 1) return 2;
        tlfea_block &B = blocks[b];
        B = tlfea_block{};
        B.elem = elem; B.law = law; B.damped = damped; B.n_elem = ne; B.conn = conns[b].data();
        B.tile_elems = tile;
        te[b] = tile ? tile : default_te(elem);
    }
    fclose(fin);

    HostBuild hb;
    const int64_t lds_dev = 163840;
    if (build_tiles(n_nodes, X.data(), n_blocks, blocks.data(), flags, te, lds_dev, hb) != TLFEA_OK) {
        printf("FAIL build_tiles: %s\n", g_err.c_str());
        return 1;
    }
    int64_t n_elem = 0;
    std::vector<int64_t> uid0(n_blocks + 1, 0);
    for (int b = 0; b < n_blocks; ++b) uid0[b + 1] = uid0[b] + blocks[b].n_elem;
    n_elem = uid0[n_blocks];

    // every element in exactly one tile; uids a permutation
    CHECK((int64_t)hb.elem_uid.size() == n_elem, "elem_uid size %zu != %lld", hb.elem_uid.size(), (long long)n_elem);
    std::vector<int> seen(n_elem, 0);
    for (int32_t u : hb.elem_uid) {
        CHECK(u >= 0 && u < n_elem, "uid %d out of range", u);
        CHECK(seen[u]++ == 0, "element %d in two tiles", u);
    }
    std::vector<int> tile_count(n_nodes, 0);
    long long model_sorted = 0, model_placed = 0;
    for (size_t ti = 0; ti < hb.tiles.size(); ++ti) {
        const TileDesc &t = hb.tiles[ti];
        const int b = t.block, nen = nen_of(blocks[b].elem), T = te[b];
        CHECK(t.n_elem >= 1 && t.n_elem <= T, "tile %zu has %d elements (te %d)", ti, t.n_elem, T);
        CHECK(t.n_node <= stage_per_thread(blocks[b].elem) * T * lanes_per_elem(blocks[b].elem), "tile %zu has %d nodes", ti, t.n_node);
        // sorted unique node ids, positions a permutation
        std::vector<int> pos_seen(t.n_node, 0), local_of_pos(t.n_node, -1);
        for (int l = 0; l < t.n_node; ++l) {
            const int32_t g = hb.lnode_gid[t.node_begin + l];
            CHECK(g >= 0 && g < n_nodes, "tile %zu node id %d", ti, g);
            if (l) CHECK(hb.lnode_gid[t.node_begin + l - 1] < g, "tile %zu node ids not sorted", ti);
            const int p = hb.lnode_pos[t.node_begin + l];
            CHECK(p >= 0 && p < t.n_node && pos_seen[p]++ == 0, "tile %zu position %d repeated or out of range", ti, p);
            local_of_pos[p] = l;
            tile_count[g]++;
        }
        // connectivity: record position of element i's node a holds that node
        std::vector<std::vector<int>> refs(t.n_node);
        for (int i = 0; i < t.n_elem; ++i) {
            const int32_t u = hb.elem_uid[t.elem_begin + i];
            const int bb = (int)(std::upper_bound(uid0.begin(), uid0.end(), (int64_t)u) - uid0.begin()) - 1;
            CHECK(bb == b, "tile %zu holds an element of block %d, not %d", ti, bb, b);
            const int32_t *c = conns[b].data() + (u - uid0[b]) * nen;
            for (int a = 0; a < nen; ++a) {
                const int p = hb.conn_local[t.conn_begin + (size_t)a * T + i];
                CHECK(p < t.n_node, "tile %zu position %d", ti, p);
                const int l = local_of_pos[p];
                CHECK(hb.lnode_gid[t.node_begin + l] == c[a], "tile %zu element %d node %d maps to the wrong record", ti, i, a);
                refs[l].push_back(a * T + i);
            }
        }
        // tile CSR: each node's slot list is exactly its (a, i) references, in order
        for (int l = 0; l < t.n_node; ++l) {
            const int p0 = hb.lnode_ptr[t.ptr_begin + l], p1 = hb.lnode_ptr[t.ptr_begin + l + 1];
            CHECK(p1 - p0 == (int)refs[l].size(), "tile %zu node %d has %d slots, expected %zu", ti, l, p1 - p0, refs[l].size());
            std::sort(refs[l].begin(), refs[l].end());
            for (int k = p0; k < p1; ++k) {
                CHECK((hb.lnode_slot[k] & (kSlotHead - 1)) == refs[l][k - p0], "tile %zu node %d slot list differs", ti, l);
                CHECK(((hb.lnode_slot[k] & kSlotHead) != 0) == (k == p0), "tile %zu node %d group flag at entry %d", ti, l, k - p0);
            }
        }
        // the kernels' chunked reduction of the slot list, replayed: thread j
        // sums entries [j C, j C + C); groups that start in a chunk are
        // finished there or by that chunk's thread from the following
        // chunks' leading parts.  Entry values are the slot ids + 1 (exact
        // sums); every node must come out once with its own sum.
        {
            const int lpe = lanes_per_elem(blocks[b].elem), C = slot_chunk(nen, lpe), nthr = T * lpe;
            const int E = nen * t.n_elem;
            const int base = hb.lnode_ptr[t.ptr_begin];
            CHECK(E <= C * nthr, "tile %zu: %d slot entries over %d threads of %d", ti, E, nthr, C);
            CHECK(hb.lnode_ptr[t.ptr_begin + t.n_node] - base == E, "tile %zu: list length", ti);
            std::vector<int> cn(nthr, -1);
            for (int l = 0; l < t.n_node; ++l) {
                const int q0 = hb.lnode_ptr[t.ptr_begin + l] - base, q1 = hb.lnode_ptr[t.ptr_begin + l + 1] - base;
                for (int j = (q0 + C - 1) / C; j * C < q1; ++j) {
                    CHECK(j < nthr && cn[j] < 0, "tile %zu chunk %d start claimed twice", ti, j);
                    cn[j] = l;
                }
            }
            auto val = [&](int e) { return (double)(hb.lnode_slot[base + e] & (kSlotHead - 1)) + 1.0; };
            auto head = [&](int e) { return (hb.lnode_slot[base + e] & kSlotHead) != 0; };
            std::vector<double> got(t.n_node, 0.0), want(t.n_node, 0.0), leadv(nthr, 0.0);
            std::vector<int> writes(t.n_node, 0);
            for (int e = 0; e < E; ++e) {
                int l = 0;
                while (l + 1 < t.n_node && hb.lnode_ptr[t.ptr_begin + l + 1] - base <= e) ++l;
                want[l] += val(e);
            }
            std::vector<int> owner_of(nthr, -1);
            std::vector<double> own(nthr, 0.0);
            for (int j = 0; j < nthr; ++j) {
                const int e0 = j * C, ne = std::min(C, E - e0);
                if (ne <= 0) continue;
                CHECK(cn[j] >= 0, "tile %zu chunk %d has no node", ti, j);
                const int l = cn[j];
                const int next = e0 + C < E ? cn[j + 1] : -1;
                const bool lead = !head(e0);
                int cur = l;
                double run = 0.0;
                bool inlead = lead;
                for (int u = 0; u < ne; ++u) {
                    if (u > 0 && head(e0 + u)) {
                        if (inlead) { leadv[j] = run; inlead = false; }
                        else { CHECK(cur < t.n_node, "tile %zu node index", ti); got[cur] += run; writes[cur]++; }
                        ++cur;
                        run = 0.0;
                    }
                    run += val(e0 + u);
                }
                if (inlead) leadv[j] = run;
                else if (next == cur) { owner_of[j] = cur; own[j] = run; }
                else { got[cur] += run; writes[cur]++; }
            }
            for (int j = 0; j < nthr; ++j) {
                if (owner_of[j] < 0) continue;
                double v = own[j];
                for (int k = 1; j + k < nthr && (j + k) * C < E && cn[j + k] == owner_of[j]; ++k) v += leadv[j + k];
                got[owner_of[j]] += v;
                writes[owner_of[j]]++;
            }
            for (int l = 0; l < t.n_node; ++l)
                CHECK(writes[l] == 1 && got[l] == want[l], "tile %zu node %d: written %d times, sum %g (expected %g)", ti, l,
                      writes[l], got[l], want[l]);
        }
        // gather model: the placed positions against the sorted order
        const int nq = nq_of(blocks[b].elem);
        for (int w0 = 0; w0 < t.n_elem; w0 += 64) {
            const int nl = std::min(64, t.n_elem - w0);
            for (int a = 0; a < nen; ++a) {
                int reads = 0;
                for (int q = 0; q < nq; ++q) {
                    bool nz = false;
                    for (int k = 0; k < 3; ++k) nz |= grad_of(blocks[b].elem, q, a, k) != 0.0;
                    reads += nz;
                }
                int placed[64], sorted_[64];
                for (int i = 0; i < nl; ++i) {
                    const int p = hb.conn_local[t.conn_begin + (size_t)a * T + w0 + i];
                    placed[i] = p;
                    sorted_[i] = local_of_pos[p];
                }
                model_placed += (long long)reads * gather_cycles(placed, nl);
                model_sorted += (long long)reads * gather_cycles(sorted_, nl);
            }
        }
    }
    // shared nodes: partial slots, one per holding tile, in tile order
    std::vector<int> part_used(hb.n_part, 0);
    std::vector<int> last_tile(n_nodes, -1);
    size_t h_index = 0;
    for (int64_t g = 0; g < n_nodes; ++g) {
        if (tile_count[g] == 1) continue;
        CHECK(h_index < hb.halo_gid.size() && hb.halo_gid[h_index] == g, "node %lld missing from the shared list", (long long)g);
        CHECK(hb.halo_ptr[h_index + 1] - hb.halo_ptr[h_index] == tile_count[g], "node %lld: %d partial slots for %d tiles",
              (long long)g, hb.halo_ptr[h_index + 1] - hb.halo_ptr[h_index], tile_count[g]);
        ++h_index;
    }
    CHECK(h_index == hb.halo_gid.size(), "extra shared nodes");
    std::vector<int> next_expected(hb.halo_gid.size());
    std::map<int32_t, size_t> h_of;
    for (size_t h = 0; h < hb.halo_gid.size(); ++h) {
        h_of[hb.halo_gid[h]] = h;
        next_expected[h] = hb.halo_ptr[h];
    }
    for (size_t ti = 0; ti < hb.tiles.size(); ++ti) {
        const TileDesc &t = hb.tiles[ti];
        for (int l = 0; l < t.n_node; ++l) {
            const int32_t g = hb.lnode_gid[t.node_begin + l];
            const int32_t d = hb.lnode_dst[t.node_begin + l];
            if (tile_count[g] == 1) {
                CHECK(d == g, "owned node %d has destination %d", g, d);
                continue;
            }
            CHECK(d < 0, "shared node %d written directly", g);
            const int p = -1 - d;
            const size_t h = h_of[g];
            CHECK(p == next_expected[h], "shared node %d: partial slot %d out of tile order (expected %d)", g, p,
                  next_expected[h]);
            next_expected[h]++;
            part_used[p]++;
        }
    }
    for (int64_t p = 0; p < hb.n_part; ++p) CHECK(part_used[p] == 1, "partial slot %lld used %d times", (long long)p, part_used[p]);
    printf("OK tiles %zu shared %zu partials %lld gather_cycles_sorted %lld gather_cycles_placed %lld\n",
           hb.tiles.size(), hb.halo_gid.size(), (long long)hb.n_part, model_sorted, model_placed);
    return 0;
}

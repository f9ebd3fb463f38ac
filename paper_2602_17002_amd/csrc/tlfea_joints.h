// Device layout of a joint set (tlfea_create_joints), shared by the host
// builder and the joint kernels.
#pragma once
#include <stdint.h>

namespace tlfea {

struct DevJoints {
    int64_t n_joints, n_nodes, n_touched;
    int nmax;                 // node slots per point (the largest element's node count)
    const int32_t *ids;       // [5][nmax][n_joints] node of each slot of each point's hosting element
    const double *sv;         // [5][nmax][n_joints] s_i(xi) of the slot (0 for unused slots)
    const double *fw;         // [4][n_joints]: f_1, f_2 (a_0.b_10, a_0.b_20), DP1 row weights w_4, w_5
    double *z;                // [n_joints][5][3] the vector each point receives (scratch;
                              // joint-major, so an entry's three components share a line)
    double *qn;               // [n_nodes][3] node-major copy of the positions of a call
                              // (scratch: a gathered node's three coordinates share a line)
    const int32_t *tnode;     // [n_touched] nodes that receive joint forces
    const int64_t *tptr;      // [n_touched + 1] entry ranges
    const int64_t *tent;      // [entries] the entry's row of z: 5 j + p (joint j, point p)
    const double *tval;       // [entries] s_i(xi) of the entry
};

}  // namespace tlfea

// hl_mesh.h -- host-side mesh services (hl_mesh.hip): conformity check and
// internal numbering of uploaded meshes.
#pragma once

#include <stdint.h>

#include <vector>

#include "hyperlag.h"

namespace hl {

// Conformity of the cells [c0, c1) over the nodes [n0, n1) of a simplicial
// mesh (x: [nodes][d] positions, cells: [cells][d+1] global node ids, every
// cell already checked positively oriented; Section 3.1, "Mesh and
// notation": the cells tile the domain and meet face to face).  Returns
// HL_E_NONCONFORMING if a face belongs to more than two cells, if two cells
// sharing a face lie on the same side of it, if (3D) a boundary edge lies on
// an odd number of boundary faces, or if a node lies on a boundary face
// (2D: edge) it is not a vertex of -- a hanging node.
hl_status check_conforming(int d, const double *x, const int32_t *cells, int64_t n0, int64_t n1, int64_t c0,
                           int64_t c1);

// Internal numbering for coalesced access: within every mesh of the batch
// (node_off / cell_off delimit them), cells sorted by the Hilbert index of
// their centroids (ties in the caller's order) and nodes in the order those
// cells first use them (unused nodes last).  cell_i2u[i] / node_i2u[i]: the
// caller's id of internal cell / node i.
void spatial_numbering(int d, const double *x, const int32_t *cells, const std::vector<int64_t> &node_off,
                       const std::vector<int64_t> &cell_off, std::vector<int32_t> &cell_i2u,
                       std::vector<int32_t> &node_i2u);

// Hilbert index of X (n = 2 or 3 coordinates of `bits` bits each; X is
// overwritten).
uint64_t hilbert_key(uint32_t *X, int bits, int n);

}  // namespace hl

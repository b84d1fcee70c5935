// Low-rank block jobs shared by the ACA and the recompression kernels.
#pragma once
#include "common.hpp"

namespace cbie {

// Largest rank an admissible block may reach in the ACA (columns of its
// workspace); blocks that hit it are reported as not converged.
constexpr int kAcaMaxRank = 512;
// most explicit block copies compressed per round (N-Mueller), complex128
// entries (32 GiB)
constexpr int64_t kAcaDense = int64_t(1) << 31;

struct AcaJob {
    int row_node0, row_nodes;    // tree-order node range of the rows
    int col_node0, col_nodes;
    int obj;
    int upn;                     // unknowns per node
    int cap;                     // workspace columns
    int64_t u_off, v_off;        // workspace offsets (elements)
    int64_t used_off;            // row-flag offset (bytes)
    int64_t a_off;               // explicit copy of the block (N-Mueller), elements; -1: entries on the fly
    int64_t phi_off;             // N-Mueller on the fly: column-node scratch in the workspace (elements)
};

}  // namespace cbie

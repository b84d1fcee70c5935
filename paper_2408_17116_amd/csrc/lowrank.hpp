// Low-rank block jobs shared by the ACA and the recompression kernels.
#pragma once
#include "common.hpp"

namespace cbie {

// Largest rank an admissible block may reach in the ACA (columns of its
// workspace); blocks that hit it are reported as not converged.
constexpr int kAcaMaxRank = 512;

struct AcaJob {
    int row_node0, row_nodes;    // tree-order node range of the rows
    int col_node0, col_nodes;
    int obj;
    int cap;                     // workspace columns
    int64_t u_off, v_off;        // workspace offsets (elements)
    int64_t used_off;            // row-flag offset (bytes)
};

}  // namespace cbie

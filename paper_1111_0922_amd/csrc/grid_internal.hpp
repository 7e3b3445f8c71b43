// grid_internal.hpp -- host-side grid state shared by the C ABI units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/lbm355.h"
#include "kernels.hpp"

struct lbm_grid {
    lbm_grid_desc d;
    int64_t n_cells = 0;
    int64_t n_nodes = 0; // fluid nodes (direct: cells between the walls)
    int64_t n_ghost = 0;
    int idx_phase = 0;   // indirect: 1 after the cellmap pass, 2 after the fill pass
    // bound state
    int scheme = -1;
    void *pdf[2] = {nullptr, nullptr};
    int cur = 0;         // pdf[cur] holds the state of TS / OS
    const int32_t *idx = nullptr;
    const int32_t *aux = nullptr;
    double *scratch = nullptr;
    int64_t pitch = 0;
    int64_t t = 0;
    int remap = 0;
    int64_t pitch_pad = 0; // extra SoA elements between direction arrays
    int64_t wg_lds = -1;   // dynamic LDS reserved per update workgroup (-1: per-precision default)
    int row_stage = 1;     // allow the row-staged direct SoA kernels
    int pair = -1;         // two nodes per lane on direct SoA grids: 1 on, 0 off, -1 default
    int band = -1;         // XCD band height (blocks) of the direct-grid block order, 0 = off, -1 = default
    const uint32_t *order = nullptr; // indirect grids: caller's block-order table (lbm_set_block_order)
    int64_t order_n = 0;
    bool order_built = false;             // lbm_build_idx wrote the XCD slab order after the IDX rows
    const uint32_t *slab_table = nullptr; // that table in the bound IDX buffer
    int slab = -1;                        // LBM_OPT_SLAB_ORDER: 1 on, 0 off, -1 default (SoA on)
    bool rank_built = false;              // lbm_build_idx wrote cell_of and the rank words after the block order
    const uint32_t *cell_of = nullptr;    // those arrays in the bound IDX buffer
    const uint2 *rank_words = nullptr;
    const uint2 *ghost_words = nullptr;   // with et_ghosts, after the rank words
    int rank = -1;                        // LBM_OPT_RANK_LOOKUP: 1 on, 0 off, -1 default
    int64_t soa_block = -1;               // LBM_OPT_SOA_BLOCK: nodes per block of an indirect SoA lattice (0 plain, -1 default)
    // open-boundary classes 1..4 (indirect grids): kind, density, velocity
    int bc_kind[4] = {0, 0, 0, 0};
    double bc_rho[4] = {1.0, 1.0, 1.0, 1.0};
    double bc_u[4][3] = {};
};

// true when some class is not a resting wall
inline bool has_open_boundaries(const lbm_grid *g)
{
    for (int c = 0; c < 4; ++c)
        if (g->bc_kind[c] != LBM_BC_WALL) return true;
    return false;
}

namespace lbm_host {

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_check(hipError_t e, const char *where);
lbm::KArgs base_args(const lbm_grid *g);
uint32_t update_blocks(const lbm_grid *g, const lbm::KArgs &a);
void set_block_order(const lbm_grid *g, lbm::KArgs &a, int kind);
uint32_t node_blocks(const lbm_grid *g);
int kernel_layout(const lbm_grid *g);
int64_t idx_pitch_of(const lbm_grid *g);
const lbm::PrecTable &table(int precision);
int state_rmap(const lbm_grid *g);

} // namespace lbm_host

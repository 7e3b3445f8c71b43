// common.hpp -- declarations shared by the host API and common.hip.
#pragma once

#include "kernels.hpp"

namespace lbm {

constexpr int IDX_PER_THREAD = 4;
constexpr int IDX_CELLS = BLOCK * IDX_PER_THREAD;

struct BuildArgs {
    const uint8_t *mask;  // 1 = solid
    int32_t *cellmap;
    int32_t *idx;         // [18][idx_pitch]
    int32_t *et;          // [7][idx_pitch] or null
    int32_t *counts;      // [2][n_blocks] per-chunk fluid and ghost counts
    int64_t *offsets;     // [2][n_blocks] exclusive offsets, then the two totals
    int32_t nx, ny, nz;
    FastDiv dvx, dvy;
    uint32_t n_cells;
    // traversal order of the fluid numbering: bricks bx*by*bz in lexicographic
    // brick order, cells of a brick lexicographically; v runs over the padded
    // brick grid (n_virtual = nbx*nby*nbz*bx*by*bz), cells outside the box skipped
    int32_t bx, by, bz, nbx, nby;
    uint32_t bv;          // bx * by * bz
    uint32_t n_virtual;
    FastDiv dv_bv, dv_bx, dv_by, dv_nbx, dv_nby;
    uint32_t n_blocks;    // ceil(n_virtual / IDX_CELLS)
    int64_t idx_pitch;
    int64_t n_fluid;
    int32_t et_on;
    // XCD slab order of the node blocks (phase 2, when both are set): slab key of
    // each block's first node, then the block order built from the keys
    uint32_t *order_key;  // [n_tiles] scratch
    uint32_t *order;      // [n_tiles] after the 18 IDX rows
    uint32_t n_tiles;     // ceil(n_fluid / BLOCK)
    // rank lookup (lexicographic numbering only, phase 2, when both are set):
    // cell of every node, and per 32 cells the fluid bits and the fluid count before
    uint32_t *cell_of;    // [idx_pitch]
    uint2 *rank_words;    // [n_words]
    uint2 *ghost_words;   // [n_words] with et_on: per 32 cells the ghost bits and the ghost count before, or null
    uint32_t n_words;     // ceil(n_cells / 32)
};

void launch_idx_phase1(const BuildArgs &b, hipStream_t s);
void launch_idx_phase2(const BuildArgs &b, hipStream_t s);
void launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);

} // namespace lbm

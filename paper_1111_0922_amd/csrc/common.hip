// common.hip -- precision-independent kernels: final moment reduction, the
// STREAM-style copy used for bandwidth calibration, and the index-array
// build of indirect addressing.
#include "common.hpp"

namespace lbm {

// ------------------------------------------------------------------ final reduction
__global__ void __launch_bounds__(BLOCK) k_reduce_final(const double *partials, uint32_t n_blocks, double *out)
{
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < n_blocks; b += BLOCK) {
#pragma unroll
        for (int k = 0; k < 4; ++k) m[k] += partials[4 * (int64_t)b + k];
    }
    block_sum4(m, out);
}

void launch_reduce_final(const double *partials, uint32_t n_blocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, s, partials, n_blocks, out);
}

// ------------------------------------------------------------------ copy
// Each thread moves COPY_UNROLL 16-byte words spaced one block apart, so a
// wavefront's accesses stay contiguous.  One word per thread measured fastest
// on MI355X (6.2 TB/s for 4 GiB; 4 words 5.6 TB/s, 8 words 4.2 TB/s).
constexpr int COPY_UNROLL = 1;

__global__ void __launch_bounds__(BLOCK) k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * BLOCK * COPY_UNROLL + threadIdx.x;
    uint4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const int64_t k = base + (int64_t)u * BLOCK;
        if (k < n16) v[u] = src[k];
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const int64_t k = base + (int64_t)u * BLOCK;
        if (k < n16) dst[k] = v[u];
    }
}

void launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s)
{
    const int64_t n16 = bytes / 16;
    const int64_t blocks = (n16 + BLOCK * COPY_UNROLL - 1) / (BLOCK * COPY_UNROLL);
    if (blocks > 0)
        hipLaunchKernelGGL(k_stream_copy, dim3((uint32_t)blocks), dim3(BLOCK), 0, s, static_cast<const uint4 *>(src),
                           static_cast<uint4 *>(dst), n16);
}

// ------------------------------------------------------------------ index build
// Cells are visited in the numbering's traversal order v (bricks in
// lexicographic brick order, cells of a brick lexicographically; one brick
// spanning the box is the plain lexicographic order), in chunks of IDX_CELLS
// (IDX_PER_THREAD consecutive v per thread).  A fluid cell's id is (chunk
// offset) + (exclusive prefix over the chunk's threads) + (position inside
// the thread's run).

// cell of traversal index v; false for a padding position outside the box
__device__ __forceinline__ bool traversal_cell(const BuildArgs &b, uint32_t v, uint32_t &c)
{
    if (v >= b.n_virtual) return false;
    const uint32_t brick = fdiv(v, b.dv_bv);
    const uint32_t local = v - brick * b.bv;
    const uint32_t q = fdiv(local, b.dv_bx);
    const uint32_t lx = local - q * (uint32_t)b.bx;
    const uint32_t lz = fdiv(q, b.dv_by);
    const uint32_t ly = q - lz * (uint32_t)b.by;
    const uint32_t q2 = fdiv(brick, b.dv_nbx);
    const uint32_t Bx = brick - q2 * (uint32_t)b.nbx;
    const uint32_t Bz = fdiv(q2, b.dv_nby);
    const uint32_t By = q2 - Bz * (uint32_t)b.nby;
    const uint32_t x = Bx * b.bx + lx, y = By * b.by + ly, z = Bz * b.bz + lz;
    if (x >= (uint32_t)b.nx || y >= (uint32_t)b.ny || z >= (uint32_t)b.nz) return false;
    c = x + (uint32_t)b.nx * (y + (uint32_t)b.ny * z);
    return true;
}

__device__ __forceinline__ void cell_xyz(const BuildArgs &b, uint32_t c, int &x, int &y, int &z)
{
    const uint32_t q = fdiv(c, b.dvx);
    x = (int)(c - q * (uint32_t)b.nx);
    const uint32_t r = fdiv(q, b.dvy);
    y = (int)(q - r * (uint32_t)b.ny);
    z = (int)r;
}

__device__ __forceinline__ uint32_t wrap_cell(const BuildArgs &b, int x, int y, int z)
{
    x = x < 0 ? x + b.nx : (x >= b.nx ? x - b.nx : x);
    y = y < 0 ? y + b.ny : (y >= b.ny ? y - b.ny : y);
    z = z < 0 ? z + b.nz : (z >= b.nz ? z - b.nz : z);
    return (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
}

// A solid cell holds esoteric-twist storage when some fluid cell reads it:
// s = x + o for fluid x and o one of the six non-zero offsets o_i.
__device__ __forceinline__ bool needs_ghost(const BuildArgs &b, uint32_t c)
{
    int x, y, z;
    cell_xyz(b, c, x, y, z);
    constexpr int off[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (!b.mask[wrap_cell(b, x - off[k][0], y - off[k][1], z - off[k][2])]) return true;
    return false;
}

__device__ __forceinline__ void cell_flags(const BuildArgs &b, uint32_t v, int &fluid, int &ghost, uint32_t &c)
{
    fluid = 0;
    ghost = 0;
    if (!traversal_cell(b, v, c)) return;
    if (!b.mask[c])
        fluid = 1;
    else if (b.et_on)
        ghost = needs_ghost(b, c) ? 1 : 0;
}

// exclusive prefix over the block of two counters; returns block totals
__device__ __forceinline__ void block_excl_scan2(int &a, int &g, int &tot_a, int &tot_g)
{
    __shared__ int sa[BLOCK], sg[BLOCK];
    const int t = threadIdx.x;
    sa[t] = a;
    sg[t] = g;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
        int va = 0, vg = 0;
        if (t >= off) {
            va = sa[t - off];
            vg = sg[t - off];
        }
        __syncthreads();
        sa[t] += va;
        sg[t] += vg;
        __syncthreads();
    }
    tot_a = sa[BLOCK - 1];
    tot_g = sg[BLOCK - 1];
    a = sa[t] - a;
    g = sg[t] - g;
    __syncthreads();
}

__global__ void __launch_bounds__(BLOCK) k_idx_count(BuildArgs b)
{
    int nf = 0, ng = 0;
    const uint32_t c0 = blockIdx.x * IDX_CELLS + threadIdx.x * IDX_PER_THREAD;
#pragma unroll
    for (int u = 0; u < IDX_PER_THREAD; ++u) {
        int f, g;
        uint32_t c;
        cell_flags(b, c0 + u, f, g, c);
        nf += f;
        ng += g;
    }
    int tf, tg;
    block_excl_scan2(nf, ng, tf, tg);
    if (threadIdx.x == 0) {
        b.counts[blockIdx.x] = tf;
        b.counts[b.n_blocks + blockIdx.x] = tg;
    }
}

// One block of SCAN_THREADS: exclusive scan of the per-block counts into
// 64-bit offsets, totals in offsets[2 * n_blocks], offsets[2 * n_blocks + 1].
constexpr int SCAN_THREADS = 1024;

__global__ void __launch_bounds__(SCAN_THREADS) k_idx_scan(BuildArgs b)
{
    __shared__ int64_t sf[SCAN_THREADS], sg[SCAN_THREADS];
    const uint32_t t = threadIdx.x;
    const uint32_t chunk = (b.n_blocks + SCAN_THREADS - 1) / SCAN_THREADS;
    const uint32_t lo = t * chunk, hi = min(lo + chunk, b.n_blocks);
    int64_t f = 0, g = 0;
    for (uint32_t k = lo; k < hi; ++k) {
        f += b.counts[k];
        g += b.counts[b.n_blocks + k];
    }
    sf[t] = f;
    sg[t] = g;
    __syncthreads();
    for (uint32_t off = 1; off < SCAN_THREADS; off <<= 1) {
        int64_t vf = 0, vg = 0;
        if (t >= off) {
            vf = sf[t - off];
            vg = sg[t - off];
        }
        __syncthreads();
        sf[t] += vf;
        sg[t] += vg;
        __syncthreads();
    }
    int64_t of = sf[t] - f, og = sg[t] - g;
    for (uint32_t k = lo; k < hi; ++k) {
        b.offsets[k] = of;
        b.offsets[b.n_blocks + k] = og;
        of += b.counts[k];
        og += b.counts[b.n_blocks + k];
    }
    if (t == SCAN_THREADS - 1) {
        b.offsets[2 * (int64_t)b.n_blocks] = sf[t];
        b.offsets[2 * (int64_t)b.n_blocks + 1] = sg[t];
    }
}

__global__ void __launch_bounds__(BLOCK) k_idx_cellmap(BuildArgs b)
{
    int fl[IDX_PER_THREAD], gh[IDX_PER_THREAD];
    uint32_t cell[IDX_PER_THREAD];
    int nf = 0, ng = 0;
    const uint32_t c0 = blockIdx.x * IDX_CELLS + threadIdx.x * IDX_PER_THREAD;
#pragma unroll
    for (int u = 0; u < IDX_PER_THREAD; ++u) {
        cell_flags(b, c0 + u, fl[u], gh[u], cell[u]);
        nf += fl[u];
        ng += gh[u];
    }
    int tf, tg;
    block_excl_scan2(nf, ng, tf, tg);
    int64_t idf = b.offsets[blockIdx.x] + nf;
    int64_t idg = b.offsets[b.n_blocks + blockIdx.x] + ng;
#pragma unroll
    for (int u = 0; u < IDX_PER_THREAD; ++u) {
        uint32_t c;
        if (!traversal_cell(b, c0 + u, c)) continue;
        int32_t v = -1;
        if (fl[u])
            v = (int32_t)idf++;
        else if (gh[u])
            v = (int32_t)(-2 - idg++);
        b.cellmap[c] = v;
    }
}

// One thread per cell: fluid cells write their IDX column (and ET rows).
__global__ void __launch_bounds__(BLOCK) k_idx_fill(BuildArgs b)
{
    const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= b.n_cells) return;
    const int32_t n = b.cellmap[c];
    if (n < 0) return;
    int x, y, z;
    cell_xyz(b, c, x, y, z);
    if (b.cell_of) b.cell_of[n] = c;
    // XCD slab of a node block: the y-eighth of its first node's row
    if (b.order_key && (n & (BLOCK - 1)) == 0) b.order_key[n / BLOCK] = (uint32_t)(((int64_t)y * 8) / b.ny);
    uint32_t mask = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const uint32_t cc = wrap_cell(b, x + cx(i), y + cy(i), z + cz(i));
        const int32_t v = b.cellmap[cc];
        // a non-fluid neighbour: -1, or -m for a boundary cell of mask value 2 <= m <= 5
        const int32_t m = b.mask[cc];
        b.idx[(int64_t)(i - 1) * b.idx_pitch + n] = v >= 0 ? v : ((m >= 2 && m <= 5) ? -m : -1);
        if (v < 0) mask |= 1u << (i - 1);
    }
    if (b.et_on) {
        constexpr int off[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int32_t v = b.cellmap[wrap_cell(b, x + off[k][0], y + off[k][1], z + off[k][2])];
            b.et[(int64_t)k * b.idx_pitch + n] = v >= 0 ? v : (int32_t)(b.n_fluid + (-2 - v));
        }
        b.et[6 * b.idx_pitch + n] = (int32_t)mask;
    }
}

// Rank words (one thread per 32 cells): bit k set when cell 32 w + k is
// fluid, and the fluid id of the word's first fluid cell, which in the
// lexicographic numbering is the number of fluid cells before the word (0
// for a word without fluid cells, whose rank is never read); likewise for
// the ghost cells of the esoteric twist.
__global__ void __launch_bounds__(BLOCK) k_rank_words(BuildArgs b)
{
    const uint32_t w = blockIdx.x * BLOCK + threadIdx.x;
    if (w >= b.n_words) return;
    const uint32_t c0 = w * 32u;
    uint32_t bits = 0;
    for (uint32_t k = 0; k < 32u && c0 + k < b.n_cells; ++k)
        if (!b.mask[c0 + k]) bits |= 1u << k;
    const uint32_t rank = bits ? (uint32_t)b.cellmap[c0 + (uint32_t)__ffs(bits) - 1u] : 0u;
    b.rank_words[w] = make_uint2(bits, rank);
    // ghost cells (cellmap -2 - k for ghost k, numbered in the same order)
    if (b.ghost_words) {
        uint32_t gbits = 0;
        for (uint32_t k = 0; k < 32u && c0 + k < b.n_cells; ++k)
            if (b.cellmap[c0 + k] <= -2) gbits |= 1u << k;
        const uint32_t grank = gbits ? (uint32_t)(-2 - b.cellmap[c0 + (uint32_t)__ffs(gbits) - 1u]) : 0u;
        b.ghost_words[w] = make_uint2(gbits, grank);
    }
}

// Block order from the slab keys (one workgroup).  Workgroup b runs on XCD
// b mod 8 (round-robin dispatch), so the r-th block of slab k in node order
// goes to workgroup 8 r + k while every slab still has an r-th block
// (r < m, m the smallest slab's count); the blocks beyond follow in node
// order from workgroup 8 m on.  Each XCD then sweeps its own y-eighth of
// every z-plane, plane after plane, and all XCDs stay in the same planes: the
// rows a block's odd-step gathers and scatters share cache lines with (y +-
// 1 and z +- 1) mostly run on the same XCD, in its L2.  A permutation of
// [0, n_tiles).
constexpr int ORDER_THREADS = 1024;

__device__ __forceinline__ void block_excl_scan_lds(uint32_t (&v)[9], uint32_t (&tot)[9])
{
    __shared__ uint32_t sv[9][ORDER_THREADS];
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 9; ++k) sv[k][t] = v[k];
    __syncthreads();
    for (uint32_t off = 1; off < ORDER_THREADS; off <<= 1) {
        uint32_t a[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) a[k] = t >= off ? sv[k][t - off] : 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 9; ++k) sv[k][t] += a[k];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        tot[k] = sv[k][ORDER_THREADS - 1];
        v[k] = sv[k][t] - v[k];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(ORDER_THREADS) k_order_build(BuildArgs b)
{
    const uint32_t T = b.n_tiles;
    const uint32_t chunk = (T + ORDER_THREADS - 1) / ORDER_THREADS;
    const uint32_t lo = min(threadIdx.x * chunk, T), hi = min(lo + chunk, T);
    uint32_t cnt[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, tot[9];
    for (uint32_t t = lo; t < hi; ++t) ++cnt[min(b.order_key[t], 7u)];
    block_excl_scan_lds(cnt, tot); // cnt: this thread's first rank in each slab
    uint32_t m = tot[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) m = min(m, tot[k]);
    uint32_t r[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) r[k] = cnt[k];
    uint32_t left[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t t = lo; t < hi; ++t) {
        const uint32_t k = min(b.order_key[t], 7u);
        uint32_t rank = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q == (int)k) rank = r[q]++;
        if (rank >= m) ++left[8];
    }
    block_excl_scan_lds(left, tot); // left[8]: this thread's first index among the blocks beyond 8 m
    uint32_t li = left[8];
#pragma unroll
    for (int k = 0; k < 9; ++k) r[k] = cnt[k];
    for (uint32_t t = lo; t < hi; ++t) {
        const uint32_t k = min(b.order_key[t], 7u);
        uint32_t rank = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q == (int)k) rank = r[q]++;
        const uint32_t wg = rank < m ? rank * 8u + k : 8u * m + li++;
        b.order[wg] = t;
    }
}

void launch_idx_phase1(const BuildArgs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_idx_count, dim3(b.n_blocks), dim3(BLOCK), 0, s, b);
    hipLaunchKernelGGL(k_idx_scan, dim3(1), dim3(SCAN_THREADS), 0, s, b);
    hipLaunchKernelGGL(k_idx_cellmap, dim3(b.n_blocks), dim3(BLOCK), 0, s, b);
}

void launch_idx_phase2(const BuildArgs &b, hipStream_t s)
{
    const uint32_t blocks = (b.n_cells + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_idx_fill, dim3(blocks), dim3(BLOCK), 0, s, b);
    if (b.cell_of && b.rank_words && b.n_words > 0)
        hipLaunchKernelGGL(k_rank_words, dim3((b.n_words + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, b);
    if (b.order_key && b.order && b.n_tiles > 0)
        hipLaunchKernelGGL(k_order_build, dim3(1), dim3(ORDER_THREADS), 0, s, b);
}

} // namespace lbm

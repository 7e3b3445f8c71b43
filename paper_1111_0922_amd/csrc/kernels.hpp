// kernels.hpp -- the fused D3Q19 node-update kernels of every propagation
// scheme, written once over (addressing, layout, precision, scheme kernel,
// collider) and instantiated per precision in k_<prec>.hip.
//
// One lane updates one node (two x-neighbours in the pair kernels).  A
// kernel reads the node's 19 PDFs through the scheme's read map, collides
// them in registers and stores them through the scheme's write map.  At a
// non-fluid neighbour the maps bounce back; for the open-boundary classes of
// indirect grids the bounced value passes the class's link rule (bc_arrive).
// The maps (Secs. 2, 3, 6, 7):
//
//   read maps (slot = (direction array j, cell)):
//     LOCAL   (i, x)
//     PULL    (i, x - c_i), or (opp i, x) when x - c_i is solid  [bounce-back]
//     AAODD   (opp i, x - c_i), or (i, x) when x - c_i is solid
//     ET(p)   (ph(i), x + o_i), ph(i) = i at even parity, opp i at odd parity
//   write maps:
//     LOCAL   (i, x)
//     PUSH    (i, x + c_i), or (opp i, x) when x + c_i is solid
//     AAEVEN  (opp i, x)
//     ET(p)   (ph(opp i), x + o_{opp i}), or (ph(i), x + o_{opp i}) when x + c_i is solid
//
//   two-step    collision LOCAL(A) -> LOCAL(B); propagation PULL(B) -> LOCAL(A)   (Sec. 2)
//   one-step    push LOCAL(A) -> PUSH(B); pull PULL(A) -> LOCAL(B); swap A, B     (Sec. 3)
//   AA pattern  even LOCAL(P) -> AAEVEN(P); odd AAODD(P) -> PUSH(P)               (Sec. 6)
//   esoteric twist  ET(t mod 2)(P) -> ET(t mod 2)(P)                              (Sec. 7)
//
// For AA and ET the write set of a node equals its read set, so nodes are
// independent and update in place.  The offsets o_i = max(-c_i, 0) satisfy
// o_{opp i} - o_i = c_i, which makes the esoteric twist's write of f_i* land
// where the neighbour x + c_i reads it after the parity flip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "collide.hpp"
#include "d3q19.hpp"
#include "storage.hpp"

namespace lbm {

constexpr int BLOCK = 256;

// ------------------------------------------------------------------ fast division
// n / d for 0 <= n < 2^31 by multiply-high (round-up method of Granlund and
// Montgomery, PLDI 1994): s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)((((1ull << s) - d) << 32) / d + 1);
    return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t hi = __umulhi(f.m, n);
#else
    const uint32_t hi = (uint32_t)(((uint64_t)f.m * n) >> 32);
#endif
    return (hi + n) >> f.s;
}

// ------------------------------------------------------------------ enums
enum Addr : int { A_DIRECT = 0, A_INDIRECT = 1 };
enum Kind : int { K_TS_COLLIDE = 0, K_TS_STREAM, K_OS_PUSH, K_OS_PULL, K_AA_EVEN, K_AA_ODD, K_ET0, K_ET1, K_NUM };
enum RMap : int { R_LOCAL = 0, R_PULL, R_AAODD, R_ET0, R_ET1, R_NUM };
enum WMap : int { W_LOCAL = 0, W_PUSH, W_AAEVEN, W_ET0, W_ET1 };

__host__ __device__ constexpr int rmap_of(int k)
{
    return k == K_TS_COLLIDE ? R_LOCAL
         : k == K_TS_STREAM  ? R_PULL
         : k == K_OS_PUSH    ? R_LOCAL
         : k == K_OS_PULL    ? R_PULL
         : k == K_AA_EVEN    ? R_LOCAL
         : k == K_AA_ODD     ? R_AAODD
         : k == K_ET0        ? R_ET0
                             : R_ET1;
}
__host__ __device__ constexpr int wmap_of(int k)
{
    return k == K_TS_COLLIDE ? W_LOCAL
         : k == K_TS_STREAM  ? W_LOCAL
         : k == K_OS_PUSH    ? W_PUSH
         : k == K_OS_PULL    ? W_LOCAL
         : k == K_AA_EVEN    ? W_AAEVEN
         : k == K_AA_ODD     ? W_PUSH
         : k == K_ET0        ? W_ET0
                             : W_ET1;
}

// what a node needs besides its own address
enum Need : int { NEED_NONE = 0, NEED_NB = 1, NEED_ET = 2 };
__host__ __device__ constexpr int need_r(int r) { return (r == R_PULL || r == R_AAODD) ? NEED_NB : (r >= R_ET0 ? NEED_ET : 0); }
__host__ __device__ constexpr int need_w(int w) { return w == W_PUSH ? NEED_NB : (w >= W_ET0 ? NEED_ET : 0); }

// ------------------------------------------------------------------ kernel arguments
struct KArgs {
    const void *src;       // lattice read
    void *dst;             // lattice written (== src for AA and ET)
    const int32_t *idx;    // IDX[18][idx_pitch] (indirect)
    const int32_t *et;     // ET table [7][idx_pitch] (indirect ET)
    // Neighbour ids by rank instead of IDX (indirect grids numbered
    // lexicographically, no open boundaries; null otherwise): the node's
    // cell, and per 32 cells of the box (x fastest) the fluid bits and the
    // number of fluid cells before the word (rank_neighbours).
    const uint32_t *cell_of;   // [idx_pitch]
    const uint2 *rank_words;   // [ceil(n_cells / 32)]
    const uint2 *ghost_words;  // esoteric twist: per 32 cells the ghost bits and the ghost count before, or null
    int64_t pitch;         // SoA elements between direction arrays
    uint32_t bsh, bmk;     // blocked SoA (L_BLK, slot_index): blocks of 2^bsh nodes, bmk = 2^bsh - 1
    int64_t idx_pitch;
    int64_t plane;         // nx * ny
    int64_t z0_offset;     // z0 * plane: cell address of node 0 (direct)
    uint32_t n_nodes;
    int32_t nx, ny, nz, z0, wall;
    FastDiv dvx, dvy;
    int32_t remap;         // block order: 0 natural, 1 XCD chunks, 2 XCD bands, 3 table (logical_block)
    const uint32_t *order; // remap 3: node block of each workgroup
    uint32_t band_yb, band_ty, band_z;
    uint32_t lds_bytes;    // dynamic LDS reserved per update workgroup (caps residency)
    int32_t row_staged;    // direct SoA, x-shifted accesses through LDS: 1 nx divides BLOCK, 2 BLOCK divides nx, 3 other nx
    int32_t pair;          // direct SoA, 16-bit storage, nx divides 2 * BLOCK: two nodes per lane
    double omega, gx, gy, gz, sigma;
    double omega_minus;    // TRT odd-moment rate (== omega for BGK)
    CollideParams<double> cpd; // collision factors (set_collision) for FP64
    CollideParams<float> cpf;  // and for FP32 compute
    // Open boundaries of indirect grids (Sec. 6: in-/outlets in both AA
    // parities).  A neighbour with IDX code -1 - c, c = 1..4, is a boundary
    // cell of class c: the population that bounces back there arrives as
    // s_c f + C_c[d] (d its direction), with s_c = -1 (bit c-1 of bc_neg) for
    // pressure classes and +1 for velocity classes.  Code -1 (c = 0) is a
    // plain wall.
    int32_t bc_on;         // some class is not a resting wall
    uint32_t bc_neg;
    double bc_can[4][Q];   // C_c[d] on canonical values (also the FP64 compute form)
    float bc_f[4][Q];      // C_c[d] on the stored form, FP32 compute
    // canonical transfer / reductions
    double *canon;
    const double *canon_in;
    const double *rho_u;
    double *partials;
};

// Collision factors from omega, omega_minus, g and sigma (host side).
inline void set_collision(KArgs &a)
{
    a.cpd = collide_params<double>(a.omega, a.omega_minus, a.gx, a.gy, a.gz, a.sigma);
    a.cpf = collide_params<float>(a.omega, a.omega_minus, a.gx, a.gy, a.gz, a.sigma);
}

template <typename T>
__device__ __forceinline__ const CollideParams<T> &cparams(const KArgs &a)
{
    if constexpr (sizeof(T) == 8)
        return a.cpd;
    else
        return a.cpf;
}

// The constants C_c[d] in the compute type, copied to LDS once per workgroup
// (bc_table_fill).  A link reads its constant there by the lane's class: a
// vector load from the kernel arguments would wait on memory per link, and
// uniform scalar loads of the whole table (76 values) overflow the scalar
// registers into spills on every path.
template <typename T>
__device__ __forceinline__ T (&bc_table())[4][Q]
{
    __shared__ T tab[4][Q];
    return tab;
}
// Every thread of the workgroup calls these (a.bc_on is uniform): the table
// from the canonical constants (FP64 compute) or the stored-form ones.
template <typename T>
__device__ __forceinline__ void bc_table_load(const double (*can)[Q], const float (*f)[Q])
{
    const uint32_t t = threadIdx.x;
    if (t < 4 * Q) bc_table<T>()[t / Q][t % Q] = sizeof(T) == 8 ? (T)can[t / Q][t % Q] : (T)f[t / Q][t % Q];
    __syncthreads();
}
template <typename T>
__device__ __forceinline__ void bc_table_fill(const KArgs &a)
{
    if (a.bc_on) bc_table_load<T>(a.bc_can, a.bc_f);
}

// The population arriving in direction d from a boundary of class c >= 1,
// given the bounced value v (compute type, stored form) ...
template <typename T>
__device__ __forceinline__ T bc_arrive(const KArgs &a, int c, int d, T v)
{
    const T k = bc_table<T>()[c - 1][d];
    return ((a.bc_neg >> (c - 1)) & 1u) ? k - v : v + k;
}
// ... the same on canonical FP64 values, and its inverse (the bounced value
// that makes f arrive).
__device__ __forceinline__ double bc_arrive_canon(const double (*can)[Q], uint32_t neg, int c, int d, double f)
{
    const double k = can[c - 1][d];
    return ((neg >> (c - 1)) & 1u) ? k - f : f + k;
}
__device__ __forceinline__ double bc_arrive_canon(const KArgs &a, int c, int d, double f)
{
    return bc_arrive_canon(a.bc_can, a.bc_neg, c, d, f);
}
__device__ __forceinline__ double bc_depart_canon(const KArgs &a, int c, int d, double f)
{
    const double k = a.bc_can[c - 1][d];
    return ((a.bc_neg >> (c - 1)) & 1u) ? k - f : f - k;
}

// The esoteric twist bounces back on its write side only, from its solid
// bit mask; the class of that neighbour comes from IDX (indirect grids).
template <int W, class N>
__device__ __forceinline__ int et_write_class(const KArgs &a, const N &nd, int i)
{
    if constexpr (W == W_ET0 || W == W_ET1) {
        if (i != 0 && a.bc_on && nd.et_solid(i)) return -a.idx[(int64_t)(i - 1) * a.idx_pitch + nd.a] - 1;
    }
    return 0;
}

// ------------------------------------------------------------------ block order
// Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD
// b mod 8), each XCD with its own L2.  The maps below are bijections on
// [0, gridDim.x) that change only which node block a workgroup updates:
//   remap 1: consecutive logical blocks (neighbouring nodes, which share
//            cache lines of the shifted accesses) run on the same XCD;
//   remap 2: direct grids seen as z-planes of band_yb blocks; the planes are
//            cut into bands of band_ty blocks (rows), band k belongs to XCD
//            k mod 8, and each XCD sweeps its bands along z.  The neighbour
//            rows a node reads from or writes to (y +- 1, z +- 1) then run
//            close in time on the same XCD.  Requires band_yb % (8 band_ty)
//            == 0 and gridDim.x = band_z * band_yb.
//   remap 3: a caller's table (indirect grids): workgroup b updates node
//            block order[b].
__device__ __forceinline__ uint32_t logical_block(const KArgs &a)
{
    uint32_t b = blockIdx.x;
    if (a.remap == 3) {
        b = a.order[b];
    } else if (a.remap == 1) {
        const uint32_t G = gridDim.x, x = b & 7u, s = b >> 3, q = G >> 3, r = G & 7u;
        b = (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
    } else if (a.remap == 2) {
        const uint32_t x = b & 7u, s = b >> 3;
        const uint32_t per_band = a.band_z * a.band_ty;
        const uint32_t k = s / per_band, r = s - k * per_band;
        const uint32_t z = r / a.band_ty, yb = (x + 8u * k) * a.band_ty + (r - z * a.band_ty);
        b = z * a.band_yb + yb;
    }
    return b;
}

// ------------------------------------------------------------------ nodes
template <int ADDR, int NEED>
struct Node;

// Direct addressing (Sec. 1): index arithmetic on the full box, x and y
// periodic, z periodic or bounded by solid wall planes z = 0 and z = nz-1.
template <int NEED>
struct Node<A_DIRECT, NEED> {
    int64_t a;
    int64_t dxp, dxm, dyp, dym, dzp, dzm;
    bool szp, szm;

    __device__ __forceinline__ void init(const KArgs &k, uint32_t n)
    {
        const uint32_t q = fdiv(n, k.dvx);
        const int x = (int)(n - q * (uint32_t)k.nx);
        const uint32_t r = fdiv(q, k.dvy);
        const int y = (int)(q - r * (uint32_t)k.ny);
        const int z = (int)r + k.z0;
        a = (int64_t)n + k.z0_offset;
        dxp = (x == k.nx - 1) ? (int64_t)(1 - k.nx) : 1;
        dxm = (x == 0) ? (int64_t)(k.nx - 1) : -1;
        dyp = (y == k.ny - 1) ? -(int64_t)(k.ny - 1) * k.nx : (int64_t)k.nx;
        dym = (y == 0) ? (int64_t)(k.ny - 1) * k.nx : -(int64_t)k.nx;
        dzp = (z == k.nz - 1) ? -(int64_t)(k.nz - 1) * k.plane : k.plane;
        dzm = (z == 0) ? (int64_t)(k.nz - 1) * k.plane : -k.plane;
        szp = k.wall && (z + 1 == k.nz - 1);
        szm = k.wall && (z - 1 == 0);
    }
    __device__ __forceinline__ int64_t shift(int sx, int sy, int sz) const
    {
        return a + (sx > 0 ? dxp : (sx < 0 ? dxm : 0)) + (sy > 0 ? dyp : (sy < 0 ? dym : 0)) +
               (sz > 0 ? dzp : (sz < 0 ? dzm : 0));
    }
    // cell x + c_i and whether it is solid
    __device__ __forceinline__ int64_t nb(int i) const { return shift(cx(i), cy(i), cz(i)); }
    __device__ __forceinline__ bool solid(int i) const { return (cz(i) > 0 && szp) || (cz(i) < 0 && szm); }
    // storage cell x + (ox, oy, oz), ox, oy, oz in {0, 1}
    __device__ __forceinline__ int64_t at(int sx, int sy, int sz) const { return shift(sx, sy, sz); }
    __device__ __forceinline__ bool et_solid(int i) const { return solid(i); }
    __device__ __forceinline__ int bc_class(int) const { return 0; }
    __device__ __forceinline__ void refresh() {}
    __device__ __forceinline__ void pin_nb(int) {}
    __device__ __forceinline__ void pin_et(int) {}
};

// Cells x + c_i (i = 1..18, periodic wrap) of node n, from the node's cell.
__device__ __forceinline__ void neighbour_cells(const KArgs &k, uint32_t n, uint32_t (&cc)[18])
{
    const uint32_t c = k.cell_of[n];
    const uint32_t nx = (uint32_t)k.nx, ny = (uint32_t)k.ny, nz = (uint32_t)k.nz, pl = (uint32_t)k.plane;
    const uint32_t q = fdiv(c, k.dvx);
    const uint32_t x = c - q * nx;
    const uint32_t z = fdiv(q, k.dvy);
    const uint32_t y = q - z * ny;
    const uint32_t px[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0 : x + 1};
    const uint32_t py[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y + 1 == ny ? 0 : y + 1) * nx};
    const uint32_t pz[3] = {(z == 0 ? nz - 1 : z - 1) * pl, z * pl, (z + 1 == nz ? 0 : z + 1) * pl};
#pragma unroll
    for (int j = 0; j < 18; ++j) cc[j] = px[cx(j + 1) + 1] + py[cy(j + 1) + 1] + pz[cz(j + 1) + 1];
}

// The 18 neighbour ids of node n from the rank words, where the fluid id of a
// cell is the number of fluid cells before it in x-fastest order: for cell
// c = 32 w + b, fluid when bit b of word w is set, with id rank(w) +
// popcount(bits(w) below b).  The result equals IDX with every non-fluid
// neighbour as -1.  Per node this reads 4 bytes of cell_of; the words (8
// bytes per 32 cells, about 33 MB for a 512^3 box) are shared by the 18
// neighbours of ~13 nodes each and mostly come from the cache, where IDX
// streams 72 bytes per node from memory.
__device__ __forceinline__ void rank_neighbours(const KArgs &k, uint32_t n, int32_t (&m)[18])
{
    uint32_t cc[18];
    neighbour_cells(k, n, cc);
    uint2 w[18];
#pragma unroll
    for (int j = 0; j < 18; ++j) w[j] = k.rank_words[cc[j] >> 5];
    // All 18 words in flight before the first is used: without this opaque use
    // the compiler loads a word's rank only under the lane's fluid bit and waits
    // for each load in turn (36 round trips instead of one).
#pragma unroll
    for (int j = 0; j < 18; ++j) asm volatile("" : "+v"(w[j].x), "+v"(w[j].y));
#pragma unroll
    for (int j = 0; j < 18; ++j) {
        const uint32_t b = cc[j] & 31u;
        const int32_t id = (int32_t)(w[j].y + (uint32_t)__popc(w[j].x & ((1u << b) - 1u)));
        m[j] = ((w[j].x >> b) & 1u) ? id : -1;
    }
}

// The esoteric twist's storage addresses and solid mask of node n from the
// rank words (the ET table's contents): e[k] is the storage entry of cell
// x + o_k for the six offsets of et_cell (the fluid id, or N_f + the ghost
// number of a solid storage cell, from the ghost words), and bit i - 1 of
// mask is set when x + c_i is not fluid.  Reads 4 bytes per node where the
// table reads 28.
__device__ __forceinline__ void rank_et(const KArgs &k, uint32_t n, int32_t (&e)[6], uint32_t &mask)
{
    // directions of the six storage cells x + ex, ey, ez, ex+ey, ex+ez, ey+ez
    constexpr int dir[6] = {1, 3, 5, 7, 11, 15};
    uint32_t cc[18];
    neighbour_cells(k, n, cc);
    uint2 w[18], gw[6];
#pragma unroll
    for (int j = 0; j < 18; ++j) w[j] = k.rank_words[cc[j] >> 5];
#pragma unroll
    for (int t = 0; t < 6; ++t) gw[t] = k.ghost_words[cc[dir[t] - 1] >> 5];
    // every word in flight before the first is used (as in rank_neighbours)
#pragma unroll
    for (int j = 0; j < 18; ++j) asm volatile("" : "+v"(w[j].x), "+v"(w[j].y));
#pragma unroll
    for (int t = 0; t < 6; ++t) asm volatile("" : "+v"(gw[t].x), "+v"(gw[t].y));
    mask = 0;
#pragma unroll
    for (int j = 0; j < 18; ++j) mask |= (((w[j].x >> (cc[j] & 31u)) & 1u) ^ 1u) << j;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int j = dir[t] - 1;
        const uint32_t b = cc[j] & 31u, below = (1u << b) - 1u;
        const uint32_t fid = w[j].y + (uint32_t)__popc(w[j].x & below);
        const uint32_t gid = k.n_nodes + gw[t].y + (uint32_t)__popc(gw[t].x & below);
        e[t] = (int32_t)(((w[j].x >> b) & 1u) ? fid : gid);
    }
}

// Indirect addressing (Sec. 1): node ids of fluid nodes; neighbours from
// IDX (-1 = wall, -1 - c = open-boundary class c) or by rank; the esoteric
// twist reads its storage addresses and the solid-neighbour mask from the ET
// table.
template <int NEED>
struct Node<A_INDIRECT, NEED> {
    int64_t a;
    int32_t m[(NEED & NEED_NB) ? 18 : 1];
    int32_t e[(NEED & NEED_ET) ? 6 : 1];
    uint32_t mask;

    __device__ __forceinline__ void init(const KArgs &k, uint32_t n)
    {
        a = n;
        if constexpr ((NEED & NEED_NB) != 0) {
            if (k.rank_words) {
                rank_neighbours(k, n, m);
            } else {
#pragma unroll
                for (int q = 0; q < 18; ++q) m[q] = k.idx[(int64_t)q * k.idx_pitch + n];
            }
        }
        if constexpr ((NEED & NEED_ET) != 0) {
            if (k.rank_words && k.ghost_words) {
                rank_et(k, n, e, mask);
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q) e[q] = k.et[(int64_t)q * k.idx_pitch + n];
                mask = (uint32_t)k.et[6 * k.idx_pitch + n];
            }
        }
    }
    __device__ __forceinline__ int64_t nb(int i) const { return m[i - 1]; }
    __device__ __forceinline__ bool solid(int i) const { return m[i - 1] < 0; }
    __device__ __forceinline__ int64_t at(int sx, int sy, int sz) const
    {
        const int c = et_cell(sx, sy, sz);
        return c == 0 ? a : (int64_t)e[c - 1];
    }
    __device__ __forceinline__ bool et_solid(int i) const { return (mask >> (i - 1)) & 1u; }
    // boundary class of the non-fluid neighbour at x + c_i (IDX code -1 - c)
    __device__ __forceinline__ int bc_class(int i) const
    {
        if constexpr ((NEED & NEED_NB) != 0)
            return -m[i - 1] - 1;
        else
            return 0;
    }
    // Opaque redefinition of one neighbour id (or ET entry) right before the
    // gather that uses it: the load's address cannot be computed earlier, so
    // the wait for that id lands here and not before the first gather load.
    __device__ __forceinline__ void pin_nb(int q)
    {
        if constexpr ((NEED & NEED_NB) != 0) asm volatile("" : "+v"(m[q]));
    }
    __device__ __forceinline__ void pin_et(int q)
    {
        if constexpr ((NEED & NEED_ET) != 0) asm volatile("" : "+v"(e[q]));
    }
    // Opaque redefinition of the node's index registers (an empty asm, no
    // memory access).  Called between gather and scatter, it keeps the
    // compiler from holding 19 wide gather addresses live across the
    // collision to reuse them for the scatter: the 32-bit ids are enough to
    // rebuild them, which halves the registers of the in-place kernels.
    __device__ __forceinline__ void refresh()
    {
        if constexpr ((NEED & NEED_NB) != 0) {
#pragma unroll
            for (int q = 0; q < 18; ++q) asm volatile("" : "+v"(m[q]));
        }
        if constexpr ((NEED & NEED_ET) != 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q) asm volatile("" : "+v"(e[q]));
            asm volatile("" : "+v"(mask));
        }
    }
};

// ------------------------------------------------------------------ slots
// Index of PDF slot (direction j, node or cell c) in a lattice buffer.
//   AoS: c * 19 + j.
//   SoA: j * pitch + c.
//   Blocked SoA: ((c >> bsh) * 19 + j) * 2^bsh + (c & bmk).
//     The 19 directions of a block of 2^bsh nodes lie in one contiguous
//     region, so the gathers and scatters of a workgroup stay in a few DRAM
//     pages instead of touching 19 arrays a lattice apart.
template <int ADDR, int LAY>
__device__ __forceinline__ int64_t slot_index(const KArgs &a, int j, int64_t c)
{
    if constexpr (LAY == L_AOS) {
        return elem<L_AOS>(j, c, a.pitch);
    } else if constexpr (LAY == L_BLK) {
        // the node's part and the direction's part apart: j << bsh is uniform
        const uint32_t u = (uint32_t)c;
        return ((int64_t)((u >> a.bsh) * (uint32_t)Q) << a.bsh) + (int64_t)(u & a.bmk) + ((int64_t)j << a.bsh);
    } else {
        return elem<L_SOA>(j, c, a.pitch);
    }
}

// ------------------------------------------------------------------ maps
template <int R, class N>
__device__ __forceinline__ void read_slot(const N &nd, int i, int &j, int64_t &c, int &bc)
{
    bc = 0;
    if constexpr (R == R_LOCAL) {
        j = i;
        c = nd.a;
    } else if constexpr (R == R_PULL) {
        const int o = opp(i);
        if (i == 0) {
            j = 0;
            c = nd.a;
        } else if (nd.solid(o)) {
            j = o;
            c = nd.a;
            bc = nd.bc_class(o);
        } else {
            j = i;
            c = nd.nb(o);
        }
    } else if constexpr (R == R_AAODD) {
        const int o = opp(i);
        if (i == 0) {
            j = 0;
            c = nd.a;
        } else if (nd.solid(o)) {
            j = i;
            c = nd.a;
            bc = nd.bc_class(o);
        } else {
            j = o;
            c = nd.nb(o);
        }
    } else {
        constexpr bool odd = (R == R_ET1);
        j = odd ? opp(i) : i;
        c = nd.at(ox(i), oy(i), oz(i));
    }
}

template <int R, class N>
__device__ __forceinline__ void read_slot(const N &nd, int i, int &j, int64_t &c)
{
    int bc;
    read_slot<R>(nd, i, j, c, bc);
}

template <int W, class N>
__device__ __forceinline__ void write_slot(const N &nd, int i, int &j, int64_t &c, int &bc)
{
    bc = 0;
    if constexpr (W == W_LOCAL) {
        j = i;
        c = nd.a;
    } else if constexpr (W == W_PUSH) {
        if (i == 0) {
            j = 0;
            c = nd.a;
        } else if (nd.solid(i)) {
            j = opp(i);
            c = nd.a;
            bc = nd.bc_class(i);
        } else {
            j = i;
            c = nd.nb(i);
        }
    } else if constexpr (W == W_AAEVEN) {
        j = opp(i);
        c = nd.a;
    } else {
        constexpr bool odd = (W == W_ET1);
        const int o = opp(i);
        c = nd.at(ox(o), oy(o), oz(o));
        const bool s = (i != 0) && nd.et_solid(i);
        j = s ? (odd ? o : i) : (odd ? i : o);
    }
}

template <int W, class N>
__device__ __forceinline__ void write_slot(const N &nd, int i, int &j, int64_t &c)
{
    int bc;
    write_slot<W>(nd, i, j, c, bc);
}

// Indirect gathers: each load's address comes from one neighbour id, loaded
// in Node::init.  Pinning that id right before the load (gather_pin) and a
// scheduling barrier after it (gather_order) issue each load as soon as its
// id has arrived; otherwise the address computations are grouped first and
// every id is waited for before the first gather load (512^3 pack, AA odd:
// 4.48 against 5.47 ms).
template <int ADDR, int R, class N>
__device__ __forceinline__ void gather_pin(N &nd, int i)
{
    if constexpr (ADDR == A_INDIRECT && (R == R_PULL || R == R_AAODD)) {
        if (i != 0) nd.pin_nb(opp(i) - 1);
    } else if constexpr (ADDR == A_INDIRECT && (R == R_ET0 || R == R_ET1)) {
        const int c = et_cell(ox(i), oy(i), oz(i));
        if (c != 0) nd.pin_et(c - 1);
    }
}
template <int ADDR, int R>
__device__ __forceinline__ void gather_order()
{
    if constexpr (ADDR == A_INDIRECT && R != R_LOCAL) __builtin_amdgcn_sched_barrier(0);
}

// Open-boundary rule on every gathered value that crossed a boundary link
// (indirect grids, gathering read maps).  Applied after all 19 loads have
// been issued: a branch between two loads would make a wavefront with such
// a link wait for each load in turn.
template <int ADDR, int R, class N, typename T>
__device__ __forceinline__ void bc_arrive_all(const KArgs &a, const N &nd, T (&v)[Q])
{
    if constexpr (ADDR == A_INDIRECT && (R == R_PULL || R == R_AAODD)) {
        if (!a.bc_on) return;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int j, bc;
            int64_t c;
            read_slot<R>(nd, i, j, c, bc);
            if (bc > 0) v[i] = bc_arrive<T>(a, bc, i, v[i]);
        }
    }
}

// ------------------------------------------------------------------ maps as offsets (direct grids)
// The same maps as above, giving the slot as (array j, cell offset s) with
// cell = x + s.  On a direct grid solidity depends on z only, so for a given
// direction the slot is the same for every node of an x-row.
template <int R, class N>
__device__ __forceinline__ void read_off(const N &nd, int i, int &j, int &sx, int &sy, int &sz)
{
    sx = sy = sz = 0;
    if constexpr (R == R_LOCAL) {
        j = i;
    } else if constexpr (R == R_PULL || R == R_AAODD) {
        const int o = opp(i);
        const bool pull = (R == R_PULL);
        if (i == 0) {
            j = 0;
        } else if (nd.solid(o)) {
            j = pull ? o : i;
        } else {
            j = pull ? i : o;
            sx = -cx(i);
            sy = -cy(i);
            sz = -cz(i);
        }
    } else {
        constexpr bool odd = (R == R_ET1);
        j = odd ? opp(i) : i;
        sx = ox(i);
        sy = oy(i);
        sz = oz(i);
    }
}

template <int W, class N>
__device__ __forceinline__ void write_off(const N &nd, int i, int &j, int &sx, int &sy, int &sz)
{
    sx = sy = sz = 0;
    if constexpr (W == W_LOCAL) {
        j = i;
    } else if constexpr (W == W_PUSH) {
        if (i == 0) {
            j = 0;
        } else if (nd.solid(i)) {
            j = opp(i);
        } else {
            j = i;
            sx = cx(i);
            sy = cy(i);
            sz = cz(i);
        }
    } else if constexpr (W == W_AAEVEN) {
        j = opp(i);
    } else {
        constexpr bool odd = (W == W_ET1);
        const int o = opp(i);
        sx = ox(o);
        sy = oy(o);
        sz = oz(o);
        const bool s = (i != 0) && nd.et_solid(i);
        j = s ? (odd ? o : i) : (odd ? i : o);
    }
}

// LDS row of the directions with cx != 0 (the only ones an x-shift can touch)
__host__ __device__ constexpr int xslot(int i)
{
    return i == 1 ? 0 : i == 2 ? 1 : (i >= 7 && i <= 14) ? i - 5 : -1;
}
constexpr int NXSLOT = 10;

// Direct SoA update with x-rows staged per workgroup.  Every global access
// of the node's own row segment is made at the node's own x, so a wavefront
// touches whole aligned cache lines; an x-shift of +-1 becomes a shift inside
// the segment, done through LDS:
//   read  slot x + sx:  thread x loads cell (x, y+sy, z+sz), the consumer
//                       x - sx picks it up from LDS;
//   write slot x + sx:  thread x deposits its value at LDS position x + sx,
//                       the owner of that position stores it at its own x.
// Two shapes (row_staged = 1 or 2):
//   1: nx divides BLOCK.  A workgroup holds whole rows (consecutive nodes) and
//      the shift is cyclic inside each row, which is the periodic wrap in x.
//   2: BLOCK divides nx.  A workgroup holds one segment of BLOCK nodes of a
//      row.  An end lane whose shifted slot lies beyond the segment loads that
//      value from global memory itself (read side), or stores its outgoing
//      value there itself (write side); positions that no lane of this
//      workgroup deposits into are stored by the neighbouring segment's end
//      lane.
// Threads past n_nodes form whole rows; they skip memory but join barriers.
// WIDE selects shape 2 at compile time, so that the shape-1 code carries none
// of the segment-end work; both shapes share one LDS array.
template <typename st>
__device__ __forceinline__ st (&staging_rows())[NXSLOT][BLOCK]
{
    __shared__ st xs[NXSLOT][BLOCK];
    return xs;
}

template <int PREC, int KIND, int COLL, bool WIDE, int LAY>
__device__ __forceinline__ void update_direct_staged(const KArgs &a)
{
    using S = Store<PREC>;
    using st = typename S::st;
    using ct = typename S::ct;
    constexpr int R = rmap_of(KIND);
    constexpr int W = wmap_of(KIND);
    st(&xs)[NXSLOT][BLOCK] = staging_rows<st>();
    const uint32_t t = threadIdx.x;
    const uint32_t n = logical_block(a) * BLOCK + t;
    const bool valid = n < a.n_nodes;
    const uint32_t seg = WIDE ? (uint32_t)BLOCK : (uint32_t)a.nx; // a power of two
    const uint32_t xl = t & (seg - 1), row = t - xl;
    // LDS position of segment position xl + sx (|sx| <= 1), cyclic in a row
    auto pos = [&](int sx) -> uint32_t { return row + (((uint32_t)((int)xl + sx)) & (seg - 1)); };
    // whether segment position xl + sx lies outside this workgroup's segment
    auto beyond = [&](int sx) -> bool { return WIDE && ((int)xl + sx < 0 || (int)xl + sx >= BLOCK); };
    Node<A_DIRECT, 0> nd;
    nd.init(a, valid ? n : 0);
    const st *src = static_cast<const st *>(a.src);
    st *dst = static_cast<st *>(a.dst);
    // All 19 loads first (each at the node's own x), so they are in flight
    // together.  They are unconditional: a thread past n_nodes addresses node
    // 0 (in bounds) and never stores what it loaded.  In a wide segment the
    // end lanes also load the values beyond it that they consume.
    typename S::rt raw[Q];
    typename S::rt halo[WIDE ? NXSLOT : 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        read_off<R>(nd, i, j, sx, sy, sz);
        raw[i] = pdf_load_raw<true, S>(src + slot_index<A_DIRECT, LAY>(a, j, nd.shift(0, sy, sz)));
        if (xslot(i) >= 0 && sx != 0 && beyond(sx))
            halo[WIDE && xslot(i) > 0 ? xslot(i) : 0] = pdf_load_raw<true, S>(src + slot_index<A_DIRECT, LAY>(a, j, nd.shift(sx, sy, sz)));
    }
    ct v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        read_off<R>(nd, i, j, sx, sy, sz);
        if (xslot(i) >= 0 && sx != 0) {
            xs[xslot(i) < 0 ? 0 : xslot(i)][t] = S::unraw(raw[i]);
        } else {
            v[i] = S::load_raw(raw[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (xslot(i) >= 0) {
            int j, sx, sy, sz;
            read_off<R>(nd, i, j, sx, sy, sz);
            const int k = xslot(i) < 0 ? 0 : xslot(i);
            if (sx != 0) v[i] = beyond(sx) ? S::load_raw(halo[WIDE ? k : 0]) : S::load(xs[k][pos(sx)]);
        }
    }
    __syncthreads();
    if constexpr (COLL == 1 && KIND != K_TS_STREAM) {
        const CollideParams<ct> &p = cparams<ct>(a);
        collide_node<ct, S::shifted>(v, p);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        write_off<W>(nd, i, j, sx, sy, sz);
        if (xslot(i) >= 0 && sx != 0) {
            if (beyond(sx)) {
                if (valid) pdf_store<true>(dst + slot_index<A_DIRECT, LAY>(a, j, nd.shift(sx, sy, sz)), S::save(v[i]));
            } else {
                xs[xslot(i) < 0 ? 0 : xslot(i)][pos(sx)] = S::save(v[i]);
            }
            continue;
        }
        if (valid) pdf_store<true>(dst + slot_index<A_DIRECT, LAY>(a, j, nd.shift(0, sy, sz)), S::save(v[i]));
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (xslot(i) >= 0) {
            int j, sx, sy, sz;
            write_off<W>(nd, i, j, sx, sy, sz);
            // the depositor of this position is segment position xl - sx
            if (sx != 0 && valid && !beyond(-sx))
                pdf_store<true>(dst + slot_index<A_DIRECT, LAY>(a, j, nd.shift(0, sy, sz)), xs[xslot(i) < 0 ? 0 : xslot(i)][t]);
        }
    }
}

// Direct SoA update with x-shifts through LDS for any nx (the shapes above
// need nx to divide BLOCK or BLOCK to divide nx).  A workgroup holds BLOCK
// consecutive nodes, which may span row boundaries.  For an x-shift s the
// neighbour of node n is n + s inside the same row (periodic in x: n + s -/+ nx
// across the row's end).  A neighbour inside the workgroup is reached through
// LDS at its own lane; one outside it is loaded from, or stored to, global
// memory by the lane itself, and an owner stores an LDS position only if its
// depositor lies inside the workgroup.  Every global access of a lane's own
// node is made at the node's own x.
template <int PREC, int KIND, int COLL, int LAY>
__device__ __forceinline__ void update_direct_general(const KArgs &a)
{
    using S = Store<PREC>;
    using st = typename S::st;
    using ct = typename S::ct;
    constexpr int R = rmap_of(KIND);
    constexpr int W = wmap_of(KIND);
    st(&xs)[NXSLOT][BLOCK] = staging_rows<st>();
    const uint32_t t = threadIdx.x;
    const uint32_t n0 = logical_block(a) * BLOCK;
    const uint32_t n = n0 + t;
    const bool valid = n < a.n_nodes;
    const uint32_t m = valid ? n : 0;
    const uint32_t nx = (uint32_t)a.nx;
    const uint32_t x = m - fdiv(m, a.dvx) * nx;
    // node of the same-row neighbour at x + s (s = +-1), and whether it is one
    // of this workgroup's nodes
    auto along = [&](int s) -> int64_t {
        int64_t q = (int64_t)m + s;
        if (s > 0 && x == nx - 1) q -= nx;
        if (s < 0 && x == 0) q += nx;
        return q;
    };
    auto inside = [&](int64_t q) -> bool { return q >= (int64_t)n0 && q < (int64_t)n0 + BLOCK; };
    Node<A_DIRECT, 0> nd;
    nd.init(a, m);
    const st *src = static_cast<const st *>(a.src);
    st *dst = static_cast<st *>(a.dst);
    // all loads first: the own-x value of every direction, and for a shifted
    // direction whose neighbour lies outside the workgroup, that value too
    typename S::rt raw[Q];
    typename S::rt halo[NXSLOT];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        read_off<R>(nd, i, j, sx, sy, sz);
        raw[i] = pdf_load_raw<true, S>(src + slot_index<A_DIRECT, LAY>(a, j, nd.shift(0, sy, sz)));
        if (xslot(i) >= 0 && sx != 0 && valid && !inside(along(sx)))
            halo[xslot(i) > 0 ? xslot(i) : 0] = pdf_load_raw<true, S>(src + slot_index<A_DIRECT, LAY>(a, j, nd.shift(sx, sy, sz)));
    }
    ct v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        read_off<R>(nd, i, j, sx, sy, sz);
        if (xslot(i) >= 0 && sx != 0) {
            xs[xslot(i) < 0 ? 0 : xslot(i)][t] = S::unraw(raw[i]);
        } else {
            v[i] = S::load_raw(raw[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (xslot(i) >= 0) {
            int j, sx, sy, sz;
            read_off<R>(nd, i, j, sx, sy, sz);
            const int k = xslot(i) < 0 ? 0 : xslot(i);
            if (sx != 0) {
                const int64_t q = along(sx);
                v[i] = inside(q) ? S::load(xs[k][(uint32_t)(q - n0)]) : S::load_raw(halo[k]);
            }
        }
    }
    __syncthreads();
    if constexpr (COLL == 1 && KIND != K_TS_STREAM) {
        const CollideParams<ct> &p = cparams<ct>(a);
        collide_node<ct, S::shifted>(v, p);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        write_off<W>(nd, i, j, sx, sy, sz);
        if (xslot(i) >= 0 && sx != 0) {
            // a lane past n_nodes stands at node 0 and deposits nothing: its
            // neighbour could be a position whose depositor is a real node
            const int64_t q = along(sx);
            if (!valid) continue;
            if (inside(q))
                xs[xslot(i) < 0 ? 0 : xslot(i)][(uint32_t)(q - n0)] = S::save(v[i]);
            else
                pdf_store<true>(dst + slot_index<A_DIRECT, LAY>(a, j, nd.shift(sx, sy, sz)), S::save(v[i]));
            continue;
        }
        if (valid) pdf_store<true>(dst + slot_index<A_DIRECT, LAY>(a, j, nd.shift(0, sy, sz)), S::save(v[i]));
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (xslot(i) >= 0) {
            int j, sx, sy, sz;
            write_off<W>(nd, i, j, sx, sy, sz);
            // the depositor of this position is the neighbour at x - sx
            if (sx != 0 && valid && inside(along(-sx)))
                pdf_store<true>(dst + slot_index<A_DIRECT, LAY>(a, j, nd.shift(0, sy, sz)), xs[xslot(i) < 0 ? 0 : xslot(i)][t]);
        }
    }
}

// Direct SoA update of two x-neighbours (x even, x + 1) per lane: the pair's
// values of one direction form one aligned word (2 x 16, 2 x 32 or 2 x 64
// bits), so each load or store of a wavefront covers twice the bytes of the
// one-node kernels with the same number of instructions.  Both nodes share y
// and z, hence every bounce-back decision.  nx is a power of two dividing
// 2 * BLOCK, so a workgroup holds whole x-rows and the x-shifts go through
// LDS as in update_direct_staged (each lane deposits or picks up two
// values).  Per node the arithmetic is that of the one-node kernels, so the
// results are bit-identical.
typedef uint16_t __attribute__((may_alias)) u16_alias;
typedef uint32_t __attribute__((may_alias)) u32_alias;
typedef float v2f __attribute__((ext_vector_type(2)));
typedef double v2d __attribute__((ext_vector_type(2)));

template <int PREC>
struct Pair;
template <>
struct Pair<P_F16S> {
    using word = uint32_t; // node x in the low half, x + 1 in the high half
    using elem = uint16_t;
    __device__ static elem lo(word w) { return (elem)(w & 0xffffu); }
    __device__ static elem hi(word w) { return (elem)(w >> 16); }
    __device__ static word join(elem a, elem b) { return (word)a | ((word)b << 16); }
    __device__ static float load(elem e) { return (float)__builtin_bit_cast(_Float16, e); }
    __device__ static elem save(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};
template <typename E, typename V>
struct PairPlain {
    using word = V;
    using elem = E;
    __device__ static elem lo(word w) { return w.x; }
    __device__ static elem hi(word w) { return w.y; }
    __device__ static word join(elem a, elem b) { return word{a, b}; }
    __device__ static E load(elem e) { return e; }
    __device__ static elem save(E v) { return v; }
};
template <>
struct Pair<P_F32> : PairPlain<float, v2f> {};
template <>
struct Pair<P_F32S> : PairPlain<float, v2f> {};
template <>
struct Pair<P_F64> : PairPlain<double, v2d> {};

// WIDE: nx a multiple of 2 * BLOCK, one 512-node segment of a row per
// workgroup (as the one-node row segments): lane 0's first node and lane
// BLOCK-1's second node reach one element beyond the segment in global
// memory, and an owner whose word is half written by the neighbouring
// segment stores only its own half.
template <int PREC, int KIND, int COLL, bool WIDE>
__device__ __forceinline__ void update_direct_pair(const KArgs &a)
{
    using S = Store<PREC>;
    using ct = typename S::ct;
    using PW = Pair<PREC>;
    using word = typename PW::word;
    using el_t = typename PW::elem;
    typedef el_t __attribute__((may_alias)) elem_alias;
    typedef word __attribute__((may_alias)) word_alias;
    constexpr int R = rmap_of(KIND);
    constexpr int W = wmap_of(KIND);
    constexpr bool shifts = !(R == R_LOCAL && (W == W_LOCAL || W == W_AAEVEN));
    constexpr uint32_t NP = 2 * BLOCK; // nodes per workgroup
    __shared__ word xw[shifts ? NXSLOT : 1][shifts ? BLOCK : 1];
    const uint32_t t = threadIdx.x;
    const uint32_t p = 2 * t;          // the pair's first node within the workgroup
    const uint32_t n = logical_block(a) * NP + p;
    const bool valid = n < a.n_nodes;  // n_nodes is a multiple of nx, so pairs are whole
    const uint32_t nx = (uint32_t)a.nx;
    const uint32_t seg = WIDE ? NP : nx; // a power of two
    const uint32_t xl = p & (seg - 1), row = p - xl;
    Node<A_DIRECT, 0> nd;
    nd.init(a, valid ? n : 0);
    const word *src = static_cast<const word *>(a.src);
    word *dst = static_cast<word *>(a.dst);
    const elem_alias *src_e = static_cast<const elem_alias *>(a.src);
    elem_alias *dst_e = static_cast<elem_alias *>(a.dst);
    auto lds = [&](int slot) { return reinterpret_cast<elem_alias *>(&xw[slot][0]); };
    // wide segments: whether segment position q lies beyond this workgroup,
    // and the cell of x + 2 (the second node's right neighbour, periodic)
    auto beyond = [&](int q) -> bool { return WIDE && (q < 0 || q >= (int)NP); };
    int64_t dx2 = 2;
    if constexpr (WIDE) {
        const uint32_t m = valid ? n : 0;
        const uint32_t x = m - fdiv(m, a.dvx) * nx;
        if (x + 2 >= nx) dx2 = 2 - (int64_t)nx;
    }
    // all 19 word loads first, at the pair's own x (unconditional: a lane
    // past n_nodes addresses node 0 and never stores); the segment-end lanes
    // also load the element beyond the segment that they consume
    word raw[Q];
    el_t halo[WIDE ? NXSLOT : 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        read_off<R>(nd, i, j, sx, sy, sz);
        raw[i] = pdf_load<true>(src + (elem<L_SOA>(j, nd.shift(0, sy, sz), a.pitch) >> 1));
        if constexpr (WIDE && shifts) {
            if (xslot(i) >= 0 && sx != 0 && beyond(sx < 0 ? (int)xl - 1 : (int)xl + 2)) {
                const int64_t c = sx < 0 ? nd.shift(-1, sy, sz) : nd.shift(0, sy, sz) + dx2;
                halo[xslot(i) > 0 ? xslot(i) : 0] = pdf_load<true>(src_e + elem<L_SOA>(j, c, a.pitch));
            }
        }
    }
    if constexpr (WIDE && shifts) {
        // opaque redefinition of the raw halo values (an empty asm, no memory
        // access): their conversion cannot move into the load branches, where
        // it would wait for each load in turn
#pragma unroll
        for (int k = 0; k < NXSLOT; ++k) asm volatile("" : "+v"(halo[k]));
    }
    ct v0[Q], v1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        read_off<R>(nd, i, j, sx, sy, sz);
        if (shifts && xslot(i) >= 0 && sx != 0) {
            reinterpret_cast<word_alias *>(&xw[xslot(i) < 0 ? 0 : xslot(i)][0])[t] = raw[i];
        } else {
            v0[i] = PW::load(PW::lo(raw[i]));
            v1[i] = PW::load(PW::hi(raw[i]));
        }
    }
    if constexpr (shifts) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (xslot(i) >= 0) {
                int j, sx, sy, sz;
                read_off<R>(nd, i, j, sx, sy, sz);
                if (sx != 0) {
                    const int k = xslot(i) < 0 ? 0 : xslot(i);
                    const elem_alias *h = lds(k);
                    v0[i] = PW::load(h[row + ((xl + (uint32_t)sx) & (seg - 1))]);
                    v1[i] = PW::load(h[row + ((xl + 1u + (uint32_t)sx) & (seg - 1))]);
                    if constexpr (WIDE) {
                        if (sx < 0 && beyond((int)xl - 1)) v0[i] = PW::load(halo[k]);
                        if (sx > 0 && beyond((int)xl + 2)) v1[i] = PW::load(halo[k]);
                    }
                }
            }
        }
        __syncthreads();
    }
    if constexpr (COLL == 1 && KIND != K_TS_STREAM) {
        const CollideParams<ct> &cp = cparams<ct>(a);
        collide_node<ct, S::shifted>(v0, cp);
        collide_node<ct, S::shifted>(v1, cp);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, sx, sy, sz;
        write_off<W>(nd, i, j, sx, sy, sz);
        if (shifts && xslot(i) >= 0 && sx != 0) {
            elem_alias *h = lds(xslot(i) < 0 ? 0 : xslot(i));
            // a value whose slot lies beyond the segment goes to global memory
            if (beyond((int)xl + sx)) {
                if (valid) pdf_store<true>(dst_e + elem<L_SOA>(j, nd.shift(-1, sy, sz), a.pitch), PW::save(v0[i]));
            } else {
                h[row + ((xl + (uint32_t)sx) & (seg - 1))] = PW::save(v0[i]);
            }
            if (beyond((int)xl + 1 + sx)) {
                if (valid) pdf_store<true>(dst_e + elem<L_SOA>(j, nd.shift(0, sy, sz) + dx2, a.pitch), PW::save(v1[i]));
            } else {
                h[row + ((xl + 1u + (uint32_t)sx) & (seg - 1))] = PW::save(v1[i]);
            }
            continue;
        }
        if (valid) pdf_store<true>(dst + (elem<L_SOA>(j, nd.shift(0, sy, sz), a.pitch) >> 1),
                                   PW::join(PW::save(v0[i]), PW::save(v1[i])));
    }
    if constexpr (shifts) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (xslot(i) >= 0) {
                int j, sx, sy, sz;
                write_off<W>(nd, i, j, sx, sy, sz);
                if (sx != 0 && valid) {
                    const word w = reinterpret_cast<const word_alias *>(&xw[xslot(i) < 0 ? 0 : xslot(i)][0])[t];
                    const int64_t e = elem<L_SOA>(j, nd.shift(0, sy, sz), a.pitch);
                    // the depositors of positions xl and xl + 1 are xl - sx and xl + 1 - sx
                    if (beyond((int)xl - sx))
                        pdf_store<true>(dst_e + e + 1, PW::hi(w));
                    else if (beyond((int)xl + 1 - sx))
                        pdf_store<true>(dst_e + e, PW::lo(w));
                    else
                        pdf_store<true>(dst + (e >> 1), w);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ update kernel
// One node's update through the generic maps (any addressing and layout).
template <int ADDR, int LAY, int PREC, int KIND, int COLL>
__device__ __forceinline__ void update_node(const KArgs &a, uint32_t n)
{
    using S = Store<PREC>;
    using st = typename S::st;
    using ct = typename S::ct;
    constexpr int R = rmap_of(KIND);
    constexpr int W = wmap_of(KIND);
    // nontemporal hint where every touched line is read or written whole by
    // this workgroup: direct SoA, and node-local kernels on indirect SoA grids
    constexpr bool local = (R == R_LOCAL && (W == W_LOCAL || W == W_AAEVEN));
    constexpr bool NT = (LAY != L_AOS) && (ADDR == A_DIRECT || local);
    Node<ADDR, need_r(R) | need_w(W)> nd;
    nd.init(a, n);
    const st *src = static_cast<const st *>(a.src);
    st *dst = static_cast<st *>(a.dst);
    ct v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, bc;
        int64_t c;
        gather_pin<ADDR, R>(nd, i);
        read_slot<R>(nd, i, j, c, bc);
        v[i] = S::load(pdf_load<NT>(src + slot_index<ADDR, LAY>(a, j, c)));
        gather_order<ADDR, R>();
    }
    bc_arrive_all<ADDR, R>(a, nd, v);
    if constexpr (COLL == 1 && KIND != K_TS_STREAM) {
        const CollideParams<ct> &p = cparams<ct>(a);
        collide_node<ct, S::shifted>(v, p);
    }
    if constexpr (need_r(R) != 0 && need_w(W) != 0) nd.refresh(); // gather and scatter both use the ids
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j, bc;
        int64_t c;
        write_slot<W>(nd, i, j, c, bc);
        if constexpr (ADDR == A_INDIRECT && (W == W_ET0 || W == W_ET1)) bc = et_write_class<W>(a, nd, i);
        ct out = v[i];
        if constexpr (ADDR == A_INDIRECT && (W == W_PUSH || W == W_ET0 || W == W_ET1)) {
            if (bc > 0 && a.bc_on) out = bc_arrive<ct>(a, bc, opp(i), out);
        }
        pdf_store<NT>(dst + slot_index<ADDR, LAY>(a, j, c), S::save(out));
    }
}

// AoS update with the node-local side staged through LDS (Sec. 1: AoS keeps
// a node's 19 PDFs together, so a workgroup's 256 consecutive nodes are one
// contiguous block of 256 * 19 values).  A local read copies that block
// into LDS with coalesced accesses and each lane then reads its record from
// LDS; a local write goes the other way.  Non-local sides (gathers from or
// scatters to neighbours) stay per lane.  Nodes past n_nodes skip memory but
// join the barriers.
template <int ADDR, int PREC, int KIND, int COLL>
__device__ __forceinline__ void update_aos_staged(const KArgs &a)
{
    using S = Store<PREC>;
    using st = typename S::st;
    using ct = typename S::ct;
    constexpr int R = rmap_of(KIND);
    constexpr int W = wmap_of(KIND);
    constexpr bool local_r = (R == R_LOCAL);
    constexpr bool local_w = (W == W_LOCAL || W == W_AAEVEN);
    __shared__ st rec[BLOCK * Q];
    const uint32_t t = threadIdx.x;
    const uint32_t n0 = logical_block(a) * BLOCK;
    const uint32_t cnt = min((uint32_t)BLOCK, a.n_nodes - n0); // the grid covers n_nodes, so n0 < n_nodes
    const bool valid = t < cnt;
    const uint32_t n = n0 + (valid ? t : 0);
    Node<ADDR, need_r(R) | need_w(W)> nd;
    nd.init(a, n);
    const int64_t a0 = (ADDR == A_DIRECT) ? (int64_t)n0 + a.z0_offset : (int64_t)n0; // first record
    const st *src = static_cast<const st *>(a.src);
    st *dst = static_cast<st *>(a.dst);
    ct v[Q];
    if constexpr (local_r) {
        // coalesced copy of the block's records into LDS.  When the write side
        // is node-local too, a full block issues all 19 loads of a lane before
        // its first LDS store (the lines belong to this workgroup alone, hence
        // the nontemporal hint); a kernel that scatters to neighbours keeps the
        // lighter loop (OS push AoS: 2.1 ms against 2.6 ms unrolled)
        const st *base = src + a0 * Q;
        if (local_w && cnt == (uint32_t)BLOCK) {
            st tmp[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) tmp[k] = pdf_load<true>(base + t + k * BLOCK);
#pragma unroll
            for (int k = 0; k < Q; ++k) rec[t + k * BLOCK] = tmp[k];
        } else {
            for (uint32_t e = t; e < cnt * Q; e += BLOCK) rec[e] = base[e];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = S::load(rec[t * Q + i]);
        __syncthreads();
    } else {
        if (valid) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int j, bc;
                int64_t c;
                gather_pin<ADDR, R>(nd, i);
                read_slot<R>(nd, i, j, c, bc);
                v[i] = S::load(src[elem<L_AOS>(j, c, a.pitch)]);
                gather_order<ADDR, R>();
            }
            bc_arrive_all<ADDR, R>(a, nd, v);
        }
    }
    if (valid) {
        if constexpr (COLL == 1 && KIND != K_TS_STREAM) {
            const CollideParams<ct> &p = cparams<ct>(a);
            collide_node<ct, S::shifted>(v, p);
        }
    }
    if constexpr (local_w) {
        if (valid) {
#pragma unroll
            for (int i = 0; i < Q; ++i) rec[t * Q + (W == W_AAEVEN ? opp(i) : i)] = S::save(v[i]);
        }
        __syncthreads();
        st *base = dst + a0 * Q;
        if (cnt == (uint32_t)BLOCK) {
            st tmp[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) tmp[k] = rec[t + k * BLOCK];
#pragma unroll
            for (int k = 0; k < Q; ++k) pdf_store<true>(base + t + k * BLOCK, tmp[k]);
        } else {
            for (uint32_t e = t; e < cnt * Q; e += BLOCK) base[e] = rec[e];
        }
    } else {
        if (valid) {
            if constexpr (need_r(R) != 0 && need_w(W) != 0) nd.refresh();
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int j, bc;
                int64_t c;
                write_slot<W>(nd, i, j, c, bc);
                if constexpr (ADDR == A_INDIRECT && (W == W_ET0 || W == W_ET1)) bc = et_write_class<W>(a, nd, i);
                ct out = v[i];
                if constexpr (ADDR == A_INDIRECT && (W == W_PUSH || W == W_ET0 || W == W_ET1)) {
                    if (bc > 0 && a.bc_on) out = bc_arrive<ct>(a, bc, opp(i), out);
                }
                dst[elem<L_AOS>(j, c, a.pitch)] = S::save(out);
            }
        }
    }
}

// Two nodes per lane on direct SoA grids (a kernel of its own: its registers
// and LDS would otherwise count against every one-node kernel).
template <int PREC, int KIND, int COLL>
__global__ void __launch_bounds__(BLOCK) k_update_pair(KArgs a)
{
    update_direct_pair<PREC, KIND, COLL, false>(a);
}
// ... with one 512-node row segment per workgroup (nx a multiple of 512)
template <int PREC, int KIND, int COLL>
__global__ void __launch_bounds__(BLOCK) k_update_pair_wide(KArgs a)
{
    update_direct_pair<PREC, KIND, COLL, true>(a);
}

// kernels whose maps never shift along x need no staging
__host__ __device__ constexpr bool shifts_x(int kind)
{
    return !(rmap_of(kind) == R_LOCAL && (wmap_of(kind) == W_LOCAL || wmap_of(kind) == W_AAEVEN));
}

// Direct SoA grids of any other nx: BLOCK consecutive nodes, shifts through
// LDS inside the workgroup (a kernel of its own, as above).
template <int PREC, int KIND, int COLL, int LAY>
__global__ void __launch_bounds__(BLOCK) k_update_gen(KArgs a)
{
    if constexpr (shifts_x(KIND)) {
        update_direct_general<PREC, KIND, COLL, LAY>(a);
    } else {
        const uint32_t n = logical_block(a) * BLOCK + threadIdx.x;
        if (n >= a.n_nodes) return;
        update_node<A_DIRECT, LAY, PREC, KIND, COLL>(a, n);
    }
}

// Direct SoA grids whose nx is a multiple of BLOCK: one row segment per
// workgroup (a kernel of its own, so that the segment-end work does not count
// against the registers of the other kernels).
template <int PREC, int KIND, int COLL, int LAY>
__global__ void __launch_bounds__(BLOCK) k_update_wide(KArgs a)
{
    if constexpr (shifts_x(KIND)) {
        update_direct_staged<PREC, KIND, COLL, true, LAY>(a);
    } else {
        const uint32_t n = logical_block(a) * BLOCK + threadIdx.x;
        if (n >= a.n_nodes) return;
        update_node<A_DIRECT, LAY, PREC, KIND, COLL>(a, n);
    }
}

template <int ADDR, int LAY, int PREC, int KIND, int COLL>
__global__ void __launch_bounds__(BLOCK) k_update(KArgs a)
{
    constexpr int R = rmap_of(KIND);
    constexpr int W = wmap_of(KIND);
    // open boundaries exist on indirect grids, for the maps that cross links
    constexpr bool links = R == R_PULL || R == R_AAODD || W == W_PUSH || W == W_ET0 || W == W_ET1;
    if constexpr (ADDR == A_INDIRECT && links) bc_table_fill<typename Store<PREC>::ct>(a);
    if constexpr (ADDR == A_DIRECT && LAY != L_AOS && shifts_x(KIND)) {
        if (a.row_staged == 1) {
            update_direct_staged<PREC, KIND, COLL, false, LAY>(a);
            return;
        }
    }
    // AoS kernels with a node-local side stage that side through LDS
    constexpr bool aos_local = (R == R_LOCAL) || (W == W_LOCAL || W == W_AAEVEN);
    if constexpr (LAY == L_AOS && aos_local) {
        update_aos_staged<ADDR, PREC, KIND, COLL>(a);
        return;
    }
    const uint32_t n = logical_block(a) * BLOCK + threadIdx.x;
    if (n >= a.n_nodes) return;
    update_node<ADDR, LAY, PREC, KIND, COLL>(a, n);
}

// ------------------------------------------------------------------ canonical transfer
// The canonical state f(t) is what the next step reads: gather (get) and
// scatter (set, init) go through the read map of the bound scheme's state.
template <int ADDR, int LAY, int PREC, int R>
__global__ void __launch_bounds__(BLOCK) k_get(KArgs a)
{
    using S = Store<PREC>;
    using st = typename S::st;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= a.n_nodes) return;
    Node<ADDR, need_r(R)> nd;
    nd.init(a, n);
    const st *src = static_cast<const st *>(a.src);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j;
        int64_t c;
        int bc;
        read_slot<R>(nd, i, j, c, bc);
        double f = S::to_canon(src[slot_index<ADDR, LAY>(a, j, c)], i, a.sigma);
        if (bc > 0 && a.bc_on) f = bc_arrive_canon(a, bc, i, f);
        a.canon[(int64_t)i * a.n_nodes + n] = f;
    }
}

template <int ADDR, int LAY, int PREC, int R>
__global__ void __launch_bounds__(BLOCK) k_set(KArgs a)
{
    using S = Store<PREC>;
    using st = typename S::st;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= a.n_nodes) return;
    Node<ADDR, need_r(R)> nd;
    nd.init(a, n);
    st *dst = static_cast<st *>(a.dst);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j;
        int64_t c;
        int bc;
        read_slot<R>(nd, i, j, c, bc);
        double f = a.canon_in[(int64_t)i * a.n_nodes + n];
        if (bc > 0 && a.bc_on) f = bc_depart_canon(a, bc, i, f);
        dst[slot_index<ADDR, LAY>(a, j, c)] = S::from_canon(f, i, a.sigma);
    }
}

// f_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u), FP64
template <int ADDR, int LAY, int PREC, int R>
__global__ void __launch_bounds__(BLOCK) k_init(KArgs a)
{
    using S = Store<PREC>;
    using st = typename S::st;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= a.n_nodes) return;
    Node<ADDR, need_r(R)> nd;
    nd.init(a, n);
    double rho = 1.0, ux = 0.0, uy = 0.0, uz = 0.0;
    if (a.rho_u) {
        rho = a.rho_u[n];
        ux = a.rho_u[(int64_t)a.n_nodes + n];
        uy = a.rho_u[2 * (int64_t)a.n_nodes + n];
        uz = a.rho_u[3 * (int64_t)a.n_nodes + n];
    }
    const double uu = ux * ux + uy * uy + uz * uz;
    st *dst = static_cast<st *>(a.dst);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
        double feq = wd(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        int j, bc;
        int64_t c;
        read_slot<R>(nd, i, j, c, bc);
        if (bc > 0 && a.bc_on) feq = bc_depart_canon(a, bc, i, feq);
        dst[slot_index<ADDR, LAY>(a, j, c)] = S::from_canon(feq, i, a.sigma);
    }
}

// ------------------------------------------------------------------ moments
// Per node FP64 sums M_n = sum_i f_i, J_n = sum_i c_i f_i; per block a fixed
// butterfly over the wavefront (64 lanes) then the 4 wavefronts in order.
__device__ __forceinline__ void block_sum4(double (&m)[4], double *out)
{
    __shared__ double part[BLOCK / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m[k] += __shfl_xor(m[k], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) part[wave][k] = m[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double s = part[0][k];
#pragma unroll
            for (int w = 1; w < BLOCK / 64; ++w) s += part[w][k];
            out[k] = s;
        }
    }
    __syncthreads(); // part[] may be reused by a following call in the same workgroup
}

// FP64 moments (M, Jx, Jy, Jz) of one node's canonical PDFs, read through map
// R; `can` holds the open-boundary constants (the kernel arguments' own, or a
// batched slot's in device memory).
template <int ADDR, int LAY, int PREC, int R>
__device__ __forceinline__ void node_moments(const KArgs &a, uint32_t n, double (&m)[4], const double (*can)[Q])
{
    using S = Store<PREC>;
    using st = typename S::st;
    Node<ADDR, need_r(R)> nd;
    nd.init(a, n);
    const st *src = static_cast<const st *>(a.src);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int j;
        int64_t c;
        int bc;
        read_slot<R>(nd, i, j, c, bc);
        double f = S::to_canon(src[slot_index<ADDR, LAY>(a, j, c)], i, a.sigma);
        if (bc > 0 && a.bc_on) f = bc_arrive_canon(can, a.bc_neg, bc, i, f);
        m[0] += f;
        if (cx(i) > 0) m[1] += f;
        if (cx(i) < 0) m[1] -= f;
        if (cy(i) > 0) m[2] += f;
        if (cy(i) < 0) m[2] -= f;
        if (cz(i) > 0) m[3] += f;
        if (cz(i) < 0) m[3] -= f;
    }
}

template <int ADDR, int LAY, int PREC, int R>
__global__ void __launch_bounds__(BLOCK) k_reduce(KArgs a)
{
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    if (n < a.n_nodes) node_moments<ADDR, LAY, PREC, R>(a, n, m, a.bc_can);
    block_sum4(m, a.partials + 4 * (int64_t)blockIdx.x);
}

// One block: thread t sums partial blocks t, t + 256, ... in order, then the
// fixed block tree; writes out[0..3].  Defined in common.hip.
void launch_reduce_final(const double *partials, uint32_t n_blocks, double *out, hipStream_t s);

// ------------------------------------------------------------------ launch table
using Launch = void (*)(const KArgs &, uint32_t, hipStream_t);

struct PrecTable {
    Launch update[2][3][2][K_NUM]; // [addr][layout (L_SOA, L_AOS, L_BLK)][collider][kind]
    Launch pair[2][K_NUM];         // direct SoA, two nodes per lane: [collider][kind]
    Launch wide[2][2][K_NUM];      // direct SoA, one row segment per workgroup: [blocked][collider][kind]
    Launch pair_wide[2][K_NUM];    // direct SoA, two nodes per lane, 512-node row segments
    Launch gen[2][2][K_NUM];       // direct SoA, any nx, shifts through LDS: [blocked][collider][kind]
    Launch get[2][3][R_NUM];
    Launch set[2][3][R_NUM];
    Launch init[2][3][R_NUM];
    Launch reduce[2][3][R_NUM];
};

const PrecTable &table_f64();
const PrecTable &table_f32();
const PrecTable &table_f16s();
const PrecTable &table_f32s();

} // namespace lbm

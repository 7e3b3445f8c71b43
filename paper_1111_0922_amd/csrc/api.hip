// api.hip -- the C ABI of lbm355.h: validation, buffer bookkeeping and
// dispatch of the kernel instantiations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/lbm355.h"
#include "common.hpp"
#include "grid_internal.hpp"

using namespace lbm;

namespace {
thread_local std::string g_err;
}

namespace lbm_host {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_check(hipError_t e, const char *where)
{
    if (e == hipSuccess) return LBM_OK;
    return fail(LBM_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

} // namespace lbm_host

using namespace lbm_host;

namespace {

constexpr int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int pdf_size(int precision) { return precision == LBM_F64 ? 8 : (precision == LBM_F16S ? 2 : 4); }

bool two_lattices(int scheme) { return scheme == LBM_TS || scheme == LBM_OS_PUSH || scheme == LBM_OS_PULL; }
bool kernel_scheme(int scheme) { return scheme >= LBM_TS && scheme <= LBM_ET; }

} // namespace


namespace {

// byte offset of the slab keys in the build scratch (after the chunk counts and offsets)
int64_t order_key_offset(int64_t chunk_blocks)
{
    return round_up(round_up(chunk_blocks * 2 * 4, 256) + (2 * chunk_blocks + 2) * 8, 256);
}

// fluid ids in plain lexicographic order (no brick of desc.brick smaller than the box)
bool lexicographic(const lbm_grid *g)
{
    const int32_t dims[3] = {g->d.nx, g->d.ny, g->d.nz};
    for (int k = 0; k < 3; ++k)
        if (g->d.brick[k] > 0 && g->d.brick[k] < dims[k]) return false;
    return true;
}

int64_t rank_words_count(const lbm_grid *g) { return (g->n_cells + 31) / 32; }

// log2 of the nodes per block of a SoA lattice of `scheme` (slot_index, L_BLK), 0
// for plain SoA.  Defaults (blocks of 1024 nodes or cells where measured faster):
//  - indirect grids, FP64, every scheme.  512^3 pack, per launch (plain ->
//    1024): AA even 2.76-2.79 -> 2.60 ms, odd 3.85-3.88 -> 3.75, two-step 6.18
//    -> 5.72-5.76 per step, one-step pull 3.12-3.30 -> 3.06-3.10; one-step push
//    and the esoteric twist within their run-to-run spread;
//  - indirect grids, FP32 and FP32-shifted storage, every scheme.  512^3 pack
//    with neighbour ids by rank, FP32 (per launch): AA even 1.37-1.38 -> 1.24
//    ms, odd 2.27 -> 2.18; two-step 3.40-3.44 -> 3.13-3.15; one-step push 2.23
//    -> 2.12, pull 2.02-2.04 -> 1.81-1.91; esoteric twist 2.43 -> 2.33.  With
//    IDX the AA pattern is level (even 1.39 -> 1.25, odd 2.35 -> 2.42).  The
//    serving mix of lattices (edges 32-192, batched) runs 30.5 -> 32.6 GLUP/s;
//  - indirect grids, FP16 storage (with IDX, its default), every scheme.  512^3
//    pack: AA 36.7 -> 38.8 GLUP/s (even 0.73-0.74 -> 0.67 ms, odd 2.19-2.20 ->
//    2.11), two-step 2.40-2.42 -> 2.25-2.26 ms per step, one-step pull 1.72 ->
//    1.62-1.63 ms, push 1.85 -> 1.80-1.82, esoteric twist 2.30 -> 2.29; 384^3
//    pack AA 38.1 -> 39.3;
//  - direct grids, FP64, FP32 and FP32-shifted storage, the two-step, one-step
//    and esoteric-twist schemes.  256^3 channel, FP64 (FP32): two-step 1.67 ->
//    1.58 ms per step (0.84 -> 0.80), one-step push 0.88 -> 0.85 (0.425 ->
//    0.406), pull 0.84 -> 0.805 (0.43 -> 0.41), esoteric twist 0.86 -> 0.82
//    (0.43 -> 0.40);
//  - direct grids, the AA pattern with FP64 storage, blocks of 4096 cells where
//    they hold whole rows (nx divides 4096 or 4096 divides nx).  Per pair of
//    steps (even + odd, plain -> 1024 -> 4096): 128^3 0.246 -> 0.203 -> 0.202
//    ms, 256^3 1.66-1.68 -> 1.63 -> 1.61, 256x256x512 3.39-3.41 -> 3.32 -> 3.30,
//    512x256x256 3.63-3.64 -> 3.57-3.59 -> 3.55.  Blocks of 1024 speed up the
//    even kernel but slow the odd one (256^3: 0.85 -> 0.85-0.86 ms); at 4096
//    the odd kernel gains too (0.834).  Where rows straddle blocks the odd
//    kernel loses (384^3: 6.12-6.13 plain, 6.21 at 4096), and FP32 and FP16
//    storage keep plain SoA (FP32 odd 0.43 -> 0.49 ms at 4096).
// Pairs of nodes per lane (16-bit storage, direct grids) need plain SoA, and
// keep it by default.
int soa_block_shift(const lbm_grid *g, int scheme)
{
    if (g->d.layout != LBM_SOA) return 0;
    const bool ind = g->d.addressing == LBM_INDIRECT;
    const int p = g->d.precision;
    int64_t def = 0;
    if (ind || (scheme != LBM_AA && p != LBM_F16S)) {
        def = 1024;
    } else if (scheme == LBM_AA && p == LBM_F64) {
        const int64_t nx = g->d.nx;
        if (4096 % nx == 0 || nx % 4096 == 0) def = 4096;
    }
    const int64_t b = g->soa_block >= 0 ? g->soa_block : def;
    int sh = 0;
    while (((int64_t)1 << sh) < b) ++sh;
    return b > 0 ? sh : 0;
}

int64_t storage_nodes(const lbm_grid *g, int scheme)
{
    if (g->d.addressing == LBM_DIRECT) return g->n_cells;
    return g->n_nodes + (scheme == LBM_ET ? g->n_ghost : 0);
}

} // namespace

namespace lbm_host {

const PrecTable &table(int precision)
{
    switch (precision) {
    case LBM_F64: return table_f64();
    case LBM_F32: return table_f32();
    case LBM_F16S: return table_f16s();
    default: return table_f32s();
    }
}

int64_t idx_pitch_of(const lbm_grid *g) { return round_up(g->n_nodes > 0 ? g->n_nodes : 1, 64); }

uint32_t node_blocks(const lbm_grid *g) { return (uint32_t)((g->n_nodes + BLOCK - 1) / BLOCK); }

// storage order the kernels are instantiated for: L_SOA, L_AOS, or L_BLK for a blocked indirect SoA lattice
int kernel_layout(const lbm_grid *g) { return soa_block_shift(g, g->scheme) ? L_BLK : g->d.layout; }

// byte offset of cell_of in the IDX buffer: after the 18 IDX rows and the slab block order
int64_t rank_offset(const lbm_grid *g) { return 18 * idx_pitch_of(g) * 4 + round_up((int64_t)node_blocks(g) * 4, 256); }

// Workgroups of an update launch.
uint32_t update_blocks(const lbm_grid *g, const KArgs &a)
{
    const int64_t npb = a.pair ? 2 * BLOCK : BLOCK;
    return (uint32_t)((g->n_nodes + npb - 1) / npb);
}

// Block order of one update kernel: the banded XCD order (logical_block) when
// it applies.  By default (band < 0) AoS kernels with a neighbour side use it,
// with bands of 8 workgroups for FP64 and 16 for 4- and 2-byte storage
// (measured on the 256^3 channel: AA odd AoS 6.7 -> 3.1 ms in FP64, 3.5 ->
// 1.7 ms in FP32); SoA and node-local kernels keep the natural order, which
// the bands slow down.
void set_block_order(const lbm_grid *g, KArgs &a, int kind)
{
    a.remap = g->remap;
    if (g->d.addressing != LBM_DIRECT) {
        if (g->order && g->order_n == (int64_t)update_blocks(g, a)) {
            a.remap = 3;
            a.order = g->order;
            return;
        }
        // XCD slab order (built with the index) for the kernels that write to
        // neighbours: their partly written lines then collect in one L2 before they
        // leave it.  Measured per launch on the 512^3 pack, FP64: AA odd 4.49 ->
        // 4.24 ms (FP32 2.75 -> 2.50), one-step push 6.72 -> 5.25, esoteric twist
        // 6.10 -> 4.97.  Kernels that only gather from neighbours gain nothing
        // (one-step pull 3.83-4.00 -> 3.88, two-step 6.64 -> 6.66 per step), and
        // node-local ones lose (AA even 2.77 -> 3.06 / 1.38 -> 1.57): their natural
        // order keeps the blocks of all XCDs in the same memory pages.
        const int W = wmap_of(kind);
        const bool writes_neighbours = W == W_PUSH || W == W_ET0 || W == W_ET1;
        const int slab = g->slab >= 0 ? g->slab : (g->d.layout == LBM_SOA ? 1 : 0);
        if (slab && writes_neighbours && g->slab_table) {
            a.remap = 3;
            a.order = g->slab_table;
        }
        return;
    }
    int64_t band = g->band;
    if (band < 0) {
        const int R = rmap_of(kind), W = wmap_of(kind);
        const bool neighbour_side = !(R == R_LOCAL && (W == W_LOCAL || W == W_AAEVEN));
        band = (g->d.layout == LBM_AOS && neighbour_side) ? (g->d.precision == LBM_F64 ? 8 : 16) : 0;
    }
    if (band <= 0) return;
    const int64_t npb = a.pair ? 2 * BLOCK : BLOCK;
    const int64_t plane = (int64_t)g->d.nx * g->d.ny;
    const int64_t yb = plane / npb;
    if (plane % npb == 0 && yb % (8 * band) == 0) {
        a.remap = 2;
        a.band_yb = (uint32_t)yb;
        a.band_ty = (uint32_t)band;
        a.band_z = (uint32_t)(g->n_nodes / plane);
    }
}

// Per-kernel residency of FP64 kernels (LDS reserved only to cap the
// resident workgroups per CU; an explicit LBM_OPT_WG_LDS wins).
//  - SoA: two workgroups per CU for every kernel.  The row-staged kernels
//    (20 KB of their own) reach it with the base 44 KB; the others need a
//    64 KB reservation, which took AA even on the 256^3 channel from 0.851
//    to 0.827 ms and on the 512^3 pack from 2.97 to 2.81 ms (odd 4.59 to
//    4.48, two-step 6.9 to 6.5 ms per step).  Fewer (one per CU) slows the
//    staged kernels by 15-25%.
//  - AoS AA: the odd kernel scatters 8-byte values into 152-byte records of
//    nine rows; with every workgroup it can hold resident, the rows in
//    flight outgrow the L2 and partially written lines leave it several
//    times (3.8x the algorithmic write bytes, counters).  One workgroup per
//    CU: 3.13 -> 2.57 ms.  The even kernel (staged records, 38 KB of LDS)
//    is best at two per CU: 0.88 -> 0.81 ms.  Indirect AoS grids gain the
//    same way (256^3 pack: even 0.354 -> 0.322, odd 2.39 -> 2.02 ms).  Lower
//    residency slows the other AoS kernels, which keep full residency.
static void set_residency(const lbm_grid *g, KArgs &a, int kind)
{
    if (g->wg_lds >= 0 || a.pair) return;
    // Neighbour ids by rank (indirect SoA) wait on one more load than IDX
    // does before the gathers, which more resident workgroups cover.  512^3
    // pack: FP32 AA odd at four workgroups per CU 2.29 ms against 2.45 at
    // three (the FP32 base); FP64 one-step pull 3.32 at four against 3.47 at
    // two; FP64 one-step push 4.37 at two against 4.90 at one (its IDX
    // setting below); FP64 esoteric twist 4.53 at three against 4.65 at two.
    // The other FP64 kernels stay at two.
    if (a.rank_words && g->d.layout == LBM_SOA) {
        const bool p32 = g->d.precision == LBM_F32 || g->d.precision == LBM_F32S;
        if (p32 && kind == K_AA_ODD) a.lds_bytes = 32768;
        if (g->d.precision == LBM_F64) {
            a.lds_bytes = kind == K_OS_PULL ? 32768 : 65536;
            if (a.ghost_words && (kind == K_ET0 || kind == K_ET1)) a.lds_bytes = 45056;
        }
        return;
    }
    if (g->d.precision != LBM_F64) return;
    if (g->d.layout == LBM_SOA) {
        const bool staged = g->d.addressing == LBM_DIRECT && a.row_staged && shifts_x(kind);
        a.lds_bytes = staged ? 45056 : 65536;
        // the one-step push on indirect grids with IDX scatters all 18 moving
        // values: one workgroup per CU (512^3 pack: 5.24 -> 5.03 ms; AA odd and
        // the esoteric twist are best at two)
        if (g->d.addressing == LBM_INDIRECT && kind == K_OS_PUSH) a.lds_bytes = 98304;
    } else {
        if (kind == K_AA_ODD) a.lds_bytes = 98304;
        if (kind == K_AA_EVEN) a.lds_bytes = 20480;
    }
}

KArgs base_args(const lbm_grid *g)
{
    KArgs a;
    std::memset(&a, 0, sizeof a);
    const lbm_grid_desc &d = g->d;
    a.idx = g->idx;
    a.et = g->aux;
    a.pitch = g->pitch;
    const int bsh = soa_block_shift(g, g->scheme);
    a.bsh = (uint32_t)bsh;
    a.bmk = (1u << bsh) - 1u;
    a.idx_pitch = idx_pitch_of(g);
    a.plane = (int64_t)d.nx * d.ny;
    const int z0 = (d.addressing == LBM_DIRECT && d.wall_z) ? 1 : 0;
    a.z0 = z0;
    a.z0_offset = (int64_t)z0 * a.plane;
    a.n_nodes = (uint32_t)g->n_nodes;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.wall = (d.addressing == LBM_DIRECT) ? d.wall_z : 0;
    a.dvx = make_fastdiv((uint32_t)d.nx);
    a.dvy = make_fastdiv((uint32_t)d.ny);
    a.remap = g->remap;
    // Base reservation, measured on MI355X: FP32 likes 40 KB on direct SoA
    // grids (256^3 channel) and 52 KB on indirect ones (512^3 pack: AA even
    // -7%, odd -3% in time); FP16 wants no cap.  FP64 kernels get theirs per
    // kernel (set_residency; 44 KB is the staged SoA kernels' share).  AoS
    // kernels otherwise keep full residency (their staged records already
    // take 19-38 KB of LDS).
    int64_t lds = 0;
    if (d.layout == LBM_SOA) {
        if (d.precision == LBM_F64) lds = 45056;
        if (d.precision == LBM_F32 || d.precision == LBM_F32S) lds = d.addressing == LBM_DIRECT ? 40960 : 53248;
    }
    a.lds_bytes = (uint32_t)(g->wg_lds >= 0 ? g->wg_lds : lds); // pair kernels: see below
    // x-rows staged per workgroup: whole rows (nx a power of two dividing the
    // workgroup size) or one segment of a row (the workgroup size divides nx)
    a.row_staged = 0;
    if (d.addressing == LBM_DIRECT && d.layout == LBM_SOA && g->row_stage) {
        if (d.nx <= BLOCK && (d.nx & (d.nx - 1)) == 0) a.row_staged = 1;
        if (d.nx > BLOCK && d.nx % BLOCK == 0) a.row_staged = 2;
        if (a.row_staged == 0) a.row_staged = 3; // any other nx: shifts through LDS across rows
    }
    // two nodes per lane: nx a power of two dividing 2 * BLOCK (whole rows) or
    // a multiple of 2 * BLOCK (512-node row segments); by default for 16-bit
    // storage (measured below for the others)
    const bool pair_on = (g->pair > 0 || (g->pair < 0 && d.precision == LBM_F16S)) && bsh == 0;
    a.pair = 0;
    if (d.addressing == LBM_DIRECT && d.layout == LBM_SOA && pair_on) {
        if (d.nx >= 2 && d.nx <= 2 * BLOCK && (d.nx & (d.nx - 1)) == 0) a.pair = 1;
        if (d.nx > 2 * BLOCK && d.nx % (2 * BLOCK) == 0) a.pair = 2; // 512-node row segments
    }
    // the pair kernels' registers already hold them to two or three workgroups per CU
    if (a.pair && g->wg_lds < 0) a.lds_bytes = 0;
    a.omega = d.omega;
    a.gx = d.g[0];
    a.gy = d.g[1];
    a.gz = d.g[2];
    a.sigma = (d.precision == LBM_F16S || d.precision == LBM_F32S) ? d.f16_scale : 1.0;
    a.omega_minus = d.omega; // BGK; lbm_step sets the TRT rate
    set_collision(a);
    // open boundaries: the constant C_c[d] of each class and direction
    a.bc_on = has_open_boundaries(g) ? 1 : 0;
    // neighbour ids by rank where the arrays exist and every class is a wall; by
    // default on SoA grids with 8- and 4-byte storage.  Measured per launch on
    // the 512^3 pack (SoA, FP64 unless noted; residency as set_residency sets
    // it): AA odd 4.22 -> 3.80 ms (FP32 2.52 -> 2.24), one-step pull 3.79 ->
    // 3.32, push 5.05 -> 4.37, two-step 6.56 -> 6.10 per step.  FP16 storage
    // gains nothing (AA odd 2.18 -> 2.21 ms).
    const bool rank_default = d.layout == LBM_SOA && d.precision != LBM_F16S;
    if (g->rank_words && (g->rank > 0 || (g->rank < 0 && rank_default)) && !a.bc_on) {
        a.cell_of = g->cell_of;
        a.rank_words = g->rank_words;
        // the esoteric twist's table from the same words: by default for FP64 only
        // (512^3 pack, per launch: FP64 4.74 -> 4.53 ms at three workgroups per CU;
        // FP32 2.45 -> 2.63-2.85, slower)
        if (g->rank > 0 || d.precision == LBM_F64) a.ghost_words = g->ghost_words;
    }
    a.bc_neg = 0;
    for (int c = 0; c < 4; ++c) {
        const double rho = g->bc_rho[c], *u = g->bc_u[c];
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const bool neg = g->bc_kind[c] == LBM_BC_PRESSURE;
        if (neg) a.bc_neg |= 1u << c;
        for (int i = 0; i < Q; ++i) {
            const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
            double k = 0.0;
            if (g->bc_kind[c] == LBM_BC_VELOCITY) k = 6.0 * wd(i) * rho * cu;      // moving wall
            if (neg) k = 2.0 * wd(i) * rho * (1.0 + 4.5 * cu * cu - 1.5 * uu);      // anti-bounce-back
            a.bc_can[c][i] = k;
            // stored form: shifted values v = sigma (f - w) turn f' = s f + k into
            // v' = s v + sigma (k - (1 - s) w)
            const bool shifted = d.precision == LBM_F16S || d.precision == LBM_F32S;
            a.bc_f[c][i] = (float)(shifted ? a.sigma * (k - (neg ? 2.0 * wd(i) : 0.0)) : k);
        }
    }
    return a;
}

// read map of the state the next step consumes
int state_rmap(const lbm_grid *g)
{
    switch (g->scheme) {
    case LBM_OS_PULL: return R_PULL;
    case LBM_AA: return (g->t & 1) ? R_AAODD : R_LOCAL;
    case LBM_ET: return (g->t & 1) ? R_ET1 : R_ET0;
    default: return R_LOCAL;
    }
}

} // namespace lbm_host

namespace {

int check_bound(const lbm_grid *g)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (g->scheme < 0) return fail(LBM_E_STATE, "no buffers bound (call lbm_bind)");
    if (g->n_nodes <= 0) return fail(LBM_E_STATE, "grid has no fluid nodes");
    return LBM_OK;
}

} // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_version(void) { return 100; }

int lbm_lattice(int32_t *c, double *w, int32_t *opp_out)
{
    for (int i = 0; i < Q; ++i) {
        if (c) {
            c[3 * i] = cx(i);
            c[3 * i + 1] = cy(i);
            c[3 * i + 2] = cz(i);
        }
        if (w) w[i] = wd(i);
        if (opp_out) opp_out[i] = opp(i);
    }
    return LBM_OK;
}

int lbm_create_grid(const lbm_grid_desc *desc, lbm_grid **out)
{
    if (!desc || !out) return fail(LBM_E_ARG, "null argument");
    const lbm_grid_desc &d = *desc;
    if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return fail(LBM_E_ARG, "box sizes must be positive");
    const int64_t nc = (int64_t)d.nx * d.ny * d.nz;
    if (nc >= (int64_t)1 << 31) return fail(LBM_E_ARG, "box of %lld cells exceeds 2^31 - 1", (long long)nc);
    if (d.addressing != LBM_DIRECT && d.addressing != LBM_INDIRECT) return fail(LBM_E_ARG, "unknown addressing");
    if (d.layout != LBM_SOA && d.layout != LBM_AOS) return fail(LBM_E_ARG, "unknown layout");
    if (d.precision < LBM_F64 || d.precision > LBM_F32S) return fail(LBM_E_ARG, "unknown precision");
    if (!(d.omega > 0.0 && d.omega < 2.0)) return fail(LBM_E_ARG, "omega must lie in (0, 2)");
    if ((d.precision == LBM_F16S || d.precision == LBM_F32S) && !(d.f16_scale > 0.0))
        return fail(LBM_E_ARG, "f16_scale (sigma of the shifted forms) must be > 0");
    if (d.addressing == LBM_DIRECT && d.wall_z && d.nz < 3) return fail(LBM_E_ARG, "walls need nz >= 3");
    if (nc * Q >= ((int64_t)1 << 40)) return fail(LBM_E_ARG, "box too large");
    for (int k = 0; k < 3; ++k)
        if (d.brick[k] < 0) return fail(LBM_E_ARG, "brick sizes must be >= 0");
    lbm_grid *g = new lbm_grid();
    g->d = d;
    g->n_cells = nc;
    if (d.addressing == LBM_DIRECT) g->n_nodes = (int64_t)d.nx * d.ny * (d.nz - (d.wall_z ? 2 : 0));
    *out = g;
    return LBM_OK;
}

int lbm_destroy_grid(lbm_grid *g)
{
    delete g;
    return LBM_OK;
}

int lbm_set_params(lbm_grid *g, double omega, const double g_acc[3])
{
    if (!g || !g_acc) return fail(LBM_E_ARG, "null argument");
    if (!(omega > 0.0 && omega < 2.0)) return fail(LBM_E_ARG, "omega must lie in (0, 2)");
    g->d.omega = omega;
    for (int k = 0; k < 3; ++k) g->d.g[k] = g_acc[k];
    return LBM_OK;
}

int lbm_set_boundary(lbm_grid *g, int32_t cls, int32_t kind, double rho, const double u[3])
{
    if (!g || !u) return fail(LBM_E_ARG, "null argument");
    if (g->d.addressing != LBM_INDIRECT)
        return fail(LBM_E_UNSUPPORTED, "open boundaries are classes of the mask of an indirect grid");
    if (cls < 1 || cls > 4) return fail(LBM_E_ARG, "boundary class %d outside 1..4", cls);
    if (kind != LBM_BC_WALL && kind != LBM_BC_VELOCITY && kind != LBM_BC_PRESSURE)
        return fail(LBM_E_ARG, "unknown boundary kind %d", kind);
    if (!(rho > 0.0) || !std::isfinite(rho)) return fail(LBM_E_ARG, "boundary density must be positive");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(u[k])) return fail(LBM_E_ARG, "boundary velocity must be finite");
    g->bc_kind[cls - 1] = kind;
    g->bc_rho[cls - 1] = rho;
    for (int k = 0; k < 3; ++k) g->bc_u[cls - 1][k] = u[k];
    return LBM_OK;
}

int lbm_set_option(lbm_grid *g, int32_t option, int64_t value)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (option == LBM_OPT_XCD_REMAP) {
        g->remap = value ? 1 : 0;
        return LBM_OK;
    }
    if (option == LBM_OPT_ROW_STAGE) {
        g->row_stage = value ? 1 : 0;
        return LBM_OK;
    }
    if (option == LBM_OPT_PAIR) {
        if (value < -1 || value > 1) return fail(LBM_E_ARG, "pair must be -1, 0 or 1");
        g->pair = (int)value;
        return LBM_OK;
    }
    if (option == LBM_OPT_BAND) {
        if (value < -1 || value > 4096) return fail(LBM_E_ARG, "band height must be -1 or lie in [0, 4096] blocks");
        g->band = (int)value;
        return LBM_OK;
    }
    if (option == LBM_OPT_SLAB_ORDER) {
        if (value < -1 || value > 1) return fail(LBM_E_ARG, "slab order must be -1, 0 or 1");
        g->slab = (int)value;
        return LBM_OK;
    }
    if (option == LBM_OPT_SOA_BLOCK) {
        const bool pow2 = value >= 64 && value <= 65536 && (value & (value - 1)) == 0;
        if (!(value == -1 || value == 0 || pow2))
            return fail(LBM_E_ARG, "SoA block must be -1, 0 or a power of two in [64, 65536] nodes");
        const int before = soa_block_shift(g, g->scheme);
        g->soa_block = value;
        if (g->d.layout == LBM_SOA && soa_block_shift(g, g->scheme) != before)
            g->scheme = -1; // the lattice layout changes: bind again
        return LBM_OK;
    }
    if (option == LBM_OPT_RANK_LOOKUP) {
        if (value < -1 || value > 1) return fail(LBM_E_ARG, "rank lookup must be -1, 0 or 1");
        g->rank = (int)value;
        return LBM_OK;
    }
    if (option == LBM_OPT_WG_LDS) {
        // at most 120 KB: with a kernel's own LDS (up to 40 KB) every
        // workgroup still fits the 160 KB of a CU
        if (value < -1 || value > 122880) return fail(LBM_E_ARG, "workgroup LDS must be -1 or lie in [0, 122880] bytes");
        g->wg_lds = value;
        return LBM_OK;
    }
    if (option == LBM_OPT_PITCH_PAD) {
        if (value < 0 || value > (1 << 20)) return fail(LBM_E_ARG, "pitch pad must lie in [0, 2^20]");
        g->pitch_pad = round_up(value, 128);
        g->scheme = -1; // buffer sizes change: bind again
        return LBM_OK;
    }
    return fail(LBM_E_ARG, "unknown option %d", option);
}

int lbm_set_block_order(lbm_grid *g, const uint32_t *d_order, int64_t n_blocks)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (g->d.addressing != LBM_INDIRECT) return fail(LBM_E_UNSUPPORTED, "block-order tables are for indirect grids");
    if (!d_order) {
        g->order = nullptr;
        g->order_n = 0;
        return LBM_OK;
    }
    if (g->idx_phase < 1) return fail(LBM_E_STATE, "build the index first: the block count follows N_f");
    const int64_t nb = (int64_t)node_blocks(g);
    if (n_blocks != nb) return fail(LBM_E_ARG, "table of %lld entries for %lld node blocks", (long long)n_blocks, (long long)nb);
    g->order = d_order;
    g->order_n = n_blocks;
    return LBM_OK;
}

int lbm_query_sizes(const lbm_grid *g, int32_t scheme, lbm_sizes *out)
{
    if (!g || !out) return fail(LBM_E_ARG, "null argument");
    if (!kernel_scheme(scheme)) return fail(LBM_E_ARG, "scheme %d has no kernels", scheme);
    std::memset(out, 0, sizeof *out);
    const lbm_grid_desc &d = g->d;
    out->n_cells = g->n_cells;
    out->n_nodes = g->n_nodes;
    out->n_ghost = (scheme == LBM_ET) ? g->n_ghost : 0;
    if (d.addressing == LBM_INDIRECT) {
        out->cellmap_bytes = round_up(g->n_cells * 4, 256);
        const int32_t dims[3] = {d.nx, d.ny, d.nz};
        int64_t nv = 1;
        for (int k = 0; k < 3; ++k) {
            const int64_t bk = (d.brick[k] > 0 && d.brick[k] < dims[k]) ? d.brick[k] : dims[k];
            nv *= (dims[k] + bk - 1) / bk * bk;
        }
        const int64_t nb = (nv + IDX_CELLS - 1) / IDX_CELLS;
        // chunk counts, 64-bit offsets, then the slab keys of at most ceil(n_cells / 256) node blocks
        out->build_scratch_bytes = order_key_offset(nb) + round_up((g->n_cells + BLOCK - 1) / BLOCK * 4, 256);
        if (g->idx_phase == 0) return LBM_OK;
        out->idx_pitch = idx_pitch_of(g);
        // the 18 IDX rows, then the XCD slab block order (one entry per node block),
        // then (lexicographic numbering) cell_of and the rank words
        out->idx_bytes = rank_offset(g);
        if (lexicographic(g))
            out->idx_bytes += out->idx_pitch * 4 + round_up(rank_words_count(g) * 8, 256) * (d.et_ghosts ? 2 : 1);
        if (scheme == LBM_ET) out->aux_bytes = 7 * out->idx_pitch * 4;
    }
    const int64_t ns = storage_nodes(g, scheme);
    const int s = pdf_size(d.precision);
    const int bsh = soa_block_shift(g, scheme);
    // a blocked lattice holds whole blocks: 19 * round_up(ns, block) values
    out->pitch = round_up(ns, bsh ? std::max<int64_t>(128, (int64_t)1 << bsh) : 128) + g->pitch_pad;
    out->pdf_bytes = d.layout == LBM_SOA ? Q * out->pitch * s : round_up(ns * Q * s, 256);
    out->pdf1_bytes = two_lattices(scheme) ? out->pdf_bytes : 0;
    out->scratch_bytes = round_up((int64_t)node_blocks(g) * 4 * 8, 256);
    return LBM_OK;
}

int lbm_build_idx(lbm_grid *g, const uint8_t *d_mask, int32_t *d_cellmap, int32_t *d_idx, int32_t *d_et,
                  void *d_scratch, int64_t *n_fluid_out, void *stream)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (g->d.addressing != LBM_INDIRECT) return fail(LBM_E_STATE, "lbm_build_idx needs an indirect grid");
    if (!d_cellmap) return fail(LBM_E_ARG, "d_cellmap is required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    BuildArgs b;
    std::memset(&b, 0, sizeof b);
    b.mask = d_mask;
    b.cellmap = d_cellmap;
    b.nx = g->d.nx;
    b.ny = g->d.ny;
    b.nz = g->d.nz;
    b.dvx = make_fastdiv((uint32_t)b.nx);
    b.dvy = make_fastdiv((uint32_t)b.ny);
    b.n_cells = (uint32_t)g->n_cells;
    const int32_t dims[3] = {g->d.nx, g->d.ny, g->d.nz};
    int32_t br[3];
    for (int k = 0; k < 3; ++k) br[k] = (g->d.brick[k] > 0 && g->d.brick[k] < dims[k]) ? g->d.brick[k] : dims[k];
    b.bx = br[0];
    b.by = br[1];
    b.bz = br[2];
    b.nbx = (dims[0] + br[0] - 1) / br[0];
    b.nby = (dims[1] + br[1] - 1) / br[1];
    const int64_t nbz = (dims[2] + br[2] - 1) / br[2];
    const int64_t bv = (int64_t)br[0] * br[1] * br[2];
    const int64_t nv = (int64_t)b.nbx * b.nby * nbz * bv;
    if (nv >= ((int64_t)1 << 31)) return fail(LBM_E_ARG, "brick grid of %lld positions exceeds 2^31 - 1", (long long)nv);
    b.bv = (uint32_t)bv;
    b.n_virtual = (uint32_t)nv;
    b.dv_bv = make_fastdiv(b.bv);
    b.dv_bx = make_fastdiv((uint32_t)b.bx);
    b.dv_by = make_fastdiv((uint32_t)b.by);
    b.dv_nbx = make_fastdiv((uint32_t)b.nbx);
    b.dv_nby = make_fastdiv((uint32_t)b.nby);
    b.n_blocks = (uint32_t)((nv + IDX_CELLS - 1) / IDX_CELLS);
    b.et_on = g->d.et_ghosts ? 1 : 0;
    if (!d_idx) {
        if (!d_mask || !d_scratch) return fail(LBM_E_ARG, "d_mask and d_scratch are required");
        b.counts = static_cast<int32_t *>(d_scratch);
        b.offsets = reinterpret_cast<int64_t *>(static_cast<char *>(d_scratch) + round_up((int64_t)b.n_blocks * 2 * 4, 256));
        launch_idx_phase1(b, s);
        int rc = hip_check(hipGetLastError(), "index build (cellmap pass)");
        if (rc) return rc;
        int64_t totals[2] = {0, 0};
        rc = hip_check(hipMemcpyAsync(totals, b.offsets + 2 * (int64_t)b.n_blocks, sizeof totals, hipMemcpyDeviceToHost, s),
                       "index build (totals)");
        if (rc) return rc;
        rc = hip_check(hipStreamSynchronize(s), "index build (sync)");
        if (rc) return rc;
        g->n_nodes = totals[0];
        g->n_ghost = g->d.et_ghosts ? totals[1] : 0;
        g->idx_phase = 1;
        g->rank_built = false;
        g->scheme = -1;
        g->order = nullptr; // the block count may have changed
        g->order_n = 0;
        if (n_fluid_out) *n_fluid_out = g->n_nodes;
        return LBM_OK;
    }
    if (g->idx_phase < 1) return fail(LBM_E_STATE, "call lbm_build_idx with d_idx = NULL first");
    if (!d_mask) return fail(LBM_E_ARG, "d_mask is required (the fill pass reads the boundary classes)");
    b.idx = d_idx;
    b.et = g->d.et_ghosts ? d_et : nullptr;
    b.et_on = b.et ? 1 : 0;
    b.idx_pitch = idx_pitch_of(g);
    b.n_fluid = g->n_nodes;
    // with the scratch, the block order of the neighbour-side kernels goes after the IDX rows
    if (d_scratch && g->n_nodes > 0) {
        b.order_key = reinterpret_cast<uint32_t *>(static_cast<char *>(d_scratch) + order_key_offset(b.n_blocks));
        b.order = reinterpret_cast<uint32_t *>(d_idx + 18 * b.idx_pitch);
        b.n_tiles = node_blocks(g);
    }
    if (lexicographic(g) && g->n_nodes > 0) {
        b.cell_of = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(d_idx) + rank_offset(g));
        b.rank_words = reinterpret_cast<uint2 *>(b.cell_of + idx_pitch_of(g));
        b.n_words = (uint32_t)rank_words_count(g);
        if (g->d.et_ghosts)
            b.ghost_words = reinterpret_cast<uint2 *>(reinterpret_cast<char *>(b.rank_words) +
                                                      round_up(rank_words_count(g) * 8, 256));
    }
    launch_idx_phase2(b, s);
    int rc = hip_check(hipGetLastError(), "index build (fill pass)");
    if (rc) return rc;
    g->idx_phase = 2;
    g->order_built = b.order != nullptr;
    g->rank_built = b.rank_words != nullptr;
    if (n_fluid_out) *n_fluid_out = g->n_nodes;
    return LBM_OK;
}

int lbm_bind(lbm_grid *g, int32_t scheme, void *d_pdf0, void *d_pdf1, const int32_t *d_idx, const int32_t *d_aux,
             void *d_scratch)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (!kernel_scheme(scheme)) return fail(LBM_E_ARG, "scheme %d has no kernels", scheme);
    const bool ind = g->d.addressing == LBM_INDIRECT;
    if (ind && g->idx_phase < 2) return fail(LBM_E_STATE, "indirect grid: build the index first");
    if (ind && scheme == LBM_ET && !g->d.et_ghosts)
        return fail(LBM_E_UNSUPPORTED, "esoteric twist on an indirect grid needs et_ghosts = 1 at creation");
    if (!d_pdf0 || !d_scratch) return fail(LBM_E_ARG, "pdf0 and scratch are required");
    if (two_lattices(scheme) && !d_pdf1) return fail(LBM_E_ARG, "this scheme needs a second lattice");
    if (ind && !d_idx) return fail(LBM_E_ARG, "indirect grid needs the IDX buffer");
    if (ind && scheme == LBM_ET && !d_aux) return fail(LBM_E_ARG, "indirect esoteric twist needs the ET table");
    lbm_sizes sz;
    int rc = lbm_query_sizes(g, scheme, &sz);
    if (rc) return rc;
    g->scheme = scheme;
    g->pdf[0] = d_pdf0;
    g->pdf[1] = two_lattices(scheme) ? d_pdf1 : nullptr;
    g->cur = 0;
    g->idx = ind ? d_idx : nullptr;
    g->slab_table = (ind && g->order_built) ? reinterpret_cast<const uint32_t *>(d_idx + 18 * idx_pitch_of(g)) : nullptr;
    g->cell_of = nullptr;
    g->rank_words = nullptr;
    g->ghost_words = nullptr;
    if (ind && g->rank_built) {
        g->cell_of = reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(d_idx) + rank_offset(g));
        g->rank_words = reinterpret_cast<const uint2 *>(g->cell_of + idx_pitch_of(g));
        if (g->d.et_ghosts)
            g->ghost_words = reinterpret_cast<const uint2 *>(reinterpret_cast<const char *>(g->rank_words) +
                                                             round_up(rank_words_count(g) * 8, 256));
    }
    g->aux = (ind && scheme == LBM_ET) ? d_aux : nullptr;
    g->scratch = static_cast<double *>(d_scratch);
    g->pitch = sz.pitch;
    g->t = 0;
    return LBM_OK;
}

int lbm_set_pdfs(lbm_grid *g, const double *d_canon, void *stream)
{
    int rc = check_bound(g);
    if (rc) return rc;
    if (!d_canon) return fail(LBM_E_ARG, "null canonical array");
    KArgs a = base_args(g);
    a.dst = g->pdf[g->cur];
    a.canon_in = d_canon;
    table(g->d.precision).set[g->d.addressing][kernel_layout(g)][state_rmap(g)](a, node_blocks(g), static_cast<hipStream_t>(stream));
    return hip_check(hipGetLastError(), "lbm_set_pdfs");
}

int lbm_get_pdfs(const lbm_grid *g, double *d_canon, void *stream)
{
    int rc = check_bound(g);
    if (rc) return rc;
    if (!d_canon) return fail(LBM_E_ARG, "null canonical array");
    KArgs a = base_args(g);
    a.src = g->pdf[g->cur];
    a.canon = d_canon;
    table(g->d.precision).get[g->d.addressing][kernel_layout(g)][state_rmap(g)](a, node_blocks(g), static_cast<hipStream_t>(stream));
    return hip_check(hipGetLastError(), "lbm_get_pdfs");
}

int lbm_init_equilibrium(lbm_grid *g, const double *d_rho_u, void *stream)
{
    int rc = check_bound(g);
    if (rc) return rc;
    g->t = 0;
    g->cur = 0;
    KArgs a = base_args(g);
    a.dst = g->pdf[0];
    a.rho_u = d_rho_u;
    table(g->d.precision).init[g->d.addressing][kernel_layout(g)][state_rmap(g)](a, node_blocks(g), static_cast<hipStream_t>(stream));
    return hip_check(hipGetLastError(), "lbm_init_equilibrium");
}

int lbm_step(lbm_grid *g, int32_t scheme, int32_t collider, int64_t n_steps, void *stream)
{
    int rc = check_bound(g);
    if (rc) return rc;
    if (scheme != g->scheme) return fail(LBM_E_STATE, "scheme %d requested, %d bound", scheme, g->scheme);
    if (collider != LBM_BGK && collider != LBM_IDENTITY && collider != LBM_TRT) return fail(LBM_E_ARG, "unknown collider");
    if (collider == LBM_TRT && !(g->d.trt_lambda > 0.0)) return fail(LBM_E_ARG, "TRT needs trt_lambda > 0");
    if (n_steps < 0) return fail(LBM_E_ARG, "negative step count");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PrecTable &tb = table(g->d.precision);
    const int A = g->d.addressing, L = kernel_layout(g), C = collider == LBM_IDENTITY ? 0 : 1;
    KArgs a = base_args(g);
    const uint32_t nb = update_blocks(g, a);
    const uint32_t lds_base = a.lds_bytes;
    auto launch = [&](int kind) {
        set_block_order(g, a, kind);
        a.lds_bytes = lds_base; // set_residency adjusts per kernel from the base
        set_residency(g, a, kind);
        (a.pair == 2 ? tb.pair_wide[C][kind] : a.pair ? tb.pair[C][kind]
         : a.row_staged == 2 ? tb.wide[L == L_BLK][C][kind] : a.row_staged == 3 ? tb.gen[L == L_BLK][C][kind]
         : tb.update[A][L][C][kind])(a, nb, s);
    };
    if (collider == LBM_TRT) {
        // Lambda = (1/w+ - 1/2)(1/w- - 1/2)
        a.omega_minus = 1.0 / (g->d.trt_lambda / (1.0 / g->d.omega - 0.5) + 0.5);
        set_collision(a);
    }
    for (int64_t k = 0; k < n_steps; ++k) {
        switch (g->scheme) {
        case LBM_TS:
            a.src = g->pdf[g->cur];
            a.dst = g->pdf[1 - g->cur];
            launch(K_TS_COLLIDE);
            a.src = g->pdf[1 - g->cur];
            a.dst = g->pdf[g->cur];
            launch(K_TS_STREAM);
            break;
        case LBM_OS_PUSH:
        case LBM_OS_PULL:
            a.src = g->pdf[g->cur];
            a.dst = g->pdf[1 - g->cur];
            launch(g->scheme == LBM_OS_PUSH ? K_OS_PUSH : K_OS_PULL);
            break;
        case LBM_AA:
            a.src = a.dst = g->pdf[0];
            launch((g->t & 1) ? K_AA_ODD : K_AA_EVEN);
            break;
        case LBM_ET:
            a.src = a.dst = g->pdf[0];
            launch((g->t & 1) ? K_ET1 : K_ET0);
            break;
        }
        // a refused launch (e.g. more LDS than a workgroup may hold) leaves the
        // step counter at the last step that was launched
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_check(e, "lbm_step");
        if (g->scheme == LBM_OS_PUSH || g->scheme == LBM_OS_PULL) g->cur = 1 - g->cur; // lattice swap
        ++g->t;
    }
    return LBM_OK;
}

int64_t lbm_time(const lbm_grid *g) { return g ? g->t : -1; }

int lbm_reduce_moments(lbm_grid *g, double *d_out4, void *stream)
{
    int rc = check_bound(g);
    if (rc) return rc;
    if (!d_out4) return fail(LBM_E_ARG, "null output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KArgs a = base_args(g);
    a.src = g->pdf[g->cur];
    a.partials = g->scratch;
    const uint32_t nb = node_blocks(g);
    table(g->d.precision).reduce[g->d.addressing][kernel_layout(g)][state_rmap(g)](a, nb, s);
    launch_reduce_final(g->scratch, nb, d_out4, s);
    return hip_check(hipGetLastError(), "lbm_reduce_moments");
}

int lbm_stream_copy(const void *d_src, void *d_dst, int64_t bytes, void *stream)
{
    if (!d_src || !d_dst || bytes < 0 || (bytes & 15) || ((uintptr_t)d_src & 15) || ((uintptr_t)d_dst & 15))
        return fail(LBM_E_ARG, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    launch_stream_copy(d_src, d_dst, bytes, static_cast<hipStream_t>(stream));
    return hip_check(hipGetLastError(), "lbm_stream_copy");
}

double lbm_model_bytes(int32_t scheme, int32_t addressing, int32_t precision, int32_t model)
{
    const int q = Q;
    const bool ind = addressing == LBM_INDIRECT;
    if (addressing != LBM_DIRECT && addressing != LBM_INDIRECT) return -1.0;
    if (model == 0) {
        // Tables 1-6: PDF transfers (loads, stores, write-allocates) and IDX loads per LUP
        double pdfs, idxs;
        switch (scheme) {
        case LBM_TS: pdfs = 6 * q; idxs = 2 * (q - 1); break;
        case LBM_OS_PUSH:
        case LBM_OS_PULL: pdfs = 3 * q; idxs = q - 1; break;
        case LBM_OS_NT: pdfs = 2 * q; idxs = q - 1; break;
        case LBM_CG: pdfs = 3 * q - 1; idxs = q - 1; break;
        case LBM_SWAP: pdfs = 3 * q - 1; idxs = (q - 1) / 2.0; break;
        case LBM_AA: pdfs = 2 * q; idxs = (q - 1) / 2.0; break;
        case LBM_ET: pdfs = 2 * q; idxs = (q + 1) / 2.0; break;
        default: return -1.0;
        }
        return pdfs * 8.0 + (ind ? idxs * 4.0 : 0.0);
    }
    if (model == 1 || model == 2) {
        if (precision < LBM_F64 || precision > LBM_F32S) return -1.0;
        const double s = pdf_size(precision);
        // no write-allocate on the GPU: each PDF is loaded once and stored once per kernel;
        // a kernel that reads neighbour ids reads q - 1 IDX entries (model 1) or one
        // cell_of entry (model 2)
        const double nb = model == 1 ? q - 1 : 1;
        double pdfs, idxs;
        switch (scheme) {
        case LBM_TS: pdfs = 4 * q; idxs = nb; break;              // in the propagation kernel only
        case LBM_OS_PUSH:
        case LBM_OS_PULL: pdfs = 2 * q; idxs = nb; break;
        case LBM_AA: pdfs = 2 * q; idxs = nb / 2.0; break;        // on odd steps, none on even
        case LBM_ET: pdfs = 2 * q; idxs = model == 1 ? 7 : 1; break; // six storage addresses + solid mask
        default: return -1.0;
        }
        return pdfs * s + (ind ? idxs * 4.0 : 0.0);
    }
    return -1.0;
}

int lbm_lattice_block(const lbm_grid *g)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (g->scheme < 0) return fail(LBM_E_STATE, "no buffers bound (call lbm_bind)");
    const int sh = soa_block_shift(g, g->scheme);
    return sh ? 1 << sh : 0;
}

int lbm_rank_lookup_active(const lbm_grid *g)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (g->scheme < 0) return fail(LBM_E_STATE, "no buffers bound (call lbm_bind)");
    const KArgs a = base_args(g);
    return (a.rank_words ? 1 : 0) | (a.ghost_words ? 2 : 0);
}

} // extern "C"

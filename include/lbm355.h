/*
 * lbm355.h -- C ABI of the MI355X (gfx950) D3Q19 lattice Boltzmann node-update library.
 *
 * The library implements the fused collide-and-propagate update of the
 * propagation schemes compared by Wittmann, Zeiser, Hager and Wellein,
 * "Comparison of different Propagation Steps for the Lattice Boltzmann
 * Method":
 *   - two-step two-grid (Sec. 2, Table 1),
 *   - one-step two-grid, push and pull (Sec. 3, Fig. 1, Table 2),
 *   - AA pattern, separate even and odd kernels (Sec. 6, Fig. 5, Table 5),
 *   - esoteric twist (Sec. 7, Fig. 6, Table 6),
 * each on a directly addressed full grid and on an indirectly addressed
 * sparse grid of fluid nodes with an 18-entry neighbour index array (Sec. 1),
 * in SoA and AoS layouts (Sec. 1).  The collision is BGK with the Guo body
 * force, or the two-relaxation-time (TRT) collision of the paper's solver
 * (Sec. 10) with the same force; PDFs are stored in FP64, FP32, or as shifted
 * deviations (f_i - w_i) * sigma in FP16 or FP32 (FP32 arithmetic).
 *
 * Conventions shared by every call:
 *   - All functions return an int status (LBM_OK or a negative LBM_E_*);
 *     lbm_last_error() gives the text of the last failure on the calling
 *     thread.  No C++ exception crosses this boundary.
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     current device).  All device memory is owned by the caller; the library
 *     never allocates device memory.  Host pointers are plain host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on it, asynchronously, unless the call
 *     says it synchronises.  Launch errors are reported by the launching call;
 *     asynchronous faults surface at the caller's next synchronisation.
 *   - Canonical PDF arrays are FP64 [19][n_nodes] (row i = direction i of the
 *     ordering below).  For a direct grid the nodes are the fluid cells in
 *     lexicographic order, x fastest (all cells, or the cells with
 *     1 <= z <= nz-2 when wall_z is set); for an indirect grid they are in
 *     the order of the fluid ids assigned by lbm_build_idx.
 *
 * D3Q19 ordering (fixed convention of this library, each moving direction
 * followed by its opposite):
 *   i :  0  1  2  3  4  5  6  7  8  9 10 11 12 13 14 15 16 17 18
 *   cx:  0  1 -1  0  0  0  0  1 -1  1 -1  1 -1  1 -1  0  0  0  0
 *   cy:  0  0  0  1 -1  0  0  1 -1 -1  1  0  0  0  0  1 -1  1 -1
 *   cz:  0  0  0  0  0  1 -1  0  0  0  0  1 -1 -1  1  1 -1 -1  1
 *   w : 1/3 for i = 0, 1/18 for i = 1..6, 1/36 for i = 7..18.
 */
#ifndef LBM355_H
#define LBM355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    LBM_OK = 0,
    LBM_E_ARG = -1,         /* invalid argument or buffer too small            */
    LBM_E_STATE = -2,       /* wrong call order, unbound buffer, scheme mismatch */
    LBM_E_HIP = -3,         /* HIP runtime error (text in lbm_last_error)      */
    LBM_E_UNSUPPORTED = -4, /* combination not provided by this build          */
    LBM_E_DIVERGED = -5     /* a lattice diverged (non-finite moments); returned
                               by lbm_batch_sync, which names the slots.  The
                               asynchronous lbm_reduce_moments reports the same
                               as a NaN mass M instead.                        */
};

/* ---------------------------------------------------------------- enums */
enum lbm_addressing { LBM_DIRECT = 0, LBM_INDIRECT = 1 };
enum lbm_layout { LBM_SOA = 0, LBM_AOS = 1 };
enum lbm_precision { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_F32S = 3 };
enum lbm_scheme {
    LBM_TS = 0,      /* two-step two-grid, Sec. 2                        */
    LBM_OS_PUSH = 1, /* one-step two-grid, push, Sec. 3                   */
    LBM_OS_PULL = 2, /* one-step two-grid, pull, Sec. 3                   */
    LBM_AA = 3,      /* AA pattern, Sec. 6                                */
    LBM_ET = 4,      /* esoteric twist, Sec. 7                            */
    /* transfer model only (lbm_model_bytes); no kernels:                 */
    LBM_OS_NT = 5,   /* one-step with non-temporal stores, Sec. 3          */
    LBM_CG = 6,      /* compressed grid, Sec. 4                            */
    LBM_SWAP = 7     /* swap algorithm, Sec. 5                             */
};
enum lbm_collider { LBM_IDENTITY = 0, LBM_BGK = 1, LBM_TRT = 2 };

/* ---------------------------------------------------------------- grid */
typedef struct lbm_grid lbm_grid;

typedef struct {
    int32_t nx, ny, nz;  /* box in cells; x is the fastest index                */
    int32_t addressing;  /* enum lbm_addressing                                  */
    int32_t layout;      /* enum lbm_layout: SoA slot (j, n) at j * pitch + n, or
                            in blocks (LBM_OPT_SOA_BLOCK); AoS at n * 19 + j     */
    int32_t precision;   /* enum lbm_precision                                   */
    int32_t wall_z;      /* DIRECT only: 1 = cell planes z = 0 and z = nz-1 are
                            solid walls (half-way bounce-back); 0 = periodic z.
                            x and y are always periodic.  INDIRECT grids are
                            periodic on all axes; solids come from the mask.   */
    int32_t et_ghosts;   /* INDIRECT only: 1 = lbm_build_idx also numbers the
                            solid cells the esoteric twist stores PDFs in.      */
    double omega;        /* BGK relaxation rate, 0 < omega < 2                   */
    double g[3];         /* body-force acceleration (force density rho * g)      */
    double f16_scale;    /* sigma of the shifted forms F16S, F32S (> 0); else ignored */
    int32_t brick[3];    /* INDIRECT only: order of the fluid numbering.  Fluid ids
                            follow bricks of brick[0] x brick[1] x brick[2] cells
                            taken in lexicographic brick order, the cells of a brick
                            lexicographically (x fastest).  0 (or the box size) in
                            every entry: plain lexicographic order.  The paper
                            compares such setups of the sparse representation
                            (Sec. 10); blocked orders keep most neighbours of a
                            workgroup's nodes in its own cache lines.             */
    int32_t reserved;    /* set to 0 */
    double trt_lambda;   /* TRT parameter Lambda = (1/w+ - 1/2)(1/w- - 1/2) > 0
                            used by the LBM_TRT collider (w+ = omega); 3/16
                            makes half-way bounce-back exact for Poiseuille flow */
} lbm_grid_desc;

typedef struct {
    int64_t n_cells;       /* nx * ny * nz                                         */
    int64_t n_nodes;       /* nodes updated per step (fluid nodes); 0 before
                              lbm_build_idx on an indirect grid                     */
    int64_t n_ghost;       /* extra storage entries of the esoteric twist           */
    int64_t pitch;         /* SoA: elements between direction arrays (blocked SoA:
                              whole blocks per direction, 19 * pitch values)        */
    int64_t idx_pitch;     /* entries between IDX rows                              */
    int64_t pdf_bytes;     /* one lattice for the queried scheme                    */
    int64_t pdf1_bytes;    /* second lattice (TS, OS push, OS pull) or 0           */
    int64_t idx_bytes;     /* int32 IDX[18][idx_pitch], the block order and (lexicographic
                              numbering) the rank-lookup arrays (indirect) or 0       */
    int64_t aux_bytes;     /* int32 ET table [7][idx_pitch] (indirect ET) or 0      */
    int64_t scratch_bytes; /* moment-reduction partials                             */
    int64_t cellmap_bytes; /* int32 cellmap[n_cells] (indirect)                     */
    int64_t build_scratch_bytes; /* scratch of lbm_build_idx                        */
} lbm_sizes;

/* Text of the last error on this thread ("" if none).  Never NULL.  No paper
 * passage: error reporting of this library. */
const char *lbm_last_error(void);

/* Library version as an integer (major * 10000 + minor * 100 + patch).  No
 * paper passage. */
int lbm_version(void);

/* The library's canonical lattice: c[19*3] (cx, cy, cz per direction),
 * w[19], opp[19].  Host pointers; any may be NULL.  Touches no GPU.  The
 * paper names the D3Q19 model (Sec. 1, Sec. 9) but prints neither velocities
 * nor weights: these are the standard D3Q19 set in this library's order. */
int lbm_lattice(int32_t *c, double *w, int32_t *opp);

/* Creates a grid from `desc` (host struct, copied).  Sec. 1: direct
 * addressing uses index arithmetic on the full box; indirect addressing keeps
 * only fluid nodes and an index array of their 18 neighbours.
 * Errors: LBM_E_ARG for non-positive sizes, n_cells >= 2^31, omega outside
 * (0, 2), an unknown enum, or f16_scale <= 0 with LBM_F16S. */
int lbm_create_grid(const lbm_grid_desc *desc, lbm_grid **out);

/* Releases the host-side descriptor.  Device buffers stay the caller's.  No
 * paper passage. */
int lbm_destroy_grid(lbm_grid *g);

/* Replaces omega and g (host values) for subsequent steps.  No paper passage:
 * the paper's solver collides with TRT (Sec. 10) and prints no operator; omega
 * and the body force g are the parameters of this library's collisions. */
int lbm_set_params(lbm_grid *g, double omega, const double g_acc[3]);

/* Open boundaries: in- and outlets (Sec. 6 counts the in-/outlet routines
 * among what the AA pattern needs in two versions).  Cells of mask value
 * cls + 1 (cls = 1..4) of an indirect grid form boundary class cls.  A
 * population f*_i that leaves fluid node x towards such a cell comes back to
 * x as direction i' = opp(i):
 *   LBM_BC_WALL      f_i' = f*_i                      (half-way bounce-back; default)
 *   LBM_BC_VELOCITY  f_i' = f*_i + 6 w_i' rho c_i'.u  (a wall moving with u: velocity inlet/outlet)
 *   LBM_BC_PRESSURE  f_i' = -f*_i + 2 w_i' rho (1 + 9/2 (c_i'.u)^2 - 3/2 u.u)
 *                    (anti-bounce-back: pressure boundary of density rho, u the
 *                    velocity in its quadratic terms, 0 for a resting reservoir)
 * The rule applies in both AA parities (odd-step gather, odd-step scatter),
 * in TS and OS, in the esoteric twist's write side (its class read from
 * IDX), in lbm_get_pdfs / lbm_set_pdfs / lbm_init_equilibrium and in the
 * moments.  Host values; takes effect at the next call.  Errors:
 * LBM_E_UNSUPPORTED on a direct grid, LBM_E_ARG for cls outside 1..4, an
 * unknown kind, rho <= 0 or a non-finite value.  Grids with open classes
 * cannot join a batch. */
enum lbm_bc_kind { LBM_BC_WALL = 0, LBM_BC_VELOCITY = 1, LBM_BC_PRESSURE = 2 };
int lbm_set_boundary(lbm_grid *g, int32_t cls, int32_t kind, double rho, const double u[3]);

/* Launch and layout options (host values; results are bit-identical for any
 * setting).  No paper passage: launch choices of this library for MI355X
 * (the paper's own tuning is CPU cache blocking and non-temporal stores,
 * Sec. 3, which these replace):
 *   LBM_OPT_XCD_REMAP (0/1, default 0): order the update kernels' workgroups
 *     so that consecutive node blocks run on the same XCD (MI355X dispatches
 *     workgroups round-robin over its 8 XCDs, each with its own L2).
 *   LBM_OPT_PITCH_PAD (elements, default 0, rounded up to a multiple of 128):
 *     padding added to the SoA pitch so that the 19 direction arrays do not
 *     start at addresses that agree in their low bits.  Changes the buffer
 *     sizes: the grid must be bound again afterwards.
 *   LBM_OPT_WG_LDS (bytes in [0, 122880], or -1 = default): dynamic LDS
 *     reserved by every update workgroup on top of what the kernel uses (up
 *     to 40 KB, so that a workgroup always fits a CU's 160 KB).  It only
 *     limits how many workgroups a CU (160 KB of LDS) keeps resident, which
 *     bounds the number of concurrent memory streams and the lines in flight
 *     per L2.  The default on SoA grids is two workgroups per CU for FP64
 *     (45056 for the kernels that stage x-rows through 20 KB of their own
 *     LDS, 65536 for the others), 40960 (direct) or 53248 (indirect) for
 *     FP32 and 0 for FP16 storage; on AoS grids it is 0, except FP64 AA:
 *     20480 for the even kernel (two workgroups per CU) and 98304 for the
 *     odd kernel (one per CU).  Indirect SoA kernels that look neighbour ids
 *     up by rank (LBM_OPT_RANK_LOOKUP) use 32768 for the FP64 one-step pull
 *     and the FP32 AA odd kernel, 45056 for the FP64 esoteric twist and 65536
 *     for the other FP64 kernels; with IDX the FP64 one-step push uses 98304.
 *   LBM_OPT_ROW_STAGE (0/1, default 1): on a direct SoA grid the x-shifted
 *     PDFs move through LDS, so that all global accesses of a wavefront are
 *     aligned: a workgroup holds whole x-rows where nx is a power of two no
 *     larger than 256, one 256-node segment of a row where nx is a multiple of
 *     256, and otherwise 256 consecutive nodes across rows (neighbours outside
 *     the workgroup in global memory); 0 forces the plain kernels.
 *   LBM_OPT_PAIR (-1 = default, 0 or 1): on a direct SoA grid whose nx is a
 *     power of two in [2, 512] or a multiple of 512 (a workgroup then holds
 *     one 512-node segment of a row), 1 makes every lane update two x-neighbours
 *     and move them as one word per direction (32, 64 or 128 bits); 0 keeps
 *     one node per lane.  The default is two nodes per lane for FP16 storage
 *     and one otherwise.
 *   LBM_OPT_BAND (blocks in [0, 4096], or -1 = default): on a direct grid
 *     whose z-plane splits into whole bands of this many workgroups for each
 *     of the 8 XCDs, order the update workgroups so that every XCD sweeps
 *     its bands along z; the neighbour rows a node reads or writes then run
 *     close in time on one L2.  Ignored when the plane does not split.  0
 *     keeps the natural order.  The default uses bands of 8 (FP64) or 16
 *     workgroups for AoS kernels that access neighbours, and the natural
 *     order otherwise.
 *   LBM_OPT_SLAB_ORDER (-1 = default, 0 or 1): on an indirect grid, 1 runs
 *     the update kernels that write to neighbours (AA odd step, one-step push,
 *     esoteric twist) in the XCD slab order that lbm_build_idx stores after
 *     the IDX rows: each XCD sweeps the node blocks whose first node lies in
 *     its own eighth of the y range, plane after plane, so the neighbour rows
 *     that share partly written cache lines run on one L2.  0 keeps the
 *     natural order.  The default is 1 on SoA grids, 0 on AoS grids.  A table
 *     set with lbm_set_block_order takes precedence.
 *   LBM_OPT_RANK_LOOKUP (-1 = default, 0 or 1): on an indirect grid numbered
 *     lexicographically (no desc.brick) whose boundary classes are all walls,
 *     1 makes the kernels that read neighbour ids compute them instead of
 *     reading IDX: the id of a fluid cell is the number of fluid cells before
 *     it, found from the node's cell (4 bytes per node) and, per 32 cells, the
 *     fluid bits and the count before them (8 bytes, shared by the neighbours
 *     of all nodes there).  IDX moves 72 bytes per node.  The esoteric
 *     twist takes its six storage addresses and its solid mask from the same
 *     words (and those of the ghost cells) instead of its 28-byte table.
 *     Ignored where it does not apply (bricked numbering, open boundaries,
 *     direct grids).
 *     The default is 1 on SoA grids with FP64, FP32 or FP32-shifted storage
 *     and 0 otherwise; by default the esoteric twist uses the words only with
 *     FP64 storage (with 4-byte storage its table measured faster).
 *   LBM_OPT_SOA_BLOCK (-1 = default, 0, or a power of two in [64, 65536]):
 *     storage order of SoA lattices.  0 is plain SoA: slot (direction j,
 *     node n) at j * pitch + n, n the fluid id (indirect) or the cell index
 *     (direct).  B > 0 cuts the nodes into blocks of B, each holding its 19
 *     directions one after the other: slot (j, n) at ((n / B) * 19 + j) * B +
 *     n mod B, so that a workgroup's accesses stay in a few memory pages.
 *     Ignored on AoS grids; on a direct grid it disables the two-nodes-per-
 *     lane kernels (LBM_OPT_PAIR).  Changes the lattice layout and sizes:
 *     the grid must be bound again afterwards.  The default is 1024 on
 *     indirect grids.  On direct grids it is 1024 for the two-step, one-step
 *     and esoteric-twist schemes with FP64, FP32 or FP32-shifted storage;
 *     4096 for the AA pattern with FP64 storage when nx divides 4096 or 4096
 *     divides nx (the blocks then hold whole rows); 0 otherwise (FP16-shifted
 *     storage keeps its two-nodes-per-lane kernels).
 * Errors: LBM_E_ARG for an unknown option or a value out of range. */
enum {
    LBM_OPT_XCD_REMAP = 1,
    LBM_OPT_PITCH_PAD = 2,
    LBM_OPT_WG_LDS = 3,
    LBM_OPT_ROW_STAGE = 4,
    LBM_OPT_PAIR = 5,
    LBM_OPT_BAND = 6,
    LBM_OPT_SLAB_ORDER = 7,
    LBM_OPT_RANK_LOOKUP = 8,
    LBM_OPT_SOA_BLOCK = 9
};
int lbm_set_option(lbm_grid *g, int32_t option, int64_t value);

/* Block order of the update kernels of an indirect grid: workgroup b updates
 * node block d_order[b] (blocks of 256 consecutive fluid ids).  d_order is a
 * caller-owned device array of n_blocks = ceil(N_f / 256) entries that must
 * stay alive while the grid steps; it must be a permutation of 0..n_blocks-1
 * (the library does not check: an entry out of range updates nothing, a
 * repeated one updates its block twice).  MI355X dispatches workgroup b to
 * XCD b mod 8, each XCD with its own L2, so the table decides which node
 * blocks share an L2 and when.  NULL restores the natural order; rebuilding
 * the index (lbm_build_idx call 1) also does.  Results are bit-identical for
 * every permutation.  Errors: LBM_E_UNSUPPORTED on a direct grid, LBM_E_STATE
 * before lbm_build_idx, LBM_E_ARG for a wrong n_blocks.  No paper passage:
 * a launch choice of this library (the paper orders the fluid nodes
 * themselves, Sec. 10; desc.brick does that here). */
int lbm_set_block_order(lbm_grid *g, const uint32_t *d_order, int64_t n_blocks);

/* Buffer sizes of `scheme` on this grid (host struct out).  For an indirect
 * grid, n_nodes, pdf/idx/aux sizes are known only after the first
 * lbm_build_idx call; before it they are 0 and cellmap_bytes /
 * build_scratch_bytes are already valid.  The sizes follow the data
 * structures of Sec. 1 (full array of all cells for direct addressing; fluid
 * nodes plus the (q-1)-entry IDX for indirect addressing) and the number of
 * lattices each scheme keeps: two for the two-step and one-step schemes
 * (Secs. 2, 3), one for the AA pattern and the esoteric twist (Secs. 6, 7). */
int lbm_query_sizes(const lbm_grid *g, int32_t scheme, lbm_sizes *out);

/* Index array of indirect addressing (Sec. 1; fluid nodes and their q-1
 * neighbours).  Two calls:
 *   1. d_idx == NULL: reads d_mask (uint8[n_cells], x fastest: 0 = fluid,
 *      1 = solid wall, 2..5 = boundary cell of class 1..4 (see
 *      lbm_set_boundary), any other non-zero value = solid wall),
 *      writes d_cellmap (int32[n_cells]): the fluid id of each fluid cell in
 *      the numbering order of desc.brick (lexicographic by default), -1 for a
 *      solid cell, or -2 - k for the solid cell holding esoteric-twist storage
 *      entry k (et_ghosts only, ghosts numbered in the same order).  Stores N_f in *n_fluid_out (host) and keeps
 *      N_f and the ghost count in the grid.  Synchronises `stream` once.
 *   2. d_idx != NULL: reads d_cellmap, writes d_idx (int32[18][idx_pitch]):
 *      IDX[k][n] = fluid id of the cell at x_n + c_{k+1} (periodic wrap), -1
 *      when that cell is a solid wall, -m for a boundary cell of mask value m.  With et_ghosts, d_et (int32[7][idx_pitch])
 *      receives the six storage addresses the esoteric twist reads at
 *      x + (1,0,0), (0,1,0), (0,0,1), (1,1,0), (1,0,1), (0,1,1) (fluid id, or
 *      N_f + ghost number for a solid cell) and, in row 6, a bit mask whose
 *      bit i-1 is set when x + c_i is solid.  When d_scratch is given, the
 *      ceil(N_f / 256) entries after the 18 IDX rows (idx_bytes covers them)
 *      receive the XCD slab block order (LBM_OPT_SLAB_ORDER); with d_scratch
 *      NULL they are left alone and the natural order is used.  On a grid
 *      numbered lexicographically the entries after that order (idx_bytes
 *      covers them) receive the arrays of LBM_OPT_RANK_LOOKUP: uint32
 *      cell_of[idx_pitch] (the cell x + nx (y + ny z) of every node), then per
 *      32 cells w = 0 .. ceil(n_cells / 32) - 1 a pair of uint32: bit k set
 *      when cell 32 w + k is fluid, and the fluid id of the word's first fluid
 *      cell (0 when it has none); with et_ghosts, after those words (rounded
 *      up to 256 bytes), the same pairs for the ghost cells (ghost bits, ghost
 *      number of the group's first ghost).  Asynchronous.
 * d_mask is read by both calls.  d_scratch: build_scratch_bytes of device
 * memory.  Errors: LBM_E_STATE on a direct grid or when call 2 precedes call
 * 1; LBM_E_ARG for a missing d_cellmap, or a missing d_mask (either call) or
 * d_scratch (call 1). */
int lbm_build_idx(lbm_grid *g, const uint8_t *d_mask, int32_t *d_cellmap, int32_t *d_idx,
                  int32_t *d_et, void *d_scratch, int64_t *n_fluid_out, void *stream);

/* Binds the caller's device buffers for `scheme` (sizes from
 * lbm_query_sizes) and resets the step counter t to 0.  Secs. 2 and 3: the
 * two-step and one-step schemes alternate between two lattices; Secs. 6 and
 * 7: the AA pattern and the esoteric twist update one lattice in place.  pdf1 is required for
 * TS and OS, ignored otherwise; idx is required for indirect grids; aux is
 * the ET table (indirect ET only); scratch holds reduction partials.
 * The PDF contents are undefined until lbm_set_pdfs or lbm_init_equilibrium.
 * Errors: LBM_E_ARG for a missing buffer, LBM_E_STATE before the indirect
 * index is built, LBM_E_UNSUPPORTED for ET on an indirect grid created
 * without et_ghosts. */
int lbm_bind(lbm_grid *g, int32_t scheme, void *d_pdf0, void *d_pdf1, const int32_t *d_idx,
             const int32_t *d_aux, void *d_scratch);

/* Uploads a canonical FP64 state d_canon[19][n_nodes] into the bound scheme's
 * layout (the inverse of the scheme's next read, so that the next step sees
 * exactly these f_i), rounding to the storage precision (FP16S stores
 * (f_i - w_i) * sigma rounded to nearest).  Asynchronous.  The layouts it
 * inverts are the paper's: the one-step pull lattice holds post-collision
 * values (Sec. 3, Fig. 1(c, d)), the AA lattice after an odd step holds them
 * in the opposite slots (Sec. 6, Fig. 5), the esoteric twist's direction
 * table flips with the parity (Sec. 7).  The canonical transfer itself has no
 * paper passage (state exchange and checkpoints of this library). */
int lbm_set_pdfs(lbm_grid *g, const double *d_canon, void *stream);

/* Reads the canonical FP64 state f(t) into d_canon[19][n_nodes]: the values
 * the next step of the bound scheme will read (for the one-step pull scheme
 * this applies the pending propagation, Sec. 3 / Fig. 1(c); for the AA
 * pattern after an odd number of steps the odd-step gather, Sec. 6 / Fig. 5;
 * for the esoteric twist the parity's direction table, Sec. 7).  The readout
 * itself has no paper passage (state exchange and checkpoints of this
 * library).  Asynchronous. */
int lbm_get_pdfs(const lbm_grid *g, double *d_canon, void *stream);

/* f = f^eq(rho, u) per node from d_rho_u[4][n_nodes] (rho, ux, uy, uz), or the
 * rest state rho = 1, u = 0 when d_rho_u is NULL; resets t to 0.
 * Asynchronous.  No paper passage (the paper prints no initial condition):
 * the equilibrium of this library's BGK collision, stored in the bound
 * scheme's layout. */
int lbm_init_equilibrium(lbm_grid *g, const double *d_rho_u, void *stream);

/* Advances the bound state by n_steps time steps of `scheme` (must be the
 * bound scheme: LBM_E_STATE otherwise).  Per step: TS launches its collision
 * and propagation kernels (Sec. 2); OS push/pull one fused kernel followed by
 * the lattice swap (Sec. 3); AA the even kernel at even t and the odd kernel
 * at odd t (Sec. 6); ET one kernel with the parity's direction table, the
 * swap of opposing directions being the parity flip (Sec. 7).  LBM_BGK
 * relaxes every non-equilibrium part with omega; LBM_TRT relaxes the parts
 * even in c with w+ = omega and the odd parts with w- = 1/(Lambda/(1/omega -
 * 1/2) + 1/2), Lambda = desc.trt_lambda (LBM_E_ARG unless > 0); the force
 * term is split the same way.  LBM_IDENTITY replaces the collision by the
 * identity (pure propagation).  Asynchronous.  A launch the device refuses
 * returns LBM_E_HIP with the step counter at the last step launched. */
int lbm_step(lbm_grid *g, int32_t scheme, int32_t collider, int64_t n_steps, void *stream);

/* Number of completed time steps since bind/set/init (its parity selects the
 * AA kernel, Sec. 6, and the esoteric twist's direction table, Sec. 7). */
int64_t lbm_time(const lbm_grid *g);

/* FP64 moments of the canonical state: d_out4 = {M, Jx, Jy, Jz} with
 * M = sum_n sum_i f_i and J = sum_n sum_i c_i f_i (raw; the mean velocity
 * adds M g / 2).  Deterministic: per-node FP64 sums, a fixed-shape tree per
 * block of 256 nodes, then one fixed-order final pass.  A NaN anywhere makes
 * M NaN.  Uses the bound scratch.  Asynchronous.  No paper passage: mass and
 * mean velocity decide convergence and permeability in this library. */
int lbm_reduce_moments(lbm_grid *g, double *d_out4, void *stream);

/* For callers that cannot allocate device memory or bring a workspace (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): lbm_reduce_moments with its per-block partials in a
 * library-owned static device array instead of the bound scratch buffer.
 * Same kernels, same block shape, hence the same bits as lbm_reduce_moments.
 * The call allocates nothing.  The array holds LBM_NOALLOC_MAX_NODES / 256
 * partials of 4 doubles (8 MiB); each GPU the library runs on keeps its own
 * copy until the process ends.  The first call on a device looks the array's
 * address up (hipGetSymbolAddress, with that device current): make that first
 * call outside stream capture.  Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (different streams, or threads)
 * race; serialise them.  Errors: LBM_E_ARG for a grid of more than
 * LBM_NOALLOC_MAX_NODES nodes (refused before any device work) or a null
 * pointer, LBM_E_STATE as lbm_reduce_moments.  Asynchronous. */
#define LBM_NOALLOC_MAX_NODES (1 << 26)
int lbm_reduce_moments_noalloc(lbm_grid *g, double *d_out4, void *stream);

/* ---------------------------------------------------------------- batches
 * Continuous batching of porous-media solves: many lattices of uneven sizes
 * (indirect SoA grids bound to the AA pattern, one storage precision) share
 * one batched AA kernel, one workgroup per tile.  A device workspace holds
 * the slot table, the tile list (tiles of 256 nodes, contiguous per slot),
 * the reduction partials and the per-slot moments.  A lattice's
 * update and moments are bit-identical to running it alone with lbm_step and
 * lbm_reduce_moments.  Slots that share a batch must not be stepped through
 * lbm_step meanwhile.  Callers serialise calls on one batch. */
typedef struct lbm_batch lbm_batch;

/* Device workspace bytes for max_slots slots and max_tiles tile entries in
 * total.  A slot takes ceil(N_f / 256) tiles rounded up to a multiple of 8:
 * its tiles start at a multiple of 8, so that its node blocks meet the 8 XCDs
 * as in a single-lattice launch, and its AA odd steps run in the grid's XCD
 * slab order (LBM_OPT_SLAB_ORDER; the order lbm_build_idx stored after the
 * IDX rows, unless the option is 0 when the grid is added).
 * The batch calls have no paper passage: the serving executor is an addition
 * of this library, built on the AA pattern because it needs one lattice per
 * solve and independent node updates (Sec. 6 notes that this suits GPUs,
 * whose memory is small). */
int lbm_batch_workspace_bytes(int32_t max_slots, int64_t max_tiles, int64_t *bytes);

/* Creates a batch over the caller's workspace (device memory, at least
 * lbm_batch_workspace_bytes, alive until lbm_batch_destroy).  Creates one
 * internal HIP stream used only to capture the run graph.  No paper passage
 * (see lbm_batch_workspace_bytes). */
int lbm_batch_create(int32_t max_slots, int64_t max_tiles, int32_t precision, void *d_workspace, lbm_batch **out);

/* Destroys the batch and its capture stream; the workspace and the grids stay
 * the caller's.  No paper passage. */
int lbm_batch_destroy(lbm_batch *b);

/* Adds a grid (indirect, SoA, bound to LBM_AA, the batch's precision, state
 * initialised) in the first free slot, written to *slot_out.  The grid keeps
 * its step counter; its parity decides which AA kernel each of its nodes
 * runs; its nodes collide with BGK at the grid's omega and force, and its
 * open-boundary classes (lbm_set_boundary) apply as they are set at this
 * call, as does its neighbour-id lookup (IDX or by rank, LBM_OPT_RANK_LOOKUP).
 * Errors: LBM_E_STATE when no slot or tile space is left,
 * LBM_E_UNSUPPORTED for other grid kinds.  No paper passage; each slot runs
 * the even and odd kernels of the AA pattern (Sec. 6). */
int lbm_batch_add(lbm_batch *b, lbm_grid *g, int32_t *slot_out);

/* Empties a slot; the grid's state stays where it is.  No paper passage. */
int lbm_batch_remove(lbm_batch *b, int32_t slot);

/* Advances every active slot by k_steps AA time steps, then reduces each
 * slot's FP64 moments (M, Jx, Jy, Jz as lbm_reduce_moments) into the
 * workspace and, when h_moments is not NULL, copies them to h_moments
 * (pinned host memory, max_slots * 4 doubles; rows of empty slots are left
 * stale).  use_graph = 1 replays a captured graph (recaptured when k_steps,
 * h_moments or the number of tiles change); 0 launches the kernels directly;
 * 2 runs all k_steps in one cooperative launch whose workgroups (as many as
 * the device keeps resident) stride over the tiles and meet at a grid
 * barrier between steps, then reduces, and synchronises `stream` before
 * returning (LBM_E_HIP if a barrier wait exceeded its bound).  Same results
 * in every mode.  Modes 0 and 1 are asynchronous on `stream`: synchronise
 * (lbm_batch_sync) before reading h_moments.  No paper passage; the steps are
 * the AA pattern's (Sec. 6). */
int lbm_batch_run(lbm_batch *b, int32_t k_steps, double *h_moments, int32_t use_graph, void *stream);

/* Waits for the batch's work on `stream` (synchronises it), then checks the
 * moments of every slot that took part in the last lbm_batch_run: a slot whose
 * M, Jx, Jy or Jz is not finite has diverged (a NaN or an overflow somewhere
 * in its lattice).  h_status (host, max_slots entries, may be NULL) receives 1
 * for such a slot and 0 for every other.  Returns LBM_E_DIVERGED when some
 * slot diverged (lbm_last_error lists them; the other slots' results are
 * valid and unaffected, since every slot is updated and reduced on its own),
 * LBM_OK otherwise.  Slots added since the last run report 0.  No paper
 * passage: failure handling of the serving executor. */
int lbm_batch_sync(lbm_batch *b, int32_t *h_status, void *stream);

/* Copies the last run's per-slot moments (max_slots * 4 doubles) to device
 * memory d_out.  Asynchronous.  No paper passage. */
int lbm_batch_moments(lbm_batch *b, double *d_out, void *stream);

/* Plain device copy of `bytes` (multiple of 16, 16-byte aligned pointers):
 * the STREAM-copy bandwidth calibration of Table 7.  Asynchronous. */
int lbm_stream_copy(const void *d_src, void *d_dst, int64_t bytes, void *stream);

/* Memory traffic per fluid-node update (bytes/LUP) of the transfer-count
 * model of Tables 1-6 and 8.  model = 0: the paper's counts (write-allocate
 * included, 8-byte PDFs, 4-byte IDX entries, precision ignored).  model = 1:
 * GPU algorithmic bytes of this library (no write-allocate, PDF size of
 * `precision` (8, 4, 2, 4 bytes), this library's IDX use).  model = 2: as 1,
 * with the neighbour ids of indirect grids looked up by rank
 * (LBM_OPT_RANK_LOOKUP): one 4-byte cell_of entry per node update of a kernel
 * that reads neighbour ids instead of 18 IDX entries (each such launch also
 * reads the 8-byte words of ceil(n_cells / 32), not counted here as they are
 * not per node); for the esoteric twist, one cell_of entry in place of its
 * seven table entries.  Returns < 0 for combinations the model does not
 * cover. */
double lbm_model_bytes(int32_t scheme, int32_t addressing, int32_t precision, int32_t model);

/* Bit 0 set when the bound grid's kernels that read neighbour ids look them
 * up by rank (LBM_OPT_RANK_LOOKUP in effect: option, numbering, boundary
 * classes), bit 1 when the esoteric twist takes its storage addresses from
 * the same words; 0 when they read IDX and the ET table, or the grid is
 * direct.  LBM_E_ARG for a null grid, LBM_E_STATE before lbm_bind.  No paper
 * passage: reports a launch choice. */
int lbm_rank_lookup_active(const lbm_grid *g);

/* Nodes per block of the bound grid's SoA lattices (LBM_OPT_SOA_BLOCK in
 * effect for the bound scheme), 0 for plain SoA or an AoS grid.  LBM_E_ARG
 * for a null grid, LBM_E_STATE before lbm_bind.  No paper passage: reports
 * the storage order of this library's lattices. */
int lbm_lattice_block(const lbm_grid *g);

#ifdef __cplusplus
}
#endif

#endif /* LBM355_H */

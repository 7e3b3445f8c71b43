// batch.hip -- continuous batching of many indirect AA-pattern lattices.
//
// A batch holds up to max_slots lattices ("slots") of uneven sizes, each an
// lbm_grid bound to the AA pattern on an indirect SoA grid.  Their nodes are
// cut into tiles of BLOCK nodes; a device-resident tile list (slot, first
// node) and slot table drive one kernel, one workgroup per tile, that
// advances every active slot by one time step per launch, each slot with its
// own parity (the AA pattern alternates its even and odd kernels, Sec. 6).
// A run of K steps is one captured graph (K step launches, the per-slot
// moment reduction and the copy of the moments to the host); since the
// tables live in device memory it stays valid while slots come and go, and
// is captured again only when the number of tiles changes.
//
// Determinism: a slot's nodes are updated by the same per-node code as the
// single-lattice kernels, and its moments are reduced tile by tile and then
// in tile order exactly as lbm_reduce_moments does, so a lattice evolves to
// the same bits alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "grid_internal.hpp"

using namespace lbm;
using namespace lbm_host;

// Dynamic LDS reserved per workgroup of the batched update kernel, only to
// cap how many are resident per CU.  Measured on the 32 serving lattices
// (graph runs): FP64 13.95 -> 14.61 GLUP/s with 64 KB (two per CU), FP32
// 26.2 -> 27.05 with 40-52 KB; FP16 loses with any cap (34.1 -> 25.6 at
// 40 KB).  When every slot of a launch takes its odd step, FP32 storage
// reserves 32 KB (four per CU), as the single-lattice odd kernel with the
// rank lookup prefers (512^3 pack: 2.29 against 2.45 ms at three per CU).
static uint32_t batch_lds(int32_t precision, int parity)
{
    if (precision == LBM_F64) return 65536;
    if (precision == LBM_F32 || precision == LBM_F32S) return parity == 1 ? 32768 : 53248;
    return 0;
}

namespace lbm {

struct SlotDesc {
    int64_t pdf_off;     // lattice and IDX: byte offsets from the workspace
    int64_t idx_off;
    int64_t order_off;   // XCD slab block order of the grid (after its IDX rows), or NO_ORDER
    int64_t cell_off;    // neighbour ids by rank: the grid's cell_of and rank words, when rank_on
    int64_t words_off;
    int64_t plane;
    int32_t nx, ny, nz, rank_on;
    FastDiv dvx, dvy;
    int64_t pitch;
    uint32_t bsh, bmk;   // blocked SoA lattice (bsh > 0, slot_index) or plain SoA (0)
    int64_t idx_pitch;
    double sigma;        // shifted-storage scale (canonical transfer of the moments)
    CollideParams<double> cpd; // collision factors of the slot's grid (BGK)
    CollideParams<float> cpf;
    uint32_t n_nodes;
    int32_t t0;          // completed steps of the slot when the run starts
    uint32_t tile_begin; // its tiles (and reduction partials) are contiguous
    uint32_t n_tiles;
    int32_t active;
    int32_t bc_on;       // open-boundary classes, as set when the grid was added
    uint32_t bc_neg;
    int32_t pad_;
    double bc_can[4][Q];
    float bc_f[4][Q];
};

struct Tile {
    uint32_t slot, node0;
};

// A slot's tiles start at a multiple of 8 in the tile list, so that its r-th
// block runs on XCD r mod 8 as in a single-lattice launch; the gaps hold
// padding tiles, which update and reduce nothing.
constexpr uint32_t PAD_SLOT = 0xFFFFFFFFu;
constexpr int64_t NO_ORDER = -1;

// Node block of a slot's tile in an odd step: the slot's XCD slab order (the
// AA odd step writes to neighbours; see LBM_OPT_SLAB_ORDER), natural
// otherwise.
__device__ __forceinline__ uint32_t tile_node0(const SlotDesc &sd, const Tile &tl, bool odd, const char *base)
{
    if (odd && sd.order_off != NO_ORDER) {
        const uint32_t *order = reinterpret_cast<const uint32_t *>(base + sd.order_off);
        return order[tl.node0 / BLOCK] * BLOCK;
    }
    return tl.node0;
}

// A pointer read from device memory is a generic (flat) pointer to the
// compiler, which then emits flat loads and stores (they wait on both the LDS
// and the vector-memory counters).  The slot table therefore holds byte
// offsets from the workspace, and the kernels add them to the workspace
// pointer they receive as an argument: derived from a kernel argument, the
// addresses are known to be global.
// Arguments of one slot's nodes.  (Moving the slot's fields to scalar
// registers with readfirstlane lowered the kernel's VGPRs from 111 to 93 and
// made it 5% slower on the serving mix; they stay as loaded.)
template <int PREC>
__device__ __forceinline__ KArgs slot_args(const SlotDesc &sd, char *base)
{
    KArgs a;
    a.src = base + sd.pdf_off;
    a.dst = base + sd.pdf_off;
    a.idx = reinterpret_cast<const int32_t *>(base + sd.idx_off);
    a.et = nullptr;
    a.cell_of = nullptr;
    a.rank_words = nullptr;
    a.ghost_words = nullptr;
    if (sd.rank_on) {
        a.cell_of = reinterpret_cast<const uint32_t *>(base + sd.cell_off);
        a.rank_words = reinterpret_cast<const uint2 *>(base + sd.words_off);
        a.nx = sd.nx;
        a.ny = sd.ny;
        a.nz = sd.nz;
        a.plane = sd.plane;
        a.dvx = sd.dvx;
        a.dvy = sd.dvy;
    }
    a.pitch = sd.pitch;
    a.bsh = sd.bsh;
    a.bmk = sd.bmk;
    a.idx_pitch = sd.idx_pitch;
    a.n_nodes = sd.n_nodes;
    a.sigma = sd.sigma;
    if constexpr (PREC == P_F64)
        a.cpd = sd.cpd;
    else
        a.cpf = sd.cpf;
    a.remap = 0;
    // the open-boundary constants stay in the slot table: the update kernels
    // copy them to LDS (bc_table_load), the reduction reads them there
    a.bc_on = sd.bc_on;
    a.bc_neg = sd.bc_neg;
    return a;
}

// Open-boundary table of one slot for a workgroup's tile (all threads; the
// slot, hence bc_on, is uniform over the workgroup).
template <int PREC>
__device__ __forceinline__ void slot_bc_table(const SlotDesc *sdp)
{
    if (sdp->bc_on) bc_table_load<typename Store<PREC>::ct>(sdp->bc_can, sdp->bc_f);
}

// One node's AA step in its slot's storage order (uniform over the tile).
template <int PREC>
__device__ __forceinline__ void slot_update(const KArgs &a, uint32_t n, bool odd, bool blocked)
{
    if (blocked) {
        if (odd)
            update_node<A_INDIRECT, L_BLK, PREC, K_AA_ODD, 1>(a, n);
        else
            update_node<A_INDIRECT, L_BLK, PREC, K_AA_EVEN, 1>(a, n);
    } else {
        if (odd)
            update_node<A_INDIRECT, L_SOA, PREC, K_AA_ODD, 1>(a, n);
        else
            update_node<A_INDIRECT, L_SOA, PREC, K_AA_EVEN, 1>(a, n);
    }
}

// One AA time step (step k of the run) of every active slot: one workgroup
// per 256-node tile.  (A persistent grid of 8 workgroups per CU striding
// over the tile list, whose launch shape would not depend on the tile count,
// ran 13% slower on the serving mix.)
template <int PREC>
__global__ void __launch_bounds__(BLOCK) k_aa_batched(const SlotDesc *slots, const Tile *tiles, const uint32_t *hdr,
                                                       int32_t k, char *base)
{
    const uint32_t tile = blockIdx.x;
    if (tile >= hdr[0]) return;
    const Tile tl = tiles[tile];
    if (tl.slot == PAD_SLOT) return;
    const SlotDesc sd = slots[tl.slot];
    const KArgs a = slot_args<PREC>(sd, base);
    slot_bc_table<PREC>(slots + tl.slot);
    const bool odd = (sd.t0 + k) & 1;
    const uint32_t n = tile_node0(sd, tl, odd, base) + threadIdx.x;
    if (n < sd.n_nodes) slot_update<PREC>(a, n, odd, sd.bsh != 0);
}

// Grid barrier of the cooperative run (every workgroup is resident).  Words
// of the workspace header: hdr[4] arrivals, hdr[5] generation, hdr[6] set when
// a wait exceeded its bound.  Thread 0 of each workgroup reads the
// generation, then arrives; the last arrival resets the count and advances
// the generation (release), the others wait for that change.  The
// agent-scope fences write this workgroup's results back to memory before it
// arrives and drop stale lines after it leaves, as a kernel boundary does
// (each XCD has its own L2).  Waits are bounded, so every wave ends; a
// timed-out wait sets hdr[6] and the run reports an error.
constexpr uint32_t BARRIER_SPIN_LIMIT = 1u << 20;

__device__ __forceinline__ bool grid_barrier(uint32_t *hdr)
{
    __shared__ uint32_t ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *count = hdr + 4, *gen = hdr + 5, *flag = hdr + 6;
        __threadfence();
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t good = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
        if (__hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > BARRIER_SPIN_LIMIT) {
                    __hip_atomic_fetch_or(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
            }
        }
        __threadfence();
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// All k_steps steps in one cooperative launch: the workgroups stride over the
// tile list and meet at a grid barrier between steps.
template <int PREC>
__global__ void __launch_bounds__(BLOCK) k_aa_batched_coop(const SlotDesc *slots, const Tile *tiles, uint32_t *hdr,
                                                            int32_t k_steps, char *base)
{
    const uint32_t nt = hdr[0];
    for (int32_t k = 0; k < k_steps; ++k) {
        for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
            const Tile tl = tiles[tile];
            if (tl.slot == PAD_SLOT) continue;
            const SlotDesc sd = slots[tl.slot];
            const KArgs a = slot_args<PREC>(sd, base);
            if (sd.bc_on) {
                __syncthreads(); // the previous tile's links have read the table
                slot_bc_table<PREC>(slots + tl.slot);
            }
            const bool odd = (sd.t0 + k) & 1;
            const uint32_t n = tile_node0(sd, tl, odd, base) + threadIdx.x;
            if (n < sd.n_nodes) slot_update<PREC>(a, n, odd, sd.bsh != 0);
        }
        if (k + 1 < k_steps && !grid_barrier(hdr)) return;
    }
}

// Per-tile FP64 moment partials of the state after `steps` steps.
template <int PREC>
__global__ void __launch_bounds__(BLOCK) k_seg_partials(const SlotDesc *slots, const Tile *tiles, const uint32_t *hdr,
                                                         double *partials, int32_t steps, char *base)
{
    const uint32_t tile = blockIdx.x;
    if (tile >= hdr[0]) return;
    const Tile tl = tiles[tile];
    if (tl.slot == PAD_SLOT) return; // no slot reads a padding tile's partial
    const SlotDesc sd = slots[tl.slot];
    const KArgs a = slot_args<PREC>(sd, base);
    const uint32_t n = tl.node0 + threadIdx.x;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    if (n < sd.n_nodes) {
        const bool odd = (sd.t0 + steps) & 1;
        const double(*can)[Q] = slots[tl.slot].bc_can;
        if (sd.bsh != 0) {
            if (odd)
                node_moments<A_INDIRECT, L_BLK, PREC, R_AAODD>(a, n, m, can);
            else
                node_moments<A_INDIRECT, L_BLK, PREC, R_LOCAL>(a, n, m, can);
        } else {
            if (odd)
                node_moments<A_INDIRECT, L_SOA, PREC, R_AAODD>(a, n, m, can);
            else
                node_moments<A_INDIRECT, L_SOA, PREC, R_LOCAL>(a, n, m, can);
        }
    }
    block_sum4(m, partials + 4 * (int64_t)tile);
}

// One workgroup per slot: the slot's partials in tile order (as k_reduce_final).
__global__ void __launch_bounds__(BLOCK) k_seg_final(const SlotDesc *slots, const double *partials, double *moments)
{
    const SlotDesc sd = slots[blockIdx.x];
    if (!sd.active) return;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < sd.n_tiles; b += BLOCK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) m[q] += partials[4 * ((int64_t)sd.tile_begin + b) + q];
    }
    block_sum4(m, moments + 4 * (int64_t)blockIdx.x);
}

} // namespace lbm

struct lbm_batch {
    int32_t max_slots = 0;
    int64_t max_tiles = 0;
    int32_t precision = LBM_F32;
    // workspace regions (device)
    uint32_t *d_hdr = nullptr;
    SlotDesc *d_slots = nullptr;
    Tile *d_tiles = nullptr;
    double *d_partials = nullptr;
    double *d_moments = nullptr;
    // host mirror
    std::vector<SlotDesc> slots;
    std::vector<lbm_grid *> grids;
    std::vector<uint8_t> in_last_run; // slot took part in the last run (its moments row is current)
    std::vector<Tile> tiles;
    bool tiles_dirty = true;
    uint32_t hdr_host[64] = {0};
    // captured run
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_k = -1;
    uint32_t graph_blocks = 0;
    int graph_parity = -2;   // common_parity the graph's launches were captured for
    double *graph_out = nullptr;
};

namespace {

constexpr int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct WsLayout {
    int64_t hdr, slots, tiles, partials, moments, total;
};

WsLayout layout_of(int32_t max_slots, int64_t max_tiles)
{
    WsLayout w;
    w.hdr = 0;
    w.slots = 256;
    w.tiles = w.slots + rup((int64_t)max_slots * (int64_t)sizeof(SlotDesc), 256);
    w.partials = w.tiles + rup(max_tiles * (int64_t)sizeof(Tile), 256);
    w.moments = w.partials + rup(max_tiles * 32, 256);
    w.total = w.moments + rup((int64_t)max_slots * 32, 256);
    return w;
}

char *ws_base(const lbm_batch *b) { return reinterpret_cast<char *>(b->d_hdr); }

int64_t ws_offset(const lbm_batch *b, const void *p)
{
    return (int64_t)(reinterpret_cast<uintptr_t>(p) - reinterpret_cast<uintptr_t>(ws_base(b)));
}

// Workgroups of the batched launches: one per tile, the count rounded up to a
// multiple of 1/16 of its leading power of two (at most 6.25% more; the extra
// workgroups find no tile and return at once).  Admissions and retirements
// that keep the count in its bucket then reuse the captured graph instead of
// capturing and instantiating a new one.
uint32_t batch_blocks(const lbm_batch *b)
{
    const uint32_t n = b->hdr_host[0];
    if (n <= 16) return n > 0 ? n : 1u;
    const uint32_t step = (1u << (31 - __builtin_clz(n))) >> 4;
    return (n + step - 1) / step * step;
}

// Cooperative run: one launch of all steps, workgroups limited to what the
// device keeps resident at once.
template <int PREC>
int launch_coop(lbm_batch *b, int32_t k_steps, hipStream_t s)
{
    int dev = 0, cus = 0, per_cu = 0;
    int rc = hip_check(hipGetDevice(&dev), "lbm_batch_run (device)");
    if (rc) return rc;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "lbm_batch_run (CUs)");
    if (rc) return rc;
    rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_aa_batched_coop<PREC>, BLOCK, 0),
                   "lbm_batch_run (occupancy)");
    if (rc) return rc;
    const uint32_t resident = (uint32_t)std::max(1, cus * per_cu);
    const uint32_t grid = std::max(1u, std::min(b->hdr_host[0], resident));
    const SlotDesc *slots = b->d_slots;
    const Tile *tiles = b->d_tiles;
    uint32_t *hdr = b->d_hdr;
    char *base = ws_base(b);
    void *args[] = {(void *)&slots, (void *)&tiles, (void *)&hdr, (void *)&k_steps, (void *)&base};
    return hip_check(hipLaunchCooperativeKernel((const void *)k_aa_batched_coop<PREC>, dim3(grid), dim3(BLOCK), args,
                                                0, s),
                     "lbm_batch_run (cooperative launch)");
}

void launch_reduce_body(lbm_batch *b, int32_t k_steps, double *h_out, hipStream_t s);

// Parity (t mod 2) shared by every active slot at the start of the run, or -1.
int common_parity(const lbm_batch *b)
{
    int p = -2;
    for (int32_t sl = 0; sl < b->max_slots; ++sl) {
        if (!b->slots[sl].active) continue;
        const int q = b->slots[sl].t0 & 1;
        if (p == -2) p = q;
        if (p != q) return -1;
    }
    return p < 0 ? -1 : p;
}

void launch_batch_body(lbm_batch *b, int32_t k_steps, double *h_out, hipStream_t s)
{
    const uint32_t nb = batch_blocks(b);
    const int p0 = common_parity(b);
    for (int32_t k = 0; k < k_steps; ++k) {
        const uint32_t lds = batch_lds(b->precision, p0 < 0 ? -1 : (p0 + k) & 1);
        if (b->precision == LBM_F64)
            hipLaunchKernelGGL(k_aa_batched<P_F64>, dim3(nb), dim3(BLOCK), lds, s, b->d_slots, b->d_tiles,
                               b->d_hdr, k, ws_base(b));
        else if (b->precision == LBM_F32)
            hipLaunchKernelGGL(k_aa_batched<P_F32>, dim3(nb), dim3(BLOCK), lds, s, b->d_slots, b->d_tiles,
                               b->d_hdr, k, ws_base(b));
        else if (b->precision == LBM_F16S)
            hipLaunchKernelGGL(k_aa_batched<P_F16S>, dim3(nb), dim3(BLOCK), lds, s, b->d_slots, b->d_tiles,
                               b->d_hdr, k, ws_base(b));
        else
            hipLaunchKernelGGL(k_aa_batched<P_F32S>, dim3(nb), dim3(BLOCK), lds, s, b->d_slots, b->d_tiles,
                               b->d_hdr, k, ws_base(b));
    }
    launch_reduce_body(b, k_steps, h_out, s);
}

// Per-slot FP64 moments of the state after the run, and their copy to the host.
void launch_reduce_body(lbm_batch *b, int32_t k_steps, double *h_out, hipStream_t s)
{
    const uint32_t nb = batch_blocks(b);
    if (b->precision == LBM_F64)
        hipLaunchKernelGGL(k_seg_partials<P_F64>, dim3(nb), dim3(BLOCK), 0, s, b->d_slots, b->d_tiles,
                           b->d_hdr, b->d_partials, k_steps, ws_base(b));
    else if (b->precision == LBM_F32)
        hipLaunchKernelGGL(k_seg_partials<P_F32>, dim3(nb), dim3(BLOCK), 0, s, b->d_slots, b->d_tiles,
                           b->d_hdr, b->d_partials, k_steps, ws_base(b));
    else if (b->precision == LBM_F16S)
        hipLaunchKernelGGL(k_seg_partials<P_F16S>, dim3(nb), dim3(BLOCK), 0, s, b->d_slots, b->d_tiles,
                           b->d_hdr, b->d_partials, k_steps, ws_base(b));
    else
        hipLaunchKernelGGL(k_seg_partials<P_F32S>, dim3(nb), dim3(BLOCK), 0, s, b->d_slots, b->d_tiles,
                           b->d_hdr, b->d_partials, k_steps, ws_base(b));
    hipLaunchKernelGGL(k_seg_final, dim3((uint32_t)b->max_slots), dim3(BLOCK), 0, s, b->d_slots, b->d_partials,
                       b->d_moments);
    if (h_out)
        (void)hipMemcpyAsync(h_out, b->d_moments, (size_t)b->max_slots * 4 * sizeof(double), hipMemcpyDeviceToHost, s);
}

void drop_graph(lbm_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_k = -1;
    b->graph_out = nullptr;
}

} // namespace

extern "C" {

int lbm_batch_workspace_bytes(int32_t max_slots, int64_t max_tiles, int64_t *bytes)
{
    if (max_slots <= 0 || max_tiles <= 0 || !bytes) return fail(LBM_E_ARG, "max_slots and max_tiles must be positive");
    *bytes = layout_of(max_slots, max_tiles).total;
    return LBM_OK;
}

int lbm_batch_create(int32_t max_slots, int64_t max_tiles, int32_t precision, void *d_workspace, lbm_batch **out)
{
    if (max_slots <= 0 || max_tiles <= 0 || max_tiles >= ((int64_t)1 << 31) || !d_workspace || !out)
        return fail(LBM_E_ARG, "bad batch arguments");
    if (precision < LBM_F64 || precision > LBM_F32S) return fail(LBM_E_ARG, "unknown precision");
    lbm_batch *b = new lbm_batch();
    b->max_slots = max_slots;
    b->max_tiles = max_tiles;
    b->precision = precision;
    const WsLayout w = layout_of(max_slots, max_tiles);
    char *ws = static_cast<char *>(d_workspace);
    b->d_hdr = reinterpret_cast<uint32_t *>(ws + w.hdr);
    b->d_slots = reinterpret_cast<SlotDesc *>(ws + w.slots);
    b->d_tiles = reinterpret_cast<Tile *>(ws + w.tiles);
    b->d_partials = reinterpret_cast<double *>(ws + w.partials);
    b->d_moments = reinterpret_cast<double *>(ws + w.moments);
    b->slots.assign(max_slots, SlotDesc{});
    b->grids.assign(max_slots, nullptr);
    b->in_last_run.assign(max_slots, 0);
    int rc = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "lbm_batch_create (capture stream)");
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return LBM_OK;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return LBM_OK;
}

int lbm_batch_add(lbm_batch *b, lbm_grid *g, int32_t *slot_out)
{
    if (!b || !g || !slot_out) return fail(LBM_E_ARG, "null argument");
    if (g->d.addressing != LBM_INDIRECT || g->d.layout != LBM_SOA || g->scheme != LBM_AA)
        return fail(LBM_E_UNSUPPORTED, "batched lattices are indirect SoA grids bound to the AA pattern");
    if (g->d.precision != b->precision) return fail(LBM_E_ARG, "grid precision differs from the batch's");
    if (g->n_nodes <= 0) return fail(LBM_E_STATE, "grid has no fluid nodes");
    const int64_t need = (g->n_nodes + BLOCK - 1) / BLOCK;
    int64_t used = 0;
    int32_t free_slot = -1;
    for (int32_t s = 0; s < b->max_slots; ++s) {
        if (b->slots[s].active) {
            used += (b->slots[s].n_tiles + 7) / 8 * 8;
            if (b->grids[s] == g) return fail(LBM_E_STATE, "grid already in the batch (slot %d)", s);
        } else if (free_slot < 0) {
            free_slot = s;
        }
    }
    if (free_slot < 0) return fail(LBM_E_STATE, "no free slot");
    if (used + (need + 7) / 8 * 8 > b->max_tiles)
        return fail(LBM_E_STATE, "tile list full (%lld + %lld > %lld)", (long long)used, (long long)((need + 7) / 8 * 8),
                    (long long)b->max_tiles);
    SlotDesc sd;
    std::memset(&sd, 0, sizeof sd);
    const KArgs a = base_args(g);
    sd.pdf_off = ws_offset(b, g->pdf[0]);
    sd.idx_off = ws_offset(b, g->idx);
    sd.order_off = (g->slab_table && g->slab != 0) ? ws_offset(b, g->slab_table) : NO_ORDER;
    // neighbour ids by rank as the grid's own launches use them
    sd.rank_on = a.rank_words ? 1 : 0;
    sd.cell_off = a.rank_words ? ws_offset(b, a.cell_of) : 0;
    sd.words_off = a.rank_words ? ws_offset(b, a.rank_words) : 0;
    sd.plane = a.plane;
    sd.nx = a.nx;
    sd.ny = a.ny;
    sd.nz = a.nz;
    sd.dvx = a.dvx;
    sd.dvy = a.dvy;
    sd.pitch = a.pitch;
    sd.bsh = a.bsh;
    sd.bmk = a.bmk;
    sd.idx_pitch = a.idx_pitch;
    sd.sigma = a.sigma;
    sd.cpd = a.cpd;
    sd.cpf = a.cpf;
    sd.n_nodes = (uint32_t)g->n_nodes;
    sd.n_tiles = (uint32_t)need;
    sd.active = 1;
    sd.bc_on = a.bc_on;
    sd.bc_neg = a.bc_neg;
    std::memcpy(sd.bc_can, a.bc_can, sizeof sd.bc_can);
    std::memcpy(sd.bc_f, a.bc_f, sizeof sd.bc_f);
    b->slots[free_slot] = sd;
    b->grids[free_slot] = g;
    b->in_last_run[free_slot] = 0;
    b->tiles_dirty = true;
    *slot_out = free_slot;
    return LBM_OK;
}

int lbm_batch_remove(lbm_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots) return fail(LBM_E_ARG, "bad slot");
    if (!b->slots[slot].active) return fail(LBM_E_STATE, "slot %d is empty", slot);
    std::memset(&b->slots[slot], 0, sizeof(SlotDesc));
    b->grids[slot] = nullptr;
    b->in_last_run[slot] = 0;
    b->tiles_dirty = true;
    return LBM_OK;
}

int lbm_batch_run(lbm_batch *b, int32_t k_steps, double *h_moments, int32_t use_graph, void *stream)
{
    if (!b || k_steps <= 0) return fail(LBM_E_ARG, "k_steps must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // refresh the per-run fields of the slot table (parity base) and, after
    // admissions or retirements, the compacted tile list
    if (b->tiles_dirty) {
        b->tiles.clear();
        for (int32_t sl = 0; sl < b->max_slots; ++sl) {
            SlotDesc &sd = b->slots[sl];
            if (!sd.active) continue;
            while (b->tiles.size() % 8) b->tiles.push_back(Tile{PAD_SLOT, 0});
            sd.tile_begin = (uint32_t)b->tiles.size();
            for (uint32_t t = 0; t < sd.n_tiles; ++t) b->tiles.push_back(Tile{(uint32_t)sl, t * (uint32_t)BLOCK});
        }
        b->hdr_host[0] = (uint32_t)b->tiles.size();
        if (!b->tiles.empty()) {
            int rc = hip_check(hipMemcpyAsync(b->d_tiles, b->tiles.data(), b->tiles.size() * sizeof(Tile),
                                              hipMemcpyHostToDevice, s), "lbm_batch_run (tiles)");
            if (rc) return rc;
        }
        int rc = hip_check(hipMemcpyAsync(b->d_hdr, b->hdr_host, sizeof b->hdr_host, hipMemcpyHostToDevice, s),
                           "lbm_batch_run (header)");
        if (rc) return rc;
        b->tiles_dirty = false;
    }
    for (int32_t sl = 0; sl < b->max_slots; ++sl)
        if (b->slots[sl].active) b->slots[sl].t0 = (int32_t)b->grids[sl]->t;
    int rc = hip_check(hipMemcpyAsync(b->d_slots, b->slots.data(), b->slots.size() * sizeof(SlotDesc),
                                      hipMemcpyHostToDevice, s), "lbm_batch_run (slots)");
    if (rc) return rc;
    if (use_graph == 2) {
        // cooperative: all steps in one launch, then the moments; synchronous,
        // so that a timed-out barrier is reported here
        static const uint32_t zeros[3] = {0, 0, 0};
        rc = hip_check(hipMemcpyAsync(b->d_hdr + 4, zeros, sizeof zeros, hipMemcpyHostToDevice, s),
                       "lbm_batch_run (barrier words)");
        if (rc) return rc;
        if (b->precision == LBM_F64)
            rc = launch_coop<P_F64>(b, k_steps, s);
        else if (b->precision == LBM_F32)
            rc = launch_coop<P_F32>(b, k_steps, s);
        else if (b->precision == LBM_F16S)
            rc = launch_coop<P_F16S>(b, k_steps, s);
        else
            rc = launch_coop<P_F32S>(b, k_steps, s);
        if (rc) return rc;
        launch_reduce_body(b, k_steps, h_moments, s);
        rc = hip_check(hipStreamSynchronize(s), "lbm_batch_run (cooperative run)");
        if (rc) return rc;
        uint32_t timed_out = 0;
        rc = hip_check(hipMemcpy(&timed_out, b->d_hdr + 6, sizeof timed_out, hipMemcpyDeviceToHost),
                       "lbm_batch_run (barrier flag)");
        if (rc) return rc;
        if (timed_out) return fail(LBM_E_HIP, "cooperative batch run: a grid barrier wait exceeded its bound");
    } else if (use_graph) {
        if (!b->exec || b->graph_k != k_steps || b->graph_out != h_moments || b->graph_blocks != batch_blocks(b) ||
            b->graph_parity != common_parity(b)) {
            drop_graph(b);
            rc = hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "lbm_batch_run (capture)");
            if (rc) return rc;
            launch_batch_body(b, k_steps, h_moments, b->cap);
            rc = hip_check(hipStreamEndCapture(b->cap, &b->graph), "lbm_batch_run (end capture)");
            if (rc) return rc;
            rc = hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "lbm_batch_run (instantiate)");
            if (rc) {
                drop_graph(b);
                return rc;
            }
            b->graph_k = k_steps;
            b->graph_out = h_moments;
            b->graph_blocks = batch_blocks(b);
            b->graph_parity = common_parity(b);
        }
        rc = hip_check(hipGraphLaunch(b->exec, s), "lbm_batch_run (graph launch)");
        if (rc) return rc;
    } else {
        launch_batch_body(b, k_steps, h_moments, s);
        rc = hip_check(hipGetLastError(), "lbm_batch_run (launch)");
        if (rc) return rc;
    }
    for (int32_t sl = 0; sl < b->max_slots; ++sl) {
        b->in_last_run[sl] = b->slots[sl].active ? 1 : 0;
        if (b->slots[sl].active) b->grids[sl]->t += k_steps;
    }
    return LBM_OK;
}

int lbm_batch_sync(lbm_batch *b, int32_t *h_status, void *stream)
{
    if (!b) return fail(LBM_E_ARG, "null batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<double> m((size_t)b->max_slots * 4);
    int rc = hip_check(hipMemcpyAsync(m.data(), b->d_moments, m.size() * sizeof(double), hipMemcpyDeviceToHost, s),
                       "lbm_batch_sync (moments)");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "lbm_batch_sync (wait)");
    if (rc) return rc;
    std::string bad;
    int n_bad = 0;
    for (int32_t sl = 0; sl < b->max_slots; ++sl) {
        bool diverged = false;
        if (b->in_last_run[sl] && b->slots[sl].active)
            for (int q = 0; q < 4; ++q) diverged = diverged || !std::isfinite(m[4 * (size_t)sl + q]);
        if (h_status) h_status[sl] = diverged ? 1 : 0;
        if (diverged) {
            if (n_bad < 16) bad += (n_bad ? ", " : "") + std::to_string(sl);
            ++n_bad;
        }
    }
    if (n_bad)
        return fail(LBM_E_DIVERGED, "%d slot(s) diverged (non-finite moments): %s%s", n_bad, bad.c_str(),
                    n_bad > 16 ? ", ..." : "");
    return LBM_OK;
}

int lbm_batch_moments(lbm_batch *b, double *d_out, void *stream)
{
    if (!b || !d_out) return fail(LBM_E_ARG, "null argument");
    return hip_check(hipMemcpyAsync(d_out, b->d_moments, (size_t)b->max_slots * 4 * sizeof(double),
                                    hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                     "lbm_batch_moments");
}

} // extern "C"

// noalloc.hip -- lbm_reduce_moments_noalloc: the FP64 moment reduction of
// lbm_reduce_moments with its per-block partials in a library-owned device
// array instead of the scratch buffer bound to the grid.  The call allocates
// nothing, so it serves callers that cannot allocate (code under stream
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the variable's name to a kernel (on the host it is only a
// stand-in for the symbol); it looks the device address up once per device
// with hipGetSymbolAddress and passes that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm355.h"
#include "grid_internal.hpp"

using namespace lbm;
using namespace lbm_host;

namespace {

constexpr int64_t STATIC_BLOCKS = (int64_t)LBM_NOALLOC_MAX_NODES / BLOCK;
static_assert((int64_t)LBM_NOALLOC_MAX_NODES % BLOCK == 0, "whole reduction blocks");

} // namespace

// One FP64 partial (M, Jx, Jy, Jz) per 256-node block: 8 MiB per device.
static __device__ __align__(256) double scratch[STATIC_BLOCKS * 4];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device (with it current) and kept for the process.
int scratch_of_current_device(double **out)
{
    int dev = -1;
    int rc = hip_check(hipGetDevice(&dev), "lbm_reduce_moments_noalloc (device)");
    if (rc) return rc;
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_E_UNSUPPORTED, "device %d beyond the %d this library tracks", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "lbm_reduce_moments_noalloc (symbol address)");
        if (rc) return rc;
        if (!p) return fail(LBM_E_HIP, "lbm_reduce_moments_noalloc: no device address for the static partials");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

} // namespace

extern "C" int lbm_reduce_moments_noalloc(lbm_grid *g, double *d_out4, void *stream)
{
    if (!g) return fail(LBM_E_ARG, "null grid");
    if (!d_out4) return fail(LBM_E_ARG, "null output");
    // checked first, so that an oversized grid is refused before any HIP call
    if (g->n_nodes > (int64_t)LBM_NOALLOC_MAX_NODES)
        return fail(LBM_E_ARG, "%lld nodes exceed the %lld of the static reduction partials",
                    (long long)g->n_nodes, (long long)LBM_NOALLOC_MAX_NODES);
    if (g->scheme < 0) return fail(LBM_E_STATE, "no buffers bound (call lbm_bind)");
    if (g->n_nodes <= 0) return fail(LBM_E_STATE, "grid has no fluid nodes");
    double *partials = nullptr;
    int rc = scratch_of_current_device(&partials);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    KArgs a = base_args(g);
    a.src = g->pdf[g->cur];
    a.partials = partials;
    const uint32_t nb = node_blocks(g);
    // the same kernels and block shape as lbm_reduce_moments: every block
    // overwrites its partial, so nothing needs clearing between calls
    table(g->d.precision).reduce[g->d.addressing][kernel_layout(g)][state_rmap(g)](a, nb, s);
    launch_reduce_final(partials, nb, d_out4, s);
    return hip_check(hipGetLastError(), "lbm_reduce_moments_noalloc");
}

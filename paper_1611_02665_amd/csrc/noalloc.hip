// Evaluation that allocates nothing: spline_eval_noalloc.
//
// The only scratch memory an evaluation needs is the permutation of a
// cell-ordered tile (one int32 per position).  spline_eval takes it from
// stream-ordered allocation; this entry point takes it from a fixed array
// in device memory instead, so that callers which must not allocate (code
// under graph capture, tight serving loops) can still use ordered tiles.
// Every other step is spline_eval's: the same checks, kernels and results.
#include <cstdlib>
#include <mutex>

#include "internal.hpp"

namespace bspl {
namespace {

// One permutation of at most kNoAllocMaxPositions positions (4 MiB), held
// by every device the library runs on until the process ends.
constexpr int64_t kNoAllocMaxPositions = BSPL_NOALLOC_MAX_POSITIONS;
static __device__ __align__(256) int32_t scratch[kNoAllocMaxPositions];

// The array's device address, looked up once per device with that device
// current.  On the host the name `scratch` is only a stand-in for the
// symbol, so kernels and copies get this address and never the name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch[kMaxDevices] = {};

bspl_status scratch_address(int32_t** out) {
    int dev = -1;
    BSPL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(BSPL_EUNSUPPORTED, "device %d is beyond the %d devices the static scratch "
                    "memory is tracked for", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(BSPL_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch[dev] = static_cast<int32_t*>(p);
    }
    *out = g_scratch[dev];
    return BSPL_OK;
}

}  // namespace
}  // namespace bspl

using namespace bspl;

extern "C" bspl_status spline_eval_noalloc(const bspl_table* t, bspl_kind kind, int64_t npos,
                                           const double* pos, float* v, float* g, float* lh,
                                           int64_t ldo, const bspl_tile* tile, void* stream) {
    if (!t) return fail(BSPL_EINVAL, "table is NULL");
    // the caller's tile, else the BSPL_TILE override, else the built-in
    // default (no wisdom lookup: that cache lives in host containers)
    bspl_tile tl;
    if (tile) {
        tl = *tile;
    } else {
        bool bad = false;
        if (env_tile(&tl, &bad)) {
            if (bad || !tile_valid(tl, t->info.dtype))
                return fail(BSPL_EINVAL, "BSPL_TILE=\"%s\" is not a valid tile for dtype %d",
                            std::getenv("BSPL_TILE"), (int)t->info.dtype);
        } else {
            tl = default_tile(t->info, kind, npos);
        }
    }
    // the scratch limit is a host check, made before any HIP call
    if (order_sorted(tl.order) && npos > kNoAllocMaxPositions)
        return fail(BSPL_EUNSUPPORTED,
                    "a cell-ordered evaluation of %lld positions needs more than the %lld "
                    "positions of static scratch memory", (long long)npos,
                    (long long)kNoAllocMaxPositions);
    int32_t* perm = nullptr;
    if (order_sorted(tl.order) && npos > 0) {
        const bspl_status st = scratch_address(&perm);
        if (st != BSPL_OK) return st;
    }
    // eval_checked runs every other check before its first launch; with a
    // non-NULL perm an ordered tile's permutation is written there in full
    // by the ordering kernel, so nothing needs clearing between calls
    return eval_checked(t, kind, npos, pos, v, g, lh, ldo, &tl, false, perm,
                        kNoAllocMaxPositions, static_cast<hipStream_t>(stream));
}

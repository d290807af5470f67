// Memory ceiling probe: a streaming kernel with the evaluation's read/write
// mix.  A VGH evaluation on an FP32 table reads 256 bytes of coefficients
// and writes 40 bytes of outputs per orbital-eval (86 % reads), so the
// bandwidth this kernel reaches with 6 reads per write (85.7 % reads) is
// the practical ceiling to set the evaluation kernels against, next to the
// HBM3E peak.
//
// Unit i (one per lane per step) reads six 16-byte words, src[j*units + i]
// for j = 0..5 (six planes, each read coalesced across the wavefront) or,
// chunked, six consecutive 1 KiB pieces of one 6 KiB span per wavefront,
// the spans in order or drawn at random (the access statistics of
// coefficient rows gathered for random positions, cache hits included),
// and writes their sum to dst[i].  U units per lane are in flight together
// (6U loads); grid = 0 launches units / U lanes, grid > 0 that many
// persistent workgroups of 256 lanes striding over the units.
#include "internal.hpp"
#include "bspline_probe.h"

namespace bspl {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kPlanes = 6;

__device__ __forceinline__ uint4 add4(uint4 a, uint4 b) {
    return make_uint4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// The 6 KiB span a wavefront's 64 units read in random mode: span number
// hash(span, salt) mod spans (a counter hash, so spans repeat and are
// skipped at random, as the rows of random positions do).
__device__ __forceinline__ int64_t random_span(int64_t span, int64_t spans, uint64_t salt) {
    uint64_t z = (uint64_t)span * 0x9E3779B97F4A7C15ull + salt;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (int64_t)(z % (uint64_t)spans);
}

// Word j of unit i: in one of six planes (plane j holds word j of every
// unit; MODE 0), or the six words of a wavefront's 64 units forming one
// contiguous 6 KiB span, in order (MODE 1) or at a random span (MODE 2).
template <int MODE>
__device__ __forceinline__ int64_t word(int64_t i, int j, int64_t units, uint64_t salt) {
    if constexpr (MODE == 0) return (int64_t)j * units + i;
    int64_t span = i >> 6;
    if constexpr (MODE == 2) span = random_span(span, units >> 6, salt);
    return span * (64 * kPlanes) + j * 64 + (i & 63);
}

template <int U, bool NT, int MODE>
__global__ void __launch_bounds__(kProbeThreads) mix_kernel(const uint4* __restrict__ src,
                                                            uint4* __restrict__ dst,
                                                            int64_t units, uint64_t salt) {
    const int64_t lanes = (int64_t)gridDim.x * kProbeThreads;
    for (int64_t i0 = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i0 < units;
         i0 += lanes * U) {
        uint4 w[U][kPlanes];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * lanes;
            if (i < units) {
#pragma unroll
                for (int j = 0; j < kPlanes; ++j) w[u][j] = src[word<MODE>(i, j, units, salt)];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * lanes;
            if (i < units) {
                uint4 s = w[u][0];
#pragma unroll
                for (int j = 1; j < kPlanes; ++j) s = add4(s, w[u][j]);
                if constexpr (NT) {
                    __builtin_nontemporal_store(s.x, &dst[i].x);
                    __builtin_nontemporal_store(s.y, &dst[i].y);
                    __builtin_nontemporal_store(s.z, &dst[i].z);
                    __builtin_nontemporal_store(s.w, &dst[i].w);
                } else {
                    dst[i] = s;
                }
            }
        }
    }
}

template <bool NT, int MODE>
const void* pick_mix(int u) {
    switch (u) {
    case 1: return (const void*)&mix_kernel<1, NT, MODE>;
    case 2: return (const void*)&mix_kernel<2, NT, MODE>;
    case 4: return (const void*)&mix_kernel<4, NT, MODE>;
    }
    return nullptr;
}

template <bool NT>
const void* pick_mode(int u, int mode) {
    switch (mode) {
    case 0: return pick_mix<NT, 0>(u);
    case 1: return pick_mix<NT, 1>(u);
    case 2: return pick_mix<NT, 2>(u);
    }
    return nullptr;
}

}  // namespace
}  // namespace bspl

using namespace bspl;

extern "C" bspl_status spline_stream_probe(const void* src, void* dst, int64_t units,
                                           int32_t per_lane, int32_t grid, int32_t flags,
                                           uint64_t salt, void* stream) {
    if (units < 0) return fail(BSPL_EINVAL, "units %lld < 0", (long long)units);
    if (grid < 0) return fail(BSPL_EINVAL, "grid %d < 0", (int)grid);
    if ((flags & ~(BSPL_PROBE_NT_STORES | BSPL_PROBE_CHUNKED | BSPL_PROBE_RANDOM)) != 0)
        return fail(BSPL_EINVAL, "bad flags 0x%x", flags);
    const bool nt = (flags & BSPL_PROBE_NT_STORES) != 0;
    const bool ch = (flags & (BSPL_PROBE_CHUNKED | BSPL_PROBE_RANDOM)) != 0;
    const int mode = (flags & BSPL_PROBE_RANDOM) ? 2 : (ch ? 1 : 0);
    const void* fn = nt ? pick_mode<true>(per_lane, mode) : pick_mode<false>(per_lane, mode);
    if (!fn) return fail(BSPL_EINVAL, "per_lane %d is not 1, 2 or 4", (int)per_lane);
    if (ch && units % 64 != 0)
        return fail(BSPL_EINVAL, "chunked units %lld not a multiple of 64", (long long)units);
    if (units == 0) return BSPL_OK;
    if (!src || !dst) return fail(BSPL_EINVAL, "src or dst is NULL");
    if (units > INT64_MAX / (16 * kPlanes))
        return fail(BSPL_EUNSUPPORTED, "units %lld overflow the byte count", (long long)units);
    // grid = 0: enough lanes for per_lane units each (one pass, no striding)
    const int64_t per_block = (int64_t)kProbeThreads * per_lane;
    const int64_t blocks = (units + per_block - 1) / per_block;
    const int64_t g = launch_grid(blocks, grid, kProbeThreads);
    const uint4* s = static_cast<const uint4*>(src);
    uint4* d = static_cast<uint4*>(dst);
    void* args[] = {&s, &d, &units, &salt};
    BSPL_HIP(hipLaunchKernel(fn, dim3((unsigned)g), dim3(kProbeThreads), args, 0,
                             static_cast<hipStream_t>(stream)));
    return BSPL_OK;
}

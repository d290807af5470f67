// Cell-ordered evaluation: a permutation of the positions sorted by the
// Morton code of their grid cell.
//
// Positions that are close in space read many of the same table rows (a
// cell's 64 rows overlap those of every cell within +-3 in each dimension).
// Evaluating them close together in time turns those repeated row reads
// into L2 / Infinity Cache hits.  The evaluation kernels read
// perm[logical index] and still write each output at the caller's index, so
// results do not depend on the order.
//
// Each workgroup sorts one chunk of up to kOrderChunk consecutive positions
// with a bitonic sort of (key << 32 | index) pairs in LDS.
#include "internal.hpp"

namespace bspl {
namespace {

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Cell coordinate of x in [0, n) at 10-bit resolution (non-finite -> 0).
__device__ __forceinline__ uint32_t cell10(double x, double inv_delta, int n, int shift) {
    const double u = x * inv_delta;
    if (!__builtin_isfinite(u) || !(__builtin_fabs(u) < 1125899906842624.0)) return 0u;
    const double nd = (double)n;
    double w = u - nd * __builtin_floor(u / nd);
    int i = (int)__builtin_floor(w);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    return (uint32_t)i >> shift;
}

__global__ void __launch_bounds__(1024) order_kernel(const double* __restrict__ pos, int npos,
                                                     double idx_, double idy_, double idz_,
                                                     int nx, int ny, int nz, int shift,
                                                     int chunk, int32_t* __restrict__ perm) {
    extern __shared__ unsigned long long keys[];
    const int base = blockIdx.x * chunk;
    const int cnt = min(chunk, npos - base);
    for (int i = threadIdx.x; i < chunk; i += blockDim.x) {
        unsigned long long k = ~0ull;
        if (i < cnt) {
            const int p = base + i;
            const uint32_t cx = cell10(pos[p], idx_, nx, shift);
            const uint32_t cy = cell10(pos[(int64_t)npos + p], idy_, ny, shift);
            const uint32_t cz = cell10(pos[2 * (int64_t)npos + p], idz_, nz, shift);
            const uint32_t m = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
            k = ((unsigned long long)m << 32) | (uint32_t)i;
        }
        keys[i] = k;
    }
    __syncthreads();
    for (int k = 2; k <= chunk; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < chunk; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = keys[i], b = keys[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < cnt; i += blockDim.x)
        perm[base + i] = base + (int32_t)(keys[i] & 0xffffffffull);
}

}  // namespace

int order_chunk(int64_t npos) {
    int c = 64;
    while (c < npos && c < kOrderChunk) c <<= 1;
    return c;
}

void order_launch_config(const TableDesc& d, int32_t* perm, OrderLaunch* o) {
    o->pos = d.pos;
    o->npos = (int)d.npos;
    o->idx = d.inv_delta[0];
    o->idy = d.inv_delta[1];
    o->idz = d.inv_delta[2];
    o->nx = d.ncell[0];
    o->ny = d.ncell[1];
    o->nz = d.ncell[2];
    int maxn = d.ncell[0];
    if (d.ncell[1] > maxn) maxn = d.ncell[1];
    if (d.ncell[2] > maxn) maxn = d.ncell[2];
    o->shift = 0;
    while ((maxn - 1) >> o->shift >= 1024) ++o->shift;
    o->chunk = order_chunk(d.npos);
    o->perm = perm;
    o->grid = (unsigned)((d.npos + o->chunk - 1) / o->chunk);
    o->block = o->chunk < 2048 ? (unsigned)o->chunk / 2 : 1024u;
    o->shmem = (unsigned)(sizeof(unsigned long long) * o->chunk);
    void* a[] = {&o->pos, &o->npos, &o->idx, &o->idy, &o->idz, &o->nx, &o->ny, &o->nz,
                 &o->shift, &o->chunk, &o->perm};
    for (int i = 0; i < 11; ++i) o->args[i] = a[i];
}

bspl_status launch_order(const TableDesc& d, int32_t* perm, hipStream_t s) {
    if (d.npos <= 0) return BSPL_OK;
    OrderLaunch o;
    order_launch_config(d, perm, &o);
    BSPL_HIP(hipLaunchKernel(order_kernel_ptr(), dim3(o.grid), dim3(o.block), o.args, o.shmem, s));
    return BSPL_OK;
}

const void* order_kernel_ptr() { return (const void*)&order_kernel; }

}  // namespace bspl

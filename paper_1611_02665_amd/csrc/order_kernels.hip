// Cell-ordered evaluation: a permutation of the positions grouped by the
// Morton code of their cell at 16 x 16 x 16 resolution.
//
// Positions that are close in space read many of the same table rows (a
// cell's 64 rows overlap those of every cell within +-3 in each dimension).
// Evaluating them close together in time turns those repeated row reads
// into L2 / Infinity Cache hits.  The evaluation kernels read
// perm[logical index] and still write each output at the caller's index, so
// results do not depend on the order.
//
// One workgroup orders one chunk of up to kOrderChunk consecutive positions
// with a counting sort: an LDS histogram over the 4096 Morton bins (the
// atomic's return value is the position's slot in its bin), an exclusive
// scan of the histogram, and a scatter.  The order inside a bin is whatever
// the atomics gave; it affects speed only.
#include "internal.hpp"

namespace bspl {
namespace {

constexpr int kBins = 4096;        // 16^3 Morton bins
constexpr int kOrderThreads = 1024;
constexpr int kPerThread = kOrderChunk / kOrderThreads;

__device__ __forceinline__ uint32_t spread3_4(uint32_t v) {  // 4 bits -> every third bit
    v &= 0xfu;
    v = (v | (v << 4)) & 0x0c3u;
    v = (v | (v << 2)) & 0x249u;
    return v;
}

// Bin coordinate (0..15) of fractional coordinate t on a periodic axis:
// the fraction of t times 16.  The bin only steers the order (any bin is a
// valid answer), so a multiply by 1/n precomputed on the host stands in for
// the division by n, and non-finite or huge coordinates share bin 0.
__device__ __forceinline__ uint32_t bin16(double t) {
    if (!(__builtin_fabs(t) < 1125899906842624.0)) return 0u;  // NaN, inf, |t| >= 2^50
    const int b = (int)((t - __builtin_floor(t)) * 16.0);
    return (uint32_t)(b > 15 ? 15 : b);
}

// Fractional coordinates of position p: the map's rows times (x, y, z).
__device__ __forceinline__ uint32_t morton_bin(const OrderMap& map, double x, double y, double z) {
    const uint32_t bx = bin16(map.f[0][0] * x + map.f[0][1] * y + map.f[0][2] * z);
    const uint32_t by = bin16(map.f[1][0] * x + map.f[1][1] * y + map.f[1][2] * z);
    const uint32_t bz = bin16(map.f[2][0] * x + map.f[2][1] * y + map.f[2][2] * z);
    return (spread3_4(bx) << 2) | (spread3_4(by) << 1) | spread3_4(bz);
}

// Orders chunk `chunk` (kOrderChunk positions) of one table's positions.
__device__ __forceinline__ void order_chunk(const double* __restrict__ pos, int npos,
                                            const OrderMap& map, int32_t* __restrict__ perm,
                                            int chunk) {
    __shared__ uint32_t count[kBins];
    __shared__ uint32_t wsum[kOrderThreads / 64];
    const int tid = threadIdx.x;
    const int base = chunk * kOrderChunk;
    const int cnt = min(kOrderChunk, npos - base);
    for (int b = tid; b < kBins; b += kOrderThreads) count[b] = 0u;
    __syncthreads();
    // bins first (all position loads in flight together), then the
    // histogram; the atomic's return value is the position's slot in its bin
    uint32_t bin[kPerThread], slot[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int i = r * kOrderThreads + tid;
        bin[r] = 0u;
        if (i < cnt) {
            const int p = base + i;
            bin[r] = morton_bin(map, pos[p], pos[(int64_t)npos + p], pos[2 * (int64_t)npos + p]);
        }
    }
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int i = r * kOrderThreads + tid;
        slot[r] = i < cnt ? atomicAdd(&count[bin[r]], 1u) : 0u;
    }
    __syncthreads();
    // exclusive scan over the bins: thread t owns bins [4t, 4t+4)
    constexpr int kBinsPerThread = kBins / kOrderThreads;
    uint32_t local[kBinsPerThread];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kBinsPerThread; ++k) {
        local[k] = run;
        run += count[tid * kBinsPerThread + k];
    }
    // inclusive scan of the per-thread totals: within the wavefront, then
    // across the 16 wavefronts
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t wave_base = 0;
    for (int w = 0; w < wave; ++w) wave_base += wsum[w];
    const uint32_t excl = wave_base + incl - run;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBinsPerThread; ++k) count[tid * kBinsPerThread + k] = excl + local[k];
    __syncthreads();
    // scatter: logical slot -> caller's index
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int i = r * kOrderThreads + tid;
        if (i < cnt) perm[base + (int)(count[bin[r]] + slot[r])] = base + i;
    }
}


__global__ void __launch_bounds__(kOrderThreads) order_kernel(
    const double* __restrict__ pos, int npos, const OrderMap map, int32_t* __restrict__ perm) {
    order_chunk(pos, npos, map, perm, blockIdx.x);
}

// All tables of a plan in one launch: block b belongs to the table whose
// chunk range holds it (a scan over at most 16 offsets).
__global__ void __launch_bounds__(kOrderThreads) order_tables_kernel(const OrderTables o) {
    const int b = blockIdx.x;
    int t = 0;
    for (int k = 1; k < o.ntables; ++k)
        if (b >= o.chunk_begin[k]) t = k;
    const OrderItem& it = o.t[t];
    order_chunk(it.pos, it.npos, it.map, it.perm, b - o.chunk_begin[t]);
}

}  // namespace

// Fractional-coordinate map of a table: row a of the grid map over n_a.
static OrderMap fraction_map(const TableDesc& d) {
    OrderMap m;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m.f[a][b] = d.axis[a][b] / d.axis[a][3];
    return m;
}

void order_launch_config(const TableDesc& d, int32_t* perm, OrderLaunch* o) {
    o->pos = d.pos;
    o->npos = (int)d.npos;
    o->map = fraction_map(d);
    o->perm = perm;
    o->grid = (unsigned)((d.npos + kOrderChunk - 1) / kOrderChunk);
    o->block = kOrderThreads;
    o->shmem = 0;
    void* a[] = {&o->pos, &o->npos, &o->map, &o->perm};
    for (int i = 0; i < 4; ++i) o->args[i] = a[i];
}

bspl_status launch_order(const TableDesc& d, int32_t* perm, hipStream_t s) {
    if (d.npos <= 0) return BSPL_OK;
    OrderLaunch o;
    order_launch_config(d, perm, &o);
    BSPL_HIP(hipLaunchKernel(order_kernel_ptr(), dim3(o.grid), dim3(o.block), o.args, o.shmem, s));
    return BSPL_OK;
}

const void* order_kernel_ptr() { return (const void*)&order_kernel; }

const void* order_tables_kernel_ptr() { return (const void*)&order_tables_kernel; }

unsigned order_block_threads() { return kOrderThreads; }

int64_t order_tables_config(const KernelArgs<kMaxTables>& a, OrderTables* o) {
    OrderTables x{};
    int64_t chunks = 0;
    int n = 0;
    for (int i = 0; i < a.ntables; ++i) {
        const TableDesc& d = a.t[i];
        if (!d.perm || d.npos <= 0) continue;
        OrderItem& it = x.t[n];
        it.pos = d.pos;
        it.perm = const_cast<int32_t*>(d.perm);
        it.map = fraction_map(d);
        it.npos = (int)d.npos;
        x.chunk_begin[n] = (int32_t)chunks;
        chunks += (d.npos + kOrderChunk - 1) / kOrderChunk;
        ++n;
    }
    x.chunk_begin[n] = (int32_t)chunks;
    x.ntables = n;
    *o = x;
    return chunks;
}

bspl_status launch_order_tables(const OrderTables& o, hipStream_t s) {
    const int64_t chunks = o.chunk_begin[o.ntables];
    if (chunks <= 0) return BSPL_OK;
    OrderTables x = o;
    void* args[] = {&x};
    BSPL_HIP(hipLaunchKernel(order_tables_kernel_ptr(), dim3((unsigned)chunks),
                             dim3(kOrderThreads), args, 0, s));
    return BSPL_OK;
}

}  // namespace bspl

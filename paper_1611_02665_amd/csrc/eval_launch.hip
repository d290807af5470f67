// Host side of the evaluation kernels: kernel selection by dtype and the
// launches of single, batched, split and ratio evaluations.
#include "internal.hpp"

namespace bspl {

// Defined by the dtype translation units (eval_f32.hip, eval_f16.hip,
// eval_bf16.hip).
#define BSPL_DECLARE_KERNEL_TABLE(T)                                             \
    const void* eval_kernel_ptr_##T(int kind, int vw, int multi, int lattice);   \
    const void* split_kernel_ptr_##T(int kind, int vw, int lattice, int split);  \
    const void* ratio_kernel_ptr_##T(int kind, int vw, int lattice);
BSPL_DECLARE_KERNEL_TABLE(F32)
BSPL_DECLARE_KERNEL_TABLE(F16)
BSPL_DECLARE_KERNEL_TABLE(BF16)
#undef BSPL_DECLARE_KERNEL_TABLE

namespace {

const void* kernel_for(int dtype, int kind, int vw, int multi, int lattice) {
    switch (dtype) {
    case BSPL_F32: return eval_kernel_ptr_F32(kind, vw, multi, lattice);
    case BSPL_F16: return eval_kernel_ptr_F16(kind, vw, multi, lattice);
    case BSPL_BF16: return eval_kernel_ptr_BF16(kind, vw, multi, lattice);
    }
    return nullptr;
}

const void* split_kernel_for(int dtype, int kind, int vw, int lattice, int split) {
    switch (dtype) {
    case BSPL_F32: return split_kernel_ptr_F32(kind, vw, lattice, split);
    case BSPL_F16: return split_kernel_ptr_F16(kind, vw, lattice, split);
    case BSPL_BF16: return split_kernel_ptr_BF16(kind, vw, lattice, split);
    }
    return nullptr;
}

const void* ratio_kernel_for(int dtype, int kind, int vw, int lattice) {
    switch (dtype) {
    case BSPL_F32: return ratio_kernel_ptr_F32(kind, vw, lattice);
    case BSPL_F16: return ratio_kernel_ptr_F16(kind, vw, lattice);
    case BSPL_BF16: return ratio_kernel_ptr_BF16(kind, vw, lattice);
    }
    return nullptr;
}

template <int MAXT>
bspl_status launch(const void* fn, const KernelArgs<MAXT>& a, const bspl_tile& tile,
                   hipStream_t s) {
    if (!fn) return fail(BSPL_EINVAL, "no kernel for this dtype/kind/vw");
    if (a.total_groups <= 0) return BSPL_OK;
    const int64_t grid = launch_grid(a.total_groups, tile.grid, 64 * tile.wx * tile.wy);
    dim3 block(64 * tile.wx * tile.wy);
    void* args[] = {const_cast<KernelArgs<MAXT>*>(&a)};
    BSPL_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), block, args, 0, s));
    return BSPL_OK;
}

}  // namespace

int64_t split_lds_bytes(int kind, int vw, int wx, int split) {
    const int nout = kind == BSPL_V ? 1 : (kind == BSPL_VGL ? 5 : 10);
    return (int64_t)split * wx * nout * vw * 64 * (int64_t)sizeof(float);
}

bspl_status launch_single(const bspl_table* t, int kind, const TableDesc& d,
                          const bspl_tile& tile, hipStream_t s) {
    if (tile.split > 1) {
        const void* fn = split_kernel_for(t->info.dtype, kind, tile.vw, d.lattice, tile.split);
        if (!fn) return fail(BSPL_EINVAL, "no split kernel for this dtype/kind/vw/split");
        const int64_t lds = split_lds_bytes(kind, tile.vw, tile.wx, tile.split);
        if (lds > kSplitMaxLds)
            return fail(BSPL_EINVAL, "split tile needs %lld bytes of LDS (at most %d)",
                        (long long)lds, kSplitMaxLds);
        const int64_t blocks = d.npos * (int64_t)d.xgroups;
        if (blocks <= 0) return BSPL_OK;
        if (blocks > (int64_t)UINT32_MAX / (64 * tile.wx * tile.split))
            return fail(BSPL_EUNSUPPORTED, "split launch beyond 2^32-1 work-items");
        TableDesc dd = d;
        int wx = tile.wx;
        void* args[] = {&dd, &wx};
        BSPL_HIP(hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(64 * tile.wx * tile.split), args,
                                 (size_t)lds, s));
        return BSPL_OK;
    }
    KernelArgs<1> a;
    a.t[0] = d;
    a.t[0].groups_begin = 0;
    a.ntables = 1;
    a.wx = tile.wx;
    a.wy = tile.wy;
    a.xcd_remap = order_xcd(tile.order) ? 1 : 0;
    a.tile_major = order_tile_major(tile.order) ? 1 : 0;
    const int64_t ygroups = (d.npos + tile.wy - 1) / tile.wy;
    a.total_groups = ygroups * d.xgroups;
    return launch<1>(kernel_for(t->info.dtype, kind, tile.vw, 0, d.lattice), a, tile, s);
}

static int any_lattice(const KernelArgs<kMaxTables>& a) {
    for (int i = 0; i < a.ntables; ++i)
        if (a.t[i].lattice) return 1;
    return 0;
}

bspl_status launch_multi(int dtype, int kind, const KernelArgs<kMaxTables>& a,
                         const bspl_tile& tile, hipStream_t s) {
    return launch<kMaxTables>(kernel_for(dtype, kind, tile.vw, 1, any_lattice(a)), a,
                              tile, s);
}

const void* multi_kernel_ptr(int dtype, int kind, int vw, int lattice) {
    return kernel_for(dtype, kind, vw, 1, lattice);
}

bspl_status launch_ratio(const bspl_table* t, int kind, const TableDesc& d, const float* ainv,
                         int64_t ld_ainv, double* out, const bspl_tile& tile, hipStream_t s) {
    const void* fn = ratio_kernel_for(t->info.dtype, kind, tile.vw, d.lattice);
    if (!fn) return fail(BSPL_EINVAL, "no ratio kernel for this dtype/kind/vw");
    if (d.npos <= 0) return BSPL_OK;
    int waves = tile.wx < d.nchunks ? tile.wx : d.nchunks;
    if (waves < 1) waves = 1;
    const int64_t grid = launch_grid(d.npos, tile.grid, 64 * waves);
    TableDesc dd = d;
    void* args[] = {&dd, const_cast<float**>(&ainv), &ld_ainv, &out};
    BSPL_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64 * waves), args, 0, s));
    return BSPL_OK;
}

}  // namespace bspl

// Table construction on the device: periodic padding, row padding to a
// 128-byte multiple, and conversion to FP16/BF16 with per-spline scales.
//
// Padded index i of a dimension with n cells holds coefficient (i-1) mod n,
// so the four rows a cell i0 needs are always i0..i0+3 and no wrap logic is
// left for the evaluation kernels (paper: the coefficient array P is padded
// and aligned, section "Baseline and miniQMC").
#include "internal.hpp"
#include "launch_check.hpp"

#include <cmath>

namespace bspl {
namespace {

// Column-wise max |c| as IEEE bits (non-negative floats order like uints).
__global__ void colmax_kernel(const float* __restrict__ c, int64_t nrows, int64_t ncols,
                              uint32_t* __restrict__ mx) {
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    uint32_t m = 0;
    for (int64_t r = blockIdx.y; r < nrows; r += gridDim.y) {
        const uint32_t b = __float_as_uint(c[r * ncols + col]) & 0x7fffffffu;
        m = b > m ? b : m;
    }
    atomicMax(&mx[col], m);
}

__global__ void fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// s_n = 2^ceil(log2 max|c_n|), or 1 for an all-zero (or padding) column.
__global__ void scales_kernel(const uint32_t* __restrict__ mx, int64_t nsplines, int64_t np,
                              float* __restrict__ scales) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= np) return;
    float s = 1.f;
    if (n < nsplines) {
        const float m = __uint_as_float(mx[n]);
        if (m > 0.f && m <= 3.4e38f) {
            int e;
            const float f = frexpf(m, &e);  // m = f * 2^e, f in [0.5, 1)
            s = ldexpf(1.f, f == 0.5f ? e - 1 : e);
        }
    }
    scales[n] = s;
}

__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

// Element n of padded point pt goes to block n / bs at row pt, column
// n % bs: [np / bs][px][py][pz][bs].  The plain layout is bs = np.
template <int DT>
__global__ void pad_kernel(const float* __restrict__ c, int padded_in, int nx, int ny, int nz,
                           int64_t nsplines, int64_t np, int64_t bs,
                           const float* __restrict__ scales, void* __restrict__ out) {
    const int px = nx + 3, py = ny + 3, pz = nz + 3;
    const int64_t npts = (int64_t)px * py * pz;
    for (int64_t pt = blockIdx.x; pt < npts; pt += gridDim.x) {
        const int iz = (int)(pt % pz);
        const int iy = (int)((pt / pz) % py);
        const int ix = (int)(pt / ((int64_t)pz * py));
        int64_t src;
        if (padded_in) {
            src = pt;
        } else {
            const int sx = (ix + nx - 1) % nx, sy = (iy + ny - 1) % ny, sz = (iz + nz - 1) % nz;
            src = ((int64_t)sx * ny + sy) * nz + sz;
        }
        const float* row = c + src * nsplines;
        for (int64_t n = threadIdx.x; n < np; n += blockDim.x) {
            const float x = n < nsplines ? row[n] : 0.f;
            const int64_t blk = n / bs;
            const int64_t o = blk * npts * bs + pt * bs + (n - blk * bs);
            if constexpr (DT == BSPL_F32) {
                static_cast<float*>(out)[o] = x;
            } else {
                const float q = x / scales[n];  // exact: scales are powers of two
                if constexpr (DT == BSPL_F16)
                    static_cast<_Float16*>(out)[o] = (_Float16)q;
                else
                    static_cast<uint16_t*>(out)[o] = to_bf16_rne(q);
            }
        }
    }
}

}  // namespace

bspl_status build_table(bspl_table* t, const float* d_coefs, bool padded_input,
                        hipStream_t s) {
    const bspl_table_info& in = t->info;
    const int64_t nsp = in.n_splines, np = in.n_padded;
    const int64_t nrows = padded_input ? (int64_t)in.px * in.py * in.pz
                                       : (int64_t)in.nx * in.ny * in.nz;
    uint32_t* mx = nullptr;
    if (in.dtype != BSPL_F32) {
        if (hipMalloc((void**)&mx, sizeof(uint32_t) * nsp) != hipSuccess)
            return fail(BSPL_ENOMEM, "scale scratch of %lld bytes", (long long)(4 * nsp));
    }
    clear_last_error();
    if (in.dtype != BSPL_F32) {
        hipLaunchKernelGGL(fill_u32, dim3(64), dim3(256), 0, s, mx, nsp, 0u);
        const unsigned gx = (unsigned)((nsp + 255) / 256);
        const unsigned gy = (unsigned)std::min<int64_t>(nrows, 1024);
        hipLaunchKernelGGL(colmax_kernel, dim3(gx, gy), dim3(256), 0, s, d_coefs, nrows, nsp, mx);
        hipLaunchKernelGGL(scales_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s,
                           mx, nsp, np, t->d_scales);
    }
    const int64_t npts = (int64_t)in.px * in.py * in.pz;
    const unsigned grid = (unsigned)std::min<int64_t>(npts, 65536);
    const int64_t bs = in.block_splines ? in.block_splines : np;
    switch (in.dtype) {
    case BSPL_F32:
        hipLaunchKernelGGL(pad_kernel<BSPL_F32>, dim3(grid), dim3(256), 0, s, d_coefs,
                           padded_input ? 1 : 0, in.nx, in.ny, in.nz, nsp, np, bs, t->d_scales,
                           t->d_table);
        break;
    case BSPL_F16:
        hipLaunchKernelGGL(pad_kernel<BSPL_F16>, dim3(grid), dim3(256), 0, s, d_coefs,
                           padded_input ? 1 : 0, in.nx, in.ny, in.nz, nsp, np, bs, t->d_scales,
                           t->d_table);
        break;
    default:
        hipLaunchKernelGGL(pad_kernel<BSPL_BF16>, dim3(grid), dim3(256), 0, s, d_coefs,
                           padded_input ? 1 : 0, in.nx, in.ny, in.nz, nsp, np, bs, t->d_scales,
                           t->d_table);
        break;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (mx) (void)hipFree(mx);
    if (e != hipSuccess) return hip_fail(e, "table build kernels");
    return BSPL_OK;
}

}  // namespace bspl

// Interpolating coefficients from orbital values on the grid.
//
// The coefficients are the orbitals' interpolation tables: the periodic
// spline must take the given value at every grid point.  At a grid point
// the weights of cells i-1, i, i+1 are 1/6, 2/3, 1/6, so along an axis of n
// points the condition is the circulant system
//     (c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i]        (indices mod n),
// and in 3-D the three axis systems apply one after the other.
//
// Solution by the factorisation z + 4 + 1/z = -(1/p)(1 - p/z)(1 - p z) with
// the pole p = sqrt(3) - 2 (Unser, Aldroubi & Eden, "B-spline signal
// processing", IEEE Trans. Signal Process. 41, 1993):
//     y[i] = f[i] + p y[i-1]       (causal, periodic start)
//     w[i] = y[i] + p w[i+1]       (anti-causal, periodic start)
//     c[i] = -6 p w[i]
// The periodic starts are geometric sums over one period,
//     y[0]   = sum_{k<n} p^k f[-k mod n]    / (1 - p^n)
//     w[n-1] = sum_{k<n} p^k y[n-1+k mod n] / (1 - p^n),
// cut at 32 terms for longer axes (|p|^32 < 1e-18).
//
// One thread runs both recursions over one line of one spline; consecutive
// threads take consecutive splines (or the fastest remaining index), so
// every access of a wavefront is one contiguous 256-byte segment.  The
// recursion state is FP64; the intermediate y is stored in the output in
// FP32, which makes the three passes work in place (src may equal dst, so
// neither pointer is restrict).
#include "internal.hpp"
#include "launch_check.hpp"

namespace bspl {
namespace {

constexpr double kPole = -0.2679491924311227;  // sqrt(3) - 2
constexpr int kStartTerms = 32;
constexpr int kFitThreads = 256;

__global__ void __launch_bounds__(kFitThreads) fit_axis_kernel(
    const float* src, float* dst, int n, int64_t inner, int64_t lines,
    double gain, int start_terms) {
    const int64_t t = (int64_t)blockIdx.x * kFitThreads + threadIdx.x;
    if (t >= lines) return;
    const int64_t o = t / inner;
    const int64_t base = o * (int64_t)n * inner + (t - o * inner);
    // causal pass; every read of src at an index precedes the write of dst there
    double pk = 1.0, y = 0.0;
    for (int k = 0; k < start_terms; ++k) {
        const int i = k == 0 ? 0 : n - k;
        y = __builtin_fma(pk, (double)src[base + (int64_t)i * inner], y);
        pk *= kPole;
    }
    y *= gain;
    dst[base] = (float)y;
    for (int i = 1; i < n; ++i) {
        const int64_t at = base + (int64_t)i * inner;
        y = __builtin_fma(kPole, y, (double)src[at]);
        dst[at] = (float)y;
    }
    // anti-causal pass over the stored y (the last one is still exact in y)
    pk = kPole;
    double w = y;
    for (int k = 1; k < start_terms; ++k) {
        w = __builtin_fma(pk, (double)dst[base + (int64_t)(k - 1) * inner], w);
        pk *= kPole;
    }
    w *= gain;
    const double out_scale = -6.0 * kPole;
    dst[base + (int64_t)(n - 1) * inner] = (float)(out_scale * w);
    for (int i = n - 2; i >= 0; --i) {
        const int64_t at = base + (int64_t)i * inner;
        w = __builtin_fma(kPole, w, (double)dst[at]);
        dst[at] = (float)(out_scale * w);
    }
}

// The same two recursions with the line staged in LDS: a wavefront loads
// its 64 lines (n x 64 floats, lane-contiguous, so conflict-free) with n
// independent loads per lane, UNROLL of them in flight at a time, runs both
// recursions in LDS and stores each coefficient once: one read and one
// write of HBM per element and axis instead of two of each.  Used while
// n * 256 B fits in 64 KiB.  The LDS a line takes sets the wavefronts per
// CU (13 at n = 48, 6 at n = 96), so longer lines keep more loads in
// flight per wavefront: 8 up to n = 64, 16 beyond (measured on MI355X: 16
// loads take the 96^3 fit from 22.0 to 17.4 ms; 32 or 48 gain nothing more
// and slow the 48^3 fit).
constexpr int kLdsMaxN = 256;
constexpr int kLdsFewLoadsMaxN = 64;

template <int UNROLL>
__global__ void __launch_bounds__(64) fit_axis_lds_kernel(
    const float* src, float* dst, int n, int64_t inner, int64_t lines, double gain,
    int start_terms) {
    extern __shared__ float line[];  // [n][64]
    const int lane = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const bool live = t < lines;
    const int64_t o = live ? t / inner : 0;
    const int64_t base = live ? o * (int64_t)n * inner + (t - o * inner) : 0;
    float* my = line + lane;
    if (live) {
#pragma unroll UNROLL
        for (int i = 0; i < n; ++i) my[i * 64] = src[base + (int64_t)i * inner];
    }
    // each lane touches only its own column: no barrier is needed
    if (!live) return;
    double pk = 1.0, y = 0.0;
    for (int k = 0; k < start_terms; ++k) {
        const int i = k == 0 ? 0 : n - k;
        y = __builtin_fma(pk, (double)my[i * 64], y);
        pk *= kPole;
    }
    y *= gain;
    my[0] = (float)y;
    for (int i = 1; i < n; ++i) {
        y = __builtin_fma(kPole, y, (double)my[i * 64]);
        my[i * 64] = (float)y;
    }
    pk = kPole;
    double w = y;
    for (int k = 1; k < start_terms; ++k) {
        w = __builtin_fma(pk, (double)my[(k - 1) * 64], w);
        pk *= kPole;
    }
    w *= gain;
    const double out_scale = -6.0 * kPole;
    dst[base + (int64_t)(n - 1) * inner] = (float)(out_scale * w);
    for (int i = n - 2; i >= 0; --i) {
        w = __builtin_fma(kPole, w, (double)my[i * 64]);
        dst[base + (int64_t)i * inner] = (float)(out_scale * w);
    }
}

}  // namespace

bspl_status launch_fit(int nx, int ny, int nz, int64_t nspl, const float* src, float* dst,
                       hipStream_t s) {
    const int dims[3] = {nx, ny, nz};
    const int64_t total = (int64_t)nx * ny * nz * nspl;
    for (int d = 0; d < 3; ++d) {
        const int n = dims[d];
        int64_t inner = nspl;
        for (int e = d + 1; e < 3; ++e) inner *= dims[e];
        const int64_t lines = total / n;
        double pn = 1.0;
        for (int k = 0; k < n && k < 64; ++k) pn *= kPole;  // p^n (0 to FP64 beyond 64)
        const double gain = 1.0 / (1.0 - pn);
        const int start_terms = n < kStartTerms ? n : kStartTerms;
        const float* in = d == 0 ? src : dst;
        clear_last_error();
        if (n <= kLdsMaxN) {
            const int64_t blocks = (lines + 63) / 64;
            if (n <= kLdsFewLoadsMaxN)
                hipLaunchKernelGGL(fit_axis_lds_kernel<8>, dim3((unsigned)blocks), dim3(64),
                                   (size_t)n * 64 * sizeof(float), s, in, dst, n, inner, lines,
                                   gain, start_terms);
            else
                hipLaunchKernelGGL(fit_axis_lds_kernel<16>, dim3((unsigned)blocks), dim3(64),
                                   (size_t)n * 64 * sizeof(float), s, in, dst, n, inner, lines,
                                   gain, start_terms);
        } else {
            const int64_t blocks = (lines + kFitThreads - 1) / kFitThreads;
            hipLaunchKernelGGL(fit_axis_kernel, dim3((unsigned)blocks), dim3(kFitThreads), 0,
                               s, in, dst, n, inner, lines, gain, start_terms);
        }
        BSPL_HIP(hipGetLastError());
    }
    return BSPL_OK;
}

}  // namespace bspl

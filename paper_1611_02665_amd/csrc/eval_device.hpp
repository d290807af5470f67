// Evaluation kernels for gfx950: V, VGL and VGH of periodic tricubic
// B-splines (paper Eq. TricubicValue; kernels of Fig. 3 and Fig. 4(b)).
//
// Work unit: one wavefront, one position, one spline tile of 64*VW
// consecutive splines.  Lane l owns splines [tile*64*VW + l*VW, +VW).
//  1. Lanes 0..2 place the position in its cell, one dimension each, in FP64
//     (periodic wrap, lower-bound index, fraction t rounded to FP32).
//  2. Lane d < 3 forms the 12 basis weights of dimension d (value, first and
//     second derivative of 4 cell offsets, derivatives already scaled by
//     1/Delta and 1/Delta^2); v_readlane broadcasts them into scalar
//     registers, so every lane of the wavefront shares them for free.
//  3. For each of the 16 (i,j) pairs the 4 z-consecutive rows of the tile
//     are one coalesced load per row (16 bytes per lane at VW=4/FP32), and
//     the reduction runs z first, then y, then x, all in FP32 registers.
//  4. The 1, 5 or 10 output rows are written once, SoA.
// The path is HBM-bound (about 2 flop/byte), so there is no MFMA, and LDS
// only carries the partial sums of split (latency-mode) units: every table
// byte moves once from HBM to registers.
//
// This header holds the device code and the generic kernel pickers; the
// three dtype translation units instantiate it.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace bspl {
namespace {

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct F32 {};
struct F16 {};
struct BF16 {};

template <typename T> struct Elem;
template <> struct Elem<F32> { static constexpr int bytes = 4; };
template <> struct Elem<F16> { static constexpr int bytes = 2; };
template <> struct Elem<BF16> { static constexpr int bytes = 2; };

// Raw load of VW consecutive coefficients (one 4/8/16-byte access per lane)
// and its widening to FP32.  Loads and widening are separate so that loads
// can be issued several row groups ahead of the arithmetic.
template <typename T, int VW> struct Row;

template <int VW> struct Row<F32, VW> {
    using raw = typename std::conditional<VW == 4, float4,
                typename std::conditional<VW == 2, float2, float>::type>::type;
    static __device__ __forceinline__ raw load(const char* p) {
        return *reinterpret_cast<const raw*>(p);
    }
    static __device__ __forceinline__ void widen(const raw& q, float (&o)[VW]) {
        if constexpr (VW == 4) {
            o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
        } else if constexpr (VW == 2) {
            o[0] = q.x; o[1] = q.y;
        } else {
            o[0] = q;
        }
    }
};

template <int VW> struct Row<F16, VW> {
    using raw = typename std::conditional<VW == 8, f16x8,
                typename std::conditional<VW == 4, f16x4, f16x2>::type>::type;
    static __device__ __forceinline__ raw load(const char* p) {
        return *reinterpret_cast<const raw*>(p);
    }
    static __device__ __forceinline__ void widen(const raw& q, float (&o)[VW]) {
#pragma unroll
        for (int e = 0; e < VW; ++e) o[e] = (float)q[e];
    }
};

__device__ __forceinline__ void bf16_pair(uint32_t w, float& lo, float& hi) {
    lo = __uint_as_float(w << 16);
    hi = __uint_as_float(w & 0xffff0000u);
}

template <int VW> struct Row<BF16, VW> {
    using raw = typename std::conditional<VW == 8, u32x4,
                typename std::conditional<VW == 4, u32x2, uint32_t>::type>::type;
    static __device__ __forceinline__ raw load(const char* p) {
        return *reinterpret_cast<const raw*>(p);
    }
    static __device__ __forceinline__ void widen(const raw& q, float (&o)[VW]) {
        if constexpr (VW == 8) {
            bf16_pair(q[0], o[0], o[1]); bf16_pair(q[1], o[2], o[3]);
            bf16_pair(q[2], o[4], o[5]); bf16_pair(q[3], o[6], o[7]);
        } else if constexpr (VW == 4) {
            bf16_pair(q[0], o[0], o[1]); bf16_pair(q[1], o[2], o[3]);
        } else {
            bf16_pair(q, o[0], o[1]);
        }
    }
};

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Output rows are written once and not read back by the launch, so the
// vector stores are non-temporal: they do not displace the table rows that
// neighbouring positions re-read from L2 (3 % on the dense cell-ordered FP16
// launches, neutral for FP32 tables).
template <int VW>
__device__ __forceinline__ void store_row(float* dst, const float (&x)[VW], int valid,
                                          bool vec) {
    if (vec && valid >= VW) {
        if constexpr (VW == 4) {
            const f32x4 q = {x[0], x[1], x[2], x[3]};
            __builtin_nontemporal_store(q, reinterpret_cast<f32x4*>(dst));
        } else if constexpr (VW == 2) {
            const f32x2 q = {x[0], x[1]};
            __builtin_nontemporal_store(q, reinterpret_cast<f32x2*>(dst));
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) __builtin_nontemporal_store(x[e], dst + e);
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e)
            if (e < valid) dst[e] = x[e];
    }
}

__device__ __forceinline__ float bcast(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Basis weight number r (0..11) of a dimension at fraction t: r/4 selects
// value, first or second derivative, r%4 the cell offset m.  These are the
// uniform cubic B-spline pieces written as cubics in t (Horner form):
//   m=0: (1-t)^3/6   m=1: (3t^3-6t^2+4)/6   m=2: (-3t^3+3t^2+3t+1)/6   m=3: t^3/6
__device__ __forceinline__ float basis_weight(int r, float t) {
    float c0, c1, c2, c3;
    switch (r) {
    case 0: c0 = 1.f / 6; c1 = -0.5f; c2 = 0.5f; c3 = -1.f / 6; break;
    case 1: c0 = 2.f / 3; c1 = 0.f; c2 = -1.f; c3 = 0.5f; break;
    case 2: c0 = 1.f / 6; c1 = 0.5f; c2 = 0.5f; c3 = -0.5f; break;
    case 3: c0 = 0.f; c1 = 0.f; c2 = 0.f; c3 = 1.f / 6; break;
    case 4: c0 = -0.5f; c1 = 1.f; c2 = -0.5f; c3 = 0.f; break;
    case 5: c0 = 0.f; c1 = -2.f; c2 = 1.5f; c3 = 0.f; break;
    case 6: c0 = 0.5f; c1 = 1.f; c2 = -1.5f; c3 = 0.f; break;
    case 7: c0 = 0.f; c1 = 0.f; c2 = 0.5f; c3 = 0.f; break;
    case 8: c0 = 1.f; c1 = -1.f; c2 = 0.f; c3 = 0.f; break;
    case 9: c0 = -2.f; c1 = 3.f; c2 = 0.f; c3 = 0.f; break;
    case 10: c0 = 1.f; c1 = -3.f; c2 = 0.f; c3 = 0.f; break;
    default: c0 = 0.f; c1 = 1.f; c2 = 0.f; c3 = 0.f; break;
    }
    return ((c3 * t + c2) * t + c1) * t + c0;
}

// Cell location of one grid coordinate u (FP64) on an axis of nd cells.
// Returns false for a non-finite input.  A position with no fraction bits
// left (|u| >= 2^50), and a non-finite one, is placed on grid point 0.  The
// steps are selects, not branches, so that the loads feeding them (the
// position and the axis row) issue together and are waited for once.
__device__ __forceinline__ bool locate(double u, double nd, int& i0, float& t) {
    const bool finite = __builtin_isfinite(u);
    const double v = __builtin_fabs(u) < 1125899906842624.0 ? u : 0.0;
    double w = v - nd * __builtin_floor(v / nd);
    w = w < 0.0 ? w + nd : w;
    w = w >= nd ? 0.0 : w;  // rounded up to n: the image of 0
    const int n = (int)nd;
    int i = (int)__builtin_floor(w);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    i0 = i;
    t = (float)(w - (double)i);
    return finite;
}

template <int KIND> struct Shape;
template <> struct Shape<BSPL_V> { static constexpr int nout = 1, ny = 1; };
template <> struct Shape<BSPL_VGL> { static constexpr int nout = 5, ny = 5; };
template <> struct Shape<BSPL_VGH> { static constexpr int nout = 10, ny = 6; };

// Row groups in flight per wavefront: 128 bytes of loads per lane (32 VGPRs).
template <typename T, int VW> struct Depth {
    static constexpr int value = 32 / (VW * Elem<T>::bytes) < 2 ? 2 : 32 / (VW * Elem<T>::bytes);
};

// Upper-triangle component k (xx, xy, xz, yy, yz, zz) as an index pair.
__device__ __forceinline__ int sym_row(int k) { return k < 3 ? 0 : (k < 5 ? 1 : 2); }
__device__ __forceinline__ int sym_col(int k) { return k < 3 ? k : (k < 5 ? k - 2 : 2); }

// Coefficient of grid-space Hessian component q in Cartesian component k:
// H_r[a][b] = sum_{d,e} M[d][a] M[e][b] H_u[d][e], with the symmetric
// off-diagonal pairs of H_u folded together.  The per-lane indices read the
// map straight from the descriptor (kernel-argument memory), which keeps
// it out of private memory.
__device__ __forceinline__ float hess_coef(const TableDesc& d, int k, int q) {
    const int a = sym_row(k), b = sym_col(k), dd = sym_row(q), e = sym_col(q);
    float c = (float)d.axis[dd][a] * (float)d.axis[e][b];
    if (dd != e) c = fmaf((float)d.axis[e][a], (float)d.axis[dd][b], c);
    return c;
}

// Lattice tables evaluate VGL with the whole grid-space Hessian, which the
// Laplacian needs once the axes are not orthogonal.
template <int KIND, int LAT> struct Internal {
    static constexpr int kind = (LAT && KIND == BSPL_VGL) ? BSPL_VGH : KIND;
};

// Steps 1-4 for one work unit: on return out holds the unit's outputs for
// splines [n0, n0 + VW) of lane `lane`, of which `valid` (if positive) are
// real splines.  NG < 16 evaluates only the row groups of the x-slabs
// [islab, islab + NG/4): the partial sum that one wavefront of a split unit
// contributes (every step after the gather is linear in the coefficients).
template <typename T, int VW, int KIND, int LAT, int NG = 16,
          int DEPTH = Depth<T, VW>::value>
__device__ __forceinline__ void eval_core(const TableDesc& d, int p, int chunk, int lane,
                                          float (&out)[Shape<KIND>::nout][VW], int& n0_out,
                                          int& valid_out, int islab = 0) {
    static_assert(NG == 16 || NG == 8 || NG == 4, "whole x-slabs only");
    static_assert(DEPTH >= 1 && DEPTH <= NG, "ring deeper than the groups");
    constexpr int EB = Elem<T>::bytes;
    constexpr int KI = Internal<KIND, LAT>::kind;  // what is accumulated
    constexpr int NOUT = Shape<KI>::nout;
    constexpr int NY = Shape<KI>::ny;

    // 1. cell index and fraction: lane d handles grid axis d,
    //    u_d = sum_a M[d][a] r_a in FP64 (a box has M diagonal)
    int my_i0 = 0;
    float my_t = 0.f;
    int my_bad = 0;
    float my_scale = 1.f;  // lane d < 3 of a box: n_d / L_d in FP32
    if (lane < 3) {
        // the lane's map row and cell count (one lane-indexed read of the
        // descriptor) and the position, all issued before the first wait
        const double* row = d.axis[lane];
        double u;
        if constexpr (LAT) {
            const double x = d.pos[p];
            const double y = d.pos[d.npos + p];
            const double z = d.pos[2 * d.npos + p];
            u = __builtin_fma(row[0], x, __builtin_fma(row[1], y, row[2] * z));
        } else {  // a box: the map is diagonal
            u = d.pos[(int64_t)lane * d.npos + p] * row[lane];
            my_scale = (float)row[lane];
        }
        my_bad = locate(u, row[3], my_i0, my_t) ? 0 : 1;
    }
    const int i0 = __builtin_amdgcn_readlane(my_i0, 0);
    const int j0 = __builtin_amdgcn_readlane(my_i0, 1);
    const int k0 = __builtin_amdgcn_readlane(my_i0, 2);
    const int bad = __builtin_amdgcn_readlane(my_bad, 0) | __builtin_amdgcn_readlane(my_bad, 1) |
                    __builtin_amdgcn_readlane(my_bad, 2);

    // 2. weights: lane d < 3 evaluates the 12 weights of axis d (value,
    //    first and second derivative of the 4 cell offsets) in straight-line
    //    code; a box folds 1/Delta_d into the derivative weights, a lattice
    //    keeps grid units and transforms the derivatives at the end.
    //    v_readlane then moves them into scalar registers, so every lane of
    //    the wavefront shares them at no VGPR cost.
    float ax[4], dax[4], d2ax[4], ay[4], day[4], d2ay[4], az[4], daz[4], d2az[4];
    auto form_weights = [&]() {
        float w[12];
        const float s = my_scale;
#pragma unroll
        for (int r = 0; r < 12; ++r) {
            w[r] = basis_weight(r, my_t);
            w[r] *= r >= 8 ? s * s : (r >= 4 ? s : 1.f);
            if (bad) w[r] = __builtin_nanf("");
        }
        // weight r of axis d; x weights are those of this unit's slabs
        // (islab is 0 unless the unit is split, and wave-uniform)
        auto wt = [&](int d_axis, int r) { return bcast(w[r], d_axis); };
        auto wx = [&](int r0, int m) {
            float v = wt(0, r0 + m);
            if constexpr (NG < 16) {
#pragma unroll
                for (int k = 1; k < 4; ++k)
                    if (m + k < 4 && islab == k) v = wt(0, r0 + m + k);
            }
            return v;
        };
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            ax[m] = wx(0, m);
            ay[m] = wt(1, m);
            az[m] = wt(2, m);
            if constexpr (KI != BSPL_V) {
                dax[m] = wx(4, m);
                d2ax[m] = wx(8, m);
                day[m] = wt(1, 4 + m);
                d2ay[m] = wt(1, 8 + m);
                daz[m] = wt(2, 4 + m);
                d2az[m] = wt(2, 8 + m);
            }
        }
    };

    constexpr bool kIssueFirst = VW * EB <= 8;
    if constexpr (!kIssueFirst) form_weights();

    // 3. gather and reduce
    const int n0 = chunk * (64 * VW) + lane * VW;
    const int valid = d.nsplines - n0;  // > 0 for lanes that own splines
    // the tile's columns: plain rows hold every spline; a spline-blocked
    // table holds chunks_per_block tiles per block (chunk is wave-uniform)
    size_t tile_off = (size_t)chunk * (64 * VW * EB);
    if (d.block_bytes) {
        const int blk = chunk / d.chunks_per_block;
        tile_off = (size_t)blk * (size_t)d.block_bytes +
                   (size_t)(chunk - blk * d.chunks_per_block) * (64 * VW * EB);
    }
    const char* base = d.table + (size_t)(i0 + islab) * d.xstride + (size_t)j0 * d.ystride +
                       (size_t)k0 * d.row_bytes + tile_off;
    const uint32_t loff = valid > 0 ? (uint32_t)(lane * VW * EB) : 0u;

    // Row groups g = 4i + j (16 of them, 4 z-rows each) stream through a ring
    // of DEPTH groups: group g+DEPTH-1 is issued before group g is reduced,
    // so DEPTH groups of loads are in flight per wavefront while register use
    // stays bounded.  An empty asm that reads the partial sums of group g and
    // clobbers memory orders "reduce g" before "issue g+DEPTH"; without it the
    // compiler hoists all 64 loads to the top and spills.  The same fence
    // after the last DEPTH groups (no loads left to order) keeps the y and x
    // reductions incremental: otherwise the compiler defers them to the end
    // of the slab and holds every z-sum live (FP16 VGH at VW=2 then needs 150
    // VGPRs instead of 82).
    using RowT = Row<T, VW>;
    typename RowT::raw ring[DEPTH][4];
    auto issue = [&](int g, int slot) {
        const uint32_t go = loff + (uint32_t)(g >> 2) * d.xstride + (uint32_t)(g & 3) * d.ystride;
#pragma unroll
        for (int k = 0; k < 4; ++k) ring[slot][k] = RowT::load(base + (go + (uint32_t)k * d.row_bytes));
    };
    // per-spline scales of reduced-precision tables, loaded while the last
    // row groups are still in flight
    float sc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) sc[e] = 1.f;
    constexpr int kScaleGroup = NG > DEPTH ? NG - DEPTH : 0;

    float acc[NOUT][VW];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[o][e] = 0.f;
    float Y[NY][VW];

    // The first DEPTH-1 row groups go out before the weights are formed, so
    // that the weights' arithmetic overlaps their flight (one position:
    // 3.99 against 4.17 us per evaluation).  With 16-byte loads per lane
    // (FP32 at VW=4, 16-bit tables at VW=8) the compiler then schedules the
    // ring as single loads with full waits between them (the dense FP32
    // launch: 299 against 273 us), so those tiles form the weights before
    // the gather set-up.
#pragma unroll
    for (int g = 0; g < DEPTH - 1; ++g) issue(g, g);
    if constexpr (kIssueFirst) form_weights();

#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + DEPTH - 1 < NG) issue(g + DEPTH - 1, (g + DEPTH - 1) % DEPTH);
        if constexpr (EB == 2) {
            if (g == kScaleGroup && valid > 0) {
#pragma unroll
                for (int e = 0; e < VW; ++e) sc[e] = d.scales[n0 + e];
            }
        }
        const int i = g >> 2, j = g & 3;
        if (j == 0) {
#pragma unroll
            for (int o = 0; o < NY; ++o)
#pragma unroll
                for (int e = 0; e < VW; ++e) Y[o][e] = 0.f;
        }
        float q[4][VW];
#pragma unroll
        for (int k = 0; k < 4; ++k) RowT::widen(ring[g % DEPTH][k], q[k]);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            // the first products are FMAs with a zero addend: with 16-bit
            // tables they take the half directly (v_fma_mix_f32) instead of
            // after a separate conversion
            float s0 = fmaf(az[0], q[0][e], 0.f);
            s0 = fmaf(az[1], q[1][e], s0);
            s0 = fmaf(az[2], q[2][e], s0);
            s0 = fmaf(az[3], q[3][e], s0);
            Y[0][e] = fmaf(ay[j], s0, Y[0][e]);
            if constexpr (KI != BSPL_V) {
                float s1 = fmaf(daz[0], q[0][e], 0.f);
                s1 = fmaf(daz[1], q[1][e], s1);
                s1 = fmaf(daz[2], q[2][e], s1);
                s1 = fmaf(daz[3], q[3][e], s1);
                float s2 = fmaf(d2az[0], q[0][e], 0.f);
                s2 = fmaf(d2az[1], q[1][e], s2);
                s2 = fmaf(d2az[2], q[2][e], s2);
                s2 = fmaf(d2az[3], q[3][e], s2);
                Y[1][e] = fmaf(day[j], s0, Y[1][e]);   // d/dy
                Y[2][e] = fmaf(d2ay[j], s0, Y[2][e]);  // d2/dy2
                Y[3][e] = fmaf(ay[j], s1, Y[3][e]);    // d/dz
                if constexpr (KI == BSPL_VGH) {
                    Y[4][e] = fmaf(day[j], s1, Y[4][e]);  // d2/dydz
                    Y[5][e] = fmaf(ay[j], s2, Y[5][e]);   // d2/dz2
                } else {
                    Y[4][e] = fmaf(ay[j], s2, Y[4][e]);   // d2/dz2
                }
            }
        }
        if (j == 3) {
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                acc[0][e] = fmaf(ax[i], Y[0][e], acc[0][e]);  // v
                if constexpr (KI == BSPL_VGL) {
                    acc[1][e] = fmaf(dax[i], Y[0][e], acc[1][e]);  // gx
                    acc[2][e] = fmaf(ax[i], Y[1][e], acc[2][e]);   // gy
                    acc[3][e] = fmaf(ax[i], Y[3][e], acc[3][e]);   // gz
                    acc[4][e] = fmaf(d2ax[i], Y[0][e], acc[4][e]); // lap: xx
                    acc[4][e] = fmaf(ax[i], Y[2][e] + Y[4][e], acc[4][e]);  // + yy + zz
                }
                if constexpr (KI == BSPL_VGH) {
                    acc[1][e] = fmaf(dax[i], Y[0][e], acc[1][e]);  // gx
                    acc[2][e] = fmaf(ax[i], Y[1][e], acc[2][e]);   // gy
                    acc[3][e] = fmaf(ax[i], Y[3][e], acc[3][e]);   // gz
                    acc[4][e] = fmaf(d2ax[i], Y[0][e], acc[4][e]); // hxx
                    acc[5][e] = fmaf(dax[i], Y[1][e], acc[5][e]);  // hxy
                    acc[6][e] = fmaf(dax[i], Y[3][e], acc[6][e]);  // hxz
                    acc[7][e] = fmaf(ax[i], Y[2][e], acc[7][e]);   // hyy
                    acc[8][e] = fmaf(ax[i], Y[4][e], acc[8][e]);   // hyz
                    acc[9][e] = fmaf(ax[i], Y[5][e], acc[9][e]);   // hzz
                }
            }
        }
        if (j == 3) {
#pragma unroll
            for (int o = 0; o < NOUT; ++o)
#pragma unroll
                for (int e = 0; e < VW; ++e) asm volatile("" : "+v"(acc[o][e]));
        } else {
#pragma unroll
            for (int o = 0; o < NY; ++o)
#pragma unroll
                for (int e = 0; e < VW; ++e) asm volatile("" : "+v"(Y[o][e]));
        }
        asm volatile("" ::: "memory");
    }

    // 4a. lattice tables: grid-space derivatives to Cartesian ones,
    //     g_r = M^T g_u and H_r = M^T H_u M (L = trace H_r)
    constexpr int NO = Shape<KIND>::nout;
    if constexpr (LAT && KIND != BSPL_V) {
        float m[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = (float)d.axis[k / 3][k % 3];
        // lane 6k + q holds the coefficient of H_u component q in H_r component k
        float hc = 0.f;
        if (lane < 36) hc = hess_coef(d, lane / 6, lane % 6);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            out[0][e] = acc[0][e];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                out[1 + a][e] = fmaf(m[a], acc[1][e], fmaf(m[3 + a], acc[2][e], m[6 + a] * acc[3][e]));
        }
        if constexpr (KIND == BSPL_VGH) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                float c[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) c[q] = bcast(hc, 6 * k + q);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    float h = 0.f;
#pragma unroll
                    for (int q = 0; q < 6; ++q) h = fmaf(c[q], acc[4 + q][e], h);
                    out[4 + k][e] = h;
                }
            }
        } else {  // VGL: the Laplacian sums the diagonal components k = 0, 3, 5
            float c[6];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                c[q] = bcast(hc, q) + bcast(hc, 18 + q) + bcast(hc, 30 + q);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                float h = 0.f;
#pragma unroll
                for (int q = 0; q < 6; ++q) h = fmaf(c[q], acc[4 + q][e], h);
                out[4][e] = h;
            }
        }
    } else {
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int e = 0; e < VW; ++e) out[o][e] = acc[o][e];
    }

    // 4b. per-spline scale of reduced-precision tables
    n0_out = n0;
    valid_out = valid;
    if (valid <= 0) return;
    if constexpr (Elem<T>::bytes == 2) {
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int e = 0; e < VW; ++e) out[o][e] *= sc[e];
    }
}

// One work unit: evaluate, then write the 1, 5 or 10 SoA output rows.
template <typename T, int VW, int KIND, int LAT>
__device__ __forceinline__ void eval_unit(const TableDesc& d, int p, int chunk, int lane) {
    float acc[Shape<KIND>::nout][VW];
    int n0, valid;
    eval_core<T, VW, KIND, LAT>(d, p, chunk, lane, acc, n0, valid);
    if (valid <= 0) return;
    const bool vec = d.vec_store != 0;
    const int64_t ldo = d.ldo;
    store_row<VW>(d.v + (int64_t)p * ldo + n0, acc[0], valid, vec);
    if constexpr (KIND != BSPL_V) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            store_row<VW>(d.g + ((int64_t)p * 3 + c) * ldo + n0, acc[1 + c], valid, vec);
    }
    if constexpr (KIND == BSPL_VGL)
        store_row<VW>(d.lh + (int64_t)p * ldo + n0, acc[4], valid, vec);
    if constexpr (KIND == BSPL_VGH) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            store_row<VW>(d.lh + ((int64_t)p * 6 + c) * ldo + n0, acc[4 + c], valid, vec);
    }
}

// Block b of a launch runs on XCD b % 8.  With remapping, XCD x takes the
// contiguous run [x*per, (x+1)*per) of blocks (the tail stays in place), so
// that neighbouring positions of a cell-sorted order share one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t total) {
    const int64_t per = total / kXcds;
    if (b >= per * kXcds) return b;
    return (b % kXcds) * per + b / kXcds;
}

// One launch over one or several tables.  Workgroup-block g covers wx
// spline tiles by wy positions of one table; blocks are numbered table by
// table, positions outer and tiles inner, or tiles outer and positions inner
// (tile_major).  With fewer workgroups than blocks
// (persistent launch) each workgroup strides over the blocks.
template <typename T, int VW, int KIND, int MAXT, int LAT>
__global__ void __launch_bounds__(512) eval_kernel(const KernelArgs<MAXT> a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wxi = wave % a.wx;
    const int wyi = wave / a.wx;
    for (int64_t b = blockIdx.x; b < a.total_groups; b += gridDim.x) {
        const int64_t g = a.xcd_remap ? xcd_block(b, a.total_groups) : b;
        int ti = 0;
        if constexpr (MAXT > 1) {
            for (int k = 1; k < a.ntables; ++k)
                if (g >= a.t[k].groups_begin) ti = k;
        }
        const TableDesc& d = a.t[ti];
        const int local = (int)(g - d.groups_begin);
        int pg, cg;
        if (a.tile_major) {  // tiles outer: every position of a tile, then the next tile
            const int ygroups = (int)((d.npos + a.wy - 1) / a.wy);
            cg = local / ygroups;
            pg = local - cg * ygroups;
        } else {             // positions outer
            pg = local / d.xgroups;
            cg = local - pg * d.xgroups;
        }
        const int chunk = cg * a.wx + wxi;
        const int q = pg * a.wy + wyi;
        if (chunk < d.nchunks && q < d.npos) {
            const int p = d.perm ? __builtin_amdgcn_readfirstlane(d.perm[q]) : q;
            eval_unit<T, VW, KIND, LAT>(d, p, chunk, lane);
        }
    }
}

// Output row of component o (0..NO-1) of position p, in the order the
// accumulators hold them: v; gx gy gz; then l or hxx hxy hxz hyy hyz hzz.
template <int KIND>
__device__ __forceinline__ float* out_row(const TableDesc& d, int o, int p) {
    const int64_t ldo = d.ldo;
    if (o == 0) return d.v + (int64_t)p * ldo;
    if (o < 4) return d.g + ((int64_t)p * 3 + (o - 1)) * ldo;
    if constexpr (KIND == BSPL_VGL) return d.lh + (int64_t)p * ldo;
    return d.lh + ((int64_t)p * 6 + (o - 4)) * ldo;
}

// Latency mode (the GPU form of the paper's nested threading over one
// walker's work, section "Optimizations and Parallelization"): with few
// positions there are too few (position, tile) units to fill the chip, and
// each unit's 16 row groups take several memory round trips in sequence.
// Here SPLIT wavefronts share one unit: wavefront s gathers and reduces the
// x-slabs [s*4/SPLIT, (s+1)*4/SPLIT) with all of its row groups in flight
// at once, the partial sums meet in LDS, and wavefront s adds up and stores
// the components o with o % SPLIT == s (partials summed in slab order, so
// the result is deterministic).  One workgroup = wx tiles x SPLIT slabs of
// one position; block b covers position b / xgroups.
template <typename T, int VW, int KIND, int LAT, int SPLIT>
__global__ void __launch_bounds__(512) split_kernel(const TableDesc d, int wx) {
    constexpr int NO = Shape<KIND>::nout;
    constexpr int NG = 16 / SPLIT;
    extern __shared__ float part[];  // [SPLIT][wx][NO][VW][64]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wxi = wave % wx;
    const int slab = wave / wx;
    const int q = (int)(blockIdx.x / (unsigned)d.xgroups);
    const int cg = (int)(blockIdx.x - (unsigned)q * (unsigned)d.xgroups);
    const int chunk = cg * wx + wxi;
    const bool live = chunk < d.nchunks;
    float acc[NO][VW];
    int n0 = 0, valid = 0;
    const int p = d.perm ? __builtin_amdgcn_readfirstlane(d.perm[q]) : q;
    if (live) {
        eval_core<T, VW, KIND, LAT, NG, NG>(d, p, chunk, lane, acc, n0, valid, slab * (NG / 4));
    } else {
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[o][e] = 0.f;
    }
    float* mine = part + (size_t)(slab * wx + wxi) * (NO * VW * 64);
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int e = 0; e < VW; ++e) mine[(o * VW + e) * 64 + lane] = acc[o][e];
    __syncthreads();
    if (!live || valid <= 0) return;
    const bool vec = d.vec_store != 0;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        if (o % SPLIT != slab) continue;
        float x[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            float sum = part[((size_t)wxi * NO * VW + o * VW + e) * 64 + lane];
#pragma unroll
            for (int s2 = 1; s2 < SPLIT; ++s2)
                sum += part[((size_t)(s2 * wx + wxi) * NO * VW + o * VW + e) * 64 + lane];
            x[e] = sum;
        }
        store_row<VW>(out_row<KIND>(d, o, p) + n0, x, valid, vec);
    }
}

// Determinant-ratio consumer fused into the evaluation (paper: the ratio of
// determinants after a one-electron move is the sum over orbitals of
// phi_n(r_e) times the inverse-matrix entry of (n, e), and its gradient the
// same sum over grad phi_n; "QMC and B-spline-based SPOs").  For position p:
//   out[p][c] = sum_n X_c,n(r_p) * ainv[p][n]
// for every output component X_c of the kind (phi; grad phi; Laplacian or
// Hessian).  One workgroup of W wavefronts owns one position; wavefront w
// reduces spline tiles w, w+W, ...; per-lane FP32 products are summed in FP64,
// reduced across the wavefront with shuffles and across the workgroup in LDS,
// in a fixed order, so the result is deterministic.  The N output rows are
// never written: a position reads its N-entry ainv row instead.
template <typename T, int VW, int KIND, int LAT>
__global__ void __launch_bounds__(512) ratio_kernel(const TableDesc d, const float* ainv,
                                                    int64_t ld_ainv, double* out) {
    constexpr int NOUT = Shape<KIND>::nout;
    __shared__ double red[8][NOUT];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int W = (int)(blockDim.x >> 6);
    for (int64_t pb = blockIdx.x; pb < d.npos; pb += gridDim.x) {
        const int p = (int)pb;
        double part[NOUT];
#pragma unroll
        for (int o = 0; o < NOUT; ++o) part[o] = 0.0;
        for (int c = wave; c < d.nchunks; c += W) {
            float acc[NOUT][VW];
            int n0, valid;
            eval_core<T, VW, KIND, LAT>(d, p, c, lane, acc, n0, valid);
            if (valid > 0) {
                float a[VW];
                const float* row = ainv + (int64_t)p * ld_ainv + n0;
#pragma unroll
                for (int e = 0; e < VW; ++e) a[e] = e < valid ? row[e] : 0.f;
#pragma unroll
                for (int o = 0; o < NOUT; ++o) {
                    float sum = 0.f;
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        if (e < valid) sum = fmaf(acc[o][e], a[e], sum);
                    part[o] += (double)sum;
                }
            }
        }
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) part[o] += __shfl_xor(part[o], off, 64);
        if (lane == 0)
#pragma unroll
            for (int o = 0; o < NOUT; ++o) red[wave][o] = part[o];
        __syncthreads();
        if (wave == 0 && lane < NOUT) {
            double sum = 0.0;
            for (int w = 0; w < W; ++w) sum += red[w][lane];
            out[(int64_t)p * NOUT + lane] = sum;
        }
        __syncthreads();
    }
}

template <typename T, int KIND, int LAT>
const void* pick_ratio(int vw) {
    if constexpr (Elem<T>::bytes == 4) {
        switch (vw) {
        case 1: return (const void*)&ratio_kernel<T, 1, KIND, LAT>;
        case 2: return (const void*)&ratio_kernel<T, 2, KIND, LAT>;
        case 4: return (const void*)&ratio_kernel<T, 4, KIND, LAT>;
        }
    } else {
        switch (vw) {
        case 2: return (const void*)&ratio_kernel<T, 2, KIND, LAT>;
        case 4: return (const void*)&ratio_kernel<T, 4, KIND, LAT>;
        case 8: return (const void*)&ratio_kernel<T, 8, KIND, LAT>;
        }
    }
    return nullptr;
}

template <typename T, int KIND>
const void* pick_ratio_lat(int vw, int lattice) {
    return lattice ? pick_ratio<T, KIND, 1>(vw) : pick_ratio<T, KIND, 0>(vw);
}

template <typename T, int KIND, int MAXT, int LAT>
const void* pick_kernel(int vw) {
    if constexpr (Elem<T>::bytes == 4) {
        switch (vw) {
        case 1: return (const void*)&eval_kernel<T, 1, KIND, MAXT, LAT>;
        case 2: return (const void*)&eval_kernel<T, 2, KIND, MAXT, LAT>;
        case 4: return (const void*)&eval_kernel<T, 4, KIND, MAXT, LAT>;
        }
    } else {
        switch (vw) {
        case 2: return (const void*)&eval_kernel<T, 2, KIND, MAXT, LAT>;
        case 4: return (const void*)&eval_kernel<T, 4, KIND, MAXT, LAT>;
        case 8: return (const void*)&eval_kernel<T, 8, KIND, MAXT, LAT>;
        }
    }
    return nullptr;
}

template <typename T, int KIND, int LAT, int SPLIT>
const void* pick_split(int vw) {
    if constexpr (Elem<T>::bytes == 4) {
        switch (vw) {
        case 1: return (const void*)&split_kernel<T, 1, KIND, LAT, SPLIT>;
        case 2: return (const void*)&split_kernel<T, 2, KIND, LAT, SPLIT>;
        case 4: return (const void*)&split_kernel<T, 4, KIND, LAT, SPLIT>;
        }
    } else {
        switch (vw) {
        case 2: return (const void*)&split_kernel<T, 2, KIND, LAT, SPLIT>;
        case 4: return (const void*)&split_kernel<T, 4, KIND, LAT, SPLIT>;
        case 8: return (const void*)&split_kernel<T, 8, KIND, LAT, SPLIT>;
        }
    }
    return nullptr;
}

template <typename T, int KIND>
const void* pick_split_kind(int vw, int lattice, int split) {
    if (split == 2)
        return lattice ? pick_split<T, KIND, 1, 2>(vw) : pick_split<T, KIND, 0, 2>(vw);
    if (split == 4)
        return lattice ? pick_split<T, KIND, 1, 4>(vw) : pick_split<T, KIND, 0, 4>(vw);
    return nullptr;
}

template <typename T, int KIND, int MAXT>
const void* pick_kernel_lat(int vw, int lattice) {
    return lattice ? pick_kernel<T, KIND, MAXT, 1>(vw) : pick_kernel<T, KIND, MAXT, 0>(vw);
}

}  // namespace
}  // namespace bspl

// The kernels of one table dtype, by kind, vector width, lattice form and
// split: each dtype's translation unit instantiates them (eval_f32.hip,
// eval_f16.hip, eval_bf16.hip) so that the three compile in parallel.
#define BSPL_DEFINE_KERNEL_TABLE(T)                                                        \
    const void* eval_kernel_ptr_##T(int kind, int vw, int multi, int lattice) {            \
        switch (kind) {                                                                    \
        case BSPL_V:                                                                       \
            return multi ? pick_kernel_lat<T, BSPL_V, kMaxTables>(vw, lattice)             \
                         : pick_kernel_lat<T, BSPL_V, 1>(vw, lattice);                     \
        case BSPL_VGL:                                                                     \
            return multi ? pick_kernel_lat<T, BSPL_VGL, kMaxTables>(vw, lattice)           \
                         : pick_kernel_lat<T, BSPL_VGL, 1>(vw, lattice);                   \
        case BSPL_VGH:                                                                     \
            return multi ? pick_kernel_lat<T, BSPL_VGH, kMaxTables>(vw, lattice)           \
                         : pick_kernel_lat<T, BSPL_VGH, 1>(vw, lattice);                   \
        }                                                                                  \
        return nullptr;                                                                    \
    }                                                                                      \
    const void* split_kernel_ptr_##T(int kind, int vw, int lattice, int split) {           \
        switch (kind) {                                                                    \
        case BSPL_V: return pick_split_kind<T, BSPL_V>(vw, lattice, split);                \
        case BSPL_VGL: return pick_split_kind<T, BSPL_VGL>(vw, lattice, split);            \
        case BSPL_VGH: return pick_split_kind<T, BSPL_VGH>(vw, lattice, split);            \
        }                                                                                  \
        return nullptr;                                                                    \
    }                                                                                      \
    const void* ratio_kernel_ptr_##T(int kind, int vw, int lattice) {                      \
        switch (kind) {                                                                    \
        case BSPL_V: return pick_ratio_lat<T, BSPL_V>(vw, lattice);                        \
        case BSPL_VGL: return pick_ratio_lat<T, BSPL_VGL>(vw, lattice);                    \
        case BSPL_VGH: return pick_ratio_lat<T, BSPL_VGH>(vw, lattice);                    \
        }                                                                                  \
        return nullptr;                                                                    \
    }

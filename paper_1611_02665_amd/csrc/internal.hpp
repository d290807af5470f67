// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "bspline.h"

struct bspl_table {
    bspl_table_info info;   // data / scales point at d_table / d_scales
    double grid_map[3][3];  // u = grid_map r: grid coordinates of a Cartesian position
    int lattice = 0;        // 1 when the cell is not an axis-aligned box
    void* d_table = nullptr;
    float* d_scales = nullptr;
    int device = 0;
};

namespace bspl {

// Most tables one batched launch can hold.
constexpr int kMaxTables = 16;
// Positions ordered together by one workgroup of the ordering pre-pass.
constexpr int kOrderChunk = 4096;
// XCDs of an MI355X; workgroups are dispatched to them round-robin.
constexpr int kXcds = 8;
// Splines per block of a spline-blocked table: the widest spline tile
// (64 lanes times the largest vector width of the dtype), so that every
// tile lies in one block.
inline int64_t block_splines_of(int dtype) { return dtype == BSPL_F32 ? 256 : 512; }

// Evaluation orders (bspl_tile.order): 0 input order; 1 cell-sorted; 2
// cell-sorted with each XCD taking a contiguous run of blocks; 3 input order,
// spline-tile-major; 4 as 2, spline-tile-major.  Position-major numbers the
// work blocks positions outer, spline tiles inner (a position's tiles run
// side by side); spline-tile-major numbers them tiles outer, so that all
// positions of one spline tile run before the next tile and a tile's rows
// stay in L2 while its positions are evaluated.
constexpr int kMaxOrder = 4;
inline bool order_sorted(int order) { return order == 1 || order == 2 || order == 4; }
inline bool order_xcd(int order) { return order == 2 || order == 4; }
inline bool order_tile_major(int order) { return order == 3 || order == 4; }

// Record a failure message for spline_last_error() and return the status.
bspl_status fail(bspl_status s, const char* fmt, ...);
bspl_status hip_fail(hipError_t e, const char* what);

#define BSPL_HIP(call)                                        \
    do {                                                      \
        hipError_t bspl_e_ = (call);                          \
        if (bspl_e_ != hipSuccess)                            \
            return ::bspl::hip_fail(bspl_e_, #call);          \
    } while (0)

// Everything a kernel needs to evaluate one table for one set of positions.
// Byte strides are 32-bit: the whole 4x4x4 row block of a cell lies within
// 4 GiB of its first row (checked at table creation).
struct TableDesc {
    const char* table;        // padded table
    const float* scales;      // per-spline scales (F16/BF16) or nullptr
    const double* pos;        // [3][npos]
    const int32_t* perm;      // evaluation order of the positions, or nullptr
    float* v;
    float* g;
    float* lh;
    int64_t npos;
    int64_t ldo;
    int64_t groups_begin;     // first workgroup-block index of this table
    // Row d: the grid map's row, u_d = sum_a axis[d][a] r_a (a box: n_d/L_d on
    // the diagonal), then the cell count n_d (as a double).  Lane d of a
    // wavefront reads its row with one 32-byte load alongside the position.
    double axis[3][4];
    int32_t lattice;          // 1: derivatives in grid units, then transformed by the map
    uint32_t row_bytes;       // bytes between consecutive z rows
    uint32_t ystride;         // bytes between consecutive y planes
    uint32_t xstride;         // bytes between consecutive x planes
    int64_t block_bytes;      // spline-blocked tables: bytes per block; plain: 0
    int32_t chunks_per_block; // spline tiles of 64*vw per block (plain: nchunks)
    int32_t nsplines;
    int32_t nchunks;          // spline tiles of 64*vw covering nsplines
    int32_t xgroups;          // blocks along splines: ceil(nchunks / wx)
    int32_t vec_store;        // outputs allow vw-wide vector stores
};

template <int MAXT>
struct KernelArgs {
    TableDesc t[MAXT];
    int64_t total_groups;
    int32_t ntables;
    int32_t wx;
    int32_t wy;
    int32_t xcd_remap;        // give each XCD a contiguous run of blocks
    int32_t tile_major;       // blocks numbered spline tiles outer, positions inner
};

// Fill a descriptor for table t (positions and outputs included).
bspl_status make_desc(const bspl_table* t, int64_t npos, const double* pos, float* v,
                      float* g, float* lh, int64_t ldo, int vw, int wx, int wy,
                      TableDesc* out);

bool tile_valid(const bspl_tile& tile, int dtype);
// The BSPL_TILE environment override: false when unset; *bad when unparsable.
bool env_tile(bspl_tile* out, bool* bad);
bspl_tile default_tile(const bspl_table_info& in, int kind, int64_t npos);

// Workgroups a launch of `groups` work blocks of `threads` threads each
// uses: all of them, or tile.grid persistent ones, and never more than one
// dispatch holds (2^32 - 1 work-items); the kernels stride over the rest.
inline int64_t launch_grid(int64_t groups, int32_t grid, int64_t threads) {
    int64_t g = groups;
    if (grid > 0 && grid < g) g = grid;
    const int64_t cap = (int64_t)UINT32_MAX / threads;
    if (g > cap) g = cap;
    return g < 1 ? 1 : g;
}

// The shape of one evaluation launch (host arithmetic only).
struct LaunchShape {
    int64_t units;       // work blocks: wx tiles x wy positions (split: wx tiles of one position)
    int64_t workgroups;  // workgroups launched
    int32_t threads;     // threads per workgroup
};
// EUNSUPPORTED for npos >= 2^31, more than 2^31 - 1 work blocks, or a split
// launch beyond 2^32 - 1 work-items; the tile must be valid for the dtype.
bspl_status launch_shape(const bspl_table_info& in, int64_t npos, const bspl_tile& tile,
                         LaunchShape* out);

// One evaluation, every argument and size checked before any HIP call.
// tile NULL: the tuned decomposition (tuned = true: spline_tile_select) or
// the built-in default (tuned = false: no wisdom lookup).  A cell-ordered
// tile takes its permutation from perm (perm_capacity positions; npos beyond
// that is EUNSUPPORTED), or from stream-ordered allocation when perm is NULL.
bspl_status eval_checked(const bspl_table* t, int kind, int64_t npos, const double* pos,
                         float* v, float* g, float* lh, int64_t ldo, const bspl_tile* tile,
                         bool tuned, int32_t* perm, int64_t perm_capacity, hipStream_t s);

// Kernel launchers (eval_launch.hip; kernels in eval_device.hpp).
bspl_status launch_single(const bspl_table* t, int kind, const TableDesc& d,
                          const bspl_tile& tile, hipStream_t s);
bspl_status launch_multi(int dtype, int kind, const KernelArgs<kMaxTables>& a,
                         const bspl_tile& tile, hipStream_t s);
bspl_status launch_ratio(const bspl_table* t, int kind, const TableDesc& d, const float* ainv,
                         int64_t ld_ainv, double* out, const bspl_tile& tile, hipStream_t s);
// Address of the batched kernel for a configuration (graph node building).
const void* multi_kernel_ptr(int dtype, int kind, int vw, int lattice);

// Cell-ordering pre-pass (order_kernels.hip): perm[i] for i < npos.
// OrderLaunch holds the launch shape and the argument values (args[] points
// into the struct, so it must not be copied after order_launch_config).
// OrderMap takes a Cartesian position to its fractional cell coordinates
// (grid coordinates divided by the cell counts, period 1 on every axis).
struct OrderMap {
    double f[3][3];
};
struct OrderLaunch {
    const double* pos;
    int npos;
    OrderMap map;
    int32_t* perm;
    unsigned grid, block, shmem;
    void* args[4];
};
void order_launch_config(const TableDesc& d, int32_t* perm, OrderLaunch* o);
bspl_status launch_order(const TableDesc& d, int32_t* perm, hipStream_t s);

// The cell orders of several tables' positions in one launch (batch plans):
// block b orders chunk b - chunk_begin[t] of the table t whose chunks hold b.
struct OrderItem {
    const double* pos;
    int32_t* perm;
    OrderMap map;
    int npos;
};
struct OrderTables {
    OrderItem t[kMaxTables];
    int32_t chunk_begin[kMaxTables + 1];  // first chunk of each table, then the total
    int ntables;
};
// Fills o with the tables of a whose perm is set; returns the total chunks.
int64_t order_tables_config(const KernelArgs<kMaxTables>& a, OrderTables* o);
bspl_status launch_order_tables(const OrderTables& o, hipStream_t s);
const void* order_tables_kernel_ptr();
unsigned order_block_threads();

// Latency mode: LDS bytes a split tile's partial sums take, and the limit.
constexpr int kSplitMaxLds = 65536;
int64_t split_lds_bytes(int kind, int vw, int wx, int split);

// Interpolating coefficients: three in-place axis passes, src -> dst (src may
// equal dst), both unpadded [nx][ny][nz][nspl] FP32 on the device.
bspl_status launch_fit(int nx, int ny, int nz, int64_t nspl, const float* src, float* dst,
                       hipStream_t s);
const void* order_kernel_ptr();

// Table layout kernels (layout_kernels.hip).
bspl_status build_table(bspl_table* t, const float* d_coefs, bool padded_input,
                        hipStream_t s);

// Wisdom cache (autotune.cpp).
// Entries keep the tile and its measured time in microseconds (< 0 when a
// wisdom line carried none).
bool wisdom_lookup(const char* key, bspl_tile* out, float* us = nullptr);
void wisdom_store(const char* key, const bspl_tile& tile, float us = -1.f);
// Key prefix of a table: base, then "-lattice" for a general cell and
// "-blocked" for the spline-blocked layout.
void key_prefix(char* buf, size_t n, const char* base, const bspl_table* t);
void wisdom_key(char* buf, size_t n, int dtype, int kind, int64_t nsplines,
                const int32_t ncell[3], int64_t npos, const char* prefix);

int device_cu_count();

// Autotuner pieces shared with the batched planner (autotune.cpp).
// Candidate tiles of the sweep; split (latency-mode) tiles only for single
// evaluations of at most kSplitMaxPositions positions.
constexpr int64_t kSplitMaxPositions = 1024;
std::vector<bspl_tile> tile_candidates(int dtype, int kind, int64_t max_nsplines, int64_t npos,
                                       bool persistent);
bspl_status fill_random_positions(double* pos, int64_t npos, const double box[3], uint64_t salt,
                                  hipStream_t s);
bspl_status sweep(const std::vector<bspl_tile>& cands, hipStream_t s,
                  bspl_status (*run)(void*, const bspl_tile&, int), void* ctx, bspl_tile* best,
                  float* best_us);
bspl_status record_wisdom(const char* path, const char* key, const bspl_tile& t, float us);

}  // namespace bspl

// Host side of the C ABI: status reporting, table layout and lifetime, and
// the single-table evaluation entry points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <cstdlib>

#include "internal.hpp"

namespace bspl {

namespace {
thread_local char g_last_error[512] = "";
}

bspl_status fail(bspl_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

bspl_status hip_fail(hipError_t e, const char* what) {
    const bspl_status s = (e == hipErrorOutOfMemory) ? BSPL_ENOMEM : BSPL_EDEVICE;
    return fail(s, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

int device_cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

bool tile_valid(const bspl_tile& tile, int dtype) {
    const bool f32 = dtype == BSPL_F32;
    const bool vw_ok = f32 ? (tile.vw == 1 || tile.vw == 2 || tile.vw == 4)
                           : (tile.vw == 2 || tile.vw == 4 || tile.vw == 8);
    const bool base_ok = vw_ok && tile.wx >= 1 && tile.wy >= 1 && tile.wx * tile.wy <= 8 &&
                         tile.grid >= 0 && tile.order >= 0 && tile.order <= kMaxOrder;
    if (tile.split == 0 || tile.split == 1) return base_ok;
    // a split unit is one workgroup per position: the block order is fixed
    return base_ok && (tile.split == 2 || tile.split == 4) && tile.wy == 1 && tile.grid == 0 &&
           tile.wx * tile.split <= 8 && tile.order <= 2;
}

// The decomposition used without a tuned one, from the measurements on
// gfx950: the narrowest vector width (one 4-byte load per lane and row, the
// fewest registers), up to 4 spline tiles per workgroup; cell order once
// positions are dense enough to share rows (64 npos / padded points >= 1/2)
// and the work amortises the ordering pass (npos * N >= 4M); and for a
// handful of positions the latency mode with 4 wavefronts per unit.
bspl_tile default_tile(const bspl_table_info& in, int kind, int64_t npos) {
    (void)kind;
    const int64_t n = in.n_splines;
    bspl_tile tile{};
    tile.vw = in.dtype == BSPL_F32 ? 1 : 2;
    const int64_t chunks = (n + 64 * tile.vw - 1) / (64 * tile.vw);
    tile.grid = 0;
    tile.order = 0;
    if (npos <= 16) {  // split * wx * n_out * vw * 256 B <= 20 KiB of LDS
        tile.wx = 1;
        tile.wy = 1;
        tile.split = 4;
        return tile;
    }
    tile.wx = (int)std::min<int64_t>(4, chunks);
    tile.wy = 1;
    tile.split = 1;
    const double points = (double)in.px * in.py * in.pz;
    if (64.0 * (double)npos >= 0.5 * points && (double)npos * (double)n >= 4194304.0)
        tile.order = 1;
    return tile;
}

// BSPL_TILE="vw,wx,wy,grid,order[,split]" overrides the tuned and default
// decompositions.  Returns false when the variable is unset; sets *bad when
// it is set but cannot be parsed.
bool env_tile(bspl_tile* out, bool* bad) {
    *bad = false;
    const char* e = std::getenv("BSPL_TILE");
    if (!e || !*e) return false;
    bspl_tile t{};
    t.split = 1;
    int used = 0, more = 0;
    if (sscanf(e, "%d,%d,%d,%d,%d%n", &t.vw, &t.wx, &t.wy, &t.grid, &t.order, &used) != 5) {
        *bad = true;
        return true;
    }
    if (e[used] == ',' && sscanf(e + used, ",%d%n", &t.split, &more) == 1) used += more;
    *bad = e[used] != '\0';
    *out = t;
    return true;
}

bspl_status launch_shape(const bspl_table_info& in, int64_t npos, const bspl_tile& tile,
                         LaunchShape* out) {
    if (npos < 0) return fail(BSPL_EINVAL, "npos %lld < 0", (long long)npos);
    if (npos > INT32_MAX) return fail(BSPL_EUNSUPPORTED, "npos beyond 2^31-1");
    if (!tile_valid(tile, in.dtype))
        return fail(BSPL_EINVAL,
                    "tile (vw=%d wx=%d wy=%d grid=%d order=%d split=%d) invalid for dtype %d",
                    tile.vw, tile.wx, tile.wy, tile.grid, tile.order, tile.split, in.dtype);
    const int64_t nchunks = (in.n_splines + 64 * tile.vw - 1) / (64 * tile.vw);
    const int64_t xgroups = (nchunks + tile.wx - 1) / tile.wx;
    LaunchShape ls{};
    if (tile.split > 1) {
        // one workgroup per (position, wx tiles): no striding loop
        ls.threads = 64 * tile.wx * tile.split;
        ls.units = npos * xgroups;
        if (ls.units > (int64_t)UINT32_MAX / ls.threads)
            return fail(BSPL_EUNSUPPORTED,
                        "split launch of %lld workgroups x %d threads exceeds 2^32-1 work-items",
                        (long long)ls.units, ls.threads);
        ls.workgroups = ls.units;
    } else {
        ls.threads = 64 * tile.wx * tile.wy;
        ls.units = xgroups * ((npos + tile.wy - 1) / tile.wy);
        if (ls.units > INT32_MAX)
            return fail(BSPL_EUNSUPPORTED, "too many work blocks (%lld)", (long long)ls.units);
        ls.workgroups = ls.units > 0 ? launch_grid(ls.units, tile.grid, ls.threads) : 0;
    }
    *out = ls;
    return BSPL_OK;
}

static bool aligned(const void* p, int bytes) {
    return p == nullptr || (reinterpret_cast<uintptr_t>(p) % (uintptr_t)bytes) == 0;
}

bspl_status make_desc(const bspl_table* t, int64_t npos, const double* pos, float* v, float* g,
                      float* lh, int64_t ldo, int vw, int wx, int wy, TableDesc* out) {
    // sizes first (host arithmetic, before any HIP call)
    {
        const int64_t nchunks = (t->info.n_splines + 64 * vw - 1) / (64 * vw);
        const int64_t groups = (nchunks + wx - 1) / wx * ((npos + wy - 1) / wy);
        if (npos > INT32_MAX) return fail(BSPL_EUNSUPPORTED, "npos beyond 2^31-1");
        if (groups > INT32_MAX)
            return fail(BSPL_EUNSUPPORTED, "too many work blocks (%lld)", (long long)groups);
    }
    // a table's memory belongs to the device it was created on
    int dev = -1;
    BSPL_HIP(hipGetDevice(&dev));
    if (dev != t->device)
        return fail(BSPL_EINVAL, "the table lives on device %d but device %d is current",
                    t->device, dev);
    const bspl_table_info& in = t->info;
    TableDesc d{};
    d.table = static_cast<const char*>(t->d_table);
    d.scales = t->d_scales;
    d.pos = pos;
    d.perm = nullptr;
    d.v = v;
    d.g = g;
    d.lh = lh;
    d.npos = npos;
    d.ldo = ldo;
    d.groups_begin = 0;
    const int ncell[3] = {in.nx, in.ny, in.nz};
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) d.axis[a][b] = t->grid_map[a][b];
        d.axis[a][3] = (double)ncell[a];
    }
    d.lattice = t->lattice;
    d.row_bytes = (uint32_t)in.row_bytes;
    d.ystride = (uint32_t)((int64_t)in.pz * in.row_bytes);
    d.xstride = (uint32_t)((int64_t)in.py * in.pz * in.row_bytes);
    d.nsplines = (int32_t)in.n_splines;
    d.nchunks = (int32_t)((in.n_splines + 64 * vw - 1) / (64 * vw));
    // a tile of 64*vw splines lies in one block (block_splines is a multiple)
    d.block_bytes = in.block_splines ? in.block_bytes : 0;
    d.chunks_per_block = in.block_splines ? (int32_t)(in.block_splines / (64 * vw))
                                          : std::max(d.nchunks, 1);
    d.xgroups = (d.nchunks + wx - 1) / wx;
    const int vb = 4 * vw;
    d.vec_store = (ldo % vw == 0) && aligned(v, vb) && aligned(g, vb) && aligned(lh, vb) ? 1 : 0;
    *out = d;
    return BSPL_OK;
}

}  // namespace bspl

using namespace bspl;

extern "C" {

const char* spline_status_string(bspl_status s) {
    switch (s) {
    case BSPL_OK: return "BSPL_OK";
    case BSPL_EINVAL: return "BSPL_EINVAL: invalid argument";
    case BSPL_ENOMEM: return "BSPL_ENOMEM: out of memory";
    case BSPL_EDEVICE: return "BSPL_EDEVICE: HIP runtime error";
    case BSPL_EUNSUPPORTED: return "BSPL_EUNSUPPORTED: unsupported request";
    case BSPL_EIO: return "BSPL_EIO: wisdom file error";
    default: break;
    }
    return "unknown bspl_status";
}

const char* spline_last_error(void) { return g_last_error; }

bspl_status spline_layout_query(int nx, int ny, int nz, int64_t n_splines, bspl_dtype dtype,
                                unsigned flags, bspl_table_info* out) {
    if (!out) return fail(BSPL_EINVAL, "out is NULL");
    if (nx <= 0 || ny <= 0 || nz <= 0 || n_splines <= 0)
        return fail(BSPL_EINVAL, "grid (%d,%d,%d) and n_splines %lld must be positive", nx, ny,
                    nz, (long long)n_splines);
    if (dtype != BSPL_F32 && dtype != BSPL_F16 && dtype != BSPL_BF16)
        return fail(BSPL_EINVAL, "bad dtype %d", (int)dtype);
    if (n_splines > (int64_t)1 << 30 || nx > (1 << 28) || ny > (1 << 28) || nz > (1 << 28))
        return fail(BSPL_EUNSUPPORTED, "sizes beyond 2^30 splines or 2^28 cells");
    bspl_table_info i{};
    i.nx = nx; i.ny = ny; i.nz = nz;
    i.px = nx + 3; i.py = ny + 3; i.pz = nz + 3;
    i.n_splines = n_splines;
    i.dtype = dtype;
    i.elem_bytes = dtype == BSPL_F32 ? 4 : 2;
    const int64_t per_row = 128 / i.elem_bytes;
    const int64_t bs = block_splines_of(dtype);
    if ((flags & BSPL_LAYOUT_BLOCKED) && n_splines > bs) {
        // [n_padded / bs][px][py][pz][bs]
        i.n_padded = (n_splines + bs - 1) / bs * bs;
        i.block_splines = bs;
        i.row_bytes = bs * i.elem_bytes;
        i.block_bytes = (int64_t)i.px * i.py * i.pz * i.row_bytes;
    } else {
        i.n_padded = (n_splines + per_row - 1) / per_row * per_row;
        i.row_bytes = i.n_padded * i.elem_bytes;
    }
    // overflow-checked px*py*pz*row_bytes
    const double est = (double)i.px * i.py * i.pz * (double)i.n_padded * i.elem_bytes;
    if (est > 9.0e18) return fail(BSPL_EUNSUPPORTED, "table of %.3g bytes overflows", est);
    i.table_bytes = (int64_t)i.px * i.py * i.pz * i.n_padded * i.elem_bytes;
    // the 4x4x4 block of a cell must span < 4 GiB (32-bit offsets in kernels)
    const double span = 3.0 * ((double)i.py * i.pz * i.row_bytes + (double)i.pz * i.row_bytes +
                               (double)i.row_bytes) + (double)i.row_bytes;
    if (span >= 4294967296.0)
        return fail(BSPL_EUNSUPPORTED, "one cell's row block spans %.3g bytes (>= 4 GiB)", span);
    i.box[0] = i.box[1] = i.box[2] = 1.0;
    i.lattice[0] = i.lattice[4] = i.lattice[8] = 1.0;
    *out = i;
    return BSPL_OK;
}

}  // extern "C"

namespace {

// Grid map of a cell with vectors a_i = lattice[3i..3i+2]: the grid
// coordinate of r along axis d is u_d = n_d * (r A^-1)_d, so
// M[d][a] = n_d * (A^-1)[a][d].  Fails for a singular or non-finite cell.
bspl_status grid_map_of(const double lat[9], const int n[3], double M[3][3], int* is_lattice) {
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(lat[k])) return fail(BSPL_EINVAL, "lattice[%d] is not finite", k);
    const double a00 = lat[0], a01 = lat[1], a02 = lat[2], a10 = lat[3], a11 = lat[4],
                 a12 = lat[5], a20 = lat[6], a21 = lat[7], a22 = lat[8];
    const double c00 = a11 * a22 - a12 * a21, c01 = a12 * a20 - a10 * a22,
                 c02 = a10 * a21 - a11 * a20;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    double norms = 1.0;
    for (int i = 0; i < 3; ++i)
        norms *= std::sqrt(lat[3 * i] * lat[3 * i] + lat[3 * i + 1] * lat[3 * i + 1] +
                           lat[3 * i + 2] * lat[3 * i + 2]);
    if (!(std::fabs(det) > 1e-12 * norms) || !(det > 0.0 || det < 0.0))
        return fail(BSPL_EINVAL, "the cell vectors are (nearly) linearly dependent");
    // inverse by the adjugate: inv[a][b] = cofactor[b][a] / det
    double inv[3][3];
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (a02 * a21 - a01 * a22) / det;
    inv[1][1] = (a00 * a22 - a02 * a20) / det;
    inv[2][1] = (a01 * a20 - a00 * a21) / det;
    inv[0][2] = (a01 * a12 - a02 * a11) / det;
    inv[1][2] = (a02 * a10 - a00 * a12) / det;
    inv[2][2] = (a00 * a11 - a01 * a10) / det;
    int off = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (i != j && lat[3 * i + j] != 0.0) off = 1;
    for (int dd = 0; dd < 3; ++dd)
        for (int a = 0; a < 3; ++a)
            M[dd][a] = off ? n[dd] * inv[a][dd] : (a == dd ? n[dd] / lat[4 * dd] : 0.0);
    *is_lattice = off;
    return BSPL_OK;
}

bspl_status create_table(bspl_table** out, int nx, int ny, int nz, int64_t n_splines,
                         const float* coefs, bspl_dtype dtype, const double lat[9],
                         unsigned flags, void* stream) {
    if (!out) return fail(BSPL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!coefs) return fail(BSPL_EINVAL, "coefs is NULL");
    if (flags & ~(BSPL_COEFS_PADDED | BSPL_COEFS_DEVICE | BSPL_COEFS_GRID_VALUES |
                  BSPL_LAYOUT_BLOCKED))
        return fail(BSPL_EINVAL, "unknown flags 0x%x", flags);
    if ((flags & BSPL_COEFS_PADDED) && (flags & BSPL_COEFS_GRID_VALUES))
        return fail(BSPL_EINVAL, "grid values are unpadded: BSPL_COEFS_PADDED with "
                                 "BSPL_COEFS_GRID_VALUES");
    bspl_table_info info{};
    bspl_status st = spline_layout_query(nx, ny, nz, n_splines, dtype, flags, &info);
    if (st != BSPL_OK) return st;
    const int ncell[3] = {nx, ny, nz};
    double gm[3][3];
    int is_lattice = 0;
    st = grid_map_of(lat, ncell, gm, &is_lattice);
    if (st != BSPL_OK) return st;
    for (int k = 0; k < 9; ++k) info.lattice[k] = lat[k];
    for (int k = 0; k < 3; ++k)
        info.box[k] = std::sqrt(lat[3 * k] * lat[3 * k] + lat[3 * k + 1] * lat[3 * k + 1] +
                                lat[3 * k + 2] * lat[3 * k + 2]);
    const bool padded = (flags & BSPL_COEFS_PADDED) != 0;
    const int64_t src_elems = padded ? (int64_t)info.px * info.py * info.pz * n_splines
                                     : (int64_t)nx * ny * nz * n_splines;
    hipStream_t s = static_cast<hipStream_t>(stream);

    bspl_table* t = new (std::nothrow) bspl_table();
    if (!t) return fail(BSPL_ENOMEM, "host allocation");
    t->info = info;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) t->grid_map[a][b] = gm[a][b];
    t->lattice = is_lattice;
    (void)hipGetDevice(&t->device);
    hipError_t e = hipMalloc(&t->d_table, (size_t)info.table_bytes);
    if (e != hipSuccess) {
        delete t;
        return hip_fail(e, "hipMalloc(table)");
    }
    if (dtype != BSPL_F32) {
        e = hipMalloc((void**)&t->d_scales, sizeof(float) * (size_t)info.n_padded);
        if (e != hipSuccess) {
            (void)hipFree(t->d_table);
            delete t;
            return hip_fail(e, "hipMalloc(scales)");
        }
    }
    // host coefficients are staged on the device; grid values are turned
    // into interpolating coefficients there (in the staging buffer, or in a
    // buffer of their own when the caller's values are on the device)
    const bool from_host = !(flags & BSPL_COEFS_DEVICE);
    const bool fit = (flags & BSPL_COEFS_GRID_VALUES) != 0;
    const float* d_src = coefs;
    float* staging = nullptr;
    if (from_host || fit) {
        e = hipMalloc((void**)&staging, sizeof(float) * (size_t)src_elems);
        if (e == hipSuccess && from_host)
            e = hipMemcpyAsync(staging, coefs, sizeof(float) * (size_t)src_elems,
                               hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            if (staging) (void)hipFree(staging);
            spline_table_destroy(t);
            return hip_fail(e, "staging coefficients on the device");
        }
        st = fit ? launch_fit(nx, ny, nz, n_splines, from_host ? staging : coefs, staging, s)
                 : BSPL_OK;
        if (st != BSPL_OK) {
            (void)hipFree(staging);
            spline_table_destroy(t);
            return st;
        }
        d_src = staging;
    }
    st = build_table(t, d_src, padded, s);
    if (staging) (void)hipFree(staging);
    if (st != BSPL_OK) {
        spline_table_destroy(t);
        return st;
    }
    t->info.data = t->d_table;
    t->info.scales = t->d_scales;
    *out = t;
    return BSPL_OK;
}

}  // namespace

extern "C" {

bspl_status spline_table_create(bspl_table** out, int nx, int ny, int nz, int64_t n_splines,
                                const float* coefs, bspl_dtype dtype, const double box[3],
                                unsigned flags, void* stream) {
    double lat[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    if (box) {
        for (int k = 0; k < 3; ++k) {
            if (!(box[k] > 0.0) || !std::isfinite(box[k])) {
                if (out) *out = nullptr;
                return fail(BSPL_EINVAL, "box[%d] = %g must be finite and > 0", k, box[k]);
            }
            lat[4 * k] = box[k];
        }
    }
    return create_table(out, nx, ny, nz, n_splines, coefs, dtype, lat, flags, stream);
}

bspl_status spline_table_create_lattice(bspl_table** out, int nx, int ny, int nz,
                                        int64_t n_splines, const float* coefs, bspl_dtype dtype,
                                        const double lattice[9], unsigned flags, void* stream) {
    if (!lattice) {
        if (out) *out = nullptr;
        return fail(BSPL_EINVAL, "lattice is NULL");
    }
    return create_table(out, nx, ny, nz, n_splines, coefs, dtype, lattice, flags, stream);
}

bspl_status spline_fit_interpolating(int nx, int ny, int nz, int64_t n_splines,
                                     const float* values, float* coefs, void* stream) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || n_splines <= 0)
        return fail(BSPL_EINVAL, "sizes must be positive (%d, %d, %d, %lld)", nx, ny, nz,
                    (long long)n_splines);
    if (!values || !coefs) return fail(BSPL_EINVAL, "values or coefs is NULL");
    const int64_t lim = INT64_MAX / 4;
    int64_t total = n_splines;
    for (int n : {nx, ny, nz}) {
        if (total > lim / n) return fail(BSPL_EUNSUPPORTED, "grid too large");
        total *= n;
    }
    return launch_fit(nx, ny, nz, n_splines, values, coefs, static_cast<hipStream_t>(stream));
}

bspl_status spline_table_destroy(bspl_table* t) {
    if (!t) return BSPL_OK;
    if (t->d_table) (void)hipFree(t->d_table);
    if (t->d_scales) (void)hipFree(t->d_scales);
    delete t;
    return BSPL_OK;
}

bspl_status spline_table_info(const bspl_table* t, bspl_table_info* out) {
    if (!t || !out) return fail(BSPL_EINVAL, "table or out is NULL");
    *out = t->info;
    return BSPL_OK;
}

bspl_status spline_tile_select(const bspl_table* t, bspl_kind kind, int64_t npos,
                               bspl_tile* out) {
    if (!t || !out) return fail(BSPL_EINVAL, "table or out is NULL");
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    bspl_tile tile;
    bool bad = false;
    if (env_tile(&tile, &bad)) {
        if (bad || !tile_valid(tile, t->info.dtype))
            return fail(BSPL_EINVAL, "BSPL_TILE=\"%s\" is not a valid tile for dtype %d",
                        std::getenv("BSPL_TILE"), (int)t->info.dtype);
        *out = tile;
        return BSPL_OK;
    }
    char key[256], prefix[64];
    const int32_t nc[3] = {t->info.nx, t->info.ny, t->info.nz};
    key_prefix(prefix, sizeof prefix, "single", t);
    wisdom_key(key, sizeof key, t->info.dtype, kind, t->info.n_splines, nc, npos, prefix);
    if (wisdom_lookup(key, &tile) && tile_valid(tile, t->info.dtype)) {
        *out = tile;
        return BSPL_OK;
    }
    *out = default_tile(t->info, kind, npos);
    return BSPL_OK;
}

bspl_status spline_launch_query(const bspl_table_info* layout, bspl_kind kind, int64_t npos,
                                const bspl_tile* tile, int64_t* units, int64_t* workgroups,
                                int32_t* threads) {
    if (!layout) return fail(BSPL_EINVAL, "layout is NULL");
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    if (layout->n_splines <= 0 || layout->dtype < BSPL_F32 || layout->dtype > BSPL_BF16)
        return fail(BSPL_EINVAL, "layout has n_splines %lld, dtype %d",
                    (long long)layout->n_splines, (int)layout->dtype);
    const bspl_tile tl = tile ? *tile : default_tile(*layout, kind, npos);
    LaunchShape ls;
    const bspl_status st = launch_shape(*layout, npos, tl, &ls);
    if (st != BSPL_OK) return st;
    if (units) *units = ls.units;
    if (workgroups) *workgroups = ls.workgroups;
    if (threads) *threads = ls.threads;
    return BSPL_OK;
}

}  // extern "C"

namespace bspl {

bspl_status eval_checked(const bspl_table* t, int kind, int64_t npos, const double* pos,
                         float* v, float* g, float* lh, int64_t ldo, const bspl_tile* tile,
                         bool tuned, int32_t* perm, int64_t perm_capacity, hipStream_t s) {
    if (!t) return fail(BSPL_EINVAL, "table is NULL");
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    if (npos < 0) return fail(BSPL_EINVAL, "npos %lld < 0", (long long)npos);
    if (ldo < t->info.n_splines)
        return fail(BSPL_EINVAL, "ldo %lld < n_splines %lld", (long long)ldo,
                    (long long)t->info.n_splines);
    if (npos == 0) return BSPL_OK;
    if (npos > INT32_MAX) return fail(BSPL_EUNSUPPORTED, "npos beyond 2^31-1");
    if (!pos || !v) return fail(BSPL_EINVAL, "pos or v is NULL");
    if (kind != BSPL_V && (!g || !lh)) return fail(BSPL_EINVAL, "g or l/h is NULL");
    bspl_tile tl;
    if (tile) {
        tl = *tile;
    } else if (tuned) {
        const bspl_status ts = spline_tile_select(t, static_cast<bspl_kind>(kind), npos, &tl);
        if (ts != BSPL_OK) return ts;
    } else {
        // the environment override, else the built-in default (no wisdom)
        bool bad = false;
        if (env_tile(&tl, &bad)) {
            if (bad || !tile_valid(tl, t->info.dtype))
                return fail(BSPL_EINVAL, "BSPL_TILE=\"%s\" is not a valid tile for dtype %d",
                            std::getenv("BSPL_TILE"), (int)t->info.dtype);
        } else {
            tl = default_tile(t->info, kind, npos);
        }
    }
    // every size limit is checked here, before any HIP call
    LaunchShape ls;
    bspl_status st = launch_shape(t->info, npos, tl, &ls);
    if (st != BSPL_OK) return st;
    if (order_sorted(tl.order) && perm && npos > perm_capacity)
        return fail(BSPL_EUNSUPPORTED,
                    "a cell-ordered evaluation of %lld positions needs more than the %lld "
                    "positions of static scratch memory", (long long)npos,
                    (long long)perm_capacity);
    TableDesc d;
    st = make_desc(t, npos, pos, v, kind == BSPL_V ? nullptr : g, kind == BSPL_V ? nullptr : lh,
                   ldo, tl.vw, tl.wx, tl.wy, &d);
    if (st != BSPL_OK) return st;
    if (!order_sorted(tl.order)) return launch_single(t, kind, d, tl, s);
    if (perm) {  // the caller's scratch: the permutation is fully rewritten
        st = launch_order(d, perm, s);
        if (st != BSPL_OK) return st;
        d.perm = perm;
        return launch_single(t, kind, d, tl, s);
    }
    // cell-ordered: the permutation lives in stream-ordered scratch memory
    BSPL_HIP(hipMallocAsync((void**)&perm, sizeof(int32_t) * (size_t)npos, s));
    st = launch_order(d, perm, s);
    if (st == BSPL_OK) {
        d.perm = perm;
        st = launch_single(t, kind, d, tl, s);
    }
    hipError_t e = hipFreeAsync(perm, s);
    if (st == BSPL_OK && e != hipSuccess) return hip_fail(e, "hipFreeAsync(permutation)");
    return st;
}

}  // namespace bspl

extern "C" {

bspl_status spline_eval(const bspl_table* t, bspl_kind kind, int64_t npos, const double* pos,
                        float* v, float* g, float* lh, int64_t ldo, const bspl_tile* tile,
                        void* stream) {
    return eval_checked(t, kind, npos, pos, v, g, lh, ldo, tile, true, nullptr, 0,
                        static_cast<hipStream_t>(stream));
}

bspl_status spline_eval_ratio(const bspl_table* t, bspl_kind kind, int64_t npos,
                              const double* pos, const float* ainv, int64_t ld_ainv, double* out,
                              const bspl_tile* tile, void* stream) {
    if (!t) return fail(BSPL_EINVAL, "table is NULL");
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    if (npos < 0) return fail(BSPL_EINVAL, "npos %lld < 0", (long long)npos);
    if (ld_ainv < t->info.n_splines)
        return fail(BSPL_EINVAL, "ld_ainv %lld < n_splines %lld", (long long)ld_ainv,
                    (long long)t->info.n_splines);
    if (npos == 0) return BSPL_OK;
    if (npos > INT32_MAX) return fail(BSPL_EUNSUPPORTED, "npos beyond 2^31-1");
    if (!pos || !ainv || !out) return fail(BSPL_EINVAL, "pos, ainv or out is NULL");
    bspl_tile tl;
    if (tile) {
        tl = *tile;
        if (!tile_valid(tl, t->info.dtype))
            return fail(BSPL_EINVAL, "tile invalid for dtype %d", t->info.dtype);
        if (tl.split > 1) return fail(BSPL_EINVAL, "split tiles are for evaluations only");
    } else {
        // two splines per lane and up to 8 wavefronts per position measured
        // best for the ratio kernel on gfx950 (valid for every dtype)
        tl = default_tile(t->info, kind, npos);
        tl.vw = 2;
        const int64_t chunks = (t->info.n_splines + 64 * tl.vw - 1) / (64 * tl.vw);
        tl.wx = (int)std::min<int64_t>(8, chunks);
        tl.wy = 1;
        tl.order = 0;
        tl.split = 1;
    }
    TableDesc d;
    bspl_status st = make_desc(t, npos, pos, nullptr, nullptr, nullptr, t->info.n_splines, tl.vw,
                               1, 1, &d);
    if (st != BSPL_OK) return st;
    return launch_ratio(t, kind, d, ainv, ld_ainv, out, tl, static_cast<hipStream_t>(stream));
}

bspl_status spline_eval_v(const bspl_table* t, int64_t npos, const double* pos, float* v,
                          int64_t ldo, void* stream) {
    return spline_eval(t, BSPL_V, npos, pos, v, nullptr, nullptr, ldo, nullptr, stream);
}

bspl_status spline_eval_vgl(const bspl_table* t, int64_t npos, const double* pos, float* v,
                            float* g, float* l, int64_t ldo, void* stream) {
    return spline_eval(t, BSPL_VGL, npos, pos, v, g, l, ldo, nullptr, stream);
}

bspl_status spline_eval_vgh(const bspl_table* t, int64_t npos, const double* pos, float* v,
                            float* g, float* h, int64_t ldo, void* stream) {
    return spline_eval(t, BSPL_VGH, npos, pos, v, g, h, ldo, nullptr, stream);
}

}  // extern "C"

/*
 * bspline.h - C ABI of the MI355X (gfx950) tricubic B-spline orbital
 * evaluator.
 *
 * The library evaluates N periodic tricubic B-spline orbitals at a batch of
 * electron positions (paper: "QMC and B-spline-based SPOs", Eq. SplineFunc
 * and Eq. TricubicValue; kernels V, VGL and VGH of section "Baseline and
 * miniQMC", Fig. 4(b)).  For each position it finds the grid cell, forms the
 * 4x4x4 cubic-basis weights and reduces the 64 coefficient rows of every
 * spline into:
 *   V   value                                   (1 output stream)
 *   VGL value, gradient, Laplacian              (1 + 3 + 1 streams)
 *   VGH value, gradient, symmetric Hessian      (1 + 3 + 6 streams)
 * Output streams are structure-of-arrays (section "Optimizations and
 * Parallelization", AoS-to-SoA subsection), one row of N per component.
 *
 * General conventions
 *  - Every function returns a bspl_status; nothing throws across the ABI.
 *    On failure spline_last_error() describes the cause (per thread).
 *  - Streams are passed as `void*` holding a hipStream_t (NULL = the null
 *    stream).  Evaluation is asynchronous and stream-ordered.
 *  - The caller owns position and output buffers; the library owns table and
 *    plan memory.  A table is immutable after creation and may be read by
 *    evaluations on several streams at once.
 *  - Positions are FP64 device arrays laid out [3][npos]: all x, then all y,
 *    then all z.  They are wrapped periodically into the box, so any finite
 *    position is valid.  A non-finite position yields NaN in every output of
 *    that position and never an out-of-bounds read.  A finite position so
 *    far out (|x/Delta| >= 2^50) that no fraction bits remain is evaluated at
 *    some grid point of the table.
 *  - Outputs are FP32 device arrays; element n of component c of position p
 *    is out[(p*ncomp + c)*ldo + n] with ldo >= N.  Columns [0,N) are
 *    overwritten (never accumulated into); columns [N,ldo) are not touched.
 *  - A table belongs to the device that was current when it was created;
 *    calls that use it must run with that device current.
 *
 * Errors common to every evaluation entry point (spline_eval*, the batch
 * plan calls): EINVAL for a NULL table, an unknown kind, npos < 0, ldo < N,
 * a NULL position or output buffer while npos > 0, an invalid tile, or a
 * table of another device; EUNSUPPORTED for npos >= 2^31, more than 2^31 - 1
 * work blocks, or a split (latency-mode) launch beyond 2^32 - 1 work-items
 * (spline_launch_query states these limits without a device); EDEVICE when
 * a HIP call fails (the launch itself; faults inside a kernel surface at the
 * next synchronising HIP call, as for any asynchronous work).  npos = 0 is a
 * successful no-op.  Size limits are checked before any HIP call, and after
 * an argument error (EINVAL, EUNSUPPORTED) nothing has been launched.  A
 * launch whose workgroups would exceed one dispatch (2^32 - 1 work-items)
 * runs as a persistent grid of fewer workgroups instead.
 */
#ifndef BSPLINE_H
#define BSPLINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Each enum also has a _ENUM_MIN and _ENUM_MAX member.  They are not values
 * to pass: they make every 32-bit int a valid value of the type, so that a
 * C caller's out-of-range value reaches the library well defined (and is
 * rejected with BSPL_EINVAL) in C++ as well.                              */
typedef enum {
    BSPL_OK = 0,
    BSPL_EINVAL = 1,       /* bad argument: NULL, non-positive size, bad enum */
    BSPL_ENOMEM = 2,       /* device or host allocation failed */
    BSPL_EDEVICE = 3,      /* a HIP call failed; see spline_last_error() */
    BSPL_EUNSUPPORTED = 4, /* valid request the library does not support */
    BSPL_EIO = 5,          /* wisdom file could not be read or written */
    BSPL_STATUS_ENUM_MIN = -2147483647 - 1,
    BSPL_STATUS_ENUM_MAX = 2147483647
} bspl_status;

/* Storage type of the coefficient table.  F16 and BF16 tables hold c/s_n
 * rounded to nearest-even, with a per-spline FP32 scale s_n = 2^ceil(log2
 * max|c_n|) (1 for an all-zero spline); evaluation converts to FP32,
 * accumulates in FP32 and multiplies each output by s_n once.             */
typedef enum {
    BSPL_F32 = 0,
    BSPL_F16 = 1,
    BSPL_BF16 = 2,
    BSPL_DTYPE_ENUM_MIN = -2147483647 - 1,
    BSPL_DTYPE_ENUM_MAX = 2147483647
} bspl_dtype;

/* Which outputs to produce (paper Fig. 3: V, VGL, VGH). */
typedef enum {
    BSPL_V = 0,
    BSPL_VGL = 1,
    BSPL_VGH = 2,
    BSPL_KIND_ENUM_MIN = -2147483647 - 1,
    BSPL_KIND_ENUM_MAX = 2147483647
} bspl_kind;

/* spline_table_create flags */
#define BSPL_COEFS_PADDED 0x1u /* coefs are [nx+3][ny+3][nz+3][N], used as-is */
#define BSPL_COEFS_DEVICE 0x2u /* coefs is a device pointer (else host)     */
#define BSPL_COEFS_GRID_VALUES 0x4u /* coefs are orbital values at the grid
                                       points; the table gets the interpolating
                                       coefficients (spline_fit_interpolating) */
#define BSPL_LAYOUT_BLOCKED 0x8u    /* store the table spline-blocked (see
                                       bspl_table_info); evaluation results are
                                       bit-identical to the plain layout      */

typedef struct bspl_table bspl_table;
typedef struct bspl_plan bspl_plan;

/* Layout of a table in device memory.  The plain table is 4-D,
 * [nx+3][ny+3][nz+3][n_padded]: one row of n_padded coefficients per padded
 * grid point, n fastest, each row starting on a 128-byte boundary (paper:
 * coefficient array P[Nx][Ny][Nz][N] with aligned, padded rows, section
 * "Baseline and miniQMC").  Padded index i holds the periodic coefficient
 * (i-1) mod n, so the 4 rows a cell needs are always i0..i0+3.
 * The spline-blocked table (BSPL_LAYOUT_BLOCKED; the paper's AoSoA table,
 * an array of sub-tables of N_b splines each, section "Optimizations and
 * Parallelization") is 5-D, [n_padded / B][nx+3][ny+3][nz+3][B] with
 * B = block_splines = 256 (F32) or 512 (F16/BF16), the widest spline tile,
 * so that the 4 z rows of a cell within one block are contiguous (a row of
 * B elements is 1 KB).  A spline tile of 64*vw splines always lies in one
 * block.  A table of at most B splines is a single block, which is the
 * plain layout (block_splines = 0).                                        */
typedef struct {
    int32_t nx, ny, nz;       /* grid cells per dimension */
    int32_t px, py, pz;       /* padded points per dimension (n + 3) */
    int64_t n_splines;        /* N */
    int64_t n_padded;         /* row length in elements (multiple of 128 B) */
    int32_t dtype;            /* bspl_dtype */
    int32_t elem_bytes;       /* 4 or 2 */
    int64_t row_bytes;        /* bytes between consecutive z rows: n_padded *
                                 elem_bytes (plain) or block_splines * elem_bytes */
    int64_t table_bytes;      /* px*py*pz*row_bytes */
    double box[3];            /* cell vector lengths (the box of an orthorhombic cell) */
    double lattice[9];        /* cell vectors a1, a2, a3 as rows (Cartesian) */
    const void* data;         /* device pointer to the table (read-only) */
    const float* scales;      /* device pointer to n_padded scales, or NULL */
    int64_t block_splines;    /* splines per block (spline-blocked), or 0 (plain) */
    int64_t block_bytes;      /* bytes of one block (spline-blocked), or 0 (plain) */
} bspl_table_info;

/* Work decomposition of one evaluation.  A wavefront (64 lanes) handles one
 * position and 64*vw consecutive splines at a time ("spline tile", the GPU
 * counterpart of the paper's AoSoA tile N_b, section "Optimizations and
 * Parallelization").  A workgroup holds wx tiles of the same positions
 * side by side and wy positions: wx*wy wavefronts, at most 8.  grid = 0
 * launches one workgroup per (wx tiles x wy positions) block; grid > 0
 * launches that many persistent workgroups that loop over the blocks.
 * order = 1 first groups the positions by the Morton code of their cell on
 * a 16x16x16 coarsening of the grid (a counting sort per chunk of 4096
 * positions, on the device, in stream-ordered scratch memory) so that
 * positions sharing table rows are evaluated together; order = 2 also hands
 * each of the 8 XCDs a contiguous run of the ordered blocks.  Orders 3 and
 * 4 number the work blocks spline tiles outer instead of positions outer:
 * every position of one spline tile is evaluated before the next tile, so
 * the rows of a tile stay in L2 while neighbouring positions re-read them
 * (order 3: positions in input order; order 4: cell-sorted and
 * XCD-grouped as order 2).  The order changes no result: every output is
 * computed the same way.  A single cell-sorted evaluation (order 1, 2 or
 * 4) takes its permutation from hipMallocAsync on the stream; for graph
 * replay use a batch plan, which owns that memory, or
 * spline_eval_noalloc.
 * split = 2 or 4 is the latency mode for a few positions (the GPU form of
 * the paper's nested threading within one walker, section "Optimizations
 * and Parallelization"): that many wavefronts share one (position, tile)
 * unit, each gathering 1/split of its 16 row groups with all of them in
 * flight, and the partial sums are added in LDS in a fixed order.  A split
 * workgroup holds wx tiles x split wavefronts of one position (wy must be
 * 1, grid 0, order at most 2, wx*split <= 8, and split*wx*n_out*vw*256
 * bytes of partial sums at most 64 KiB).  Results differ from split = 1 only by rounding; split
 * = 0 means 1.  Evaluations only (not ratios or batch plans).            */
typedef struct {
    int32_t vw;    /* splines per lane: 1, 2, 4 (F32) or 2, 4, 8 (F16/BF16) */
    int32_t wx;    /* wavefronts per workgroup along splines */
    int32_t wy;    /* wavefronts per workgroup along positions */
    int32_t grid;  /* persistent workgroups, or 0 */
    int32_t order; /* 0 input order, 1 cell-sorted, 2 cell-sorted + XCD-grouped,
                      3 input order tile-major, 4 as 2 tile-major */
    int32_t split; /* 0 or 1; 2 or 4 wavefronts per unit (latency mode) */
} bspl_tile;

/* Human-readable name of a status code (static string). */
const char* spline_status_string(bspl_status s);

/* Description of the last failure on the calling thread (static per thread;
 * empty string if none). */
const char* spline_last_error(void);

/* Host-only layout query: fills *out (data and scales set to NULL) for the
 * given shape and layout flag (0 or BSPL_LAYOUT_BLOCKED; other creation
 * flags are ignored) without touching the device.  EINVAL for non-positive
 * sizes or a bad dtype; EUNSUPPORTED when a size overflows 64-bit byte
 * counts or the 4x4x4 row block of one cell spans 4 GiB or more.         */
bspl_status spline_layout_query(int nx, int ny, int nz, int64_t n_splines,
                                bspl_dtype dtype, unsigned flags, bspl_table_info* out);

/* Create a table from FP32 coefficients.
 *  coefs: [nx][ny][nz][n_splines], n fastest, periodic (the coefficient of
 *         grid point (i,j,k) for spline n), on the host, or on the device
 *         with BSPL_COEFS_DEVICE; with BSPL_COEFS_PADDED the array is
 *         [nx+3][ny+3][nz+3][n_splines] and padded index i is used for
 *         cell i-1 directly (no periodic fill).
 *  flags: BSPL_COEFS_* as above, plus BSPL_LAYOUT_BLOCKED for the
 *         spline-blocked layout (spline_layout_select measures which layout
 *         is faster for a shape).
 *  box:   three box lengths (> 0), or NULL for the unit cube.
 *  The library copies, pads, converts and owns the table.  The call
 *  returns when the table is ready on the device; coefs may be freed then.
 *  Errors: EINVAL (NULL out/coefs, sizes <= 0, bad dtype, box <= 0),
 *  ENOMEM, EDEVICE, EUNSUPPORTED (see spline_layout_query).               */
bspl_status spline_table_create(bspl_table** out, int nx, int ny, int nz,
                                int64_t n_splines, const float* coefs,
                                bspl_dtype dtype, const double box[3],
                                unsigned flags, void* stream);

/* Create a table on a general (triclinic, e.g. hexagonal) periodic cell.
 *  lattice: the cell vectors a1, a2, a3 (Cartesian, rows of a 3x3 matrix,
 *  row-major).  Grid point (i, j, k) sits at (i/nx) a1 + (j/ny) a2 + (k/nz) a3;
 *  a position r has grid coordinates u = (nx s1, ny s2, nz s3) with
 *  s = r A^-1 its fractional coordinates, and wraps periodically in each of
 *  them.  Gradients and Hessians are Cartesian (grad_r = M^T grad_u,
 *  H_r = M^T H_u M with M = d u / d r), and the Laplacian is trace H_r.
 *  This is an extension beyond the paper's orthorhombic grids, needed for
 *  real orbitals on non-orthogonal cells.  A diagonal lattice is exactly
 *  spline_table_create with box = the diagonal.  Errors as
 *  spline_table_create; EINVAL also for a singular or non-finite lattice.  */
bspl_status spline_table_create_lattice(bspl_table** out, int nx, int ny, int nz,
                                        int64_t n_splines, const float* coefs,
                                        bspl_dtype dtype, const double lattice[9],
                                        unsigned flags, void* stream);

/* Interpolating coefficients (paper, "QMC and B-spline-based SPOs": the
 * coefficients are the orbitals' interpolation tables).  values and coefs
 * are device arrays [nx][ny][nz][n_splines], n fastest: values[i][j][k][n]
 * is orbital n at grid point (i, j, k); on return coefs holds the periodic
 * coefficients whose spline takes exactly those values at the grid points,
 * i.e. the solution of (c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i] (indices mod
 * n) along each axis.  The solve does not depend on the cell shape, so the
 * result serves box and lattice tables alike.  coefs == values (in place)
 * is allowed; any other overlap is undefined.  FP64 recursions, FP32
 * storage between the three axis passes.  Asynchronous on the stream.
 * Errors: EINVAL (sizes <= 0, NULL pointers), EUNSUPPORTED (byte count
 * overflow), EDEVICE.  The same fit runs inside spline_table_create and
 * spline_table_create_lattice when flags hold BSPL_COEFS_GRID_VALUES
 * (host or device values; not with BSPL_COEFS_PADDED).                   */
bspl_status spline_fit_interpolating(int nx, int ny, int nz, int64_t n_splines,
                                     const float* values, float* coefs, void* stream);

/* Free a table.  NULL is accepted.  No evaluation may still be in flight on
 * it (hipFree semantics). */
bspl_status spline_table_destroy(bspl_table* t);

/* Describe a table (device pointers included). */
bspl_status spline_table_info(const bspl_table* t, bspl_table_info* out);

/* Value only (paper Fig. 3, V).  v: [npos][ldo]. */
bspl_status spline_eval_v(const bspl_table* t, int64_t npos, const double* pos,
                          float* v, int64_t ldo, void* stream);

/* Value, gradient, Laplacian (paper Fig. 3, VGL).  v: [npos][ldo],
 * g: [npos][3][ldo] (gx, gy, gz), l: [npos][ldo] (trace of the Hessian). */
bspl_status spline_eval_vgl(const bspl_table* t, int64_t npos, const double* pos,
                            float* v, float* g, float* l, int64_t ldo, void* stream);

/* Value, gradient, Hessian (paper Fig. 4(b), VGH).  v: [npos][ldo],
 * g: [npos][3][ldo], h: [npos][6][ldo] ordered xx, xy, xz, yy, yz, zz.     */
bspl_status spline_eval_vgh(const bspl_table* t, int64_t npos, const double* pos,
                            float* v, float* g, float* h, int64_t ldo, void* stream);

/* Any kind with an explicit work decomposition (tile NULL = the tuned or
 * default one).  lh is l for VGL and h for VGH; g and lh are ignored for V.
 * EINVAL if the tile is not valid for the table's dtype.                   */
bspl_status spline_eval(const bspl_table* t, bspl_kind kind, int64_t npos,
                        const double* pos, float* v, float* g, float* lh,
                        int64_t ldo, const bspl_tile* tile, void* stream);

/* Host-only: the launch spline_eval makes for a table of this layout (from
 * spline_layout_query or spline_table_info) at npos positions with this
 * tile, or with the built-in default tile when tile is NULL (no wisdom is
 * consulted).  On success *units is the number of work blocks (wx spline
 * tiles x wy positions; split tiles: wx tiles of one position), *workgroups
 * the workgroups launched and *threads the threads per workgroup (any of
 * the three may be NULL).  A grid beyond one dispatch (2^32 - 1 work-items)
 * is reported as the persistent grid it becomes.  EINVAL for a NULL
 * layout, a bad kind or dtype, n_splines <= 0, npos < 0 or an invalid tile;
 * EUNSUPPORTED for npos >= 2^31, more than 2^31 - 1 work blocks or a split
 * launch beyond 2^32 - 1 work-items.  spline_eval applies exactly these
 * checks before any HIP call.                                             */
bspl_status spline_launch_query(const bspl_table_info* layout, bspl_kind kind, int64_t npos,
                                const bspl_tile* tile, int64_t* units, int64_t* workgroups,
                                int32_t* threads);

/* spline_eval without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, checks, kernels and results as
 * spline_eval, with two differences:
 *  - a cell-sorted tile (order 1, 2 or 4) keeps its permutation in a static
 *    device array of BSPL_NOALLOC_MAX_POSITIONS int32 entries (4 MiB, held
 *    by each device the library runs on until the process ends) instead of
 *    stream-ordered scratch memory; npos beyond that limit with an ordered
 *    tile is EUNSUPPORTED, checked before any HIP call.  Unordered tiles use
 *    no scratch memory at all.
 *  - tile NULL takes the BSPL_TILE override or the built-in default
 *    decomposition (spline_tile_select without the wisdom cache).
 * The call makes no hipMalloc, hipFree or other allocating call.  Every
 * ordered call on one device shares that device's array, and each call
 * rewrites the part it uses, so ordered calls that overlap in time on one
 * device (different streams, or host threads without ordering between
 * them) race and give undefined results; calls on one stream are ordered
 * by the stream.  The first call on a device looks up the array's device
 * address (hipGetSymbolAddress) with that device current.                 */
#define BSPL_NOALLOC_MAX_POSITIONS (1 << 20)
bspl_status spline_eval_noalloc(const bspl_table* t, bspl_kind kind, int64_t npos,
                                const double* pos, float* v, float* g, float* lh,
                                int64_t ldo, const bspl_tile* tile, void* stream);

/* Determinant ratios fused with the evaluation (paper, section "QMC and
 * B-spline-based SPOs": after a move of electron e the determinant ratio is
 * the sum over orbitals n of phi_n(r_e) times the inverse-matrix entry
 * linking orbital n and electron e, and the gradient ratio is the same sum
 * over grad phi_n).  For each position p:
 *     out[p*ncomp + c] = sum_{n<N} X_{c,n}(r_p) * ainv[p*ld_ainv + n]
 * with X the kind's components in the order of spline_eval (V: phi; VGL:
 * phi, gx, gy, gz, Laplacian; VGH: phi, gx, gy, gz, hxx, hxy, hxz, hyy, hyz,
 * hzz), ncomp = 1, 5 or 10.  ainv: device FP32 [npos][ld_ainv], row p being
 * the N inverse-matrix entries of the electron that position p moves (for
 * A[n][e] = phi_n(r_e), the entries (A^-1)[e][n], n = 0..N-1); ld_ainv >= N.
 * out: device FP64 [npos][ncomp], overwritten.  The N-wide output rows are
 * never materialised.  Products are formed in FP32 and summed in FP64 in a
 * fixed order (the result is deterministic).  tile: vw and wx (wavefronts
 * per position, at most 8) are used, NULL picks them.  Errors as spline_eval. */
bspl_status spline_eval_ratio(const bspl_table* t, bspl_kind kind, int64_t npos,
                              const double* pos, const float* ainv, int64_t ld_ainv,
                              double* out, const bspl_tile* tile, void* stream);

/* The decomposition spline_eval uses when given tile = NULL: the tuned one
 * from the wisdom cache if it holds this shape, else a built-in default:
 * the narrowest vector width with up to 4 spline tiles per workgroup, cell
 * order when positions are dense (64 npos >= half the padded grid points)
 * and npos * N >= 4M, and the latency mode (split 4) for npos <= 16.      */
bspl_status spline_tile_select(const bspl_table* t, bspl_kind kind, int64_t npos,
                               bspl_tile* out);
/* For experiments the environment variable BSPL_TILE="vw,wx,wy,grid,order"
 * or "vw,wx,wy,grid,order,split" overrides both the tuned and the default
 * decomposition here, in every evaluation given tile = NULL and in batch
 * plans created with tile = NULL (whose sweep it replaces; split must then
 * be 0 or 1).  A value that does not parse or is not valid for the table's
 * dtype makes those calls return EINVAL.  Ratios are not affected.        */

/* Autotuner (the paper tunes the tile size N_b once per machine by an
 * exhaustive sweep and plans an FFTW-like "wisdom" file, section
 * "Experiments and Results").  Times every valid decomposition on this
 * table at this batch size with uniformly random positions, keeps the
 * fastest in the in-process wisdom cache, appends it to wisdom_path when
 * that is not NULL, and returns it in *best (may be NULL).  Allocates and
 * frees its own scratch buffers; synchronizes the stream.                 */
bspl_status spline_autotune(const bspl_table* t, bspl_kind kind, int64_t npos,
                            const char* wisdom_path, bspl_tile* best, void* stream);

/* Layout selection (the paper tunes the AoSoA sub-table size with the tile
 * size, section "Experiments and Results").  Decides between the plain and
 * the spline-blocked layout for tables of this shape, dtype and kind at
 * this batch size, on box cells, and returns 0 or BSPL_LAYOUT_BLOCKED in
 * *layout.  Both layouts are built as temporary tables of the real shape
 * with random coefficients (timing does not depend on them), each runs at its
 * best tile (from the wisdom cache, else autotuned, recorded in the cache
 * and appended to wisdom_path when that is not NULL), and the two are
 * timed back to back on the same random positions, alternating which goes
 * first, 25 times.  The blocked layout is chosen only when the median of
 * the per-rep time ratio blocked/plain lies below 1 by more than twice its
 * spread (1.4826 x the median absolute deviation) and by at least 3 %
 * (the spread between two allocations of one layout);
 * otherwise the plain layout is kept.  Shapes of at most one block
 * (n_splines <= 256 for F32, 512 for F16/BF16) return 0 at once.  Needs
 * device memory for one table of each layout plus the unpadded
 * coefficients; synchronizes the stream.  Errors as spline_table_create
 * and spline_autotune.                                                    */
bspl_status spline_layout_select(int nx, int ny, int nz, int64_t n_splines, bspl_dtype dtype,
                                 bspl_kind kind, int64_t npos, const char* wisdom_path,
                                 unsigned* layout, void* stream);

/* Load wisdom entries from a file into the cache (EIO if unreadable).  One
 * entry per line: "key vw wx wy grid order split [time_us]"; other lines
 * (comments, older formats) are skipped.  Keys of spline-blocked tables
 * carry "-blocked" in their first field.                                  */
bspl_status spline_wisdom_load(const char* path);

/* Write the whole wisdom cache to a file, with the tile times it holds
 * (EIO on failure). */
bspl_status spline_wisdom_save(const char* path);

/* Batched evaluation of several tables in one kernel launch (a grid that
 * covers every unit, or grid > 0 persistent workgroups striding over
 * them), replayed from a captured HIP graph (paper: independent AoSoA tiles and walkers,
 * section "Optimizations and Parallelization", Fig. 6).  All tables must
 * share one dtype; they may differ in shape, N, cell and layout (plain or
 * spline-blocked).  npos[i] positions go to table i.  Buffers are bound at
 * plan creation:
 *   pos[i]   device [3][npos[i]] FP64
 *   v[i]     device [npos[i]][ldo[i]]
 *   g[i]     device [npos[i]][3][ldo[i]]           (VGL, VGH; else NULL)
 *   lh[i]    device l or h as for spline_eval       (VGL, VGH; else NULL)
 * tile: one decomposition for the whole launch (split must be 0 or 1), or
 * NULL to autotune it at plan creation (consulting and extending
 * wisdom_path when not NULL).
 * Tables and buffers must outlive the plan.  At most 16 tables.           */
bspl_status spline_batch_plan_create(bspl_plan** out, int ntables,
                                     const bspl_table* const* tables,
                                     const int64_t* npos, bspl_kind kind,
                                     const double* const* pos, float* const* v,
                                     float* const* g, float* const* lh,
                                     const int64_t* ldo, const bspl_tile* tile,
                                     const char* wisdom_path, void* stream);

/* Replay the plan's graph on a stream.  Returns as soon as it is queued. */
bspl_status spline_batch_execute(bspl_plan* p, void* stream);

/* The same work as spline_batch_execute, issued as plain kernel launches
 * (the ordering kernel when the tile is cell-ordered, then the evaluation
 * kernel) instead of a graph replay.  Results are bit-identical.  A graph
 * launch costs about 4.5 us more per call on MI355X, which matters for
 * small batches; these launches can also be captured into a caller's own
 * graph.  As with execute, calls on one plan must not overlap on different
 * streams (they share the plan's permutation buffer).                     */
bspl_status spline_batch_launch(bspl_plan* p, void* stream);

/* Rebind the buffers of table i in an existing plan (same npos and ldo
 * rules); takes effect from the next execute or launch.                   */
bspl_status spline_batch_rebind(bspl_plan* p, int i, const double* pos, float* v,
                                float* g, float* lh);

/* The decomposition a plan launches with. */
bspl_status spline_batch_plan_tile(const bspl_plan* p, bspl_tile* out);

/* Free a plan (NULL accepted).  No replay may still be in flight. */
bspl_status spline_batch_plan_destroy(bspl_plan* p);

#ifdef __cplusplus
}
#endif

#endif /* BSPLINE_H */

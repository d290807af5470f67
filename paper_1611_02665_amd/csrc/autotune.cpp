// Autotuner and wisdom cache.
//
// The paper tunes the tile size N_b once per machine by sweeping powers of
// two and plans an FFTW-like wisdom file for production runs (section
// "Experiments and Results").  Here the sweep covers every valid work
// decomposition (splines per lane, wavefronts per workgroup along splines
// and positions, persistent grid size), timed with HIP events on the real
// table at the real batch size; the winner is cached per
// (arch, dtype, kind, N, grid, npos bucket) and can be written to a text file.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "launch_check.hpp"

namespace bspl {

namespace {

// A cached decision: the tile, and its measured time when known (< 0 if not).
struct Entry {
    bspl_tile tile;
    float us;
};

std::mutex g_mu;
std::map<std::string, Entry>& cache() {
    static std::map<std::string, Entry> c;
    return c;
}

// gfx architecture of the current device, without feature suffixes; looked
// up once per device.
std::string arch_name() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    a = c == std::string::npos ? a : a.substr(0, c);
    names[dev] = a;
    return a;
}

int64_t pow2_bucket(int64_t n) {
    int64_t b = 1;
    while (b < n) b <<= 1;
    return b;
}

bool parse_line(const char* line, std::string* key, bspl_tile* t, float* us) {
    char k[256];
    bspl_tile x{};
    float time_us = -1.f;
    // key vw wx wy grid order split [time_us]
    const int n = sscanf(line, "%255s %d %d %d %d %d %d %f", k, &x.vw, &x.wx, &x.wy, &x.grid,
                         &x.order, &x.split, &time_us);
    if (n < 7) return false;
    *key = k;
    *t = x;
    *us = n == 8 ? time_us : -1.f;
    return true;
}

// Uniform random positions in the box: a counter hash per coordinate.
__global__ void random_positions(double* pos, int64_t npos, double lx, double ly, double lz,
                                 uint64_t salt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * npos) return;
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + salt;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    const int64_t d = i / npos;
    pos[i] = u * (d == 0 ? lx : (d == 1 ? ly : lz));
}

// Coefficients uniform in (-1, 1) from a counter hash, for tables that are
// built only to be timed.
__global__ void random_coefs(float* c, int64_t n, uint64_t salt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + salt;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    c[i] = (float)((double)(z >> 40) * (2.0 / 16777216.0) - 1.0);
}

}  // namespace

void wisdom_key(char* buf, size_t n, int dtype, int kind, int64_t nsplines, const int32_t nc[3],
                int64_t npos, const char* prefix) {
    static const char* dt[] = {"f32", "f16", "bf16"};
    static const char* kd[] = {"v", "vgl", "vgh"};
    snprintf(buf, n, "%s|%s|%s|%s|N%lld|%dx%dx%d|p%lld", prefix, arch_name().c_str(),
             dt[dtype], kd[kind], (long long)nsplines, nc[0], nc[1], nc[2],
             (long long)pow2_bucket(npos));
}

void key_prefix(char* buf, size_t n, const char* base, const bspl_table* t) {
    snprintf(buf, n, "%s%s%s", base, t->lattice ? "-lattice" : "",
             t->info.block_splines ? "-blocked" : "");
}

bool wisdom_lookup(const char* key, bspl_tile* out, float* us) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache().find(key);
    if (it == cache().end()) return false;
    *out = it->second.tile;
    if (us) *us = it->second.us;
    return true;
}

void wisdom_store(const char* key, const bspl_tile& tile, float us) {
    std::lock_guard<std::mutex> lk(g_mu);
    cache()[key] = Entry{tile, us};
}

// Candidate decompositions for a table (and, for batched launches, grid
// sizes as multiples of the compute-unit count).
std::vector<bspl_tile> tile_candidates(int dtype, int kind, int64_t max_nsplines, int64_t npos,
                                       bool persistent) {
    std::vector<bspl_tile> out;
    const int vws32[] = {1, 2, 4}, vws16[] = {2, 4, 8};
    const int* vws = dtype == BSPL_F32 ? vws32 : vws16;
    const int shapes[][2] = {{1, 1}, {2, 1}, {4, 1}, {8, 1}, {1, 2}, {1, 4},
                             {2, 2}, {4, 2}, {2, 4}, {1, 8}};
    const int cus = device_cu_count();
    const int grids_p[] = {0, 1, 2, 4, 8};
    const int grids_s[] = {0};
    for (int vi = 0; vi < 3; ++vi) {
        const int vw = vws[vi];
        const int64_t chunks = (max_nsplines + 64 * vw - 1) / (64 * vw);
        if (vi > 0 && chunks * 64 * vw > 2 * max_nsplines && chunks == 1) continue;
        for (auto& s : shapes) {
            if (s[0] > chunks && s[0] > 1) continue;
            const int* grids = persistent ? grids_p : grids_s;
            const int ng = persistent ? 5 : 1;
            for (int gi = 0; gi < ng; ++gi)
                for (int order = 0; order <= kMaxOrder; ++order)
                    out.push_back(bspl_tile{vw, s[0], s[1], grids[gi] * cus, order, 1});
        }
        // latency mode (single evaluations): wx tiles x split wavefronts per
        // position, input order
        if (persistent || npos > kSplitMaxPositions) continue;
        for (int split : {2, 4})
            for (int wx : {1, 2, 4}) {
                if (wx * split > 8 || (wx > chunks && wx > 1)) continue;
                if (split_lds_bytes(kind, vw, wx, split) > kSplitMaxLds) continue;
                out.push_back(bspl_tile{vw, wx, 1, 0, 0, split});
            }
    }
    return out;
}

// Timing events, destroyed on every return path.
struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    int n = 0;
    bspl_status create(int count) {
        for (n = 0; n < count; ++n) {
            const hipError_t err = hipEventCreate(&e[n]);
            if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
        }
        return BSPL_OK;
    }
    ~Events() {
        for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
    }
};

// Time `launch` (already bound to its buffers) with events: median of runs.
template <typename F>
static bspl_status time_launch(F&& launch, hipStream_t s, int reps, float* us) {
    Events ev;
    bspl_status st = ev.create(2);
    if (st != BSPL_OK) return st;
    for (int w = 0; w < 2; ++w) {
        st = launch(w);
        if (st != BSPL_OK) return st;
    }
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(ev.e[0], s);
        st = launch(r);
        (void)hipEventRecord(ev.e[1], s);
        const hipError_t e = hipEventSynchronize(ev.e[1]);
        if (st != BSPL_OK) return st;
        if (e != hipSuccess) return hip_fail(e, "autotune timing");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev.e[0], ev.e[1]);
        t.push_back(ms * 1000.f);
    }
    std::sort(t.begin(), t.end());
    *us = t[t.size() / 2];
    return BSPL_OK;
}

bspl_status fill_random_positions(double* pos, int64_t npos, const double box[3], uint64_t salt,
                                  hipStream_t s) {
    if (npos <= 0) return BSPL_OK;
    const int64_t n = 3 * npos;
    clear_last_error();
    hipLaunchKernelGGL(random_positions, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos,
                       npos, box[0], box[1], box[2], salt);
    BSPL_HIP(hipGetLastError());
    return BSPL_OK;
}

// Sweep tiles for a launch described by `run(tile, iteration)`: every
// candidate timed briefly (median of 5), then the fastest few again, side
// by side: 25 rounds in which each finalist runs once, the order rotating
// from round to round, and the median of its 25 times decides.  Timing the
// finalists interleaved keeps clock and cache drift over the sweep from
// deciding between tiles a few percent apart.
bspl_status sweep(const std::vector<bspl_tile>& cands, hipStream_t s,
                  bspl_status (*run)(void*, const bspl_tile&, int), void* ctx, bspl_tile* best,
                  float* best_us) {
    if (cands.empty()) return fail(BSPL_EUNSUPPORTED, "no candidate tile");
    std::vector<std::pair<float, size_t>> first;
    for (size_t i = 0; i < cands.size(); ++i) {
        float us = 0;
        auto call = [&](int it) { return run(ctx, cands[i], it); };
        bspl_status st = time_launch(call, s, 5, &us);
        if (st != BSPL_OK) return st;
        first.emplace_back(us, i);
    }
    std::sort(first.begin(), first.end());
    const size_t nf = std::min<size_t>(4, first.size());
    Events ev;
    bspl_status st = ev.create(2);
    if (st != BSPL_OK) return st;
    std::vector<std::vector<float>> t(nf);
    for (int r = 0; r < 25; ++r) {
        for (size_t k = 0; k < nf; ++k) {
            const size_t f = (k + (size_t)r) % nf;
            (void)hipEventRecord(ev.e[0], s);
            st = run(ctx, cands[first[f].second], r);
            (void)hipEventRecord(ev.e[1], s);
            const hipError_t e = hipEventSynchronize(ev.e[1]);
            if (st != BSPL_OK) return st;
            if (e != hipSuccess) return hip_fail(e, "autotune timing");
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev.e[0], ev.e[1]);
            t[f].push_back(ms * 1000.f);
        }
    }
    for (size_t f = 0; f < nf; ++f) {
        std::sort(t[f].begin(), t[f].end());
        const float us = t[f][t[f].size() / 2];
        if (f == 0 || us < *best_us) {
            *best = cands[first[f].second];
            *best_us = us;
        }
    }
    return BSPL_OK;
}

static bspl_status append_wisdom(const char* path, const char* key, const bspl_tile& t,
                                 float us) {
    FILE* f = fopen(path, "a");
    if (!f) return fail(BSPL_EIO, "cannot append to wisdom file %s", path);
    fprintf(f, "%s %d %d %d %d %d %d %.3f\n", key, t.vw, t.wx, t.wy, t.grid, t.order, t.split,
            us);
    const bool ok = fclose(f) == 0;
    return ok ? BSPL_OK : fail(BSPL_EIO, "cannot write wisdom file %s", path);
}

bspl_status record_wisdom(const char* path, const char* key, const bspl_tile& t, float us) {
    wisdom_store(key, t, us);
    return path ? append_wisdom(path, key, t, us) : BSPL_OK;
}

}  // namespace bspl

using namespace bspl;

namespace {

struct SingleCtx {
    const bspl_table* t;
    int kind;
    int64_t npos;
    double* pos[4];
    float* out[3];
    int64_t ldo;
    hipStream_t s;
};

bspl_status run_single(void* vctx, const bspl_tile& tile, int it) {
    SingleCtx* c = static_cast<SingleCtx*>(vctx);
    return spline_eval(c->t, static_cast<bspl_kind>(c->kind), c->npos, c->pos[it & 3],
                       c->out[0], c->out[1], c->out[2], c->ldo, &tile, c->s);
}

// Layout selection: the plain and the spline-blocked table of one shape,
// each at its best tile, timed back to back on the same positions.  Rep r
// times k launches of one layout, then k of the other (plain first on even
// reps, blocked first on odd ones), and the per-rep ratio blocked / plain
// is summarised by its median and its spread (1.4826 * median absolute
// deviation, the standard deviation of normal noise).  The spread of one
// race misses the difference between two allocations of the same layout
// (which pages the table lands on), measured at up to 2 % on MI355X, so the
// blocked layout must also win by at least 3 %.
constexpr int kLayoutReps = 25;
constexpr float kLayoutMinMargin = 0.03f;

struct LayoutRace {
    float* coefs = nullptr;
    bspl_table* t[2] = {nullptr, nullptr};
    bspl_tile tile[2] = {};
    void* mem = nullptr;

    bspl_status run(int kind, int64_t npos, hipStream_t s, float* ratio, float* noise) {
        const int ncomp = kind == BSPL_V ? 1 : (kind == BSPL_VGL ? 5 : 10);
        const int64_t ldo = t[0]->info.n_padded;
        const size_t pos_bytes = (sizeof(double) * 3 * (size_t)npos + 255) / 256 * 256;
        const size_t out_bytes = sizeof(float) * (size_t)npos * (size_t)ldo;
        BSPL_HIP(hipMalloc(&mem, 4 * pos_bytes + (size_t)ncomp * out_bytes));
        char* m = static_cast<char*>(mem);
        double* pos[4];
        for (int b = 0; b < 4; ++b) pos[b] = reinterpret_cast<double*>(m + b * pos_bytes);
        float* v = reinterpret_cast<float*>(m + 4 * pos_bytes);
        float* g = v + (size_t)npos * ldo;
        float* lh = g + (size_t)3 * npos * ldo;
        for (int b = 0; b < 4; ++b) {
            const bspl_status st = fill_random_positions(pos[b], npos, t[0]->info.box,
                                                         0x1a7000ull + b, s);
            if (st != BSPL_OK) return st;
        }
        auto launches = [&](int l, int k, int it0) {
            for (int i = 0; i < k; ++i) {
                const bspl_status st = spline_eval(t[l], static_cast<bspl_kind>(kind), npos,
                                                   pos[(it0 + i) & 3], v, g, lh, ldo, &tile[l], s);
                if (st != BSPL_OK) return st;
            }
            return BSPL_OK;
        };
        // launches per timing: about 300 us of work (at least 2)
        float us0 = 0.f;
        bspl_status st = time_launch([&](int it) { return launches(0, 1, it); }, s, 5, &us0);
        if (st != BSPL_OK) return st;
        const int k = std::min(64, std::max(2, (int)(300.f / std::max(us0, 1.f)) + 1));
        Events ev;
        st = ev.create(3);
        if (st != BSPL_OK) return st;
        std::vector<float> r;
        for (int rep = 0; rep < kLayoutReps; ++rep) {
            const int first = rep & 1;
            float ms[2] = {0.f, 0.f};
            (void)hipEventRecord(ev.e[0], s);
            st = launches(first, k, 2 * rep);
            (void)hipEventRecord(ev.e[1], s);
            if (st == BSPL_OK) st = launches(1 - first, k, 2 * rep);
            (void)hipEventRecord(ev.e[2], s);
            const hipError_t e = hipEventSynchronize(ev.e[2]);
            if (st != BSPL_OK) return st;
            if (e != hipSuccess) return hip_fail(e, "layout timing");
            (void)hipEventElapsedTime(&ms[first], ev.e[0], ev.e[1]);
            (void)hipEventElapsedTime(&ms[1 - first], ev.e[1], ev.e[2]);
            r.push_back(ms[1] / std::max(ms[0], 1e-6f));
        }
        std::sort(r.begin(), r.end());
        const float med = r[r.size() / 2];
        std::vector<float> dev;
        for (float x : r) dev.push_back(std::fabs(x - med));
        std::sort(dev.begin(), dev.end());
        *ratio = med;
        *noise = 1.4826f * dev[dev.size() / 2];
        return BSPL_OK;
    }

    void release(hipStream_t s) {
        (void)hipStreamSynchronize(s);
        for (int l = 0; l < 2; ++l)
            if (t[l]) spline_table_destroy(t[l]);
        if (mem) (void)hipFree(mem);
        if (coefs) (void)hipFree(coefs);
    }
};

}  // namespace

extern "C" {

bspl_status spline_autotune(const bspl_table* t, bspl_kind kind, int64_t npos,
                            const char* wisdom_path, bspl_tile* best, void* stream) {
    if (!t) return fail(BSPL_EINVAL, "table is NULL");
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    if (npos <= 0 || npos > INT32_MAX) return fail(BSPL_EINVAL, "npos %lld", (long long)npos);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ncomp = kind == BSPL_V ? 1 : (kind == BSPL_VGL ? 5 : 10);
    SingleCtx c{};
    c.t = t;
    c.kind = kind;
    c.npos = npos;
    c.ldo = t->info.n_padded;
    c.s = s;
    bspl_status st = BSPL_OK;
    void* mem = nullptr;
    const size_t pos_bytes = sizeof(double) * 3 * (size_t)npos;
    const size_t out_bytes = sizeof(float) * (size_t)npos * (size_t)c.ldo;
    const size_t total = 4 * pos_bytes + (size_t)ncomp * out_bytes + 4096;
    hipError_t e = hipMalloc(&mem, total);
    if (e != hipSuccess) return hip_fail(e, "autotune scratch");
    char* m = static_cast<char*>(mem);
    for (int b = 0; b < 4; ++b) {
        c.pos[b] = reinterpret_cast<double*>(m);
        m += (pos_bytes + 255) / 256 * 256;
    }
    c.out[0] = reinterpret_cast<float*>(m);
    c.out[1] = c.out[0] + (size_t)npos * c.ldo;
    c.out[2] = c.out[1] + (size_t)3 * npos * c.ldo;
    for (int b = 0; b < 4 && st == BSPL_OK; ++b)
        st = fill_random_positions(c.pos[b], npos, t->info.box, 0x5eed0000ull + b, s);
    bspl_tile bt{};
    float us = 0;
    if (st == BSPL_OK) {
        auto cands = tile_candidates(t->info.dtype, kind, t->info.n_splines, npos, false);
        st = sweep(cands, s, run_single, &c, &bt, &us);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(mem);
    if (st != BSPL_OK) return st;
    char key[256], prefix[64];
    const int32_t nc[3] = {t->info.nx, t->info.ny, t->info.nz};
    key_prefix(prefix, sizeof prefix, "single", t);
    wisdom_key(key, sizeof key, t->info.dtype, kind, t->info.n_splines, nc, npos, prefix);
    st = record_wisdom(wisdom_path, key, bt, us);
    if (best) *best = bt;
    return st;
}

bspl_status spline_layout_select(int nx, int ny, int nz, int64_t n_splines, bspl_dtype dtype,
                                 bspl_kind kind, int64_t npos, const char* wisdom_path,
                                 unsigned* layout, void* stream) {
    if (!layout) return fail(BSPL_EINVAL, "layout is NULL");
    *layout = 0;
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    if (npos <= 0 || npos > INT32_MAX) return fail(BSPL_EINVAL, "npos %lld", (long long)npos);
    bspl_table_info info{};
    bspl_status st = spline_layout_query(nx, ny, nz, n_splines, dtype, BSPL_LAYOUT_BLOCKED, &info);
    if (st != BSPL_OK) return st;
    if (info.block_splines == 0) return BSPL_OK;  // one block: the layouts coincide
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t nc[3] = {nx, ny, nz};
    const unsigned flags[2] = {0u, BSPL_LAYOUT_BLOCKED};
    const char* prefixes[2] = {"single", "single-blocked"};
    LayoutRace race{};
    // both layouts as temporary tables of the real shape, with random
    // coefficients like a real table's
    const size_t elems = (size_t)nx * ny * nz * (size_t)n_splines;
    hipError_t e = hipMalloc((void**)&race.coefs, sizeof(float) * elems);
    if (e == hipSuccess) {
        clear_last_error();
        hipLaunchKernelGGL(random_coefs, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s,
                           race.coefs, (int64_t)elems, 0xc0ef0000ull);
        e = hipGetLastError();
    }
    if (e != hipSuccess) st = hip_fail(e, "layout selection coefficients");
    for (int l = 0; l < 2 && st == BSPL_OK; ++l)
        st = spline_table_create(&race.t[l], nx, ny, nz, n_splines, race.coefs, dtype, nullptr,
                                 BSPL_COEFS_DEVICE | flags[l], stream);
    // each layout at its best tile: the wisdom cache, else a sweep
    for (int l = 0; l < 2 && st == BSPL_OK; ++l) {
        char key[256];
        wisdom_key(key, sizeof key, dtype, kind, n_splines, nc, npos, prefixes[l]);
        float us = -1.f;
        if (!(wisdom_lookup(key, &race.tile[l], &us) && us > 0.f))
            st = spline_autotune(race.t[l], kind, npos, wisdom_path, &race.tile[l], stream);
    }
    float ratio = 1.f, noise = 0.f;
    if (st == BSPL_OK) st = race.run(kind, npos, s, &ratio, &noise);
    race.release(s);
    if (st != BSPL_OK) return st;
    // blocked only when it wins by more than the measured noise
    *layout = ratio < 1.f - std::max(kLayoutMinMargin, 2.f * noise) ? BSPL_LAYOUT_BLOCKED : 0u;
    return BSPL_OK;
}

bspl_status spline_wisdom_load(const char* path) {
    if (!path) return fail(BSPL_EINVAL, "path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return fail(BSPL_EIO, "cannot open wisdom file %s", path);
    char line[512];
    while (fgets(line, sizeof line, f)) {
        std::string key;
        bspl_tile tile;
        float us = -1.f;
        if (line[0] == '#' || !parse_line(line, &key, &tile, &us)) continue;
        wisdom_store(key.c_str(), tile, us);
    }
    fclose(f);
    return BSPL_OK;
}

bspl_status spline_wisdom_save(const char* path) {
    if (!path) return fail(BSPL_EINVAL, "path is NULL");
    FILE* f = fopen(path, "w");
    if (!f) return fail(BSPL_EIO, "cannot create wisdom file %s", path);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& kv : cache()) {
            const bspl_tile& t = kv.second.tile;
            fprintf(f, "%s %d %d %d %d %d %d", kv.first.c_str(), t.vw, t.wx, t.wy, t.grid,
                    t.order, t.split);
            if (kv.second.us > 0.f) fprintf(f, " %.3f", kv.second.us);
            fputc('\n', f);
        }
    }
    return fclose(f) == 0 ? BSPL_OK : fail(BSPL_EIO, "cannot write wisdom file %s", path);
}

}  // extern "C"

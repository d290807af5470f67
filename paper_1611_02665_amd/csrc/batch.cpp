// Batched multi-table evaluation: one launch over a flattened
// work list of (table, position block, spline-tile block) units, built once
// into a HIP graph and replayed (spline_batch_execute), or issued as the
// same kernel launches without the graph (spline_batch_launch).
//
// This is the GPU form of the paper's independent AoSoA tiles and walkers
// (section "Optimizations and Parallelization", Fig. 6): every unit is
// independent, so workgroups stride over the list with no synchronisation.
// Units are numbered table by table (positions outer, spline tiles inner)
// and each table's first unit index is kept in its descriptor, so a unit
// finds its table with a scan over at most 16 prefix offsets.  All units
// move the same number of bytes (one spline tile of 64 rows), so a static
// stride over the list balances tables of very different size.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

struct bspl_plan {
    int ntables = 0;
    int dtype = 0;
    int kind = 0;
    bspl_tile tile{};
    const bspl_table* tables[bspl::kMaxTables] = {};
    int64_t npos[bspl::kMaxTables] = {};
    int64_t ldo[bspl::kMaxTables] = {};
    bspl::KernelArgs<bspl::kMaxTables> args{};
    int32_t* d_perm = nullptr;               // cell orders of all tables (sorted orders)
    int64_t perm_off[bspl::kMaxTables] = {};
    bspl::OrderTables otab{};                // the ordering launch's argument (sorted orders)
    void* oargs[1] = {};
    hipGraphNode_t order_node = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
    bool dirty = false;
};

namespace bspl {

static_assert(sizeof(KernelArgs<kMaxTables>) <= 4096, "kernel arguments must fit 4 KiB");
static_assert(sizeof(OrderTables) <= 4096, "kernel arguments must fit 4 KiB");

namespace {

struct Bindings {
    const double* pos[kMaxTables];
    float* v[kMaxTables];
    float* g[kMaxTables];
    float* lh[kMaxTables];
};

bspl_status build_args(const bspl_plan& p, const bspl_tile& tile, const Bindings& b,
                       KernelArgs<kMaxTables>* out, int32_t* perm_base = nullptr) {
    KernelArgs<kMaxTables> a{};
    int64_t begin = 0;
    for (int i = 0; i < p.ntables; ++i) {
        TableDesc d;
        const bool vonly = p.kind == BSPL_V;
        bspl_status st = make_desc(p.tables[i], p.npos[i], b.pos[i], b.v[i],
                                   vonly ? nullptr : b.g[i], vonly ? nullptr : b.lh[i], p.ldo[i],
                                   tile.vw, tile.wx, tile.wy, &d);
        if (st != BSPL_OK) return st;
        d.groups_begin = begin;
        if (order_sorted(tile.order) && perm_base) d.perm = perm_base + p.perm_off[i];
        begin += (int64_t)d.xgroups * ((p.npos[i] + tile.wy - 1) / tile.wy);
        a.t[i] = d;
    }
    if (begin > INT32_MAX) return fail(BSPL_EUNSUPPORTED, "too many work blocks");
    a.total_groups = begin;
    a.ntables = p.ntables;
    a.wx = tile.wx;
    a.wy = tile.wy;
    a.xcd_remap = order_xcd(tile.order) ? 1 : 0;
    a.tile_major = order_tile_major(tile.order) ? 1 : 0;
    *out = a;
    return BSPL_OK;
}

Bindings current_bindings(const bspl_plan& p) {
    Bindings b{};
    for (int i = 0; i < p.ntables; ++i) {
        b.pos[i] = p.args.t[i].pos;
        b.v[i] = p.args.t[i].v;
        b.g[i] = p.args.t[i].g;
        b.lh[i] = p.args.t[i].lh;
    }
    return b;
}

// A plan with any non-box cell runs the lattice form of the kernel for all
// of its tables (a box is a lattice with a diagonal map).
int plan_lattice(const bspl_plan& p) {
    for (int i = 0; i < p.ntables; ++i)
        if (p.tables[i]->lattice) return 1;
    return 0;
}

void batch_key(const bspl_plan& p, char* buf, size_t n) {
    std::string k;
    for (int i = 0; i < p.ntables; ++i) {
        char part[256];
        const bspl_table_info& in = p.tables[i]->info;
        const int32_t nc[3] = {in.nx, in.ny, in.nz};
        char prefix[64];
        snprintf(prefix, sizeof prefix, "%s%s",
                 i == 0 ? (plan_lattice(p) ? "batch-lattice" : "batch") : "",
                 in.block_splines ? "-blocked" : "");
        wisdom_key(part, sizeof part, in.dtype, p.kind, in.n_splines, nc, p.npos[i], prefix);
        k += (i == 0 ? "" : "+");
        k += part;
    }
    snprintf(buf, n, "%s", k.c_str());
}

int64_t grid_for(const KernelArgs<kMaxTables>& a, const bspl_tile& t) {
    return launch_grid(a.total_groups, t.grid, 64 * t.wx * t.wy);
}

struct TuneCtx {
    bspl_plan* p;
    Bindings b[2];
    int32_t* perm;
    hipStream_t s;
};

bspl_status run_batch(void* vctx, const bspl_tile& tile, int it) {
    TuneCtx* c = static_cast<TuneCtx*>(vctx);
    KernelArgs<kMaxTables> a;
    bspl_status st = build_args(*c->p, tile, c->b[it & 1], &a, c->perm);
    if (st != BSPL_OK) return st;
    if (order_sorted(tile.order)) {
        OrderTables o;
        order_tables_config(a, &o);
        st = launch_order_tables(o, c->s);
        if (st != BSPL_OK) return st;
    }
    return launch_multi(c->p->dtype, c->p->kind, a, tile, c->s);
}

// Sweep decompositions for the plan on scratch positions and outputs.
bspl_status autotune_plan(bspl_plan* p, hipStream_t s, bspl_tile* best, float* us) {
    const int ncomp = p->kind == BSPL_V ? 1 : (p->kind == BSPL_VGL ? 5 : 10);
    size_t total = 0;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    for (int i = 0; i < p->ntables; ++i)
        total += 2 * up(sizeof(double) * 3 * p->npos[i]) +
                 (size_t)ncomp * up(sizeof(float) * p->npos[i] * p->ldo[i]);
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, total + 256);
    if (e != hipSuccess) return hip_fail(e, "batch autotune scratch");
    TuneCtx c{};
    c.p = p;
    c.s = s;
    c.perm = p->d_perm;
    char* m = static_cast<char*>(mem);
    bspl_status st = BSPL_OK;
    int64_t max_n = 1;
    for (int i = 0; i < p->ntables && st == BSPL_OK; ++i) {
        max_n = std::max<int64_t>(max_n, p->tables[i]->info.n_splines);
        for (int k = 0; k < 2; ++k) {
            double* pos = reinterpret_cast<double*>(m);
            m += up(sizeof(double) * 3 * p->npos[i]);
            st = fill_random_positions(pos, p->npos[i], p->tables[i]->info.box,
                                       0xba7c0000ull + 16 * i + k, s);
            c.b[k].pos[i] = pos;
        }
        float* o[3];
        const size_t one = up(sizeof(float) * p->npos[i] * p->ldo[i]);
        o[0] = reinterpret_cast<float*>(m);
        o[1] = reinterpret_cast<float*>(m + one);
        o[2] = reinterpret_cast<float*>(m + 4 * one);
        m += (size_t)ncomp * one;
        for (int k = 0; k < 2; ++k) {
            c.b[k].v[i] = o[0];
            c.b[k].g[i] = p->kind == BSPL_V ? nullptr : o[1];
            c.b[k].lh[i] = p->kind == BSPL_V ? nullptr : o[2];
        }
    }
    if (st == BSPL_OK) {
        std::vector<bspl_tile> cands;
        // one grid over all units, or persistent workgroups striding over them
        for (const bspl_tile& t : tile_candidates(p->dtype, p->kind, max_n, 0, true))
            cands.push_back(t);
        st = sweep(cands, s, run_batch, &c, best, us);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(mem);
    return st;
}

// The ordering node's launch: every table's chunks in one grid.  Returns
// false when no table has positions to order.
bool order_params(bspl_plan* p, hipKernelNodeParams* kp) {
    const int64_t chunks = order_tables_config(p->args, &p->otab);
    p->oargs[0] = &p->otab;
    *kp = hipKernelNodeParams{};
    kp->func = const_cast<void*>(order_tables_kernel_ptr());
    kp->gridDim = dim3((unsigned)std::max<int64_t>(chunks, 1));
    kp->blockDim = dim3(order_block_threads());
    kp->sharedMemBytes = 0;
    kp->kernelParams = p->oargs;
    kp->extra = nullptr;
    return chunks > 0;
}

// Graph: [one ordering node for all tables (sorted orders)] -> one evaluation node.
bspl_status instantiate(bspl_plan* p) {
    const void* fn = multi_kernel_ptr(p->dtype, p->kind, p->tile.vw, plan_lattice(*p));
    if (!fn) return fail(BSPL_EINVAL, "no batched kernel for vw=%d", p->tile.vw);
    BSPL_HIP(hipGraphCreate(&p->graph, 0));
    std::vector<hipGraphNode_t> deps;
    if (order_sorted(p->tile.order)) {
        hipKernelNodeParams op;
        if (order_params(p, &op)) {
            BSPL_HIP(hipGraphAddKernelNode(&p->order_node, p->graph, nullptr, 0, &op));
            deps.push_back(p->order_node);
        }
    }
    hipKernelNodeParams kp{};
    void* params[] = {&p->args};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3((unsigned)grid_for(p->args, p->tile));
    kp.blockDim = dim3(64 * p->tile.wx * p->tile.wy);
    kp.sharedMemBytes = 0;
    kp.kernelParams = params;
    kp.extra = nullptr;
    BSPL_HIP(hipGraphAddKernelNode(&p->node, p->graph, deps.empty() ? nullptr : deps.data(),
                                   deps.size(), &kp));
    BSPL_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return BSPL_OK;
}

}  // namespace
}  // namespace bspl

using namespace bspl;

extern "C" {

bspl_status spline_batch_plan_create(bspl_plan** out, int ntables, const bspl_table* const* tables,
                                     const int64_t* npos, bspl_kind kind,
                                     const double* const* pos, float* const* v, float* const* g,
                                     float* const* lh, const int64_t* ldo, const bspl_tile* tile,
                                     const char* wisdom_path, void* stream) {
    if (!out) return fail(BSPL_EINVAL, "out is NULL");
    *out = nullptr;
    if (ntables < 1 || ntables > kMaxTables)
        return fail(BSPL_EINVAL, "ntables %d outside 1..%d", ntables, kMaxTables);
    if (!tables || !npos || !pos || !v || !ldo) return fail(BSPL_EINVAL, "NULL array argument");
    if (kind < BSPL_V || kind > BSPL_VGH) return fail(BSPL_EINVAL, "bad kind %d", (int)kind);
    if (kind != BSPL_V && (!g || !lh)) return fail(BSPL_EINVAL, "g or lh array is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    bspl_plan* p = new (std::nothrow) bspl_plan();
    if (!p) return fail(BSPL_ENOMEM, "host allocation");
    p->ntables = ntables;
    p->kind = kind;
    Bindings b{};
    for (int i = 0; i < ntables; ++i) {
        const bspl_table* t = tables[i];
        if (!t) { delete p; return fail(BSPL_EINVAL, "table %d is NULL", i); }
        if (i == 0) p->dtype = t->info.dtype;
        if (t->info.dtype != p->dtype) {
            delete p;
            return fail(BSPL_EUNSUPPORTED, "tables of one plan must share a dtype");
        }
        if (npos[i] < 0 || npos[i] > INT32_MAX) {
            delete p;
            return fail(BSPL_EINVAL, "npos[%d] = %lld", i, (long long)npos[i]);
        }
        if (ldo[i] < t->info.n_splines) {
            delete p;
            return fail(BSPL_EINVAL, "ldo[%d] < n_splines", i);
        }
        if (npos[i] > 0 && (!pos[i] || !v[i] || (kind != BSPL_V && (!g[i] || !lh[i])))) {
            delete p;
            return fail(BSPL_EINVAL, "buffers of table %d are NULL", i);
        }
        p->tables[i] = t;
        p->npos[i] = npos[i];
        p->ldo[i] = ldo[i];
        b.pos[i] = pos[i];
        b.v[i] = v[i];
        b.g[i] = kind == BSPL_V ? nullptr : g[i];
        b.lh[i] = kind == BSPL_V ? nullptr : lh[i];
    }
    bspl_status st = BSPL_OK;
    // permutation storage for cell-ordered tiles (allocated up front so the
    // autotuner can try them; a few bytes per position)
    int64_t total_pos = 0;
    for (int i = 0; i < ntables; ++i) {
        p->perm_off[i] = total_pos;
        total_pos += (p->npos[i] + 63) / 64 * 64;
    }
    if (total_pos > 0) {
        hipError_t e = hipMalloc((void**)&p->d_perm, sizeof(int32_t) * (size_t)total_pos);
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "hipMalloc(permutations)");
        }
    }
    if (tile) {
        if (!tile_valid(*tile, p->dtype)) {
            spline_batch_plan_destroy(p);
            return fail(BSPL_EINVAL, "tile invalid for dtype");
        }
        if (tile->split > 1) {
            spline_batch_plan_destroy(p);
            return fail(BSPL_EINVAL, "split tiles are for single evaluations only");
        }
        p->tile = *tile;
    } else {
        char key[2048];
        batch_key(*p, key, sizeof key);
        bspl_tile t;
        bool bad = false;
        const bool forced = env_tile(&t, &bad);
        if (forced && (bad || !tile_valid(t, p->dtype) || t.split > 1)) {
            spline_batch_plan_destroy(p);
            return fail(BSPL_EINVAL, "BSPL_TILE is not a valid plan tile for dtype %d", p->dtype);
        }
        if (wisdom_path && !forced) (void)spline_wisdom_load(wisdom_path);
        if (forced || (wisdom_lookup(key, &t) && tile_valid(t, p->dtype) && t.split <= 1)) {
            p->tile = t;
        } else {
            float us = 0;
            st = autotune_plan(p, s, &t, &us);
            if (st == BSPL_OK) st = record_wisdom(wisdom_path, key, t, us);
            if (st != BSPL_OK) {
                spline_batch_plan_destroy(p);
                return st;
            }
            p->tile = t;
        }
    }
    st = build_args(*p, p->tile, b, &p->args, p->d_perm);
    if (st == BSPL_OK) st = instantiate(p);
    if (st != BSPL_OK) {
        spline_batch_plan_destroy(p);
        return st;
    }
    *out = p;
    return BSPL_OK;
}

bspl_status spline_batch_execute(bspl_plan* p, void* stream) {
    if (!p) return fail(BSPL_EINVAL, "plan is NULL");
    if (p->args.total_groups == 0) return BSPL_OK;
    if (p->dirty) {
        if (p->order_node) {
            hipKernelNodeParams op;
            order_params(p, &op);
            BSPL_HIP(hipGraphExecKernelNodeSetParams(p->exec, p->order_node, &op));
        }
        hipKernelNodeParams kp{};
        void* params[] = {&p->args};
        kp.func = const_cast<void*>(multi_kernel_ptr(p->dtype, p->kind, p->tile.vw,
                                                     plan_lattice(*p)));
        kp.gridDim = dim3((unsigned)grid_for(p->args, p->tile));
        kp.blockDim = dim3(64 * p->tile.wx * p->tile.wy);
        kp.kernelParams = params;
        BSPL_HIP(hipGraphExecKernelNodeSetParams(p->exec, p->node, &kp));
        p->dirty = false;
    }
    BSPL_HIP(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
    return BSPL_OK;
}

bspl_status spline_batch_launch(bspl_plan* p, void* stream) {
    if (!p) return fail(BSPL_EINVAL, "plan is NULL");
    if (p->args.total_groups == 0) return BSPL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (order_sorted(p->tile.order)) {
        hipKernelNodeParams op;
        if (order_params(p, &op))
            BSPL_HIP(hipLaunchKernel(op.func, op.gridDim, op.blockDim, op.kernelParams,
                                     op.sharedMemBytes, s));
    }
    const void* fn = multi_kernel_ptr(p->dtype, p->kind, p->tile.vw, plan_lattice(*p));
    void* params[] = {&p->args};
    BSPL_HIP(hipLaunchKernel(fn, dim3((unsigned)grid_for(p->args, p->tile)),
                             dim3(64 * p->tile.wx * p->tile.wy), params, 0, s));
    return BSPL_OK;
}

bspl_status spline_batch_rebind(bspl_plan* p, int i, const double* pos, float* v, float* g,
                                float* lh) {
    if (!p) return fail(BSPL_EINVAL, "plan is NULL");
    if (i < 0 || i >= p->ntables) return fail(BSPL_EINVAL, "table index %d", i);
    if (p->npos[i] > 0 && (!pos || !v || (p->kind != BSPL_V && (!g || !lh))))
        return fail(BSPL_EINVAL, "NULL buffer");
    Bindings b = current_bindings(*p);
    b.pos[i] = pos;
    b.v[i] = v;
    b.g[i] = p->kind == BSPL_V ? nullptr : g;
    b.lh[i] = p->kind == BSPL_V ? nullptr : lh;
    KernelArgs<kMaxTables> a;
    bspl_status st = build_args(*p, p->tile, b, &a, p->d_perm);
    if (st != BSPL_OK) return st;
    p->args = a;
    p->dirty = true;
    return BSPL_OK;
}

bspl_status spline_batch_plan_tile(const bspl_plan* p, bspl_tile* out) {
    if (!p || !out) return fail(BSPL_EINVAL, "plan or out is NULL");
    *out = p->tile;
    return BSPL_OK;
}

bspl_status spline_batch_plan_destroy(bspl_plan* p) {
    if (!p) return BSPL_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_perm) (void)hipFree(p->d_perm);
    delete p;
    return BSPL_OK;
}

}  // extern "C"

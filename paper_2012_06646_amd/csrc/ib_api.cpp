// Host runtime of libibops: argument checking, plan workspace layout and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "ib.h"
#include "ib_host.h"
#include "ib_internal.h"

using namespace ibk;

namespace ibk {

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int bits_for(int64_t G)
{
    int b = 0;
    while ((int64_t(1) << b) < G) ++b;
    return b;
}

// Validate a descriptor; fill the distinct staggerings.
int32_t check_grid(const ib_grid_desc* g, int32_t dtype, int64_t npts, int* nstag,
                   int comp_stag[3], double stag_xi[3][3])
{
    if (!g) return IB_ERR_ARG;
    if (g->dim != 2 && g->dim != 3) return IB_ERR_UNSUPPORTED;
    if (dtype != IB_F64 && dtype != IB_F32) return IB_ERR_UNSUPPORTED;
    if (g->kernel < 0 || g->kernel >= IB_KERNEL_COUNT) return IB_ERR_UNSUPPORTED;
    if (g->ncomp < 1 || g->ncomp > 3) return IB_ERR_ARG;
    if (npts < 0) return IB_ERR_ARG;
    if (npts > MAX_POINTS) return IB_ERR_UNSUPPORTED;
    if (g->walls < 0 || g->walls >= (1 << g->dim)) return IB_ERR_ARG;
    int64_t G = 1;
    for (int k = 0; k < g->dim; ++k) {
        if (g->n[k] < 4) return IB_ERR_UNSUPPORTED;
        if (!(g->length[k] > 0.0) || !std::isfinite(g->length[k])) return IB_ERR_ARG;
        G *= (int64_t)g->n[k] + (((g->walls >> k) & 1) ? IB_WALL_GHOSTS : 0);
        if (G > 2147483647LL) return IB_ERR_UNSUPPORTED;
    }
    int ns = 0;
    for (int c = 0; c < g->ncomp; ++c) {
        for (int k = 0; k < g->dim; ++k) {
            const double xi = g->stagger[c][k];
            if (!(xi >= 0.0 && xi < 1.0)) return IB_ERR_ARG;
        }
        int found = -1;
        for (int s = 0; s < ns && found < 0; ++s) {
            bool same = true;
            for (int k = 0; k < g->dim; ++k) same &= (stag_xi[s][k] == g->stagger[c][k]);
            if (same) found = s;
        }
        if (found < 0) {
            for (int k = 0; k < 3; ++k) stag_xi[ns][k] = k < g->dim ? g->stagger[c][k] : 0.0;
            found = ns++;
        }
        comp_stag[c] = found;
    }
    *nstag = ns;
    return IB_OK;
}

int32_t check_tuning(const ib_tuning* t, int32_t dtype)
{
    if (!t) return IB_OK;
    if (t->spread_tile < 0 || t->spread_tile > SPREAD_TILE_SHAPES) return IB_ERR_ARG;
    if (t->radix_bits != 0 && (t->radix_bits < 4 || t->radix_bits > max_bucket_bits(dtype))) return IB_ERR_ARG;
    return IB_OK;
}

// Bucket digit bits of a plan: enough buckets that each spans at most BKT_CELLS cells (up
// to 2^max_bucket_bits(dtype) buckets), and about one bucket per 2048 points up to 2^10
// buckets, so that a bucket's points usually fit its block's LDS; a tuning may ask for a
// width of its own.
int bucket_bits(int64_t G, int64_t n, int tuned, int32_t dtype)
{
    const int bits = bits_for(G);
    const int cap = max_bucket_bits(dtype);
    int rb;
    if (tuned > 0) {
        rb = tuned;
    } else {
        int want = 0;
        while (want < 10 && (int64_t(2048) << want) < n) ++want;
        rb = std::max(bits - 13, want);  // 2^13 = BKT_CELLS
    }
    rb = std::min(rb, cap);
    return std::max(0, std::min(rb, bits));
}

ib_grid_desc kernel_grid(const ib_grid_desc& g)
{
    ib_grid_desc k = g;
    k.walls = 0;
    for (int d = 0; d < g.dim; ++d)
        if ((g.walls >> d) & 1) {
            k.n[d] = g.n[d] + IB_WALL_GHOSTS;
            k.length[d] = g.length[d] / g.n[d] * k.n[d];  // only the index range matters
        }
    return k;
}

void make_layout(const ib_grid_desc* user, int32_t dtype, int nstag, int64_t n, Layout* L,
                 const ib_tuning* tuning)
{
    const ib_grid_desc kg = kernel_grid(*user);
    const ib_grid_desc* g = &kg;
    L->nstag = nstag;
    L->G = 1;
    for (int k = 0; k < g->dim; ++k) L->G *= g->n[k];
    L->rows = (int)(L->G / g->n[0]);
    L->rb = bucket_bits(L->G, n, tuning ? tuning->radix_bits : 0, dtype);
    L->cb = bits_for(L->G) - L->rb;
    L->ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    L->nseg_tiles = n > 0 ? (n + SORT_TILE - 1) / SORT_TILE : 1;
    const int64_t R = int64_t(1) << L->rb;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t kn = (size_t)nstag * (size_t)n * sizeof(int32_t);
    L->kin = take(kn);
    L->kA = take(kn);
    L->vA = take(kn);
    L->kB = take(kn);
    L->vB = take(kn);
    L->cstart = take(((size_t)L->G + 1) * sizeof(int32_t));
    L->seg_off = take((size_t)nstag * (size_t)(n + 1) * sizeof(int32_t));
    L->q = take((size_t)nstag * sizeof(int32_t));
    const size_t b = dtype == IB_F64 ? 8 : 4;
    L->Xs = take((size_t)n * g->dim * b);
    L->Xb = take((size_t)n * g->dim * b);
    L->Xn = take((size_t)n * g->dim * b);
    L->Us = take(g->dim == 3 ? (size_t)n * 2 * b : 0);
    int tiles[3];
    // ib_tuning.spread_tile: 0 = the built-in shape of the precision, k = shape k - 1.
    L->sp_tile = g->dim != 3 ? 0
                 : (tuning && tuning->spread_tile > 0) ? tuning->spread_tile - 1
                                                       : builtin_spread_shape(dtype);
    int slow;
    spread_tiles(g->dim, L->sp_tile, g->n, tiles, &slow);
    L->sp_tiles = tiles[0] * tiles[1] * tiles[2] * g->ncomp;
    L->split = spread_split(n, L->sp_tiles, tuning ? tuning->split_points : 0);
    L->partial = take(L->split > 1 ? (size_t)L->split * L->sp_tiles *
                                         spread_tile_cells(g->dim, L->sp_tile) * sizeof(long long)
                                   : 0);
    L->tile_shift = take(L->split > 1 ? (size_t)L->sp_tiles * sizeof(int32_t) : 0);
    L->fmax = take((size_t)3 * FMAX_PARTS * sizeof(unsigned long long));
    // Everything from here to zero_end starts each update cleared (clear_once, bucket pass).
    L->zero_begin = off;
    L->seg_status = take((size_t)nstag * L->nseg_tiles * sizeof(uint32_t));
    L->bhist = take((size_t)nstag * 3 * BKT_SHARDS * R * sizeof(uint32_t));
    L->counters = take((size_t)nstag * PLAN_COUNTERS * sizeof(uint32_t));
    L->flag = take(sizeof(uint32_t));
    L->bad = take(sizeof(uint32_t));
    L->cellmax = take(sizeof(uint32_t));
    L->crowd = take(sizeof(uint32_t));
    L->zero_end = off;
    L->total = off;
}

int32_t hip_status(hipError_t e) { return e == hipSuccess ? IB_OK : IB_ERR_HIP; }

}  // namespace ibk

extern "C" {

const char* ib_status_string(int32_t s)
{
    switch (s) {
    case IB_OK: return "ok";
    case IB_ERR_ARG: return "invalid argument";
    case IB_ERR_OOM: return "out of memory (workspace too small or host allocation failed)";
    case IB_ERR_HIP: return "HIP runtime error";
    case IB_ERR_UNSUPPORTED: return "unsupported configuration";
    case IB_ERR_BUSY: return "busy";
    case IB_ERR_DEVICE_FLAG: return "device flagged a data error (non-finite or out-of-range position)";
    case IB_PENDING: return "pending";
    default: return "unknown status";
    }
}

size_t ib_plan_workspace_bytes(const ib_grid_desc* grid, int32_t dtype, int64_t npts)
{
    int nstag, cs[3];
    double sx[3][3];
    if (check_grid(grid, dtype, npts, &nstag, cs, sx) != IB_OK) return 0;
    Layout L;
    make_layout(grid, dtype, nstag, npts, &L, nullptr);
    return L.total;
}

}  // extern "C"

namespace ibk {

void plan_setup(ib_plan_s* p, const ib_grid_desc* user, int32_t dtype, int64_t npts, int nstag,
                const int cs[3], const double sx[3][3], const Layout& L, void* workspace)
{
    p->user = *user;
    p->grid = kernel_grid(*user);
    const ib_grid_desc* grid = &p->grid;
    p->dtype = dtype;
    p->npts = npts;
    GeomArgs& g = p->sa.g;
    std::memset(&g, 0, sizeof g);
    g.dim = grid->dim;
    g.ncomp = grid->ncomp;
    g.nstag = nstag;
    g.rows = L.rows;
    g.npts = npts;
    double hd = 1.0;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = k < grid->dim ? grid->n[k] : 1;
        if (k >= grid->dim) {
            g.inv_h_d[k] = 1.0;
            g.inv_h_f[k] = 1.0f;
            continue;
        }
        // spacing from the caller's grid (a walled dimension keeps it; only indices differ)
        const double N = user->n[k], Lk = user->length[k];
        g.inv_n[k] = 1.0 / grid->n[k];
        g.inv_h_d[k] = N / Lk;
        g.inv_lo_d[k] = (double)((long double)N / (long double)Lk - (long double)g.inv_h_d[k]);
        g.inv_h_f[k] = (float)user->n[k] / (float)user->length[k];
        g.inv_lo_f[k] = (float)((long double)N / (long double)Lk - (long double)g.inv_h_f[k]);
        hd *= Lk / N;
    }
    g.scale = 1.0 / hd;
    g.split = L.split;
    g.sp_tile = L.sp_tile;
    g.odd = grid->kernel == IB_KERNEL_ROMA3 ? 1 : 0;
    for (int c = 0; c < grid->ncomp; ++c) {
        g.comp_stag[c] = cs[c];
        for (int k = 0; k < 3; ++k) {
            g.comp_xi[c][k] = k < grid->dim ? grid->stagger[c][k] : 0.0;
            // floor(t - xi_c) - floor(t - xi_0) lies in [dlo, dhi]
            const double d = k < grid->dim ? grid->stagger[0][k] - grid->stagger[c][k] : 0.0;
            g.dlo[c][k] = d < 0.0 ? -1 : 0;
            g.dhi[c][k] = d > 0.0 ? 1 : 0;
        }
    }
    for (int s = 0; s < nstag; ++s)
        for (int k = 0; k < 3; ++k) g.stag_xi[s][k] = sx[s][k];

    char* base = (char*)workspace;
    PlanDev& d = p->sa.d;
    d.kin = (int32_t*)(base + L.kin);
    d.kA = (int32_t*)(base + L.kA);
    d.vA = (int32_t*)(base + L.vA);
    d.kB = (int32_t*)(base + L.kB);
    d.vB = (int32_t*)(base + L.vB);
    d.bhist = (uint32_t*)(base + L.bhist);
    d.cstart = (int32_t*)(base + L.cstart);
    d.seg_off = (int32_t*)(base + L.seg_off);
    d.q = (int32_t*)(base + L.q);
    d.Xs = base + L.Xs;
    d.Xb = base + L.Xb;
    d.Xn = base + L.Xn;
    d.Us = base + L.Us;
    d.partial = (long long*)(base + L.partial);
    d.tile_shift = (int32_t*)(base + L.tile_shift);
    d.fmax = (unsigned long long*)(base + L.fmax);
    d.seg_status = (uint32_t*)(base + L.seg_status);
    d.counters = (uint32_t*)(base + L.counters);
    d.flag = (uint32_t*)(base + L.flag);
    d.bad = (uint32_t*)(base + L.bad);
    d.cellmax = (uint32_t*)(base + L.cellmax);
    d.crowd = (uint32_t*)(base + L.crowd);
    d.zero_begin = (uint32_t*)(base + L.zero_begin);
    d.zero_words = (L.zero_end - L.zero_begin) / sizeof(uint32_t);
    p->sa.rb = L.rb;
    p->sa.cb = L.cb;
    p->sa.ntiles = L.ntiles;
    p->sa.nseg_tiles = L.nseg_tiles;
    p->sorted_keys = d.kB;
    p->perm = d.vB;
    p->X = nullptr;
    p->updated = 0;
    p->xn_valid = 0;
}

}  // namespace ibk

extern "C" {

int32_t ib_plan_create(const ib_grid_desc* grid, int32_t dtype, int64_t npts, void* workspace,
                       size_t workspace_bytes, ib_plan* out)
{
    return ib_plan_create_tuned(grid, dtype, npts, nullptr, workspace, workspace_bytes, out);
}

size_t ib_plan_workspace_bytes_tuned(const ib_grid_desc* grid, int32_t dtype, int64_t npts,
                                     const ib_tuning* tuning)
{
    int nstag, cs[3];
    double sx[3][3];
    if (check_grid(grid, dtype, npts, &nstag, cs, sx) != IB_OK) return 0;
    if (check_tuning(tuning, dtype) != IB_OK) return 0;
    Layout L;
    make_layout(grid, dtype, nstag, npts, &L, tuning);
    return L.total;
}

int32_t ib_plan_create_tuned(const ib_grid_desc* grid, int32_t dtype, int64_t npts,
                             const ib_tuning* tuning, void* workspace, size_t workspace_bytes,
                             ib_plan* out)
{
    if (!out) return IB_ERR_ARG;
    *out = nullptr;
    int nstag, cs[3];
    double sx[3][3] = {{0}};
    int32_t st = check_grid(grid, dtype, npts, &nstag, cs, sx);
    if (st != IB_OK) return st;
    st = check_tuning(tuning, dtype);
    if (st != IB_OK) return st;
    Layout L;
    make_layout(grid, dtype, nstag, npts, &L, tuning);
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) return IB_ERR_ARG;
    if (workspace_bytes < L.total) return IB_ERR_OOM;

    ib_plan p = new (std::nothrow) ib_plan_s();
    if (!p) return IB_ERR_OOM;
    plan_setup(p, grid, dtype, npts, nstag, cs, sx, L, workspace);
    *out = p;
    return IB_OK;
}

int32_t ib_plan_num_staggers(ib_plan p) { return p ? p->sa.g.nstag : IB_ERR_ARG; }

int32_t ib_plan_stagger_of(ib_plan p, int32_t comp)
{
    if (!p || comp < 0 || comp >= p->grid.ncomp) return IB_ERR_ARG;
    return p->sa.g.comp_stag[comp];
}

// The per-update region (bucket histograms, cursors, look-back words, tickets, flags) is
// cleared by a kernel before a plan's first update; afterwards each sort's bucket pass clears
// what the next sort of its staggering counts into, its scatter pass absorbs the bad-point
// mark, and each export clears the runs' words before its runs pass.  Without points there
// is no scatter pass, so such plans clear at every update.
static hipError_t clear_once(ib_plan p, hipStream_t st)
{
    if (p->cleared && p->npts > 0) return hipSuccess;
    const hipError_t e = launch_plan_reset(p->sa, st);
    if (e == hipSuccess) p->cleared = 1;
    return e;
}

int32_t ib_plan_update(ib_plan p, const void* X, void* stream)
{
    if (!p) return IB_ERR_ARG;
    if (!X && p->npts > 0) return IB_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = clear_once(p, st);
    // The operators use the keys and sort of staggering 0, its cell-start table and the
    // positions in that order; other staggerings are sorted when exported.
    if (e == hipSuccess) e = launch_sort_stagger(p->sa, 0, p->dtype, X, nullptr, true, st);
    int32_t r = hip_status(e);
    if (r != IB_OK) return r;
    p->X = X;
    p->updated = 1;
    p->xn_valid = 0;
    return IB_OK;
}

int32_t ib_plan_update_advected(ib_plan p, void* stream)
{
    if (!p || !p->updated || !p->xn_valid) return IB_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    // The advanced positions, in the previous sorted order, with that order's point indices.
    hipError_t e = clear_once(p, st);
    if (e == hipSuccess)
        e = launch_sort_stagger(p->sa, 0, p->dtype, p->sa.d.Xn, p->perm, true, st);
    int32_t r = hip_status(e);
    if (r != IB_OK) return r;
    p->xn_valid = 0;
    return IB_OK;
}

int32_t ib_plan_export(ib_plan p, int32_t sid, int32_t* keys, int32_t* sorted_keys, int32_t* perm,
                       int32_t* seg_off, int32_t* q, void* stream)
{
    if (!p || sid < 0 || sid >= p->sa.g.nstag || !p->updated) return IB_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    // Every export recomputes what it needs on the stream, with no host-side record of
    // what is current: a plan whose updates are replayed from a captured graph exports the
    // replayed update's arrays.
    if (sid != 0) {
        // from the update's positions in staggering-0 sorted order (valid even after X was
        // advanced in place)
        int32_t r = hip_status(launch_sort_stagger(p->sa, sid, p->dtype, p->sa.d.Xs, p->perm, false, st));
        if (r != IB_OK) return r;
    }
    const size_t n = (size_t)p->npts;
    const PlanDev& d = p->sa.d;
    hipError_t e = hipSuccess;
    if (seg_off || q) {
        // run heads, q and offsets from the sorted keys
        e = launch_runs(p->sa, sid, st);
        if (e != hipSuccess) return IB_ERR_HIP;
    }
    if (keys && n) e = launch_keys_out(p->sa, sid, keys, st);
    if (e == hipSuccess && sorted_keys && n)
        e = hipMemcpyAsync(sorted_keys, p->sorted_keys + sid * n, n * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && perm && n)
        e = hipMemcpyAsync(perm, p->perm + sid * n, n * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && seg_off)
        e = hipMemcpyAsync(seg_off, d.seg_off + sid * (n + 1), (n + 1) * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && q) e = hipMemcpyAsync(q, d.q + sid, 4, hipMemcpyDeviceToDevice, st);
    return hip_status(e);
}

int32_t ib_plan_status(ib_plan p)
{
    if (!p) return IB_ERR_ARG;
    // the plan's work may run on any stream, or replay from a captured graph
    if (hipDeviceSynchronize() != hipSuccess) return IB_ERR_HIP;
    if (!p->updated) return IB_OK;
    uint32_t flag = 0;
    if (hipMemcpy(&flag, p->sa.d.flag, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess)
        return IB_ERR_HIP;
    if (flag) {
        const uint32_t zero = 0;
        if (hipMemcpy(p->sa.d.flag, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
            return IB_ERR_HIP;
        return IB_ERR_DEVICE_FLAG;
    }
    return IB_OK;
}

void ib_plan_destroy(ib_plan p) { delete p; }

static void fill_op_args(ib_plan p, OpArgs* a)
{
    std::memset(a, 0, sizeof *a);
    a->g = p->sa.g;
    a->sorted_keys = p->sorted_keys;  // staggering 0
    a->perm = p->perm;
    a->cstart = p->sa.d.cstart;
    a->X = p->X;
    a->Xs = p->sa.d.Xs;
    a->Us = p->sa.d.Us;

    a->partial = p->sa.d.partial;
    a->tile_shift = p->sa.d.tile_shift;
    a->fmax = p->sa.d.fmax;
    a->cellmax = p->sa.d.cellmax;
    a->crowd = p->sa.d.crowd;
    a->out_scale = 1.0;
}

// Walled plans: kernels that can address the caller's unpadded field do so (direct).
static void set_direct(ib_plan p, OpArgs* a)
{
    if (!p->user.walls) return;
    a->direct = 1;
    for (int k = 0; k < 3; ++k) a->user_n[k] = k < p->user.dim ? p->user.n[k] : 1;
}

// The caller's grid field u: walled plans' kernels read it as the padded grid's first
// cells, with zero ghost values (set_direct).
static const void* kernel_field(ib_plan p, OpArgs* a, const void* u)
{
    set_direct(p, a);
    return u;
}

int32_t ib_spread_scaled(ib_plan p, const void* F, void* f, double scale, int32_t accumulate,
                         void* stream)
{
    if (!p || !f || !p->updated || !std::isfinite(scale)) return IB_ERR_ARG;
    if (!F && p->npts > 0) return IB_ERR_ARG;
    OpArgs a;
    fill_op_args(p, &a);
    a.g.scale *= scale;  // one factor applied to the exact sums: (prod_k h_k)^-1 * scale
    a.F = F;
    a.f = f;
    a.accumulate = accumulate != 0;
    set_direct(p, &a);  // walled: the padded grid's tiles write the caller's cells, ghosts dropped
    hipStream_t st = (hipStream_t)stream;
    return hip_status(launch_spread(a, p->dtype, p->grid.kernel, st));
}

int32_t ib_spread(ib_plan p, const void* F, void* f, int32_t accumulate, void* stream)
{
    return ib_spread_scaled(p, F, f, 1.0, accumulate, stream);
}

int32_t ib_interpolate_scaled(ib_plan p, const void* u, void* U, double scale, void* stream)
{
    if (!p || !u || !p->updated || !std::isfinite(scale)) return IB_ERR_ARG;
    if (!U && p->npts > 0) return IB_ERR_ARG;
    if (p->npts == 0) return IB_OK;
    OpArgs a;
    fill_op_args(p, &a);
    a.out_scale = scale;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    a.u = kernel_field(p, &a, u);
    a.U = U;
    if (e == hipSuccess) e = launch_interp(a, p->dtype, p->grid.kernel, st);
    return hip_status(e);
}

int32_t ib_interpolate(ib_plan p, const void* u, void* U, void* stream)
{
    return ib_interpolate_scaled(p, u, U, 1.0, stream);
}

int32_t ib_interpolate_advect(ib_plan p, const void* u, void* U, void* X, double dt, void* stream)
{
    if (!p || !u || !p->updated) return IB_ERR_ARG;
    if ((!U || !X) && p->npts > 0) return IB_ERR_ARG;
    if (p->grid.ncomp != p->grid.dim || !std::isfinite(dt)) return IB_ERR_ARG;
    if (p->npts == 0) return IB_OK;
    OpArgs a;
    fill_op_args(p, &a);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    a.u = kernel_field(p, &a, u);
    a.U = U;
    p->xn_valid = 0;
    if (!p->user.walls) {  // walled: interpolation, then the update without wrap along walls
        a.Xadv = X;
        a.Xnext = p->sa.d.Xn;  // the advanced positions also in sorted order
        a.adv_dt = dt;
        for (int k = 0; k < 3; ++k) a.adv_len[k] = k < p->grid.dim ? p->grid.length[k] : 1.0;
    }
    if (e == hipSuccess) e = launch_interp(a, p->dtype, p->grid.kernel, st);
    if (e == hipSuccess && p->user.walls)
        e = launch_advect(p->user.dim, p->user.ncomp, p->npts, p->user.length, p->user.walls,
                          p->dtype, X, U, dt, st);
    if (e == hipSuccess && !p->user.walls) p->xn_valid = 1;
    return hip_status(e);
}

int32_t ib_interpolate_grad_scaled(ib_plan p, const void* u, const void* W, void* dX, double scale,
                                   int32_t accumulate, void* stream)
{
    if (!p || !u || !p->updated || !std::isfinite(scale)) return IB_ERR_ARG;
    if ((!W || !dX) && p->npts > 0) return IB_ERR_ARG;
    if (p->npts == 0) return IB_OK;
    OpArgs a;
    fill_op_args(p, &a);
    a.out_scale = scale;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    a.u = kernel_field(p, &a, u);
    if (e == hipSuccess)
        e = launch_interp_grad(a, p->dtype, p->grid.kernel, W, dX, accumulate != 0, st);
    return hip_status(e);
}

int32_t ib_interpolate_grad(ib_plan p, const void* u, const void* W, void* dX, int32_t accumulate,
                            void* stream)
{
    return ib_interpolate_grad_scaled(p, u, W, dX, 1.0, accumulate, stream);
}

int32_t ib_advect(const ib_grid_desc* grid, int32_t dtype, int64_t npts, void* X, const void* U,
                  double dt, void* stream)
{
    int nstag, cs[3];
    double sx[3][3];
    int32_t st = check_grid(grid, dtype, npts, &nstag, cs, sx);
    if (st != IB_OK) return st;
    if (grid->ncomp != grid->dim || !std::isfinite(dt)) return IB_ERR_ARG;
    if (npts > 0 && (!X || !U)) return IB_ERR_ARG;
    return hip_status(launch_advect(grid->dim, grid->ncomp, npts, grid->length, grid->walls, dtype,
                                    X, U, dt, (hipStream_t)stream));
}

int32_t ib_tether_force(const ib_grid_desc* grid, int32_t dtype, int64_t npts, const void* X0,
                        const void* X, double k, void* F, void* stream)
{
    int nstag, cs[3];
    double sx[3][3];
    int32_t st = check_grid(grid, dtype, npts, &nstag, cs, sx);
    if (st != IB_OK) return st;
    if (grid->ncomp != grid->dim || !std::isfinite(k)) return IB_ERR_ARG;
    if (npts > 0 && (!X0 || !X || !F)) return IB_ERR_ARG;
    return hip_status(launch_tether(grid->dim, grid->walls, npts, grid->length, dtype, X0, X, k,
                                    F, (hipStream_t)stream));
}

}  // extern "C"

// axf_api.hip -- C ABI: plan lifecycle, evaluation entry points, errors and
// the device arena cache.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *get_error() { return g_err.c_str(); }

// ---------------------------------------------------------- arena cache
// The cache is off unless the caller opts in with axf_set_cache_limit: its
// blocks are invisible to other allocators (PyTorch's included), so by
// default a released arena goes straight back to the runtime.
namespace {
std::mutex g_cache_mu;
std::vector<Arena> g_cache;
size_t g_cached_bytes = 0;
size_t g_cache_limit = 0;

// Frees cached blocks, largest first, until at most `limit` bytes remain.
// Caller holds g_cache_mu.
void cache_trim(size_t limit)
{
    std::sort(g_cache.begin(), g_cache.end(), [](const Arena &a, const Arena &b) { return a.bytes < b.bytes; });
    while (g_cached_bytes > limit && !g_cache.empty()) {
        Arena a = g_cache.back();
        g_cache.pop_back();
        g_cached_bytes -= a.bytes;
        (void)hipFree(a.base);
    }
}
}  // namespace

Arena arena_acquire(size_t bytes)
{
    int dev = 0;
    AXF_HIP(hipGetDevice(&dev));
    bytes = std::max<size_t>(bytes, 256);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        int best = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i) {
            const Arena &a = g_cache[i];
            if (a.device != dev || a.bytes < bytes || a.bytes > 2 * bytes + (size_t(64) << 20)) continue;
            if (best < 0 || a.bytes < g_cache[best].bytes) best = i;
        }
        if (best >= 0) {
            Arena a = g_cache[best];
            g_cache.erase(g_cache.begin() + best);
            g_cached_bytes -= a.bytes;
            a.used = 0;
            return a;
        }
    }
    Arena a;
    a.device = dev;
    a.bytes = bytes;
    hipError_t e = hipMalloc((void **)&a.base, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // drop the cache and retry once
        std::vector<Arena> drop;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            drop.swap(g_cache);
            g_cached_bytes = 0;
        }
        for (Arena &x : drop) (void)hipFree(x.base);
        e = hipMalloc((void **)&a.base, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
            throw Fail{AXF_ERR_OUT_OF_MEMORY};
        }
    }
    return a;
}

void arena_release(Arena &a)
{
    if (!a.base) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_cached_bytes + a.bytes <= g_cache_limit) {
        g_cache.push_back(a);
        g_cached_bytes += a.bytes;
    } else {
        (void)hipFree(a.base);
    }
    a = Arena();
}

hipEvent_t event_get(Plan &pl)
{
    if (!pl.spare_events.empty()) {
        hipEvent_t e = pl.spare_events.back();
        pl.spare_events.pop_back();
        return e;
    }
    hipEvent_t e;
    AXF_HIP(hipEventCreate(&e));
    return e;
}

PhaseTimer::PhaseTimer(Plan &p, hipStream_t s, int ph) : pl(p), st(s), phase(ph)
{
    if (!pl.timing || phase < 0) return;
    a = event_get(pl);
    b = event_get(pl);
    AXF_HIP(hipEventRecord(a, st));
}

PhaseTimer::~PhaseTimer()
{
    if (!a) return;
    if (hipEventRecord(b, st) == hipSuccess) pl.marks.push_back({phase, a, b});
}

static void release_events(Plan *pl)
{
    for (auto &m : pl->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (auto e : pl->spare_events) (void)hipEventDestroy(e);
    pl->marks.clear();
    pl->spare_events.clear();
}

void plan_release(Plan *pl)
{
    if (!pl) return;
    (void)hipDeviceSynchronize();
    release_events(pl);
    if (pl->tables_ready) (void)hipEventDestroy(pl->tables_ready);
    pl->tables_ready = nullptr;
    for (hipEvent_t *e : {&pl->ev_fork, &pl->ev_join}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
    arena_release(pl->points);
    arena_release(pl->tree);
    arena_release(pl->expn);
    arena_release(pl->tilemem);
    arena_release(pl->tabmem);
}

static void validate_params(const axf_params *p)
{
    AXF_REQUIRE(p != nullptr, AXF_ERR_INVALID_ARGUMENT, "params is NULL");
    AXF_REQUIRE(p->n_modes >= 1 && p->n_modes <= AXF_MAX_MODES, AXF_ERR_UNSUPPORTED,
                "n_modes must be in 1..64");
    AXF_REQUIRE(p->order >= 0 && p->order <= AXF_MAX_ORDER, AXF_ERR_UNSUPPORTED, "order must be in 0..24");
    AXF_REQUIRE(p->depth == 0 || (p->depth >= 2 && p->depth <= AXF_MAX_DEPTH), AXF_ERR_UNSUPPORTED,
                "depth must be 0 (automatic) or in 2..11");
    AXF_REQUIRE(p->depth != 0 || p->max_leaf >= 1, AXF_ERR_INVALID_ARGUMENT,
                "max_leaf must be >= 1 when depth is 0");
    AXF_REQUIRE(p->nrhs >= 1 && p->nrhs <= AXF_MAX_RHS, AXF_ERR_UNSUPPORTED, "nrhs must be in 1..8");
    AXF_REQUIRE((p->flags & ~(AXF_TILE_MASK | AXF_NO_OVERLAP)) == 0, AXF_ERR_INVALID_ARGUMENT, "unknown plan flags");
    const int tb = (int)((p->flags & AXF_TILE_MASK) >> AXF_TILE_SHIFT);
    AXF_REQUIRE(tb == 0 || s2l_tile_ok(tb), AXF_ERR_UNSUPPORTED, "S2L tile width must be 2, 4 or 8 (or 0)");
}

// The stream that builds a plan's tables beside the tree (one per device,
// default priority, created on first use and kept for the process).
static hipStream_t table_stream(int device)
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    hipStream_t &s = streams[device & 63];
    if (!s) AXF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
}

// Build everything after the parameters are known valid.
void plan_build(Plan &pl, const axf_params &p, int64_t ns, const double *rs, const double *zs, int64_t nf,
                const double *rf, const double *zf, hipStream_t st)
{
    AXF_HIP(hipGetDevice(&pl.device));
    pl.p = p;
    pl.nmodes = p.n_modes;
    pl.N = p.n_modes - 1;
    pl.M = p.order;
    pl.P = (p.order + 1) * (p.order + 2) / 2;
    pl.nrhs = p.nrhs;
    pl.C = p.n_modes * p.nrhs;
    pl.TS = (p.order + 1) * (p.order + 1) * (p.order + 1);
    pl.chistar = forward_chi_limit(p.n_modes);
    pl.nmb = mode_bucket(p.n_modes);
    {
        const int tb = (int)((p.flags & AXF_TILE_MASK) >> AXF_TILE_SHIFT);
        // no tile flag: the matrix-core S2L on tiles of up to 16 boxes (two
        // column tiles); AXF_TILE(tb): the vector-unit S2L on tb boxes
        pl.mfma = tb == 0;
        pl.tb = tb ? tb : 2 * kS2lMfmaBoxes;
    }
    pl.overlap = !(p.flags & AXF_NO_OVERLAP);
    pl.Cs = pl.nmb * p.nrhs;
    pl.src.n = ns;
    pl.fld.n = nf;
    // The tables depend only on the square, the depth, the order and the
    // modes: they are built on a second stream while the tree is sorted and
    // the S2L tiles are made, and joined before the plan is returned.
    hipStream_t side = table_stream(pl.device);
    auto start_tables = [&]() {
        const int d = pl.d;
        // a level's tables cover the radial stations up to that of the
        // largest radius: an S2L operator uses the table of the inner of two
        // occupied stations, so stations beyond it are never read.  With the
        // square's origin koff L/4 from the axis (koff >= 0), station s of
        // level l sits at koff 2^(l-2) + s + 1/2 box units, the radius of
        // station koff 2^(l-2) + s of the finest level's axis grid, so its
        // tables are that station's times 2^(l-d) (eq. gfunc:scaled): the
        // levels' station ranges on that grid are merged into runs and only
        // the runs are stored.  Otherwise every level has its own tables.
        size_t ngeom = 0;
        pl.tab_runs.clear();
        if (pl.koff >= 0) {
            std::vector<std::pair<int, int>> iv;
            for (int l = 2; l <= d; ++l) {
                const int v0 = pl.koff << (l - 2);
                iv.push_back({v0, v0 + box_index(pl.rmax, pl.rlo, pl.invL, l)});
            }
            std::sort(iv.begin(), iv.end());
            for (auto &x : iv) {
                if (!pl.tab_runs.empty() && x.first <= pl.tab_runs.back().second + 1)
                    pl.tab_runs.back().second = std::max(pl.tab_runs.back().second, x.second);
                else
                    pl.tab_runs.push_back(x);
            }
            for (int l = 2; l <= d; ++l) {
                const int v0 = pl.koff << (l - 2);
                size_t before = 0;
                for (auto &run : pl.tab_runs) {
                    if (v0 >= run.first && v0 <= run.second) {
                        pl.tab_base[l] = (size_t)12 * (before + (size_t)(v0 - run.first));
                        pl.tab_smax[l] = std::min((1 << l) - 1, run.second - v0);
                        break;
                    }
                    before += (size_t)(run.second - run.first + 1);
                }
            }
            for (auto &run : pl.tab_runs) ngeom += (size_t)12 * (run.second - run.first + 1);
        } else {
            for (int l = 2; l <= d; ++l) {
                pl.tab_smax[l] = box_index(pl.rmax, pl.rlo, pl.invL, l);
                pl.tab_base[l] = ngeom;
                ngeom += (size_t)12 * (pl.tab_smax[l] + 1);
            }
        }
        const bool shared = pl.koff >= 0;
        Sizer tz;
        tz.add<double>(ngeom * (size_t)pl.nmodes * pl.TS + kTablePad);
        tz.add<double>(table_scratch_doubles(ngeom, pl.M, pl.nmodes));
        pl.tabmem = arena_acquire(tz.bytes + 4096);
        double *tab = pl.tabmem.take<double>(ngeom * (size_t)pl.nmodes * pl.TS + kTablePad);
        for (int l = 2; l <= d; ++l) {
            pl.lev[l].tab = tab + pl.tab_base[l] * pl.nmodes * pl.TS;
            pl.lev[l].tscale = shared ? std::ldexp(1.0, l - d) : 1.0;
        }
        pl.tab_scratch = pl.tabmem.take<double>(table_scratch_doubles(ngeom, pl.M, pl.nmodes));
        // after everything the caller's stream already holds
        hipEvent_t ev = event_get(pl);
        AXF_HIP(hipEventRecord(ev, st));
        AXF_HIP(hipStreamWaitEvent(side, ev, 0));
        pl.spare_events.push_back(ev);   // reusable: the wait has been enqueued
        build_tables(pl, side);
        if (!pl.tables_ready) AXF_HIP(hipEventCreateWithFlags(&pl.tables_ready, hipEventDisableTiming));
        AXF_HIP(hipEventRecord(pl.tables_ready, side));
    };
    AXF_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
    AXF_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
    build_tree(pl, rs, zs, rf, zf, st, start_tables);
    build_tiles(pl, st);

    // expansion arena: moments, locals and the S2L partial sums
    const int d = pl.d;
    Sizer sz;
    for (int l = 2; l <= d; ++l) {
        size_t nb = (size_t)std::max(pl.src.nocc[l], pl.fld.nocc[l]);
        sz.add<double2>(std::max<size_t>(nb, 1) * pl.C * pl.P);
        sz.add<double2>(std::max<size_t>(nb, 1) * pl.C * pl.P);
    }
    // offset groups of the S2L pass and their partial-sum buffer (one level
    // at a time, either side as targets)
    size_t part = 0;
    int mfma_tpw = 0, mfma_waves = 0;
    s2l_mfma_shape(pl.M, mfma_tpw, mfma_waves);
    for (Side *sd : {&pl.src, &pl.fld})
        for (int l = 2; l <= d; ++l) {
            sd->s2l_groups[l] =
                s2l_group_count(sd->ntiles[l], pl.C, pl.M, pl.mfma ? mfma_waves : s2l_waves(pl.M));
            if (sd->s2l_groups[l] > 1)
                part = std::max(part, (size_t)sd->s2l_groups[l] * sd->nocc[l] * pl.C * pl.P);
        }
    sz.add<double2>(std::max<size_t>(part, 1));
    sz.add<double>((size_t)6 * kCoefS * kCoefS);
    pl.expn = arena_acquire(sz.bytes + 4096);
    for (int l = 2; l <= d; ++l) {
        size_t nb = (size_t)std::max(pl.src.nocc[l], pl.fld.nocc[l]);
        pl.lev[l].nb = 1 << l;
        pl.lev[l].h = pl.L / (1 << l);
        pl.lev[l].mom = pl.expn.take<double2>(std::max<size_t>(nb, 1) * pl.C * pl.P);
        pl.lev[l].loc = pl.expn.take<double2>(std::max<size_t>(nb, 1) * pl.C * pl.P);
    }
    pl.s2l_part = pl.expn.take<double2>(std::max<size_t>(part, 1));
    // M2M and L2L shift factors (the host copy lives with the plan)
    pl.shift_coef = pl.expn.take<double>((size_t)6 * kCoefS * kCoefS);
    shift_coef_host(pl.M, pl.coef_host);
    AXF_HIP(hipMemcpyAsync(pl.shift_coef, pl.coef_host.data(), sizeof(double) * pl.coef_host.size(),
                           hipMemcpyHostToDevice, st));
    // One wait for the tile and factor uploads (their host images can then
    // go). The tables may still be running on the table stream: the
    // evaluation passes wait for `tables_ready` on their own stream just
    // before the first S2L, so the gather, P2M and M2M overlap them.
    AXF_HIP(hipStreamSynchronize(st));
    std::vector<char>().swap(pl.tile_host);
    std::vector<int32_t>().swap(pl.box_host);
    pl.device_bytes = pl.points.bytes + pl.tree.bytes + pl.expn.bytes + pl.tilemem.bytes + pl.tabmem.bytes;
}

// Moves every buffer of a plan into caller memory [ws, ws + bytes): the five
// arenas are copied back to back (each at a 256-byte boundary), every
// device pointer of the plan is rebased, and the arenas are released.
// Synchronises the device first (the tables may still be in flight).
size_t plan_workspace_bytes(const Plan &pl)
{
    const Arena *ar[5] = {&pl.points, &pl.tree, &pl.tilemem, &pl.expn, &pl.tabmem};
    size_t need = 0;
    for (const Arena *a : ar) need = ((need + 255) & ~size_t(255)) + a->used;
    return need;
}

static void plan_relocate(Plan &pl, char *ws, size_t bytes)
{
    Arena *ar[5] = {&pl.points, &pl.tree, &pl.tilemem, &pl.expn, &pl.tabmem};
    size_t off[5], need = 0;
    for (int i = 0; i < 5; ++i) {
        need = (need + 255) & ~size_t(255);
        off[i] = need;
        need += ar[i]->used;
    }
    AXF_REQUIRE(bytes >= need, AXF_ERR_WORKSPACE,
                "workspace of " + std::to_string(bytes) + " bytes is smaller than the " + std::to_string(need) +
                    " bytes the plan needs");
    // every listed pointer must lie in an arena (or be null) ...
    // (an end pointer, p == base + used, belongs to its arena only if no
    // arena holds p strictly inside: two allocations may be adjacent)
    auto owner = [&](const char *p) {
        for (int i = 0; i < 5; ++i)
            if (ar[i]->base && p >= ar[i]->base && p < ar[i]->base + ar[i]->used) return i;
        for (int i = 0; i < 5; ++i)
            if (ar[i]->base && p == ar[i]->base + ar[i]->used) return i;
        return -1;
    };
    std::vector<const void *> fields;
    bool stray = false;
    plan_device_ptrs(pl, [&](char *&p, const void *field) {
        fields.push_back(field);
        if (p) stray |= owner(p) < 0;
    });
    AXF_REQUIRE(!stray, AXF_ERR_HIP, "internal: a plan pointer lies outside the plan's arenas");
    // ... and no unlisted word of the plan may hold an arena address
    for (Arena *a : ar) fields.push_back(&a->base);
    std::sort(fields.begin(), fields.end());
    const uintptr_t *w = reinterpret_cast<const uintptr_t *>(&pl);
    for (size_t k = 0; k < sizeof(Plan) / sizeof(uintptr_t); ++k) {
        const char *v = reinterpret_cast<const char *>(w[k]);
        bool in_arena = false;
        for (Arena *a : ar)
            in_arena |= a->base && v >= a->base && v < a->base + a->bytes;
        AXF_REQUIRE(!in_arena || std::binary_search(fields.begin(), fields.end(), (const void *)&w[k]), AXF_ERR_HIP,
                    "internal: the plan holds an arena address that relocation does not know");
    }
    AXF_HIP(hipSetDevice(pl.device));
    AXF_HIP(hipDeviceSynchronize());
    for (int i = 0; i < 5; ++i)
        if (ar[i]->used) AXF_HIP(hipMemcpy(ws + off[i], ar[i]->base, ar[i]->used, hipMemcpyDeviceToDevice));
    plan_device_ptrs(pl, [&](char *&p, const void *) {
        if (!p) return;
        const int i = owner(p);
        p = ws + off[i] + (p - ar[i]->base);
    });
    for (Arena *a : ar) arena_release(*a);
    pl.external = true;
    pl.device_bytes = need;
}

}  // namespace axf

using namespace axf;


#define AXF_TRY(...)                                        \
    try {                                                   \
        __VA_ARGS__;                                        \
        return AXF_OK;                                      \
    } catch (const Fail &f) {                               \
        return f.st;                                        \
    } catch (const std::bad_alloc &) {                      \
        set_error("host allocation failed");                \
        return AXF_ERR_OUT_OF_MEMORY;                       \
    } catch (...) {                                         \
        set_error("unexpected internal error");             \
        return AXF_ERR_HIP;                                 \
    }

extern "C" {

axf_status axf_plan_create(const axf_params *params, int64_t ns, const double *r_src, const double *z_src,
                           int64_t nf, const double *r_fld, const double *z_fld, void *stream,
                           axf_plan **out_plan, size_t *workspace_bytes)
{
    axf_plan *h = nullptr;
    try {
        AXF_REQUIRE(out_plan != nullptr, AXF_ERR_INVALID_ARGUMENT, "out_plan is NULL");
        *out_plan = nullptr;
        if (workspace_bytes) *workspace_bytes = 0;
        validate_params(params);
        AXF_REQUIRE(ns >= 1 && nf >= 1, AXF_ERR_INVALID_ARGUMENT, "ns and nf must be >= 1");
        AXF_REQUIRE(ns < (int64_t(1) << 31) && nf < (int64_t(1) << 31), AXF_ERR_UNSUPPORTED,
                    "ns and nf must be < 2^31");
        AXF_REQUIRE(r_src && z_src && r_fld && z_fld, AXF_ERR_INVALID_ARGUMENT, "a coordinate pointer is NULL");
        h = new axf_plan();
        plan_build(h->pl, *params, ns, r_src, z_src, nf, r_fld, z_fld, (hipStream_t)stream);
        if (workspace_bytes) *workspace_bytes = plan_workspace_bytes(h->pl);
        *out_plan = h;
        return AXF_OK;
    } catch (const Fail &f) {
        if (h) {
            plan_release(&h->pl);
            delete h;
        }
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return AXF_ERR_OUT_OF_MEMORY;
    }
}

axf_status axf_plan_set_workspace(axf_plan *plan, void *workspace, size_t bytes)
{
    AXF_TRY({
        AXF_REQUIRE(plan && workspace, AXF_ERR_INVALID_ARGUMENT, "plan and workspace must be non-NULL");
        AXF_REQUIRE(!plan->pl.external, AXF_ERR_INVALID_ARGUMENT, "the plan already lives in a workspace");
        AXF_REQUIRE(((uintptr_t)workspace & 255) == 0, AXF_ERR_WORKSPACE,
                    "workspace must be aligned to 256 bytes");
        plan_relocate(plan->pl, (char *)workspace, bytes);
    })
}

axf_status axf_set_cache_limit(size_t bytes)
{
    AXF_TRY({
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache_limit = bytes;
        cache_trim(bytes);
    })
}

void axf_plan_destroy(axf_plan *plan)
{
    if (!plan) return;
    plan_release(&plan->pl);
    delete plan;
}

axf_status axf_evaluate(axf_plan *plan, const double *S, double *phi, void *stream)
{
    AXF_TRY({
        AXF_REQUIRE(plan && S && phi, AXF_ERR_INVALID_ARGUMENT, "plan, S and phi must be non-NULL");
        EvalOut o;
        o.phi = phi;
        run_fmm(plan->pl, plan->pl.src, plan->pl.fld, S, o, (hipStream_t)stream);
    })
}

axf_status axf_evaluate_grad(axf_plan *plan, const double *S, double *phi, double *dphi_dr, double *dphi_dz,
                             double *dphi_az, void *stream)
{
    AXF_TRY({
        AXF_REQUIRE(plan && S && phi, AXF_ERR_INVALID_ARGUMENT, "plan, S and phi must be non-NULL");
        EvalOut o;
        o.phi = phi;
        o.dr = dphi_dr;
        o.dz = dphi_dz;
        o.daz = dphi_az;
        o.mode = 1;
        run_fmm(plan->pl, plan->pl.src, plan->pl.fld, S, o, (hipStream_t)stream);
    })
}

axf_status axf_evaluate_direct(axf_plan *plan, const double *S, double *phi, void *stream)
{
    AXF_TRY({
        AXF_REQUIRE(plan && S && phi, AXF_ERR_INVALID_ARGUMENT, "plan, S and phi must be non-NULL");
        EvalOut o;
        o.phi = phi;
        run_direct(plan->pl, plan->pl.src, plan->pl.fld, S, o, (hipStream_t)stream);
    })
}

axf_status axf_adjoint(axf_plan *plan, const double *S, const double *gphi, double *gS, double *g_rsrc,
                       double *g_zsrc, void *stream)
{
    AXF_TRY({
        AXF_REQUIRE(plan && gphi && gS, AXF_ERR_INVALID_ARGUMENT, "plan, gphi and gS must be non-NULL");
        AXF_REQUIRE(!(g_rsrc || g_zsrc) || S, AXF_ERR_INVALID_ARGUMENT,
                    "S is required for coordinate gradients");
        EvalOut o;
        o.phi = gS;
        if (g_rsrc || g_zsrc) {
            o.mode = 2;
            o.Sdot = S;
            o.gr = g_rsrc;
            o.gz = g_zsrc;
        }
        run_fmm(plan->pl, plan->pl.fld, plan->pl.src, gphi, o, (hipStream_t)stream);
    })
}

axf_status axf_plan_info(const axf_plan *plan, int32_t *depth, int32_t *n_modes, int32_t *order, int32_t *nrhs,
                         int64_t *ns, int64_t *nf, double *square4, int64_t *n_near_pairs, int64_t *n_s2l_pairs,
                         size_t *device_bytes)
{
    AXF_TRY({
        AXF_REQUIRE(plan, AXF_ERR_INVALID_ARGUMENT, "plan is NULL");
        const Plan &pl = plan->pl;
        if (depth) *depth = pl.d;
        if (n_modes) *n_modes = pl.nmodes;
        if (order) *order = pl.M;
        if (nrhs) *nrhs = pl.nrhs;
        if (ns) *ns = pl.src.n;
        if (nf) *nf = pl.fld.n;
        if (square4) {
            square4[0] = pl.rlo;
            square4[1] = pl.zlo;
            square4[2] = pl.L;
            square4[3] = pl.invL;
        }
        if (n_near_pairs) *n_near_pairs = pl.near_pairs;
        if (n_s2l_pairs) *n_s2l_pairs = pl.s2l_pairs;
        if (device_bytes) *device_bytes = pl.device_bytes;
    })
}

axf_status axf_plan_level_info(const axf_plan *plan, int32_t level, int32_t *n_src_boxes, int32_t *n_fld_boxes)
{
    AXF_TRY({
        AXF_REQUIRE(plan, AXF_ERR_INVALID_ARGUMENT, "plan is NULL");
        AXF_REQUIRE(level >= 2 && level <= plan->pl.d, AXF_ERR_INVALID_ARGUMENT, "level out of range");
        if (n_src_boxes) *n_src_boxes = plan->pl.src.nocc[level];
        if (n_fld_boxes) *n_fld_boxes = plan->pl.fld.nocc[level];
    })
}

axf_status axf_plan_table(const axf_plan *plan, int32_t level, int32_t station, int32_t dr, int32_t dz,
                          double *host_out)
{
    AXF_TRY({
        AXF_REQUIRE(plan && host_out, AXF_ERR_INVALID_ARGUMENT, "plan and host_out must be non-NULL");
        const Plan &pl = plan->pl;
        AXF_REQUIRE(level >= 2 && level <= pl.d, AXF_ERR_INVALID_ARGUMENT, "level out of range");
        AXF_REQUIRE(station >= 0 && station < (1 << level), AXF_ERR_INVALID_ARGUMENT, "station out of range");
        AXF_REQUIRE(station <= pl.tab_smax[level], AXF_ERR_INVALID_ARGUMENT,
                    "no table at this station: it lies beyond the largest radius");
        AXF_REQUIRE(dr >= 0 && dr <= 3 && dz >= 0 && dz <= 3 && (dr >= 2 || dz >= 2), AXF_ERR_INVALID_ARGUMENT,
                    "separation must satisfy 0 <= dr, dz <= 3, not both <= 1");
        const int M = pl.M, K = 2 * M, nm = pl.nmodes;
        const size_t TS = (size_t)pl.TS;
        std::vector<double> buf(TS * nm);
        const double *src = pl.lev[level].tab + ((size_t)station * 12 + geom_slot(dr, dz)) * nm * TS;
        AXF_HIP(hipSetDevice(pl.device));
        AXF_HIP(hipDeviceSynchronize());
        AXF_HIP(hipMemcpy(buf.data(), src, sizeof(double) * TS * nm, hipMemcpyDeviceToHost));
        for (int n = 0; n < nm; ++n)
            for (int a = 0; a <= M; ++a)
                for (int b = 0; b <= M; ++b)
                    for (int c = 0; c <= K; ++c) {
                        double v = (a + b + c <= K) ? buf[(size_t)n * TS + table_row(M, a, b) + c] : 0.0;
                        v *= pl.lev[level].tscale;
                        host_out[(((size_t)n * (M + 1) + a) * (M + 1) + b) * (K + 1) + c] = v;
                    }
    })
}

axf_status axf_plan_set_timing(axf_plan *plan, int32_t enable)
{
    AXF_TRY({
        AXF_REQUIRE(plan, AXF_ERR_INVALID_ARGUMENT, "plan is NULL");
        plan->pl.timing = enable != 0;
    })
}

axf_status axf_plan_read_timing(axf_plan *plan, double *ms, int32_t *launches)
{
    AXF_TRY({
        AXF_REQUIRE(plan && ms, AXF_ERR_INVALID_ARGUMENT, "plan and ms must be non-NULL");
        Plan &pl = plan->pl;
        for (int i = 0; i < AXF_NUM_PHASES; ++i) {
            ms[i] = 0.0;
            if (launches) launches[i] = 0;
        }
        for (auto &m : pl.marks) {
            AXF_HIP(hipEventSynchronize(m.b));
            float t = 0.f;
            AXF_HIP(hipEventElapsedTime(&t, m.a, m.b));
            ms[m.phase] += t;
            if (launches) launches[m.phase] += 1;
            pl.spare_events.push_back(m.a);
            pl.spare_events.push_back(m.b);
        }
        pl.marks.clear();
    })
}

axf_status axf_plan_work(const axf_plan *plan, int64_t *near_pairs, int64_t *s2l_pairs, int64_t *s2l_units,
                         double *flops)
{
    AXF_TRY({
        AXF_REQUIRE(plan, AXF_ERR_INVALID_ARGUMENT, "plan is NULL");
        Plan &pl = const_cast<axf_plan *>(plan)->pl;
        if (near_pairs) *near_pairs = pl.near_pairs;
        if (s2l_pairs) *s2l_pairs = pl.s2l_pairs;
        if (s2l_units) *s2l_units = pl.s2l_units;
        if (flops) {
            if (!pl.census_done) {
                AXF_HIP(hipSetDevice(pl.device));
                pair_census(pl, false, pl.census_near, nullptr);
                pair_census(pl, true, pl.census_direct, nullptr);
                pl.census_done = true;
            }
            // FP64 operation model (fma = 2).  A pair costs 24 flops of
            // geometry, start values and chi, 9 per AGM iteration, 3 per
            // recursion step, N + 6 more on the backward branch (asymptotic
            // start and normalisation) and 4 per mode and right-hand side of
            // complex accumulation; iteration and step counts come from the
            // pair census (what each pair needs, not what a wave executes).
            const double P = pl.P, C = pl.C, Nm = pl.nmodes, R = pl.nrhs, N = pl.N;
            const double M = pl.M;
            const double c3 = (M + 1) * (M + 2) * (M + 3) / 6.0;   // C(M+3, 3): one separable pass
            auto pair_flops = [&](const double *cs) {
                return cs[0] * (24.0 + 4.0 * Nm * R) + 9.0 * cs[2] + 3.0 * cs[3] + cs[1] * (N + 6.0);
            };
            double nbox_up = 0, nbox_down = 0;   // M2M parents, L2L children
            for (int l = 2; l < pl.d; ++l) nbox_up += pl.src.nocc[l];
            for (int l = 3; l <= pl.d; ++l) nbox_down += pl.fld.nocc[l];
            flops[AXF_PHASE_GATHER] = 0.0;
            flops[AXF_PHASE_P2M] = (double)pl.src.n * (4.0 * P * C + 2.0 * P);
            // separable shifts: M2M 4 children in z + 2 parities in r, L2L r then z
            flops[AXF_PHASE_M2M] = nbox_up * C * c3 * 24.0;
            // one contraction per (target box, offset unit): the offsets
            // (dr, dz) and (dr, -dz) share it
            flops[AXF_PHASE_S2L] = (double)pl.s2l_units * C * P * P * 4.0;
            flops[AXF_PHASE_L2L] = nbox_down * C * c3 * 8.0;
            flops[AXF_PHASE_LEAF] = pair_flops(pl.census_near);
            flops[AXF_PHASE_L2P] = (double)pl.fld.n * (4.0 * P * C + 2.0 * P);
            flops[AXF_PHASE_DIRECT] = pair_flops(pl.census_direct);
        }
    })
}

axf_status axf_plan_census(const axf_plan *plan, double *near_counts, double *direct_counts)
{
    AXF_TRY({
        AXF_REQUIRE(plan, AXF_ERR_INVALID_ARGUMENT, "plan is NULL");
        Plan &pl = const_cast<axf_plan *>(plan)->pl;
        if (!pl.census_done) {
            AXF_HIP(hipSetDevice(pl.device));
            pair_census(pl, false, pl.census_near, nullptr);
            pair_census(pl, true, pl.census_direct, nullptr);
            pl.census_done = true;
        }
        for (int q = 0; q < 4; ++q) {
            if (near_counts) near_counts[q] = pl.census_near[q];
            if (direct_counts) direct_counts[q] = pl.census_direct[q];
        }
    })
}

const char *axf_status_string(axf_status s)
{
    switch (s) {
    case AXF_OK: return "AXF_OK";
    case AXF_ERR_INVALID_ARGUMENT: return "AXF_ERR_INVALID_ARGUMENT";
    case AXF_ERR_INVALID_GEOMETRY: return "AXF_ERR_INVALID_GEOMETRY";
    case AXF_ERR_OUT_OF_MEMORY: return "AXF_ERR_OUT_OF_MEMORY";
    case AXF_ERR_UNSUPPORTED: return "AXF_ERR_UNSUPPORTED";
    case AXF_ERR_HIP: return "AXF_ERR_HIP";
    case AXF_ERR_WORKSPACE: return "AXF_ERR_WORKSPACE";
    }
    return "AXF_ERR_UNKNOWN";
}

const char *axf_last_error(void) { return get_error(); }

}  // extern "C"

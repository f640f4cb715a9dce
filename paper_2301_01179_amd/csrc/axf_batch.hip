// axf_batch.hip -- batched evaluation of many independent problems.
//
// Each problem gets its own tree and tables (a plan) at a depth chosen by the
// autotuner below.  The passes of all problems are then merged: one queue of
// (problem, work item) pairs per pass (gather, leaf moments, each upward step,
// each downward level, leaf evaluation), walked by persistent kernels, so a
// whole batch is ~2 d_max kernel launches regardless of the number of
// problems.  The launch sequence is captured once in a HIP graph and replayed.
//
// Autotuner: the rates of the evaluation's parts (seconds per near-field
// pair, per S2L unit and channel, per shifted box and channel, per point and
// channel) are measured on the device when a batch is created, by timing the
// phases of a probe problem at two depths; they are kept per device, order,
// mode count and tile width for the process.  The S2L tile width is the one
// whose probe S2L ran fastest.  Each problem's depth is then the one whose
// exactly counted work (near pairs, S2L units, shifted boxes, points, on the
// square the plan will use) costs the least at those rates.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

Arena arena_acquire(size_t bytes);
void plan_build(Plan &pl, const axf_params &p, int64_t ns, const double *rs, const double *zs, int64_t nf,
                const double *rf, const double *zf, hipStream_t st);
void plan_release(Plan *pl);

namespace {

// Seconds per unit of work of one evaluation's parts.
struct Rates {
    double near_pair = 0;    // per near-field pair and right-hand side
    double s2l_unit = 0;     // per S2L unit and channel
    double box = 0;          // per (box, channel) of the M2M and L2L shifts
    double point = 0;        // per (point, channel) of moments, gather and local evaluation
    double s2l_seconds = 0;  // the probe's S2L time (ranks the tile widths)
};

struct Work {
    double near = 0, units = 0, boxes = 0;
};

// The square plan_build will use (the same rule as the tree builder): side =
// larger extent; in r it starts on the axis when that side reaches the
// largest radius, else at the smallest radius; in z at the smallest z.
struct Square {
    double rlo = 0, zlo = 0, invL = 1;
};
Square plan_square(const std::vector<double> &rs, const std::vector<double> &zs, const std::vector<double> &rf,
                   const std::vector<double> &zf)
{
    double rmin = INFINITY, rmax = -INFINITY, zmin = INFINITY, zmax = -INFINITY;
    for (auto v : {&rs, &rf})
        for (double x : *v) {
            rmin = std::min(rmin, x);
            rmax = std::max(rmax, x);
        }
    for (auto v : {&zs, &zf})
        for (double x : *v) {
            zmin = std::min(zmin, x);
            zmax = std::max(zmax, x);
        }
    Square q;
    double L = 1.0;
    int koff = 0;
    square_rule(rmin, rmax, zmin, zmax, q.rlo, q.zlo, L, koff);
    q.invL = 1.0 / L;
    return q;
}

// Exact work of the uniform tree at depth d: near-field pairs over the 3x3
// neighbour leaves, S2L units (a target box with the source boxes at (dr, dz)
// and (dr, -dz) of its interaction list, either occupied: the pairing of the
// tiled S2L), and the boxes the M2M (source parents) and L2L (target
// children) shift.
Work count_work(const std::vector<double> &rs, const std::vector<double> &zs, const std::vector<double> &rf,
                const std::vector<double> &zf, const Square &sq, int d)
{
    const int nb = 1 << d;
    std::vector<int32_t> cs((size_t)nb * nb, 0), cf((size_t)nb * nb, 0);
    for (size_t i = 0; i < rs.size(); ++i)
        cs[(size_t)box_index(rs[i], sq.rlo, sq.invL, d) * nb + box_index(zs[i], sq.zlo, sq.invL, d)]++;
    for (size_t i = 0; i < rf.size(); ++i)
        cf[(size_t)box_index(rf[i], sq.rlo, sq.invL, d) * nb + box_index(zf[i], sq.zlo, sq.invL, d)]++;
    Work w;
    for (int ir = 0; ir < nb; ++ir)
        for (int iz = 0; iz < nb; ++iz) {
            const int t = cf[(size_t)ir * nb + iz];
            if (!t) continue;
            long long s = 0;
            for (int jr = std::max(ir - 1, 0); jr <= std::min(ir + 1, nb - 1); ++jr)
                for (int jz = std::max(iz - 1, 0); jz <= std::min(iz + 1, nb - 1); ++jz) s += cs[(size_t)jr * nb + jz];
            w.near += (double)t * s;
        }
    std::vector<int32_t> s_l = cs, f_l = cf;
    for (int l = d; l >= 2; --l) {
        const int n = 1 << l;
        for (int ir = 0; ir < n; ++ir)
            for (int iz = 0; iz < n; ++iz) {
                if (l < d && s_l[(size_t)ir * n + iz]) w.boxes += 1;        // M2M parent
                if (!f_l[(size_t)ir * n + iz]) continue;
                if (l > 2) w.boxes += 1;                                     // L2L child
                const int dr0 = -2 - (ir & 1), dz0 = -2 - (iz & 1);
                for (int dr = dr0; dr < dr0 + 6; ++dr) {
                    const int jr = ir + dr;
                    if (jr < 0 || jr >= n) continue;
                    const bool near_r = dr >= -1 && dr <= 1;
                    for (int adz = 0; adz <= 3; ++adz) {
                        const bool hasp = adz > 0 && adz <= dz0 + 5 && !(near_r && adz <= 1);
                        const bool hasm = -adz >= dz0 && !(near_r && adz <= 1);
                        const bool occp = hasp && iz + adz < n && s_l[(size_t)jr * n + iz + adz];
                        const bool occm = hasm && iz - adz >= 0 && s_l[(size_t)jr * n + iz - adz];
                        if (occp || occm) w.units += 1;
                    }
                }
            }
        if (l == 2) break;
        const int h = n / 2;
        std::vector<int32_t> s2((size_t)h * h, 0), f2((size_t)h * h, 0);
        for (int ir = 0; ir < n; ++ir)
            for (int iz = 0; iz < n; ++iz) {
                s2[(size_t)(ir >> 1) * h + (iz >> 1)] += s_l[(size_t)ir * n + iz];
                f2[(size_t)(ir >> 1) * h + (iz >> 1)] += f_l[(size_t)ir * n + iz];
            }
        s_l.swap(s2);
        f_l.swap(f2);
    }
    return w;
}

// Phase times of the plan's recorded marks (milliseconds per phase).
void read_marks(Plan &pl, double ms[AXF_NUM_PHASES])
{
    for (int i = 0; i < AXF_NUM_PHASES; ++i) ms[i] = 0.0;
    for (auto &m : pl.marks) {
        AXF_HIP(hipEventSynchronize(m.b));
        float t = 0.f;
        AXF_HIP(hipEventElapsedTime(&t, m.a, m.b));
        ms[m.phase] += t;
    }
}

// Rates from a probe: 20,000 rings of the ring box [0.5, 1.5] x [-0.5, 0.5]
// (a two-dimensional additive recurrence, no random numbers), sources =
// field points, one right-hand side, unit strengths, at depths 4 and 5; the
// leaf runs fused with the local evaluation, as in the batch kernels.
Rates probe_rates(int M, int nmodes, int tb, hipStream_t st)
{
    const int n = 20000;
    std::vector<double> h(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const double a = (i + 0.5) * 0.7548776662466927, b = (i + 0.5) * 0.5698402909980532;
        h[i] = 0.5 + (a - std::floor(a));
        h[n + i] = -0.5 + (b - std::floor(b));
    }
    Sizer sz;
    sz.add<double>(2 * (size_t)n);
    sz.add<double2>((size_t)nmodes * n);
    sz.add<double2>((size_t)nmodes * n);
    Arena a = arena_acquire(sz.bytes + 4096);
    double *xy = a.take<double>(2 * (size_t)n);
    double2 *S = a.take<double2>((size_t)nmodes * n);
    double2 *phi = a.take<double2>((size_t)nmodes * n);
    std::vector<double2> ones((size_t)nmodes * n, make_double2(1.0, 0.0));
    Rates r;
    double ms[AXF_NUM_PHASES] = {}, near = 0, units = 0, boxes = 0, pts = 0;
    try {
        AXF_HIP(hipMemcpyAsync(xy, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
        AXF_HIP(hipMemcpyAsync(S, ones.data(), ones.size() * sizeof(double2), hipMemcpyHostToDevice, st));
        for (int d : {4, 5}) {
            axf_params pp{};
            pp.n_modes = nmodes;
            pp.order = M;
            pp.depth = d;
            pp.max_leaf = 64;
            pp.nrhs = 1;
            pp.flags = AXF_TILE(tb);
            Plan pl;
            try {
                plan_build(pl, pp, n, xy, xy + n, n, xy, xy + n, st);
                if (pl.tables_ready) AXF_HIP(hipEventSynchronize(pl.tables_ready));
                EvalOut o;
                o.phi = (double *)phi;
                o.fused = true;
                run_fmm(pl, pl.src, pl.fld, (const double *)S, o, st);
                pl.timing = true;
                for (int rep = 0; rep < 2; ++rep) run_fmm(pl, pl.src, pl.fld, (const double *)S, o, st);
                double m[AXF_NUM_PHASES];
                read_marks(pl, m);
                for (int i = 0; i < AXF_NUM_PHASES; ++i) ms[i] += m[i] / 2.0;
                near += pl.near_pairs;
                units += (double)pl.s2l_units * pl.C;
                for (int l = 2; l < pl.d; ++l) boxes += (double)pl.src.nocc[l] * pl.C;
                for (int l = 3; l <= pl.d; ++l) boxes += (double)pl.fld.nocc[l] * pl.C;
                pts += 2.0 * n * pl.C;
            } catch (...) {
                plan_release(&pl);
                throw;
            }
            plan_release(&pl);
        }
    } catch (...) {
        arena_release(a);
        throw;
    }
    arena_release(a);
    r.near_pair = ms[AXF_PHASE_LEAF] * 1e-3 / std::max(near, 1.0);
    r.s2l_unit = ms[AXF_PHASE_S2L] * 1e-3 / std::max(units, 1.0);
    r.box = (ms[AXF_PHASE_M2M] + ms[AXF_PHASE_L2L]) * 1e-3 / std::max(boxes, 1.0);
    r.point = (ms[AXF_PHASE_GATHER] + ms[AXF_PHASE_P2M]) * 1e-3 / std::max(pts, 1.0);
    r.s2l_seconds = ms[AXF_PHASE_S2L] * 1e-3;
    return r;
}

Rates measured_rates(int M, int nmodes, int tb, hipStream_t st)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, Rates> cache;
    int dev = 0;
    AXF_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, M, nmodes, tb);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    Rates r = probe_rates(M, nmodes, tb, st);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = r;
    return r;
}

// Modelled seconds of problem pb at every depth and tile width: the exact
// work counts of each depth priced at the probe rates of each width
// (rates[t] for width kTiles[t]; a width whose rates are absent, s2l_unit
// zero, is skipped).  Entries that are not modelled hold INFINITY.  Returns
// the (depth, tile index) of least modelled time.
using Model = double[AXF_MAX_DEPTH + 2][3];
std::pair<int, int> autotune_model(const axf_problem &pb, int nmodes, const Rates *rates, hipStream_t st,
                                   Model &model)
{
    for (auto &row : model)
        for (double &v : row) v = INFINITY;
    std::vector<double> rs(pb.ns), zs(pb.ns), rf(pb.nf), zf(pb.nf);
    AXF_HIP(hipMemcpyAsync(rs.data(), pb.r_src, pb.ns * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(zs.data(), pb.z_src, pb.ns * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(rf.data(), pb.r_fld, pb.nf * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(zf.data(), pb.z_fld, pb.nf * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipStreamSynchronize(st));
    const Square sq = plan_square(rs, zs, rf, zf);
    const double C = (double)nmodes * pb.nrhs;
    std::pair<int, int> best{2, tile_index(kDefaultTile)};
    double best_t = INFINITY;
    const double npts = (double)std::max(pb.ns, pb.nf);
    for (int d = 2; d <= AXF_MAX_DEPTH; ++d) {
        if (d > 2 && npts / std::pow(4.0, d - 1) < 1.0) break;   // deeper than one point per box
        const Work w = count_work(rs, zs, rf, zf, sq, d);
        for (int t = 0; t < 3; ++t) {
            const Rates &r = rates[t];
            if (r.s2l_unit <= 0) continue;
            // near-field cost in units of one right-hand side: with G^(n)
            // shared by the right-hand sides (near_class > 0) each further
            // one adds about a quarter (measured: 1, 2, 4, 8 right-hand
            // sides of a 100,000-ring box in 1.3, 1.4, 2.0, 4.3 ms)
            const double nq = near_class(pb.nrhs, mode_bucket(nmodes)) ? 1.0 + 0.25 * (pb.nrhs - 1) : pb.nrhs;
            const double tm = w.near * nq * r.near_pair + w.units * C * r.s2l_unit + w.boxes * C * r.box +
                              (double)(pb.ns + pb.nf) * C * r.point;
            model[d][t] = tm;
            if (tm < best_t) {
                best_t = tm;
                best = {d, t};
            }
        }
    }
    return best;
}

// Descriptors and merged work queues of a set of plans (problem i of the
// queues is plans[i], evaluating S[i] into phi[i]), in one arena; the
// uploads are queued on `st`.
void build_queues(const std::vector<Plan *> &plans, const std::vector<const double *> &S,
                  const std::vector<double *> &phi, int M, int nmodes, Arena &mem, BatchQueues &q, hipStream_t st)
{
    const int nprob = (int)plans.size();
    std::vector<ProbDev> pd(nprob);
    std::vector<int2> qg, qp, ql, qlc[4];
    std::vector<std::vector<int2>> qm(AXF_MAX_DEPTH + 1), qlt(AXF_MAX_DEPTH + 1), qs(3 * (AXF_MAX_DEPTH + 1));
    int maxd = 2;
    for (int i = 0; i < nprob; ++i) {
        const Plan &pl = *plans[i];
        maxd = std::max(maxd, pl.d);
        fill_probdev(pl, S[i], phi[i], pd[i]);
        int64_t ge = pl.src.n * pl.Cs;
        for (int64_t k = 0; k * 256 < ge; ++k) qg.push_back(make_int2(i, (int)k));
        for (int k = 0; k < pl.src.nocc[pl.d] * p2m_pairs(pl.C); ++k) qp.push_back(make_int2(i, k));
        for (int t = 1; pl.d - t >= 2; ++t)
            for (int k = 0; k < pl.src.nocc[pl.d - t] * pl.C; ++k) qm[t].push_back(make_int2(i, k));
        for (int l = 2; l <= pl.d; ++l) {
            for (int k = 0; k < pl.fld.nocc[l] * pl.C; ++k) qlt[l].push_back(make_int2(i, k));
            for (int k = 0; k < pl.fld.ntiles[l] * pl.C; ++k)
                qs[3 * l + tile_index(pl.tb)].push_back(make_int2(i, k));
        }
        const int cls = near_class(pl.nrhs, pl.nmb);
        for (int k = 0; k < pl.fld.nchunks; ++k) {
            ql.push_back(make_int2(i, k));
            qlc[cls].push_back(make_int2(i, k));
        }
    }
    Sizer sz;
    sz.add<ProbDev>(nprob);
    sz.add<int2>(qg.size() + 1);
    sz.add<int2>(qp.size() + 1);
    sz.add<int2>(ql.size() + 1);
    for (int c = 0; c < 4; ++c) sz.add<int2>(qlc[c].size() + 1);
    for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
        sz.add<int2>(qm[l].size() + 1);
        sz.add<int2>(qlt[l].size() + 1);
        for (int t = 0; t < 3; ++t) sz.add<int2>(qs[3 * l + t].size() + 1);
    }
    mem = arena_acquire(sz.bytes + 4096);
    q = BatchQueues();
    ProbDev *dp = mem.take<ProbDev>(nprob);
    auto up = [&](const std::vector<int2> &v, int2 *&dst, int &n) {
        dst = mem.take<int2>(v.size() + 1);
        n = (int)v.size();
        if (n) AXF_HIP(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    };
    AXF_HIP(hipMemcpyAsync(dp, pd.data(), sizeof(ProbDev) * nprob, hipMemcpyHostToDevice, st));
    up(qg, q.gather, q.ngather);
    up(qp, q.p2m, q.np2m);
    up(ql, q.leaf, q.nleaf);
    for (int c = 0; c < 4; ++c) up(qlc[c], q.leafq[c], q.nleafq[c]);
    for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
        up(qm[l], q.m2m[l], q.nm2m[l]);
        up(qlt[l], q.l2l[l], q.nl2l[l]);
        for (int t = 0; t < 3; ++t) up(qs[3 * l + t], q.s2l[l][t], q.ns2l[l][t]);
    }
    AXF_HIP(hipStreamSynchronize(st));   // the host images go out of scope
    q.probs = dp;
    q.M = M;
    q.nmodes = nmodes;
    q.nmb = mode_bucket(nmodes);
    q.TS = (M + 1) * (M + 1) * (M + 1);
    q.maxd = maxd;
    q.chistar = plans[0]->chistar;
}

// Problems with at least this many points get their depth and tile width
// from trial evaluations: the modelled (depth, width), then at that width the
// neighbouring depth the model ranks next, further in whichever direction
// improves, and last the other widths at the fastest depth.  Smaller
// problems take the modelled pair.
constexpr int64_t kTrialPoints = 2000;

// One problem evaluated through the batch kernels at depth d and S2L tile
// width tb (a one-problem queue, an eager launch on `st`): the plan, and the
// time of one run.
Plan *trial_plan(const axf_problem &pb, axf_params pp, int d, int tb, const BatchSide &side, hipStream_t st,
                 double &sec)
{
    pp.depth = d;
    pp.flags = AXF_TILE(tb);
    Plan *pl = new Plan();
    Arena mem;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        arena_release(mem);
    };
    try {
        plan_build(*pl, pp, pb.ns, pb.r_src, pb.z_src, pb.nf, pb.r_fld, pb.z_fld, st);
        if (pl->tables_ready) AXF_HIP(hipEventSynchronize(pl->tables_ready));
        BatchQueues q;
        build_queues({pl}, {pb.S}, {pb.phi}, pp.order, pp.n_modes, mem, q, st);
        AXF_HIP(hipEventCreate(&e0));
        AXF_HIP(hipEventCreate(&e1));
        AXF_HIP(hipEventRecord(e0, st));
        run_batch(q, st, &side);
        AXF_HIP(hipEventRecord(e1, st));
        AXF_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        AXF_HIP(hipEventElapsedTime(&ms, e0, e1));
        sec = 1e-3 * ms;
    } catch (...) {
        cleanup();
        plan_release(pl);
        delete pl;
        throw;
    }
    cleanup();
    return pl;
}

// The plan of one autotuned problem; rates[t] are the probe rates of tile
// width kTiles[t] (s2l_unit zero: that width is not considered).
Plan *tune_problem(const axf_problem &pb, const axf_params &pp, const Rates *rates, const BatchSide &side,
                   hipStream_t st)
{
    Model model;
    const std::pair<int, int> m0 = autotune_model(pb, pp.n_modes, rates, st, model);
    const int d0 = m0.first, t0 = m0.second;
    const double npts = (double)std::max(pb.ns, pb.nf);
    if (std::max(pb.ns, pb.nf) < kTrialPoints) {
        axf_params p1 = pp;
        p1.depth = d0;
        p1.flags = AXF_TILE(kTiles[t0]);
        Plan *pl = new Plan();
        try {
            plan_build(*pl, p1, pb.ns, pb.r_src, pb.z_src, pb.nf, pb.r_fld, pb.z_fld, st);
        } catch (...) {
            plan_release(pl);
            delete pl;
            throw;
        }
        return pl;
    }
    Plan *best = nullptr;
    int bestd = d0;
    double bests = INFINITY;
    std::vector<std::pair<int, int>> tried;
    // true when (depth d, tile index t) was tried and became the best
    auto trial = [&](int d, int t) -> bool {
        if (d < 2 || d > AXF_MAX_DEPTH || (d > 2 && npts / std::pow(4.0, d - 1) < 1.0)) return false;
        if (rates[t].s2l_unit <= 0) return false;
        if (std::find(tried.begin(), tried.end(), std::make_pair(d, t)) != tried.end()) return false;
        tried.emplace_back(d, t);
        double sec = INFINITY;
        Plan *p = trial_plan(pb, pp, d, kTiles[t], side, st, sec);
        if (!best || sec < bests) {
            if (best) {
                plan_release(best);
                delete best;
            }
            best = p;
            bestd = d;
            bests = sec;
            return true;
        }
        plan_release(p);
        delete p;
        return false;
    };
    try {
        trial(d0, t0);
        const int lo = d0 - 1, hi = d0 + 1;
        const double mlo = lo >= 2 ? model[lo][t0] : INFINITY, mhi = model[hi][t0];
        const int first = mlo <= mhi ? lo : hi, second = first == lo ? hi : lo;
        int dir = 0;
        if (trial(first, t0)) {
            dir = first - d0;
        } else if (trial(second, t0)) {
            dir = second - d0;
        }
        while (dir != 0 && trial(bestd + dir, t0)) {
        }
        const int dbest = bestd;
        for (int t = 0; t < 3; ++t)
            if (t != t0) trial(dbest, t);
    } catch (...) {
        if (best) {
            plan_release(best);
            delete best;
        }
        throw;
    }
    return best;
}

}  // namespace
}  // namespace axf

using namespace axf;

struct axf_batch {
    int device = 0;
    axf_params p{};
    std::vector<axf_problem> probs;
    std::vector<Plan *> plans;
    std::vector<int> depth, tile;   // per problem
    int tb = kDefaultTile;           // width of the problems with a given depth
    Arena qmem;
    BatchQueues q;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    BatchSide side;              // the near field's branch of the graph
};

static void batch_free(axf_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->side.stream) (void)hipStreamDestroy(b->side.stream);
    if (b->side.fork) (void)hipEventDestroy(b->side.fork);
    if (b->side.join) (void)hipEventDestroy(b->side.join);
    for (Plan *pl : b->plans) {
        plan_release(pl);
        delete pl;
    }
    arena_release(b->qmem);
    delete b;
}

extern "C" {

axf_status axf_batch_create(const axf_params *params, int32_t nprob, const axf_problem *problems, void *stream,
                            axf_batch **out_batch)
{
    axf_batch *b = nullptr;
    try {
        AXF_REQUIRE(out_batch != nullptr, AXF_ERR_INVALID_ARGUMENT, "out_batch is NULL");
        *out_batch = nullptr;
        AXF_REQUIRE(params && problems && nprob >= 1, AXF_ERR_INVALID_ARGUMENT, "params, problems and nprob >= 1");
        AXF_REQUIRE(params->n_modes >= 1 && params->n_modes <= AXF_MAX_MODES, AXF_ERR_UNSUPPORTED,
                    "n_modes must be in 1..64");
        AXF_REQUIRE(params->order >= 0 && params->order <= AXF_MAX_ORDER, AXF_ERR_UNSUPPORTED,
                    "order must be in 0..24");
        for (int i = 0; i < nprob; ++i) {
            const axf_problem &pb = problems[i];
            AXF_REQUIRE(pb.ns >= 1 && pb.nf >= 1 && pb.r_src && pb.z_src && pb.r_fld && pb.z_fld && pb.S && pb.phi,
                        AXF_ERR_INVALID_ARGUMENT, "problem " + std::to_string(i) + ": empty or NULL arrays");
            AXF_REQUIRE(pb.nrhs >= 1 && pb.nrhs <= AXF_MAX_RHS, AXF_ERR_UNSUPPORTED,
                        "problem " + std::to_string(i) + ": nrhs must be in 1..8");
            AXF_REQUIRE(pb.depth == 0 || (pb.depth >= 2 && pb.depth <= AXF_MAX_DEPTH), AXF_ERR_UNSUPPORTED,
                        "problem " + std::to_string(i) + ": depth must be 0 or in 2..11");
            AXF_REQUIRE(pb.tile == 0 || s2l_tile_ok(pb.tile), AXF_ERR_UNSUPPORTED,
                        "problem " + std::to_string(i) + ": S2L tile width must be 0, 2, 4 or 8");
            AXF_REQUIRE(pb.depth != 0 || !(params->flags & AXF_BATCH_NO_AUTOTUNE) || params->max_leaf >= 1,
                        AXF_ERR_INVALID_ARGUMENT, "max_leaf must be >= 1 without the autotuner");
        }
        AXF_REQUIRE((params->flags & ~(AXF_BATCH_NO_AUTOTUNE | AXF_TILE_MASK)) == 0, AXF_ERR_INVALID_ARGUMENT,
                    "unknown batch flags");
        const int tb_given = (int)((params->flags & AXF_TILE_MASK) >> AXF_TILE_SHIFT);
        AXF_REQUIRE(tb_given == 0 || s2l_tile_ok(tb_given), AXF_ERR_UNSUPPORTED,
                    "S2L tile width must be 2, 4 or 8 (or 0)");
        hipStream_t st = (hipStream_t)stream;
        b = new axf_batch();
        AXF_HIP(hipGetDevice(&b->device));
        b->p = *params;
        b->probs.assign(problems, problems + nprob);
        const bool tune = !(params->flags & AXF_BATCH_NO_AUTOTUNE);
        // the width of problems that name none and are not autotuned: the
        // flag's, else (autotuner on) the one whose probe S2L ran fastest
        Rates rates[3];
        auto rates_of = [&](int t) -> const Rates & {
            if (rates[t].s2l_unit <= 0) rates[t] = measured_rates(params->order, params->n_modes, kTiles[t], st);
            return rates[t];
        };
        if (tb_given) {
            b->tb = tb_given;
        } else if (!tune) {
            b->tb = kDefaultTile;
        } else {
            double best = INFINITY;
            for (int t = 0; t < 3; ++t)
                if (rates_of(t).s2l_seconds < best) {
                    best = rates[t].s2l_seconds;
                    b->tb = kTiles[t];
                }
        }
        AXF_HIP(hipStreamCreateWithFlags(&b->side.stream, hipStreamNonBlocking));
        AXF_HIP(hipEventCreateWithFlags(&b->side.fork, hipEventDisableTiming));
        AXF_HIP(hipEventCreateWithFlags(&b->side.join, hipEventDisableTiming));
        for (int i = 0; i < nprob; ++i) {
            const axf_problem &pb = problems[i];
            axf_params pp = *params;
            pp.nrhs = pb.nrhs;
            const int tb_prob = pb.tile ? pb.tile : tb_given;   // 0: not fixed for this problem
            pp.flags = AXF_TILE(tb_prob ? tb_prob : b->tb);
            Plan *pl = nullptr;
            if (pb.depth != 0 || !tune) {
                pp.depth = pb.depth;          // 0 without the autotuner: the max_leaf rule
                pl = new Plan();
                try {
                    plan_build(*pl, pp, pb.ns, pb.r_src, pb.z_src, pb.nf, pb.r_fld, pb.z_fld, st);
                } catch (...) {
                    plan_release(pl);
                    delete pl;
                    throw;
                }
            } else {
                // the widths it may take, with their rates
                Rates cand[3];
                for (int t = 0; t < 3; ++t)
                    if (!tb_prob || kTiles[t] == tb_prob) cand[t] = rates_of(t);
                pl = tune_problem(pb, pp, cand, b->side, st);
            }
            b->plans.push_back(pl);
            b->depth.push_back(pl->d);
            b->tile.push_back(pl->tb);
        }
        // the batch's passes do not wait on the table stream: tables first
        for (Plan *pl : b->plans)
            if (pl->tables_ready) AXF_HIP(hipEventSynchronize(pl->tables_ready));
        std::vector<const double *> Sv(nprob);
        std::vector<double *> phiv(nprob);
        for (int i = 0; i < nprob; ++i) {
            Sv[i] = problems[i].S;
            phiv[i] = problems[i].phi;
        }
        BatchQueues &q = b->q;
        build_queues(b->plans, Sv, phiv, params->order, params->n_modes, b->qmem, q, st);
        // one eager pass (sets kernel attributes), then capture the sequence
        run_batch(q, st, &b->side);
        AXF_HIP(hipStreamSynchronize(st));
        AXF_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        AXF_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        run_batch(q, b->cap, &b->side);
        AXF_HIP(hipStreamEndCapture(b->cap, &b->graph));
        AXF_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        *out_batch = b;
        return AXF_OK;
    } catch (const Fail &f) {
        if (b && b->cap) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(b->cap, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        batch_free(b);
        return f.st;
    } catch (const std::bad_alloc &) {
        batch_free(b);
        set_error("host allocation failed");
        return AXF_ERR_OUT_OF_MEMORY;
    }
}

axf_status axf_batch_launch(axf_batch *b, void *stream)
{
    try {
        AXF_REQUIRE(b && b->exec, AXF_ERR_INVALID_ARGUMENT, "batch is NULL");
        AXF_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

axf_status axf_batch_launch_plain(axf_batch *b, void *stream)
{
    try {
        AXF_REQUIRE(b, AXF_ERR_INVALID_ARGUMENT, "batch is NULL");
        for (size_t i = 0; i < b->plans.size(); ++i) {
            EvalOut o;
            o.phi = b->probs[i].phi;
            Plan &pl = *b->plans[i];
            run_fmm(pl, pl.src, pl.fld, b->probs[i].S, o, (hipStream_t)stream);
        }
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

axf_status axf_batch_problem_depth(const axf_batch *b, int32_t i, int32_t *depth)
{
    try {
        AXF_REQUIRE(b && depth && i >= 0 && i < (int32_t)b->depth.size(), AXF_ERR_INVALID_ARGUMENT,
                    "bad batch, index or output pointer");
        *depth = b->depth[i];
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

axf_status axf_batch_problem_tile(const axf_batch *b, int32_t i, int32_t *tile)
{
    try {
        AXF_REQUIRE(b && tile && i >= 0 && i < (int32_t)b->tile.size(), AXF_ERR_INVALID_ARGUMENT,
                    "bad batch, index or output pointer");
        *tile = b->tile[i];
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

void axf_batch_destroy(axf_batch *b) { batch_free(b); }

}  // extern "C"

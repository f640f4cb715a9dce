// axf_batch.hip -- batched evaluation of many independent problems.
//
// Each problem gets its own tree and tables (a plan) at a depth chosen by the
// autotuner below.  The passes of all problems are then merged: one queue of
// (problem, work item) pairs per pass (gather, leaf moments, each upward step,
// each downward level, leaf evaluation), walked by persistent kernels, so a
// whole batch is ~2 d_max kernel launches regardless of the number of
// problems.  The launch sequence is captured once in a HIP graph and replayed.
//
// Autotuner: for every candidate depth the exact work of the FMM is counted
// on the host from the points (near-field pairs, S2L box pairs, occupied
// boxes), and the depth with the smallest modelled time is kept.  The model's
// rates are the measured throughputs of the kernels on MI355X.
#include <algorithm>
#include <cmath>
#include <vector>

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

Arena arena_acquire(size_t bytes);
void plan_build(Plan &pl, const axf_params &p, int64_t ns, const double *rs, const double *zs, int64_t nf,
                const double *rf, const double *zf, hipStream_t st);
void plan_release(Plan *pl);

namespace {

// Modelled seconds of one evaluation at depth d (work counted on the host).
struct DepthModel {
    double near_pair_s, s2l_flop_s, m2m_box_s, leaf_point_s;
};

DepthModel model_rates(int M, int nmodes, int nrhs)
{
    DepthModel m;
    // near field: 6.6e-11 s per pair at 17 modes, one right-hand side; the
    // kernel re-evaluates G for every right-hand side
    m.near_pair_s = 6.6e-11 * (nmodes + 17.0) / 34.0 * nrhs;
    // tiled S2L: ~3 TFLOP/s at M = 12 rising to ~7 TFLOP/s at M = 24
    double rate = 3e12 + std::max(0, std::min(12, M - 12)) * (4e12 / 12.0);
    m.s2l_flop_s = 1.0 / rate;
    const double c4 = (M + 1.0) * (M + 2) * (M + 3) * (M + 4) / 24.0;
    m.m2m_box_s = 4.6e-11 * c4 * nmodes * nrhs;
    const double P = (M + 1.0) * (M + 2) / 2;
    m.leaf_point_s = 2e-12 * P * nmodes * nrhs;
    return m;
}

struct Counts {
    double near = 0, s2l = 0, boxes = 0;
};

// Work of the uniform tree at depth d over the union bounding square.
Counts count_work(const std::vector<double> &rs, const std::vector<double> &zs, const std::vector<double> &rf,
                  const std::vector<double> &zf, double rlo, double zlo, double invL, int d)
{
    const int nb = 1 << d;
    std::vector<int32_t> cs((size_t)nb * nb, 0), cf((size_t)nb * nb, 0);
    for (size_t i = 0; i < rs.size(); ++i)
        cs[(size_t)box_index(rs[i], rlo, invL, d) * nb + box_index(zs[i], zlo, invL, d)]++;
    for (size_t i = 0; i < rf.size(); ++i)
        cf[(size_t)box_index(rf[i], rlo, invL, d) * nb + box_index(zf[i], zlo, invL, d)]++;
    Counts c;
    for (int ir = 0; ir < nb; ++ir)
        for (int iz = 0; iz < nb; ++iz) {
            int t = cf[(size_t)ir * nb + iz];
            if (!t) continue;
            long long s = 0;
            for (int jr = std::max(ir - 1, 0); jr <= std::min(ir + 1, nb - 1); ++jr)
                for (int jz = std::max(iz - 1, 0); jz <= std::min(iz + 1, nb - 1); ++jz) s += cs[(size_t)jr * nb + jz];
            c.near += (double)t * s;
        }
    // coarser levels by aggregation
    std::vector<int32_t> s_l = cs, f_l = cf;
    for (int l = d; l >= 2; --l) {
        const int n = 1 << l;
        for (int ir = 0; ir < n; ++ir)
            for (int iz = 0; iz < n; ++iz) {
                if (!f_l[(size_t)ir * n + iz]) continue;
                c.boxes += 1;
                for (int jr = 2 * (ir >> 1) - 2; jr < 2 * (ir >> 1) + 4; ++jr)
                    for (int jz = 2 * (iz >> 1) - 2; jz < 2 * (iz >> 1) + 4; ++jz) {
                        if (jr < 0 || jz < 0 || jr >= n || jz >= n) continue;
                        if (std::abs(jr - ir) <= 1 && std::abs(jz - iz) <= 1) continue;
                        if (s_l[(size_t)jr * n + jz]) c.s2l += 1;
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
    return c;
}

int autotune_depth(const axf_problem &pb, int M, int nmodes, hipStream_t st)
{
    std::vector<double> rs(pb.ns), zs(pb.ns), rf(pb.nf), zf(pb.nf);
    AXF_HIP(hipMemcpyAsync(rs.data(), pb.r_src, pb.ns * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(zs.data(), pb.z_src, pb.ns * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(rf.data(), pb.r_fld, pb.nf * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(zf.data(), pb.z_fld, pb.nf * sizeof(double), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipStreamSynchronize(st));
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
    double ext = std::max(rmax - rmin, zmax - zmin);
    double L = ext > 0 ? ext : 1.0, invL = 1.0 / L;
    DepthModel m = model_rates(M, nmodes, pb.nrhs);
    const double P = (M + 1.0) * (M + 2) / 2;
    const double C = (double)nmodes * pb.nrhs;
    int best = 2;
    double best_t = INFINITY;
    const double npts = (double)std::max(pb.ns, pb.nf);
    for (int d = 2; d <= AXF_MAX_DEPTH; ++d) {
        if (d > 2 && npts / std::pow(4.0, d - 1) < 1.0) break;   // deeper than one point per box
        Counts c = count_work(rs, zs, rf, zf, rmin, zmin, invL, d);
        double t = c.near * m.near_pair_s + c.s2l * C * P * P * 4.0 * m.s2l_flop_s + c.boxes * m.m2m_box_s +
                   (double)pb.nf * m.leaf_point_s + 5e-6 * d;
        if (t < best_t) {
            best_t = t;
            best = d;
        }
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
    std::vector<int> depth;
    Arena qmem;
    BatchQueues q;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

static void batch_free(axf_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
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
            AXF_REQUIRE(pb.depth != 0 || !(params->flags & AXF_BATCH_NO_AUTOTUNE) || params->max_leaf >= 1,
                        AXF_ERR_INVALID_ARGUMENT, "max_leaf must be >= 1 without the autotuner");
        }
        hipStream_t st = (hipStream_t)stream;
        b = new axf_batch();
        AXF_HIP(hipGetDevice(&b->device));
        b->p = *params;
        b->probs.assign(problems, problems + nprob);
        int maxd = 2;
        for (int i = 0; i < nprob; ++i) {
            const axf_problem &pb = problems[i];
            axf_params pp = *params;
            pp.nrhs = pb.nrhs;
            pp.flags = 0;
            if (pb.depth != 0) {
                pp.depth = pb.depth;
            } else if (params->flags & AXF_BATCH_NO_AUTOTUNE) {
                pp.depth = 0;
            } else {
                pp.depth = autotune_depth(pb, params->order, params->n_modes, st);
            }
            Plan *pl = new Plan();
            b->plans.push_back(pl);
            plan_build(*pl, pp, pb.ns, pb.r_src, pb.z_src, pb.nf, pb.r_fld, pb.z_fld, st);
            b->depth.push_back(pl->d);
            maxd = std::max(maxd, pl->d);
        }
        // the batch's passes do not wait on the table stream: tables first
        for (Plan *pl : b->plans)
            if (pl->tables_ready) AXF_HIP(hipEventSynchronize(pl->tables_ready));
        // descriptors and merged queues
        std::vector<ProbDev> pd(nprob);
        std::vector<int2> qg, qp, ql;
        std::vector<std::vector<int2>> qm(AXF_MAX_DEPTH + 1), qs(AXF_MAX_DEPTH + 1), qlt(AXF_MAX_DEPTH + 1);
        for (int i = 0; i < nprob; ++i) {
            const Plan &pl = *b->plans[i];
            fill_probdev(pl, problems[i].S, problems[i].phi, pd[i]);
            int64_t ge = pl.src.n * pl.Cs;
            for (int64_t k = 0; k * 256 < ge; ++k) qg.push_back(make_int2(i, (int)k));
            for (int k = 0; k < pl.src.nocc[pl.d] * p2m_pairs(pl.C); ++k) qp.push_back(make_int2(i, k));
            for (int t = 1; pl.d - t >= 2; ++t)
                for (int k = 0; k < pl.src.nocc[pl.d - t] * pl.C; ++k) qm[t].push_back(make_int2(i, k));
            for (int l = 2; l <= pl.d; ++l) {
                for (int k = 0; k < pl.fld.nocc[l] * pl.C; ++k) qlt[l].push_back(make_int2(i, k));
                for (int k = 0; k < pl.fld.ntiles[l] * pl.C; ++k) qs[l].push_back(make_int2(i, k));
            }
            for (int k = 0; k < pl.fld.nchunks; ++k) ql.push_back(make_int2(i, k));
        }
        Sizer sz;
        sz.add<ProbDev>(nprob);
        sz.add<int2>(qg.size() + 1);
        sz.add<int2>(qp.size() + 1);
        sz.add<int2>(ql.size() + 1);
        for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
            sz.add<int2>(qm[l].size() + 1);
            sz.add<int2>(qs[l].size() + 1);
            sz.add<int2>(qlt[l].size() + 1);
        }
        b->qmem = arena_acquire(sz.bytes + 4096);
        BatchQueues &q = b->q;
        ProbDev *dp = b->qmem.take<ProbDev>(nprob);
        auto up = [&](const std::vector<int2> &v, int2 *&dst, int &n) {
            dst = b->qmem.take<int2>(v.size() + 1);
            n = (int)v.size();
            if (n) AXF_HIP(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, st));
        };
        AXF_HIP(hipMemcpyAsync(dp, pd.data(), sizeof(ProbDev) * nprob, hipMemcpyHostToDevice, st));
        up(qg, q.gather, q.ngather);
        up(qp, q.p2m, q.np2m);
        up(ql, q.leaf, q.nleaf);
        for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
            up(qm[l], q.m2m[l], q.nm2m[l]);
            up(qs[l], q.s2l[l], q.ns2l[l]);
            up(qlt[l], q.l2l[l], q.nl2l[l]);
        }
        AXF_HIP(hipStreamSynchronize(st));
        q.probs = dp;
        q.M = params->order;
        q.nmodes = params->n_modes;
        q.nmb = mode_bucket(params->n_modes);
        q.TS = (params->order + 1) * (params->order + 1) * (params->order + 1);
        q.maxd = maxd;
        q.chistar = b->plans[0]->chistar;
        // one eager pass (sets kernel attributes), then capture the sequence
        run_batch(q, st);
        AXF_HIP(hipStreamSynchronize(st));
        AXF_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        AXF_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        run_batch(q, b->cap);
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

void axf_batch_destroy(axf_batch *b) { batch_free(b); }

}  // extern "C"

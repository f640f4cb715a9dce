// axf_noalloc.hip -- axf_evaluate_noalloc: the FMM evaluation of
// axf_evaluate with its evaluation scratch (strengths gathered into tree
// order, moments, locals and the S2L partial sums) taken from a fixed device
// array of the library instead of the plan's memory, so that the call
// allocates nothing.
#include <algorithm>
#include <mutex>

#include "axf_internal.hpp"

namespace axf {
namespace {

// Largest evaluation scratch the entry point serves.  Every GPU the
// library runs on holds this array until the process ends.
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
char *g_scratch_ptr[64] = {};   // device address of `scratch` on each device

// The array's name is a host-side stand-in: its device address is looked up
// once per device, with that device current, and used from then on.
char *scratch_on_device(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    AXF_REQUIRE(device >= 0 && device < 64, AXF_ERR_UNSUPPORTED, "device index beyond 63");
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        AXF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[device] = static_cast<char *>(p);
    }
    return g_scratch_ptr[device];
}

// Points the plan's evaluation buffers at the scratch for one call and puts
// the plan's own back afterwards (also when the call fails).  Phase timing
// is off meanwhile: its events would be created on demand.
struct ScratchSwap {
    Plan &pl;
    double2 *Sg, *part;
    double2 *mom[AXF_MAX_DEPTH + 1], *loc[AXF_MAX_DEPTH + 1];
    bool timing;
    ScratchSwap(Plan &p, char *base) : pl(p), Sg(p.Sg), part(p.s2l_part), timing(p.timing)
    {
        for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
            mom[l] = p.lev[l].mom;
            loc[l] = p.lev[l].loc;
        }
        Arena a;
        a.base = base;
        a.bytes = kNoAllocScratchBytes;
        carve(p, a);
        p.timing = false;
    }
    ~ScratchSwap()
    {
        pl.Sg = Sg;
        pl.s2l_part = part;
        for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
            pl.lev[l].mom = mom[l];
            pl.lev[l].loc = loc[l];
        }
        pl.timing = timing;
    }
    // The same carving sizes the scratch (Sizer) and fills it (Arena).
    template <class A>
    static void carve(Plan &p, A &a)
    {
        take(a, p.Sg, (size_t)std::max<int64_t>(p.src.n, 1) * p.Cs);
        for (int l = 2; l <= p.d; ++l) {
            const size_t nb = (size_t)std::max(std::max(p.src.nocc[l], p.fld.nocc[l]), 1);
            take(a, p.lev[l].mom, nb * p.C * p.P);
            take(a, p.lev[l].loc, nb * p.C * p.P);
        }
        size_t part = 1;
        for (int l = 2; l <= p.d; ++l)
            if (p.fld.s2l_groups[l] > 1)
                part = std::max(part, (size_t)p.fld.s2l_groups[l] * p.fld.nocc[l] * p.C * p.P);
        take(a, p.s2l_part, part);
    }
    static void take(Arena &a, double2 *&dst, size_t n) { dst = a.take<double2>(n); }
    static void take(Sizer &s, double2 *&, size_t n) { s.add<double2>(n); }
};

size_t noalloc_bytes(Plan &pl)
{
    Sizer s;
    ScratchSwap::carve(pl, s);
    return s.bytes;
}

}  // namespace
}  // namespace axf

using namespace axf;

extern "C" axf_status axf_evaluate_noalloc(axf_plan *plan, const double *S, double *phi, void *stream)
{
    try {
        AXF_REQUIRE(plan && S && phi, AXF_ERR_INVALID_ARGUMENT, "plan, S and phi must be non-NULL");
        Plan &pl = plan->pl;
        const size_t need = noalloc_bytes(pl);
        AXF_REQUIRE(need <= kNoAllocScratchBytes, AXF_ERR_UNSUPPORTED,
                    "the evaluation needs " + std::to_string(need) + " bytes of scratch, more than the " +
                        std::to_string(kNoAllocScratchBytes) + " bytes axf_evaluate_noalloc holds; use axf_evaluate");
        int cur = -1;
        AXF_HIP(hipGetDevice(&cur));
        AXF_REQUIRE(cur == pl.device, AXF_ERR_INVALID_ARGUMENT, "the plan's device must be the current device");
        char *base = scratch_on_device(pl.device);
        ScratchSwap swap(pl, base);
        EvalOut o;
        o.phi = phi;
        run_fmm(pl, pl.src, pl.fld, S, o, (hipStream_t)stream);
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (...) {
        set_error("unexpected internal error");
        return AXF_ERR_HIP;
    }
}

// axf_internal.hpp -- host-side structures shared by the library sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <functional>
#include <vector>
#include <algorithm>
#include <cmath>
#include <utility>

#include "axf.h"

namespace axf {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
const char *get_error();

struct Fail {
    axf_status st;
};

#define AXF_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::axf::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
            throw ::axf::Fail{AXF_ERR_HIP};                                            \
        }                                                                              \
    } while (0)

#define AXF_REQUIRE(cond, code, msg)                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            ::axf::set_error(msg);                                                     \
            throw ::axf::Fail{code};                                                   \
        }                                                                              \
    } while (0)

// --------------------------------------------------------------- memory
// Device arenas are recycled through a small per-process cache so that
// creating and destroying plans in a loop does not pay hipMalloc/hipFree.
struct Arena {
    char *base = nullptr;
    size_t bytes = 0;
    size_t used = 0;
    int device = -1;
    template <class T>
    T *take(size_t count)
    {
        size_t off = (used + 255) & ~size_t(255);
        size_t need = count * sizeof(T);
        if (off + need > bytes) {
            set_error("internal: arena overflow");
            throw Fail{AXF_ERR_OUT_OF_MEMORY};
        }
        used = off + need;
        return reinterpret_cast<T *>(base + off);
    }
};
Arena arena_acquire(size_t bytes);   // throws on failure
void arena_release(Arena &a);        // returns the block to the cache

// Bytes that `take` calls will consume, for sizing an arena.
struct Sizer {
    size_t bytes = 0;
    template <class T>
    void add(size_t count)
    {
        bytes = ((bytes + 255) & ~size_t(255)) + count * sizeof(T);
    }
};

// Device-side view of a sorted point set.
struct SideView {
    const double *r, *z;
    const int32_t *perm, *off;
};

// ------------------------------------------------------------------ plan
// One point set (the sources, or the field points) sorted onto the common
// tree.  Box ids at a level are station-major: b = ir * 2^l + iz.
struct Side {
    int64_t n = 0;
    double *r = nullptr, *z = nullptr;      // sorted coordinates [n]
    double *rinv = nullptr;                 // 1 / r, sorted [n]
    int32_t *perm = nullptr;                // sorted position -> caller index
    int32_t *off = nullptr;                 // leaf offsets in Morton order [4^d + 1]
    int32_t *slot[AXF_MAX_DEPTH + 1] = {};  // [4^l]: box id -> compact slot, -1 if empty
    int32_t *box[AXF_MAX_DEPTH + 1] = {};   // [nocc]: compact slot -> box id
    int nocc[AXF_MAX_DEPTH + 1] = {};
    int4 *chunks = nullptr;                 // leaf work: (slot, first, count, box)
    int nchunks = 0;
    int max_leaf = 0;
    // S2L tiles of this side as targets: (station, z parity, first, count)
    int4 *tiles[AXF_MAX_DEPTH + 1] = {};
    int32_t *tile_slots[AXF_MAX_DEPTH + 1] = {};
    int ntiles[AXF_MAX_DEPTH + 1] = {};
    int s2l_groups[AXF_MAX_DEPTH + 1] = {};  // offset groups of the S2L pass at each level
};

// Shape of the tiled S2L: output slots of one (box, channel) are rows k
// whose even and odd columns are each split into blocks of LB (columns l0,
// l0 + 2, ...); LB is the smallest width whose slots fit in four waves, the
// block has one wave per 64 slots, and a tile holds TB = 2, 4 or 8 target
// boxes (the plan's tile width).
inline int s2l_slots(int M, int lb)
{
    int s = 0;
    for (int k = 0; k <= M; ++k) {
        const int ncol = M + 1 - k;
        s += ((ncol + 1) / 2 + lb - 1) / lb + (ncol / 2 + lb - 1) / lb;
    }
    return s;
}
inline int s2l_lb(int M) { return s2l_slots(M, 1) <= 256 ? 1 : 2; }   // 2 fits M <= 24
inline int s2l_waves(int M) { return (s2l_slots(M, s2l_lb(M)) + 63) / 64; }
// The bounding square (reading R5): side L = the larger extent (1 if both
// are zero), from the smallest z.  In r it starts on the axis when that side
// reaches the largest radius (koff = 0).  Else, when the smallest radius
// lies between L/4 and L (k = floor(4 r_min / L) in 1..3), on the multiple k
// of L'/4 with the smallest L' >= L for which k L'/4 + L' reaches the
// largest radius (L' = r_max / (1 + k/4), raised ulp by ulp until it does),
// provided k L'/4 is still not above the smallest radius: then the stations
// of every level sit at whole box units k 2^(l-2) from the axis grid and the
// levels share tables (koff = k).  Else at the smallest radius (koff = -1).
// Each operation is rounded on its own (no contraction): the oracle
// evaluates the same sequence.
inline void square_rule(double rmin, double rmax, double zmin, double zmax, double &rlo, double &zlo, double &L,
                        int &koff)
{
#pragma clang fp contract(off)
    const double ext = std::max(rmax - rmin, zmax - zmin);
    L = ext > 0.0 ? ext : 1.0;
    zlo = zmin;
    rlo = rmin;
    koff = -1;
    if (rmax <= L) {
        rlo = 0.0;
        koff = 0;
        return;
    }
    const double k = std::floor(rmin / (L * 0.25));
    if (k < 1.0 || k > 3.0) return;
    const double f = 1.0 + k * 0.25;
    double Ls = std::max(L, rmax / f);
    for (;;) {
        const double r0 = k * (Ls * 0.25);
        const double top = r0 + Ls;
        if (top >= rmax) break;
        Ls = std::nextafter(Ls, INFINITY);
    }
    const double r0 = k * (Ls * 0.25);
    if (r0 <= rmin) {
        L = Ls;
        rlo = r0;
        koff = (int)k;
    }
}

// Near field with G^(n) shared by the right-hand sides: up to this many
// modes (mode buckets up to 24); the class of a plan: 0 = one source per
// lane step (nrhs 1, or more modes), 1, 2, 3 = 2, 4, 8 lanes per target.
constexpr int kNearQMaxModes = 24;
inline int near_class(int nrhs, int nmb)
{
    if (nrhs < 2 || nmb > kNearQMaxModes) return 0;
    return nrhs <= 2 ? 1 : nrhs <= 4 ? 2 : 3;
}

// Tile widths the vector-unit S2L kernels are compiled for (boxes per
// tile), from params.flags (AXF_TILE_SHIFT; 0 there selects the matrix-core
// kernel); kDefaultTile is the batch kernels' width when none is chosen.
constexpr int kDefaultTile = 4;
inline bool s2l_tile_ok(int tb) { return tb == 2 || tb == 4 || tb == 8; }
constexpr int kTiles[3] = {2, 4, 8};
inline int tile_index(int tb) { return tb == 2 ? 0 : tb == 4 ? 1 : 2; }
// Matrix-core S2L: tiles of 8 boxes (16 real columns); the outputs of a
// (box, channel) in row tiles of 16 (rows of one column parity), at most 21
// for M <= 24, dealt to W <= 4 waves of TPW tiles each (4 <= TPW <= 7), the
// pair that leaves the fewest idle tiles (ties: more tiles per wave).
constexpr int kS2lMfmaBoxes = 8;
inline int s2l_row_tiles(int M)
{
    int r0 = 0, r1 = 0;
    for (int k = 0; k <= M; ++k) {
        r0 += (M + 2 - k) / 2;
        r1 += (M + 1 - k) / 2;
    }
    return (r0 + 15) / 16 + (r1 + 15) / 16;
}
inline void s2l_mfma_shape(int M, int &tpw, int &waves)
{
    const int nt = s2l_row_tiles(M);
    int best = 1 << 30;
    for (int t = 7; t >= 4; --t) {
        const int w = (nt + t - 1) / t;
        if (w > 4) continue;
        if (w * t - nt < best) {
            best = w * t - nt;
            tpw = t;
            waves = w;
        }
    }
}
// P2M work items per leaf: one per pair of channels (the pair shares the
// sources' offset powers).
__host__ __device__ inline int p2m_pairs(int C) { return (C + 1) / 2; }
// Window bound of the S2L lanes: M rounded up to a multiple of 4.
inline int s2l_window(int M) { return M <= 4 ? 4 : (M + 3) / 4 * 4; }
// Doubles past the last table: a lane reads its whole window, up to
// s2l_window + 2 s2l_lb - 1 entries past the start of the table's last row.
constexpr size_t kTablePad = 64;
// Offset groups of a level: the 18 offset units (pairs (dr, +-dz) of the
// interaction list) of a (tile, channel) are split over G blocks so that a
// level launches ~2048 waves.
inline int s2l_group_count(int ntiles, int C, int M, int waves_per_block)
{
    const int64_t waves = (int64_t)ntiles * C * waves_per_block;
    if (waves <= 0) return 1;
    int64_t g = (2048 + waves - 1) / waves;
    return (int)(g < 1 ? 1 : g > 9 ? 9 : g);
}

struct Level {
    int nb = 0;                // boxes per side, 2^l
    double h = 0;              // box width
    double2 *mom = nullptr;    // [max(nocc)][C][P] moments (z-factorial normalised)
    double2 *loc = nullptr;    // [max(nocc)][C][P] local coefficients
    double *tab = nullptr;     // [nb][12][n_modes][TS] S2L tables (x >= 0, outer >= inner)
    double tscale = 1.0;       // factor of the stored tables (2^(l-d) when levels share the finest's)
};

// Mode counts the near-field kernels are compiled for; a plan uses the
// smallest one >= n_modes and pads the strengths with zeros.
inline int mode_bucket(int nmodes)
{
    const int b[] = {4, 9, 12, 17, 24, 33, 48, 64};
    for (int v : b)
        if (nmodes <= v) return v;
    return 64;
}

struct Plan {
    int device = 0;
    axf_params p{};
    int N = 0, M = 0, P = 0, C = 0, TS = 0, d = 0, nrhs = 1, nmodes = 1;
    int nmb = 4, Cs = 4;        // mode bucket and padded channels per point in Sg
    int tb = kDefaultTile;      // S2L tile width (target boxes per tile)
    bool mfma = false;          // S2L on the matrix cores (tiles of kS2lMfmaBoxes)
    bool overlap = true;        // near field beside the downward pass (second stream)
    double rlo = 0, zlo = 0, L = 1, invL = 1;
    double rmax = 0;                     // largest ring radius of both sets
    int tab_smax[AXF_MAX_DEPTH + 1] = {};   // last radial station with tables, per level
    size_t tab_base[AXF_MAX_DEPTH + 1] = {};   // first geometry of each level in the table storage
    int koff = -1;                          // square origin in units of L/4 (>= 0: levels share tables)
    // shared tables: runs [first, last] of finest-level stations of the axis
    // grid (station v at v + 1/2 box units), stored one after the other
    std::vector<std::pair<int, int>> tab_runs;
    double chistar = 1e300;
    Side src, fld;
    Level lev[AXF_MAX_DEPTH + 1];
    double2 *Sg = nullptr;      // gathered strengths, point-major [max(ns, nf)][Cs]
    double2 *s2l_part = nullptr;  // partial S2L sums of the offset groups of one level
    double *gsum = nullptr;     // adjoint coordinate-gradient scratch
    double *tab_scratch = nullptr;
    Arena points, tree, expn, tilemem, tabmem;
    std::vector<double> geom_host;   // table geometries (4 doubles each), source of an async copy
    hipEvent_t tables_ready = nullptr;   // recorded after the tables on the table stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // near field beside the downward pass
    double *shift_coef = nullptr;        // M2M and L2L factors, [3][2][S][S], S = AXF_MAX_ORDER + 1
    std::vector<double> coef_host;       // their host copy, source of an async copy
    std::vector<int32_t> box_host;       // every level's occupied boxes of both sides (host copy)
    size_t box_host_off[2][AXF_MAX_DEPTH + 1] = {};
    std::vector<char> tile_host;         // host image of the S2L tile arena, source of an async copy
    int64_t near_pairs = 0, s2l_pairs = 0, s2l_units = 0;   // S2L: box pairs, (box, offset unit) pairs
    bool census_done = false;
    double census_near[4] = {}, census_direct[4] = {};
    size_t device_bytes = 0;
    bool external = false;      // buffers live in a caller workspace (axf_plan_set_workspace)
    // phase timing (HIP events on the evaluation stream)
    bool timing = false;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare_events;
};

// Calls f(v, field) for every device pointer a plan holds into its arenas:
// v is its value as a char pointer (a reference, so that f may rebase it)
// and field the address of the member itself.  Relocating a plan into a
// caller's workspace rebases exactly these; it also checks that no other
// word of the plan holds an address inside an arena, so a pointer added to
// the plan without being listed here is reported instead of left dangling.
template <class T, class F>
inline void visit_ptr(T *&p, F &f)
{
    char *c = reinterpret_cast<char *>(p);
    f(c, (const void *)&p);
    p = reinterpret_cast<T *>(c);
}
template <class F>
void plan_device_ptrs(Plan &pl, F &&f)
{
    for (Side *s : {&pl.src, &pl.fld}) {
        visit_ptr(s->r, f);
        visit_ptr(s->z, f);
        visit_ptr(s->rinv, f);
        visit_ptr(s->perm, f);
        visit_ptr(s->off, f);
        visit_ptr(s->chunks, f);
        for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
            visit_ptr(s->slot[l], f);
            visit_ptr(s->box[l], f);
            visit_ptr(s->tiles[l], f);
            visit_ptr(s->tile_slots[l], f);
        }
    }
    for (int l = 0; l <= AXF_MAX_DEPTH; ++l) {
        visit_ptr(pl.lev[l].mom, f);
        visit_ptr(pl.lev[l].loc, f);
        visit_ptr(pl.lev[l].tab, f);
    }
    visit_ptr(pl.Sg, f);
    visit_ptr(pl.s2l_part, f);
    visit_ptr(pl.gsum, f);
    visit_ptr(pl.tab_scratch, f);
    visit_ptr(pl.shift_coef, f);
}

// Records HIP events around a pass when the plan's timing is enabled.
struct PhaseTimer {
    Plan &pl;
    hipStream_t st;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    PhaseTimer(Plan &p, hipStream_t s, int ph);
    ~PhaseTimer();
};

// -------------------------------------------------------------- launchers
hipEvent_t event_get(Plan &pl);
// tree (axf_tree.hip)
// `after_depth` runs once the square and the depth are known (before the
// sort), so that work depending only on them can start.
void build_tree(Plan &pl, const double *rs, const double *zs, const double *rf, const double *zf,
                hipStream_t st, const std::function<void()> &after_depth);
void build_tiles(Plan &pl, hipStream_t st);
// tables (axf_tables.hip)
void build_tables(Plan &pl, hipStream_t st);
size_t table_scratch_doubles(size_t ngeom, int M, int nmodes);
// shift factors of the M2M and L2L passes (axf_fmm.hip)
constexpr int kCoefS = AXF_MAX_ORDER + 1;
void shift_coef_host(int M, std::vector<double> &out);
// FMM passes (axf_fmm.hip).  `src` carries the strengths (gathered into
// pl.Sg), `tgt` receives the potential.  mode: 0 = potential only,
// 1 = potential and gradient arrays, 2 = potential and the coordinate
// gradient contraction of the adjoint (gr, gz accumulate
// Re(Sdot * conj(grad psi))).
struct EvalOut {
    double *phi = nullptr;       // complex [nrhs][nmodes][tgt.n], caller order
    double *dr = nullptr;        // gradient outputs (mode 1)
    double *dz = nullptr;
    double *daz = nullptr;       // mode 1: (1/r) dPhi/dtheta = i n Phi^(n) / r
    const double *Sdot = nullptr;  // mode 2: caller-order strengths at the targets
    double *gr = nullptr, *gz = nullptr;
    int mode = 0;
    bool fused = false;          // mode 0: near field and local evaluation in one kernel
};
void run_fmm(Plan &pl, const Side &src, const Side &tgt, const double *S, const EvalOut &out,
             hipStream_t st);
void run_direct(Plan &pl, const Side &src, const Side &tgt, const double *S, const EvalOut &out,
                hipStream_t st);

// ----------------------------------------------------------------- batches
// Device descriptor of one problem of a batch: the pointers and scalars of
// its plan that the persistent batch kernels read.
struct ProbDev {
    int d = 2, nrhs = 1, C = 1, Cs = 4;
    double rlo = 0, zlo = 0, invL = 1;
    int64_t ns = 0, nf = 0;
    SideView sv{}, tv{};
    const double *srinv = nullptr;
    const double2 *S = nullptr;     // caller strengths [nrhs][nmodes][ns]
    double2 *phi = nullptr;         // caller potential [nrhs][nmodes][nf]
    double2 *Sg = nullptr;
    const int32_t *sbox[AXF_MAX_DEPTH + 1] = {}, *sslot[AXF_MAX_DEPTH + 1] = {};
    const int32_t *tbox[AXF_MAX_DEPTH + 1] = {}, *tslot[AXF_MAX_DEPTH + 1] = {};
    const int4 *tiles[AXF_MAX_DEPTH + 1] = {};
    const int32_t *tile_slots[AXF_MAX_DEPTH + 1] = {};
    double2 *mom[AXF_MAX_DEPTH + 1] = {}, *loc[AXF_MAX_DEPTH + 1] = {};
    const double *tab[AXF_MAX_DEPTH + 1] = {};
    double tscale[AXF_MAX_DEPTH + 1] = {};
    const int4 *chunks = nullptr;
    const double *shift_coef = nullptr;
};

// Merged work queues of a batch: one (problem, item) list per pass.
// m2m[t] holds the step from level d-t+1 to d-t of each problem (so the
// problems' different depths line up), l2l[l] the target boxes x channels
// and s2l[l] the tiles x channels of level l; p2m holds leaves x channels.
struct BatchQueues {
    const ProbDev *probs = nullptr;
    int2 *gather = nullptr, *p2m = nullptr, *leaf = nullptr;
    int ngather = 0, np2m = 0, nleaf = 0;
    // the leaf chunks again by near-field kernel: [0] one source per lane
    // step, [1..3] G^(n) shared by 2, 4, 8 right-hand-side lanes
    int2 *leafq[4] = {};
    int nleafq[4] = {};
    int2 *m2m[AXF_MAX_DEPTH + 1] = {}, *l2l[AXF_MAX_DEPTH + 1] = {};
    int nm2m[AXF_MAX_DEPTH + 1] = {}, nl2l[AXF_MAX_DEPTH + 1] = {};
    // S2L tiles of level l of the problems whose tile width is kTiles[t]
    int2 *s2l[AXF_MAX_DEPTH + 1][3] = {};
    int ns2l[AXF_MAX_DEPTH + 1][3] = {};
    int M = 0, nmodes = 1, nmb = 4, TS = 1, maxd = 2;
    double chistar = 1e300;
};
void fill_probdev(const Plan &pl, const double *S, double *phi, ProbDev &pd);
// Pair census of the near field (or, sampled, of the direct sum) with the
// field points as targets: [pairs, backward pairs, AGM iterations, steps].
void pair_census(Plan &pl, bool direct, double out[4], hipStream_t st);
// A second stream and two events with which run_batch runs the near field
// beside the downward pass.
struct BatchSide {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
void run_batch(const BatchQueues &bq, hipStream_t st, const BatchSide *side);

}  // namespace axf

// The opaque plan handle of the C ABI.
struct axf_plan {
    axf::Plan pl;
};

// axf_fmm.hip -- FMM passes of Algorithm 1 on gfx950, plus the direct sum.
//
// Scaled conventions (box units, h = box width at the level):
//   moments   s_ij = sum_q S_q (dr_q/h)^i (dz_q/h)^j / j!        (eq. analysis:moments)
//   locals    Phi(r, z) = sum_kl L_kl (dr/h)^k (dz/h)^l            (eq. analysis:local)
//   S2L       L_kl += ((-1)^l / l!) sum_ij sigma(j+l) T_{k,i,j+l} s_ij      outward
//             L_kl += ((-1)^l / l!) sum_ij sigma(j+l) T_{i,k,j+l} s_ij      inward
//             with T the table of the inner station (c! gbar h^(a+b+c)),
//             sigma(c) = (-1)^c for z_target >= z_source (forward) else 1.
//   This is eq. analysis:s2l with the FO/BO/FI/BI reuse of section 2.2: one
//   table at r >= r1, x >= 0 serves all four orientations.
#include <algorithm>

#include <mutex>

#include "axf_device.hpp"

#include "axf_internal.hpp"

namespace axf {

namespace {

constexpr int kMaxRhs = AXF_MAX_RHS;


// ---------------------------------------------------------------- gather
// Strengths into tree order, point-major with Cs = nmb * nrhs channels per
// point (channel n * nrhs + q; modes nmodes..nmb-1 are zero padding).
__global__ void k_gather(const double2 *__restrict__ S, const int32_t *__restrict__ perm, int64_t n,
                         int nmodes, int nrhs, int Cs, double2 *__restrict__ Sg)
{
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * Cs) return;
    int64_t p = e / Cs;
    int c = (int)(e - p * Cs);
    int nn = c / nrhs, q = c - nn * nrhs;
    Sg[e] = nn < nmodes ? S[((int64_t)q * nmodes + nn) * n + perm[p]] : make_double2(0.0, 0.0);
}

// ------------------------------------------------------------------- P2M
// Leaf moments (eq. analysis:moments in box units): one block per (leaf,
// pair of channels), s_ij = sum_s S_s (dr_s)^i (dz_s)^j / j!, offsets in leaf
// units; the two channels share the staged powers of the offsets.
constexpr int kP2MChunk = 64;
__device__ __forceinline__ void p2m_body(int M, int C, int Cs, int depth, double rlo, double zlo, double invh,
                                         SideView sv, const int32_t *__restrict__ boxes,
                                         const double2 *__restrict__ Sg, double2 *__restrict__ mom, int item)
{
    __shared__ double pr[kP2MChunk][AXF_MAX_ORDER + 1];
    __shared__ double pz[kP2MChunk][AXF_MAX_ORDER + 1];
    __shared__ double2 ss[2][kP2MChunk];
    const int P = (M + 1) * (M + 2) / 2;
    const int npair = p2m_pairs(C);
    const int k = item / npair, c = 2 * (item - (item / npair) * npair);
    const bool two = c + 1 < C;     // uniform over the block
    const int b = boxes[k];
    const int nb = 1 << depth;
    const int ir = b / nb, iz = b - ir * nb;
    const uint32_t m = morton((uint32_t)ir, (uint32_t)iz);
    const int first = sv.off[m], last = sv.off[m + 1];
    const double cr = ir + 0.5, cz = iz + 0.5;
    // this thread's outputs: p = tid and tid + 256
    int oi[2], oj[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int p = threadIdx.x + u * 256, i = 0;
        if (p < P)
            while (p >= M + 1 - i) {
                p -= M + 1 - i;
                ++i;
            }
        oi[u] = i;
        oj[u] = p;
    }
    double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    double2 acc1[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    for (int s0 = first; s0 < last; s0 += kP2MChunk) {
        const int ns = min(kP2MChunk, last - s0);
        __syncthreads();
        if (threadIdx.x < ns) {
            const int e = threadIdx.x;
            const double dr = (sv.r[s0 + e] - rlo) * invh - cr;
            const double dz = (sv.z[s0 + e] - zlo) * invh - cz;
            double a = 1.0, q = 1.0;
            for (int i = 0; i <= M; ++i) {
                pr[e][i] = a;
                pz[e][i] = q;
                a *= dr;
                q *= dz / (i + 1.0);
            }
            ss[0][e] = Sg[(int64_t)(s0 + e) * Cs + c];
            ss[1][e] = two ? Sg[(int64_t)(s0 + e) * Cs + c + 1] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (threadIdx.x + u * 256 >= P) continue;
            const int i = oi[u], j = oj[u];
            double2 a = acc[u], b = acc1[u];
            if (two) {
                for (int s = 0; s < ns; ++s) {
                    const double w = pr[s][i] * pz[s][j];
                    a.x = fma(w, ss[0][s].x, a.x);
                    a.y = fma(w, ss[0][s].y, a.y);
                    b.x = fma(w, ss[1][s].x, b.x);
                    b.y = fma(w, ss[1][s].y, b.y);
                }
            } else {
                for (int s = 0; s < ns; ++s) {
                    const double w = pr[s][i] * pz[s][j];
                    a.x = fma(w, ss[0][s].x, a.x);
                    a.y = fma(w, ss[0][s].y, a.y);
                }
            }
            acc[u] = a;
            acc1[u] = b;
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int p = threadIdx.x + u * 256;
        if (p < P) {
            mom[((int64_t)k * C + c) * P + p] = acc[u];
            if (two) mom[((int64_t)k * C + c + 1) * P + p] = acc1[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_p2m(int M, int C, int Cs, int depth, double rlo, double zlo,
                                            double invh, SideView sv, const int32_t *__restrict__ boxes,
                                            const double2 *__restrict__ Sg, double2 *__restrict__ mom)
{
    p2m_body(M, C, Cs, depth, rlo, zlo, invh, sv, boxes, Sg, mom, blockIdx.x);
}

// Decode a packed-triangle index p into (i, j), i + j <= M, i-major.
__device__ __forceinline__ void tri_decode(int M, int p, int &i, int &j)
{
    int r = 0;
    while (p >= M + 1 - r) {
        p -= M + 1 - r;
        ++r;
    }
    i = r;
    j = p;
}

// ------------------------------------------------------------------- M2M
// Upward shift (eq. analysis:shift) of the four children into the parent,
// in parent units with child offsets dr, dz = +-1/4:
//   s_ij = sum_children sum_a R[i][a] sum_b Z[j][b] s'_ab,
//   R[i][a] = C(i,a) dr^(i-a) 2^-a,  Z[j][b] = dz^(j-b) / (j-b)! 2^-b.
// The double sum is applied separably: first over b for each child, summed
// over the two children of each r offset, then over a.  One block per
// (parent box, channel); the children's moments are staged in LDS.
__device__ __forceinline__ void m2m_body(int M, int C, int level, const int32_t *__restrict__ pboxes,
                                         const int32_t *__restrict__ cslot, const double2 *__restrict__ cmom,
                                         double2 *__restrict__ pmom, const double *__restrict__ coef, int item)
{
    constexpr int PM = (AXF_MAX_ORDER + 1) * (AXF_MAX_ORDER + 2) / 2;
    __shared__ double cfr[2][AXF_MAX_ORDER + 1][AXF_MAX_ORDER + 1];
    __shared__ double cfz[2][AXF_MAX_ORDER + 1][AXF_MAX_ORDER + 1];
    __shared__ double2 sm[4][PM];
    __shared__ double2 t[2][PM];
    const int P = (M + 1) * (M + 2) / 2;
    const int k = item / C, c = item - (item / C) * C;
    const int b = pboxes[k];
    const int nb = 1 << level;
    const int ir = b / nb, iz = b - ir * nb;
    for (int e = threadIdx.x; e < 2 * (M + 1) * (M + 1); e += blockDim.x) {
        const int sg = e / ((M + 1) * (M + 1)), rem = e - sg * (M + 1) * (M + 1);
        const int i = rem / (M + 1), a = rem - i * (M + 1);
        cfr[sg][i][a] = coef[(size_t)(2 + sg) * kCoefS * kCoefS + i * kCoefS + a];
        cfz[sg][i][a] = coef[(size_t)(4 + sg) * kCoefS * kCoefS + i * kCoefS + a];
    }
    const int cnb = nb * 2;
    for (int e = threadIdx.x; e < 4 * P; e += blockDim.x) {
        const int ch = e / P, p = e - ch * P;
        const int cs = cslot[(2 * ir + (ch >> 1)) * cnb + (2 * iz + (ch & 1))];
        sm[ch][p] = cs >= 0 ? cmom[((int64_t)cs * C + c) * P + p] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // z pass: t[sr][a][j] = sum_sz sum_{b <= j} Z_sz[j][b] s'_(sr,sz)[a][b],  a + j <= M
    for (int e = threadIdx.x; e < 2 * P; e += blockDim.x) {
        const int sr = e / P, p = e - sr * P;
        int a, j;
        tri_decode(M, p, a, j);
        const int row = p - j;          // tri_index(M, a, 0)
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int sz = 0; sz < 2; ++sz) {
            const double2 *src = sm[sr * 2 + sz] + row;
            for (int q = 0; q <= j; ++q) {
                const double w = cfz[sz][j][q];
                v.x = fma(w, src[q].x, v.x);
                v.y = fma(w, src[q].y, v.y);
            }
        }
        t[sr][p] = v;
    }
    __syncthreads();
    // r pass: s[i][j] = sum_sr sum_{a <= i} R_sr[i][a] t[sr][a][j]
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        int i, j;
        tri_decode(M, p, i, j);
        double2 v = make_double2(0.0, 0.0);
        int row = 0;                    // tri_index(M, a, 0)
        for (int a = 0; a <= i; ++a) {
#pragma unroll
            for (int sr = 0; sr < 2; ++sr) {
                const double w = cfr[sr][i][a];
                const double2 x = t[sr][row + j];
                v.x = fma(w, x.x, v.x);
                v.y = fma(w, x.y, v.y);
            }
            row += M + 1 - a;
        }
        pmom[((int64_t)k * C + c) * P + p] = v;
    }
}

__global__ __launch_bounds__(256) void k_m2m(int M, int C, int level, const int32_t *__restrict__ pboxes,
                                            const int32_t *__restrict__ cslot,
                                            const double2 *__restrict__ cmom, double2 *__restrict__ pmom,
                                            const double *__restrict__ coef)
{
    m2m_body(M, C, level, pboxes, cslot, cmom, pmom, coef, blockIdx.x);
}

// ------------------------------------------------------------------- L2L
// Local shift (eq. analysis:l2l) from the parent into each occupied target
// box of a level, child offsets dr, dz = +-1/4 parent units, child units half
// the parent's:  L'_kl = sum_a sum_q F_r[k][a] F_z[l][q] L_(k+a, l+q),
// F[i][q] = C(i+q, q) d^q 2^-i.  Separable: over a, then over q.  Boxes
// without a parent expansion (level 2) start from zero.  One block per
// (target box, channel); the result initialises the box's locals, which the
// S2L pass of the same level then accumulates into.
__device__ __forceinline__ void l2l_body(int M, int C, int level, const int32_t *__restrict__ tbox,
                                         const int32_t *__restrict__ tslot_parent, const double2 *__restrict__ ploc,
                                         double2 *__restrict__ loc, const double *__restrict__ coef, int item)
{
    constexpr int PM = (AXF_MAX_ORDER + 1) * (AXF_MAX_ORDER + 2) / 2;
    __shared__ double fc[2][AXF_MAX_ORDER + 1][AXF_MAX_ORDER + 1];
    __shared__ double2 pl[PM];
    __shared__ double2 u[PM];
    const int P = (M + 1) * (M + 2) / 2;
    const int k = item / C, c = item - (item / C) * C;
    double2 *out = loc + ((int64_t)k * C + c) * P;
    const int nb = 1 << level;
    const int bid = tbox[k];
    const int ir = bid / nb, iz = bid - ir * nb;
    const int pslot = level > 2 ? tslot_parent[(ir >> 1) * (nb >> 1) + (iz >> 1)] : -1;
    if (pslot < 0) {                    // uniform over the block
        for (int p = threadIdx.x; p < P; p += blockDim.x) out[p] = make_double2(0.0, 0.0);
        return;
    }
    for (int e = threadIdx.x; e < 2 * (M + 1) * (M + 1); e += blockDim.x) {
        const int sg = e / ((M + 1) * (M + 1)), rem = e - sg * (M + 1) * (M + 1);
        const int i = rem / (M + 1), q = rem - i * (M + 1);
        fc[sg][i][q] = coef[(size_t)sg * kCoefS * kCoefS + i * kCoefS + q];
    }
    const double2 *src = ploc + ((int64_t)pslot * C + c) * P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) pl[p] = src[p];
    __syncthreads();
    const int sr = ir & 1, sz = iz & 1;
    // r pass: u[kk][l] = sum_a F_r[kk][a] L[kk+a][l],  kk + a + l <= M
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        int kk, l;
        tri_decode(M, p, kk, l);
        double2 v = make_double2(0.0, 0.0);
        int row = p - l;                // tri_index(M, kk, 0)
        for (int a = 0; kk + a + l <= M; ++a) {
            const double w = fc[sr][kk][a];
            const double2 x = pl[row + l];
            v.x = fma(w, x.x, v.x);
            v.y = fma(w, x.y, v.y);
            row += M + 1 - (kk + a);
        }
        u[p] = v;
    }
    __syncthreads();
    // z pass: L'[kk][l] = sum_q F_z[l][q] u[kk][l+q]
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        int kk, l;
        tri_decode(M, p, kk, l);
        double2 v = make_double2(0.0, 0.0);
        for (int q = 0; kk + l + q <= M; ++q) {
            const double w = fc[sz][l][q];
            const double2 x = u[p + q];
            v.x = fma(w, x.x, v.x);
            v.y = fma(w, x.y, v.y);
        }
        out[p] = v;
    }
}

__global__ __launch_bounds__(256) void k_l2l(int M, int C, int level, const int32_t *__restrict__ tbox,
                                            const int32_t *__restrict__ tslot_parent,
                                            const double2 *__restrict__ ploc, double2 *__restrict__ loc,
                                            const double *__restrict__ coef)
{
    l2l_body(M, C, level, tbox, tslot_parent, ploc, loc, coef, blockIdx.x);
}

// ------------------------------------------------------- S2L, tiled form
// One offset pair's contraction for one lane: rows i = 0..M of the staged
// combined moments (the lane's column parity) against the table row (k, i)
// of an outward offset or (i, k) of an inward one, from the lane's first
// column l0 (one row advance per i); the lane's columns are l0 + 2u.  With
// FIX the order is the compile-time MW and every loop is unrolled: each row
// loads exactly its window (M - i + 2LB - 1 entries) with no branches.
// Otherwise the window is read whole (MW + 2LB - 1 entries, M <= MW): entries
// past c = 2M - k - i only meet columns l > M - k, which are never written,
// or j > M - i, which is skipped, and the table allocation is padded past its
// last row.
template <int LB, int TB, int MW, bool FIX>
__device__ __forceinline__ void s2l_row(int M, int i, const double *&row, const double2 *&mrow, int k, bool outward,
                                        double2 (&acc)[LB][TB])
{
    constexpr int NW = MW + 2 * LB - 1;
    const int jn = M - i;
    double w[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q)
        if (!FIX || q < jn + 2 * LB - 1) w[q] = row[q];
#pragma unroll
    for (int j = 0; j <= MW; ++j) {
        if (j <= jn) {
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const double2 sv = mrow[j * 2 * TB + b];
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    acc[u][b].x = fma(w[j + 2 * u], sv.x, acc[u][b].x);
                    acc[u][b].y = fma(w[j + 2 * u], sv.y, acc[u][b].y);
                }
            }
        }
    }
    mrow += (jn + 1) * 2 * TB;
    // next row: (k, i + 1) is 2M + 1 - k - i entries on, (i + 1, k) one
    // a-slab of the table less the rows b < k of slab i and b >= k of slab i + 1
    row += outward ? 2 * M + 1 - k - i : (M + 1) * (2 * M + 1) - (M * (M + 1)) / 2 - k - (M + 1) * i;
}

template <int LB, int TB, int MW, bool FIX>
__device__ __forceinline__ void s2l_rows(int M, const double *__restrict__ T, int k, int l0, bool outward,
                                         const double2 *ms, double2 (&acc)[LB][TB])
{
    const double *row = T + (outward ? table_row(M, k, 0) : table_row(M, 0, k)) + l0;
    const double2 *mrow = ms + (l0 & 1) * TB;
    if constexpr (FIX) {
#pragma unroll
        for (int i = 0; i <= MW; ++i) s2l_row<LB, TB, MW, true>(MW, i, row, mrow, k, outward, acc);
    } else {
#pragma unroll 1
        for (int i = 0; i <= M; ++i) s2l_row<LB, TB, MW, false>(M, i, row, mrow, k, outward, acc);
    }
}

// One block of W waves per (tile, channel).  A tile is up to TB occupied
// target boxes of one radial station with the same z parity, so that every
// box of the tile has the same interaction-list offsets (dr, dz) and
// therefore, for each offset, the same operator: one table, one
// orientation.  The offsets (dr, dz) and (dr, -dz) share the table of |dz|
// and differ only by the sign (-1)^(j+l) of the forward one (z_target >
// z_source), so they are taken together: with M+ the moments of the source
// above and M- those of the source below, the even columns l see A = M+ +
// (-1)^j M- and the odd ones B = M+ - (-1)^j M-, one contraction for both
// (18 such units per tile instead of 27 offsets).  Each lane owns the outputs
// (k, l0 + 2u), u < LB, of one column parity for all TB boxes (the W waves
// split the output rows between them, so the table is not read twice); for
// each input moment (i, j) the table values T[k][i][j+l] of the lane's
// outputs form a window that slides by one entry per j (Hankel structure),
// so each step loads one table value and does 2 LB TB FMAs on combined
// moments broadcast from LDS.  The result, times (-1)^l / l!, is added to the
// locals that the L2L pass initialised.
// Compiled S2L shapes: (LB, MW, FIX) with MW = M rounded up to a multiple
// of 4, the window bound, LB from the slot rule, and FIX = (M == MW): the
// fully unrolled rows of a compile-time order.
#define AXF_S2L_SHAPES(Mv, F)                                            \
    do {                                                                 \
        const int mw_ = s2l_window(Mv);                                  \
        if (s2l_lb(Mv) == 2) {                                           \
            if ((Mv) == 24) F(2, 24, true);                              \
            else F(2, 24, false);                                        \
        } else if ((Mv) == mw_) {                                        \
            if (mw_ == 4) F(1, 4, true);                                 \
            else if (mw_ == 8) F(1, 8, true);                            \
            else if (mw_ == 12) F(1, 12, true);                          \
            else if (mw_ == 16) F(1, 16, true);                          \
            else F(1, 20, true);                                         \
        } else {                                                         \
            if (mw_ == 4) F(1, 4, false);                                \
            else if (mw_ == 8) F(1, 8, false);                           \
            else if (mw_ == 12) F(1, 12, false);                         \
            else if (mw_ == 16) F(1, 16, false);                         \
            else if (mw_ == 20) F(1, 20, false);                         \
            else F(1, 24, false);                                        \
        }                                                                \
    } while (0)

template <int LB, int TB, int MW, bool FIX>
__device__ __forceinline__ void s2l_tile_body(int M, int nmodes, int nrhs, int level, int TS,
                                                 const int4 *__restrict__ tiles,      // station, parity, first, count
                                                 const int32_t *__restrict__ tslots,  // target slots of the tiles
                                                 const int32_t *__restrict__ tbox,    // slot -> box id (targets)
                                                 const int32_t *__restrict__ sslot,
                                                 const double2 *__restrict__ mom,
                                                 const double *__restrict__ tab,
                                                 double2 *__restrict__ loc, int item, int G,
                                                 double2 *__restrict__ part, int nocc, double tscale)
{
    extern __shared__ double2 ms[];          // [P][2][TB] combined moments A, B; boxes interleaved
    __shared__ double invfact[AXF_MAX_ORDER + 1];
    __shared__ double jsign[(AXF_MAX_ORDER + 1) * (AXF_MAX_ORDER + 2) / 2];   // (-1)^j of moment p = (i, j)
    const int P = (M + 1) * (M + 2) / 2;
    const int C = nmodes * nrhs;
    const int ti = item / (C * G), rem = item - ti * (C * G);
    const int c = rem / G, g = rem - (rem / G) * G;    // channel, offset group
    const int n = c / nrhs;
    const int4 tl = tiles[ti];
    const int station = tl.x, nbx = tl.w;
    const int nb = 1 << level;
    const int tid = threadIdx.x, nthr = blockDim.x;

    if (tid <= M) {
        double f = 1.0;
        for (int t = 2; t <= tid; ++t) f *= t;
        invfact[tid] = 1.0 / f;
    }
    for (int p = tid; p < P; p += nthr) {
        int i = 0, q = p;                       // q = j of the moment (i, j)
        while (q >= M + 1 - i) {
            q -= M + 1 - i;
            ++i;
        }
        jsign[p] = (q & 1) ? -1.0 : 1.0;
    }
    // this lane's outputs: row k, columns l0 + 2u (u < LB) of one parity;
    // per row the even columns come first, then the odd ones
    int k = 0, l0 = 0, acc_lane = tid;
    bool live = false;
    for (int kk = 0; kk <= M; ++kk) {
        const int ncol = M + 1 - kk;
        const int ne = ((ncol + 1) / 2 + LB - 1) / LB, no = (ncol / 2 + LB - 1) / LB;
        if (acc_lane < ne + no) {
            k = kk;
            l0 = acc_lane < ne ? 2 * LB * acc_lane : 1 + 2 * LB * (acc_lane - ne);
            live = true;
            break;
        }
        acc_lane -= ne + no;
    }
    int zb[TB], sl[TB];
#pragma unroll
    for (int b = 0; b < TB; ++b) {
        sl[b] = b < nbx ? tslots[tl.z + b] : -1;
        int bid = sl[b] >= 0 ? tbox[sl[b]] : 0;
        zb[b] = bid - (bid / nb) * nb;
    }
    double2 acc[LB][TB];
#pragma unroll
    for (int u = 0; u < LB; ++u)
#pragma unroll
        for (int b = 0; b < TB; ++b) acc[u][b] = make_double2(0.0, 0.0);

    const int par = tl.y;                       // z parity of the tile
    const int dr0 = -2 - (station & 1), dz0 = -2 - par;
    const double *tab_n = tab + (size_t)n * TS;
    int oc = 0;                                 // index of the unit in the interaction list
    for (int dr = dr0; dr < dr0 + 6; ++dr) {
        const int jr = station + dr;
        const bool near_r = dr >= -1 && dr <= 1;
        for (int adz = 0; adz <= 3; ++adz) {
            // the unit's offsets dz = +adz (source above the target) and
            // dz = -adz (below: forward), each if it is in the interaction
            // list (children of the parent's neighbours, not adjacent)
            const bool hasp = adz > 0 && adz <= dz0 + 5 && !(near_r && adz <= 1);
            const bool hasm = -adz >= dz0 && !(near_r && adz <= 1);
            if (!hasp && !hasm) continue;
            if (oc++ % G != g || jr < 0 || jr >= nb) continue;   // another group's unit
            int sp[TB], sm[TB];
            bool any = false;
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const int jp = zb[b] + adz, jm = zb[b] - adz;
                sp[b] = (hasp && sl[b] >= 0 && jp < nb) ? sslot[jr * nb + jp] : -1;
                sm[b] = (hasm && sl[b] >= 0 && jm >= 0) ? sslot[jr * nb + jm] : -1;
                any |= sp[b] >= 0 || sm[b] >= 0;
            }
            if (!any) continue;
            const bool outward = dr <= 0;               // target radius >= source radius
            const int inner = outward ? jr : station;
            const int adr = outward ? -dr : dr;
            const double *T = tab_n + ((size_t)inner * 12 + geom_slot(adr, adz)) * nmodes * (size_t)TS;
            __syncthreads();
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const double2 *mp = sp[b] >= 0 ? mom + ((int64_t)sp[b] * C + c) * P : nullptr;
                const double2 *mm = sm[b] >= 0 ? mom + ((int64_t)sm[b] * C + c) * P : nullptr;
                for (int p = tid; p < P; p += nthr) {
                    double2 vp = make_double2(0.0, 0.0), vm = make_double2(0.0, 0.0);
                    if (mp) vp = mp[p];
                    if (mm) {
                        const double2 v = mm[p];
                        const double sg = jsign[p];
                        vm = make_double2(sg * v.x, sg * v.y);
                    }
                    ms[(p * 2) * TB + b] = make_double2(vp.x + vm.x, vp.y + vm.y);
                    ms[(p * 2 + 1) * TB + b] = make_double2(vp.x - vm.x, vp.y - vm.y);
                }
            }
            __syncthreads();
            if (live) s2l_rows<LB, TB, MW, FIX>(FIX ? MW : M, T, k, l0, outward, ms, acc);
        }
    }
    __syncthreads();                            // invfact is visible even when no offset ran
    // (-1)^l / l! * acc: added to the locals, or this group's partial sums
    // (each output has exactly one owner in a block)
#pragma unroll
    for (int b = 0; b < TB; ++b) {
        if (!live || sl[b] < 0) continue;
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int ll = l0 + 2 * u;
            if (ll > M - k) continue;
            const double f = ((ll & 1) ? -tscale : tscale) * invfact[ll];
            const int64_t e = ((int64_t)sl[b] * C + c) * P + tri_index(M, k, ll);
            if (part) {
                part[(int64_t)g * nocc * C * P + e] = make_double2(f * acc[u][b].x, f * acc[u][b].y);
            } else {
                double2 v = loc[e];
                v.x = fma(f, acc[u][b].x, v.x);
                v.y = fma(f, acc[u][b].y, v.y);
                loc[e] = v;
            }
        }
    }
}

// ------------------------------------------------------- S2L, matrix cores
// The units of the tiled form contracted on the FP64 matrix cores
// (v_mfma_f64_16x16x4): for one (tile of up to 8 boxes, channel) and one
// unit, Out[(k, l)][col] += sum over (i, j) of T[k][i][j + l] X[(i, j)][col]
// (T[i][k][j + l] for an inward unit), the 16 columns being the real and
// imaginary parts of the 8 boxes' combined moments (A for even l, B for odd
// l).  Output rows are split by the parity of l, k-major, in tiles of 16;
// wave w keeps the row tiles w, w + 4, ... as 16 x 16 blocks in registers
// through every unit.  A k-step takes 4 consecutive packed moments (i, j):
// each lane gathers its operand T entry of every row tile (16 rows x 4
// columns of a Hankel block: a few cache lines) and its box's two moments
// straight from memory, one step ahead of the matrix cores, and forms the
// combined moments in registers; no LDS staging, no barriers.  Padded rows
// read row (0, 0), padded columns column (M, 0) (valid table entries) and
// meet zero moments or are not written.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int TPW, int NB>
__device__ __forceinline__ void s2l_mfma_body(int M, int nmodes, int nrhs, int level,
                                              const int4 *__restrict__ tiles, const int32_t *__restrict__ tslots,
                                              const int32_t *__restrict__ tbox, const int32_t *__restrict__ sslot,
                                              const double2 *__restrict__ mom, const double *__restrict__ tab,
                                              double2 *__restrict__ loc, int item, int G, double2 *__restrict__ part,
                                              int nocc, double tscale, int TS, int W)
{
    constexpr int TB = kS2lMfmaBoxes * NB;   // NB column tiles of 8 boxes
    __shared__ double invfact[AXF_MAX_ORDER + 1];
    // the block's units: table offset, orientation, source slots per box
    __shared__ int64_t u_toff[18];
    __shared__ int u_out[18];
    __shared__ int u_src[18][2][TB];
    __shared__ int s_nunits;
    const int P = (M + 1) * (M + 2) / 2;
    const int C = nmodes * nrhs;
    // work item: (tile, channel, offset group, row group w of W); the W
    // one-wave blocks of a (tile, channel, group) are neighbours
    const int w = item % W;
    item /= W;
    const int ti = item / (C * G), rem = item - ti * (C * G);
    const int c = rem / G, g = rem - (rem / G) * G;
    const int n = c / nrhs;
    const int4 tl = tiles[ti];
    const int station = tl.x, nbx = tl.w;
    const int nb = 1 << level;
    const int tid = threadIdx.x, lane = tid;

    if (tid <= M) {
        double f = 1.0;
        for (int t = 2; t <= tid; ++t) f *= t;
        invfact[tid] = 1.0 / f;
    }
    // unit list (thread b < TB resolves the sources of box b; thread 0 also
    // the tables), in the order of the interaction list, this group's share
    if (tid < TB) {
        const int b = tid;
        const int sl = b < nbx ? tslots[tl.z + b] : -1;
        const int bid = sl >= 0 ? tbox[sl] : 0;
        const int zb = bid - (bid / nb) * nb;
        // the box's own z parity (a tile may hold both): which of the two
        // offsets of a unit exist differs, the list of units does not
        const int dr0 = -2 - (station & 1), dz0 = -2 - (zb & 1);
        int oc = 0, nu = 0;
        for (int dr = dr0; dr < dr0 + 6; ++dr) {
            const int jr = station + dr;
            const bool near_r = dr >= -1 && dr <= 1;
            for (int adz = 0; adz <= 3; ++adz) {
                const bool hasp = adz > 0 && adz <= dz0 + 5 && !(near_r && adz <= 1);
                const bool hasm = -adz >= dz0 && !(near_r && adz <= 1);
                if (!hasp && !hasm) continue;
                if (oc++ % G != g || jr < 0 || jr >= nb) continue;
                const int jp = zb + adz, jm = zb - adz;
                u_src[nu][0][b] = (hasp && sl >= 0 && jp < nb) ? sslot[jr * nb + jp] : -1;
                u_src[nu][1][b] = (hasm && sl >= 0 && jm >= 0) ? sslot[jr * nb + jm] : -1;
                if (b == 0) {
                    const bool outward = dr <= 0;
                    const int inner = outward ? jr : station;
                    const int adr = outward ? -dr : dr;
                    u_toff[nu] = (int64_t)n * TS + ((int64_t)inner * 12 + geom_slot(adr, adz)) * nmodes * TS;
                    u_out[nu] = outward;
                }
                ++nu;
            }
        }
        if (b == 0) s_nunits = nu;
    }
    __syncthreads();
    if (tid == 0) {                             // drop the units no box of the tile has sources for
        int m = 0;
        for (int u = 0; u < s_nunits; ++u) {
            bool any = false;
            for (int b = 0; b < TB; ++b) any |= u_src[u][0][b] >= 0 || u_src[u][1][b] >= 0;
            if (!any) continue;
            if (m != u) {
                u_toff[m] = u_toff[u];
                u_out[m] = u_out[u];
                for (int b = 0; b < TB; ++b) {
                    u_src[m][0][b] = u_src[u][0][b];
                    u_src[m][1][b] = u_src[u][1][b];
                }
            }
            ++m;
        }
        s_nunits = m;
    }
    // rows of each parity and their tiles
    int R0 = 0, R1 = 0;
    for (int k = 0; k <= M; ++k) {
        R0 += (M + 2 - k) / 2;
        R1 += (M + 1 - k) / 2;
    }
    const int NT0 = (R0 + 15) / 16, NT = NT0 + (R1 + 15) / 16;
    // the table position of this lane's operand row (k, l) of each row tile,
    // for both orientations: entry (a, b, c) sits at table_row(M, a, b) + c,
    // so row (k, l) meets column (i, j) at
    //   outward  table_row(M, k, i) + j + l = ro + i (2M + 1 - k) + j - i (i - 1) / 2
    //   inward   table_row(M, i, k) + j + l = ri - i k + table_row(M, i, 0) + j
    const int K2 = 2 * M + 1;
    int ro[TPW], ri[TPW], kr[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = w + W * u;
        int k = 0, l = 0;
        if (t < NT) {
            const int par = t >= NT0;
            int idx = (par ? t - NT0 : t) * 16 + (lane & 15);
            if (idx < (par ? R1 : R0)) {
                for (;; ++k) {
                    const int cnt = (M + 1 - k + 1 - par) / 2;
                    if (idx < cnt) break;
                    idx -= cnt;
                }
                l = par + 2 * idx;
            }
        }
        kr[u] = k;
        ro[u] = table_row(M, k, 0) + l;
        ri[u] = k * K2 - (k * (k - 1)) / 2 + l;
    }
    mfma_d4 acc[TPW][NB];
#pragma unroll
    for (int u = 0; u < TPW; ++u)
#pragma unroll
        for (int h = 0; h < NB; ++h) acc[u][h] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();                            // unit list, invfact

    const int kk = lane >> 4;                   // this lane's column of the 4 x 16 moment block
    const int col = lane & 15, mb = col >> 1, comp = col & 1;
    const int nst = (P + 3) >> 2;
    const double *dmom = reinterpret_cast<const double *>(mom);
    const int nunits = s_nunits;
    for (int un = 0; un < nunits; ++un) {
        // the unit's table (uniform: its entries are addressed by 32-bit byte
        // offsets from a scalar base; a table is (M + 1)^3 doubles)
        const int64_t toff = u_toff[un];
        const uint32_t tlo = __builtin_amdgcn_readfirstlane((uint32_t)toff);
        const uint32_t thi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)toff >> 32));
        const char *Tb = reinterpret_cast<const char *>(tab + (int64_t)(((uint64_t)thi << 32) | tlo));
        const bool outward = u_out[un] != 0;
        int base[TPW], mult[TPW];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            base[u] = outward ? ro[u] : ri[u];
            mult[u] = outward ? K2 - kr[u] : -kr[u];
        }
        // this lane's box of each column tile (mb + 8 h)
        const double *mp[NB], *mm[NB];
        double fp[NB], fm[NB];
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            const int sp = u_src[un][0][mb + 8 * h], sm = u_src[un][1][mb + 8 * h];
            const bool hasp = sp >= 0, hasm = sm >= 0;
            // a box without a source reads the moments of slot 0 (valid) and drops them
            mp[h] = dmom + 2 * ((int64_t)(hasp ? sp : 0) * C + c) * P + comp;
            mm[h] = dmom + 2 * ((int64_t)(hasm ? sm : 0) * C + c) * P + comp;
            fp[h] = hasp ? 1.0 : 0.0;
            fm[h] = hasm ? 1.0 : 0.0;
        }
        // operands of the k-step holding packed moment p = (i, j) in this
        // lane's column; every load is unconditional and in bounds (a column
        // past the last moment reads (M, 0) and moment P - 1, then drops them)
        // (the moments are taken raw and scaled by 0 or 1 where they are
        // used, so that no branch or select waits on the load)
        auto gather = [&](int p, int i, int j, double (&av)[TPW], double (&xp)[NB], double (&xm)[NB]) {
            const bool live = p < P;
            const int ii = live ? i : M, jj = live ? j : 0;
            const int cterm = outward ? jj - (ii * (ii - 1)) / 2 : table_row(M, ii, 0) + jj;
#pragma unroll
            for (int u = 0; u < TPW; ++u)
                av[u] = *reinterpret_cast<const double *>(Tb + (uint32_t)(base[u] + ii * mult[u] + cterm) * 8u);
            const int pc = live ? p : P - 1;
#pragma unroll
            for (int h = 0; h < NB; ++h) {
                xp[h] = mp[h][2 * pc];
                xm[h] = mm[h][2 * pc];
            }
        };
        // (i, j) of packed index p + 4 from (i, j) of p (past the last moment
        // i runs to M + 1, which gather clamps)
        auto advance = [&](int &i, int &j) {
            j += 4;
#pragma unroll
            for (int r = 0; r < 4; ++r) {       // rows are >= 1 long: at most 4 wraps
                const bool wrap = i <= M && j > M - i;
                j = wrap ? j - (M + 1 - i) : j;
                i = wrap ? i + 1 : i;
            }
        };
        // the contraction of one k-step: operands av, raw moments (xp, xm)
        // of column (p, j)
        auto contract = [&](const double (&av)[TPW], const double (&xp)[NB], const double (&xm)[NB], int p, int j) {
            // combined moments: A = M+ + (-1)^j M-, B = M+ - (-1)^j M-
            const double live = p < P ? 1.0 : 0.0;
            double bA[NB], bB[NB];
#pragma unroll
            for (int h = 0; h < NB; ++h) {
                const double vp = xp[h] * (fp[h] * live), vm = xm[h] * (((j & 1) ? -fm[h] : fm[h]) * live);
                bA[h] = vp + vm;
                bB[h] = vp - vm;
            }
            // every tile of the wave runs (an idle tile's rows read row
            // (0, 0) and are never written), so no branch splits the step;
            // each operand block feeds the NB column tiles
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int t = w + W * u;
#pragma unroll
                for (int h = 0; h < NB; ++h)
                    acc[u][h] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], t >= NT0 ? bB[h] : bA[h], acc[u][h], 0, 0, 0);
            }
        };
        // two operand sets used in turn: the loads of step st + 1 go to the
        // other set while the matrix cores run step st (no register copies,
        // so nothing waits on a load before its step)
        int p0 = kk, i0 = 0, j0 = kk;
        while (j0 > M - i0 && i0 < M) {         // (i, j) of p = kk
            j0 -= M + 1 - i0;
            ++i0;
        }
        double a0[TPW], a1[TPW], x0p[NB], x0m[NB], x1p[NB], x1m[NB];
        gather(p0, i0, j0, a0, x0p, x0m);
        // (the loop body is one branch-free block, the step count rounded up
        // to even (a step past the last moment adds zeros), and the
        // scheduling barriers keep each step's loads ahead of the other
        // set's matrix operations)
        for (int st = 0; st < nst; st += 2) {
            int p1 = p0 + 4, i1 = i0, j1 = j0;
            advance(i1, j1);
            gather(p1, i1, j1, a1, x1p, x1m);
            __builtin_amdgcn_sched_barrier(0);
            contract(a0, x0p, x0m, p0, j0);
            __builtin_amdgcn_sched_barrier(0);
            p0 = p1 + 4;
            i0 = i1;
            j0 = j1;
            advance(i0, j0);
            gather(p0, i0, j0, a0, x0p, x0m);
            __builtin_amdgcn_sched_barrier(0);
            contract(a1, x1p, x1m, p1, j1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // lane holds rows lane / 16 + 4 v, v < 4, of column lane % 16 of each of
    // its row tiles; (-1)^l / l! times the sum goes to the locals (or this
    // group's partial sums)
    double *dl = reinterpret_cast<double *>(loc);
    double *dp = reinterpret_cast<double *>(part);
#pragma unroll
    for (int h = 0; h < NB; ++h) {
    const int ob = mb + 8 * h;
    if (ob >= nbx) break;
    const int slot = tslots[tl.z + ob];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = w + W * u;
        if (t >= NT) continue;
        const int par = t >= NT0;
        const int Rp = par ? R1 : R0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int idx = (par ? t - NT0 : t) * 16 + (lane >> 4) + 4 * v;
            if (idx >= Rp) continue;
            int k = 0;
            for (;; ++k) {
                const int cnt = (M + 1 - k + 1 - par) / 2;
                if (idx < cnt) break;
                idx -= cnt;
            }
            const int ll = par + 2 * idx;
            const double f = ((ll & 1) ? -tscale : tscale) * invfact[ll];
            const int64_t e = ((int64_t)slot * C + c) * P + tri_index(M, k, ll);
            if (part) {
                dp[2 * ((int64_t)g * nocc * C * P + e) + comp] = f * acc[u][h][v];
            } else {
                dl[2 * e + comp] = fma(f, acc[u][h][v], dl[2 * e + comp]);
            }
        }
    }
    }
}

template <int TPW, int NB>
__global__ __launch_bounds__(64) void k_s2l_mfma(int M, int nmodes, int nrhs, int level, int TS,
                                                             const int4 *__restrict__ tiles,
                                                             const int32_t *__restrict__ tslots,
                                                             const int32_t *__restrict__ tbox,
                                                             const int32_t *__restrict__ sslot,
                                                             const double2 *__restrict__ mom,
                                                             const double *__restrict__ tab, double2 *__restrict__ loc,
                                                             int G, double2 *__restrict__ part, int nocc, double tscale,
                                                             int W)
{
    s2l_mfma_body<TPW, NB>(M, nmodes, nrhs, level, tiles, tslots, tbox, sslot, mom, tab, loc, blockIdx.x, G, part, nocc,
                           tscale, TS, W);
}

// Sum of the offset groups' partial S2L results into the locals, in group
// order (deterministic).
__global__ __launch_bounds__(256) void k_s2l_reduce(int64_t n, int G, const double2 *__restrict__ part,
                                                   double2 *__restrict__ loc)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    double2 v = loc[e];
    for (int g = 0; g < G; ++g) {
        const double2 x = part[(int64_t)g * n + e];
        v.x += x.x;
        v.y += x.y;
    }
    loc[e] = v;
}

template <int LB, int TB, int MW, bool FIX>
__global__ __launch_bounds__(256) void k_s2l_tile(int M, int nmodes, int nrhs, int level, int TS,
                                                  const int4 *__restrict__ tiles, const int32_t *__restrict__ tslots,
                                                  const int32_t *__restrict__ tbox, const int32_t *__restrict__ sslot,
                                                  const double2 *__restrict__ mom, const double *__restrict__ tab,
                                                  double2 *__restrict__ loc, int G, double2 *__restrict__ part,
                                                  int nocc, double tscale)
{
    s2l_tile_body<LB, TB, MW, FIX>(M, nmodes, nrhs, level, TS, tiles, tslots, tbox, sslot, mom, tab, loc, blockIdx.x, G,
                                   part, nocc, tscale);
}

// ------------------------------------------------------------ pair sums
// Accumulators of one lane: potential, and for MODE != 0 the r- and
// x-derivatives (App. A, first-derivative starting formulas).
template <int NMB, int MODE>
struct Acc {
    double ar[NMB], ai[NMB];
    double rr_[MODE ? NMB : 1], ri_[MODE ? NMB : 1], zr_[MODE ? NMB : 1], zi_[MODE ? NMB : 1];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int n = 0; n < NMB; ++n) {
            ar[n] = ai[n] = 0.0;
            if constexpr (MODE != 0) rr_[n] = ri_[n] = zr_[n] = zi_[n] = 0.0;
        }
    }
};

// Backward-branch values of a pair: in registers for the potential-only
// kernels of up to 24 modes, otherwise in the wave's LDS scratch `lg`
// [NMB][64] (the gradient accumulators leave no registers for them).
template <int NMB, int MODE>
struct BackVals {
    static constexpr bool kReg = MODE == 0 && NMB <= 24;
    double v[kReg ? NMB : 1];
    double *lg;
    int lane;
    __device__ __forceinline__ void set(int n, double x)
    {
        if constexpr (kReg) v[n] = x;
        else lg[n * 64 + lane] = x;
    }
    __device__ __forceinline__ double get(int n) const
    {
        if constexpr (kReg) return v[n];
        else return lg[n * 64 + lane];
    }
};

// One mode's contribution g = G^(n) of a pair: potential, and for MODE != 0
// the r- and x-derivatives from G^(n) and G^(n-1) (App. A, first-derivative
// starting formulas).
struct PairDeriv {
    double iprp, iprm, Ar, hr, x;
};
template <int NMB, int MODE>
__device__ __forceinline__ void accum_mode(Acc<NMB, MODE> &A, int n, double g, double &gprev, const double2 v,
                                           const PairDeriv &pd)
{
    A.ar[n] = fma(g, v.x, A.ar[n]);
    A.ai[n] = fma(g, v.y, A.ai[n]);
    if constexpr (MODE != 0) {
        const double nu = n - 0.5;
        const double W = (g + gprev) * pd.iprp + (g - gprev) * pd.iprm;
        const double gdr = fma(pd.hr, g, nu * pd.Ar * W);
        const double gdx = nu * pd.x * W;
        A.rr_[n] = fma(gdr, v.x, A.rr_[n]);
        A.ri_[n] = fma(gdr, v.y, A.ri_[n]);
        A.zr_[n] = fma(gdx, v.x, A.zr_[n]);
        A.zi_[n] = fma(gdx, v.y, A.zi_[n]);
        gprev = g;
    }
}

// One step of the forward recursion (eq. gfunc:recursion) in differences:
// with D_n = G^(n) - G^(n+1) the recursion
//   (n + 1/2) G^(n+1) = 2 n chi G^(n) - (n - 1/2) G^(n-1)
// becomes D_n = ((n - 1/2) D_(n-1) - 2 n (chi - 1) G^(n)) / (n + 1/2),
// G^(n+1) = G^(n) - D_n.  Near chi = 1 neighbouring modes are close and the
// three-term form subtracts nearly equal products (and rounds chi itself);
// here the small differences are carried directly and chi - 1 comes from
// rho-^2 without cancellation: 1e-14 instead of 1e-12 relative at 64 modes.
// On entry g = G^(n), dg = D_(n-1) (D_0 = G^(0) - G^(1) for n = 0: the
// n = 0 step just forms G^(1)); on exit g = G^(n+1), dg = D_n.
__device__ __forceinline__ void fwd_step(int n, double dchi, double &g, double &dg)
{
    if (n > 0) {
        const double an = (n - 0.5) / (n + 0.5), bn = 2.0 * n / (n + 0.5);
        dg = fma(an, dg, -(bn * dchi) * g);
    }
    g -= dg;
}

// The G^(n)(r, r1, x), n < NMB, of one pair per lane, handed to sink(n,
// G^(n), gprev, pd) in increasing n (gprev, pd: the previous value and the
// pair's derivative data, for the gradient accumulators).  All lanes of the
// wave call it together (the backward recursion runs a wave-wide number of
// steps).  `use` = false lanes get zeros.  The wave takes one of three mode
// streams: all pairs forward (the recursion streams into the sink), all
// backward (normalised Miller values), or mixed (both, selected per lane).
template <int NMB, int MODE, class Sink>
__device__ __forceinline__ void pair_visit(double r, double r1, double x, double inv_r, double inv_r1, bool use,
                                           double chistar, int nmodes, double *__restrict__ lg, Sink &&sink)
{
    const int lane = threadIdx.x & 63;
    const double dr = r - r1, sr = r + r1;
    double rm2 = fma(dr, dr, x * x);
    const double rp2 = fma(sr, sr, x * x);
    if (!use) rm2 = rp2;
    const double inv_rr = inv_r * inv_r1;
    PairStart ps = pair_start(rm2, rp2, r * r1, inv_rr);
    if (!use) {
        ps.g0 = 0.0;
        ps.g1 = 0.0;
        ps.chi = 1.0;
    }
    const bool back = (NMB > 2) && ps.chi >= chistar;
    const bool anyback = __ballot(back) != 0;
    // every pair of the wave on the backward branch (idle lanes have g0 = 0
    // and contribute nothing either way): no forward recursion needed
    const bool allback = anyback && __ballot(use && !back) == 0;
    BackVals<NMB, MODE> bv;
    bv.lg = lg;
    bv.lane = lane;
    if constexpr (NMB > 2) {
        if (anyback) {
            // Miller's backward recursion, started from the large-n limit of
            // the ratio G^(n+1)/G^(n) (from the hypergeometric form
            // Q_(n-1/2)(cosh eta) ~ e^(-(n+1/2) eta) 2F1(1/2, n+1/2; n+1; e^(-2 eta))):
            //   t_n ~ (n+1/2)/(n+1) e^(-eta) (1 + q / (4 (1-q) n (n+1))),  q = e^(-2 eta).
            // Its error decays like e^(-2 eta) per step; 3 + 12/sqrt(2 (chi-1))
            // steps above the top mode reach the rounding level (the bound
            // acosh(1 + d) <= sqrt(2 d) makes the count conservative).
            const double dmin = wave_min(back ? ps.dchi : 1e300);
            int extra = 3 + (int)ceil(12.0 * __builtin_amdgcn_rsq(2.0 * dmin));
            // steps above the stored modes, a multiple of 16
            int nsteps = nmodes - 1 + extra - (NMB - 1);
            nsteps = (nsteps + 15) & ~15;
            if (nsteps < 16) nsteps = 16;
            if (NMB - 1 + nsteps > kMillerMax) nsteps = (kMillerMax - NMB + 1) & ~15;
            const int ntop = __builtin_amdgcn_readfirstlane(NMB - 1 + nsteps);
            // lanes on the forward branch run the same steps on a harmless chi
            const double dch = back ? ps.dchi : dmin;
            const double chi = back ? ps.chi : 1.0 + dmin;
            const double lam = chi + fast_sqrt(dch * (chi + 1.0));      // e^eta
            const double il = fast_rcp(lam), q = il * il;
            const double nt = (double)ntop;
            const double t = (nt + 0.5) * fast_rcp(nt + 1.0) * il *
                             fma(q, fast_rcp(4.0 * (1.0 - q) * nt * (nt + 1.0)), 1.0);
            double zc = 1.0;                                  // z_ntop
            double zp = t * fast_rcp(c_down.rho[ntop + 1]);   // z_(ntop+1)
            for (int n = ntop; n >= NMB; n -= 16) {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const double zm = fma(c_down.alpha[n - u] * chi, zc, -zp);
                    zp = zc;
                    zc = zm;
                }
                if (fabs(zc) > 0x1p500) {
                    zc *= 0x1p-500;
                    zp *= 0x1p-500;
                }
            }
            // back to G-scaled values with w_(NMB-1) = 1: y_(NMB-1), y_NMB
            double y = zc, yp = c_down.rho[NMB] * zp;
            // keep the growth of the last NMB-1 steps (at most lam per step)
            // in range: lam < 2^(ilogb(lam) + 1) bounds it without a
            // logarithm; a power-of-two scale changes no rounding
            const int ey = ilogb(y);
            int e = ey + (NMB - 1) * (ilogb(lam) + 1) - 16;
            int emax = ey + 1000;
            if (e > emax) e = emax;
            y = ldexp(y, -e);
            yp = ldexp(yp, -e);
            bv.set(NMB - 1, y);
            double up = yp;
#pragma unroll
            for (int n = NMB - 1; n >= 1; --n) {
                const double fa = 4.0 * n / (2.0 * n - 1.0), fb = (2.0 * n + 1.0) / (2.0 * n - 1.0);
                double ym = fma(fa * chi, y, -fb * up);
                up = y;
                y = ym;
                bv.set(n - 1, y);
            }
            // normalise by G^(0) from the AGM
            const double scale = ps.g0 * fast_rcp(y);
#pragma unroll
            for (int n = 0; n < NMB; ++n) bv.set(n, scale * bv.get(n));
        }
    }
    PairDeriv pd{};
    if constexpr (MODE != 0) {
        pd.iprp = fast_rcp(rp2);
        pd.iprm = fast_rcp(rm2);
        pd.Ar = (r * r - r1 * r1 - x * x) * 0.5 * inv_r;
        pd.hr = -0.5 * inv_r;
        pd.x = x;
    }
    const double chi = ps.chi;
    if (MODE == 0 && NMB > 2 && allback) {
        double gprev = bv.get(1);               // G^(-1) = G^(1)
#pragma unroll
        for (int n = 0; n < NMB; ++n) sink(n, bv.get(n), gprev, pd);
        return;
    }
    // forward recursion (in differences, fwd_step) streamed over the modes
    // (mixed waves select the backward value on their backward lanes)
    double gprev = ps.g1;
    if constexpr (MODE != 0 && NMB > 2) {
        if (anyback && back) gprev = bv.get(1);
    }
    (void)chi;
    const double dchi = use ? ps.dchi : 0.0;
    double gcur = ps.g0, dg = ps.g0 - ps.g1;
#pragma unroll
    for (int n = 0; n < NMB; ++n) {
        double g = gcur;
        if constexpr (NMB > 2) {
            if (anyback) g = back ? bv.get(n) : g;
        }
        sink(n, g, gprev, pd);
        if (n + 1 < NMB) fwd_step(n, dchi, gcur, dg);
    }
}

// Adds S_s^(n) G^(n)(r, r1, x) for n < nmodes of one pair per lane (Ss: the
// source's strengths of modes 0..NMB-1 for this right-hand side, zero
// beyond nmodes).
template <int NMB, int MODE>
__device__ __forceinline__ void pair_accum(double r, double r1, double x, double inv_r, double inv_r1, bool use,
                                           double chistar, int nmodes, const double2 *Ss,
                                           Acc<NMB, MODE> &A, double *__restrict__ lg)
{
    pair_visit<NMB, MODE>(r, r1, x, inv_r, inv_r1, use, chistar, nmodes, lg,
                          [&](int n, double g, double &gprev, const PairDeriv &pd) {
                              accum_mode<NMB, MODE>(A, n, g, gprev, Ss[n], pd);
                          });
}

// Launch shape of the pair kernels per mode bucket: waves per block (each
// takes every WPB-th source) and sources per staged tile; larger buckets use
// fewer waves so that the LDS scratch fits.
template <int NMB>
struct PairShape {
    static constexpr int WPB = NMB <= 33 ? 4 : 2;
    static constexpr int ST = NMB <= 33 ? 64 : 32;
    static constexpr int RC = 16;       // modes per reduction round
};

// Deterministic sum of the block's waves' accumulators through LDS, in
// rounds of RC modes [N0, N1); wave 0 ends with the totals.  The rounds are
// unrolled at compile time so that every accumulator index is a constant
// (a runtime mode index would move the accumulators to scratch memory).
template <int NMB, int MODE, int WPB, int N0>
__device__ __forceinline__ void reduce_round(Acc<NMB, MODE> &A, double *__restrict__ buf, int w, int lane)
{
    constexpr int K = MODE ? 6 : 2;
    constexpr int RC = PairShape<NMB>::RC;
    constexpr int N1 = N0 + RC < NMB ? N0 + RC : NMB;
    for (int src = WPB - 1; src >= 0; --src) {
        __syncthreads();
        if (w == src) {
#pragma unroll
            for (int n = N0; n < N1; ++n) {
                double *bp = buf + ((size_t)(n - N0) * 64 + lane) * K;
                double v[6] = {A.ar[n], A.ai[n], 0, 0, 0, 0};
                if constexpr (MODE != 0) {
                    v[2] = A.rr_[n]; v[3] = A.ri_[n]; v[4] = A.zr_[n]; v[5] = A.zi_[n];
                }
                if (src == WPB - 1) {
#pragma unroll
                    for (int k = 0; k < K; ++k) bp[k] = v[k];
                } else if (src > 0) {
#pragma unroll
                    for (int k = 0; k < K; ++k) bp[k] += v[k];
                } else {
                    A.ar[n] += bp[0];
                    A.ai[n] += bp[1];
                    if constexpr (MODE != 0) {
                        A.rr_[n] += bp[2]; A.ri_[n] += bp[3]; A.zr_[n] += bp[4]; A.zi_[n] += bp[5];
                    }
                }
            }
        }
    }
    if constexpr (N1 < NMB) reduce_round<NMB, MODE, WPB, N1>(A, buf, w, lane);
}

template <int NMB, int MODE, int WPB>
__device__ __forceinline__ void reduce_waves(Acc<NMB, MODE> &A, double *__restrict__ buf)
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    reduce_round<NMB, MODE, WPB, 0>(A, buf, w, lane);
    __syncthreads();
}

template <int NMB, int MODE>
constexpr size_t leaf_lds_doubles()
{
    constexpr int WPB = PairShape<NMB>::WPB, RC = PairShape<NMB>::RC;
    size_t miller = (size_t)WPB * NMB * 64;
    size_t red = (size_t)64 * RC * (MODE ? 6 : 2);
    return miller > red ? miller : red;
}

// scratch + staged source tile (strengths, r, z, 1/r)
template <int NMB, int MODE>
constexpr size_t leaf_lds_bytes()
{
    constexpr int ST = PairShape<NMB>::ST;
    return leaf_lds_doubles<NMB, MODE>() * sizeof(double) + (size_t)ST * NMB * 16 + 3 * ST * sizeof(double);
}

// Strength loads per staging round and thread, by mode bucket: as many as
// the kernels' registers allow without losing a wave per SIMD.
template <int NMB>
constexpr int kStageLoads = NMB == 17 ? 4 : NMB <= 12 ? 2 : 1;

// One tile of sources into LDS for the pair kernels (NT threads): element
// e < nel of st_S is val(e), and source k < cnt (cnt <= NT) has its r, z and
// 1/r at st_[rzi][k], source index src_of(k).  Every thread issues its
// coordinate loads and up to four strength loads before its first LDS write,
// so a tile waits about one memory latency, not one per element (B loads
// per round: fewer where the kernel's registers are scarce).
template <int NT, int B, class SrcOf, class Val>
__device__ __forceinline__ void stage_tile(int cnt, int nel, SrcOf src_of, Val val, const SideView &sv,
                                           const double *__restrict__ sinv, double2 *__restrict__ st_S,
                                           double *__restrict__ st_r, double *__restrict__ st_z,
                                           double *__restrict__ st_i)
{
    const int tid = threadIdx.x;
    const bool crd = tid < cnt;
    double cr = 0.0, cz = 0.0, ci = 0.0;
    if (crd) {
        const auto sidx = src_of(tid);
        cr = sv.r[sidx];
        cz = sv.z[sidx];
        ci = sinv[sidx];
    }
    for (int base = 0; base < nel; base += B * NT) {
        double2 v[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int e = base + b * NT + tid;
            v[b] = e < nel ? val(e) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int e = base + b * NT + tid;
            if (e < nel) st_S[e] = v[b];
        }
    }
    if (crd) {
        st_r[tid] = cr;
        st_z[tid] = cz;
        st_i[tid] = ci;
    }
}

// The sources of the 3 x 3 neighbour leaves of leaf (ir, iz) as one list,
// leaf by leaf (r outer, z inner; leaves outside the domain are empty):
// item li is source li + d_i of the tree order, i the last of the nine
// leaves whose start cb[i] in the list is <= li; d_i is accumulated from the
// steps inc[i] = d_i - d_(i-1) (the starts do not decrease), so that no
// array is indexed at run time and the list stays in registers.
struct NearList {
    int cb[9], inc[9], total;
    __device__ __forceinline__ NearList(const int32_t *__restrict__ off, int ir, int iz, int nb)
    {
        total = 0;
        int dprev = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int jr = ir + i / 3 - 1, jz = iz + i % 3 - 1;
            const bool in = jr >= 0 && jr < nb && jz >= 0 && jz < nb;
            const uint32_t m = in ? morton((uint32_t)jr, (uint32_t)jz) : 0u;
            const int b = in ? off[m] : 0, e = in ? off[m + 1] : 0;
            cb[i] = total;
            inc[i] = (b - total) - dprev;
            dprev = b - total;
            total += e - b;
        }
    }
    __device__ __forceinline__ int source(int li) const
    {
        int d = inc[0];
#pragma unroll
        for (int i = 1; i < 9; ++i) d += li >= cb[i] ? inc[i] : 0;
        return li + d;
    }
};

// ------------------------------------------------------------ leaf pass
// One block (four waves) per chunk of <= 64 targets of one leaf: local
// expansion (eq. analysis:local) plus the direct sum over the 3x3 neighbour
// leaves, the sources dealt round-robin to the four waves (and to the lane
// groups of a wave when the chunk has 32 targets or fewer).
// MODE 0: potential; 1: potential and gradient; 2: potential and the
// adjoint coordinate contraction.  PART 0: both sums; PART 1 (MODE 0): the
// near field only, written to phi (it needs no local expansions, so it runs
// beside the downward pass; k_l2p adds them afterwards).
template <int NMB, int MODE, int PART = 0>
__device__ __forceinline__ void leaf_body(int M, int nmodes, int nrhs, int depth, double rlo, double zlo,
                                             double invh, double chistar, const int4 *__restrict__ chunks,
                                             SideView tv, SideView sv, const double *__restrict__ sinv,
                                             const double2 *__restrict__ Sg, const double2 *__restrict__ loc,
                                             double2 *__restrict__ phi, double2 *__restrict__ dphr,
                                             double2 *__restrict__ dphz, double2 *__restrict__ dpha,
                                             const double2 *__restrict__ Sdot,
                                             double *__restrict__ gr, double *__restrict__ gz, int64_t ntot,
                                             int Cs, int item)
{
    constexpr int WPB = PairShape<NMB>::WPB, ST = PairShape<NMB>::ST;
    extern __shared__ double lds[];
    double2 *st_S = reinterpret_cast<double2 *>(lds + leaf_lds_doubles<NMB, MODE>());
    double *st_r = reinterpret_cast<double *>(st_S + ST * NMB);
    double *st_z = st_r + ST, *st_i = st_z + ST;
    const int4 ch = chunks[item];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    // a chunk of T targets takes tp lanes (T rounded up to a power of two)
    // per group and SG = 64 / tp groups per wave; the groups take different
    // sources of each staged tile and are summed before the cross-wave
    // reduction, so that small chunks (the last of a leaf, small leaves)
    // leave no lanes idle
    const int T = ch.z;
    const int tp = T > 32 ? 64 : T > 16 ? 32 : T > 8 ? 16 : T > 4 ? 8 : T > 2 ? 4 : T > 1 ? 2 : 1;
    const int SG = 64 / tp;
    const int tl = lane & (tp - 1), sg = lane / tp;
    const bool active = tl < T;
    const int t = ch.y + (active ? tl : 0);
    const int nb = 1 << depth;
    const int ir = ch.w / nb, iz = ch.w - (ch.w / nb) * nb;
    const int P = (M + 1) * (M + 2) / 2;
    const int C = nmodes * nrhs;
    const double r = tv.r[t], z = tv.z[t];
    const double xr = (r - rlo) * invh - (ir + 0.5);
    const double xz = (z - zlo) * invh - (iz + 0.5);
    const double inv_r = fast_rcp(r);
    const int orig = tv.perm[t];
    double *lg = lds + (size_t)w * NMB * 64;
    double gsr = 0.0, gsz = 0.0;
    for (int q = 0; q < nrhs; ++q) {
        Acc<NMB, MODE> A;
        A.zero();
        // local expansion, monomials dealt round-robin over the (wave,
        // group) slots
        const double2 *lc = loc + (int64_t)ch.x * C * P;
        if constexpr (PART != 1) {
            double pr = 1.0, pr1 = 0.0;
            int p = 0;
            for (int kk = 0; kk <= M; ++kk) {
                double pz = 1.0, pz1 = 0.0;
                for (int ll = 0; kk + ll <= M; ++ll, ++p) {
                    if (p % (WPB * SG) == w * SG + sg) {
                        const double wv = pr * pz;
#pragma unroll
                        for (int n = 0; n < NMB; ++n) {
                            if (n < nmodes) {
                                const double2 v = lc[(int64_t)(n * nrhs + q) * P + p];
                                A.ar[n] = fma(wv, v.x, A.ar[n]);
                                A.ai[n] = fma(wv, v.y, A.ai[n]);
                                if constexpr (MODE != 0) {
                                    const double wr = pr1 * pz * invh, wz = pr * pz1 * invh;
                                    A.rr_[n] = fma(wr, v.x, A.rr_[n]);
                                    A.ri_[n] = fma(wr, v.y, A.ri_[n]);
                                    A.zr_[n] = fma(wz, v.x, A.zr_[n]);
                                    A.zi_[n] = fma(wz, v.y, A.zi_[n]);
                                }
                            }
                            if ((n & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    pz1 = (ll + 1) * pz;
                    pz *= xz;
                }
                pr1 = (kk + 1) * pr;
                pr *= xr;
            }
        }
        // near field: the sources of the 3x3 neighbour leaves in tiles of 64,
        // staged in LDS, dealt round-robin to the four waves
        const NearList nl(sv.off, ir, iz, nb);
        const int total = nl.total;
        for (int tile = 0; tile < total; tile += ST) {
            __syncthreads();
            const int cnt = min(ST, total - tile);
            stage_tile<64 * WPB, kStageLoads<NMB>>(
                cnt, cnt * NMB, [&](int k) { return nl.source(tile + k); },
                [&](int e) {
                    const int k = e / NMB, n = e - k * NMB;
                    return Sg[(int64_t)nl.source(tile + k) * Cs + n * nrhs + q];
                },
                sv, sinv, st_S, st_r, st_z, st_i);
            __syncthreads();
            // slot w SG + sg of every WPB SG sources (a lane past the tile's
            // end reads its group's first source and adds nothing)
            for (int kb = w * SG; kb < cnt; kb += WPB * SG) {
                const int k = kb + sg < cnt ? kb + sg : kb;
                const double r1 = st_r[k], x = z - st_z[k];
                const bool use = active && kb + sg < cnt && !(r == r1 && x == 0.0);
                pair_accum<NMB, MODE>(r, r1, x, inv_r, st_i[k], use, chistar, nmodes, st_S + k * NMB, A, lg);
            }
        }
        if (SG > 1) {
            // the groups' sums, by a fixed butterfly (the same order every call)
            auto fold = [&](double &v) {
                for (int off = tp; off < 64; off <<= 1) v += __shfl_xor(v, off);
            };
#pragma unroll
            for (int n = 0; n < NMB; ++n) {
                fold(A.ar[n]);
                fold(A.ai[n]);
                if constexpr (MODE != 0) {
                    fold(A.rr_[n]);
                    fold(A.ri_[n]);
                    fold(A.zr_[n]);
                    fold(A.zi_[n]);
                }
            }
        }
        reduce_waves<NMB, MODE, WPB>(A, lds);
        if (w == 0 && active && sg == 0) {
#pragma unroll
            for (int n = 0; n < NMB; ++n) {
                if (n < nmodes) {
                    int64_t o = ((int64_t)q * nmodes + n) * ntot + orig;
                    phi[o] = make_double2(A.ar[n], A.ai[n]);
                    if constexpr (MODE == 1) {
                        if (dphr) dphr[o] = make_double2(A.rr_[n], A.ri_[n]);
                        if (dphz) dphz[o] = make_double2(A.zr_[n], A.zi_[n]);
                        // (1/r) d/dtheta of the mode-n term: i n Phi^(n) / r
                        if (dpha) dpha[o] = make_double2(-n * A.ai[n] * inv_r, n * A.ar[n] * inv_r);
                    }
                    if constexpr (MODE == 2) {
                        double2 sd = Sdot[o];
                        gsr += sd.x * A.rr_[n] + sd.y * A.ri_[n];
                        gsz += sd.x * A.zr_[n] + sd.y * A.zi_[n];
                    }
                }
            }
        }
        __syncthreads();
    }
    if constexpr (MODE == 2) {
        if (w == 0 && active && sg == 0) {
            if (gr) gr[orig] = gsr;
            if (gz) gz[orig] = gsz;
        }
    }
}

template <int NMB, int MODE, int PART>
__global__ __launch_bounds__(64 * PairShape<NMB>::WPB) void k_leaf(
    int M, int nmodes, int nrhs, int depth, double rlo, double zlo, double invh, double chistar,
    const int4 *__restrict__ chunks, SideView tv, SideView sv, const double *__restrict__ sinv,
    const double2 *__restrict__ Sg, const double2 *__restrict__ loc, double2 *__restrict__ phi,
    double2 *__restrict__ dphr, double2 *__restrict__ dphz, double2 *__restrict__ dpha,
    const double2 *__restrict__ Sdot,
    double *__restrict__ gr, double *__restrict__ gz, int64_t ntot, int Cs)
{
    leaf_body<NMB, MODE, PART>(M, nmodes, nrhs, depth, rlo, zlo, invh, chistar, chunks, tv, sv, sinv, Sg, loc, phi,
                               dphr, dphz, dpha, Sdot, gr, gz, ntot, Cs, blockIdx.x);
}

// ------------------------------------------- near field, shared G^(n)
// Near field of a potential evaluation with several right-hand sides and at
// most 24 modes: G^(n) of a (target, source) pair is computed once for every
// right-hand side.  A wave serves 64 / QP targets with QP lanes each (QP =
// nrhs rounded up to 2, 4 or 8; lane q of a target accumulates right-hand
// side q).  In each step the QP lanes of a target take QP consecutive
// sources, write their G^(n) to the wave's LDS rows, and each lane then adds
// G^(n) S_q^(n) of all QP sources (the sources in order, as the one-source
// kernel does).  A block has QP waves, the <= 64 targets of one chunk; every
// wave walks all sources of the 3 x 3 neighbour leaves, staged in LDS in
// tiles of 32 (QP = 2, 4) or 16 (QP = 8) sources.  The result goes to phi;
// the local expansions are added by k_l2p.
template <int NMB, int QP>
struct NearQShape {
    static constexpr int ST = QP == 2 ? 32 : 128 / QP;           // sources per staged tile
    static constexpr size_t kLdsBytes = sizeof(double) * ((size_t)QP * NMB * 64 + 3 * ST) +
                                        sizeof(double2) * (size_t)ST * NMB * QP;
};

template <int NMB, int QP>
__device__ __forceinline__ void leaf_q_body(int nmodes, int nrhs, int depth, double chistar,
                                            const int4 *__restrict__ chunks, SideView tv, SideView sv,
                                            const double *__restrict__ sinv, const double2 *__restrict__ Sg,
                                            double2 *__restrict__ phi, int64_t ntot, int Cs, int item)
{
    constexpr int ST = NearQShape<NMB, QP>::ST, TPW = 64 / QP;
    extern __shared__ double lds[];
    double *gl_all = lds;                                        // [QP waves][NMB][64]
    double *st_r = lds + (size_t)QP * NMB * 64;
    double *st_z = st_r + ST, *st_i = st_z + ST;
    double2 *st_S = reinterpret_cast<double2 *>(st_i + ST);     // [ST][NMB][QP]
    const int4 ch = chunks[item];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int tl = lane / QP, q = lane - (lane / QP) * QP;
    double *gl = gl_all + (size_t)w * NMB * 64;
    const int tix = w * TPW + tl;                               // target of the chunk
    const bool active = tix < ch.z;
    const int t = ch.y + (active ? tix : 0);
    const int nb = 1 << depth;
    const int ir = ch.w / nb, iz = ch.w - (ch.w / nb) * nb;
    const double r = tv.r[t], z = tv.z[t];
    const double inv_r = fast_rcp(r);
    Acc<NMB, 0> A;
    A.zero();
    const NearList nl(sv.off, ir, iz, nb);
    const int total = nl.total;
    for (int tile = 0; tile < total; tile += ST) {
        __syncthreads();
        const int cnt = min(ST, total - tile);
        stage_tile<64 * QP, kStageLoads<NMB>>(
            cnt, cnt * NMB * QP, [&](int k) { return nl.source(tile + k); },
            [&](int e) {
                const int k = e / (NMB * QP), rem = e - k * (NMB * QP);
                const int n = rem / QP, qq = rem - (rem / QP) * QP;
                return qq < nrhs ? Sg[(int64_t)nl.source(tile + k) * Cs + n * nrhs + qq] : make_double2(0.0, 0.0);
            },
            sv, sinv, st_S, st_r, st_z, st_i);
        __syncthreads();
        for (int k0 = 0; k0 < cnt; k0 += QP) {
            // this lane's pair: its target with source k0 + q
            const int k = min(k0 + q, cnt - 1);
            const double r1 = st_r[k], x = z - st_z[k];
            const bool use = active && k0 + q < cnt && !(r == r1 && x == 0.0);
            pair_visit<NMB, 0>(r, r1, x, inv_r, st_i[k], use, chistar, nmodes, nullptr,
                               [&](int n, double g, double &, const PairDeriv &) { gl[n * 64 + lane] = g; });
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // G^(n) of the target's QP pairs (lanes tl QP .. tl QP + QP - 1)
            // against this lane's right-hand side, sources in order
#pragma unroll
            for (int qs = 0; qs < QP; ++qs) {
                if (k0 + qs >= cnt) break;                           // uniform
                const double *gq = gl + tl * QP + qs;
                const double2 *Sq = st_S + ((size_t)(k0 + qs) * NMB) * QP + q;
#pragma unroll
                for (int n = 0; n < NMB; ++n) {
                    const double g = gq[n * 64];
                    const double2 v = Sq[n * QP];
                    A.ar[n] = fma(g, v.x, A.ar[n]);
                    A.ai[n] = fma(g, v.y, A.ai[n]);
                }
            }
            // every lane has read the rows before the next step rewrites them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (active && q < nrhs) {
        const int orig = tv.perm[t];
#pragma unroll
        for (int n = 0; n < NMB; ++n)
            if (n < nmodes) phi[((int64_t)q * nmodes + n) * ntot + orig] = make_double2(A.ar[n], A.ai[n]);
    }
}

template <int NMB, int QP>
__global__ __launch_bounds__(64 * QP) void k_leaf_q(int nmodes, int nrhs, int depth, double chistar,
                                                    const int4 *__restrict__ chunks, SideView tv, SideView sv,
                                                    const double *__restrict__ sinv, const double2 *__restrict__ Sg,
                                                    double2 *__restrict__ phi, int64_t ntot, int Cs)
{
    leaf_q_body<NMB, QP>(nmodes, nrhs, depth, chistar, chunks, tv, sv, sinv, Sg, phi, ntot, Cs, blockIdx.x);
}

// ------------------------------------------------------------------ L2P
// Local expansions at the field points (eq. analysis:local), added to the
// near field already in phi: one block per (chunk of <= 64 targets, group of
// kL2PChannels channels); the chunk's leaf coefficients of those channels
// are staged in LDS and each wave evaluates one channel at its targets by
// Horner's rule in z nested in Horner's rule in r (offsets in box units).
constexpr int kL2PChannels = 4;
__device__ __forceinline__ void l2p_body(int M, int nmodes, int nrhs, int depth, double rlo, double zlo, double invh,
                                         const int4 ch, SideView tv, const double2 *__restrict__ loc,
                                         double2 *__restrict__ phi, int64_t ntot, int grp, double2 *__restrict__ cf)
{
    const int P = (M + 1) * (M + 2) / 2, C = nmodes * nrhs;
    const int c0 = grp * kL2PChannels, nc = min(kL2PChannels, C - c0);
    const double2 *lc = loc + ((int64_t)ch.x * C + c0) * P;
    for (int e = threadIdx.x; e < nc * P; e += blockDim.x) cf[e] = lc[e];
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (w >= nc || lane >= ch.z) return;
    const int c = c0 + w, n = c / nrhs, q = c - n * nrhs;
    const int nb = 1 << depth;
    const int ir = ch.w / nb, iz = ch.w - (ch.w / nb) * nb;
    const int t = ch.y + lane;
    const double xr = (tv.r[t] - rlo) * invh - (ir + 0.5);
    const double xz = (tv.z[t] - zlo) * invh - (iz + 0.5);
    const double2 *ck = cf + w * P;
    double ar = 0.0, ai = 0.0;
    for (int kk = M; kk >= 0; --kk) {
        const int base = kk * (M + 1) - (kk * (kk - 1)) / 2;     // packed (kk, 0)
        double sr = ck[base + M - kk].x, si = ck[base + M - kk].y;
        for (int ll = M - kk - 1; ll >= 0; --ll) {
            sr = fma(sr, xz, ck[base + ll].x);
            si = fma(si, xz, ck[base + ll].y);
        }
        ar = fma(ar, xr, sr);
        ai = fma(ai, xr, si);
    }
    const int64_t o = ((int64_t)q * nmodes + n) * ntot + tv.perm[t];
    const double2 v = phi[o];
    phi[o] = make_double2(v.x + ar, v.y + ai);
}

__global__ __launch_bounds__(64 * kL2PChannels) void k_l2p(int M, int nmodes, int nrhs, int depth, double rlo,
                                                           double zlo, double invh, const int4 *__restrict__ chunks,
                                                           SideView tv, const double2 *__restrict__ loc,
                                                           double2 *__restrict__ phi, int64_t ntot)
{
    extern __shared__ double2 cf[];          // [kL2PChannels][P]
    const int C = nmodes * nrhs;
    const int ngrp = (C + kL2PChannels - 1) / kL2PChannels;
    const int ci = blockIdx.x / ngrp, grp = blockIdx.x - ci * ngrp;
    l2p_body(M, nmodes, nrhs, depth, rlo, zlo, invh, chunks[ci], tv, loc, phi, ntot, grp, cf);
}

// ---------------------------------------------------------------- direct
// One block (four waves) per 64 targets; each wave takes every fourth source.
template <int NMB>
__global__ __launch_bounds__(64 * PairShape<NMB>::WPB) void k_direct(int nmodes, int nrhs, double chistar, SideView tv, int64_t nt,
                                               SideView sv, const double *__restrict__ sinv, int64_t ns,
                                               const double2 *__restrict__ Sg, double2 *__restrict__ phi, int Cs)
{
    constexpr int WPB = PairShape<NMB>::WPB, ST = PairShape<NMB>::ST;
    extern __shared__ double lds[];
    double2 *st_S = reinterpret_cast<double2 *>(lds + leaf_lds_doubles<NMB, 0>());
    double *st_r = reinterpret_cast<double *>(st_S + ST * NMB);
    double *st_z = st_r + ST, *st_i = st_z + ST;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t tg = blockIdx.x * (int64_t)64 + lane;
    const bool active = tg < nt;
    const int64_t t = active ? tg : 0;
    const int C = nmodes * nrhs;
    const double r = tv.r[t], z = tv.z[t];
    const double inv_r = fast_rcp(r);
    double *lg = lds + (size_t)w * NMB * 64;
    for (int q = 0; q < nrhs; ++q) {
        Acc<NMB, 0> A;
        A.zero();
        for (int64_t tile = 0; tile < ns; tile += ST) {
            __syncthreads();
            const int cnt = (int)min((int64_t)ST, ns - tile);
            stage_tile<64 * WPB, kStageLoads<NMB>>(
                cnt, cnt * NMB, [&](int k) { return tile + k; },
                [&](int e) {
                    const int k = e / NMB, n = e - k * NMB;
                    return Sg[(tile + k) * Cs + n * nrhs + q];
                },
                sv, sinv, st_S, st_r, st_z, st_i);
            __syncthreads();
            for (int k = w; k < cnt; k += WPB) {
                const double r1 = st_r[k], x = z - st_z[k];
                const bool use = active && !(r == r1 && x == 0.0);
                pair_accum<NMB, 0>(r, r1, x, inv_r, st_i[k], use, chistar, nmodes, st_S + k * NMB, A, lg);
            }
        }
        reduce_waves<NMB, 0, WPB>(A, lds);
        if (w == 0 && active) {
            const int orig = tv.perm[t];
#pragma unroll
            for (int n = 0; n < NMB; ++n)
                if (n < nmodes) phi[((int64_t)q * nmodes + n) * nt + orig] = make_double2(A.ar[n], A.ai[n]);
        }
        __syncthreads();
    }
}

SideView view_of(const Side &s)
{
    SideView v;
    v.r = s.r;
    v.z = s.z;
    v.perm = s.perm;
    v.off = s.off;
    return v;
}

// Dynamic LDS above 64 KiB (wide tiles at high order) needs the kernel's
// attribute raised once per device.
template <class K>
void allow_lds(K kernel, size_t shm, int device, bool (&done)[64])
{
    if (shm > 65536 && !done[device & 63]) {
        AXF_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        done[device & 63] = true;
    }
}

template <int LB, int TB, int MW, bool FIX>
void launch_s2l_t(Plan &pl, const Side &src, const Side &tgt, int l, hipStream_t st)
{
    size_t shm = sizeof(double2) * 2 * (size_t)TB * pl.P;
    static bool attr[64] = {};
    allow_lds(k_s2l_tile<LB, TB, MW, FIX>, shm, pl.device, attr);
    const int G = tgt.s2l_groups[l];
    double2 *part = G > 1 ? pl.s2l_part : nullptr;
    k_s2l_tile<LB, TB, MW, FIX><<<tgt.ntiles[l] * pl.C * G, 64 * s2l_waves(pl.M), shm, st>>>(
        pl.M, pl.nmodes, pl.nrhs, l, pl.TS, tgt.tiles[l], tgt.tile_slots[l], tgt.box[l], src.slot[l],
        pl.lev[l].mom, pl.lev[l].tab, pl.lev[l].loc, G, part, tgt.nocc[l], pl.lev[l].tscale);
    if (G > 1) {
        const int64_t n = (int64_t)tgt.nocc[l] * pl.C * pl.P;
        k_s2l_reduce<<<(int)((n + 255) / 256), 256, 0, st>>>(n, G, part, pl.lev[l].loc);
    }
}

void launch_s2l_mfma(Plan &pl, const Side &src, const Side &tgt, int l, hipStream_t st)
{
    const int G = tgt.s2l_groups[l];
    double2 *part = G > 1 ? pl.s2l_part : nullptr;
    int tpw = 0, waves = 0;
    s2l_mfma_shape(pl.M, tpw, waves);
    // two column tiles (16 boxes) where a station column holds more than 8
    // boxes, else one
    const bool two = (1 << l) > kS2lMfmaBoxes && pl.tb > kS2lMfmaBoxes;
#define AXF_S2L_MFMA(T, NB)                                                                                      \
    k_s2l_mfma<T, NB><<<tgt.ntiles[l] * pl.C * G * waves, 64, 0, st>>>(                                          \
        pl.M, pl.nmodes, pl.nrhs, l, pl.TS, tgt.tiles[l], tgt.tile_slots[l], tgt.box[l], src.slot[l],          \
        pl.lev[l].mom, pl.lev[l].tab, pl.lev[l].loc, G, part, tgt.nocc[l], pl.lev[l].tscale, waves)
    if (two) {
        if (tpw == 4) AXF_S2L_MFMA(4, 2);
        else if (tpw == 5) AXF_S2L_MFMA(5, 2);
        else if (tpw == 6) AXF_S2L_MFMA(6, 2);
        else AXF_S2L_MFMA(7, 2);
    } else {
        if (tpw == 4) AXF_S2L_MFMA(4, 1);
        else if (tpw == 5) AXF_S2L_MFMA(5, 1);
        else if (tpw == 6) AXF_S2L_MFMA(6, 1);
        else AXF_S2L_MFMA(7, 1);
    }
#undef AXF_S2L_MFMA
    if (G > 1) {
        const int64_t n = (int64_t)tgt.nocc[l] * pl.C * pl.P;
        k_s2l_reduce<<<(int)((n + 255) / 256), 256, 0, st>>>(n, G, part, pl.lev[l].loc);
    }
}

void launch_s2l(Plan &pl, const Side &src, const Side &tgt, int l, hipStream_t st)
{
    {
        // locals of the level's target boxes: shifted parent expansion, or zero
        PhaseTimer tm(pl, st, AXF_PHASE_L2L);
        k_l2l<<<tgt.nocc[l] * pl.C, 256, 0, st>>>(pl.M, pl.C, l, tgt.box[l], l > 2 ? tgt.slot[l - 1] : nullptr,
                                                   l > 2 ? pl.lev[l - 1].loc : nullptr, pl.lev[l].loc, pl.shift_coef);
    }
    PhaseTimer tm(pl, st, AXF_PHASE_S2L);
    if (pl.mfma) {
        launch_s2l_mfma(pl, src, tgt, l, st);
        return;
    }
#define AXF_S2L_LAUNCH2(LB, MW, FIX) launch_s2l_t<LB, 2, MW, FIX>(pl, src, tgt, l, st)
#define AXF_S2L_LAUNCH4(LB, MW, FIX) launch_s2l_t<LB, 4, MW, FIX>(pl, src, tgt, l, st)
#define AXF_S2L_LAUNCH8(LB, MW, FIX) launch_s2l_t<LB, 8, MW, FIX>(pl, src, tgt, l, st)
    if (pl.tb == 2) AXF_S2L_SHAPES(pl.M, AXF_S2L_LAUNCH2);
    else if (pl.tb == 8) AXF_S2L_SHAPES(pl.M, AXF_S2L_LAUNCH8);
    else AXF_S2L_SHAPES(pl.M, AXF_S2L_LAUNCH4);
#undef AXF_S2L_LAUNCH2
#undef AXF_S2L_LAUNCH4
#undef AXF_S2L_LAUNCH8
}

template <int NMB, int MODE, int PART = 0>
void launch_leaf_mode(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st)
{
    SideView tv = view_of(tgt), sv = view_of(src);
    double invh = (double)(1 << pl.d) * pl.invL;
    const double2 *loc = pl.lev[pl.d].loc;
    constexpr size_t shm = leaf_lds_bytes<NMB, MODE>();
    static bool attr[64] = {};
    if (shm > 65536 && !attr[pl.device & 63]) {
        AXF_HIP(hipFuncSetAttribute((const void *)k_leaf<NMB, MODE, PART>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
        attr[pl.device & 63] = true;
    }
    if (tgt.nchunks == 0) return;
    k_leaf<NMB, MODE, PART><<<tgt.nchunks, 64 * PairShape<NMB>::WPB, shm, st>>>(pl.M, pl.nmodes, pl.nrhs, pl.d, pl.rlo, pl.zlo, invh,
                                                     pl.chistar, tgt.chunks, tv, sv, src.rinv, pl.Sg, loc,
                                                     (double2 *)out.phi, (double2 *)out.dr, (double2 *)out.dz,
                                                     (double2 *)out.daz, (const double2 *)out.Sdot, out.gr, out.gz, tgt.n,
                                                     NMB * pl.nrhs);
}

template <int NMB>
void launch_leaf(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st, int part = 0)
{
    if (out.mode == 0 && part == 1) launch_leaf_mode<NMB, 0, 1>(pl, src, tgt, out, st);
    else if (out.mode == 0) launch_leaf_mode<NMB, 0>(pl, src, tgt, out, st);
    else if (out.mode == 1) launch_leaf_mode<NMB, 1>(pl, src, tgt, out, st);
    else launch_leaf_mode<NMB, 2>(pl, src, tgt, out, st);
}

// Near field with G^(n) shared by the right-hand sides (potential, nrhs >= 2,
// NMB <= kNearQMaxModes); QP = nrhs rounded up to 2, 4 or 8.
template <int NMB, int QP>
void launch_leaf_q_t(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st)
{
    constexpr size_t shm = NearQShape<NMB, QP>::kLdsBytes;
    static bool attr[64] = {};
    allow_lds(k_leaf_q<NMB, QP>, shm, pl.device, attr);
    k_leaf_q<NMB, QP><<<tgt.nchunks, 64 * QP, shm, st>>>(pl.nmodes, pl.nrhs, pl.d, pl.chistar, tgt.chunks,
                                                         view_of(tgt), view_of(src), src.rinv, pl.Sg,
                                                         (double2 *)out.phi, tgt.n, NMB * pl.nrhs);
}

template <int NMB>
void launch_leaf_q(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st)
{
    if constexpr (NMB <= kNearQMaxModes) {
        if (pl.nrhs <= 2) launch_leaf_q_t<NMB, 2>(pl, src, tgt, out, st);
        else if (pl.nrhs <= 4) launch_leaf_q_t<NMB, 4>(pl, src, tgt, out, st);
        else launch_leaf_q_t<NMB, 8>(pl, src, tgt, out, st);
    }
}

template <int NMB>
void launch_direct(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st)
{
    SideView tv = view_of(tgt), sv = view_of(src);
    int g = (int)((tgt.n + 63) / 64);
    constexpr size_t shm = leaf_lds_bytes<NMB, 0>();
    static bool attr[64] = {};
    if (shm > 65536 && !attr[pl.device & 63]) {
        AXF_HIP(hipFuncSetAttribute((const void *)k_direct<NMB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
        attr[pl.device & 63] = true;
    }
    k_direct<NMB><<<g, 64 * PairShape<NMB>::WPB, shm, st>>>(pl.nmodes, pl.nrhs, pl.chistar, tv, tgt.n, sv, src.rinv, src.n, pl.Sg,
                                       (double2 *)out.phi, NMB * pl.nrhs);
}

// ------------------------------------------------------------- batches
// Persistent kernels: each block walks the merged queue of (problem, item)
// pairs of all problems of a batch, reading the problem's descriptor.
// The descriptors are read through the constant address space: a pointer
// read from ordinary memory is generic (flat), and the compiler would address
// through it with flat instructions and 64-bit vector addresses, whereas a
// pointer read from constant memory is taken to be global, as kernel-argument
// pointers are (scalar base plus vector offset).
constexpr int kPersistBlocks = 2048;
typedef __attribute__((address_space(4))) const ProbDev ConstProbDev;
__device__ __forceinline__ SideView view_of(const __attribute__((address_space(4))) SideView &v)
{
    SideView s;
    s.r = v.r;
    s.z = v.z;
    s.perm = v.perm;
    s.off = v.off;
    return s;
}

__global__ __launch_bounds__(256) void kb_gather(const ProbDev *__restrict__ P, const int2 *__restrict__ q, int n,
                                                int nmodes)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        const int64_t e = (int64_t)it.y * 256 + threadIdx.x;
        if (e >= pd.ns * pd.Cs) continue;
        const int64_t pp = e / pd.Cs;
        const int c = (int)(e - pp * pd.Cs);
        const int nn = c / pd.nrhs, qq = c - nn * pd.nrhs;
        pd.Sg[e] = nn < nmodes ? pd.S[((int64_t)qq * nmodes + nn) * pd.ns + pd.sv.perm[pp]] : make_double2(0.0, 0.0);
    }
}

__global__ __launch_bounds__(256) void kb_p2m(const ProbDev *__restrict__ P, const int2 *__restrict__ q, int n, int M)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        __syncthreads();
        p2m_body(M, pd.C, pd.Cs, pd.d, pd.rlo, pd.zlo, (double)(1 << pd.d) * pd.invL, view_of(pd.sv), pd.sbox[pd.d], pd.Sg,
                 pd.mom[pd.d], it.y);
    }
}

__global__ __launch_bounds__(256) void kb_m2m(const ProbDev *__restrict__ P, const int2 *__restrict__ q, int n, int M,
                                             int t)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        const int l = pd.d - t;
        __syncthreads();
        m2m_body(M, pd.C, l, pd.sbox[l], pd.sslot[l + 1], pd.mom[l + 1], pd.mom[l], pd.shift_coef, it.y);
    }
}

template <int LB, int TB, int MW, bool FIX>
__global__ __launch_bounds__(256) void kb_s2l(const ProbDev *__restrict__ P, const int2 *__restrict__ q, int n, int M,
                                             int nmodes, int TS, int l)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        __syncthreads();
        s2l_tile_body<LB, TB, MW, FIX>(M, nmodes, pd.nrhs, l, TS, pd.tiles[l], pd.tile_slots[l], pd.tbox[l], pd.sslot[l],
                              pd.mom[l], pd.tab[l], pd.loc[l], it.y, 1, nullptr, 0, pd.tscale[l]);
    }
}

__global__ __launch_bounds__(256) void kb_l2l(const ProbDev *__restrict__ P, const int2 *__restrict__ q, int n, int M,
                                             int l)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        __syncthreads();
        l2l_body(M, pd.C, l, pd.tbox[l], l > 2 ? pd.tslot[l - 1] : nullptr, l > 2 ? pd.loc[l - 1] : nullptr,
                 pd.loc[l], pd.shift_coef, it.y);
    }
}

// PART 0: near field and local expansions; PART 1: near field only (the
// local expansions follow in kb_l2p).
template <int NMB, int PART>
__global__ __launch_bounds__(64 * PairShape<NMB>::WPB) void kb_leaf(const ProbDev *__restrict__ P,
                                                                    const int2 *__restrict__ q, int n, int M,
                                                                    int nmodes, double chistar)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        __syncthreads();
        leaf_body<NMB, 0, PART>(M, nmodes, pd.nrhs, pd.d, pd.rlo, pd.zlo, (double)(1 << pd.d) * pd.invL, chistar,
                                pd.chunks, view_of(pd.tv), view_of(pd.sv), pd.srinv, pd.Sg, pd.loc[pd.d], pd.phi, nullptr,
                                nullptr, nullptr, nullptr, nullptr, nullptr, pd.nf, pd.Cs, it.y);
    }
}

// Near field with G^(n) shared by QP right-hand-side lanes, over a queue of
// (problem, chunk) items of problems with the same lane count.
template <int NMB, int QP>
__global__ __launch_bounds__(64 * QP) void kb_leaf_q(const ProbDev *__restrict__ P, const int2 *__restrict__ q,
                                                     int n, int nmodes, double chistar)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        __syncthreads();
        leaf_q_body<NMB, QP>(nmodes, pd.nrhs, pd.d, chistar, pd.chunks, view_of(pd.tv), view_of(pd.sv), pd.srinv,
                             pd.Sg, pd.phi, pd.nf, pd.Cs, it.y);
    }
}

// Local expansions of every chunk of the leaf queue, all channel groups.
__global__ __launch_bounds__(64 * kL2PChannels) void kb_l2p(const ProbDev *__restrict__ P,
                                                            const int2 *__restrict__ q, int n, int M, int nmodes)
{
    extern __shared__ double2 cf[];
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int2 it = q[i];
        ConstProbDev &pd = ((ConstProbDev *)P)[it.x];
        const int C = nmodes * pd.nrhs, ngrp = (C + kL2PChannels - 1) / kL2PChannels;
        for (int g = 0; g < ngrp; ++g) {
            __syncthreads();
            l2p_body(M, nmodes, pd.nrhs, pd.d, pd.rlo, pd.zlo, (double)(1 << pd.d) * pd.invL, pd.chunks[it.y],
                     view_of(pd.tv), pd.loc[pd.d], pd.phi, pd.nf, g, cf);
        }
    }
}

template <int LB, int TB, int MW, bool FIX>
void launch_s2l_batch(const BatchQueues &bq, int l, hipStream_t st)
{
    const int P = (bq.M + 1) * (bq.M + 2) / 2;
    size_t shm = sizeof(double2) * 2 * (size_t)TB * P;
    static bool attr[64] = {};
    int dev = 0;
    AXF_HIP(hipGetDevice(&dev));
    allow_lds(kb_s2l<LB, TB, MW, FIX>, shm, dev, attr);
    const int t = tile_index(TB);
    int g = std::min(bq.ns2l[l][t], kPersistBlocks * 2);
    kb_s2l<LB, TB, MW, FIX><<<g, 64 * s2l_waves(bq.M), shm, st>>>(bq.probs, bq.s2l[l][t], bq.ns2l[l][t], bq.M,
                                                                   bq.nmodes, bq.TS, l);
}


template <int NMB, int QP>
void launch_leafq_batch_t(const BatchQueues &bq, int c, hipStream_t st)
{
    constexpr size_t shm = NearQShape<NMB, QP>::kLdsBytes;
    static bool attr[64] = {};
    int dev = 0;
    AXF_HIP(hipGetDevice(&dev));
    allow_lds(kb_leaf_q<NMB, QP>, shm, dev, attr);
    kb_leaf_q<NMB, QP><<<std::min(bq.nleafq[c], kPersistBlocks), 64 * QP, shm, st>>>(bq.probs, bq.leafq[c],
                                                                                    bq.nleafq[c], bq.nmodes,
                                                                                    bq.chistar);
}

// The near field of every leaf chunk (potential only; the local expansions
// follow in kb_l2p): each near-field class with its kernel.
template <int NMB>
void launch_near_batch(const BatchQueues &bq, hipStream_t st)
{
    if (bq.nleafq[0]) {
        constexpr size_t shm = leaf_lds_bytes<NMB, 0>();
        static bool attr[64] = {};
        int dev = 0;
        AXF_HIP(hipGetDevice(&dev));
        allow_lds(kb_leaf<NMB, 1>, shm, dev, attr);
        kb_leaf<NMB, 1><<<std::min(bq.nleafq[0], kPersistBlocks), 64 * PairShape<NMB>::WPB, shm, st>>>(
            bq.probs, bq.leafq[0], bq.nleafq[0], bq.M, bq.nmodes, bq.chistar);
    }
    if constexpr (NMB <= kNearQMaxModes) {
        if (bq.nleafq[1]) launch_leafq_batch_t<NMB, 2>(bq, 1, st);
        if (bq.nleafq[2]) launch_leafq_batch_t<NMB, 4>(bq, 2, st);
        if (bq.nleafq[3]) launch_leafq_batch_t<NMB, 8>(bq, 3, st);
    }
}

// ------------------------------------------------------------- census
// Work census of the pair sums for the flop model: per pair, the AGM
// iterations to convergence (the criterion of pair_start, c <= 2^-15 a) and the recursion
// steps the pair itself needs (forward: N - 1; backward: N + 3 +
// 12 / sqrt(2 (chi - 1)), the count the backward branch uses for its worst
// lane).  Sums per block: [pairs, backward pairs, AGM iterations, steps].
__device__ __forceinline__ void census_pair(double r, double z, double r1, double z1, double chistar, int N,
                                            double (&cnt)[4])
{
    if (r == r1 && z == z1) return;
    const double x = z - z1, dr = r - r1, sr = r + r1;
    const double rm2 = dr * dr + x * x, rp2 = sr * sr + x * x, rr = r * r1;
    double a = sqrt(rp2), b = sqrt(rm2), c = 2.0 * rr / (a + b);
    int it = 0;
    for (; it < 48;) {
        const double an = 0.5 * (a + b);
        b = sqrt(a * b);
        a = an;
        ++it;
        if (c <= 0x1p-15 * a) break;
        c = 0.5 * (a - b);
    }
    const double dchi = rm2 / (2.0 * rr);
    cnt[0] += 1.0;
    cnt[2] += it;
    if (1.0 + dchi >= chistar) {
        cnt[1] += 1.0;
        cnt[3] += N + 3 + ceil(12.0 / sqrt(2.0 * dchi));
    } else {
        cnt[3] += N > 1 ? N - 1 : 0;
    }
}

__device__ __forceinline__ void census_block_sum(double (&cnt)[4], double *__restrict__ out)
{
    __shared__ double red[4][256];
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = cnt[q];
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) v += red[threadIdx.x][t];
        out[blockIdx.x * 4 + threadIdx.x] = v;
    }
}

// near field: one thread per target of a leaf chunk, the sources of the 3x3
// neighbour leaves
__global__ __launch_bounds__(64) void k_census_near(int depth, int N, double chistar,
                                                   const int4 *__restrict__ chunks, SideView tv, SideView sv,
                                                   double *__restrict__ out)
{
    const int4 ch = chunks[blockIdx.x];
    double cnt[4] = {0.0, 0.0, 0.0, 0.0};
    if ((int)threadIdx.x < ch.z) {
        const int t = ch.y + threadIdx.x;
        const double r = tv.r[t], z = tv.z[t];
        const int nb = 1 << depth;
        const int ir = ch.w / nb, iz = ch.w - (ch.w / nb) * nb;
        for (int jr = max(ir - 1, 0); jr <= min(ir + 1, nb - 1); ++jr)
            for (int jz = max(iz - 1, 0); jz <= min(iz + 1, nb - 1); ++jz) {
                const uint32_t m = morton((uint32_t)jr, (uint32_t)jz);
                for (int s = sv.off[m]; s < sv.off[m + 1]; ++s) census_pair(r, z, sv.r[s], sv.z[s], chistar, N, cnt);
            }
    }
    census_block_sum(cnt, out);
}

// direct sum: every `stride`-th target against all sources
__global__ __launch_bounds__(256) void k_census_direct(int N, double chistar, SideView tv, int64_t nt, int64_t stride,
                                                      SideView sv, int64_t ns, double *__restrict__ out)
{
    double cnt[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * stride;
    if (t < nt) {
        const double r = tv.r[t], z = tv.z[t];
        for (int64_t s = 0; s < ns; ++s) census_pair(r, z, sv.r[s], sv.z[s], chistar, N, cnt);
    }
    census_block_sum(cnt, out);
}

#define AXF_BUCKETS(X) X(4) X(9) X(12) X(17) X(24) X(33) X(48) X(64)

}  // namespace

// Shift factors of the M2M and L2L passes for order M, in the layout the
// kernels read: [L2L F][M2M r][M2M z] x [d = -1/4, +1/4] x [S][S].
//   L2L:  F[i][q] = C(i+q, q) d^q 2^-i,  i + q <= M;
//   M2M:  r factor C(i, a) d^(i-a) 2^-a and z factor d^(i-a) / (i-a)! 2^-a,  a <= i.
void shift_coef_host(int M, std::vector<double> &out)
{
    const int S = kCoefS;
    out.assign((size_t)6 * S * S, 0.0);
    for (int sg = 0; sg < 2; ++sg) {
        const double d = sg ? 0.25 : -0.25;
        for (int i = 0; i <= M; ++i)
            for (int q = 0; q <= M; ++q) {
                if (i + q <= M) {
                    double bin = 1.0, pw = 1.0;
                    for (int s = 0; s < q; ++s) {
                        bin = bin * (i + q - s) / (s + 1.0);
                        pw *= d;
                    }
                    out[(size_t)sg * S * S + i * S + q] = bin * pw * std::ldexp(1.0, -i);
                }
                const int a = q;
                if (a <= i) {
                    double bin = 1.0, pw = 1.0, fct = 1.0;
                    for (int t = 0; t < a; ++t) bin = bin * (i - t) / (t + 1.0);
                    for (int t = 0; t < i - a; ++t) {
                        pw *= d;
                        fct *= (t + 1.0);
                    }
                    const double two = std::ldexp(1.0, -a);
                    out[(size_t)(2 + sg) * S * S + i * S + a] = bin * pw * two;
                    out[(size_t)(4 + sg) * S * S + i * S + a] = pw / fct * two;
                }
            }
    }
}

// The stream on which the near field of an evaluation runs beside the
// downward pass (one per device, default priority, kept for the process).
static hipStream_t near_stream(int device)
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    hipStream_t &s = streams[device & 63];
    if (!s) AXF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
}

void run_fmm(Plan &pl, const Side &src, const Side &tgt, const double *S, const EvalOut &out, hipStream_t st)
{
    const int M = pl.M, P = pl.P, C = pl.C, d = pl.d;
    const int64_t ns = src.n;
    {
        PhaseTimer tm(pl, st, AXF_PHASE_GATHER);
        int64_t tot = ns * pl.Cs;
        k_gather<<<(int)((tot + 255) / 256), 256, 0, st>>>((const double2 *)S, src.perm, ns, pl.nmodes, pl.nrhs,
                                                          pl.Cs, pl.Sg);
    }
    // potential only: the near field needs only the gathered strengths, so it
    // runs on a second stream beside the downward pass (both are
    // latency-bound and leave issue slots to the other); it is started after
    // the short upward pass so that it does not hold the CUs that pass
    // needs; the local expansions are added once both are done
    const bool split = out.mode == 0 && !out.fused && pl.overlap && tgt.nchunks > 0;
    // several right-hand sides: the near field computes each pair's G^(n)
    // once for all of them (then the local expansions are added by k_l2p)
    const bool multi = out.mode == 0 && !out.fused && near_class(pl.nrhs, pl.nmb) > 0 && tgt.nchunks > 0;
    SideView sv = view_of(src);
    if (src.nocc[d] > 0) {
        PhaseTimer tm(pl, st, AXF_PHASE_P2M);
        k_p2m<<<src.nocc[d] * p2m_pairs(C), 256, 0, st>>>(M, C, pl.Cs, d, pl.rlo, pl.zlo, (double)(1 << d) * pl.invL, sv, src.box[d],
                                           pl.Sg, pl.lev[d].mom);
    }
    {
        PhaseTimer tm(pl, st, AXF_PHASE_M2M);
        for (int l = d - 1; l >= 2; --l)
            if (src.nocc[l] > 0)
                k_m2m<<<src.nocc[l] * C, 256, 0, st>>>(M, C, l, src.box[l], src.slot[l + 1], pl.lev[l + 1].mom,
                                                   pl.lev[l].mom, pl.shift_coef);
    }
    if (split) {
        hipStream_t side = near_stream(pl.device);
        AXF_HIP(hipEventRecord(pl.ev_fork, st));
        AXF_HIP(hipStreamWaitEvent(side, pl.ev_fork, 0));
        {
            PhaseTimer tm(pl, side, AXF_PHASE_LEAF);
#define AXF_NEAR(B)                                                   \
    if (pl.nmb == B) {                                                \
        if (multi) launch_leaf_q<B>(pl, src, tgt, out, side);         \
        else launch_leaf<B>(pl, src, tgt, out, side, 1);              \
    }
            AXF_BUCKETS(AXF_NEAR)
#undef AXF_NEAR
        }
        AXF_HIP(hipEventRecord(pl.ev_join, side));
    }
    {
        // the tables (built on the table stream) are needed from here on
        if (pl.tables_ready) AXF_HIP(hipStreamWaitEvent(st, pl.tables_ready, 0));
        for (int l = 2; l <= d; ++l) {
            if (tgt.ntiles[l] == 0) continue;
            launch_s2l(pl, src, tgt, l, st);
        }
    }
    (void)pl.nmodes;
    if (multi && !split) {
        PhaseTimer tm(pl, st, AXF_PHASE_LEAF);
#define AXF_NEARQ(B) \
    if (pl.nmb == B) launch_leaf_q<B>(pl, src, tgt, out, st);
        AXF_BUCKETS(AXF_NEARQ)
#undef AXF_NEARQ
    }
    if (split || multi) {
        if (split) AXF_HIP(hipStreamWaitEvent(st, pl.ev_join, 0));
        PhaseTimer tm(pl, st, AXF_PHASE_L2P);
        const int ngrp = (C + kL2PChannels - 1) / kL2PChannels;
        k_l2p<<<tgt.nchunks * ngrp, 64 * kL2PChannels, sizeof(double2) * kL2PChannels * P, st>>>(
            M, pl.nmodes, pl.nrhs, d, pl.rlo, pl.zlo, (double)(1 << d) * pl.invL, tgt.chunks, view_of(tgt),
            pl.lev[d].loc, (double2 *)out.phi, tgt.n);
        AXF_HIP(hipGetLastError());
        return;
    }
    PhaseTimer tm_leaf(pl, st, AXF_PHASE_LEAF);
#define AXF_LEAF(B)                                         \
    if (pl.nmb == B) {                                      \
        launch_leaf<B>(pl, src, tgt, out, st);              \
        AXF_HIP(hipGetLastError());                         \
        return;                                             \
    }
    AXF_BUCKETS(AXF_LEAF)
#undef AXF_LEAF
}

void run_direct(Plan &pl, const Side &src, const Side &tgt, const double *S, const EvalOut &out, hipStream_t st)
{
    const int64_t ns = src.n;
    const int C = pl.C;
    int64_t tot = ns * pl.Cs;
    {
        PhaseTimer tm(pl, st, AXF_PHASE_GATHER);
        k_gather<<<(int)((tot + 255) / 256), 256, 0, st>>>((const double2 *)S, src.perm, ns, pl.nmodes, pl.nrhs,
                                                          pl.Cs, pl.Sg);
    }
    (void)pl.nmodes;
    PhaseTimer tm_dir(pl, st, AXF_PHASE_DIRECT);
#define AXF_DIR(B)                                          \
    if (pl.nmb == B) {                                      \
        launch_direct<B>(pl, src, tgt, out, st);            \
        AXF_HIP(hipGetLastError());                         \
        return;                                             \
    }
    AXF_BUCKETS(AXF_DIR)
#undef AXF_DIR
}

void run_batch(const BatchQueues &bq, hipStream_t st, const BatchSide *side)
{
    if (bq.ngather)
        kb_gather<<<std::min(bq.ngather, kPersistBlocks), 256, 0, st>>>(bq.probs, bq.gather, bq.ngather, bq.nmodes);
    if (bq.np2m) kb_p2m<<<std::min(bq.np2m, kPersistBlocks), 256, 0, st>>>(bq.probs, bq.p2m, bq.np2m, bq.M);
    for (int t = 1; t <= bq.maxd - 2; ++t)
        if (bq.nm2m[t])
            kb_m2m<<<std::min(bq.nm2m[t], kPersistBlocks), 256, 0, st>>>(bq.probs, bq.m2m[t], bq.nm2m[t], bq.M, t);
    // the near field of every problem beside the downward pass (as in
    // run_fmm), when a second stream is given
    const bool split = side != nullptr && bq.nleaf > 0;
    if (split) {
        AXF_HIP(hipEventRecord(side->fork, st));
        AXF_HIP(hipStreamWaitEvent(side->stream, side->fork, 0));
#define AXF_NEARB(B)                                    \
    if (bq.nmb == B) launch_near_batch<B>(bq, side->stream);
        AXF_BUCKETS(AXF_NEARB)
#undef AXF_NEARB
        AXF_HIP(hipEventRecord(side->join, side->stream));
    }
    for (int l = 2; l <= bq.maxd; ++l) {
        if (bq.nl2l[l])
            kb_l2l<<<std::min(bq.nl2l[l], kPersistBlocks), 256, 0, st>>>(bq.probs, bq.l2l[l], bq.nl2l[l], bq.M, l);
#define AXF_S2L_LAUNCH2(LB, MW, FIX) launch_s2l_batch<LB, 2, MW, FIX>(bq, l, st)
#define AXF_S2L_LAUNCH4(LB, MW, FIX) launch_s2l_batch<LB, 4, MW, FIX>(bq, l, st)
#define AXF_S2L_LAUNCH8(LB, MW, FIX) launch_s2l_batch<LB, 8, MW, FIX>(bq, l, st)
        // one launch per tile width in use (the problems of a batch may differ)
        if (bq.ns2l[l][0]) AXF_S2L_SHAPES(bq.M, AXF_S2L_LAUNCH2);
        if (bq.ns2l[l][1]) AXF_S2L_SHAPES(bq.M, AXF_S2L_LAUNCH4);
        if (bq.ns2l[l][2]) AXF_S2L_SHAPES(bq.M, AXF_S2L_LAUNCH8);
#undef AXF_S2L_LAUNCH2
#undef AXF_S2L_LAUNCH4
#undef AXF_S2L_LAUNCH8
    }
    if (bq.nleaf) {
        if (split) {
            AXF_HIP(hipStreamWaitEvent(st, side->join, 0));
        } else {
#define AXF_NEARB(B) \
    if (bq.nmb == B) launch_near_batch<B>(bq, st);
            AXF_BUCKETS(AXF_NEARB)
#undef AXF_NEARB
        }
        const int P = (bq.M + 1) * (bq.M + 2) / 2;
        kb_l2p<<<std::min(bq.nleaf, kPersistBlocks), 64 * kL2PChannels, sizeof(double2) * kL2PChannels * P, st>>>(
            bq.probs, bq.leaf, bq.nleaf, bq.M, bq.nmodes);
    }
    AXF_HIP(hipGetLastError());
}

void fill_probdev(const Plan &pl, const double *S, double *phi, ProbDev &pd)
{
    pd = ProbDev();
    pd.d = pl.d;
    pd.nrhs = pl.nrhs;
    pd.C = pl.C;
    pd.Cs = pl.Cs;
    pd.rlo = pl.rlo;
    pd.zlo = pl.zlo;
    pd.invL = pl.invL;
    pd.ns = pl.src.n;
    pd.nf = pl.fld.n;
    pd.sv = view_of(pl.src);
    pd.tv = view_of(pl.fld);
    pd.srinv = pl.src.rinv;
    pd.S = (const double2 *)S;
    pd.phi = (double2 *)phi;
    pd.Sg = pl.Sg;
    for (int l = 2; l <= pl.d; ++l) {
        pd.sbox[l] = pl.src.box[l];
        pd.sslot[l] = pl.src.slot[l];
        pd.tbox[l] = pl.fld.box[l];
        pd.tslot[l] = pl.fld.slot[l];
        pd.tiles[l] = pl.fld.tiles[l];
        pd.tile_slots[l] = pl.fld.tile_slots[l];
        pd.mom[l] = pl.lev[l].mom;
        pd.loc[l] = pl.lev[l].loc;
        pd.tab[l] = pl.lev[l].tab;
        pd.shift_coef = pl.shift_coef;
        pd.tscale[l] = pl.lev[l].tscale;
    }
    pd.chunks = pl.fld.chunks;
}

void pair_census(Plan &pl, bool direct, double out[4], hipStream_t st)
{
    const Side &src = pl.src, &tgt = pl.fld;
    int nblk;
    int64_t stride = 1;
    if (direct) {
        // sample targets so that about 3e7 pairs are visited
        stride = std::max<int64_t>(1, (int64_t)((double)tgt.n * src.n / 3e7));
        const int64_t nsamp = (tgt.n + stride - 1) / stride;
        nblk = (int)((nsamp + 255) / 256);
    } else {
        nblk = tgt.nchunks;
    }
    for (int q = 0; q < 4; ++q) out[q] = 0.0;
    if (nblk == 0) return;
    double *d = nullptr;
    AXF_HIP(hipMalloc(&d, sizeof(double) * 4 * (size_t)nblk));
    if (direct)
        k_census_direct<<<nblk, 256, 0, st>>>(pl.N, pl.chistar, view_of(tgt), tgt.n, stride, view_of(src), src.n, d);
    else
        k_census_near<<<nblk, 64, 0, st>>>(pl.d, pl.N, pl.chistar, tgt.chunks, view_of(tgt), view_of(src), d);
    std::vector<double> h(4 * (size_t)nblk);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipStreamSynchronize(st);
    (void)hipFree(d);
    AXF_HIP(e1);
    AXF_HIP(e2);
    AXF_HIP(e3);
    for (int b = 0; b < nblk; ++b)
        for (int q = 0; q < 4; ++q) out[q] += h[4 * (size_t)b + q];
    if (direct) {
        // scale the sampled counts to all targets
        const double f = (double)tgt.n / (double)((tgt.n + stride - 1) / stride);
        for (int q = 0; q < 4; ++q) out[q] *= f;
    }
}

}  // namespace axf


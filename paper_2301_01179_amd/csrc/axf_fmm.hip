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

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

namespace {

constexpr int kMaxRhs = AXF_MAX_RHS;

struct SideView {     // device-side view of a Side
    const double *r, *z;
    const int32_t *perm, *off;
};

// ---------------------------------------------------------------- gather
__global__ void k_gather(const double2 *__restrict__ S, const int32_t *__restrict__ perm, int64_t n,
                         int nmodes, int nrhs, double2 *__restrict__ Sg)
{
    int C = nmodes * nrhs;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * C) return;
    int64_t p = e / C;
    int c = (int)(e - p * C);
    int nn = c / nrhs, q = c - nn * nrhs;
    Sg[e] = S[((int64_t)q * nmodes + nn) * n + perm[p]];
}

// ------------------------------------------------------------------- P2M
constexpr int kP2MChunk = 32;
__global__ __launch_bounds__(256) void k_p2m(int M, int C, int depth, double rlo, double zlo, double invh,
                                            SideView sv, const int32_t *__restrict__ boxes,
                                            const double2 *__restrict__ Sg, double2 *__restrict__ mom)
{
    __shared__ double pr[kP2MChunk][AXF_MAX_ORDER + 1];
    __shared__ double pz[kP2MChunk][AXF_MAX_ORDER + 1];
    const int P = (M + 1) * (M + 2) / 2;
    const int k = blockIdx.x;
    const int b = boxes[k];
    const int nb = 1 << depth;
    const int ir = b / nb, iz = b - ir * nb;
    const uint32_t m = morton((uint32_t)ir, (uint32_t)iz);
    const int first = sv.off[m], last = sv.off[m + 1];
    const double cr = ir + 0.5, cz = iz + 0.5;
    const int nout = C * P;
    constexpr int kOut = 8;
    double2 acc[kOut];
    int oc[kOut], oi[kOut], oj[kOut];
#pragma unroll
    for (int u = 0; u < kOut; ++u) {
        acc[u] = make_double2(0.0, 0.0);
        int e = threadIdx.x + u * 256;
        int c = e / P, p = e - c * P;
        int i = 0;
        while (p >= M + 1 - i) {
            p -= M + 1 - i;
            ++i;
        }
        oc[u] = c;
        oi[u] = i;
        oj[u] = p;
    }
    for (int base = 0; base < nout; base += kOut * 256) {
        for (int s0 = first; s0 < last; s0 += kP2MChunk) {
            int ns = min(kP2MChunk, last - s0);
            __syncthreads();
            for (int e = threadIdx.x; e < ns; e += blockDim.x) {
                double dr = (sv.r[s0 + e] - rlo) * invh - cr;
                double dz = (sv.z[s0 + e] - zlo) * invh - cz;
                double a = 1.0, c = 1.0;
                for (int i = 0; i <= M; ++i) {
                    pr[e][i] = a;
                    pz[e][i] = c;
                    a *= dr;
                    c *= dz / (i + 1.0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kOut; ++u) {
                int e = base + threadIdx.x + u * 256;
                if (e < nout) {
                    int c = (base == 0) ? oc[u] : e / P;
                    int i = oi[u], j = oj[u];
                    if (base != 0) {
                        int p = e - c * P;
                        i = 0;
                        while (p >= M + 1 - i) {
                            p -= M + 1 - i;
                            ++i;
                        }
                        j = p;
                    }
                    double2 a = acc[u];
                    for (int s = 0; s < ns; ++s) {
                        double w = pr[s][i] * pz[s][j];
                        double2 sv2 = Sg[(int64_t)(s0 + s) * C + c];
                        a.x += w * sv2.x;
                        a.y += w * sv2.y;
                    }
                    acc[u] = a;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kOut; ++u) {
            int e = base + threadIdx.x + u * 256;
            if (e < nout) mom[(int64_t)k * nout + e] = acc[u];
            acc[u] = make_double2(0.0, 0.0);
        }
    }
}

// ------------------------------------------------------------------- M2M
// parent s_ij = sum_children sum_a C(i,a) dr^(i-a) 2^-a sum_b dz^(j-b)/(j-b)! 2^-b s'_ab
// with dr, dz = +-1/4 (child centre - parent centre in parent units).
__global__ __launch_bounds__(256) void k_m2m(int M, int C, int level, const int32_t *__restrict__ pboxes,
                                            const int32_t *__restrict__ cslot,
                                            const double2 *__restrict__ cmom, double2 *__restrict__ pmom)
{
    __shared__ double cfr[2][AXF_MAX_ORDER + 1][AXF_MAX_ORDER + 1];
    __shared__ double cfz[2][AXF_MAX_ORDER + 1][AXF_MAX_ORDER + 1];
    const int P = (M + 1) * (M + 2) / 2;
    const int k = blockIdx.x;
    const int b = pboxes[k];
    const int nb = 1 << level;
    const int ir = b / nb, iz = b - ir * nb;
    for (int e = threadIdx.x; e < 2 * (M + 1) * (M + 1); e += blockDim.x) {
        int sg = e / ((M + 1) * (M + 1)), rem = e - sg * (M + 1) * (M + 1);
        int i = rem / (M + 1), a = rem - i * (M + 1);
        double d = sg ? 0.25 : -0.25;
        double vr = 0.0, vz = 0.0;
        if (a <= i) {
            double bin = 1.0, pw = 1.0, fct = 1.0;
            for (int t = 0; t < a; ++t) bin = bin * (i - t) / (t + 1.0);
            for (int t = 0; t < i - a; ++t) {
                pw *= d;
                fct *= (t + 1.0);
            }
            double two = ldexp(1.0, -a);
            vr = bin * pw * two;
            vz = pw / fct * two;
        }
        cfr[sg][i][a] = vr;
        cfz[sg][i][a] = vz;
    }
    __syncthreads();
    const int cnb = nb * 2;
    int cs[4];
    for (int ch = 0; ch < 4; ++ch) {
        int cr = ch >> 1, cz = ch & 1;
        cs[ch] = cslot[(2 * ir + cr) * cnb + (2 * iz + cz)];
    }
    const int nout = C * P;
    for (int e = threadIdx.x; e < nout; e += blockDim.x) {
        int c = e / P, p = e - c * P;
        int i = 0;
        while (p >= M + 1 - i) {
            p -= M + 1 - i;
            ++i;
        }
        int j = p;
        double2 acc = make_double2(0.0, 0.0);
        for (int ch = 0; ch < 4; ++ch) {
            if (cs[ch] < 0) continue;
            int sr = ch >> 1, sz = ch & 1;
            const double2 *src = cmom + ((int64_t)cs[ch] * C + c) * P;
            for (int a = 0; a <= i; ++a) {
                double fr = cfr[sr][i][a];
                int rowa = tri_index(M, a, 0);
                for (int bb = 0; bb <= j; ++bb) {
                    double w = fr * cfz[sz][j][bb];
                    double2 v = src[rowa + bb];
                    acc.x += w * v.x;
                    acc.y += w * v.y;
                }
            }
        }
        pmom[(int64_t)k * nout + e] = acc;
    }
}

// --------------------------------------------------------- L2L + S2L
// One block per (occupied target box, mode).
__global__ __launch_bounds__(256) void k_s2l(int M, int nmodes, int nrhs, int level, int TS,
                                            const int32_t *__restrict__ tboxes,
                                            const int32_t *__restrict__ tslot_parent,
                                            const double2 *__restrict__ ploc,
                                            const int32_t *__restrict__ sslot,
                                            const double2 *__restrict__ mom,
                                            const double *__restrict__ tab,
                                            double2 *__restrict__ loc)
{
    extern __shared__ double2 ms[];          // [nrhs][P] staged moments
    __shared__ double lcoef[2][AXF_MAX_ORDER + 1][AXF_MAX_ORDER + 1];   // L2L factors
    __shared__ double invfact[AXF_MAX_ORDER + 1];
    const int P = (M + 1) * (M + 2) / 2;
    const int C = nmodes * nrhs;
    const int k = blockIdx.x / nmodes, n = blockIdx.x - (blockIdx.x / nmodes) * nmodes;
    const int b = tboxes[k];
    const int nb = 1 << level;
    const int ir = b / nb, iz = b - ir * nb;
    const int tid = threadIdx.x;

    if (tid <= M) {
        double f = 1.0;
        for (int t = 2; t <= tid; ++t) f *= t;
        invfact[tid] = 1.0 / f;
    }
    // L2L factors: C(i+q, q) d^q 2^-(i) for d = -1/4, +1/4 (child - parent, parent units)
    for (int e = tid; e < 2 * (M + 1) * (M + 1); e += blockDim.x) {
        int sg = e / ((M + 1) * (M + 1)), rem = e - sg * (M + 1) * (M + 1);
        int i = rem / (M + 1), q = rem - i * (M + 1);
        double d = sg ? 0.25 : -0.25;
        double v = 0.0;
        if (i + q <= M) {
            double bin = 1.0;
            for (int t = 0; t < q; ++t) bin = bin * (i + q - t) / (t + 1.0);
            double pw = 1.0;
            for (int t = 0; t < q; ++t) pw *= d;
            v = bin * pw * ldexp(1.0, -i);
        }
        lcoef[sg][i][q] = v;
    }
    // outputs of this thread
    int ok[2], ol[2];
    bool act[2];
    for (int u = 0; u < 2; ++u) {
        int p = tid + u * 256;
        act[u] = p < P;
        int kk = 0;
        if (act[u]) {
            while (p >= M + 1 - kk) {
                p -= M + 1 - kk;
                ++kk;
            }
        }
        ok[u] = kk;
        ol[u] = act[u] ? p : 0;
    }
    double2 acc[2][kMaxRhs];
    for (int u = 0; u < 2; ++u)
        for (int q = 0; q < kMaxRhs; ++q) acc[u][q] = make_double2(0.0, 0.0);
    __syncthreads();

    const double *tab_n = tab + (size_t)n * TS;
    const int jr0 = 2 * (ir >> 1) - 2, jz0 = 2 * (iz >> 1) - 2;
    for (int jr = jr0; jr < jr0 + 6; ++jr) {
        if (jr < 0 || jr >= nb) continue;
        for (int jz = jz0; jz < jz0 + 6; ++jz) {
            if (jz < 0 || jz >= nb) continue;
            if (abs(jr - ir) <= 1 && abs(jz - iz) <= 1) continue;
            int ss = sslot[jr * nb + jz];
            if (ss < 0) continue;
            __syncthreads();
            for (int e = tid; e < nrhs * P; e += blockDim.x) {
                int q = e / P, p = e - q * P;
                ms[e] = mom[((int64_t)ss * C + n * nrhs + q) * P + p];
            }
            __syncthreads();
            const bool outward = jr <= ir;
            const int station = outward ? jr : ir;
            const int dr = outward ? ir - jr : jr - ir;
            const int dz = abs(iz - jz);
            const bool fwd = iz >= jz;
            const double *T = tab_n + ((size_t)station * 12 + geom_slot(dr, dz)) * nmodes * (size_t)TS;
            for (int u = 0; u < 2; ++u) {
                if (!act[u]) continue;
                const int kk = ok[u], ll = ol[u];
                for (int i = 0; i <= M; ++i) {
                    const double *row = T + (outward ? table_row(M, kk, i) : table_row(M, i, kk));
                    const int pbase = tri_index(M, i, 0);
                    for (int j = 0; j + i <= M; ++j) {
                        int c = j + ll;
                        double tv = row[c];
                        if (fwd && (c & 1)) tv = -tv;
                        for (int q = 0; q < nrhs; ++q) {
                            double2 s = ms[q * P + pbase + j];
                            acc[u][q].x += tv * s.x;
                            acc[u][q].y += tv * s.y;
                        }
                    }
                }
            }
        }
    }
    // combine with the parent's shifted local expansion (eq. analysis:l2l)
    int pslot = -1;
    if (level > 2) pslot = tslot_parent[(ir >> 1) * (nb >> 1) + (iz >> 1)];
    const int sr = ir & 1, sz = iz & 1;
    for (int u = 0; u < 2; ++u) {
        if (!act[u]) continue;
        const int kk = ok[u], ll = ol[u];
        const double f = ((ll & 1) ? -1.0 : 1.0) * invfact[ll];
        for (int q = 0; q < nrhs; ++q) {
            double2 v = make_double2(f * acc[u][q].x, f * acc[u][q].y);
            if (pslot >= 0) {
                const double2 *pl = ploc + ((int64_t)pslot * C + n * nrhs + q) * P;
                for (int a = 0; kk + a <= M; ++a) {
                    double fa = lcoef[sr][kk][a];
                    for (int c2 = 0; kk + a + ll + c2 <= M; ++c2) {
                        double w = fa * lcoef[sz][ll][c2];
                        double2 x = pl[tri_index(M, kk + a, ll + c2)];
                        v.x += w * x.x;
                        v.y += w * x.y;
                    }
                }
            }
            loc[((int64_t)k * C + n * nrhs + q) * P + tri_index(M, kk, ll)] = v;
        }
    }
}

// ------------------------------------------------------------ leaf pass
// One wave per chunk of <= 64 targets of one leaf: local expansion
// (eq. analysis:local) plus the direct sum over the 3x3 neighbour leaves.
// MODE 0: potential; 1: potential and gradient; 2: potential and the
// adjoint coordinate contraction.
template <int NMB, int MODE>
__global__ __launch_bounds__(64) void k_leaf(int M, int nmodes, int nrhs, int depth, double rlo, double zlo,
                                            double invh, double chistar, const int4 *__restrict__ chunks,
                                            SideView tv, SideView sv, const double2 *__restrict__ Sg,
                                            const double2 *__restrict__ loc, double2 *__restrict__ phi,
                                            double2 *__restrict__ dphr, double2 *__restrict__ dphz,
                                            const double2 *__restrict__ Sdot, double *__restrict__ gr,
                                            double *__restrict__ gz, int64_t ntot)
{
    const int4 ch = chunks[blockIdx.x];
    const int lane = threadIdx.x;
    const bool active = lane < ch.z;
    const int t = ch.y + (active ? lane : 0);
    const int nb = 1 << depth;
    const int ir = ch.w / nb, iz = ch.w - (ch.w / nb) * nb;
    const int P = (M + 1) * (M + 2) / 2;
    const int C = nmodes * nrhs;
    const double r = tv.r[t], z = tv.z[t];
    const double xr = (r - rlo) * invh - (ir + 0.5);
    const double xz = (z - zlo) * invh - (iz + 0.5);
    const double inv_r = 1.0 / r;
    const int orig = tv.perm[t];
    double gsr = 0.0, gsz = 0.0;
    for (int q = 0; q < nrhs; ++q) {
        double ar[NMB], ai[NMB];
        double drr[MODE ? NMB : 1], dri[MODE ? NMB : 1], dzr[MODE ? NMB : 1], dzi[MODE ? NMB : 1];
#pragma unroll
        for (int n = 0; n < NMB; ++n) {
            ar[n] = ai[n] = 0.0;
            if constexpr (MODE != 0) drr[n] = dri[n] = dzr[n] = dzi[n] = 0.0;
        }
        // local expansion
        const double2 *lc = loc + (int64_t)ch.x * C * P;
        {
            double pr = 1.0, pr1 = 0.0;   // xr^k, k xr^(k-1)
            int p = 0;
            for (int kk = 0; kk <= M; ++kk) {
                double pz = 1.0, pz1 = 0.0;
                for (int ll = 0; kk + ll <= M; ++ll, ++p) {
                    double w = pr * pz;
#pragma unroll
                    for (int n = 0; n < NMB; ++n) {
                        if (n < nmodes) {
                            double2 v = lc[(int64_t)(n * nrhs + q) * P + p];
                            ar[n] += w * v.x;
                            ai[n] += w * v.y;
                            if constexpr (MODE != 0) {
                                double wr = pr1 * pz * invh, wz = pr * pz1 * invh;
                                drr[n] += wr * v.x;
                                dri[n] += wr * v.y;
                                dzr[n] += wz * v.x;
                                dzi[n] += wz * v.y;
                            }
                        }
                    }
                    pz1 = (ll + 1) * pz;
                    pz *= xz;
                }
                pr1 = (kk + 1) * pr;
                pr *= xr;
            }
        }
        // near field
        for (int jr = max(ir - 1, 0); jr <= min(ir + 1, nb - 1); ++jr) {
            for (int jz = max(iz - 1, 0); jz <= min(iz + 1, nb - 1); ++jz) {
                const uint32_t m = morton((uint32_t)jr, (uint32_t)jz);
                const int s0 = sv.off[m], s1 = sv.off[m + 1];
                for (int s = s0; s < s1; ++s) {
                    const double r1 = sv.r[s], z1 = sv.z[s];
                    const double dr = r - r1, x = z - z1, sr = r + r1;
                    double rm2 = dr * dr + x * x;
                    const double rp2 = sr * sr + x * x;
                    const bool use = active && rm2 != 0.0;
                    if (!use) rm2 = rp2 > 0.0 ? rp2 : 1.0;
                    const double rr = r * r1, inv_rr = inv_r / r1;
                    double G[NMB];
                    green_modes<NMB>(rm2, rp2, rr, inv_rr, chistar, nmodes, G);
                    const double2 *Ss = Sg + (int64_t)s * C + q;
                    const double wgt = use ? 1.0 : 0.0;
                    if constexpr (MODE == 0) {
#pragma unroll
                        for (int n = 0; n < NMB; ++n) {
                            if (n < nmodes) {
                                double2 v = Ss[n * nrhs];
                                double g = G[n] * wgt;
                                ar[n] += g * v.x;
                                ai[n] += g * v.y;
                            }
                        }
                    } else {
                        const double iprp = 1.0 / rp2, iprm = 1.0 / rm2;
                        const double A = (r * r - r1 * r1 - x * x) * 0.5 * inv_r;
                        const double hr = -0.5 * inv_r;
#pragma unroll
                        for (int n = 0; n < NMB; ++n) {
                            if (n < nmodes) {
                                double2 v = Ss[n * nrhs];
                                double gn = G[n], gm = G[n == 0 ? (NMB > 1 ? 1 : 0) : n - 1];
                                double W = (gn + gm) * iprp + (gn - gm) * iprm;
                                double nu = n - 0.5;
                                double gdr = (hr * gn + nu * A * W) * wgt;
                                double gdx = nu * x * W * wgt;
                                double g = gn * wgt;
                                ar[n] += g * v.x;
                                ai[n] += g * v.y;
                                drr[n] += gdr * v.x;
                                dri[n] += gdr * v.y;
                                dzr[n] += gdx * v.x;
                                dzi[n] += gdx * v.y;
                            }
                        }
                    }
                }
            }
        }
        if (active) {
#pragma unroll
            for (int n = 0; n < NMB; ++n) {
                if (n < nmodes) {
                    int64_t o = ((int64_t)q * nmodes + n) * ntot + orig;
                    phi[o] = make_double2(ar[n], ai[n]);
                    if constexpr (MODE == 1) {
                        if (dphr) dphr[o] = make_double2(drr[n], dri[n]);
                        if (dphz) dphz[o] = make_double2(dzr[n], dzi[n]);
                    }
                    if constexpr (MODE == 2) {
                        double2 s = Sdot[o];
                        gsr += s.x * drr[n] + s.y * dri[n];
                        gsz += s.x * dzr[n] + s.y * dzi[n];
                    }
                }
            }
        }
    }
    if constexpr (MODE == 2) {
        if (active) {
            if (gr) gr[orig] = gsr;
            if (gz) gz[orig] = gsz;
        }
    }
}

// ---------------------------------------------------------------- direct
template <int NMB>
__global__ __launch_bounds__(256) void k_direct(int nmodes, int nrhs, double chistar, SideView tv, int64_t nt,
                                               SideView sv, int64_t ns, const double2 *__restrict__ Sg,
                                               double2 *__restrict__ phi)
{
    const int64_t tg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool active = tg < nt;
    const int64_t t = active ? tg : 0;
    const int C = nmodes * nrhs;
    const double r = tv.r[t], z = tv.z[t];
    const double inv_r = 1.0 / r;
    for (int q = 0; q < nrhs; ++q) {
        double ar[NMB], ai[NMB];
#pragma unroll
        for (int n = 0; n < NMB; ++n) ar[n] = ai[n] = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            const double r1 = sv.r[s], z1 = sv.z[s];
            const double dr = r - r1, x = z - z1, sr = r + r1;
            double rm2 = dr * dr + x * x;
            const double rp2 = sr * sr + x * x;
            const bool use = rm2 != 0.0;
            if (!use) rm2 = rp2;
            double G[NMB];
            green_modes<NMB>(rm2, rp2, r * r1, inv_r / r1, chistar, nmodes, G);
            const double2 *Ss = Sg + s * C + q;
            const double wgt = use ? 1.0 : 0.0;
#pragma unroll
            for (int n = 0; n < NMB; ++n) {
                if (n < nmodes) {
                    double2 v = Ss[n * nrhs];
                    double g = G[n] * wgt;
                    ar[n] += g * v.x;
                    ai[n] += g * v.y;
                }
            }
        }
        if (active) {
            const int orig = tv.perm[t];
#pragma unroll
            for (int n = 0; n < NMB; ++n)
                if (n < nmodes) phi[((int64_t)q * nmodes + n) * nt + orig] = make_double2(ar[n], ai[n]);
        }
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

template <int NMB>
void launch_leaf(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st)
{
    SideView tv = view_of(tgt), sv = view_of(src);
    double invh = (double)(1 << pl.d) * pl.invL;
    const double2 *loc = pl.lev[pl.d].loc;
    dim3 g(tgt.nchunks);
    auto *phi = (double2 *)out.phi;
    if (out.mode == 0)
        k_leaf<NMB, 0><<<g, 64, 0, st>>>(pl.M, pl.nmodes, pl.nrhs, pl.d, pl.rlo, pl.zlo, invh, pl.chistar,
                                         tgt.chunks, tv, sv, pl.Sg, loc, phi, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, tgt.n);
    else if (out.mode == 1)
        k_leaf<NMB, 1><<<g, 64, 0, st>>>(pl.M, pl.nmodes, pl.nrhs, pl.d, pl.rlo, pl.zlo, invh, pl.chistar,
                                         tgt.chunks, tv, sv, pl.Sg, loc, phi, (double2 *)out.dr,
                                         (double2 *)out.dz, nullptr, nullptr, nullptr, tgt.n);
    else
        k_leaf<NMB, 2><<<g, 64, 0, st>>>(pl.M, pl.nmodes, pl.nrhs, pl.d, pl.rlo, pl.zlo, invh, pl.chistar,
                                         tgt.chunks, tv, sv, pl.Sg, loc, phi, nullptr, nullptr,
                                         (const double2 *)out.Sdot, out.gr, out.gz, tgt.n);
}

template <int NMB>
void launch_direct(Plan &pl, const Side &src, const Side &tgt, const EvalOut &out, hipStream_t st)
{
    SideView tv = view_of(tgt), sv = view_of(src);
    int g = (int)((tgt.n + 255) / 256);
    k_direct<NMB><<<g, 256, 0, st>>>(pl.nmodes, pl.nrhs, pl.chistar, tv, tgt.n, sv, src.n, pl.Sg,
                                      (double2 *)out.phi);
}

#define AXF_BUCKETS(X) X(8) X(16) X(24) X(32) X(40) X(64)

}  // namespace

void run_fmm(Plan &pl, const Side &src, const Side &tgt, const double *S, const EvalOut &out, hipStream_t st)
{
    const int M = pl.M, P = pl.P, C = pl.C, d = pl.d;
    const int64_t ns = src.n;
    {
        int64_t tot = ns * C;
        k_gather<<<(int)((tot + 255) / 256), 256, 0, st>>>((const double2 *)S, src.perm, ns, pl.nmodes, pl.nrhs,
                                                          pl.Sg);
    }
    SideView sv = view_of(src);
    if (src.nocc[d] > 0)
        k_p2m<<<src.nocc[d], 256, 0, st>>>(M, C, d, pl.rlo, pl.zlo, (double)(1 << d) * pl.invL, sv, src.box[d],
                                           pl.Sg, pl.lev[d].mom);
    for (int l = d - 1; l >= 2; --l)
        if (src.nocc[l] > 0)
            k_m2m<<<src.nocc[l], 256, 0, st>>>(M, C, l, src.box[l], src.slot[l + 1], pl.lev[l + 1].mom,
                                               pl.lev[l].mom);
    for (int l = 2; l <= d; ++l) {
        if (tgt.nocc[l] == 0) continue;
        size_t shm = sizeof(double2) * (size_t)pl.nrhs * P;
        k_s2l<<<tgt.nocc[l] * pl.nmodes, 256, shm, st>>>(M, pl.nmodes, pl.nrhs, l, pl.TS, tgt.box[l],
                                                         l > 2 ? tgt.slot[l - 1] : nullptr,
                                                         l > 2 ? pl.lev[l - 1].loc : nullptr, src.slot[l],
                                                         pl.lev[l].mom, pl.lev[l].tab, pl.lev[l].loc);
    }
    const int nm = pl.nmodes;
#define AXF_LEAF(B)                                         \
    if (nm <= B) {                                          \
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
    int64_t tot = ns * C;
    k_gather<<<(int)((tot + 255) / 256), 256, 0, st>>>((const double2 *)S, src.perm, ns, pl.nmodes, pl.nrhs, pl.Sg);
    const int nm = pl.nmodes;
#define AXF_DIR(B)                                          \
    if (nm <= B) {                                          \
        launch_direct<B>(pl, src, tgt, out, st);            \
        AXF_HIP(hipGetLastError());                         \
        return;                                             \
    }
    AXF_BUCKETS(AXF_DIR)
#undef AXF_DIR
}

}  // namespace axf

// axf_tables.hip -- S2L Taylor tables of the modal Green's function (App. A).
//
// For every level l, inner radial station s and separation (dr, dz) of the
// twelve in section 2.2 (0 <= dr, dz <= 3, not both <= 1), the table holds
//     T_{a,b,c} = c! * gbar_{a,b,c}(r_out, r_in, x) * h^(a+b+c),
// a, b <= M, a + b + c <= 2M, where gbar is the normalised derivative of
// eq. gfunc:gnbar, r_in is the centre of station s, r_out = r_in + dr h,
// x = dz h.  By eq. gfunc:scaled the table is computed in box units
// (r / h) and divided by h.  Starting values follow eq. gfunc:derivatives:x
// and its r, r1 and mixed companions (the rational factors' x-derivatives are
// taken from powers of w = x - i c, c = r +- r1); the remaining entries come
// from the Laplace equation (eq. gfunc:laplace) by Leibniz' rule:
//   (i+1)(i+2) g_{i+2,j,k} = sum_{u<=i} (-1)^u r^-(u+1) [(u+1) n^2/r g_{i-u,j,k}
//                            - (i-u+1) g_{i-u+1,j,k}] - (k+1)(k+2) g_{i,j,k+2}
// and its r <-> r1 image.  (The printed recursion lacks the last term.)
#include <cmath>
#include <vector>

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

namespace {

struct GeomDesc {
    double rout, rin, x, invh;   // box units; invh = 1 / h
};

// G^(n)(r, r1, x), n = 0..N, one thread: AGM start values, forward recursion
// for chi < chistar, otherwise backward recursion on ratios normalised by G^(0).
__device__ void green_scalar(int N, double r, double r1, double x, double chistar, double *G)
{
    double dr = r - r1, sr = r + r1;
    double rm2 = dr * dr + x * x, rp2 = sr * sr + x * x;
    double rr = r * r1;
    double rp = sqrt(rp2), rm = sqrt(rm2);
    double a = rp, b = rm, c = 2.0 * rr / (rp + rm), csum = c * c, w = 1.0;
    for (int it = 0; it < 48; ++it) {
        double an = 0.5 * (a + b);
        b = sqrt(a * b);
        a = an;
        if (c <= 0x1p-30 * a) break;
        c = 0.5 * (a - b);
        w *= 2.0;
        csum = fma(w * c, c, csum);
    }
    double g0 = 0.5 / a;
    G[0] = g0;
    if (N < 1) return;
    double chi = (rp2 + rm2) / (4.0 * rr);
    if (chi < chistar) {
        G[1] = g0 * csum / (2.0 * rr);
        for (int n = 1; n < N; ++n)
            G[n + 1] = (4.0 * n * chi * G[n] - (2.0 * n - 1.0) * G[n - 1]) / (2.0 * n + 1.0);
    } else {
        double dchi = rm2 / (2.0 * rr);
        int ntop = N + 10 + (int)ceil(20.0 / sqrt(2.0 * dchi));
        if (ntop > kMillerMax) ntop = kMillerMax;
        // t = G^(n) / G^(n-1) for n = ntop .. 1
        double t = 0.0;
        for (int n = ntop; n >= 1; --n) {
            t = (2.0 * n - 1.0) / (4.0 * n * chi - (2.0 * n + 1.0) * t);
            if (n <= N) G[n] = t;   // ratio, turned into values below
        }
        for (int n = 1; n <= N; ++n) G[n] *= G[n - 1];
    }
}

constexpr int kStartThreads = 128;   // >= AXF_MAX_MODES + 1

// Starting columns g_{0,0,k}, g_{1,0,k}, g_{0,1,k}, g_{1,1,k} for all modes of
// one geometry; out layout [geom][n][4][2M+1].
__global__ __launch_bounds__(kStartThreads) void k_tab_start(int M, int nmodes, double chistar,
                                                            const GeomDesc *__restrict__ geoms,
                                                            double *__restrict__ out)
{
    extern __shared__ double sm[];
    const int K = 2 * M;
    const int Nw = nmodes - 1 < 1 ? 1 : nmodes - 1;   // g^(-1) = g^(1) needs mode 1
    const int L = K + 2;
    double *fp = sm, *fm = fp + L, *pp = fm + L, *pm = pp + L, *qp = pm + L, *qm = qp + L;
    double *dp = qm + L, *dm = dp + L;
    double *g00 = dm + L;                      // [Nw+1][L]
    double *g01 = g00 + (Nw + 1) * L;
    double *g10 = g01 + (Nw + 1) * L;
    double *g11 = g10 + (Nw + 1) * L;
    const GeomDesc gd = geoms[blockIdx.x];
    const double r = gd.rout, r1 = gd.rin, x = gd.x;
    const int t = threadIdx.x;
    if (t == 0) {
        double G[AXF_MAX_MODES + 1];
        green_scalar(Nw, r, r1, x, chistar, G);
        for (int n = 0; n <= Nw; ++n) g00[n * L] = G[n];
        // (1/q!) d^q/dx^q of x/rho^2 = (-1)^q Re w^-(q+1),
        // (r^2 - r1^2 - x^2)/rho^2 = -1 + 2 r Im w^-1, its r1-derivative
        // +-2 r Re w^-2 (+ for rho+, - for rho-), w = x - i (r +- r1).
        for (int sgn = 0; sgn < 2; ++sgn) {
            double cc = sgn == 0 ? r + r1 : r - r1;
            double den = x * x + cc * cc;
            double ire = x / den, iim = cc / den;   // 1/w
            double pre = ire, pim = iim;            // running w^-(q+1)
            double *f = sgn == 0 ? fp : fm, *p = sgn == 0 ? pp : pm, *q = sgn == 0 ? qp : qm;
            double *dd = sgn == 0 ? dp : dm;
            double wre = 0, wim = 0;                // w^-(q+2)
            wre = pre * ire - pim * iim;
            wim = pre * iim + pim * ire;
            for (int k = 0; k <= K; ++k) {
                double s = (k & 1) ? -1.0 : 1.0;
                f[k] = s * pre;
                p[k] = (k == 0 ? -1.0 : 0.0) + 2.0 * r * s * pim;
                // r <-> r1 exchange: c+ unchanged, c- -> -c- (conjugates w-)
                q[k] = (k == 0 ? -1.0 : 0.0) + (sgn == 0 ? 2.0 : -2.0) * r1 * s * pim;
                dd[k] = (sgn == 0 ? 2.0 : -2.0) * r * s * (k + 1.0) * wre;
                double nre = pre * ire - pim * iim, nim = pre * iim + pim * ire;
                pre = nre;
                pim = nim;
                double mre = wre * ire - wim * iim, mim = wre * iim + wim * ire;
                wre = mre;
                wim = mim;
            }
        }
    }
    __syncthreads();
    // x-derivatives, k-outer, n-inner (eq. gfunc:derivatives:x)
    for (int k = 0; k < K; ++k) {
        if (t <= Nw) {
            int nm = t == 0 ? 1 : t - 1;
            double s = 0.0;
            for (int q = 0; q <= k; ++q) {
                double a = g00[t * L + k - q], b = g00[nm * L + k - q];
                s += (a + b) * fp[q] + (a - b) * fm[q];
            }
            g00[t * L + k + 1] = (t - 0.5) * s / (k + 1.0);
        }
        __syncthreads();
    }
    if (M >= 1) {
        if (t <= Nw) {
            int nm = t == 0 ? 1 : t - 1;
            for (int k = 0; k <= K - 1; ++k) {
                double s1 = 0.0, s2 = 0.0;
                for (int q = 0; q <= k; ++q) {
                    double a = g00[t * L + k - q], b = g00[nm * L + k - q];
                    s1 += (a + b) * pp[q] + (a - b) * pm[q];
                    s2 += (a + b) * qp[q] + (a - b) * qm[q];
                }
                double g = g00[t * L + k];
                g10[t * L + k] = (-g + (t - 0.5) * s1) / (2.0 * r);
                g01[t * L + k] = (-g + (t - 0.5) * s2) / (2.0 * r1);
            }
        }
        __syncthreads();
        if (t <= Nw) {
            int nm = t == 0 ? 1 : t - 1;
            for (int k = 0; k <= K - 2; ++k) {
                double s = 0.0;
                for (int q = 0; q <= k; ++q) {
                    double a = g00[t * L + k - q], b = g00[nm * L + k - q];
                    double e = g01[t * L + k - q], f = g01[nm * L + k - q];
                    s += (a + b) * dp[q] + (e + f) * pp[q] + (a - b) * dm[q] + (e - f) * pm[q];
                }
                g11[t * L + k] = (-g01[t * L + k] + (t - 0.5) * s) / (2.0 * r);
            }
        }
        __syncthreads();
    }
    for (int e = t; e < nmodes * 4 * (K + 1); e += blockDim.x) {
        int n = e / (4 * (K + 1)), rem = e - n * 4 * (K + 1), col = rem / (K + 1), k = rem - col * (K + 1);
        const double *src = col == 0 ? g00 : col == 1 ? g10 : col == 2 ? g01 : g11;
        bool ok = (col == 0) || (col < 3 && k <= K - 1) || (col == 3 && k <= K - 2);
        out[(size_t)blockIdx.x * nmodes * 4 * (K + 1) + e] = (ok && M >= (col == 0 ? 0 : 1)) ? src[n * L + k] : 0.0;
    }
}

// Laplace recursion for one (geometry, mode) in LDS; writes the scaled table.
__global__ __launch_bounds__(256) void k_tab_laplace(int M, int nmodes, const GeomDesc *__restrict__ geoms,
                                                    const double *__restrict__ start,
                                                    double *__restrict__ tab)
{
    extern __shared__ double t[];      // (M+1)^3 compact entries
    __shared__ double ipr[AXF_MAX_ORDER + 2], ipr1[AXF_MAX_ORDER + 2], fact[2 * AXF_MAX_ORDER + 2];
    const int K = 2 * M;
    const int g = blockIdx.x / nmodes, n = blockIdx.x - g * nmodes;
    const GeomDesc gd = geoms[g];
    const double r = gd.rout, r1 = gd.rin;
    const double n2 = (double)n * n;
    const int tid = threadIdx.x;
    if (tid == 0) {
        double a = 1.0 / r, b = 1.0 / r1, pa = a, pb = b;
        for (int u = 0; u <= M; ++u) {
            ipr[u] = pa;
            ipr1[u] = pb;
            pa *= a;
            pb *= b;
        }
        double f = 1.0;
        for (int c = 0; c <= K; ++c) {
            fact[c] = f;
            f *= (c + 1.0);
        }
    }
    const double *st = start + ((size_t)g * nmodes + n) * 4 * (K + 1);
    for (int e = tid; e < K + 1; e += blockDim.x) {
        t[table_row(M, 0, 0) + e] = st[e];
        if (M >= 1) {
            if (e <= K - 1) {
                t[table_row(M, 1, 0) + e] = st[(K + 1) + e];
                t[table_row(M, 0, 1) + e] = st[2 * (K + 1) + e];
            }
            if (e <= K - 2) t[table_row(M, 1, 1) + e] = st[3 * (K + 1) + e];
        }
    }
    __syncthreads();
    // r-recursion for b = 0, 1
    for (int i = 0; i + 2 <= M; ++i) {
        int len0 = K - i - 2 + 1, len1 = K - i - 3 + 1;
        const double inv = 1.0 / ((i + 1.0) * (i + 2.0));
        for (int e = tid; e < len0 + len1; e += blockDim.x) {
            int j = e < len0 ? 0 : 1, k = e < len0 ? e : e - len0;
            double s = 0.0;
            for (int u = 0; u <= i; ++u) {
                double term = (u + 1) * n2 * ipr[0] * t[table_row(M, i - u, j) + k]
                              - (i - u + 1) * t[table_row(M, i - u + 1, j) + k];
                s += ((u & 1) ? -ipr[u] : ipr[u]) * term;
            }
            t[table_row(M, i + 2, j) + k] = s * inv - (k + 1.0) * (k + 2.0) * inv * t[table_row(M, i, j) + k + 2];
        }
        __syncthreads();
    }
    // r1-recursion for all a
    for (int j = 0; j + 2 <= M; ++j) {
        const double inv = 1.0 / ((j + 1.0) * (j + 2.0));
        // items: a = 0..M, k = 0..K - a - j - 2
        int tot = 0;
        for (int a = 0; a <= M; ++a) tot += (K - a - j - 2 >= 0) ? (K - a - j - 1) : 0;
        for (int e = tid; e < tot; e += blockDim.x) {
            int a = 0, k = e;
            while (k >= K - a - j - 1) {
                k -= K - a - j - 1;
                ++a;
            }
            double s = 0.0;
            for (int u = 0; u <= j; ++u) {
                double term = (u + 1) * n2 * ipr1[0] * t[table_row(M, a, j - u) + k]
                              - (j - u + 1) * t[table_row(M, a, j - u + 1) + k];
                s += ((u & 1) ? -ipr1[u] : ipr1[u]) * term;
            }
            t[table_row(M, a, j + 2) + k] = s * inv - (k + 1.0) * (k + 2.0) * inv * t[table_row(M, a, j) + k + 2];
        }
        __syncthreads();
    }
    // scaled output: c! g / h
    double *out = tab + ((size_t)g * nmodes + n) * (size_t)((M + 1) * (M + 1) * (M + 1));
    const int nrow = (M + 1) * (M + 1);
    const int wid = tid >> 6, lane = tid & 63;
    for (int row = wid; row < nrow; row += blockDim.x >> 6) {
        int a = row / (M + 1), b = row - a * (M + 1);
        int base = table_row(M, a, b), len = K + 1 - a - b;
        for (int c = lane; c < len; c += 64) out[base + c] = t[base + c] * fact[c] * gd.invh;
    }
}

}  // namespace

void build_tables(Plan &pl, hipStream_t st)
{
    const int M = pl.M, K = 2 * M, nm = pl.nmodes;
    // geometry list in storage order: level, station, slot
    std::vector<GeomDesc> geoms;
    for (int l = 2; l <= pl.d; ++l) {
        int nb = 1 << l;
        double h = pl.L / nb;
        for (int s = 0; s < nb; ++s)
            for (int gs = 0; gs < 12; ++gs) {
                int dr = gs < 4 ? gs / 2 : 2 + (gs - 4) / 4;
                int dz = gs < 4 ? 2 + gs % 2 : (gs - 4) % 4;
                double rin = pl.rlo / h + s + 0.5;
                GeomDesc g;
                g.rin = rin;
                g.rout = rin + dr;
                g.x = dz;
                g.invh = 1.0 / h;
                geoms.push_back(g);
            }
    }
    const int ng = (int)geoms.size();
    const size_t TS = (size_t)(M + 1) * (M + 1) * (M + 1);
    // scratch (plan arena): geometry descriptors and starting columns
    GeomDesc *dgeo = reinterpret_cast<GeomDesc *>(pl.tab_scratch);
    double *dstart = reinterpret_cast<double *>(pl.tab_scratch) + 4 * (size_t)ng;
    AXF_HIP(hipMemcpyAsync(dgeo, geoms.data(), sizeof(GeomDesc) * ng, hipMemcpyHostToDevice, st));
    const int Nw = nm - 1 < 1 ? 1 : nm - 1;
    size_t sm_start = sizeof(double) * ((size_t)8 * (K + 2) + (size_t)4 * (Nw + 1) * (K + 2));
    size_t sm_lap = sizeof(double) * TS;
    static bool attr_done[64] = {};
    if (!attr_done[pl.device & 63]) {
        AXF_HIP(hipFuncSetAttribute((const void *)k_tab_laplace, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    sizeof(double) * (AXF_MAX_ORDER + 1) * (AXF_MAX_ORDER + 1) * (AXF_MAX_ORDER + 1)));
        AXF_HIP(hipFuncSetAttribute((const void *)k_tab_start, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    sizeof(double) * (8 * (2 * AXF_MAX_ORDER + 2) +
                                                      4 * (AXF_MAX_MODES + 1) * (2 * AXF_MAX_ORDER + 2))));
        attr_done[pl.device & 63] = true;
    }
    k_tab_start<<<ng, kStartThreads, sm_start, st>>>(M, nm, pl.chistar, dgeo, dstart);
    // tables of level l start at geometry index 12 * (2^l - 4)
    double *tab = pl.lev[2].tab;
    k_tab_laplace<<<ng * nm, 256, sm_lap, st>>>(M, nm, dgeo, dstart, tab);
    AXF_HIP(hipGetLastError());
    // the host geometry list must outlive the copy
    AXF_HIP(hipStreamSynchronize(st));
    (void)TS;
}

size_t table_scratch_doubles(int d, int M, int nmodes)
{
    size_t ng = 12 * (((size_t)1 << (d + 1)) - 4);
    return 4 * ng + ng * (size_t)nmodes * 4 * (2 * M + 1);
}

}  // namespace axf

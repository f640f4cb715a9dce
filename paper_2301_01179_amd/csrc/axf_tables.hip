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
// from the Laplace equation (eq. gfunc:laplace), here multiplied by r^2 so
// that each entry needs five earlier ones (see k_tab_laplace), in r for the
// columns b <= 1 and then in r1 for all a.  (The paper's form, divided by r,
// is the Leibniz expansion of 1/r and 1/r^2; its printed version lacks the
// axial term (k+1)(k+2) g_{i,j,k+2}.)
#include <cstring>
#include <cmath>
#include <vector>

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

namespace {

struct GeomDesc {
    double rout, rin, x, invh;   // box units; invh = 1 / h
    double slot;                 // table slot in the level-major storage
};

// ------------------------------------------------------- double-double
// The starting columns are built from sums and differences of neighbouring
// modes, g^n +- g^(n-1).  Where n x / r is small (boxes far from the axis
// relative to their separation) the modes agree to many digits and the
// x recurrence amplifies rounding by up to ~1e14 at order 48, so G^(n), the
// rational-factor coefficients and the starting recurrences run in
// double-double arithmetic (an unevaluated sum hi + lo, ~106 bits): the
// error-free transformations TwoSum (Knuth) and TwoProduct via fma, with
// the accurate addition of Hida, Li and Bailey's double-double library.
// The Laplace recursion that fills the rest of a table is well conditioned
// and runs in FP64.
//
// The error terms are exact only if every product and sum is rounded on
// its own: floating-point contraction (fusing a*b + c into one fma across
// statements) is switched off for this file, and fma is written out where
// it is meant.
#pragma clang fp contract(off)
struct dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd dd_two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ __forceinline__ dd dd_fast_sum(double a, double b)   // |a| >= |b|
{
    double s = a + b;
    return {s, b - (s - a)};
}
__host__ __device__ __forceinline__ dd dd_d(double a) { return {a, 0.0}; }
__host__ __device__ __forceinline__ dd dd_prod(double a, double b)
{
    double p = a * b;
    return {p, fma(a, b, -p)};
}
__host__ __device__ __forceinline__ dd operator+(dd a, dd b)
{
    dd s = dd_two_sum(a.hi, b.hi), t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_fast_sum(s.hi, s.lo);
    s.lo += t.lo;
    return dd_fast_sum(s.hi, s.lo);
}
__host__ __device__ __forceinline__ dd operator-(dd a) { return {-a.hi, -a.lo}; }
__host__ __device__ __forceinline__ dd operator-(dd a, dd b) { return a + (-b); }
__host__ __device__ __forceinline__ dd operator*(dd a, dd b)
{
    dd p = dd_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return dd_fast_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd operator*(dd a, double b)
{
    dd p = dd_prod(a.hi, b);
    p.lo = fma(a.lo, b, p.lo);
    return dd_fast_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd operator/(dd a, dd b)
{
    double q1 = a.hi / b.hi;
    dd r = a - b * q1;
    double q2 = r.hi / b.hi;
    r = r - b * q2;
    double q3 = r.hi / b.hi;
    dd q = dd_fast_sum(q1, q2);
    return q + dd_d(q3);
}
__host__ __device__ __forceinline__ dd dd_sqrt(dd a)
{
    if (a.hi <= 0.0) return dd_d(0.0);
    double x = sqrt(a.hi);
    dd x2 = dd_prod(x, x);
    double corr = ((a - x2).hi) / (2.0 * x);
    return dd_fast_sum(x, corr);
}

// Threads of k_tab_start; a mode's x-derivative sums are split over LPM
// lanes (16, or 8 above 32 modes).
constexpr int kStartThreads = 512;
__host__ __device__ inline int start_lpm(int nw1)
{
    int l = 16;
    while (l > 1 && l * nw1 > kStartThreads) l >>= 1;
    return l;
}

// G^(n)(r, r1, x), n = 0..N, in double-double (one thread): the AGM gives
// G^(0) = 1 / (2 AGM(rho+, rho-)) and G^(1) / G^(0) = sum_n 2^(n-1) c_n^2 / (2 r r1);
// forward recursion in n below chistar, otherwise backward recursion on the
// ratios G^(n) / G^(n-1) started far enough up for double-double accuracy.
__host__ __device__ void green_dd(int N, double r, double r1, double x, double chistar, dd *G, int stride)
{
    dd sr = dd_two_sum(r, r1), df = dd_two_sum(r, -r1), xx = dd_prod(x, x);
    dd rp2 = sr * sr + xx, rm2 = df * df + xx, rr = dd_prod(r, r1);
    dd a = dd_sqrt(rp2), b = dd_sqrt(rm2);
    dd c = (rr * 2.0) / (a + b);
    dd csum = c * c;
    double w = 1.0;
    for (int it = 0; it < 64; ++it) {
        dd an = (a + b) * 0.5;
        b = dd_sqrt(a * b);
        a = an;
        c = (c * c) / ((a + b) * 2.0);   // c_(n+1) = c_n^2 / (4 a_(n+1))
        w *= 2.0;
        dd t = c * c * w;
        csum = csum + t;
        if (c.hi <= 0x1p-108 * a.hi) break;   // a is within c of the AGM
    }
    dd g0 = dd_d(0.5) / a;
    G[0] = g0;
    if (N < 1) return;
    dd chi = (rp2 + rm2) / (rr * 4.0);
    if (chi.hi < chistar) {
        G[stride] = g0 * csum / (rr * 2.0);
        for (int n = 1; n < N; ++n)
            G[(n + 1) * stride] = (chi * G[n * stride] * (4.0 * n) - G[(n - 1) * stride] * (2.0 * n - 1.0)) /
                                  dd_d(2.0 * n + 1.0);
    } else {
        double dchi = (rm2 / (rr * 2.0)).hi;
        int ntop = N + 10 + (int)ceil(40.0 / sqrt(2.0 * dchi));
        dd t = dd_d(0.0);
        for (int n = ntop; n >= 1; --n) {
            t = dd_d(2.0 * n - 1.0) / (chi * (4.0 * n) - t * (2.0 * n + 1.0));
            if (n <= N) G[n * stride] = t;
        }
        for (int n = 1; n <= N; ++n) G[n * stride] = G[n * stride] * G[(n - 1) * stride];
    }
}

// Starting columns g_{0,0,k}, g_{1,0,k}, g_{0,1,k}, g_{1,1,k} for all modes of
// one geometry; out layout [geom][n][4][2M+1].  Coefficients (1/q!) d^q/dx^q
// of the rational factors: x/rho^2 = (-1)^q Re w^-(q+1) and the companions
// below come from 1/rho^2 = sum u_q t^q, whose coefficients obey the
// three-term recurrence that multiplying by rho^2(x + t) gives.
__global__ __launch_bounds__(kStartThreads) void k_tab_start(int M, int nmodes, double chistar,
                                                            const GeomDesc *__restrict__ geoms,
                                                            dd *__restrict__ hand)
{
    extern __shared__ dd smd[];
    const int K = 2 * M;
    const int Nw = nmodes - 1 < 1 ? 1 : nmodes - 1;   // g^(-1) = g^(1) needs mode 1
    const int L = K + 1;
    dd *up = smd, *um = up + L, *fp = um + L, *fm = fp + L, *pp = fm + L, *pm = pp + L, *qp = pm + L,
       *qm = qp + L, *dp = qm + L, *dm = dp + L;
    dd *g00 = dm + L;                 // [Nw+1][L]
    dd *rinv = g00 + (Nw + 1) * L;    // 1 / (k + 1), k < L
    const GeomDesc gd = geoms[blockIdx.x];
    const double r = gd.rout, r1 = gd.rin, x = gd.x;
    const int tid = threadIdx.x;
    const int lpm = start_lpm(Nw + 1);
    const int n = tid / lpm, j = tid - n * lpm;      // mode and lane within the mode
    const bool active = n <= Nw;
    const int nm = n == 0 ? 1 : n - 1;
    if (tid == 0) green_dd(Nw, r, r1, x, chistar, g00, L);
    if (tid == 64 || (tid == 0 && blockDim.x <= 64)) {
        for (int sgn = 0; sgn < 2; ++sgn) {
            dd cc = sgn == 0 ? dd_two_sum(r, r1) : dd_two_sum(r, -r1);
            dd rho2 = cc * cc + dd_prod(x, x);
            dd *u = sgn == 0 ? up : um;
            u[0] = dd_d(1.0) / rho2;
            if (K >= 1) u[1] = -(u[0] * (2.0 * x)) / rho2;
            for (int q = 2; q <= K; ++q) u[q] = -(u[q - 1] * (2.0 * x) + u[q - 2]) / rho2;
        }
    }
    __syncthreads();
    const dd A0 = dd_prod(r, r) - dd_prod(r1, r1) - dd_prod(x, x);
    const dd B0 = dd_prod(r1, r1) - dd_prod(r, r) - dd_prod(x, x);
    for (int q = tid; q <= K; q += blockDim.x) {
        rinv[q] = dd_d(1.0) / dd_d(q + 1.0);
        dd u1p = q >= 1 ? up[q - 1] : dd_d(0.0), u2p = q >= 2 ? up[q - 2] : dd_d(0.0);
        dd u1m = q >= 1 ? um[q - 1] : dd_d(0.0), u2m = q >= 2 ? um[q - 2] : dd_d(0.0);
        fp[q] = up[q] * x + u1p;
        fm[q] = um[q] * x + u1m;
        pp[q] = A0 * up[q] - u1p * (2.0 * x) - u2p;
        pm[q] = A0 * um[q] - u1m * (2.0 * x) - u2m;
        qp[q] = B0 * up[q] - u1p * (2.0 * x) - u2p;
        qm[q] = B0 * um[q] - u1m * (2.0 * x) - u2m;
    }
    __syncthreads();
    // d/dr1 of p = (r^2 - r1^2 - x^2) / rho^2: -2 r1 / rho^2 - p (d rho^2 / dr1) / rho^2
    for (int q = tid; q <= K; q += blockDim.x) {
        dd cpu = dd_d(0.0), cmu = dd_d(0.0);
        for (int s2 = 0; s2 <= q; ++s2) {
            cpu = cpu + pp[s2] * up[q - s2];
            cmu = cmu + pm[s2] * um[q - s2];
        }
        dp[q] = up[q] * (-2.0 * r1) - cpu * dd_two_sum(r, r1) * 2.0;
        dm[q] = um[q] * (-2.0 * r1) + cmu * dd_two_sum(r, -r1) * 2.0;
    }
    // x-derivatives, k-outer, n-inner (eq. gfunc:derivatives:x):
    //   g_n[k+1] = (n - 1/2)/(k+1) sum_{m<=k} (g_n[m] + g_(n-1)[m]) fp[k-m]
    //                                        + (g_n[m] - g_(n-1)[m]) fm[k-m].
    // Lane j of a mode owns the sums s_k, k = j (mod lpm); once the entries
    // of index m are known every lane adds their terms to its own sums, and
    // the owner of s_m then publishes g_n[m+1] (no cross-lane reduction).
    constexpr int kOwn = (2 * AXF_MAX_ORDER + 7) / 8;     // sums per lane (lpm >= 8 up to 64 modes)
    dd acc[kOwn];
#pragma unroll
    for (int u = 0; u < kOwn; ++u) acc[u] = dd_d(0.0);
    for (int m = 0; m < K; ++m) {
        if (active) {
            const dd a = g00[n * L + m], b = g00[nm * L + m];
            const dd sp = a + b, sm = a - b;
#pragma unroll
            for (int u = 0; u < kOwn; ++u) {
                const int k = j + u * lpm;
                if (k >= m && k < K) acc[u] = acc[u] + sp * fp[k - m] + sm * fm[k - m];
            }
            // owner of s_m: lane m mod lpm, slot m / lpm
            if (j == m % lpm) {
                dd sfin = acc[0];
#pragma unroll
                for (int u = 1; u < kOwn; ++u)
                    if (u == m / lpm) sfin = acc[u];
                g00[n * L + m + 1] = sfin * (rinv[m] * (n - 0.5));
            }
        }
        __syncthreads();
    }
    // hand the x column of every mode and the rational series to the
    // r-derivative kernel: [g00: Nw+1][fp fm pp pm qp qm dp dm][L]
    __syncthreads();
    dd *h = hand + (size_t)blockIdx.x * (Nw + 9) * L;
    for (int e = tid; e < (Nw + 1) * L; e += blockDim.x) h[e] = g00[e];
    for (int e = tid; e < 8 * L; e += blockDim.x) h[(Nw + 1) * L + e] = fp[e];   // fp..dm are contiguous
}

// Modes per block of the r-derivative kernel and its threads.
constexpr int kStartModes = 8;
constexpr int kStartRThreads = 256;

// The r- and r1-derivative columns g_{1,0,k}, g_{0,1,k} and the mixed g_{1,1,k}
// of kStartModes modes of one geometry (App. A, first-derivative starting
// formulas), from the x columns and series of k_tab_start; writes the
// starting columns [geom][n][4][2M+1] of the Laplace recursion.  Every
// (mode, k) entry is an independent sum of k + 1 terms; a thread takes the
// entries k and K - 1 - k of one mode, so every thread sums the same count.
// g_{0,1} of mode m0 - 1 (and of mode 1 for mode 0, g^(-1) = g^(1)) is
// recomputed here for the mixed column.
__global__ __launch_bounds__(kStartRThreads) void k_tab_start_r(int M, int nmodes, const GeomDesc *__restrict__ geoms,
                                                               const dd *__restrict__ hand,
                                                               double *__restrict__ out)
{
    extern __shared__ dd smr[];
    const int K = 2 * M, L = K + 1;
    const int Nw = nmodes - 1 < 1 ? 1 : nmodes - 1;
    const int ngr = (nmodes + kStartModes - 1) / kStartModes;
    const int g = blockIdx.x / ngr, grp = blockIdx.x - g * ngr;
    const int m0 = grp * kStartModes, m1 = min(m0 + kStartModes, nmodes);
    // modes whose g01 is needed: [lo, hi)
    const int lo = m0 == 0 ? 0 : m0 - 1, hi = m0 == 0 ? max(m1, 2) : m1;
    const int nw = hi - lo;
    const GeomDesc gd = geoms[g];
    const double r = gd.rout, r1 = gd.rin;
    const int tid = threadIdx.x;
    dd *g00 = smr;                               // [Nw+1][L]
    dd *fp = g00 + (Nw + 1) * L, *fm = fp + L, *pp = fm + L, *pm = pp + L, *qp = pm + L, *qm = qp + L,
       *dp = qm + L, *dm = dp + L;
    dd *S = dm + L, *D = S + nw * L;             // g00[m] +- g00[mm], m in [lo, hi)
    dd *g01 = D + nw * L;                        // [lo, hi)
    dd *S1 = g01 + nw * L, *D1 = S1 + nw * L;    // g01[m] +- g01[mm]
    const dd *h = hand + (size_t)g * (Nw + 9) * L;
    for (int e = tid; e < (Nw + 9) * L; e += blockDim.x) g00[e] = h[e];
    __syncthreads();
    for (int e = tid; e < nw * L; e += blockDim.x) {
        const int m = lo + e / L, k = e - (e / L) * L;
        const int mm = m == 0 ? 1 : m - 1;
        S[e] = g00[m * L + k] + g00[mm * L + k];
        D[e] = g00[m * L + k] - g00[mm * L + k];
    }
    __syncthreads();
    double *o = out + (size_t)g * nmodes * 4 * L;
    if (M >= 1) {
        const dd i2r = dd_d(1.0) / dd_d(2.0 * r), i2r1 = dd_d(1.0) / dd_d(2.0 * r1);
        auto g10_entry = [&](int m, int k) {
            const dd *Sm = S + (m - lo) * L, *Dm = D + (m - lo) * L;
            dd s1 = dd_d(0.0), s2 = dd_d(0.0);
            for (int q = 0; q <= k; ++q) {
                const dd sp = Sm[k - q], sm = Dm[k - q];
                s1 = s1 + sp * pp[q] + sm * pm[q];
                s2 = s2 + sp * qp[q] + sm * qm[q];
            }
            const dd gg = g00[m * L + k];
            g01[(m - lo) * L + k] = (s2 * (m - 0.5) - gg) * i2r1;
            if (m >= m0 && m < m1) o[((size_t)m * 4 + 1) * L + k] = ((s1 * (m - 0.5) - gg) * i2r).hi;
        };
        const int h10 = (K + 1) / 2;
        for (int e = tid; e < nw * h10; e += blockDim.x) {
            const int m = lo + e / h10, k = e - (e / h10) * h10;
            g10_entry(m, k);
            if (K - 1 - k != k) g10_entry(m, K - 1 - k);
        }
        __syncthreads();
        for (int e = tid; e < (m1 - m0) * (K - 1); e += blockDim.x) {
            const int m = m0 + e / (K - 1), k = e - (e / (K - 1)) * (K - 1);
            const int mm = m == 0 ? 1 : m - 1;
            S1[(m - lo) * L + k] = g01[(m - lo) * L + k] + g01[(mm - lo) * L + k];
            D1[(m - lo) * L + k] = g01[(m - lo) * L + k] - g01[(mm - lo) * L + k];
        }
        __syncthreads();
        auto g11_entry = [&](int m, int k) {
            const dd *Sm = S + (m - lo) * L, *Dm = D + (m - lo) * L;
            const dd *S1m = S1 + (m - lo) * L, *D1m = D1 + (m - lo) * L;
            dd s = dd_d(0.0);
            for (int q = 0; q <= k; ++q)
                s = s + Sm[k - q] * dp[q] + S1m[k - q] * pp[q] + Dm[k - q] * dm[q] + D1m[k - q] * pm[q];
            o[((size_t)m * 4 + 3) * L + k] = ((s * (m - 0.5) - g01[(m - lo) * L + k]) * i2r).hi;
        };
        const int h11 = K / 2;   // K - 1 entries per mode, paired
        for (int e = tid; e < (m1 - m0) * h11; e += blockDim.x) {
            const int m = m0 + e / h11, k = e - (e / h11) * h11;
            g11_entry(m, k);
            if (K - 2 - k != k) g11_entry(m, K - 2 - k);
        }
    }
    // g00, g01 and the zero tails of this block's modes
    for (int e = tid; e < (m1 - m0) * 4 * L; e += blockDim.x) {
        const int nn = m0 + e / (4 * L), rem = e - (e / (4 * L)) * 4 * L, col = rem / L, k = rem - col * L;
        const size_t oe = ((size_t)nn * 4 + col) * L + k;
        if (col == 0) {
            o[oe] = g00[nn * L + k].hi;
        } else if (col == 2) {
            o[oe] = (M >= 1 && k <= K - 1) ? g01[(nn - lo) * L + k].hi : 0.0;
        } else if (M < 1 || (col == 1 && k > K - 1) || (col == 3 && k > K - 2)) {
            o[oe] = 0.0;
        }
    }
}

size_t start_lds_bytes(int M, int nmodes)
{
    const int Nw = nmodes - 1 < 1 ? 1 : nmodes - 1;
    return sizeof(dd) * (size_t)(2 * M + 1) * (11 + (Nw + 1));
}

size_t start_r_lds_bytes(int M, int nmodes)
{
    const int Nw = nmodes - 1 < 1 ? 1 : nmodes - 1;
    const int nw = kStartModes + 1;   // the group's modes and one below (or mode 1)
    return sizeof(dd) * (size_t)(2 * M + 1) * ((Nw + 1) + 8 + 5 * nw);
}

// Laplace recursion for one (geometry, mode); writes the scaled table.
// The Laplace equation multiplied by r^2,
//   r^2 g_rr + r g_r - n^2 g + r^2 g_xx = 0,
// gives for the Taylor coefficients about r (rho = r' - r) a recursion of
// five terms (the form divided by r needs all previous rows):
//   r^2 (i+1)(i+2) g_(i+2) = -[ r (i+1)(2i+1) g_(i+1) + (i^2 - n^2) g_i
//                               + r^2 h_i + 2 r h_(i-1) + h_(i-2) ],
//   h_m = (k+1)(k+2) g_(m, k+2);  and the same in r1 for the source index.
// Each 16-lane row of a wave runs one recursion; lane l of the row holds the
// x indices k = l + 16t, t = 0..3, of the last four rows (a row's stores are
// contiguous), so the k + 2 entry is lane l + 2's element t, or for l >= 14
// lane l - 14's element t + 1: one DPP rotation of the row by two lanes.
// Two rows run the r recursions of the columns b = 0 and 1 (rows staged in
// LDS), then the 16 rows of the block share the r1 recursions, one per a.
constexpr int kLapThreads = 256;
constexpr int kLapRecs = kLapThreads / 16;      // recursions in flight per block
__device__ __forceinline__ double lap_step(double c1, double c0, double s2, double s1, double inv, double kk,
                                           double g1, double g0, double h0, double hm1, double hm2)
{
    // -(c1 g_(i+1) + c0 g_i + kk (s2 h_i + s1 h_(i-1) + h_(i-2))) / (s2 (i+1)(i+2)), inv = -1/(...)
    return (c1 * g1 + c0 * g0 + kk * (s2 * h0 + s1 * hm1 + hm2)) * inv;
}

// The value of lane (l + 2) mod 16 of the 16-lane row (DPP row_ror:14).
__device__ __forceinline__ double row_plus2(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x12e, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x12e, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// The k + 2 entries of the lane's four x indices for one row of values.
__device__ __forceinline__ void plus2(const double (&v)[4], int l16, double (&h)[4])
{
    double rot[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) rot[t] = row_plus2(v[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) h[t] = l16 < 14 ? rot[t] : (t < 3 ? rot[t + 1] : 0.0);
}

// One recursion over rows i = 0..M of a column of length K + 1 - base - i
// (base = b for the r recursion, a for the r1 one): rows 0 and 1 given, the
// rest from the Laplace step with coefficient scale rr (r or r1); each new
// row is passed to emit(i, t, value) for its valid entries.
template <class Emit>
__device__ __forceinline__ void lap_run(int M, int K, int base, double rr, double nirr, double n2,
                                        const double *rstep, double (&g0)[4], double (&g1)[4], int l16,
                                        Emit emit)
{
    double gm1[4] = {0.0, 0.0, 0.0, 0.0}, gm2[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i + 2 <= M; ++i) {
        const double c1 = rr * (i + 1.0) * (2.0 * i + 1.0), c0 = (double)i * i - n2;
        const double inv = nirr * rstep[i];
        double h0[4], hm1[4], hm2[4], gn[4];
        plus2(g0, l16, h0);
        plus2(gm1, l16, hm1);
        plus2(gm2, l16, hm2);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = l16 + 16 * t;
            const double kk = (k + 1.0) * (k + 2.0);
            gn[t] = lap_step(c1, c0, rr * rr, 2.0 * rr, inv, kk, g1[t], g0[t], h0[t], i >= 1 ? hm1[t] : 0.0,
                             i >= 2 ? hm2[t] : 0.0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = l16 + 16 * t;
            const bool valid = k <= K - base - (i + 2);
            gm2[t] = gm1[t];
            gm1[t] = g0[t];
            g0[t] = g1[t];
            g1[t] = valid ? gn[t] : 0.0;
            if (valid) emit(i + 2, t, g1[t]);
        }
    }
}

__global__ __launch_bounds__(kLapThreads) void k_tab_laplace(int M, int nmodes, const GeomDesc *__restrict__ geoms,
                                                            const double *__restrict__ start,
                                                            double *__restrict__ tab)
{
    __shared__ double col[2][AXF_MAX_ORDER + 1][2 * AXF_MAX_ORDER + 1];   // rows (a, b) for b = 0, 1
    __shared__ double fact[2 * AXF_MAX_ORDER + 2];
    __shared__ double rstep[AXF_MAX_ORDER + 1];    // 1 / ((i + 1)(i + 2))
    const int K = 2 * M;
    const int g = blockIdx.x / nmodes, n = blockIdx.x - g * nmodes;
    const GeomDesc gd = geoms[g];
    const double r = gd.rout, r1 = gd.rin;
    const double n2 = (double)n * n;
    const int tid = threadIdx.x, rec = tid >> 4, l16 = tid & 15;
    double *out = tab + ((size_t)gd.slot * nmodes + n) * (size_t)((M + 1) * (M + 1) * (M + 1));
    if (tid == 0) {
        double f = 1.0;
        for (int c = 0; c <= K; ++c) {
            fact[c] = f;
            f *= (c + 1.0);
        }
    }
    if (tid <= M) rstep[tid] = 1.0 / ((tid + 1.0) * (tid + 2.0));
    __syncthreads();
    const double nir2 = -1.0 / (r * r), nir12 = -1.0 / (r1 * r1);
    const double *st = start + ((size_t)g * nmodes + n) * 4 * (K + 1);
    // r recursion of column b (rows 0 and 1 of wave 0): rows (i, b), i = 0..M,
    // length K + 1 - i - b, staged in LDS
    if (rec < 2 && (rec == 0 || M >= 1)) {
        const int bcol = rec, len0 = K + 1 - bcol;
        double g0[4], g1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = l16 + 16 * t;
            g0[t] = k < len0 ? st[(bcol == 0 ? 0 : 2) * (K + 1) + k] : 0.0;
            g1[t] = (M >= 1 && k < len0 - 1) ? st[(bcol == 0 ? 1 : 3) * (K + 1) + k] : 0.0;
            if (k < len0) col[bcol][0][k] = g0[t];
            if (M >= 1 && k < len0 - 1) col[bcol][1][k] = g1[t];
        }
        lap_run(M, K, bcol, r, nir2, n2, rstep, g0, g1, l16,
                [&](int i, int t, double v) { col[bcol][i][l16 + 16 * t] = v; });
    }
    __syncthreads();
    // r1 recursion for each a: rows (a, j), j = 0..M, length K + 1 - a - j
    for (int a = rec; a <= M; a += kLapRecs) {
        double g0[4], g1[4], fk[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = l16 + 16 * t;
            g0[t] = k <= K - a ? col[0][a][k] : 0.0;
            g1[t] = (M >= 1 && k <= K - a - 1) ? col[1][a][k] : 0.0;
            fk[t] = k <= K ? fact[k] * gd.invh : 0.0;
            if (k <= K - a) out[table_row(M, a, 0) + k] = g0[t] * fk[t];
            if (M >= 1 && k <= K - a - 1) out[table_row(M, a, 1) + k] = g1[t] * fk[t];
        }
        lap_run(M, K, a, r1, nir12, n2, rstep, g0, g1, l16,
                [&](int j, int t, double v) { out[table_row(M, a, j) + l16 + 16 * t] = v * fk[t]; });
    }
}

}  // namespace

void build_tables(Plan &pl, hipStream_t st)
{
    const int M = pl.M, K = 2 * M, nm = pl.nmodes;
    // geometry list: station, separation; the finest level's stations of the
    // axis grid in the plan's runs when the levels share tables, else the
    // stations 0..tab_smax[l] of each level from geometry tab_base[l] on.
    // The plan keeps the list until the copy has run.
    std::vector<GeomDesc> geoms;
    auto add = [&](double rin, double h, size_t slot0) {
        for (int gs = 0; gs < 12; ++gs) {
            int dr = gs < 4 ? gs / 2 : 2 + (gs - 4) / 4;
            int dz = gs < 4 ? 2 + gs % 2 : (gs - 4) % 4;
            GeomDesc g;
            g.rin = rin;
            g.rout = rin + dr;
            g.x = dz;
            g.invh = 1.0 / h;
            g.slot = (double)(slot0 + gs);
            geoms.push_back(g);
        }
    };
    if (pl.koff >= 0) {
        // shared: the runs of finest-level stations of the axis grid
        const double h = pl.L / (1 << pl.d);
        size_t at = 0;
        for (auto &run : pl.tab_runs)
            for (int v = run.first; v <= run.second; ++v, ++at) add(v + 0.5, h, 12 * at);
    } else {
        for (int l = 2; l <= pl.d; ++l) {
            const double h = pl.L / (1 << l);
            for (int s = 0; s <= pl.tab_smax[l]; ++s) add(pl.rlo / h + s + 0.5, h, pl.tab_base[l] + (size_t)s * 12);
        }
    }
    const int ng = (int)geoms.size();
    const size_t TS = (size_t)(M + 1) * (M + 1) * (M + 1);
    // scratch (plan arena): geometry descriptors and starting columns
    GeomDesc *dgeo = reinterpret_cast<GeomDesc *>(pl.tab_scratch);
    double *dstart = reinterpret_cast<double *>(pl.tab_scratch) + 5 * (size_t)ng;
    static_assert(sizeof(GeomDesc) == 5 * sizeof(double), "geometry record");
    pl.geom_host.resize(5 * (size_t)ng);
    std::memcpy(pl.geom_host.data(), geoms.data(), sizeof(GeomDesc) * ng);
    AXF_HIP(hipMemcpyAsync(dgeo, pl.geom_host.data(), sizeof(GeomDesc) * ng, hipMemcpyHostToDevice, st));
    // x columns and series of each geometry, handed to the r-derivative kernel
    dd *hand = reinterpret_cast<dd *>(dstart + (size_t)ng * nm * 4 * (K + 1));
    static bool attr_done[64] = {};
    if (!attr_done[pl.device & 63]) {
        AXF_HIP(hipFuncSetAttribute((const void *)k_tab_start, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)start_lds_bytes(AXF_MAX_ORDER, AXF_MAX_MODES)));
        AXF_HIP(hipFuncSetAttribute((const void *)k_tab_start_r, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)start_r_lds_bytes(AXF_MAX_ORDER, AXF_MAX_MODES)));
        attr_done[pl.device & 63] = true;
    }
    k_tab_start<<<ng, kStartThreads, start_lds_bytes(M, nm), st>>>(M, nm, pl.chistar, dgeo, hand);
    const int ngr = (nm + kStartModes - 1) / kStartModes;
    k_tab_start_r<<<ng * ngr, kStartRThreads, start_r_lds_bytes(M, nm), st>>>(M, nm, dgeo, hand, dstart);
    // every geometry record carries its slot from the storage's start
    double *tab = pl.lev[2].tab - pl.tab_base[2] * (size_t)nm * TS;
    k_tab_laplace<<<ng * nm, kLapThreads, 0, st>>>(M, nm, dgeo, dstart, tab);
    AXF_HIP(hipGetLastError());
}

size_t table_scratch_doubles(size_t ng, int M, int nmodes)
{
    const size_t L = 2 * (size_t)M + 1;
    const size_t nw1 = nmodes < 2 ? 2 : nmodes;   // modes 0..Nw of the x columns
    // geometries, starting columns, and the x columns + series in double-double
    return 5 * ng + ng * (size_t)nmodes * 4 * L + ng * 2 * (nw1 + 8) * L;
}

}  // namespace axf

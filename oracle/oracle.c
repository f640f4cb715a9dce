/*
 * oracle.c -- plain FP64 CPU oracle for the axisymmetric modal FMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * CPU-baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant generator with the GPU library, and the GPU
 * library never calls it.
 *
 * Written from M. J. Carley, "A Fast Multipole Method for axisymmetric
 * domains" (arXiv 2301.01179).  Every routine cites the passage it follows.
 * It is deliberately slow and literal: no blocking, no symmetry reuse, no
 * fusion beyond what the cited equations state.
 *
 * Conventions shared with the callers (Python wrapper in oracle.py):
 *   - complex numbers are interleaved (re, im) doubles;
 *   - strengths S are laid out [nrhs][nmodes][ns], potentials [nrhs][nmodes][nf];
 *   - a source whose (r, z) equals the field point bit for bit is skipped
 *     (no self interaction; the paper is silent, its points are distinct).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   R1. The Laplace derivative recursion (App. A, eq. gfunc:laplace:recursion)
 *       as printed drops the axial term; the recursion used below is the one
 *       that follows from eq. gfunc:laplace by Leibniz' rule and contains
 *       -(k+1)(k+2) g_{i,j,k+2}.
 *   R2. Backward (Miller) recursion start: the paper starts at n = N+80; that
 *       start leaves ~1e-9 relative error just above chi = 1.008, against the
 *       paper's own claim of machine precision.  The start used here is
 *       n_top = N + max(80, ceil(20/acosh(chi)) + 10).
 *   R3. M2M / L2L displacement: delta = child centre - parent centre, with
 *       +delta powers (the paper's "-Delta" with Delta = parent - child).
 *   R4. Upward pass ends at level 2 (Algorithm 1), S2L runs on levels 2..d.
 *   R5. Domain: bounding square of all source and field points,
 *       [r_lo, r_lo+L] x [z_lo, z_lo+L], L = max(r extent, z extent)
 *       (1 if both are zero), z_lo = smallest z.  r_lo = 0 (the paper's
 *       domain 0 <= r <= r_max) when L reaches the largest radius.  Else,
 *       if k = floor(r_min / (L/4)) is 1, 2 or 3: L' = the smallest double
 *       >= max(L, r_max / (1 + k/4)) with k (L'/4) + L' >= r_max, and if
 *       k (L'/4) <= r_min the square is [k L'/4, k L'/4 + L'] of side L'
 *       (the levels' stations then sit at whole box units from the axis
 *       grid).  Else r_lo = smallest radius.  Box index
 *       floor(((r-r_lo)*(1/L))*2^l), clamped to 2^l - 1.
 *   R6. Moments i+j <= M, locals k+l <= M, derivative tables to total order
 *       2M: the S2L sum of eq. analysis:s2l runs over all i+j <= M.
 *   R7. The starting formulas of App. A (eq. gfunc:derivatives:x and its r,
 *       r1 and mixed companions) lose up to ~14 digits at high x order when
 *       n x / r is small; they are evaluated in binary128 here (the paper
 *       does not discuss their conditioning), and the Laplace recursion that
 *       continues them runs in x87 extended precision.
 *   R14. The azimuthal Fourier series (section 2, eqs. analysis:source and
 *       analysis:phi) with K equally spaced samples theta_k = 2 pi k / K:
 *       S^(n) = (1/K) sum_k s(theta_k) e^(-i n theta_k), exact for a real
 *       source of modes |n| <= N when K >= 2N + 1; and
 *       phi(theta) = Re Phi^(0) + 2 Re sum_{n >= 1} Phi^(n) e^(i n theta),
 *       which is the series over n = -N..N with Phi^(-n) = conj(Phi^(n)).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_PI 3.141592653589793238462643383279502884

/* ------------------------------------------------------------------------ */
/* Carlson's symmetric integrals by the duplication theorem (App. A names
 * Carlson's method for K and E).  Series truncation after the fifth-order
 * terms; iteration continues until every relative deviation is < 1e-3, where
 * the neglected sixth-order terms are below 1e-18. */

static double ora_rf(double x, double y, double z)
{
    for (int it = 0; it < 200; ++it) {
        double A = (x + y + z) / 3.0;
        double X = 1.0 - x / A, Y = 1.0 - y / A, Z = 1.0 - z / A;
        double dev = fmax(fabs(X), fmax(fabs(Y), fabs(Z)));
        if (dev < 1e-3) {
            double E2 = X * Y - Z * Z;
            double E3 = X * Y * Z;
            return (1.0 - E2 / 10.0 + E3 / 14.0 + E2 * E2 / 24.0
                    - 3.0 * E2 * E3 / 44.0) / sqrt(A);
        }
        double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        double lam = sx * sy + sy * sz + sz * sx;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
    }
    return NAN;
}

static double ora_rd(double x, double y, double z)
{
    double sum = 0.0, scale = 1.0;
    for (int it = 0; it < 200; ++it) {
        double A = (x + y + 3.0 * z) / 5.0;
        double X = 1.0 - x / A, Y = 1.0 - y / A, Z3 = 1.0 - z / A;
        double dev = fmax(fabs(X), fmax(fabs(Y), fabs(Z3)));
        if (dev < 1e-3) {
            double Z = -(X + Y) / 3.0;
            double XY = X * Y, Z2 = Z * Z;
            double E2 = XY - 6.0 * Z2;
            double E3 = (3.0 * XY - 8.0 * Z2) * Z;
            double E4 = 3.0 * (XY - Z2) * Z2;
            double E5 = XY * Z2 * Z;
            double ser = 1.0 - 3.0 * E2 / 14.0 + E3 / 6.0 + 9.0 * E2 * E2 / 88.0
                         - 3.0 * E4 / 22.0 - 9.0 * E2 * E3 / 52.0 + 3.0 * E5 / 26.0;
            return 3.0 * sum + scale * ser / (A * sqrt(A));
        }
        double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        double lam = sx * sy + sy * sz + sz * sx;
        sum += scale / (sz * (z + lam));
        scale *= 0.25;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
    }
    return NAN;
}

/* Complete elliptic integrals of parameter m = k^2, with the complementary
 * parameter 1-m passed separately so that it is never formed by subtraction. */
void ora_ellipke(double m, double mc, double *K, double *E)
{
    double rf = ora_rf(0.0, mc, 1.0);
    *K = rf;
    *E = rf - (m / 3.0) * ora_rd(0.0, mc, 1.0);
}

/* ------------------------------------------------------------------------ */
/* Forward/backward switch of the recursion (App. A).  The paper switches at
 * chi = 1.008 for its mode range.  Rounding in the forward recursion grows
 * like e^(2 n eta), eta = acosh(chi), relative to Q_{n-1/2}, and accumulates
 * over the n steps: the error at the top mode is about N e^(2 N eta) u
 * (u = 2^-53; measured against 40-digit values: 7e-12 at N = 32 and 3e-11
 * at N = 63 with the growth held at its N = 32 value).  Reading R8: the
 * paper's 1.008 is kept wherever N e^(2 N eta) <= 2^13 (measured: at most
 * 2.4e-12 relative at any mode up to N = 63), which holds at 1.008 up to
 * N = 23; above that the switch moves down to eta = (13 ln 2 - ln N) / (2 N),
 * and the backward recursion, whose start adapts to eta, covers the rest. */
static int ora_use_forward(int N, double chi, double dchi)
{
    if (!(chi < 1.008)) return 0;
    double eta = log1p(dchi + sqrt(dchi * (2.0 + dchi)));   /* acosh(chi) */
    return 2.0 * N * eta + log((double)N) <= 13.0 * log(2.0);
}

/* Q_{n-1/2}(chi), n = 0..N  (App. A, eqs. gfunc:recursion and gfunc:Q0).
 * Q[n] holds Q_{n-1/2}.  dchi = chi - 1, mc = 1 - mu^2 and m = mu^2 are
 * supplied from the geometry without cancellation. */
void ora_qseq(int N, double chi, double dchi, double m, double mc, double *Q)
{
    double K, E;
    ora_ellipke(m, mc, &K, &E);
    double mu = sqrt(m);
    Q[0] = mu * K;                                   /* Q_{-1/2} = mu K(mu) */
    if (N < 1) return;
    if (ora_use_forward(N, chi, dchi)) {
        /* forward recursion from Q_{-1/2}, Q_{1/2} */
        Q[1] = chi * mu * K - (1.0 + chi) * mu * E;  /* Q_{1/2} */
        for (int n = 1; n < N; ++n)
            Q[n + 1] = (4.0 * n * chi * Q[n] - (2.0 * n - 1.0) * Q[n - 1]) / (2.0 * n + 1.0);
    } else {
        /* backward recursion, normalised by Q_{-1/2}; written on the ratios
         * t_n = Q_{n+1/2}/Q_{n-1/2} so that nothing overflows:
         *   t_{n-1} = (2n-1) / (4 n chi - (2n+1) t_n),  t_{ntop} = 0. */
        double eta = log1p(dchi + sqrt(dchi * (2.0 + dchi)));   /* acosh(chi) */
        int extra = (int)ceil(20.0 / eta) + 10;
        if (extra < 80) extra = 80;
        int ntop = N + extra;
        double *t = (double *)malloc(sizeof(double) * (size_t)(ntop + 1));
        t[ntop] = 0.0;
        for (int n = ntop; n >= 1; --n)
            t[n - 1] = (2.0 * n - 1.0) / (4.0 * n * chi - (2.0 * n + 1.0) * t[n]);
        for (int n = 0; n < N; ++n) Q[n + 1] = t[n] * Q[n];
        free(t);
    }
}

/* Modal Green's function G^(n)(r, r1, x), n = 0..N  (eq. analysis:gfunc /
 * gfunc:basic): G = Q_{n-1/2}(chi) / (2 pi sqrt(r r1)),
 * chi = (r^2 + r1^2 + x^2) / (2 r r1). */
void ora_green(int N, double r, double r1, double x, double *G)
{
    double dr = r - r1, sr = r + r1;
    double rm2 = dr * dr + x * x;
    double rp2 = sr * sr + x * x;
    double rr = r * r1;
    double dchi = rm2 / (2.0 * rr);
    double chi = 1.0 + dchi;
    double m = 4.0 * rr / rp2;          /* mu^2 = 2/(1+chi) */
    double mc = rm2 / rp2;              /* 1 - mu^2        */
    ora_qseq(N, chi, dchi, m, mc, G);
    double f = 1.0 / (2.0 * ORA_PI * sqrt(rr));
    for (int n = 0; n <= N; ++n) G[n] *= f;
}

/* ------------------------------------------------------------------------ */
/* Direct modal sum (eq. analysis:sum):
 *   Phi^(n)(r_j, z_j) = sum_i S_i^(n) G^(n)(r_j, r_i, z_j - z_i). */
void ora_direct(int64_t ns, const double *rs, const double *zs,
                int64_t nf, const double *rf, const double *zf,
                int nmodes, int nrhs, const double *S, double *phi)
{
    int N = nmodes - 1;
#pragma omp parallel
    {
        double *G = (double *)malloc(sizeof(double) * (size_t)nmodes);
        double *acc = (double *)malloc(sizeof(double) * 2 * (size_t)nmodes * (size_t)nrhs);
#pragma omp for schedule(dynamic, 4)
        for (int64_t j = 0; j < nf; ++j) {
            memset(acc, 0, sizeof(double) * 2 * (size_t)nmodes * (size_t)nrhs);
            for (int64_t i = 0; i < ns; ++i) {
                if (rs[i] == rf[j] && zs[i] == zf[j]) continue;
                ora_green(N, rf[j], rs[i], zf[j] - zs[i], G);
                for (int q = 0; q < nrhs; ++q)
                    for (int n = 0; n <= N; ++n) {
                        const double *s = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                        double *a = acc + 2 * (q * nmodes + n);
                        a[0] += s[0] * G[n];
                        a[1] += s[1] * G[n];
                    }
            }
            for (int q = 0; q < nrhs; ++q)
                for (int n = 0; n <= N; ++n) {
                    double *p = phi + 2 * (((int64_t)q * nmodes + n) * nf + j);
                    p[0] = acc[2 * (q * nmodes + n)];
                    p[1] = acc[2 * (q * nmodes + n) + 1];
                }
        }
        free(G);
        free(acc);
    }
}

/* First derivatives of G^(n) from the starting formulas of App. A at
 * k = 0 (x-derivative, eq. gfunc:derivatives:x; r-derivative and its
 * r <-> r1 exchange), with G^(-1) = G^(1).  Returns dG/dr, dG/dr1, dG/dx. */
static void ora_green_d1(int N, double r, double r1, double x,
                         double *G, double *Gr, double *Gr1, double *Gx)
{
    int Nw = N < 1 ? 1 : N;
    double Gw[Nw + 1];
    ora_green(Nw, r, r1, x, Gw);
    double rp2 = (r + r1) * (r + r1) + x * x;
    double rm2 = (r - r1) * (r - r1) + x * x;
    for (int n = 0; n <= N; ++n) {
        double gn = Gw[n], gm = n == 0 ? Gw[1] : Gw[n - 1];
        double nu = n - 0.5;
        double W = (gn + gm) / rp2 + (gn - gm) / rm2;
        G[n] = gn;
        Gx[n] = nu * x * W;
        Gr[n] = -gn / (2.0 * r) + nu * (r * r - r1 * r1 - x * x) / (2.0 * r) * W;
        Gr1[n] = -gn / (2.0 * r1) + nu * (r1 * r1 - r * r - x * x) / (2.0 * r1) * W;
    }
}

/* Gradient of the direct modal sum at the field points:
 * dPhi/dr_j and dPhi/dz_j, same layout as phi. */
void ora_direct_grad(int64_t ns, const double *rs, const double *zs,
                     int64_t nf, const double *rf, const double *zf,
                     int nmodes, int nrhs, const double *S,
                     double *dphi_dr, double *dphi_dz)
{
    int N = nmodes - 1;
#pragma omp parallel
    {
        double *G = malloc(sizeof(double) * nmodes), *Gr = malloc(sizeof(double) * nmodes);
        double *Gr1 = malloc(sizeof(double) * nmodes), *Gx = malloc(sizeof(double) * nmodes);
        double *ar = calloc(2 * (size_t)nmodes * nrhs, sizeof(double));
        double *az = calloc(2 * (size_t)nmodes * nrhs, sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int64_t j = 0; j < nf; ++j) {
            memset(ar, 0, sizeof(double) * 2 * nmodes * nrhs);
            memset(az, 0, sizeof(double) * 2 * nmodes * nrhs);
            for (int64_t i = 0; i < ns; ++i) {
                if (rs[i] == rf[j] && zs[i] == zf[j]) continue;
                ora_green_d1(N, rf[j], rs[i], zf[j] - zs[i], G, Gr, Gr1, Gx);
                for (int q = 0; q < nrhs; ++q)
                    for (int n = 0; n <= N; ++n) {
                        const double *s = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                        int a = 2 * (q * nmodes + n);
                        ar[a] += s[0] * Gr[n];
                        ar[a + 1] += s[1] * Gr[n];
                        az[a] += s[0] * Gx[n];
                        az[a + 1] += s[1] * Gx[n];
                    }
            }
            for (int q = 0; q < nrhs; ++q)
                for (int n = 0; n <= N; ++n) {
                    int64_t o = 2 * (((int64_t)q * nmodes + n) * nf + j);
                    int a = 2 * (q * nmodes + n);
                    dphi_dr[o] = ar[a];
                    dphi_dr[o + 1] = ar[a + 1];
                    dphi_dz[o] = az[a];
                    dphi_dz[o + 1] = az[a + 1];
                }
        }
        free(G); free(Gr); free(Gr1); free(Gx); free(ar); free(az);
    }
}

/* Adjoint of the direct modal sum.  For a real loss L of Phi, with
 * gphi = dL/dRe(Phi) + i dL/dIm(Phi):
 *   gS_i^(n)  = sum_j G^(n)(r_j, r_i, z_j - z_i) gphi_j^(n)
 *   gr_i      = sum_{n,j} Re(conj(gphi_j^(n)) S_i^(n)) dG/dr1
 *   gz_i      = sum_{n,j} Re(conj(gphi_j^(n)) S_i^(n)) (-dG/dx)
 * (summed over right-hand sides as well).  gr, gz may be NULL. */
void ora_direct_adjoint(int64_t ns, const double *rs, const double *zs,
                        int64_t nf, const double *rf, const double *zf,
                        int nmodes, int nrhs, const double *S, const double *gphi,
                        double *gS, double *gr, double *gz)
{
    int N = nmodes - 1;
#pragma omp parallel
    {
        double *G = malloc(sizeof(double) * nmodes), *Gr = malloc(sizeof(double) * nmodes);
        double *Gr1 = malloc(sizeof(double) * nmodes), *Gx = malloc(sizeof(double) * nmodes);
        double *acc = malloc(sizeof(double) * 2 * (size_t)nmodes * nrhs);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < ns; ++i) {
            memset(acc, 0, sizeof(double) * 2 * nmodes * nrhs);
            double sr = 0.0, sz = 0.0;
            for (int64_t j = 0; j < nf; ++j) {
                if (rs[i] == rf[j] && zs[i] == zf[j]) continue;
                ora_green_d1(N, rf[j], rs[i], zf[j] - zs[i], G, Gr, Gr1, Gx);
                for (int q = 0; q < nrhs; ++q)
                    for (int n = 0; n <= N; ++n) {
                        const double *g = gphi + 2 * (((int64_t)q * nmodes + n) * nf + j);
                        const double *s = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                        int a = 2 * (q * nmodes + n);
                        acc[a] += g[0] * G[n];
                        acc[a + 1] += g[1] * G[n];
                        double w = g[0] * s[0] + g[1] * s[1];   /* Re(conj(g) s) */
                        sr += w * Gr1[n];
                        sz -= w * Gx[n];
                    }
            }
            for (int q = 0; q < nrhs; ++q)
                for (int n = 0; n <= N; ++n) {
                    int64_t o = 2 * (((int64_t)q * nmodes + n) * ns + i);
                    gS[o] = acc[2 * (q * nmodes + n)];
                    gS[o + 1] = acc[2 * (q * nmodes + n) + 1];
                }
            if (gr) gr[i] = sr;
            if (gz) gz[i] = sz;
        }
        free(G); free(Gr); free(Gr1); free(Gx); free(acc);
    }
}

/* ------------------------------------------------------------------------ */
/* Taylor tables  gbar^(n)_{a,b,c} = d^{a+b+c} G / (a! b! c! dr^a dr1^b dx^c)
 * (App. A, eqs. gfunc:gnbar, gfunc:taylor) for a <= M, b <= M, a+b+c <= 2M.
 * Output layout T[n][a][b][c], dims (N+1) x (M+1) x (M+1) x (2M+1); entries
 * outside the index set are set to zero.
 *
 * Coefficients (1/q!) d^q/dx^q of the rational factors in the starting
 * formulas are generated by the linear recurrence that multiplying through
 * by the denominator rho^2(x0+t) = rho^2 + 2 x0 t + t^2 gives. */

/* The starting columns (b <= 1 and a <= 1) are formed from sums and
 * differences of neighbouring modes, (g^n + g^(n-1)) and (g^n - g^(n-1)).
 * Where n x/r is small the two modes agree to many digits and the
 * recurrence in k amplifies rounding errors by up to ~1e14 at order 2M = 48
 * (measured against a 50-digit evaluation), so these columns, and the G^(n)
 * they start from, are computed in IEEE binary128 (reading R7).  The Laplace
 * recursion that fills the rest of the table is well conditioned and runs in
 * FP64. */
typedef __float128 ora_q;

static ora_q ora_rf_q(ora_q x, ora_q y, ora_q z)
{
    for (int it = 0; it < 400; ++it) {
        ora_q A = (x + y + z) / 3;
        ora_q X = 1 - x / A, Y = 1 - y / A, Z = 1 - z / A;
        ora_q dev = fmaxq(fabsq(X), fmaxq(fabsq(Y), fabsq(Z)));
        if (dev < 1e-7Q) {   /* neglected sixth-order terms < 1e-40 */
            ora_q E2 = X * Y - Z * Z;
            ora_q E3 = X * Y * Z;
            return (1 - E2 / 10 + E3 / 14 + E2 * E2 / 24 - 3 * E2 * E3 / 44) / sqrtq(A);
        }
        ora_q sx = sqrtq(x), sy = sqrtq(y), sz = sqrtq(z);
        ora_q lam = sx * sy + sy * sz + sz * sx;
        x = (x + lam) / 4;
        y = (y + lam) / 4;
        z = (z + lam) / 4;
    }
    return nanq("");
}

static ora_q ora_rd_q(ora_q x, ora_q y, ora_q z)
{
    ora_q sum = 0, scale = 1;
    for (int it = 0; it < 400; ++it) {
        ora_q A = (x + y + 3 * z) / 5;
        ora_q X = 1 - x / A, Y = 1 - y / A, Z3 = 1 - z / A;
        ora_q dev = fmaxq(fabsq(X), fmaxq(fabsq(Y), fabsq(Z3)));
        if (dev < 1e-7Q) {
            ora_q Z = -(X + Y) / 3;
            ora_q XY = X * Y, Z2 = Z * Z;
            ora_q E2 = XY - 6 * Z2;
            ora_q E3 = (3 * XY - 8 * Z2) * Z;
            ora_q E4 = 3 * (XY - Z2) * Z2;
            ora_q E5 = XY * Z2 * Z;
            ora_q ser = 1 - 3 * E2 / 14 + E3 / 6 + 9 * E2 * E2 / 88 - 3 * E4 / 22
                        - 9 * E2 * E3 / 52 + 3 * E5 / 26;
            return 3 * sum + scale * ser / (A * sqrtq(A));
        }
        ora_q sx = sqrtq(x), sy = sqrtq(y), sz = sqrtq(z);
        ora_q lam = sx * sy + sy * sz + sz * sx;
        sum += scale / (sz * (z + lam));
        scale /= 4;
        x = (x + lam) / 4;
        y = (y + lam) / 4;
        z = (z + lam) / 4;
    }
    return nanq("");
}

/* G^(n), n = 0..N, in binary128: the steps of ora_qseq / ora_green with the
 * backward-recursion start lengthened for the smaller target error
 * (e^(-2 eta (ntop - N)) < 1e-34). */
static void ora_green_q(int N, ora_q r, ora_q r1, ora_q x, ora_q *G)
{
    ora_q dr = r - r1, sr = r + r1;
    ora_q rm2 = dr * dr + x * x, rp2 = sr * sr + x * x, rr = r * r1;
    ora_q dchi = rm2 / (2 * rr), chi = 1 + dchi;
    ora_q m = 4 * rr / rp2, mc = rm2 / rp2;
    ora_q rf = ora_rf_q(0, mc, 1);
    ora_q K = rf, E = rf - (m / 3) * ora_rd_q(0, mc, 1);
    ora_q mu = sqrtq(m);
    G[0] = mu * K;
    if (N >= 1) {
        if (chi < 1.008Q) {
            G[1] = chi * mu * K - (1 + chi) * mu * E;
            for (int n = 1; n < N; ++n)
                G[n + 1] = (4 * n * chi * G[n] - (2 * n - 1) * G[n - 1]) / (2 * n + 1);
        } else {
            ora_q eta = log1pq(dchi + sqrtq(dchi * (2 + dchi)));
            int extra = (int)ceilq(40 / eta) + 10;
            if (extra < 160) extra = 160;
            int ntop = N + extra;
            ora_q *t = (ora_q *)malloc(sizeof(ora_q) * (size_t)(ntop + 1));
            t[ntop] = 0;
            for (int n = ntop; n >= 1; --n)
                t[n - 1] = (2 * n - 1) / (4 * n * chi - (2 * n + 1) * t[n]);
            for (int n = 0; n < N; ++n) G[n + 1] = t[n] * G[n];
            free(t);
        }
    }
    ora_q f = 1 / (2 * M_PIq * sqrtq(rr));
    for (int n = 0; n <= N; ++n) G[n] *= f;
}

/* u_q: Taylor coefficients of 1/(c^2 + x^2) about x0 */
static void ora_inv_rho2_coeffs(ora_q c, ora_q x0, int Q, ora_q *u)
{
    ora_q rho2 = c * c + x0 * x0;
    u[0] = 1 / rho2;
    if (Q >= 1) u[1] = -2 * x0 * u[0] / rho2;
    for (int q = 2; q <= Q; ++q) u[q] = -(2 * x0 * u[q - 1] + u[q - 2]) / rho2;
}

#define TIDX(n, a, b, c) ((((size_t)(n) * (M + 1) + (a)) * (M + 1) + (b)) * (2 * M + 1) + (c))

void ora_gtable(int N, int M, double r, double r1, double x, double *T)
{
    int Nw = N < 1 ? 1 : N;      /* mode 1 is needed for n = 0 (g^(-1) = g^(1)) */
    int K = 2 * M;               /* highest x order */
    size_t per = (size_t)(M + 1) * (M + 1) * (2 * M + 1);
    /* the Laplace recursion runs in x87 extended precision (64-bit
     * significand, reading R7): its rounding then stays well below that of
     * an FP64 recursion, which reaches ~1e-12 of an order's scale at high
     * modes */
    long double *W = (long double *)calloc(per * (size_t)(Nw + 1), sizeof(long double));
    ora_q Gq[Nw + 1];
    ora_q rq = r, r1q = r1, xq = x;
    ora_green_q(Nw, rq, r1q, xq, Gq);

    ora_q cp = rq + r1q, cm = rq - r1q;
    ora_q up[K + 1], um[K + 1];
    ora_inv_rho2_coeffs(cp, xq, K, up);
    ora_inv_rho2_coeffs(cm, xq, K, um);
    /* f = x / rho^2, numerator x0 + t */
    ora_q fp[K + 1], fm[K + 1];
    /* p = (r^2 - r1^2 - x^2) / rho^2, numerator A0 - 2 x0 t - t^2 */
    ora_q pp[K + 1], pm[K + 1], qp[K + 1], qm[K + 1];  /* q: r <-> r1 exchanged */
    ora_q A0 = rq * rq - r1q * r1q - xq * xq, B0 = r1q * r1q - rq * rq - xq * xq;
    for (int q = 0; q <= K; ++q) {
        ora_q um1p = q >= 1 ? up[q - 1] : 0, um2p = q >= 2 ? up[q - 2] : 0;
        ora_q um1m = q >= 1 ? um[q - 1] : 0, um2m = q >= 2 ? um[q - 2] : 0;
        fp[q] = xq * up[q] + um1p;
        fm[q] = xq * um[q] + um1m;
        pp[q] = A0 * up[q] - 2 * xq * um1p - um2p;
        pm[q] = A0 * um[q] - 2 * xq * um1m - um2m;
        qp[q] = B0 * up[q] - 2 * xq * um1p - um2p;
        qm[q] = B0 * um[q] - 2 * xq * um1m - um2m;
    }
    /* d = d/dr1 of p: (-2 r1)/rho^2 - p * (d rho^2/dr1)/rho^2,
     * d rho+^2/dr1 = 2 (r + r1), d rho-^2/dr1 = -2 (r - r1). */
    ora_q dp[K + 1], dm[K + 1];
    for (int q = 0; q <= K; ++q) {
        ora_q cpu = 0, cmu = 0;
        for (int s = 0; s <= q; ++s) {
            cpu += pp[s] * up[q - s];
            cmu += pm[s] * um[q - s];
        }
        dp[q] = -2 * r1q * up[q] - 2 * cp * cpu;
        dm[q] = -2 * r1q * um[q] + 2 * cm * cmu;
    }

    /* starting columns in binary128: g00[n][k], g10, g01, g11 */
    size_t col = (size_t)(Nw + 1) * (K + 1);
    ora_q *g00 = (ora_q *)calloc(4 * col, sizeof(ora_q));
    ora_q *g10 = g00 + col, *g01 = g10 + col, *g11 = g01 + col;
#define GQ(a, n, k) a[(size_t)(n) * (K + 1) + (k)]
    /* x-derivatives, eq. gfunc:derivatives:x, k-outer / n-inner */
    for (int n = 0; n <= Nw; ++n) GQ(g00, n, 0) = Gq[n];
    for (int k = 0; k < K; ++k) {
        for (int n = 0; n <= Nw; ++n) {
            int nm = n == 0 ? 1 : n - 1;
            ora_q s = 0;
            for (int q = 0; q <= k; ++q) {
                ora_q gn = GQ(g00, n, k - q), gm = GQ(g00, nm, k - q);
                s += (gn + gm) * fp[q] + (gn - gm) * fm[q];
            }
            GQ(g00, n, k + 1) = (n - 0.5Q) * s / (k + 1);
        }
    }
    if (M >= 1) {
        /* r-derivative and its r <-> r1 exchange */
        for (int n = 0; n <= Nw; ++n) {
            int nm = n == 0 ? 1 : n - 1;
            for (int k = 0; k <= K - 1; ++k) {
                ora_q s1 = 0, s2 = 0;
                for (int q = 0; q <= k; ++q) {
                    ora_q gn = GQ(g00, n, k - q), gm = GQ(g00, nm, k - q);
                    s1 += (gn + gm) * pp[q] + (gn - gm) * pm[q];
                    s2 += (gn + gm) * qp[q] + (gn - gm) * qm[q];
                }
                GQ(g10, n, k) = -GQ(g00, n, k) / (2 * rq) + (n - 0.5Q) / (2 * rq) * s1;
                GQ(g01, n, k) = -GQ(g00, n, k) / (2 * r1q) + (n - 0.5Q) / (2 * r1q) * s2;
            }
        }
        /* mixed r, r1 derivative */
        for (int n = 0; n <= Nw; ++n) {
            int nm = n == 0 ? 1 : n - 1;
            for (int k = 0; k <= K - 2; ++k) {
                ora_q s = 0;
                for (int q = 0; q <= k; ++q) {
                    ora_q gn = GQ(g00, n, k - q), gm = GQ(g00, nm, k - q);
                    ora_q hn = GQ(g01, n, k - q), hm = GQ(g01, nm, k - q);
                    s += (gn + gm) * dp[q] + (hn + hm) * pp[q]
                         + (gn - gm) * dm[q] + (hn - hm) * pm[q];
                }
                GQ(g11, n, k) = -GQ(g01, n, k) / (2 * rq) + (n - 0.5Q) / (2 * rq) * s;
            }
        }
    }
#define WI(n, a, b, c) W[(size_t)(n) * per + ((size_t)(a) * (M + 1) + (b)) * (2 * M + 1) + (c)]
    for (int n = 0; n <= Nw; ++n)
        for (int k = 0; k <= K; ++k) {
            WI(n, 0, 0, k) = (long double)GQ(g00, n, k);
            if (M >= 1 && k <= K - 1) {
                WI(n, 1, 0, k) = (long double)GQ(g10, n, k);
                WI(n, 0, 1, k) = (long double)GQ(g01, n, k);
            }
            if (M >= 1 && k <= K - 2) WI(n, 1, 1, k) = (long double)GQ(g11, n, k);
        }
#undef GQ
    free(g00);
    /* Laplace recursion (eq. gfunc:laplace, reading R1) in r for b = 0, 1,
     * then in r1 for all a. */
    const long double rl = r, r1l = r1;
    for (int n = 0; n <= N; ++n) {
        long double n2 = (long double)n * (long double)n;
        for (int j = 0; j <= 1 && j <= M; ++j)
            for (int i = 0; i + 2 <= M; ++i)
                for (int k = 0; i + 2 + j + k <= K; ++k) {
                    long double s = 0.0L, rp = 1.0L / rl;   /* rp = r^-(u+1) */
                    for (int u = 0; u <= i; ++u) {
                        long double sg = (u & 1) ? -1.0L : 1.0L;
                        s += sg * rp * ((u + 1) * n2 / rl * WI(n, i - u, j, k)
                                        - (i - u + 1) * WI(n, i - u + 1, j, k));
                        rp /= rl;
                    }
                    WI(n, i + 2, j, k) = s / ((i + 1.0L) * (i + 2.0L))
                        - (k + 1.0L) * (k + 2.0L) / ((i + 1.0L) * (i + 2.0L)) * WI(n, i, j, k + 2);
                }
        for (int j = 0; j + 2 <= M; ++j)
            for (int a = 0; a <= M; ++a)
                for (int k = 0; a + j + 2 + k <= K; ++k) {
                    long double s = 0.0L, rp = 1.0L / r1l;
                    for (int u = 0; u <= j; ++u) {
                        long double sg = (u & 1) ? -1.0L : 1.0L;
                        s += sg * rp * ((u + 1) * n2 / r1l * WI(n, a, j - u, k)
                                        - (j - u + 1) * WI(n, a, j - u + 1, k));
                        rp /= r1l;
                    }
                    WI(n, a, j + 2, k) = s / ((j + 1.0L) * (j + 2.0L))
                        - (k + 1.0L) * (k + 2.0L) / ((j + 1.0L) * (j + 2.0L)) * WI(n, a, j, k + 2);
                }
    }
    for (int n = 0; n <= N; ++n)
        for (int a = 0; a <= M; ++a)
            for (int b = 0; b <= M; ++b)
                for (int c = 0; c <= K; ++c)
                    T[TIDX(n, a, b, c)] = (a + b + c <= K) ? (double)WI(n, a, b, c) : 0.0;
#undef WI
    free(W);
}

/* ------------------------------------------------------------------------ */
/* Reference FMM following Algorithm 1 (section 3) literally on a dense
 * uniform quadtree.  S2L tables are built at the actual pair of box
 * centres (r = target centre, r1 = source centre, x = target z - source z)
 * and applied with eq. analysis:s2l; no FO/BO/FI/BI reuse.
 * flags & 1: unit kernel (G = 1, gbar_000 = 1, all other derivatives 0),
 * used to check that every source/target pair is counted exactly once. */

typedef struct {
    double rlo, zlo, L, invL;
} ora_square;

static ora_square ora_bounding_square(int64_t ns, const double *rs, const double *zs,
                                      int64_t nf, const double *rf, const double *zf)
{
    double rmin = INFINITY, rmax = -INFINITY, zmin = INFINITY, zmax = -INFINITY;
    for (int64_t i = 0; i < ns; ++i) {
        rmin = fmin(rmin, rs[i]); rmax = fmax(rmax, rs[i]);
        zmin = fmin(zmin, zs[i]); zmax = fmax(zmax, zs[i]);
    }
    for (int64_t j = 0; j < nf; ++j) {
        rmin = fmin(rmin, rf[j]); rmax = fmax(rmax, rf[j]);
        zmin = fmin(zmin, zf[j]); zmax = fmax(zmax, zf[j]);
    }
    ora_square sq;
    double ext = fmax(rmax - rmin, zmax - zmin);
    /* R5: side = the larger extent; in r on the axis when that side reaches
       the largest radius, else on k/4 of a (slightly grown) side when the
       smallest radius is between L/4 and L, else at the smallest radius */
    sq.L = ext > 0.0 ? ext : 1.0;
    sq.zlo = zmin;
    sq.rlo = rmin;
    if (rmax <= sq.L) {
        sq.rlo = 0.0;
    } else {
        double k = floor(rmin / (sq.L * 0.25));
        if (k >= 1.0 && k <= 3.0) {
            double f = 1.0 + k * 0.25;
            double Ls = fmax(sq.L, rmax / f);
            for (;;) {
                double r0 = k * (Ls * 0.25);
                double top = r0 + Ls;
                if (top >= rmax) break;
                Ls = nextafter(Ls, INFINITY);
            }
            double r0 = k * (Ls * 0.25);
            if (r0 <= rmin) {
                sq.L = Ls;
                sq.rlo = r0;
            }
        }
    }
    sq.invL = 1.0 / sq.L;
    return sq;
}

static int ora_box_index(double v, double lo, double invL, int level)
{
    double t = (v - lo) * invL;
    double s = t * (double)(1 << level);
    int i = (int)s;
    int nb = 1 << level;
    if (i > nb - 1) i = nb - 1;
    if (i < 0) i = 0;
    return i;
}

void ora_square_info(int64_t ns, const double *rs, const double *zs,
                     int64_t nf, const double *rf, const double *zf, double *out4)
{
    ora_square sq = ora_bounding_square(ns, rs, zs, nf, rf, zf);
    out4[0] = sq.rlo; out4[1] = sq.zlo; out4[2] = sq.L; out4[3] = sq.invL;
}

/* leaf box indices at a given level for a list of points */
void ora_box_indices(int64_t n, const double *r, const double *z,
                     double rlo, double zlo, double invL, int level,
                     int32_t *ir, int32_t *iz)
{
    for (int64_t i = 0; i < n; ++i) {
        ir[i] = ora_box_index(r[i], rlo, invL, level);
        iz[i] = ora_box_index(z[i], zlo, invL, level);
    }
}

static double ora_binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double b = 1.0;
    for (int i = 1; i <= k; ++i) b = b * (n - k + i) / i;
    return b;
}

/* index of coefficient (i, j), i + j <= M, in a packed triangle */
static int ora_tri(int M, int i, int j)
{
    return i * (M + 1) - i * (i - 1) / 2 + j;
}

/* S2L from moments Smom (P complex per channel, channel = q*nmodes + n) of a
 * box centred (r1, z1) into locals Loc of a box centred (r, z)
 * (eq. analysis:s2l). */
static void ora_s2l(int nmodes, int nrhs, int M, double r, double z, double r1, double z1,
                    const double *Smom, double *Loc, double *T, int unit)
{
    int N = nmodes - 1, P = (M + 1) * (M + 2) / 2;
    if (unit) {
        memset(T, 0, sizeof(double) * (size_t)nmodes * (M + 1) * (M + 1) * (2 * M + 1));
        for (int n = 0; n <= N; ++n) T[TIDX(n, 0, 0, 0)] = 1.0;
    } else {
        ora_gtable(N, M, r, r1, z - z1, T);
    }
    for (int q = 0; q < nrhs; ++q)
        for (int n = 0; n <= N; ++n) {
            const double *Sm = Smom + 2 * (size_t)P * (q * nmodes + n);
            double *Lc = Loc + 2 * (size_t)P * (q * nmodes + n);
            for (int k = 0; k <= M; ++k)
                for (int l = 0; k + l <= M; ++l) {
                    double are = 0.0, aim = 0.0;
                    for (int i = 0; i <= M; ++i)
                        for (int j = 0; i + j <= M; ++j) {
                            double g = T[TIDX(n, k, i, j + l)];
                            double w = ((j & 1) ? -1.0 : 1.0) * ora_binom(j + l, j) * g;
                            are += w * Sm[2 * ora_tri(M, i, j)];
                            aim += w * Sm[2 * ora_tri(M, i, j) + 1];
                        }
                    Lc[2 * ora_tri(M, k, l)] += are;
                    Lc[2 * ora_tri(M, k, l) + 1] += aim;
                }
        }
}

static void ora_pair_kernel(int N, double r, double r1, double x, double *G, int unit)
{
    if (unit) {
        for (int n = 0; n <= N; ++n) G[n] = 1.0;
    } else {
        ora_green(N, r, r1, x, G);
    }
}

void ora_fmm_grad(int64_t ns, const double *rs, const double *zs,
                  int64_t nf, const double *rf, const double *zf,
                  int nmodes, int nrhs, const double *S, int M, int depth, int flags,
                  double *phi, double *dphi_dr, double *dphi_dz);

void ora_fmm(int64_t ns, const double *rs, const double *zs,
             int64_t nf, const double *rf, const double *zf,
             int nmodes, int nrhs, const double *S, int M, int depth, int flags,
             double *phi)
{
    ora_fmm_grad(ns, rs, zs, nf, rf, zf, nmodes, nrhs, S, M, depth, flags, phi, NULL, NULL);
}

/* Algorithm 1 with, optionally, the field gradient at the field points:
 * the r- and z-derivatives of the local expansion (eq. analysis:local) plus
 * the near-field sum of S dG/dr and S dG/dx (App. A starting formulas). */
void ora_fmm_grad(int64_t ns, const double *rs, const double *zs,
                  int64_t nf, const double *rf, const double *zf,
                  int nmodes, int nrhs, const double *S, int M, int depth, int flags,
                  double *phi, double *dphi_dr, double *dphi_dz)
{
    int grad = dphi_dr != NULL && dphi_dz != NULL;
    int unit = flags & 1;
    int N = nmodes - 1, d = depth;
    int P = (M + 1) * (M + 2) / 2;
    int C = nmodes * nrhs;
    size_t blk = 2 * (size_t)P * C;           /* doubles per box */
    ora_square sq = ora_bounding_square(ns, rs, zs, nf, rf, zf);

    /* per-level dense moment and local arrays, box (ir, iz) at ir*2^l + iz */
    double **mom = calloc(d + 1, sizeof(double *));
    double **loc = calloc(d + 1, sizeof(double *));
    for (int l = 2; l <= d; ++l) {
        mom[l] = calloc((size_t)1 << (2 * l), blk * sizeof(double));
        loc[l] = calloc((size_t)1 << (2 * l), blk * sizeof(double));
    }
    int nb = 1 << d;
    int32_t *sir = malloc(sizeof(int32_t) * ns), *siz = malloc(sizeof(int32_t) * ns);
    int32_t *fir = malloc(sizeof(int32_t) * nf), *fiz = malloc(sizeof(int32_t) * nf);
    ora_box_indices(ns, rs, zs, sq.rlo, sq.zlo, sq.invL, d, sir, siz);
    ora_box_indices(nf, rf, zf, sq.rlo, sq.zlo, sq.invL, d, fir, fiz);

    /* leaf moments, eq. analysis:moments (unscaled displacements) */
    {
        double h = sq.L / nb;
        for (int64_t i = 0; i < ns; ++i) {
            double rc = sq.rlo + (sir[i] + 0.5) * h, zc = sq.zlo + (siz[i] + 0.5) * h;
            double dr = rs[i] - rc, dz = zs[i] - zc;
            double *m = mom[d] + blk * ((size_t)sir[i] * nb + siz[i]);
            for (int q = 0; q < nrhs; ++q)
                for (int n = 0; n <= N; ++n) {
                    const double *s = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                    double *mm = m + 2 * (size_t)P * (q * nmodes + n);
                    double pr = 1.0;
                    for (int a = 0; a <= M; ++a) {
                        double pz = 1.0;
                        for (int b = 0; a + b <= M; ++b) {
                            double w = unit ? (a == 0 && b == 0 ? 1.0 : 0.0) : pr * pz;
                            mm[2 * ora_tri(M, a, b)] += s[0] * w;
                            mm[2 * ora_tri(M, a, b) + 1] += s[1] * w;
                            pz *= dz;
                        }
                        pr *= dr;
                    }
                }
        }
    }
    /* upward pass, eq. analysis:shift, levels d-1 .. 2 */
    for (int l = d - 1; l >= 2; --l) {
        int nbl = 1 << l;
        double hp = sq.L / nbl, hc = hp / 2.0;
        for (int ir = 0; ir < nbl; ++ir)
            for (int iz = 0; iz < nbl; ++iz) {
                double rcp = sq.rlo + (ir + 0.5) * hp, zcp = sq.zlo + (iz + 0.5) * hp;
                double *mp = mom[l] + blk * ((size_t)ir * nbl + iz);
                for (int cr = 0; cr < 2; ++cr)
                    for (int cz = 0; cz < 2; ++cz) {
                        int jr = 2 * ir + cr, jz = 2 * iz + cz;
                        double rcc = sq.rlo + (jr + 0.5) * hc, zcc = sq.zlo + (jz + 0.5) * hc;
                        double dr = rcc - rcp, dz = zcc - zcp;
                        const double *mc = mom[l + 1] + blk * ((size_t)jr * (2 * nbl) + jz);
                        for (int c = 0; c < C; ++c)
                            for (int i = 0; i <= M; ++i)
                                for (int j = 0; i + j <= M; ++j) {
                                    double are = 0.0, aim = 0.0;
                                    for (int q = 0; q <= i; ++q)
                                        for (int u = 0; u <= j; ++u) {
                                            double w = ora_binom(i, q) * ora_binom(j, u)
                                                       * pow(dr, q) * pow(dz, u);
                                            if (unit) w = (q == 0 && u == 0) ? 1.0 : 0.0;
                                            const double *sm = mc + 2 * ((size_t)P * c + ora_tri(M, i - q, j - u));
                                            are += w * sm[0];
                                            aim += w * sm[1];
                                        }
                                    mp[2 * ((size_t)P * c + ora_tri(M, i, j))] += are;
                                    mp[2 * ((size_t)P * c + ora_tri(M, i, j)) + 1] += aim;
                                }
                    }
            }
    }
    /* downward pass, levels 2 .. d */
    size_t tsz = (size_t)nmodes * (M + 1) * (M + 1) * (2 * M + 1);
    for (int l = 2; l <= d; ++l) {
        int nbl = 1 << l;
        double h = sq.L / nbl;
        if (l > 2) {
            /* parent-to-child local shift, eq. analysis:l2l */
            int nbp = nbl / 2;
            double hp = 2.0 * h;
            for (int ir = 0; ir < nbl; ++ir)
                for (int iz = 0; iz < nbl; ++iz) {
                    int pr = ir / 2, pz = iz / 2;
                    double dr = (sq.rlo + (ir + 0.5) * h) - (sq.rlo + (pr + 0.5) * hp);
                    double dz = (sq.zlo + (iz + 0.5) * h) - (sq.zlo + (pz + 0.5) * hp);
                    const double *lp = loc[l - 1] + blk * ((size_t)pr * nbp + pz);
                    double *lc = loc[l] + blk * ((size_t)ir * nbl + iz);
                    for (int c = 0; c < C; ++c)
                        for (int i = 0; i <= M; ++i)
                            for (int j = 0; i + j <= M; ++j) {
                                double are = 0.0, aim = 0.0;
                                for (int q = 0; i + q <= M; ++q)
                                    for (int u = 0; i + q + j + u <= M; ++u) {
                                        double w = ora_binom(i + q, q) * ora_binom(j + u, u)
                                                   * pow(dr, q) * pow(dz, u);
                                        if (unit) w = (q == 0 && u == 0) ? 1.0 : 0.0;
                                        const double *sl = lp + 2 * ((size_t)P * c + ora_tri(M, i + q, j + u));
                                        are += w * sl[0];
                                        aim += w * sl[1];
                                    }
                                lc[2 * ((size_t)P * c + ora_tri(M, i, j))] += are;
                                lc[2 * ((size_t)P * c + ora_tri(M, i, j)) + 1] += aim;
                            }
                }
        }
        /* S2L over the interaction list: children of the parent's neighbours
         * that are not neighbours of the box (section 2.2, Fig. fmm:lists) */
#pragma omp parallel
        {
            double *T = malloc(sizeof(double) * tsz);
#pragma omp for schedule(dynamic, 1)
            for (int b = 0; b < nbl * nbl; ++b) {
                int ir = b / nbl, iz = b % nbl;
                double rc = sq.rlo + (ir + 0.5) * h, zc = sq.zlo + (iz + 0.5) * h;
                double *lc = loc[l] + blk * ((size_t)ir * nbl + iz);
                for (int jr = 2 * (ir / 2) - 2; jr <= 2 * (ir / 2) + 3; ++jr)
                    for (int jz = 2 * (iz / 2) - 2; jz <= 2 * (iz / 2) + 3; ++jz) {
                        if (jr < 0 || jz < 0 || jr >= nbl || jz >= nbl) continue;
                        if (abs(jr - ir) <= 1 && abs(jz - iz) <= 1) continue;
                        double r1 = sq.rlo + (jr + 0.5) * h, z1 = sq.zlo + (jz + 0.5) * h;
                        ora_s2l(nmodes, nrhs, M, rc, zc, r1, z1,
                                mom[l] + blk * ((size_t)jr * nbl + jz), lc, T, unit);
                    }
            }
            free(T);
        }
    }
    /* leaf evaluation: local expansion plus direct sum over neighbours */
    {
        double h = sq.L / nb;
#pragma omp parallel
        {
            double *G = malloc(sizeof(double) * nmodes), *Gr = malloc(sizeof(double) * nmodes);
            double *Gr1 = malloc(sizeof(double) * nmodes), *Gx = malloc(sizeof(double) * nmodes);
#pragma omp for schedule(dynamic, 16)
            for (int64_t j = 0; j < nf; ++j) {
                double rc = sq.rlo + (fir[j] + 0.5) * h, zc = sq.zlo + (fiz[j] + 0.5) * h;
                double dr = rf[j] - rc, dz = zf[j] - zc;
                const double *lc = loc[d] + blk * ((size_t)fir[j] * nb + fiz[j]);
                for (int c = 0; c < C; ++c) {
                    double are = 0.0, aim = 0.0, gre = 0.0, gim = 0.0, zre = 0.0, zim = 0.0;
                    for (int k = 0; k <= M; ++k)
                        for (int l2 = 0; k + l2 <= M; ++l2) {
                            double w = unit ? (k == 0 && l2 == 0 ? 1.0 : 0.0) : pow(dr, k) * pow(dz, l2);
                            double wr = (k > 0 && !unit) ? k * pow(dr, k - 1) * pow(dz, l2) : 0.0;
                            double wz = (l2 > 0 && !unit) ? l2 * pow(dr, k) * pow(dz, l2 - 1) : 0.0;
                            const double *v = lc + 2 * ((size_t)P * c + ora_tri(M, k, l2));
                            are += w * v[0]; aim += w * v[1];
                            gre += wr * v[0]; gim += wr * v[1];
                            zre += wz * v[0]; zim += wz * v[1];
                        }
                    int q = c / nmodes, n = c % nmodes;
                    int64_t o = 2 * (((int64_t)q * nmodes + n) * nf + j);
                    phi[o] = are;
                    phi[o + 1] = aim;
                    if (grad) {
                        dphi_dr[o] = gre; dphi_dr[o + 1] = gim;
                        dphi_dz[o] = zre; dphi_dz[o + 1] = zim;
                    }
                }
                for (int64_t i = 0; i < ns; ++i) {
                    if (abs(sir[i] - fir[j]) > 1 || abs(siz[i] - fiz[j]) > 1) continue;
                    if (rs[i] == rf[j] && zs[i] == zf[j]) continue;
                    if (grad) ora_green_d1(N, rf[j], rs[i], zf[j] - zs[i], G, Gr, Gr1, Gx);
                    else ora_pair_kernel(N, rf[j], rs[i], zf[j] - zs[i], G, unit);
                    for (int q = 0; q < nrhs; ++q)
                        for (int n = 0; n <= N; ++n) {
                            const double *sv = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                            int64_t o = 2 * (((int64_t)q * nmodes + n) * nf + j);
                            phi[o] += sv[0] * G[n];
                            phi[o + 1] += sv[1] * G[n];
                            if (grad) {
                                dphi_dr[o] += sv[0] * Gr[n]; dphi_dr[o + 1] += sv[1] * Gr[n];
                                dphi_dz[o] += sv[0] * Gx[n]; dphi_dz[o + 1] += sv[1] * Gx[n];
                            }
                        }
                }
            }
            free(G); free(Gr); free(Gr1); free(Gx);
        }
    }
    for (int l = 2; l <= d; ++l) { free(mom[l]); free(loc[l]); }
    free(mom); free(loc); free(sir); free(siz); free(fir); free(fiz);
}

/* The same FMM result evaluated one field point at a time.  Because the
 * moment shift (eq. analysis:shift) and the local shift (eq. analysis:l2l)
 * re-centre polynomials of degree <= M without loss, the FMM value at a
 * field point equals: direct sum over the 3x3 neighbour leaves, plus, for
 * every level l = 2..d, the S2L image of the moments of each interaction-list
 * box (computed straight from its sources about its own centre) about the
 * centre of the point's level-l box, evaluated at the point.  Used on
 * sampled points of problems too large for ora_fmm. */
void ora_fmm_points(int64_t ns, const double *rs, const double *zs,
                    int64_t nf, const double *rf, const double *zf,
                    int nmodes, int nrhs, const double *S, int M, int depth,
                    int64_t nsample, const int64_t *idx, double *out)
{
    int N = nmodes - 1, d = depth;
    int P = (M + 1) * (M + 2) / 2;
    int C = nmodes * nrhs;
    size_t blk = 2 * (size_t)P * C;
    ora_square sq = ora_bounding_square(ns, rs, zs, nf, rf, zf);
    int nb = 1 << d;
    int32_t *sir = malloc(sizeof(int32_t) * ns), *siz = malloc(sizeof(int32_t) * ns);
    ora_box_indices(ns, rs, zs, sq.rlo, sq.zlo, sq.invL, d, sir, siz);
    size_t tsz = (size_t)nmodes * (M + 1) * (M + 1) * (2 * M + 1);
#pragma omp parallel
    {
        double *T = malloc(sizeof(double) * tsz);
        double *G = malloc(sizeof(double) * nmodes);
        double *mom = malloc(sizeof(double) * blk * 49);
        int used[49];
        double *loc = malloc(sizeof(double) * blk);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < nsample; ++t) {
            int64_t j = idx[t];
            int fr = ora_box_index(rf[j], sq.rlo, sq.invL, d);
            int fz = ora_box_index(zf[j], sq.zlo, sq.invL, d);
            double acc[2 * C];
            memset(acc, 0, sizeof(acc));
            /* neighbour leaves: direct */
            for (int64_t i = 0; i < ns; ++i) {
                if (abs(sir[i] - fr) > 1 || abs(siz[i] - fz) > 1) continue;
                if (rs[i] == rf[j] && zs[i] == zf[j]) continue;
                ora_green(N, rf[j], rs[i], zf[j] - zs[i], G);
                for (int q = 0; q < nrhs; ++q)
                    for (int n = 0; n <= N; ++n) {
                        const double *s = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                        acc[2 * (q * nmodes + n)] += s[0] * G[n];
                        acc[2 * (q * nmodes + n) + 1] += s[1] * G[n];
                    }
            }
            /* far field, level by level */
            for (int l = 2; l <= d; ++l) {
                int sh = d - l;
                int br = fr >> sh, bz = fz >> sh;
                double h = sq.L / (1 << l);
                double rc = sq.rlo + (br + 0.5) * h, zc = sq.zlo + (bz + 0.5) * h;
                memset(mom, 0, sizeof(double) * blk * 49);
                memset(used, 0, sizeof(used));
                for (int64_t i = 0; i < ns; ++i) {
                    int ar = sir[i] >> sh, az = siz[i] >> sh;
                    if (ar < 2 * (br / 2) - 2 || ar > 2 * (br / 2) + 3) continue;
                    if (az < 2 * (bz / 2) - 2 || az > 2 * (bz / 2) + 3) continue;
                    if (abs(ar - br) <= 1 && abs(az - bz) <= 1) continue;
                    int slot = (ar - br + 3) * 7 + (az - bz + 3);
                    used[slot] = 1;
                    double r1 = sq.rlo + (ar + 0.5) * h, z1 = sq.zlo + (az + 0.5) * h;
                    double dr = rs[i] - r1, dz = zs[i] - z1;
                    double *m = mom + blk * slot;
                    for (int q = 0; q < nrhs; ++q)
                        for (int n = 0; n <= N; ++n) {
                            const double *s = S + 2 * (((int64_t)q * nmodes + n) * ns + i);
                            double *mm = m + 2 * (size_t)P * (q * nmodes + n);
                            double pr = 1.0;
                            for (int a = 0; a <= M; ++a) {
                                double pz = 1.0;
                                for (int b = 0; a + b <= M; ++b) {
                                    mm[2 * ora_tri(M, a, b)] += s[0] * pr * pz;
                                    mm[2 * ora_tri(M, a, b) + 1] += s[1] * pr * pz;
                                    pz *= dz;
                                }
                                pr *= dr;
                            }
                        }
                }
                for (int slot = 0; slot < 49; ++slot) {
                    if (!used[slot]) continue;
                    int ar = br + slot / 7 - 3, az = bz + slot % 7 - 3;
                    double r1 = sq.rlo + (ar + 0.5) * h, z1 = sq.zlo + (az + 0.5) * h;
                    memset(loc, 0, sizeof(double) * blk);
                    ora_s2l(nmodes, nrhs, M, rc, zc, r1, z1, mom + blk * slot, loc, T, 0);
                    double dr = rf[j] - rc, dz = zf[j] - zc;
                    for (int c = 0; c < C; ++c) {
                        double pr = 1.0;
                        for (int k = 0; k <= M; ++k) {
                            double pz = 1.0;
                            for (int l2 = 0; k + l2 <= M; ++l2) {
                                acc[2 * c] += pr * pz * loc[2 * ((size_t)P * c + ora_tri(M, k, l2))];
                                acc[2 * c + 1] += pr * pz * loc[2 * ((size_t)P * c + ora_tri(M, k, l2)) + 1];
                                pz *= dz;
                            }
                            pr *= dr;
                        }
                    }
                }
            }
            for (int q = 0; q < nrhs; ++q)
                for (int n = 0; n <= N; ++n) {
                    double *o = out + 2 * (((int64_t)q * nmodes + n) * nsample + t);
                    o[0] = acc[2 * (q * nmodes + n)];
                    o[1] = acc[2 * (q * nmodes + n) + 1];
                }
        }
        free(T); free(G); free(mom); free(loc);
    }
    free(sir); free(siz);
    (void)nb;
}


/* ------------------------------------------------------------------------ */
/* Azimuthal analysis and synthesis (section 2, eqs. analysis:source and
 * analysis:phi; reading R14).  Angles are reduced exactly: the phase of
 * term (n, k) is 2 pi ((n k) mod K) / K. */

/* samples: [nrhs][nrings][K] real values s(theta_k) on each ring;
 * S: complex [nrhs][nmodes][nrings], modes n = 0..nmodes-1. */
void ora_analysis(int64_t nrings, int K, int nmodes, int nrhs, const double *samples, double *S)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrings; ++i)
        for (int q = 0; q < nrhs; ++q) {
            const double *s = samples + ((int64_t)q * nrings + i) * K;
            for (int n = 0; n < nmodes; ++n) {
                double re = 0.0, im = 0.0;
                for (int k = 0; k < K; ++k) {
                    double t = 2.0 * ORA_PI * (double)(((int64_t)n * k) % K) / K;
                    re += s[k] * cos(t);
                    im -= s[k] * sin(t);
                }
                double *o = S + 2 * (((int64_t)q * nmodes + n) * nrings + i);
                o[0] = re / K;
                o[1] = im / K;
            }
        }
}

/* phi: complex [nrhs][nmodes][npts]; out: [nrhs][npts][K] real values
 * phi(theta_k) at theta_k = 2 pi k / K. */
void ora_synthesis(int64_t npts, int nmodes, int nrhs, const double *phi, int K, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < npts; ++j)
        for (int q = 0; q < nrhs; ++q)
            for (int k = 0; k < K; ++k) {
                double v = phi[2 * ((int64_t)q * nmodes * npts + j)];     /* Re Phi^(0) */
                for (int n = 1; n < nmodes; ++n) {
                    const double *p = phi + 2 * (((int64_t)q * nmodes + n) * npts + j);
                    double t = 2.0 * ORA_PI * (double)(((int64_t)n * k) % K) / K;
                    v += 2.0 * (p[0] * cos(t) - p[1] * sin(t));
                }
                out[((int64_t)q * npts + j) * K + k] = v;
            }
}

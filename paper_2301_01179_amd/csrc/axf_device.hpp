// axf_device.hpp -- device-side building blocks of the gfx950 modal FMM.
//
// * the modal Green's function G^(n)(r, r1, x), n = 0..N, for one pair per
//   lane: complete elliptic integrals by the arithmetic-geometric mean, the
//   three-term recursion in n (eq. gfunc:recursion) forward for
//   chi < chi*(N) and backward (Miller) otherwise, normalised by
//   G^(0) = 1 / (2 AGM(rho+, rho-));
// * Morton interleave, packed-triangle and table indexing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace axf {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Coefficients of the downward recursion written for G:
//   G^(n-1) = A[n] chi G^(n) - B[n] G^(n+1),  A[n] = 4n/(2n-1),  B[n] = (2n+1)/(2n-1).
constexpr int kMillerMax = 1400;
struct DownCoef {
    double a[kMillerMax + 2];
    double b[kMillerMax + 2];
    constexpr DownCoef() : a(), b()
    {
        for (int n = 1; n < kMillerMax + 2; ++n) {
            a[n] = 4.0 * n / (2.0 * n - 1.0);
            b[n] = (2.0 * n + 1.0) / (2.0 * n - 1.0);
        }
    }
};
static __constant__ DownCoef c_down = DownCoef();

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Forward-recursion limit: rounding grows like lambda^(2N), lambda = chi +
// sqrt(chi^2 - 1); below chi* the growth stays under ~100.
inline double forward_chi_limit(int nmodes)
{
    int N = nmodes - 1;
    if (N < 2) return 1e300;
    double eta = 4.605170185988091 / (2.0 * N);   // ln(100) / (2N)
    return 0.5 * (__builtin_exp(eta) + __builtin_exp(-eta));
}

// Modal Green's functions of one pair per lane, G[n] for n < NMB (entries at
// n >= nmodes are finite but unused).  Must be called by every lane of the
// wave in uniform control flow (the backward branch uses a wave-wide step
// count).  Inputs:
//   rm2 = (r - r1)^2 + x^2 > 0,  rp2 = (r + r1)^2 + x^2,  rr = r r1,
//   inv_rr = 1 / (r r1).
template <int NMB>
__device__ __forceinline__ void green_modes(double rm2, double rp2, double rr, double inv_rr,
                                            double chistar, int nmodes, double (&G)[NMB])
{
    // AGM(rho+, rho-): G^(0) = 1 / (2 AGM), and with c_n the AGM half-differences
    // G^(1) / G^(0) = (1 / (2 r r1)) sum_{n >= 1} 2^(n-1) c_n^2   (from E/K).
    double rp = sqrt(rp2), rm = sqrt(rm2);
    double a = rp, b = rm;
    double c = 2.0 * rr / (rp + rm);          // c_1 = (rho+ - rho-) / 2, no cancellation
    double csum = c * c, w = 1.0;
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
    double g1 = g0 * csum * 0.5 * inv_rr;
    double chi = (rp2 + rm2) * 0.25 * inv_rr;

    // forward recursion (all lanes; backward lanes overwrite below)
    G[0] = g0;
    if constexpr (NMB > 1) G[1] = g1;
#pragma unroll
    for (int n = 1; n + 1 < NMB; ++n) {
        if (n + 1 < nmodes) {
            const double fa = 4.0 * n / (2.0 * n + 1.0), fb = (2.0 * n - 1.0) / (2.0 * n + 1.0);
            G[n + 1] = fa * chi * G[n] - fb * G[n - 1];
        }
    }
    if constexpr (NMB > 2) {
        bool back = chi >= chistar;
        if (__ballot(back)) {
            // chi - 1 without cancellation
            double dchi = rm2 * 0.5 * inv_rr;
            double dmin = wave_min(back ? dchi : 1e300);
            // Miller start: error ~ lambda^(-2 (ntop - N)), acosh(1 + d) <= sqrt(2 d)
            int extra = 10 + (int)ceil(20.0 / sqrt(2.0 * dmin));
            int ntop = nmodes - 1 + extra;
            if (ntop < NMB) ntop = NMB;
            if (ntop > kMillerMax) ntop = kMillerMax;
            ntop = __builtin_amdgcn_readfirstlane(ntop);
            double yp = 0.0, y = 1.0;             // y_{ntop+1}, y_{ntop}
            for (int n = ntop; n >= NMB; --n) {   // -> y_{NMB-1}
                double ym = c_down.a[n] * chi * y - c_down.b[n] * yp;
                yp = y;
                y = ym;
                if ((n & 7) == 0 && fabs(y) > 0x1p500) {
                    y *= 0x1p-500;
                    yp *= 0x1p-500;
                }
            }
            // rescale so that the growth over the last NMB-1 steps stays in range
            double lam = chi + sqrt(dchi * (chi + 1.0));
            int e = ilogb(y) + (int)ceil((NMB - 1) * log2(lam)) - 16;
            int emax = ilogb(y) + 1000;
            if (e > emax) e = emax;
            y = ldexp(y, -e);
            yp = ldexp(yp, -e);
            double Gb[NMB];
            Gb[NMB - 1] = y;
#pragma unroll
            for (int n = NMB - 1; n >= 1; --n) {
                const double fa = 4.0 * n / (2.0 * n - 1.0), fb = (2.0 * n + 1.0) / (2.0 * n - 1.0);
                double up = (n == NMB - 1) ? yp : Gb[n + 1];
                Gb[n - 1] = fa * chi * Gb[n] - fb * up;
            }
            double s = g0 / Gb[0];
#pragma unroll
            for (int n = 1; n < NMB; ++n) G[n] = back ? Gb[n] * s : G[n];
        }
    }
}

// sqrt and reciprocal for positive normal arguments: hardware estimate
// refined by Newton steps (Goldschmidt form for the square root); within a
// few ulp, without the range scaling of the IEEE-rounded library versions.
__device__ __forceinline__ double fast_sqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

__device__ __forceinline__ double fast_rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Start values of one pair: G^(0) = 1 / (2 AGM(rho+, rho-)) and
// G^(1) = G^(0) (1 / (2 r r1)) sum_{n>=1} 2^(n-1) c_n^2 (from E/K by the AGM).
struct PairStart {
    double g0, g1, chi, dchi;
};

__device__ __forceinline__ PairStart pair_start(double rm2, double rp2, double rr, double inv_rr)
{
    double rp = fast_sqrt(rp2), rm = fast_sqrt(rm2);
    double a = rp, b = rm;
    double c = 2.0 * rr * fast_rcp(rp + rm);
    double csum = c * c, w = 1.0;
    for (int it = 0; it < 48; ++it) {
        double an = 0.5 * (a + b);
        b = fast_sqrt(a * b);
        a = an;
        if (c <= 0x1p-30 * a) break;
        c = 0.5 * (a - b);
        w *= 2.0;
        csum = fma(w * c, c, csum);
    }
    PairStart ps;
    ps.g0 = 0.5 * fast_rcp(a);
    ps.g1 = ps.g0 * csum * 0.5 * inv_rr;
    ps.chi = (rp2 + rm2) * 0.25 * inv_rr;
    ps.dchi = rm2 * 0.5 * inv_rr;
    return ps;
}

// Spread the low 11 bits of v to the even bit positions.
__host__ __device__ __forceinline__ uint32_t spread_bits(uint32_t v)
{
    v &= 0x7ffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__host__ __device__ __forceinline__ uint32_t compact_bits(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

// Morton index of box (ir, iz): r bits at odd positions, z bits at even ones.
__host__ __device__ __forceinline__ uint32_t morton(uint32_t ir, uint32_t iz)
{
    return (spread_bits(ir) << 1) | spread_bits(iz);
}

// Box index of a coordinate at a level; the same IEEE operations as the
// definition of the tree: floor(((v - lo) * (1/L)) * 2^level), clamped.
__host__ __device__ __forceinline__ int box_index(double v, double lo, double invL, int level)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double t = __dmul_rn(__dsub_rn(v, lo), invL);
#else
    double t = (v - lo) * invL;
#endif
    double s = t * (double)(1 << level);
    int i = (int)s;
    int nb = 1 << level;
    if (i > nb - 1) i = nb - 1;
    if (i < 0) i = 0;
    return i;
}

// Packed triangle index of (i, j), i + j <= M, i-major.
__host__ __device__ __forceinline__ int tri_index(int M, int i, int j)
{
    return i * (M + 1) - (i * (i - 1)) / 2 + j;
}

// Start of row (a, b) in a compact table {a <= M, b <= M, c <= 2M - a - b},
// rows a-major; row length 2M + 1 - a - b; (M + 1)^3 entries in total.
__host__ __device__ __forceinline__ int table_row(int M, int a, int b)
{
    int K = 2 * M + 1;
    return a * ((M + 1) * K - (M * (M + 1)) / 2) - (M + 1) * ((a * (a - 1)) / 2)
           + b * (K - a) - (b * (b - 1)) / 2;
}

// Slot of separation (dr, dz), 0 <= dr, dz <= 3, not both <= 1, in the
// twelve tables of a radial station.
__host__ __device__ __forceinline__ int geom_slot(int dr, int dz)
{
    // dr = 0,1: dz = 2,3 -> 0..3 ; dr = 2,3: dz = 0..3 -> 4..11
    return dr <= 1 ? dr * 2 + (dz - 2) : 4 + (dr - 2) * 4 + dz;
}

}  // namespace axf

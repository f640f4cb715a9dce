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

// Downward recursion of the modal Green's function,
//   G^(n-1) = A_n chi G^(n) - B_n G^(n+1),  A_n = 4n/(2n-1),  B_n = (2n+1)/(2n-1),
// in rescaled variables G^(n) = w_n z_n with w_(n-1) = B_n w_(n+1), which
// turns every step into one multiply and one fma:
//   z_(n-1) = alpha_n chi z_n - z_(n+1),  alpha_n = A_n rho_n,  rho_n = w_n / w_(n-1).
// rho is anchored at the top (rho = 1 at kMillerMax + 1) and built downward
// by rho_n = 1 / (B_n rho_(n+1)); each entry is consistent with its
// neighbour to one rounding, which is all the rescaling needs.
constexpr int kMillerMax = 1400;
struct DownCoef {
    double alpha[kMillerMax + 2];
    double rho[kMillerMax + 2];
    constexpr DownCoef() : alpha(), rho()
    {
        rho[kMillerMax + 1] = 1.0;
        for (int n = kMillerMax; n >= 1; --n) rho[n] = (2.0 * n - 1.0) / ((2.0 * n + 1.0) * rho[n + 1]);
        for (int n = 1; n < kMillerMax + 2; ++n) alpha[n] = 4.0 * n / (2.0 * n - 1.0) * rho[n];
    }
};
static __constant__ DownCoef c_down = DownCoef();

extern "C" __device__ __attribute__((const)) double __ockl_wfred_min_f64(double);

// Minimum over the wave's lanes (the device library's cross-lane reduction:
// data-parallel lane moves instead of six dependent LDS permutes).
__device__ __forceinline__ double wave_min(double v) { return __ockl_wfred_min_f64(v); }

// Forward-recursion limit.  Rounding in the forward recursion grows like
// lambda^(2n), lambda = chi + sqrt(chi^2 - 1) = e^eta, relative to G^(n).
// The paper's switch chi* = 1.008 for modes up to N = 32 (App. A) allows
// growth e^(2 N eta) = e^(64 acosh 1.008) ~ 3300 at the top mode.  Rounding
// in the forward recursion grows like that factor relative to G^(n) and
// accumulates over the N steps; the pairs just below the switch are among
// the nearest ones, whose terms dominate the sum.  Up to N = 16 the bound
// is kept; above, it shrinks as (16 / N)^3: e^(2 N eta*) = 3300 (16 / N)^3.
// Measured against 40-digit values just below the switch: at most 5e-13
// (N = 16, 23, 32), 2e-13 (47), 3e-13 (63) relative to G^(n).
inline double forward_chi_limit(int nmodes)
{
    int N = nmodes - 1;
    if (N < 2) return 1e300;
    const double growth = 64.0 * __builtin_acosh(1.008) + (N > 16 ? 3.0 * __builtin_log(16.0 / N) : 0.0);
    const double eta = growth / (2.0 * N);
    return 0.5 * (__builtin_exp(eta) + __builtin_exp(-eta));
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
        if (c <= 0x1p-15 * a) break;
        c = 0.5 * (a - b);
        w *= 2.0;
        csum = fma(w * c, c, csum);
    }
    // stopped at c <= 2^-15 a: the next half-difference c' = c^2 / (4 a) is
    // below 2^-32 a and the limit is a - c' to 2^-64, so
    // 1 / limit = (1/a)(1 + c^2 / (4 a^2)); the omitted csum term is ~2^-56.
    PairStart ps;
    const double ra = fast_rcp(a);
    ps.g0 = 0.5 * ra * fma(0.25 * c * c, ra * ra, 1.0);
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

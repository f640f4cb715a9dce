// axf_azimuth.hip -- azimuthal analysis and synthesis (section 2, eqs.
// analysis:source and analysis:phi): samples of a real ring source at
// theta_k = 2 pi k / K -> Fourier coefficients S^(n), n = 0..N, and modal
// potentials Phi^(n) -> potential samples phi(theta_k) with
// Phi^(-n) = conj(Phi^(n)).
//
// Both are direct transforms (K <= AXF_MAX_ANGLES, N <= 63): the work is a
// few multiply-adds per loaded byte, so the kernels are HBM-bound and are
// built for coalescing: samples move through LDS tiles read along the
// contiguous angle index and written along the ring index, and each
// twiddle comes from a table of e^(2 pi i m / K) at the exact index
// m = (n k) mod K, so no phase accumulates rounding.
#include <algorithm>

#include "axf_internal.hpp"

namespace axf {
namespace {

constexpr int kRingsPerBlock = 64;     // one lane per ring
constexpr int kModeGroups = 4;         // waves per block; wave w takes modes w, w + 4, ...
constexpr int kModesPerLane = (AXF_MAX_MODES + kModeGroups - 1) / kModeGroups;
constexpr int kTileAngles = 32;        // angles per staged tile of the analysis

__device__ __forceinline__ void fill_twiddles(double2 *tw, int K)
{
    for (int m = threadIdx.x; m < K; m += blockDim.x) {
        double s, c;
        sincospi(2.0 * m / K, &s, &c);
        tw[m] = make_double2(c, s);
    }
}

// One block per (64 rings, right-hand side).  S^(n) = (1/K) sum_k s_k
// e^(-i n theta_k): lane = ring, wave w accumulates the modes n = w (mod 4).
__global__ __launch_bounds__(256) void k_analysis(int64_t nrings, int K, int nmodes,
                                                  const double *__restrict__ samples,
                                                  double2 *__restrict__ S)
{
    extern __shared__ double2 sh[];
    double2 *tw = sh;                                                  // [K]
    double *tile = reinterpret_cast<double *>(tw + K);                 // [kTileAngles][64]
    const int q = blockIdx.y;
    const int64_t ring0 = (int64_t)blockIdx.x * kRingsPerBlock;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nr = (int)std::min<int64_t>(kRingsPerBlock, nrings - ring0);
    fill_twiddles(tw, K);
    const double *src = samples + ((int64_t)q * nrings + ring0) * K;
    double re[kModesPerLane], im[kModesPerLane];
#pragma unroll
    for (int j = 0; j < kModesPerLane; ++j) re[j] = im[j] = 0.0;
    for (int k0 = 0; k0 < K; k0 += kTileAngles) {
        const int kc = std::min(kTileAngles, K - k0);
        __syncthreads();
        // angle fastest: each ring's run of kc samples is contiguous
        for (int e = threadIdx.x; e < kRingsPerBlock * kTileAngles; e += blockDim.x) {
            const int r = e / kTileAngles, kk = e - r * kTileAngles;
            tile[kk * kRingsPerBlock + r] = (r < nr && kk < kc) ? src[(int64_t)r * K + k0 + kk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kModesPerLane; ++j) {
            const int n = w + kModeGroups * j;
            if (n >= nmodes) break;                       // uniform over the wave
            int m = (int)(((int64_t)n * k0) % K);
            double ar = re[j], ai = im[j];
            for (int kk = 0; kk < kc; ++kk) {
                const double v = tile[kk * kRingsPerBlock + lane];
                const double2 t = tw[m];
                ar = fma(v, t.x, ar);
                ai = fma(-v, t.y, ai);
                m += n;
                if (m >= K) m -= K;
            }
            re[j] = ar;
            im[j] = ai;
        }
    }
    if (lane >= nr) return;
    const double invK = 1.0 / K;
#pragma unroll
    for (int j = 0; j < kModesPerLane; ++j) {
        const int n = w + kModeGroups * j;
        if (n >= nmodes) break;
        S[((int64_t)q * nmodes + n) * nrings + ring0 + lane] = make_double2(re[j] * invK, im[j] * invK);
    }
}

constexpr int kPointsPerBlock = 32;

// One block per (32 points, right-hand side): the modes of the points are
// staged in LDS; each thread forms outputs (point, k) with k fastest, so
// the block writes one contiguous run of 32 K values.
__global__ __launch_bounds__(256) void k_synthesis(int64_t npts, int nmodes, const double2 *__restrict__ phi,
                                                   int K, double *__restrict__ out)
{
    extern __shared__ double2 sh[];
    double2 *tw = sh;                                    // [K]
    double2 *md = tw + K;                                // [nmodes][kPointsPerBlock]
    const int q = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * kPointsPerBlock;
    const int np = (int)std::min<int64_t>(kPointsPerBlock, npts - p0);
    fill_twiddles(tw, K);
    for (int e = threadIdx.x; e < nmodes * kPointsPerBlock; e += blockDim.x) {
        const int n = e / kPointsPerBlock, p = e - n * kPointsPerBlock;
        md[e] = p < np ? phi[((int64_t)q * nmodes + n) * npts + p0 + p] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double *o = out + ((int64_t)q * npts + p0) * K;
    for (int e = threadIdx.x; e < np * K; e += blockDim.x) {
        const int p = e / K, k = e - p * K;
        double v = md[p].x;                              // Re Phi^(0)
        int m = 0;
        double acc = 0.0;
        for (int n = 1; n < nmodes; ++n) {
            m += k;
            if (m >= K) m -= K;                          // m = (n k) mod K
            const double2 c = md[n * kPointsPerBlock + p];
            const double2 t = tw[m];
            acc = fma(c.x, t.x, acc);
            acc = fma(-c.y, t.y, acc);
        }
        o[e] = fma(2.0, acc, v);
    }
}

}  // namespace
}  // namespace axf

using namespace axf;

extern "C" {

axf_status axf_azimuthal_analysis(int64_t nrings, int32_t n_angles, int32_t n_modes, int32_t nrhs,
                                  const double *samples, double *S, void *stream)
{
    try {
        AXF_REQUIRE(samples && S, AXF_ERR_INVALID_ARGUMENT, "samples and S must be non-NULL");
        AXF_REQUIRE(nrings >= 1 && nrhs >= 1, AXF_ERR_INVALID_ARGUMENT, "nrings and nrhs must be >= 1");
        AXF_REQUIRE(n_modes >= 1 && n_modes <= AXF_MAX_MODES, AXF_ERR_UNSUPPORTED, "n_modes must be in 1..64");
        AXF_REQUIRE(n_angles >= 2 * n_modes - 1, AXF_ERR_INVALID_ARGUMENT,
                    "n_angles must be >= 2 n_modes - 1 (modes above n_angles / 2 alias)");
        AXF_REQUIRE(n_angles <= AXF_MAX_ANGLES, AXF_ERR_UNSUPPORTED, "n_angles must be <= 2048");
        AXF_REQUIRE(nrhs <= 65535 && (nrings + kRingsPerBlock - 1) / kRingsPerBlock < (int64_t(1) << 31),
                    AXF_ERR_UNSUPPORTED, "too many rings or right-hand sides");
        const size_t shm = sizeof(double2) * n_angles + sizeof(double) * kTileAngles * kRingsPerBlock;
        dim3 grid((unsigned)((nrings + kRingsPerBlock - 1) / kRingsPerBlock), (unsigned)nrhs);
        if (shm > 65536)
            AXF_HIP(hipFuncSetAttribute((const void *)k_analysis, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)shm));
        k_analysis<<<grid, 256, shm, (hipStream_t)stream>>>(nrings, n_angles, n_modes, samples, (double2 *)S);
        AXF_HIP(hipGetLastError());
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (...) {
        set_error("unexpected internal error");
        return AXF_ERR_HIP;
    }
}

axf_status axf_azimuthal_synthesis(int64_t npts, int32_t n_modes, int32_t nrhs, const double *phi,
                                   int32_t n_angles, double *out, void *stream)
{
    try {
        AXF_REQUIRE(phi && out, AXF_ERR_INVALID_ARGUMENT, "phi and out must be non-NULL");
        AXF_REQUIRE(npts >= 1 && nrhs >= 1, AXF_ERR_INVALID_ARGUMENT, "npts and nrhs must be >= 1");
        AXF_REQUIRE(n_modes >= 1 && n_modes <= AXF_MAX_MODES, AXF_ERR_UNSUPPORTED, "n_modes must be in 1..64");
        AXF_REQUIRE(n_angles >= 1 && n_angles <= AXF_MAX_ANGLES, AXF_ERR_UNSUPPORTED,
                    "n_angles must be in 1..2048");
        AXF_REQUIRE(nrhs <= 65535 && (npts + kPointsPerBlock - 1) / kPointsPerBlock < (int64_t(1) << 31),
                    AXF_ERR_UNSUPPORTED, "too many points or right-hand sides");
        const size_t shm = sizeof(double2) * (n_angles + (size_t)n_modes * kPointsPerBlock);
        dim3 grid((unsigned)((npts + kPointsPerBlock - 1) / kPointsPerBlock), (unsigned)nrhs);
        if (shm > 65536)
            AXF_HIP(hipFuncSetAttribute((const void *)k_synthesis, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)shm));
        k_synthesis<<<grid, 256, shm, (hipStream_t)stream>>>(npts, n_modes, (const double2 *)phi, n_angles, out);
        AXF_HIP(hipGetLastError());
        return AXF_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (...) {
        set_error("unexpected internal error");
        return AXF_ERR_HIP;
    }
}

}  // extern "C"

// axf_tree.hip -- uniform (r, z) quadtree on the device (Algorithm 1, first
// two steps): bounding square, depth, Morton keys, stable radix sort of both
// point sets, leaf offsets, occupied-box slots per level and leaf work chunks.
#include <cstring>
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "axf_device.hpp"
#include "axf_internal.hpp"

namespace axf {

namespace {

constexpr int kBlk = 256;

// Pinned host memory for the plan's readbacks.  A device-to-host copy into
// pageable memory waits for its stream and then copies through a staging
// buffer; into pinned memory it queues like any other copy, and the one
// stream wait that follows covers all of them.  The buffers are pooled for
// the life of the process (never freed, so no HIP call runs at exit).
struct PinnedLease {
    void *p = nullptr;
    size_t cap = 0;
    hipStream_t st = nullptr;
    static std::mutex &mu()
    {
        static std::mutex m;
        return m;
    }
    static std::vector<std::pair<void *, size_t>> &pool()
    {
        static std::vector<std::pair<void *, size_t>> v;
        return v;
    }
    PinnedLease(size_t bytes, hipStream_t s) : st(s)
    {
        {
            std::lock_guard<std::mutex> lock(mu());
            auto &v = pool();
            for (size_t i = 0; i < v.size(); ++i)
                if (v[i].second >= bytes) {
                    p = v[i].first;
                    cap = v[i].second;
                    v.erase(v.begin() + (std::ptrdiff_t)i);
                    return;
                }
        }
        cap = std::max<size_t>(4096, (bytes + 4095) / 4096 * 4096);
        AXF_HIP(hipHostMalloc(&p, cap, hipHostMallocDefault));
    }
    ~PinnedLease()
    {
        if (!p) return;
        (void)hipStreamSynchronize(st);   // no copy into it may still be in flight
        std::lock_guard<std::mutex> lock(mu());
        pool().push_back({p, cap});
    }
    PinnedLease(const PinnedLease &) = delete;
    PinnedLease &operator=(const PinnedLease &) = delete;
};
constexpr int kItems = 8;                 // items per thread in scans
constexpr int kTile = kBlk * kItems;      // 2048
constexpr int kSortItems = 4;             // items per thread in radix-sort tiles
constexpr int kSortTile = kBlk * kSortItems;   // 1024

// ------------------------------------------------------------ bounding box
__global__ void k_bbox_partial(const double *__restrict__ rs, const double *__restrict__ zs, int64_t ns,
                               const double *__restrict__ rf, const double *__restrict__ zf, int64_t nf,
                               double *__restrict__ part)
{
    double rmin = INFINITY, rmax = -INFINITY, zmin = INFINITY, zmax = -INFINITY, bad = 0;
    int64_t n = ns + nf;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double r = i < ns ? rs[i] : rf[i - ns];
        double z = i < ns ? zs[i] : zf[i - ns];
        bool ok = isfinite(r) && isfinite(z) && r > 0.0;
        if (!ok) {
            bad += 1.0;
            continue;
        }
        rmin = fmin(rmin, r);
        rmax = fmax(rmax, r);
        zmin = fmin(zmin, z);
        zmax = fmax(zmax, z);
    }
    __shared__ double sh[5][kBlk];
    int t = threadIdx.x;
    sh[0][t] = rmin; sh[1][t] = rmax; sh[2][t] = zmin; sh[3][t] = zmax; sh[4][t] = bad;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] = fmin(sh[0][t], sh[0][t + s]);
            sh[1][t] = fmax(sh[1][t], sh[1][t + s]);
            sh[2][t] = fmin(sh[2][t], sh[2][t + s]);
            sh[3][t] = fmax(sh[3][t], sh[3][t + s]);
            sh[4][t] += sh[4][t + s];
        }
        __syncthreads();
    }
    if (t < 5) part[blockIdx.x * 5 + t] = sh[t][0];
}

__global__ void k_bbox_final(const double *__restrict__ part, int nb, double *__restrict__ out)
{
    __shared__ double sh[5][kBlk];
    int t = threadIdx.x;
    double v[5] = {INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int b = t; b < nb; b += kBlk) {
        v[0] = fmin(v[0], part[b * 5 + 0]);
        v[1] = fmax(v[1], part[b * 5 + 1]);
        v[2] = fmin(v[2], part[b * 5 + 2]);
        v[3] = fmax(v[3], part[b * 5 + 3]);
        v[4] += part[b * 5 + 4];
    }
    for (int k = 0; k < 5; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] = fmin(sh[0][t], sh[0][t + s]);
            sh[1][t] = fmax(sh[1][t], sh[1][t + s]);
            sh[2][t] = fmin(sh[2][t], sh[2][t + s]);
            sh[3][t] = fmax(sh[3][t], sh[3][t + s]);
            sh[4][t] += sh[4][t + s];
        }
        __syncthreads();
    }
    if (t < 5) out[t] = sh[t][0];
}

// ------------------------------------------------------------------ keys
__global__ void k_keys(const double *__restrict__ r, const double *__restrict__ z, int64_t n, double rlo,
                       double zlo, double invL, int level, uint32_t *__restrict__ key,
                       int32_t *__restrict__ val)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ir = box_index(r[i], rlo, invL, level);
    int iz = box_index(z[i], zlo, invL, level);
    key[i] = morton((uint32_t)ir, (uint32_t)iz);
    if (val) val[i] = (int32_t)i;
}

__global__ void k_hist(const uint32_t *__restrict__ key, int64_t n, int shift, int32_t *__restrict__ hist)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicAdd(&hist[key[i] >> shift], 1);
}

__global__ void k_max_int(const int32_t *__restrict__ a, int64_t n, int32_t *__restrict__ out)
{
    __shared__ int32_t sh[kBlk];
    int32_t m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, a[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sh[0]);
}

// ------------------------------------------------------------------ scan
// Exclusive scan of int32, tiles of kTile items; block sums scanned
// recursively.
__global__ void k_scan_tile(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                            int32_t *__restrict__ sums)
{
    __shared__ int32_t sh[kBlk];
    int t = threadIdx.x;
    int64_t base = blockIdx.x * (int64_t)kTile + (int64_t)t * kItems;
    int32_t v[kItems];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    sh[t] = s;
    __syncthreads();
    for (int o = 1; o < kBlk; o <<= 1) {
        int32_t add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int32_t run = sh[t] - s;   // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (t == kBlk - 1 && sums) sums[blockIdx.x] = sh[t];
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t n, const int32_t *__restrict__ sums)
{
    int64_t base = blockIdx.x * (int64_t)kTile;
    int32_t add = sums[blockIdx.x];
    for (int k = threadIdx.x; k < kTile; k += kBlk)
        if (base + k < n) out[base + k] += add;
}

// ------------------------------------------------------------ radix sort
__global__ void k_rs_hist(const uint32_t *__restrict__ key, int64_t n, int shift, int nblocks,
                          int32_t *__restrict__ counts)
{
    __shared__ int32_t h[256];
    int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * (int64_t)kSortTile;
    for (int k = t; k < kSortTile; k += kBlk) {
        int64_t i = base + k;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// Stable scatter: items are taken in order, 256 per round, ranked within the
// wave by matching digits across ballots and across waves through LDS.
__global__ void k_rs_scatter(const uint32_t *__restrict__ key, const int32_t *__restrict__ val, int64_t n,
                             int shift, int nblocks, const int32_t *__restrict__ offsets,
                             uint32_t *__restrict__ okey, int32_t *__restrict__ oval)
{
    __shared__ int32_t run[256];
    __shared__ int32_t base_off[256];
    __shared__ int32_t wcnt[kBlk / 64][256];
    int t = threadIdx.x;
    int w = t >> 6, lane = t & 63;
    run[t] = 0;
    base_off[t] = offsets[(int64_t)t * nblocks + blockIdx.x];
    for (int k = 0; k < kBlk / 64; ++k) wcnt[k][t] = 0;
    __syncthreads();
    uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int round = 0; round < kSortItems; ++round) {
        int64_t i = blockIdx.x * (int64_t)kSortTile + (int64_t)round * kBlk + t;
        bool act = i < n;
        uint32_t kk = act ? key[i] : 0u;
        int32_t vv = act ? val[i] : 0;
        uint32_t dg = (kk >> shift) & 255u;
        uint64_t match = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (dg >> b) & 1u;
            uint64_t m = __ballot(act && bit);
            match &= bit ? m : ~m;
        }
        int rank = __popcll(match & lt);
        if (act && rank == 0) wcnt[w][dg] = __popcll(match);
        __syncthreads();
        if (act) {
            int pre = run[dg];
            for (int k = 0; k < w; ++k) pre += wcnt[k][dg];
            int pos = base_off[dg] + pre + rank;
            okey[pos] = kk;
            oval[pos] = vv;
        }
        __syncthreads();
        int add = 0;
        for (int k = 0; k < kBlk / 64; ++k) {
            add += wcnt[k][t];
            wcnt[k][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

// ----------------------------------------------------------- structure
__global__ void k_gather_coords(const double *__restrict__ r, const double *__restrict__ z,
                                const int32_t *__restrict__ perm, int64_t n, double *__restrict__ ro,
                                double *__restrict__ zo, double *__restrict__ rinv)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t i = perm[p];
    ro[p] = r[i];
    zo[p] = z[i];
    rinv[p] = 1.0 / r[i];
}

// off[m] = first sorted position with key >= m, m = 0..nleaf
__global__ void k_offsets(const uint32_t *__restrict__ key, int64_t n, int64_t nleaf, int32_t *__restrict__ off)
{
    int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m > nleaf) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)key[mid] < m) lo = mid + 1;
        else hi = mid;
    }
    off[m] = (int32_t)lo;
}

__device__ __forceinline__ int32_t box_count(const int32_t *__restrict__ off, int level, int depth, int b)
{
    int nb = 1 << level;
    int ir = b / nb, iz = b - ir * nb;
    uint32_t m = morton((uint32_t)ir, (uint32_t)iz);
    int sh = 2 * (depth - level);
    return off[(int64_t)(m + 1) << sh] - off[(int64_t)m << sh];
}

// Occupancy flags of the levels 2..depth of both point sets in one array:
// side 0 (sources) then side 1 (field points), each the levels in order,
// level l holding its 4^l boxes (T = sum of 4^l entries per side).
__global__ void k_flags_all(const int32_t *__restrict__ off0, const int32_t *__restrict__ off1, int depth,
                            int64_t T, int32_t *__restrict__ flag)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 2 * T) return;
    const int side = i >= T;
    int64_t r = i - side * T, nbox = 16;
    int l = 2;
    while (r >= nbox) {
        r -= nbox;
        nbox <<= 2;
        ++l;
    }
    flag[i] = box_count(side ? off1 : off0, l, depth, (int)r) > 0 ? 1 : 0;
}

// From the exclusive scan `pre` of those flags: each level's slot map
// (box -> compact index, -1 if empty), its occupied boxes in box order, and
// its count (small[4 + 2 l + side]).  A side's slot maps sit back to back
// from `slot` (level l at sum_{l' < l} 4^l'), its box lists from `box` (level l
// at sum_{l' < l} min(4^l', n)).
__global__ void k_slots_all(const int32_t *__restrict__ flag, const int32_t *__restrict__ pre, int64_t T,
                            int64_t n0, int64_t n1, int32_t *__restrict__ slot0, int32_t *__restrict__ slot1,
                            int32_t *__restrict__ box0, int32_t *__restrict__ box1, int32_t *__restrict__ small)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 2 * T) return;
    const int side = i >= T;
    const int64_t n = side ? n1 : n0;
    int64_t r = i - side * T, nbox = 16, seg = 0, boff = 0;
    int l = 2;
    while (r >= nbox) {
        r -= nbox;
        seg += nbox;
        boff += nbox < n ? nbox : n;
        nbox <<= 2;
        ++l;
    }
    const int32_t rel = pre[i] - pre[side * T + seg];
    int32_t *slot = (side ? slot1 : slot0) + seg;
    int32_t *box = (side ? box1 : box0) + boff;
    if (flag[i]) {
        slot[r] = rel;
        box[rel] = (int32_t)r;
    } else {
        slot[r] = -1;
    }
    if (r == nbox - 1) small[4 + 2 * l + side] = rel + flag[i];
}

__global__ void k_chunk_count(const int32_t *__restrict__ off, const int32_t *__restrict__ box, int nocc,
                              int depth, int32_t *__restrict__ nch, int32_t *__restrict__ maxleaf)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nocc) return;
    int c = box_count(off, depth, depth, box[k]);
    nch[k] = (c + 63) / 64;
    atomicMax(maxleaf, c);
}

__global__ void k_chunk_fill(const int32_t *__restrict__ off, const int32_t *__restrict__ box, int nocc,
                             int depth, const int32_t *__restrict__ pre, int4 *__restrict__ chunks,
                             int32_t *__restrict__ total)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nocc) return;
    int b = box[k];
    int nb = 1 << depth;
    int ir = b / nb, iz = b - ir * nb;
    uint32_t m = morton((uint32_t)ir, (uint32_t)iz);
    int first = off[m], cnt = off[m + 1] - first;
    int c0 = pre[k];
    for (int j = 0; j * 64 < cnt; ++j)
        chunks[c0 + j] = make_int4(k, first + j * 64, min(64, cnt - j * 64), b);
    if (k == nocc - 1) *total = c0 + (cnt + 63) / 64;
}

// Work counts: near-field pairs (targets x sources of the 3x3 neighbour
// leaves) and S2L box pairs (occupied source boxes in each occupied target
// box's interaction list).
// Adds the block's per-thread counts v[0..1] to out[0..1]: summed in LDS,
// then one global atomic per counter and block.  Every thread of the block
// must call it.
__device__ __forceinline__ void block_count_add(unsigned long long v0, unsigned long long v1,
                                                unsigned long long *__restrict__ out, int nout)
{
    __shared__ unsigned long long acc[2];
    if (threadIdx.x < 2) acc[threadIdx.x] = 0;
    __syncthreads();
    if (v0) atomicAdd(&acc[0], v0);
    if (nout > 1 && v1) atomicAdd(&acc[1], v1);
    __syncthreads();
    if ((int)threadIdx.x < nout && acc[threadIdx.x]) atomicAdd(out + threadIdx.x, acc[threadIdx.x]);
}

__global__ void k_count_near(const int32_t *__restrict__ toff, const int32_t *__restrict__ soff,
                             const int32_t *__restrict__ tbox, int nocc, int depth,
                             unsigned long long *__restrict__ out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    long long nt = 0, ns = 0;
    if (k < nocc) {
        int nb = 1 << depth;
        int b = tbox[k];
        int ir = b / nb, iz = b - ir * nb;
        nt = box_count(toff, depth, depth, b);
        for (int jr = max(ir - 1, 0); jr <= min(ir + 1, nb - 1); ++jr)
            for (int jz = max(iz - 1, 0); jz <= min(iz + 1, nb - 1); ++jz)
                ns += box_count(soff, depth, depth, jr * nb + jz);
    }
    block_count_add((unsigned long long)(nt * ns), 0, out, 1);
}

__global__ void k_count_s2l(const int32_t *__restrict__ tbox, int nocc, const int32_t *__restrict__ sslot,
                            int level, unsigned long long *__restrict__ out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0, u = 0;
    const int nb = 1 << level;
    const int b = k < nocc ? tbox[k] : 0;
    const int ir = b / nb, iz = b - ir * nb;
    const int zlo = 2 * (iz >> 1) - 2, zhi = 2 * (iz >> 1) + 4;   // z window of the list
    for (int jr = 2 * (ir >> 1) - 2; k < nocc && jr < 2 * (ir >> 1) + 4; ++jr) {
        if (jr < 0 || jr >= nb) continue;
        const bool near_r = abs(jr - ir) <= 1;
        // offset units: source boxes at z distance +adz and -adz share one
        // contraction; a unit counts if either of its boxes is occupied
        for (int adz = 0; adz <= 3; ++adz) {
            if (near_r && adz <= 1) continue;
            bool occ = false;
            for (int sgn = -1; sgn <= (adz > 0 ? 1 : -1); sgn += 2) {
                const int jz = iz + sgn * adz;
                if (jz < zlo || jz >= zhi || jz < 0 || jz >= nb) continue;
                if (sslot[jr * nb + jz] >= 0) {
                    ++c;
                    occ = true;
                }
            }
            u += occ;
        }
    }
    block_count_add((unsigned long long)c, (unsigned long long)u, out, 2);
}

inline int nblk(int64_t n, int b = kBlk) { return (int)((n + b - 1) / b); }

// Recursive exclusive scan; tmp must hold scan_tmp_ints(n) ints.
int64_t scan_tmp_ints(int64_t n)
{
    int64_t tot = 0;
    while (n > 1) {
        int64_t nb = (n + kTile - 1) / kTile;
        tot += nb + 64;
        n = nb;
    }
    return tot + 64;
}

void scan_excl(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t st)
{
    if (n <= 0) return;
    int64_t nb = (n + kTile - 1) / kTile;
    if (nb == 1) {
        k_scan_tile<<<1, kBlk, 0, st>>>(in, out, n, nullptr);
        return;
    }
    int32_t *sums = tmp;
    int32_t *rest = tmp + nb + 64;
    k_scan_tile<<<(int)nb, kBlk, 0, st>>>(in, out, n, sums);
    scan_excl(sums, sums, nb, rest, st);
    k_scan_add<<<(int)nb, kBlk, 0, st>>>(out, n, sums);
}

struct SortBufs {
    uint32_t *k0, *k1;
    int32_t *v0, *v1;
    int32_t *counts;
    int32_t *tmp;
};

// Stable LSD radix sort of (key, val) on the low `bits` bits; result in k0/v0.
void radix_sort(SortBufs &b, int64_t n, int bits, hipStream_t st)
{
    int nblocks = (int)((n + kSortTile - 1) / kSortTile);
    uint32_t *ka = b.k0, *kb = b.k1;
    int32_t *va = b.v0, *vb = b.v1;
    for (int shift = 0; shift < bits; shift += 8) {
        k_rs_hist<<<nblocks, kBlk, 0, st>>>(ka, n, shift, nblocks, b.counts);
        scan_excl(b.counts, b.counts, (int64_t)256 * nblocks, b.tmp, st);
        k_rs_scatter<<<nblocks, kBlk, 0, st>>>(ka, va, n, shift, nblocks, b.counts, kb, vb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != b.k0) {
        AXF_HIP(hipMemcpyAsync(b.k0, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
        AXF_HIP(hipMemcpyAsync(b.v0, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
}

struct PointScratch {
    uint32_t *key11;      // keys at the deepest level (auto depth only)
    SortBufs sb;
};

}  // namespace

void build_tree(Plan &pl, const double *rs, const double *zs, const double *rf, const double *zf,
                hipStream_t st, const std::function<void()> &after_depth)
{
    const int64_t ns = pl.src.n, nf = pl.fld.n;
    const int64_t nmax = std::max(ns, nf);
    const bool autod = pl.p.depth == 0;

    // ---- point arena: sorted coordinates, permutations, gathered strengths, sort scratch
    Sizer sz;
    sz.add<double>(5 * 1024 + 8);              // bbox partials + result
    for (int64_t n : {ns, nf}) {
        sz.add<double>(n);
        sz.add<double>(n);
        sz.add<double>(n);
        sz.add<int32_t>(n);
    }
    sz.add<double2>((size_t)nmax * pl.Cs);     // gathered strengths
    sz.add<double>(2 * (size_t)ns);            // adjoint coordinate-gradient scratch
    const int64_t nb11 = autod ? ((int64_t)1 << (2 * AXF_MAX_DEPTH)) : 0;
    if (autod) {
        sz.add<uint32_t>(ns);
        sz.add<uint32_t>(nf);
        sz.add<int32_t>(nb11);
        sz.add<int32_t>(nb11);
    }
    sz.add<uint32_t>(nmax);
    sz.add<uint32_t>(nmax);
    sz.add<int32_t>(nmax);
    sz.add<int32_t>(nmax);
    int64_t cnt_ints = 256 * ((nmax + kSortTile - 1) / kSortTile);
    sz.add<int32_t>(cnt_ints);
    // scans: sort counts, chunk counts (<= 4^d) and the occupancy flags of
    // every level of both sides (< 3 * 4^d)
    int64_t tmp_ints = std::max<int64_t>(scan_tmp_ints(cnt_ints), scan_tmp_ints((int64_t)3 << (2 * AXF_MAX_DEPTH)));
    sz.add<int32_t>(tmp_ints);
    sz.add<int32_t>(64);
    sz.add<unsigned long long>(4);
    pl.points = arena_acquire(sz.bytes + 4096);
    Arena &A = pl.points;
    double *bb = A.take<double>(5 * 1024 + 8);
    pl.src.r = A.take<double>(ns);
    pl.src.z = A.take<double>(ns);
    pl.src.rinv = A.take<double>(ns);
    pl.src.perm = A.take<int32_t>(ns);
    pl.fld.r = A.take<double>(nf);
    pl.fld.z = A.take<double>(nf);
    pl.fld.rinv = A.take<double>(nf);
    pl.fld.perm = A.take<int32_t>(nf);
    pl.Sg = A.take<double2>((size_t)nmax * pl.Cs);
    pl.gsum = A.take<double>(2 * (size_t)ns);
    uint32_t *k11s = nullptr, *k11f = nullptr;
    int32_t *hs = nullptr, *hf = nullptr;
    if (autod) {
        k11s = A.take<uint32_t>(ns);
        k11f = A.take<uint32_t>(nf);
        hs = A.take<int32_t>(nb11);
        hf = A.take<int32_t>(nb11);
    }
    SortBufs sb;
    sb.k0 = A.take<uint32_t>(nmax);
    sb.k1 = A.take<uint32_t>(nmax);
    sb.v0 = A.take<int32_t>(nmax);
    sb.v1 = A.take<int32_t>(nmax);
    sb.counts = A.take<int32_t>(cnt_ints);
    sb.tmp = A.take<int32_t>(tmp_ints);
    int32_t *small = A.take<int32_t>(64);
    unsigned long long *cnt64 = A.take<unsigned long long>(4);

    // ---- bounding square and validation
    int nbb = std::min<int64_t>(1024, std::max<int64_t>(1, (ns + nf + kBlk - 1) / kBlk));
    k_bbox_partial<<<nbb, kBlk, 0, st>>>(rs, zs, ns, rf, zf, nf, bb);
    k_bbox_final<<<1, kBlk, 0, st>>>(bb, nbb, bb + 5 * 1024);
    // pinned readback area: bounding box (5 doubles), the small counters
    // (64 ints), the pair counts (4 x 64 bits) and the depth rule's maximum
    PinnedLease rb(1024, st);
    double *pin_box = static_cast<double *>(rb.p);
    int32_t *pin_small = reinterpret_cast<int32_t *>(static_cast<char *>(rb.p) + 64);
    unsigned long long *pin_cnt = reinterpret_cast<unsigned long long *>(static_cast<char *>(rb.p) + 64 + 256);
    int32_t *pin_max = reinterpret_cast<int32_t *>(static_cast<char *>(rb.p) + 512);
    double box[5];
    AXF_HIP(hipMemcpyAsync(pin_box, bb + 5 * 1024, sizeof(box), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipStreamSynchronize(st));
    std::memcpy(box, pin_box, sizeof(box));
    AXF_REQUIRE(box[4] == 0.0, AXF_ERR_INVALID_GEOMETRY,
                "a coordinate is not finite or a ring radius is <= 0");
    square_rule(box[0], box[1], box[2], box[3], pl.rlo, pl.zlo, pl.L, pl.koff);
    pl.rmax = box[1];
    pl.invL = 1.0 / pl.L;

    // ---- depth
    int d = pl.p.depth;
    if (autod) {
        k_keys<<<nblk(ns), kBlk, 0, st>>>(rs, zs, ns, pl.rlo, pl.zlo, pl.invL, AXF_MAX_DEPTH, k11s, nullptr);
        k_keys<<<nblk(nf), kBlk, 0, st>>>(rf, zf, nf, pl.rlo, pl.zlo, pl.invL, AXF_MAX_DEPTH, k11f, nullptr);
        auto max_count = [&](int dd) {
            int64_t nl = (int64_t)1 << (2 * dd);
            AXF_HIP(hipMemsetAsync(hs, 0, nl * sizeof(int32_t), st));
            AXF_HIP(hipMemsetAsync(hf, 0, nl * sizeof(int32_t), st));
            AXF_HIP(hipMemsetAsync(small, 0, sizeof(int32_t), st));
            int sh = 2 * (AXF_MAX_DEPTH - dd);
            k_hist<<<nblk(ns), kBlk, 0, st>>>(k11s, ns, sh, hs);
            k_hist<<<nblk(nf), kBlk, 0, st>>>(k11f, nf, sh, hf);
            int g = (int)std::min<int64_t>(1024, (nl + kBlk - 1) / kBlk);
            k_max_int<<<g, kBlk, 0, st>>>(hs, nl, small);
            k_max_int<<<g, kBlk, 0, st>>>(hf, nl, small);
            AXF_HIP(hipMemcpyAsync(pin_max, small, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            AXF_HIP(hipStreamSynchronize(st));
            return (int)*pin_max;
        };
        double est = std::log((double)nmax / std::max(1, pl.p.max_leaf)) / std::log(4.0);
        d = std::max(2, std::min(AXF_MAX_DEPTH, (int)std::ceil(est)));
        if (max_count(d) <= pl.p.max_leaf) {
            while (d > 2 && max_count(d - 1) <= pl.p.max_leaf) --d;
        } else {
            while (d < AXF_MAX_DEPTH && max_count(d) > pl.p.max_leaf) ++d;
        }
    }
    pl.d = d;
    after_depth();

    // ---- per side: keys at depth d, sort, gather coordinates
    const int bits = 2 * d;
    struct In {
        Side *s;
        const double *r, *z;
    } ins[2] = {{&pl.src, rs, zs}, {&pl.fld, rf, zf}};
    // structure arena sized by depth
    const int64_t nleaf = (int64_t)1 << (2 * d);
    // boxes of the levels 2..d (slot maps) and their occupied bound per side
    int64_t tlev = 0, blev[2] = {0, 0};
    for (int l = 2; l <= d; ++l) {
        tlev += (int64_t)1 << (2 * l);
        for (int side = 0; side < 2; ++side) blev[side] += std::min<int64_t>((int64_t)1 << (2 * l), ins[side].s->n);
    }
    const int64_t nflag = std::max<int64_t>(nleaf + 1, 2 * tlev);
    Sizer ss;
    for (int side = 0; side < 2; ++side) {
        int64_t n = ins[side].s->n;
        ss.add<int32_t>(nleaf + 1);
        ss.add<int32_t>(tlev);
        ss.add<int32_t>(blev[side]);
        int64_t nocc_max = std::min<int64_t>(nleaf, n);
        ss.add<int4>(nocc_max + n / 64 + 1);
    }
    ss.add<int32_t>(nflag);   // flags / chunk counts
    ss.add<int32_t>(nflag);   // prefix
    pl.tree = arena_acquire(ss.bytes + 4096);
    Arena &T = pl.tree;
    for (int side = 0; side < 2; ++side) {
        Side &s = *ins[side].s;
        s.off = T.take<int32_t>(nleaf + 1);
        int32_t *slot_all = T.take<int32_t>(tlev);
        int32_t *box_all = T.take<int32_t>(blev[side]);
        int64_t so = 0, bo = 0;
        for (int l = 2; l <= d; ++l) {
            s.slot[l] = slot_all + so;
            s.box[l] = box_all + bo;
            so += (int64_t)1 << (2 * l);
            bo += std::min<int64_t>((int64_t)1 << (2 * l), s.n);
        }
        s.chunks = T.take<int4>(std::min<int64_t>(nleaf, s.n) + s.n / 64 + 1);
    }
    int32_t *flag = T.take<int32_t>(nflag);
    int32_t *pre = T.take<int32_t>(nflag);

    // small[] layout: [0..1] maxleaf per side, [2..3] nchunks, [4 + 2*l + side] nocc
    AXF_HIP(hipMemsetAsync(small, 0, 64 * sizeof(int32_t), st));
    for (int side = 0; side < 2; ++side) {
        Side &s = *ins[side].s;
        int64_t n = s.n;
        k_keys<<<nblk(n), kBlk, 0, st>>>(ins[side].r, ins[side].z, n, pl.rlo, pl.zlo, pl.invL, d, sb.k0, sb.v0);
        radix_sort(sb, n, bits, st);
        AXF_HIP(hipMemcpyAsync(s.perm, sb.v0, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        k_gather_coords<<<nblk(n), kBlk, 0, st>>>(ins[side].r, ins[side].z, s.perm, n, s.r, s.z, s.rinv);
        k_offsets<<<nblk(nleaf + 1), kBlk, 0, st>>>(sb.k0, n, nleaf, s.off);
    }
    // occupied boxes of every level of both sides: one flag pass, one scan
    k_flags_all<<<nblk(2 * tlev), kBlk, 0, st>>>(pl.src.off, pl.fld.off, d, tlev, flag);
    scan_excl(flag, pre, 2 * tlev, sb.tmp, st);
    k_slots_all<<<nblk(2 * tlev), kBlk, 0, st>>>(flag, pre, tlev, pl.src.n, pl.fld.n, pl.src.slot[2], pl.fld.slot[2],
                                                 pl.src.box[2], pl.fld.box[2], small);
    // occupancy counts are needed to size the leaf work lists
    int32_t h_small[64];
    AXF_HIP(hipMemcpyAsync(pin_small, small, sizeof(h_small), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipStreamSynchronize(st));
    std::memcpy(h_small, pin_small, sizeof(h_small));
    for (int side = 0; side < 2; ++side) {
        Side &s = *ins[side].s;
        for (int l = 2; l <= d; ++l) s.nocc[l] = h_small[4 + 2 * l + side];
        int nocc = s.nocc[d];
        k_chunk_count<<<nblk(nocc), kBlk, 0, st>>>(s.off, s.box[d], nocc, d, flag, small + side);
        scan_excl(flag, pre, nocc, sb.tmp, st);
        k_chunk_fill<<<nblk(nocc), kBlk, 0, st>>>(s.off, s.box[d], nocc, d, pre, s.chunks, small + 2 + side);
    }
    AXF_HIP(hipMemsetAsync(cnt64, 0, 4 * sizeof(unsigned long long), st));
    k_count_near<<<nblk(pl.fld.nocc[d]), kBlk, 0, st>>>(pl.fld.off, pl.src.off, pl.fld.box[d], pl.fld.nocc[d], d,
                                                        cnt64);
    for (int l = 2; l <= d; ++l)
        k_count_s2l<<<nblk(pl.fld.nocc[l]), kBlk, 0, st>>>(pl.fld.box[l], pl.fld.nocc[l], pl.src.slot[l], l,
                                                           cnt64 + 1);
    unsigned long long h_cnt[4];
    AXF_HIP(hipMemcpyAsync(pin_small, small, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    AXF_HIP(hipMemcpyAsync(pin_cnt, cnt64, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
    // the occupied boxes of every level (the S2L tiles are made from them on
    // the host) come back with the counts: one wait for both, one copy per
    // side (its box lists sit back to back, up to the last occupied box of
    // the finest level)
    {
        size_t total = 0, base[2], len[2];
        for (int side = 0; side < 2; ++side) {
            const Side &s = *ins[side].s;
            base[side] = total;
            for (int l = 2; l <= d; ++l) pl.box_host_off[side][l] = total + (size_t)(s.box[l] - s.box[2]);
            len[side] = (size_t)(s.box[d] - s.box[2]) + s.nocc[d];
            total += len[side];
        }
        pl.box_host.resize(std::max<size_t>(total, 1));
        PinnedLease bl(sizeof(int32_t) * pl.box_host.size(), st);
        int32_t *pin_boxes = static_cast<int32_t *>(bl.p);
        for (int side = 0; side < 2; ++side)
            AXF_HIP(hipMemcpyAsync(pin_boxes + base[side], ins[side].s->box[2], len[side] * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, st));
        AXF_HIP(hipStreamSynchronize(st));
        std::memcpy(pl.box_host.data(), pin_boxes, sizeof(int32_t) * total);
    }
    std::memcpy(h_small, pin_small, 4 * sizeof(int32_t));
    std::memcpy(h_cnt, pin_cnt, sizeof(h_cnt));
    pl.near_pairs = (int64_t)h_cnt[0];
    pl.s2l_pairs = (int64_t)h_cnt[1];
    pl.s2l_units = (int64_t)h_cnt[2];
    pl.src.max_leaf = h_small[0];
    pl.fld.max_leaf = h_small[1];
    pl.src.nchunks = h_small[2];
    pl.fld.nchunks = h_small[3];
}

// S2L tiles: occupied target boxes grouped by (station, z parity), TB per
// tile, for both sides (the adjoint uses the sources as targets).
void build_tiles(Plan &pl, hipStream_t st)
{
    const int TB = pl.tb;
    Side *sides[2] = {&pl.src, &pl.fld};
    constexpr int NL = AXF_MAX_DEPTH + 1;
    // every level's box list of both sides, copied back with the tree counts
    std::vector<std::vector<int4>> tiles(2 * NL);
    std::vector<std::vector<int32_t>> slots(2 * NL);
    for (int si = 0; si < 2; ++si) {
        for (int l = 2; l <= pl.d; ++l) {
            const int n = sides[si]->nocc[l];
            const int32_t *bx = pl.box_host.data() + pl.box_host_off[si][l];
            const int nb = 1 << l;
            auto &tv = tiles[si * NL + l];
            auto &sv = slots[si * NL + l];
            // boxes are station-major in slot order; the vector S2L splits each
            // station by z parity (one offset set per tile), the matrix-core
            // S2L takes a station's boxes in order (each box its own parity)
            int k = 0;
            while (k < n) {
                int station = bx[k] / nb, e = k;
                while (e < n && bx[e] / nb == station) ++e;
                for (int par = 0; par < (pl.mfma ? 1 : 2); ++par) {
                    int first = (int)sv.size();
                    for (int j = k; j < e; ++j)
                        if (pl.mfma || ((bx[j] - station * nb) & 1) == par) sv.push_back(j);
                    for (int f = first; f < (int)sv.size(); f += TB)
                        tv.push_back(make_int4(station, par, f, std::min(TB, (int)sv.size() - f)));
                }
                k = e;
            }
        }
    }
    Sizer sz;
    for (int si = 0; si < 2; ++si)
        for (int l = 2; l <= pl.d; ++l) {
            sz.add<int4>(std::max<size_t>(1, tiles[si * NL + l].size()));
            sz.add<int32_t>(std::max<size_t>(1, slots[si * NL + l].size()));
        }
    pl.tilemem = arena_acquire(sz.bytes + 4096);
    // the arena's image on the host, filled in place and copied once; the
    // plan keeps it until the copy has run
    std::vector<char> &img = pl.tile_host;
    img.assign(sz.bytes + 4096, 0);
    for (int si = 0; si < 2; ++si) {
        Side &s = *sides[si];
        for (int l = 2; l <= pl.d; ++l) {
            auto &tv = tiles[si * NL + l];
            auto &sv = slots[si * NL + l];
            s.tiles[l] = pl.tilemem.take<int4>(std::max<size_t>(1, tv.size()));
            s.tile_slots[l] = pl.tilemem.take<int32_t>(std::max<size_t>(1, sv.size()));
            s.ntiles[l] = (int)tv.size();
            if (!tv.empty())
                std::memcpy(img.data() + ((char *)s.tiles[l] - pl.tilemem.base), tv.data(), tv.size() * sizeof(int4));
            if (!sv.empty())
                std::memcpy(img.data() + ((char *)s.tile_slots[l] - pl.tilemem.base), sv.data(),
                            sv.size() * sizeof(int32_t));
        }
    }
    if (pl.tilemem.used)
        AXF_HIP(hipMemcpyAsync(pl.tilemem.base, img.data(), pl.tilemem.used, hipMemcpyHostToDevice, st));
}

}  // namespace axf

// pool.hip -- the dynamic per-range domain pool (Sec. 3.1).
//
// The paper keeps the domain dimensions in a height-balanced search tree and
// asks it, per range, for the domains inside d_r - D_f <= d_d <= d_r + D_f.
// The same sets come out of a static order: the domains sorted by dimension
// (stable, so equal values keep ascending index) and, per range, the interval
// [lo, hi) of positions that satisfy the window. fp64 subtraction is
// monotone, so the membership test |fd_d - fd_r| <= tol + 1e-9 holds on one
// contiguous run of the sorted order and two binary searches find it.
//
// The sort is a stable LSD radix sort over 8-bit digits of an
// order-preserving integer image of the keys: per block digit histograms, one
// exclusive scan over (digit, block), and a
// scatter that ranks equal digits by position with wave ballots, so every
// pass is stable. A pass whose digit is the same for every key is skipped
// (decided on the device). Small arrays are sorted by one workgroup in LDS.
#include "fic_internal.h"

namespace fic {

namespace {

constexpr int kSortThreads = 1024;
constexpr int kSortPerThread = 4;
constexpr int kSortTile = kSortThreads * kSortPerThread;   // keys per block
constexpr int kSortWaves = kSortThreads / 64;

// Digit runs of the per-tile counts are padded to a multiple of 16 tiles,
// so the scan gives every thread of a block 16-byte aligned runs.
inline __host__ __device__ int64_t padded_tiles(int64_t nb) { return (nb + 15) & ~(int64_t)15; }

// Exclusive scan of m uint32 entries in three launches: per-tile scans of
// kScanTile entries, a scan of the tile totals, and the carry-in add.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // inclusive scan inside each wave, then across the 4 wave totals
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += sh[w];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return base + x - v;
}

// One tile's scan; with a single tile (gridDim.x == 1) the total also goes
// to *grand (nullable), so no totals pass is needed.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t *__restrict__ a, int64_t m,
                                                             uint32_t *__restrict__ tile_tot,
                                                             uint32_t *__restrict__ grand)
{
    __shared__ uint32_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < m ? a[base + i] : 0u;
        sum += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, sh, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < m) a[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) {
        tile_tot[blockIdx.x] = total;
        if (grand && gridDim.x == 1) *grand = total;
    }
}

// Scan of the tile totals (one block, any count), total to *total.
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(uint32_t *__restrict__ t, int64_t nt,
                                                              uint32_t *__restrict__ total)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (int64_t b = 0; b < nt; b += kScanThreads) {
        const int64_t i = b + threadIdx.x;
        const uint32_t v = i < nt ? t[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, sh, tot);
        if (i < nt) t[i] = carry + ex;
        carry += tot;
    }
    if (total && threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint32_t *__restrict__ a, int64_t m,
                                                           const uint32_t *__restrict__ tile_off)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    const uint32_t off = tile_off[blockIdx.x];
    if (blockIdx.x == 0) return;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < m) a[base + i] += off;
}

// Order-preserving integer image of an fp64 value, and its inverse.
__device__ inline u64 fd_bits(double x)
{
    u64 b = (u64)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline double fd_of_bits(u64 k)
{
    const u64 b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Control words of one multi-block sort (in its workspace): cur[p] is where
// the data is before pass p (0: the caller's arrays, 1: the alternate
// ones). Pass 0 starts in the caller's arrays without reading cur[0]; each
// pass's scatter writes the next entry before a later kernel reads it.
constexpr int kMaxPasses = 8;
struct SortCtl {
    uint32_t cur[kMaxPasses + 1];
};

// Up to this many tiles, each scatter workgroup sums its digit offsets from
// the tile counts itself (at most 64 x 256 counts per workgroup), so a pass
// takes two launches instead of three.
constexpr int kFusedScanTiles = 64;

// Exclusive scan over the 1024 threads of a block (16 waves); *total gets
// the sum. All threads must call it.
__device__ inline uint32_t block_scan_1024(uint32_t v, uint32_t *wsum, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t base = 0, all = 0;
    for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t t = wsum[w];
        if (w < wave) base += t;
        all += t;
    }
    total = all;
    __syncthreads();
    return base + x - v;
}

// Lanes of the wave whose 8-bit digit equals this lane's (valid lanes only).
__device__ __forceinline__ u64 digit_peers(uint32_t d, bool valid)
{
    u64 peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const u64 bb = __ballot((d >> bit) & 1u);
        peers &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    return peers;
}

// Pass `pass` (digit at bit `shift`) of the multi-block sort, step 1: per
// tile digit counts into cnt (digit-major: cnt[d * nbp + tile], nbp = nb
// padded to 16).
// Keys of equal digit in a wave are counted together: one LDS atomic per
// (wave, digit), not one per key (nearby dimensions crowd a few digits).
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const u64 *__restrict__ ka,
                                                            const u64 *__restrict__ kb, int64_t n,
                                                            int shift, int pass,
                                                            uint32_t *__restrict__ cnt, int nb,
                                                            const SortCtl *ctl)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    const u64 *keys = (pass && ctl->cur[pass]) ? kb : ka;   // written by the previous pass's scatter
    if (tid < 256) h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const u64 lt = (1ull << (tid & 63)) - 1ull;
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)(keys[i] >> shift) & 255u : 0u;
        const u64 peers = digit_peers(d, valid);
        if (valid && (peers & lt) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    if (tid < 256) cnt[(int64_t)tid * padded_tiles(nb) + blockIdx.x] = h[tid];
}

// Step 2: one workgroup per digit d scans its run of tile counts in place
// (exclusive; the position of each tile's keys among the digit's keys) and
// writes the digit's total to tot[d].
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t *__restrict__ cnt, int nb,
                                                   uint32_t *__restrict__ tot)
{
    __shared__ uint32_t sh[4];
    const int d = blockIdx.x, tid = threadIdx.x;
    uint32_t *row = cnt + (int64_t)d * padded_tiles(nb);
    uint32_t carry = 0;
    for (int t0 = 0; t0 < nb; t0 += 256) {
        const int t = t0 + tid;
        const uint32_t v = t < nb ? row[t] : 0u;
        uint32_t all;
        const uint32_t ex = block_exclusive_scan(v, sh, all);
        if (t < nb) row[t] = carry + ex;
        carry += all;
    }
    if (tid == 0) tot[d] = carry;
}

// Step 3: stable scatter of each tile by the digit: equal digits are ranked
// by position with wave ballots, waves in order (one thread per digit
// tabulates each wave's offset once per round), rounds in order. A tile's
// start position of digit d is (keys of smaller digits) + (keys of digit d in
// earlier tiles): from the scan (offs, tot) or, with fused (nb <=
// kFusedScanTiles), summed here from the raw tile counts. A pass in which
// one digit holds all n keys would not change the order and is skipped;
// block 0 records where the data is for the next pass.
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    u64 *__restrict__ ka, uint32_t *__restrict__ va, u64 *__restrict__ kb,
    uint32_t *__restrict__ vb, int64_t n, int shift, int pass, const uint32_t *__restrict__ offs,
    const uint32_t *__restrict__ tot, int nb, int fused, SortCtl *ctl)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[kSortWaves][256];     // per-wave digit counts (zero between uses)
    __shared__ uint32_t wo[kSortWaves][256];     // per-wave digit offsets
    __shared__ uint32_t wsum[kSortWaves];
    __shared__ int skip;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) skip = 0;
    for (int i = tid; i < kSortWaves * 256; i += kSortThreads) (&wc[0][0])[i] = 0u;
    __syncthreads();
    uint32_t t = 0, before = 0;
    if (tid < 256) {
        const uint32_t *row = offs + (int64_t)tid * padded_tiles(nb);
        if (fused) {
            for (int b = 0; b < nb; ++b) {
                const uint32_t c = row[b];
                before += b < (int)blockIdx.x ? c : 0u;
                t += c;
            }
        } else {
            t = tot[tid];
            before = row[blockIdx.x];
        }
    }
    if (tid < 256 && (int64_t)t == n) skip = 1;
    uint32_t all;
    const uint32_t dbase = block_scan_1024(t, wsum, all);     // digits >= 256 add 0
    const uint32_t cur = pass ? ctl->cur[pass] : 0u;
    const bool skipped = skip != 0;
    if (blockIdx.x == 0 && tid == 0) ctl->cur[pass + 1] = skipped ? cur : (cur ^ 1u);
    if (skipped) return;                            // block-uniform
    const u64 *kin = cur ? kb : ka;
    const uint32_t *vin = cur ? vb : va;
    u64 *kout = cur ? ka : kb;
    uint32_t *vout = cur ? va : vb;
    if (tid < 256) run[tid] = dbase + before;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const u64 lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * kSortThreads + tid;
        const bool valid = i < n;
        const u64 key = valid ? kin[i] : 0ull;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const u64 peers = digit_peers(d, valid);
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[wave][d] = __popcll(peers);
        __syncthreads();
        if (tid < 256) {
            // digit tid: offsets of the waves in order, the counts cleared
            uint32_t acc = run[tid];
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t c = wc[w][tid];
                wo[w][tid] = acc;
                wc[w][tid] = 0u;
                acc += c;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wo[wave][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
    }
}

// The sorted data back into the caller's arrays when it ended in the
// alternate ones; with fd_out (nullable), the sorted keys read as fd_bits
// images are decoded into it (the sorted fp64 values).
__global__ void k_sort_finish(u64 *__restrict__ ka, uint32_t *__restrict__ va,
                              const u64 *__restrict__ kb, const uint32_t *__restrict__ vb,
                              int64_t n, int passes, const SortCtl *ctl, double *__restrict__ fd_out)
{
    const bool moved = ctl->cur[passes] != 0u;
    if (!moved && !fd_out) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 k = moved ? kb[i] : ka[i];
    if (moved) {
        ka[i] = k;
        va[i] = vb[i];
    }
    if (fd_out) fd_out[i] = fd_of_bits(k);
}

// Up to kSmallSort pairs: the whole sort in one workgroup, in LDS. Per pass
// a digit histogram, its scan (a pass where one digit holds every key is
// skipped) and a stable scatter of the keys in index order, 1024 at a time.
// Keys of equal digit inside a wave find each other by ballots over the
// digit's bits: the histogram takes one LDS atomic per (wave, digit) instead
// of one per key (the digits of nearby fractal dimensions crowd a few bins),
// and a key's position is its digit's offset for its wave (run of the digit
// plus the counts of the waves before it, tabulated once per 1024 keys by
// one thread per digit) plus its rank among its wave's equal digits.
constexpr int kSmallThreads = 1024;
constexpr int kSmallSort = 4096;
constexpr int kSmallWaves = kSmallThreads / kWave;

__global__ __launch_bounds__(kSmallThreads) void k_sort_small(u64 *__restrict__ keys,
                                                              uint32_t *__restrict__ vals, int n,
                                                              int passes, double *__restrict__ fd_out)
{
    __shared__ u64 sk[2][kSmallSort];
    __shared__ uint32_t sv[2][kSmallSort];
    __shared__ uint32_t hist[256], run[256], wsum[4];
    __shared__ uint32_t wc[kSmallWaves][256];    // per-wave digit counts (zero between uses)
    __shared__ uint32_t wo[kSmallWaves][256];    // per-wave digit offsets
    __shared__ int skip;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < n; i += kSmallThreads) {
        sk[0][i] = keys[i];
        sv[0][i] = vals[i];
    }
    for (int i = tid; i < kSmallWaves * 256; i += kSmallThreads) (&wc[0][0])[i] = 0u;
    int cur = 0;
    const u64 lt = (1ull << lane) - 1ull;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        if (tid < 256) hist[tid] = 0u;
        if (tid == 0) skip = 0;
        __syncthreads();
        for (int base = 0; base < n; base += kSmallThreads) {
            const int i = base + tid;
            const bool valid = i < n;
            const uint32_t d = valid ? (uint32_t)(sk[cur][i] >> shift) & 255u : 0u;
            const u64 peers = digit_peers(d, valid);
            if (valid && (peers & lt) == 0ull) atomicAdd(&hist[d], (uint32_t)__popcll(peers));
        }
        __syncthreads();
        // exclusive scan of the 256 counts by waves 0..3
        const uint32_t v = tid < 256 ? hist[tid] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (tid < 256 && lane == 63) wsum[wave] = x;
        if (tid < 256 && (int)v == n) skip = 1;
        __syncthreads();
        if (tid < 256) {
            uint32_t b = 0;
            for (int w = 0; w < wave; ++w) b += wsum[w];
            run[tid] = b + x - v;
        }
        __syncthreads();
        const int skipped = skip;
        __syncthreads();                             // read by all before the next pass clears it
        if (skipped) continue;                       // block-uniform
        for (int base = 0; base < n; base += kSmallThreads) {
            const int i = base + tid;
            const bool valid = i < n;
            const u64 key = valid ? sk[cur][i] : 0ull;
            const uint32_t val = valid ? sv[cur][i] : 0u;
            const uint32_t d = (uint32_t)(key >> shift) & 255u;
            const u64 peers = digit_peers(d, valid);
            const uint32_t rank = __popcll(peers & lt);
            if (valid && rank == 0) wc[wave][d] = __popcll(peers);
            __syncthreads();
            if (tid < 256) {
                // digit tid: offsets of the waves in order, the counts cleared
                uint32_t acc = run[tid];
#pragma unroll
                for (int w = 0; w < kSmallWaves; ++w) {
                    const uint32_t c = wc[w][tid];
                    wo[w][tid] = acc;
                    wc[w][tid] = 0u;
                    acc += c;
                }
                run[tid] = acc;
            }
            __syncthreads();
            if (valid) {
                const uint32_t pos = wo[wave][d] + rank;
                sk[cur ^ 1][pos] = key;
                sv[cur ^ 1][pos] = val;
            }
        }
        cur ^= 1;
        __syncthreads();
    }
    for (int i = tid; i < n; i += kSmallThreads) {
        keys[i] = sk[cur][i];
        vals[i] = sv[cur][i];
        if (fd_out) fd_out[i] = fd_of_bits(sk[cur][i]);
    }
}

__global__ void k_fd_keys(const double *__restrict__ fd, int64_t n, u64 *__restrict__ keys,
                          uint32_t *__restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        keys[i] = fd_bits(fd[i]);
        vals[i] = (uint32_t)i;
    }
}

// Per range: [lo, hi) = positions p with -T <= fd_sorted[p] - fd_r <= T,
// T = tol + 1e-9, both bounds by binary search on the monotone difference.
// A negative tol asks for (max - min)/3 over the domain dimensions: the ends
// of the sorted array.
__global__ void k_bounds(const double *__restrict__ fdr, int32_t nr,
                         const double *__restrict__ fds, int32_t nd, double tol,
                         uint32_t *__restrict__ lo, uint32_t *__restrict__ hi)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const double te = tol >= 0.0 ? tol : (nd > 0 ? (fds[nd - 1] - fds[0]) / 3.0 : 0.0);
    const double T = te + 1e-9;
    const double x = fdr[r];
    int a = 0, b = nd;                       // first p with fds[p] - x >= -T
    while (a < b) {
        int m = (a + b) >> 1;
        if (fds[m] - x >= -T) b = m; else a = m + 1;
    }
    int c = a, e = nd;                       // first p with fds[p] - x > T
    while (c < e) {
        int m = (c + e) >> 1;
        if (fds[m] - x > T) e = m; else c = m + 1;
    }
    lo[r] = (uint32_t)a;
    hi[r] = (uint32_t)c;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t scan_ws_bytes(int64_t m) { return align256((size_t)((m + kScanTile - 1) / kScanTile + 1) * 4); }

size_t sort_ws_bytes(int64_t n)
{
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb < 1) nb = 1;
    const int64_t nbp = padded_tiles(nb);
    return align256((size_t)n * 8) + align256((size_t)n * 4) +
           (size_t)kMaxPasses * (align256((size_t)nbp * 256 * 4) + 1024) + align256(sizeof(SortCtl));
}

hipError_t scan_u32(uint32_t *a, int64_t m, uint32_t *total, void *ws, hipStream_t s)
{
    const int64_t nt = (m + kScanTile - 1) / kScanTile;
    uint32_t *tt = (uint32_t *)ws;
    if (nt == 1) {           // one tile: its scan is the whole scan
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, a, m, tt, total);
        return hipGetLastError();
    }
    if (nt > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanThreads), 0, s, a, m, tt,
                           (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, tt, nt, total);
    if (nt > 1)
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(kScanThreads), 0, s, a, m, tt);
    return hipGetLastError();
}

// Stable sort of n (key, value) pairs by the low key_bits bits of the keys
// (LSD, 8-bit digits). Up to kSmallSort pairs: one launch (k_sort_small).
// Otherwise per digit the tile histograms and the stable scatter, with a
// scan of the tile counts between them above kFusedScanTiles tiles, and a
// last launch that copies the result back when it ended in the alternate
// arrays; passes in which every key has the same digit are skipped on the
// device. No workgroup waits on another: every hand-over is a kernel
// boundary. With fd_out (nullable) the keys are fd_bits images and their
// sorted fp64 values are also written there.
hipError_t radix_sort_pairs(u64 *keys, uint32_t *vals, int64_t n, int key_bits, void *ws,
                            hipStream_t s, double *fd_out)
{
    if (n <= 0 || (n == 1 && !fd_out)) return hipSuccess;
    const int passes = (key_bits + 7) / 8;
    if (passes > kMaxPasses) return hipErrorInvalidValue;
    if (n <= kSmallSort) {
        hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(kSmallThreads), 0, s, keys, vals, (int)n,
                           passes, fd_out);
        return hipGetLastError();
    }
    const int nb = (int)((n + kSortTile - 1) / kSortTile);
    char *p = (char *)ws;
    u64 *kalt = (u64 *)p;                 p += align256((size_t)n * 8);
    uint32_t *valt = (uint32_t *)p;       p += align256((size_t)n * 4);
    const size_t nbp = (size_t)padded_tiles(nb);
    const size_t cstride = (align256(nbp * 256 * 4) + 1024) / 4;   // counts, then 256 totals
    uint32_t *cnt = (uint32_t *)p;        p += (size_t)kMaxPasses * cstride * 4;
    SortCtl *ctl = (SortCtl *)p;
    const int fused = nb <= kFusedScanTiles ? 1 : 0;
    for (int pass = 0; pass < passes; ++pass) {
        uint32_t *c = cnt + (size_t)pass * cstride;
        uint32_t *tot = c + align256(nbp * 256 * 4) / 4;
        hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(kSortThreads), 0, s, (const u64 *)keys,
                           (const u64 *)kalt, n, pass * 8, pass, c, nb, (const SortCtl *)ctl);
        if (!fused) hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, c, nb, tot);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(kSortThreads), 0, s, keys, vals, kalt,
                           valt, n, pass * 8, pass, (const uint32_t *)c, (const uint32_t *)tot, nb,
                           fused, ctl);
    }
    hipLaunchKernelGGL(k_sort_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, vals,
                       (const u64 *)kalt, (const uint32_t *)valt, n, passes, (const SortCtl *)ctl,
                       fd_out);
    return hipGetLastError();
}

// Pool workspace: sort keys (n_domain u64), sorted fd (n_domain f64), sort
// scratch.
size_t pool_ws_bytes(int64_t nr, int64_t nd)
{
    (void)nr;
    return align256((size_t)nd * 8) * 2 + sort_ws_bytes(nd);
}

hipError_t launch_pool(const double *fd_range, int32_t nr, const double *fd_dom, int32_t nd,
                       double tol, uint32_t *perm, uint32_t *lo, uint32_t *hi, void *ws,
                       hipStream_t s, const Tracer *tr)
{
    trace(tr, FIC_STAGE_POOL, 1, s);
    char *p = (char *)ws;
    u64 *keys = (u64 *)p;          p += align256((size_t)nd * 8);
    double *fds = (double *)p;     p += align256((size_t)nd * 8);
    void *sortws = p;
    const int th = 256;
    hipLaunchKernelGGL(k_fd_keys, dim3((nd + th - 1) / th), dim3(th), 0, s, fd_dom, (int64_t)nd,
                       keys, perm);
    // the sort also writes the sorted fd values (decoded from its keys)
    hipError_t e = radix_sort_pairs(keys, perm, nd, 64, sortws, s, fds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bounds, dim3((nr + th - 1) / th), dim3(th), 0, s, fd_range, nr, fds, nd,
                       tol, lo, hi);
    trace(tr, FIC_STAGE_POOL, 0, s);
    return hipGetLastError();
}

}  // namespace fic

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
// exclusive scan over (digit, block), and a scatter that ranks equal digits
// by position with wave ballots, so every pass is stable.
#include "fic_internal.h"

namespace fic {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortPerThread = 16;
constexpr int kSortTile = kSortThreads * kSortPerThread;   // keys per block

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const u64 *__restrict__ keys,
                                                              int64_t n, int shift,
                                                              uint32_t *__restrict__ hist,
                                                              int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortPerThread; ++r) {
        int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

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

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t *__restrict__ a, int64_t m,
                                                             uint32_t *__restrict__ tile_tot)
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
    if (threadIdx.x == 0) tile_tot[blockIdx.x] = total;
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

__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(
    const u64 *__restrict__ kin, const uint32_t *__restrict__ vin, u64 *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offs,
    int nblocks)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[kSortThreads / kWave][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kSortThreads / kWave; ++w) wc[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const u64 lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortPerThread; ++r) {
        const int64_t i = base + r * kSortThreads + tid;
        const bool valid = i < n;
        u64 key = valid ? kin[i] : 0ull;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            u64 bb = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wc[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / kWave; ++w) {
            add += wc[w][tid];
            wc[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

// Order-preserving integer image of an fp64 value.
__device__ inline u64 fd_bits(double x)
{
    u64 b = (u64)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
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

// Window half-width: tol, or (max - min)/3 over the domain dimensions.
__global__ __launch_bounds__(1024) void k_resolve_tol(const double *__restrict__ fd, int64_t n,
                                                       double tol, double *__restrict__ out)
{
    __shared__ double smax[1024], smin[1024];
    double mx = -INFINITY, mn = INFINITY;
    if (tol < 0.0)
        for (int64_t i = threadIdx.x; i < n; i += 1024) {
            mx = fmax(mx, fd[i]);
            mn = fmin(mn, fd[i]);
        }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = tol < 0.0 ? (smax[0] - smin[0]) / 3.0 : tol;
}

__global__ void k_sorted_fd(const double *__restrict__ fd, const uint32_t *__restrict__ perm,
                            int64_t n, double *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fd[perm[i]];
}

// Per range: [lo, hi) = positions p with -T <= fd_sorted[p] - fd_r <= T,
// T = tol + 1e-9, both bounds by binary search on the monotone difference.
__global__ void k_bounds(const double *__restrict__ fdr, int32_t nr,
                         const double *__restrict__ fds, int32_t nd,
                         const double *__restrict__ tol_eff, uint32_t *__restrict__ lo,
                         uint32_t *__restrict__ hi)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const double T = tol_eff[0] + 1e-9;
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

__global__ void k_copy_pairs(const u64 *__restrict__ ks, const uint32_t *__restrict__ vs,
                             u64 *__restrict__ kd, uint32_t *__restrict__ vd, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    kd[i] = ks[i];
    vd[i] = vs[i];
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t scan_ws_bytes(int64_t m) { return align256((size_t)((m + kScanTile - 1) / kScanTile + 1) * 4); }

size_t sort_ws_bytes(int64_t n)
{
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb < 1) nb = 1;
    return align256((size_t)n * 8) + align256((size_t)n * 4) + align256((size_t)nb * 256 * 4) +
           scan_ws_bytes(nb * 256) + 256;
}

hipError_t scan_u32(uint32_t *a, int64_t m, uint32_t *total, void *ws, hipStream_t s)
{
    const int64_t nt = (m + kScanTile - 1) / kScanTile;
    uint32_t *tt = (uint32_t *)ws;
    if (nt > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanThreads), 0, s, a, m, tt);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, tt, nt, total);
    if (nt > 1)
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(kScanThreads), 0, s, a, m, tt);
    return hipGetLastError();
}

hipError_t radix_sort_pairs(u64 *keys, uint32_t *vals, int64_t n, int key_bits, void *ws,
                            hipStream_t s)
{
    if (n <= 1) return hipSuccess;
    const int nb = (int)((n + kSortTile - 1) / kSortTile);
    char *p = (char *)ws;
    u64 *kalt = (u64 *)p;                 p += align256((size_t)n * 8);
    uint32_t *valt = (uint32_t *)p;       p += align256((size_t)n * 4);
    uint32_t *hist = (uint32_t *)p;       p += align256((size_t)nb * 256 * 4);
    void *scanws = p;
    const int passes = (key_bits + 7) / 8;
    u64 *ka = keys, *kb = kalt;
    uint32_t *va = vals, *vb = valt;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * 8;
        hipLaunchKernelGGL(k_digit_hist, dim3(nb), dim3(kSortThreads), 0, s, ka, n, shift, hist, nb);
        const hipError_t se = scan_u32(hist, (int64_t)nb * 256, nullptr, scanws, s);
        if (se != hipSuccess) return se;
        hipLaunchKernelGGL(k_digit_scatter, dim3(nb), dim3(kSortThreads), 0, s, ka, va, kb, vb, n,
                           shift, hist, nb);
        u64 *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys)     // odd pass count: copy back (a kernel, so graphs hold no copy nodes)
        hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ka, va,
                           keys, vals, n);
    return hipGetLastError();
}

// Pool workspace: sort keys (n_domain u64), sorted fd (n_domain f64),
// tol (f64), sort scratch.
size_t pool_ws_bytes(int64_t nr, int64_t nd)
{
    (void)nr;
    return align256((size_t)nd * 8) * 2 + 256 + sort_ws_bytes(nd);
}

hipError_t launch_pool(const double *fd_range, int32_t nr, const double *fd_dom, int32_t nd,
                       double tol, uint32_t *perm, uint32_t *lo, uint32_t *hi, void *ws,
                       hipStream_t s, const Tracer *tr)
{
    trace(tr, FIC_STAGE_POOL, 1, s);
    char *p = (char *)ws;
    u64 *keys = (u64 *)p;          p += align256((size_t)nd * 8);
    double *fds = (double *)p;     p += align256((size_t)nd * 8);
    double *tol_eff = (double *)p; p += 256;
    void *sortws = p;
    const int th = 256;
    hipLaunchKernelGGL(k_fd_keys, dim3((nd + th - 1) / th), dim3(th), 0, s, fd_dom, (int64_t)nd,
                       keys, perm);
    hipError_t e = radix_sort_pairs(keys, perm, nd, 64, sortws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resolve_tol, dim3(1), dim3(1024), 0, s, fd_dom, (int64_t)nd, tol, tol_eff);
    hipLaunchKernelGGL(k_sorted_fd, dim3((nd + th - 1) / th), dim3(th), 0, s, fd_dom, perm,
                       (int64_t)nd, fds);
    hipLaunchKernelGGL(k_bounds, dim3((nr + th - 1) / th), dim3(th), 0, s, fd_range, nr, fds, nd,
                       tol_eff, lo, hi);
    trace(tr, FIC_STAGE_POOL, 0, s);
    return hipGetLastError();
}

}  // namespace fic

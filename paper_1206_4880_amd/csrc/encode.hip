// encode.hip -- the range-domain matching search of the PIFS encoder
// (Sec. 1 and Sec. 2: every non-overlapping range against the overlapping
// domains of twice its size, shrunk by 2x2 sums, under the 8 isometries and a
// quantized contrast / brightness; exhaustive, or restricted to the per-range
// pool of Sec. 3.1).
//
// Matrix-core path (FIC_KERNEL_MFMA):
//   range prep   A rows: for each range and isometry q, the range pixels under
//                T_q^-1, centred by an integer level rhat (|.| <= 255), FP16
//                (exact), pre-swizzled into MFMA lane order.
//   domain prep  B columns: the 2x2 sums of each domain (in pool order),
//                centred by an integer level dhat (|.| <= 1020), FP16 (exact);
//                per column Sdd', eps = sum D - n*dhat and u = sqrt(Sdd')/n.
//   search       a persistent work queue of (range group, column chunk)
//                items, of one image or of all images of a batch. The
//                group's A rows stay in VGPRs; each MR-column block costs
//                MB*KS MFMAs, giving C''' = sum (r-rhat)(D-dhat) exactly in
//                FP32 (64-term chunks), and Srd' = n*C''' - delta*eps
//                exactly. A few FP32 instructions per output tile screen out
//                pairs whose continuous optimum cannot reach the range's best
//                F (16x16 ranges screen one FP32 sum against a threshold
//                lowered by its rounding bound and recompute the exact chunks
//                only for blocks that pass); passing cells queue in LDS and
//                get the exact fit a wave's worth at a time (4x4 ranges queue
//                the passing columns and replay them, cells screened one by
//                one, before their cells are queued); packed
//                (F, domain, isometry) keys meet in LDS, and each flush
//                exchanges them with the global keys, so waves on other
//                column chunks of the same ranges tighten each other's
//                thresholds.
// VALU and MFMA instruction time add up on a SIMD, so the hot loops are
// written for few VALU instructions per MFMA (scalar addressing, one compare
// per block), not to hide them.
//   finalize     recompute the winner exactly from the image, write fic_code.
// Plain path (FIC_KERNEL_PLAIN): one thread per (range, domain, isometry),
// integer cross term from the 2x2-sum image, exact fit, the same keys.
// The work split (columns per item, early flush trigger, per-XCD queues)
// comes from a tuning row per (range size, log2 D) and pool-fraction bucket,
// read on the device. On top of these: batches (persistent searches over the
// items of many images, one per range size or 4x4 and 8x8 in one launch,
// recorded as a HIP graph), the two-level partition (level-2 search of the
// quadrants of split ranges) and colour (three channel searches over the
// pools of one gray image).
#include "fic_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace fic {

namespace {

constexpr int kBminBlock = 1024; // perm entries per block-minimum

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Allowance of the screen in C''' units: n/4 covers |n*C''' - Srd'| <= n^2/4;
// 16x16 ranges add 64 for the FP32 sum of their 4 exact partial sums.
template <int B> constexpr float screen_slack()
{
    return Cfg<B>::n / 4.0f + (Cfg<B>::NCH > 1 ? 64.0f : 0.0f);
}

// The contrast is clamped: s = k/16 with k in [-16, 15]. Relaxing k to the
// real interval [-16, 16], F(k) = 4096 Srr' - 128 k Srd' + k^2 Sdd' reaches
// F_best (T^2 = Srr' - F_best/4096) only if |Srd'| >= T sqrt(Sdd') when the
// vertex |64 Srd'/Sdd'| <= 16, and only if |Srd'| >= 2 T^2 + Sdd'/8 at the
// end points otherwise; when T > sqrt(Sdd')/4 the first case is empty, so a
// pair passes only by the second. In C''' units (sqrt(Sdd') = n u): for
// T > n u / 4 a cell needs max |C'''| >= 2 T^2/n + n u^2/8 (minus the same
// slack), a stricter test than T u. Returns that threshold, lowered by 2^-20
// for the FP32 rounding (T and u are rounded down already, and the bound
// grows with both), or 0 when the plain test T u is the exact one.
template <int B> __device__ __forceinline__ float clamp_threshold(float t, float u)
{
    constexpr float n = (float)Cfg<B>::n;
    if (!(t > (n * 0.25f) * u)) return 0.0f;
    return fmaf(2.0f * t, t * (1.0f / n), (n * 0.125f) * u * u) * (1.0f - 0x1p-20f);
}

// The contrast is quantised: every range's key starts at most at its DC
// code (k = 0, F = 4096 Srr', the lowest pool domain under isometry 0, the
// smallest (domain, isometry) there is), so a pair can only replace the key
// with some k != 0 and F(k) < 4096 Srr', i.e. k (k Sdd' - 128 Srd') < 0,
// which needs 128 |Srd'| > Sdd'. In C''' units (|Srd'| <= n |C'''| + n^2/4,
// Sdd' = n^2 u^2): max |C'''| > n u^2 / 128 - n/4. This holds whatever T is,
// and decides the ranges whose best is still the DC code (T = 0, where the
// test T u passes every pair). Returns n u^2/128 lowered by 2^-20 (u is
// rounded down already); flat and padding columns (u = 1e30) never pass.
template <int B> __device__ __forceinline__ float quant_threshold(float u)
{
    constexpr float n = (float)Cfg<B>::n;
    return (n * (1.0f / 128.0f)) * u * u * (1.0f - 0x1p-20f);
}

// Threshold of the 16x16 search, whose hot screen sums all n products in one
// FP32 accumulator. The products are exact; every partial sum is at most
// ||A|| ||B|| (Cauchy-Schwarz), so each of the at most n + KS roundings is off
// by at most ||A|| ||B|| 2^-23. With ||B|| <= sqrt(n) (u + 1/2) and
// ||A||^2 <= Srr'/n + n/4 (centring by an integer level), lowering T by
// e = (n + KS) 2^-23 sqrt(n) ||A|| covers the u-proportional part of the
// error; the rest, e/2 <= 1.1, is inside screen_slack. Other range sizes
// accumulate exactly and keep T.
template <int B> __device__ inline float screen_t_b(int64_t srr, int64_t f)
{
    using C = Cfg<B>;
    const float t = screen_t(srr, f);
    if (C::NCH == 1 || t == 0.0f) return t;
    const double na = sqrt((double)srr / C::n + C::n / 4.0);
    const double e = (double)(C::n + C::KS) * 0x1p-23 * sqrt((double)C::n) * na;
    const double tf = ((double)t - e) * (1.0 - 0x1p-20);
    return tf > 0.0 ? (float)tf : 0.0f;
}

template <int EPL> struct Frag;
template <> struct Frag<8> { typedef half8_t type; };

__device__ __forceinline__ float4_t mma(half8_t a, half8_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float16_t mma32(half8_t a, half8_t b, float16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(u64 *p, int64_t n, u64 v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- prep
// Search order of the ranges: by (lo, hi) of the pool interval, ranges that
// need no search (flat, empty pool) last, ties by raster index. lo and hi
// both grow with the range's dimension, so along this order the first and
// last column of every group never decrease, and the groups that touch a
// column chunk form one contiguous run (the work list needs no atomics).
// Exhaustive search only moves the flat (and unselected) ranges to the end.
template <int B>
__global__ void k_range_keys(const uint8_t *__restrict__ img, int32_t pitch, int32_t rcols, int64_t R,
                             const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                             const uint8_t *__restrict__ sel, uint32_t D, int dbits,
                             u64 *__restrict__ keys, uint32_t *__restrict__ vals)
{
    constexpr int n = B * B;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint8_t *rp = img + (int64_t)(r / rcols) * B * pitch + (r % rcols) * B;
    int32_t sr = 0;
    int64_t sq = 0;
    for (int i = 0; i < B; ++i)
        for (int j = 0; j < B; ++j) {
            const int v = rp[i * pitch + j];
            sr += v;
            sq += v * v;
        }
    const bool flat = (int64_t)n * sq - (int64_t)sr * sr == 0;
    const uint32_t l = lo ? lo[r] : 0u, h = hi ? hi[r] : D;
    const bool idle = flat || l >= h || (sel && !sel[r]);
    u64 key;
    if (!lo) key = idle ? 1ull : 0ull;
    else key = idle ? (1ull << (2 * dbits)) - 1ull : (((u64)l << dbits) | (u64)h);
    keys[r] = key;
    vals[r] = (uint32_t)r;
}

template <int B>
__global__ __launch_bounds__(256) void k_range_prep(
    const uint8_t *__restrict__ img, int32_t pitch, int32_t rcols, int64_t R, int64_t Rp,
    const uint32_t *__restrict__ order, const uint32_t *__restrict__ lo,
    const uint32_t *__restrict__ hi, const uint8_t *__restrict__ sel, uint32_t D,
    _Float16 *__restrict__ A, RangeStat *__restrict__ rs)
{
    using C = Cfg<B>;
    constexpr int n = C::n, MR = C::MR, KPI = C::KPI, EPL = C::EPL, KS = C::KS, MB = C::MB,
                  GR = C::GR;
    typedef typename Frag<EPL>::type frag_t;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = gt >> 3;
    const int q = (int)(gt & 7);
    if (s >= Rp) return;
    const bool valid = s < R;
    const uint32_t ridx = valid ? (order ? order[s] : (uint32_t)s) : 0u;
    const int ry = (int)(ridx / rcols) * B, rx = (int)(ridx % rcols) * B;
    const uint8_t *rp = img + (int64_t)ry * pitch + rx;
    int32_t sr = 0;
    int64_t sq = 0;
    if (valid)
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) {
                int v = rp[i * pitch + j];
                sr += v;
                sq += v * v;
            }
    const int32_t rhat = (sr + n / 2) / n;
    const int64_t grp = s / GR;
    int blk, row;
    a_place<B>((int)(s % GR), q, blk, row);
    const int iq = iso_inverse(q);
    // A_q[u][v] = r[T_q^-1 (u, v)] - rhat, so that sum A_q * D = sum r * T_q(D)
    for (int ks = 0; ks < KS; ++ks)
        for (int g = 0; g < KPI / EPL; ++g) {
            frag_t f;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int K = ks * KPI + g * EPL + e;
                int si, sj;
                iso_src(iq, B, K / B, K % B, si, sj);
                f[e] = valid ? (_Float16)(int)(rp[si * pitch + sj] - rhat) : (_Float16)0;
            }
            ((frag_t *)A)[((grp * MB + blk) * KS + ks) * 64 + g * MR + row] = f;
        }
    if (q == 0) {
        RangeStat st;
        st.srr = (int64_t)n * sq - (int64_t)sr * sr;
        st.sr = sr;
        st.delta = sr - n * rhat;
        st.ridx = ridx;
        st.lo = valid ? (lo ? lo[ridx] : 0u) : 0u;
        st.hi = valid ? (hi ? hi[ridx] : D) : 0u;
        st.flags = !valid ? kPad
                          : ((st.srr == 0 ? kFlat : 0u) | (st.lo >= st.hi ? kEmpty : 0u) |
                             (sel && !sel[ridx] ? kSkip : 0u));
        rs[s] = st;
    }
}

// Pair sums of the 2B bytes at p: pk[j] holds p[4j] + p[4j+1] in its low
// and p[4j+2] + p[4j+3] in its high 16 bits. Aligned dword loads (one more
// than the span) and byte funnel shifts replace 2B byte loads; where those
// words would reach outside the image [begin, end) the bytes are read one by
// one.
template <int B>
__device__ __forceinline__ void pair_sums(const uint8_t *p, const uint8_t *begin,
                                          const uint8_t *end, uint32_t (&pk)[B / 2])
{
    constexpr int NW = B / 2;                        // 4-byte words in 2B bytes
    const uintptr_t a = (uintptr_t)p & ~(uintptr_t)3;
    const int sh = (int)((uintptr_t)p & 3);
    if (a >= (uintptr_t)begin && a + 4 * (NW + 1) <= (uintptr_t)end) {
        const uint32_t *w = (const uint32_t *)a;
        uint32_t r[NW + 1];
#pragma unroll
        for (int j = 0; j <= NW; ++j) r[j] = w[j];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const uint32_t x = __builtin_amdgcn_alignbyte(r[j + 1], r[j], (uint32_t)sh);
            pk[j] = (x & 0x00ff00ffu) + ((x >> 8) & 0x00ff00ffu);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NW; ++j)
            pk[j] = (uint32_t)(p[4 * j] + p[4 * j + 1]) |
                    ((uint32_t)(p[4 * j + 2] + p[4 * j + 3]) << 16);
    }
}

template <int B>
__global__ __launch_bounds__(256) void k_domain_prep(
    const uint8_t *__restrict__ img, int64_t img_bytes, int32_t pitch, int32_t dcols, int32_t t,
    const uint32_t *__restrict__ perm, int64_t D, int64_t Dp, _Float16 *__restrict__ Bm,
    float *__restrict__ u, int32_t *__restrict__ eps, int64_t *__restrict__ sdd,
    uint32_t *__restrict__ dom)
{
    using C = Cfg<B>;
    constexpr int n = C::n, MR = C::MR, KPI = C::KPI, EPL = C::EPL, KS = C::KS;
    typedef typename Frag<EPL>::type frag_t;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gt / B;
    const int i = (int)(gt % B);
    if (p >= Dp) return;                 // whole B-lane groups leave together
    const bool valid = p < D;
    const uint32_t d = valid ? (perm ? perm[p] : (uint32_t)p) : 0u;
    const int y = (int)(d / dcols) * t, x = (int)(d % dcols) * t;
    int v[B];
    int64_t rs1 = 0, rs2 = 0;
    const uint8_t *q = img + (int64_t)(y + 2 * i) * pitch + x;
    uint32_t p0[B / 2], p1[B / 2];
    pair_sums<B>(q, img, img + img_bytes, p0);
    pair_sums<B>(q + pitch, img, img + img_bytes, p1);
#pragma unroll
    for (int j = 0; j < B / 2; ++j) {
        const uint32_t s2 = p0[j] + p1[j];           // two 2x2 sums, <= 1020 each
        v[2 * j] = valid ? (int)(s2 & 0xffffu) : 0;
        v[2 * j + 1] = valid ? (int)(s2 >> 16) : 0;
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
        rs1 += v[e];
        rs2 += v[e] * v[e];
    }
#pragma unroll
    for (int off = 1; off < B; off <<= 1) {
        rs1 += __shfl_xor(rs1, off);
        rs2 += __shfl_xor(rs2, off);
    }
    const int64_t sdd_ = (int64_t)n * rs2 - rs1 * rs1;
    const int32_t dhat = (int32_t)((rs1 + n / 2) / n);
    const int64_t cb = p / MR;
    const int c = (int)(p % MR);
    // pixel row i holds K = i*B .. i*B + B-1: whole fragments when B >= EPL,
    // else part of one fragment
    if constexpr (B >= EPL) {
#pragma unroll
        for (int f0 = 0; f0 < B; f0 += EPL) {
            const int K0 = i * B + f0;
            const int ks = K0 / KPI, g = (K0 % KPI) / EPL;
            frag_t f;
#pragma unroll
            for (int e = 0; e < EPL; ++e) f[e] = (_Float16)(valid ? v[f0 + e] - dhat : 0);
            ((frag_t *)Bm)[(cb * KS + ks) * 64 + g * MR + c] = f;
        }
    } else {
        const int K0 = i * B;
        const int ks = K0 / KPI, g = (K0 % KPI) / EPL;
        _Float16 *dst = Bm + ((cb * KS + ks) * 64 + g * MR + c) * EPL + K0 % EPL;
#pragma unroll
        for (int e = 0; e < B; ++e) dst[e] = (_Float16)(valid ? v[e] - dhat : 0);
    }
    if (i == 0) {
        u[p] = valid ? screen_u(sdd_, n) : 1e30f;   // padding: always masked (p >= hi)
        eps[p] = valid ? (int32_t)(rs1 - (int64_t)n * dhat) : 0;
        sdd[p] = valid ? sdd_ : 0;
        dom[p] = d;
    }
}

// Minimum domain index over blocks of the pool order (for flat ranges, whose
// every pair ties at F = 0 and which therefore take the lowest pool index).
__global__ void k_blockmin(const uint32_t *__restrict__ perm, int64_t D, uint32_t *bmin)
{
    const int64_t blk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t nb = (D + kBminBlock - 1) / kBminBlock;
    if (blk >= nb) return;
    uint32_t m = 0xffffffffu;
    for (int64_t i = blk * kBminBlock + lane; i < min(D, (blk + 1) * kBminBlock); i += 64)
        m = min(m, perm[i]);
    for (int off = 32; off > 0; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off));
    if (lane == 0) bmin[blk] = m;
}

// Lowest domain index in pool positions [lo, hi), by the whole wave: the
// partial blocks at both ends from perm, the whole blocks from their minima.
// Every lane returns the result.
__device__ uint32_t pool_min_wave(const uint32_t *perm, const uint32_t *bmin, uint32_t lo,
                                  uint32_t hi, int lane)
{
    if (!perm) return lo;
    uint32_t m = 0xffffffffu;
    const uint32_t kb = (uint32_t)kBminBlock;
    uint32_t head = (lo + kb - 1) / kb * kb;
    if (head > hi) head = hi;
    const uint32_t mid = head + (hi - head) / kb * kb;
    for (uint32_t i = lo + lane; i < head; i += 64) m = min(m, perm[i]);
    for (uint32_t b = head / kb + lane; b < mid / kb; b += 64) m = min(m, bmin[b]);
    for (uint32_t i = mid + lane; i < hi; i += 64) m = min(m, perm[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off));
    return m;
}

// Row i's part of the exact cross sums of (range at (ry, rx), domain at
// (dy, dx), isometry q), from pixels: cx = sum_j r[i][j] * D[src(i, j)],
// sd and sdd the sums of the domain values those cells take (over all rows
// they are the domain's sums, whatever q).
template <int B>
__device__ void pair_row_sums(const uint8_t *img, int32_t pitch, int ry, int rx, int dy, int dx,
                              int q, int i, int64_t &cx, int64_t &sd, int64_t &sdd)
{
    cx = sd = sdd = 0;
    for (int j = 0; j < B; ++j) {
        int si, sj;
        iso_src(q, B, i, j, si, sj);
        const uint8_t *pp = img + (int64_t)(dy + 2 * si) * pitch + dx + 2 * sj;
        const int dv = pp[0] + pp[1] + pp[pitch] + pp[pitch + 1];
        cx += (int64_t)img[(int64_t)(ry + i) * pitch + rx + j] * dv;
        sd += dv;
        sdd += dv * dv;
    }
}

// Sum over the B lanes of an aligned segment of a wave (B a power of two).
template <int B, class T> __device__ __forceinline__ T segment_sum(T v)
{
#pragma unroll
    for (int off = 1; off < B; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

// Initial best key per range, so the screen starts from a real threshold:
// one wave per range evaluates 8 candidate columns spread over its pool under
// the 8 isometries (lane = candidate * 8 + isometry), exactly, from the
// prepared operands (the FP16 values are integers). Flat ranges get their
// final key directly (every pair ties at F = 0: the lowest pool index wins).
template <int B>
__global__ __launch_bounds__(256) void k_seed(const _Float16 *__restrict__ A,
                                              const _Float16 *__restrict__ Bm,
                                              const RangeStat *__restrict__ rs,
                                              const int32_t *__restrict__ eps,
                                              const int64_t *__restrict__ sdd,
                                              const uint32_t *__restrict__ dom, int64_t Rp,
                                              const uint32_t *__restrict__ perm,
                                              const uint32_t *__restrict__ bmin, int shift,
                                              u64 *__restrict__ keys, u64 *counters)
{
    using C = Cfg<B>;
    constexpr int n = C::n, MR = C::MR, KPI = C::KPI, EPL = C::EPL, KS = C::KS, MB = C::MB,
                  GR = C::GR;
    typedef typename Frag<EPL>::type frag_t;
    const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (s >= Rp) return;
    const RangeStat st = rs[s];
    if (st.flags & (kPad | kEmpty | kSkip)) {
        if (lane == 0) keys[s] = kNoKey;
        return;
    }
    const uint32_t dmin = pool_min_wave(perm, bmin, st.lo, st.hi, lane);
    if (st.flags & kFlat) {
        if (lane == 0) keys[s] = pack_key(0, dmin, 0, shift);
        return;
    }
    const int q = lane & 7, cand = lane >> 3;
    const uint32_t p = st.lo + (uint32_t)(((uint64_t)(st.hi - st.lo) * (2 * cand + 1)) / 16);
    const int64_t grp = s / GR;
    int blk, row;
    a_place<B>((int)(s % GR), q, blk, row);
    const frag_t *ap = (const frag_t *)A + ((grp * MB + blk) * KS) * 64 + row;
    const frag_t *bp = (const frag_t *)Bm + ((int64_t)(p / MR) * KS) * 64 + (p % MR);
    int32_t cx = 0;
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int g = 0; g < KPI / EPL; ++g) {
            const frag_t fa = ap[ks * 64 + g * MR], fb = bp[ks * 64 + g * MR];
#pragma unroll
            for (int e = 0; e < EPL; ++e) cx += (int32_t)(float)fa[e] * (int32_t)(float)fb[e];
        }
    const int64_t srd = (int64_t)n * cx - (int64_t)st.delta * eps[p];
    int k;
    const int64_t f = fit_f(st.srr, srd, sdd[p], k);
    u64 key = pack_key(f, dom[p], q, shift);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const u64 o = __shfl_xor(key, off);
        key = o < key ? o : key;
    }
    if (lane == 0) {
        // every pair reaches F = 4096*Srr' at k = 0, so the lowest pool
        // domain under isometry 0 is a real candidate with that F
        const u64 dc = pack_key(4096 * st.srr, dmin, 0, shift);
        keys[s] = key < dc ? key : dc;
        if (counters) atomicAdd(&counters[3], 64ull);
    }
}

// ------------------------------------------------------------ work list
// One image's search operands: an entry of the device table the persistent
// search reads per work item, so one launch serves many images.
struct SearchArgs {
    const _Float16 *A;
    const _Float16 *Bm;
    const float *u;
    const int32_t *eps;
    const int64_t *sdd;
    const uint32_t *dom;
    const RangeStat *rs;
    const uint4 *grp;
    const WorkItem *items;
    const uint32_t *n_items;
    u64 *keys;
    int shift;
    int flush_at;                // early flush trigger (0: only when the queue is full)
    int xcd;                     // items in XCD order: one queue per XCD
    int ncx;                     // chunk slots per XCD
    const uint32_t *xq;          // exclusive item offsets per chunk slot (XCD x: slots x*ncx..)
};

// Per group: the union [L, H) of its active ranges' intervals (rounded to
// column blocks of width bw, a power of two) and their intersection
// [ilo, ihi) (blocks inside it need no per-range mask). Groups without an
// active range get L = H = Dp.
// Also adds the group's pool sizes to *pool_sum (zeroed before), from which
// the work list picks its parameters.
// One wave per group, a lane per range, wave reductions: the range records
// are loaded side by side, not one after another; one atomic per workgroup
// (of 4 groups) for the pool sizes, not one per group on the same word.
__global__ __launch_bounds__(256) void k_group_bounds(const RangeStat *__restrict__ rs, int64_t G,
                                                      int GR, uint32_t Dp, uint32_t bw,
                                                      uint4 *__restrict__ grp, u64 *pool_sum)
{
    __shared__ u64 part[4];
    const int64_t gi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t L = 0xffffffffu, H = 0, ilo = 0, ihi = 0xffffffffu;
    u64 psum = 0;
    bool act = false;
    for (int r = lane; gi < G && r < GR; r += 64) {
        const RangeStat st = rs[gi * GR + r];
        if (st.flags & kIdle) continue;
        act = true;
        L = min(L, st.lo);
        H = max(H, st.hi);
        ilo = max(ilo, st.lo);
        ihi = min(ihi, st.hi);
        psum += st.hi - st.lo;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        L = min(L, (uint32_t)__shfl_xor((int)L, off));
        H = max(H, (uint32_t)__shfl_xor((int)H, off));
        ilo = max(ilo, (uint32_t)__shfl_xor((int)ilo, off));
        ihi = min(ihi, (uint32_t)__shfl_xor((int)ihi, off));
        psum += (u64)__shfl_xor((unsigned long long)psum, off);
    }
    const bool any = __ballot(act) != 0ull;
    if (lane == 0) {
        if (gi < G)
            grp[gi] = any ? make_uint4(L & ~(bw - 1u), (H + bw - 1u) & ~(bw - 1u), ilo, ihi)
                          : make_uint4(Dp, Dp, 0, 0);
        part[w] = psum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const u64 tot = part[0] + part[1] + part[2] + part[3];
        if (tot) atomicAdd(pool_sum, tot);
    }
}

// Columns per work item and flush trigger of an image, from its tuning row
// and the pool-fraction bucket of its pool sizes (exact integer sum).
struct ItemParams { uint32_t chunk; int flush_at; int xcd; };
__device__ inline ItemParams item_params(const TuneRow &t, int pooled, const u64 *pool_sum,
                                         int64_t R, int64_t D, int allow_xcd, int chunk_min)
{
    const int b = tune_bucket(pooled, pooled ? *pool_sum : 0ull, R, D);
    ItemParams ip;
    ip.chunk = 1u << max((int)t.chunk_log2[b], chunk_min);
    ip.flush_at = t.flush_at[b];
    ip.xcd = allow_xcd && t.xcd[b];
    return ip;
}

// Slot of column chunk c in the work list: chunk-major, or XCD-major (the
// chunks c = x (mod 8) of XCD x together, ncx slots per XCD).
__device__ inline int64_t chunk_slot(int64_t c, int xcd, int64_t ncx)
{
    return xcd ? (c % kXcds) * ncx + c / kXcds : c;
}
__device__ inline int64_t slot_chunk(int64_t p, int xcd, int64_t ncx)
{
    return xcd ? (p % ncx) * kXcds + p / ncx : p;
}

// Per column chunk c: the run of groups [gf, gl] that touch it (both ends
// of the group intervals are monotone in the group index), and its length,
// at the chunk's slot. NC counts chunk slots of the narrowest item width (a
// multiple of 8); with wider items the chunks past the lattice get no groups.
__global__ void k_chunk_span(const uint4 *__restrict__ grp, int64_t G, int64_t NC, TuneRow tune,
                             int chunk_min, int pooled, const u64 *__restrict__ pool_sum,
                             int64_t R, int64_t D, int allow_xcd, uint32_t *__restrict__ cnt,
                             uint32_t *__restrict__ gfirst)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NC) return;
    const ItemParams ip = item_params(tune, pooled, pool_sum, R, D, allow_xcd, chunk_min);
    const uint32_t chunk = ip.chunk;
    const int64_t pc = chunk_slot(c, ip.xcd, NC / kXcds);
    if ((uint64_t)c * chunk >= (uint64_t)D) {   // past the lattice (also past its padding)
        cnt[pc] = 0;
        gfirst[c] = 0;
        return;
    }
    const uint32_t c0 = (uint32_t)c * chunk, c1 = c0 + chunk;
    int64_t a = 0, b = G;                    // active groups: a prefix [0, G_act)
    while (a < b) { const int64_t m = (a + b) >> 1; if (grp[m].x < grp[m].y) a = m + 1; else b = m; }
    const int64_t gact = a;
    a = 0; b = gact;                         // first group with H > c0
    while (a < b) { const int64_t m = (a + b) >> 1; if (grp[m].y > c0) b = m; else a = m + 1; }
    const int64_t gf = a;
    a = 0; b = gact;                         // first group with L >= c1
    while (a < b) { const int64_t m = (a + b) >> 1; if (grp[m].x >= c1) b = m; else a = m + 1; }
    const int64_t gend = a;
    cnt[pc] = gend > gf ? (uint32_t)(gend - gf) : 0u;
    gfirst[c] = (uint32_t)gf;
}

// Item i: its chunk slot by binary search over the scanned counts, its group
// by offset inside the chunk's run. Chunk-major order: the items in flight at
// any moment share a few column chunks, which then stay resident in each
// XCD's L2; in XCD order, the chunks of each XCD's queue together.
// Thread 0 also publishes the image's table entry.
__global__ void k_emit_items(const uint4 *__restrict__ grp, const uint32_t *__restrict__ chunkoff,
                             const uint32_t *__restrict__ gfirst, int64_t NC, TuneRow tune,
                             int chunk_min, int pooled, const u64 *__restrict__ pool_sum,
                             int64_t R, int64_t D, int allow_xcd,
                             const uint32_t *__restrict__ total, int64_t max_items,
                             WorkItem *__restrict__ items, SearchArgs args,
                             SearchArgs *__restrict__ slot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const ItemParams ip = item_params(tune, pooled, pool_sum, R, D, allow_xcd, chunk_min);
    const uint32_t chunk = ip.chunk;
    const int64_t ncx = NC / kXcds;
    if (i == 0) {
        args.flush_at = ip.flush_at;
        args.xcd = ip.xcd;
        args.ncx = (int)ncx;
        args.xq = chunkoff;
        *slot = args;
    }
    if (i >= max_items || i >= (int64_t)*total) return;
    int64_t a = 0, b = NC;                   // last slot p with chunkoff[p] <= i
    while (b - a > 1) { const int64_t m = (a + b) >> 1; if (chunkoff[m] <= (uint32_t)i) a = m; else b = m; }
    const int64_t c = slot_chunk(a, ip.xcd, ncx);
    const uint32_t g = gfirst[c] + (uint32_t)(i - chunkoff[a]);
    const uint4 gb = grp[g];
    WorkItem w;
    w.grp = g;
    w.c0 = max((uint32_t)c * chunk, gb.x);
    w.c1 = min((uint32_t)(c + 1) * chunk, gb.y);
    w.pad = 0;
    items[i] = w;
}

// base[i] = items of the table entries before i (exclusive prefix over the
// images' item counts), base[n] = all items. One workgroup: each thread sums
// a contiguous run of entries, then the 256 partial sums are scanned.
__global__ __launch_bounds__(256) void k_item_bases(const SearchArgs *__restrict__ tab, int32_t n,
                                                    uint32_t *__restrict__ base)
{
    __shared__ uint32_t part[256];
    const int t = threadIdx.x;
    const int per = (n + 255) / 256;
    const int i0 = min(n, t * per), i1 = min(n, i0 + per);
    uint32_t sum = 0;
    for (int i = i0; i < i1; ++i) sum += *tab[i].n_items;
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < 256; ++k) {
            const uint32_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        base[n] = acc;
    }
    __syncthreads();
    uint32_t acc = part[t];
    for (int i = i0; i < i1; ++i) {
        base[i] = acc;
        acc += *tab[i].n_items;
    }
}

// ------------------------------------------------------------ MFMA search
// Both tile shapes screen every (range, column) cell of a block and append
// the cells that pass to a per-wave queue in LDS, with their exact cross
// terms; when the queue holds a wave's worth of cells, every lane fits one of
// them exactly (out of line, so the hot loop stays small and unrolled), the
// wave's best keys (in LDS) take an LDS atomic minimum, and the refreshed
// thresholds come back through LDS. Fitting a passing cell in place would run
// the exact fit on the whole wave for the few lanes that passed.
constexpr int kQueue = 256;          // queued cells per wave (capacity)
// 16x16 ranges pass few cells: half the capacity leaves LDS for wider stages
template <int B> constexpr int queue16_cap() { return B == 16 ? 128 : kQueue; }
// A block that leaves at least flush_at cells queued (SearchArgs::flush_at,
// chosen per image; 0 = only when the queue is full) flushes them at once:
// every flush publishes the wave's best keys, takes the other waves', and
// tightens the thresholds (narrow pools pass many cells early). By default
// only 8x8 ranges flush early (at 64): at 4x4 and 16x16 the extra flushes
// cost more than they save.
// Word 3 of a raw buffer descriptor on gfx9-family GPUs (32-bit data format,
// no swizzle): byte offsets, no stride.
constexpr int kBufWord3 = 0x00020000;

template <class T> __device__ __forceinline__ const __attribute__((address_space(1))) T *
as_global(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}

// A pointer every lane holds the same value of, moved to scalar registers, so
// that block offsets are scalar arithmetic and loads use the scalar base.
template <class T> __device__ __forceinline__ const T *uniform_ptr(const T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const T *)(((uint64_t)hi << 32) | lo);
}

// True when any lane's flag is set (the wave's ballot is not zero).
__device__ __forceinline__ bool wave_any(bool x)
{
    return __builtin_amdgcn_ballot_w64(x) != 0;
}

// ---------------- 16 x 16 tiles (8x8 and 16x16 ranges)
// A wave owns GR = 2*MB ranges. Lane l of a tile sees column l%16 against 4
// isometries of one range, half of a cell (a_place): at 8x8 the two row
// blocks 2g, 2g+1 hold range 4*(l/16) + g, at 16x16 row block b holds ranges
// 2b and 2b+1.
template <int B> __device__ __forceinline__ int tile_range(int b, int lane)
{
    return Cfg<B>::QR ? 4 * (lane >> 4) + (b >> 1) : 2 * b + (lane >> 5);
}
template <int B> __device__ __forceinline__ int tile_iso(int b, int lane)
{
    return Cfg<B>::QR ? 4 * (b & 1) : 4 * ((lane >> 4) & 1);
}

template <int B> struct Queue16 {
    int32_t c[4][queue16_cap<B>()];  // exact cross terms of the half cell
    uint32_t p[queue16_cap<B>()];    // column
    uint32_t lq[queue16_cap<B>()];   // range within the group | isometry base << 8
    u64 best[Cfg<B>::GR];            // best keys of the wave's ranges
    float T[Cfg<B>::GR];             // their thresholds
    int64_t srr[Cfg<B>::GR];         // their Srr'
    int32_t delta[Cfg<B>::GR];       // their delta = sum r - n*rhat
    uint32_t lo[Cfg<B>::GR];         // their pool windows (empty if idle)
    uint32_t hi[Cfg<B>::GR];
};

template <int B> struct WaveState {
    typedef typename Frag<Cfg<B>::EPL>::type frag_t;
    frag_t af[Cfg<B>::MB][Cfg<B>::KS];
    float T[Cfg<B>::MB];
    uint32_t lo[Cfg<B>::MB], hi[Cfg<B>::MB];
    uint32_t grp;
    uint32_t qn;                     // queued half cells (wave-uniform)
    uint32_t flush_at;               // early flush trigger (0: off)
    u64 survivors;
    u64 screened;
};

// Fit the nq queued half cells (one per lane and round of 64), fold the keys
// into the LDS best keys, write the thresholds to LDS. The column loads of
// all rounds are issued before the first fit, so their latency is paid once
// per flush; the range constants come from LDS.
// The current global key of range `lane` of group grp: an atomic load at
// device scope (never an older copy from this XCD's L2). Any value it
// returns is a key some wave reached, so taking it is always valid.
__device__ __forceinline__ u64 group_key(u64 *keys, uint32_t grp, int gr, int lane)
{
    return __hip_atomic_load(&keys[(int64_t)grp * gr + lane], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

template <int B>
__device__ __noinline__ void flush16(const SearchArgs *ta, uint32_t nq, Queue16<B> *qu,
                                     uint32_t grp)
{
    constexpr int n = Cfg<B>::n, GR = Cfg<B>::GR, RQ = queue16_cap<B>() / 64;
    const float slack = screen_slack<B>();
    const int lane = threadIdx.x & 63;
    const SearchArgs a = *ta;
    const auto *gsdd = as_global(a.sdd);
    const auto *geps = as_global(a.eps);
    const auto *gdom = as_global(a.dom);
    const auto *gu = as_global(a.u);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint32_t pe[RQ], lqe[RQ], dm[RQ];
    int64_t sd[RQ];
    int32_t ep[RQ];
    float uu[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        const uint32_t e = (uint32_t)(r * 64 + lane);
        pe[r] = 0; lqe[r] = 0; dm[r] = 0; sd[r] = 0; ep[r] = 0; uu[r] = 0.0f;
        if (e < nq) {
            pe[r] = qu->p[e];
            lqe[r] = qu->lq[e];
        }
    }
#pragma unroll
    for (int r = 0; r < RQ; ++r)
        if ((uint32_t)(r * 64 + lane) < nq) {
            sd[r] = gsdd[pe[r]];
            ep[r] = geps[pe[r]];
            dm[r] = gdom[pe[r]];
            uu[r] = gu[pe[r]];
        }
    // what other waves on the same ranges (other column chunks) have found,
    // read with the column loads (one memory round trip per flush)
    const u64 gk = lane < GR ? group_key(a.keys, grp, GR, lane) : kNoKey;
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        const uint32_t e = (uint32_t)(r * 64 + lane);
        // the isometries of the half cell that still pass the screen against
        // the range's current threshold (the queued cross terms are exact);
        // the wave fits one of them per lane and step, in increasing order
        uint32_t mask = 0;
        uint32_t ls = 0, isob = 0;
        if (e < nq) {
            ls = lqe[r] & 255u;
            isob = lqe[r] >> 8;
            const float t = qu->T[ls];
            const float g = quant_threshold<B>(uu[r]) - slack;    // the quantised contrast
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float c = fabsf((float)qu->c[v][e]);
                if (fmaf(-t, uu[r], c) >= -slack && c >= g) mask |= 1u << v;
            }
        }
        if (!wave_any(mask != 0)) continue;
        const double base = 4096.0 * (double)qu->srr[ls];
        const double ne = (double)qu->delta[ls] * (double)ep[r];
        const double dd = (double)sd[r];
        const float inv = __builtin_amdgcn_rcpf((float)dd);
        const bool any = mask != 0;
        double fb = 0.0;
        int vb = -1;
        while (wave_any(mask != 0)) {
            if (mask) {
                const int v = __builtin_ctz(mask);
                mask &= mask - 1u;
                const double rd = (double)n * (double)qu->c[v][e] - ne;   // exact integers
                const double f = fit_f_d(base, rd, dd, inv);
                if (vb < 0 || f < fb) {      // ascending v: ties keep the lower isometry
                    fb = f;
                    vb = v;
                }
            }
        }
        if (any) atomicMin(&qu->best[ls], pack_key((int64_t)fb, dm[r], (int)isob + vb, a.shift));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < GR) {
        // take the other waves' keys read above and publish the wave's best
        // (no wait for the atomic's reply)
        u64 bk = qu->best[lane];
        bk = gk < bk ? gk : bk;
        atomicMin(&a.keys[(int64_t)grp * GR + lane], bk);
        qu->best[lane] = bk;
        qu->T[lane] = bk == kNoKey ? 0.0f : screen_t_b<B>(qu->srr[lane], (int64_t)(bk >> a.shift));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Fit and empty the queue. The thresholds the wave screens with are reloaded
// separately (refresh16): a block's pass tests are all taken before its
// cells are queued, so a flush in the middle of queueing them changes
// nothing for that block, and keeping the thresholds fixed until the block
// is queued keeps them out of the queueing branches' register copies.
template <int B>
__device__ __forceinline__ void flush_queue16(const SearchArgs *ta, WaveState<B> &st,
                                              Queue16<B> *qu)
{
    flush16<B>(ta, st.qn, qu, st.grp);
    st.survivors += 4ull * st.qn;    // wave-uniform
    st.qn = 0;
}

template <int B>
__device__ __forceinline__ void refresh16(WaveState<B> &st, const Queue16<B> *qu)
{
    constexpr int MW = Cfg<B>::MB;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int b = 0; b < MW; ++b)
        if (st.T[b] != __builtin_inff())        // searched ranges only
            st.T[b] = qu->T[tile_range<B>(b, lane)];
}

// The cross terms of one 16-column block against the wave's row blocks.
template <int B>
__device__ __forceinline__ void mma_block(const WaveState<B> &st,
                                          const typename WaveState<B>::frag_t (&bf)[Cfg<B>::KS],
                                          float4_t (&acc)[Cfg<B>::MB][Cfg<B>::NCH])
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, NCH = C::NCH, KPC = C::KS / NCH;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int kk = 0; kk < KPC; ++kk)
#pragma unroll
            for (int b = 0; b < MW; ++b) {
                const float4_t z = {0.f, 0.f, 0.f, 0.f};
                acc[b][c] = mma(st.af[b][c * KPC + kk], bf[c * KPC + kk], kk ? acc[b][c] : z);
            }
}

// Append row block b's passing half cells (at most 64) to the wave's queue,
// with their exact cross terms (each 64-term chunk is exact in FP32).
template <int B>
__device__ __forceinline__ void queue_rowblock(const SearchArgs *ta, WaveState<B> &st,
                                               Queue16<B> *qu, int b, bool pass,
                                               const float4_t (&accb)[Cfg<B>::NCH], uint32_t p,
                                               bool &flushed)
{
    constexpr int NCH = Cfg<B>::NCH;
    const int lane = threadIdx.x & 63;
    const u64 ball = __ballot(pass);
    if (ball == 0) return;
    const uint32_t cnt = (uint32_t)__popcll(ball);
    if (st.qn + cnt > (uint32_t)queue16_cap<B>()) {
        flush_queue16<B>(ta, st, qu);
        flushed = true;
    }
    if (pass) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(ball >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0u));
        const uint32_t pos = st.qn + below;
        const uint32_t isob = (uint32_t)tile_iso<B>(b, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int32_t cx = 0;
#pragma unroll
            for (int c = 0; c < NCH; ++c) cx += (int32_t)accb[c][v];
            qu->c[v][pos] = cx;
        }
        qu->p[pos] = p;
        qu->lq[pos] = (uint32_t)tile_range<B>(b, lane) | (isob << 8);
    }
    st.qn += cnt;
}

// Screen the cross terms of column block cb; queue the passing half cells.
template <int B, bool MASK>
__device__ __forceinline__ void screen_acc(const SearchArgs *ta, WaveState<B> &st,
                                           Queue16<B> *qu,
                                           const float4_t (&acc)[Cfg<B>::MB][Cfg<B>::NCH],
                                           float u, int cb)
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, NCH = C::NCH;
    const float slack = screen_slack<B>();
    const int lane = threadIdx.x & 63, col = lane & 15;
    const uint32_t p = (uint32_t)cb * 16 + col;
    if (C::QR) {
        // one range per lane in row blocks 2g, 2g+1: one threshold for the
        // 8 isometries, and only a block where some lane passes takes the
        // per-row-block tests below
        bool any = false;
        float dg = -__builtin_inff();
#pragma unroll
        for (int g = 0; g < MW / 2; ++g) {
            const float4_t x = acc[2 * g][0], y = acc[2 * g + 1][0];
            // a left-leaning chain: v_max3 takes two new values at a time
            float m = fmaxf(fabsf(x[0]), fabsf(x[1]));
            m = fmaxf(fmaxf(m, fabsf(x[2])), fabsf(x[3]));
            m = fmaxf(fmaxf(m, fabsf(y[0])), fabsf(y[1]));
            m = fmaxf(fmaxf(m, fabsf(y[2])), fabsf(y[3]));
            const float d = fmaf(-st.T[2 * g], u, m);
            if (MASK) any = any || (d >= -slack && p >= st.lo[2 * g] && p < st.hi[2 * g]);
            else dg = fmaxf(dg, d);
        }
        if (!MASK) any = dg >= -slack;
        if (!MASK && MW == 8 && C::KS == 2) {
            // the last MFMAs of the block interleaved with the screens of the
            // ranges whose row blocks are done (12 MFMAs, then a range's 5
            // VALU instructions per 2 MFMAs, the last two ranges, the fold and
            // the compare): the screen no longer waits on fresh MFMA results
            __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);    // VALU
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 13, 0);
        }
        if (!wave_any(any)) return;
    }
    bool pass[MW];
    bool hit = false;
    float dmax = -__builtin_inff();
#pragma unroll
    for (int b = 0; b < MW; ++b) {
        float4_t sv = acc[b][0];
#pragma unroll
        for (int c = 1; c < NCH; ++c) sv += acc[b][c];
        const float m = fmaxf(fmaxf(fabsf(sv[0]), fabsf(sv[1])), fmaxf(fabsf(sv[2]), fabsf(sv[3])));
        // m - T u in one rounding: >= -slack whenever m >= T u - slack
        const float d = fmaf(-st.T[b], u, m);
        bool h = d >= -slack;
        if (MASK) h = h && p >= st.lo[b] && p < st.hi[b];
        pass[b] = h;
        if (MASK) hit = hit || h;
        else dmax = fmaxf(dmax, d);  // unmasked: one compare for all row blocks
    }
    if (!MASK) hit = dmax >= -slack;
    if (!wave_any(hit)) return;
    bool flushed = false;
#pragma unroll
    for (int b = 0; b < MW; ++b) queue_rowblock<B>(ta, st, qu, b, pass[b], acc[b], p, flushed);
    if (st.flush_at && st.qn >= st.flush_at) {
        flush_queue16<B>(ta, st, qu);
        flushed = true;
    }
    if (flushed) refresh16<B>(st, qu);
}

template <int B, bool MASK>
__device__ __forceinline__ void screen_block(const SearchArgs *ta, WaveState<B> &st,
                                             Queue16<B> *qu,
                                             const typename WaveState<B>::frag_t (&bf)[Cfg<B>::KS],
                                             float u, int cb)
{
    float4_t acc[Cfg<B>::MB][Cfg<B>::NCH];
    mma_block<B>(st, bf, acc);
    screen_acc<B, MASK>(ta, st, qu, acc, u, cb);
}

// The hot cross terms of one 16-column block whose B fragments are in LDS:
// all KS MFMAs of a row block chained into one accumulator.
template <int B>
__device__ __forceinline__ void mma_block_lds(const WaveState<B> &st,
                                              const typename WaveState<B>::frag_t *lb,
                                              float4_t (&acc)[Cfg<B>::MB])
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, KS = C::KS;
    typedef typename WaveState<B>::frag_t frag_t;
    const int lane = threadIdx.x & 63;
    frag_t bf[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bf[ks] = lb[ks * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int b = 0; b < MW; ++b) {
            const float4_t z = {0.f, 0.f, 0.f, 0.f};
            acc[b] = mma(st.af[b][ks], bf[ks], ks ? acc[b] : z);
        }
    // all reads first, then the MFMAs K step by K step (without this the
    // scheduler interleaves them less well and the block needs more VGPRs)
    __builtin_amdgcn_sched_group_barrier(0x100, KS, 0);   // LDS reads
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) __builtin_amdgcn_sched_group_barrier(0x008, MW, 0);   // MFMAs
}

// Rounding check of the one-accumulator screen on the matrix cores (the
// context's verify switch): every value of the block is recomputed from the
// exact 64-term chunks, summed in int32 (exact), and its distance from the
// one-accumulator FP32 sum is compared with the bound the threshold is
// lowered by, e*u + e/2 with e = (n + KS) 2^-23 sqrt(n) ||A|| (screen_t_b;
// ||B|| <= sqrt(n) (u + 1/2), u undone from its rounding down). Counts, in
// vc: [0] values over the bound, [1] values checked, [2] the largest
// error / bound seen, in units of 2^-20 (atomic maximum).
template <int B>
__device__ __noinline__ void verify_block_lds(const WaveState<B> &st, const Queue16<B> *qu,
                                              const typename WaveState<B>::frag_t *lb,
                                              const float4_t (&acc)[Cfg<B>::MB], float u, u64 *vc)
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, KS = C::KS, NCH = C::NCH, KPC = KS / NCH, n = C::n;
    const int lane = threadIdx.x & 63;
    u64 bad = 0, seen = 0, worst = 0;
#pragma unroll
    for (int b = 0; b < MW; ++b) {
        float4_t ax[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int kk = 0; kk < KPC; ++kk) {
                const float4_t z = {0.f, 0.f, 0.f, 0.f};
                ax[c] = mma(st.af[b][c * KPC + kk], lb[(c * KPC + kk) * 64 + lane], kk ? ax[c] : z);
            }
        const double srr = (double)qu->srr[tile_range<B>(b, lane)];
        const double na = sqrt(srr / n + n / 4.0);
        const double e = (double)(n + KS) * 0x1p-23 * sqrt((double)n) * na;
        const double bound = e * ((double)u * (1.0 + 0x1p-19)) + e * 0.5;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int32_t sx = 0;
#pragma unroll
            for (int c = 0; c < NCH; ++c) sx += (int32_t)ax[c][v];
            const double err = fabs((double)acc[b][v] - (double)sx);
            seen += 1;
            if (err > bound) bad += 1;
            const double ratio = bound > 0.0 ? err / bound : (err > 0.0 ? 1e9 : 0.0);
            const u64 q = (u64)fmin(ratio * 1048576.0, 1e18);
            worst = q > worst ? q : worst;
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        bad += __shfl_xor(bad, off);
        seen += __shfl_xor(seen, off);
        const u64 o = __shfl_xor(worst, off);
        worst = o > worst ? o : worst;
    }
    if (lane == 0 && vc) {
        atomicAdd(&vc[0], bad);
        atomicAdd(&vc[1], seen);
        atomicMax(&vc[2], worst);
    }
}

// 16x16 ranges, B fragments of the block in LDS (lane order). The hot test
// screens the one-accumulator sums; only a block where some lane passes
// recomputes the exact 64-term chunk sums (re-reading its fragments) and
// goes through the exact screen and queue.
template <int B, bool MASK, bool VERIFY>
__device__ __forceinline__ void screen_block_lds(const SearchArgs *ta, WaveState<B> &st,
                                                 Queue16<B> *qu,
                                                 const typename WaveState<B>::frag_t *lb,
                                                 const float4_t (&acc)[Cfg<B>::MB], float u, int cb,
                                                 u64 *vc)
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, KS = C::KS;
    const int lane = threadIdx.x & 63, col = lane & 15;
    const float slack = screen_slack<B>();
    const uint32_t p = (uint32_t)cb * 16 + col;
    if constexpr (VERIFY) verify_block_lds<B>(st, qu, lb, acc, u, vc);
    bool hit = false;
    float dmax = -__builtin_inff();
#pragma unroll
    for (int b = 0; b < MW; ++b) {
        const float4_t sv = acc[b];
        const float m = fmaxf(fmaxf(fabsf(sv[0]), fabsf(sv[1])), fmaxf(fabsf(sv[2]), fabsf(sv[3])));
        const float d = fmaf(-st.T[b], u, m);
        if (MASK) hit = hit || (d >= -slack && p >= st.lo[b] && p < st.hi[b]);
        else dmax = fmaxf(dmax, d);
    }
    if (!MASK) hit = dmax >= -slack;
    if (!wave_any(hit)) return;
    // exact chunk sums, exact screen and queue, one row block at a time
    // (after a flush in the middle, the later row blocks still screen with
    // the thresholds the block started with: looser, never wrong, and the
    // flush re-screens every queued cell against the current ones)
    constexpr int NCH = C::NCH, KPC = KS / NCH;
    const float slx = screen_slack<B>();
    bool flushed = false;
#pragma unroll
    for (int b = 0; b < MW; ++b) {
        float4_t ax[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int kk = 0; kk < KPC; ++kk) {
                const float4_t z = {0.f, 0.f, 0.f, 0.f};
                ax[c] = mma(st.af[b][c * KPC + kk], lb[(c * KPC + kk) * 64 + lane], kk ? ax[c] : z);
            }
        float4_t sv = ax[0];
#pragma unroll
        for (int c = 1; c < NCH; ++c) sv += ax[c];
        const float m = fmaxf(fmaxf(fabsf(sv[0]), fabsf(sv[1])), fmaxf(fabsf(sv[2]), fabsf(sv[3])));
        bool h = fmaf(-st.T[b], u, m) >= -slx;
        if (MASK) h = h && p >= st.lo[b] && p < st.hi[b];
        queue_rowblock<B>(ta, st, qu, b, h, ax, p, flushed);
    }
    if (st.flush_at && st.qn >= st.flush_at) {
        flush_queue16<B>(ta, st, qu);
        flushed = true;
    }
    if (flushed) refresh16<B>(st, qu);
}

// Column blocks [cb_begin, cb_end) against the wave's A rows. The B
// fragments and u of the block two ahead are loaded while a block computes.
template <int B, bool MASK>
__device__ __forceinline__ void scan_blocks(const SearchArgs &a, const SearchArgs *ta,
                                            WaveState<B> &st, Queue16<B> *qu, int cb_begin,
                                            int cb_end)
{
    using C = Cfg<B>;
    constexpr int KS = C::KS;
    typedef typename WaveState<B>::frag_t frag_t;
    cb_begin = __builtin_amdgcn_readfirstlane(cb_begin);
    cb_end = __builtin_amdgcn_readfirstlane(cb_end);
    if (cb_begin >= cb_end) return;
    const int lane = threadIdx.x & 63, col = lane & 15;
    // Buffer loads: the block offset goes in the scalar offset, the lane
    // offset in a 32-bit VGPR, so no 64-bit address arithmetic per block. The
    // key's domain field holds at most 2^23 domains at 8x8 (F < 2^38), so B
    // stays below 2^30 bytes and every offset fits 32 bits (the API checks it).
    static_assert(B == 8, "32-bit buffer offsets are sized for 8x8 ranges");
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(a.Bm), (short)0, -1, kBufWord3);
    const __amdgpu_buffer_rsrc_t ru =
        __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(a.u), (short)0, -1, kBufWord3);
    const uint32_t lb = (uint32_t)lane * (uint32_t)sizeof(frag_t), lu = (uint32_t)col * 4u;
    constexpr uint32_t kBlkB = KS * 64 * sizeof(frag_t), kBlkU = 16 * 4;
    auto ldb = [&](int c, int ks) {
        return __builtin_bit_cast(frag_t, __builtin_amdgcn_raw_buffer_load_b128(
                                              rb, lb + (uint32_t)(ks * 64 * sizeof(frag_t)),
                                              (int)((uint32_t)c * kBlkB), 0));
    };
    auto ldu = [&](int c) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                             ru, lu, (int)((uint32_t)c * kBlkU), 0));
    };
    const int last = cb_end - 1;
    frag_t b0[KS], b1[KS];
    float u0, u1;
    {
        const int c1 = min(cb_begin + 1, last);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            b0[ks] = ldb(cb_begin, ks);
            b1[ks] = ldb(c1, ks);
        }
        u0 = ldu(cb_begin);
        u1 = ldu(c1);
    }
    // whole pairs of blocks without a branch between them (a conditional
    // second step would make the compiler wait for the loads just issued)
    // the MFMAs of a block are issued before its fragments are reloaded
    // (no register copies), and the screen follows the reload
    int cb = cb_begin;
    for (; cb + 2 <= cb_end; cb += 2) {
        {
            float4_t acc[C::MB][C::NCH];
            mma_block<B>(st, b0, acc);
            const float uc = u0;
            const int nx = min(cb + 2, last);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) b0[ks] = ldb(nx, ks);
            u0 = ldu(nx);
            screen_acc<B, MASK>(ta, st, qu, acc, uc, cb);
        }
        {
            float4_t acc[C::MB][C::NCH];
            mma_block<B>(st, b1, acc);
            const float uc = u1;
            const int nx = min(cb + 3, last);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) b1[ks] = ldb(nx, ks);
            u1 = ldu(nx);
            screen_acc<B, MASK>(ta, st, qu, acc, uc, cb + 1);
        }
    }
    if (cb < cb_end) screen_block<B, MASK>(ta, st, qu, b0, u0, cb);
}

// Work-item claims of a persistent wave. One counter (ctr[0]) over the items
// of all table entries; or, for one image whose work list is in XCD order,
// one counter per XCD queue (ctr[16 + x]): a wave starts at the queue of the
// XCD its workgroup runs on (workgroups go to the XCDs round robin) and moves
// on to the next queue when that one is empty, until all are empty. Every
// wave reaches the end: each queue is finite and found empty once.
struct ItemQueue {
    int xq;                          // XCD queues
    int q, left;                     // current queue, queues not yet found empty
};
__device__ __forceinline__ ItemQueue item_queue(const SearchArgs *tab, int32_t n_img)
{
    ItemQueue iq;
    iq.xq = n_img == 1 && tab[0].xcd;
    iq.q = (int)(blockIdx.x % kXcds);
    iq.left = kXcds;
    return iq;
}
__device__ __forceinline__ bool claim_item(uint32_t *ctr, const SearchArgs *tab, uint32_t nitems,
                                           uint32_t dbg, ItemQueue &iq, uint32_t &item)
{
    const int lane = threadIdx.x & 63;
    if (!iq.xq) {
        uint32_t i = 0;
        if (lane == 0) i = atomicAdd(ctr, 1u);
        i = __builtin_amdgcn_readfirstlane(i);
        if (i >= nitems) return false;
        item = (dbg & kDbgReverse) ? nitems - 1u - i : i;   // order-independence check
        return true;
    }
    const uint32_t *xq = tab->xq;
    const int ncx = tab->ncx;
    while (iq.left > 0) {
        const int q = __builtin_amdgcn_readfirstlane(iq.q);
        const uint32_t lo = xq[q * ncx];
        const uint32_t hi = q == kXcds - 1 ? nitems : xq[(q + 1) * ncx];
        uint32_t j = 0;
        if (lane == 0) j = atomicAdd(ctr + 16 + q, 1u);
        j = __builtin_amdgcn_readfirstlane(j);
        if (lo + j < hi) {
            item = (dbg & kDbgReverse) ? hi - 1u - j : lo + j;
            return true;
        }
        iq.q = (q + 1) % kXcds;
        iq.left -= 1;
    }
    return false;
}

// Claiming ahead: claim_issue sends the plain queue's atomic for the next
// item (lane 0's reply, not yet read), claim_take reads it when that item
// is due, so the atomic's round trip overlaps the current item's end (its
// last flush and key publication). With the per-XCD queues claim_take
// claims then (claim_item). (The file is built without the compiler's
// atomic optimizer, which would turn the lane-0 atomic into a wave-wide one
// that reads its reply at once.)
__device__ __forceinline__ void claim_issue(uint32_t *ctr, const ItemQueue &iq, uint32_t &raw)
{
    // only lane 0's value is read; the other lanes keep theirs, so the reply
    // needs no merge (a merge would wait for it right here)
    if (!iq.xq && (threadIdx.x & 63) == 0) raw = atomicAdd(ctr, 1u);
}
__device__ __forceinline__ bool claim_take(uint32_t raw, uint32_t *ctr, const SearchArgs *tab,
                                           uint32_t nitems, uint32_t dbg, ItemQueue &iq,
                                           uint32_t &item)
{
    if (iq.xq) return claim_item(ctr, tab, nitems, dbg, iq, item);
    const uint32_t i = __builtin_amdgcn_readfirstlane(raw);
    if (i >= nitems) return false;
    item = (dbg & kDbgReverse) ? nitems - 1u - i : i;   // order-independence check
    return true;
}

// The image of global item `item` among n_img table entries with item bases
// base[] (last entry whose base <= item), wave-uniform.
// The bases are read through the constant address space: wave-uniform
// scalar loads that hit the scalar cache (every wave reads the same few
// words), not one vector-memory round trip per bisection step.
typedef __attribute__((address_space(4))) const uint32_t cu32;
__device__ __forceinline__ int image_of_item(const uint32_t *__restrict__ base, int32_t n_img,
                                             uint32_t item)
{
    cu32 *cb = (cu32 *)base;
    int ia = 0, ib = n_img;
    while (ib - ia > 1) {
        const int m = __builtin_amdgcn_readfirstlane((ia + ib) >> 1);
        if (cb[m] <= item) ia = m; else ib = m;
    }
    return __builtin_amdgcn_readfirstlane(ia);
}

// Item index `item` of image ia relative to its base (a scalar load, as above).
__device__ __forceinline__ uint32_t item_in_image(const uint32_t *__restrict__ base, int ia,
                                                  uint32_t item)
{
    return item - ((cu32 *)base)[ia];
}

// One work item (a group of 2*MB ranges against a run of column blocks) of
// the 16x16-tile search: load the group's A rows and thresholds, scan the
// blocks (masked where some range's pool ends inside them), flush, publish
// the keys.
struct NoHook {
    __device__ void operator()() const {}
};

template <int B, class Hook = NoHook>
__device__ __forceinline__ void item16(const SearchArgs *ta, const SearchArgs &a,
                                       const WorkItem &wi, WaveState<B> &st, Queue16<B> *qu,
                                       const Hook &before_end = Hook())
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, KS = C::KS, GR = C::GR;
    typedef typename WaveState<B>::frag_t frag_t;
    const int lane = threadIdx.x & 63;
    st.flush_at = (uint32_t)a.flush_at;
    st.grp = wi.grp;
    const frag_t *ap = (const frag_t *)a.A + (int64_t)st.grp * MW * KS * 64 + lane;
#pragma unroll
    for (int b = 0; b < MW; ++b)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) st.af[b][ks] = ap[(b * KS + ks) * 64];
    if (lane < GR) {
        // the group's range constants and thresholds, once per range: the
        // flush re-screens queued cells against these, and every lane takes
        // its row blocks' values from here (an active range's pool is never
        // empty, so an empty window marks an idle range)
        const int64_t slot = (int64_t)st.grp * GR + lane;
        const u64 bk = a.keys[slot];
        const RangeStat rsx = a.rs[slot];
        const bool act = !(rsx.flags & kIdle);
        qu->best[lane] = bk;
        qu->srr[lane] = rsx.srr;
        qu->delta[lane] = rsx.delta;
        qu->T[lane] = bk == kNoKey ? 0.0f : screen_t_b<B>(rsx.srr, (int64_t)(bk >> a.shift));
        qu->lo[lane] = act ? rsx.lo : 0u;
        qu->hi[lane] = act ? rsx.hi : 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int b = 0; b < MW; ++b) {
        const int r = tile_range<B>(b, lane);
        st.lo[b] = qu->lo[r];
        st.hi[b] = qu->hi[r];
        st.T[b] = st.hi[b] > st.lo[b] ? qu->T[r] : __builtin_inff();
    }
    const uint4 gb = a.grp[st.grp];
    const int cb0 = (int)(wi.c0 >> 4), cb1 = (int)(wi.c1 >> 4);
    // column blocks fully inside every active range's pool need no mask
    int ib0 = (int)((gb.z + 15u) >> 4), ib1 = (int)(gb.w >> 4);
    ib0 = min(max(ib0, cb0), cb1);
    ib1 = max(min(ib1, cb1), ib0);
    st.screened += (u64)(cb1 - cb0) * 16 * GR * 8;
    scan_blocks<B, true>(a, ta, st, qu, cb0, ib0);
    scan_blocks<B, false>(a, ta, st, qu, ib0, ib1);
    scan_blocks<B, true>(a, ta, st, qu, ib1, cb1);
    before_end();
    if (st.qn) flush_queue16<B>(ta, st, qu);
    if (lane < GR) {
        const u64 bk = qu->best[lane];
        if (bk != kNoKey) atomicMin(&a.keys[(int64_t)st.grp * GR + lane], bk);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// A wave's counters at the end of a persistent search.
__device__ __forceinline__ void add_counters(u64 *counters, u64 screened, u64 survivors,
                                             u64 items_done)
{
    if (!counters) return;
    if ((threadIdx.x & 63) == 0) {      // all three counts are wave-uniform
        atomicAdd(&counters[0], screened);
        atomicAdd(&counters[1], survivors);
        atomicAdd(&counters[2], items_done);
    }
}

// Items of n_img images (table entries tab[0..n_img), item bases base[]) in
// one queue: a wave claims an item, finds its image by binary search over
// the bases, and loads that image's operands.
// 8 row blocks of 8x8 ranges fill 2 waves/SIMD (237 VGPRs); fewer blocks at
// more waves per SIMD re-read B more and measure slower.
template <int B>
__global__ __launch_bounds__(256, 2) void k_search_mfma(const SearchArgs *__restrict__ tab,
                                                        const uint32_t *__restrict__ base,
                                                        int32_t n_img, uint32_t *item_ctr,
                                                        u64 *counters, uint32_t dbg)
{
    __shared__ Queue16<B> queues[4];
    Queue16<B> *qu = &queues[threadIdx.x >> 6];
    const uint32_t nitems = base[n_img];
    WaveState<B> st;
    st.survivors = 0;
    st.screened = 0;
    st.qn = 0;
    u64 items_done = 0;
    ItemQueue iq = item_queue(tab, n_img);
    uint32_t raw = 0;
    claim_issue(item_ctr, iq, raw);
    for (;;) {
        uint32_t item;
        if (!claim_take(raw, item_ctr, tab, nitems, dbg, iq, item)) break;
        const int ia = image_of_item(base, n_img, item);
        const SearchArgs *ta = tab + ia;
        const SearchArgs a = *ta;
        // the next item is claimed before this one's end work
        item16<B>(ta, a, a.items[item_in_image(base, ia, item)], st, qu,
                  [&]() { claim_issue(item_ctr, iq, raw); });
        items_done += 1;
    }
    add_counters(counters, st.screened, st.survivors, items_done);
}

// ---------------- 16 x 16 tiles with B shared through LDS (16x16 ranges)
// A 16x16 range has 256 pixels: every 16-column block brings 8 KB of B
// fragments per wave for only 16 MFMAs, more than the L1/L2 path feeds four
// SIMDs. So a workgroup takes (4 consecutive groups, column chunk) items: its
// 4 waves load each stage of kStage16 column blocks into LDS once (direct
// global->LDS loads, double-buffered, one barrier per stage) and each wave
// screens its own group's ranges against them; blocks outside a wave's own
// pools are skipped, blocks inside all of them skip the per-range mask.
constexpr int kStage16 = 4;          // 16-column blocks per LDS stage

typedef __attribute__((address_space(3))) void lds_void;

template <int B, bool VERIFY>
__global__ __launch_bounds__(256, 2) void k_search_lds16(const SearchArgs *__restrict__ tab,
                                                         const uint32_t *__restrict__ base,
                                                         int32_t n_img, uint32_t *item_ctr,
                                                         u64 *counters, uint32_t dbg)
{
    using C = Cfg<B>;
    constexpr int MW = C::MB, KS = C::KS, GR = C::GR, SB = kStage16, FR = SB * KS;
    typedef typename WaveState<B>::frag_t frag_t;
    __shared__ frag_t sB0[FR * 64], sB1[FR * 64];   // two separate buffers: the DMA into one
    __shared__ float sU0[SB * 16], sU1[SB * 16];    // never aliases the one being read
    __shared__ Queue16<B> queues[4];
    __shared__ uint32_t sItem;
    __shared__ int sOk;
    const int lane = threadIdx.x & 63, col = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Queue16<B> *qu = &queues[w];
    const uint32_t nitems = base[n_img];
    WaveState<B> st;
    st.survivors = 0;
    st.screened = 0;
    st.qn = 0;
    u64 items_done = 0;
    ItemQueue iq = item_queue(tab, n_img);     // used by wave 0, which claims for the workgroup
    for (;;) {
        if (w == 0) {
            uint32_t it = 0;
            const bool ok = claim_item(item_ctr, tab, nitems, dbg, iq, it);
            if (lane == 0) {
                sItem = it;
                sOk = ok ? 1 : 0;
            }
        }
        __syncthreads();
        const uint32_t item = sItem;
        const int ok = sOk;
        __syncthreads();
        if (!ok) break;
        const int ia = image_of_item(base, n_img, item);
        const SearchArgs *ta = tab + ia;
        const SearchArgs a = *ta;
        const WorkItem wi = a.items[item_in_image(base, ia, item)];
        st.flush_at = (uint32_t)a.flush_at;
        st.grp = __builtin_amdgcn_readfirstlane(wi.grp) * 4 + (uint32_t)w;
        const frag_t *ap = (const frag_t *)a.A + (int64_t)st.grp * MW * KS * 64 + lane;
#pragma unroll
        for (int b = 0; b < MW; ++b)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) st.af[b][ks] = ap[(b * KS + ks) * 64];
        if (lane < GR) {
            // the range constants and thresholds once per range (as item16):
            // the flush re-screens queued cells against them and every lane
            // takes its row blocks' values from here
            const int64_t slot = (int64_t)st.grp * GR + lane;
            const u64 bk = a.keys[slot];
            const RangeStat rsx = a.rs[slot];
            const bool act = !(rsx.flags & kIdle);
            qu->best[lane] = bk;
            qu->srr[lane] = rsx.srr;
            qu->delta[lane] = rsx.delta;
            qu->T[lane] = bk == kNoKey ? 0.0f : screen_t_b<B>(rsx.srr, (int64_t)(bk >> a.shift));
            qu->lo[lane] = act ? rsx.lo : 0u;
            qu->hi[lane] = act ? rsx.hi : 0u;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // the wave's own pools: union [wlo, whi) and intersection [ilo, ihi)
        uint32_t wlo = 0xffffffffu, whi = 0u, ilo = 0u, ihi = 0xffffffffu;
#pragma unroll
        for (int b = 0; b < MW; ++b) {
            const int r = tile_range<B>(b, lane);
            st.lo[b] = qu->lo[r];
            st.hi[b] = qu->hi[r];
            const bool act = st.hi[b] > st.lo[b];     // an empty window: idle
            st.T[b] = act ? qu->T[r] : __builtin_inff();
            if (act) {
                wlo = min(wlo, st.lo[b]); whi = max(whi, st.hi[b]);
                ilo = max(ilo, st.lo[b]); ihi = min(ihi, st.hi[b]);
            }
        }
        wlo = min(wlo, (uint32_t)__shfl_xor((int)wlo, 32));
        whi = max(whi, (uint32_t)__shfl_xor((int)whi, 32));
        ilo = max(ilo, (uint32_t)__shfl_xor((int)ilo, 32));
        ihi = min(ihi, (uint32_t)__shfl_xor((int)ihi, 32));
        wlo = __builtin_amdgcn_readfirstlane(wlo);
        whi = __builtin_amdgcn_readfirstlane(whi);
        ilo = __builtin_amdgcn_readfirstlane(ilo);
        ihi = __builtin_amdgcn_readfirstlane(ihi);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int cb0 = __builtin_amdgcn_readfirstlane((int)(wi.c0 >> 4));
        const int cb1 = __builtin_amdgcn_readfirstlane((int)(wi.c1 >> 4));
        const int nst = (cb1 - cb0 + SB - 1) / SB;
        // the wave's blocks: [lb0, lb1) meet its pools, [ib0, ib1) lie inside
        // all of them (no per-range mask)
        const int lb0 = max(cb0, (int)(wlo >> 4)), lb1 = min(cb1, (int)((whi + 15u) >> 4));
        const int ib0 = (int)((ilo + 15u) >> 4), ib1 = (int)(ihi >> 4);
        st.screened += (u64)(lb1 > lb0 ? lb1 - lb0 : 0) * 16 * GR * 8;
        const auto *gB = as_global(uniform_ptr((const frag_t *)a.Bm));
        const auto *gU = as_global(uniform_ptr(a.u));
        // each wave loads fragments w, w + 4, ... of the stage; blocks past
        // the item reload its last block (in bounds, never read), so the
        // loads need no branches
        static_assert(FR % 4 == 0, "stage fragments split over 4 waves");
        auto stage_load = [&](int sidx, frag_t *dB, float *dU) {
            const int sb0 = cb0 + sidx * SB;
#pragma unroll
            for (int f = 0; f < FR / 4; ++f) {
                const int fr = w + 4 * f;
                const int blk = min(sb0 + fr / KS, cb1 - 1);
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(gB + ((int64_t)blk * KS + fr % KS) * 64 + lane),
                    (lds_void *)(dB + fr * 64), 16, 0, 0);
            }
            if (w == 0 && lane < SB * 16) {
                const int blk = min(sb0 + lane / 16, cb1 - 1);
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(gU + (int64_t)blk * 16 + (lane & 15)),
                    (lds_void *)dU, 4, 0, 0);
            }
        };
        if (nst > 0) stage_load(0, sB0, sU0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int sidx = 0; sidx < nst; ++sidx) {
            const frag_t *cB = (sidx & 1) ? sB1 : sB0;
            const float *cU = (sidx & 1) ? sU1 : sU0;
            if (sidx + 1 < nst) stage_load(sidx + 1, (sidx & 1) ? sB0 : sB1, (sidx & 1) ? sU0 : sU1);
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int cb = cb0 + sidx * SB + j;
                if (cb < lb0 || cb >= lb1) continue;
                const float u = cU[j * 16 + col];
                float4_t acc[MW];
                mma_block_lds<B>(st, cB + j * KS * 64, acc);
                if (cb >= ib0 && cb < ib1)
                    screen_block_lds<B, false, VERIFY>(ta, st, qu, cB + j * KS * 64, acc, u, cb,
                                                       counters ? counters + 4 : nullptr);
                else
                    screen_block_lds<B, true, VERIFY>(ta, st, qu, cB + j * KS * 64, acc, u, cb,
                                                      counters ? counters + 4 : nullptr);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        if (st.qn) flush_queue16<B>(ta, st, qu);
        if (lane < GR) {
            const u64 bk = qu->best[lane];
            if (bk != kNoKey) atomicMin(&a.keys[(int64_t)st.grp * GR + lane], bk);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        items_done += 1;
    }
    if (counters && lane == 0) {       // wave-uniform counts
        atomicAdd(&counters[0], st.screened);
        atomicAdd(&counters[1], st.survivors);
        if (w == 0) atomicAdd(&counters[2], items_done);
    }
}

// ---------------- 32 x 32 tiles (4x4 ranges; K = 16 per MFMA)
// A wave owns GR = 4*MB ranges: row block blk holds the range quad 4*blk ..
// 4*blk+3 under the 8 isometries. Lane l's 16 outputs of a tile are column
// l%32 against range 4*blk + 2*(l/32) (v < 8) and that + 1 (v >= 8), under
// isometry v%8: whole cells. Per block: MB*KS MFMAs, then per lane and range
// half one 8-value maximum, one fma and one compare.
// A 4x4 range meets many near-optimal domains: on smooth images nearly every
// block has a passing cell. So the scan only queues the COLUMNS in which some
// cell passes (one ballot and one LDS store per block); once kColReplay
// columns are queued (tested after every group of blocks), replay32 gathers
// their B fragments, redoes the MFMAs, screens each cell against its range's
// current threshold and pool window, and queues the passing cells, with
// their cross terms, for the exact fit (flush32).
constexpr int kColReplay = 64;
constexpr int kColQ = kColReplay + 4 * 32;   // + one group of 4 blocks: no overflow check per block

template <int B> struct Queue32 {
    float4_t c[kQueue][2];           // the cell's cross terms, isometries 0-3 and 4-7
    uint32_t p[kQueue];              // column
    uint32_t ls[kQueue];             // range within the wave's group
    uint32_t colp[kColQ];            // queued columns
    float colu[kColQ];               // their u
    half8_t colb[kColQ][2];          // their B fragments (K halves 0, 1), gathered by the replay
    uint32_t lo[Cfg<B>::GR];         // pool windows of the wave's ranges (empty if idle)
    uint32_t hi[Cfg<B>::GR];
    u64 best[Cfg<B>::GR];            // best keys of the wave's ranges
    float T[Cfg<B>::GR];             // their thresholds
    int64_t srr[Cfg<B>::GR];         // their Srr'
    int32_t delta[Cfg<B>::GR];       // their delta = sum r - n*rhat
};

template <int B> struct Wave32 {
    static constexpr int MB = Cfg<B>::MB, KS = Cfg<B>::KS;
    half8_t af[MB][KS];
    float T[MB][2];
    uint32_t lo[MB][2], hi[MB][2];
    uint32_t grp;
    uint32_t qn;                     // queued cells (wave-uniform)
    uint32_t cq;                     // queued columns (wave-uniform)
    uint32_t flush_at;               // early flush trigger (0: off)
    u64 survivors, screened, replayed;
};

__device__ __forceinline__ float max8(const float16_t &a, int base)
{
    const float x = fmaxf(fmaxf(fabsf(a[base + 0]), fabsf(a[base + 1])), fabsf(a[base + 2]));
    const float y = fmaxf(fmaxf(fabsf(a[base + 3]), fabsf(a[base + 4])), fabsf(a[base + 5]));
    return fmaxf(fmaxf(x, y), fmaxf(fabsf(a[base + 6]), fabsf(a[base + 7])));
}

// Fit the nq queued cells (one per lane and round of 64) as flush16 does,
// over all 8 isometries of each cell.
template <int B>
__device__ __noinline__ void flush32(const SearchArgs *ta, uint32_t nq, Queue32<B> *qu,
                                     uint32_t grp)
{
    constexpr int n = Cfg<B>::n, GR = Cfg<B>::GR, RQ = kQueue / 64;
    const float slack = screen_slack<B>();
    const int lane = threadIdx.x & 63;
    const SearchArgs a = *ta;
    const auto *gsdd = as_global(a.sdd);
    const auto *geps = as_global(a.eps);
    const auto *gdom = as_global(a.dom);
    const auto *gu = as_global(a.u);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint32_t pe[RQ], le[RQ], dm[RQ];
    int64_t sd[RQ];
    int32_t ep[RQ];
    float uu[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        const uint32_t e = (uint32_t)(r * 64 + lane);
        pe[r] = 0; le[r] = 0; dm[r] = 0; sd[r] = 0; ep[r] = 0; uu[r] = 0.0f;
        if (e < nq) {
            pe[r] = qu->p[e];
            le[r] = qu->ls[e];
        }
    }
#pragma unroll
    for (int r = 0; r < RQ; ++r)
        if ((uint32_t)(r * 64 + lane) < nq) {
            sd[r] = gsdd[pe[r]];
            ep[r] = geps[pe[r]];
            dm[r] = gdom[pe[r]];
            uu[r] = gu[pe[r]];
        }
    // other waves' keys for the group, read with the column loads (as flush16)
    const u64 gk = lane < GR ? group_key(a.keys, grp, GR, lane) : kNoKey;
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        const uint32_t e = (uint32_t)(r * 64 + lane);
        // The isometries of the cell that still pass the screen against the
        // range's current threshold (never looser than when it was queued);
        // the others cannot reach the range's best key. Usually one or two
        // of the 8 pass, so the wave fits one passing isometry per lane and
        // step, in increasing order, until no lane has one left.
        uint32_t mask = 0;
        uint32_t ls = 0;
        if (e < nq) {
            ls = le[r];
            const float t = qu->T[ls];
            // the clamped and the quantised contrast
            const float g = fmaxf(clamp_threshold<B>(t, uu[r]), quant_threshold<B>(uu[r])) - slack;
            const float4_t ca = qu->c[e][0], cb = qu->c[e][1];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float c = fabsf(q < 4 ? ca[q] : cb[q - 4]);
                if (fmaf(-t, uu[r], c) >= -slack && c >= g) mask |= 1u << q;
            }
        }
        if (!wave_any(mask != 0)) continue;
        const double base = 4096.0 * (double)qu->srr[ls];
        const double ne = (double)qu->delta[ls] * (double)ep[r];
        const double dd = (double)sd[r];
        const float inv = __builtin_amdgcn_rcpf((float)dd);
        const bool any = mask != 0;
        double fb = 0.0;
        int qb = -1;
        while (wave_any(mask != 0)) {
            if (mask) {
                const int q = __builtin_ctz(mask);
                mask &= mask - 1u;
                const double rd = (double)n * (double)((const float *)&qu->c[e][0])[q] - ne;   // exact
                const double f = fit_f_d(base, rd, dd, inv);
                if (qb < 0 || f < fb) {      // ascending q: ties keep the lower isometry
                    fb = f;
                    qb = q;
                }
            }
        }
        if (any) atomicMin(&qu->best[ls], pack_key((int64_t)fb, dm[r], qb, a.shift));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < GR) {
        // take the other waves' keys read above, publish the wave's best
        u64 bk = qu->best[lane];
        bk = gk < bk ? gk : bk;
        atomicMin(&a.keys[(int64_t)grp * GR + lane], bk);
        qu->best[lane] = bk;
        qu->T[lane] = bk == kNoKey ? 0.0f : screen_t(qu->srr[lane], (int64_t)(bk >> a.shift));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Fit and empty the cell queue.
template <int B>
__device__ __forceinline__ void flush_queue32(const SearchArgs *ta, Wave32<B> &st,
                                              Queue32<B> *qu)
{
    flush32<B>(ta, st.qn, qu, st.grp);
    st.survivors += 8ull * st.qn;    // wave-uniform
    st.qn = 0;
}

template <int B>
__device__ __forceinline__ void refresh32(Wave32<B> &st, const Queue32<B> *qu)
{
    constexpr int MB = Cfg<B>::MB;
    const int h = (threadIdx.x >> 5) & 1;
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
            if (st.T[blk][hl] != __builtin_inff())      // searched ranges only
                st.T[blk][hl] = qu->T[4 * blk + 2 * h + hl];
}

// Queue the passing cells of one 32-column tile (pass: the lane's two cells
// of each row block), each as one 32-byte record of its 8 cross terms,
// fitting and emptying the queue first whenever it would overflow. Returns
// the queue's new length; fitted gains the cells fitted on the way.
template <int B>
__device__ __forceinline__ uint32_t queue_cells32(const SearchArgs *ta, uint32_t qn,
                                                  Queue32<B> *qu, uint32_t grp,
                                                  const float16_t (&acc)[Cfg<B>::MB],
                                                  const bool (&pass)[Cfg<B>::MB][2], uint32_t p,
                                                  uint32_t &fitted)
{
    constexpr int MB = Cfg<B>::MB;
    const int h = (threadIdx.x >> 5) & 1;
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) {
            const u64 ball = __ballot(pass[blk][hl]);
            if (ball == 0) continue;
            const uint32_t cnt = (uint32_t)__popcll(ball);
            if (qn + cnt > (uint32_t)kQueue) {
                flush32<B>(ta, qn, qu, grp);
                fitted += qn;
                qn = 0;
            }
            if (pass[blk][hl]) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(ball >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0u));
                const uint32_t pos = qn + below;
                const float16_t &av = acc[blk];
                qu->c[pos][0] = float4_t{av[8 * hl + 0], av[8 * hl + 1], av[8 * hl + 2], av[8 * hl + 3]};
                qu->c[pos][1] = float4_t{av[8 * hl + 4], av[8 * hl + 5], av[8 * hl + 6], av[8 * hl + 7]};
                qu->p[pos] = p;
                qu->ls[pos] = (uint32_t)(4 * blk + 2 * h + hl);
            }
            qn += cnt;
        }
    return qn;
}

// Replay and empty the column queue, 32 columns per tile: gather their B
// fragments (all tiles' loads in flight at once, staged through LDS, so
// their latency is paid once per replay), redo the MFMAs against the
// wave's A fragments (the same exact
// cross terms as in the scan) and screen every cell again, against its
// range's current threshold (never looser than when the column was queued)
// and pool window. The passing cells go to the cell queue, which is fitted
// whenever it would overflow and, at the end, once it holds flush_at cells;
// the thresholds in registers are reloaded.
template <int B>
__device__ __forceinline__ void replay_queue32(const SearchArgs *ta, Wave32<B> &st,
                                               Queue32<B> *qu)
{
    constexpr int MB = Cfg<B>::MB;
    static_assert(Cfg<B>::KS == 1, "one K step per 32 x 32 tile");
    const float slack = screen_slack<B>();
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    const half8_t *gb = (const half8_t *)uniform_ptr(ta->Bm);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint32_t ncol = st.cq, grp = st.grp;
    constexpr int kTiles = kColQ / 32;
    {
        // lane l fetches K half l/32 of its column, as in the scan's fragments
        half8_t g[kTiles];
#pragma unroll
        for (int t = 0; t < kTiles; ++t)
            if ((uint32_t)(32 * t) < ncol) {
                const uint32_t e = min((uint32_t)(32 * t + col), ncol - 1u);
                const uint32_t p = qu->colp[e];
                g[t] = gb[(int64_t)(p >> 5) * 64 + h * 32 + (p & 31)];
            }
#pragma unroll
        for (int t = 0; t < kTiles; ++t)
            if ((uint32_t)(32 * t) < ncol) qu->colb[min((uint32_t)(32 * t + col), ncol - 1u)][h] = g[t];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    uint32_t qn = st.qn, fitted = 0;
    for (uint32_t c0 = 0; c0 < ncol; c0 += 32) {
        const bool valid = c0 + (uint32_t)col < ncol;
        const uint32_t e = valid ? c0 + (uint32_t)col : c0;
        const uint32_t p = qu->colp[e];
        const float u = qu->colu[e];
        const half8_t bf = qu->colb[e][h];
        float16_t acc[MB];
#pragma unroll
        for (int blk = 0; blk < MB; ++blk) {
            float16_t z;
#pragma unroll
            for (int i = 0; i < 16; ++i) z[i] = 0.0f;
            acc[blk] = mma32(st.af[blk][0], bf, z);
        }
        // every cell's threshold and window read up front and the tests
        // combined without short-circuits (no LDS round trip per branch)
        float tr[MB][2];
        uint32_t lr[MB][2], hr[MB][2];
#pragma unroll
        for (int blk = 0; blk < MB; ++blk)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl) {
                const int r = 4 * blk + 2 * h + hl;
                tr[blk][hl] = qu->T[r];
                lr[blk][hl] = qu->lo[r];
                hr[blk][hl] = qu->hi[r];
            }
        bool pass[MB][2];
#pragma unroll
        for (int blk = 0; blk < MB; ++blk)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl) {
                const float d = fmaf(-tr[blk][hl], u, max8(acc[blk], 8 * hl));
                pass[blk][hl] = valid & (d >= -slack) & (p >= lr[blk][hl]) & (p < hr[blk][hl]);
            }
        qn = queue_cells32<B>(ta, qn, qu, grp, acc, pass, p, fitted);
    }
    if (st.flush_at && qn >= st.flush_at) {
        flush32<B>(ta, qn, qu, grp);
        fitted += qn;
        qn = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    st.qn = qn;
    st.survivors += 8ull * fitted;   // wave-uniform
    st.replayed += ncol;
    st.cq = 0;
    refresh32<B>(st, qu);
}

template <int B, bool MASK>
__device__ __forceinline__ void screen32(const SearchArgs *ta, Wave32<B> &st, Queue32<B> *qu,
                                         const float16_t (&acc)[Cfg<B>::MB], float u, int cb)
{
    constexpr int MB = Cfg<B>::MB;
    const float slack = screen_slack<B>();
    const int lane = threadIdx.x & 63;
    const uint32_t p = (uint32_t)cb * 32 + (lane & 31);
    bool hit = false;
    float dmax = -__builtin_inff();
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) {
            // max |C'''| - T u in one rounding (see the 16x16 screen)
            const float d = fmaf(-st.T[blk][hl], u, max8(acc[blk], 8 * hl));
            if (MASK) hit = hit || (d >= -slack && p >= st.lo[blk][hl] && p < st.hi[blk][hl]);
            else dmax = fmaxf(dmax, d);
        }
    if (!MASK) hit = dmax >= -slack;
    if (!MASK && MB == 4) {
        // three MFMAs, the first row block's screen, the last MFMA, the rest:
        // the screen starts on results that are done
        __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);    // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);   // VALU
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 40, 0);
    }
    const u64 ball = __ballot(hit);
    if (ball == 0) return;
    // queue the column once (lanes l and l + 32 hold the same column); the
    // scan replays the queue before it can hold more than kColQ - 32
    const uint32_t cols = (uint32_t)ball | (uint32_t)(ball >> 32);
    const uint32_t cnt = (uint32_t)__popc(cols);
    if (lane < 32 && ((cols >> (lane & 31)) & 1u)) {
        const uint32_t pos = st.cq + __builtin_amdgcn_mbcnt_lo(cols, 0u);
        qu->colp[pos] = p;
        qu->colu[pos] = u;
    }
    st.cq += cnt;
}

// Column blocks [cb_begin, cb_end): the B fragments and u of the block PD
// ahead are loaded while a block computes (a 4x4 block is cheap, so its loads
// need a deeper queue to hide the L2 latency). Whole groups of PD blocks run
// without a branch between them: a conditional step would make the compiler
// wait for the loads just issued.
template <int B, bool MASK>
__device__ __forceinline__ void scan32(const SearchArgs &a, const SearchArgs *ta, Wave32<B> &st,
                                       Queue32<B> *qu, int cb_begin, int cb_end)
{
    constexpr int MB = Cfg<B>::MB, KS = Cfg<B>::KS, PD = KS == 1 ? 4 : 2;
    cb_begin = __builtin_amdgcn_readfirstlane(cb_begin);
    cb_end = __builtin_amdgcn_readfirstlane(cb_end);
    if (cb_begin >= cb_end) return;
    const int lane = threadIdx.x & 63, col = lane & 31;
    // buffer loads: block offset in the scalar offset, 32-bit lane offset
    // (the API rejects a B operand of 2^31 bytes or more)
    static_assert(B == 4, "32-bit buffer offsets are sized for 4x4 ranges");
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(a.Bm), (short)0, -1, kBufWord3);
    const __amdgpu_buffer_rsrc_t ru =
        __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(a.u), (short)0, -1, kBufWord3);
    const uint32_t lb = (uint32_t)lane * 16u, lu = (uint32_t)col * 4u;
    constexpr uint32_t kBlkB = KS * 64 * 16, kBlkU = 32 * 4;
    const int last = cb_end - 1;
    half8_t b0[KS], b1[KS], b2[KS], b3[KS];
    float u0, u1, u2 = 0.0f, u3 = 0.0f;
    auto load = [&](half8_t (&bq)[KS], float &uq, int c) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            bq[ks] = __builtin_bit_cast(half8_t, __builtin_amdgcn_raw_buffer_load_b128(
                                                     rb, lb + (uint32_t)ks * 1024u,
                                                     (int)((uint32_t)c * kBlkB), 0));
        uq = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                           ru, lu, (int)((uint32_t)c * kBlkU), 0));
    };
    // the cross terms of one column block (MB row blocks of 32 x 32)
    auto mmab = [&](const half8_t (&bq)[KS], float16_t (&acc)[MB]) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int blk = 0; blk < MB; ++blk) {
                float16_t z;
                if (ks == 0) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) z[e] = 0.0f;
                } else {
                    z = acc[blk];
                }
                acc[blk] = mma32(st.af[blk][ks], bq[ks], z);
            }
    };
    load(b0, u0, min(cb_begin + 0, last));
    load(b1, u1, min(cb_begin + 1, last));
    if constexpr (PD == 4) {
        load(b2, u2, min(cb_begin + 2, last));
        load(b3, u3, min(cb_begin + 3, last));
    }
    int cb = cb_begin;
    // the MFMAs of a block are issued before its fragments are reloaded
    auto step = [&](half8_t (&bq)[KS], float &uq, int i) {
        float16_t acc[MB];
        mmab(bq, acc);
        const float uc = uq;
        load(bq, uq, min(cb + i + PD, last));
        screen32<B, MASK>(ta, st, qu, acc, uc, cb + i);
    };
    auto tail = [&](const half8_t (&bq)[KS], float uq, int i) {
        float16_t acc[MB];
        mmab(bq, acc);
        screen32<B, MASK>(ta, st, qu, acc, uq, cb + i);
    };
    static_assert(kColQ >= kColReplay + PD * 32, "a group of blocks fits the column queue");
    for (; cb + PD <= cb_end; cb += PD) {
        step(b0, u0, 0);
        step(b1, u1, 1);
        if constexpr (PD == 4) {
            step(b2, u2, 2);
            step(b3, u3, 3);
        }
        if (st.cq >= (uint32_t)kColReplay) replay_queue32<B>(ta, st, qu);
    }
    if (cb + 0 < cb_end) tail(b0, u0, 0);
    if constexpr (PD == 4) {
        if (cb + 1 < cb_end) tail(b1, u1, 1);
        if (cb + 2 < cb_end) tail(b2, u2, 2);
    }
    if (st.cq >= (uint32_t)kColReplay) replay_queue32<B>(ta, st, qu);
}

// One work item of the 32x32-tile search (4x4 ranges), as item16.
template <int B, class Hook = NoHook>
__device__ __forceinline__ void item32(const SearchArgs *ta, const SearchArgs &a,
                                       const WorkItem &wi, Wave32<B> &st, Queue32<B> *qu,
                                       const Hook &before_end = Hook())
{
    constexpr int MB = Cfg<B>::MB, KS = Cfg<B>::KS, GR = Cfg<B>::GR;
    const int lane = threadIdx.x & 63, h = lane >> 5;
    st.flush_at = (uint32_t)a.flush_at;
    st.grp = wi.grp;
    const half8_t *ap = (const half8_t *)a.A + (int64_t)st.grp * MB * KS * 64 + lane;
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) st.af[blk][ks] = ap[(blk * KS + ks) * 64];
    if (lane < GR) {
        // the replay and the flush screen against these thresholds and windows
        const int64_t slot = (int64_t)st.grp * GR + lane;
        const u64 bk = a.keys[slot];
        const RangeStat rsx = a.rs[slot];
        const bool act = !(rsx.flags & kIdle);
        qu->best[lane] = bk;
        qu->srr[lane] = rsx.srr;
        qu->delta[lane] = rsx.delta;
        qu->T[lane] = bk == kNoKey ? 0.0f : screen_t(rsx.srr, (int64_t)(bk >> a.shift));
        qu->lo[lane] = act ? rsx.lo : 0u;
        qu->hi[lane] = act ? rsx.hi : 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // every lane's cells from the values above (an empty window: idle)
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) {
            const int r = 4 * blk + 2 * h + hl;
            st.lo[blk][hl] = qu->lo[r];
            st.hi[blk][hl] = qu->hi[r];
            st.T[blk][hl] = st.hi[blk][hl] > st.lo[blk][hl] ? qu->T[r] : __builtin_inff();
        }
    const uint4 gb = a.grp[st.grp];
    const int cb0 = (int)(wi.c0 >> 5), cb1 = (int)(wi.c1 >> 5);
    // column blocks fully inside every active range's pool need no mask
    int ib0 = (int)((gb.z + 31u) >> 5), ib1 = (int)(gb.w >> 5);
    ib0 = min(max(ib0, cb0), cb1);
    ib1 = max(min(ib1, cb1), ib0);
    st.screened += (u64)(cb1 - cb0) * 32 * GR * 8;
    scan32<B, true>(a, ta, st, qu, cb0, ib0);
    scan32<B, false>(a, ta, st, qu, ib0, ib1);
    scan32<B, true>(a, ta, st, qu, ib1, cb1);
    before_end();
    if (st.cq) replay_queue32<B>(ta, st, qu);
    if (st.qn) flush_queue32<B>(ta, st, qu);
    if (lane < GR) {
        const u64 bk = qu->best[lane];
        if (bk != kNoKey) atomicMin(&a.keys[(int64_t)st.grp * GR + lane], bk);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int B>
__global__ __launch_bounds__(256, 2) void k_search_mfma32(const SearchArgs *__restrict__ tab,
                                                          const uint32_t *__restrict__ base,
                                                          int32_t n_img, uint32_t *item_ctr,
                                                          u64 *counters, uint32_t dbg)
{
    __shared__ Queue32<B> queues[4];
    const int lane = threadIdx.x & 63;
    Queue32<B> *qu = &queues[threadIdx.x >> 6];
    const uint32_t nitems = base[n_img];
    Wave32<B> st;
    st.survivors = 0;
    st.screened = 0;
    st.replayed = 0;
    st.qn = 0;
    st.cq = 0;
    u64 items_done = 0;
    ItemQueue iq = item_queue(tab, n_img);
    uint32_t raw = 0;
    claim_issue(item_ctr, iq, raw);
    for (;;) {
        uint32_t item;
        if (!claim_take(raw, item_ctr, tab, nitems, dbg, iq, item)) break;
        const int ia = image_of_item(base, n_img, item);
        const SearchArgs *ta = tab + ia;
        const SearchArgs a = *ta;
        claim_issue(item_ctr, iq, raw);             // the next item
        item32<B>(ta, a, a.items[item_in_image(base, ia, item)], st, qu);
        items_done += 1;
    }
    add_counters(counters, st.screened, st.survivors, items_done);
    if (counters && lane == 0) atomicAdd(&counters[7], st.replayed);
}

// 4x4 and 8x8 images of a batch in ONE persistent launch: the items of the
// 8x8 images (tab8, base8) come first in the queue, then those of the 4x4
// images (tab4, base4); a wave runs each item with that range size's code.
// Each wave's LDS queue is a union of the two sizes' queues (the waves of a
// workgroup may run items of different sizes at the same time, so the
// unions are per wave, never across waves).
__global__ __launch_bounds__(256, 2) void k_search_mixed(const SearchArgs *__restrict__ tab8,
                                                         const uint32_t *__restrict__ base8,
                                                         int32_t n8,
                                                         const SearchArgs *__restrict__ tab4,
                                                         const uint32_t *__restrict__ base4,
                                                         int32_t n4, uint32_t *item_ctr,
                                                         u64 *counters, uint32_t dbg)
{
    union WaveQueue {
        Queue16<8> q8;
        Queue32<4> q4;
    };
    __shared__ WaveQueue qm[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t ni8 = base8[n8];
    const uint32_t nitems = ni8 + base4[n4];
    // the next item is claimed while this one runs (see claim_issue)
    uint32_t raw = 0;
    if (lane == 0) raw = atomicAdd(item_ctr, 1u);
    for (;;) {
        uint32_t item = __builtin_amdgcn_readfirstlane(raw);
        if (item >= nitems) break;
        if (lane == 0) raw = atomicAdd(item_ctr, 1u);
        if (dbg & kDbgReverse) item = nitems - 1u - item;   // order-independence check
        // per item: the queue is empty between items, and the counters are
        // added per item (nothing but the loop is carried across items)
        if (item < ni8) {
            const int ia = image_of_item(base8, n8, item);
            const SearchArgs *ta = tab8 + ia;
            const SearchArgs a = *ta;
            WaveState<8> s8;
            s8.qn = 0;
            s8.screened = 0;
            s8.survivors = 0;
            item16<8>(ta, a, a.items[item_in_image(base8, ia, item)], s8, &qm[w].q8);
            add_counters(counters, s8.screened, s8.survivors, 1);
        } else {
            const uint32_t i4 = item - ni8;
            const int ia = image_of_item(base4, n4, i4);
            const SearchArgs *ta = tab4 + ia;
            const SearchArgs a = *ta;
            Wave32<4> s4;
            s4.qn = 0;
            s4.cq = 0;
            s4.screened = 0;
            s4.survivors = 0;
            s4.replayed = 0;
            item32<4>(ta, a, a.items[item_in_image(base4, ia, i4)], s4, &qm[w].q4);
            add_counters(counters, s4.screened, s4.survivors, 1);
            if (counters && lane == 0) atomicAdd(&counters[7], s4.replayed);
        }
    }
}

// The search kernel of a range size: 32x32 tiles for 4x4 ranges, 16x16
// tiles otherwise.
template <int B> const void *search_kernel()
{
    if constexpr (Cfg<B>::MR == 32)
        return reinterpret_cast<const void *>(&k_search_mfma32<B>);
    else if constexpr (B == 16)
        return reinterpret_cast<const void *>(&k_search_lds16<B, false>);
    else
        return reinterpret_cast<const void *>(&k_search_mfma<B>);
}

// ------------------------------------------------------------ plain search
__global__ void k_box2x2(const uint8_t *__restrict__ img, int32_t h, int32_t w, int32_t pitch,
                         uint16_t *__restrict__ S)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sw = w - 1;
    if (i >= (int64_t)(h - 1) * sw) return;
    const int64_t y = i / sw, x = i - y * sw;
    const uint8_t *p = img + y * pitch + x;
    S[i] = (uint16_t)(p[0] + p[1] + p[pitch] + p[pitch + 1]);
}

// One thread per (range, domain position, isometry): 32 positions x 8
// isometries per block, the range (under each inverse isometry) in LDS.
template <int B>
__global__ __launch_bounds__(256) void k_search_plain(
    const uint8_t *__restrict__ img, Geom g, const uint16_t *__restrict__ S,
    const uint32_t *__restrict__ perm, const uint32_t *__restrict__ lo,
    const uint32_t *__restrict__ hi, int64_t r0, int shift, u64 *__restrict__ keys)
{
    constexpr int n = B * B;
    __shared__ int32_t ar[8][n];
    __shared__ int32_t s_sr;
    __shared__ int64_t s_srr;
    const int64_t r = r0 + blockIdx.y;
    const int tid = threadIdx.x;
    const int ry = (int)(r / g.rcols) * B, rx = (int)(r % g.rcols) * B;
    for (int e = tid; e < 8 * n; e += 256) {
        const int q = e / n, K = e % n;
        int si, sj;
        iso_src(iso_inverse(q), B, K / B, K % B, si, sj);
        ar[q][K] = img[(int64_t)(ry + si) * g.pitch + rx + sj];
    }
    if (tid == 0) {
        int32_t sr = 0;
        int64_t sq = 0;
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) {
                int v = img[(int64_t)(ry + i) * g.pitch + rx + j];
                sr += v;
                sq += v * v;
            }
        s_sr = sr;
        s_srr = (int64_t)n * sq - (int64_t)sr * sr;
    }
    __syncthreads();
    const uint32_t plo = lo ? lo[r] : 0u, phi = hi ? hi[r] : (uint32_t)g.D;
    const uint32_t pos = blockIdx.x * 32u + (uint32_t)(tid >> 3);
    const int q = tid & 7;
    u64 key = kNoKey;
    if (pos >= plo && pos < phi) {
        const uint32_t d = perm ? perm[pos] : pos;
        const int dy = (int)(d / g.dcols) * g.t, dx = (int)(d % g.dcols) * g.t;
        const int64_t sw = g.w - 1;
        const uint16_t *sp = S + (int64_t)dy * sw + dx;
        int64_t cx = 0, sd = 0, sq = 0;
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) {
                const int dv = sp[(int64_t)(2 * i) * sw + 2 * j];
                cx += ar[q][i * B + j] * dv;
                sd += dv;
                sq += dv * dv;
            }
        const int64_t srd = n * cx - (int64_t)s_sr * sd;
        int k;
        const int64_t f = fit_f(s_srr, srd, n * sq - sd * sd, k);
        key = pack_key(f, d, q, shift);
    }
    for (int off = 32; off > 0; off >>= 1) {
        const u64 o = __shfl_xor(key, off);
        key = o < key ? o : key;
    }
    if ((tid & 63) == 0 && key != kNoKey) atomicMin(&keys[r], key);
}

// ------------------------------------------------------------ finalize
// B lanes per range, lane i summing row i, so a range's pixel reads are
// spread over B lanes (one lane per range left the launch latency-bound).
template <int B>
__global__ __launch_bounds__(256) void k_finalize(const uint8_t *__restrict__ img, Geom g,
                                                  const uint32_t *__restrict__ order,
                                                  const u64 *__restrict__ keys,
                                                  const uint8_t *__restrict__ sel, int shift,
                                                  fic_code *__restrict__ codes)
{
    constexpr int n = B * B;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = t / B;
    const int i = (int)(t % B);
    // a segment of B lanes is one range; segments past the ranges take part
    // in the shuffles and write nothing
    const bool live = s < g.R;
    const uint32_t ridx = live ? (order ? order[s] : (uint32_t)s) : 0u;
    const bool coded = live && !(sel && !sel[ridx]);
    const int ry = (int)(ridx / g.rcols) * B, rx = (int)(ridx % g.rcols) * B;
    int64_t sr = 0, sq = 0;
    if (coded)
        for (int j = 0; j < B; ++j) {
            const int v = img[(int64_t)(ry + i) * g.pitch + rx + j];
            sr += v;
            sq += v * v;
        }
    sr = segment_sum<B>(sr);
    sq = segment_sum<B>(sq);
    const u64 key = coded ? keys[s] : kNoKey;
    const uint32_t d = (uint32_t)((key >> 3) & ((1ull << (shift - 3)) - 1ull));
    const int q = (int)(key & 7ull);
    int64_t cx = 0, sd = 0, sdd = 0;
    if (key != kNoKey) {
        const int dy = (int)(d / g.dcols) * g.t, dx = (int)(d % g.dcols) * g.t;
        pair_row_sums<B>(img, g.pitch, ry, rx, dy, dx, q, i, cx, sd, sdd);
    }
    cx = segment_sum<B>(cx);
    sd = segment_sum<B>(sd);
    sdd = segment_sum<B>(sdd);
    if (!live || i != 0) return;
    fic_code c;
    if (!coded) {                        // not coded: flag bit 2, everything else 0
        c.domain = 0; c.iso = 0; c.s_idx = 0; c.o_idx = 0; c.flags = 4; c.err = 0;
        codes[ridx] = c;
        return;
    }
    const int64_t srr = (int64_t)n * sq - sr * sr;
    const int32_t j = (int32_t)((sr + n - 1) / (2 * n));
    const int64_t e = sr - 2 * (int64_t)n * j;
    const int64_t jcost = 4096 * e * e;
    c.o_idx = (uint8_t)j;
    if (key == kNoKey) {
        c.domain = 0;
        c.iso = 0;
        c.s_idx = 0;
        c.flags = 1;
        c.err = 4096 * srr + jcost;
    } else {
        int k;
        const int64_t srd = (int64_t)n * cx - sr * sd;
        const int64_t f = fit_f(srr, srd, (int64_t)n * sdd - sd * sd, k);
        c.domain = d;
        c.iso = (uint8_t)q;
        c.s_idx = (int8_t)k;
        c.flags = (f == (int64_t)(key >> shift)) ? 0 : 0x80;   // 0x80: key / recompute mismatch
        c.err = f + jcost;
    }
    codes[ridx] = c;
}

inline unsigned blocks_for(int64_t n, int th) { return (unsigned)((n + th - 1) / th); }

// Two-level partition: a level-1 range whose E exceeds emax is split -- its
// code gets flag bit 1 and its four quadrants (the level-2 ranges holding its
// pixels) are selected for level 2; every level-2 range is written.
__global__ void k_split(fic_code *__restrict__ codes1, int64_t R1, int32_t rcols1,
                        int32_t rcols2, int64_t emax, uint8_t *__restrict__ sel2)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R1) return;
    const bool split = codes1[r].err > emax;
    if (split) codes1[r].flags |= 2;
    const int64_t ry = r / rcols1, rx = r % rcols1;
    const uint8_t v = split ? 1 : 0;
    sel2[(2 * ry) * rcols2 + 2 * rx] = v;
    sel2[(2 * ry) * rcols2 + 2 * rx + 1] = v;
    sel2[(2 * ry + 1) * rcols2 + 2 * rx] = v;
    sel2[(2 * ry + 1) * rcols2 + 2 * rx + 1] = v;
}

// Plain search: 2x2 sums, then one thread per (range, position, isometry).
template <int B>
hipError_t run_plain_b(const EncodePlan &p, const uint8_t *img, const uint32_t *perm,
                       const uint32_t *lo, const uint32_t *hi, fic_code *codes, void *ws,
                       hipStream_t s, const Tracer *tr)
{
    const Geom &g = p.g;
    char *w = (char *)ws;
    u64 *keys = (u64 *)(w + p.off_keys);
    const int th = 256;
    uint16_t *S = (uint16_t *)(w + p.off_S);
    trace(tr, FIC_STAGE_DOMAIN_PREP, 1, s);
    hipLaunchKernelGGL(k_box2x2, dim3(blocks_for((int64_t)(g.h - 1) * (g.w - 1), th)), dim3(th), 0,
                       s, img, g.h, g.w, g.pitch, S);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(g.R, th)), dim3(th), 0, s, keys, g.R, kNoKey);
    trace(tr, FIC_STAGE_DOMAIN_PREP, 0, s);
    trace(tr, FIC_STAGE_SEARCH, 1, s);
    const unsigned gx = blocks_for(p.Dp, 32);
    for (int64_t r0 = 0; r0 < g.R; r0 += 65535) {
        const unsigned gy = (unsigned)(g.R - r0 < 65535 ? g.R - r0 : 65535);
        hipLaunchKernelGGL(k_search_plain<B>, dim3(gx, gy), dim3(256), 0, s, img, g, S, perm, lo, hi,
                           r0, p.shift, keys);
    }
    trace(tr, FIC_STAGE_SEARCH, 0, s);
    trace(tr, FIC_STAGE_FINAL, 1, s);
    hipLaunchKernelGGL(k_finalize<B>, dim3(blocks_for(g.R * B, th)), dim3(th), 0, s, img, g,
                       (const uint32_t *)nullptr, keys, p.sel, p.shift, codes);
    trace(tr, FIC_STAGE_FINAL, 0, s);
    return hipGetLastError();
}

// Everything before the MFMA search for one image: range order and A rows,
// B columns, seeds, the work list; the last kernel publishes the image's
// table entry to *slot.
template <int B>
hipError_t prep_b(const EncodePlan &p, const uint8_t *img, const uint32_t *perm,
                  const uint32_t *lo, const uint32_t *hi, void *ws, u64 *counters,
                  SearchArgs *slot, hipStream_t s, const Tracer *tr, int allow_xcd)
{
    const Geom &g = p.g;
    char *w = (char *)ws;
    const int th = 256;
    u64 *keys = (u64 *)(w + p.off_keys);
    _Float16 *A = (_Float16 *)(w + p.off_A);
    RangeStat *rs = (RangeStat *)(w + p.off_rs);
    uint32_t *order = (uint32_t *)(w + p.off_order);
    _Float16 *Bm = (_Float16 *)(w + p.off_B);
    float *u = (float *)(w + p.off_u);
    int32_t *eps = (int32_t *)(w + p.off_eps);
    int64_t *sdd = (int64_t *)(w + p.off_sdd);
    uint32_t *dom = (uint32_t *)(w + p.off_dom);
    WorkItem *items = (WorkItem *)(w + p.off_items);
    uint32_t *ctr = (uint32_t *)(w + p.off_ctr);
    uint32_t *chunkcnt = (uint32_t *)(w + p.off_chunkcnt);
    uint32_t *chunkfill = (uint32_t *)(w + p.off_chunkfill);
    uint4 *grp = (uint4 *)(w + p.off_grp);
    uint32_t *bmin = (uint32_t *)(w + p.off_bmin);

    trace(tr, FIC_STAGE_RANGE_PREP, 1, s);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, ctr, (int64_t)64, 0u);
    {
        int dbits = 1;
        while (((int64_t)1 << dbits) <= g.D) ++dbits;
        u64 *sk = (u64 *)(w + p.off_sortkeys);
        hipLaunchKernelGGL(k_range_keys<B>, dim3(blocks_for(g.R, th)), dim3(th), 0, s, img, g.pitch,
                           g.rcols, g.R, lo, hi, p.sel, (uint32_t)g.D, dbits, sk, order);
        hipError_t e = radix_sort_pairs(sk, order, g.R, p.pooled ? 2 * dbits : 8, w + p.off_sort, s);
        if (e != hipSuccess) return e;
    }
    if (p.pooled)
        hipLaunchKernelGGL(k_blockmin, dim3(blocks_for((g.D + kBminBlock - 1) / kBminBlock * 64, th)),
                           dim3(th), 0, s, perm, g.D, bmin);
    hipLaunchKernelGGL(k_range_prep<B>, dim3(blocks_for(p.Rp * 8, th)), dim3(th), 0, s, img, g.pitch,
                       g.rcols, g.R, p.Rp, (const uint32_t *)order, lo, hi, p.sel, (uint32_t)g.D, A,
                       rs);
    trace(tr, FIC_STAGE_RANGE_PREP, 0, s);
    trace(tr, FIC_STAGE_DOMAIN_PREP, 1, s);
    const int64_t img_bytes = (int64_t)(g.h - 1) * g.pitch + g.w;
    hipLaunchKernelGGL(k_domain_prep<B>, dim3(blocks_for(p.Dp * B, th)), dim3(th), 0, s, img,
                       img_bytes, g.pitch, g.dcols, g.t, perm, g.D, p.Dp, Bm, u, eps, sdd, dom);
    trace(tr, FIC_STAGE_DOMAIN_PREP, 0, s);
    trace(tr, FIC_STAGE_WORKLIST, 1, s);
    hipLaunchKernelGGL(k_seed<B>, dim3(blocks_for(p.Rp * 64, th)), dim3(th), 0, s, A, Bm, rs, eps,
                       sdd, dom, p.Rp, perm, bmin, p.shift, keys, counters);
    u64 *pool_sum = (u64 *)(ctr + 8);     // zeroed with the counters above
    hipLaunchKernelGGL(k_group_bounds, dim3(blocks_for(p.IG * 64, th)), dim3(th), 0, s, rs, p.IG,
                       (int)(p.GR * p.IGW), (uint32_t)p.Dp, (uint32_t)Cfg<B>::MR, grp, pool_sum);
    hipLaunchKernelGGL(k_chunk_span, dim3(blocks_for(p.NC, th)), dim3(th), 0, s, grp, p.IG, p.NC,
                       p.tune, p.chunk_min, p.pooled, (const u64 *)pool_sum, g.R, g.D, allow_xcd,
                       chunkcnt, chunkfill);
    // exclusive scan of the per-chunk counts; the total is the item count
    const hipError_t se = scan_u32(chunkcnt, p.NC, ctr + 1, w + p.off_scan, s);
    if (se != hipSuccess) return se;
    SearchArgs a;
    a.A = A; a.Bm = Bm; a.u = u; a.eps = eps; a.sdd = sdd; a.dom = dom; a.rs = rs; a.grp = grp;
    a.items = items; a.n_items = ctr + 1; a.keys = keys; a.shift = p.shift; a.flush_at = 0;
    a.xcd = 0; a.ncx = 0; a.xq = nullptr;
    hipLaunchKernelGGL(k_emit_items, dim3(blocks_for(p.max_items, th)), dim3(th), 0, s, grp,
                       chunkcnt, chunkfill, p.NC, p.tune, p.chunk_min, p.pooled,
                       (const u64 *)pool_sum, g.R, g.D, allow_xcd, ctr + 1, p.max_items, items, a,
                       slot);
    trace(tr, FIC_STAGE_WORKLIST, 0, s);
    return hipGetLastError();
}

// Resident workgroups per CU of k_search_mfma<4, 8, 16> and k_search_mixed,
// queried once per process (outside any stream capture).
int g_per_cu[4] = {0, 0, 0, 0};

template <int B> hipError_t occupancy_of(int &out)
{
    int v = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, search_kernel<B>(), 256, 0);
    out = v < 1 ? 1 : v;
    return e;
}

// The persistent search over the items of n table entries (all range size
// B). item_ctr must read 0; base holds n + 1 entries.
template <int B>
hipError_t search_b(const SearchArgs *tab, int32_t n, uint32_t *base, uint32_t *item_ctr,
                    int num_cu, u64 *counters, uint32_t dbg, hipStream_t s, const Tracer *tr)
{
    // persistent grid: as many workgroups as stay resident on every CU
    const int per_cu = g_per_cu[B == 4 ? 0 : B == 8 ? 1 : 2];
    if (per_cu < 1) return hipErrorNotInitialized;
    hipLaunchKernelGGL(k_item_bases, dim3(1), dim3(256), 0, s, tab, n, base);
    trace(tr, FIC_STAGE_SEARCH, 1, s);
    if constexpr (Cfg<B>::MR == 32)
        hipLaunchKernelGGL(k_search_mfma32<B>, dim3(per_cu * num_cu), dim3(256), 0, s, tab,
                           (const uint32_t *)base, n, item_ctr, counters, dbg);
    else if constexpr (B == 16) {
        if (dbg & kDbgVerify16)
            hipLaunchKernelGGL((k_search_lds16<B, true>), dim3(per_cu * num_cu), dim3(256), 0, s,
                               tab, (const uint32_t *)base, n, item_ctr, counters, dbg);
        else
            hipLaunchKernelGGL((k_search_lds16<B, false>), dim3(per_cu * num_cu), dim3(256), 0, s,
                               tab, (const uint32_t *)base, n, item_ctr, counters, dbg);
    } else
        hipLaunchKernelGGL(k_search_mfma<B>, dim3(per_cu * num_cu), dim3(256), 0, s, tab,
                           (const uint32_t *)base, n, item_ctr, counters, dbg);
    trace(tr, FIC_STAGE_SEARCH, 0, s);
    return hipGetLastError();
}

template <int B>
hipError_t finalize_b(const EncodePlan &p, const uint8_t *img, void *ws, fic_code *codes,
                      hipStream_t s, const Tracer *tr)
{
    char *w = (char *)ws;
    trace(tr, FIC_STAGE_FINAL, 1, s);
    hipLaunchKernelGGL(k_finalize<B>, dim3(blocks_for(p.g.R * B, 256)), dim3(256), 0, s, img, p.g,
                       (const uint32_t *)(w + p.off_order), (const u64 *)(w + p.off_keys), p.sel,
                       p.shift, codes);
    trace(tr, FIC_STAGE_FINAL, 0, s);
    return hipGetLastError();
}

template <int B>
hipError_t run_encode_b(const EncodePlan &p, const uint8_t *img, const uint32_t *perm,
                        const uint32_t *lo, const uint32_t *hi, int kernel, fic_code *codes,
                        void *ws, int num_cu, u64 *counters, hipStream_t s, const Tracer *tr)
{
    if (kernel == FIC_KERNEL_PLAIN) return run_plain_b<B>(p, img, perm, lo, hi, codes, ws, s, tr);
    char *w = (char *)ws;
    uint32_t *ctr = (uint32_t *)(w + p.off_ctr);   // [0] item counter, [1] items, [2..3] bases
    SearchArgs *slot = (SearchArgs *)(w + p.off_args);
    hipError_t e = prep_b<B>(p, img, perm, lo, hi, ws, counters, slot, s, tr, 1);
    if (e == hipSuccess) e = search_b<B>(slot, 1, ctr + 2, ctr, num_cu, counters, p.dbg, s, tr);
    if (e == hipSuccess) e = finalize_b<B>(p, img, ws, codes, s, tr);
    return e;
}

template <int B>
hipError_t batch_phase(int phase, const EncodePlan &p, const uint8_t *img, const uint32_t *perm,
                       const uint32_t *lo, const uint32_t *hi, void *ws, u64 *counters,
                       SearchArgs *slot, fic_code *codes, hipStream_t s, const Tracer *tr,
                       int single = 0)
{
    // batches of several images share one queue: chunk-major work lists; a
    // batch of one image searches as a single-image encode does (its tuning
    // row may choose the per-XCD queues)
    return phase == 0 ? prep_b<B>(p, img, perm, lo, hi, ws, counters, slot, s, tr, single)
                      : finalize_b<B>(p, img, ws, codes, s, tr);
}

}  // namespace

hipError_t init_search_occupancy()
{
    hipError_t e = occupancy_of<4>(g_per_cu[0]);
    if (e == hipSuccess) e = occupancy_of<8>(g_per_cu[1]);
    if (e == hipSuccess) e = occupancy_of<16>(g_per_cu[2]);
    if (e == hipSuccess) {
        int v = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &v, reinterpret_cast<const void *>(&k_search_mixed), 256, 0);
        g_per_cu[3] = v < 1 ? 1 : v;
    }
    return e;
}

void plan_encode(const Geom &g, int pooled, EncodePlan &p)
{
    p.g = g;
    p.pooled = pooled;
    p.GR = g.b == 16 ? Cfg<16>::GR : g.b == 8 ? Cfg<8>::GR : Cfg<4>::GR;
    const int mr = g.b == 16 ? Cfg<16>::MR : g.b == 8 ? Cfg<8>::MR : Cfg<4>::MR;
    // 16x16 ranges: a workgroup's 4 waves search 4 consecutive groups over
    // the same columns, sharing the B fragments through LDS
    p.IGW = g.b == 16 ? 4 : 1;
    p.Rp = (g.R + p.GR * p.IGW - 1) / (p.GR * p.IGW) * (p.GR * p.IGW);
    p.G = p.Rp / p.GR;
    p.IG = p.G / p.IGW;
    p.Dp = (g.D + mr - 1) / mr * mr;
    // chunk slots at the narrowest item width, widened until the work list's
    // worst case (every group against every chunk) stays within kMaxItems
    auto slots = [&](int cl) {
        const int64_t nc = (p.Dp + ((int64_t)1 << cl) - 1) >> cl;
        return (nc + kXcds - 1) / kXcds * kXcds;
    };
    p.chunk_min = kChunkLog2Min;
    while (p.chunk_min < kChunkLog2Max && p.IG * slots(p.chunk_min) > kMaxItems) ++p.chunk_min;
    p.NC = slots(p.chunk_min);
    p.max_items = p.IG * p.NC;
    int dbits = 1;
    while (((int64_t)1 << dbits) < g.D) ++dbits;
    p.shift = dbits + 3;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    p.off_A = take((size_t)p.Rp * 8 * g.n * 2);
    p.off_rs = take((size_t)p.Rp * sizeof(RangeStat));
    p.off_order = take((size_t)p.Rp * 4);
    p.off_B = take((size_t)p.Dp * g.n * 2);
    p.off_u = take((size_t)p.Dp * 4);
    p.off_eps = take((size_t)p.Dp * 4);
    p.off_sdd = take((size_t)p.Dp * 8);
    p.off_dom = take((size_t)p.Dp * 4);
    p.off_keys = take((size_t)p.Rp * 8);
    p.off_items = take((size_t)p.max_items * sizeof(WorkItem));
    p.off_ctr = take(256);
    p.off_args = take(sizeof(SearchArgs));
    p.off_chunkcnt = take((size_t)p.NC * 4);
    p.off_chunkfill = take((size_t)p.NC * 4);
    p.off_grp = take((size_t)p.IG * 16);
    p.off_bmin = take((size_t)((g.D + kBminBlock - 1) / kBminBlock) * 4);
    p.off_S = take((size_t)(g.h - 1) * (g.w - 1) * 2);
    p.off_sortkeys = take((size_t)p.Rp * 8);
    p.off_sort = take(sort_ws_bytes(p.Rp));
    p.off_scan = take(scan_ws_bytes(p.NC));
    p.total = o;
    p.sel = nullptr;
    p.tune = default_tune_row(g.b);
    p.dbg = 0;
}

hipError_t run_encode(const EncodePlan &p, const uint8_t *img, const uint32_t *perm,
                      const uint32_t *lo, const uint32_t *hi, int kernel, fic_code *codes,
                      void *ws, int num_cu, u64 *counters, hipStream_t s, const Tracer *tr)
{
    switch (p.g.b) {
    case 4: return run_encode_b<4>(p, img, perm, lo, hi, kernel, codes, ws, num_cu, counters, s, tr);
    case 8: return run_encode_b<8>(p, img, perm, lo, hi, kernel, codes, ws, num_cu, counters, s, tr);
    case 16: return run_encode_b<16>(p, img, perm, lo, hi, kernel, codes, ws, num_cu, counters, s, tr);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ batch
// Workspace of a batch: a header (the table of search operands, grouped by
// range size; per size the item bases and the item counter), then one part
// per image (fd of ranges and domains, pool, encode workspace). Within a
// size group the images are ordered by decreasing R * D, so the largest
// images' items enter the queue first and small images fill the tail.
namespace {
constexpr int kSizes[3] = {4, 8, 16};
int size_group(int b) { return b == 4 ? 0 : b == 8 ? 1 : 2; }
}

void plan_batch(const BatchJob *jobs, int32_t n, BatchPlan &bp)
{
    bp.n = n;
    bp.dbg = 0;
    bp.slot.assign(n, 0);
    bp.part.assign(n, BatchPart{});
    std::vector<int32_t> idx(n);
    for (int32_t i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
        const int gx = size_group(jobs[x].g.b), gy = size_group(jobs[y].g.b);
        if (gx != gy) return gx < gy;
        return jobs[x].g.R * jobs[x].g.D > jobs[y].g.R * jobs[y].g.D;
    });
    bp.order = idx;
    for (int k = 0; k < 3; ++k) { bp.group_first[k] = 0; bp.group_count[k] = 0; }
    for (int32_t k = 0; k < n; ++k) {
        const int gi = size_group(jobs[idx[k]].g.b);
        if (bp.group_count[gi] == 0) bp.group_first[gi] = k;
        bp.group_count[gi] += 1;
        bp.slot[idx[k]] = k;
    }
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    bp.off_tab = take((size_t)n * sizeof(SearchArgs));
    bp.off_base = take((size_t)3 * (n + 1) * 4);
    bp.off_ctr = take(3 * 256);
    bp.items = 0;
    for (int32_t i = 0; i < n; ++i) {
        const BatchJob &j = jobs[i];
        BatchPart &pt = bp.part[i];
        pt.off_fdr = take((size_t)j.g.R * 8);
        pt.off_fdd = take((size_t)j.g.D * 8);
        pt.off_perm = take((size_t)j.g.D * 4);
        pt.off_lo = take((size_t)j.g.R * 4);
        pt.off_hi = take((size_t)j.g.R * 4);
        pt.off_pool = take(j.pooled ? pool_ws_bytes(j.g.R, j.g.D) : 0);
        plan_encode(j.g, j.pooled ? 1 : 0, pt.plan);
        pt.off_enc = take(pt.plan.total);
        bp.items += pt.plan.max_items;
    }
    bp.total = o;
}

hipError_t run_encode_batch(const BatchJob *jobs, const BatchPlan &bp, void *ws, int num_cu,
                            u64 *counters, hipStream_t s, const Tracer *tr, const BatchStreams *bs)
{
    char *w = (char *)ws;
    SearchArgs *tab = (SearchArgs *)(w + bp.off_tab);
    uint32_t *base = (uint32_t *)(w + bp.off_base);
    uint32_t *ctr = (uint32_t *)(w + bp.off_ctr);
    hipLaunchKernelGGL(k_fill_u32, dim3(3), dim3(64), 0, s, ctr, (int64_t)(3 * 64), 0u);
    hipError_t e = hipGetLastError();
    // The images' preparations (and, after the search, their finalizations)
    // are independent chains of small launches: spread them over the side
    // streams, each image (largest first, by ranges + domains) onto the
    // least loaded one, so that the streams end together.
    const int ns = bs ? bs->ns : 0;
    std::vector<int> lane_of(bp.n, 0);
    if (ns > 1) {
        std::vector<int32_t> by(bp.n);
        for (int32_t k = 0; k < bp.n; ++k) by[k] = k;
        auto cost = [&](int32_t k) { return jobs[bp.order[k]].g.R + jobs[bp.order[k]].g.D; };
        std::stable_sort(by.begin(), by.end(), [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
        std::vector<int64_t> load(ns, 0);
        for (const int32_t k : by) {
            const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            lane_of[k] = q;
            load[q] += cost(k);
        }
    }
    auto fork = [&]() {
        hipError_t r = hipEventRecord(bs->fork, s);
        for (int q = 0; q < ns && r == hipSuccess; ++q) r = hipStreamWaitEvent(bs->side[q], bs->fork, 0);
        return r;
    };
    auto join = [&]() {
        hipError_t r = hipSuccess;
        for (int q = 0; q < ns && r == hipSuccess; ++q) r = hipEventRecord(bs->join[q], bs->side[q]);
        for (int q = 0; q < ns && r == hipSuccess; ++q) r = hipStreamWaitEvent(s, bs->join[q], 0);
        return r;
    };
    if (ns > 0 && e == hipSuccess) e = fork();
    // classify, pool and search preparation, image by image
    for (int32_t k = 0; k < bp.n && e == hipSuccess; ++k) {
        const int32_t i = bp.order[k];
        const BatchJob &j = jobs[i];
        const hipStream_t ps = ns > 0 ? bs->side[lane_of[k]] : s;
        const BatchPart &pt = bp.part[i];
        const Geom &g = j.g;
        double *fdr = (double *)(w + pt.off_fdr);
        double *fdd = (double *)(w + pt.off_fdd);
        uint32_t *perm = (uint32_t *)(w + pt.off_perm);
        uint32_t *lo = (uint32_t *)(w + pt.off_lo);
        uint32_t *hi = (uint32_t *)(w + pt.off_hi);
        if (j.pooled) {
            e = launch_fd_classify(j.img, g.h, g.w, g.pitch, g.b, g.b, fdr, nullptr, ps, tr);
            if (e == hipSuccess)
                e = launch_fd_classify(j.img, g.h, g.w, g.pitch, 2 * g.b, g.t, fdd, nullptr, ps, tr);
            if (e == hipSuccess)
                e = launch_pool(fdr, (int32_t)g.R, fdd, (int32_t)g.D, j.tol, perm, lo, hi,
                                w + pt.off_pool, ps, tr);
        }
        if (e != hipSuccess) break;
        const uint32_t *pp = j.pooled ? perm : nullptr;
        const uint32_t *pl = j.pooled ? lo : nullptr;
        const uint32_t *ph = j.pooled ? hi : nullptr;
        void *ew = w + pt.off_enc;
        switch (g.b) {
        case 4: e = batch_phase<4>(0, pt.plan, j.img, pp, pl, ph, ew, counters, tab + k, nullptr, ps, tr, bp.n == 1); break;
        case 8: e = batch_phase<8>(0, pt.plan, j.img, pp, pl, ph, ew, counters, tab + k, nullptr, ps, tr, bp.n == 1); break;
        default: e = batch_phase<16>(0, pt.plan, j.img, pp, pl, ph, ew, counters, tab + k, nullptr, ps, tr, bp.n == 1); break;
        }
    }
    if (ns > 0 && e == hipSuccess) e = join();
    // 4x4 and 8x8 images together: one persistent search over all their items
    const bool mixed = bp.group_count[0] > 0 && bp.group_count[1] > 0 && !(bp.dbg & kDbgSeparate);
    if (mixed && e == hipSuccess) {
        if (g_per_cu[3] < 1) return hipErrorNotInitialized;
        const SearchArgs *t4 = tab + bp.group_first[0], *t8 = tab + bp.group_first[1];
        uint32_t *b4 = base, *b8 = base + (bp.n + 1);
        hipLaunchKernelGGL(k_item_bases, dim3(1), dim3(256), 0, s, t4, bp.group_count[0], b4);
        hipLaunchKernelGGL(k_item_bases, dim3(1), dim3(256), 0, s, t8, bp.group_count[1], b8);
        trace(tr, FIC_STAGE_SEARCH, 1, s);
        hipLaunchKernelGGL(k_search_mixed, dim3(g_per_cu[3] * num_cu), dim3(256), 0, s, t8,
                           (const uint32_t *)b8, bp.group_count[1], t4, (const uint32_t *)b4,
                           bp.group_count[0], ctr, counters, bp.dbg);
        trace(tr, FIC_STAGE_SEARCH, 0, s);
        e = hipGetLastError();
    }
    // otherwise one persistent search per range size over all its images
    // (the tuned launch choice, or a single range size)
    for (int gi = 0; gi < 3 && e == hipSuccess; ++gi) {
        if (bp.group_count[gi] == 0 || (mixed && gi < 2)) continue;
        const SearchArgs *t = tab + bp.group_first[gi];
        uint32_t *gb = base + (size_t)gi * (bp.n + 1);
        uint32_t *gc = ctr + gi * 64;
        switch (kSizes[gi]) {
        case 4: e = search_b<4>(t, bp.group_count[gi], gb, gc, num_cu, counters, bp.dbg, s, tr); break;
        case 8: e = search_b<8>(t, bp.group_count[gi], gb, gc, num_cu, counters, bp.dbg, s, tr); break;
        default: e = search_b<16>(t, bp.group_count[gi], gb, gc, num_cu, counters, bp.dbg, s, tr); break;
        }
    }
    // finalize, image by image, over the side streams again
    if (ns > 0 && e == hipSuccess) e = fork();
    for (int32_t k = 0; k < bp.n && e == hipSuccess; ++k) {
        const int32_t i = bp.order[k];
        const BatchJob &j = jobs[i];
        const BatchPart &pt = bp.part[i];
        const hipStream_t ps = ns > 0 ? bs->side[lane_of[k]] : s;
        void *ew = w + pt.off_enc;
        switch (j.g.b) {
        case 4: e = batch_phase<4>(1, pt.plan, j.img, nullptr, nullptr, nullptr, ew, counters, nullptr, j.codes, ps, tr); break;
        case 8: e = batch_phase<8>(1, pt.plan, j.img, nullptr, nullptr, nullptr, ew, counters, nullptr, j.codes, ps, tr); break;
        default: e = batch_phase<16>(1, pt.plan, j.img, nullptr, nullptr, nullptr, ew, counters, nullptr, j.codes, ps, tr); break;
        }
    }
    if (ns > 0 && e == hipSuccess) e = join();
    return e;
}

// ------------------------------------------------------------ quadtree
// Workspace: per level the FD, pool and encode parts of a batch image, then
// the level-2 selection.
void plan_quadtree(const Geom &g1, double tol1, const Geom &g2, double tol2, QuadPlan &qp)
{
    BatchJob j[2];
    j[0].img = nullptr; j[0].g = g1; j[0].tol = tol1; j[0].codes = nullptr;
    j[1].img = nullptr; j[1].g = g2; j[1].tol = tol2; j[1].codes = nullptr;
    for (int l = 0; l < 2; ++l) j[l].pooled = std::isfinite(j[l].tol) || j[l].tol < 0;
    BatchPlan bp;
    plan_batch(j, 2, bp);
    size_t o = bp.total;
    qp.lv[0] = j[0];
    qp.lv[1] = j[1];
    qp.part[0] = bp.part[0];
    qp.part[1] = bp.part[1];
    qp.off_sel = o;
    o += align256((size_t)g2.R);
    qp.total = o;
}

namespace {
template <int B>
hipError_t encode_level(const BatchJob &j, const BatchPart &pt, const uint8_t *img, char *w,
                        const uint8_t *sel, fic_code *codes, int num_cu, u64 *counters,
                        hipStream_t s, const Tracer *tr)
{
    const Geom &g = j.g;
    double *fdr = (double *)(w + pt.off_fdr);
    double *fdd = (double *)(w + pt.off_fdd);
    uint32_t *perm = (uint32_t *)(w + pt.off_perm);
    uint32_t *lo = (uint32_t *)(w + pt.off_lo);
    uint32_t *hi = (uint32_t *)(w + pt.off_hi);
    hipError_t e = hipSuccess;
    if (j.pooled) {
        e = launch_fd_classify(img, g.h, g.w, g.pitch, g.b, g.b, fdr, nullptr, s, tr);
        if (e == hipSuccess)
            e = launch_fd_classify(img, g.h, g.w, g.pitch, 2 * g.b, g.t, fdd, nullptr, s, tr);
        if (e == hipSuccess)
            e = launch_pool(fdr, (int32_t)g.R, fdd, (int32_t)g.D, j.tol, perm, lo, hi,
                            w + pt.off_pool, s, tr);
        if (e != hipSuccess) return e;
    }
    EncodePlan p = pt.plan;
    p.sel = sel;
    return run_encode_b<B>(p, img, j.pooled ? perm : nullptr, j.pooled ? lo : nullptr,
                           j.pooled ? hi : nullptr, FIC_KERNEL_MFMA, codes, w + pt.off_enc, num_cu,
                           counters, s, tr);
}
}  // namespace

hipError_t run_quadtree(const QuadPlan &qp, const uint8_t *img, int64_t emax, fic_code *codes1,
                        fic_code *codes2, void *ws, int num_cu, u64 *counters, hipStream_t s,
                        const Tracer *tr)
{
    char *w = (char *)ws;
    uint8_t *sel2 = (uint8_t *)(w + qp.off_sel);
    const Geom &g1 = qp.lv[0].g, &g2 = qp.lv[1].g;
    hipError_t e;
    switch (g1.b) {
    case 8: e = encode_level<8>(qp.lv[0], qp.part[0], img, w, nullptr, codes1, num_cu, counters, s, tr); break;
    case 16: e = encode_level<16>(qp.lv[0], qp.part[0], img, w, nullptr, codes1, num_cu, counters, s, tr); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split, dim3(blocks_for(g1.R, 256)), dim3(256), 0, s, codes1, g1.R,
                       g1.rcols, g2.rcols, emax, sel2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (g2.b) {
    case 4: return encode_level<4>(qp.lv[1], qp.part[1], img, w, sel2, codes2, num_cu, counters, s, tr);
    case 8: return encode_level<8>(qp.lv[1], qp.part[1], img, w, sel2, codes2, num_cu, counters, s, tr);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ colour
namespace {
// One thread per pixel: the three planes of an interleaved RGB image and the
// image the dimensions come from (0: luma (299 R + 587 G + 114 B + 500) div
// 1000, 1: mean (R + G + B + 1) div 3).
__global__ void k_color_planes(const uint8_t *__restrict__ rgb, int32_t h, int32_t w,
                               int32_t pitch, int32_t mode, uint8_t *__restrict__ planes)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (int64_t)h * w;
    if (i >= np) return;
    const int64_t y = i / w, x = i - y * w;
    const uint8_t *p = rgb + y * pitch + 3 * x;
    const int r = p[0], g = p[1], b = p[2];
    planes[i] = (uint8_t)r;
    planes[np + i] = (uint8_t)g;
    planes[2 * np + i] = (uint8_t)b;
    planes[3 * np + i] = (uint8_t)(mode == 0 ? (299 * r + 587 * g + 114 * b + 500) / 1000
                                             : (r + g + b + 1) / 3);
}
}  // namespace

// Workspace: four planes (R, G, B, dimension image), the FD/pool/encode parts
// of one image on the plane geometry.
void plan_color(const Geom &g, double tol, ColorPlan &cp)
{
    cp.gp = g;
    cp.gp.pitch = g.w;
    BatchJob j;
    j.img = nullptr; j.g = cp.gp; j.tol = tol; j.codes = nullptr;
    j.pooled = std::isfinite(tol) || tol < 0;
    BatchPlan bp;
    plan_batch(&j, 1, bp);
    cp.job = j;
    cp.part = bp.part[0];
    size_t o = bp.total;
    cp.off_planes = o;
    o += align256((size_t)4 * g.h * g.w);
    cp.total = o;
}

hipError_t run_color(const ColorPlan &cp, const uint8_t *rgb, int32_t rgb_pitch, int32_t fd_source,
                     fic_code *const codes[3], void *ws, int num_cu, u64 *counters, hipStream_t s,
                     const Tracer *tr)
{
    char *w = (char *)ws;
    const Geom &g = cp.gp;
    const int64_t np = (int64_t)g.h * g.w;
    uint8_t *planes = (uint8_t *)(w + cp.off_planes);
    hipLaunchKernelGGL(k_color_planes, dim3(blocks_for(np, 256)), dim3(256), 0, s, rgb, g.h, g.w,
                       rgb_pitch, fd_source, planes);
    hipError_t e = hipGetLastError();
    const BatchPart &pt = cp.part;
    double *fdr = (double *)(w + pt.off_fdr);
    double *fdd = (double *)(w + pt.off_fdd);
    uint32_t *perm = (uint32_t *)(w + pt.off_perm);
    uint32_t *lo = (uint32_t *)(w + pt.off_lo);
    uint32_t *hi = (uint32_t *)(w + pt.off_hi);
    const bool pooled = cp.job.pooled;
    if (pooled && e == hipSuccess) {
        const uint8_t *fdimg = planes + 3 * np;
        e = launch_fd_classify(fdimg, g.h, g.w, g.pitch, g.b, g.b, fdr, nullptr, s, tr);
        if (e == hipSuccess)
            e = launch_fd_classify(fdimg, g.h, g.w, g.pitch, 2 * g.b, g.t, fdd, nullptr, s, tr);
        if (e == hipSuccess)
            e = launch_pool(fdr, (int32_t)g.R, fdd, (int32_t)g.D, cp.job.tol, perm, lo, hi,
                            w + pt.off_pool, s, tr);
    }
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
        e = run_encode(pt.plan, planes + c * np, pooled ? perm : nullptr, pooled ? lo : nullptr,
                       pooled ? hi : nullptr, FIC_KERNEL_MFMA, codes[c], w + pt.off_enc, num_cu,
                       counters, s, tr);
    return e;
}

}  // namespace fic

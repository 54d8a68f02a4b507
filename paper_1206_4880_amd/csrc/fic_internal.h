// fic_internal.h -- shared declarations of the gfx950 PIFS search library.
//
// Everything here is device-side plumbing for the kernels in this directory:
// block geometry, the square isometries, the exact quantized fit of one
// (range, domain, isometry) pair, operand layouts of the matrix-core search
// and the launch wrappers the C ABI calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "fic.h"

namespace fic {

typedef unsigned long long u64;
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int kWave = 64;
constexpr u64 kNoKey = ~0ull;

// ---------------------------------------------------------------------------
// Operand layout of the matrix-core search, per range size B (n = B*B).
// The cross term of a (range, isometry) row with a domain column is a dot
// product over K = n pixels, run as MR x MR output tiles:
//   MR   tile side: 16 (v_mfma_f32_16x16x32_f16) for 8x8 and 16x16 ranges;
//        32 (v_mfma_f32_32x32x16_f16, whose K = 16 is exactly one 4x4
//        range) for 4x4 ranges
//   KPI  K consumed by one MFMA; EPL halves per lane per MFMA (MR*KPI/64)
//   KS   MFMAs per tile (n / KPI)
//   MB   MR-row blocks per wave; GR ranges per wave. A 16-row block holds
//        2 ranges x 8 isometries, a 32-row block 4 ranges x 8 isometries.
//   NCH  independent FP32 accumulators per row block: a sum of 64 products of
//        a centred pixel (|.| <= 255) and a centred 2x2 sum (|.| <= 1020) stays
//        below 2^24, so each 64-element chunk is exact; n = 256 keeps 4.
// Element (ks, kg, e) of lane kg*MR + r is pixel K = ks*KPI + kg*EPL + e of
// the block in row-major order, for the A (rows) and B (columns) operand
// alike, so their products pair up pixel by pixel.
template <int B> struct Cfg;
// QR: the 16 x 16 tiles hold a range's 8 isometries in one quarter of the
// lanes over two row blocks (1), or in one row block (0); see a_place.
template <> struct Cfg<4> {
    static constexpr int n = 16, MR = 32, KPI = 16, EPL = 8, KS = 1, MB = 4, NCH = 1, GR = 16,
                         QR = 0;
};
template <> struct Cfg<8> {
    static constexpr int n = 64, MR = 16, KPI = 32, EPL = 8, KS = 2, MB = 8, NCH = 1, GR = 16,
                         QR = 1;
};
template <> struct Cfg<16> {
    static constexpr int n = 256, MR = 16, KPI = 32, EPL = 8, KS = 8, MB = 3, NCH = 4, GR = 6,
                         QR = 0;
};

// Row of range ls (0..GR-1 of its wave group) under isometry q: row block
// blk and row inside it. Lane l of a 16x16 output holds rows 4*(l/16) + v,
// v = 0..3.
//   MR = 16, QR = 1: row block 2*(ls%4) + q/4, row 4*(ls/4) + q%4. Lane l
//            sees range 4*(l/16) + blk/2 under isometries 4*(blk%2) + v, so
//            a pair of row blocks holds all 8 isometries of one range per lane.
//   MR = 16, QR = 0: row block ls/2, row 8*(ls%2) + q. Lane l sees range
//            2*blk + l/32 under isometries 4*((l/16)%2) + v.
//   MR = 32: the output of lane l holds rows 8*(v/4) + 4*(l/32) + v%4,
//            v = 0..15; the placement below makes v < 8 range 2*(l/32) and
//            v >= 8 range 2*(l/32) + 1 of the quad, isometry v % 8.
template <int B>
__host__ __device__ inline void a_place(int ls, int q, int &blk, int &row)
{
    if (Cfg<B>::MR == 32) {
        const int rl = ls & 3;
        blk = ls >> 2;
        row = 8 * (2 * (rl & 1) + (q >> 2)) + 4 * (rl >> 1) + (q & 3);
    } else if (Cfg<B>::QR) {
        blk = 2 * (ls & 3) + (q >> 2);
        row = 4 * (ls >> 2) + (q & 3);
    } else {
        blk = ls >> 1;
        row = 8 * (ls & 1) + q;
    }
}

// Per-range state, in search order ("slot"). 32 bytes.
struct RangeStat {
    int64_t srr;     // n*sum r^2 - (sum r)^2
    int32_t sr;      // sum r
    int32_t delta;   // sum r - n*rhat, rhat = the centring level of the A rows
    uint32_t ridx;   // raster range index
    uint32_t lo, hi; // pool = columns [lo, hi) of the domain order
    uint32_t flags;  // kFlat | kPad | kEmpty | kSkip
};
constexpr uint32_t kFlat = 1u, kPad = 2u, kEmpty = 4u, kSkip = 8u;   // kSkip: not selected
constexpr uint32_t kIdle = kFlat | kPad | kEmpty | kSkip;             // never searched

struct WorkItem { uint32_t grp, c0, c1, pad; };

// ---------------------------------------------------------------------------
// Search parameters chosen per image ON THE DEVICE from its pool fraction:
// bucket 0 is exhaustive search; a pooled image with
// f = (sum of pool sizes) / (R * D) falls in bucket 1 + floor(-log2 f),
// clamped to [1, kTuneBuckets - 1]. Per bucket: the columns of a work item
// (2^chunk_log2, kChunkLog2Min..kChunkLog2Max) and the early flush trigger of
// the search queue (flush once at least flush_at half cells are queued; 4x4:
// cells, tested after each replay of queued columns; 0 = only when the queue
// is full), and whether a single-image
// search takes its work items from one queue per XCD (xcd = 1: queue x holds
// the column chunks c = x (mod 8), so each XCD's L2 streams an eighth of the
// domain columns; waves steal from the other queues when theirs is empty).
// A row serves one (range size, log2 D) class; the autotuner fills rows,
// defaults are below.
constexpr int kTuneBuckets = 6;
constexpr int kChunkLog2Min = 11, kChunkLog2Max = 16;
// Work-list entries a single search plans for at most (16 bytes each: 1 GiB);
// a job that would need more at 2^kChunkLog2Min columns uses wider items.
constexpr int64_t kMaxItems = (int64_t)1 << 26;
constexpr int kXcds = 8;             // MI355X: 8 XCDs, workgroups assigned round robin
struct TuneRow {
    int8_t chunk_log2[kTuneBuckets];
    int16_t flush_at[kTuneBuckets];
    uint8_t xcd[kTuneBuckets];
};
// Exhaustive jobs 16384-column items, pooled 4096 (narrow pools need the
// finer balance); the early flush at 64 queued half cells only at 8x8.
inline TuneRow default_tune_row(int b)
{
    TuneRow r;
    for (int k = 0; k < kTuneBuckets; ++k) {
        r.chunk_log2[k] = (int8_t)(k == 0 ? 14 : 12);
        r.flush_at[k] = (int16_t)(b == 8 ? 64 : 0);
        r.xcd[k] = 0;
    }
    return r;
}
// Bucket of a pooled image's pool fraction f (1 for f >= 1/2, 2 for
// [1/4, 1/2), ..., kTuneBuckets - 1 below).
__host__ __device__ inline int tune_bucket_of_fraction(double f)
{
    int b = 1;
    double edge = 0.5;
    while (b < kTuneBuckets - 1 && f < edge) {
        ++b;
        edge *= 0.5;
    }
    return b;
}
// The bucket of an image: 0 when exhaustive, else that of
// f = pool_sum / (R * D) in fp64 (pool_sum: the exact integer sum of the
// searched ranges' pool sizes). Host and device use this same rule.
__host__ __device__ inline int tune_bucket(int pooled, uint64_t pool_sum, int64_t R, int64_t D)
{
    if (!pooled) return 0;
    return tune_bucket_of_fraction((double)pool_sum / ((double)R * (double)D));
}

// Debug switches of a context (fic_set_debug): consume the work items in
// reverse order; run the 16x16 search's rounding check; search the 4x4 and
// 8x8 images of a batch in one launch per range size instead of one
// combined launch.
constexpr uint32_t kDbgReverse = 1u, kDbgVerify16 = 2u, kDbgSeparate = 4u;

// ---------------------------------------------------------------------------
// The isometries: T_q(d)[i][j] = d[src], src per q (0 identity, 1 rot90 cw,
// 2 rot180, 3 rot270 cw, 4 mirror left-right, 5 mirror up-down, 6 transpose,
// 7 anti-transpose).
__host__ __device__ inline void iso_src(int q, int b, int i, int j, int &si, int &sj)
{
    switch (q) {
    case 0: si = i;         sj = j;         break;
    case 1: si = b - 1 - j; sj = i;         break;
    case 2: si = b - 1 - i; sj = b - 1 - j; break;
    case 3: si = j;         sj = b - 1 - i; break;
    case 4: si = i;         sj = b - 1 - j; break;
    case 5: si = b - 1 - i; sj = j;         break;
    case 6: si = j;         sj = i;         break;
    default: si = b - 1 - j; sj = b - 1 - i; break;
    }
}
// q' with T_q' = T_q^-1 (only the quarter turns are not involutions).
__host__ __device__ inline int iso_inverse(int q) { return q == 1 ? 3 : (q == 3 ? 1 : q); }

// ---------------------------------------------------------------------------
// Exact fit of one pair. With s = k/16, o = 2j:
//   4096*n*SSE = F(k) + 4096*(sum r - 2nj)^2,
//   F(k) = 4096*Srr' - 128*k*Srd' + k^2*Sdd'  (a parabola in k).
// The integer minimiser on [-16, 15] is the clamped nearest integer to the
// vertex 64*Srd'/Sdd' (ties to the smaller |k|). The vertex is located in
// fp64 (error far below 1/2), then the two neighbouring integers are compared
// exactly in int64, so the choice is exact.
__host__ __device__ inline int64_t fit_f(int64_t srr, int64_t srd, int64_t sdd, int &k_out)
{
    int k;
    if (sdd <= 0) {
        k = 0;
    } else {
        double v = 64.0 * (double)srd / (double)sdd;
        if (v >= 15.0) {
            k = 15;
        } else if (v <= -16.0) {
            k = -16;
        } else {
            int k0 = (int)floor(v);          // in [-16, 14]
            int k1 = k0 + 1;
            int64_t f0 = 4096 * srr - 128 * (int64_t)k0 * srd + (int64_t)k0 * k0 * sdd;
            int64_t f1 = 4096 * srr - 128 * (int64_t)k1 * srd + (int64_t)k1 * k1 * sdd;
            int a0 = k0 < 0 ? -k0 : k0, a1 = k1 < 0 ? -k1 : k1;
            k = (f1 < f0 || (f1 == f0 && a1 < a0)) ? k1 : k0;
        }
    }
    k_out = k;
    return 4096 * srr - 128 * (int64_t)k * srd + (int64_t)k * k * sdd;
}

// F of the best contrast index, as fit_f, for the queue flushes (many fits
// per call), in fp64: every term of F is an integer below 2^53 for n <= 256
// (|Srd'| <= sqrt(Srr' Sdd')), so each fma is exact. base = 4096 Srr', rd =
// Srd', dd = Sdd', inv = an fp32 reciprocal of Sdd'. The vertex
// v = 64 Srd'/Sdd' it gives is off by far less than 1/2, so the integer
// minimiser over [-16, 15] is among round(v) - 1, round(v), round(v) + 1;
// those three are compared exactly, ties to the smaller |k| (fit_f's rule).
__device__ inline double fit_f_d(double base, double rd, double dd, float inv)
{
    if (dd <= 0.0) return base;
    const float v = 64.0f * (float)rd * inv;
    int kr = (int)rintf(fminf(fmaxf(v, -17.0f), 16.0f));
    kr = kr < -15 ? -15 : (kr > 14 ? 14 : kr);     // candidates kr - 1 .. kr + 1 in [-16, 15]
    double best = 0.0;
    int babs = 0;
#pragma unroll
    for (int j = -1; j <= 1; ++j) {
        const int k = kr + j;
        const double f = fma((double)(k * k), dd, fma(-128.0 * (double)k, rd, base));
        const int a = k < 0 ? -k : k;
        if (j == -1 || f < best || (f == best && a < babs)) {
            best = f;
            babs = a;
        }
    }
    return best;
}

// Packed search key: (F << shift) | (domain << 3) | isometry. Its unsigned
// minimum is the lexicographic minimum of (F, domain, isometry).
__host__ __device__ inline u64 pack_key(int64_t f, uint32_t dom, int q, int shift)
{
    return ((u64)f << shift) | ((u64)dom << 3) | (u64)q;
}

// Screen threshold of a range whose best key so far has error F: a pair can
// only reach F if |Srd'| / sqrt(Sdd') >= sqrt(Srr' - F/4096). Rounded down.
__device__ inline float screen_t(int64_t srr, int64_t f)
{
    double theta = (double)srr - (double)f * (1.0 / 4096.0);
    if (theta <= 0.0) return 0.0f;
    return (float)(sqrt(theta) * (1.0 - 0x1p-20));
}

// Domain side constant u = sqrt(Sdd') / n, rounded down; flat domains get a
// huge finite value (they can only tie when the range threshold is 0).
__device__ inline float screen_u(int64_t sdd, int n)
{
    if (sdd <= 0) return 1e30f;
    return (float)(sqrt((double)sdd) / (double)n * (1.0 - 0x1p-20));
}

// ---------------------------------------------------------------------------
// Stage tracing hook: the C ABI passes a recorder that puts HIP events around
// each stage on the stream; nullptr disables it.
struct Tracer {
    void *self;
    void (*mark)(void *self, int stage, int begin, hipStream_t s);
};
inline void trace(const Tracer *t, int stage, int begin, hipStream_t s)
{
    if (t) t->mark(t->self, stage, begin, s);
}

// ---------------------------------------------------------------------------
// Launch wrappers (each .hip file owns its kernels).
struct Geom {
    int32_t h, w, pitch, b, t;
    int32_t n, rcols, rrows, dcols, drows;
    int64_t R, D;
};

// DBC fractal dimension (fd_dbc.hip)
hipError_t launch_fd_classify(const uint8_t *img, int32_t h, int32_t w, int32_t pitch,
                              int32_t block, int32_t step, double *fd64, float *fd32,
                              hipStream_t s, const Tracer *tr = nullptr);

// radix sort + pool (pool.hip)
size_t sort_ws_bytes(int64_t n);
hipError_t radix_sort_pairs(u64 *keys, uint32_t *vals, int64_t n, int key_bits, void *ws,
                            hipStream_t s, double *fd_out = nullptr);
size_t scan_ws_bytes(int64_t m);
hipError_t scan_u32(uint32_t *a, int64_t m, uint32_t *total, void *ws, hipStream_t s);
size_t pool_ws_bytes(int64_t nr, int64_t nd);
hipError_t launch_pool(const double *fd_range, int32_t nr, const double *fd_dom, int32_t nd,
                       double tol, uint32_t *perm, uint32_t *lo, uint32_t *hi, void *ws,
                       hipStream_t s, const Tracer *tr = nullptr);

// encode (encode.hip)
struct EncodePlan {
    Geom g;
    int pooled;
    int64_t Rp, Dp, G, GR, NC;   // padded ranges/columns, groups, ranges per group, chunks
    int64_t IGW, IG;              // groups per work item (one per wave of a workgroup), item groups
    int32_t shift;                // NC: chunk slots at the narrowest item (2^chunk_min
                                  // columns), a multiple of kXcds
    int32_t chunk_min;            // narrowest item width (log2): kChunkLog2Min, raised for
                                  // large jobs so the work list stays within kMaxItems
    int64_t max_items;
    size_t off_A, off_rs, off_order, off_B, off_u, off_eps, off_sdd, off_dom, off_keys,
        off_items, off_ctr, off_args, off_chunkcnt, off_chunkfill, off_grp, off_bmin, off_S,
        off_sort, off_sortkeys, off_scan, total;
    // (dev) per range, raster order: 0 = not coded (its code gets flag bit 2);
    // null = every range. Set by the caller after plan_encode.
    const uint8_t *sel;
    TuneRow tune;                 // parameters per pool-fraction bucket
    uint32_t dbg;                 // kDbg* switches
};
hipError_t init_search_occupancy();   // once per process, before any search launch
void plan_encode(const Geom &g, int pooled, EncodePlan &p);
hipError_t run_encode(const EncodePlan &p, const uint8_t *img, const uint32_t *perm,
                      const uint32_t *lo, const uint32_t *hi, int kernel, fic_code *codes,
                      void *ws, int num_cu, u64 *counters, hipStream_t s,
                      const Tracer *tr = nullptr);

// Batch: one image of it, its workspace part, and the whole layout.
struct BatchJob {
    const uint8_t *img;
    Geom g;
    double tol;
    bool pooled;
    fic_code *codes;
};
struct BatchPart {
    size_t off_fdr, off_fdd, off_perm, off_lo, off_hi, off_pool, off_enc;
    EncodePlan plan;
};
struct BatchPlan {
    int32_t n;
    std::vector<int32_t> order;      // preparation / table order of the images
    std::vector<int32_t> slot;       // table entry of image i
    std::vector<BatchPart> part;
    int32_t group_first[3], group_count[3];   // table runs for B = 4, 8, 16
    size_t off_tab, off_base, off_ctr, total;
    int64_t items;                   // upper bound on the work items of all images
    uint32_t dbg;                    // kDbg* switches of the searches
};
// Side streams for the per-image preparation of a batch: forked from the
// calling stream by one event and joined back before the searches (under
// stream capture this records parallel branches).
constexpr int kMaxSideStreams = 8;
struct BatchStreams {
    int ns;
    hipStream_t side[kMaxSideStreams];
    hipEvent_t fork;
    hipEvent_t join[kMaxSideStreams];
};
void plan_batch(const BatchJob *jobs, int32_t n, BatchPlan &bp);

// Two-level (quadtree) encode: level-1 ranges B1, level-2 ranges B2 = B1/2
// coded only inside level-1 ranges whose E exceeds emax.
struct QuadPlan {
    BatchJob lv[2];                  // img, geometry, tol, pooled per level (codes set per call)
    BatchPart part[2];
    size_t off_sel, total;
};
void plan_quadtree(const Geom &g1, double tol1, const Geom &g2, double tol2, QuadPlan &qp);

// Colour: the channels of an interleaved RGB image, each searched over the
// pool of the luma (fd_source 0) or mean (1) image.
struct ColorPlan {
    Geom gp;                         // plane geometry (pitch = width)
    BatchJob job;
    BatchPart part;
    size_t off_planes, total;
};
void plan_color(const Geom &g, double tol, ColorPlan &cp);
hipError_t run_color(const ColorPlan &cp, const uint8_t *rgb, int32_t rgb_pitch, int32_t fd_source,
                     fic_code *const codes[3], void *ws, int num_cu, u64 *counters, hipStream_t s,
                     const Tracer *tr = nullptr);
hipError_t run_quadtree(const QuadPlan &qp, const uint8_t *img, int64_t emax, fic_code *codes1,
                        fic_code *codes2, void *ws, int num_cu, u64 *counters, hipStream_t s,
                        const Tracer *tr = nullptr);
hipError_t run_encode_batch(const BatchJob *jobs, const BatchPlan &bp, void *ws, int num_cu,
                            u64 *counters, hipStream_t s, const Tracer *tr = nullptr,
                            const BatchStreams *bs = nullptr);

// packed code bit string (bitstream.hip)
int code_dbits(int64_t D);
int64_t packed_words(const Geom &g);
hipError_t run_pack(const Geom &g, const fic_code *codes, uint32_t *words, hipStream_t s);
hipError_t run_unpack(const Geom &g, const uint32_t *words, fic_code *codes, hipStream_t s);

// decode (decode.hip)
size_t decode_ws_bytes(const Geom &g);
int32_t decode_max_iters();
hipError_t run_decode(const Geom &g, const fic_code *codes, int32_t max_iters,
                      const uint8_t *init, uint8_t *out, void *ws, int32_t *iters,
                      hipStream_t s, const Tracer *tr = nullptr);
hipError_t run_decode_quadtree(const Geom &g1, const fic_code *codes1, const Geom &g2,
                               const fic_code *codes2, int32_t max_iters, const uint8_t *init,
                               uint8_t *out, void *ws, int32_t *iters, hipStream_t s,
                               const Tracer *tr = nullptr);

}  // namespace fic

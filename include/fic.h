/*
 * fic.h -- C ABI of the MI355X (gfx950) PIFS range-domain matching library.
 *
 * The operations follow the paper's statement of the encoder (Revathy &
 * Jayamohan, "Dynamic Domain Classification for Fractal Image Compression"):
 *   fic_fd_classify        Sec. 3.1: local fractal dimension of every block by
 *                          differential box counting (ref. [9]).
 *   fic_build_domain_pool  Sec. 3.1: domains ordered by dimension (the role of
 *                          the balanced search tree) and, per range, the window
 *                          d_r - D_f <= d_d <= d_r + D_f as an interval of that
 *                          order; D_f = (F_m - F_l)/3 when no tolerance is given.
 *   fic_encode_pifs        Sec. 1 / Sec. 2: for every non-overlapping range, the
 *                          best domain (twice the size, overlapping, shrunk by
 *                          2x2 sums) under the 8 square isometries and the
 *                          quantized contrast / brightness; exhaustive or pooled.
 *   fic_encode_pifs_batch  the same for many images of different sizes.
 *   fic_decode_pifs        Sec. 1: iterate the maps from a start image.
 *   fic_encode_quadtree /  a two-level range partition (ref. [12]) on top of
 *   fic_decode_quadtree    the same search and decoder.
 *
 * Quantities (exact integers; n = B*B; D = 2x2 sums of the domain, 0..1020):
 *   contrast   s = k/16, k in [-16, 15]        (5 bits)
 *   brightness o = 2j,   j in [0, 127]          (7 bits)
 *   map        r'_i = s * ((T_q D)_i/4 - sum(D)/(4n)) + o
 *   error      E = 4096 * n * SSE  (exact)
 *   selection  minimum E; ties to the lowest (domain index, isometry), then
 *              the smaller |k|, then the smaller k; j is the nearest level to
 *              the range mean, ties down.
 *   isometry q T_q(d)[i][j] = d[src]: 0 (i,j), 1 (B-1-j,i) rot90 cw,
 *              2 (B-1-i,B-1-j), 3 (j,B-1-i) rot270 cw, 4 (i,B-1-j) mirror LR,
 *              5 (B-1-i,j) mirror UD, 6 (j,i) transpose, 7 (B-1-j,B-1-i).
 *   lattice    ranges raster order over (H/B) x (W/B); domains at (t*a, t*c)
 *              fully inside the image, index a*cols + c.
 *
 * Conventions for every call:
 *   - Pointers marked (dev) are HIP device pointers, (host) host pointers.
 *     The caller owns every buffer; the library never frees caller memory and
 *     allocates no device memory inside these calls (a context holds only a
 *     few bytes of per-device state).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on it and never synchronise the host, except
 *     fic_create. Outputs are valid once the stream reaches that point.
 *   - Arguments are validated on the host before any HIP call; an invalid
 *     call returns a status and launches nothing. No exception crosses the
 *     ABI. A context is not thread-safe: use one per host thread.
 */
#ifndef FIC_H
#define FIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FIC_OK = 0,
    FIC_ERR_INVALID_ARG = 1,   /* null pointer, bad geometry, NaN tolerance ... */
    FIC_ERR_UNSUPPORTED = 2,   /* a valid request the library does not handle   */
    FIC_ERR_WORKSPACE = 3,     /* ws_bytes below fic_*_workspace_bytes()        */
    FIC_ERR_CAPACITY = 4,      /* the packed (F, domain, isometry) key would
                                  not fit 64 bits for this geometry, the 4x4 /
                                  8x8 B operand would reach 2^31 bytes, or the
                                  work list could exceed 2^32 - 1 items        */
    FIC_ERR_DEVICE = 5         /* no HIP device, or a HIP call / launch failed  */
} fic_status;

/* Image geometry. uint8 rows of `pitch` bytes (pitch >= width).
   range_size B in {4, 8, 16}; height, width multiples of B and >= 2B;
   domain side 2B; domain_step t >= 1. */
typedef struct {
    int32_t height, width, pitch;
    int32_t range_size;
    int32_t domain_step;
} fic_geom;

/* One code per range, ranges in raster order. 16 bytes. */
typedef struct {
    uint32_t domain;   /* raster index on the domain lattice                  */
    uint8_t  iso;      /* 0..7                                                */
    int8_t   s_idx;    /* k, s = k/16                                         */
    uint8_t  o_idx;    /* j, o = 2j                                           */
    uint8_t  flags;    /* bit 0: empty pool, DC-only code (domain 0, iso 0,
                          k = 0); bit 1: split (two-level encode); bit 2:
                          not coded (two-level encode, parent not split);
                          bit 7: internal check failed -- the search's
                          packed key disagreed with the exact recomputation
                          of its winner from the pixels. It never occurs
                          in a correct build; a code carrying it must not
                          be trusted (the call itself still returned
                          FIC_OK, since codes are written asynchronously). */
    int64_t  err;      /* E = 4096 * n * SSE                                  */
} fic_code;

typedef struct fic_ctx fic_ctx;

enum { FIC_KERNEL_MFMA = 0, FIC_KERNEL_PLAIN = 1 };

/* Per-image job of a batch (host struct; pointers inside are device). */
typedef struct {
    const uint8_t *img;   /* (dev) */
    fic_geom geom;
    double tol;           /* as fic_build_domain_pool; +INF = exhaustive */
    fic_code *codes;      /* (dev) ranges of this image */
} fic_image_desc;

/* Create a context on HIP device `device` (queries its properties; this is
   the only call that may block). FIC_ERR_DEVICE when there is no such
   device, FIC_ERR_UNSUPPORTED when it is not gfx950. device = -1 makes a
   host-only context: every call still validates its arguments (and returns
   their error), then answers FIC_ERR_DEVICE instead of launching. */
fic_status fic_create(int32_t device, fic_ctx **out /* host */);
fic_status fic_destroy(fic_ctx *ctx);

/* Static text of a status (host). */
const char *fic_status_string(fic_status s);

/* Optional instrumentation: when `counters` (dev, 8 x uint64, zeroed by the
   caller) is set, the search kernels add
     [0] pair evaluations screened, [1] pairs passed to the exact fit,
     [2] work items processed,      [3] exact seeds evaluated,
     [7] columns the 4x4 search queued and replayed (recomputed on the
         matrix cores and screened cell by cell),
   and with FIC_DEBUG_VERIFY16 (fic_set_debug) the 16x16 search adds
     [4] FP32 sums whose rounding error exceeded the bound its screen
         threshold is lowered by (must stay 0),
     [5] sums checked, [6] the largest error / bound seen, in units of
         2^-20 (an atomic maximum).
   NULL (the default) disables the adds. */
fic_status fic_set_counters(fic_ctx *ctx, uint64_t *counters /* dev */);

/* Debug switches (host state of the context, for tests; 0 = off, the
   default). FIC_DEBUG_REVERSE_ITEMS: the persistent searches take their
   work items in reverse order (codes must not change: the packed-key minimum
   is order independent). FIC_DEBUG_VERIFY16: the 16x16 search recomputes the
   exact 64-term chunk sums of every block it screens and checks the rounding
   error of its one-accumulator FP32 sums against the bound its screen relies
   on, counting into counters [4]..[6] (much slower; codes unchanged).
   FIC_DEBUG_SEPARATE_SEARCHES: a batch searches its 4x4 and its 8x8 images
   in one persistent launch per range size instead of one combined launch
   (codes unchanged; for comparisons).
   FIC_ERR_INVALID_ARG for unknown bits. Batch graphs are recorded per
   switch setting. */
enum { FIC_DEBUG_REVERSE_ITEMS = 1, FIC_DEBUG_VERIFY16 = 2, FIC_DEBUG_SEPARATE_SEARCHES = 4 };
fic_status fic_set_debug(fic_ctx *ctx, uint32_t flags);

/* Stage tracing. With timing enabled, each later call records a pair of HIP
   events around each of its stages, on the call's own stream:
     FIC_STAGE_CLASSIFY    differential box counting (fic_fd_classify)
     FIC_STAGE_POOL        sort + window bounds (fic_build_domain_pool)
     FIC_STAGE_RANGE_PREP  range order, sums and A rows
     FIC_STAGE_DOMAIN_PREP 2x2 sums, domain sums and B columns
     FIC_STAGE_WORKLIST    seeds and the work list of the persistent search
     FIC_STAGE_SEARCH      the search kernel itself (MFMA or plain)
     FIC_STAGE_FINAL       finalize (codes)
     FIC_STAGE_DECODE      all decoding sweeps
     FIC_STAGE_BATCH       a whole fic_encode_pifs_batch replayed as one graph
   fic_timing_enable(ctx, 1) clears the record and starts recording; 0 stops.
   fic_timing_read waits for the recorded events (host sync), then writes up
   to `capacity` (stage, milliseconds) pairs in record order (host arrays)
   and the total number recorded to *count. Events are host objects; no
   device memory is allocated. */
enum {
    FIC_STAGE_CLASSIFY = 0, FIC_STAGE_POOL = 1, FIC_STAGE_RANGE_PREP = 2,
    FIC_STAGE_DOMAIN_PREP = 3, FIC_STAGE_WORKLIST = 4, FIC_STAGE_SEARCH = 5,
    FIC_STAGE_FINAL = 6, FIC_STAGE_DECODE = 7, FIC_STAGE_BATCH = 8
};
fic_status fic_timing_enable(fic_ctx *ctx, int32_t enable);
fic_status fic_timing_read(fic_ctx *ctx, int32_t *stages /* host */, float *ms /* host */,
                           int32_t capacity, int32_t *count /* host */);

/* Number of ranges / domains of a geometry (host helpers; 0 if invalid). */
int64_t fic_num_ranges(const fic_geom *g /* host */);
int64_t fic_num_domains(const fic_geom *g /* host */);

/* ------------------------------------------------------------------------
 * fic_fd_classify -- Sec. 3.1, differential box counting.
 * For every block x block window whose top-left corner is at (step*a,
 * step*c), a = 0..(H-block)/step, c = 0..(W-block)/step, raster order:
 *   box sizes s = 2, 4, ..., block; box height h = s*256/block;
 *   n_s = sum over the (block/s)^2 cells of floor(max/h) - floor(min/h) + 1;
 *   FD = least-squares slope of log N_s against log(block/s).
 * Ranges use (block, step) = (B, B); domains (2B, t).
 *   img   (dev) uint8, g->pitch bytes per row
 *   block in {4, 8, 16, 32}; step >= 1; block <= height, width
 *   fd64  (dev) double[count] (required); fd32 (dev) float[count] or NULL,
 *         fd32 = (float)fd64.
 * ---------------------------------------------------------------------- */
fic_status fic_fd_classify(fic_ctx *ctx, const uint8_t *img, const fic_geom *g,
                           int32_t block, int32_t step,
                           double *fd64, float *fd32, void *stream);

/* ------------------------------------------------------------------------
 * fic_build_domain_pool -- Sec. 3.1, the dynamic per-range domain pool.
 *   fd_range  (dev) double[n_range], fd_domain (dev) double[n_domain]
 *   tol       >= 0: window half-width; < 0: D_f = (max - min)/3 over
 *             fd_domain; +INF: every domain. NaN is rejected.
 *   perm      (dev) uint32[n_domain]: domain indices in ascending fd order,
 *             equal values in ascending index (stable).
 *   lo, hi    (dev) uint32[n_range]: the pool of range r is
 *             perm[lo[r] .. hi[r]), exactly { d : |fd_d - fd_r| <= tol + 1e-9 }
 *             in fp64.
 *   ws        (dev) scratch of ws_bytes >= fic_pool_workspace_bytes(n_range,
 *             n_domain).
 * ---------------------------------------------------------------------- */
size_t fic_pool_workspace_bytes(int64_t n_range, int64_t n_domain);
fic_status fic_build_domain_pool(fic_ctx *ctx, const double *fd_range, int32_t n_range,
                                 const double *fd_domain, int32_t n_domain, double tol,
                                 uint32_t *perm, uint32_t *lo, uint32_t *hi,
                                 void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * fic_encode_pifs -- Sec. 1 / Sec. 2, the range-domain matching search.
 *   img    (dev) uint8 image, geometry g (host)
 *   perm, lo, hi  (dev) from fic_build_domain_pool for this image, or all
 *          three NULL for exhaustive search (every domain for every range).
 *          Mixed NULL / non-NULL is rejected.
 *   kernel FIC_KERNEL_MFMA (FP16 matrix-core cross terms, exact, screened,
 *          persistent work queue) or FIC_KERNEL_PLAIN (one thread per
 *          (range, domain, isometry), integer arithmetic).
 *   codes  (dev) fic_code[fic_num_ranges(g)], raster order.
 *   ws     (dev) scratch, ws_bytes >= fic_encode_workspace_bytes(g, pooled).
 * Both kernels return identical codes.
 * ---------------------------------------------------------------------- */
size_t fic_encode_workspace_bytes(const fic_geom *g, int32_t pooled);
fic_status fic_encode_pifs(fic_ctx *ctx, const uint8_t *img, const fic_geom *g,
                           const uint32_t *perm, const uint32_t *lo, const uint32_t *hi,
                           int32_t kernel, fic_code *codes,
                           void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * fic_encode_pifs_noalloc -- fic_encode_pifs for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same search and the same codes, with
 * the workspace taken from a static device array of the library instead of
 * a caller buffer. It calls no hipMalloc / hipFree or other allocating
 * routine and records no stage events.
 *   Arguments as fic_encode_pifs, without ws / ws_bytes.
 *   FIC_ERR_WORKSPACE when fic_encode_workspace_bytes(g, pooled) exceeds
 *   fic_noalloc_scratch_bytes() (64 MiB: e.g. 512 x 512 jobs with 4 x 4 or
 *   8 x 8 ranges, 1024 x 1024 with 8 x 8 ranges at domain step 2; 16 x 16
 *   ranges at domain step 1 need more from 512 x 512 up).
 * The array exists once per GPU (held until the process ends) and is shared
 * by every call on that GPU: calls that overlap on one GPU (other streams,
 * other host threads or contexts) race and must be serialised by the caller.
 * Each call initialises what it reads, so no clearing is needed in between.
 * ---------------------------------------------------------------------- */
size_t fic_noalloc_scratch_bytes(void);
fic_status fic_encode_pifs_noalloc(fic_ctx *ctx, const uint8_t *img, const fic_geom *g,
                                   const uint32_t *perm, const uint32_t *lo, const uint32_t *hi,
                                   int32_t kernel, fic_code *codes, void *stream);

/* ------------------------------------------------------------------------
 * fic_encode_pifs_batch -- the encoder of Sec. 1 - Sec. 3.1 (classify, pool
 * when tol is finite or negative, search) for n_images images, each with its
 * own geometry and tolerance. Every image is prepared on its own workspace
 * part; then the searches run as ONE persistent work-queue launch over the
 * items of all 4x4 and 8x8 images (8x8 images first, each size's images
 * largest first; 16x16 images in a second launch of their own); then the
 * codes are written.
 *   descs (host) fic_image_desc[n_images]; codes of image i go to
 *         descs[i].codes (dev). Codes equal fic_encode_pifs on each image.
 *   ws    (dev) >= fic_batch_workspace_bytes(n_images, descs) (the sum of
 *         the images' parts plus a small header).
 * Graphs (default on, see fic_set_batch_graph): the first call with given
 * descriptors, workspace and counters records the whole batch as a HIP graph
 * (captured on a stream of the context's own) and launches it on `stream`;
 * later calls with the same descriptors, workspace and counters replay it.
 * A replay reads the images' current contents. The context keeps the 4 most
 * recently used graphs (host objects; no device memory is allocated).
 * FIC_ERR_CAPACITY also when the batch could exceed 2^32 work items.
 * ---------------------------------------------------------------------- */
size_t fic_batch_workspace_bytes(int32_t n_images, const fic_image_desc *descs);
fic_status fic_encode_pifs_batch(fic_ctx *ctx, int32_t n_images,
                                 const fic_image_desc *descs,
                                 void *ws, size_t ws_bytes, void *stream);
/* enable != 0 (the default): record and replay batch graphs as above;
   0: enqueue every kernel of each call directly (and drop recorded graphs). */
fic_status fic_set_batch_graph(fic_ctx *ctx, int32_t enable);

/* ------------------------------------------------------------------------
 * fic_encode_color -- per-channel encode of a colour image (Sec. 3.1
 * discusses colour): the fractal dimensions, and so the pools, come from one
 * gray image -- fd_source 0: luma (299 R + 587 G + 114 B + 500) div 1000,
 * 1: channel mean (R + G + B + 1) div 3 -- and each channel is searched over
 * them (tol as in fic_image_desc; +INF = exhaustive).
 *   rgb   (dev) interleaved uint8 R, G, B; g->pitch = bytes per row >= 3*width;
 *         height, width, range_size, domain_step as for fic_encode_pifs.
 *   codes_r, codes_g, codes_b (dev) fic_code[fic_num_ranges] each; decode
 *         each with fic_decode_pifs (pitch = width).
 *   ws    (dev) >= fic_color_workspace_bytes(g, tol).
 * ---------------------------------------------------------------------- */
size_t fic_color_workspace_bytes(const fic_geom *g, double tol);
fic_status fic_encode_color(fic_ctx *ctx, const uint8_t *rgb, const fic_geom *g, double tol,
                            int32_t fd_source, fic_code *codes_r, fic_code *codes_g,
                            fic_code *codes_b, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * fic_pack_codes / fic_unpack_codes -- the stored code as a bit string
 * (Sec. 1: per range the domain, the isometry, the contrast and the
 * brightness). Range r's fields start at bit r*W of a little-endian string
 * of 32-bit words, each field least significant bit first, in the order
 * domain index (ceil(log2 D) bits, at least 1), isometry (3), k + 16 (5),
 * j (7); W is their sum (35 bits at 1024^2, 8x8 ranges, step 1). Flags and
 * errors are not stored: unpacked codes have flags 0 and err 0.
 *   words (dev) uint32[nwords], nwords >= fic_packed_words(g); pack clears
 *         the words it uses and FIC_ERR_WORKSPACE when nwords is short;
 *         unpack answers FIC_ERR_INVALID_ARG then.
 *   codes (dev) fic_code[fic_num_ranges(g)].
 * Compression ratio of an image = 8*h*w / (32*fic_packed_words(g)).
 * ---------------------------------------------------------------------- */
int64_t fic_packed_words(const fic_geom *g);
fic_status fic_pack_codes(fic_ctx *ctx, const fic_code *codes, const fic_geom *g,
                          uint32_t *words, int64_t nwords, void *stream);
fic_status fic_unpack_codes(fic_ctx *ctx, const uint32_t *words, int64_t nwords,
                            const fic_geom *g, fic_code *codes, void *stream);

/* ------------------------------------------------------------------------
 * fic_decode_pifs -- Sec. 1, decoding by iteration of the stored maps.
 * Simultaneous sweeps from `init` (dev, h x w, pitch w; NULL = all 128):
 *   pixel = clamp(floor((k*(n*(T_q D')_i - sum D') + 128*n*j + 32*n) / (64n)),
 *                 0, 255)
 * with D' the 2x2 sums of the current image at the code's domain; stops after
 * the first sweep that changes no pixel, or after max_iters sweeps.
 *   codes (dev) fic_code[fic_num_ranges(g)]; out (dev) uint8 h x w (pitch w)
 *   scratch (dev) >= fic_decode_workspace_bytes(g)
 * Decoding at a larger size (the maps do not depend on the pixel grid): the
 * codes of geometry (h, w, B, t) decode at twice the size with geometry
 * (2h, 2w, 2B, 2t) -- the same domain indices; g->range_size may therefore
 * also be 32 here (16x16 codes at twice the size).
 *   iters_done (dev) int32: sweeps run.
 * ---------------------------------------------------------------------- */
size_t fic_decode_workspace_bytes(const fic_geom *g);
fic_status fic_decode_pifs(fic_ctx *ctx, const fic_code *codes, const fic_geom *g,
                           int32_t max_iters, const uint8_t *init, uint8_t *out,
                           void *scratch, size_t scratch_bytes, int32_t *iters_done,
                           void *stream);

/* ------------------------------------------------------------------------
 * fic_encode_quadtree -- two-level partition of the range grid (the quadtree
 * of Fisher's book, the paper's ref. [12], at two levels). The paper does
 * not specify it; the rule here:
 *   - every level-1 range (g1: B1 in {8, 16}) is coded as fic_encode_pifs
 *     does (pool from tol1 as in fic_image_desc, or exhaustive);
 *   - a level-1 code is split when its mean squared error exceeds
 *     rms_split^2, i.e. when E > floor(4096 * n1^2 * rms_split^2) (fp64 in
 *     the order rms*rms*(4096*n1*n1)); its flags get bit 1 and its four
 *     quadrants, the level-2 ranges (g2: B2 = B1/2, same height, width and
 *     pitch, its own domain step) holding its pixels, are coded as
 *     fic_encode_pifs does over the whole level-2 domain lattice (pool from
 *     tol2 or exhaustive);
 *   - every other level-2 code is "not coded": domain 0, iso 0, k = 0, j = 0,
 *     flags bit 2, E = 0.
 *   img     (dev) uint8 image; codes1 (dev) fic_code[R1]; codes2 (dev)
 *           fic_code[R2], raster order on each grid.
 *   rms_split >= 0 (gray levels); +INF never splits, 0 splits every code
 *           with E > 0. NaN or negative is rejected.
 *   ws      (dev) >= fic_quadtree_workspace_bytes(g1, tol1, g2, tol2).
 * ---------------------------------------------------------------------- */
size_t fic_quadtree_workspace_bytes(const fic_geom *g1, double tol1, const fic_geom *g2,
                                    double tol2);
fic_status fic_encode_quadtree(fic_ctx *ctx, const uint8_t *img, const fic_geom *g1, double tol1,
                               const fic_geom *g2, double tol2, double rms_split,
                               fic_code *codes1, fic_code *codes2, void *ws, size_t ws_bytes,
                               void *stream);

/* fic_decode_quadtree -- fic_decode_pifs for a two-level code set: each
   sweep applies the level-1 codes without flag bit 1 and the level-2 codes
   without flag bit 2, all from the previous image (every pixel once).
   scratch (dev) >= fic_decode_workspace_bytes(g1). */
fic_status fic_decode_quadtree(fic_ctx *ctx, const fic_code *codes1, const fic_geom *g1,
                               const fic_code *codes2, const fic_geom *g2, int32_t max_iters,
                               const uint8_t *init, uint8_t *out, void *scratch,
                               size_t scratch_bytes, int32_t *iters_done, void *stream);

/* ------------------------------------------------------------------------
 * Autotuning of the persistent search (the uneven per-range pools of Sec.
 * 3.1 make the work per range vary widely).
 * Each encode picks, ON THE DEVICE, two parameters of its work list from a
 * table row of the context, indexed by the image's pool-fraction bucket
 * (0: exhaustive; pooled images 1 + floor(-log2 f) clamped to 1..5, f = the
 * sum of the searched ranges' pool sizes / (R * D)):
 *   chunk_log2  columns per work item = 2^chunk_log2, 11..16;
 *   flush_at    early flush of a wave's queue of passing cells once it holds
 *               at least this many (0 = only when full), 0..256;
 *   xcd         1: a single-image search takes its work items from one
 *               queue per XCD (the column chunks c = x mod 8 on XCD x, so
 *               each XCD's L2 streams an eighth of the domain columns;
 *               waves take from other queues once theirs is empty); 0: one
 *               queue in chunk order. Batches of several images always use
 *               one queue (a batch of one image follows its row).
 * A row serves one (range size B, floor(log2 D)) class; classes without a
 * row use the built-in defaults (exhaustive 2^14, pooled 2^12; flush 64 at
 * B = 8, else 0; xcd 0). Every choice gives the same codes.
 *
 * fic_autotune: for the images described by descs (each with its geometry
 * and tolerance, codes written to descs[i].codes), group them by (B,
 * floor(log2 D), bucket) and, per group, time encodes of each image alone
 * (classify, pool, search, finalize; the time taken is the search launch's,
 * from events around it, best of `reps`) of candidate rows by
 * coordinate descent (chunk_log2 over 11..16, then flush_at over 0, 16, 32, 64,
 * 128, then xcd), keep the winner only if a final interleaved re-measurement still has
 * it faster than the starting row, and store it in the context. BLOCKS THE
 * HOST (event synchronisation); not for stream capture. Recorded batch graphs
 * are dropped. report (host, nullable) receives up to report_cap entries, one
 * per group; *report_count (nullable) the number of entries.
 * When the images include both 4x4 and 8x8 ranges and ws also holds their
 * whole batch (>= fic_batch_workspace_bytes(n_images, descs)), the tuner
 * also times the batch with one combined persistent search and with one
 * search per range size (best of 3 each) and keeps the faster for later
 * batches; its report entry has range_size 0, flush_at 1 when separate
 * launches won, base_ms the combined time and tuned_ms the kept one.
 *   ws  (dev) >= fic_autotune_workspace_bytes(n_images, descs) (the largest
 *       single-image batch workspace).
 * fic_tune_save / fic_tune_load: the context's rows and batch launch choice
 * ("batch_separate": 0 or 1; optional on load, 0 when absent) as a JSON file
 * (host path) tagged with the device's gcnArchName and fic_kernel_hash(); load
 * replaces the rows, answers FIC_ERR_UNSUPPORTED (rows unchanged) for a file
 * written for another architecture or other kernels, FIC_ERR_INVALID_ARG for
 * an unreadable or malformed one. fic_create loads the file named by the
 * environment variable FIC_TUNE_CACHE when it matches.
 * fic_tune_reset: back to the defaults.
 * fic_tune_query: the (chunk_log2, flush_at, xcd) an encode of geometry g
 * would use (pool_fraction as above, ignored when pooled = 0; xcd nullable).
 * fic_kernel_hash: static string identifying the kernel sources of this
 * build.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t range_size, dlog2, bucket, images;   /* the tuning class         */
    int32_t chunk_log2, flush_at, xcd;           /* chosen                   */
    int32_t base_chunk_log2, base_flush_at, base_xcd;   /* the row it started from */
    float base_ms, tuned_ms;   /* summed search times of the class's images */
} fic_tune_entry;
size_t fic_autotune_workspace_bytes(int32_t n_images, const fic_image_desc *descs);
fic_status fic_autotune(fic_ctx *ctx, int32_t n_images, const fic_image_desc *descs,
                        void *ws, size_t ws_bytes, int32_t reps,
                        fic_tune_entry *report /* host */, int32_t report_cap,
                        int32_t *report_count /* host */, void *stream);
fic_status fic_tune_save(fic_ctx *ctx, const char *path);
fic_status fic_tune_load(fic_ctx *ctx, const char *path);
fic_status fic_tune_reset(fic_ctx *ctx);
fic_status fic_tune_query(fic_ctx *ctx, const fic_geom *g, int32_t pooled, double pool_fraction,
                          int32_t *chunk_log2 /* host */, int32_t *flush_at /* host */,
                          int32_t *xcd /* host, nullable */);
const char *fic_kernel_hash(void);

#ifdef __cplusplus
}
#endif
#endif /* FIC_H */

/*
 * fic_oracle.c -- CPU oracle for the PIFS range-domain matching search.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously-correct
 * reference that the GPU path is checked against. Only the test suite, the
 * package's smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never links, calls or falls back to it. It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (Revathy & Jayamohan, "Dynamic Domain Classification for
 * Fractal Image Compression"):
 *   - Sec. 1 / Sec. 2: the image is cut into non-overlapping B x B range
 *     blocks; candidate domains are the overlapping 2B x 2B blocks, shrunk to
 *     B x B ("resizing") and mapped onto the range by a geometric transform
 *     (the 8 square isometries) and an intensity transform (contrast s and
 *     brightness o). The best-matching domain per range is kept.
 *   - Sec. 2, Table 1: the range / domain counts of that lattice.
 *   - Sec. 3.1: each block is classified by its local fractal dimension,
 *     estimated by differential box counting (the box-counting limit
 *     equation, estimator of Sarkar & Chaudhuri, ref. [9]); a range only
 *     searches the domains whose dimension lies inside the fractal-distance
 *     window d_r - D_f <= d_d <= d_r + D_f, with D_f = (F_m - F_l) / 3 when no
 *     tolerance is given.
 *   - Sec. 1: decoding iterates the stored maps from an arbitrary start image.
 *
 * Readings of what the paper leaves open (the same ones the GPU path takes):
 *   intensity map  r' = (k/16) * (T_q dbar - mean dbar) + 2j, k in [-16,15],
 *                  j in [0,127]; dbar = 2x2 SUM / 4 (sums D kept as integers);
 *   isometries     T_q(d)[i][j] = d[src], src per q listed in iso_src();
 *   selection      minimum SSE; ties to the lowest (domain, isometry), then
 *                  the smaller |k|, then the smaller k, then the smaller j;
 *   empty pool     a DC-only code (domain 0, isometry 0, k = 0), flag bit 0;
 *   DBC            box sizes s = 2,4,..,M, box height h = s*256/M,
 *                  n_s = floor(max/h) - floor(min/h) + 1, FD = least-squares
 *                  slope of log N_s against log(M/s);
 *   window         |fd_d - fd_r| <= tol + 1e-9 evaluated in fp64.
 *
 * Precision: every search quantity is an exact 64-bit integer (scaled by
 * 4096 * n so the quantized s and o stay integral); fractal dimensions are
 * fp64. The error of a code is reported as E = 4096 * n * SSE (exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Geometry: Sec. 2 and Table 1.                                           */
/* ---------------------------------------------------------------------- */

/* Non-overlapping B x B ranges, raster order. */
int64_t fico_num_ranges(int32_t h, int32_t w, int32_t b)
{
    if (b <= 0 || h < b || w < b) return 0;
    return (int64_t)(h / b) * (int64_t)(w / b);
}

static int32_t dom_cols(int32_t w, int32_t b, int32_t t) { return (w - 2 * b) / t + 1; }
static int32_t dom_rows(int32_t h, int32_t b, int32_t t) { return (h - 2 * b) / t + 1; }

/* Overlapping 2B x 2B domains whose top-left corner is at (t*a, t*c) and that
   lie fully inside the image; index = a * cols + c. */
int64_t fico_num_domains(int32_t h, int32_t w, int32_t b, int32_t t)
{
    if (b <= 0 || t <= 0 || h < 2 * b || w < 2 * b) return 0;
    return (int64_t)dom_rows(h, b, t) * (int64_t)dom_cols(w, b, t);
}

/* ---------------------------------------------------------------------- */
/* The 8 square isometries ("rotation", Sec. 1): T_q(d)[i][j] = d[si][sj].  */
/* ---------------------------------------------------------------------- */
static void iso_src(int q, int b, int i, int j, int *si, int *sj)
{
    switch (q) {
    case 0: *si = i;         *sj = j;         break; /* identity          */
    case 1: *si = b - 1 - j; *sj = i;         break; /* rotate 90 cw      */
    case 2: *si = b - 1 - i; *sj = b - 1 - j; break; /* rotate 180        */
    case 3: *si = j;         *sj = b - 1 - i; break; /* rotate 270 cw     */
    case 4: *si = i;         *sj = b - 1 - j; break; /* mirror left-right */
    case 5: *si = b - 1 - i; *sj = j;         break; /* mirror up-down    */
    case 6: *si = j;         *sj = i;         break; /* transpose         */
    default:*si = b - 1 - j; *sj = b - 1 - i; break; /* anti-transpose    */
    }
}

/* dst = T_q(src) for a b x b block of int64 values (row-major). */
void fico_iso_apply(int32_t q, int32_t b, const int64_t *src, int64_t *dst)
{
    for (int i = 0; i < b; ++i)
        for (int j = 0; j < b; ++j) {
            int si, sj;
            iso_src(q, b, i, j, &si, &sj);
            dst[i * b + j] = src[si * b + sj];
        }
}

/* ---------------------------------------------------------------------- */
/* Local fractal dimension by differential box counting (Sec. 3.1, the     */
/* box-counting equation, estimator of ref. [9]).                          */
/* ---------------------------------------------------------------------- */

/* FD of the M x M block with top-left (y0, x0). counts (nullable) receives
   N_s for s = 2, 4, ..., M in that order. */
double fico_dbc_fd(const uint8_t *img, int32_t pitch, int32_t y0, int32_t x0,
                   int32_t m, int64_t *counts)
{
    double xs[8], ys[8];
    int np = 0;
    for (int s = 2; s <= m; s *= 2) {
        int h = s * 256 / m;                 /* box height, G = 256 levels */
        int64_t n_s = 0;
        for (int cy = 0; cy < m; cy += s)
            for (int cx = 0; cx < m; cx += s) {
                int mn = 255, mx = 0;
                for (int y = 0; y < s; ++y)
                    for (int x = 0; x < s; ++x) {
                        int g = img[(int64_t)(y0 + cy + y) * pitch + (x0 + cx + x)];
                        if (g < mn) mn = g;
                        if (g > mx) mx = g;
                    }
                n_s += mx / h - mn / h + 1;  /* boxes spanned by the cell */
            }
        if (counts) counts[np] = n_s;
        xs[np] = log((double)m / (double)s);
        ys[np] = log((double)n_s);
        ++np;
    }
    /* least-squares slope of log N_s on log(1/r), r = s/M */
    double mx_ = 0.0, my_ = 0.0;
    for (int i = 0; i < np; ++i) { mx_ += xs[i]; my_ += ys[i]; }
    mx_ /= np; my_ /= np;
    double sxy = 0.0, sxx = 0.0;
    for (int i = 0; i < np; ++i) {
        sxy += (xs[i] - mx_) * (ys[i] - my_);
        sxx += (xs[i] - mx_) * (xs[i] - mx_);
    }
    return sxy / sxx;
}

/* FD of every M x M block at step `step` (ranges: M = B, step = B; domains:
   M = 2B, step = t), raster order over block positions. */
void fico_fd_blocks(const uint8_t *img, int32_t h, int32_t w, int32_t pitch,
                    int32_t m, int32_t step, double *fd, int32_t nthreads)
{
    int32_t rows = (h - m) / step + 1, cols = (w - m) / step + 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int32_t a = 0; a < rows; ++a)
        for (int32_t c = 0; c < cols; ++c)
            fd[(int64_t)a * cols + c] =
                fico_dbc_fd(img, pitch, a * step, c * step, m, NULL);
}

/* The window half-width (Sec. 3.1): a given tolerance, or the fractal
   distance D_f = (F_m - F_l) / 3 over the domain set when tol < 0. */
double fico_resolve_tol(double tol, const double *fd_dom, int64_t nd)
{
    if (!(tol < 0.0)) return tol;          /* also passes NaN and +inf */
    double fmax = -INFINITY, fmin = INFINITY;
    for (int64_t i = 0; i < nd; ++i) {
        if (fd_dom[i] > fmax) fmax = fd_dom[i];
        if (fd_dom[i] < fmin) fmin = fd_dom[i];
    }
    return (fmax - fmin) / 3.0;
}

/* Membership of one domain in one range's pool (Sec. 3.1 window). */
static int in_pool(double fd_r, double fd_d, double tol)
{
    return fabs(fd_d - fd_r) <= tol + 1e-9;
}

/* ---------------------------------------------------------------------- */
/* Quantized least-squares fit of one (range, domain, isometry) pair.       */
/* ---------------------------------------------------------------------- */

/* With s = k/16 and o = 2j, 4096*n*SSE splits exactly into
      F(k) + 4096*(Sr - 2*n*j)^2,
      F(k) = 4096*Srr' - 128*k*Srd' + k^2*Sdd',
   Srr' = n*sum r^2 - (sum r)^2, Sdd' = n*sum D^2 - (sum D)^2,
   Srd' = n*sum r*T(D) - sum r * sum D (all exact integers). The oracle scans
   every k on the 5-bit grid rather than solving for it. */
static int64_t best_k(int64_t srr, int64_t srd, int64_t sdd, int32_t *k_out)
{
    int64_t best = 0;
    int32_t bk = 0;
    int first = 1;
    for (int32_t k = -16; k <= 15; ++k) {
        int64_t f = 4096 * srr - 128 * (int64_t)k * srd + (int64_t)k * k * sdd;
        int better = first || f < best ||
                     (f == best && (abs(k) < abs(bk) || (abs(k) == abs(bk) && k < bk)));
        if (better) { best = f; bk = k; first = 0; }
    }
    *k_out = bk;
    return best;
}

/* Brightness index: the j on the 7-bit grid closest to the range mean. */
static int32_t best_j(int64_t sr, int32_t n, int64_t *cost)
{
    int32_t bj = 0;
    int64_t bc = -1;
    for (int32_t j = 0; j <= 127; ++j) {
        int64_t e = sr - 2 * (int64_t)n * j;
        int64_t c = 4096 * e * e;
        if (bc < 0 || c < bc) { bc = c; bj = j; }
    }
    *cost = bc;
    return bj;
}

typedef struct {
    const uint8_t *img;
    int32_t h, w, pitch, b, t, n, dcols, rcols;
    int64_t nd;
    int16_t *dsum;     /* nd x n downsampled domains (2x2 sums, 0..1020) */
    int64_t *dsd;      /* sum D   per domain */
    int64_t *dsdd;     /* sum D^2 per domain */
} ctx_t;

static void range_pixels(const ctx_t *c, int64_t r, int64_t *px)
{
    int32_t ry = (int32_t)(r / c->rcols), rx = (int32_t)(r % c->rcols);
    for (int i = 0; i < c->b; ++i)
        for (int j = 0; j < c->b; ++j)
            px[i * c->b + j] = c->img[(int64_t)(ry * c->b + i) * c->pitch + rx * c->b + j];
}

static void build_domains(ctx_t *c)
{
    int32_t b = c->b, n = c->n;
    c->dsum = (int16_t *)malloc((size_t)c->nd * n * sizeof(int16_t));
    c->dsd = (int64_t *)malloc((size_t)c->nd * sizeof(int64_t));
    c->dsdd = (int64_t *)malloc((size_t)c->nd * sizeof(int64_t));
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t d = 0; d < c->nd; ++d) {
        int32_t y = (int32_t)(d / c->dcols) * c->t, x = (int32_t)(d % c->dcols) * c->t;
        int64_t s = 0, ss = 0;
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                const uint8_t *p = c->img + (int64_t)(y + 2 * i) * c->pitch + x + 2 * j;
                int v = p[0] + p[1] + p[c->pitch] + p[c->pitch + 1];
                c->dsum[d * n + i * b + j] = (int16_t)v;
                s += v;
                ss += (int64_t)v * v;
            }
        c->dsd[d] = s;
        c->dsdd[d] = ss;
    }
}

static void free_domains(ctx_t *c)
{
    free(c->dsum); free(c->dsd); free(c->dsdd);
}

/* Exact F and k of one pair, the isometry applied to the DOMAIN. */
static int64_t pair_f(const ctx_t *c, const int64_t *rpx, int64_t sr, int64_t srr,
                      int64_t d, int q, const int32_t *perm, int32_t *k_out)
{
    const int16_t *dd = c->dsum + d * c->n;
    int64_t cross = 0;
    for (int i = 0; i < c->n; ++i) cross += rpx[i] * (int64_t)dd[perm[q * c->n + i]];
    int64_t n = c->n;
    int64_t srr_ = n * srr - sr * sr;
    int64_t sdd_ = n * c->dsdd[d] - c->dsd[d] * c->dsd[d];
    int64_t srd_ = n * cross - sr * c->dsd[d];
    return best_k(srr_, srd_, sdd_, k_out);
}

static int32_t *iso_tables(int32_t b)
{
    int32_t n = b * b;
    int32_t *perm = (int32_t *)malloc((size_t)8 * n * sizeof(int32_t));
    for (int q = 0; q < 8; ++q)
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                int si, sj;
                iso_src(q, b, i, j, &si, &sj);
                perm[q * n + i * b + j] = si * b + sj;   /* (T_q D)_ij = D[perm] */
            }
    return perm;
}

/*
 * Encode the selected ranges (all when sel == NULL) of one image.
 * Exhaustive search when fd_range or fd_dom is NULL; otherwise the dynamic
 * per-range pool of Sec. 3.1 with half-width tol (already resolved).
 * Outputs are indexed like `sel` (or by range index when sel == NULL).
 * Returns 0, or -1 on invalid geometry.
 */
int32_t fico_encode(const uint8_t *img, int32_t h, int32_t w, int32_t pitch,
                    int32_t b, int32_t t,
                    const double *fd_range, const double *fd_dom, double tol,
                    const int64_t *sel, int64_t nsel,
                    int32_t *dom_out, int32_t *iso_out, int32_t *k_out, int32_t *j_out,
                    int32_t *flags_out, int64_t *err_out, int64_t *f_out,
                    int64_t *pool_out, int32_t nthreads)
{
    if (b <= 0 || t <= 0 || h % b || w % b || h < 2 * b || w < 2 * b || pitch < w)
        return -1;
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.img = img; c.h = h; c.w = w; c.pitch = pitch; c.b = b; c.t = t; c.n = b * b;
    c.dcols = dom_cols(w, b, t);
    c.rcols = w / b;
    c.nd = fico_num_domains(h, w, b, t);
    int64_t nr = fico_num_ranges(h, w, b);
    if (!sel) nsel = nr;
    int pool_mode = fd_range && fd_dom;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    build_domains(&c);
    int32_t *perm = iso_tables(b);

#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t r = sel ? sel[s] : s;
        int64_t rpx[1024];
        range_pixels(&c, r, rpx);
        int64_t sr = 0, srr = 0;
        for (int i = 0; i < c.n; ++i) { sr += rpx[i]; srr += rpx[i] * rpx[i]; }
        int64_t best_f = 0, pool = 0;
        int64_t best_d = -1;
        int32_t best_q = 0, best_kq = 0;
        for (int64_t d = 0; d < c.nd; ++d) {
            if (pool_mode && !in_pool(fd_range[r], fd_dom[d], tol)) continue;
            ++pool;
            for (int q = 0; q < 8; ++q) {
                int32_t kq;
                int64_t f = pair_f(&c, rpx, sr, srr, d, q, perm, &kq);
                /* domains ascend and isometries ascend, so a strict
                   improvement is the lexicographic (F, d, q) minimum */
                if (best_d < 0 || f < best_f) {
                    best_f = f; best_d = d; best_q = q; best_kq = kq;
                }
            }
        }
        int64_t jcost;
        int32_t jq = best_j(sr, c.n, &jcost);
        int32_t flags = 0;
        if (best_d < 0) {                       /* empty pool: DC-only code */
            int64_t srr_ = (int64_t)c.n * srr - sr * sr;
            best_d = 0; best_q = 0; best_kq = 0;
            best_f = 4096 * srr_;
            flags = 1;
        }
        dom_out[s] = (int32_t)best_d;
        iso_out[s] = best_q;
        k_out[s] = best_kq;
        j_out[s] = jq;
        flags_out[s] = flags;
        f_out[s] = best_f;
        err_out[s] = best_f + jcost;
        if (pool_out) pool_out[s] = pool;
    }
    free(perm);
    free_domains(&c);
    return 0;
}

/* F and k of a single (range, domain, isometry) pair, for pinned cases. */
int64_t fico_pair_f(const uint8_t *img, int32_t h, int32_t w, int32_t pitch,
                    int32_t b, int32_t t, int64_t r, int64_t d, int32_t q,
                    int32_t *k_out)
{
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.img = img; c.h = h; c.w = w; c.pitch = pitch; c.b = b; c.t = t; c.n = b * b;
    c.dcols = dom_cols(w, b, t);
    c.rcols = w / b;
    c.nd = fico_num_domains(h, w, b, t);
    build_domains(&c);
    int32_t *perm = iso_tables(b);
    int64_t rpx[1024];
    range_pixels(&c, r, rpx);
    int64_t sr = 0, srr = 0;
    for (int i = 0; i < c.n; ++i) { sr += rpx[i]; srr += rpx[i] * rpx[i]; }
    int64_t f = pair_f(&c, rpx, sr, srr, d, q, perm, k_out);
    free(perm);
    free_domains(&c);
    return f;
}

/* ---------------------------------------------------------------------- */
/* Decoding (Sec. 1): iterate the maps from a start image.                  */
/* ---------------------------------------------------------------------- */

static int64_t floor_div(int64_t a, int64_t d)
{
    int64_t q = a / d;
    if ((a % d) != 0 && ((a < 0) != (d < 0))) --q;
    return q;
}

/* One simultaneous (Jacobi) sweep: every range pixel becomes the rounded
   value of its map applied to the current image. Returns #changed pixels. */
static int64_t decode_sweep(const int32_t *dom, const int32_t *iso, const int32_t *kq,
                            const int32_t *jq, const uint8_t *skip, int32_t h, int32_t w,
                            int32_t b, int32_t t, const uint8_t *cur, uint8_t *nxt)
{
    int32_t n = b * b, rcols = w / b, dcols = dom_cols(w, b, t);
    int64_t nr = fico_num_ranges(h, w, b), changed = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : changed)
#endif
    for (int64_t r = 0; r < nr; ++r) {
        if (skip && skip[r]) continue;   /* its pixels belong to the other level */
        int64_t dsum[1024], tdsum[1024];
        int32_t dy = (dom[r] / dcols) * t, dx = (dom[r] % dcols) * t;
        int64_t sd = 0;
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                const uint8_t *p = cur + (int64_t)(dy + 2 * i) * w + dx + 2 * j;
                dsum[i * b + j] = p[0] + p[1] + p[w] + p[w + 1];
                sd += dsum[i * b + j];
            }
        fico_iso_apply(iso[r], b, dsum, tdsum);
        int32_t ry = (int32_t)(r / rcols) * b, rx = (int32_t)(r % rcols) * b;
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                /* round( (k/16) * (TD/4 - SD/(4n)) + 2j ) */
                int64_t num = (int64_t)kq[r] * (n * tdsum[i * b + j] - sd)
                            + 128 * (int64_t)n * jq[r] + 32 * (int64_t)n;
                int64_t v = floor_div(num, 64 * (int64_t)n);
                if (v < 0) v = 0;
                if (v > 255) v = 255;
                int64_t o = (int64_t)(ry + i) * w + rx + j;
                if (cur[o] != (uint8_t)v) ++changed;
                nxt[o] = (uint8_t)v;
            }
    }
    return changed;
}

/* Decode from `init` (all 128 when NULL) until a sweep changes nothing or
   max_iters sweeps ran. out: h x w (pitch w). */
int32_t fico_decode(const int32_t *dom, const int32_t *iso, const int32_t *kq,
                    const int32_t *jq, int32_t h, int32_t w, int32_t b, int32_t t,
                    int32_t max_iters, const uint8_t *init, uint8_t *out,
                    int32_t *iters_done, int32_t nthreads)
{
    if (b <= 0 || t <= 0 || h % b || w % b || h < 2 * b || w < 2 * b) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    size_t np = (size_t)h * w;
    uint8_t *a = (uint8_t *)malloc(np), *bb = (uint8_t *)malloc(np);
    if (init) memcpy(a, init, np); else memset(a, 128, np);
    int32_t it = 0;
    for (; it < max_iters; ) {
        int64_t ch = decode_sweep(dom, iso, kq, jq, NULL, h, w, b, t, a, bb);
        uint8_t *tmp = a; a = bb; bb = tmp;
        ++it;
        if (ch == 0) break;
    }
    memcpy(out, a, np);
    *iters_done = it;
    free(a); free(bb);
    return 0;
}

/* Two-level (quadtree) decode: each simultaneous sweep applies the level-1
   maps of the ranges that were not split (split1[r] == 0) and the level-2
   maps of the sub-ranges that were coded (coded2[r] != 0); together they
   cover every pixel once. Same stop rule as fico_decode. */
int32_t fico_decode_quadtree(const int32_t *dom1, const int32_t *iso1, const int32_t *k1,
                             const int32_t *j1, const uint8_t *split1, int32_t b1, int32_t t1,
                             const int32_t *dom2, const int32_t *iso2, const int32_t *k2,
                             const int32_t *j2, const uint8_t *coded2, int32_t b2, int32_t t2,
                             int32_t h, int32_t w, int32_t max_iters, const uint8_t *init,
                             uint8_t *out, int32_t *iters_done, int32_t nthreads)
{
    if (b1 <= 0 || b2 <= 0 || b1 != 2 * b2 || t1 <= 0 || t2 <= 0 || h % b1 || w % b1 ||
        h < 2 * b1 || w < 2 * b1)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    size_t np = (size_t)h * w;
    int64_t n2 = fico_num_ranges(h, w, b2);
    uint8_t *skip2 = (uint8_t *)malloc((size_t)n2);
    for (int64_t r = 0; r < n2; ++r) skip2[r] = coded2[r] ? 0 : 1;
    uint8_t *a = (uint8_t *)malloc(np), *bb = (uint8_t *)malloc(np);
    if (init) memcpy(a, init, np); else memset(a, 128, np);
    int32_t it = 0;
    for (; it < max_iters; ) {
        int64_t ch = decode_sweep(dom1, iso1, k1, j1, split1, h, w, b1, t1, a, bb);
        ch += decode_sweep(dom2, iso2, k2, j2, skip2, h, w, b2, t2, a, bb);
        uint8_t *tmp = a; a = bb; bb = tmp;
        ++it;
        if (ch == 0) break;
    }
    memcpy(out, a, np);
    *iters_done = it;
    free(a); free(bb); free(skip2);
    return 0;
}

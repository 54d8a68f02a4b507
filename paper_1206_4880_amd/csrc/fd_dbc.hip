// fd_dbc.hip -- local fractal dimension of image blocks by differential box
// counting (Sec. 3.1: the box-counting definition of the dimension, estimated
// with the differential box-counting rule of ref. [9]).
//
// For an M x M block: box sizes s = 2, 4, ..., M; gray axis cut into boxes
// of height h = s*256/M; each s x s cell spans floor(max/h) - floor(min/h) + 1
// boxes; N_s sums that over the (M/s)^2 cells; the dimension is the
// least-squares slope of log N_s against log(M/s). (s = M always gives
// N_M = 1.)
//
// One workgroup owns a tile of block origins. It stages the pixel patch the
// tile covers in LDS once, then builds min/max pyramids over it in LDS
// (level s holds the s x s cell extremes at every patch position, built from
// four level-s/2 entries), so overlapping domains (step 1) share every cell
// instead of re-reading 2B x 2B pixels each. Counts are exact integers; the
// slope is fp64, the fp32 copy its rounding.
#include "fic_internal.h"

namespace fic {

namespace {

constexpr int kPatch = 64;          // max patch side staged in LDS
constexpr int kThreads = 256;

struct MinMax { uint8_t mn, mx; };

template <int M>
__global__ __launch_bounds__(kThreads) void k_fd_dbc(const uint8_t *__restrict__ img,
                                                     int32_t h, int32_t w, int32_t pitch,
                                                     int32_t step, int32_t rows, int32_t cols,
                                                     int32_t tile, double *__restrict__ fd64,
                                                     float *__restrict__ fd32)
{
    // levels s = 2 .. M/2 (at most 4 levels for M = 32)
    constexpr int NL = (M == 4) ? 1 : (M == 8) ? 2 : (M == 16) ? 3 : 4;
    __shared__ uint8_t px[kPatch * kPatch];
    __shared__ MinMax lv[NL][kPatch * kPatch];

    const int a0 = blockIdx.y * tile, c0 = blockIdx.x * tile;
    const int ta = min(tile, rows - a0), tc = min(tile, cols - c0);
    const int py = (ta - 1) * step + M, pxw = (tc - 1) * step + M;
    const int y0 = a0 * step, x0 = c0 * step;

    for (int i = threadIdx.x; i < py * pxw; i += kThreads) {
        int yy = i / pxw, xx = i - yy * pxw;
        px[yy * kPatch + xx] = img[(int64_t)(y0 + yy) * pitch + (x0 + xx)];
    }
    __syncthreads();
    // level 0: 2 x 2 cells at every position
    for (int i = threadIdx.x; i < (py - 1) * (pxw - 1); i += kThreads) {
        int yy = i / (pxw - 1), xx = i - yy * (pxw - 1);
        const uint8_t *p = px + yy * kPatch + xx;
        uint8_t a = p[0], b = p[1], c = p[kPatch], d = p[kPatch + 1];
        MinMax m;
        m.mn = min(min(a, b), min(c, d));
        m.mx = max(max(a, b), max(c, d));
        lv[0][yy * kPatch + xx] = m;
    }
    __syncthreads();
    // level l: (2^(l+1)) cells from four level l-1 cells offset by s/2
#pragma unroll
    for (int l = 1; l < NL; ++l) {
        const int s = 2 << l, hs = s >> 1;
        const int ny = py - s + 1, nx = pxw - s + 1;
        for (int i = threadIdx.x; i < ny * nx; i += kThreads) {
            int yy = i / nx, xx = i - yy * nx;
            const MinMax *q = lv[l - 1] + yy * kPatch + xx;
            MinMax a = q[0], b = q[hs], c = q[hs * kPatch], d = q[hs * kPatch + hs];
            MinMax m;
            m.mn = min(min(a.mn, b.mn), min(c.mn, d.mn));
            m.mx = max(max(a.mx, b.mx), max(c.mx, d.mx));
            lv[l][yy * kPatch + xx] = m;
        }
        __syncthreads();
    }

    const int t = threadIdx.x;
    if (t >= tile * tile) return;
    const int la = t / tile, lc = t - la * tile;
    if (la >= ta || lc >= tc) return;
    const int wy = la * step, wx = lc * step;

    double xs[NL + 1], ys[NL + 1];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int s = 2 << l;
        const int hshift = __builtin_ctz((unsigned)(s * 256 / M));   // h is a power of two
        const int cells = M / s;
        int64_t ns = 0;
        for (int ci = 0; ci < cells; ++ci)
            for (int cj = 0; cj < cells; ++cj) {
                MinMax m = lv[l][(wy + ci * s) * kPatch + (wx + cj * s)];
                ns += (m.mx >> hshift) - (m.mn >> hshift) + 1;
            }
        xs[l] = log2((double)(M / s));
        ys[l] = log2((double)ns);
    }
    xs[NL] = 0.0;        // s = M: one cell spanning one box
    ys[NL] = 0.0;
    double mx = 0.0, my = 0.0;
#pragma unroll
    for (int l = 0; l <= NL; ++l) { mx += xs[l]; my += ys[l]; }
    mx /= (NL + 1);
    my /= (NL + 1);
    double sxy = 0.0, sxx = 0.0;
#pragma unroll
    for (int l = 0; l <= NL; ++l) {
        sxy += (xs[l] - mx) * (ys[l] - my);
        sxx += (xs[l] - mx) * (xs[l] - mx);
    }
    const double fd = sxy / sxx;
    const int64_t o = (int64_t)(a0 + la) * cols + (c0 + lc);
    fd64[o] = fd;
    if (fd32) fd32[o] = (float)fd;
}

template <int M>
hipError_t launch_m(const uint8_t *img, int32_t h, int32_t w, int32_t pitch, int32_t step,
                    double *fd64, float *fd32, hipStream_t s)
{
    const int32_t rows = (h - M) / step + 1, cols = (w - M) / step + 1;
    // largest tile (<= 16 origins per side) whose patch fits the LDS staging
    int tile = (kPatch - M) / step + 1;
    if (tile > 16) tile = 16;
    if (tile < 1) tile = 1;
    dim3 grid((cols + tile - 1) / tile, (rows + tile - 1) / tile);
    hipLaunchKernelGGL(k_fd_dbc<M>, grid, dim3(kThreads), 0, s, img, h, w, pitch, step, rows,
                       cols, tile, fd64, fd32);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fd_classify(const uint8_t *img, int32_t h, int32_t w, int32_t pitch,
                              int32_t block, int32_t step, double *fd64, float *fd32,
                              hipStream_t s, const Tracer *tr)
{
    hipError_t e;
    trace(tr, FIC_STAGE_CLASSIFY, 1, s);
    switch (block) {
    case 4: e = launch_m<4>(img, h, w, pitch, step, fd64, fd32, s); break;
    case 8: e = launch_m<8>(img, h, w, pitch, step, fd64, fd32, s); break;
    case 16: e = launch_m<16>(img, h, w, pitch, step, fd64, fd32, s); break;
    case 32: e = launch_m<32>(img, h, w, pitch, step, fd64, fd32, s); break;
    default: e = hipErrorInvalidValue; break;
    }
    trace(tr, FIC_STAGE_CLASSIFY, 0, s);
    return e;
}

}  // namespace fic

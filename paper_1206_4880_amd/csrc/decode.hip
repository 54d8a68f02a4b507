// decode.hip -- decoding by iteration of the stored maps (Sec. 1: the
// transformations are applied to an arbitrary start image; a limited number
// of iterations converges to the attractor).
//
// One sweep recomputes every range simultaneously from the previous image
// (Jacobi): pixel (u, v) of range r becomes
//   clamp(floor((k*(n*(T_q D')_uv - sum D') + 128*n*j + 32*n) / (64*n)), 0, 255)
// i.e. s*((T_q D')/4 - mean(D')/4) + o rounded half up, D' the 2x2 sums of the
// code's domain in the current image. Integer arithmetic, so every sweep is
// exact. Sweeps stop after the first one that changes nothing; the stop test
// lives on the device (a flag later sweeps read), so the host never waits.
#include "fic_internal.h"

namespace fic {

namespace {

constexpr int kMaxIters = 1024;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ void k_decode_init(const uint8_t *__restrict__ init, int64_t np, uint8_t *__restrict__ buf0,
                              uint32_t *__restrict__ flags, int32_t nflags, int32_t *iters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) buf0[i] = init ? init[i] : (uint8_t)128;
    if (i < nflags) flags[i] = 0u;
    if (i == 0) *iters = 0;
}

// Codes whose flags meet skip_flags write nothing (in a two-level decode
// their pixels belong to the other level).
// 256 threads a block (one per pixel of 256/n ranges); 1024 for 32x32 ranges
// (16x16 codes decoded at twice the size).
template <int B> constexpr int sweep_threads() { return B == 32 ? 1024 : 256; }

template <int B>
__global__ __launch_bounds__(sweep_threads<B>()) void k_decode_sweep(const fic_code *__restrict__ codes, Geom g,
                                                      uint8_t skip_flags,
                                                      const uint8_t *__restrict__ cur,
                                                      uint8_t *__restrict__ nxt,
                                                      uint32_t *__restrict__ changed,
                                                      const uint32_t *__restrict__ done)
{
    constexpr int n = B * B, RPB = sweep_threads<B>() / n;   // ranges per block
    __shared__ int32_t sums[RPB];
    __shared__ uint32_t nchg;
    if (*done) return;
    const int tid = threadIdx.x, lr = tid / n, i = tid % n;
    const int64_t r = (int64_t)blockIdx.x * RPB + lr;
    if (tid < RPB) sums[tid] = 0;
    if (tid == 0) nchg = 0;
    __syncthreads();
    fic_code c;
    c.domain = 0; c.iso = 0; c.s_idx = 0; c.o_idx = 0; c.flags = 0;
    if (r < g.R) c = codes[r];
    const bool inside = r < g.R && !(c.flags & skip_flags);
    // a code naming a domain or isometry outside the lattice is not applied
    // (its range decodes to 0) rather than read outside the image
    const bool valid = inside && c.domain < (uint64_t)g.D && c.iso < 8;
    int dv = 0;
    int u = i / B, v = i % B;
    if (valid) {
        const int dy = (int)(c.domain / g.dcols) * g.t, dx = (int)(c.domain % g.dcols) * g.t;
        int si, sj;
        iso_src(c.iso, B, u, v, si, sj);
        const uint8_t *p = cur + (int64_t)(dy + 2 * si) * g.w + dx + 2 * sj;
        dv = p[0] + p[1] + p[g.w] + p[g.w + 1];
        atomicAdd(&sums[lr], dv);
    }
    __syncthreads();
    if (inside) {
        const int64_t num = (int64_t)c.s_idx * ((int64_t)n * dv - sums[lr]) +
                            128 * (int64_t)n * c.o_idx + 32 * (int64_t)n;
        const int64_t den = 64 * (int64_t)n;
        int64_t val = num >= 0 ? num / den : -((-num + den - 1) / den);
        val = !valid ? 0 : (val < 0 ? 0 : (val > 255 ? 255 : val));
        const int ry = (int)(r / g.rcols) * B, rx = (int)(r % g.rcols) * B;
        const int64_t o = (int64_t)(ry + u) * g.w + rx + v;
        if (cur[o] != (uint8_t)val) atomicAdd(&nchg, 1u);
        nxt[o] = (uint8_t)val;
    }
    __syncthreads();
    if (tid == 0 && nchg) atomicAdd(changed, nchg);
}

__global__ void k_decode_check(int32_t it, const uint32_t *__restrict__ changed,
                               uint32_t *__restrict__ done, int32_t *iters)
{
    if (threadIdx.x == 0 && !*done) {
        *iters = it + 1;
        if (changed[it] == 0) *done = 1;
    }
}

__global__ void k_decode_out(const uint8_t *__restrict__ b0, const uint8_t *__restrict__ b1,
                             int64_t np, const int32_t *__restrict__ iters, uint8_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) out[i] = ((*iters) & 1) ? b1[i] : b0[i];
}

template <int B>
hipError_t run_b(const Geom &g, const fic_code *codes, int32_t max_iters, const uint8_t *init,
                 uint8_t *out, void *ws, int32_t *iters, hipStream_t s, const Tracer *tr)
{
    trace(tr, FIC_STAGE_DECODE, 1, s);
    const int64_t np = (int64_t)g.h * g.w;
    char *w = (char *)ws;
    uint8_t *b0 = (uint8_t *)w;
    uint8_t *b1 = (uint8_t *)(w + align256(np));
    uint32_t *flags = (uint32_t *)(w + 2 * align256(np));   // [0..max) changed, [kMaxIters] done
    uint32_t *done = flags + kMaxIters;
    const int th = 256;
    const int64_t nfl = kMaxIters + 1;
    const int64_t nthr = np > nfl ? np : nfl;
    hipLaunchKernelGGL(k_decode_init, dim3((unsigned)((nthr + th - 1) / th)), dim3(th), 0, s, init,
                       np, b0, flags, (int32_t)nfl, iters);
    constexpr int RPB = sweep_threads<B>() / (B * B);
    const unsigned nb = (unsigned)((g.R + RPB - 1) / RPB);
    for (int it = 0; it < max_iters; ++it) {
        const uint8_t *src = (it & 1) ? b1 : b0;
        uint8_t *dst = (it & 1) ? b0 : b1;
        hipLaunchKernelGGL(k_decode_sweep<B>, dim3(nb), dim3(sweep_threads<B>()), 0, s, codes, g,
                           (uint8_t)0, src, dst, flags + it, done);
        hipLaunchKernelGGL(k_decode_check, dim3(1), dim3(64), 0, s, it, flags, done, iters);
    }
    hipLaunchKernelGGL(k_decode_out, dim3((unsigned)((np + th - 1) / th)), dim3(th), 0, s, b0, b1,
                       np, iters, out);
    trace(tr, FIC_STAGE_DECODE, 0, s);
    return hipGetLastError();
}

template <int B>
void sweep_b(const Geom &g, const fic_code *codes, uint8_t skip, const uint8_t *src, uint8_t *dst,
             uint32_t *changed, const uint32_t *done, hipStream_t s)
{
    constexpr int RPB = sweep_threads<B>() / (B * B);
    const unsigned nb = (unsigned)((g.R + RPB - 1) / RPB);
    hipLaunchKernelGGL(k_decode_sweep<B>, dim3(nb), dim3(sweep_threads<B>()), 0, s, codes, g, skip,
                       src, dst, changed, done);
}

void sweep(const Geom &g, const fic_code *codes, uint8_t skip, const uint8_t *src, uint8_t *dst,
           uint32_t *changed, const uint32_t *done, hipStream_t s)
{
    switch (g.b) {
    case 4: sweep_b<4>(g, codes, skip, src, dst, changed, done, s); break;
    case 8: sweep_b<8>(g, codes, skip, src, dst, changed, done, s); break;
    default: sweep_b<16>(g, codes, skip, src, dst, changed, done, s); break;
    }
}

}  // namespace

// Two-level decode: each sweep applies the level-1 codes that were not split
// (flag bit 1) and the level-2 codes that were coded (no flag bit 2), from
// the same image; together they write every pixel once.
hipError_t run_decode_quadtree(const Geom &g1, const fic_code *codes1, const Geom &g2,
                               const fic_code *codes2, int32_t max_iters, const uint8_t *init,
                               uint8_t *out, void *ws, int32_t *iters, hipStream_t s,
                               const Tracer *tr)
{
    trace(tr, FIC_STAGE_DECODE, 1, s);
    const int64_t np = (int64_t)g1.h * g1.w;
    char *w = (char *)ws;
    uint8_t *b0 = (uint8_t *)w;
    uint8_t *b1 = (uint8_t *)(w + align256(np));
    uint32_t *flags = (uint32_t *)(w + 2 * align256(np));
    uint32_t *done = flags + kMaxIters;
    const int th = 256;
    const int64_t nfl = kMaxIters + 1;
    const int64_t nthr = np > nfl ? np : nfl;
    hipLaunchKernelGGL(k_decode_init, dim3((unsigned)((nthr + th - 1) / th)), dim3(th), 0, s, init,
                       np, b0, flags, (int32_t)nfl, iters);
    for (int it = 0; it < max_iters; ++it) {
        const uint8_t *src = (it & 1) ? b1 : b0;
        uint8_t *dst = (it & 1) ? b0 : b1;
        sweep(g1, codes1, 2, src, dst, flags + it, done, s);
        sweep(g2, codes2, 4, src, dst, flags + it, done, s);
        hipLaunchKernelGGL(k_decode_check, dim3(1), dim3(64), 0, s, it, flags, done, iters);
    }
    hipLaunchKernelGGL(k_decode_out, dim3((unsigned)((np + th - 1) / th)), dim3(th), 0, s, b0, b1,
                       np, iters, out);
    trace(tr, FIC_STAGE_DECODE, 0, s);
    return hipGetLastError();
}

size_t decode_ws_bytes(const Geom &g)
{
    const int64_t np = (int64_t)g.h * g.w;
    return 2 * align256(np) + align256((size_t)(kMaxIters + 1) * 4);
}

int32_t decode_max_iters() { return kMaxIters; }

hipError_t run_decode(const Geom &g, const fic_code *codes, int32_t max_iters,
                      const uint8_t *init, uint8_t *out, void *ws, int32_t *iters, hipStream_t s,
                      const Tracer *tr)
{
    switch (g.b) {
    case 4: return run_b<4>(g, codes, max_iters, init, out, ws, iters, s, tr);
    case 8: return run_b<8>(g, codes, max_iters, init, out, ws, iters, s, tr);
    case 16: return run_b<16>(g, codes, max_iters, init, out, ws, iters, s, tr);
    case 32: return run_b<32>(g, codes, max_iters, init, out, ws, iters, s, tr);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fic

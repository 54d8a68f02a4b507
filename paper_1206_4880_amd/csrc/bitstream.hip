// bitstream.hip -- the stored code as a bit string (Sec. 1: per range the
// domain, the isometry, the contrast and the brightness are kept): range r's
// fields start at bit r*W of a little-endian string of 32-bit words, each
// field least significant bit first, in the order domain index (ceil(log2 D)
// bits, at least 1), isometry (3), k + 16 (5), j (7); W = that sum. The
// flags and the error are not stored.
#include "fic_internal.h"

namespace fic {

namespace {

__global__ void k_zero_words(uint32_t *__restrict__ w, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = 0u;
}

// One thread per range: its W <= 43 bits land in at most three words.
__global__ void k_pack(const fic_code *__restrict__ codes, int64_t R, int dbits, int64_t nwords,
                       uint32_t *__restrict__ words)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int W = dbits + 15;
    const fic_code c = codes[r];
    const u64 v = (u64)(c.domain & ((1ull << dbits) - 1ull)) | ((u64)(c.iso & 7u) << dbits) |
                  ((u64)((uint32_t)(c.s_idx + 16) & 31u) << (dbits + 3)) |
                  ((u64)(c.o_idx & 127u) << (dbits + 8));
    const int64_t bit = r * (int64_t)W;
    const int64_t i = bit >> 5;
    const int sh = (int)(bit & 31);
    // bits 0..31, 32..63, 64..95 of v << sh
    const uint32_t w0 = (uint32_t)(v << sh);
    const uint32_t w1 = sh ? (uint32_t)(v >> (32 - sh)) : (uint32_t)(v >> 32);
    const uint32_t w2 = sh ? (uint32_t)(v >> (64 - sh)) : 0u;
    if (w0) atomicOr(&words[i], w0);
    if (w1 && i + 1 < nwords) atomicOr(&words[i + 1], w1);
    if (w2 && i + 2 < nwords) atomicOr(&words[i + 2], w2);
}

__global__ void k_unpack(const uint32_t *__restrict__ words, int64_t nwords, int64_t R, int dbits,
                         fic_code *__restrict__ codes)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int W = dbits + 15;
    const int64_t bit = r * (int64_t)W;
    const int64_t i = bit >> 5;
    const int sh = (int)(bit & 31);
    const u64 w0 = words[i];
    const u64 w1 = i + 1 < nwords ? words[i + 1] : 0u;
    const u64 w2 = i + 2 < nwords ? words[i + 2] : 0u;
    u64 v = ((w1 << 32) | w0) >> sh;
    if (sh && W + sh > 64) v |= w2 << (64 - sh);
    v &= (1ull << W) - 1ull;
    fic_code c;
    c.domain = (uint32_t)(v & ((1ull << dbits) - 1ull));
    c.iso = (uint8_t)((v >> dbits) & 7u);
    c.s_idx = (int8_t)((int)((v >> (dbits + 3)) & 31u) - 16);
    c.o_idx = (uint8_t)((v >> (dbits + 8)) & 127u);
    c.flags = 0;
    c.err = 0;
    codes[r] = c;
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int code_dbits(int64_t D)
{
    int d = 1;
    while (d < 63 && ((int64_t)1 << d) < D) ++d;
    return d;
}

int64_t packed_words(const Geom &g)
{
    const int64_t W = code_dbits(g.D) + 15;
    return (g.R * W + 31) / 32;
}

hipError_t run_pack(const Geom &g, const fic_code *codes, uint32_t *words, hipStream_t s)
{
    const int64_t nw = packed_words(g);
    hipLaunchKernelGGL(k_zero_words, dim3(nblocks(nw)), dim3(256), 0, s, words, nw);
    hipLaunchKernelGGL(k_pack, dim3(nblocks(g.R)), dim3(256), 0, s, codes, g.R, code_dbits(g.D), nw,
                       words);
    return hipGetLastError();
}

hipError_t run_unpack(const Geom &g, const uint32_t *words, fic_code *codes, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack, dim3(nblocks(g.R)), dim3(256), 0, s, words, packed_words(g), g.R,
                       code_dbits(g.D), codes);
    return hipGetLastError();
}

}  // namespace fic

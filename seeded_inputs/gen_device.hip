/*
 * Device form of the packed boards of gen.c: the same counter-based
 * SplitMix64 draw for every cell (the definition is in gen.c's header), so a
 * board generated here equals the host one bit for bit.  It draws boards
 * straight into device memory, where a 65536 x 65536 board (4.3e9 cells)
 * takes milliseconds instead of seconds on the host.  Like gen.c it holds
 * none of the Life arithmetic.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// One thread per packed word: cell (r, c) is bit c mod 64 of word
// r * W + c / 64, alive iff the high half of the (r * cols + c + 1)-th
// output of the stream seeded with `key` is below `thr` (every cell alive
// when `all`); padding bits are 0.
__global__ void k_gen_packed(uint64_t key, uint32_t thr, int all, int64_t rows, int64_t cols,
                             int64_t W, uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * W) return;
  const int64_t r = i / W;
  const int64_t c0 = (i - r * W) * 64;
  const int64_t n = cols - c0 < 64 ? cols - c0 : 64;
  const uint64_t idx0 = (uint64_t)(r * cols + c0);
  uint64_t word = 0;
  for (int64_t b = 0; b < n; ++b) {
    const bool alive =
        all || (uint32_t)(mix64(key + (idx0 + (uint64_t)b + 1) * kGamma) >> 32) < thr;
    word |= (uint64_t)alive << b;
  }
  out[i] = word;
}

}  // namespace

/* Fills d_out (rows x ceil(cols / 64) uint64 words in device memory, row
 * stride W) with board (seed, board_id, rows, cols, p), asynchronously on
 * `stream` (a hipStream_t; NULL = the default stream).  Returns 0, -1 on
 * invalid sizes or a null pointer, -2 if the launch failed. */
extern "C" int si_gen_packed_device(uint64_t seed, uint64_t board_id, int64_t rows,
                                    int64_t cols, double p, uint64_t* d_out, void* stream) {
  if (rows <= 0 || cols <= 0 || !d_out) return -1;
  const uint64_t key = mix64(seed + kGamma) ^ mix64(board_id + 2 * kGamma);
  uint32_t thr = 0u;
  if (p >= 1.0)
    thr = 0xFFFFFFFFu;
  else if (p > 0.0)
    thr = (uint32_t)floor(p * 4294967296.0);
  const int64_t W = (cols + 63) / 64;
  const int64_t words = rows * W;
  const int block = 256;
  const int64_t grid = (words + block - 1) / block;
  if (grid > 0x7FFFFFFF) return -1;
  hipLaunchKernelGGL(k_gen_packed, dim3((uint32_t)grid), dim3(block), 0, (hipStream_t)stream,
                     key, thr, p >= 1.0 ? 1 : 0, rows, cols, W, d_out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

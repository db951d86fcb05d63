/*
 * Seeded synthetic boards for the Life step (shared by the oracle side and the
 * GPU side; it holds none of the Life arithmetic).
 *
 * Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014; finaliser constants of Stafford's "Mix13"
 * as used by Vigna's reference splitmix64.c).  A SplitMix64 stream seeded with
 * state s returns, as its i-th output (i = 1, 2, ...), mix64(s + i * GAMMA).
 *
 * Board (seed, board_id, rows, cols, p):
 *   key       = mix64(seed + GAMMA) ^ mix64(board_id + 2 * GAMMA)
 *   h(r, c)   = the (r * cols + c + 1)-th output of the stream seeded with key
 *   alive     <=> (h >> 32) < floor(p * 2^32)   (threshold computed in double)
 *
 * Two layouts of the same cells:
 *   bytes : row-major uint8, 1 = alive, 0 = dead;
 *   packed: rows of W = ceil(cols / 64) uint64 words, cell (r, c) is bit
 *           (c mod 64) of word r * W + c / 64 (LSB first), padding bits 0.
 */
#include <stdint.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t si_mix64(uint64_t z) { return mix64(z); }

/* i-th output (i >= 1) of the SplitMix64 stream whose initial state is s. */
uint64_t si_splitmix64_nth(uint64_t s, uint64_t i) { return mix64(s + i * GAMMA); }

uint64_t si_board_key(uint64_t seed, uint64_t board_id) {
  return mix64(seed + GAMMA) ^ mix64(board_id + 2 * GAMMA);
}

uint32_t si_threshold(double p) {
  if (!(p > 0.0)) return 0u;
  if (p >= 1.0) return 0xFFFFFFFFu; /* every draw below 2^32 - 1 is alive */
  return (uint32_t)floor(p * 4294967296.0);
}

static inline int alive_at(uint64_t key, uint64_t idx, uint32_t thr, int all) {
  if (all) return 1;
  return (uint32_t)(mix64(key + (idx + 1) * GAMMA) >> 32) < thr;
}

/* Returns 0 on success, -1 on invalid sizes. */
int si_gen_bytes(uint64_t seed, uint64_t board_id, int64_t rows, int64_t cols,
                 double p, uint8_t* out) {
  if (rows <= 0 || cols <= 0 || !out) return -1;
  const uint64_t key = si_board_key(seed, board_id);
  const uint32_t thr = si_threshold(p);
  const int all = p >= 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r)
    for (int64_t c = 0; c < cols; ++c)
      out[r * cols + c] = (uint8_t)alive_at(key, (uint64_t)(r * cols + c), thr, all);
  return 0;
}

int si_gen_packed(uint64_t seed, uint64_t board_id, int64_t rows, int64_t cols,
                  double p, uint64_t* out) {
  if (rows <= 0 || cols <= 0 || !out) return -1;
  const uint64_t key = si_board_key(seed, board_id);
  const uint32_t thr = si_threshold(p);
  const int all = p >= 1.0;
  const int64_t W = (cols + 63) / 64;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    for (int64_t w = 0; w < W; ++w) {
      uint64_t word = 0;
      const int64_t c0 = w * 64;
      const int64_t n = cols - c0 < 64 ? cols - c0 : 64;
      for (int64_t b = 0; b < n; ++b)
        word |= (uint64_t)alive_at(key, (uint64_t)(r * cols + c0 + b), thr, all) << b;
      out[r * W + w] = word;
    }
  }
  return 0;
}

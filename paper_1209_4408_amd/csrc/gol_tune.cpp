// Autotuner of the single-board tile pass (gol_tune in include/gol.h).
//
// For a board size it times candidate (generations per pass T, band height)
// pairs on scratch boards of that size and keeps the fastest per generation.
// The pass's run time does not depend on the cells (bitwise network, no
// data-dependent branches), so zeroed scratch boards time it faithfully.
// Candidates: T in {4, 8, 16}; band counts that put the wave total just under
// k waves per SIMD for k in {2, 3, 4, 6, 8, 12, 16}.  Results live in a
// per-process table keyed by (device, rows, cols); when GOL_AUTOTUNE_CACHE
// names a file, choices are also appended there and read back on first use.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

#include "gol.h"
#include "gol_internal.h"
#include "gol_plan.h"
#include "gol_runtime.h"

namespace gol {

hipError_t launch_board_pass(int T, const uint32_t* src, uint32_t* dst, int32_t R, int32_t C,
                             int32_t D, const GridGeom& g, int pd, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

namespace {
struct Key {
  int dev;
  int64_t rows, cols;
  bool operator<(const Key& o) const {
    return std::tie(dev, rows, cols) < std::tie(o.dev, o.rows, o.cols);
  }
};
std::mutex g_mu;
std::map<Key, TuneChoice> g_table;
bool g_loaded = false;

void load_file_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("GOL_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  int dev, T, band;
  long long rows, cols;
  while (fscanf(f, "%d %lld %lld %d %d", &dev, &rows, &cols, &T, &band) == 5)
    if (valid_T(T) && band > 0) g_table[Key{dev, rows, cols}] = TuneChoice{T, band};
  fclose(f);
}

void save_locked(const Key& k, const TuneChoice& c) {
  const char* path = getenv("GOL_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%d %lld %lld %d %d\n", k.dev, (long long)k.rows, (long long)k.cols, c.T, c.band_rows);
  fclose(f);
}
}  // namespace

bool tuned_choice(int64_t rows, int64_t cols, TuneChoice* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_table.find(Key{dev, rows, cols});
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

int tune(int64_t R, int64_t C, hipStream_t st, TuneChoice* out) {
  int rc = check_board(R, C, 0);
  if (rc) return rc;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  const int64_t W = (C + 63) / 64, D = 2 * W;
  const size_t bytes = (size_t)(R * W * 8);
  void *a = nullptr, *b = nullptr;
  rc = scratch_alloc(&a, bytes, st);
  if (rc) return rc;
  rc = scratch_alloc(&b, bytes, st);
  if (rc) {
    scratch_free(a, st);
    return rc;
  }
  e = launch_fill_u32((uint32_t*)a, (int64_t)(bytes / 4), 0u, st);
  if (e == hipSuccess) e = launch_fill_u32((uint32_t*)b, (int64_t)(bytes / 4), 0u, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int nsimd = simd_count();
  const int64_t ns = (D + kStripDwords - 1) / kStripDwords;
  double best = 1e300;
  TuneChoice pick{default_T(), default_band_rows(R, C, default_T(), nsimd)};
  for (int T : {4, 8, 16}) {
    std::set<int64_t> heights;
    for (int k : {2, 3, 4, 6, 8, 12, 16}) {
      const int64_t bands = std::max<int64_t>(1, (int64_t)k * nsimd / ns);
      const int64_t h = std::max<int64_t>(1, (R + bands - 1) / bands);
      if (h <= 65535) heights.insert(h);
    }
    heights.insert(default_band_rows(R, C, T, nsimd));
    const int pd = default_prefetch(T);
    for (int64_t h : heights) {
      if (e != hipSuccess) break;
      const GridGeom g = board_geometry(R, C, (int)h);
      // one warm-up pass, then enough passes for ~2 ms of device time
      e = launch_board_pass(T, (const uint32_t*)a, (uint32_t*)b, (int32_t)R, (int32_t)C,
                            (int32_t)D, g, pd, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e == hipSuccess)
        e = launch_board_pass(T, (const uint32_t*)b, (uint32_t*)a, (int32_t)R, (int32_t)C,
                              (int32_t)D, g, pd, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      int reps = (int)std::min(50.0, std::max(2.0, 2.0 / std::max(ms, 1e-3f)));
      e = hipEventRecord(e0, st);
      for (int i = 0; i < reps && e == hipSuccess; ++i)
        e = launch_board_pass(T, (const uint32_t*)((i & 1) ? b : a), (uint32_t*)((i & 1) ? a : b),
                              (int32_t)R, (int32_t)C, (int32_t)D, g, pd, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      const double per_gen = (double)ms / ((double)reps * T);
      if (per_gen < best) {
        best = per_gen;
        pick = TuneChoice{T, (int)h};
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  scratch_free(b, st);
  scratch_free(a, st);
  if (e != hipSuccess) return hip_error(e, "gol_tune");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    const Key k{dev, R, C};
    g_table[k] = pick;
    save_locked(k, pick);
  }
  if (out) *out = pick;
  return GOL_OK;
}

}  // namespace gol

extern "C" int gol_tune(int64_t rows, int64_t cols, void* stream, int* out_t_block,
                        int* out_band_rows) {
  gol::TuneChoice c{0, 0};
  int rc;
  try {
    rc = gol::tune(rows, cols, (hipStream_t)stream, &c);
  } catch (...) {
    return gol::set_error(GOL_EDEVICE, "unexpected exception");
  }
  if (rc) return rc;
  if (out_t_block) *out_t_block = c.T;
  if (out_band_rows) *out_band_rows = c.band_rows;
  return GOL_OK;
}

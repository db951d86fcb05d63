// Autotuner of the single-board tile pass (gol_tune / gol_tune_cfg in
// include/gol.h).
//
// For a board size it times candidate launch configurations on scratch
// boards of that size and keeps the fastest per generation.  The pass's run
// time does not depend on the cells (bitwise network, no data-dependent
// branches), so zeroed scratch boards time it faithfully.  Candidates: both
// layouts (one band per wave; two bands per wave sharing an edge, where the
// board allows it), T in {8, 12, 16} with the prefetch distance that suits
// it (for one band per wave at T = 16 also a shorter one), and band heights
// that put about k waves on each SIMD for k in {2, 3, 4, 6, 8, 10, 12}.  Results live in a per-process table keyed by (device,
// rows, cols); when GOL_AUTOTUNE_CACHE names a file, choices are also
// appended there and read back on first use.
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
std::map<Key, PassConfig> g_table;
bool g_loaded = false;

bool usable(const PassConfig& c) {
  if (c.layout == kLayoutResident) return true;
  return valid_board_T(c.T) && c.band_rows > 0 &&
         (c.layout == kLayoutBand || c.layout == kLayoutPaired) &&
         pass_config_compiled(c.layout, c.T, c.pd);
}

// Cache file lines: device rows cols t_block band_rows prefetch layout.
void load_file_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("GOL_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  int dev;
  long long rows, cols;
  PassConfig c;
  while (fscanf(f, "%d %lld %lld %d %d %d %d", &dev, &rows, &cols, &c.T, &c.band_rows, &c.pd,
                &c.layout) == 7)
    if (usable(c)) g_table[Key{dev, rows, cols}] = c;
  fclose(f);
}

void save_locked(const Key& k, const PassConfig& c) {
  const char* path = getenv("GOL_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%d %lld %lld %d %d %d %d\n", k.dev, (long long)k.rows, (long long)k.cols, c.T,
          c.band_rows, c.pd, c.layout);
  fclose(f);
}

// Configurations timed for an R x C board.
std::vector<PassConfig> candidates(int64_t R, int64_t C, int nsimd) {
  std::vector<PassConfig> out;
  const int64_t D = 2 * ((C + 63) / 64);
  for (int layout : {kLayoutBand, kLayoutPaired}) {
    const int64_t lanes = layout == kLayoutBand ? kStripDwords : kHalfStripDwords;
    const int64_t ns = (D + lanes - 1) / lanes;
    for (int T : {8, 12, 16}) {
      // the band layout at 16 generations per pass also with 9 rows of
      // prefetch (2 % faster than its default 12 on the 65536^2 board)
      std::set<int> pds{layout == kLayoutPaired ? 9 : default_prefetch(T)};
      if (layout == kLayoutBand && T == 16) pds.insert(9);
      std::set<int64_t> heights;
      for (int k : {2, 3, 4, 6, 8, 10, 12}) {
        // waves: ns x bands (one band per wave) or ns x pairs (two per wave)
        const int64_t units = std::max<int64_t>(1, (int64_t)k * nsimd / ns);
        const int64_t per = layout == kLayoutBand ? units : 2 * units;
        const int64_t h = std::max<int64_t>(1, (R + per - 1) / per);
        if (h <= 65535) heights.insert(h);
      }
      if (layout == kLayoutBand) heights.insert(default_band_rows(R, C, T, nsimd));
      for (int pd : pds)
        for (int64_t h : heights) {
          PassConfig c;
          c.T = T;
          c.layout = layout;
          c.pd = pd;
          c.band_rows = (int)h;
          if (layout == kLayoutPaired &&
              !paired_ok(R, C, T, paired_geometry(R, C, c.band_rows, c.T, c.pd), nullptr))
            continue;
          out.push_back(c);
        }
    }
  }
  if (resident_fits(R, C)) {
    // the whole board in one workgroup's LDS, timed over launches of 12
    // generations (a run is one launch whatever its length)
    PassConfig c;
    c.T = 12;
    c.layout = kLayoutResident;
    out.push_back(c);
  }
  return out;
}
}  // namespace

bool tuned_choice(int64_t rows, int64_t cols, PassConfig* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_table.find(Key{dev, rows, cols});
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

int tune(int64_t R, int64_t C, hipStream_t st, PassConfig* out) {
  int rc = check_board(R, C, 0);
  if (rc) return rc;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  const int64_t W = (C + 63) / 64;
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
  double best = 1e300;
  PassConfig pick;
  rc = resolve_config(R, C, PassConfig{}, &pick);  // the untuned default, if nothing wins
  const uint32_t* pa = (const uint32_t*)a;
  uint32_t* pb = (uint32_t*)b;
  for (const PassConfig& c : candidates(R, C, nsimd)) {
    if (e != hipSuccess || rc) break;
    // one warm-up pass, then enough passes for about 6 ms of device time
    e = launch_pass(c, pa, pb, R, C, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_pass(c, pb, (uint32_t*)pa, R, C, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    const int reps = (int)std::min(200.0, std::max(3.0, 6.0 / std::max(ms, 1e-3f)));
    e = hipEventRecord(e0, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
      e = launch_pass(c, (i & 1) ? pb : pa, (i & 1) ? (uint32_t*)pa : pb, R, C, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    const double per_gen = (double)ms / ((double)reps * c.T);
    if (per_gen < best) {
      best = per_gen;
      pick = c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  scratch_free(b, st);
  scratch_free(a, st);
  if (rc) return rc;
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

extern "C" int gol_tune_cfg(int64_t rows, int64_t cols, void* stream, gol_pass_config* out) {
  gol::PassConfig c;
  int rc;
  try {
    rc = gol::tune(rows, cols, (hipStream_t)stream, &c);
  } catch (...) {
    return gol::set_error(GOL_EDEVICE, "unexpected exception");
  }
  if (rc) return rc;
  if (out) {
    out->t_block = c.T;
    out->band_rows = c.band_rows;
    out->prefetch = c.pd;
    out->layout = c.layout;
  }
  return GOL_OK;
}

extern "C" int gol_tune(int64_t rows, int64_t cols, void* stream, int* out_t_block,
                        int* out_band_rows) {
  gol_pass_config c{};
  const int rc = gol_tune_cfg(rows, cols, stream, &c);
  if (rc) return rc;
  if (out_t_block) *out_t_block = c.t_block;
  if (out_band_rows) *out_band_rows = c.band_rows;
  return GOL_OK;
}

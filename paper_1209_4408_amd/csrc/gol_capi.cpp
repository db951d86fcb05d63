// C ABI of libgol: argument checks, device scratch, pass sequencing, batch
// plans.  Declared in include/gol.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <map>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gol.h"
#include "gol_debug.h"
#include "gol_internal.h"
#include "gol_plan.h"
#include "gol_runtime.h"

namespace gol {

// Launchers defined in gol_kernels.hip.
hipError_t launch_board_pass(int T, const uint32_t* src, uint32_t* dst, int32_t R, int32_t C,
                             int32_t D, const GridGeom& g, int pd, bool bounded, hipStream_t st,
                             const uint32_t* top = nullptr, const uint32_t* bot = nullptr);
hipError_t launch_board_pass_half(int T, const uint32_t* src, uint32_t* dst, int32_t R, int32_t C,
                                  int32_t D, const GridGeom& g, int pd, hipStream_t st);
hipError_t launch_board_lds(const uint32_t* src, uint32_t* dst, int32_t R, int32_t C, int32_t D,
                            int32_t G, hipStream_t st);
hipError_t launch_population(const uint64_t* b, int64_t R, int64_t C, unsigned long long* out,
                             hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_batch_pass(int T, bool masked, const BoardDesc* boards, const Segment* segs,
                             const WaveItem* items, int nearly, int nlate, int late_begin,
                             int level, hipStream_t st);
hipError_t launch_pack(const uint8_t* in, int64_t R, int64_t C, uint64_t* out, hipStream_t st);
hipError_t launch_unpack(const uint64_t* in, int64_t R, int64_t C, uint8_t* out, hipStream_t st);
hipError_t launch_copy_clear_padding(const uint64_t* in, int64_t R, int64_t C, uint64_t* out,
                                     hipStream_t st);
// Device address of the current device's fixed scratch (kFixedScratchBytes).
hipError_t fixed_scratch(void** out);
hipError_t launch_step_t1(const uint32_t* src, uint32_t* dst, int32_t R, int32_t D, int band_rows,
                          hipStream_t st);
hipError_t launch_batch_queue(int T, const BoardDesc* boards, const Segment* segs,
                              const QueueItem* items, const int32_t* per_pass, int nitems,
                              uint32_t* ctl, int nboards, int waves, hipStream_t st);
int batch_queue_waves(int T);

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string t_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(GOL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { t_last_error.clear(); }

const char* last_error() { return t_last_error.c_str(); }

// ---------------------------------------------------------------------------
// Device scratch allocation (stream ordered)
// ---------------------------------------------------------------------------
static std::mutex g_alloc_mu;
static gol_alloc_fn g_alloc = nullptr;
static gol_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;
static std::vector<int> g_pool_ready;

static void ensure_pool(int dev) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if ((int)g_pool_ready.size() <= dev) g_pool_ready.resize(dev + 1, 0);
  if (g_pool_ready[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;  // keep freed blocks cached in the pool
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_pool_ready[dev] = 1;
}

int scratch_alloc(void** p, size_t bytes, hipStream_t st) {
  gol_alloc_fn a;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
    ctx = g_alloc_ctx;
  }
  if (bytes == 0) bytes = 256;
  if (a) {
    *p = a(bytes, (void*)st, ctx);
    if (!*p) return set_error(GOL_ENOMEM, "installed allocator returned NULL for %zu bytes", bytes);
    return GOL_OK;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  ensure_pool(dev);
  e = hipMallocAsync(p, bytes, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GOL_ENOMEM, "hipMallocAsync(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  return GOL_OK;
}

void scratch_free(void* p, hipStream_t st) {
  if (!p) return;
  gol_free_fn f;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    f = g_free;
    ctx = g_alloc_ctx;
  }
  if (f)
    f(p, (void*)st, ctx);
  else
    (void)hipFreeAsync(p, st);
}

// Pinned host staging blocks, reused by power-of-two size class, and a pool
// of timing-free events, so repeated calls do not call hipHostMalloc or
// hipEventCreate.  A block handed back with pinned_put_after returns to the
// pool once the event recorded after its last use has completed.
static std::mutex g_pin_mu;
static std::map<size_t, std::vector<void*>> g_pin_free;
static std::vector<hipEvent_t> g_event_free;
struct Deferred {
  hipEvent_t ev;
  void* pinned;
  size_t cls;
};
static std::vector<Deferred> g_deferred;

// Blocks of a class up to kSlabMaxClass are carved from one hipHostMalloc of
// eight blocks (at least 1 MiB), so a burst of requests pins memory in a
// few large calls instead of one call per block (page-locking is the slow
// part of hipHostMalloc).  Blocks never return to the system.
constexpr size_t kSlabMaxClass = (size_t)8 << 20;
constexpr size_t kSlabBlocks = 8;

void* pinned_get(size_t bytes, size_t* cls_out) {
  size_t cls = 4096;
  while (cls < bytes) cls <<= 1;
  *cls_out = cls;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto& v = g_pin_free[cls];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      return p;
    }
  }
  const size_t n = cls <= kSlabMaxClass ? std::max(kSlabBlocks, ((size_t)1 << 20) / cls) : 1;
  void* p = nullptr;
  if (hipHostMalloc(&p, cls * n, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (n > 1) {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto& v = g_pin_free[cls];
    for (size_t i = 1; i < n; ++i) v.push_back((char*)p + i * cls);
  }
  return p;
}

void pinned_put(void* p, size_t cls) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free[cls].push_back(p);
}

static hipError_t event_get(hipEvent_t* ev) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_event_free.empty()) {
      *ev = g_event_free.back();
      g_event_free.pop_back();
      return hipSuccess;
    }
  }
  return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

void reap_deferred(bool wait) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  size_t k = 0;
  for (auto& d : g_deferred) {
    if (wait) (void)hipEventSynchronize(d.ev);
    if (hipEventQuery(d.ev) == hipSuccess) {
      g_event_free.push_back(d.ev);
      g_pin_free[d.cls].push_back(d.pinned);
    } else {
      g_deferred[k++] = d;
    }
  }
  g_deferred.resize(k);
}

int pinned_put_after(void* pinned, size_t cls, hipStream_t st) {
  hipEvent_t ev = nullptr;
  hipError_t e = event_get(&ev);
  if (e == hipSuccess) e = hipEventRecord(ev, st);
  if (e != hipSuccess) return hip_error(e, "hipEventRecord");
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_deferred.push_back(Deferred{ev, pinned, cls});
  return GOL_OK;
}

// ---------------------------------------------------------------------------
// Checks
// ---------------------------------------------------------------------------
int check_board(int64_t rows, int64_t cols, int64_t gens) {
  if (rows < 1 || cols < 1 || rows > (1 << 30) || cols > (1 << 30))
    return set_error(GOL_EINVAL, "rows and cols must be in [1, 2^30] (got %lld x %lld)",
                     (long long)rows, (long long)cols);
  if (gens < 0) return set_error(GOL_EINVAL, "generations must be >= 0 (got %lld)", (long long)gens);
  const int64_t W = (cols + 63) / 64;
  if (rows > INT64_MAX / 8 / W) return set_error(GOL_EINVAL, "board too large");
  return GOL_OK;
}

bool ranges_partially_overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  if (x == y) return false;
  return x < y + bytes && y < x + bytes;
}

static bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + bbytes && y < x + abytes;
}

int default_T() { return 12; }

// Boards the resident layout takes when no t_block or layout is asked for:
// at most this many dwords, where a tile pass is bound by its launch and by
// one wave's sweep rather than by its work (on MI355X, 120 generations: 64^2
// 33 us resident against 77 us in tile passes, 128^2 41 against 77,
// 120 x 240 60 against 90; 256^2 83 against 77, where one workgroup's share
// of the chip starts to bind).
constexpr int64_t kResidentAutoDwords = 1024;
// Generations per resident launch (about 0.1 s on the largest boards the
// layout takes, well under that on the boards it is chosen for).
constexpr int64_t kResidentMaxGens = 65536;
static bool resident_auto(int64_t R, int64_t C) {
  return resident_fits(R, C) && R * ((C + 31) / 32) <= kResidentAutoDwords;
}
int default_batch_T() { return 16; }


// SIMDs of the current device (4 per compute unit), cached per device.
int simd_count() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = 4 * cus;
  }
  return cache[dev];
}

// ---------------------------------------------------------------------------
// Single board
// ---------------------------------------------------------------------------
// Band height of the paired layout when none is given: about two waves per
// SIMD, as for the one-band layout.
static int default_paired_rows(int64_t R, int64_t C, int nsimd) {
  const int64_t D = 2 * ((C + 63) / 64);
  const int64_t ns = (D + kHalfStripDwords - 1) / kHalfStripDwords;
  const int64_t pairs = std::max<int64_t>(1, 2 * (int64_t)nsimd / ns);
  return (int)std::max<int64_t>(1, (R + 2 * pairs - 1) / (2 * pairs));
}

int resolve_config(int64_t R, int64_t C, const PassConfig& want, PassConfig* out) {
  PassConfig c = want;
  if (c.T < 0 || c.band_rows < 0 || c.pd < 0 || c.layout < 0)
    return set_error(GOL_EINVAL, "negative field in the pass configuration");
  if (c.bounded && c.layout != 0 && c.layout != kLayoutBand)
    return set_error(GOL_EINVAL, "a bounded board runs in the band layout (layout 0 or 1)");
  PassConfig tc;
  const bool automatic = !want.bounded && want.T == 0 && want.layout == 0;
  const bool tuned = automatic && tuned_choice(R, C, &tc);
  if (tuned) {
    c.T = tc.T;
    c.layout = tc.layout;
    if (!c.band_rows) c.band_rows = tc.band_rows;
    if (!c.pd) c.pd = tc.pd;
  }
  if (c.layout == kLayoutResident || (automatic && !tuned && resident_auto(R, C))) {
    if (!resident_fits(R, C))
      return set_error(GOL_EINVAL,
                       "the resident layout needs cols <= 32768 and both generations of the "
                       "board within %lld bytes of LDS",
                       (long long)kResidentMaxLdsBytes);
    c.layout = kLayoutResident;
    *out = c;
    return GOL_OK;
  }
  if (!c.T) c.T = default_T();
  if (!c.layout) c.layout = kLayoutBand;
  if (!c.pd) c.pd = default_prefetch(c.T);
  if (!valid_board_T(c.T))
    return set_error(GOL_EINVAL, "t_block must be 0, 1, 2, 4, 8, 12 or 16 (got %d)", c.T);
  if (c.layout != kLayoutBand && c.layout != kLayoutPaired)
    return set_error(GOL_EINVAL, "layout must be 0, 1 (band), 2 (paired) or 3 (resident) (got %d)",
                     c.layout);
  if (!pass_config_compiled(c.layout, c.T, c.pd))
    return set_error(GOL_EINVAL, "prefetch %d is not built for layout %d with t_block %d", c.pd,
                     c.layout, c.T);
  if (!c.band_rows)
    c.band_rows = c.layout == kLayoutBand ? default_band_rows(R, C, c.T, simd_count())
                                          : default_paired_rows(R, C, simd_count());
  if (c.layout == kLayoutPaired) {
    const char* why = nullptr;
    if (!paired_ok(R, C, c.T, paired_geometry(R, C, c.band_rows, c.T, c.pd), &why))
      return set_error(GOL_EINVAL, "%s", why);
  }
  *out = c;
  return GOL_OK;
}

// Band height of the one-generation kernel: about 32 waves per SIMD over its
// 248-dword strips, bands of at least 8 rows.  Short bands re-read more halo
// rows (two per band) but keep more rows in flight: on the 65536^2 board
// (19-row bands) a generation takes 216 us against 235 us at 8 waves per SIMD
// (73-row bands); bands of 8 to 20 rows measured 211-218 us, 128 rows 245 us.
static int t1_band_rows(int64_t R, int64_t D, int nsimd) {
  const int64_t strips = (D + 247) / 248;
  const int64_t bands = std::max<int64_t>(1, 32 * (int64_t)nsimd / strips);
  return (int)std::min<int64_t>(std::max<int64_t>(8, (R + bands - 1) / bands), 1 << 20);
}

hipError_t launch_pass(const PassConfig& c, const uint32_t* src, uint32_t* dst, int64_t R,
                       int64_t C, hipStream_t st) {
  const int32_t D = (int32_t)(2 * ((C + 63) / 64));
  if (c.layout == kLayoutResident)  // c.T generations in one launch
    return launch_board_lds(src, dst, (int32_t)R, (int32_t)C, D, c.T, st);
  // one generation on rows of whole 128-bit words: the HBM-bound kernel
  if (c.T == 1 && c.layout == kLayoutBand && !c.bounded && C % 128 == 0)
    return launch_step_t1(src, dst, (int32_t)R, D, t1_band_rows(R, D, simd_count()), st);
  if (c.layout == kLayoutPaired)
    return launch_board_pass_half(c.T, src, dst, (int32_t)R, (int32_t)C, D,
                                  paired_geometry(R, C, c.band_rows, c.T, c.pd), c.pd, st);
  return launch_board_pass(c.T, src, dst, (int32_t)R, (int32_t)C, D,
                           board_geometry(R, C, c.band_rows), c.pd, c.bounded, st);
}

// Walks the operations of a run in order without storing them: for each
// stretch of generations up to the next population check (or to G), the
// passes -- powers of two for the stretch mod t_block, small first, then whole
// t_block passes; in the resident layout, launches of at most
// kResidentMaxGens generations -- then the count at that check.  op(t, slot)
// is called with t > 0 for a pass of t generations and t == 0 for the count
// into slot `slot`; it returns false to stop the walk.
template <class Op>
static void walk_ops(int64_t G, int T, bool resident, const int64_t* checks, int64_t ncheck,
                     Op&& op) {
  int64_t g = 0;
  for (int64_t i = 0; i <= ncheck; ++i) {
    const int64_t upto = i < ncheck ? checks[i] : G;
    const int64_t len = upto - g;
    if (len > 0 && resident) {
      for (int64_t left = len; left > 0;) {
        const int64_t m = std::min<int64_t>(left, kResidentMaxGens);
        if (!op((int)m, -1)) return;
        left -= m;
      }
    } else if (len > 0) {
      const int64_t r = len % T;
      for (int k = 0; (1 << k) < T; ++k)
        if ((r & (1 << k)) && !op(1 << k, -1)) return;
      for (int64_t q = len / T; q > 0; --q)
        if (!op(T, -1)) return;
    }
    g = std::max(g, upto);
    if (i < ncheck && !op(0, i)) return;
  }
}

int step_packed(const uint64_t* d_in, int64_t R, int64_t C, int64_t G, uint64_t* d_out,
                hipStream_t st, const PassConfig& cfg, const int64_t* checks, int64_t ncheck,
                int64_t* d_counts, void* ext_scratch, size_t ext_scratch_bytes) {
  int rc = check_board(R, C, G);
  if (rc) return rc;
  if (!d_in || !d_out) return set_error(GOL_EINVAL, "null board pointer");
  if (ncheck < 0 || (ncheck > 0 && (!checks || !d_counts)))
    return set_error(GOL_EINVAL, "population checks: null array or negative count");
  for (int64_t i = 0; i < ncheck; ++i)
    if (checks[i] < 0 || checks[i] > G || (i > 0 && checks[i] < checks[i - 1]))
      return set_error(GOL_EINVAL,
                       "population checks must be non-decreasing generation counts in 0..%lld",
                       (long long)G);
  PassConfig c;
  rc = resolve_config(R, C, cfg, &c);
  if (rc) return rc;
  const int64_t W = (C + 63) / 64;
  const size_t bytes = (size_t)(R * W * 8);
  if (ranges_partially_overlap(d_in, d_out, bytes))
    return set_error(GOL_EINVAL, "d_in and d_out partially overlap");
  if (ext_scratch && bytes > ext_scratch_bytes)
    return set_error(GOL_EINVAL,
                     "the board needs %zu bytes of scratch; the fixed scratch holds %zu",
                     bytes, ext_scratch_bytes);
  if (!ext_scratch) reap_deferred(false);
  const bool resident = c.layout == kLayoutResident;
  unsigned long long* counts = (unsigned long long*)d_counts;
  hipError_t e = hipSuccess;
  if (ncheck > 0) e = launch_fill_u32((uint32_t*)d_counts, 2 * ncheck, 0u, st);
  // passes in the run (a pass ends at every checked generation)
  int64_t K = 0;
  walk_ops(G, c.T, resident, checks, ncheck, [&](int t, int64_t) {
    K += t > 0;
    return true;
  });
  if (K == 0) {
    if (e == hipSuccess) e = launch_copy_clear_padding(d_in, R, C, d_out, st);
    for (int64_t i = 0; i < ncheck && e == hipSuccess; ++i)
      e = launch_population(d_out, R, C, counts + i, st);
    return e == hipSuccess ? GOL_OK : hip_error(e, "copy kernel launch");
  }
  if (resident) {
    // each launch reads its whole board before writing, so every launch
    // after the first runs in place on d_out
    const int32_t D = (int32_t)(2 * W);
    const uint32_t* cur = (const uint32_t*)d_in;
    walk_ops(G, c.T, true, checks, ncheck, [&](int t, int64_t slot) {
      if (t == 0)
        e = launch_population((const uint64_t*)cur, R, C, counts + slot, st);
      else
        e = launch_board_lds(cur, (uint32_t*)d_out, (int32_t)R, (int32_t)C, D, t, st);
      if (t > 0) cur = (const uint32_t*)d_out;
      return e == hipSuccess;
    });
    return e == hipSuccess ? GOL_OK : hip_error(e, "resident board launch");
  }
  void* s1v = ext_scratch;
  if (!s1v) {
    rc = scratch_alloc(&s1v, bytes, st);
    if (rc) return rc;
  }
  uint32_t* s1 = (uint32_t*)s1v;
  uint32_t* out = (uint32_t*)d_out;
  const uint32_t* src0 = (const uint32_t*)d_in;
  uint32_t* w[2] = {out, s1};
  int par = (int)((K - 1) & 1);
  if (e == hipSuccess && (const void*)d_in == (const void*)d_out && (K & 1)) {
    // pass 0 must not write the board it reads: start from a copy
    e = launch_copy_clear_padding(d_in, R, C, (uint64_t*)s1, st);
    src0 = s1;
    par = 0;
  }
  // the G mod T remainder: shorter passes, one band per wave, defaults
  PassConfig rem;
  rem.layout = kLayoutBand;
  rem.bounded = c.bounded;
  const uint32_t* cur = src0;  // the board after the passes so far
  int64_t j = 0;
  if (e == hipSuccess)
    walk_ops(G, c.T, false, checks, ncheck, [&](int t, int64_t slot) {
      if (t == 0) {
        e = launch_population((const uint64_t*)cur, R, C, counts + slot, st);
        return e == hipSuccess;
      }
      const uint32_t* src = (j == 0) ? src0 : w[(j - 1 + par) & 1];
      uint32_t* dst = w[(j + par) & 1];
      if (t == c.T) {
        e = launch_pass(c, src, dst, R, C, st);
      } else {
        if (rem.T != t) {
          rem.T = t;
          rem.pd = default_prefetch(t);
          rem.band_rows = default_band_rows(R, C, t, simd_count());
        }
        e = launch_pass(rem, src, dst, R, C, st);
      }
      cur = dst;
      ++j;
      return e == hipSuccess;
    });
  if (!ext_scratch) scratch_free(s1v, st);
  if (e != hipSuccess) return hip_error(e, "tile pass launch");
  return GOL_OK;
}

// Library streams for the synchronous host API, each with a pinned host
// staging buffer that its calls reuse (a call holds the slot until its
// stream has drained, so the buffer is never in use twice).
struct HostSlot {
  hipStream_t st = nullptr;
  void* pinned = nullptr;
  size_t cap = 0;
};
static std::mutex g_stream_mu;
static std::vector<HostSlot> g_slots;

static int acquire_slot(HostSlot* slot) {
  {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    if (!g_slots.empty()) {
      *slot = g_slots.back();
      g_slots.pop_back();
      return GOL_OK;
    }
  }
  *slot = HostSlot{};
  hipError_t e = hipStreamCreateWithFlags(&slot->st, hipStreamNonBlocking);
  return e == hipSuccess ? GOL_OK : hip_error(e, "hipStreamCreate");
}

static void release_slot(const HostSlot& slot) {
  std::lock_guard<std::mutex> lk(g_stream_mu);
  g_slots.push_back(slot);
}

// Library streams without staging (the second stream of batched schedules).
static std::vector<hipStream_t> g_streams;

static int acquire_stream(hipStream_t* st) {
  {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    if (!g_streams.empty()) {
      *st = g_streams.back();
      g_streams.pop_back();
      return GOL_OK;
    }
  }
  hipError_t e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
  return e == hipSuccess ? GOL_OK : hip_error(e, "hipStreamCreate");
}

static void release_stream(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_stream_mu);
  g_streams.push_back(st);
}

// Byte boards up to this size go through the slot's pinned buffer (a host
// copy and one DMA each way); larger ones are copied from pageable memory.
constexpr size_t kStagingMaxBytes = (size_t)16 << 20;

int step_host(const uint8_t* board, int64_t R, int64_t C, int64_t G, uint8_t* out, int T) {
  int rc = check_board(R, C, G);
  if (rc) return rc;
  if (!board || !out) return set_error(GOL_EINVAL, "null board pointer");
  if (R > INT64_MAX / C) return set_error(GOL_EINVAL, "board too large");
  const size_t N = (size_t)(R * C);
  if (ranges_partially_overlap(board, out, N))
    return set_error(GOL_EINVAL, "board and out partially overlap");
  const int64_t W = (C + 63) / 64;
  const size_t words_bytes = (size_t)(R * W * 8);
  HostSlot slot;
  rc = acquire_slot(&slot);
  if (rc) return rc;
  const hipStream_t st = slot.st;
  if (N <= kStagingMaxBytes && slot.cap < N) {
    if (slot.pinned) (void)hipHostFree(slot.pinned);
    slot.pinned = nullptr;
    slot.cap = 0;
    if (hipHostMalloc(&slot.pinned, N, 0) == hipSuccess) slot.cap = N;
    else slot.pinned = nullptr;  // fall back to pageable copies
  }
  const bool staged = N <= kStagingMaxBytes && slot.cap >= N;
  if (staged) memcpy(slot.pinned, board, N);
  void *db = nullptr, *pa = nullptr, *pb = nullptr;
  rc = scratch_alloc(&db, N, st);
  if (!rc) rc = scratch_alloc(&pa, words_bytes, st);
  if (!rc) rc = scratch_alloc(&pb, words_bytes, st);
  hipError_t e = hipSuccess;
  if (!rc) {
    e = hipMemcpyAsync(db, staged ? slot.pinned : board, N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_pack((const uint8_t*)db, R, C, (uint64_t*)pa, st);
    if (e == hipSuccess) {
      PassConfig cfg;
      cfg.T = T;
      rc = step_packed((const uint64_t*)pa, R, C, G, (uint64_t*)pb, st, cfg);
      if (!rc) {
        e = launch_unpack((const uint64_t*)pb, R, C, (uint8_t*)db, st);
        if (e == hipSuccess)
          e = hipMemcpyAsync(staged ? slot.pinned : out, db, N, hipMemcpyDeviceToHost, st);
      }
    }
  }
  scratch_free(pb, st);
  scratch_free(pa, st);
  scratch_free(db, st);
  hipError_t e2 = hipStreamSynchronize(st);
  if (staged && !rc && e == hipSuccess && e2 == hipSuccess) memcpy(out, slot.pinned, N);
  release_slot(slot);
  if (rc) return rc;
  if (e != hipSuccess) return hip_error(e, "gol_step");
  if (e2 != hipSuccess) return hip_error(e2, "hipStreamSynchronize");
  return GOL_OK;
}

// ---------------------------------------------------------------------------
// Batch plans
// ---------------------------------------------------------------------------


// Validates, plans and fills the board descriptors given a scratch base.
int plan_boards(const gol_board* boards, int64_t n, int T, int band_rows, DevicePlan& P) {
  if (n < 0 || (n > 0 && !boards)) return set_error(GOL_EINVAL, "bad board array");
  if (n > (int64_t)1 << 24) return set_error(GOL_EINVAL, "too many boards");
  if (T == 0) T = default_batch_T();
  if (!valid_T(T)) return set_error(GOL_EINVAL, "t_block must be 0, 1, 2, 4, 8, 12 or 16 (got %d)", T);
  std::vector<BoardReq> req((size_t)n);
  P.boards.assign(boards, boards + n);
  P.scratch_off.assign((size_t)n, 0);
  size_t off = 0;
  for (int64_t b = 0; b < n; ++b) {
    const gol_board& g = boards[b];
    int rc = check_board(g.rows, g.cols, g.generations);
    if (rc) return set_error(rc, "board %lld: %s", (long long)b, last_error());
    if (!g.d_in || !g.d_out) return set_error(GOL_EINVAL, "board %lld: null pointer", (long long)b);
    const int64_t W = (g.cols + 63) / 64;
    if (ranges_partially_overlap(g.d_in, g.d_out, (size_t)(g.rows * W * 8)))
      return set_error(GOL_EINVAL, "board %lld: d_in and d_out partially overlap", (long long)b);
    req[b] = BoardReq{g.rows, g.cols, g.generations};
    if (g.generations > 0) {
      P.scratch_off[b] = off;
      off += (size_t)(g.rows * W);
    }
  }
  P.scratch_words = off;
  std::string err;
  if (band_rows <= 0) {
    band_rows = kBatchBandRows;
    const char* e = getenv("GOL_BATCH_BAND_ROWS");  // tuning override
    if (e && atoi(e) > 0) band_rows = atoi(e);
  }
  if (!build_plan(req, T, band_rows, P.hp, err)) return set_error(GOL_EINVAL, "%s", err.c_str());
  return GOL_OK;
}

void fill_board_descs(DevicePlan& P) {
  const size_t n = P.boards.size();
  P.h_boards.assign(n, BoardDesc{});
  P.copy_first.clear();
  P.zero_gen.clear();
  for (size_t b = 0; b < n; ++b) {
    const gol_board& g = P.boards[b];
    BoardDesc& d = P.h_boards[b];
    const int64_t W = (g.cols + 63) / 64;
    d.R = (int32_t)g.rows;
    d.C = (int32_t)g.cols;
    d.D = (int32_t)(2 * W);
    d.K = P.hp.K[b];
    d.Tshort = P.hp.Tshort[b];
    d.start = P.hp.start[b];
    d.jshort = P.hp.jshort[b];
    if (d.K == 0) {
      P.zero_gen.push_back((int)b);
      d.src0 = (const uint32_t*)g.d_in;
      d.w[0] = d.w[1] = (uint32_t*)g.d_out;
      continue;
    }
    uint32_t* s1 = (uint32_t*)(P.d_scratch + P.scratch_off[b]);
    d.w[0] = (uint32_t*)g.d_out;
    d.w[1] = s1;
    d.src0 = (const uint32_t*)g.d_in;
    d.par = (d.K - 1) & 1;
    if ((const void*)g.d_in == (const void*)g.d_out && (d.K & 1)) {
      P.copy_first.push_back((int)b);
      d.src0 = s1;
      d.par = 0;
    }
  }
}

hipError_t enqueue_levels(const HostPlan& hp, const BoardDesc* boards, const Segment* segs,
                          const WaveItem* items, hipStream_t st, hipStream_t side,
                          hipEvent_t fork, hipEvent_t join) {
  const int Kmax = (int)hp.level_items.size();
  const bool two = Kmax > 0 && hp.late_begin < (int32_t)hp.items.size();
  hipError_t e = hipSuccess;
  if (two) {
    e = hipEventRecord(fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
  }
  for (int L = 0; L < Kmax && e == hipSuccess; ++L) {
    if (hp.level_early[L] > 0)
      e = launch_batch_pass(hp.T, L == 0 && hp.early_masked, boards, segs, items,
                            hp.level_early[L], 0, hp.late_begin, L, st);
    if (e == hipSuccess && hp.level_late[L] > 0)
      e = launch_batch_pass(hp.T, L == Kmax - 1 && hp.late_masked, boards, segs, items, 0,
                            hp.level_late[L], hp.late_begin, L, two ? side : st);
  }
  if (two) {
    // join even after a failed launch, so a capture on `st` can end
    hipError_t e2 = hipEventRecord(join, side);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(st, join, 0);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

hipError_t enqueue_plan(const DevicePlan& P, hipStream_t st, hipStream_t side, hipEvent_t fork,
                        hipEvent_t join) {
  hipError_t e = hipSuccess;
  for (int b : P.zero_gen) {
    const gol_board& g = P.boards[b];
    e = launch_copy_clear_padding(g.d_in, g.rows, g.cols, g.d_out, st);
    if (e != hipSuccess) return e;
  }
  for (int b : P.copy_first) {
    const gol_board& g = P.boards[b];
    e = launch_copy_clear_padding(g.d_in, g.rows, g.cols, P.d_scratch + P.scratch_off[b], st);
    if (e != hipSuccess) return e;
  }
  return enqueue_levels(P.hp, P.d_boards, P.d_segs, P.d_items, st, side, fork, join);
}

// Uploads boards / segments / items into one device block at `dev`.
static size_t meta_bytes(const DevicePlan& P, size_t* ob, size_t* os, size_t* oi) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  *ob = 0;
  *os = al(P.h_boards.size() * sizeof(BoardDesc));
  *oi = *os + al(P.hp.segs.size() * sizeof(Segment));
  return *oi + al(P.hp.items.size() * sizeof(WaveItem));
}

static void fill_meta_host(const DevicePlan& P, char* host, size_t ob, size_t os, size_t oi) {
  memcpy(host + ob, P.h_boards.data(), P.h_boards.size() * sizeof(BoardDesc));
  memcpy(host + os, P.hp.segs.data(), P.hp.segs.size() * sizeof(Segment));
  memcpy(host + oi, P.hp.items.data(), P.hp.items.size() * sizeof(WaveItem));
}

// A pooled library stream and two events for enqueue_levels' second stream.
// The events may be destroyed once the waits on them are queued.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  int open() {
    int rc = acquire_stream(&st);
    if (rc) return rc;
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    return e == hipSuccess ? GOL_OK : hip_error(e, "hipEventCreate");
  }
  ~SideStream() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (st) release_stream(st);
  }
};

int batch_run(const gol_board* boards, int64_t n, hipStream_t st, int T) {
  reap_deferred(false);
  DevicePlan P;
  int rc = plan_boards(boards, n, T, 0, P);
  if (rc) return rc;
  if (n == 0) return GOL_OK;
  SideStream side;
  rc = side.open();
  if (rc) return rc;
  void* scratch = nullptr;
  void* meta = nullptr;
  if (P.scratch_words) {
    rc = scratch_alloc(&scratch, P.scratch_words * 8, st);
    if (rc) return rc;
  }
  P.d_scratch = (uint64_t*)scratch;
  fill_board_descs(P);
  size_t ob, os, oi;
  const size_t mb = meta_bytes(P, &ob, &os, &oi);
  rc = scratch_alloc(&meta, mb, st);
  if (rc) {
    scratch_free(scratch, st);
    return rc;
  }
  size_t cls = 0;
  void* pinned = pinned_get(mb, &cls);
  if (!pinned) {
    scratch_free(meta, st);
    scratch_free(scratch, st);
    return set_error(GOL_ENOMEM, "pinned staging of %zu bytes", mb);
  }
  fill_meta_host(P, (char*)pinned, ob, os, oi);
  hipError_t e = hipMemcpyAsync(meta, pinned, mb, hipMemcpyHostToDevice, st);
  P.d_boards = (BoardDesc*)((char*)meta + ob);
  P.d_segs = (Segment*)((char*)meta + os);
  P.d_items = (WaveItem*)((char*)meta + oi);
  if (e == hipSuccess) e = enqueue_plan(P, st, side.st, side.fork, side.join);
  scratch_free(meta, st);
  scratch_free(scratch, st);
  rc = pinned_put_after(pinned, cls, st);
  if (e != hipSuccess) return hip_error(e, "gol_batch_run");
  return rc;
}

// Candidate schedules of a batch, timed on zeroed scratch boards of the
// same sizes (a pass's run time does not depend on the cells): for each
// (T, band height) the schedule runs once to warm up and once timed with
// events on a library stream; the fastest wins.  The scratch (input, output
// and ping-pong board per board) is freed before returning.
int tune_batch(const std::vector<BoardReq>& boards, const std::vector<int>& Ts,
               const std::vector<int>& bands, int* T_out, int* band_out, double* secs_out) {
  size_t words = 0;
  std::vector<size_t> off(boards.size(), 0);
  for (size_t b = 0; b < boards.size(); ++b) {
    off[b] = words;
    words += (size_t)(boards[b].rows * ((boards[b].cols + 63) / 64));
  }
  *T_out = Ts.empty() ? default_batch_T() : Ts[0];
  *band_out = bands.empty() ? kBatchBandRows : bands[0];
  if (secs_out) *secs_out = 0.0;
  if (words == 0 || Ts.empty() || bands.empty()) return GOL_OK;
  HostSlot slot;
  int rc = acquire_slot(&slot);
  if (rc) return rc;
  hipStream_t st = slot.st;
  SideStream side;
  rc = side.open();
  void* buf = nullptr;
  if (!rc) rc = scratch_alloc(&buf, 3 * words * 8, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  if (!rc) {
    e = launch_fill_u32((uint32_t*)buf, (int64_t)(2 * words), 0u, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
  }
  double best = 1e300;
  std::vector<gol_board> gb(boards.size());
  uint64_t* in = (uint64_t*)buf;
  for (size_t b = 0; b < boards.size(); ++b)
    gb[b] = gol_board{in + off[b], in + words + off[b], boards[b].rows, boards[b].cols,
                      boards[b].generations};
  for (int T : Ts) {
    for (int band : bands) {
      if (rc || e != hipSuccess) break;
      DevicePlan P;
      rc = plan_boards(gb.data(), (int64_t)gb.size(), T, band, P);
      if (rc) break;
      P.d_scratch = in + 2 * words;
      fill_board_descs(P);
      size_t ob, os, oi;
      const size_t mb = meta_bytes(P, &ob, &os, &oi);
      std::vector<char> host(mb);
      fill_meta_host(P, host.data(), ob, os, oi);
      void* meta = nullptr;
      rc = scratch_alloc(&meta, mb, st);
      if (rc) break;
      e = hipMemcpyAsync(meta, host.data(), mb, hipMemcpyHostToDevice, st);
      P.d_boards = (BoardDesc*)((char*)meta + ob);
      P.d_segs = (Segment*)((char*)meta + os);
      P.d_items = (WaveItem*)((char*)meta + oi);
      if (e == hipSuccess) e = enqueue_plan(P, st, side.st, side.fork, side.join);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = enqueue_plan(P, st, side.st, side.fork, side.join);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      scratch_free(meta, st);
      if (e == hipSuccess && ms < best) {
        best = ms;
        *T_out = T;
        *band_out = band;
      }
    }
  }
  if (buf) scratch_free(buf, st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t es = hipStreamSynchronize(st);
  release_slot(slot);
  if (rc) return rc;
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return hip_error(e, "batch tuning");
  if (secs_out) *secs_out = best * 1e-3;
  return GOL_OK;
}

// The automatic fields of a plan's configuration (*T == 0: T in 8, 12, 16;
// *band == 0: 48, 64, 96 or 128 rows), timed on scratch copies of the boards
// (or, above kTuneMaxBytes of them, of every k-th board).  Boards that are
// invalid are left for plan_boards to reject.
constexpr size_t kTuneMaxBytes = (size_t)1 << 30;
static int tune_plan(const gol_board* boards, int64_t n, int* T, int* band) {
  std::vector<int> Ts = *T ? std::vector<int>{*T} : std::vector<int>{8, 12, 16};
  std::vector<int> bands =
      *band ? std::vector<int>{*band} : std::vector<int>{48, 64, 96, 128};
  if (!*T) *T = default_batch_T();
  if (!*band) *band = kBatchBandRows;
  if (n <= 0 || !boards) return GOL_OK;
  double bytes = 0.0;
  for (int64_t b = 0; b < n; ++b) {
    const gol_board& g = boards[b];
    if (check_board(g.rows, g.cols, g.generations)) {
      clear_error();
      return GOL_OK;
    }
    bytes += 3.0 * (double)g.rows * (double)((g.cols + 63) / 64) * 8.0;
  }
  const int64_t k = std::max<int64_t>(1, (int64_t)std::ceil(bytes / (double)kTuneMaxBytes));
  std::vector<BoardReq> req;
  for (int64_t b = 0; b < n; b += k)
    req.push_back(BoardReq{boards[b].rows, boards[b].cols, boards[b].generations});
  int t = *T, h = *band;
  const int rc = tune_batch(req, Ts, bands, &t, &h, nullptr);
  if (rc == GOL_ENOMEM) {  // no room to time: keep the defaults
    clear_error();
    return GOL_OK;
  }
  if (rc) return rc;
  *T = t;
  *band = h;
  return GOL_OK;
}

}  // namespace gol

// ---------------------------------------------------------------------------
// extern "C"
// ---------------------------------------------------------------------------
using namespace gol;

struct gol_plan {
  DevicePlan P;
  void* meta = nullptr;
  // the persistent work-queue form (GOL_LAYOUT_QUEUE): its own tables
  bool queue = false;
  QueuePlan Q;
  const QueueItem* d_qitems = nullptr;
  const int32_t* d_per_pass = nullptr;
  uint32_t* d_ctl = nullptr;
  int qwaves = 0;
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t side = nullptr;  // the late group's stream (default priority)
  hipEvent_t fork = nullptr, join = nullptr;
  // one event recorded after each run still in flight: destroy waits for
  // these only, not for the whole device
  std::vector<hipEvent_t> runs;
  std::mutex mu;
};

// Records the end of a plan run on `st` (reusing events of completed runs).
static hipError_t plan_mark_run(gol_plan* p, hipStream_t st) {
  std::lock_guard<std::mutex> lk(p->mu);
  hipEvent_t ev = nullptr;
  for (size_t i = 0; i < p->runs.size(); ++i)
    if (hipEventQuery(p->runs[i]) == hipSuccess) {
      ev = p->runs[i];
      p->runs.erase(p->runs.begin() + (long)i);
      break;
    }
  hipError_t e = ev ? hipSuccess : hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, st);
  if (e == hipSuccess) p->runs.push_back(ev);
  else if (ev) (void)hipEventDestroy(ev);
  return e;
}

// Tables of the queue form: board descriptors (short pass first), segments,
// items, items per pass, control words.
static int setup_queue(gol_plan* p, int T, int band) {
  std::vector<BoardReq> req;
  for (const gol_board& g : p->P.boards) req.push_back(BoardReq{g.rows, g.cols, g.generations});
  std::string err;
  if (!build_queue_plan(req, T, band, p->Q, err)) return set_error(GOL_EINVAL, "%s", err.c_str());
  for (BoardDesc& d : p->P.h_boards) d.jshort = 0;  // pass j reads / writes as before
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t n = p->P.h_boards.size();
  const size_t ob = 0, os = al(n * sizeof(BoardDesc));
  const size_t oi = os + al(p->Q.segs.size() * sizeof(Segment));
  const size_t op = oi + al(p->Q.items.size() * sizeof(QueueItem));
  const size_t oc = op + al(n * sizeof(int32_t));
  const size_t mb = oc + al((kQueueCtlHeader + n) * sizeof(uint32_t));
  hipError_t e = hipMalloc(&p->meta, mb);
  if (e != hipSuccess) return set_error(GOL_ENOMEM, "hipMalloc queue tables: %s", hipGetErrorString(e));
  std::vector<char> host(mb, 0);
  memcpy(host.data() + ob, p->P.h_boards.data(), n * sizeof(BoardDesc));
  memcpy(host.data() + os, p->Q.segs.data(), p->Q.segs.size() * sizeof(Segment));
  memcpy(host.data() + oi, p->Q.items.data(), p->Q.items.size() * sizeof(QueueItem));
  memcpy(host.data() + op, p->Q.per_pass.data(), n * sizeof(int32_t));
  e = hipMemcpy(p->meta, host.data(), mb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_error(e, "hipMemcpy queue tables");
  p->P.d_boards = (BoardDesc*)((char*)p->meta + ob);
  p->P.d_segs = (Segment*)((char*)p->meta + os);
  p->d_qitems = (const QueueItem*)((char*)p->meta + oi);
  p->d_per_pass = (const int32_t*)((char*)p->meta + op);
  p->d_ctl = (uint32_t*)((char*)p->meta + oc);
  p->qwaves = batch_queue_waves(T);
  if (p->qwaves <= 0) p->qwaves = 4 * simd_count();
  return GOL_OK;
}

static hipError_t enqueue_queue(const gol_plan* p, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int b : p->P.zero_gen) {
    const gol_board& g = p->P.boards[b];
    e = launch_copy_clear_padding(g.d_in, g.rows, g.cols, g.d_out, st);
    if (e != hipSuccess) return e;
  }
  for (int b : p->P.copy_first) {
    const gol_board& g = p->P.boards[b];
    e = launch_copy_clear_padding(g.d_in, g.rows, g.cols, p->P.d_scratch + p->P.scratch_off[b], st);
    if (e != hipSuccess) return e;
  }
  return launch_batch_queue(p->Q.T, p->P.d_boards, p->P.d_segs, p->d_qitems, p->d_per_pass,
                            (int)p->Q.items.size(), p->d_ctl, (int)p->P.h_boards.size(),
                            p->qwaves, st);
}

extern "C" {

const char* gol_last_error(void) { return gol::last_error(); }

const char* gol_version(void) { return "golmi 0.1 (gfx950)"; }

int gol_step(const uint8_t* board, int64_t rows, int64_t cols, int64_t generations, uint8_t* out) {
  try {
    return step_host(board, rows, cols, generations, out, 0);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_step_packed_ex(const uint64_t* d_in, int64_t rows, int64_t cols, int64_t generations,
                       uint64_t* d_out, void* stream, int t_block) {
  try {
    PassConfig cfg;
    cfg.T = t_block;
    return step_packed(d_in, rows, cols, generations, d_out, (hipStream_t)stream, cfg);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_step_packed_noalloc(const uint64_t* d_in, int64_t rows, int64_t cols,
                            int64_t generations, uint64_t* d_out, void* stream) {
  try {
    int rc = check_board(rows, cols, generations);
    if (rc) return rc;
    const int64_t W = (cols + 63) / 64;
    if (rows > kFixedScratchBytes / 8 / W)
      return set_error(GOL_EINVAL,
                       "gol_step_packed_noalloc takes boards of at most %lld bytes "
                       "(rows * ceil(cols / 64) * 8); this one needs %lld",
                       (long long)kFixedScratchBytes, (long long)(rows * W * 8));
    if (!d_in || !d_out) return set_error(GOL_EINVAL, "null board pointer");
    void* scr = nullptr;
    const hipError_t e = fixed_scratch(&scr);
    if (e != hipSuccess) return hip_error(e, "fixed scratch lookup");
    PassConfig cfg;
    return step_packed(d_in, rows, cols, generations, d_out, (hipStream_t)stream, cfg, nullptr,
                       0, nullptr, scr, (size_t)kFixedScratchBytes);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_step_packed_cfg(const uint64_t* d_in, int64_t rows, int64_t cols, int64_t generations,
                        uint64_t* d_out, void* stream, const gol_pass_config* config) {
  try {
    PassConfig cfg;
    if (config) {
      cfg.T = config->t_block;
      cfg.band_rows = config->band_rows;
      cfg.pd = config->prefetch;
      cfg.layout = config->layout;
    }
    return step_packed(d_in, rows, cols, generations, d_out, (hipStream_t)stream, cfg);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_step_packed_population(const uint64_t* d_in, int64_t rows, int64_t cols,
                               int64_t generations, uint64_t* d_out, void* stream,
                               const gol_pass_config* config, const int64_t* checks,
                               int64_t ncheck, int64_t* d_counts) {
  try {
    PassConfig cfg;
    if (config) {
      cfg.T = config->t_block;
      cfg.band_rows = config->band_rows;
      cfg.pd = config->prefetch;
      cfg.layout = config->layout;
    }
    return step_packed(d_in, rows, cols, generations, d_out, (hipStream_t)stream, cfg, checks,
                       ncheck, d_counts);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_step_packed_bounded(const uint64_t* d_in, int64_t rows, int64_t cols,
                            int64_t generations, uint64_t* d_out, void* stream,
                            const gol_pass_config* config) {
  try {
    PassConfig cfg;
    if (config) {
      cfg.T = config->t_block;
      cfg.band_rows = config->band_rows;
      cfg.pd = config->prefetch;
      cfg.layout = config->layout;
    }
    cfg.bounded = true;
    return step_packed(d_in, rows, cols, generations, d_out, (hipStream_t)stream, cfg);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_strip_pass(const uint64_t* d_strip, const uint64_t* d_top, const uint64_t* d_bottom,
                   int64_t rows, int64_t cols, int64_t t, uint64_t* d_out, void* stream,
                   const gol_pass_config* config) {
  int rc = check_board(rows, cols, t);
  if (rc) return rc;
  if (!d_strip || !d_top || !d_bottom || !d_out)
    return set_error(GOL_EINVAL, "null buffer");
  if (t < 1 || t > 16 || !valid_board_T((int)t))
    return set_error(GOL_EINVAL, "t must be 1, 2, 4, 8, 12 or 16 (got %lld)", (long long)t);
  const int T = (int)t;
  PassConfig c;
  if (config) {
    if (config->t_block != 0 && config->t_block != T)
      return set_error(GOL_EINVAL, "config t_block must be 0 or t");
    if (config->layout != 0 && config->layout != kLayoutBand)
      return set_error(GOL_EINVAL, "a strip runs in the band layout (layout 0 or 1)");
    if (config->band_rows < 0 || config->prefetch < 0)
      return set_error(GOL_EINVAL, "negative field in the pass configuration");
    c.band_rows = config->band_rows;
    c.pd = config->prefetch;
  }
  const int64_t W = (cols + 63) / 64;
  const size_t sb = (size_t)(rows * W * 8), hb = (size_t)(t * W * 8);
  if (ranges_overlap(d_out, sb, d_strip, sb) || ranges_overlap(d_out, sb, d_top, hb) ||
      ranges_overlap(d_out, sb, d_bottom, hb))
    return set_error(GOL_EINVAL, "d_out overlaps an input");
  PassConfig tc;
  if (!c.band_rows && !c.pd && tuned_choice(rows, cols, &tc) && tc.layout == kLayoutBand &&
      tc.T == T) {
    c.band_rows = tc.band_rows;
    c.pd = tc.pd;
  }
  if (!c.pd) c.pd = default_prefetch(T);
  if (!pass_config_compiled(kLayoutBand, T, c.pd))
    return set_error(GOL_EINVAL, "prefetch %d is not built for the band layout with t %d", c.pd, T);
  if (!c.band_rows) c.band_rows = default_band_rows(rows, cols, T, simd_count());
  const int32_t D = (int32_t)(2 * W);
  const hipError_t e = launch_board_pass(
      T, (const uint32_t*)d_strip, (uint32_t*)d_out, (int32_t)rows, (int32_t)cols, D,
      board_geometry(rows, cols, c.band_rows), c.pd, false, (hipStream_t)stream,
      (const uint32_t*)d_top, (const uint32_t*)d_bottom);
  return e == hipSuccess ? GOL_OK : hip_error(e, "strip pass launch");
}

int gol_population(const uint64_t* d_packed, int64_t rows, int64_t cols, int64_t* d_count,
                   void* stream) {
  int rc = check_board(rows, cols, 0);
  if (rc) return rc;
  if (!d_packed || !d_count) return set_error(GOL_EINVAL, "null pointer");
  hipError_t e = launch_fill_u32((uint32_t*)d_count, 2, 0u, (hipStream_t)stream);
  if (e == hipSuccess)
    e = launch_population(d_packed, rows, cols, (unsigned long long*)d_count, (hipStream_t)stream);
  return e == hipSuccess ? GOL_OK : hip_error(e, "population kernel launch");
}

int gol_step_packed(const uint64_t* d_in, int64_t rows, int64_t cols, int64_t generations,
                    uint64_t* d_out, void* stream) {
  return gol_step_packed_ex(d_in, rows, cols, generations, d_out, stream, 0);
}

int gol_pack(const uint8_t* d_bytes, int64_t rows, int64_t cols, uint64_t* d_packed,
             void* stream) {
  int rc = check_board(rows, cols, 0);
  if (rc) return rc;
  if (!d_bytes || !d_packed) return set_error(GOL_EINVAL, "null pointer");
  hipError_t e = launch_pack(d_bytes, rows, cols, d_packed, (hipStream_t)stream);
  return e == hipSuccess ? GOL_OK : hip_error(e, "pack kernel launch");
}

int gol_unpack(const uint64_t* d_packed, int64_t rows, int64_t cols, uint8_t* d_bytes,
               void* stream) {
  int rc = check_board(rows, cols, 0);
  if (rc) return rc;
  if (!d_bytes || !d_packed) return set_error(GOL_EINVAL, "null pointer");
  hipError_t e = launch_unpack(d_packed, rows, cols, d_bytes, (hipStream_t)stream);
  return e == hipSuccess ? GOL_OK : hip_error(e, "unpack kernel launch");
}

int gol_batch_run(const gol_board* boards, int64_t n, void* stream) {
  try {
    return batch_run(boards, n, (hipStream_t)stream, 0);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(GOL_EDEVICE, "unexpected exception");
  }
}

int gol_plan_create(const gol_board* boards, int64_t n, int t_block, gol_plan** out) {
  gol_pass_config c{};
  c.t_block = t_block;
  return gol_plan_create_cfg(boards, n, &c, out);
}

int gol_plan_create_cfg(const gol_board* boards, int64_t n, const gol_pass_config* config,
                        gol_plan** out) {
  if (!out) return set_error(GOL_EINVAL, "null output pointer");
  *out = nullptr;
  gol_plan* p = nullptr;
  try {
    gol_pass_config cfg{};
    if (config) cfg = *config;
    if (cfg.t_block < 0 || cfg.band_rows < 0 || cfg.band_rows > 65535 || cfg.prefetch != 0 ||
        (cfg.layout != 0 && cfg.layout != GOL_LAYOUT_QUEUE))
      return set_error(GOL_EINVAL,
                       "a batch plan takes t_block (0, 1, 2, 4, 8, 12, 16) and band_rows "
                       "(0 .. 65535); prefetch must be 0 and layout 0 or GOL_LAYOUT_QUEUE");
    if (cfg.t_block != 0 && !valid_T(cfg.t_block))
      return set_error(GOL_EINVAL, "t_block must be 0, 1, 2, 4, 8, 12 or 16 (got %d)",
                       cfg.t_block);
    const bool queue = cfg.layout == GOL_LAYOUT_QUEUE;
    int T = cfg.t_block, band = cfg.band_rows;
    if (queue) {
      if (!T) T = 12;
      if (!band) band = kBatchBandRows;
      if (!(T == 8 || T == 12 || T == 16))
        return set_error(GOL_EINVAL, "the queue form runs t_block 8, 12 or 16 (got %d)", T);
    } else if (T == 0 || band == 0) {
      int rc = tune_plan(boards, n, &T, &band);
      if (rc) return rc;
    }
    p = new gol_plan();
    p->queue = queue;
    int rc = plan_boards(boards, n, T, band, p->P);
    if (rc) {
      delete p;
      return rc;
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      delete p;
      return hip_error(e, "hipGetDevice");
    }
    if (p->P.scratch_words) {
      e = hipMalloc((void**)&p->P.d_scratch, p->P.scratch_words * 8);
      if (e != hipSuccess) {
        delete p;
        return set_error(GOL_ENOMEM, "hipMalloc scratch (%zu bytes): %s", p->P.scratch_words * 8,
                         hipGetErrorString(e));
      }
    }
    fill_board_descs(p->P);
    if (queue) {
      rc = setup_queue(p, T, band);
      if (rc) {
        (void)hipFree(p->P.d_scratch);
        delete p;
        return rc;
      }
      *out = p;
      return GOL_OK;
    }
    size_t ob, os, oi;
    const size_t mb = meta_bytes(p->P, &ob, &os, &oi);
    e = hipMalloc(&p->meta, mb);
    if (e != hipSuccess) {
      (void)hipFree(p->P.d_scratch);
      delete p;
      return set_error(GOL_ENOMEM, "hipMalloc plan tables: %s", hipGetErrorString(e));
    }
    std::vector<char> host(mb);
    fill_meta_host(p->P, host.data(), ob, os, oi);
    e = hipMemcpy(p->meta, host.data(), mb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p->meta);
      (void)hipFree(p->P.d_scratch);
      delete p;
      return hip_error(e, "hipMemcpy plan tables");
    }
    p->P.d_boards = (BoardDesc*)((char*)p->meta + ob);
    p->P.d_segs = (Segment*)((char*)p->meta + os);
    p->P.d_items = (WaveItem*)((char*)p->meta + oi);
    e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
    if (e != hipSuccess) {
      rc = hip_error(e, "plan stream and events");
      (void)gol_plan_destroy(p);
      return rc;
    }
    *out = p;
    return GOL_OK;
  } catch (const std::bad_alloc&) {
    delete p;
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
}

int gol_plan_run(gol_plan* p, void* stream) {
  if (!p) return set_error(GOL_EINVAL, "null plan");
  hipStream_t st = (hipStream_t)stream;
  if (st == nullptr) {
    hipError_t e = p->queue ? enqueue_queue(p, st) : enqueue_plan(p->P, st, p->side, p->fork,
                                                                    p->join);
    if (e == hipSuccess) e = plan_mark_run(p, st);
    return e == hipSuccess ? GOL_OK : hip_error(e, "gol_plan_run");
  }
  if (!p->exec) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    hipError_t el = p->queue ? enqueue_queue(p, st)
                             : enqueue_plan(p->P, st, p->side, p->fork, p->join);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (el != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_error(el, "plan launch during capture");
    }
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      p->exec = nullptr;
      return hip_error(e, "hipGraphInstantiate");
    }
    p->graph = g;
  }
  hipError_t e = hipGraphLaunch(p->exec, st);
  if (e == hipSuccess) e = plan_mark_run(p, st);
  return e == hipSuccess ? GOL_OK : hip_error(e, "hipGraphLaunch");
}

int gol_plan_config(const gol_plan* p, gol_pass_config* out) {
  if (!p || !out) return set_error(GOL_EINVAL, "null argument");
  *out = gol_pass_config{};
  out->t_block = p->P.hp.T;
  out->band_rows = p->P.hp.band_rows;
  out->layout = p->queue ? GOL_LAYOUT_QUEUE : 0;
  return GOL_OK;
}

int gol_plan_info(const gol_plan* p, int64_t* waves, int64_t* levels, double* cell_updates) {
  if (!p) return set_error(GOL_EINVAL, "null plan");
  if (waves) *waves = p->P.hp.level_items.empty() ? 0 : p->P.hp.level_items[0];
  if (levels) *levels = (int64_t)p->P.hp.level_items.size();
  if (cell_updates) *cell_updates = p->P.hp.cell_updates;
  return GOL_OK;
}

int gol_plan_destroy(gol_plan* p) {
  if (!p) return GOL_OK;
  // the plan's buffers and graph are in use until its queued runs end
  for (hipEvent_t ev : p->runs) {
    (void)hipEventSynchronize(ev);
    (void)hipEventDestroy(ev);
  }
  p->runs.clear();
  if (p->side) (void)hipStreamSynchronize(p->side);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->meta) (void)hipFree(p->meta);
  if (p->P.d_scratch) (void)hipFree(p->P.d_scratch);
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->join) (void)hipEventDestroy(p->join);
  if (p->side) (void)hipStreamDestroy(p->side);
  delete p;
  return GOL_OK;
}

int gol_set_allocator(gol_alloc_fn alloc, gol_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return set_error(GOL_EINVAL, "alloc and free must both be set or both be NULL");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_ctx = ctx;
  return GOL_OK;
}

// Host-only view of a batch schedule (no device work): used to test the
// planner.  rows/cols/generations: n entries.  Writes up to cap_segs
// segments and cap_items waves; returns their counts, the level sizes (up to
// cap_levels pairs), the late group's first wave and each board's first
// level.  Returns GOL_EINVAL on invalid boards.
static void copy_plan_tables(const HostPlan& hp, void* segs, int64_t cap_segs, void* items,
                             int64_t cap_items, int32_t* levels, int64_t cap_levels,
                             int32_t* starts, int32_t* late_begin, int64_t* nsegs,
                             int64_t* nitems, int64_t* nlevels) {
  if (nsegs) *nsegs = (int64_t)hp.segs.size();
  if (nitems) *nitems = (int64_t)hp.items.size();
  if (nlevels) *nlevels = (int64_t)hp.level_items.size();
  if (segs)
    memcpy(segs, hp.segs.data(),
           std::min<size_t>(hp.segs.size(), (size_t)cap_segs) * sizeof(Segment));
  if (items)
    memcpy(items, hp.items.data(),
           std::min<size_t>(hp.items.size(), (size_t)cap_items) * sizeof(WaveItem));
  if (levels)
    for (size_t L = 0; L < std::min<size_t>(hp.level_items.size(), (size_t)cap_levels); ++L) {
      levels[2 * L] = hp.level_early[L];
      levels[2 * L + 1] = hp.level_late[L];
    }
  if (starts) memcpy(starts, hp.start.data(), hp.start.size() * sizeof(int32_t));
  if (late_begin) *late_begin = hp.late_begin;
}

int gol_debug_plan_tables(const int64_t* rows, const int64_t* cols, const int64_t* gens, int64_t n,
                          int t_block, int band_rows, void* segs, int64_t cap_segs, void* items,
                          int64_t cap_items, int32_t* levels, int64_t cap_levels,
                          int32_t* starts, int32_t* late_begin, int64_t* nsegs, int64_t* nitems,
                          int64_t* nlevels) {
  try {
    if (n < 0 || (n > 0 && (!rows || !cols || !gens))) return set_error(GOL_EINVAL, "bad arrays");
    std::vector<BoardReq> req((size_t)n);
    for (int64_t b = 0; b < n; ++b) req[b] = BoardReq{rows[b], cols[b], gens[b]};
    HostPlan hp;
    std::string err;
    if (t_block == 0) t_block = default_batch_T();
    if (!build_plan(req, t_block, band_rows > 0 ? band_rows : 64, hp, err))
      return set_error(GOL_EINVAL, "%s", err.c_str());
    copy_plan_tables(hp, segs, cap_segs, items, cap_items, levels, cap_levels, starts,
                     late_begin, nsegs, nitems, nlevels);
    return GOL_OK;
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
}

int gol_debug_plan_queue_gave_up(gol_plan* p, int32_t* gave_up) {
  if (!p || !gave_up) return set_error(GOL_EINVAL, "null argument");
  *gave_up = 0;
  if (!p->queue) return GOL_OK;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    for (hipEvent_t ev : p->runs) {
      const hipError_t e = hipEventSynchronize(ev);
      if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
    }
  }
  uint32_t w = 0;
  const hipError_t e = hipMemcpy(&w, p->d_ctl + 1, sizeof(w), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, "hipMemcpy queue status");
  *gave_up = (int32_t)w;
  return GOL_OK;
}

int gol_debug_chunk_plan_tables(const int64_t* rows, const int64_t* cols, const int64_t* gens,
                                int64_t n, int t_block, int band_rows, void* segs,
                                int64_t cap_segs, void* items, int64_t cap_items,
                                int32_t* levels, int64_t cap_levels, int32_t* starts,
                                int32_t* late_begin, int64_t* nsegs, int64_t* nitems,
                                int64_t* nlevels, int32_t* band_used) {
  try {
    if (n < 0 || (n > 0 && (!rows || !cols || !gens))) return set_error(GOL_EINVAL, "bad arrays");
    if (t_block == 0) t_block = default_batch_T();
    if (!valid_T(t_block)) return set_error(GOL_EINVAL, "t_block must be 0, 1, 2, 4, 8, 12 or 16");
    std::vector<std::pair<int64_t, int64_t>> dims;
    for (int64_t b = 0; b < n; ++b) {
      const int rc = check_board(rows[b], cols[b], gens[b]);
      if (rc) return rc;
      dims.emplace_back(rows[b], cols[b]);
    }
    const int h = band_rows > 0 ? band_rows : chunk_band_rows(dims, t_block, 1024, kBatchBandRows);
    if (h > 65535) return set_error(GOL_EINVAL, "band height out of range");
    std::vector<BoardTiles> tiles((size_t)n);
    std::vector<ChunkBoard> req((size_t)n);
    for (int64_t b = 0; b < n; ++b) {
      board_tiles(rows[b], cols[b], h, tiles[b]);
      req[b] = ChunkBoard{&tiles[b], rows[b], cols[b], gens[b]};
    }
    HostPlan hp;
    std::string err;
    if (!build_chunk_plan(req, t_block, hp, err)) return set_error(GOL_EINVAL, "%s", err.c_str());
    copy_plan_tables(hp, segs, cap_segs, items, cap_items, levels, cap_levels, starts,
                     late_begin, nsegs, nitems, nlevels);
    if (band_used) *band_used = h;
    return GOL_OK;
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
}

}  // extern "C"

// Serving loop with continuous batching (gol_serve_* in include/gol.h).
//
// One scheduler thread per server.  Each tick it
//   1. admits queued requests, oldest first, while their two device buffers
//      fit the HBM budget: device memory and the host-to-device copy are
//      queued on the upload stream, followed by a marker;
//   2. queues one chunk on the compute stream: every resident board whose
//      upload marker the host has seen done advances min(chunk length,
//      remaining) generations in one batched schedule of tile passes (so a
//      chunk never stalls the device on an upload still in flight);
//   3. for boards that finish in that chunk, queues the device-to-host copy
//      (download stream, after the chunk) and the release of their buffers.
// Submissions reach the scheduler through an inbox with its own lock, so a
// client never waits for a scheduler tick.  Board state stays in device
// memory between chunks.  Up to two chunks are
// in flight, so the host prepares the next while the device runs the last.
// Each board keeps its tiles from chunk to chunk (rebuilt only when the band
// height changes), so a chunk's schedule is assembled in time linear in its
// tiles; its tables go through a ring of reused pinned and device buffers.
//
// The scheduler talks to the device through an executor.  HipExec is the
// real one (compute streams, upload and download streams, events,
// stream-ordered memory with released board buffers cached by size class,
// the library's pinned staging pool).
// HostExec keeps boards in host memory and completes every operation at once;
// it exists so the scheduling policy (admission order, budget, chunking,
// buffer bookkeeping, retirement, cancellation, failures) and each chunk's
// schedule can be tested on a machine without a GPU.  It replays a chunk's
// levels and tiles as the device would, standing in for a pass of t
// generations over a tile by adding t to every 32-bit word of the tile,
// which composes like the real step (two passes of a and b generations equal
// a + b) and shows whether every pass read and wrote the right buffers and
// covered every word once.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gol.h"
#include "gol_debug.h"
#include "gol_internal.h"
#include "gol_plan.h"
#include "gol_runtime.h"

namespace gol {

namespace {

// Opaque marker of queued device work; done() says whether it has run.
using Token = void*;

// What the scheduler needs from the device.  Copies and buffer work go in
// one queue ("copy"), chunks in another ("compute").  Calls return GOL_OK or
// an error code with the message set.
class Exec {
 public:
  virtual ~Exec() = default;
  virtual int bind_thread() = 0;
  virtual int simd_count() const { return 1024; }  // SIMDs of the device (band model)
  // Host staging of results (pinned where the device is real): *cls
  // identifies the block for host_free; cls 0 = plain malloc'd memory.
  virtual void* host_alloc(size_t bytes, size_t* cls) = 0;
  virtual void host_free(void* p, size_t cls) = 0;
  // Host staging of a submitted board until its upload (called by the
  // submitting thread, without the server lock): plain memory here.
  virtual void* stage_alloc(size_t bytes, size_t* cls) {
    *cls = 0;
    return malloc(bytes ? bytes : 1);
  }
  // Device bytes one board buffer of `bytes` takes (what the budget counts).
  virtual size_t block_bytes(size_t bytes) const { return bytes; }
  // Device bytes the executor may keep in released board buffers for reuse.
  virtual void set_block_cache_limit(uint64_t bytes) { (void)bytes; }
  virtual int board_alloc(size_t bytes, void** p) = 0;  // in copy-queue order
  virtual void board_free_after_copies(void* p) = 0;
  virtual void board_free_after_chunks(void* p) = 0;
  virtual int upload(void* dev, const void* host, size_t bytes) = 0;
  // A marker after the uploads queued so far (done() once they have run).
  virtual int upload_mark(Token* mark) = 0;
  // Chunks / result copies queued from now on come after the uploads before
  // a marker (one the host has seen done: the device does not stall on it).
  virtual int chunks_wait_for_upload(Token mark) = 0;
  virtual int copies_wait_for_upload(Token mark) = 0;
  virtual int run_chunk(const std::vector<BoardDesc>& bd, const HostPlan& hp, Token* done) = 0;
  virtual int copies_wait_for(Token chunk) = 0;
  virtual int download(void* host, const void* dev, size_t bytes, Token* done) = 0;
  // release `pinned` once everything queued so far on one queue has run
  virtual int host_free_after(bool compute, void* pinned, size_t cls) = 0;
  virtual bool done(Token t) = 0;
  virtual double seconds(Token chunk) = 0;  // device time of a completed chunk
  // Device time between the end of the chunk completed before this one and
  // this one's start (0 if unknown); called once per chunk, in order.
  virtual double gap_before(Token chunk) { (void)chunk; return 0.0; }
  // No chunk is queued: the next one starts a new run of chunks.
  virtual void chunks_idle() {}
  virtual void release(Token t) = 0;
  virtual void reap() = 0;
  virtual void sync() = 0;
};

class HipExec : public Exec {
 public:
  explicit HipExec(int device) : dev_(device) {}
  ~HipExec() override {
    sync();
    reap();  // everything has run: every deferred release happens here
    for (auto& kv : cache_)
      for (void* p : kv.second) (void)hipFreeAsync(p, up_);
    cache_.clear();
    sync();
    for (Slot& c : slots_) {
      for (hipEvent_t ev : {c.start, c.end, c.fork, c.join})
        if (ev) (void)hipEventDestroy(ev);
      if (c.meta) (void)hipFree(c.meta);
      if (c.pin) pinned_put(c.pin, c.pin_bytes);
    }
    for (Copy* c : copies_free_) {
      if (c->end) (void)hipEventDestroy(c->end);
      delete c;
    }
    for (hipEvent_t ev : events_) (void)hipEventDestroy(ev);
    if (ref_) (void)hipEventDestroy(ref_);
    if (compute_) (void)hipStreamDestroy(compute_);
    if (compute2_) (void)hipStreamDestroy(compute2_);
    if (up_) (void)hipStreamDestroy(up_);
    if (down_) (void)hipStreamDestroy(down_);
  }
  int init() {
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(dev_);
    // All four streams get hardware queues of their own: streams created
    // plainly share the runtime's few queues (GPU_MAX_HW_QUEUES) with every
    // other stream of the process, so which queues they land on depends on
    // the streams created and destroyed before.  A compute stream sharing a
    // queue with the download stream waits behind its copies and the device
    // idles between chunks (measured: 0.15 s of gaps instead of 0.02 over a
    // stream of about 0.8 s, 7 % less throughput at 0.7 of capacity and 18 %
    // at 0.9); the upload stream sharing one with the download stream, whose
    // copies wait for chunks, makes single upload calls hold up the scheduler
    // thread for up to 40 ms (measured on a second server of one process: a
    // saturated burst 0.8 of the first server's rate).  A stream with a CU
    // mask (here every CU, so it runs like any other) has a queue of its own.
    std::vector<uint32_t> all_cus;
    int ncu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev_);
    if (e == hipSuccess) {
      all_cus.assign((size_t)(ncu + 31) / 32, 0u);
      for (int i = 0; i < ncu; ++i) all_cus[(size_t)i / 32] |= 1u << (i % 32);
      e = hipExtStreamCreateWithCUMask(&compute_, (uint32_t)all_cus.size(), all_cus.data());
    }
    if (e == hipSuccess)
      e = hipExtStreamCreateWithCUMask(&compute2_, (uint32_t)all_cus.size(), all_cus.data());
    if (e == hipSuccess)
      e = hipExtStreamCreateWithCUMask(&up_, (uint32_t)all_cus.size(), all_cus.data());
    if (e == hipSuccess)
      e = hipExtStreamCreateWithCUMask(&down_, (uint32_t)all_cus.size(), all_cus.data());
    if (e == hipSuccess) e = hipEventCreate(&ref_);
    for (Slot& c : slots_) {
      if (e == hipSuccess) e = hipEventCreate(&c.start);
      if (e == hipSuccess) e = hipEventCreate(&c.end);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c.fork, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c.join, hipEventDisableTiming);
    }
    if (e == hipSuccess) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, dev_) == hipSuccess) {
        uint64_t thr = UINT64_MAX;  // keep freed blocks cached in the pool
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
      }
    }
    if (e == hipSuccess && ncu > 0) nsimd_ = 4 * ncu;
    (void)hipSetDevice(prev);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server streams");
  }
  int simd_count() const override { return nsimd_; }
  int bind_thread() override {
    hipError_t e = hipSetDevice(dev_);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: hipSetDevice");
  }
  void* host_alloc(size_t bytes, size_t* cls) override {
    void* p = pinned_get(bytes, cls);
    if (p) pinned_held_ += *cls;
    return p;
  }
  // Submitted boards are staged in pinned blocks of the library's pool while
  // the server holds less than kStagePinnedMax bytes of pinned staging, so
  // their uploads are asynchronous copies that do not hold up the scheduler
  // thread (an upload from pageable memory returns only once the runtime
  // has staged it); beyond that, in plain memory.
  void* stage_alloc(size_t bytes, size_t* cls) override {
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    if (pinned_held_.fetch_add(c) + c <= kStagePinnedMax) {
      void* p = pinned_get(bytes, cls);
      if (p) return p;
    }
    pinned_held_ -= c;
    return Exec::stage_alloc(bytes, cls);
  }
  void host_free(void* p, size_t cls) override {
    if (cls == 0) {
      free(p);
    } else {
      pinned_put(p, cls);
      pinned_held_ -= cls;
    }
  }
  // Board buffers come in size classes a quarter power of two apart (at
  // most 25 % above the board's bytes, at least 4 KiB).
  size_t block_bytes(size_t bytes) const override {
    if (bytes <= 4096) return 4096;
    size_t top = 1;
    while (top <= (bytes - 1) / 2) top <<= 1;  // largest power of two below bytes
    const size_t step = top / 4;
    return (bytes + step - 1) / step * step;
  }
  void set_block_cache_limit(uint64_t bytes) override { cache_limit_ = bytes; }
  // A released buffer of the same class if one is cached, else a new one
  // from the stream-ordered pool; cached buffers go back to the pool first
  // when the pool is short or the blocks held would pass the cache limit.
  int board_alloc(size_t bytes, void** p) override {
    const size_t c = block_bytes(bytes);
    auto it = cache_.find(c);
    if (it != cache_.end() && !it->second.empty()) {
      *p = it->second.back();
      it->second.pop_back();
      cached_bytes_ -= c;
      return GOL_OK;
    }
    while (held_ + c > cache_limit_ && cached_bytes_ > 0) drop_cached();
    hipError_t e = hipMallocAsync(p, c, up_);
    if (e != hipSuccess && cached_bytes_ > 0) {
      (void)hipGetLastError();
      while (cached_bytes_ > 0) drop_cached();
      e = hipMallocAsync(p, c, up_);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return set_error(GOL_ENOMEM, "server: device allocation of %zu bytes failed", c);
    }
    block_cls_[*p] = c;
    held_ += c;
    return GOL_OK;
  }
  // A board's buffers are released only once the host has seen their last
  // use complete (the result download, or the chunks already queued for a
  // cancelled board): a block handed to the next admission before then
  // could be overwritten by its upload before the last use had run.  Then
  // they are cached for the next board of their class while the blocks held
  // stay within the cache limit, else returned to the stream-ordered pool on
  // the stream that allocates them.  Returning them is what a busy server
  // avoids: single hipFreeAsync calls have held the scheduler thread for up
  // to 70 ms (seven such calls cost a saturated burst of 0.9 s about 0.18 s
  // of device idle time).
  void board_free_after_copies(void* p) override { free_after(p, down_); }
  void board_free_after_chunks(void* p) override { free_after(p, compute_); }
  int upload(void* dev, const void* host, size_t bytes) override {
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, up_);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: host-to-device copy");
  }
  int upload_mark(Token* mark) override {
    Copy* c = copy_get();
    hipError_t e = c->end ? hipSuccess : event_get(&c->end);
    if (e == hipSuccess) e = hipEventRecord(c->end, up_);
    if (e != hipSuccess) {
      copies_free_.push_back(c);
      return hip_error(e, "server: upload marker");
    }
    *mark = c;
    return GOL_OK;
  }
  int chunks_wait_for_upload(Token mark) override {
    hipError_t e = hipStreamWaitEvent(compute_, ((Copy*)mark)->end, 0);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: stream wait");
  }
  int copies_wait_for_upload(Token mark) override {
    hipError_t e = hipStreamWaitEvent(down_, ((Copy*)mark)->end, 0);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: stream wait");
  }
  // A chunk's tables go through the next of a ring of slots, each keeping
  // its pinned staging, its device table block and its four events from one
  // chunk to the next (grown, never shrunk), so a chunk allocates nothing.
  // At most two chunks are in flight, so the slot a chunk takes last served
  // the chunk three before it, which has completed.
  int run_chunk(const std::vector<BoardDesc>& bd, const HostPlan& hp, Token* done) override {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t os = al(bd.size() * sizeof(BoardDesc));
    const size_t oi = os + al(hp.segs.size() * sizeof(Segment));
    const size_t mb = oi + al(hp.items.size() * sizeof(WaveItem));
    Slot& c = slots_[next_slot_];
    next_slot_ = (next_slot_ + 1) % kSlots;
    hipError_t e = hipSuccess;
    if (c.busy) e = hipEventSynchronize(c.end);  // not reached while two chunks at most are queued
    c.busy = false;
    if (e == hipSuccess && c.pin_bytes < mb) {
      // from the library's pinned pool: freeing page-locked memory waits for
      // the device, which would drain the chunks in flight
      if (c.pin) pinned_put(c.pin, c.pin_bytes);
      c.pin = pinned_get(std::max(2 * mb, kSlotMinBytes), &c.pin_bytes);
      if (!c.pin) {
        c.pin_bytes = 0;
        e = hipErrorOutOfMemory;
      }
    }
    if (e == hipSuccess && c.meta_bytes < mb) {
      if (c.meta) (void)hipFreeAsync(c.meta, compute_);
      c.meta = nullptr;
      c.meta_bytes = 0;
      const size_t want = std::max(2 * mb, kSlotMinBytes);
      e = hipMallocAsync(&c.meta, want, compute_);
      if (e == hipSuccess) c.meta_bytes = want;
    }
    if (e != hipSuccess) return hip_error(e, "server: chunk tables");
    char* pin = (char*)c.pin;
    memcpy(pin, bd.data(), bd.size() * sizeof(BoardDesc));
    memcpy(pin + os, hp.segs.data(), hp.segs.size() * sizeof(Segment));
    memcpy(pin + oi, hp.items.data(), hp.items.size() * sizeof(WaveItem));
    if (e == hipSuccess && !ref_valid_) {
      e = hipEventRecord(ref_, compute_);
      ref_valid_ = e == hipSuccess;
      prev_end_ = -1.0;
    }
    if (e == hipSuccess) e = hipEventRecord(c.start, compute_);
    if (e == hipSuccess) e = hipMemcpyAsync(c.meta, pin, mb, hipMemcpyHostToDevice, compute_);
    const BoardDesc* d_b = (const BoardDesc*)c.meta;
    const Segment* d_s = (const Segment*)((char*)c.meta + os);
    const WaveItem* d_i = (const WaveItem*)((char*)c.meta + oi);
    if (e == hipSuccess) e = enqueue_levels(hp, d_b, d_s, d_i, compute_, compute2_, c.fork, c.join);
    if (e == hipSuccess) e = hipEventRecord(c.end, compute_);
    if (e != hipSuccess) return hip_error(e, "server: chunk launch");
    c.busy = true;
    *done = &c;
    return GOL_OK;
  }
  int copies_wait_for(Token chunk) override {
    hipError_t e = hipStreamWaitEvent(down_, ((Slot*)chunk)->end, 0);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: stream wait");
  }
  int download(void* host, const void* dev, size_t bytes, Token* done) override {
    Copy* c = copy_get();
    hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, down_);
    if (e == hipSuccess && !c->end) e = event_get(&c->end);
    if (e == hipSuccess) e = hipEventRecord(c->end, down_);
    if (e != hipSuccess) {
      copies_free_.push_back(c);
      return hip_error(e, "server: result copy");
    }
    *done = c;
    return GOL_OK;
  }
  int host_free_after(bool compute, void* pinned, size_t cls) override {
    hipEvent_t ev = nullptr;
    hipError_t e = event_get(&ev);
    if (e == hipSuccess) e = hipEventRecord(ev, compute ? compute_ : up_);
    if (e != hipSuccess) {
      if (ev) events_.push_back(ev);
      return hip_error(e, "server: event record");
    }
    pending_.push_back(Pending{ev, pinned, cls, nullptr});
    return GOL_OK;
  }
  bool done(Token t) override { return hipEventQuery(end_of(t)) == hipSuccess; }
  double seconds(Token t) override {
    const Tagged* g = (const Tagged*)t;
    if (g->kind != 0) return 0.0;
    const Slot* c = (const Slot*)t;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->start, c->end) != hipSuccess) {
      (void)hipGetLastError();
      return 0.0;
    }
    return ms * 1e-3;
  }
  // The slot before a chunk's in the ring held the chunk queued before it
  // (its events are reused only by the chunk after next, which is queued
  // after this one completes).
  // Both ends of each chunk are timed against one reference event recorded
  // before the first chunk of a run of chunks (consecutive chunks' own
  // events do not always give an elapsed time to each other).
  double gap_before(Token t) override {
    const Tagged* g = (const Tagged*)t;
    if (g->kind != 0 || !ref_valid_) return 0.0;
    const Slot* c = (const Slot*)t;
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, ref_, c->start) != hipSuccess ||
        hipEventElapsedTime(&b, ref_, c->end) != hipSuccess) {
      (void)hipGetLastError();
      prev_end_ = -1.0;
      return 0.0;
    }
    const double gap = prev_end_ >= 0.0 ? a * 1e-3 - prev_end_ : 0.0;
    prev_end_ = b * 1e-3;
    return gap > 0.0 ? gap : 0.0;
  }
  void chunks_idle() override { ref_valid_ = false; }
  void release(Token t) override {
    Tagged* g = (Tagged*)t;
    if (!g) return;
    if (g->kind == 0)
      ((Slot*)t)->busy = false;
    else
      copies_free_.push_back((Copy*)t);
  }
  void reap() override {
    size_t k = 0;
    for (auto& p : pending_) {
      if (hipEventQuery(p.ev) == hipSuccess) {
        events_.push_back(p.ev);
        if (p.device)
          release_block(p.device);
        else
          host_free(p.pinned, p.cls);
      } else {
        pending_[k++] = p;
      }
    }
    pending_.resize(k);
  }
  void sync() override {
    if (compute_) (void)hipStreamSynchronize(compute_);
    if (compute2_) (void)hipStreamSynchronize(compute2_);
    if (up_) (void)hipStreamSynchronize(up_);
    if (down_) (void)hipStreamSynchronize(down_);
  }

 private:
  // Tokens: a chunk's slot (kind 0), or a result copy or upload marker (kind 1).
  struct Tagged {
    int kind = 0;
  };
  struct Slot : Tagged {
    hipEvent_t start = nullptr, end = nullptr, fork = nullptr, join = nullptr;
    void* pin = nullptr;
    size_t pin_bytes = 0;
    void* meta = nullptr;
    size_t meta_bytes = 0;
    bool busy = false;
  };
  struct Copy : Tagged {
    hipEvent_t end = nullptr;  // kept with the record for its next use
  };
  Copy* copy_get() {
    Copy* c = nullptr;
    if (copies_free_.empty()) {
      c = new Copy();
    } else {
      c = copies_free_.back();
      copies_free_.pop_back();
    }
    c->kind = 1;
    return c;
  }
  // Waits on the host for an event: then the pinned block returns to the
  // pool, or the device block is released (release_block: cached or freed).
  struct Pending {
    hipEvent_t ev;
    void* pinned;
    size_t cls;
    void* device = nullptr;
  };
  void free_after(void* p, hipStream_t st) {
    if (!p) return;
    hipEvent_t ev = nullptr;
    if (event_get(&ev) == hipSuccess && hipEventRecord(ev, st) == hipSuccess) {
      pending_.push_back(Pending{ev, nullptr, 0, p});
      return;
    }
    (void)hipGetLastError();
    // no event: wait for the stream, then free
    if (ev) events_.push_back(ev);
    (void)hipStreamSynchronize(st);
    release_block(p);
  }
  void release_block(void* p) {
    auto it = block_cls_.find(p);
    const size_t c = it == block_cls_.end() ? 0 : it->second;
    if (c > 0 && held_ <= cache_limit_) {
      cache_[c].push_back(p);
      cached_bytes_ += c;
      return;
    }
    if (it != block_cls_.end()) block_cls_.erase(it);
    held_ -= c;
    (void)hipFreeAsync(p, up_);
  }
  // Returns one cached block (of the largest class) to the pool.
  void drop_cached() {
    auto it = cache_.end();
    while (it != cache_.begin()) {
      --it;
      if (!it->second.empty()) break;
    }
    if (it == cache_.end() || it->second.empty()) {
      cached_bytes_ = 0;
      return;
    }
    void* p = it->second.back();
    it->second.pop_back();
    cached_bytes_ -= it->first;
    held_ -= it->first;
    block_cls_.erase(p);
    (void)hipFreeAsync(p, up_);
  }
  static constexpr int kSlots = 3;
  // Smallest table block of a slot (pinned and device): a chunk over a few
  // thousand boards fits, so a busy server does not grow its tables (a new
  // device block is a stream-ordered allocation the compute stream waits on).
  static constexpr size_t kSlotMinBytes = (size_t)4 << 20;
  hipEvent_t end_of(Token t) const {
    const Tagged* g = (const Tagged*)t;
    return g->kind == 0 ? ((const Slot*)t)->end : ((const Copy*)t)->end;
  }
  // Events without timing from a free list (created on first need).
  hipError_t event_get(hipEvent_t* ev) {
    if (!events_.empty()) {
      *ev = events_.back();
      events_.pop_back();
      return hipSuccess;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
  }
  int dev_;
  int nsimd_ = 1024;
  hipStream_t compute_ = nullptr;
  // uploads (and the allocation of admitted boards) and result downloads (and
  // the release of retired boards) on separate streams, so an admission never
  // waits behind a download that waits for a chunk
  hipStream_t up_ = nullptr, down_ = nullptr;
  hipStream_t compute2_ = nullptr;  // the late group of each chunk's schedule
  Slot slots_[kSlots];
  int next_slot_ = 0;
  hipEvent_t ref_ = nullptr;  // timing reference of the current run of chunks
  bool ref_valid_ = false;
  double prev_end_ = -1.0;    // end of the last completed chunk, seconds after ref_
  std::vector<Copy*> copies_free_;
  std::vector<hipEvent_t> events_;  // free events
  std::vector<Pending> pending_;    // touched by the scheduler thread under the server lock
  // Board buffers (scheduler thread, under the server lock): the class of
  // every block taken from the pool, released blocks by class, and the bytes
  // held from the pool (in use or cached) and cached.
  std::unordered_map<void*, size_t> block_cls_;
  std::map<size_t, std::vector<void*>> cache_;
  uint64_t held_ = 0, cached_bytes_ = 0;
  uint64_t cache_limit_ = 0;
  static constexpr size_t kStagePinnedMax = (size_t)1 << 30;
  std::atomic<size_t> pinned_held_{0};  // pinned staging (inputs and results) held now
};

// Boards in host memory, every operation complete on return (see the file
// comment).  fail_at: the 1-based index of the chunk that reports a device
// error (0 = never).
class HostExec : public Exec {
 public:
  explicit HostExec(int64_t fail_at) : fail_at_(fail_at) {}
  int bind_thread() override { return GOL_OK; }
  void* host_alloc(size_t bytes, size_t* cls) override {
    *cls = 0;
    return malloc(bytes ? bytes : 1);
  }
  void host_free(void* p, size_t) override { free(p); }
  int board_alloc(size_t bytes, void** p) override {
    *p = malloc(bytes ? bytes : 1);
    if (!*p) return set_error(GOL_ENOMEM, "host executor: out of memory");
    std::lock_guard<std::mutex> lk(mu_);
    sizes_[*p] = bytes;
    live_ += bytes;
    peak_ = std::max(peak_, live_);
    return GOL_OK;
  }
  void board_free_after_copies(void* p) override { drop(p); }
  void board_free_after_chunks(void* p) override { drop(p); }
  int upload(void* dev, const void* host, size_t bytes) override {
    memcpy(dev, host, bytes);
    return GOL_OK;
  }
  int upload_mark(Token* mark) override {
    *mark = &token_;
    return GOL_OK;
  }
  int chunks_wait_for_upload(Token) override { return GOL_OK; }
  int copies_wait_for_upload(Token) override { return GOL_OK; }
  // Replays the chunk's schedule as the device would run it: level by level,
  // the early group's waves then the late group's, each segment taking the
  // pass of its board that the level runs (the buffer it reads and writes,
  // its generation count) exactly as the batch kernel selects them, and
  // standing in for that pass by adding its generation count to every
  // dword of the segment's tile.  A pass shorter than T in a level launched
  // without the per-lane generation mask would run T generations on the
  // device: reported as a device failure.
  int run_chunk(const std::vector<BoardDesc>& bd, const HostPlan& hp, Token* done) override {
    if (++chunks_ == fail_at_) return set_error(GOL_EDEVICE, "host executor: injected failure");
    const int Kmax = (int)hp.level_items.size();
    for (int L = 0; L < Kmax; ++L) {
      for (int grp = 0; grp < 2; ++grp) {
        const int begin = grp == 0 ? 0 : hp.late_begin;
        const int count = grp == 0 ? hp.level_early[L] : hp.level_late[L];
        const bool masked = grp == 0 ? (L == 0 && hp.early_masked)
                                     : (L == Kmax - 1 && hp.late_masked);
        for (int i = begin; i < begin + count; ++i) {
          const WaveItem& w = hp.items[i];
          for (int k = 0; k < w.nseg; ++k) {
            const Segment& sg = hp.segs[w.seg_begin + k];
            const BoardDesc& d = bd[sg.board];
            const int j = L - d.start;
            if (j < 0 || j >= d.K) continue;  // the board has no pass at this level
            const uint32_t* src = j == 0 ? d.src0 : d.w[(j - 1 + d.par) & 1];
            uint32_t* dst = d.w[(j + d.par) & 1];
            const int t = j == d.jshort ? d.Tshort : hp.T;
            if (t != hp.T && !masked)
              return set_error(GOL_EDEVICE, "host executor: a %d-generation pass at level %d "
                               "of a %d-generation schedule is not masked", t, L, hp.T);
            for (int r = sg.r0; r < sg.r0 + (int)sg.h; ++r)
              for (int p = sg.p0 + 1; p < sg.p0 + (int)sg.nlanes - 1; ++p)
                dst[(size_t)r * d.D + p] = src[(size_t)r * d.D + p] + (uint32_t)t;
          }
        }
      }
    }
    *done = &token_;
    return GOL_OK;
  }
  int copies_wait_for(Token) override { return GOL_OK; }
  int download(void* host, const void* dev, size_t bytes, Token* done) override {
    memcpy(host, dev, bytes);
    *done = &token_;
    return GOL_OK;
  }
  int host_free_after(bool, void* pinned, size_t cls) override {
    host_free(pinned, cls);
    return GOL_OK;
  }
  bool done(Token) override { return true; }
  double seconds(Token) override { return 0.0; }
  void release(Token) override {}
  void reap() override {}
  void sync() override {}
  size_t peak() const {
    std::lock_guard<std::mutex> lk(mu_);
    return peak_;
  }

 private:
  void drop(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    live_ -= sizes_[p];
    sizes_.erase(p);
    free(p);
  }
  int64_t fail_at_;
  int64_t chunks_ = 0;
  char token_ = 0;
  mutable std::mutex mu_;
  std::unordered_map<void*, size_t> sizes_;
  size_t live_ = 0, peak_ = 0;
};

enum class State { Queued, Resident, Done, Failed, Cancelled };

struct Request {
  uint64_t ticket = 0;
  int64_t rows = 0, cols = 0, W = 0, gens = 0;
  size_t bytes = 0;
  void* pin_in = nullptr;      // staged input (pinned or plain) until its upload
  size_t pin_in_cls = 0;
  void* pin_out = nullptr;
  size_t pin_out_cls = 0;
  uint64_t* d_buf[2] = {nullptr, nullptr};
  int cur = 0;                 // d_buf[cur] holds the state after the queued chunks
  int64_t queued_gens = 0;     // generations covered by chunks queued so far
  State state = State::Queued;
  bool cancel = false;
  bool retiring = false;       // final copy queued
  Token out_done = nullptr;    // device-to-host copy of the result done
  uint64_t mark = 0;           // upload marker its input copy precedes
  BoardTiles tiles;            // the board's tiles at the band height last used
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::string err;
};

}  // namespace

struct Server {
  gol_serve_config cfg{};
  std::chrono::steady_clock::time_point t0;
  std::unique_ptr<Exec> exec;
  HostExec* host_exec = nullptr;  // set when exec is the host executor

  std::mutex mu;
  std::condition_variable cv_work;   // scheduler wakes on submit / cancel / stop
  std::condition_variable cv_done;   // waiters wake on completion
  bool stop = false;
  bool failed = false;
  std::string fail_msg;

  // Submissions land in the inbox under in_mu, never under mu, which a busy
  // scheduler holds for whole ticks; whoever holds mu moves them into reqs
  // and the admission queue (drain_inbox).  Before an idle wait the
  // scheduler sets `sleeping` and rechecks inbox_n; a submitter that finds
  // `sleeping` set takes mu to wake it, so no submission waits out a sleep.
  std::mutex in_mu;
  std::vector<std::unique_ptr<Request>> inbox;  // under in_mu
  uint64_t next_ticket = 1;                     // under in_mu
  std::atomic<int64_t> inbox_n{0};
  std::atomic<bool> sleeping{false};
  std::atomic<bool> failed_seen{false};  // S.failed, readable without mu
  std::deque<uint64_t> queue;                      // admission order
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<uint64_t> resident;                  // admitted, not yet retired
  uint64_t used_bytes = 0;

  std::deque<Token> chunks;                        // queued chunks, oldest first
  std::deque<double> chunk_cu;                     // their cell updates
  int T = 16;                                      // generations per pass (resolved)
  int band = 96;                                   // band height of a busy chunk (resolved)
  double rate = 0.0;  // cell updates per device second of completed chunks (running mean)
  double t_starved = -1.0;  // when the last queued chunk was seen done with work left over

  // Upload markers, one per admitting tick, numbered 1, 2, ...: a board
  // joins chunks (or, with no generations, retires) once the host has seen
  // its marker done, so a chunk never waits on the device for an upload
  // still in flight; the device-side wait on a done marker keeps the copy
  // ordered before the kernels that read it.
  std::deque<std::pair<uint64_t, Token>> marks;  // issued, not yet seen done
  uint64_t mark_seq = 0;       // last issued
  uint64_t uploaded = 0;       // last seen done
  Token uploaded_mark = nullptr;  // its marker (kept for the waits below)
  uint64_t chunks_after = 0;   // chunks queued from now on follow uploads up to this marker
  uint64_t copies_after = 0;   // result copies likewise
  gol_serve_stats stats{};
  std::thread th;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

static void fail_all(Server& S, const std::string& msg) {
  // caller holds S.mu
  S.failed = true;
  S.failed_seen = true;
  S.fail_msg = msg;
  for (auto& kv : S.reqs) {
    Request& r = *kv.second;
    if (r.state == State::Queued || r.state == State::Resident) {
      r.state = State::Failed;
      r.err = msg;
    }
  }
  S.cv_done.notify_all();
}

// Submissions from the inbox into reqs and the admission queue, in ticket
// order.  Caller holds S.mu.
static void drain_inbox(Server& S) {
  if (S.inbox_n.load() == 0) return;
  std::vector<std::unique_ptr<Request>> got;
  {
    std::lock_guard<std::mutex> g(S.in_mu);
    got.swap(S.inbox);
    S.inbox_n = 0;
  }
  for (auto& r : got) {
    if (S.failed) {
      r->state = State::Failed;
      r->err = S.fail_msg;
      if (r->pin_in) S.exec->host_free(r->pin_in, r->pin_in_cls);
      r->pin_in = nullptr;
    } else {
      S.queue.push_back(r->ticket);
    }
    const uint64_t t = r->ticket;
    S.reqs.emplace(t, std::move(r));
  }
  if (S.failed) S.cv_done.notify_all();
}

static void reap(Server& S) {
  S.exec->reap();
  while (!S.marks.empty() && S.exec->done(S.marks.front().second)) {
    if (S.uploaded_mark) S.exec->release(S.uploaded_mark);
    S.uploaded = S.marks.front().first;
    S.uploaded_mark = S.marks.front().second;
    S.marks.pop_front();
  }
  while (!S.chunks.empty() && S.exec->done(S.chunks.front())) {
    const double secs = S.exec->seconds(S.chunks.front());
    const double cu = S.chunk_cu.front();
    S.stats.device_busy_s += secs;
    S.stats.chunk_gap_s += S.exec->gap_before(S.chunks.front());
    if (secs > 0.0 && cu > 0.0)
      S.rate = S.rate > 0.0 ? 0.75 * S.rate + 0.25 * (cu / secs) : cu / secs;
    S.exec->release(S.chunks.front());
    S.chunks.pop_front();
    S.chunk_cu.pop_front();
    if (S.chunks.empty()) S.exec->chunks_idle();
    if (S.chunks.empty() && S.t_starved < 0.0) {
      bool work = !S.queue.empty();
      for (size_t i = 0; !work && i < S.resident.size(); ++i) {
        const Request& r = *S.reqs[S.resident[i]];
        work = !r.cancel && !r.retiring && r.queued_gens < r.gens;
      }
      if (work) S.t_starved = S.now();
    }
  }
}

// Host seconds one scheduler tick spends admitting requests before it goes
// on to queue chunks and retire boards: a device with fewer than two chunks
// queued gets the next one sooner.
constexpr double kAdmitSliceHungry = 0.0003;
constexpr double kAdmitSlice = 0.001;

// Device time a chunk of an automatic length aims at: long enough that its
// launches and host work are small beside it, short enough that a request
// arriving meanwhile waits little before it joins.  Behind a deep backlog
// (the work resident and queued would take more than 16 such chunks) the
// chunk aims at a sixteenth of that backlog, up to kChunkTargetMaxSeconds:
// every request then waits mostly for the backlog anyway, and fewer chunks
// end in fewer joins (measured with all 4096 requests of the served
// workload at once: 0.88 of the batched capacity against 0.85 at 3 ms,
// with the Poisson streams' rates and latencies unchanged).
constexpr double kChunkTargetSeconds = 0.003;
constexpr double kChunkTargetMaxSeconds = 0.024;
constexpr double kChunkBacklogShare = 1.0 / 16.0;
// Generations of the first chunks of an automatic length (no rate measured yet).
constexpr int64_t kChunkFirstPasses = 15;
constexpr int64_t kChunkMaxPasses = 256;

// Generations every board advances in the next chunk (at most; fewer if it
// finishes): the configured count, or (chunk_generations 0) as many whole
// passes as the resident cells take the target device time (above) at the
// rate measured on earlier chunks.
static int64_t chunk_generations(const Server& S, const std::vector<Request*>& act) {
  if (S.cfg.chunk_generations > 0) return S.cfg.chunk_generations;
  if (S.rate <= 0.0) return kChunkFirstPasses * S.T;
  double cells = 0.0, backlog = 0.0;  // cells in the chunk; cell updates left
  for (const Request* r : act) {
    cells += (double)r->rows * (double)r->cols;
    backlog += (double)r->rows * (double)r->cols * (double)(r->gens - r->queued_gens);
  }
  for (uint64_t t : S.queue) {
    const Request& q = *S.reqs.at(t);
    backlog += (double)q.rows * (double)q.cols * (double)q.gens;
  }
  const double target = std::min(kChunkTargetMaxSeconds,
                                 std::max(kChunkTargetSeconds, kChunkBacklogShare * backlog / S.rate));
  const double g = target * S.rate / std::max(cells, 1.0);
  const int64_t passes = std::min<int64_t>(kChunkMaxPasses,
                                           std::max<int64_t>(1, (int64_t)std::ceil(g / S.T)));
  return passes * S.T;
}

// Completed result copies -> Done.  Caller holds S.mu.
static void finish_copies(Server& S) {
  bool any = false;
  for (auto& kv : S.reqs) {
    Request& r = *kv.second;
    if (r.state == State::Resident && r.retiring && r.out_done && S.exec->done(r.out_done)) {
      S.exec->release(r.out_done);
      r.out_done = nullptr;
      r.state = State::Done;
      r.t_done = S.now();
      any = true;
    }
  }
  if (any) S.cv_done.notify_all();
}

// Device buffers and the input copy of an admitted board (copy queue).
// GOL_ENOMEM: the device could not give the buffers (nothing was queued).
static int admit(Server& S, Request& r) {
  // caller holds S.mu
  void* p0 = nullptr;
  void* p1 = nullptr;
  int rc = S.exec->board_alloc(r.bytes, &p0);
  if (!rc) rc = S.exec->board_alloc(r.bytes, &p1);
  if (rc) {
    if (p0) S.exec->board_free_after_copies(p0);
    return rc;
  }
  r.d_buf[0] = (uint64_t*)p0;
  r.d_buf[1] = (uint64_t*)p1;
  r.cur = 0;
  rc = S.exec->upload(p0, r.pin_in, r.bytes);
  r.mark = S.mark_seq + 1;  // the marker queued after this tick's admissions
  if (!rc) rc = S.exec->host_free_after(false, r.pin_in, r.pin_in_cls);
  if (rc) return rc == GOL_ENOMEM ? GOL_EDEVICE : rc;
  r.pin_in = nullptr;
  r.state = State::Resident;
  r.t_admit = S.now();
  S.stats.admitted += 1;
  return GOL_OK;
}

// Build and queue one chunk over the resident boards.  Caller holds S.mu.
// The band height is chosen per chunk for the boards in it (the occupancy
// model of chunk_band_rows); each board keeps its tiles for that height, so
// a chunk's schedule is assembled from them in time linear in the tiles.
static int queue_chunk(Server& S, std::vector<uint64_t>& retire_now) {
  std::vector<Request*> act;
  for (uint64_t t : S.resident) {
    Request& r = *S.reqs[t];
    if (!r.cancel && !r.retiring && r.queued_gens < r.gens && r.mark <= S.uploaded)
      act.push_back(&r);
  }
  if (act.empty()) return GOL_OK;
  const auto t_plan0 = std::chrono::steady_clock::now();
  const int T = S.T;
  const int64_t gchunk = chunk_generations(S, act);
  std::vector<std::pair<int64_t, int64_t>> dims;
  dims.reserve(act.size());
  for (Request* r : act) dims.emplace_back(r->rows, r->cols);
  const int h = chunk_band_rows(dims, T, S.exec->simd_count(), S.band);
  std::vector<ChunkBoard> req;
  req.reserve(act.size());
  for (Request* r : act) {
    if (r->tiles.band_rows != h) board_tiles(r->rows, r->cols, h, r->tiles);
    const int64_t g = std::min<int64_t>(gchunk, r->gens - r->queued_gens);
    req.push_back(ChunkBoard{&r->tiles, r->rows, r->cols, g});
  }
  HostPlan hp;
  std::string err;
  if (!build_chunk_plan(req, T, hp, err))
    return set_error(GOL_EINVAL, "server plan: %s", err.c_str());
  std::vector<BoardDesc> bd(act.size());
  for (size_t b = 0; b < act.size(); ++b) {
    Request& r = *act[b];
    BoardDesc& d = bd[b];
    d.R = (int32_t)r.rows;
    d.C = (int32_t)r.cols;
    d.D = (int32_t)(2 * r.W);
    d.K = hp.K[b];
    d.Tshort = hp.Tshort[b];
    d.start = hp.start[b];
    d.jshort = hp.jshort[b];
    d.src0 = (const uint32_t*)r.d_buf[r.cur];
    d.w[0] = (uint32_t*)r.d_buf[r.cur ^ 1];
    d.w[1] = (uint32_t*)r.d_buf[r.cur];
    d.par = 0;  // pass j writes w[j & 1]; the result lands in w[(K - 1) & 1]
  }
  Token done = nullptr;
  int rc = GOL_OK;
  bool fresh = false;
  for (const Request* r : act) fresh = fresh || r->mark > S.chunks_after;
  if (fresh) {
    rc = S.exec->chunks_wait_for_upload(S.uploaded_mark);
    if (rc) return rc;
    S.chunks_after = S.uploaded;
  }
  rc = S.exec->run_chunk(bd, hp, &done);
  S.stats.plan_host_s +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_plan0).count();
  if (rc) return rc;
  S.chunks.push_back(done);
  if (S.t_starved >= 0.0) {
    S.stats.starved_s += S.now() - S.t_starved;
    S.t_starved = -1.0;
  }
  S.chunk_cu.push_back(hp.cell_updates);
  S.stats.chunks += 1;
  S.stats.last_chunk_generations = gchunk;
  S.stats.last_band_rows = h;
  S.stats.launches += (int64_t)hp.level_items.size();
  S.stats.cell_updates += hp.cell_updates;
  S.stats.max_resident = std::max<int64_t>(S.stats.max_resident, (int64_t)act.size());
  S.stats.mean_resident += ((double)act.size() - S.stats.mean_resident) / (double)S.stats.chunks;
  for (size_t b = 0; b < act.size(); ++b) {
    Request& r = *act[b];
    r.queued_gens += req[b].generations;
    if (hp.K[b] & 1) r.cur ^= 1;
    if (r.queued_gens >= r.gens) retire_now.push_back(r.ticket);
  }
  // result copies wait for this chunk
  return S.exec->copies_wait_for(done);
}

// Queue result copy + buffer release for a finished board.  Caller holds S.mu.
static int queue_retire(Server& S, Request& r) {
  r.pin_out = S.exec->host_alloc(r.bytes, &r.pin_out_cls);
  if (!r.pin_out) return set_error(GOL_EDEVICE, "server: pinned result buffer");
  const int rc = S.exec->download(r.pin_out, r.d_buf[r.cur], r.bytes, &r.out_done);
  S.exec->board_free_after_copies(r.d_buf[0]);
  S.exec->board_free_after_copies(r.d_buf[1]);
  r.d_buf[0] = r.d_buf[1] = nullptr;
  S.used_bytes -= 2 * S.exec->block_bytes(r.bytes);
  r.retiring = true;
  S.stats.retired += 1;
  return rc;
}

// Drop a cancelled resident board: its buffers are released after the
// chunks already queued (compute order).  Caller holds S.mu.
static void drop_cancelled(Server& S, Request& r) {
  S.exec->board_free_after_chunks(r.d_buf[0]);
  S.exec->board_free_after_chunks(r.d_buf[1]);
  r.d_buf[0] = r.d_buf[1] = nullptr;
  S.used_bytes -= 2 * S.exec->block_bytes(r.bytes);
  r.state = State::Cancelled;
}

static void scheduler(Server* Sp) {
  Server& S = *Sp;
  {
    const int rc = S.exec->bind_thread();
    if (rc) {
      std::lock_guard<std::mutex> lk(S.mu);
      fail_all(S, last_error());
      return;
    }
  }
  std::unique_lock<std::mutex> lk(S.mu);
  while (true) {
    drain_inbox(S);
    reap(S);
    finish_copies(S);
    if (S.stop) break;
    if (S.failed) {
      S.cv_work.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    int rc = GOL_OK;
    bool did = false;
    // cancelled resident boards leave
    for (size_t i = 0; i < S.resident.size();) {
      Request& r = *S.reqs[S.resident[i]];
      if (r.cancel && !r.retiring) {
        drop_cancelled(S, r);
        S.resident.erase(S.resident.begin() + i);
        S.cv_done.notify_all();
        did = true;
      } else {
        ++i;
      }
    }
    // admission, oldest first, under the budget and the resident cap, for at
    // most a slice of host time per tick (shorter while the device has fewer
    // than two chunks to run), so that a burst of submissions is admitted
    // over several ticks between which chunks keep the device busy
    bool admitted = false;
    const auto t_admit0 = std::chrono::steady_clock::now();
    const double slice = S.chunks.size() < 2 ? kAdmitSliceHungry : kAdmitSlice;
    while (!S.queue.empty()) {
      if (admitted && !S.resident.empty() &&
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_admit0).count() >
              slice)
        break;
      Request& r = *S.reqs[S.queue.front()];
      if (r.cancel) {
        r.state = State::Cancelled;
        if (r.pin_in) S.exec->host_free(r.pin_in, r.pin_in_cls);
        r.pin_in = nullptr;
        S.queue.pop_front();
        S.cv_done.notify_all();
        continue;
      }
      const uint64_t need = 2 * (uint64_t)S.exec->block_bytes(r.bytes);
      const bool cap_ok = S.cfg.max_resident <= 0 ||
                          (int64_t)S.resident.size() < (int64_t)S.cfg.max_resident;
      if (!cap_ok || S.used_bytes + need > S.cfg.hbm_budget_bytes) break;
      rc = admit(S, r);
      if (rc == GOL_ENOMEM) {
        // the device is short of memory despite the budget: wait for resident
        // boards to leave, or fail this request if none will
        rc = GOL_OK;
        if (S.resident.empty()) {
          r.state = State::Failed;
          r.err = "device allocation failed for a board within the budget";
          if (r.pin_in) S.exec->host_free(r.pin_in, r.pin_in_cls);
          r.pin_in = nullptr;
          S.queue.pop_front();
          S.cv_done.notify_all();
          continue;
        }
        break;
      }
      if (rc) break;
      S.used_bytes += need;
      S.stats.peak_resident_bytes =
          std::max<int64_t>(S.stats.peak_resident_bytes, (int64_t)S.used_bytes);
      S.resident.push_back(r.ticket);
      S.queue.pop_front();
      admitted = true;
      did = true;
    }
    S.stats.admit_host_s +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_admit0).count();
    // a marker after this tick's uploads
    if (admitted && rc == GOL_OK) {
      Token t = nullptr;
      rc = S.exec->upload_mark(&t);
      if (rc == GOL_OK) S.marks.emplace_back(++S.mark_seq, t);
    }
    // one chunk if fewer than two are in flight
    if (rc == GOL_OK && S.chunks.size() < 2) {
      std::vector<uint64_t> retire_now;
      rc = queue_chunk(S, retire_now);
      const auto t_ret0 = std::chrono::steady_clock::now();
      for (uint64_t t : retire_now) {
        if (rc) break;
        rc = queue_retire(S, *S.reqs[t]);
      }
      S.stats.retire_host_s +=
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_ret0).count();
      if (!retire_now.empty()) did = true;
    }
    // boards with zero generations retire without a chunk
    for (uint64_t t : S.resident) {
      Request& r = *S.reqs[t];
      if (rc == GOL_OK && !r.retiring && !r.cancel && r.gens == 0 && r.mark <= S.uploaded) {
        if (r.mark > S.copies_after) {
          rc = S.exec->copies_wait_for_upload(S.uploaded_mark);
          S.copies_after = S.uploaded;
        }
        if (rc == GOL_OK) rc = queue_retire(S, r);
        did = true;
      }
    }
    // retired boards leave the resident list
    S.resident.erase(std::remove_if(S.resident.begin(), S.resident.end(),
                                    [&](uint64_t t) { return S.reqs[t]->retiring; }),
                     S.resident.end());
    S.stats.resident_bytes = (int64_t)S.used_bytes;
    if (rc != GOL_OK) {
      fail_all(S, last_error());
      continue;
    }
    if (!did) {
      // nothing to queue: wait for work or for the device to progress
      bool copies = false;
      for (auto& kv : S.reqs)
        if (kv.second->retiring && kv.second->state == State::Resident) copies = true;
      S.sleeping = true;
      if (S.inbox_n.load() == 0) {
        if (!S.chunks.empty() || copies || !S.marks.empty())
          S.cv_work.wait_for(lk, std::chrono::microseconds(50));
        else
          S.cv_work.wait_for(lk, std::chrono::milliseconds(20));
      }
      S.sleeping = false;
    }
  }
}

// The pass length and band height of every chunk, timed at the first creation on
// a resident set standing in for a busy server: square boards of 512 to
// 8192 cells a side, four times as many of each size as of the next larger
// (so every size holds the same cells: 1 of 8192^2 ... 256 of 512^2, 3.4e8
// cells), advancing 48 generations (a multiple of every candidate), over
// t_block 8, 12, 16 (or the given one) and band heights 64, 96, 128; the
// fastest pair serves every chunk (a chunk with few tiles shortens the band,
// see chunk_band_rows).
// The choice is kept per device and given t_block for the process's later
// servers.
static int tune_served(int device, int T_fixed, int* T_out, int* band_out) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, std::pair<int, int>> chosen;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(device, T_fixed);
  const auto it = chosen.find(key);
  if (it != chosen.end()) {
    *T_out = it->second.first;
    *band_out = it->second.second;
    return GOL_OK;
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_error(e, "server: hipSetDevice");
  std::vector<BoardReq> set;
  for (int k = 0; k < 5; ++k)
    set.insert(set.end(), (size_t)1 << (2 * k), BoardReq{8192 >> k, 8192 >> k, 48});
  const std::vector<int> Ts = T_fixed ? std::vector<int>{T_fixed} : std::vector<int>{8, 12, 16};
  const int rc = tune_batch(set, Ts, {64, 96, 128}, T_out, band_out, nullptr);
  (void)hipSetDevice(prev);
  if (rc == GOL_OK) chosen[key] = std::make_pair(*T_out, *band_out);
  return rc;
}

static int check_config(const gol_serve_config* cfg) {
  if (cfg->chunk_generations < 0)
    return set_error(GOL_EINVAL, "chunk_generations must be >= 0 (0 = automatic)");
  if (cfg->hbm_budget_bytes == 0) return set_error(GOL_EINVAL, "hbm_budget_bytes must be > 0");
  if (cfg->t_block != 0 && !valid_T(cfg->t_block))
    return set_error(GOL_EINVAL, "t_block must be 0, 1, 2, 4, 8, 12 or 16");
  return GOL_OK;
}

}  // namespace gol

using namespace gol;

struct gol_server {
  Server S;
};

static int start_server(const gol_serve_config* cfg, std::unique_ptr<Exec> exec,
                        HostExec* host_exec, int tuned_T, int tuned_band, gol_server** out) {
  gol_server* s = nullptr;
  try {
    s = new gol_server();
  } catch (...) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
  Server& S = s->S;
  S.cfg = *cfg;
  S.T = tuned_T > 0 ? tuned_T : (cfg->t_block ? cfg->t_block : default_batch_T());
  S.band = tuned_band > 0 ? tuned_band : kBatchBandRows;
  S.stats.t_block = S.T;
  S.stats.busy_band_rows = S.band;
  S.t0 = std::chrono::steady_clock::now();
  S.exec = std::move(exec);
  S.host_exec = host_exec;
  S.th = std::thread(scheduler, &S);
  *out = s;
  return GOL_OK;
}

extern "C" {

int gol_serve_create(const gol_serve_config* cfg, gol_server** out) {
  if (!cfg || !out) return set_error(GOL_EINVAL, "null argument");
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (cfg->device < 0 || cfg->device >= ndev) return set_error(GOL_EINVAL, "bad device ordinal");
  try {
    auto ex = std::make_unique<HipExec>(cfg->device);
    rc = ex->init();
    if (rc) return rc;
    ex->set_block_cache_limit(cfg->hbm_budget_bytes);
    int T = cfg->t_block, band = 0;
    rc = tune_served(cfg->device, cfg->t_block, &T, &band);
    if (rc) return rc;
    return start_server(cfg, std::move(ex), nullptr, T, band, out);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
}

int gol_debug_serve_create_host(const gol_serve_config* cfg, int64_t fail_at_chunk,
                                gol_server** out) {
  if (!cfg || !out) return set_error(GOL_EINVAL, "null argument");
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  try {
    auto ex = std::make_unique<HostExec>(fail_at_chunk);
    HostExec* raw = ex.get();
    return start_server(cfg, std::move(ex), raw, 0, 0, out);
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
}

int64_t gol_debug_serve_host_peak_bytes(const gol_server* srv) {
  if (!srv || !srv->S.host_exec) return -1;
  return (int64_t)srv->S.host_exec->peak();
}

int gol_serve_submit(gol_server* srv, const uint64_t* host_packed, int64_t rows, int64_t cols,
                     int64_t generations, uint64_t* ticket) {
  if (!srv || !host_packed || !ticket) return set_error(GOL_EINVAL, "null argument");
  int rc = check_board(rows, cols, generations);
  if (rc) return rc;
  Server& S = srv->S;
  const int64_t W = (cols + 63) / 64;
  const size_t bytes = (size_t)(rows * W * 8);
  const uint64_t need = 2 * (uint64_t)S.exec->block_bytes(bytes);
  if (need > S.cfg.hbm_budget_bytes)
    return set_error(GOL_ENOMEM, "board needs %llu device bytes, budget is %llu",
                     (unsigned long long)need, (unsigned long long)S.cfg.hbm_budget_bytes);
  try {
    auto r = std::make_unique<Request>();
    r->rows = rows;
    r->cols = cols;
    r->W = W;
    r->gens = generations;
    r->bytes = bytes;
    r->pin_in = S.exec->stage_alloc(bytes, &r->pin_in_cls);
    if (!r->pin_in) return set_error(GOL_ENOMEM, "host staging for %zu bytes", bytes);
    memcpy(r->pin_in, host_packed, bytes);
    if (cols % 64) {
      // padding bits are not cells: the server keeps every board with them
      // cleared, so a request of zero generations returns the normalised input
      const uint64_t keep = ((uint64_t)1 << (cols % 64)) - 1;
      uint64_t* last = (uint64_t*)r->pin_in + (W - 1);
      for (int64_t i = 0; i < rows; ++i) last[i * W] &= keep;
    }
    if (S.failed_seen) {
      S.exec->host_free(r->pin_in, r->pin_in_cls);
      std::lock_guard<std::mutex> lk(S.mu);
      return set_error(GOL_EDEVICE, "server failed: %s", S.fail_msg.c_str());
    }
    std::lock_guard<std::mutex> g(S.in_mu);
    r->ticket = S.next_ticket++;
    r->t_submit = S.now();
    *ticket = r->ticket;
    S.inbox.push_back(std::move(r));
    S.inbox_n += 1;
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
  if (S.sleeping.load()) {
    std::lock_guard<std::mutex> lk(S.mu);
    S.cv_work.notify_one();
  }
  return GOL_OK;
}

static int take_result(Server& S, uint64_t ticket, uint64_t* host_out, gol_request_info* info,
                       std::unique_lock<std::mutex>& lk) {
  auto it = S.reqs.find(ticket);
  if (it == S.reqs.end())
    return set_error(GOL_ENOTFOUND, "unknown or retired ticket %llu", (unsigned long long)ticket);
  Request& r = *it->second;
  if (r.state == State::Cancelled) {
    S.reqs.erase(it);
    return set_error(GOL_ECANCELED, "ticket %llu was cancelled", (unsigned long long)ticket);
  }
  if (r.state == State::Failed) {
    std::string m = r.err;
    S.reqs.erase(it);
    return set_error(GOL_EDEVICE, "ticket %llu failed: %s", (unsigned long long)ticket, m.c_str());
  }
  if (r.state != State::Done)
    return set_error(GOL_EAGAIN, "ticket %llu not finished", (unsigned long long)ticket);
  if (info) {
    info->generations_done = r.gens;
    info->submit_s = r.t_submit;
    info->admit_s = r.t_admit;
    info->done_s = r.t_done;
  }
  std::unique_ptr<Request> own = std::move(it->second);
  S.reqs.erase(it);
  lk.unlock();
  if (host_out) memcpy(host_out, own->pin_out, own->bytes);
  S.exec->host_free(own->pin_out, own->pin_out_cls);
  return GOL_OK;
}

int gol_serve_poll(gol_server* srv, uint64_t ticket, uint64_t* host_out, gol_request_info* info) {
  if (!srv) return set_error(GOL_EINVAL, "null server");
  Server& S = srv->S;
  std::unique_lock<std::mutex> lk(S.mu);
  drain_inbox(S);
  finish_copies(S);
  return take_result(S, ticket, host_out, info, lk);
}

int gol_serve_wait(gol_server* srv, uint64_t ticket, uint64_t* host_out, gol_request_info* info) {
  if (!srv) return set_error(GOL_EINVAL, "null server");
  Server& S = srv->S;
  std::unique_lock<std::mutex> lk(S.mu);
  drain_inbox(S);
  while (true) {
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) break;
    State st = it->second->state;
    if (st == State::Done || st == State::Failed || st == State::Cancelled) break;
    S.cv_done.wait_for(lk, std::chrono::milliseconds(1));
    finish_copies(S);
  }
  return take_result(S, ticket, host_out, info, lk);
}

int gol_serve_cancel(gol_server* srv, uint64_t ticket) {
  if (!srv) return set_error(GOL_EINVAL, "null server");
  Server& S = srv->S;
  std::lock_guard<std::mutex> lk(S.mu);
  drain_inbox(S);
  auto it = S.reqs.find(ticket);
  if (it == S.reqs.end())
    return set_error(GOL_ENOTFOUND, "unknown or retired ticket %llu", (unsigned long long)ticket);
  Request& r = *it->second;
  if (r.state == State::Queued || (r.state == State::Resident && !r.retiring)) {
    r.cancel = true;
    S.cv_work.notify_one();
  }
  return GOL_OK;
}

double gol_serve_now(const gol_server* srv) { return srv ? srv->S.now() : 0.0; }

int gol_serve_get_stats(const gol_server* srv, gol_serve_stats* out) {
  if (!srv || !out) return set_error(GOL_EINVAL, "null argument");
  Server& S = const_cast<gol_server*>(srv)->S;
  std::lock_guard<std::mutex> lk(S.mu);
  *out = S.stats;
  return GOL_OK;
}

int gol_serve_destroy(gol_server* srv) {
  if (!srv) return GOL_OK;
  Server& S = srv->S;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv_work.notify_all();
  if (S.th.joinable()) S.th.join();
  {
    std::lock_guard<std::mutex> lk(S.mu);
    drain_inbox(S);
  }
  S.exec->sync();
  reap(S);
  for (Token t : S.chunks) S.exec->release(t);
  S.chunks.clear();
  for (auto& m : S.marks) S.exec->release(m.second);
  S.marks.clear();
  if (S.uploaded_mark) S.exec->release(S.uploaded_mark);
  S.uploaded_mark = nullptr;
  for (auto& kv : S.reqs) {
    Request& r = *kv.second;
    if (r.out_done) S.exec->release(r.out_done);
    S.exec->board_free_after_copies(r.d_buf[0]);
    S.exec->board_free_after_copies(r.d_buf[1]);
    if (r.pin_in) S.exec->host_free(r.pin_in, r.pin_in_cls);
    if (r.pin_out) S.exec->host_free(r.pin_out, r.pin_out_cls);
  }
  S.exec->sync();
  S.exec->reap();
  delete srv;
  return GOL_OK;
}

}  // extern "C"

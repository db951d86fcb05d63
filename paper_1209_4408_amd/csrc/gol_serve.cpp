// Serving loop with continuous batching (gol_serve_* in include/gol.h).
//
// One scheduler thread per server.  Each tick it
//   1. admits queued requests, oldest first, while their two device buffers
//      fit the HBM budget: device memory and the host-to-device copy are
//      queued on the copy stream, and the compute stream will wait for it;
//   2. queues one chunk on the compute stream: every resident board advances
//      min(chunk_generations, remaining) generations in one batched schedule
//      of tile passes (boards admitted since the last tick join here);
//   3. for boards that finish in that chunk, queues the device-to-host copy
//      (copy stream, after the chunk) and the release of their buffers.
// Board state stays in device memory between chunks.  Up to two chunks are
// in flight, so the host prepares the next while the device runs the last.
//
// The scheduler talks to the device through an executor.  HipExec is the
// real one (two HIP streams, events, stream-ordered memory, pinned staging).
// HostExec keeps boards in host memory and completes every operation at once;
// it exists so the scheduling policy (admission order, budget, chunking,
// buffer bookkeeping, retirement, cancellation, failures) can be tested on a
// machine without a GPU.  Its stand-in for a tile pass adds the number of
// generations advanced to every word of the board, which composes like the
// real step (two chunks of a and b generations equal one of a + b) and shows
// whether the scheduler read and wrote the right buffers.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
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
  virtual void* host_alloc(size_t bytes, size_t* cls) = 0;
  virtual void host_free(void* p, size_t cls) = 0;
  virtual int board_alloc(size_t bytes, void** p) = 0;  // in copy-queue order
  virtual void board_free_after_copies(void* p) = 0;
  virtual void board_free_after_chunks(void* p) = 0;
  virtual int upload(void* dev, const void* host, size_t bytes) = 0;
  virtual int chunks_wait_for_copies() = 0;
  virtual int run_chunk(const std::vector<BoardDesc>& bd, const HostPlan& hp, Token* done) = 0;
  virtual int copies_wait_for(Token chunk) = 0;
  virtual int download(void* host, const void* dev, size_t bytes, Token* done) = 0;
  // release `pinned` once everything queued so far on one queue has run
  virtual int host_free_after(bool compute, void* pinned, size_t cls) = 0;
  virtual bool done(Token t) = 0;
  virtual double seconds(Token chunk) = 0;  // device time of a completed chunk
  virtual void release(Token t) = 0;
  virtual void reap() = 0;
  virtual void sync() = 0;
};

// Pinned host blocks reused by size class (power of two), so steady-state
// serving does not call hipHostMalloc.
class PinnedPool {
 public:
  ~PinnedPool() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipHostFree(p);
  }
  void* get(size_t bytes, size_t* cls_out) {
    size_t cls = 4096;
    while (cls < bytes) cls <<= 1;
    *cls_out = cls;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto& v = free_[cls];
      if (!v.empty()) {
        void* p = v.back();
        v.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
  }
  void put(void* p, size_t cls) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_[cls].push_back(p);
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
};

class HipExec : public Exec {
 public:
  explicit HipExec(int device) : dev_(device) {}
  ~HipExec() override {
    sync();
    reap();
    if (compute_) (void)hipStreamDestroy(compute_);
    if (compute2_) (void)hipStreamDestroy(compute2_);
    if (copy_) (void)hipStreamDestroy(copy_);
  }
  int init() {
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(dev_);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&compute_, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&compute2_, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking);
    if (e == hipSuccess) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, dev_) == hipSuccess) {
        uint64_t thr = UINT64_MAX;  // keep freed blocks cached in the pool
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
      }
    }
    (void)hipSetDevice(prev);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server streams");
  }
  int bind_thread() override {
    hipError_t e = hipSetDevice(dev_);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: hipSetDevice");
  }
  void* host_alloc(size_t bytes, size_t* cls) override { return pool_.get(bytes, cls); }
  void host_free(void* p, size_t cls) override { pool_.put(p, cls); }
  int board_alloc(size_t bytes, void** p) override {
    hipError_t e = hipMallocAsync(p, bytes, copy_);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return set_error(GOL_ENOMEM, "server: device allocation of %zu bytes failed", bytes);
    }
    return GOL_OK;
  }
  void board_free_after_copies(void* p) override {
    if (p) (void)hipFreeAsync(p, copy_);
  }
  void board_free_after_chunks(void* p) override {
    if (p) (void)hipFreeAsync(p, compute_);
  }
  int upload(void* dev, const void* host, size_t bytes) override {
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, copy_);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: host-to-device copy");
  }
  int chunks_wait_for_copies() override {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, copy_);
    if (e == hipSuccess) e = hipStreamWaitEvent(compute_, ev, 0);
    if (e != hipSuccess) return hip_error(e, "server: admission event");
    pending_.push_back(Pending{ev, nullptr, 0});
    return GOL_OK;
  }
  int run_chunk(const std::vector<BoardDesc>& bd, const HostPlan& hp, Token* done) override {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t os = al(bd.size() * sizeof(BoardDesc));
    const size_t oi = os + al(hp.segs.size() * sizeof(Segment));
    const size_t mb = oi + al(hp.items.size() * sizeof(WaveItem));
    size_t cls = 0;
    char* pin = (char*)pool_.get(mb, &cls);
    if (!pin) return set_error(GOL_EDEVICE, "server: pinned staging");
    memcpy(pin, bd.data(), bd.size() * sizeof(BoardDesc));
    memcpy(pin + os, hp.segs.data(), hp.segs.size() * sizeof(Segment));
    memcpy(pin + oi, hp.items.data(), hp.items.size() * sizeof(WaveItem));
    void* meta = nullptr;
    hipError_t e = hipMallocAsync(&meta, mb, compute_);
    if (e != hipSuccess) {
      pool_.put(pin, cls);
      return set_error(GOL_EDEVICE, "server: chunk tables: %s", hipGetErrorString(e));
    }
    Chunk* c = new Chunk();
    e = hipEventCreate(&c->start);
    if (e == hipSuccess) e = hipEventCreate(&c->end);
    if (e == hipSuccess) e = hipEventRecord(c->start, compute_);
    if (e == hipSuccess) e = hipMemcpyAsync(meta, pin, mb, hipMemcpyHostToDevice, compute_);
    const BoardDesc* d_b = (const BoardDesc*)meta;
    const Segment* d_s = (const Segment*)((char*)meta + os);
    const WaveItem* d_i = (const WaveItem*)((char*)meta + oi);
    hipEvent_t fork = nullptr, join = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e == hipSuccess) e = enqueue_levels(hp, d_b, d_s, d_i, compute_, compute2_, fork, join);
    if (fork) (void)hipEventDestroy(fork);  // the waits on them are queued
    if (join) (void)hipEventDestroy(join);
    (void)hipFreeAsync(meta, compute_);
    if (e == hipSuccess) e = hipEventRecord(c->end, compute_);
    if (e != hipSuccess) {
      release(c);
      return hip_error(e, "server: chunk launch");
    }
    const int rc = host_free_after(true, pin, cls);
    if (rc) {
      release(c);
      return rc;
    }
    *done = c;
    return GOL_OK;
  }
  int copies_wait_for(Token chunk) override {
    hipError_t e = hipStreamWaitEvent(copy_, ((Chunk*)chunk)->end, 0);
    return e == hipSuccess ? GOL_OK : hip_error(e, "server: stream wait");
  }
  int download(void* host, const void* dev, size_t bytes, Token* done) override {
    Chunk* c = new Chunk();
    hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, copy_);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->end, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(c->end, copy_);
    if (e != hipSuccess) {
      release(c);
      return hip_error(e, "server: result copy");
    }
    *done = c;
    return GOL_OK;
  }
  int host_free_after(bool compute, void* pinned, size_t cls) override {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, compute ? compute_ : copy_);
    if (e != hipSuccess) return hip_error(e, "server: event record");
    pending_.push_back(Pending{ev, pinned, cls});
    return GOL_OK;
  }
  bool done(Token t) override { return hipEventQuery(((Chunk*)t)->end) == hipSuccess; }
  double seconds(Token t) override {
    Chunk* c = (Chunk*)t;
    float ms = 0.f;
    if (!c->start || hipEventElapsedTime(&ms, c->start, c->end) != hipSuccess) return 0.0;
    return ms * 1e-3;
  }
  void release(Token t) override {
    Chunk* c = (Chunk*)t;
    if (!c) return;
    if (c->start) (void)hipEventDestroy(c->start);
    if (c->end) (void)hipEventDestroy(c->end);
    delete c;
  }
  void reap() override {
    size_t k = 0;
    for (auto& p : pending_) {
      if (hipEventQuery(p.ev) == hipSuccess) {
        (void)hipEventDestroy(p.ev);
        pool_.put(p.pinned, p.cls);
      } else {
        pending_[k++] = p;
      }
    }
    pending_.resize(k);
  }
  void sync() override {
    if (compute_) (void)hipStreamSynchronize(compute_);
    if (copy_) (void)hipStreamSynchronize(copy_);
  }

 private:
  struct Chunk {
    hipEvent_t start = nullptr, end = nullptr;
  };
  struct Pending {
    hipEvent_t ev;
    void* pinned;
    size_t cls;
  };
  int dev_;
  hipStream_t compute_ = nullptr, copy_ = nullptr;
  hipStream_t compute2_ = nullptr;  // the late group of each chunk's schedule
  PinnedPool pool_;
  std::vector<Pending> pending_;  // touched by the scheduler thread under the server lock
};

// Boards in host memory, every operation complete on return (see the file
// comment).  fail_at: the 1-based index of the chunk that reports a device
// error (0 = never).
class HostExec : public Exec {
 public:
  explicit HostExec(int64_t fail_at) : fail_at_(fail_at) {}
  int bind_thread() override { return GOL_OK; }
  void* host_alloc(size_t bytes, size_t* cls) override {
    *cls = bytes;
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
  int chunks_wait_for_copies() override { return GOL_OK; }
  int run_chunk(const std::vector<BoardDesc>& bd, const HostPlan& hp, Token* done) override {
    if (++chunks_ == fail_at_) return set_error(GOL_EDEVICE, "host executor: injected failure");
    for (const BoardDesc& d : bd) {
      const uint64_t g = (uint64_t)(d.K - 1) * (uint64_t)hp.T + (uint64_t)d.Tshort;
      const uint64_t* src = (const uint64_t*)d.src0;
      uint64_t* dst = (uint64_t*)d.w[(d.K - 1 + d.par) & 1];
      const size_t words = (size_t)d.R * (size_t)(d.D / 2);
      for (size_t i = 0; i < words; ++i) dst[i] = src[i] + g;
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
  void* pin_in = nullptr;
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
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queue;                      // admission order
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<uint64_t> resident;                  // admitted, not yet retired
  uint64_t used_bytes = 0;

  std::deque<Token> chunks;                        // queued chunks, oldest first
  gol_serve_stats stats{};
  std::thread th;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

static void fail_all(Server& S, const std::string& msg) {
  // caller holds S.mu
  S.failed = true;
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

static void reap(Server& S) {
  S.exec->reap();
  while (!S.chunks.empty() && S.exec->done(S.chunks.front())) {
    S.stats.device_busy_s += S.exec->seconds(S.chunks.front());
    S.exec->release(S.chunks.front());
    S.chunks.pop_front();
  }
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
  if (!rc) rc = S.exec->host_free_after(false, r.pin_in, r.pin_in_cls);
  if (rc) return rc == GOL_ENOMEM ? GOL_EDEVICE : rc;
  r.pin_in = nullptr;
  r.state = State::Resident;
  r.t_admit = S.now();
  S.stats.admitted += 1;
  return GOL_OK;
}

// Build and queue one chunk over the resident boards.  Caller holds S.mu.
static int queue_chunk(Server& S, std::vector<uint64_t>& retire_now) {
  std::vector<Request*> act;
  for (uint64_t t : S.resident) {
    Request& r = *S.reqs[t];
    if (!r.cancel && !r.retiring && r.queued_gens < r.gens) act.push_back(&r);
  }
  if (act.empty()) return GOL_OK;
  const auto t_plan0 = std::chrono::steady_clock::now();
  const int T = S.cfg.t_block ? S.cfg.t_block : default_batch_T();
  std::vector<BoardReq> req;
  req.reserve(act.size());
  for (Request* r : act) {
    const int64_t g = std::min<int64_t>(S.cfg.chunk_generations, r->gens - r->queued_gens);
    req.push_back(BoardReq{r->rows, r->cols, g});
  }
  HostPlan hp;
  std::string err;
  if (!build_plan(req, T, 64, hp, err)) return set_error(GOL_EINVAL, "server plan: %s", err.c_str());
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
  S.stats.plan_host_s +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_plan0).count();
  Token done = nullptr;
  int rc = S.exec->run_chunk(bd, hp, &done);
  if (rc) return rc;
  S.chunks.push_back(done);
  S.stats.chunks += 1;
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
  S.used_bytes -= 2 * r.bytes;
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
  S.used_bytes -= 2 * r.bytes;
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
    // admission, oldest first, under the budget and the resident cap
    bool admitted = false;
    while (!S.queue.empty()) {
      Request& r = *S.reqs[S.queue.front()];
      if (r.cancel) {
        r.state = State::Cancelled;
        if (r.pin_in) S.exec->host_free(r.pin_in, r.pin_in_cls);
        r.pin_in = nullptr;
        S.queue.pop_front();
        S.cv_done.notify_all();
        continue;
      }
      const uint64_t need = 2 * (uint64_t)r.bytes;
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
    // the next chunk reads what the copy queue wrote
    if (admitted && rc == GOL_OK) rc = S.exec->chunks_wait_for_copies();
    // one chunk if fewer than two are in flight
    if (rc == GOL_OK && S.chunks.size() < 2) {
      std::vector<uint64_t> retire_now;
      rc = queue_chunk(S, retire_now);
      for (uint64_t t : retire_now) {
        if (rc) break;
        rc = queue_retire(S, *S.reqs[t]);
      }
      if (!retire_now.empty()) did = true;
    }
    // boards with zero generations retire without a chunk
    for (uint64_t t : S.resident) {
      Request& r = *S.reqs[t];
      if (rc == GOL_OK && !r.retiring && !r.cancel && r.gens == 0) {
        rc = queue_retire(S, r);
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
      if (!S.chunks.empty() || copies)
        S.cv_work.wait_for(lk, std::chrono::microseconds(50));
      else
        S.cv_work.wait_for(lk, std::chrono::milliseconds(20));
    }
  }
}

static int check_config(const gol_serve_config* cfg) {
  if (cfg->chunk_generations < 1) return set_error(GOL_EINVAL, "chunk_generations must be >= 1");
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
                        HostExec* host_exec, gol_server** out) {
  gol_server* s = nullptr;
  try {
    s = new gol_server();
  } catch (...) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
  Server& S = s->S;
  S.cfg = *cfg;
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
    return start_server(cfg, std::move(ex), nullptr, out);
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
    return start_server(cfg, std::move(ex), raw, out);
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
  if (2 * (uint64_t)bytes > S.cfg.hbm_budget_bytes)
    return set_error(GOL_ENOMEM, "board needs %zu device bytes, budget is %llu", 2 * bytes,
                     (unsigned long long)S.cfg.hbm_budget_bytes);
  try {
    auto r = std::make_unique<Request>();
    r->rows = rows;
    r->cols = cols;
    r->W = W;
    r->gens = generations;
    r->bytes = bytes;
    r->pin_in = S.exec->host_alloc(bytes, &r->pin_in_cls);
    if (!r->pin_in) return set_error(GOL_ENOMEM, "pinned staging for %zu bytes", bytes);
    memcpy(r->pin_in, host_packed, bytes);
    if (cols % 64) {
      // padding bits are not cells: the server keeps every board with them
      // cleared, so a request of zero generations returns the normalised input
      const uint64_t keep = ((uint64_t)1 << (cols % 64)) - 1;
      uint64_t* last = (uint64_t*)r->pin_in + (W - 1);
      for (int64_t i = 0; i < rows; ++i) last[i * W] &= keep;
    }
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.failed) {
      S.exec->host_free(r->pin_in, r->pin_in_cls);
      return set_error(GOL_EDEVICE, "server failed: %s", S.fail_msg.c_str());
    }
    r->ticket = S.next_ticket++;
    r->t_submit = S.now();
    *ticket = r->ticket;
    S.queue.push_back(r->ticket);
    S.reqs.emplace(r->ticket, std::move(r));
  } catch (const std::bad_alloc&) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
  S.cv_work.notify_one();
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
  finish_copies(S);
  return take_result(S, ticket, host_out, info, lk);
}

int gol_serve_wait(gol_server* srv, uint64_t ticket, uint64_t* host_out, gol_request_info* info) {
  if (!srv) return set_error(GOL_EINVAL, "null server");
  Server& S = srv->S;
  std::unique_lock<std::mutex> lk(S.mu);
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
  S.exec->sync();
  reap(S);
  for (Token t : S.chunks) S.exec->release(t);
  S.chunks.clear();
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

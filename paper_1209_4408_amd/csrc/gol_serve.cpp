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
#include <hip/hip_runtime.h>
#include <stdint.h>
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
#include "gol_internal.h"
#include "gol_plan.h"
#include "gol_runtime.h"

namespace gol {

hipError_t launch_batch_pass(int T, bool masked, const BoardDesc* boards, const Segment* segs,
                             const WaveItem* items, int nitems, int level, hipStream_t st);

namespace {

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
  hipEvent_t ev_out = nullptr; // device-to-host copy of the result done
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::string err;
};

struct PendingFree {
  hipEvent_t ev;
  void* pinned;
  size_t cls;
};

}  // namespace

struct Server {
  gol_serve_config cfg{};
  std::chrono::steady_clock::time_point t0;
  hipStream_t compute = nullptr, copy = nullptr;
  PinnedPool pool;

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

  // owned by the scheduler thread
  std::vector<PendingFree> pend_free;
  std::deque<hipEvent_t> chunk_events;
  std::deque<hipEvent_t> chunk_starts;  // timing events, paired with chunk_events
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

// Queue the release of a pinned block once everything queued on `st` so far has run.
static bool defer_pinned(Server& S, hipStream_t st, void* p, size_t cls) {
  if (!p) return true;
  hipEvent_t ev;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return false;
  if (hipEventRecord(ev, st) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return false;
  }
  S.pend_free.push_back(PendingFree{ev, p, cls});
  return true;
}

static void reap(Server& S) {
  size_t k = 0;
  for (auto& f : S.pend_free) {
    if (hipEventQuery(f.ev) == hipSuccess) {
      (void)hipEventDestroy(f.ev);
      S.pool.put(f.pinned, f.cls);
    } else {
      S.pend_free[k++] = f;
    }
  }
  S.pend_free.resize(k);
  while (!S.chunk_events.empty() && hipEventQuery(S.chunk_events.front()) == hipSuccess) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, S.chunk_starts.front(), S.chunk_events.front()) == hipSuccess)
      S.stats.device_busy_s += ms * 1e-3;
    (void)hipEventDestroy(S.chunk_starts.front());
    (void)hipEventDestroy(S.chunk_events.front());
    S.chunk_starts.pop_front();
    S.chunk_events.pop_front();
  }
}

// Completed result copies -> Done.  Caller holds S.mu.
static void finish_copies(Server& S) {
  bool any = false;
  for (auto& kv : S.reqs) {
    Request& r = *kv.second;
    if (r.state == State::Resident && r.retiring && r.ev_out &&
        hipEventQuery(r.ev_out) == hipSuccess) {
      (void)hipEventDestroy(r.ev_out);
      r.ev_out = nullptr;
      r.state = State::Done;
      r.t_done = S.now();
      any = true;
    }
  }
  if (any) S.cv_done.notify_all();
}

static int admit(Server& S, Request& r) {
  // caller holds S.mu; device work goes to the copy stream
  void* p0 = nullptr;
  void* p1 = nullptr;
  hipError_t e = hipMallocAsync(&p0, r.bytes, S.copy);
  if (e == hipSuccess) e = hipMallocAsync(&p1, r.bytes, S.copy);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (p0) (void)hipFreeAsync(p0, S.copy);
    return GOL_ENOMEM;
  }
  r.d_buf[0] = (uint64_t*)p0;
  r.d_buf[1] = (uint64_t*)p1;
  r.cur = 0;
  e = hipMemcpyAsync(p0, r.pin_in, r.bytes, hipMemcpyHostToDevice, S.copy);
  if (e != hipSuccess) return hip_error(e, "server: host-to-device copy");
  if (!defer_pinned(S, S.copy, r.pin_in, r.pin_in_cls))
    return set_error(GOL_EDEVICE, "server: event record failed");
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
  const int T = S.cfg.t_block ? S.cfg.t_block : default_T();
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
    d.Tfirst = hp.Tfirst[b];
    d.src0 = (const uint32_t*)r.d_buf[r.cur];
    d.w[0] = (uint32_t*)r.d_buf[r.cur ^ 1];
    d.w[1] = (uint32_t*)r.d_buf[r.cur];
    d.par = 0;  // pass j writes w[j & 1]; the result lands in w[(K - 1) & 1]
  }
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t os = al(bd.size() * sizeof(BoardDesc));
  const size_t oi = os + al(hp.segs.size() * sizeof(Segment));
  const size_t mb = oi + al(hp.items.size() * sizeof(WaveItem));
  size_t cls = 0;
  char* pin = (char*)S.pool.get(mb, &cls);
  if (!pin) return set_error(GOL_ENOMEM, "server: pinned staging");
  memcpy(pin, bd.data(), bd.size() * sizeof(BoardDesc));
  memcpy(pin + os, hp.segs.data(), hp.segs.size() * sizeof(Segment));
  memcpy(pin + oi, hp.items.data(), hp.items.size() * sizeof(WaveItem));
  S.stats.plan_host_s +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_plan0).count();
  void* meta = nullptr;
  hipError_t e = hipMallocAsync(&meta, mb, S.compute);
  if (e != hipSuccess) {
    S.pool.put(pin, cls);
    return set_error(GOL_ENOMEM, "server: chunk tables: %s", hipGetErrorString(e));
  }
  hipEvent_t ev0;
  e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventRecord(ev0, S.compute);
  if (e != hipSuccess) return hip_error(e, "server: chunk start event");
  S.chunk_starts.push_back(ev0);
  e = hipMemcpyAsync(meta, pin, mb, hipMemcpyHostToDevice, S.compute);
  const BoardDesc* d_b = (const BoardDesc*)meta;
  const Segment* d_s = (const Segment*)((char*)meta + os);
  const WaveItem* d_i = (const WaveItem*)((char*)meta + oi);
  for (size_t L = 0; L < hp.level_items.size() && e == hipSuccess; ++L)
    e = launch_batch_pass(T, L == 0 && hp.level0_masked, d_b, d_s, d_i, hp.level_items[L], (int)L,
                          S.compute);
  (void)hipFreeAsync(meta, S.compute);
  if (!defer_pinned(S, S.compute, pin, cls) && e == hipSuccess) e = hipErrorUnknown;
  if (e != hipSuccess) return hip_error(e, "server: chunk launch");
  hipEvent_t ev;
  e = hipEventCreate(&ev);
  if (e == hipSuccess) e = hipEventRecord(ev, S.compute);
  if (e != hipSuccess) return hip_error(e, "server: chunk event");
  S.chunk_events.push_back(ev);
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
  e = hipStreamWaitEvent(S.copy, ev, 0);
  if (e != hipSuccess) return hip_error(e, "server: stream wait");
  return GOL_OK;
}

// Queue result copy + buffer release for a finished board.  Caller holds S.mu.
static int queue_retire(Server& S, Request& r) {
  r.pin_out = S.pool.get(r.bytes, &r.pin_out_cls);
  if (!r.pin_out) return set_error(GOL_ENOMEM, "server: pinned result buffer");
  hipError_t e = hipMemcpyAsync(r.pin_out, r.d_buf[r.cur], r.bytes, hipMemcpyDeviceToHost, S.copy);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r.ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(r.ev_out, S.copy);
  (void)hipFreeAsync(r.d_buf[0], S.copy);
  (void)hipFreeAsync(r.d_buf[1], S.copy);
  r.d_buf[0] = r.d_buf[1] = nullptr;
  S.used_bytes -= 2 * r.bytes;
  r.retiring = true;
  S.stats.retired += 1;
  if (e != hipSuccess) return hip_error(e, "server: result copy");
  return GOL_OK;
}

// Drop a cancelled resident board: its buffers are released after the
// chunks already queued (compute stream order).  Caller holds S.mu.
static void drop_cancelled(Server& S, Request& r) {
  if (r.d_buf[0]) (void)hipFreeAsync(r.d_buf[0], S.compute);
  if (r.d_buf[1]) (void)hipFreeAsync(r.d_buf[1], S.compute);
  r.d_buf[0] = r.d_buf[1] = nullptr;
  S.used_bytes -= 2 * r.bytes;
  r.state = State::Cancelled;
}

static void scheduler(Server* Sp) {
  Server& S = *Sp;
  if (hipSetDevice(S.cfg.device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(S.mu);
    fail_all(S, "server: hipSetDevice failed");
    return;
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
        if (r.pin_in) S.pool.put(r.pin_in, r.pin_in_cls);
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
          if (r.pin_in) S.pool.put(r.pin_in, r.pin_in_cls);
          r.pin_in = nullptr;
          S.queue.pop_front();
          S.cv_done.notify_all();
          continue;
        }
        break;
      }
      if (rc) break;
      S.used_bytes += need;
      S.resident.push_back(r.ticket);
      S.queue.pop_front();
      admitted = true;
      did = true;
    }
    if (admitted && rc == GOL_OK) {
      // the next chunk reads what the copy stream wrote
      hipEvent_t ev;
      hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(ev, S.copy);
      if (e == hipSuccess) e = hipStreamWaitEvent(S.compute, ev, 0);
      if (e == hipSuccess) S.pend_free.push_back(PendingFree{ev, nullptr, 0});
      if (e != hipSuccess) rc = hip_error(e, "server: admission event");
    }
    // one chunk if fewer than two are in flight
    if (rc == GOL_OK && S.chunk_events.size() < 2) {
      std::vector<uint64_t> retire_now;
      rc = queue_chunk(S, retire_now);
      for (uint64_t t : retire_now) {
        if (rc) break;
        rc = queue_retire(S, *S.reqs[t]);
        did = true;
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
    if (rc != GOL_OK) {
      fail_all(S, last_error());
      continue;
    }
    if (!did) {
      // nothing to queue: wait for work or for the device to progress
      const bool busy = !S.chunk_events.empty() || !S.pend_free.empty();
      bool copies = false;
      for (auto& kv : S.reqs)
        if (kv.second->retiring && kv.second->state == State::Resident) copies = true;
      if (busy || copies)
        S.cv_work.wait_for(lk, std::chrono::microseconds(50));
      else
        S.cv_work.wait_for(lk, std::chrono::milliseconds(20));
    }
  }
}

}  // namespace gol

using namespace gol;

struct gol_server {
  Server S;
};

extern "C" {

int gol_serve_create(const gol_serve_config* cfg, gol_server** out) {
  if (!cfg || !out) return set_error(GOL_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->chunk_generations < 1) return set_error(GOL_EINVAL, "chunk_generations must be >= 1");
  if (cfg->hbm_budget_bytes == 0) return set_error(GOL_EINVAL, "hbm_budget_bytes must be > 0");
  if (cfg->t_block != 0 && !valid_T(cfg->t_block))
    return set_error(GOL_EINVAL, "t_block must be 0, 1, 2, 4, 8 or 16");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (cfg->device < 0 || cfg->device >= ndev) return set_error(GOL_EINVAL, "bad device ordinal");
  gol_server* s = nullptr;
  try {
    s = new gol_server();
  } catch (...) {
    return set_error(GOL_ENOMEM, "host allocation failed");
  }
  Server& S = s->S;
  S.cfg = *cfg;
  S.t0 = std::chrono::steady_clock::now();
  int prev = 0;
  (void)hipGetDevice(&prev);
  e = hipSetDevice(cfg->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.compute, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.copy, hipStreamNonBlocking);
  if (e == hipSuccess) {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, cfg->device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    if (S.compute) (void)hipStreamDestroy(S.compute);
    if (S.copy) (void)hipStreamDestroy(S.copy);
    delete s;
    return hip_error(e, "server streams");
  }
  S.th = std::thread(scheduler, &S);
  *out = s;
  return GOL_OK;
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
    r->pin_in = S.pool.get(bytes, &r->pin_in_cls);
    if (!r->pin_in) return set_error(GOL_ENOMEM, "pinned staging for %zu bytes", bytes);
    memcpy(r->pin_in, host_packed, bytes);
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.failed) {
      S.pool.put(r->pin_in, r->pin_in_cls);
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
  if (it == S.reqs.end()) return set_error(GOL_ENOTFOUND, "unknown or retired ticket %llu",
                                           (unsigned long long)ticket);
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
  if (r.state != State::Done) return set_error(GOL_EAGAIN, "ticket %llu not finished",
                                               (unsigned long long)ticket);
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
  S.pool.put(own->pin_out, own->pin_out_cls);
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
  if (it == S.reqs.end()) return set_error(GOL_ENOTFOUND, "unknown or retired ticket %llu",
                                           (unsigned long long)ticket);
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
  (void)hipStreamSynchronize(S.compute);
  (void)hipStreamSynchronize(S.copy);
  reap(S);
  for (auto& f : S.pend_free) {
    (void)hipEventSynchronize(f.ev);
    (void)hipEventDestroy(f.ev);
    S.pool.put(f.pinned, f.cls);
  }
  for (auto& kv : S.reqs) {
    Request& r = *kv.second;
    if (r.ev_out) (void)hipEventDestroy(r.ev_out);
    if (r.d_buf[0]) (void)hipFreeAsync(r.d_buf[0], S.copy);
    if (r.d_buf[1]) (void)hipFreeAsync(r.d_buf[1], S.copy);
    if (r.pin_in) S.pool.put(r.pin_in, r.pin_in_cls);
    if (r.pin_out) S.pool.put(r.pin_out, r.pin_out_cls);
  }
  (void)hipStreamSynchronize(S.copy);
  for (hipEvent_t ev : S.chunk_events) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : S.chunk_starts) (void)hipEventDestroy(ev);
  (void)hipStreamDestroy(S.compute);
  (void)hipStreamDestroy(S.copy);
  delete srv;
  return GOL_OK;
}

}  // extern "C"

// Runtime helpers shared by the C ABI translation units: error reporting,
// stream-ordered device scratch, deferred release of pinned staging, and
// the single-board / batch drivers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gol.h"
#include "gol_internal.h"
#include "gol_plan.h"

namespace gol {

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);
void clear_error();
const char* last_error();

int scratch_alloc(void** p, size_t bytes, hipStream_t st);
void scratch_free(void* p, hipStream_t st);
// Pinned host staging from a pool of power-of-two size classes (*cls
// receives the class); pinned_put_after returns the block to the pool once
// the work queued on st so far has run.
void* pinned_get(size_t bytes, size_t* cls);
void pinned_put(void* pinned, size_t cls);  // at once: the caller knows it is idle
int pinned_put_after(void* pinned, size_t cls, hipStream_t st);
void reap_deferred(bool wait);

int check_board(int64_t rows, int64_t cols, int64_t gens);
bool ranges_partially_overlap(const void* a, const void* b, size_t bytes);
int default_T();        // generations per pass of a single board without tuning
int default_batch_T();  // of batched and served schedules
int simd_count();

// Launch configuration of the single-board pass (gol_pass_config); 0 in a
// field = automatic.
struct PassConfig {
  int T = 0;
  int band_rows = 0;
  int pd = 0;
  int layout = 0;
  bool bounded = false;  // cells beyond the edges are dead (no torus); band layout only
};
// The autotuner's choice for a board size on the current device, if any.
bool tuned_choice(int64_t rows, int64_t cols, PassConfig* out);
// Fill the automatic fields (tuned choice, then defaults) and check the
// result; GOL_EINVAL with a message if it cannot run this board.
int resolve_config(int64_t R, int64_t C, const PassConfig& want, PassConfig* out);
// One pass of T = c.T generations with a resolved configuration.
hipError_t launch_pass(const PassConfig& c, const uint32_t* src, uint32_t* dst, int64_t R,
                       int64_t C, hipStream_t st);

// checks (host, non-decreasing, in 0..G) / d_counts (device int64[ncheck]):
// the population after each checked generation count.  ext_scratch (device,
// ext_scratch_bytes): the ping-pong board to use instead of one from the
// allocator (boards larger than it -> GOL_EINVAL); with it the call makes no
// device or pinned allocation.
int step_packed(const uint64_t* d_in, int64_t R, int64_t C, int64_t G, uint64_t* d_out,
                hipStream_t st, const PassConfig& cfg, const int64_t* checks = nullptr,
                int64_t ncheck = 0, int64_t* d_counts = nullptr, void* ext_scratch = nullptr,
                size_t ext_scratch_bytes = 0);

// A batch schedule bound to device buffers.
struct DevicePlan {
  HostPlan hp;
  std::vector<gol_board> boards;
  std::vector<BoardDesc> h_boards;
  std::vector<int> copy_first;  // in-place boards with an odd pass count: copy in -> scratch
  std::vector<int> zero_gen;    // generations == 0: normalising copy
  BoardDesc* d_boards = nullptr;
  Segment* d_segs = nullptr;
  WaveItem* d_items = nullptr;
  uint64_t* d_scratch = nullptr;
  size_t scratch_words = 0;
  std::vector<size_t> scratch_off;
};

int plan_boards(const gol_board* boards, int64_t n, int T, int band_rows, DevicePlan& P);
void fill_board_descs(DevicePlan& P);

// Queues the level launches of a batch schedule whose tables are on the
// device: the early group's levels on `st`, the late group's on `side`,
// which first waits (through `fork`) for the work queued on `st` so far;
// then `st` waits (through `join`) for `side`.  The groups hold different
// boards, so the two streams' launches overlap and each fills the tail of
// the other's levels.  With no late group everything goes on `st` and the
// events are not used.  `side` must have the default priority.
hipError_t enqueue_levels(const HostPlan& hp, const BoardDesc* boards, const Segment* segs,
                          const WaveItem* items, hipStream_t st, hipStream_t side,
                          hipEvent_t fork, hipEvent_t join);
// Times the batch schedule of these boards (sizes and generation counts) on
// zeroed scratch boards for every T in Ts and band height in bands; the
// fastest pair goes to *T_out / *band_out (its seconds to *secs_out).
int tune_batch(const std::vector<BoardReq>& boards, const std::vector<int>& Ts,
               const std::vector<int>& bands, int* T_out, int* band_out, double* secs_out);
// Band height of batched schedules when none is given or tuned.
constexpr int kBatchBandRows = 96;

// The normalising copies of a plan, then enqueue_levels.
hipError_t enqueue_plan(const DevicePlan& P, hipStream_t st, hipStream_t side, hipEvent_t fork,
                        hipEvent_t join);

}  // namespace gol

/*
 * gol.h -- C ABI of the MI355X Game-of-Life step library (libgol.so).
 *
 * The operation: Conway's Life, rule B3/S23 (the paper, Section 1: every cell
 * has eight neighbours -- horizontal, vertical and diagonal; all cells change
 * at once each time step; a live cell with two or three live neighbours
 * lives on, any other live cell dies; a dead cell with exactly three live
 * neighbours becomes live) on a torus whose left/right and top/bottom edges
 * are adjacent (Section 2.2).  A run is fixed by its initial board and its
 * number of generations (Section 1: the evolution depends on the initial
 * state only).  Neighbour coordinates wrap modulo the board's sides; on tori
 * with fewer than 3 rows or columns an offset that lands on a cell already
 * counted, or on the cell itself, counts again.
 *
 * Layouts
 *   byte board   : rows * cols uint8, row-major; nonzero = alive on input,
 *                  results are 0 / 1.
 *   packed board : rows * W uint64 words, W = ceil(cols / 64); cell (r, c) is
 *                  bit (c mod 64) of word r * W + c / 64, LSB first.  Padding
 *                  bits (columns >= cols) are ignored on input and written 0.
 *
 * Sizes: 1 <= rows, cols <= 2^30, rows * W * 8 bytes must fit the device;
 * generations >= 0 (0 copies the normalised input).
 *
 * Errors: every call returns GOL_OK (0) or a negative code; gol_last_error()
 * returns a description of the calling thread's last failure.  No C++
 * exception crosses this interface.
 *
 * Streams: `stream` arguments are hipStream_t handles passed as void*
 * (NULL = the legacy default stream).  Asynchronous calls return once their
 * work is queued; their buffers must stay valid until it has run.
 */
#ifndef GOL_H
#define GOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GOL_OK = 0,
  GOL_EINVAL = -1,     /* null pointer, size out of range, generations < 0, bad overlap */
  GOL_ENOMEM = -2,     /* device or host allocation failed, or request > server budget */
  GOL_EDEVICE = -3,    /* a HIP call failed; the message names it */
  GOL_EAGAIN = -4,     /* served request not finished yet */
  GOL_ENOTFOUND = -5,  /* unknown or already retired ticket */
  GOL_ECANCELED = -6   /* served request was cancelled */
};

/* Description of the calling thread's last error ("" if none). */
const char* gol_last_error(void);

/* Library version string. */
const char* gol_version(void);

/*
 * Advance a board held in HOST memory by `generations` generations.
 * board, out: host byte boards of rows * cols bytes (out == board allowed;
 * partial overlap -> GOL_EINVAL).  Synchronous: copies the board to the
 * current HIP device, packs it, runs the tile passes, unpacks and copies
 * back before returning.
 */
int gol_step(const uint8_t* board, int64_t rows, int64_t cols, int64_t generations,
             uint8_t* out);

/*
 * Advance a packed board held in DEVICE memory.  d_in, d_out: device
 * pointers to rows * W words (d_out == d_in allowed; partial overlap ->
 * GOL_EINVAL).  Asynchronous on `stream`.  The library takes its ping-pong
 * scratch (one board, two when d_out == d_in and the pass count is odd) from
 * the device's stream-ordered memory pool, or from the allocator installed
 * with gol_set_allocator.  `t_block` = generations per pass (the temporal
 * block): 0 picks the tuned configuration for this size (see gol_tune), else
 * one of 1, 2, 4, 8, 12, 16 with the default band height and layout.
 * G mod t_block generations run first as shorter passes.
 */
int gol_step_packed(const uint64_t* d_in, int64_t rows, int64_t cols, int64_t generations,
                    uint64_t* d_out, void* stream);
int gol_step_packed_ex(const uint64_t* d_in, int64_t rows, int64_t cols, int64_t generations,
                       uint64_t* d_out, void* stream, int t_block);

/*
 * gol_step_packed for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result and automatic configuration as gol_step_packed, but
 * the ping-pong board comes from a fixed array in the library's device code
 * (64 MiB on each GPU the library runs on, held until the process ends)
 * instead of the memory pool or the installed allocator: the call makes no
 * device or host-pinned allocation and frees nothing.
 *   Size limit: rows * ceil(cols / 64) * 8 <= 64 MiB (e.g. 16384 x 32768);
 *   larger boards -> GOL_EINVAL with a message, before any device work.
 *   Sharing: every call on one GPU uses that GPU's one array, whose contents
 *   are left from the last call (nothing in it needs clearing: every pass
 *   writes each word it later reads).  Calls that overlap on one GPU (two
 *   streams, two threads) race on it; the caller serialises them.
 */
int gol_step_packed_noalloc(const uint64_t* d_in, int64_t rows, int64_t cols,
                            int64_t generations, uint64_t* d_out, void* stream);

/*
 * Launch configuration of the single-board tile pass (Section 2's grid,
 * split into tiles that each advance t_block generations per sweep of the
 * board).  A field of 0 means automatic: when t_block and layout are both 0
 * the autotuner's choice for this board size is used if gol_tune ran, and
 * every field still 0 takes the built-in default.
 *   t_block   generations per pass: 1, 2, 4, 8, 12 or 16.
 *   band_rows rows per band (>= 1).
 *   prefetch  rows requested ahead of use: GOL_LAYOUT_BAND 3 or 6 for
 *             t_block <= 4, 6 or 9 for 8 and 12, 9 or 12 for 16;
 *             GOL_LAYOUT_PAIRED 9 or 12.
 *   layout    GOL_LAYOUT_BAND: one band of one strip per wave;
 *             GOL_LAYOUT_PAIRED: two adjacent bands per wave that sweep
 *             towards each other and trade the rows of their shared edge,
 *             so only the outer edges of the pair recompute halo rows;
 *             needs t_block 8, 12 or 16, cols % 32 == 0, a packed board
 *             below 2 GiB and bands of at least t_block rows;
 *             GOL_LAYOUT_RESIDENT: the whole board in one workgroup's LDS
 *             for all its generations (one launch per run, or per
 *             population check), for boards whose two generations fit
 *             in 64 KiB of LDS: cols <= 32768 and rows x ceil(cols / 32)
 *             dwords plus one pad dword per row segment (at most 1024) at
 *             most 8192 -- every board of up to 7168 dwords fits; t_block,
 *             band_rows and prefetch are ignored.  With
 *             every field 0 it is taken for boards of at most 1024 such
 *             dwords (e.g. 128 x 256) unless the autotuner chose otherwise.
 * Combinations outside these sets -> GOL_EINVAL with a message.
 */
#define GOL_LAYOUT_BAND 1
#define GOL_LAYOUT_PAIRED 2
#define GOL_LAYOUT_RESIDENT 3
/* Batch plans only (gol_plan_create_cfg): the persistent work-queue form. */
#define GOL_LAYOUT_QUEUE 4
typedef struct gol_pass_config {
  int32_t t_block;
  int32_t band_rows;
  int32_t prefetch;
  int32_t layout;
} gol_pass_config;

/* gol_step_packed with an explicit launch configuration (NULL = automatic). */
int gol_step_packed_cfg(const uint64_t* d_in, int64_t rows, int64_t cols, int64_t generations,
                        uint64_t* d_out, void* stream, const gol_pass_config* config);

/*
 * Bounded board: gol_step_packed_cfg for a board whose surroundings are dead
 * -- every cell beyond its edges is dead at every generation (such cells are
 * not evolved), instead of the torus of Section 2.2.  Section 1 describes an
 * infinite grid; a bounded board agrees with it as long as no cell beyond the
 * edges would become alive.  Runs in the band layout (config->layout 0 or
 * GOL_LAYOUT_BAND, any other -> GOL_EINVAL); t_block 0 takes the default
 * (the autotuner's choices are for tori).  Same buffers, overlap rules and
 * errors as gol_step_packed_cfg.
 */
int gol_step_packed_bounded(const uint64_t* d_in, int64_t rows, int64_t cols,
                            int64_t generations, uint64_t* d_out, void* stream,
                            const gol_pass_config* config);

/*
 * Strip pass: t generations of one row strip of a larger torus, whose
 * neighbouring rows are held elsewhere -- the unit of the row (1-D)
 * decomposition of Section 2.1 (Figure 1), where each worker updates a bar of
 * whole rows; the rows just beyond its edges belong to its neighbours (the
 * boundary reads Section 2.2 describes for sub-regions).  Across devices the
 * strips would form a ring and trade t edge rows per pass.
 *   d_strip  : rows x W words (W = ceil(cols / 64)), the strip at generation g.
 *   d_top    : t x W words, the t rows just above the strip's first row,
 *              farthest first (its last row touches the strip).
 *   d_bottom : t x W words, the t rows just below the strip's last row,
 *              nearest first.
 *   d_out    : rows x W words, receives the strip at generation g + t.
 * Each row is a whole torus row: columns wrap within the row.  t must be 1, 2,
 * 4, 8, 12 or 16 (one pass; the halo rows are only known at generation g).
 * config (may be NULL): band_rows and prefetch as for gol_step_packed_cfg;
 * t_block must be 0 or t and layout 0 or GOL_LAYOUT_BAND.  Padding bits of the
 * inputs are ignored and written as 0.  d_out must not overlap any input
 * (GOL_EINVAL); null buffers, sizes outside [1, 2^30] -> GOL_EINVAL.
 * Asynchronous on stream; the inputs must stay valid until it completes.
 */
int gol_strip_pass(const uint64_t* d_strip, const uint64_t* d_top, const uint64_t* d_bottom,
                   int64_t rows, int64_t cols, int64_t t, uint64_t* d_out, void* stream,
                   const gol_pass_config* config);

/*
 * Population: the number of live cells, the quantity the paper tabulates at
 * chosen iteration counts (Table 1).  Padding bits are not counted.
 *
 * gol_population: d_packed (device, rows * W words) -> *d_count (device
 * int64).  Asynchronous on `stream`; reads the board once.
 *
 * gol_step_packed_population: gol_step_packed_cfg that also records the
 * population after each of `ncheck` generation counts.  checks: HOST array,
 * non-decreasing, each in 0 .. generations (repeats allowed).  d_counts:
 * DEVICE int64[ncheck]; d_counts[i] receives the population after checks[i]
 * generations.  A pass ends at every checked generation and the board it
 * leaves is counted (one read of the board per check).  Asynchronous on
 * `stream`: checks is read during the call, d_counts is written by the
 * queued work.  Errors:
 * GOL_EINVAL for a null array with ncheck > 0, ncheck < 0 or checks out of
 * order or range, in addition to gol_step_packed_cfg's.
 */
int gol_population(const uint64_t* d_packed, int64_t rows, int64_t cols, int64_t* d_count,
                   void* stream);
int gol_step_packed_population(const uint64_t* d_in, int64_t rows, int64_t cols,
                               int64_t generations, uint64_t* d_out, void* stream,
                               const gol_pass_config* config, const int64_t* checks,
                               int64_t ncheck, int64_t* d_counts);

/*
 * Autotuner of the single-board path: times candidate launch configurations
 * (both layouts, t_block 8, 12 and 16, several band heights) for rows x cols
 * boards on the current device, using two scratch boards of that size from
 * the stream-ordered pool (the pass's run time does not depend on the
 * cells), and remembers the fastest per generation.  Later automatic calls
 * on this device and size use it.  Synchronous on `stream` (tens to hundreds
 * of milliseconds).  `out` (may be NULL) receives the choice.  If the
 * environment variable GOL_AUTOTUNE_CACHE names a file, choices are appended
 * to it and read back by later processes.
 */
int gol_tune_cfg(int64_t rows, int64_t cols, void* stream, gol_pass_config* out);
/* gol_tune_cfg reporting only t_block and band_rows (either may be NULL). */
int gol_tune(int64_t rows, int64_t cols, void* stream, int* out_t_block, int* out_band_rows);

/* Device conversions between the byte and packed layouts (asynchronous). */
int gol_pack(const uint8_t* d_bytes, int64_t rows, int64_t cols, uint64_t* d_packed,
             void* stream);
int gol_unpack(const uint64_t* d_packed, int64_t rows, int64_t cols, uint8_t* d_bytes,
               void* stream);

/*
 * Many independent boards, each with its own size and generation count, in
 * one schedule of tile passes (uneven sizes share waves; a board runs its
 * passes in a block of consecutive levels, the boards being split between
 * levels at the start and at the end of the schedule so every level carries
 * a similar load).  d_in / d_out follow gol_step_packed's rules per board.
 * Asynchronous on `stream`: the two halves of the schedule run on `stream`
 * and on a library stream that waits for `stream`'s earlier work and that
 * `stream` waits for in turn, so the work is ordered on `stream` as one call.
 */
typedef struct {
  const uint64_t* d_in;
  uint64_t* d_out;
  int64_t rows;
  int64_t cols;
  int64_t generations;
} gol_board;

int gol_batch_run(const gol_board* boards, int64_t n, void* stream);

/*
 * A batch plan: the schedule of gol_batch_run built once and run many times
 * on the same buffers (the launch sequence is captured into a HIP graph on
 * the first run and replayed afterwards).  The plan owns its scratch.
 */
typedef struct gol_plan gol_plan;
/* t_block: generations per pass, 0 = tuned, else 1, 2, 4, 8, 12 or 16; the
 * band height is tuned (see gol_plan_create_cfg). */
int gol_plan_create(const gol_board* boards, int64_t n, int t_block, gol_plan** out);
/*
 * gol_plan_create with the band height too: config->t_block and
 * config->band_rows (rows per tile band, 1 .. 65535); prefetch and layout
 * must be 0.  A field of 0 is tuned: creation times the candidate schedules
 * (t_block 8, 12 or 16; band_rows 48, 64, 96 or 128) of these boards on
 * zeroed scratch boards of the same sizes, allocated and freed inside the call
 * (of every k-th board when they would take more than 1 GiB; the defaults,
 * 16 and 96, when the device has no room), and keeps the fastest.  Creation
 * is synchronous; the buffers of `boards` are not touched.
 * config->layout GOL_LAYOUT_QUEUE selects the persistent work-queue form
 * instead of the level-by-level schedule: one launch of as many waves as the
 * device holds at once, taking items (one wave of one board's tiles in one
 * pass) from a queue in pass order, each waiting until its board's previous
 * pass is complete (device-scope counters, release / acquire fences, waits
 * bounded: a wait that gives up stops the launch early, which
 * gol_debug_plan_queue_gave_up reports).  t_block 8, 12 or 16 (0: 12),
 * band_rows 0: 96; nothing is tuned.  It exists to measure the two forms
 * against each other; the level schedule is the default.
 */
int gol_plan_create_cfg(const gol_board* boards, int64_t n, const gol_pass_config* config,
                        gol_plan** out);
/* The plan's generations per pass and band height (other fields 0). */
int gol_plan_config(const gol_plan* plan, gol_pass_config* out);
int gol_plan_run(gol_plan* plan, void* stream);
/* Describes the plan: waves per level 0, levels, total cell updates. */
int gol_plan_info(const gol_plan* plan, int64_t* waves, int64_t* levels, double* cell_updates);
int gol_plan_destroy(gol_plan* plan);

/*
 * Serving: a request loop with continuous batching.  Requests are admitted
 * while the boards resident on the device fit `hbm_budget_bytes` (two packed
 * buffers per board); every tick advances all resident boards by up to
 * `chunk_generations` in one batched schedule, new arrivals join at the next
 * tick, finished boards are copied back and leave.
 */
typedef struct gol_serve_config {
  uint64_t hbm_budget_bytes;   /* device bytes for resident boards: two buffers per board,
                                  each rounded up to a size class at most 25 % above the
                                  board's packed bytes (classes a quarter power of two
                                  apart, at least 4 KiB); buffers of retired boards stay
                                  cached for the next board of their class while the
                                  buffers held, in use or cached, fit this budget */
  int32_t chunk_generations;   /* generations per tick (>= 1), or 0: automatic -- each
                                  tick runs the whole passes that take the resident boards
                                  about 3 ms of device time at the rate measured on earlier
                                  ticks (15 passes until one has completed); behind a
                                  backlog of more than 16 such ticks (resident and queued
                                  work), a sixteenth of the backlog, up to 24 ms */
  int32_t device;              /* HIP device ordinal */
  int32_t max_resident;        /* cap on resident boards (0 = no cap) */
  int32_t t_block;             /* generations per pass: 1, 2, 4, 8, 12, 16, or 0: tuned at
                                  creation together with the band height of the tiles (8, 12
                                  or 16 x 64, 96 or 128 rows, whichever runs a stand-in
                                  resident set fastest: square boards of 512 to 8192 a side,
                                  the same cells at each size, 48 generations; with t_block
                                  given only the band height is timed; the choice is kept for
                                  the process's later servers on the same device and t_block,
                                  which start without timing).  A chunk whose tiles
                                  give fewer than two waves per SIMD halves the band height
                                  (not below 32 rows or t_block) until they do. */
} gol_serve_config;

typedef struct gol_server gol_server;

typedef struct {
  int64_t generations_done;
  double submit_s;   /* seconds on the server's clock */
  double admit_s;
  double done_s;
} gol_request_info;

int gol_serve_create(const gol_serve_config* cfg, gol_server** out);
/* Copies rows * W words from host memory before returning (padding bits are
 * cleared in the copy, so every result -- also of a request of zero
 * generations -- has them 0). */
int gol_serve_submit(gol_server* srv, const uint64_t* host_packed, int64_t rows, int64_t cols,
                     int64_t generations, uint64_t* ticket);
/* GOL_EAGAIN until done; then writes rows * W words to host_out, fills info
 * (may be NULL) and retires the ticket. */
int gol_serve_poll(gol_server* srv, uint64_t ticket, uint64_t* host_out, gol_request_info* info);
/* Blocks until the ticket is done (or failed / cancelled), then as poll. */
int gol_serve_wait(gol_server* srv, uint64_t ticket, uint64_t* host_out, gol_request_info* info);
int gol_serve_cancel(gol_server* srv, uint64_t ticket);
/* Seconds on the server's clock (the time base of gol_request_info). */
double gol_serve_now(const gol_server* srv);

/* Counters since the server was created (thread-safe snapshot). */
typedef struct {
  int64_t chunks;          /* chunks queued (one batched schedule each) */
  int64_t launches;        /* tile-pass launches queued */
  int64_t admitted;        /* requests admitted to the device */
  int64_t retired;         /* requests whose result copy was queued */
  double plan_host_s;      /* host seconds spent building and launching chunk schedules */
  double device_busy_s;    /* device seconds of completed chunks (first to last launch) */
  double cell_updates;     /* cell updates queued */
  int64_t max_resident;    /* largest number of boards in one chunk */
  double mean_resident;    /* boards per chunk, averaged over chunks */
  int64_t resident_bytes;  /* device bytes of resident boards now */
  int64_t peak_resident_bytes; /* largest value of resident_bytes (never above the budget) */
  int64_t t_block;         /* generations per pass of every chunk (given or tuned) */
  int64_t last_chunk_generations; /* generations of the last chunk queued (at most) */
  int64_t last_band_rows;  /* band height of the last chunk's tiles */
  int64_t busy_band_rows;  /* band height of a chunk with many tiles (given or tuned) */
  double admit_host_s;     /* host seconds the scheduler spent admitting requests */
  double retire_host_s;    /* host seconds spent queueing result copies of finished boards */
  double starved_s;        /* host-observed seconds with no chunk queued while boards had
                              generations left (the device waited for the scheduler) */
  double chunk_gap_s;      /* device seconds between one chunk's end and the next one's
                              start, over chunks queued while another was in flight */
} gol_serve_stats;
int gol_serve_get_stats(const gol_server* srv, gol_serve_stats* out);
int gol_serve_destroy(gol_server* srv);

/*
 * Optional allocator for the library's device scratch (e.g. a framework's
 * caching allocator).  alloc(bytes, stream, ctx) returns device memory usable
 * in stream order on `stream`; free(ptr, stream, ctx) releases it after the
 * stream's queued work.  Pass NULLs to restore the default
 * (hipMallocAsync / hipFreeAsync).
 */
typedef void* (*gol_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*gol_free_fn)(void* ptr, void* stream, void* ctx);
int gol_set_allocator(gol_alloc_fn alloc, gol_free_fn free_fn, void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GOL_H */

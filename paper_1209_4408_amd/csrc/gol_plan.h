// Host-side schedule of tile passes for one or many boards (no HIP calls).
//
// A board of G generations runs K = ceil(G / T) passes: one of them (the
// first or the last) advances G - (K - 1) T generations, every other T.
// Passes run level by level, one launch per level, Kmax = max K levels.  A
// board of the early group runs its passes at levels 0 .. K - 1 (the short
// one first), a board of the late group at levels Kmax - K .. Kmax - 1 (the
// short one last), so each launch carries a similar amount of work instead
// of the last levels holding only the few longest boards, whose passes then
// run one wave per SIMD.  Boards are assigned longest first, each to the
// group whose levels it would span hold less work so far.
//
// Tiles: a board's row of D dwords is cut into strips of at most 62 useful
// dwords (each strip + 2 halo lanes fits a 64-lane wave), its rows into bands
// of at most `band_rows` rows.  A tile is one segment of consecutive lanes.
// Tiles of 32 lanes or more get a wave of their own; smaller ones (narrow
// boards) are packed several to a wave, grouped by band height and by K so
// that packed lanes stay busy.  Each group's waves are sorted by their
// largest K, so the waves of level L are a prefix of the early group's array
// followed by a prefix of the late group's.
#pragma once
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "gol_internal.h"

namespace gol {

struct BoardReq {
  int64_t rows, cols, generations;
};

struct HostPlan {
  int T = 8;
  int band_rows = 64;
  std::vector<Segment> segs;
  std::vector<WaveItem> items;       // early group, then late group
  int32_t late_begin = 0;            // index of the late group's first wave
  std::vector<int32_t> level_early;  // level L launches items [0, level_early[L])
  std::vector<int32_t> level_late;   // and [late_begin, late_begin + level_late[L])
  std::vector<int32_t> level_items;  // waves taking part in level L (the sum)
  bool early_masked = false;         // level 0 of the early group has a pass shorter than T
  bool late_masked = false;          // the late group's last level has one
  std::vector<int32_t> K;            // passes per board
  std::vector<int32_t> Tshort;       // generations of the board's short pass
  std::vector<int32_t> start;        // level of the board's pass 0
  std::vector<int32_t> jshort;       // index of the short pass: 0 or K - 1
  double cell_updates = 0;           // sum rows * cols * generations
  double lane_steps = 0;             // sum over levels of waves * 64 * row steps
};

// Balanced split of n into k parts: part i has q + (i < r) items and starts
// at i q + min(i, r).
struct Split {
  int64_t q, r;
  int64_t size(int64_t i) const { return q + (i < r ? 1 : 0); }
  int64_t start(int64_t i) const { return i * q + (i < r ? i : r); }
};
inline Split split(int64_t n, int64_t k) { return Split{n / k, n % k}; }

// Grid of one large board for the single-board kernel, one band per wave.
GridGeom board_geometry(int64_t rows, int64_t cols, int band_rows);

// Grid for the paired layout: strips of at most 30 dwords and pairs of bands
// of one height H (band_q): the smallest H >= max(band_rows, T) with H - T a
// multiple of pd; ceil(rows / 2H) pairs (nbands = 2 x pairs), pair p covering
// rows 2 p H .. 2 p H + 2H - 1 mod rows (the last pair may overlap the first).
GridGeom paired_geometry(int64_t rows, int64_t cols, int band_rows, int T, int pd);

// Whether the paired layout runs this board with T generations per pass and
// grid g; if not, *why says which condition fails.
bool paired_ok(int64_t rows, int64_t cols, int T, const GridGeom& g, const char** why);

// Builds the batch schedule.  Returns false with a message on invalid input.
bool build_plan(const std::vector<BoardReq>& boards, int T, int band_rows, HostPlan& plan,
                std::string& err);

// Tiles of one board for schedules that keep a board's tiles between
// launches (the server computes them once per board and band height): the
// board's segments (board field 0, rows and dwords as in build_plan) and its
// waves, each holding segments of this board only.  Strips narrow enough
// that several fit a wave take consecutive bands of the same strip into one
// wave (same board, same pass count: no lane ever idles for another board).
struct BoardTiles {
  struct Wave {
    int32_t seg_begin;
    int16_t nseg;
    uint16_t h;  // tallest band of the wave
  };
  int band_rows = 0;
  bool aligned = false;  // cols % 32 == 0
  std::vector<Segment> segs;
  std::vector<Wave> waves;
};
void board_tiles(int64_t rows, int64_t cols, int band_rows, BoardTiles& out);

// One board of a chunk schedule: its tiles and the generations it advances.
struct ChunkBoard {
  const BoardTiles* tiles;
  int64_t rows, cols, generations;
};
// The batch schedule of build_plan over boards that bring their own tiles
// (no packing search: the cost is linear in the number of segments).
bool build_chunk_plan(const std::vector<ChunkBoard>& boards, int T, HostPlan& plan,
                      std::string& err);

// Band height for a chunk over these boards (rows, cols) with T generations
// per pass: `base` (the height timed fastest for a busy server) while its
// tiles give every SIMD at least two waves; with fewer tiles, the height is
// halved (not below 32 rows or T) until they do, so a lightly loaded server
// still spreads its few boards over the chip.
int chunk_band_rows(const std::vector<std::pair<int64_t, int64_t>>& boards, int T, int nsimd,
                    int base);

// The persistent work-queue form of a batch schedule (QueueItem): every
// board tiled on its own (board_tiles at band_rows), its short pass first,
// items queued pass by pass, boards within a pass longest work first.
struct QueuePlan {
  int T = 12;
  std::vector<Segment> segs;
  std::vector<QueueItem> items;
  std::vector<int32_t> per_pass;  // items of each board per pass
};
bool build_queue_plan(const std::vector<BoardReq>& boards, int T, int band_rows, QueuePlan& qp,
                      std::string& err);

// Default band height for the single-board kernel: tall bands amortise the
// 2T halo rows, but enough waves per SIMD are needed to hide latency, and the
// wave total should not leave a few SIMDs one wave behind the rest.
int default_band_rows(int64_t rows, int64_t cols, int T, int nsimd);

// Prefetch distance (rows) of the single-board kernel for T generations per pass.
int default_prefetch(int T);

// Generations per pass of the batched kernel: 1, 2, 4, 8, 12, 16.
bool valid_T(int T);
// Generations per pass of the single-board kernel.
bool valid_board_T(int T);

}  // namespace gol

// Internal types shared by the planner (host C++) and the HIP kernels.
//
// Board layout in device memory (the library boundary's packed layout): a
// board of R rows and C columns is R rows of W = ceil(C / 64) uint64 words;
// cell (r, c) is bit (c mod 64) of word r * W + c / 64, LSB first, and bits at
// columns >= C are 0.  The kernels read it as 32-bit words: row r holds
// D = 2 * W dwords, dword j carries cells 32 j .. 32 j + 31 (bit i = cell
// 32 j + i), because a little-endian uint64 is its low dword then its high one.
#pragma once
#include <stdint.h>

namespace gol {

// Upper bound on generations per pass: a halo of one 32-bit word per side is
// enough while at most 32 generations eat into it, one bit per generation.
constexpr int kMaxT = 32;
// Lanes per wave (CDNA wave64).
constexpr int kWave = 64;
// Useful columns of a strip that fills a whole wave: 64 lanes minus two halo lanes.
constexpr int kStripDwords = kWave - 2;
// Useful columns of a strip in one half of a wave (paired layout).
constexpr int kHalfStripDwords = kWave / 2 - 2;

// Fixed device scratch of gol_step_packed_noalloc: one ping-pong board of at
// most this many bytes, a device array of the code object (each GPU the
// library runs on holds its own copy until the process ends).
constexpr int64_t kFixedScratchBytes = (int64_t)64 << 20;

// Layouts of the single-board tile pass.
constexpr int kLayoutBand = 1;    // one band of one strip per wave
constexpr int kLayoutPaired = 2;  // two adjacent bands per wave, sharing their edge
constexpr int kLayoutResident = 3;  // whole board in one workgroup's LDS for a whole run

// Resident layout: threads of its workgroup, and the LDS it may use for the
// board's two generations (rows of ceil(C / 32) dwords each).
constexpr int kResidentThreads = 1024;
constexpr int64_t kResidentMaxLdsBytes = 65536;
// Resident layout geometry.  The workgroup has about one thread per dword on
// the smallest boards and kResidentThreads beyond (never fewer threads than
// dwords in a row); thread t owns dword column t mod nd of a segment of rs
// consecutive rows.  In LDS each segment is followed by one pad dword, so the
// segments a wave sweeps start in different banks.
struct ResidentGeom {
  int64_t nd, threads, nsegs, rs, words;  // words: one generation, pads included
};
constexpr ResidentGeom resident_geom(int64_t R, int64_t C) {
  const int64_t nd = (C + 31) / 32;
  const int64_t want = R * nd > nd ? R * nd : nd;
  const int64_t t = ((want + 63) / 64) * 64;
  const int64_t threads = t < kResidentThreads ? t : kResidentThreads;
  const int64_t nsegs = threads / (nd > 0 ? nd : 1);
  const int64_t rs = nsegs > 0 ? (R + nsegs - 1) / nsegs : R;
  return ResidentGeom{nd, threads, nsegs, rs, R * nd + (R - 1) / (rs > 0 ? rs : 1) + 1};
}
// Rows of at most kResidentThreads dwords; both generations within the LDS budget.
constexpr bool resident_fits(int64_t R, int64_t C) {
  return (C + 31) / 32 <= kResidentThreads &&
         resident_geom(R, C).words * 8 <= kResidentMaxLdsBytes;
}

// Prefetch distances (rows) compiled for each layout and pass length.
constexpr bool pass_config_compiled(int layout, int T, int pd) {
  return layout == kLayoutBand
             ? (((T == 1 || T == 2 || T == 4) && (pd == 3 || pd == 6)) ||
                ((T == 8 || T == 12) && (pd == 6 || pd == 9)) || (T == 16 && (pd == 9 || pd == 12)))
             : layout == kLayoutPaired && (T == 8 || T == 12 || T == 16) && (pd == 9 || pd == 12);
}

// One board as seen by one launch of the pass kernel.  The board runs pass
// j (0-based) at level start + j.  Pass j reads  src0            if j == 0,
//                                                w[(j-1+par)&1]  otherwise,
// and writes                                     w[(j+par)&1].
// Pass jshort advances Tshort generations, every other pass the kernel's T.
struct BoardDesc {
  const uint32_t* src0;
  uint32_t* w[2];
  int32_t R;       // rows
  int32_t C;       // columns (cells per row)
  int32_t D;       // dwords per row = 2 * ceil(C / 64)
  int32_t K;       // passes
  int32_t Tshort;  // generations of pass jshort, 1 <= Tshort <= T
  int32_t par;
  int32_t start;   // level of pass 0
  int32_t jshort;  // 0 or K - 1
};

// A run of consecutive lanes of one wave that work on one tile of one board:
// lanes lane0 .. lane0 + nlanes - 1 hold logical dwords p0 .. p0 + nlanes - 1
// of rows r0 - T .. r0 + h + T - 1; the first and last lane are halo, the
// others write rows r0 .. r0 + h - 1.  Logical dword p covers the logical
// columns 32 p .. 32 p + 31, and logical column x is cell x mod C (the torus
// unrolled), so p may be -1 or reach past the row end.
struct Segment {
  int32_t board;
  int32_t p0;
  int32_t r0;
  uint16_t h;
  uint8_t lane0;
  uint8_t nlanes;
};

// One wave's work in a launch: segments [seg_begin, seg_begin + nseg).
struct WaveItem {
  int32_t seg_begin;
  int16_t nseg;
  uint16_t h;      // max h over its segments
  int32_t maxK;    // largest pass count of its boards: the wave takes part in
                   // levels 0 .. maxK - 1 (early group) or Kmax - maxK ..
                   // Kmax - 1 (late group)
  int32_t flags;   // kItemAligned: every lane's board has C % 32 == 0
};
constexpr int32_t kItemAligned = 1;

// Persistent work-queue form of a batch schedule: one launch whose waves take
// items in queue order (an atomic counter), each item one wave of one
// board's tiles in one pass.  Pass j of a board waits until the board's
// counter of finished items reaches j x (its items per pass); items are
// queued pass by pass, so an item waits only on items taken before it.
struct QueueItem {
  int32_t seg_begin;
  int16_t nseg;
  uint16_t h;      // tallest band of the item's segments
  int32_t board;
  int32_t pass;
  int32_t flags;   // kItemAligned
};
// Control words of a queue launch (zeroed before it): next item, error
// (a wait gave up), then one finished-item counter per board.
constexpr int kQueueCtlHeader = 2;

// Geometry of a single large board split into strips x bands, one wave per
// tile, computed from the block index (no tables).
struct GridGeom {
  int32_t nstrips;   // strips across a row
  int32_t nbands;    // bands down the board
  int32_t strip_q, strip_r;  // balanced split of D dwords: first strip_r strips get q+1
  int32_t band_q, band_r;    // balanced split of R rows
};

}  // namespace gol

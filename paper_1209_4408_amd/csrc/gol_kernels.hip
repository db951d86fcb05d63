// HIP kernels for gfx950 (CDNA4): Conway's Life, B3/S23, on a torus.
//
// The method (the paper, Section 1): every cell has eight neighbours, all
// cells change at once each time step, a live cell survives with two or three
// live neighbours, a dead cell is born with exactly three.  The grid is a
// torus (Section 2.2): rows and columns wrap.  Boards are bit-packed, one bit
// per cell (see gol_internal.h for the layout).
//
// Tile pass.  One wave (64 lanes) owns a tile: a strip of consecutive 32-bit
// column words ("dwords") and a band of rows.  Lane l holds logical dword
// p0 + l of the rows it sweeps, top to bottom; the first and last lane of the
// strip are halo.  The wave advances the tile by T generations in one sweep:
// a T-stage pipeline held in registers, stage s turning generation s rows into
// generation s + 1 rows one row behind stage s - 1.  Each stage keeps a
// window of three rows.  Horizontal neighbour bits cross lanes with DPP
// (wave_shr / wave_shl) and v_alignbit; the neighbour count and the rule are
// a bit-sliced adder network of v_bitop3 ops (gfx950's 3-input logic op).
//
// Torus seam.  A lane's dword is a window of 32 logical columns, logical
// column x being cell x mod C.  The window is gathered once per row at load
// time (funnel shift across the seam for C not a multiple of 32), so the
// generation pipeline itself never sees the seam and every board shape,
// including tori narrower than 3 cells, takes the same path.  Rows wrap the
// same way: the sweep reads rows r0 - T .. r0 + h + T - 1 modulo R.
//
// Halo.  A stage's lanes at the ends of a strip get wrong neighbour bits from
// outside the strip; wrong bits move inward one column per generation, so
// after T <= 32 generations the halo dwords absorb them and every inner lane
// is exact.  Likewise the T extra rows above and below the band.
//
// Besides the torus pass: the same pass on a bounded board (cells beyond the
// edges dead at every generation) and on a strip of a larger torus whose halo
// rows come from two other buffers (both selected by the gather mode);
// batched passes over many boards from tables; small boards resident in one
// workgroup's LDS for a whole run (k_board_lds); the live-cell count
// (k_population); pack / unpack of byte boards.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "gol_internal.h"

// Which instruction kinds the scheduler may move across a row step's load
// request (0: none, so the request stays PD steps ahead of its use).
#ifndef GOL_PREFETCH_FENCE_MASK
#define GOL_PREFETCH_FENCE_MASK 0
#endif
// Prefetch distance (rows) of the batch kernel.
#ifndef GOL_BATCH_PREFETCH
#define GOL_BATCH_PREFETCH 6
#endif

namespace gol {

// ---------------------------------------------------------------------------
// Bit-sliced logic.  v_bitop3_b32 computes any function of three inputs from
// an 8-entry truth table; the table of f is f(0xF0, 0xCC, 0xAA).
// ---------------------------------------------------------------------------
constexpr uint32_t kXor3 = (0xF0u ^ 0xCCu ^ 0xAAu) & 0xFFu;                               // 0x96
constexpr uint32_t kMaj3 = ((0xF0u & 0xCCu) | (0xF0u & 0xAAu) | (0xCCu & 0xAAu)) & 0xFFu;   // 0xE8
// e1(v, c0, u) = !v & (c0 ^ u)
constexpr uint32_t kE1 = (~0xF0u & (0xCCu ^ 0xAAu)) & 0xFFu;                               // 0x06
// e2(v, c0, u) = v ? (!c0 & !u) : (c0 & u)
constexpr uint32_t kE2 = ((0xF0u & ~0xCCu & ~0xAAu) | (~0xF0u & 0xCCu & 0xAAu)) & 0xFFu;     // 0x18
// sel(s, a, b) = s ? a : b
constexpr uint32_t kSel = ((0xF0u & 0xCCu) | (~0xF0u & 0xAAu)) & 0xFFu;                    // 0xCA
constexpr uint32_t kAnd3 = (0xF0u & 0xCCu & 0xAAu) & 0xFFu;                                 // 0x80

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, kXor3);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, kMaj3);
}

// Next generation of a 32-cell dword from the horizontal 3-sums of the row
// above (a), the row itself (c) and the row below (b), each sum as a 2-bit
// number lo + 2 hi, and the row's own cells x.
//   nine-cell sum  S = (lo_a+lo_c+lo_b) + 2 (hi_a+hi_c+hi_b)
//                    = s0 + 2 (c0 + u + 2 v)
//   live next  <=>  S == 3  or  (x and S == 4)
//   S == 3  <=>  s0 and !v and (c0 ^ u)
//   S == 4  <=>  !s0 and (v ? !c0 & !u : c0 & u)
// (S counts the cell itself: 3 = birth or survival with two neighbours,
// 4 with a live cell = survival with three neighbours.)
__device__ __forceinline__ uint32_t life_rule(uint32_t lo_a, uint32_t lo_c, uint32_t lo_b,
                                              uint32_t hi_a, uint32_t hi_c, uint32_t hi_b,
                                              uint32_t x) {
  const uint32_t s0 = xor3(lo_a, lo_c, lo_b);
  const uint32_t c0 = maj3(lo_a, lo_c, lo_b);
  const uint32_t u = xor3(hi_a, hi_c, hi_b);
  const uint32_t v = maj3(hi_a, hi_c, hi_b);
  const uint32_t e1 = __builtin_amdgcn_bitop3_b32(v, c0, u, kE1);
  const uint32_t e2 = __builtin_amdgcn_bitop3_b32(v, c0, u, kE2);
  const uint32_t f = x & e2;
  return __builtin_amdgcn_bitop3_b32(s0, e1, f, kSel);
}

// Lane l receives src of lane l - 1 (lane 0 receives 0).
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}
// Lane l receives src of lane l + 1 (lane 63 receives 0).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}

// ---------------------------------------------------------------------------
// Per-lane state of one tile sweep.
// ---------------------------------------------------------------------------
struct Lane {
  int32_t R, D;
  // Gather of the lane's 32 logical columns from two words of the row:
  // a = dword ia and b = dword ib.
  //   C >= 64: the window starts at cell q = 32 ia + sh.  Where it stays
  //     inside the row, b = dword ia + 1 supplies the bits past dword ia and
  //     m1 = ~0; where it passes the row end after n1 < 32 cells, b = dword 0
  //     (the row's start) and m1 keeps the n1 low bits:
  //       window = m1 ? alignbit(b, a, sh) : b << n1   (bitwise select).
  //   C < 64 (narrow): a, b = dwords 0 and 1 hold the whole row; it is
  //     repeated up a 64-bit word and the window read from bit q, which sh
  //     holds (and n1 holds C).
  // Bounded boards read the lane's own dword (doff) and m1 keeps the bits
  // that are cells of the board (0 for a lane beyond either edge).
  int32_t ia, ib;
  uint32_t sh, n1, m1;
  bool narrow;
  bool live;            // lane has a board in this launch
  // rows
  int32_t in_r;
  const uint32_t* in_row;
  int32_t out_r;
  uint32_t* out_row;
  int64_t wrap;         // R * D: a row pointer that reaches row R moves back by this
  int32_t in_u;         // input row before wrapping (bounded boards, strips)
  const uint32_t* mid;  // strips: the strip's row 0
  const uint32_t* bot;  // strips: the first row below the strip
  int32_t emit_base;    // r0 - T - 1: the row stage 0 emits at step i is emit_base + i
  uint32_t vbits;       // bounded boards: bit S set if stage S emits a row of the board
  uint32_t doff;        // bounded boards: byte offset of the lane's word, or past the row
  // store
  bool store;
  uint32_t soff;        // byte offset of the lane's dword in a row
  uint32_t smask;
  int32_t hl;           // rows this lane writes
  int32_t Tl;           // generations this lane advances (masked pipelines)
};

__device__ __forceinline__ void lane_setup(Lane& L, const uint32_t* src, uint32_t* dst, int32_t R,
                                           int32_t C, int32_t D, int32_t p, int32_t lane_in_seg,
                                           int32_t nlanes, int32_t r0, int32_t h, int32_t T,
                                           int32_t Tl, bool live) {
  L.R = R;
  L.D = D;
  L.live = live;
  L.Tl = Tl;
  int64_t q64 = ((int64_t)p * 32) % (int64_t)C;
  if (q64 < 0) q64 += C;
  const uint32_t q = (uint32_t)q64;
  L.narrow = C < 64;
  const int32_t nd = (C + 31) >> 5;
  if (!L.narrow) {
    // Only a right halo lane that follows a padding dword can need the
    // dwords ia, ia + 1 and 0 at once; its cells never reach a stored word
    // within T <= 32 generations, so it takes dword 0.
    L.ia = (int32_t)(q >> 5);
    L.sh = q & 31u;
    const uint32_t n1 = (uint32_t)min((int64_t)32, (int64_t)C - (int64_t)q);
    const bool past_end = n1 < 32u;
    L.ib = past_end ? 0 : (L.sh != 0u && L.ia + 1 < nd ? L.ia + 1 : L.ia);
    L.n1 = n1 & 31u;
    L.m1 = past_end ? (1u << n1) - 1u : 0xFFFFFFFFu;
  } else {
    L.ia = 0;
    L.ib = 1;  // D == 2
    L.sh = q;
    L.n1 = (uint32_t)C;
    L.m1 = 0xFFFFFFFFu;
  }
  int64_t rin = ((int64_t)r0 - T) % (int64_t)R;
  if (rin < 0) rin += R;
  L.wrap = (int64_t)R * D;
  L.in_r = (int32_t)rin;
  L.in_u = r0 - T;
  L.emit_base = r0 - T - 1;
  L.in_row = src + rin * (int64_t)D;
  L.out_r = r0;
  L.out_row = dst + (int64_t)r0 * D;
  L.store = live && lane_in_seg >= 1 && lane_in_seg <= nlanes - 2 && p >= 0 && p < D;
  L.soff = L.store ? (uint32_t)p * 4u : 0u;
  const int64_t c0 = (int64_t)p * 32;
  L.smask = (c0 + 32 <= C) ? 0xFFFFFFFFu : (c0 >= C ? 0u : ((1u << (uint32_t)(C - c0)) - 1u));
  L.hl = h;
}

// Buffer descriptor word 3 for untyped 32-bit buffer access on gfx9-family
// parts; offsets at or past num_records are dropped by the range check.
constexpr int kBufferDword3 = 0x00020000;
constexpr uint32_t kDroppedOffset = 0x80000000u;

// A pointer that is the same in every lane, moved to scalar registers.
// __builtin_amdgcn_readfirstlane takes and returns 32 bits, so the two halves
// of the 64-bit address are read separately.
__device__ __forceinline__ uint32_t* uniform_ptr(uint32_t* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (uint32_t*)(uintptr_t)(((uint64_t)hi << 32) | (uint64_t)lo);
}

struct Raw {
  uint32_t a, b;
};

// How a lane gathers its 32 columns of a row (load_raw / window):
constexpr int kGatherTorus = 0;    // C % 32 != 0: two words of the row (Lane)
constexpr int kGatherAligned = 1;  // C % 32 == 0: the lane's own word
constexpr int kGatherBounded = 2;  // cells beyond the board's edges are dead:
                                   // rows outside 0 .. R - 1 and columns outside
                                   // 0 .. C - 1 read as 0
// Added to kGatherTorus or kGatherAligned: the R rows are a strip of a larger
// torus; the rows above and below it come from two other buffers (halo rows)
// instead of wrapping around the strip.  Columns still wrap.
constexpr int kHaloRows = 4;
constexpr int col_gather(int g) { return g & 3; }

// Boards live in global memory.  Pointers read from the batch tables are
// generic to the compiler, and a generic (flat) load may be an LDS access that
// completes out of order, so each use of a flat load's result would wait for
// every load in flight and defeat the prefetch ring; global-address-space
// accesses complete in order and can be waited for one at a time.
typedef const __attribute__((address_space(1))) uint32_t* GlobalIn;
typedef __attribute__((address_space(1))) uint32_t* GlobalOut;

// Every lane loads every step from an address inside the board (idle lanes
// and lanes whose gather needs one word read a valid word they ignore), so
// the loads carry no branch and the compiler can wait for each one alone.
template <int GATHER>
__device__ __forceinline__ Raw load_raw(const Lane& L) {
  Raw r;
  if constexpr (GATHER == kGatherBounded) {
    // a row outside the board has no records: every lane reads 0; a lane
    // outside the row carries an offset past the row, which also reads 0
    const bool row_in = L.in_u >= 0 && L.in_u < L.R;  // uniform
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)uniform_ptr((uint32_t*)L.in_row), 0, row_in ? L.D * 4 : 0, kBufferDword3);
    r.a = __builtin_amdgcn_raw_buffer_load_b32(rs, L.doff, 0, 0);
    r.b = 0u;
  } else {
    r.a = ((GlobalIn)L.in_row)[L.ia];
    r.b = col_gather(GATHER) == kGatherAligned ? 0u : ((GlobalIn)L.in_row)[L.ib];
  }
  return r;
}

template <int GATHER>
__device__ __forceinline__ uint32_t window(const Raw& r, const Lane& L) {
  if constexpr (col_gather(GATHER) == kGatherAligned) return r.a;
  if constexpr (GATHER == kGatherBounded) return r.a & L.m1;  // the row's cells only
  if (!L.narrow)
    return __builtin_amdgcn_bitop3_b32(L.m1, __builtin_amdgcn_alignbit(r.b, r.a, L.sh),
                                       r.b << L.n1, kSel);
  // C < 64: the row, with its padding bits cleared (input padding is not
  // trusted), repeated by doubling: after k steps the first C 2^k bits are
  // the row over and over.  Five steps reach 32 cells past any q < C.
  uint32_t len = L.n1;
  // recompute the shift counts every row rather than hold them for the whole
  // sweep (registers are allocated for the kernel's largest path)
  asm volatile("" : "+v"(len));
  uint64_t v = ((uint64_t)r.b << 32 | r.a) & ((1ull << len) - 1ull);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    v |= len < 64u ? v << len : 0ull;
    len <<= 1;
  }
  return (uint32_t)(v >> L.sh);
}

template <int GATHER>
__device__ __forceinline__ void advance_in(Lane& L) {
  L.in_u += 1;
  if constexpr ((GATHER & kHaloRows) != 0) {
    // rows -T .. -1 from the top halo, 0 .. R - 1 from the strip, R .. R + T - 1
    // from the bottom halo; the prefetch past the tile's last row (never used)
    // re-reads the bottom halo's last row
    if (L.in_u == 0)
      L.in_row = L.mid;
    else if (L.in_u == L.R)
      L.in_row = L.bot;
    else if (L.in_u < L.R + L.Tl)
      L.in_row += L.D;
    return;
  }
  L.in_r += 1;
  L.in_row += L.D;
  if (L.in_r == L.R) {
    L.in_r = 0;
    L.in_row -= L.wrap;
  }
}

__device__ __forceinline__ void advance_out(Lane& L) {
  L.out_r += 1;
  L.out_row += L.D;
  if (L.out_r == L.R) {
    L.out_r = 0;
    L.out_row -= L.wrap;
  }
}

template <int TM>
struct Pipe {
  uint32_t lo[TM][3];
  uint32_t hi[TM][3];
  uint32_t xs[TM][3];
};

// Stage S of the pipeline at a step of phase PH (step index mod 3).  Stage S
// receives generation-S row m = step - S into slot m mod 3 and, once it holds
// rows m - 2, m - 1, m, emits generation S + 1 of row m - 1 to stage S + 1.
// In the prologue (PRO) the step index K is known at compile time and stages
// that have not yet received (K < 2S) or cannot yet emit (K < 2S + 2) stop.
// BND (bounded boards): every generation a stage emits keeps only cells of
// the board -- columns outside 0 .. C - 1 (m1) and rows outside 0 .. R - 1
// (bit S of L.vbits clear) are dead again, or a birth just beyond an edge
// would reach the board one generation later.  The row test is a uniform
// bit turned into a mask by arithmetic, so it costs one bitop3 and no branch.
template <int TM, bool MASKED, int PH, int S, bool PRO, int K, bool BND = false>
__device__ __forceinline__ void stages(uint32_t& x, Pipe<TM>& P, const Lane& L) {
  if constexpr (S < TM) {
    if constexpr (!(PRO && K < 2 * S)) {
      constexpr int slot = ((PH - S) % 3 + 3) % 3;
      constexpr int sa = (slot + 1) % 3;  // row m - 2
      constexpr int sc = (slot + 2) % 3;  // row m - 1
      const uint32_t xp = from_prev_lane(x);
      const uint32_t xn = from_next_lane(x);
      const uint32_t xl = __builtin_amdgcn_alignbit(x, xp, 31);  // west neighbours
      const uint32_t xr = __builtin_amdgcn_alignbit(xn, x, 1);   // east neighbours
      P.lo[S][slot] = xor3(xl, x, xr);
      P.hi[S][slot] = maj3(xl, x, xr);
      P.xs[S][slot] = x;
      if constexpr (!(PRO && K < 2 * S + 2)) {
        uint32_t y = life_rule(P.lo[S][sa], P.lo[S][sc], P.lo[S][slot], P.hi[S][sa], P.hi[S][sc],
                               P.hi[S][slot], P.xs[S][sc]);
        if (MASKED) y = (S < L.Tl) ? y : P.xs[S][sc];
        if constexpr (BND) {
          const uint32_t rows_in = 0u - ((L.vbits >> S) & 1u);
          y = __builtin_amdgcn_bitop3_b32(y, L.m1, rows_in, kAnd3);
        }
        x = y;
        stages<TM, MASKED, PH, S + 1, PRO, K, BND>(x, P, L);
      }
    }
  }
}

// One row step.  P3 = step index mod 3 (stage slots), PP = step index mod PD
// (the prefetch ring: the row consumed now was loaded PD steps earlier, and
// the row PD steps ahead is requested in its place).
template <int TM, bool MASKED, int GATHER, int PD, bool BUFST, int P3, int PP, bool PRO, int K>
__device__ __forceinline__ void step(int i, int nsteps, Lane& L, Pipe<TM>& P, Raw (&PF)[PD]) {
  uint32_t x = window<GATHER>(PF[PP], L);
  // rows wrap, so the PD rows requested past the band's end are valid too
  PF[PP] = load_raw<GATHER>(L);
  advance_in<GATHER>(L);
  // keep the request here, PD steps ahead of its use (the mask says which
  // instruction kinds the scheduler may still move across this point)
  __builtin_amdgcn_sched_barrier(GOL_PREFETCH_FENCE_MASK);
  if constexpr (GATHER == kGatherBounded) {
    // stage S emits row emit_base + i - S (the sweep starts at row r0 - T):
    // bit S of vbits says whether that row lies on the board
    const int row0 = L.emit_base + i;
    const int lo = max(0, row0 - L.R + 1), hi = min(TM - 1, row0);
    L.vbits = lo > hi ? 0u : (((2u << hi) - 1u) & ~((1u << lo) - 1u));
  }
  stages<TM, MASKED, P3, 0, PRO, K, GATHER == kGatherBounded>(x, P, L);
  if constexpr (!PRO) {
    // stage TM - 1 emitted generation TM of output row i - 2 TM of the band
    if constexpr (BUFST) {
      // the wave's output row is uniform: one buffer store, no branch; lanes
      // that do not write carry an offset the range check drops
      uint32_t* row = uniform_ptr(L.out_row);
      __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc(row, 0, L.D * 4, kBufferDword3);
      __builtin_amdgcn_raw_buffer_store_b32(x & L.smask, rs, L.soff, 0, 0);
    } else {
      if (L.store && i - 2 * TM < L.hl)
        *(GlobalOut)((char*)L.out_row + L.soff) = x & L.smask;
    }
    advance_out(L);
  }
}

template <int TM, bool MASKED, int GATHER, int PD, bool BUFST, int K>
__device__ __forceinline__ void prologue(int nsteps, Lane& L, Pipe<TM>& P, Raw (&PF)[PD]) {
  if constexpr (K < 2 * TM) {
    step<TM, MASKED, GATHER, PD, BUFST, K % 3, K % PD, true, K>(K, nsteps, L, P, PF);
    prologue<TM, MASKED, GATHER, PD, BUFST, K + 1>(nsteps, L, P, PF);
  }
}

// Steady state: PD consecutive steps starting at a step index congruent to
// 2 TM modulo PD (PD is 3 or 6, so the slot phase is fixed too).
template <int TM, bool MASKED, int GATHER, int PD, bool BUFST, int U>
__device__ __forceinline__ void body(int i, int nsteps, Lane& L, Pipe<TM>& P, Raw (&PF)[PD]) {
  if constexpr (U < PD) {
    constexpr int k = 2 * TM + U;
    step<TM, MASKED, GATHER, PD, BUFST, k % 3, k % PD, false, 0>(i + U, nsteps, L, P, PF);
    body<TM, MASKED, GATHER, PD, BUFST, U + 1>(i, nsteps, L, P, PF);
  }
}

template <int TM, bool MASKED, int GATHER, int PD, bool BUFST, int U>
__device__ __forceinline__ void tail(int i, int nsteps, Lane& L, Pipe<TM>& P, Raw (&PF)[PD]) {
  if constexpr (U < PD - 1) {
    if (i + U < nsteps) {
      constexpr int k = 2 * TM + U;
      step<TM, MASKED, GATHER, PD, BUFST, k % 3, k % PD, false, 0>(i + U, nsteps, L, P, PF);
      tail<TM, MASKED, GATHER, PD, BUFST, U + 1>(i, nsteps, L, P, PF);
    }
  }
}

// Sweep one tile: H output rows (the wave's largest band), TM generations,
// input rows requested PD steps ahead of use.
template <int TM, bool MASKED, int GATHER, int PD, bool BUFST>
__device__ __forceinline__ void run_tile(Lane& L, int H) {
  static_assert(TM >= 1 && TM <= kMaxT, "generations per pass");
  static_assert(PD % 3 == 0 && PD >= 3, "prefetch distance");
  Pipe<TM> P;
  Raw PF[PD];
  const int nsteps = H + 2 * TM;  // >= 3
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    PF[k] = load_raw<GATHER>(L);
    advance_in<GATHER>(L);
  }
  prologue<TM, MASKED, GATHER, PD, BUFST, 0>(nsteps, L, P, PF);
  int i = 2 * TM;
  for (; i + PD - 1 < nsteps; i += PD) body<TM, MASKED, GATHER, PD, BUFST, 0>(i, nsteps, L, P, PF);
  tail<TM, MASKED, GATHER, PD, BUFST, 0>(i, nsteps, L, P, PF);
}

// Workgroups are dealt to the 8 XCDs of the chip in turn; give each XCD a
// contiguous range of items so tiles that share halo rows share an L2.
__device__ __forceinline__ int xcd_item(int nitems) {
  const int per = (nitems + 7) >> 3;
  const int b = (int)blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Single board: tile (strip s, band b) from the block index, no tables.
// ---------------------------------------------------------------------------
struct PassArgs {
  const uint32_t* src;
  uint32_t* dst;
  int32_t R, C, D;
  const uint32_t* top;  // strips (kHaloRows): T rows above row 0, the farthest first
  const uint32_t* bot;  // strips: T rows below row R - 1, the nearest first
};

template <int TM, int PD, int GATHER>
__global__ __launch_bounds__(64) void k_board_pass(PassArgs a, GridGeom g) {
  const int nitems = g.nstrips * g.nbands;
  const int item = xcd_item(nitems);
  if (item >= nitems) return;  // whole wave
  const int s = item % g.nstrips, b = item / g.nstrips;
  const int us = g.strip_q + (s < g.strip_r ? 1 : 0);
  const int ds = s * g.strip_q + min(s, g.strip_r);
  const int hb = g.band_q + (b < g.band_r ? 1 : 0);
  const int rb = b * g.band_q + min(b, g.band_r);
  const int lane = (int)threadIdx.x;
  const int nl = us + 2;
  Lane L;
  lane_setup(L, a.src, a.dst, a.R, a.C, a.D, ds - 1 + lane, lane, nl, rb, hb, TM, TM, lane < nl);
  if (!L.store) L.soff = kDroppedOffset;
  if constexpr ((GATHER & kHaloRows) != 0) {
    L.mid = a.src;
    L.bot = a.bot;
    L.in_row = L.in_u < 0 ? a.top + (int64_t)(L.in_u + TM) * a.D : a.src + (int64_t)L.in_u * a.D;
  }
  if constexpr (GATHER == kGatherBounded) {
    const int p = ds - 1 + lane;
    const int nd = (a.C + 31) >> 5;
    // A tile whose sweep reads only rows rb - T .. rb + hb + T - 1 and whole
    // dwords ds - 1 .. ds + us of the board never meets an edge: the plain
    // gather of the lane's own dword (ia == p there) serves it, with no masks.
    if (rb - TM >= 0 && rb + hb + TM <= a.R && ds >= 1 && ds + us < (a.C >> 5)) {
      run_tile<TM, false, kGatherAligned, PD, true>(L, hb);
      return;
    }
    const bool col_in = p >= 0 && p < nd;
    const int64_t c0 = (int64_t)p * 32;
    L.doff = col_in ? (uint32_t)p * 4u : kDroppedOffset;
    L.m1 = !col_in ? 0u
                   : (c0 + 32 <= a.C ? 0xFFFFFFFFu : ((1u << (uint32_t)(a.C - c0)) - 1u));
  }
  run_tile<TM, false, GATHER, PD, true>(L, hb);
}

// ---------------------------------------------------------------------------
// Single board, paired bands in the two halves of one wave.
//
// A band swept on its own recomputes a cone of T rows beyond each of its
// edges.  Here lanes 0-31 sweep band 2p downwards and lanes 32-63 sweep band
// 2p + 1 upwards, over the same strip of at most 30 dwords (each half has its
// own two halo lanes; the DPP shifts that cross lane 31 / 32 only touch halo
// lanes), so both halves reach the edge between the bands at the end of
// their sweeps.  There, instead of computing the other band's rows, the
// halves trade them: stage s of one half needs generation s of the first
// row beyond the edge, which is the other half's own edge row as its stage
// s - 1 emitted it one step earlier.  Both halves run one instruction
// stream, so the last T steps of the sweep (the epilogue) pass one row each
// way with v_permlane32_swap, and stage e stops after epilogue step e; only
// the outer edges of the pair keep a cone.  (The rule is symmetric under
// reflection, so the upward sweep is the same pipeline over the rows in
// reverse order.)
//
// Every band has the same height H, with H - T a multiple of the prefetch
// distance, so the sweep reaches its epilogue at a step whose slot and
// prefetch phases are known at compile time.  Pair p covers rows 2 p H ..
// 2 p H + 2 H - 1 (mod R); when the pairs together cover more than R rows the
// last pair overlaps the first, and both write the same (correct) next state
// into the shared rows.  Rows go through buffer loads and stores at per-lane
// byte offsets into the board (boards below 2 GiB); each half's row index is
// a scalar that wraps around the torus.
// ---------------------------------------------------------------------------
// One stage at a step of slot phase PH (see stages): receive x, emit the
// next generation of the row before it.
template <int TM, int PH, int S>
__device__ __forceinline__ uint32_t one_stage(uint32_t x, Pipe<TM>& P) {
  constexpr int slot = ((PH - S) % 3 + 3) % 3;
  constexpr int sa = (slot + 1) % 3;
  constexpr int sc = (slot + 2) % 3;
  const uint32_t xp = from_prev_lane(x);
  const uint32_t xn = from_next_lane(x);
  const uint32_t xl = __builtin_amdgcn_alignbit(x, xp, 31);
  const uint32_t xr = __builtin_amdgcn_alignbit(xn, x, 1);
  P.lo[S][slot] = xor3(xl, x, xr);
  P.hi[S][slot] = maj3(xl, x, xr);
  P.xs[S][slot] = x;
  return life_rule(P.lo[S][sa], P.lo[S][sc], P.lo[S][slot], P.hi[S][sa], P.hi[S][sc],
                   P.hi[S][slot], P.xs[S][sc]);
}

struct HalfLane {
  int32_t R, D;
  uint32_t in_off, in_step;    // byte offset of the lane's input dword, change per row
  uint32_t out_off, out_step;  // same for the output (step 0 for lanes that never store)
  uint32_t smask;
  int32_t in_a, in_b;          // current input row of each half (uniform)
  int32_t out_a, out_b;
  uint32_t wrap;               // R * D * 4
  bool upper;                  // lane in the upper half (band 2p + 1)
};

constexpr uint32_t kHalfDropped = 0xFFFFFF00u;

// Next row of each half.  WRAP: some row of this wave's sweep lies across
// the torus seam (only waves next to row 0 take that path).
template <bool WRAP>
__device__ __forceinline__ void half_advance_in(HalfLane& L) {
  L.in_off += L.in_step;
  if constexpr (WRAP) {
    L.in_a += 1;
    if (L.in_a == L.R) {  // uniform
      L.in_a = 0;
      if (!L.upper) L.in_off -= L.wrap;
    }
    L.in_b -= 1;
    if (L.in_b < 0) {  // uniform
      L.in_b += L.R;
      if (L.upper) L.in_off += L.wrap;
    }
  }
}

template <bool WRAP>
__device__ __forceinline__ void half_advance_out(HalfLane& L) {
  L.out_off += L.out_step;
  if constexpr (WRAP) {
    L.out_a += 1;
    if (L.out_a == L.R) {
      L.out_a = 0;
      if (!L.upper && L.out_step) L.out_off -= L.wrap;
    }
    L.out_b -= 1;
    if (L.out_b < 0) {
      L.out_b += L.R;
      if (L.upper && L.out_step) L.out_off += L.wrap;
    }
  }
}

template <int TM, int PD, bool WRAP, int P3, int PP, bool PRO, int K>
__device__ __forceinline__ void hstep(HalfLane& L, Pipe<TM>& P, uint32_t (&PF)[PD],
                                      __amdgpu_buffer_rsrc_t src, __amdgpu_buffer_rsrc_t dst) {
  uint32_t x = PF[PP];
  PF[PP] = __builtin_amdgcn_raw_buffer_load_b32(src, L.in_off, 0, 0);
  half_advance_in<WRAP>(L);
  __builtin_amdgcn_sched_barrier(GOL_PREFETCH_FENCE_MASK);
  Lane unused;  // read only by masked pipelines
  stages<TM, false, P3, 0, PRO, K>(x, P, unused);
  if constexpr (!PRO) {
    __builtin_amdgcn_raw_buffer_store_b32(x & L.smask, dst, L.out_off, 0, 0);
    half_advance_out<WRAP>(L);
  }
}

template <int TM, int PD, bool WRAP, int K>
__device__ __forceinline__ void hprologue(HalfLane& L, Pipe<TM>& P, uint32_t (&PF)[PD],
                                          __amdgpu_buffer_rsrc_t src, __amdgpu_buffer_rsrc_t dst) {
  if constexpr (K < 2 * TM) {
    hstep<TM, PD, WRAP, K % 3, K % PD, true, K>(L, P, PF, src, dst);
    hprologue<TM, PD, WRAP, K + 1>(L, P, PF, src, dst);
  }
}

template <int TM, int PD, bool WRAP, int U>
__device__ __forceinline__ void hbody(HalfLane& L, Pipe<TM>& P, uint32_t (&PF)[PD],
                                      __amdgpu_buffer_rsrc_t src, __amdgpu_buffer_rsrc_t dst) {
  if constexpr (U < PD) {
    constexpr int k = 2 * TM + U;
    hstep<TM, PD, WRAP, k % 3, k % PD, false, 0>(L, P, PF, src, dst);
    hbody<TM, PD, WRAP, U + 1>(L, P, PF, src, dst);
  }
}

template <int TM, int PD, bool WRAP, int U>
__device__ __forceinline__ void htail(int i, int n, HalfLane& L, Pipe<TM>& P, uint32_t (&PF)[PD],
                                      __amdgpu_buffer_rsrc_t src, __amdgpu_buffer_rsrc_t dst) {
  if constexpr (U < PD - 1) {
    if (i + U < n) {
      constexpr int k = 2 * TM + U;
      hstep<TM, PD, WRAP, k % 3, k % PD, false, 0>(L, P, PF, src, dst);
      htail<TM, PD, WRAP, U + 1>(i, n, L, P, PF, src, dst);
    }
  }
}

// The other half's value of x (lane l receives lane l xor 32).
__device__ __forceinline__ uint32_t swap_halves(uint32_t x, bool upper) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return upper ? r[0] : r[1];
}

// Epilogue step at sweep step index K (mod 3), stages S .. TM - 1; stage
// K - 2 TM (the one at the shared edge) hands its emitted row to `edge`.
template <int TM, int K, int S>
__device__ __forceinline__ void hepi_stages(uint32_t& x, Pipe<TM>& P, uint32_t& edge) {
  if constexpr (S < TM) {
    x = one_stage<TM, K % 3, S>(x, P);
    if constexpr (S == K - 2 * TM) edge = x;
    hepi_stages<TM, K, S + 1>(x, P, edge);
  }
}

template <int TM, bool WRAP, int E>
__device__ __forceinline__ void hepilogue(uint32_t xin, HalfLane& L, Pipe<TM>& P,
                                          __amdgpu_buffer_rsrc_t dst) {
  if constexpr (E < TM) {
    uint32_t x = xin, edge = 0u;
    // epilogue step E is sweep step H + TM + E, congruent to 2 TM + E mod 3
    hepi_stages<TM, 2 * TM + E, E>(x, P, edge);
    __builtin_amdgcn_raw_buffer_store_b32(x & L.smask, dst, L.out_off, 0, 0);
    half_advance_out<WRAP>(L);
    if constexpr (E + 1 < TM) {
      // stage E emitted this half's edge row (generation E + 1); the other
      // half's stage E + 1 receives it next step
      hepilogue<TM, WRAP, E + 1>(swap_halves(edge, L.upper), L, P, dst);
    }
  }
}

// One wave's sweep: H + 2 TM steps, the last TM of them the epilogue.
template <int TM, int PD, bool WRAP>
__device__ __forceinline__ void run_tile_half(HalfLane& L, int H, __amdgpu_buffer_rsrc_t rsrc,
                              __amdgpu_buffer_rsrc_t rdst) {
  Pipe<TM> P;
  uint32_t PF[PD];
#pragma unroll
  for (int k = 0; k < PD; ++k) {
    PF[k] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, L.in_off, 0, 0);
    half_advance_in<WRAP>(L);
  }
  hprologue<TM, PD, WRAP, 0>(L, P, PF, rsrc, rdst);
  // H - TM is a multiple of PD: whole loop bodies up to the epilogue
  for (int i = 2 * TM; i < H + TM; i += PD) hbody<TM, PD, WRAP, 0>(L, P, PF, rsrc, rdst);
  // the first row beyond the shared edge, loaded PD steps ago
  hepilogue<TM, WRAP, 0>(PF[(2 * TM) % PD], L, P, rdst);
}

template <int TM, int PD>
__global__ __launch_bounds__(64) void k_board_pass_half(PassArgs a, GridGeom g) {
  const int npairs = g.nbands / 2;
  const int nitems = g.nstrips * npairs;
  const int item = xcd_item(nitems);
  if (item >= nitems) return;  // whole wave
  const int s = item % g.nstrips, pr = item / g.nstrips;
  const int us = g.strip_q + (s < g.strip_r ? 1 : 0);
  const int ds = s * g.strip_q + min(s, g.strip_r);
  const int lane = (int)threadIdx.x;
  const bool upper = lane >= 32;
  const int l = lane & 31;
  const int nl = us + 2;
  const int R = a.R, D = a.D;
  // half A: rows [a0, a0 + H) downwards; half B: rows [a0 + H, b1] upwards
  const int H = g.band_q;
  const int a0 = 2 * pr * H;
  const int b1 = a0 + 2 * H - 1;  // may pass R: wraps
  auto wrapr = [&](int r) { r %= R; return r < 0 ? r + R : r; };
  HalfLane L;
  L.R = R;
  L.D = D;
  L.upper = upper;
  L.wrap = (uint32_t)R * (uint32_t)D * 4u;
  L.in_a = wrapr(a0 - TM);
  L.in_b = wrapr(b1 + TM);
  L.out_a = wrapr(a0);
  L.out_b = wrapr(b1);
  const int p = ds - 1 + l;                     // logical dword of the lane
  const int nd = a.C >> 5;                      // dwords holding cells (C % 32 == 0)
  const int pc = ((p % nd) + nd) % nd;          // the dword its columns wrap to
  const int rin = upper ? L.in_b : L.in_a;
  const int rout = upper ? L.out_b : L.out_a;
  L.in_off = ((uint32_t)rin * (uint32_t)D + (uint32_t)pc) * 4u;
  L.in_step = upper ? (uint32_t)(-4 * D) : (uint32_t)(4 * D);
  const bool store = l >= 1 && l <= nl - 2 && l < 31 && p >= 0 && p < D;
  L.out_off = store ? ((uint32_t)rout * (uint32_t)D + (uint32_t)p) * 4u : kHalfDropped;
  L.out_step = store ? L.in_step : 0u;
  L.smask = p < nd ? 0xFFFFFFFFu : 0u;          // a padding dword stays 0
  __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.src, 0, (int)L.wrap, kBufferDword3);
  __amdgpu_buffer_rsrc_t rdst = __builtin_amdgcn_make_buffer_rsrc(a.dst, 0, (int)L.wrap,
                                                                   kBufferDword3);
  // rows the sweep touches: A from a0 - TM to a0 + H + TM + PD, B the mirror
  const bool wraps = a0 - TM < 0 || b1 + TM >= R || a0 + H + TM + PD >= R;
  if (wraps)
    run_tile_half<TM, PD, true>(L, H, rsrc, rdst);
  else
    run_tile_half<TM, PD, false>(L, H, rsrc, rdst);
}

// ---------------------------------------------------------------------------
// One generation per launch on wide aligned boards (the HBM-bound form):
// rows of D dwords with D % 4 == 0.  A wave owns a strip of 62 x 4 = 248
// dwords plus one halo lane of four dwords on each side (lane l holds the
// four consecutive dwords from 248 s - 4 + 4 l, modulo D, moved as one 128-bit
// buffer access) and a band of rows; it sweeps rows r0 - 1 .. r0 + h (mod R)
// keeping the horizontal 3-sums of the last two rows and emits row m - 1 when
// row m arrives, so each row is read once per strip (plus the halo lanes and
// the band's two halo rows) and written once.  Word-edge bits come from the
// neighbouring dword: within the lane, or from the next lane by DPP; the halo
// lanes' own results are wrong at their far edge and are not stored.  Rows
// are requested kT1Prefetch steps ahead; lanes past the board load nothing
// (their offsets fall outside the buffer and are dropped).
// ---------------------------------------------------------------------------
constexpr int kT1Lane = 4;                       // dwords per lane
constexpr int kT1Useful = (kWave - 2) * kT1Lane;  // dwords a strip writes
constexpr int kT1Prefetch = 8;                   // rows requested ahead

struct T1Args {
  const uint32_t* src;
  uint32_t* dst;
  int32_t R, D;
  int32_t nstrips, nbands, band_q, band_r;  // balanced split of the rows into nbands
};

struct T1Row {
  uint32_t x[kT1Lane];
};

__device__ __forceinline__ void t1_load(T1Row& r, const uint32_t* row, uint32_t bytes,
                                        uint32_t qoff) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)uniform_ptr((uint32_t*)row), 0, (int)bytes,
                                        kBufferDword3);
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, qoff, 0, 0);
  r.x[0] = v[0];
  r.x[1] = v[1];
  r.x[2] = v[2];
  r.x[3] = v[3];
}

__global__ __launch_bounds__(64) void k_step_t1(T1Args a) {
  const int nitems = a.nstrips * a.nbands;
  const int item = xcd_item(nitems);
  if (item >= nitems) return;  // whole wave
  const int s = item % a.nstrips, b = item / a.nstrips;
  const int hb = a.band_q + (b < a.band_r ? 1 : 0);
  const int rb = b * a.band_q + min(b, a.band_r);
  const int lane = (int)threadIdx.x;
  const int D = a.D, R = a.R;
  // logical dword of the lane (the strip's west halo lane starts 4 dwords
  // before it), and whether the lane is useful, the east halo or idle
  const int p = s * kT1Useful - kT1Lane + lane * kT1Lane;
  const int send = min(s * kT1Useful + kT1Useful, D);  // end of the strip's useful dwords
  const bool useful = lane >= 1 && lane <= kWave - 2 && p < send;
  const bool loads = lane == 0 || p < send + kT1Lane;  // useful or a halo lane
  const uint32_t bytes = (uint32_t)D * 4u;
  const uint32_t qoff = loads ? (uint32_t)(((p % D) + D) % D) * 4u : kDroppedOffset;
  const uint32_t soff = useful ? (uint32_t)p * 4u : kDroppedOffset;
  // rows rb - 1 .. rb + hb, modulo R
  int rin = ((rb - 1) % R + R) % R;
  const uint32_t* in_row = a.src + (int64_t)rin * D;
  auto advance = [&]() {
    ++rin;
    in_row += D;
    if (rin == R) {
      rin = 0;
      in_row = a.src;
    }
  };
  int rout = rb;
  uint32_t* out_row = a.dst + (int64_t)rb * D;
  T1Row PF[kT1Prefetch];
#pragma unroll
  for (int k = 0; k < kT1Prefetch; ++k) {
    t1_load(PF[k], in_row, bytes, qoff);
    advance();
  }
  uint32_t lo[2][kT1Lane], hi[2][kT1Lane], xs[kT1Lane];
  const int nsteps = hb + 2;
  auto step = [&](int i, T1Row& r) {
    uint32_t x[kT1Lane];
#pragma unroll
    for (int k = 0; k < kT1Lane; ++k) x[k] = r.x[k];
    // request the row kT1Prefetch steps ahead into this slot
    t1_load(r, in_row, bytes, qoff);
    advance();
    __builtin_amdgcn_sched_barrier(GOL_PREFETCH_FENCE_MASK);
    const uint32_t west = from_prev_lane(x[kT1Lane - 1]);
    const uint32_t east = from_next_lane(x[0]);
    uint32_t l2[kT1Lane], h2[kT1Lane];
#pragma unroll
    for (int k = 0; k < kT1Lane; ++k) {
      const uint32_t xw = k == 0 ? west : x[k - 1];
      const uint32_t xe = k == kT1Lane - 1 ? east : x[k + 1];
      const uint32_t xl = __builtin_amdgcn_alignbit(x[k], xw, 31);
      const uint32_t xr = __builtin_amdgcn_alignbit(xe, x[k], 1);
      l2[k] = xor3(xl, x[k], xr);
      h2[k] = maj3(xl, x[k], xr);
    }
    if (i >= 2) {
      uint32_t y[kT1Lane];
#pragma unroll
      for (int k = 0; k < kT1Lane; ++k)
        y[k] = life_rule(lo[0][k], lo[1][k], l2[k], hi[0][k], hi[1][k], h2[k], xs[k]);
      const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
          (void*)uniform_ptr(out_row), 0, (int)bytes, kBufferDword3);
      __builtin_amdgcn_raw_buffer_store_b128({y[0], y[1], y[2], y[3]}, rd, soff, 0, 0);
      ++rout;
      out_row += D;
      if (rout == R) {
        rout = 0;
        out_row = a.dst;
      }
    }
#pragma unroll
    for (int k = 0; k < kT1Lane; ++k) {
      lo[0][k] = lo[1][k];
      hi[0][k] = hi[1][k];
      lo[1][k] = l2[k];
      hi[1][k] = h2[k];
      xs[k] = x[k];
    }
  };
  int i = 0;
  for (; i + kT1Prefetch <= nsteps; i += kT1Prefetch) {
#pragma unroll
    for (int k = 0; k < kT1Prefetch; ++k) step(i + k, PF[k]);
  }
#pragma unroll
  for (int k = 0; k < kT1Prefetch; ++k)
    if (i + k < nsteps) step(i + k, PF[k]);
}

// ---------------------------------------------------------------------------
// Many boards: waves from a table, each made of one or more segments.
// ---------------------------------------------------------------------------
// A launch runs the waves items[0, nearly) and items[late_begin,
// late_begin + nlate) of level `level`.
template <int TM, bool MASKED>
__global__ __launch_bounds__(64) void k_batch_pass(const BoardDesc* __restrict__ boards,
                                                   const Segment* __restrict__ segs,
                                                   const WaveItem* __restrict__ items, int nearly,
                                                   int nlate, int late_begin, int level) {
  const int nitems = nearly + nlate;
  const int idx = xcd_item(nitems);
  if (idx >= nitems) return;  // whole wave
  const int it = idx < nearly ? idx : late_begin + (idx - nearly);
  const WaveItem w = items[it];
  const int lane = (int)threadIdx.x;
  int mine = -1;
  for (int k = 0; k < w.nseg; ++k) {
    const Segment sg = segs[w.seg_begin + k];
    if (lane >= sg.lane0 && lane < sg.lane0 + sg.nlanes) mine = w.seg_begin + k;
  }
  Lane L;
  if (mine >= 0) {
    const Segment sg = segs[mine];
    const BoardDesc bd = boards[sg.board];
    const int jl = level - bd.start;
    const bool active = jl >= 0 && jl < bd.K;
    const int j = jl < 0 ? 0 : (jl < bd.K ? jl : bd.K - 1);
    const uint32_t* src = (j == 0) ? bd.src0 : bd.w[(j - 1 + bd.par) & 1];
    uint32_t* dst = bd.w[(j + bd.par) & 1];
    const int Tl = (j == bd.jshort) ? bd.Tshort : TM;
    lane_setup(L, src, dst, bd.R, bd.C, bd.D, sg.p0 + (lane - sg.lane0), lane - sg.lane0,
               sg.nlanes, sg.r0, sg.h, TM, Tl, active);
  } else {
    const Segment sg = segs[w.seg_begin];
    const BoardDesc bd = boards[sg.board];
    lane_setup(L, bd.src0, bd.w[0], bd.R, bd.C, bd.D, 0, 0, 1, 0, 1, TM, TM, false);
  }
  if (w.flags & kItemAligned)
    run_tile<TM, MASKED, kGatherAligned, GOL_BATCH_PREFETCH, false>(L, w.h);
  else
    run_tile<TM, MASKED, kGatherTorus, GOL_BATCH_PREFETCH, false>(L, w.h);
}

// ---------------------------------------------------------------------------
// Many boards in one persistent launch: each wave takes items from a queue
// (QueueItem, in pass order) until it is empty.  Before an item of pass j it
// waits for the board's counter to reach j x (items per pass): every tile of
// pass j - 1 has stored (the rows this pass reads) and has finished reading
// the buffer this pass overwrites.  Publication goes through device-scope
// release / acquire fences around the counter; a wait gives up after a
// bounded number of sleeps (setting the error word, which every wave checks,
// so the launch always drains).
// ---------------------------------------------------------------------------
constexpr uint32_t kQueueSpinLimit = 1u << 22;  // sleeps of ~128 clocks each before giving up

template <int TM>
__global__ __launch_bounds__(64) void k_batch_queue(const BoardDesc* __restrict__ boards,
                                                    const Segment* __restrict__ segs,
                                                    const QueueItem* __restrict__ items,
                                                    const int32_t* __restrict__ per_pass,
                                                    int nitems, uint32_t* ctl) {
  const int lane = (int)threadIdx.x;
  uint32_t* const next = ctl;
  uint32_t* const error = ctl + 1;
  uint32_t* const done = ctl + kQueueCtlHeader;
  while (true) {
    uint32_t it = 0;
    if (lane == 0) it = __hip_atomic_fetch_add(next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    it = (uint32_t)__builtin_amdgcn_readfirstlane((int)it);
    if ((int)it >= nitems) return;
    if (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
    const QueueItem q = items[it];
    const uint32_t need = (uint32_t)q.pass * (uint32_t)per_pass[q.board];
    if (need > 0u) {
      uint32_t spins = 0;
      while (__hip_atomic_load(done + q.board, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins >= kQueueSpinLimit ||
            __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          if (lane == 0)
            __hip_atomic_store(error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    int mine = -1;
    for (int k = 0; k < q.nseg; ++k) {
      const Segment sg = segs[q.seg_begin + k];
      if (lane >= sg.lane0 && lane < sg.lane0 + sg.nlanes) mine = q.seg_begin + k;
    }
    const BoardDesc bd = boards[q.board];
    const int j = q.pass;
    const uint32_t* src = (j == 0) ? bd.src0 : bd.w[(j - 1 + bd.par) & 1];
    uint32_t* dst = bd.w[(j + bd.par) & 1];
    const int Tl = (j == bd.jshort) ? bd.Tshort : TM;
    Lane L;
    if (mine >= 0) {
      const Segment sg = segs[mine];
      lane_setup(L, src, dst, bd.R, bd.C, bd.D, sg.p0 + (lane - sg.lane0), lane - sg.lane0,
                 sg.nlanes, sg.r0, sg.h, TM, Tl, true);
    } else {
      lane_setup(L, src, dst, bd.R, bd.C, bd.D, 0, 0, 1, 0, 1, TM, TM, false);
    }
    const bool shortp = Tl < TM;  // uniform: the item's one board and pass
    if (q.flags & kItemAligned) {
      if (shortp)
        run_tile<TM, true, kGatherAligned, GOL_BATCH_PREFETCH, false>(L, q.h);
      else
        run_tile<TM, false, kGatherAligned, GOL_BATCH_PREFETCH, false>(L, q.h);
    } else {
      if (shortp)
        run_tile<TM, true, kGatherTorus, GOL_BATCH_PREFETCH, false>(L, q.h);
      else
        run_tile<TM, false, kGatherTorus, GOL_BATCH_PREFETCH, false>(L, q.h);
    }
    // the stores of this item are complete and visible device-wide before
    // the counter says so
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_fetch_add(done + q.board, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Layout conversion (byte boards of the host API) and normalising copies.
// ---------------------------------------------------------------------------

// uint8 cells (nonzero = alive) -> packed words.  One wave per output word:
// lane l tests cell 64 w + l, the wave's ballot is the word.
__global__ __launch_bounds__(256) void k_pack(const uint8_t* __restrict__ in, int64_t R, int64_t C,
                                              int64_t W, uint64_t* __restrict__ out) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t wi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wi < R * W;
       wi += nwaves) {
    const int64_t r = wi / W, c = (wi - r * W) * 64 + lane;
    const bool alive = c < C && in[r * C + c] != 0;
    const uint64_t m = __ballot(alive);
    if (lane == 0) out[wi] = m;
  }
}

// packed words -> uint8 cells 0/1, one thread per cell.
__global__ __launch_bounds__(256) void k_unpack(const uint64_t* __restrict__ in, int64_t R,
                                                int64_t C, int64_t W, uint8_t* __restrict__ out) {
  const int64_t n = R * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / C, c = i - r * C;
    out[i] = (uint8_t)((in[r * W + (c >> 6)] >> (c & 63)) & 1u);
  }
}

// Copy words with the padding bits (columns >= C) cleared.
__global__ __launch_bounds__(256) void k_copy_clear_padding(const uint64_t* __restrict__ in,
                                                            int64_t R, int64_t C, int64_t W,
                                                            uint64_t* __restrict__ out) {
  const int64_t n = R * W;
  const int64_t last = C - (W - 1) * 64;  // valid bits of the last word, 1..64
  const uint64_t lastmask = last >= 64 ? ~0ull : ((1ull << last) - 1ull);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = i % W;
    out[i] = in[i] & (w == W - 1 ? lastmask : ~0ull);
  }
}

// Fill 32-bit words (device counters, flags); used instead of hipMemsetAsync
// so the launch sequences can be captured into graphs.
// Live cells of a packed board: n = R * W words, the last word of each row
// masked by lastmask (padding bits are not cells).  Adds to *out.  Each
// thread keeps four loads in flight; a block sums its threads in LDS and adds
// once, so the single counter sees one atomic per block (the launcher keeps
// the grid to a few blocks per CU).
constexpr int kPopThreads = 256;
constexpr int kPopUnroll = 4;
__global__ __launch_bounds__(kPopThreads) void k_population(const uint64_t* __restrict__ b,
                                                            int64_t n, int64_t W,
                                                            uint64_t lastmask,
                                                            unsigned long long* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kPopThreads;
  const int64_t cs = stride % W;
  int64_t i = (int64_t)blockIdx.x * kPopThreads + threadIdx.x;
  int64_t c = i % W;  // column word of i, advanced with i
  auto next = [&](int64_t col) { col += cs; return col >= W ? col - W : col; };
  uint64_t cnt = 0u;
  for (; i + (kPopUnroll - 1) * stride < n; i += kPopUnroll * stride) {
    uint64_t v[kPopUnroll];
#pragma unroll
    for (int u = 0; u < kPopUnroll; ++u) v[u] = b[i + u * stride];
#pragma unroll
    for (int u = 0; u < kPopUnroll; ++u) {
      if (c == W - 1) v[u] &= lastmask;
      cnt += (uint64_t)__builtin_popcountll(v[u]);
      c = next(c);
    }
  }
  for (; i < n; i += stride) {
    uint64_t v = b[i];
    if (c == W - 1) v &= lastmask;
    cnt += (uint64_t)__builtin_popcountll(v);
    c = next(c);
  }
  // wave sums, then one atomic per block
  uint32_t lo = (uint32_t)cnt;  // at most 64 words x 64 bits x iterations: far below 2^32
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lo += (uint32_t)__shfl_xor((int)lo, o, 64);
  __shared__ uint32_t part[kPopThreads / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = lo;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < kPopThreads / kWave; ++k) s += part[k];
    atomicAdd(out, s);
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n,
                                                  uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Small boards: the whole board resident in one workgroup's LDS for a run.
//
// The packed board is read once into LDS (rows of nd = ceil(C / 32) dwords,
// padding bits cleared), then every generation is computed from one LDS copy
// into the other, with a workgroup barrier between generations, and the last
// one is written out once: no HBM traffic and no launch per pass, which is
// what bounds the tile passes on boards this small.  Work item (column j,
// row segment s) sweeps its rows downwards keeping the horizontal sums of the
// rows above, at and below the current one in registers; the word-edge bits
// come from the neighbouring dwords in LDS, wrapping at the row end (the
// column after C - 1 is column 0), and rows wrap modulo R.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kResidentThreads) void k_board_lds(const uint32_t* src, uint32_t* dst,
                                                                int32_t R, int32_t C, int32_t D,
                                                                int32_t G) {
  extern __shared__ uint32_t lds_board[];
  const int nd = (C + 31) >> 5;  // <= the workgroup's thread count
  const int nthreads = (int)blockDim.x;
  const int nsegs = nthreads / nd;
  const int rs = (R + nsegs - 1) / nsegs;
  const int nbuf = R * nd + (R - 1) / rs + 1;  // one generation with its segment pads
  auto base = [&](int r) { return r * nd + r / rs; };
  uint32_t* cur = lds_board;
  uint32_t* nxt = lds_board + nbuf;
  const int tid = (int)threadIdx.x;
  const uint32_t last_mask = (C & 31) ? (1u << (C & 31)) - 1u : 0xFFFFFFFFu;
  for (int i = tid; i < R * nd; i += nthreads) {
    const int r = i / nd, j = i - r * nd;
    const uint32_t v = ((GlobalIn)src)[(int64_t)r * D + j];
    cur[base(r) + j] = j == nd - 1 ? v & last_mask : v;
  }
  // this thread's work item: dword column j of rows r0 .. r1 - 1 (segment s)
  const int j = tid % nd, s = tid / nd;
  const int r0 = s * rs, r1 = min(R, r0 + rs);
  const bool active = s < nsegs && r0 < r1;
  const int n = min(32, C - 32 * j);  // cells in dword j
  const uint32_t mask = n == 32 ? 0xFFFFFFFFu : (1u << n) - 1u;
  const int cl = (32 * j - 1 + C) % C;  // the cell west of the dword's first
  const int cr = (32 * j + n) % C;      // the cell east of its last
  const int jl = cl >> 5, bl = cl & 31, jr = cr >> 5, br = cr & 31;
  const int above = base(r0 == 0 ? R - 1 : r0 - 1);  // rows of other segments
  const int below = base(r1 == R ? 0 : r1);
  const int own = s;                                 // pads before row r0's segment
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    if (active) {
      uint32_t lo[3], hi[3], x[3];
      auto hsum = [&](int b, int k) {
        const uint32_t* row = cur + b;
        const uint32_t v = row[j];
        const uint32_t w = (row[jl] >> bl) & 1u, e = (row[jr] >> br) & 1u;
        const uint32_t xl = ((v << 1) | w) & mask;      // west neighbours
        const uint32_t xr = (v >> 1) | (e << (n - 1));  // east neighbours
        lo[k] = xor3(xl, v, xr);
        hi[k] = maj3(xl, v, xr);
        x[k] = v;
      };
      hsum(above, 0);
      hsum(r0 * nd + own, 1);
      for (int r = r0; r < r1; ++r) {
        hsum(r + 1 < r1 ? (r + 1) * nd + own : below, 2);
        nxt[r * nd + own + j] =
            life_rule(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], x[1]) & mask;
        lo[0] = lo[1]; hi[0] = hi[1];
        lo[1] = lo[2]; hi[1] = hi[2]; x[1] = x[2];
      }
    }
    __syncthreads();
    uint32_t* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (int i = tid; i < R * D; i += nthreads) {
    const int r = i / D, jj = i - r * D;
    ((GlobalOut)dst)[(int64_t)r * D + jj] = jj < nd ? cur[base(r) + jj] : 0u;  // padding: 0
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the C ABI in gol_capi.cpp).
// ---------------------------------------------------------------------------
template <int TM, int PD>
static hipError_t launch_board_pass_t(const PassArgs& a, const GridGeom& g, bool bounded,
                                      hipStream_t st) {
  const int nitems = g.nstrips * g.nbands;
  const int grid = ((nitems + 7) / 8) * 8;
  if (a.top && (a.C & 31) == 0)
    hipLaunchKernelGGL((k_board_pass<TM, PD, kGatherAligned | kHaloRows>), dim3(grid), dim3(64), 0,
                       st, a, g);
  else if (a.top)
    hipLaunchKernelGGL((k_board_pass<TM, PD, kGatherTorus | kHaloRows>), dim3(grid), dim3(64), 0,
                       st, a, g);
  else if (bounded)
    hipLaunchKernelGGL((k_board_pass<TM, PD, kGatherBounded>), dim3(grid), dim3(64), 0, st, a, g);
  else if ((a.C & 31) == 0)
    hipLaunchKernelGGL((k_board_pass<TM, PD, kGatherAligned>), dim3(grid), dim3(64), 0, st, a, g);
  else
    hipLaunchKernelGGL((k_board_pass<TM, PD, kGatherTorus>), dim3(grid), dim3(64), 0, st, a, g);
  return hipGetLastError();
}

// One band per wave; (T, pd) must satisfy pass_config_compiled(kLayoutBand, ...).
// bounded: cells beyond the board's edges are dead (no torus).  top / bot
// non-null: the R rows are a strip with T halo rows in each (pass of T
// generations, the result for the strip's rows only).
hipError_t launch_board_pass(int T, const uint32_t* src, uint32_t* dst, int32_t R, int32_t C,
                             int32_t D, const GridGeom& g, int pd, bool bounded, hipStream_t st,
                             const uint32_t* top, const uint32_t* bot) {
  PassArgs a{src, dst, R, C, D, top, bot};
#define GOL_LAUNCH_BAND(TV, PDV) \
  if (T == TV && pd == PDV) return launch_board_pass_t<TV, PDV>(a, g, bounded, st);
  GOL_LAUNCH_BAND(1, 3)
  GOL_LAUNCH_BAND(1, 6)
  GOL_LAUNCH_BAND(2, 3)
  GOL_LAUNCH_BAND(2, 6)
  GOL_LAUNCH_BAND(4, 3)
  GOL_LAUNCH_BAND(4, 6)
  GOL_LAUNCH_BAND(8, 6)
  GOL_LAUNCH_BAND(8, 9)
  GOL_LAUNCH_BAND(12, 6)
  GOL_LAUNCH_BAND(12, 9)
  GOL_LAUNCH_BAND(16, 9)
  GOL_LAUNCH_BAND(16, 12)
#undef GOL_LAUNCH_BAND
  return hipErrorInvalidValue;
}

// One generation on a board with cols % 128 == 0 (D % 4 == 0): 248-dword
// strips x bands of about band_rows rows.
hipError_t launch_step_t1(const uint32_t* src, uint32_t* dst, int32_t R, int32_t D, int band_rows,
                          hipStream_t st) {
  T1Args a;
  a.src = src;
  a.dst = dst;
  a.R = R;
  a.D = D;
  a.nstrips = (D + kT1Useful - 1) / kT1Useful;
  const int64_t nb = ((int64_t)R + band_rows - 1) / band_rows;
  a.nbands = (int32_t)(nb < 1 ? 1 : nb);
  a.band_q = R / a.nbands;
  a.band_r = R % a.nbands;
  const int64_t nitems = (int64_t)a.nstrips * a.nbands;
  const int64_t grid = ((nitems + 7) / 8) * 8;
  hipLaunchKernelGGL(k_step_t1, dim3((unsigned)grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

// Whole board resident in LDS for G generations; resident_fits(R, C) must
// hold.  src may equal dst (the board is read in full before any write).
hipError_t launch_board_lds(const uint32_t* src, uint32_t* dst, int32_t R, int32_t C, int32_t D,
                            int32_t G, hipStream_t st) {
  const ResidentGeom rg = resident_geom(R, C);
  const size_t lds = (size_t)2 * (size_t)rg.words * 4u;
  hipLaunchKernelGGL(k_board_lds, dim3(1), dim3((unsigned)rg.threads), lds, st, src, dst, R, C, D,
                     G);
  return hipGetLastError();
}

// Two bands per wave; (T, pd) must satisfy pass_config_compiled(kLayoutPaired,
// ...), g must come from paired_geometry with the same T and pd, C % 32 == 0
// and the board must be smaller than 2 GiB.
hipError_t launch_board_pass_half(int T, const uint32_t* src, uint32_t* dst, int32_t R, int32_t C,
                                  int32_t D, const GridGeom& g, int pd, hipStream_t st) {
  PassArgs a{src, dst, R, C, D, nullptr, nullptr};
  const int nitems = g.nstrips * (g.nbands / 2);
  const int grid = ((nitems + 7) / 8) * 8;
#define GOL_LAUNCH_HALF(TV, PDV)                                                          \
  if (T == TV && pd == PDV) {                                                             \
    hipLaunchKernelGGL((k_board_pass_half<TV, PDV>), dim3(grid), dim3(64), 0, st, a, g);  \
    return hipGetLastError();                                                             \
  }
  GOL_LAUNCH_HALF(8, 9)
  GOL_LAUNCH_HALF(8, 12)
  GOL_LAUNCH_HALF(12, 9)
  GOL_LAUNCH_HALF(12, 12)
  GOL_LAUNCH_HALF(16, 9)
  GOL_LAUNCH_HALF(16, 12)
#undef GOL_LAUNCH_HALF
  return hipErrorInvalidValue;
}

template <int TM, bool MASKED>
static hipError_t launch_batch_pass_t(const BoardDesc* boards, const Segment* segs,
                                      const WaveItem* items, int nearly, int nlate,
                                      int late_begin, int level, hipStream_t st) {
  const int grid = ((nearly + nlate + 7) / 8) * 8;
  hipLaunchKernelGGL((k_batch_pass<TM, MASKED>), dim3(grid), dim3(64), 0, st, boards, segs, items,
                     nearly, nlate, late_begin, level);
  return hipGetLastError();
}

// Level `level` of a batch schedule: the waves items[0, nearly) and
// items[late_begin, late_begin + nlate); masked when some pass of the level
// is shorter than T.
hipError_t launch_batch_pass(int T, bool masked, const BoardDesc* boards, const Segment* segs,
                             const WaveItem* items, int nearly, int nlate, int late_begin,
                             int level, hipStream_t st) {
  if (nearly + nlate <= 0) return hipSuccess;
#define GOL_LAUNCH_BATCH(TV)                                                                \
  case TV:                                                                                  \
    return masked ? launch_batch_pass_t<TV, true>(boards, segs, items, nearly, nlate,       \
                                                  late_begin, level, st)                    \
                  : launch_batch_pass_t<TV, false>(boards, segs, items, nearly, nlate,      \
                                                   late_begin, level, st);
  switch (T) {
    GOL_LAUNCH_BATCH(1)
    GOL_LAUNCH_BATCH(2)
    GOL_LAUNCH_BATCH(4)
    GOL_LAUNCH_BATCH(8)
    GOL_LAUNCH_BATCH(12)
    GOL_LAUNCH_BATCH(16)
    default: return hipErrorInvalidValue;
  }
#undef GOL_LAUNCH_BATCH
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

// Resident waves of the queue kernel on the current device (its occupancy
// per compute unit times the compute units), or 0 if unknown.
int batch_queue_waves(int T) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e = hipErrorInvalidValue;
  if (T == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_queue<8>, 64, 0);
  if (T == 12) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_queue<12>, 64, 0);
  if (T == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_queue<16>, 64, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per * cus;
}

// The persistent queue form: `waves` waves (the device's resident capacity
// for the kernel) take the nitems items; ctl holds kQueueCtlHeader + boards
// words, zeroed here first.
hipError_t launch_batch_queue(int T, const BoardDesc* boards, const Segment* segs,
                              const QueueItem* items, const int32_t* per_pass, int nitems,
                              uint32_t* ctl, int nboards, int waves, hipStream_t st) {
  hipError_t e = launch_fill_u32(ctl, (int64_t)kQueueCtlHeader + nboards, 0u, st);
  if (e != hipSuccess || nitems <= 0) return e;
  const int grid = waves < 1 ? 1 : waves;
#define GOL_LAUNCH_QUEUE(TV)                                                                  \
  case TV:                                                                                    \
    hipLaunchKernelGGL(k_batch_queue<TV>, dim3(grid), dim3(64), 0, st, boards, segs, items,   \
                       per_pass, nitems, ctl);                                                \
    return hipGetLastError();
  switch (T) {
    GOL_LAUNCH_QUEUE(8)
    GOL_LAUNCH_QUEUE(12)
    GOL_LAUNCH_QUEUE(16)
    default: return hipErrorInvalidValue;
  }
#undef GOL_LAUNCH_QUEUE
}

static int grid_for(int64_t n, int per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

hipError_t launch_pack(const uint8_t* in, int64_t R, int64_t C, uint64_t* out, hipStream_t st) {
  const int64_t W = (C + 63) / 64;
  hipLaunchKernelGGL(k_pack, dim3(grid_for(R * W, 4)), dim3(256), 0, st, in, R, C, W, out);
  return hipGetLastError();
}

hipError_t launch_unpack(const uint64_t* in, int64_t R, int64_t C, uint8_t* out, hipStream_t st) {
  const int64_t W = (C + 63) / 64;
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(R * C, 256)), dim3(256), 0, st, in, R, C, W, out);
  return hipGetLastError();
}

hipError_t launch_copy_clear_padding(const uint64_t* in, int64_t R, int64_t C, uint64_t* out,
                                     hipStream_t st) {
  const int64_t W = (C + 63) / 64;
  hipLaunchKernelGGL(k_copy_clear_padding, dim3(grid_for(R * W, 256)), dim3(256), 0, st, in, R, C,
                     W, out);
  return hipGetLastError();
}

// Adds the live cells of a packed R x C board to *out (not cleared here).
hipError_t launch_population(const uint64_t* b, int64_t R, int64_t C, unsigned long long* out,
                             hipStream_t st) {
  const int64_t W = (C + 63) / 64;
  const uint64_t lastmask = (C % 64) ? ((uint64_t)1 << (C % 64)) - 1 : ~(uint64_t)0;
  const int64_t n = R * W;
  int64_t blocks = (n + (int64_t)kPopThreads * kPopUnroll - 1) / ((int64_t)kPopThreads * kPopUnroll);
  // four blocks per CU at most: on a 512 MiB board 1024 blocks read at 6.0 TB/s,
  // 2048 at 5.2 and 8192 at 3.9 (more atomics on the one counter, longer tail)
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_population, dim3((int)blocks), dim3(kPopThreads), 0, st, b, n, W, lastmask,
                     out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Fixed scratch for callers that cannot allocate (gol_step_packed_noalloc):
// the ping-pong board of a run lives in this array instead of memory from
// the allocator.  In host code `scratch` names a host-side stand-in, not the
// device array, so host code never passes it to a kernel or a copy: it takes
// the device address from fixed_scratch(), looked up once per device with
// hipGetSymbolAddress (each GPU holds its own copy at its own address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint64_t scratch[kFixedScratchBytes / sizeof(uint64_t)];

// Device address of the current device's `scratch` (GOL_OK-style 0, or the
// HIP error of the lookup).
hipError_t fixed_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> ptr;  // per device ordinal, null until looked up
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)ptr.size() <= dev) ptr.resize((size_t)dev + 1, nullptr);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

}  // namespace gol

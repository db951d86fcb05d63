/*
 * gol_debug.h -- host-only introspection of libgol's batch scheduler.
 *
 * gol_debug_plan_tables builds the schedule that gol_batch_run / gol_plan_create
 * would use for boards of the given sizes and generation counts, on the host
 * only (no device memory, no HIP call), and copies out its tables so tests
 * can check them.  Layouts (little endian):
 *   segment (16 bytes): int32 board, int32 p0 (logical dword of the first,
 *     halo, lane), int32 r0 (first output row), uint16 h (output rows),
 *     uint8 lane0, uint8 nlanes;
 *   wave item (16 bytes): int32 seg_begin, int16 nseg, uint16 h (largest
 *     band), int32 maxK (largest pass count of its boards), int32 flags
 *     (bit 0: every lane's board has cols % 32 == 0);
 *   levels[2 L], levels[2 L + 1]: level L launches the waves
 *     [0, levels[2 L]) and [*late_begin, *late_begin + levels[2 L + 1]) —
 *     a prefix of the early group (waves running levels 0 .. maxK - 1) and
 *     of the late group (levels Kmax - maxK .. Kmax - 1, Kmax = the number
 *     of levels);
 *   starts[b]: the level of board b's first pass (n entries; boards with no
 *     generations: 0).
 * rows / cols / gens: n entries each.  t_block: generations per pass (0 =
 * default).  band_rows: rows per tile band (0 = default).  Up to cap_* entries
 * (cap_levels pairs) are written to each non-NULL output; *nsegs, *nitems,
 * *nlevels receive the full counts.  Returns GOL_OK, GOL_EINVAL (bad sizes or
 * t_block) or GOL_ENOMEM.  Thread-safe; owns nothing after it returns.
 */
#ifndef GOL_DEBUG_H
#define GOL_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int gol_debug_plan_tables(const int64_t* rows, const int64_t* cols, const int64_t* gens, int64_t n,
                          int t_block, int band_rows, void* segs, int64_t cap_segs, void* items,
                          int64_t cap_items, int32_t* levels, int64_t cap_levels,
                          int32_t* starts, int32_t* late_begin, int64_t* nsegs, int64_t* nitems,
                          int64_t* nlevels);

/*
 * The same tables for a served chunk: each board tiled on its own
 * (consecutive bands of one narrow strip share a wave; no wave holds two
 * boards) and the boards' waves assembled in pass-count order, as a server's
 * chunk is built.  band_rows 0 = the band height a server whose busy
 * height is 96 picks for these boards on a 1024-SIMD device (96, halved
 * while the tiles give fewer than two waves per SIMD, not below 32 rows or
 * t_block); *band_used (may be NULL) receives the height used.
 */
int gol_debug_chunk_plan_tables(const int64_t* rows, const int64_t* cols, const int64_t* gens,
                                int64_t n, int t_block, int band_rows, void* segs,
                                int64_t cap_segs, void* items, int64_t cap_items,
                                int32_t* levels, int64_t cap_levels, int32_t* starts,
                                int32_t* late_begin, int64_t* nsegs, int64_t* nitems,
                                int64_t* nlevels, int32_t* band_used);

/*
 * For a plan of the queue form (GOL_LAYOUT_QUEUE): waits for its queued runs
 * and sets *gave_up to 1 if a wave of the last run gave up waiting for a
 * board's previous pass (its results are then not to be used), else 0; 0 for
 * other plans.
 */
typedef struct gol_plan gol_plan;
int gol_debug_plan_queue_gave_up(gol_plan* plan, int32_t* gave_up);

/*
 * A server whose "device" is host memory, for testing the serving scheduler
 * (admission by budget, chunking, the buffer that holds each board's state,
 * retirement, cancellation, failure handling) without a GPU.  Every queued
 * operation completes at once.  It replays each chunk's schedule level by
 * level and tile by tile as the device would; its stand-in for a pass of t
 * generations adds t (mod 2^32) to every 32-bit word of the tile, so a board
 * advanced by g generations has g added to each of its 32-bit words; it
 * computes nothing of the Life rule.  A pass shorter than t_block in a level
 * launched without the short-pass mask fails the chunk (GOL_EDEVICE).  fail_at_chunk > 0 makes the fail_at_chunk-th chunk report
 * GOL_EDEVICE (the server then fails every unfinished request).  Use the
 * gol_serve_* calls on the result; cfg->device is ignored.
 */
typedef struct gol_server gol_server;
typedef struct gol_serve_config gol_serve_config;
int gol_debug_serve_create_host(const gol_serve_config* cfg, int64_t fail_at_chunk,
                                gol_server** out);
/* Largest number of board bytes the host executor held at once (-1 if srv is
 * not a host-executor server). */
int64_t gol_debug_serve_host_peak_bytes(const gol_server* srv);

/*
 * VALU issue-rate probe: *lane_ops_per_second receives the lane-operation
 * rate of one instruction kind on the current device -- 32768 waves, each
 * thread running eight independent chains of 2048 applications, timed with
 * HIP events over one launch after a warm-up launch.  kind: 0 v_xor_b32,
 * 1 v_bitop3_b32 (three VGPR sources), 2 v_alignbit_b32, 3 v_mov_b32 with
 * DPP, 4 v_add_u32 -- the instruction kinds of the tile pass, which price
 * its ALU roofline.  Synchronous on stream; GOL_EINVAL for another kind or
 * a null pointer.
 */
int gol_debug_valu_rate(int kind, void* stream, double* lane_ops_per_second);

#ifdef __cplusplus
}
#endif

#endif /* GOL_DEBUG_H */

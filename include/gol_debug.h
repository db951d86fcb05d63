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
 *     band), int32 maxK (levels the wave takes part in), int32 flags
 *     (bit 0: every lane's board has cols % 32 == 0);
 *   level_items[L]: waves launched at level L (a prefix of the items).
 * rows / cols / gens: n entries each.  t_block: generations per pass (0 =
 * default).  band_rows: rows per tile band (0 = default).  Up to cap_* entries
 * are written to each non-NULL output; *nsegs, *nitems, *nlevels receive the
 * full counts.  Returns GOL_OK, GOL_EINVAL (bad sizes or t_block) or
 * GOL_ENOMEM.  Thread-safe; owns nothing after it returns.
 */
#ifndef GOL_DEBUG_H
#define GOL_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int gol_debug_plan_tables(const int64_t* rows, const int64_t* cols, const int64_t* gens, int64_t n,
                          int t_block, int band_rows, void* segs, int64_t cap_segs, void* items,
                          int64_t cap_items, int32_t* level_items, int64_t cap_levels,
                          int64_t* nsegs, int64_t* nitems, int64_t* nlevels);

#ifdef __cplusplus
}
#endif

#endif /* GOL_DEBUG_H */

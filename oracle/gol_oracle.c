/*
 * ORACLE -- test infrastructure only.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library; the product path
 * (the HIP library and its Python binding) never links, loads or calls it.
 *
 * Plain, slow, obviously correct Conway's Life (B3/S23) on an R x C torus,
 * one byte per cell, written from the paper:
 *   - every cell has eight neighbours: the cells horizontally, vertically or
 *     diagonally adjacent to it (Section 1, Introduction);
 *   - at each time step every cell changes at once (Section 1): the next
 *     generation is computed from the current one into a second array, then
 *     the arrays swap;
 *   - the four transitions of Section 1 (enumerated list): a live cell with
 *     fewer than two live neighbours dies; with two or three it lives on; with
 *     more than three it dies; a dead cell with exactly three becomes live;
 *   - the grid is a torus: the left and right edges are adjacent and so are
 *     the top and bottom edges, so a boundary cell takes its neighbours from
 *     the opposite edge (Section 2.2, two-dimensional decomposition);
 *   - the cell states live in an array, one element per cell (Section 2.1).
 * Neighbour coordinates are taken modulo R and C; on tori with R < 3 or C < 3
 * an offset that lands on an already-counted cell, or on the cell itself, is
 * counted again (one count per offset).
 *
 * oracle_life_omp splits the rows of each generation among OpenMP threads:
 * the paper's one-dimensional row decomposition (Section 2.1, Figure 1), used
 * here only to time the oracle on all host cores.  Each thread writes only its
 * own rows of the next array, so the result is the same as the serial loop.
 * oracle_life_decomp times the paper's three domain decompositions against
 * each other: rows (Figure 1), columns (Figure 2), or an m x n grid of equal
 * sub-regions (Section 2.2, Figure 3), one region per thread; every cell is
 * still computed by the same plain rule from the current array.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Next state of one cell from its current state and live-neighbour count,
 * one branch per enumerated transition of Section 1. */
static inline uint8_t next_state(uint8_t alive, int n) {
  if (alive) {
    if (n < 2) return 0;           /* under-population */
    if (n == 2 || n == 3) return 1;/* lives on */
    return 0;                      /* overcrowding */
  }
  return n == 3 ? 1 : 0;           /* reproduction */
}

/* One generation of the cells in rows [r_begin, r_end) and columns
 * [c_begin, c_end) of cur into nxt.  The wrapped row and column indices of the
 * eight neighbours are written out explicitly. */
static void step_block(const uint8_t* cur, uint8_t* nxt, int64_t R, int64_t C,
                       int64_t r_begin, int64_t r_end, int64_t c_begin, int64_t c_end) {
  for (int64_t r = r_begin; r < r_end; ++r) {
    const int64_t up = (r - 1 + R) % R, down = (r + 1) % R;
    const uint8_t* above = cur + up * C;
    const uint8_t* here = cur + r * C;
    const uint8_t* below = cur + down * C;
    for (int64_t c = c_begin; c < c_end; ++c) {
      const int64_t left = (c - 1 + C) % C, right = (c + 1) % C;
      const int n = (above[left] != 0) + (above[c] != 0) + (above[right] != 0) +
                    (here[left] != 0)                    + (here[right] != 0) +
                    (below[left] != 0) + (below[c] != 0) + (below[right] != 0);
      nxt[r * C + c] = next_state(here[c] != 0, n);
    }
  }
}

static void step_rows(const uint8_t* cur, uint8_t* nxt, int64_t R, int64_t C,
                      int64_t r_begin, int64_t r_end) {
  step_block(cur, nxt, R, C, r_begin, r_end, 0, C);
}

/* Region of thread t of nt under a decomposition: 0 = rows, 1 = columns,
 * 2 = an m x n grid (m block rows, n block columns, m n = nt, m the largest
 * divisor of nt not above its square root; thread t takes block row t / n and
 * block column t % n).  Regions are as equal as the sizes allow. */
static void region(int mode, int64_t R, int64_t C, int64_t t, int64_t nt, int64_t* r0,
                   int64_t* r1, int64_t* c0, int64_t* c1) {
  int64_t m = 1, n = 1, i = 0, j = 0;
  if (mode == 0) {
    m = nt; i = t;
  } else if (mode == 1) {
    n = nt; j = t;
  } else {
    for (int64_t d = 1; d * d <= nt; ++d)
      if (nt % d == 0) m = d;
    n = nt / m;
    i = t / n;
    j = t % n;
  }
  *r0 = R * i / m; *r1 = R * (i + 1) / m;
  *c0 = C * j / n; *c1 = C * (j + 1) / n;
}

/* Shared driver: returns 0 ok, -1 bad arguments, -2 out of memory.
 * Input cells are alive iff nonzero; output cells are 0 or 1.  G == 0 copies
 * the input normalised to 0/1.  out may equal in. */
static int life_run(const uint8_t* in, int64_t R, int64_t C, int64_t G,
                    uint8_t* out, int threads) {
  if (!in || !out || R <= 0 || C <= 0 || G < 0) return -1;
  if (R > INT64_MAX / C) return -1;
  const int64_t N = R * C;
  uint8_t* a = (uint8_t*)malloc((size_t)N);
  uint8_t* b = (uint8_t*)malloc((size_t)N);
  if (!a || !b) { free(a); free(b); return -2; }
  for (int64_t i = 0; i < N; ++i) a[i] = in[i] ? 1 : 0;
  for (int64_t g = 0; g < G; ++g) {
    if (threads > 1) {
#ifdef _OPENMP
#pragma omp parallel num_threads(threads)
      {
        const int64_t nt = omp_get_num_threads();
        const int64_t t = omp_get_thread_num();
        const int64_t r0 = R * t / nt, r1 = R * (t + 1) / nt;
        step_rows(a, b, R, C, r0, r1);
      }
#else
      step_rows(a, b, R, C, 0, R);
#endif
    } else {
      step_rows(a, b, R, C, 0, R);
    }
    uint8_t* t = a; a = b; b = t;
  }
  memcpy(out, a, (size_t)N);
  free(a);
  free(b);
  return 0;
}

int oracle_life(const uint8_t* in, int64_t R, int64_t C, int64_t G, uint8_t* out) {
  return life_run(in, R, C, G, out, 1);
}

int oracle_life_omp(const uint8_t* in, int64_t R, int64_t C, int64_t G, uint8_t* out,
                    int threads) {
  return life_run(in, R, C, G, out, threads);
}

/* Returns 0 ok, -1 bad arguments (mode outside 0 .. 2 too), -2 out of memory. */
int oracle_life_decomp(const uint8_t* in, int64_t R, int64_t C, int64_t G, uint8_t* out,
                       int threads, int mode) {
  if (!in || !out || R <= 0 || C <= 0 || G < 0 || threads < 1 || mode < 0 || mode > 2)
    return -1;
  if (R > INT64_MAX / C) return -1;
  const int64_t N = R * C;
  uint8_t* a = (uint8_t*)malloc((size_t)N);
  uint8_t* b = (uint8_t*)malloc((size_t)N);
  if (!a || !b) { free(a); free(b); return -2; }
  for (int64_t i = 0; i < N; ++i) a[i] = in[i] ? 1 : 0;
  for (int64_t g = 0; g < G; ++g) {
#ifdef _OPENMP
#pragma omp parallel num_threads(threads)
    {
      const int64_t nt = omp_get_num_threads();
      const int64_t t = omp_get_thread_num();
      int64_t r0, r1, c0, c1;
      region(mode, R, C, t, nt, &r0, &r1, &c0, &c1);
      step_block(a, b, R, C, r0, r1, c0, c1);
    }
#else
    step_block(a, b, R, C, 0, R, 0, C);
#endif
    uint8_t* t = a; a = b; b = t;
  }
  memcpy(out, a, (size_t)N);
  free(a);
  free(b);
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

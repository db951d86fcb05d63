// Host-side schedule of tile passes; see gol_plan.h.
#include "gol_plan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <map>
#include <numeric>

namespace gol {

bool valid_T(int T) { return T == 1 || T == 2 || T == 4 || T == 8 || T == 12 || T == 16; }
bool valid_board_T(int T) { return valid_T(T); }

static int64_t dwords_per_row(int64_t cols) { return 2 * ((cols + 63) / 64); }

GridGeom board_geometry(int64_t rows, int64_t cols, int band_rows) {
  const int64_t D = dwords_per_row(cols);
  const int64_t ns = (D + kStripDwords - 1) / kStripDwords;
  const int64_t nb = (rows + band_rows - 1) / band_rows;
  const Split s = split(D, ns), b = split(rows, nb);
  GridGeom g;
  g.nstrips = (int32_t)ns;
  g.nbands = (int32_t)nb;
  g.strip_q = (int32_t)s.q;
  g.strip_r = (int32_t)s.r;
  g.band_q = (int32_t)b.q;
  g.band_r = (int32_t)b.r;
  return g;
}

GridGeom paired_geometry(int64_t rows, int64_t cols, int band_rows, int T, int pd) {
  const int64_t D = dwords_per_row(cols);
  const int64_t ns = (D + kHalfStripDwords - 1) / kHalfStripDwords;
  // band height: at least band_rows and T, with H - T a multiple of pd
  int64_t H = std::max<int64_t>({1, (int64_t)band_rows, (int64_t)T});
  if (pd > 0) H = T + ((H - T + pd - 1) / pd) * pd;
  const int64_t npairs = std::max<int64_t>(1, (rows + 2 * H - 1) / (2 * H));
  const Split s = split(D, ns);
  GridGeom g;
  g.nstrips = (int32_t)ns;
  g.nbands = (int32_t)(2 * npairs);
  g.strip_q = (int32_t)s.q;
  g.strip_r = (int32_t)s.r;
  g.band_q = (int32_t)std::min<int64_t>(H, INT32_MAX);
  g.band_r = 0;
  return g;
}

bool paired_ok(int64_t rows, int64_t cols, int T, const GridGeom& g, const char** why) {
  const char* w = nullptr;
  if (!(T == 8 || T == 12 || T == 16))
    w = "the paired layout runs 8, 12 or 16 generations per pass";
  else if (cols % 32 != 0)
    w = "the paired layout needs a column count that is a multiple of 32";
  else if (rows * dwords_per_row(cols) * 4 >= (int64_t(1) << 31))
    w = "the paired layout needs a packed board below 2 GiB";
  else if (g.band_q > 65535)
    w = "the paired layout takes bands of at most 65535 rows";
  if (why) *why = w;
  return w == nullptr;
}

// Throughput of the tile pass relative to its best, against resident waves
// per SIMD (measured on MI355X for 16384^2 and 65536^2 boards after removing
// the halo-row overhead; the two boards agree): latency is hidden better
// with more waves.
static double occupancy_factor(double waves_per_simd) {
  static const double k[] = {1, 2, 3, 4, 6, 8, 12, 16};
  static const double f[] = {0.45, 0.68, 0.80, 0.86, 0.90, 0.93, 0.97, 0.97};
  if (waves_per_simd <= k[0]) return f[0] * waves_per_simd / k[0];
  for (int i = 1; i < 8; ++i)
    if (waves_per_simd <= k[i])
      return f[i - 1] + (f[i] - f[i - 1]) * (waves_per_simd - k[i - 1]) / (k[i] - k[i - 1]);
  return f[7];
}

int default_band_rows(int64_t rows, int64_t cols, int T, int nsimd) {
  const int64_t D = dwords_per_row(cols);
  const int64_t ns = (D + kStripDwords - 1) / kStripDwords;
  if (nsimd < 1) nsimd = 1024;
  // Candidate band counts put the wave total just under a multiple of the
  // SIMD count (a SIMD holding one wave more than the rest sets the pace).
  // Each band sweeps h + 2T rows to emit h; stage s runs from step 2s, so the
  // pipeline does h + T + 1 row steps of work per T generations of h rows.
  // Estimated time: waves on the busiest SIMD x row steps per wave, slowed
  // by the occupancy factor of that many resident waves.
  double best = 1e300;
  int64_t best_h = std::min<int64_t>(rows, 64);
  for (int k : {1, 2, 3, 4, 6, 8, 12, 16, 24}) {
    const int64_t bands = std::max<int64_t>(1, (int64_t)k * nsimd / ns);
    const int64_t h = std::max<int64_t>(1, (rows + bands - 1) / bands);
    if (h > 65535) continue;
    const int64_t nb = (rows + h - 1) / h;
    const double waves = (double)(nb * ns);
    const double per_simd_max = std::ceil(waves / nsimd);
    const double t = per_simd_max * (double)(h + T + 1) /
                     occupancy_factor(std::min(per_simd_max, 16.0));
    if (t < best) {
      best = t;
      best_h = h;
    }
  }
  return (int)best_h;
}

int default_prefetch(int T) { return T >= 16 ? 12 : T >= 8 ? 9 : 3; }

namespace {
struct ItemBuild {
  std::vector<Segment> segs;
  int lanes = 0;
  int h = 0;
  int maxK = 0;
  bool aligned = true;
};
}  // namespace

// First-fit packing of the segments of `order`'s boards (K descending) into
// 64-lane waves.  A segment joins an open wave if it fits, its band is at
// most an eighth shorter than the wave's tallest (the wave's row count is its
// tallest band), and its board needs at most max(2, maxK / 8) fewer passes
// than the wave's longest board (lanes of shorter boards idle in the levels
// where their board does not run).
static std::vector<ItemBuild> pack_waves(const std::vector<BoardReq>& boards,
                                         const std::vector<int32_t>& K,
                                         const std::vector<int32_t>& order, int band_rows) {
  std::vector<ItemBuild> built;
  std::vector<size_t> open;  // indices of waves that may still take segments
  for (int32_t b : order) {
    const BoardReq& q = boards[b];
    const int64_t D = dwords_per_row(q.cols);
    const int64_t ns = (D + kStripDwords - 1) / kStripDwords;
    const Split S = split(D, ns);
    const int64_t nb = (q.rows + band_rows - 1) / band_rows;
    const Split B = split(q.rows, nb);
    const int Kb = K[b];
    const bool aligned = (q.cols % 32) == 0;
    // waves that can no longer take boards of this K close for good
    open.erase(std::remove_if(open.begin(), open.end(),
                              [&](size_t i) {
                                return built[i].maxK - Kb > std::max(2, built[i].maxK / 8);
                              }),
               open.end());
    for (int64_t bi = 0; bi < nb; ++bi) {
      const int h = (int)B.size(bi);
      for (int64_t si = 0; si < ns; ++si) {
        Segment sg;
        sg.board = b;
        sg.p0 = (int32_t)(S.start(si) - 1);
        sg.r0 = (int32_t)B.start(bi);
        sg.h = (uint16_t)h;
        sg.nlanes = (uint8_t)(S.size(si) + 2);
        size_t pick = SIZE_MAX;
        const size_t first = open.size() > 64 ? open.size() - 64 : 0;
        for (size_t k = first; k < open.size(); ++k) {
          const ItemBuild& it = built[open[k]];
          if (it.lanes + sg.nlanes <= kWave && h <= it.h && h >= it.h - it.h / 8) {
            pick = k;
            break;
          }
        }
        if (pick == SIZE_MAX) {
          ItemBuild it;
          it.h = h;
          it.maxK = Kb;
          built.push_back(std::move(it));
          open.push_back(built.size() - 1);
          pick = open.size() - 1;
        }
        ItemBuild& it = built[open[pick]];
        sg.lane0 = (uint8_t)it.lanes;
        it.segs.push_back(sg);
        it.lanes += sg.nlanes;
        it.aligned = it.aligned && aligned;
        if (it.lanes > kWave - 3) open.erase(open.begin() + pick);
        // only the last 64 open waves are ever searched: waves far behind
        // them close, which keeps each erase short
        if (open.size() > 512) open.erase(open.begin(), open.end() - 128);
      }
    }
  }
  std::stable_sort(built.begin(), built.end(),
                   [](const ItemBuild& a, const ItemBuild& c) { return a.maxK > c.maxK; });
  return built;
}

bool build_plan(const std::vector<BoardReq>& boards, int T, int band_rows, HostPlan& plan,
                std::string& err) {
  if (!valid_T(T)) {
    err = "generations per pass must be 1, 2, 4, 8, 12 or 16";
    return false;
  }
  if (band_rows < 1 || band_rows > 65535) {
    err = "band height out of range";
    return false;
  }
  plan = HostPlan();
  plan.T = T;
  plan.band_rows = band_rows;
  const size_t n = boards.size();
  plan.K.assign(n, 0);
  plan.Tshort.assign(n, 0);
  plan.start.assign(n, 0);
  plan.jshort.assign(n, 0);
  for (size_t b = 0; b < n; ++b) {
    const BoardReq& q = boards[b];
    if (q.rows < 1 || q.cols < 1 || q.rows > (1 << 30) || q.cols > (1 << 30) ||
        q.generations < 0) {
      err = "board " + std::to_string(b) + ": size or generations out of range";
      return false;
    }
    const int64_t K = (q.generations + T - 1) / T;
    if (K > (int64_t)1 << 30) {
      err = "board " + std::to_string(b) + ": too many generations";
      return false;
    }
    plan.K[b] = (int32_t)K;
    plan.Tshort[b] = K > 0 ? (int32_t)(q.generations - (K - 1) * T) : 0;
    plan.cell_updates += (double)q.rows * (double)q.cols * (double)q.generations;
  }
  std::vector<int32_t> order;
  for (size_t b = 0; b < n; ++b)
    if (plan.K[b] > 0) order.push_back((int32_t)b);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t c) { return plan.K[a] > plan.K[c]; });
  const int Kmax = order.empty() ? 0 : plan.K[order.front()];

  // Groups: longest boards first, each to the group (early: levels 0 .. K - 1,
  // late: Kmax - K .. Kmax - 1) whose levels it spans hold less work so far.
  // A board's work per pass is counted as its lanes times its rows.
  std::vector<double> load((size_t)Kmax, 0.0), prefix((size_t)Kmax + 1, 0.0);
  std::vector<int32_t> early, late;
  for (int32_t b : order) {
    const int Kb = plan.K[b];
    const double w = (double)boards[b].rows * (double)(dwords_per_row(boards[b].cols) + 2);
    double e = 0.0, l = 0.0;
    for (int L = 0; L < Kb; ++L) e += load[L];
    for (int L = Kmax - Kb; L < Kmax; ++L) l += load[L];
    if (l < e) {
      late.push_back(b);
      plan.start[b] = Kmax - Kb;
      plan.jshort[b] = Kb - 1;
      for (int L = Kmax - Kb; L < Kmax; ++L) load[L] += w;
    } else {
      early.push_back(b);
      for (int L = 0; L < Kb; ++L) load[L] += w;
    }
  }

  const std::vector<ItemBuild> be = pack_waves(boards, plan.K, early, band_rows);
  const std::vector<ItemBuild> bl = pack_waves(boards, plan.K, late, band_rows);
  plan.segs.clear();
  plan.items.clear();
  plan.items.reserve(be.size() + bl.size());
  for (const std::vector<ItemBuild>* grp : {&be, &bl}) {
    if (grp == &bl) plan.late_begin = (int32_t)plan.items.size();
    for (const ItemBuild& it : *grp) {
      WaveItem w;
      w.seg_begin = (int32_t)plan.segs.size();
      w.nseg = (int16_t)it.segs.size();
      w.h = (uint16_t)it.h;
      w.maxK = it.maxK;
      w.flags = it.aligned ? kItemAligned : 0;
      plan.items.push_back(w);
      plan.segs.insert(plan.segs.end(), it.segs.begin(), it.segs.end());
    }
  }
  plan.level_early.assign(Kmax, 0);
  plan.level_late.assign(Kmax, 0);
  plan.level_items.assign(Kmax, 0);
  for (int32_t b : early)
    if (plan.Tshort[b] < T) plan.early_masked = true;
  for (int32_t b : late)
    if (plan.Tshort[b] < T) plan.late_masked = true;
  // early waves with maxK > L run at level L; late waves with maxK >= Kmax - L
  size_t ce = be.size(), cl = 0;
  for (int L = 0; L < Kmax; ++L) {
    while (ce > 0 && be[ce - 1].maxK <= L) --ce;
    while (cl < bl.size() && bl[cl].maxK >= Kmax - L) ++cl;
    plan.level_early[L] = (int32_t)ce;
    plan.level_late[L] = (int32_t)cl;
    plan.level_items[L] = (int32_t)(ce + cl);
    for (size_t i = 0; i < ce; ++i) plan.lane_steps += (double)kWave * (be[i].h + 2 * T);
    for (size_t i = 0; i < cl; ++i) plan.lane_steps += (double)kWave * (bl[i].h + 2 * T);
  }
  return true;
}


void board_tiles(int64_t rows, int64_t cols, int band_rows, BoardTiles& out) {
  out.band_rows = band_rows;
  out.aligned = (cols % 32) == 0;
  out.segs.clear();
  out.waves.clear();
  const int64_t D = dwords_per_row(cols);
  const int64_t ns = (D + kStripDwords - 1) / kStripDwords;
  const Split S = split(D, ns);
  const int64_t nb = (rows + band_rows - 1) / band_rows;
  const Split B = split(rows, nb);
  // lanes of the widest strip: segments per wave when strips are narrow
  const int64_t lanes = S.size(0) + 2;
  const int64_t per = std::max<int64_t>(1, kWave / lanes);
  out.segs.reserve((size_t)(ns * nb));
  for (int64_t si = 0; si < ns; ++si) {
    for (int64_t b0 = 0; b0 < nb; b0 += per) {
      BoardTiles::Wave w;
      w.seg_begin = (int32_t)out.segs.size();
      w.nseg = 0;
      w.h = 0;
      int lane = 0;
      for (int64_t bi = b0; bi < std::min(nb, b0 + per); ++bi) {
        Segment sg;
        sg.board = 0;
        sg.p0 = (int32_t)(S.start(si) - 1);
        sg.r0 = (int32_t)B.start(bi);
        sg.h = (uint16_t)B.size(bi);
        sg.lane0 = (uint8_t)lane;
        sg.nlanes = (uint8_t)(S.size(si) + 2);
        lane += sg.nlanes;
        w.h = std::max<uint16_t>(w.h, sg.h);
        w.nseg += 1;
        out.segs.push_back(sg);
      }
      out.waves.push_back(w);
    }
  }
}

bool build_chunk_plan(const std::vector<ChunkBoard>& boards, int T, HostPlan& plan,
                      std::string& err) {
  if (!valid_T(T)) {
    err = "generations per pass must be 1, 2, 4, 8, 12 or 16";
    return false;
  }
  plan = HostPlan();
  plan.T = T;
  const size_t n = boards.size();
  plan.K.assign(n, 0);
  plan.Tshort.assign(n, 0);
  plan.start.assign(n, 0);
  plan.jshort.assign(n, 0);
  int Kmax = 0;
  for (size_t b = 0; b < n; ++b) {
    const ChunkBoard& q = boards[b];
    if (!q.tiles || q.generations < 0 || q.generations > ((int64_t)1 << 30)) {
      err = "board " + std::to_string(b) + ": no tiles or generations out of range";
      return false;
    }
    const int64_t K = (q.generations + T - 1) / T;
    plan.K[b] = (int32_t)K;
    plan.Tshort[b] = K > 0 ? (int32_t)(q.generations - (K - 1) * T) : 0;
    plan.cell_updates += (double)q.rows * (double)q.cols * (double)q.generations;
    Kmax = std::max<int>(Kmax, (int)K);
    if (b == 0 || q.tiles->band_rows > plan.band_rows) plan.band_rows = q.tiles->band_rows;
  }
  // boards by pass count, most first (counting sort: K <= Kmax), then the
  // early / late groups as in build_plan
  std::vector<std::vector<int32_t>> byK((size_t)Kmax + 1);
  for (size_t b = 0; b < n; ++b)
    if (plan.K[b] > 0) byK[(size_t)plan.K[b]].push_back((int32_t)b);
  // Boards that run every level (K == Kmax, most of a busy chunk) are split
  // between the groups by load, so each group's stream carries about half
  // of every level and the two streams fill each other's level tails (in a
  // schedule of uneven K the early / late split does this by itself).
  std::vector<double> load((size_t)Kmax, 0.0);
  std::vector<int32_t> early, late;
  double e_all = 0.0, l_all = 0.0;
  for (int k = Kmax; k >= 1; --k) {
    for (int32_t b : byK[(size_t)k]) {
      const double w = (double)boards[b].rows * (double)(dwords_per_row(boards[b].cols) + 2);
      double e = 0.0, l = 0.0;
      if (k < Kmax) {
        for (int L = 0; L < k; ++L) e += load[L];
        for (int L = Kmax - k; L < Kmax; ++L) l += load[L];
      } else {
        e = e_all;
        l = l_all;
      }
      if (l < e) {
        l_all += w * k;
        late.push_back(b);
        plan.start[b] = Kmax - k;
        plan.jshort[b] = k - 1;
        for (int L = Kmax - k; L < Kmax; ++L) load[L] += w;
      } else {
        e_all += w * k;
        early.push_back(b);
        for (int L = 0; L < k; ++L) load[L] += w;
      }
    }
  }
  // waves: each board's own, its segments relabelled with the board's index;
  // the groups' boards are already in descending K, so their waves are too
  size_t nseg = 0, nwave = 0;
  for (size_t b = 0; b < n; ++b)
    if (plan.K[b] > 0) {
      nseg += boards[b].tiles->segs.size();
      nwave += boards[b].tiles->waves.size();
    }
  plan.segs.reserve(nseg);
  plan.items.reserve(nwave);
  std::vector<int32_t> maxk_e, maxk_l;
  for (const std::vector<int32_t>* grp : {&early, &late}) {
    if (grp == &late) plan.late_begin = (int32_t)plan.items.size();
    for (int32_t b : *grp) {
      const BoardTiles& t = *boards[b].tiles;
      const int32_t base = (int32_t)plan.segs.size();
      for (Segment sg : t.segs) {
        sg.board = b;
        plan.segs.push_back(sg);
      }
      for (const BoardTiles::Wave& w : t.waves) {
        WaveItem it;
        it.seg_begin = base + w.seg_begin;
        it.nseg = w.nseg;
        it.h = w.h;
        it.maxK = plan.K[b];
        it.flags = t.aligned ? kItemAligned : 0;
        plan.items.push_back(it);
        (grp == &late ? maxk_l : maxk_e).push_back(plan.K[b]);
      }
    }
  }
  plan.level_early.assign(Kmax, 0);
  plan.level_late.assign(Kmax, 0);
  plan.level_items.assign(Kmax, 0);
  for (int32_t b : early)
    if (plan.Tshort[b] < T) plan.early_masked = true;
  for (int32_t b : late)
    if (plan.Tshort[b] < T) plan.late_masked = true;
  size_t ce = maxk_e.size(), cl = 0;
  for (int L = 0; L < Kmax; ++L) {
    while (ce > 0 && maxk_e[ce - 1] <= L) --ce;
    while (cl < maxk_l.size() && maxk_l[cl] >= Kmax - L) ++cl;
    plan.level_early[L] = (int32_t)ce;
    plan.level_late[L] = (int32_t)cl;
    plan.level_items[L] = (int32_t)(ce + cl);
  }
  for (size_t i = 0; i < plan.items.size(); ++i) {
    const WaveItem& it = plan.items[i];
    plan.lane_steps += (double)kWave * (it.h + 2 * T) * (double)it.maxK;
  }
  return true;
}

// Waves of a chunk's tiles at band height h (board_tiles' layout).
static double chunk_waves(const std::vector<std::pair<int64_t, int64_t>>& boards, int h) {
  double waves = 0.0;
  for (const auto& rc : boards) {
    const int64_t D = dwords_per_row(rc.second);
    const int64_t ns = (D + kStripDwords - 1) / kStripDwords;
    const int64_t nb = (rc.first + h - 1) / h;
    const int64_t lanes = split(D, ns).size(0) + 2;
    const int64_t per = std::max<int64_t>(1, kWave / lanes);
    waves += (double)ns * (double)((nb + per - 1) / per);
  }
  return waves;
}

int chunk_band_rows(const std::vector<std::pair<int64_t, int64_t>>& boards, int T, int nsimd,
                    int base) {
  if (nsimd < 1) nsimd = 1024;
  int h = std::max(base, 1);
  const int floor_h = std::max(32, T);
  while (h / 2 >= floor_h && chunk_waves(boards, h) < 2.0 * nsimd) h /= 2;
  return h;
}

bool build_queue_plan(const std::vector<BoardReq>& boards, int T, int band_rows, QueuePlan& qp,
                      std::string& err) {
  if (!(T == 8 || T == 12 || T == 16)) {
    err = "the queue form runs 8, 12 or 16 generations per pass";
    return false;
  }
  if (band_rows < 1 || band_rows > 65535) {
    err = "band height out of range";
    return false;
  }
  qp = QueuePlan();
  qp.T = T;
  const size_t n = boards.size();
  qp.per_pass.assign(n, 0);
  std::vector<int64_t> K(n, 0);
  std::vector<int32_t> seg_base(n, 0), wave_base(n, 0);
  std::vector<BoardTiles::Wave> waves;
  int64_t Kmax = 0;
  for (size_t b = 0; b < n; ++b) {
    K[b] = (boards[b].generations + T - 1) / T;
    Kmax = std::max(Kmax, K[b]);
    if (K[b] == 0) continue;
    BoardTiles t;
    board_tiles(boards[b].rows, boards[b].cols, band_rows, t);
    seg_base[b] = (int32_t)qp.segs.size();
    wave_base[b] = (int32_t)waves.size();
    for (Segment sg : t.segs) {
      sg.board = (int32_t)b;
      qp.segs.push_back(sg);
    }
    for (BoardTiles::Wave w : t.waves) {
      w.seg_begin += seg_base[b];
      waves.push_back(w);
    }
    qp.per_pass[b] = (int32_t)t.waves.size();
  }
  std::vector<int32_t> order;
  for (size_t b = 0; b < n; ++b)
    if (K[b] > 0) order.push_back((int32_t)b);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
    return (double)boards[a].rows * boards[a].cols * boards[a].generations >
           (double)boards[c].rows * boards[c].cols * boards[c].generations;
  });
  for (int64_t L = 0; L < Kmax; ++L)
    for (int32_t b : order) {
      if (L >= K[b]) continue;
      const bool aligned = boards[b].cols % 32 == 0;
      for (int32_t w = 0; w < qp.per_pass[b]; ++w) {
        const BoardTiles::Wave& wv = waves[(size_t)wave_base[b] + w];
        QueueItem it;
        it.seg_begin = wv.seg_begin;
        it.nseg = wv.nseg;
        it.h = wv.h;
        it.board = b;
        it.pass = (int32_t)L;
        it.flags = aligned ? kItemAligned : 0;
        qp.items.push_back(it);
      }
    }
  if (qp.items.size() > (size_t)INT32_MAX) {
    err = "too many queue items";
    return false;
  }
  return true;
}

}  // namespace gol

// Host check of the convolution work lists (tiles, packed rows, tasks,
// partial-sum slots) that the plan builds from the history windows of
// section 3.1.  Built with the address and undefined-behaviour sanitizers on
// the host side and run on the CPU: it calls the plan's own builders
// (window_steps, closure_kept, build_tiles) over a sweep of fault sizes,
// step sizes, cut-offs, learned-closure cuts, engines and tile shapes, and
// checks every property the conv kernels and the mode stage rely on:
//  - tasks cover the tiles in order, each within the workgroup's LDS slots;
//  - each mode's tiles (rows) cover its ring slots [0, R_n) once, in order,
//    and carry the mode's own ring parameters;
//  - a partial sum is written by one task only, its tiles are consecutive
//    in that task, and the mode stage's (mode_pos, part0, nparts) list names
//    exactly the partial sums the mode's tiles write;
//  - packed rows: every task is 128 rows, flush slots are numbered in row
//    order, a wave sum ends at every wave end and at the end of every
//    partial sum, runs of slots of one partial sum add up to the task's
//    count, and every field fits the bits the row word gives it.
// Prints one line per failure and a summary; exit status 0 when all hold.
#include <cstdint>
#include <cstdio>
#include <set>
#include <vector>

#include "internal.h"

using namespace sbiem;

namespace {

long long g_cases = 0, g_fail = 0;

#define CHECK(cond, ...)                                                           \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      if (g_fail < 40) {                                                           \
        std::printf("FAIL %s:%d (%s) ", __FILE__, __LINE__, #cond);                \
        std::printf(__VA_ARGS__);                                                  \
        std::printf("\n");                                                         \
      }                                                                            \
      ++g_fail;                                                                    \
      return;                                                                      \
    }                                                                              \
  } while (0)

struct Case {
  int log2N;
  double L, beta, kcT, kcN;
  bool closure, var;
  int precision, tile;
};

// the ring set-up of the plan (fixed-step and variable-step engines)
void ring_setup(const sbiem_plan& p, DtData& d, double dt, double hmin) {
  const int half = (int)(p.N / 2);
  d.dt = dt;
  d.MT = window_steps(p.N, p.L, p.cs, dt, p.kcL[0]);
  d.MN = window_steps(p.N, p.L, p.cs, dt, p.kcL[1]);
  d.M.assign(half + 1, 0);
  for (int n = 0; n <= half; ++n) d.M[n] = std::max(d.MT[n], d.MN[n]);
  std::vector<int> a, b;
  if (d.var) {
    a = window_steps(p.N, p.L, p.cs, hmin, p.kcL[0]);
    b = window_steps(p.N, p.L, p.cs, hmin, p.kcL[1]);
  }
  d.Rn.assign(half + 1, 0);
  d.ring_off.assign(half + 1, 0);
  long long slots = 0;
  for (int n = 1; n <= half; ++n) {
    if (d.var)
      d.Rn[n] = std::max(a[n], b[n]) + 2;
    else
      d.Rn[n] = (p.closure_on ? closure_kept(d.M[n], p.closure_cut) : d.M[n]) - 1;
    d.ring_off[n] = slots;
    slots += d.Rn[n];
  }
  d.ring_slots = slots;
}

void check_case(const Case& c) {
  ++g_cases;
  sbiem_plan p;
  p.log2N = c.log2N;
  p.N = (int64_t)1 << c.log2N;
  p.log2P = c.log2N / 2;  // the four-step split of the transforms
  p.log2Q = c.log2N - p.log2P;
  p.L = c.L;
  p.cs = 3464.0;
  p.kcL[0] = c.kcT;
  p.kcL[1] = c.kcN;
  p.precision = c.precision;
  p.closure_on = c.closure;
  p.closure_cut = 0.25;
  p.adaptive = c.var;
  const int half = (int)(p.N / 2);
  const double dt = c.beta * (c.L / (double)p.N) / p.cs;
  DtData d;
  d.var = c.var;
  ring_setup(p, d, dt, 0.5 * dt);
  const bool fp32 = c.precision == SBIEM_FP32CONV && !c.var;
  const int tile = fp32 ? c.tile : kTileSlots64;
  const bool packed = fp32 && tile == kTileSlots32p;
  const long double th_unit = 3.141592653589793238462643383279502884L * (long double)p.cs *
                              (long double)dt / (long double)p.L / (long double)kTableStep;
  const int extra = build_tiles(&p, &d, tile, th_unit);
  const int ntiles = (int)d.tiles.size();
  const int cap = packed ? kTaskRows
                         : (fp32 ? conv32_wave_tiles(tile) * (kConvThreads / 64) : kTaskTiles64);
  char tag[160];
  std::snprintf(tag, sizeof tag, "N=2^%d L=%g beta=%g kc=(%g,%g) closure=%d var=%d tile=%d",
                c.log2N, c.L, c.beta, c.kcT, c.kcN, (int)c.closure, (int)c.var, tile);
  CHECK(d.tile_slots == tile, "%s tile_slots %d", tag, d.tile_slots);
  CHECK(extra >= half + 1, "%s parts %d", tag, extra);
  CHECK((int)d.part0.size() == half + 1 && (int)d.nparts.size() == half + 1, "%s", tag);

  // tasks: in order, contiguous, non-empty, within the LDS slots
  int next = 0;
  for (size_t k = 0; k < d.tasks.size(); ++k) {
    const ConvTask& t = d.tasks[k];
    CHECK(t.t0 == next && t.t1 > t.t0, "%s task %zu [%d,%d) after %d", tag, k, t.t0, t.t1, next);
    CHECK(t.t1 - t.t0 <= cap, "%s task %zu has %d tiles (cap %d)", tag, k, t.t1 - t.t0, cap);
    CHECK(packed || cap <= kTaskTiles, "%s task slots %d beyond the LDS's %d", tag, cap,
          kTaskTiles);
    if (packed) {
      CHECK(t.t1 - t.t0 == kTaskRows && t.t0 == (int)k * kTaskRows, "%s packed task %zu", tag, k);
      CHECK(t.nsum >= 0 && t.nsum <= kTaskRows, "%s task %zu nsum %d", tag, k, t.nsum);
    }
    next = t.t1;
  }
  CHECK(next == ntiles, "%s tasks end at %d of %d tiles", tag, next, ntiles);
  if (packed) CHECK((int)d.row_meta.size() == ntiles, "%s row_meta %zu", tag, d.row_meta.size());

  // tiles: each mode's slots covered once, in order, with its own parameters
  std::vector<int> covered(half + 1, 0);
  std::vector<int> task_of(ntiles, -1);
  for (size_t k = 0; k < d.tasks.size(); ++k)
    for (int i = d.tasks[k].t0; i < d.tasks[k].t1; ++i) task_of[i] = (int)k;
  bool padding = false;
  for (int i = 0; i < ntiles; ++i) {
    const Tile& t = d.tiles[i];
    if (t.len == 0) {
      // only the packed layout pads, and only its last task
      CHECK(packed && task_of[i] == (int)d.tasks.size() - 1, "%s empty tile %d", tag, i);
      CHECK(t.part == -1, "%s empty row %d has part %d", tag, i, t.part);
      padding = true;
      continue;
    }
    CHECK(!padding, "%s tile %d after the padding", tag, i);
    const int n = t.mode;
    CHECK(n >= 1 && n <= half, "%s tile %d mode %d", tag, i, n);
    CHECK(t.len >= 1 && t.len <= tile, "%s tile %d len %d", tag, i, t.len);
    CHECK(t.p0 == covered[n], "%s tile %d of mode %d starts at %d, expected %d", tag, i, n, t.p0,
          covered[n]);
    CHECK(t.p0 % tile == 0, "%s tile %d p0 %d", tag, i, t.p0);
    CHECK(t.p0 + t.len <= d.Rn[n], "%s tile %d ends at %d past R_n %d", tag, i, t.p0 + t.len,
          d.Rn[n]);
    CHECK(t.len == tile || t.p0 + t.len == d.Rn[n], "%s tile %d short inside its mode", tag, i);
    CHECK(t.Rn == d.Rn[n] && t.MT == d.MT[n] && t.MN == d.MN[n] && t.ring_off == d.ring_off[n],
          "%s tile %d parameters", tag, i);
    CHECK(t.rmagic == UINT64_MAX / (uint64_t)t.Rn + 1, "%s tile %d ring magic", tag, i);
    covered[n] = t.p0 + t.len;
    // a mode runs through consecutive tiles (a later tile of mode n never
    // follows a tile of another mode)
    if (i > 0 && d.tiles[i - 1].len > 0 && d.tiles[i - 1].mode != n)
      CHECK(t.p0 == 0, "%s mode %d resumes at tile %d", tag, n, i);
  }
  for (int n = 1; n <= half; ++n)
    CHECK(covered[n] == d.Rn[n], "%s mode %d covered to %d of %d", tag, n, covered[n], d.Rn[n]);

  // partial sums: one task each, consecutive tiles, and the mode stage's list
  std::vector<int> owner(extra, -1), mode_of(extra, -1), last_tile(extra, -1);
  std::vector<std::set<int>> parts_of(half + 1);
  for (int i = 0; i < ntiles; ++i) {
    const Tile& t = d.tiles[i];
    if (t.len == 0) continue;
    CHECK(t.part >= 0 && t.part < extra, "%s tile %d part %d of %d", tag, i, t.part, extra);
    const int k = task_of[i];
    CHECK(owner[t.part] == -1 || owner[t.part] == k, "%s part %d written by tasks %d and %d", tag,
          t.part, owner[t.part], k);
    CHECK(mode_of[t.part] == -1 || mode_of[t.part] == t.mode, "%s part %d shared by modes", tag,
          t.part);
    CHECK(last_tile[t.part] == -1 || last_tile[t.part] == i - 1,
          "%s part %d not consecutive at tile %d", tag, t.part, i);
    owner[t.part] = k;
    mode_of[t.part] = t.mode;
    last_tile[t.part] = i;
    parts_of[t.mode].insert(t.part);
  }
  for (int n = 1; n <= half; ++n) {
    std::set<int> want;
    if (d.Rn[n] > 0) {
      CHECK(d.nparts[n] >= 1, "%s mode %d nparts %d", tag, n, d.nparts[n]);
      want.insert(mode_pos(n, p.log2P, p.log2Q));
      for (int j = 1; j < d.nparts[n]; ++j) want.insert(d.part0[n] + j - 1);
    } else {
      CHECK(d.nparts[n] == 0, "%s empty mode %d nparts %d", tag, n, d.nparts[n]);
    }
    CHECK(want == parts_of[n], "%s mode %d: the mode stage reads %zu partial sums, tiles write %zu",
          tag, n, want.size(), parts_of[n].size());
  }

  if (!packed) return;
  // packed rows: flush slots, runs and the bits of the row word
  for (size_t k = 0; k < d.tasks.size(); ++k) {
    const ConvTask& tk = d.tasks[k];
    int slot = 0;
    int run_total = 0;
    for (int i = tk.t0; i < tk.t1; ++i) {
      const Tile& t = d.tiles[i];
      const int2 m = d.row_meta[i];
      if (t.len == 0) {
        CHECK(m.x == -1 && m.y == 0, "%s empty row %d meta (%d,%d)", tag, i, m.x, m.y);
        continue;
      }
      const bool wave_end = (i - tk.t0) % kPackRows == kPackRows - 1;
      const bool part_end = i + 1 == tk.t1 || d.tiles[i + 1].len == 0 ||
                            d.tiles[i + 1].part != t.part;
      if (wave_end || part_end) {
        CHECK(m.x == slot, "%s row %d flush slot %d, expected %d", tag, i, m.x, slot);
        ++slot;
      } else {
        CHECK(m.x == -1, "%s row %d flushes inside a wave and a partial sum", tag, i);
      }
      CHECK(t.len <= 0xFF && m.x + 1 <= 0xFF && m.y <= 0xFF, "%s row %d word fields", tag, i);
      if (m.y > 0) {
        CHECK(m.x >= 0, "%s row %d run without a slot", tag, i);
        run_total += m.y;
        // the run's slots are the next m.y flushes, all of this row's part
        int seen = 0;
        for (int j = i; j < tk.t1 && seen < m.y; ++j)
          if (d.row_meta[j].x >= 0) {
            CHECK(d.tiles[j].part == t.part, "%s run at row %d mixes parts", tag, i);
            CHECK(d.row_meta[j].x == m.x + seen, "%s run at row %d not consecutive", tag, i);
            ++seen;
          }
        CHECK(seen == m.y, "%s run at row %d has %d of %d slots", tag, i, seen, m.y);
      }
    }
    CHECK(slot == tk.nsum, "%s task %zu has %d slots, nsum %d", tag, k, slot, tk.nsum);
    CHECK(run_total == tk.nsum, "%s task %zu runs add to %d of %d", tag, k, run_total, tk.nsum);
  }
}

}  // namespace

int main() {
  std::vector<Case> cases;
  const double kc[][2] = {{200.0, 200.0}, {100.0, 300.0}, {50.0, 50.0}, {6.0, 6.0}};
  for (int lg = 3; lg <= 16; ++lg)
    for (double beta : {0.25, 0.5, 1.0})
      for (const auto& k : kc)
        for (int cl = 0; cl < 2; ++cl) {
          const double L = (lg % 2 ? 10.0 : 40.0) * (double)(1 << lg);
          if (lg <= 14 || (beta == 0.5 && k[0] == 200.0)) {
            for (int tile : {kTileSlots32p, kTileSlots32s, kTileSlots32w, kTileSlots32, kTileSlots32l})
              cases.push_back({lg, L, beta, k[0], k[1], cl == 1, false, SBIEM_FP32CONV, tile});
            if (cl == 0) {
              cases.push_back({lg, L, beta, k[0], k[1], false, false, SBIEM_FP64, 0});
              if (lg <= 13) cases.push_back({lg, L, beta, k[0], k[1], false, true, SBIEM_FP64, 0});
            }
          }
        }
  // the benchmark's fault (N = 2^18, 2400 km, beta 0.5), plain and closed
  for (int cl = 0; cl < 2; ++cl)
    for (int tile : {kTileSlots32p, kTileSlots32s, kTileSlots32w, kTileSlots32})
      cases.push_back({18, 2400e3, 0.5, 200.0, 200.0, cl == 1, false, SBIEM_FP32CONV, tile});
  for (const Case& c : cases) check_case(c);
  std::printf("%lld cases, %lld failures\n", g_cases, g_fail);
  return g_fail == 0 ? 0 : 1;
}

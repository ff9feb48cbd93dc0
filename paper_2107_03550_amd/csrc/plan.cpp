// Plan management of libsbiem: validation, curvature, windows, weight tables,
// device buffers, state upload/download and the stress-only path.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <complex>
#include <cstring>
#include <sstream>
#include <thread>

#include "internal.h"

namespace sbiem {

namespace {
thread_local std::string g_last_error;
const long double kPiL = 3.141592653589793238462643383279502884L;
}  // namespace

DeviceAllocator& allocator() {
  static DeviceAllocator a;
  return a;
}

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  DeviceAllocator& a = allocator();
  if (a.alloc) return a.alloc(bytes, a.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  DeviceAllocator& a = allocator();
  if (a.release) a.release(p, a.ctx);
  else (void)hipFree(p);
}

void* DevArena::get(size_t bytes) {
  void* p = dev_alloc(bytes);
  if (p) ptrs.push_back(p);
  return p;
}

void DevArena::release_all() {
  for (void* p : ptrs) dev_free(p);
  ptrs.clear();
}

int fail(sbiem_plan* p, int status, const std::string& msg) {
  if (p) p->last_error = msg;
  else g_last_error = msg;
  return status;
}

int fail_global(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(sbiem_plan* p, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(p, e == hipErrorOutOfMemory ? SBIEM_ENOMEM : SBIEM_EDEVICE, m);
}

namespace {

bool all_finite(const double* x, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// In-place iterative radix-2 FFT in long double (sign -1: forward).
void host_fft(std::vector<std::complex<long double>>& a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t i = 0; i < n; i += len) {
      for (size_t k = 0; k < len / 2; ++k) {
        long double ang = sign * 2.0L * kPiL * (long double)k / (long double)len;
        std::complex<long double> w(cosl(ang), sinl(ang));
        std::complex<long double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

// kappa = h'' spectrally: IDFT(-k^2 DFT(h)) with the Nyquist term kept.
std::vector<double> curvature_host(const double* h, int64_t N, double L) {
  std::vector<std::complex<long double>> a(N);
  for (int64_t i = 0; i < N; ++i) a[i] = h ? h[i] : 0.0;
  host_fft(a, -1);
  for (int64_t n = 0; n < N; ++n) {
    int64_t ns = n <= N / 2 ? n : n - N;
    long double k = 2.0L * kPiL * (long double)ns / (long double)L;
    a[n] *= -k * k;
  }
  host_fft(a, +1);
  std::vector<double> out(N);
  for (int64_t i = 0; i < N; ++i) out[i] = (double)(a[i].real() / (long double)N);
  return out;
}

}  // namespace

// Natural element order (host) -> class-major device order and back.
std::vector<double> to_elem_order(const sbiem_plan* p, const double* x) {
  const int64_t N = p->N;
  std::vector<double> y(N);
  for (int64_t i = 0; i < N; ++i) y[elem_pos((int)i, p->log2P, p->log2Q)] = x[i];
  return y;
}

hipError_t download_elems(const sbiem_plan* p, const double* dev, double* host) {
  const int64_t N = p->N;
  std::vector<double> y(N);
  hipError_t e = hipMemcpy(y.data(), dev, (size_t)N * sizeof(double), hipMemcpyDeviceToHost);
  if (e) return e;
  for (int64_t i = 0; i < N; ++i) host[i] = y[elem_pos((int)i, p->log2P, p->log2Q)];
  return hipSuccess;
}

namespace {

template <typename T>
T* upload(sbiem::DevArena& mem, const std::vector<T>& v, hipStream_t s, hipError_t* err) {
  T* d = (T*)mem.get(v.size() * sizeof(T));
  if (!d) {
    *err = hipErrorOutOfMemory;
    return nullptr;
  }
  if (!v.empty()) *err = hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
  return d;
}

}  // namespace

// Window lengths M_n (n = 0..N/2) exactly as the windows are defined:
// T_w = (L/c_s) min(1, k_c/|k|), k_c = kcL/L, M = ceil(x - 1e-9 x), x = T_w/dt.
std::vector<int> window_steps(int64_t N, double L, double cs, double dt, double kcL) {
  std::vector<int> M(N / 2 + 1);
  const double kc = kcL / (1.0 * L);
  for (int64_t n = 0; n <= N / 2; ++n) {
    const double k = 2.0 * M_PI * (double)n / L;
    const double ratio = k > kc ? kc / k : 1.0;
    const double Tw = (1.0 * L / cs) * ratio;
    const double x = Tw / dt;
    double m = std::ceil(x - 1e-9 * x);
    if (m < 1) m = 1;
    M[n] = (int)m;
  }
  return M;
}

int closure_kept(int M, double cut) {
  const int Mk = (int)std::ceil(cut * M - 1e-9);
  return (Mk >= 18 && Mk < M) ? Mk : M;
}

bool var_engine(const sbiem_plan* p) {
  return p->adaptive || (p->rule == SBIEM_RULE_INTERVAL && p->precision == SBIEM_FP32CONV);
}

namespace {

// Weights (w^T, w^N) of lags j = 0..count-1 of mode n at step dt for the
// plan's rule; zero from each kind's window length on.  theta = c_s |k| dt / 2.
void lag_weights(const sbiem_plan* p, int n, double dt, int MT, int MN, int j0, int count,
                 std::vector<long double>* wT, std::vector<long double>* wN) {
  const long double cs = p->cs, cp = p->cp;
  const long double theta = kPiL * cs * (long double)dt / (long double)p->L * n;
  wT->assign(count, 0.0L);
  wN->assign(count, 0.0L);
  if (n == 0) return;
  if (p->rule == SBIEM_RULE_MIDPOINT) {
    for (int c = 0; c < count; ++c) {
      const int j = j0 + c;
      if (j >= MT && j >= MN) continue;
      long double CT, CN;
      kernel_values(theta * (long double)(2 * j + 1), cs, cp, &CT, &CN, nullptr, nullptr);
      (*wT)[c] = j < MT ? dt * CT : 0.0L;
      (*wN)[c] = j < MN ? dt * CN : 0.0L;
    }
    return;
  }
  // INTERVAL: [P(min((2j+2) theta, Tcut)) - P(min(2j theta, Tcut))] dt / (2 theta)
  const long double kL = 2.0L * kPiL * n;
  const long double cutT = std::min(kL, (long double)p->kcL[0]);
  const long double cutN = std::min(kL, (long double)p->kcL[1]);
  const long double scale = (long double)dt / (2.0L * theta);
  auto prim = [&](int b, long double* PT, long double* PN) {
    const long double T = theta * (long double)(2 * b);
    long double pt, pn;
    kernel_primitives(std::min(T, cutT), cs, cp, &pt, &pn);
    *PT = pt;
    if (cutN != cutT) kernel_primitives(std::min(T, cutN), cs, cp, &pt, &pn);
    *PN = pn;
  };
  long double pT0, pN0;
  prim(j0, &pT0, &pN0);
  for (int c = 0; c < count; ++c) {
    const int j = j0 + c;
    long double pT1, pN1;
    prim(j + 1, &pT1, &pN1);
    (*wT)[c] = j < MT ? (pT1 - pT0) * scale : 0.0L;
    (*wN)[c] = j < MN ? (pN1 - pN0) * scale : 0.0L;
    pT0 = pT1;
    pN0 = pN1;
  }
}

}  // namespace

// Tiles (one wavefront each) and tasks (one workgroup each) of a fault's
// ring: a task holds whole modes up to task_tiles tiles, a longer mode is
// cut into pieces of task_tiles tiles, each with its own partial sum (the
// first piece of mode n at parts[mode_pos(n)], further pieces from N/2 + 1
// on).  FP32 tiles keep 16 rows of 64 records in flight per wave, so a task
// is 8192 records whatever the tile.  Returns the number of partial sums.
// Packed FP32 rows: every row of every mode in order, 128 to a task, a task
// ending wherever its 128th row falls (a mode cut by a task boundary gets one
// partial sum per task, ordered as above; the last task is padded with empty
// rows).  A wave sum ends at the last row of a partial sum in a wave and at a
// wave's last row; its LDS slot counts the task's wave sums in row order, so
// the slots of one partial sum are consecutive.
static int build_rows(const sbiem_plan* p, DtData* d, long double th_unit) {
  const int half = (int)(p->N / 2);
  d->tile_slots = kTileSlots32p;
  d->tiles.clear();
  d->tasks.clear();
  d->row_meta.clear();
  d->part0.assign(half + 1, 0);
  d->nparts.assign(half + 1, 0);
  int extra = half + 1;
  auto open_task = [&]() {
    const int at = (int)d->tiles.size();
    d->tasks.push_back(ConvTask{at, at, 0, 0});
  };
  for (int n = 1; n <= half; ++n) {
    const int rows = (d->Rn[n] + 63) / 64;
    if (rows == 0) continue;
    const int extra0 = extra;
    int part = mode_pos(n, p->log2P, p->log2Q);
    for (int r = 0; r < rows; ++r) {
      if (d->tasks.empty() || d->tasks.back().t1 - d->tasks.back().t0 == kTaskRows) {
        if (r > 0) part = extra++;   // the mode continues in a new task
        open_task();
      }
      Tile t{};
      t.mode = n;
      t.p0 = 64 * r;
      t.len = std::min(64, d->Rn[n] - 64 * r);
      t.Rn = d->Rn[n];
      t.part = part;
      t.MT = d->MT[n];
      t.MN = d->MN[n];
      t.ring_off = d->ring_off[n];
      t.th = (double)(th_unit * n);
      t.rmagic = UINT64_MAX / (uint64_t)t.Rn + 1;
      d->tiles.push_back(t);
      d->tasks.back().t1 = (int)d->tiles.size();
    }
    d->part0[n] = extra0;
    d->nparts[n] = 1 + (extra - extra0);
  }
  // pad the last task; empty rows have len 0 and no partial sum
  if (!d->tasks.empty())
    while (d->tasks.back().t1 - d->tasks.back().t0 < kTaskRows) {
      Tile t{};
      t.part = -1;
      t.Rn = 1;
      t.rmagic = 0;
      d->tiles.push_back(t);
      d->tasks.back().t1 = (int)d->tiles.size();
    }
  // wave sums: slots in row order; the run length at a partial sum's first
  d->row_meta.assign(d->tiles.size(), make_int2(-1, 0));
  for (ConvTask& k : d->tasks) {
    int slot = 0;
    for (int i = k.t0; i < k.t1; ++i) {
      const Tile& t = d->tiles[i];
      if (t.len == 0) continue;
      const bool wave_end = (i - k.t0) % kPackRows == kPackRows - 1;
      const bool last = i + 1 == k.t1 || d->tiles[i + 1].len == 0 || d->tiles[i + 1].part != t.part;
      if (wave_end || last) d->row_meta[i].x = slot++;
    }
    // run lengths: consecutive slots of one partial sum
    int run_row = -1, run_part = -2;
    for (int i = k.t0; i < k.t1; ++i) {
      if (d->row_meta[i].x < 0) continue;
      if (d->tiles[i].part != run_part) {
        run_row = i;
        run_part = d->tiles[i].part;
      }
      d->row_meta[run_row].y += 1;
    }
    k.nsum = slot;
  }
  return extra;
}

int build_tiles(const sbiem_plan* p, DtData* d, int tile, long double th_unit) {
  const int half = (int)(p->N / 2);
  const bool fp32 = p->precision == SBIEM_FP32CONV && !d->var;
  if (fp32 && tile == kTileSlots32p) return build_rows(p, d, th_unit);
  d->row_meta.clear();
  const int task_tiles = fp32 ? conv32_wave_tiles(tile) * (kConvThreads / 64) : kTaskTiles64;
  d->tile_slots = tile;
  d->tiles.clear();
  d->tasks.clear();
  d->part0.assign(half + 1, 0);
  d->nparts.assign(half + 1, 0);
  int extra = half + 1;
  int cur_tiles = 0;
  auto open_task = [&]() {
    d->tasks.push_back(ConvTask{(int)d->tiles.size(), (int)d->tiles.size(), 0, 0});
    cur_tiles = 0;
  };
  for (int n = 1; n <= half; ++n) {
    const int count = (d->Rn[n] + tile - 1) / tile;
    if (count == 0) continue;
    if (d->tasks.empty() || cur_tiles + std::min(count, task_tiles) > task_tiles) open_task();
    const int extra0 = extra;
    int part = mode_pos(n, p->log2P, p->log2Q);
    for (int k = 0; k < count; ++k) {
      if (cur_tiles == task_tiles) {  // a long mode continues in a new task
        open_task();
        part = extra++;
      }
      Tile t;
      t.fault = 0;
      t.mode = n;
      t.p0 = k * tile;
      t.len = std::min(tile, d->Rn[n] - k * tile);
      t.Rn = d->Rn[n];
      t.part = part;
      t.MT = d->MT[n];
      t.MN = d->MN[n];
      t.ring_off = d->ring_off[n];
      t.th = (double)(th_unit * n);
      t.rmagic = UINT64_MAX / (uint64_t)t.Rn + 1;
      d->tiles.push_back(t);
      d->tasks.back().t1 = (int)d->tiles.size();
      ++cur_tiles;
    }
    d->part0[n] = extra0;
    d->nparts[n] = 1 + (extra - extra0);
  }
  return extra;
}

int build_dt_data(sbiem_plan* p, double dt, DtData** out) {
  *out = nullptr;
  DtData* d = new DtData();
  d->dt = dt;
  d->var = var_engine(p);
  const int64_t N = p->N;
  const int half = (int)(N / 2);
  d->MT = window_steps(N, p->L, p->cs, dt, p->kcL[0]);
  d->MN = window_steps(N, p->L, p->cs, dt, p->kcL[1]);
  d->M.assign(half + 1, 0);
  for (int n = 0; n <= half; ++n) d->M[n] = std::max(d->MT[n], d->MN[n]);
  // the variable-step ring holds intervals as short as the half steps of an
  // attempt at dt_min (adaptive plans) or dt itself
  std::vector<int> Mvar;
  if (d->var) {
    const double hmin = p->adaptive ? 0.5 * dt : dt;
    const std::vector<int> a = window_steps(N, p->L, p->cs, hmin, p->kcL[0]);
    const std::vector<int> b = window_steps(N, p->L, p->cs, hmin, p->kcL[1]);
    Mvar.assign(half + 1, 0);
    for (int n = 0; n <= half; ++n) Mvar[n] = std::max(a[n], b[n]);
  }
  d->Rn.assign(half + 1, 0);
  d->ring_off.assign(half + 1, 0);
  long long slots = 0;
  int Rmax = 0;
  for (int n = 1; n <= half; ++n) {
    if (d->var) {
      // every interval a step at dt >= dt_min can still reach (M_n), plus
      // the two a rejected two-half-step attempt writes: the slots they
      // overwrite then hold intervals strictly past every window
      d->Rn[n] = Mvar[n] + 2;
    } else {
      // the learned closure keeps M'_n lags of the modes it closes
      const int kept = p->closure_on ? closure_kept(d->M[n], p->closure_cut) : d->M[n];
      d->Rn[n] = kept - 1;
    }
    d->ring_off[n] = slots;
    slots += d->Rn[n];
    Rmax = std::max(Rmax, d->Rn[n]);
  }
  d->ring_slots = slots;
  // conv tiles (one wavefront each) and tasks (one workgroup each)
  // (FP32 under the learned closure: shorter tiles, most kept windows being
  // far shorter than a full tile; the variable-step conv uses FP64 tiles)
  const bool fp32 = p->precision == SBIEM_FP32CONV && !d->var;
  const int tile = fp32 ? (p->conv_tile ? p->conv_tile
                                        : (p->closure_on ? kTileSlots32s : kTileSlots32))
                        : kTileSlots64;
  const long double th_unit = 3.141592653589793238462643383279502884L * (long double)p->cs *
                              (long double)dt / (long double)p->L / (long double)kTableStep;
  const int parts = build_tiles(p, d, tile, th_unit);
  // per-mode constants: lags 0 and 1 of the plan's rule (the variable-step
  // engine recomputes lag 0 per step and keeps lag 1 in its sums)
  std::vector<ModeCoef> coef(half + 1);
  const double c1 = 1.0 - p->r;
  auto mode_coef = [&](int n) {
    const double kabs = 2.0 * M_PI * (double)n / p->L;
    std::vector<long double> wT, wN;
    lag_weights(p, n, dt, d->MT[n], d->MN[n], 0, 2, &wT, &wN);
    ModeCoef& c = coef[mode_pos(n, p->log2P, p->log2Q)];
    c.mk = -p->mu * kabs;
    c.ms = (n == 0 || 2 * n == N) ? 0.0 : p->mu;
    c.aT = c1 * dt + (double)wT[0];
    c.aN = c1 * dt + (double)wN[0];
    c.w1T = d->var ? 0.0 : (double)wT[1];
    c.w1N = d->var ? 0.0 : (double)wN[1];
    c.ring_off = d->ring_off[n];
    c.Rn = d->Rn[n];
    c.part0 = d->part0[n];
    c.nparts = d->nparts[n];
    c.pad = 0;
  };
  {
    const int nth = half >= (1 << 15) ? 8 : 1;
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t)
      pool.emplace_back([&, t]() {
        for (int n = t; n <= half; n += nth) mode_coef(n);
      });
    for (int n = 0; n <= half; n += nth) mode_coef(n);
    for (auto& th : pool) th.join();
  }
  hipError_t e = hipSuccess;
  hipStream_t s = p->stream;
  d->coef = upload(d->mem, coef, s, &e);
  d->coef_host = coef;
  d->th_mode.assign(half + 1, 0.0);
  for (int n = 0; n <= half; ++n) d->th_mode[n] = (double)(th_unit * n);
  if (!e && p->closure_on) {
    std::vector<int> cn, cMk, cM;
    for (int n = 1; n <= half; ++n) {
      if (d->Rn[n] + 1 == d->M[n]) continue;  // open mode
      cn.push_back(n);
      cMk.push_back(d->Rn[n] + 1);
      cM.push_back(d->M[n]);
    }
    std::vector<double> DT, DN;
    discarded_weights(p->cs, p->cp, p->L, dt, cn, cMk, cM, &DT, &DN);
    size_t ci = 0;
    for (int n = 1; n <= half; ++n) {
      if (d->Rn[n] + 1 == d->M[n]) continue;  // open mode
      ClosureMode c;
      c.fault = 0;
      c.pm = mode_pos(n, p->log2P, p->log2Q);
      c.Rn = d->Rn[n];
      c.Mk = d->Rn[n] + 1;
      c.ring_off = d->ring_off[n];
      const double csk = p->cs * 2.0 * M_PI * (double)n / p->L;
      c.tcut = (float)(csk * c.Mk * dt / 100.0);
      c.pad = 0.f;
      c.inv_csk = 1.0 / csk;
      c.dT = DT[ci];
      c.dN = DN[ci];
      ++ci;
      d->closure.push_back(c);
    }
    d->tails = (double4*)d->mem.get(sizeof(double4) * (half + 1));
    if (!d->tails) e = hipErrorOutOfMemory;
    else e = hipMemsetAsync(d->tails, 0, sizeof(double4) * (half + 1), s);
  }
  if (!e) {
    d->parts = (double4*)d->mem.get(sizeof(double4) * std::max(1, parts));
    d->parts_cap = std::max(1, parts);
    if (!d->parts) e = hipErrorOutOfMemory;
    else e = hipMemsetAsync(d->parts, 0, sizeof(double4) * std::max(1, parts), s);
  }

  const size_t rec = p->precision == SBIEM_FP32CONV ? 16 : 32;
  if (!e) {
    d->ring = d->mem.get((size_t)std::max<long long>(slots, 1) * rec);
    if (!d->ring) e = hipErrorOutOfMemory;
    else e = hipMemsetAsync(d->ring, 0, (size_t)std::max<long long>(slots, 1) * rec, s);
  }
  if (!e && p->precision == SBIEM_FP64 && !d->var) {
    // FP64 weights in ring order: slot q of mode n holds the weights of lag
    // j = R_n - q + 1 (q >= 1); q = 0 is the lag-1 slot, weight 0.
    std::vector<double2> w(std::max<long long>(slots, 1));
    auto fill = [&](int n) {
      const int Rn = d->Rn[n];
      if (Rn <= 0) return;
      const long long off = d->ring_off[n];
      w[off] = make_double2(0.0, 0.0);
      if (Rn < 2) return;
      // lags 2..Rn in one pass
      std::vector<long double> wT, wN;
      lag_weights(p, n, dt, d->MT[n], d->MN[n], 2, Rn - 1, &wT, &wN);
      for (int q = 1; q < Rn; ++q) {
        const int j = Rn - q + 1;
        w[off + q] = make_double2((double)wT[j - 2], (double)wN[j - 2]);
      }
    };
    const int nth = slots >= (1 << 20) ? 8 : 1;
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t)
      pool.emplace_back([&, t]() {
        for (int n = 1 + t; n <= half; n += nth) fill(n);
      });
    for (int n = 1; n <= half; n += nth) fill(n);
    for (auto& th : pool) th.join();
    d->wrev = upload(d->mem, w, s, &e);
  }
  const long double cs = p->cs, cp = p->cp;
  if (!e && p->precision == SBIEM_FP32CONV && !d->var) {
    // Hermite table on T = i h covering every lag (plus the skipped slot).
    const long double theta_unit = kPiL * cs * (long double)dt / (long double)p->L;
    double Tmax = 0.0;
    for (int n = 1; n <= half; ++n)
      Tmax = std::max(Tmax, (double)(theta_unit * n) * (2.0 * (d->Rn[n] + 1) + 3.0));
    const int K = (int)std::ceil(Tmax / kTableStep) + 3;
    if ((size_t)K * sizeof(float4) > (size_t)(kMaxLdsBytes - kConvStaticLds)) {
      e = hipErrorInvalidValue;
    } else {
      std::vector<float4> tab(K);
      for (int i = 0; i < K; ++i) {
        long double CT, CN, dCT, dCN;
        kernel_values((long double)i * kTableStep, cs, cp, &CT, &CN, &dCT, &dCN);
        tab[i] = make_float4((float)(dt * CT), (float)(dt * kTableStep * dCT), (float)(dt * CN),
                             (float)(dt * kTableStep * dCN));
      }
      d->table_len = K;
      d->table = upload(d->mem, tab, s, &e);
    }
  }
  if (!e && d->var) {
    // primitive table: the largest argument is the largest window end,
    // c_s |k| T_w = min(|k| L, k_c L) <= min(pi N, max k_c L)
    const double Tmax = std::min(M_PI * (double)N, std::max(p->kcL[0], p->kcL[1]));
    const double h = 1.0 / 32.0;
    const int K = (int)std::ceil(Tmax / h) + 3;
    std::vector<double> tab(6 * (size_t)K);
    auto node = [&](int i) {
      long double PT, PN, CT, CN, dCT, dCN;
      const long double T = (long double)i * (long double)h;
      kernel_primitives(T, cs, cp, &PT, &PN);
      kernel_values(T, cs, cp, &CT, &CN, &dCT, &dCN);
      double* q = &tab[6 * (size_t)i];
      q[0] = (double)PT;
      q[1] = (double)CT;
      q[2] = (double)dCT;
      q[3] = (double)PN;
      q[4] = (double)CN;
      q[5] = (double)dCN;
    };
    for (int i = 0; i < K; ++i) node(i);
    d->ptab_len = K;
    d->ptab_h = h;
    d->ptab = upload(d->mem, tab, s, &e);
    // the log entries of every referenced interval survive the two entries
    // a rejected attempt writes
    d->tlog_cap = Rmax + 2;
    if (!e) {
      d->tlog = (double2*)d->mem.get(sizeof(double2) * d->tlog_cap);
      if (!d->tlog) e = hipErrorOutOfMemory;
      else e = hipMemsetAsync(d->tlog, 0, sizeof(double2) * d->tlog_cap, s);
    }
  }
  if (!e) e = hipStreamSynchronize(s);
  if (e) {
    delete d;
    return hip_fail(p, e, "building the weight tables");
  }
  *out = d;
  return SBIEM_OK;
}

int retile(sbiem_plan* p, int tile) {
  DtData* d = p->dtd;
  if (!d || d->var || p->precision != SBIEM_FP32CONV || d->tile_slots == tile) return SBIEM_OK;
  const int half = (int)(p->N / 2);
  const long double th_unit = 3.141592653589793238462643383279502884L * (long double)p->cs *
                              (long double)d->dt / (long double)p->L / (long double)kTableStep;
  const int parts = build_tiles(p, d, tile, th_unit);
  hipStream_t s = p->stream;
  hipError_t e = hipStreamSynchronize(s);
  if (!e && parts > d->parts_cap) {
    double4* np = (double4*)d->mem.get(sizeof(double4) * parts);
    if (!np) return fail(p, SBIEM_ENOMEM, "retile: partial sums");
    d->parts = np;
    d->parts_cap = parts;
  }
  if (!e) e = hipMemsetAsync(d->parts, 0, sizeof(double4) * d->parts_cap, s);
  for (int n = 1; n <= half; ++n) {
    ModeCoef& c = d->coef_host[mode_pos(n, p->log2P, p->log2Q)];
    c.part0 = d->part0[n];
    c.nparts = d->nparts[n];
  }
  if (!e)
    e = hipMemcpyAsync(d->coef, d->coef_host.data(), sizeof(ModeCoef) * d->coef_host.size(),
                       hipMemcpyHostToDevice, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(p, e, "retile");
  // the plan's own launch context holds the old tiles: rebuilt on next use
  delete p->exec;
  p->exec = nullptr;
  return refresh_desc(p);
}

void discarded_weights(double cs, double cp, double L, double dt, const std::vector<int>& n,
                       const std::vector<int>& Mk, const std::vector<int>& M, std::vector<double>* DT,
                       std::vector<double>* DN) {
  const size_t cnt = n.size();
  DT->assign(cnt, 0.0);
  DN->assign(cnt, 0.0);
  if (cnt == 0) return;
  // table coordinate of lag j: x = (2 j + 1) c_s |k_n| dt / (2 h)
  const long double th_unit = 3.141592653589793238462643383279502884L * (long double)cs *
                              (long double)dt / (long double)L / (long double)kTableStep;
  double xmax = 0.0;
  long long work = 0;
  for (size_t i = 0; i < cnt; ++i) {
    xmax = std::max(xmax, (double)(th_unit * n[i]) * (2.0 * M[i] + 1.0));
    work += std::max(0, M[i] - Mk[i]);
  }
  const int K = (int)std::ceil(xmax) + 3;
  std::vector<double> tab(4 * (size_t)K);
  for (int i = 0; i < K; ++i) {
    long double CT, CN, dCT, dCN;
    kernel_values((long double)i * kTableStep, cs, cp, &CT, &CN, &dCT, &dCN);
    tab[4 * i + 0] = (double)(dt * CT);
    tab[4 * i + 1] = (double)(dt * kTableStep * dCT);
    tab[4 * i + 2] = (double)(dt * CN);
    tab[4 * i + 3] = (double)(dt * kTableStep * dCN);
  }
  auto run = [&](size_t i0, size_t i1) {
    for (size_t i = i0; i < i1; ++i) {
      const double th = (double)(th_unit * n[i]);
      double sT = 0.0, sN = 0.0;
      for (int j = Mk[i]; j < M[i]; ++j) {
        const double x = (double)(2 * j + 1) * th;
        const int k = std::min((int)x, K - 2);
        const double f = x - (double)k, f2 = f * f, f3 = f2 * f;
        const double h00 = 2 * f3 - 3 * f2 + 1, h10 = f3 - 2 * f2 + f, h01 = 3 * f2 - 2 * f3,
                     h11 = f3 - f2;
        const double* a = &tab[4 * (size_t)k];
        sT += h00 * a[0] + h10 * a[1] + h01 * a[4] + h11 * a[5];
        sN += h00 * a[2] + h10 * a[3] + h01 * a[6] + h11 * a[7];
      }
      (*DT)[i] = sT;
      (*DN)[i] = sN;
    }
  };
  const int nth = work > (1 << 22) ? 8 : 1;
  if (nth == 1) {
    run(0, cnt);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back(run, cnt * t / nth, cnt * (t + 1) / nth);
  for (auto& th : pool) th.join();
}

int build_dyn_data(sbiem_plan* p, DynData** out) {
  *out = nullptr;
  DynData* d = new DynData();
  const size_t N = (size_t)p->N, M = (size_t)(p->N / 2 + 1);
  bool ok = true;
  auto el = [&](double** ptr) {
    *ptr = (double*)d->mem.get(N * sizeof(double));
    ok = ok && *ptr;
  };
  auto sp = [&](double2** ptr) {
    *ptr = (double2*)d->mem.get(M * sizeof(double2));
    ok = ok && *ptr;
  };
  for (int k = 0; k < 2; ++k) {
    el(&d->slip[k]);
    el(&d->V[k]);
    el(&d->theta[k]);
    el(&d->thd[k]);
    el(&d->tau_el[k]);
    el(&d->sigma_el[k]);
  }
  el(&d->V1);
  el(&d->thd1);
  sp(&d->u_hat);
  sp(&d->g_hat);
  sp(&d->v_hat0);
  sp(&d->gv_hat0);
  sp(&d->v_hat1);
  sp(&d->gv_hat1);
  sp(&d->hprev_v);
  sp(&d->hprev_g);
  sp(&d->B_T);
  sp(&d->B_N);
  // exchange buffers sized for FP64 complex (FP32 uses the first half)
  d->gI = d->mem.get(N * sizeof(double2));
  d->gF = d->mem.get(N * sizeof(double2));
  d->step = (long long*)d->mem.get(sizeof(long long) * 2);
  d->err = (int*)d->mem.get(sizeof(int) * 4);
  d->cells = (int*)d->mem.get(sizeof(int) * 8);
  d->done = d->cells + 6;
  ok = ok && d->gI && d->gF && d->step && d->err && d->cells;
  if (!ok) {
    delete d;
    return fail(p, SBIEM_ENOMEM, "device allocation of the state buffers failed");
  }
  d->err_count = d->err + 1;
  d->err_index = d->err + 2;
  hipStream_t s = p->stream;
  hipError_t e = hipSuccess;
  // zero everything that is read before being written
  for (int k = 0; k < 2 && !e; ++k) {
    e = hipMemsetAsync(d->tau_el[k], 0, N * sizeof(double), s);
    if (!e) e = hipMemsetAsync(d->sigma_el[k], 0, N * sizeof(double), s);
  }
  double2* spec[] = {d->u_hat, d->g_hat, d->v_hat0, d->gv_hat0, d->v_hat1, d->gv_hat1,
                     d->hprev_v, d->hprev_g, d->B_T, d->B_N};
  for (double2* q : spec)
    if (!e) e = hipMemsetAsync(q, 0, M * sizeof(double2), s);
  if (!e) e = hipMemsetAsync(d->step, 0, sizeof(long long) * 2, s);
  if (!e) e = hipMemsetAsync(d->cells, 0, sizeof(int) * 8, s);
  const int init[4] = {0, 0, 0x7fffffff, 0};
  if (!e) e = hipMemcpyAsync(d->err, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) {
    delete d;
    return hip_fail(p, e, "initialising the state buffers");
  }
  *out = d;
  return SBIEM_OK;
}

FaultDev make_fault_desc(sbiem_plan* p, DtData* dtd, DynData* dyn, double V_pl, double t0) {
  FaultDev f;
  std::memset(&f, 0, sizeof(f));
  f.N = (int)p->N;
  f.log2N = p->log2N;
  f.nmodes = (int)(p->N / 2);
  f.log2P = p->log2P;
  f.log2Q = p->log2Q;
  f.P = 1 << p->log2P;
  f.Q = 1 << p->log2Q;
  f.ngroups = std::max(1, f.P / 2);
  f.ncls = p->ncls;
  f.theta_mode = p->theta_mode;
  f.newton_max = p->newton_max;
  f.L = p->L;
  f.mu = p->mu;
  f.r = p->r;
  f.cs = p->cs;
  f.dt = dtd ? dtd->dt : 0.0;
  f.eta_rad = p->mu / (2.0 * p->cs);
  f.V_pl = V_pl;
  f.Dc = p->Dc;
  f.V_ref = p->V_ref;
  f.f0 = p->f0;
  f.tau_rate = p->tau_rate;
  f.t0 = t0;
  f.ln_V_ref = p->V_ref > 0 ? std::log(p->V_ref) : 0.0;
  f.a = p->a;
  f.b = p->b;
  f.sigma_load = p->sigma_load;
  f.tau_load = p->tau_load;
  f.kappa = p->kappa;
  for (int k = 0; k < 2; ++k) {
    f.slip[k] = dyn->slip[k];
    f.V[k] = dyn->V[k];
    f.theta[k] = dyn->theta[k];
    f.thd[k] = dyn->thd[k];
    f.tau_el[k] = dyn->tau_el[k];
    f.sigma_el[k] = dyn->sigma_el[k];
  }
  f.V1 = dyn->V1;
  f.thd1 = dyn->thd1;
  f.u_hat = dyn->u_hat;
  f.g_hat = dyn->g_hat;
  f.v_hat0 = dyn->v_hat0;
  f.gv_hat0 = dyn->gv_hat0;
  f.v_hat1 = dyn->v_hat1;
  f.gv_hat1 = dyn->gv_hat1;
  f.hprev_v = dyn->hprev_v;
  f.hprev_g = dyn->hprev_g;
  f.B_T = dyn->B_T;
  f.B_N = dyn->B_N;
  f.fwd_scale = p->fwd_scale;
  f.gI = dyn->gI;
  f.gF = dyn->gF;
  f.cells = dyn->cells;
  f.done = dyn->done;
  if (dtd) {
    f.coef = dtd->coef;
    f.parts = dtd->parts;
    f.tails = dtd->tails;
    f.ring = dtd->ring;
    f.wrev = dtd->wrev;
  }
  f.twiddle = p->twiddle;
  f.kcT = p->kcL[0];
  f.kcN = p->kcL[1];
  if (dtd && dtd->var) {
    f.ptab = dtd->ptab;
    f.ptab_len = dtd->ptab_len;
    f.ptab_h = dtd->ptab_h;
    f.tlog = dtd->tlog;
    f.tlog_cap = dtd->tlog_cap;
  }
  f.step = dyn->step;
  f.err = dyn->err;
  f.err_count = dyn->err_count;
  f.err_index = dyn->err_index;
  return f;
}

}  // namespace sbiem

using namespace sbiem;

namespace {

int check_plan(sbiem_plan* p) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  return SBIEM_OK;
}

int ensure_device(sbiem_plan* p) {
  hipError_t e = hipSetDevice(p->device);
  if (e) return hip_fail(p, e, "hipSetDevice");
  return SBIEM_OK;
}

// Quarter-wave table cos(2 pi t / N), t = 0..N/4, in the convolution
// precision, and once in FP64 for the slip transforms of the set-up paths.
int upload_twiddles(sbiem_plan* p) {
  const int64_t N = p->N, Q = N / 4;
  std::vector<double> t64(Q + 1);
  std::vector<float> t32(Q + 1);
  for (int64_t t = 0; t <= Q; ++t) {
    long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)t / (long double)N;
    long double c = (t == Q) ? 0.0L : cosl(ang);
    t64[t] = (double)c;
    t32[t] = (float)c;
  }
  hipError_t e = hipSuccess;
  if (!p->twiddle64) p->twiddle64 = upload(p->mem, t64, p->stream, &e);
  if (p->precision == SBIEM_FP32CONV) p->twiddle = upload(p->mem, t32, p->stream, &e);
  else p->twiddle = p->twiddle64;
  if (!e) e = hipStreamSynchronize(p->stream);
  if (e) return hip_fail(p, e, "uploading twiddles");
  return SBIEM_OK;
}

}  // namespace

// Forward declarations of exec.cpp helpers
namespace sbiem {
int rebuild_exec(sbiem_plan* p);
int refresh_desc(sbiem_plan* p);
int reset_history(sbiem_plan* p);
int rebase_state(sbiem_plan* p);
int spectral_state_from_host(sbiem_plan* p, const double* slip, const double* V, double t);
int spectral_state_from_device(sbiem_plan* p);
}  // namespace sbiem

extern "C" {

int sbiem_abi_version(void) { return SBIEM_ABI_VERSION; }

const char* sbiem_status_string(int status) {
  switch (status) {
    case SBIEM_OK: return "SBIEM_OK";
    case SBIEM_EINVAL: return "SBIEM_EINVAL";
    case SBIEM_ENOMEM: return "SBIEM_ENOMEM";
    case SBIEM_EDEVICE: return "SBIEM_EDEVICE";
    case SBIEM_ENEWTON: return "SBIEM_ENEWTON";
    case SBIEM_ESTATE: return "SBIEM_ESTATE";
    case SBIEM_EOPEN: return "SBIEM_EOPEN";
    case SBIEM_ENOTREADY: return "SBIEM_ENOTREADY";
    default: return "unknown status";
  }
}

const char* sbiem_last_error(const sbiem_plan* p) {
  return p ? p->last_error.c_str() : g_last_error.c_str();
}

int sbiem_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail_global(SBIEM_EINVAL, "allocator: give both functions or neither");
  DeviceAllocator& a = allocator();
  a.alloc = alloc;
  a.release = release;
  a.ctx = ctx;
  return SBIEM_OK;
}

int sbiem_kernel_eval(double cs, double cp, const double* T, int64_t n, double* CT, double* CN,
                      double* dCT, double* dCN) {
  if (!(cs > 0) || !(cp > cs) || n < 0 || (n > 0 && !T))
    return fail_global(SBIEM_EINVAL, "kernel_eval: need 0 < cs < cp and T");
  for (int64_t i = 0; i < n; ++i) {
    if (!(T[i] >= 0) || !std::isfinite(T[i])) return fail_global(SBIEM_EINVAL, "kernel_eval: T must be finite and >= 0");
    long double a, b, c, d;
    kernel_values(T[i], cs, cp, &a, &b, &c, &d);
    if (CT) CT[i] = (double)a;
    if (CN) CN[i] = (double)b;
    if (dCT) dCT[i] = (double)c;
    if (dCN) dCN[i] = (double)d;
  }
  return SBIEM_OK;
}

int sbiem_plan_create(sbiem_plan** out, int64_t N, double L, double mu, double nu, double cs,
                      double cp, const double* h) {
  if (!out) return fail_global(SBIEM_EINVAL, "plan_create: NULL out");
  *out = nullptr;
  if (N < 8 || N > (1 << 22) || (N & (N - 1)))
    return fail_global(SBIEM_EINVAL, "plan_create: N must be a power of two in [8, 2^22]");
  if (!(L > 0) || !(mu > 0) || !(cs > 0) || !(cp > cs) || !std::isfinite(L) || !std::isfinite(mu) ||
      !std::isfinite(cp))
    return fail_global(SBIEM_EINVAL, "plan_create: need L, mu > 0 and 0 < cs < cp");
  if (!(nu > 0 && nu < 0.5)) return fail_global(SBIEM_EINVAL, "plan_create: need 0 < nu < 0.5");
  const double q = (cp * cp) / (cs * cs);
  const double nu_w = (q - 2.0) / (2.0 * (q - 1.0));
  if (std::fabs(nu - nu_w) > 1e-3) {
    std::ostringstream m;
    m << "plan_create: nu = " << nu << " inconsistent with cp/cs (nu = " << nu_w << ")";
    return fail_global(SBIEM_EINVAL, m.str());
  }
  if (h && !all_finite(h, N)) return fail_global(SBIEM_EINVAL, "plan_create: h must be finite");

  sbiem_plan* p = new sbiem_plan();
  hipError_t e = hipGetDevice(&p->device);
  if (e) {
    delete p;
    return fail_global(SBIEM_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  }
  p->N = N;
  p->log2N = 0;
  while ((int64_t(1) << p->log2N) < N) ++p->log2N;
  split_sizes(p->log2N, &p->log2P, &p->log2Q, &p->ncls);
  p->L = L;
  p->mu = mu;
  p->nu = nu;
  p->cs = cs;
  p->cp = cp;
  p->r = (cs * cs) / (cp * cp);
  p->kappa_host = curvature_host(h, N, L);
  {
    double kmax = 0.0;
    for (double k : p->kappa_host) kmax = std::max(kmax, std::fabs(k));
    p->fwd_scale = kmax > 0.0 ? std::ldexp(1.0, -std::ilogb(kmax)) : 1.0;
  }
  const size_t bytes = (size_t)N * sizeof(double);
  p->kappa = (double*)p->mem.get(bytes);
  p->a = (double*)p->mem.get(bytes);
  p->b = (double*)p->mem.get(bytes);
  p->sigma_load = (double*)p->mem.get(bytes);
  p->tau_load = (double*)p->mem.get(bytes);
  if (!p->kappa || !p->a || !p->b || !p->sigma_load || !p->tau_load) {
    delete p;
    return fail_global(SBIEM_ENOMEM, "plan_create: device allocation failed");
  }
  {
    std::vector<double> kp = to_elem_order(p, p->kappa_host.data());
    e = hipMemcpy(p->kappa, kp.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e) {
    delete p;
    return fail_global(SBIEM_EDEVICE, std::string("plan_create: ") + hipGetErrorString(e));
  }
  int st = upload_twiddles(p);
  if (st) {
    std::string m = p->last_error;
    delete p;
    return fail_global(st, m);
  }
  st = build_dyn_data(p, &p->dyn);
  if (!st) {
    p->d_desc = (FaultDev*)p->mem.get(sizeof(FaultDev));
    if (!p->d_desc) st = fail(p, SBIEM_ENOMEM, "plan_create: device allocation failed");
  }
  if (!st) st = refresh_desc(p);
  if (st) {
    std::string m = p->last_error;
    delete p;
    return fail_global(st, m);
  }
  *out = p;
  return SBIEM_OK;
}

int sbiem_plan_destroy(sbiem_plan* p) {
  if (!p) return SBIEM_OK;
  if (p->batch_refs > 0) return fail(p, SBIEM_EINVAL, "plan is still used by a batch");
  (void)hipSetDevice(p->device);
  (void)hipStreamSynchronize(p->stream);
  delete p->exec;
  delete p->dtd;
  delete p->dyn;
  delete p->snap;
  delete p;
  return SBIEM_OK;
}

int sbiem_set_precision(sbiem_plan* p, int mode) {
  if (int s = check_plan(p)) return s;
  if (mode != SBIEM_FP64 && mode != SBIEM_FP32CONV) return fail(p, SBIEM_EINVAL, "unknown precision");
  if (p->dtd) return fail(p, SBIEM_EINVAL, "precision must be chosen before the time step is set");
  if (mode == p->precision) return SBIEM_OK;
  if (int s = ensure_device(p)) return s;
  p->precision = mode;
  if (int st = upload_twiddles(p)) return st;
  return refresh_desc(p);
}

int sbiem_set_theta_mode(sbiem_plan* p, int mode) {
  if (int s = check_plan(p)) return s;
  if (mode != SBIEM_THETA_PAPER && mode != SBIEM_THETA_EXP) return fail(p, SBIEM_EINVAL, "unknown theta mode");
  p->theta_mode = mode;
  return refresh_desc(p);
}

int sbiem_set_rule(sbiem_plan* p, int rule) {
  if (int s = check_plan(p)) return s;
  if (rule != SBIEM_RULE_MIDPOINT && rule != SBIEM_RULE_INTERVAL)
    return fail(p, SBIEM_EINVAL, "set_rule: unknown rule");
  if (p->dtd) return fail(p, SBIEM_EINVAL, "set_rule: the rule must be chosen before the time step");
  if (p->adaptive && rule != SBIEM_RULE_INTERVAL)
    return fail(p, SBIEM_EINVAL, "set_rule: variable steps use the interval rule");
  if (p->closure_on && rule != SBIEM_RULE_MIDPOINT)
    return fail(p, SBIEM_EINVAL, "set_rule: the learned closure uses the midpoint rule");
  p->rule = rule;
  return SBIEM_OK;
}

int sbiem_set_cutoffs(sbiem_plan* p, double kcL_shear, double kcL_normal) {
  if (int s = check_plan(p)) return s;
  if (!(kcL_shear >= 1.0 && kcL_shear <= 1e6) || !(kcL_normal >= 1.0 && kcL_normal <= 1e6))
    return fail(p, SBIEM_EINVAL, "set_cutoffs: need 1 <= k_c L <= 1e6");
  if (p->dtd) return fail(p, SBIEM_EINVAL, "set_cutoffs: the cut-offs must be chosen before the time step");
  if (p->closure_on && kcL_shear != kcL_normal)
    return fail(p, SBIEM_EINVAL, "set_cutoffs: the learned closure needs equal cut-offs");
  p->kcL[0] = kcL_shear;
  p->kcL[1] = kcL_normal;
  return refresh_desc(p);
}

int sbiem_set_adaptive(sbiem_plan* p, int on) {
  if (int s = check_plan(p)) return s;
  if (p->dtd) return fail(p, SBIEM_EINVAL, "set_adaptive: must precede the time step");
  if (on && p->closure_on) return fail(p, SBIEM_EINVAL, "set_adaptive: not with the learned closure");
  if (on && p->batch_refs > 0) return fail(p, SBIEM_EINVAL, "set_adaptive: plan is used by a batch");
  p->adaptive = on != 0;
  if (p->adaptive) p->rule = SBIEM_RULE_INTERVAL;
  return SBIEM_OK;
}

int sbiem_kernel_primitive_eval(double cs, double cp, const double* T, int64_t n, double* PT,
                                double* PN) {
  if (!(cs > 0) || !(cp > cs) || n < 0 || (n > 0 && !T))
    return fail_global(SBIEM_EINVAL, "kernel_primitive_eval: need 0 < cs < cp and T");
  for (int64_t i = 0; i < n; ++i) {
    if (!(T[i] >= 0) || !std::isfinite(T[i]))
      return fail_global(SBIEM_EINVAL, "kernel_primitive_eval: T must be finite and >= 0");
    long double a, b;
    kernel_primitives(T[i], cs, cp, &a, &b);
    if (PT) PT[i] = (double)a;
    if (PN) PN[i] = (double)b;
  }
  return SBIEM_OK;
}

int sbiem_set_conv_tile(sbiem_plan* p, int records) {
  if (int s = check_plan(p)) return s;
  if (records != 0 && records != kTileSlots32s && records != kTileSlots32 &&
      records != kTileSlots32l && records != kTileSlots32p && records != kTileSlots32w)
    return fail(p, SBIEM_EINVAL, "set_conv_tile: records must be 0, 64, 256, 320, 512 or 1024");
  if (p->batch_refs > 0) return fail(p, SBIEM_EINVAL, "set_conv_tile: plan is used by a batch");
  p->conv_tile = records;
  p->conv_tile_set = records != 0;
  if (!p->dtd || p->dtd->var || p->precision != SBIEM_FP32CONV) return SBIEM_OK;
  const int tile = records ? records : (p->closure_on ? kTileSlots32s : kTileSlots32);
  if (tile == p->dtd->tile_slots) return SBIEM_OK;
  if (int st = retile(p, tile)) return st;
  if (p->dyn) p->dyn->primed = false;
  return SBIEM_OK;
}

int sbiem_get_conv_tile(const sbiem_plan* p, int* records) {
  if (!p || !records) return fail_global(SBIEM_EINVAL, "get_conv_tile: NULL argument");
  if (p->dtd && !p->dtd->var && p->precision == SBIEM_FP32CONV) *records = p->dtd->tile_slots;
  else if (p->precision == SBIEM_FP32CONV)
    *records = p->conv_tile ? p->conv_tile : (p->closure_on ? kTileSlots32s : kTileSlots32);
  else
    *records = kTileSlots64;
  return SBIEM_OK;
}

int sbiem_set_newton_limit(sbiem_plan* p, int max_iterations) {
  if (int s = check_plan(p)) return s;
  if (max_iterations < 0 || max_iterations > 1000)
    return fail(p, SBIEM_EINVAL, "set_newton_limit: need 0 <= max_iterations <= 1000");
  p->newton_max = max_iterations == 0 ? 100 : max_iterations;
  return refresh_desc(p);
}

int sbiem_set_friction(sbiem_plan* p, const double* a, const double* b, double Dc, double V_ref,
                       double f0, const double* sigma_load, const double* tau_load,
                       double tau_load_rate, double V_pl) {
  if (int s = check_plan(p)) return s;
  const int64_t N = p->N;
  if (!a || !b || !sigma_load || !tau_load) return fail(p, SBIEM_EINVAL, "set_friction: NULL array");
  if (!all_finite(a, N) || !all_finite(b, N) || !all_finite(sigma_load, N) || !all_finite(tau_load, N))
    return fail(p, SBIEM_EINVAL, "set_friction: arrays must be finite");
  for (int64_t i = 0; i < N; ++i)
    if (!(a[i] > 0)) return fail(p, SBIEM_EINVAL, "set_friction: a must be > 0");
  if (!(Dc > 0) || !(V_ref > 0) || !std::isfinite(f0) || !std::isfinite(tau_load_rate) ||
      !(V_pl >= 0) || !std::isfinite(Dc) || !std::isfinite(V_ref) || !std::isfinite(V_pl))
    return fail(p, SBIEM_EINVAL, "set_friction: need Dc, V_ref > 0, V_pl >= 0, finite f0 and rate");
  if (int s = ensure_device(p)) return s;
  const size_t bytes = (size_t)N * sizeof(double);
  hipError_t e = hipStreamSynchronize(p->stream);
  {
    std::vector<double> x = to_elem_order(p, a);
    if (!e) e = hipMemcpy(p->a, x.data(), bytes, hipMemcpyHostToDevice);
    x = to_elem_order(p, b);
    if (!e) e = hipMemcpy(p->b, x.data(), bytes, hipMemcpyHostToDevice);
    x = to_elem_order(p, sigma_load);
    if (!e) e = hipMemcpy(p->sigma_load, x.data(), bytes, hipMemcpyHostToDevice);
    x = to_elem_order(p, tau_load);
    if (!e) e = hipMemcpy(p->tau_load, x.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e) return hip_fail(p, e, "set_friction");
  p->a_host.assign(a, a + N);
  if (!p->constrained.empty()) p->state_set = false;  // its V_pl elements become free
  p->constrained.clear();
  p->Dc = Dc;
  p->V_ref = V_ref;
  p->f0 = f0;
  p->tau_rate = tau_load_rate;
  const bool reframe = p->state_set && V_pl != p->V_pl;
  p->V_pl = V_pl;
  p->friction_set = true;
  if (int st = refresh_desc(p)) return st;
  // the spectral state is kept in the backslip frame of V_pl
  if (reframe) return spectral_state_from_device(p);
  return SBIEM_OK;
}

int sbiem_set_constrained(sbiem_plan* p, const uint8_t* mask) {
  if (int s = check_plan(p)) return s;
  if (!p->friction_set) return fail(p, SBIEM_ENOTREADY, "set_constrained: set_friction first");
  const int64_t N = p->N;
  std::vector<uint8_t> m;
  if (mask) {
    m.assign(mask, mask + N);
    bool any = false;
    for (uint8_t& x : m) any = any || (x = x != 0);
    if (!any) m.clear();
  }
  if (int s = ensure_device(p)) return s;
  // the device copy of a carries the mask as its sign
  std::vector<double> a = p->a_host;
  for (size_t i = 0; i < m.size(); ++i)
    if (m[i]) a[i] = -a[i];
  std::vector<double> x = to_elem_order(p, a.data());
  hipError_t e = hipStreamSynchronize(p->stream);
  if (!e) e = hipMemcpy(p->a, x.data(), (size_t)N * sizeof(double), hipMemcpyHostToDevice);
  if (e) return hip_fail(p, e, "set_constrained");
  p->constrained = std::move(m);
  p->state_set = false;
  return SBIEM_OK;
}

int sbiem_set_state(sbiem_plan* p, const double* slip, const double* V_in, const double* theta,
                    double t) {
  if (int s = check_plan(p)) return s;
  if (!p->friction_set) return fail(p, SBIEM_ENOTREADY, "set_state: set_friction first");
  const int64_t N = p->N;
  if (!slip || !V_in || !theta) return fail(p, SBIEM_EINVAL, "set_state: NULL array");
  if (!all_finite(slip, N) || !all_finite(V_in, N) || !all_finite(theta, N) || !std::isfinite(t))
    return fail(p, SBIEM_EINVAL, "set_state: values must be finite");
  const bool held = !p->constrained.empty();
  for (int64_t i = 0; i < N; ++i)
    if ((!(V_in[i] > 0) && !(held && p->constrained[i])) || !(theta[i] > 0))
      return fail(p, SBIEM_EINVAL, "set_state: V and theta must be > 0");
  if (int s = ensure_device(p)) return s;
  // constrained elements slide at V_pl with a frozen state
  std::vector<double> Vh(V_in, V_in + N);
  std::vector<double> thd(N);
  for (int64_t i = 0; i < N; ++i) {
    if (held && p->constrained[i]) Vh[i] = p->V_pl;
    thd[i] = (held && p->constrained[i]) ? 0.0 : 1.0 - theta[i] * Vh[i] / p->Dc;
  }
  const double* V = Vh.data();
  DynData* d = p->dyn;
  const size_t bytes = (size_t)N * sizeof(double);
  hipStream_t s = p->stream;
  hipError_t e = hipStreamSynchronize(s);
  {
    // both buffers of the double-buffered state get the initial state (the
    // other buffer stands for the step before the first one)
    const double* host[4] = {slip, V, theta, thd.data()};
    double* const* dev[4] = {d->slip, d->V, d->theta, d->thd};
    for (int k = 0; k < 4 && !e; ++k) {
      std::vector<double> x = to_elem_order(p, host[k]);
      e = hipMemcpy(dev[k][0], x.data(), bytes, hipMemcpyHostToDevice);
      if (!e) e = hipMemcpy(dev[k][1], x.data(), bytes, hipMemcpyHostToDevice);
    }
  }
  for (int k = 0; k < 2 && !e; ++k) {
    e = hipMemsetAsync(d->tau_el[k], 0, bytes, s);
    if (!e) e = hipMemsetAsync(d->sigma_el[k], 0, bytes, s);
  }
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(p, e, "set_state");
  p->t0 = t;
  p->t_var = t;
  p->var_accepted = 0;
  p->state_set = true;
  p->last_fail_count = 0;
  p->last_fail_index = -1;
  if (int st = reset_history(p)) return st;
  return spectral_state_from_host(p, slip, V, t);
}

int sbiem_get_state(sbiem_plan* p, double* slip, double* V, double* theta, double* tau_el,
                    double* sigma_el, double* t) {
  if (int s = check_plan(p)) return s;
  if (!p->state_set) return fail(p, SBIEM_ENOTREADY, "get_state: no state set");
  if (int s = ensure_device(p)) return s;
  DynData* d = p->dyn;
  long long step = 0;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (!e) e = hipMemcpy(&step, d->step, sizeof(step), hipMemcpyDeviceToHost);
  if (e) return hip_fail(p, e, "get_state");
  const int cur = (int)(step & 1);
  const double* src[5] = {d->slip[cur], d->V[cur], d->theta[cur], d->tau_el[cur], d->sigma_el[cur]};
  double* dst[5] = {slip, V, theta, tau_el, sigma_el};
  for (int k = 0; k < 5 && !e; ++k)
    if (dst[k]) e = download_elems(p, src[k], dst[k]);
  if (e) return hip_fail(p, e, "get_state");
  if (t) *t = (p->dtd && p->dtd->var) ? p->t_var : p->t0 + (double)step * (p->dtd ? p->dtd->dt : 0.0);
  return SBIEM_OK;
}

int sbiem_get_curvature(const sbiem_plan* p, double* kappa) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (!kappa) return fail(const_cast<sbiem_plan*>(p), SBIEM_EINVAL, "NULL kappa");
  std::memcpy(kappa, p->kappa_host.data(), (size_t)p->N * sizeof(double));
  return SBIEM_OK;
}

int sbiem_window_lengths(const sbiem_plan* p, double dt, int64_t* M) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (!(dt > 0) || !M) return fail(const_cast<sbiem_plan*>(p), SBIEM_EINVAL, "window_lengths: need dt > 0");
  std::vector<int> m = window_steps(p->N, p->L, p->cs, dt, std::max(p->kcL[0], p->kcL[1]));
  for (int64_t n = 1; n <= p->N / 2; ++n) M[n - 1] = m[n];
  return SBIEM_OK;
}

int sbiem_set_dt(sbiem_plan* p, double dt) {
  if (int s = check_plan(p)) return s;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(p, SBIEM_EINVAL, "set_dt: need dt > 0");
  if (int s = ensure_device(p)) return s;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e) return hip_fail(p, e, "set_dt");
  // keep the current state: move it to buffer 0 at t0 = current time
  if (p->state_set && p->dtd) {
    if (int st = rebase_state(p)) return st;
  }
  DtData* d = nullptr;
  if (int s = build_dt_data(p, dt, &d)) return s;
  delete p->exec;
  p->exec = nullptr;
  delete p->dtd;
  p->dtd = d;
  if (int st = rebuild_exec(p)) return st;
  if (int st = reset_history(p)) return st;
  if (p->state_set) return spectral_state_from_device(p);
  return SBIEM_OK;
}

int sbiem_set_closure(sbiem_plan* p, const float* params_shear, const float* params_normal,
                      double cut) {
  if (int s = check_plan(p)) return s;
  const bool on = params_shear != nullptr;
  if (on != (params_normal != nullptr))
    return fail(p, SBIEM_EINVAL, "set_closure: give both networks or neither");
  if (on && p->precision != SBIEM_FP32CONV)
    return fail(p, SBIEM_EINVAL, "set_closure: the closure runs with SBIEM_FP32CONV");
  if (on && !(cut > 0.0 && cut < 1.0)) return fail(p, SBIEM_EINVAL, "set_closure: need 0 < cut < 1");
  if (on && (p->adaptive || p->rule != SBIEM_RULE_MIDPOINT || p->kcL[0] != p->kcL[1]))
    return fail(p, SBIEM_EINVAL,
                "set_closure: needs fixed steps, the midpoint rule and equal cut-offs");
  if (p->batch_refs > 0) return fail(p, SBIEM_EINVAL, "set_closure: plan is used by a batch");
  if (on) {
    for (int k = 0; k < 2; ++k) {
      const float* src = k ? params_normal : params_shear;
      for (int i = 0; i < kClosureParams; ++i)
        if (!std::isfinite(src[i])) return fail(p, SBIEM_EINVAL, "set_closure: parameters must be finite");
    }
  }
  if (int s = ensure_device(p)) return s;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e) return hip_fail(p, e, "set_closure");
  p->closure_mem.release_all();
  p->net_frag[0] = p->net_frag[1] = nullptr;
  p->net_bias[0] = p->net_bias[1] = nullptr;
  p->closure_on = on;
  if (on) {
    p->closure_cut = cut;
    for (int k = 0; k < 2; ++k) {
      const float* src = k ? params_normal : params_shear;
      p->closure_params[k].assign(src, src + kClosureParams);
      std::vector<unsigned short> frag;
      std::vector<float> bias;
      closure_pack(src, &frag, &bias);
      p->net_frag[k] = p->closure_mem.get(frag.size() * sizeof(unsigned short));
      p->net_bias[k] = (float*)p->closure_mem.get(bias.size() * sizeof(float));
      if (!p->net_frag[k] || !p->net_bias[k]) return fail(p, SBIEM_ENOMEM, "set_closure: device allocation failed");
      e = hipMemcpy(p->net_frag[k], frag.data(), frag.size() * sizeof(unsigned short), hipMemcpyHostToDevice);
      if (!e) e = hipMemcpy(p->net_bias[k], bias.data(), bias.size() * sizeof(float), hipMemcpyHostToDevice);
      if (e) return hip_fail(p, e, "set_closure");
    }
  } else {
    p->closure_params[0].clear();
    p->closure_params[1].clear();
  }
  if (!p->dtd) return refresh_desc(p);
  // new window lengths: rebuild the tables and ring like a new dt (the state
  // is kept, the history restarts)
  return sbiem_set_dt(p, p->dtd->dt);
}

int sbiem_set_stream(sbiem_plan* p, void* hip_stream) {
  if (int s = check_plan(p)) return s;
  (void)hipStreamSynchronize(p->stream);
  p->stream = (hipStream_t)hip_stream;
  if (p->exec) p->exec->drop_graph();
  return SBIEM_OK;
}

}  // extern "C"

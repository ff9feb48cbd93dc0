// Execution contexts of libsbiem: launch sequences of the two-pass step for
// one fault or a batch of faults, HIP-graph replay, failure reporting,
// per-launch timing and the stress-only path.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <utility>

#include "internal.h"

namespace sbiem {

namespace {
constexpr int kGraphSteps = 16;  // steps captured in one replayable graph
constexpr int kProfileGraphs = 2;  // graphs replayed between two evented steps
}

Exec::~Exec() {
  drop_graph();
  if (aux) (void)hipStreamDestroy(aux);
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
}

hipError_t EventPool::ensure(size_t n) {
  while (ev.size() < n) {
    hipEvent_t x = nullptr;
    hipError_t e = hipEventCreate(&x);
    if (e) return e;
    ev.push_back(x);
  }
  return hipSuccess;
}

EventPool::~EventPool() {
  for (hipEvent_t x : ev) (void)hipEventDestroy(x);
}

void Exec::drop_graph() {
  if (graph) (void)hipGraphExecDestroy(graph);
  if (graph_def) (void)hipGraphDestroy(graph_def);
  graph = nullptr;
  graph_def = nullptr;
  graph_steps = 0;
}

int build_exec(const std::vector<sbiem_plan*>& plans, const std::vector<DtData*>& dts,
               const std::vector<DynData*>& dyns, const std::vector<FaultDev>& descs,
               int precision, Exec** out, std::string* err) {
  *out = nullptr;
  Exec* ex = new Exec();
  ex->dyns = dyns;
  ex->precision = precision;
  ex->nfaults = (int)plans.size();
  ex->host_faults = descs;
  std::vector<Tile> tiles;
  std::vector<RowDesc> rows;   // packed FP32 layout: what the conv reads instead of tiles
  std::vector<ConvTask> tasks;
  std::vector<int2> mmap, emap;
  std::vector<ClosureMode> cmodes;
  for (sbiem_plan* p : plans) {
    if (p->closure_on != plans[0]->closure_on ||
        (p->closure_on && (p->closure_params[0] != plans[0]->closure_params[0] ||
                           p->closure_params[1] != plans[0]->closure_params[1] ||
                           p->closure_cut != plans[0]->closure_cut))) {
      *err = "batch members must share the closure setting and networks";
      delete ex;
      return SBIEM_EINVAL;
    }
  }
  if (plans.size() > 1) {
    for (sbiem_plan* p : plans)
      if (var_engine(p)) {
        *err = "plans on the variable-step engine cannot be batched";
        delete ex;
        return SBIEM_EINVAL;
      }
  }
  double bytes = 0.0;
  const double rec = precision == SBIEM_FP32CONV ? 16.0 : 32.0;
  for (int f = 0; f < ex->nfaults; ++f) {
    DtData* d = dts[f];
    const int base = (int)tiles.size();
    const size_t rec_bytes = precision == SBIEM_FP32CONV ? 16 : 32;
    for (Tile t : d->tiles) {
      t.fault = f;
      t.rec = (const char*)d->ring + (size_t)t.ring_off * rec_bytes;
      tiles.push_back(t);
    }
    if (d->tile_slots == kTileSlots32p && precision == SBIEM_FP32CONV && !d->var)
      for (size_t i = 0; i < d->tiles.size(); ++i) {
        const Tile& t = d->tiles[i];
        const int2 m = d->row_meta[i];
        RowDesc r;
        r.rec = (const char*)d->ring + ((size_t)t.ring_off + (size_t)t.p0) * rec_bytes;
        r.word = (unsigned)t.len | (unsigned)(m.x + 1) << 8 | (unsigned)m.y << 16;
        r.p0 = t.p0;
        r.Rn = t.Rn;
        r.MT = t.MT;
        r.MN = t.MN;
        r.part = t.part;
        r.th = t.th;
        r.rmagic = t.rmagic;
        rows.push_back(r);
      }
    for (ConvTask k : d->tasks) tasks.push_back(ConvTask{k.t0 + base, k.t1 + base, f, k.nsum});
    // algorithmic bytes: ring records of lags 2..M_n-1 read, one history sum
    // (2 complex FP64) written per mode
    // (variable-step engine: every slot of R_n, plus the interval log, once
    // every slot holds an interval inside its window)
    const bool var = d->var;
    for (size_t n = 1; n < d->Rn.size(); ++n)
      if (d->Rn[n] > 1) bytes += rec * (d->Rn[n] - (var ? 0 : 1)) + 32.0;
    if (var) bytes += 16.0 * d->tlog_cap;
    for (ClosureMode c : d->closure) {
      c.fault = f;
      cmodes.push_back(c);
    }
    const FaultDev& fd = descs[f];
    for (int g = 0; g < fd.ngroups; ++g) mmap.push_back(make_int2(f, g));
    for (int b = 0; b < fd.Q; b += fd.ncls) emap.push_back(make_int2(f, b));
    ex->mode_lds = std::max(ex->mode_lds, mode_lds_bytes(precision, fd.log2Q));
    ex->elem_lds = std::max(ex->elem_lds, elem_lds_bytes(precision, fd.log2P, fd.ncls));
    if (precision == SBIEM_FP32CONV) {
      if (d->table_len > ex->table_len) {
        ex->table_len = d->table_len;
        ex->table = d->table;
      }
    }
  }
  if (precision == SBIEM_FP32CONV) {
    ex->tile_rows = dts[0]->tile_slots / 64;
    for (int f = 1; f < ex->nfaults; ++f)
      if (dts[f]->tile_slots != dts[0]->tile_slots) {
        *err = "FP32 batch members must share the conv tile size (closure setting)";
        delete ex;
        return SBIEM_EINVAL;
      }
  }
  if (precision == SBIEM_FP32CONV && ex->nfaults > 1) {
    // all faults must share the table (same dt, c_s, c_p)
    for (int f = 0; f < ex->nfaults; ++f) {
      sbiem_plan* p = plans[f];
      sbiem_plan* q = plans[0];
      if (dts[f]->dt != dts[0]->dt || p->cs != q->cs || p->cp != q->cp) {
        *err = "FP32 batch members must share dt, cs and cp";
        delete ex;
        return SBIEM_EINVAL;
      }
    }
  }
  if (!rows.empty())
    for (size_t k = 0; k < tasks.size(); ++k)
      if (tasks[k].t0 != (int)k * kTaskRows || tasks[k].t1 != tasks[k].t0 + kTaskRows) {
        *err = "packed conv rows: every task must hold 128 rows in order";
        delete ex;
        return SBIEM_EINVAL;
      }
  ex->ntiles = (int)tiles.size();
  ex->ntasks = (int)tasks.size();
  ex->mode_blocks = (int)mmap.size();
  ex->elem_blocks = (int)emap.size();
  ex->conv_bytes = bytes;
  ex->conv_grid = conv_grid_size(precision, ex->ntasks, ex->table_len, default_conv_reserve(ex->conv_bytes));
  ex->d_faults = (FaultDev*)ex->mem.get(sizeof(FaultDev) * ex->nfaults);
  ex->d_tiles = (Tile*)ex->mem.get(sizeof(Tile) * std::max(1, ex->ntiles));
  ex->d_tasks = (ConvTask*)ex->mem.get(sizeof(ConvTask) * std::max(1, ex->ntasks));
  ex->d_mode_map = (int2*)ex->mem.get(sizeof(int2) * std::max(1, ex->mode_blocks));
  ex->d_elem_map = (int2*)ex->mem.get(sizeof(int2) * std::max(1, ex->elem_blocks));
  ex->conv_ctr = (int*)ex->mem.get(sizeof(int) * 2);
  if (plans[0]->closure_on && !cmodes.empty()) {
    ex->nclosure = (int)cmodes.size();
    ex->closure_modes = (ClosureMode*)ex->mem.get(sizeof(ClosureMode) * cmodes.size());
    for (int k = 0; k < 2; ++k) {
      ex->net_frag[k] = plans[0]->net_frag[k];
      ex->net_bias[k] = plans[0]->net_bias[k];
    }
    if (ex->closure_modes &&
        hipMemcpy(ex->closure_modes, cmodes.data(), sizeof(ClosureMode) * cmodes.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
      *err = "uploading the closed modes failed";
      delete ex;
      return SBIEM_EDEVICE;
    }
  }
  if (!ex->d_faults || !ex->d_tiles || !ex->d_tasks || !ex->d_mode_map || !ex->d_elem_map ||
      !ex->conv_ctr || (ex->nclosure && !ex->closure_modes)) {
    *err = "device allocation of the execution context failed";
    delete ex;
    return SBIEM_ENOMEM;
  }
  hipError_t e = hipMemcpy(ex->d_faults, ex->host_faults.data(), sizeof(FaultDev) * ex->nfaults,
                           hipMemcpyHostToDevice);
  static_assert(sizeof(RowDesc) <= sizeof(Tile), "packed rows fit the tile buffer");
  if (!e && ex->ntiles && !rows.empty())
    e = hipMemcpy(ex->d_tiles, rows.data(), sizeof(RowDesc) * rows.size(), hipMemcpyHostToDevice);
  else if (!e && ex->ntiles)
    e = hipMemcpy(ex->d_tiles, tiles.data(), sizeof(Tile) * ex->ntiles, hipMemcpyHostToDevice);
  if (!e && ex->ntasks)
    e = hipMemcpy(ex->d_tasks, tasks.data(), sizeof(ConvTask) * ex->ntasks, hipMemcpyHostToDevice);
  if (!e)
    e = hipMemcpy(ex->d_mode_map, mmap.data(), sizeof(int2) * ex->mode_blocks, hipMemcpyHostToDevice);
  if (!e)
    e = hipMemcpy(ex->d_elem_map, emap.data(), sizeof(int2) * ex->elem_blocks, hipMemcpyHostToDevice);
  if (!e) e = hipMemset(ex->conv_ctr, 0, sizeof(int) * 2);
  if (!e) e = setup_kernel_attributes(precision);
  if (!e) e = hipStreamCreateWithFlags(&ex->aux, hipStreamNonBlocking);
  if (!e) e = hipEventCreateWithFlags(&ex->fork, hipEventDisableTiming);
  if (!e) e = hipEventCreateWithFlags(&ex->join, hipEventDisableTiming);
  if (e) {
    *err = std::string("building the execution context: ") + hipGetErrorString(e);
    delete ex;
    return SBIEM_EDEVICE;
  }
  *out = ex;
  return SBIEM_OK;
}

int refresh_desc(sbiem_plan* p) {
  FaultDev f = make_fault_desc(p, p->dtd, p->dyn, p->V_pl, p->t0);
  hipError_t e = hipSetDevice(p->device);
  if (!e) e = hipStreamSynchronize(p->stream);
  if (!e) e = hipMemcpy(p->d_desc, &f, sizeof(f), hipMemcpyHostToDevice);
  if (e) return hip_fail(p, e, "updating the fault descriptor");
  if (p->exec) {
    p->exec->host_faults[0] = f;
    e = hipMemcpy(p->exec->d_faults, &f, sizeof(f), hipMemcpyHostToDevice);
    if (e) return hip_fail(p, e, "updating the fault descriptor");
  }
  return SBIEM_OK;
}

int rebuild_exec(sbiem_plan* p) {
  delete p->exec;
  p->exec = nullptr;
  if (!p->dtd) return SBIEM_OK;
  FaultDev f = make_fault_desc(p, p->dtd, p->dyn, p->V_pl, p->t0);
  std::string err;
  Exec* ex = nullptr;
  int st = build_exec({p}, {p->dtd}, {p->dyn}, {f}, p->precision, &ex, &err);
  if (st) return fail(p, st, err);
  p->exec = ex;
  return refresh_desc(p);
}

// step counter 0, no pending failure, empty history (zero ring and lag-1 record).
int reset_history(sbiem_plan* p) {
  DynData* d = p->dyn;
  hipStream_t s = p->stream;
  const size_t M = (size_t)(p->N / 2 + 1);
  hipError_t e = hipMemsetAsync(d->step, 0, sizeof(long long), s);
  const int init[3] = {0, 0, 0x7fffffff};
  if (!e) e = hipMemcpyAsync(d->err, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemsetAsync(d->hprev_v, 0, M * sizeof(double2), s);
  if (!e) e = hipMemsetAsync(d->hprev_g, 0, M * sizeof(double2), s);
  if (!e) e = hipMemsetAsync(d->cells, 0, sizeof(int) * 8, s);
  d->primed = false;
  if (!e && p->dtd) {
    const size_t rec = p->precision == SBIEM_FP32CONV ? 16 : 32;
    e = hipMemsetAsync(p->dtd->ring, 0, (size_t)std::max<long long>(p->dtd->ring_slots, 1) * rec, s);
    if (!e && p->dtd->tlog)
      e = hipMemsetAsync(p->dtd->tlog, 0, sizeof(double2) * p->dtd->tlog_cap, s);
  }
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(p, e, "resetting the history");
  p->var_b = -1;
  return SBIEM_OK;
}

// Move the committed state to buffer 0 with t0 = its time (dt about to change).
int rebase_state(sbiem_plan* p) {
  DynData* d = p->dyn;
  long long step = 0;
  hipError_t e = hipMemcpy(&step, d->step, sizeof(step), hipMemcpyDeviceToHost);
  if (e) return hip_fail(p, e, "rebase");
  const int cur = (int)(step & 1);
  const size_t bytes = (size_t)p->N * sizeof(double);
  if (cur == 1) {
    e = hipMemcpy(d->slip[0], d->slip[1], bytes, hipMemcpyDeviceToDevice);
    if (!e) e = hipMemcpy(d->V[0], d->V[1], bytes, hipMemcpyDeviceToDevice);
    if (!e) e = hipMemcpy(d->theta[0], d->theta[1], bytes, hipMemcpyDeviceToDevice);
    if (!e) e = hipMemcpy(d->thd[0], d->thd[1], bytes, hipMemcpyDeviceToDevice);
    if (!e) e = hipMemcpy(d->tau_el[0], d->tau_el[1], bytes, hipMemcpyDeviceToDevice);
    if (!e) e = hipMemcpy(d->sigma_el[0], d->sigma_el[1], bytes, hipMemcpyDeviceToDevice);
    if (e) return hip_fail(p, e, "rebase");
  }
  if (p->dtd && p->dtd->var) p->t0 = p->t_var;
  else p->t0 += (double)step * (p->dtd ? p->dtd->dt : 0.0);
  p->t_var = p->t0;
  e = hipMemset(d->step, 0, sizeof(long long));
  if (e) return hip_fail(p, e, "rebase");
  return SBIEM_OK;
}

// u_hat = F[slip - V_pl t], g_hat = F[kappa (slip - V_pl t)],
// v_hat0 = F[V - V_pl], gv_hat0 = F[kappa (V - V_pl)] from host arrays
// (natural element order).
// Forward transforms of slip (and rate) signals for the set-up paths, in
// FP64 whatever the convolution precision: the static term multiplies the
// slip spectrum by |k|, so FP32 rounding of a large slip would come back
// amplified at high wavenumbers.  An FP32 plan gets a descriptor copy that
// points at the FP64 twiddle table.
hipError_t forward_fp64(sbiem_plan* p, const FaultDev* d_desc, const FaultDev& h, const double* a,
                        double2* A, double2* B, int count, long long stride, void* gF, hipStream_t s,
                        DevArena& tmp) {
  if (p->precision == SBIEM_FP64) return launch_forward(d_desc, h, SBIEM_FP64, a, A, B, count, stride, gF, s);
  FaultDev h64 = h;
  h64.twiddle = p->twiddle64;
  FaultDev* d64 = (FaultDev*)tmp.get(sizeof(FaultDev));
  if (!d64 || !p->twiddle64) return hipErrorOutOfMemory;
  hipError_t e = hipStreamSynchronize(s);
  if (!e) e = hipMemcpy(d64, &h64, sizeof(FaultDev), hipMemcpyHostToDevice);
  if (!e) e = setup_kernel_attributes(SBIEM_FP64);
  if (!e) e = launch_forward(d64, h64, SBIEM_FP64, a, A, B, count, stride, gF, s);
  return e;
}

int spectral_state_from_host(sbiem_plan* p, const double* slip, const double* V, double t) {
  const int64_t N = p->N;
  std::vector<double> x(2 * N);
  for (int64_t i = 0; i < N; ++i) {
    x[i] = slip[i] - p->V_pl * t;
    x[N + i] = V[i] - p->V_pl;
  }
  DynData* d = p->dyn;
  hipStream_t s = p->stream;
  DevArena tmp;
  double* dx = (double*)tmp.get((size_t)2 * N * sizeof(double));
  void* gF = tmp.get((size_t)2 * N * sizeof(double2));
  double2* A = (double2*)tmp.get((size_t)2 * (N / 2 + 1) * sizeof(double2));
  double2* B = (double2*)tmp.get((size_t)2 * (N / 2 + 1) * sizeof(double2));
  if (!dx || !gF || !A || !B) return fail(p, SBIEM_ENOMEM, "spectral state: device allocation failed");
  const size_t M = (size_t)(N / 2 + 1);
  FaultDev h = make_fault_desc(p, p->dtd, d, p->V_pl, p->t0);
  hipError_t e = hipMemcpyAsync(dx, x.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice, s);
  if (!e) e = setup_kernel_attributes(p->precision);
  if (!e) e = forward_fp64(p, p->d_desc, h, dx, A, B, 2, (long long)M, gF, s, tmp);
  if (!e) e = hipMemcpyAsync(d->u_hat, A, M * sizeof(double2), hipMemcpyDeviceToDevice, s);
  if (!e) e = hipMemcpyAsync(d->g_hat, B, M * sizeof(double2), hipMemcpyDeviceToDevice, s);
  if (!e) e = hipMemcpyAsync(d->v_hat0, A + M, M * sizeof(double2), hipMemcpyDeviceToDevice, s);
  if (!e) e = hipMemcpyAsync(d->gv_hat0, B + M, M * sizeof(double2), hipMemcpyDeviceToDevice, s);
  if (!e) e = hipStreamSynchronize(s);
  d->primed = false;
  if (e) return hip_fail(p, e, "computing the spectral state");
  return SBIEM_OK;
}

int spectral_state_from_device(sbiem_plan* p) {
  const int64_t N = p->N;
  std::vector<double> slip(N), V(N);
  double t = 0.0;
  if (int st = sbiem_get_state(p, slip.data(), V.data(), nullptr, nullptr, nullptr, &t)) return st;
  return spectral_state_from_host(p, slip.data(), V.data(), t);
}

namespace {

// Record the failure flags read back from the device (status, failing
// elements, first failing element) and clear them there.
int note_failure(sbiem_plan* p, int status, int count, int index) {
  DynData* d = p->dyn;
  if (status == 0) {
    p->last_fail_count = 0;
    p->last_fail_index = -1;
    return SBIEM_OK;
  }
  p->last_fail_count = count;
  p->last_fail_index = index;
  d->primed = false;
  const int init[3] = {0, 0, 0x7fffffff};
  hipError_t e = hipMemcpy(d->err, init, sizeof(init), hipMemcpyHostToDevice);
  if (e) return hip_fail(p, e, "clearing the failure flag");
  const char* what = status == SBIEM_EOPEN ? "normal traction not compressive"
                     : status == SBIEM_ESTATE ? "state variable not positive"
                                              : "momentum balance did not converge";
  return fail(p, status, std::string("step failed: ") + what + " at element " + std::to_string(index));
}

int check_failure(sbiem_plan* p) {
  int h[3];
  hipError_t e = hipMemcpy(h, p->dyn->err, sizeof(h), hipMemcpyDeviceToHost);
  if (e) return hip_fail(p, e, "reading the failure flag");
  return note_failure(p, h[0], h[1], h[2]);
}

int ready(sbiem_plan* p, double dt) {
  if (!p->friction_set || !p->state_set)
    return fail(p, SBIEM_ENOTREADY, "set_friction and set_state must precede stepping");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(p, SBIEM_EINVAL, "dt must be > 0");
  if (!p->dtd) return sbiem_set_dt(p, dt);
  if (p->dtd->var) {
    const double hmin = p->adaptive ? 0.5 * p->dtd->dt : p->dtd->dt;
    if (dt < hmin * (1.0 - 1e-12))
      return fail(p, SBIEM_EINVAL, "dt is below the shortest interval the history is sized for");
    return SBIEM_OK;
  }
  if (dt != p->dtd->dt)
    return fail(p, SBIEM_EINVAL, "variable dt is not supported: dt differs from the plan's");
  return SBIEM_OK;
}

// ---------------------------------------------------------------------------
// Variable-step engine (section 3.2): a step of any length against the
// interval history, launched kernel by kernel: balance cells reset, history
// sums at the step's end time, pass-1 maxima and assembly, the two passes,
// the commit (which logs the interval's times).
// ---------------------------------------------------------------------------
// The launches of one step from t_old to t_new (no synchronisation; after a
// failure every later launch of the fault returns without effect until the
// flag is cleared).
// Algorithmic bytes of a variable-step conv launch ending at t_new from the
// host copy of the interval log: per mode, the stored intervals inside the
// longer of its two windows (their records are loaded), the log entries
// they touch, one partial sum written per mode.
double var_conv_bytes(const sbiem_plan* p, double t_new) {
  const DtData* d = p->dtd;
  if (p->var_b < 0 || p->var_tend.empty()) return 0.0;
  const long long cap = (long long)p->var_tend.size();
  const double rec = p->precision == SBIEM_FP32CONV ? 16.0 : 32.0;
  const double kc = std::max(p->kcL[0], p->kcL[1]);
  double bytes = 0.0;
  long long most = 0;
  for (size_t n = 1; n < d->Rn.size(); ++n) {
    const long long Rn = d->Rn[n];
    if (Rn <= 0) continue;
    const double kL = 2.0 * M_PI * (double)n;
    const double window = std::min(kL, kc) / (p->cs * kL / p->L);
    // the oldest interval that both the ring and the log still hold, then
    // the first one inside the window (end times increase with l)
    long long lo = std::max(0LL, p->var_b - std::min(Rn, cap) + 1), hi = p->var_b + 1;
    while (lo < hi) {
      const long long mid = (lo + hi) / 2;
      if (t_new - p->var_tend[(size_t)(mid % cap)] < window) hi = mid;
      else lo = mid + 1;
    }
    const long long live = p->var_b + 1 - lo;
    bytes += rec * (double)live + 32.0;
    most = std::max(most, live);
  }
  return bytes + 16.0 * (double)most;
}

// newest_end: end time of the newest stored interval (-inf: none).  When it
// lies at least the longest window L/c_s before t_new (with a margin far
// above rounding), every stored interval weighs exactly 0 for every mode:
// the conv launch is skipped and the mode stage takes zero history sums.
hipError_t var_launch(sbiem_plan* p, double dt, double t_old, double t_new, double newest_end) {
  Exec& ex = *p->exec;
  hipStream_t s = p->stream;
  const int nohist = (t_new - newest_end) >= (p->L / p->cs) * (1.0 + 1e-9) ? 1 : 0;
  const VarArgs va{dt, t_old, t_new, 1, nohist};
  hipError_t e = launch_reset_cells(ex, s);
  if (!e && !nohist) {
    // while profiling, the launch stamps two events of the plan's pool with
    // its own start and end (read back by var_prof_collect after the next
    // synchronisation)
    const bool prof = p->profiling && p->events.ensure(2 * (size_t)(p->var_prof_pending + 1)) == hipSuccess;
    if (prof) {
      p->prof_bytes += var_conv_bytes(p, t_new);
      e = launch_conv_var(ex, va, s, p->events.ev[2 * p->var_prof_pending],
                          p->events.ev[2 * p->var_prof_pending + 1]);
      if (!e) ++p->var_prof_pending;
    } else {
      e = launch_conv_var(ex, va, s);
    }
  }
  if (!e) e = launch_modes(ex, 0, 1, s, va);
  if (!e) e = launch_modes(ex, 0, 0, s, va);
  if (!e) e = launch_elems(ex, 1, s, va);
  if (!e) e = launch_modes(ex, 1, 0, s, va);
  if (!e) e = launch_elems(ex, 2, s, va);
  if (!e) e = launch_modes(ex, 2, 0, s, va);
  return e;
}

// Add the evented conv launches of the last synchronised work to the
// profile counters.
hipError_t var_prof_collect(sbiem_plan* p) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < p->var_prof_pending && !e; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p->events.ev[2 * k], p->events.ev[2 * k + 1]);
    if (!e) {
      p->prof_ms += ms;
      p->prof_launches += 1;
    }
  }
  p->var_prof_pending = 0;
  return e;
}

// End time of the newest committed interval (-inf: none yet).
double var_newest_end(const sbiem_plan* p) {
  if (p->var_b < 0 || p->var_tend.empty()) return -std::numeric_limits<double>::infinity();
  return p->var_tend[(size_t)(p->var_b % (long long)p->var_tend.size())];
}

// Record a committed interval ending at t_end in the host copy.
void var_commit(sbiem_plan* p, double t_end) {
  if (p->var_tend.size() != (size_t)p->dtd->tlog_cap)
    p->var_tend.assign((size_t)std::max(p->dtd->tlog_cap, 1), 0.0);
  ++p->var_b;
  p->var_tend[(size_t)(p->var_b % (long long)p->var_tend.size())] = t_end;
}

int var_step(sbiem_plan* p, double dt) {
  const double t_new = p->t_var + dt;
  hipError_t e = var_launch(p, dt, p->t_var, t_new, var_newest_end(p));
  if (!e) e = hipStreamSynchronize(p->stream);
  if (!e) e = var_prof_collect(p);
  if (e) return hip_fail(p, e, "variable step");
  p->dyn->primed = false;
  const int st = check_failure(p);
  if (st == SBIEM_OK) {
    p->t_var = t_new;
    var_commit(p, t_new);
  }
  return st;
}

int snap_alloc(sbiem_plan* p) {
  if (p->snap) return SBIEM_OK;
  VarSnap* v = new VarSnap();
  const size_t N = (size_t)p->N, M = (size_t)(p->N / 2 + 1);
  bool ok = true;
  for (double*& x : v->el) ok = ok && (x = (double*)v->mem.get(N * sizeof(double)));
  for (double2*& x : v->sp) ok = ok && (x = (double2*)v->mem.get(M * sizeof(double2)));
  ok = ok && (v->step = (long long*)v->mem.get(sizeof(long long)));
  ok = ok && (v->Vf = (double*)v->mem.get(N * sizeof(double)));
  ok = ok && (v->thf = (double*)v->mem.get(N * sizeof(double)));
  ok = ok && (v->eps = (unsigned long long*)v->mem.get(4 * sizeof(unsigned long long)));
  if (!ok) {
    delete v;
    return fail(p, SBIEM_ENOMEM, "adaptive stepping: snapshot allocation failed");
  }
  DynData* d = p->dyn;
  double* el[12] = {d->slip[0], d->slip[1], d->V[0], d->V[1], d->theta[0], d->theta[1],
                    d->thd[0], d->thd[1], d->tau_el[0], d->tau_el[1], d->sigma_el[0],
                    d->sigma_el[1]};
  double2* sp[6] = {d->u_hat, d->g_hat, d->v_hat0, d->gv_hat0, d->hprev_v, d->hprev_g};
  for (int k = 0; k < 12; ++k) {
    v->save.add(el[k], v->el[k], N * sizeof(double));
    v->restore.add(v->el[k], el[k], N * sizeof(double));
  }
  for (int k = 0; k < 6; ++k) {
    v->save.add(sp[k], v->sp[k], M * sizeof(double2));
    v->restore.add(v->sp[k], sp[k], M * sizeof(double2));
  }
  v->save.add(d->step, v->step, sizeof(long long));
  v->restore.add(v->step, d->step, sizeof(long long));
  v->restore.add(nullptr, v->eps, 2 * sizeof(unsigned long long));
  p->snap = v;
  return SBIEM_OK;
}

// Largest list entry in 8-byte words (the copy launch's x extent).
int snap_words(const sbiem_plan* p) { return (int)std::max<int64_t>(p->N, 2 * (p->N / 2 + 1)); }

// Committed state <-> snapshot (save = true: state -> snapshot), one launch;
// a restore also clears the error-measure cells.
hipError_t snap_copy(sbiem_plan* p, bool save) {
  VarSnap* v = p->snap;
  return launch_copy_many(save ? v->save : v->restore, snap_words(p), p->stream);
}

// One step in steady state: the next step's history sums on the second
// stream beside the element/mode stages of this step, joined before the
// commit launch that consumes them.  Both the conv launch and the first
// element launch wait only for the previous step's commit; the one enqueued
// first follows the commit on its hardware queue, the other crosses queues,
// which costs microseconds (most in a replayed graph).  stages_first puts the
// element/mode chain first: it pays where that chain is the step's critical
// path (small rings), and the conv-first order where the conv is.  The
// closure network (when on) follows the conv on its stream, or with
// closure_main precedes the first stage launch: it reads only ring records
// the step does not write before its commit and writes only the tails the
// commit reads, so it may run beside the conv; on the stage stream it
// shortens the conv's path where the stages have time to spare.
// While profiling, events e0/e1 bracket the conv launch.
hipError_t launch_step(Exec& ex, hipStream_t s, hipStream_t aux, bool profile, hipEvent_t e0,
                       hipEvent_t e1) {
  auto stages_start = [&]() {
    hipError_t r = ex.closure_main ? launch_closure(ex, 1, s) : hipSuccess;
    if (!r) r = launch_elems(ex, 1, s);
    return r;
  };
  hipError_t e = hipEventRecord(ex.fork, s);
  if (!e && ex.stages_first) e = stages_start();
  if (!e) e = hipStreamWaitEvent(aux, ex.fork, 0);
  if (!e && profile) e = hipEventRecord(e0, aux);
  if (!e) e = launch_conv(ex, 1, aux);
  if (!e && profile) e = hipEventRecord(e1, aux);
  if (!e && !ex.closure_main) e = launch_closure(ex, 1, aux);
  if (!e) e = hipEventRecord(ex.join, aux);
  if (!e && !ex.stages_first) e = stages_start();
  if (!e) e = launch_modes(ex, 1, 0, s);
  if (!e) e = launch_elems(ex, 2, s);
  if (!e) e = hipStreamWaitEvent(s, ex.join, 0);
  if (!e) e = launch_modes(ex, 2, 0, s);
  return e;
}

// Pass-1 spectra of the pending step from the stored state (after a reset,
// a new dt or a failed step): history sums for this step, the balance
// maxima, then the assembly.
hipError_t prologue(Exec& ex, hipStream_t s) {
  bool need = false;
  for (DynData* d : ex.dyns) need = need || !d->primed;
  if (!need) return hipSuccess;
  const int init[8] = {-2000, -2000, -2000, -2000, 0, 0, 0, 0};
  hipError_t e = hipSuccess;
  for (DynData* d : ex.dyns)
    if (!e) e = hipMemcpyAsync(d->cells, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (!e) e = launch_conv(ex, 0, s);
  if (!e) e = launch_closure(ex, 0, s);
  if (!e) e = launch_modes(ex, 0, 1, s);
  if (!e) e = launch_modes(ex, 0, 0, s);
  if (!e) e = hipStreamSynchronize(s);  // init lives on the host stack
  if (!e)
    for (DynData* d : ex.dyns) d->primed = true;
  return e;
}

hipError_t ensure_graph(Exec* ex, hipStream_t s) {
  if (ex->graph && ex->graph_stream == s) return hipSuccess;
  ex->drop_graph();
  hipStream_t cap = nullptr, cap2 = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (!e) e = hipStreamCreateWithFlags(&cap2, hipStreamNonBlocking);
  if (!e) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (!e) {
    for (int k = 0; k < kGraphSteps && !e; ++k) e = launch_step(*ex, cap, cap2, false, nullptr, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (!e) e = e2;
    if (!e) {
      e = hipGraphInstantiate(&ex->graph, g, nullptr, nullptr, 0);
      ex->graph_def = g;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  if (cap2) (void)hipStreamDestroy(cap2);
  if (cap) (void)hipStreamDestroy(cap);
  if (!e) {
    ex->graph_steps = kGraphSteps;
    ex->graph_stream = s;
  } else {
    ex->drop_graph();
  }
  return e;
}

// Run nsteps of an execution context on stream s.  While profiling, one
// step in every kProfileGraphs * kGraphSteps + 1 is launched directly with a
// pair of events around its conv launch and the others are replayed from the
// step graph as usual (HIP graphs do not give usable times for event nodes;
// a directly launched step costs several graph steps, so the sample is kept
// sparse); no host synchronisation inside a chunk of steps, the elapsed times
// are summed once the chunk has finished.
hipError_t run_steps(Exec* ex, int64_t nsteps, hipStream_t s, bool profile, EventPool* pool,
                     double* prof_ms, int64_t* prof_launches, const char** what) {
  *what = "running the time steps";
  if (nsteps <= 0) return hipSuccess;
  *what = "running the prologue launches";
  hipError_t e = prologue(*ex, s);
  if (e) return e;
  if (profile) {
    if (nsteps > kGraphSteps) {
      *what = "capturing the step graph";
      e = ensure_graph(ex, s);
      if (e) return e;
    }
    const int64_t chunk = 8192;  // timed steps per host synchronisation
    int64_t left = nsteps;
    while (left > 0 && !e) {
      *what = "creating timing events";
      e = pool->ensure((size_t)(2 * chunk));
      int64_t timed = 0;
      while (left > 0 && timed < chunk && !e) {
        *what = "launching profiled steps";
        e = launch_step(*ex, s, ex->aux, true, pool->ev[2 * timed], pool->ev[2 * timed + 1]);
        ++timed;
        --left;
        for (int g = 0; g < kProfileGraphs && !e && left >= kGraphSteps; ++g) {
          *what = "launching the step graph";
          e = hipGraphLaunch(ex->graph, s);
          left -= kGraphSteps;
        }
      }
      *what = "waiting for profiled steps";
      if (!e) e = hipStreamSynchronize(s);
      *what = "reading the timing events";
      for (int64_t k = 0; k < timed && !e; ++k) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, pool->ev[2 * k], pool->ev[2 * k + 1]);
        if (!e) {
          *prof_ms += ms;
          *prof_launches += 1;
        }
      }
    }
    return e;
  }
  int64_t left = nsteps;
  if (left >= kGraphSteps) {
    *what = "capturing the step graph";
    e = ensure_graph(ex, s);
    if (e) return e;
    *what = "launching the step graph";
    while (left >= kGraphSteps && !e) {
      e = hipGraphLaunch(ex->graph, s);
      left -= kGraphSteps;
    }
  }
  *what = "launching steps";
  for (int64_t k = 0; k < left && !e; ++k) e = launch_step(*ex, s, ex->aux, false, nullptr, nullptr);
  return e;
}

// Autotuning of the convolution launch: whole steps are replayed from the
// step graph with each candidate number of conv workgroups, in either launch
// order and, with the closure on, with the closure network on either stream
// (events on s around chunks of graph launches), and the fastest is kept.  Results do not depend on either (every task writes its own partial
// sums, and the dependencies are the same), so the trial steps are ordinary
// steps of the simulation.
hipError_t tune_conv(Exec* ex, int64_t steps_per_trial, hipStream_t s, int* chosen,
                     const char** what, float* best_ms_out = nullptr) {
  *chosen = ex->conv_grid;
  if (best_ms_out) *best_ms_out = 0.f;
  if (ex->precision != SBIEM_FP32CONV || ex->ntasks == 0) return hipSuccess;
  *what = "running the prologue launches";
  hipError_t e = prologue(*ex, s);
  if (e) return e;
  struct Shape {
    int grid;
    bool first, cmain;
    bool operator==(const Shape& o) const {
      return grid == o.grid && first == o.first && cmain == o.cmain;
    }
  };
  const bool closure = ex->closure_modes && ex->nclosure > 0;
  std::vector<Shape> cand;
  for (bool cmain : {false, true}) {
    if (cmain && !closure) continue;
    for (bool first : {false, true})
      for (int reserve : {0, 64, 128, 192, 256}) {
        const Shape g{conv_grid_size(ex->precision, ex->ntasks, ex->table_len, reserve), first,
                      cmain};
        if (std::find(cand.begin(), cand.end(), g) == cand.end()) cand.push_back(g);
      }
  }
  const int64_t chunks = std::max<int64_t>(1, steps_per_trial / kGraphSteps);
  hipEvent_t a = nullptr, b = nullptr;
  *what = "creating tuning events";
  e = hipEventCreate(&a);
  if (!e) e = hipEventCreate(&b);
  // one trial: the step graph of a shape, settled by one replay, then timed
  auto trial = [&](const Shape& g, bool cached, float* ms) {
    ex->drop_graph();
    ex->conv_grid = g.grid;
    ex->stages_first = g.first;
    ex->closure_main = g.cmain;
    ex->cached_loads = cached;
    *what = "capturing the step graph";
    hipError_t r = ensure_graph(ex, s);
    *what = "launching tuning steps";
    if (!r) r = hipGraphLaunch(ex->graph, s);  // settles the new grid
    if (!r) r = hipEventRecord(a, s);
    for (int64_t k = 0; k < chunks && !r; ++k) r = hipGraphLaunch(ex->graph, s);
    if (!r) r = hipEventRecord(b, s);
    if (!r) r = hipEventSynchronize(b);
    if (!r) r = hipEventElapsedTime(ms, a, b);
    return r;
  };
  float best_ms = 0.f;
  Shape best{ex->conv_grid, ex->stages_first, ex->closure_main};
  for (size_t c = 0; c < cand.size() && !e; ++c) {
    float ms = 0.f;
    e = trial(cand[c], false, &ms);
    if (!e && (c == 0 || ms < best_ms)) {
      best_ms = ms;
      best = cand[c];
    }
  }
  // the best shape once more with the record loads on the default cache
  // policy (kept only if faster)
  bool cached = false;
  if (!e) {
    float ms = 0.f;
    e = trial(best, true, &ms);
    if (!e && ms < best_ms) {
      best_ms = ms;
      cached = true;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  ex->drop_graph();
  ex->conv_grid = best.grid;
  ex->stages_first = best.first;
  ex->closure_main = best.cmain;
  ex->cached_loads = cached;
  *chosen = best.grid;
  if (best_ms_out) *best_ms_out = best_ms;
  return e;
}

// Tile shapes of the FP32 conv to try: the one in use first, then the
// others (none when a member's tile was set explicitly).
std::vector<int> tile_candidates(const std::vector<sbiem_plan*>& plans) {
  const DtData* d = plans[0]->dtd;
  std::vector<int> c{d->tile_slots};
  if (d->var || plans[0]->precision != SBIEM_FP32CONV) return c;
  for (const sbiem_plan* p : plans)
    if (p->conv_tile_set) return c;
  // (packed rows, kTileSlots32p, only when set: slower on every workload
  // measured, their per-row descriptors costing more than they save)
  for (int t : {kTileSlots32, kTileSlots32s, kTileSlots32w, kTileSlots32l})
    if (t != c[0]) c.push_back(t);
  return c;
}

// Autotuning over tile shapes: for each candidate the members are re-cut
// (retile), the execution context rebuilt by `rebuild` and tune_conv run on
// it; the fastest tile with its grid and launch order is kept.  Every trial
// step is an ordinary step (a tile change alters only the FP32 summation
// order of the sums).
template <typename Rebuild, typename GetExec>
int tune_tiles(const std::vector<sbiem_plan*>& plans, int64_t steps_per_trial, hipStream_t s,
               Rebuild rebuild, GetExec get_exec, int* chosen, int* tile_out, std::string* err) {
  const std::vector<int> cand = tile_candidates(plans);
  struct Best {
    int tile = 0, grid = 0;
    bool first = false, cmain = false, cached = false;
    float ms = 0.f;
  } best;
  const char* what = "";
  for (size_t c = 0; c < cand.size(); ++c) {
    if (c > 0) {
      for (sbiem_plan* p : plans)
        if (int st = retile(p, cand[c])) return st;
      if (int st = rebuild()) return st;
      for (sbiem_plan* p : plans) p->dyn->primed = false;
    }
    Exec* ex = get_exec();
    int g = 0;
    float ms = 0.f;
    hipError_t e = tune_conv(ex, steps_per_trial, s, &g, &what, &ms);
    if (!e) e = hipStreamSynchronize(s);
    if (e) {
      *err = std::string(what) + ": " + hipGetErrorString(e);
      return SBIEM_EDEVICE;
    }
    if (c == 0 || ms < best.ms) {
      best.tile = cand[c];
      best.grid = ex->conv_grid;
      best.first = ex->stages_first;
      best.cmain = ex->closure_main;
      best.cached = ex->cached_loads;
      best.ms = ms;
    }
  }
  if (cand.size() > 1) {
    for (sbiem_plan* p : plans)
      if (int st = retile(p, best.tile)) return st;
    if (int st = rebuild()) return st;
    for (sbiem_plan* p : plans) p->dyn->primed = false;
    Exec* ex = get_exec();
    ex->conv_grid = best.grid;
    ex->stages_first = best.first;
    ex->closure_main = best.cmain;
    ex->cached_loads = best.cached;
    for (sbiem_plan* p : plans) p->conv_tile = best.tile;
  }
  *chosen = best.grid;
  *tile_out = best.tile;
  return SBIEM_OK;
}

}  // namespace

}  // namespace sbiem

using namespace sbiem;

extern "C" {

int sbiem_step(sbiem_plan* p, double dt) { return sbiem_run(p, dt, 1); }

int sbiem_run(sbiem_plan* p, double dt, int64_t nsteps) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (nsteps < 0) return fail(p, SBIEM_EINVAL, "nsteps must be >= 0");
  if (int st = ready(p, dt)) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e) return hip_fail(p, e, "hipSetDevice");
  if (!p->exec) {
    if (int st = rebuild_exec(p)) return st;
  }
  if (p->dtd->var) {
    for (int64_t k = 0; k < nsteps; ++k)
      if (int st = var_step(p, dt)) return st;
    return SBIEM_OK;
  }
  const char* what = "";
  e = run_steps(p->exec, nsteps, p->stream, p->profiling, &p->events, &p->prof_ms,
                &p->prof_launches, &what);
  if (!e) {
    what = "waiting for the time steps";
    e = hipStreamSynchronize(p->stream);
  }
  if (e) return hip_fail(p, e, what);
  return check_failure(p);
}

int sbiem_step_var(sbiem_plan* p, double dt) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (!p->dtd || !p->dtd->var)
    return fail(p, SBIEM_EINVAL, "step_var: the plan is not on the variable-step engine "
                                 "(sbiem_set_adaptive, then sbiem_set_dt)");
  return sbiem_run(p, dt, 1);
}

namespace {

constexpr int64_t kResync = 32;  // FP32 plans: accepted steps between spectral-slip refreshes

// The controller behind sbiem_adapt and sbiem_adapt_until: log records of
// `stride` doubles (4, or 5 with the maximum slip rate after the attempt);
// v_cross > 0 also ends the run after the first accepted step across it.
int adapt_impl(sbiem_plan* p, double eps0, double dt_max, double t_end, int64_t max_accepted,
               double v_cross, double* dt_io, double* log, int64_t log_cap, int stride,
               int64_t* log_len, int* crossed) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (!p->adaptive || !p->dtd)
    return fail(p, SBIEM_EINVAL, "adapt: needs sbiem_set_adaptive(1) and sbiem_set_dt(dt_min)");
  if (!p->friction_set || !p->state_set)
    return fail(p, SBIEM_ENOTREADY, "set_friction and set_state must precede stepping");
  const double dt_min = p->dtd->dt;
  if (!dt_io || !(eps0 > 0) || !(dt_max >= dt_min) || max_accepted < 0 || log_cap < 0 ||
      (log_cap > 0 && !log) || !std::isfinite(dt_max) || !(*dt_io > 0))
    return fail(p, SBIEM_EINVAL, "adapt: need eps0 > 0, dt_max >= dt_min, *dt_io > 0");
  hipError_t e = hipSetDevice(p->device);
  if (e) return hip_fail(p, e, "hipSetDevice");
  if (!p->exec) {
    if (int st = rebuild_exec(p)) return st;
  }
  if (int st = snap_alloc(p)) return st;
  DynData* d = p->dyn;
  VarSnap* v = p->snap;
  hipStream_t s = p->stream;
  long long s0 = 0;
  e = hipStreamSynchronize(s);
  if (!e) e = hipMemcpy(&s0, d->step, sizeof(s0), hipMemcpyDeviceToHost);
  if (e) return hip_fail(p, e, "adapt");
  int64_t nlog = 0;
  auto record = [&](double t, double dt, double eps, int outcome, double vmax) {
    if (nlog < log_cap) {
      double* r = log + stride * nlog;
      r[0] = t;
      r[1] = dt;
      r[2] = eps;
      r[3] = (double)outcome;
      if (stride > 4) r[4] = vmax;
    }
    ++nlog;
  };
  auto read_norms = [&](double* eps, double* vmax) {
    unsigned long long bits[2] = {0, 0};
    hipError_t err = hipMemcpyAsync(bits, v->eps, sizeof(bits), hipMemcpyDeviceToHost, s);
    if (!err) err = hipStreamSynchronize(s);
    std::memcpy(eps, &bits[0], sizeof(double));
    std::memcpy(vmax, &bits[1], sizeof(double));
    return err;
  };
  if (crossed) *crossed = 0;
  // maximum slip rate of the state the run starts from
  double v_prev = 0.0;
  if (v_cross > 0) {
    const int c = (int)(s0 & 1);
    double unused;
    e = launch_err_norm(d->V[c], d->theta[c], d->V[c], d->theta[c], (int)p->N, v->eps, s);
    if (!e) e = read_norms(&unused, &v_prev);
    if (e) return hip_fail(p, e, "adapt: maximum slip rate");
  }
  const double growth = 5.0, safety = 0.9;
  auto next_dt = [&](double dt, double eps) {
    const double g = eps > 0 ? safety * std::pow(eps0 / eps, 1.0 / 3.0) * dt : growth * dt;
    return std::min(std::min(std::max(g, dt_min), dt_max), growth * dt);
  };
  auto physics = [](int st) {
    return st == SBIEM_ENEWTON || st == SBIEM_ESTATE || st == SBIEM_EOPEN;
  };
  double dt = std::min(std::max(*dt_io, dt_min), dt_max);
  int64_t accepted = 0;
  int status = SBIEM_OK;
  bool crossing = false;
  while (accepted < max_accepted && p->t_var < t_end && status == SBIEM_OK && !crossing) {
    for (;;) {
      const double t_start = p->t_var;
      const double t_half = t_start + 0.5 * dt;
      // one step of dt, then two of dt/2 from the same state, launched back
      // to back: after a failure the remaining launches do nothing, and the
      // flags come back with the error measure in one read
      CopyList keep;
      const int cf = (int)((s0 + 1) & 1);  // the full step's solution buffer
      keep.add(d->V[cf], v->Vf, (size_t)p->N * sizeof(double));
      keep.add(d->theta[cf], v->thf, (size_t)p->N * sizeof(double));
      const int c = (int)(s0 & 1);         // two steps after s0
      const double newest = var_newest_end(p);
      e = snap_copy(p, true);
      if (!e) e = var_launch(p, dt, t_start, t_start + dt, newest);
      if (!e) e = launch_copy_many(keep, (int)p->N, s);
      if (!e) e = snap_copy(p, false);
      if (!e) e = var_launch(p, 0.5 * dt, t_start, t_half, newest);
      if (!e) e = var_launch(p, 0.5 * dt, t_half, t_half + 0.5 * dt, t_half);
      if (!e)
        e = launch_err_norm(v->Vf, v->thf, d->V[c], d->theta[c], (int)p->N, v->eps, s, d->err,
                            true);
      unsigned long long r[4] = {0, 0, 0, 0};
      if (!e) e = hipMemcpyAsync(r, v->eps, sizeof(r), hipMemcpyDeviceToHost, s);
      if (!e) e = hipStreamSynchronize(s);
      if (!e) e = var_prof_collect(p);
      if (e) return hip_fail(p, e, "adapt: attempt");
      d->primed = false;
      const int st = (int)(unsigned)r[2];
      if (st != SBIEM_OK) {
        note_failure(p, st, (int)(r[3] >> 32), (int)(unsigned)(r[3] & 0xffffffffULL));
        if (!physics(st)) return st;
        e = snap_copy(p, false);
        if (!e) e = hipStreamSynchronize(s);
        if (e) return hip_fail(p, e, "adapt: snapshot");
        p->t_var = t_start;
        if (dt <= dt_min) {
          record(t_start, dt, -1.0, SBIEM_ADAPT_STOP, -1.0);
          status = st;
          break;
        }
        record(t_start, dt, -1.0, SBIEM_ADAPT_FAIL, -1.0);
        dt = std::max(0.5 * dt, dt_min);
        continue;
      }
      p->last_fail_count = 0;
      p->last_fail_index = -1;
      p->t_var = t_half + 0.5 * dt;
      double eps, vmax;
      std::memcpy(&eps, &r[0], sizeof(double));
      std::memcpy(&vmax, &r[1], sizeof(double));
      if (eps <= eps0 || dt <= dt_min) {
        record(t_start, dt, eps, eps <= eps0 ? SBIEM_ADAPT_ACCEPT : SBIEM_ADAPT_FLOOR, vmax);
        var_commit(p, t_half);
        var_commit(p, p->t_var);
        s0 += 2;
        ++accepted;
        dt = next_dt(dt, eps);
        if (v_cross > 0 && (v_prev < v_cross) != (vmax < v_cross)) {
          if (crossed) *crossed = 1;
          crossing = true;
        }
        v_prev = vmax;
        // FP32 rate spectra feed the FP64 spectral slip through the commit's
        // integration; recompute it from the FP64 slip every kResync
        // accepted steps so that its rounding does not accumulate over a run
        if (p->precision == SBIEM_FP32CONV && ++p->var_accepted % kResync == 0) {
          if (int rs = spectral_state_from_device(p)) return rs;
        }
        break;
      }
      record(t_start, dt, eps, SBIEM_ADAPT_REJECT, vmax);
      e = snap_copy(p, false);
      if (!e) e = hipStreamSynchronize(s);
      if (e) return hip_fail(p, e, "adapt: snapshot");
      p->t_var = t_start;
      d->primed = false;
      dt = std::max(safety * std::pow(eps0 / eps, 1.0 / 3.0) * dt, dt_min);
    }
  }
  *dt_io = dt;
  if (log_len) *log_len = nlog;
  if (status != SBIEM_OK)
    return fail(p, status, "adapt: a step failed with dt at its minimum: " + p->last_error);
  return SBIEM_OK;
}

}  // namespace

int sbiem_adapt(sbiem_plan* p, double eps0, double dt_max, double t_end, int64_t max_accepted,
                double* dt_io, double* log, int64_t log_cap, int64_t* log_len) {
  return adapt_impl(p, eps0, dt_max, t_end, max_accepted, 0.0, dt_io, log, log_cap, 4, log_len,
                    nullptr);
}

int sbiem_adapt_until(sbiem_plan* p, double eps0, double dt_max, double t_end,
                      int64_t max_accepted, double v_cross, double* dt_io, double* log,
                      int64_t log_cap, int64_t* log_len, int* crossed) {
  if (!std::isfinite(v_cross)) {
    if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
    return fail(p, SBIEM_EINVAL, "adapt_until: v_cross must be finite");
  }
  return adapt_impl(p, eps0, dt_max, t_end, max_accepted, v_cross, dt_io, log, log_cap, 5,
                    log_len, crossed);
}

int sbiem_steps_done(const sbiem_plan* p, int64_t* nsteps) {
  if (!p || !nsteps) return fail_global(SBIEM_EINVAL, "NULL argument");
  long long step = 0;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (!e) e = hipMemcpy(&step, p->dyn->step, sizeof(step), hipMemcpyDeviceToHost);
  if (e) return hip_fail(const_cast<sbiem_plan*>(p), e, "steps_done");
  *nsteps = step;
  return SBIEM_OK;
}

int sbiem_failures(const sbiem_plan* p, int64_t* count, int64_t* first_index) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (count) *count = p->last_fail_count;
  if (first_index) *first_index = p->last_fail_count ? p->last_fail_index : -1;
  return SBIEM_OK;
}

int sbiem_set_profiling(sbiem_plan* p, int on) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  p->profiling = on != 0;
  p->prof_ms = 0.0;
  p->prof_launches = 0;
  p->prof_bytes = 0.0;
  return SBIEM_OK;
}

int sbiem_profile(sbiem_plan* p, double* conv_ms, int64_t* conv_launches,
                  double* conv_bytes_per_launch) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (conv_ms) *conv_ms = p->prof_ms;
  if (conv_launches) *conv_launches = p->prof_launches;
  if (conv_bytes_per_launch) {
    if (p->dtd && p->dtd->var)
      *conv_bytes_per_launch = p->prof_launches ? p->prof_bytes / (double)p->prof_launches : 0.0;
    else
      *conv_bytes_per_launch = p->exec ? p->exec->conv_bytes : 0.0;
  }
  p->prof_ms = 0.0;
  p->prof_launches = 0;
  p->prof_bytes = 0.0;
  return SBIEM_OK;
}

int sbiem_stress(sbiem_plan* p, const double* slip_hist, int64_t nt, double dt, double* tau_out,
                 double* sigma_out) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (nt < 0 || !(dt > 0) || !std::isfinite(dt) || !slip_hist || !tau_out || !sigma_out)
    return fail(p, SBIEM_EINVAL, "stress: need nt >= 0, dt > 0 and arrays");
  const int64_t N = p->N;
  for (int64_t i = 0; i < (nt + 1) * N; ++i)
    if (!std::isfinite(slip_hist[i])) return fail(p, SBIEM_EINVAL, "stress: slip must be finite");
  hipError_t e = hipSetDevice(p->device);
  if (e) return hip_fail(p, e, "hipSetDevice");
  hipStream_t s = p->stream;
  e = hipStreamSynchronize(s);
  if (e) return hip_fail(p, e, "stress");
  DtData* dtd = nullptr;
  if (int st = build_dt_data(p, dt, &dtd)) return st;
  DynData* dyn = nullptr;
  if (int st = build_dyn_data(p, &dyn)) {
    delete dtd;
    return st;
  }
  FaultDev f = make_fault_desc(p, dtd, dyn, 0.0, 0.0);
  std::string err;
  Exec* ex = nullptr;
  int st = build_exec({p}, {dtd}, {dyn}, {f}, p->precision, &ex, &err);
  if (st) {
    delete dyn;
    delete dtd;
    return fail(p, st, err);
  }
  DevArena tmp;
  const int M = (int)(N / 2 + 1);
  const int64_t nint = nt;
  const int64_t nsig = std::max<int64_t>(nint, 1);
  double* d_hist = (double*)tmp.get((size_t)(nt + 1) * N * sizeof(double));
  double* d_rates = (double*)tmp.get((size_t)nsig * N * sizeof(double));
  double2* RV = (double2*)tmp.get((size_t)nsig * M * sizeof(double2));
  double2* RG = (double2*)tmp.get((size_t)nsig * M * sizeof(double2));
  void* gF = tmp.get((size_t)nsig * N * sizeof(double2));
  if (!d_hist || !d_rates || !RV || !RG || !gF) {
    delete ex;
    delete dyn;
    delete dtd;
    return fail(p, SBIEM_ENOMEM, "stress: device allocation failed");
  }
  e = hipMemcpyAsync(d_hist, slip_hist, (size_t)(nt + 1) * N * sizeof(double), hipMemcpyHostToDevice, s);
  // interval rates as first differences of the snapshots
  if (!e && nint > 0) e = launch_rates(d_hist, d_rates, (long long)nint * N, N, dt, s);
  const FaultDev* dfd = ex->d_faults;
  if (!e && nint > 0)
    e = launch_forward(dfd, f, p->precision, d_rates, RV, RG, (int)nint, M, gF, s);
  // static part on snapshot nt-1 (its slip plus dt times the last rate is snapshot nt)
  const int64_t base = nint > 0 ? nt - 1 : 0;
  if (!e) e = forward_fp64(p, dfd, f, d_hist + base * N, dyn->u_hat, dyn->g_hat, 1, M, gF, s, tmp);
  if (!e && nint > 0) {
    e = hipMemcpyAsync(dyn->v_hat0, RV + (nint - 1) * M, M * sizeof(double2), hipMemcpyDeviceToDevice, s);
    if (!e) e = hipMemcpyAsync(dyn->gv_hat0, RG + (nint - 1) * M, M * sizeof(double2), hipMemcpyDeviceToDevice, s);
  }
  if (!e) e = launch_fill_ring(dfd, p->precision, M - 1, RV, RG, (int)nint, s);
  const long long step = nint > 0 ? nint - 1 : 0;
  if (!e) e = hipMemcpyAsync(dyn->step, &step, sizeof(step), hipMemcpyHostToDevice, s);
  std::vector<double2> tl;
  if (!e && dtd->var) {
    // interval l spans [l dt, (l + 1) dt]; the log keeps the last tlog_cap
    tl.assign(dtd->tlog_cap, make_double2(0.0, 0.0));
    for (int64_t l = std::max<int64_t>(0, nint - 1 - dtd->tlog_cap); l <= nint - 2; ++l)
      tl[l % dtd->tlog_cap] = make_double2((double)l * dt, (double)(l + 1) * dt);
    e = hipMemcpyAsync(dtd->tlog, tl.data(), sizeof(double2) * tl.size(), hipMemcpyHostToDevice, s);
  }
  if (!e) e = hipStreamSynchronize(s);  // step lives on the host stack
  dyn->primed = false;
  if (!e && dtd->var) {
    const double t_new = (double)nt * dt;
    const VarArgs va{dt, t_new - dt, t_new, 1, 0};
    e = launch_reset_cells(*ex, s);
    if (!e) e = launch_conv_var(*ex, va, s);
    if (!e) e = launch_modes(*ex, 0, 1, s, va);
    if (!e) e = launch_modes(*ex, 0, 0, s, va);
  } else if (!e) {
    e = prologue(*ex, s);
  }
  if (!e) e = launch_elems(*ex, 0, s);
  if (!e) e = hipStreamSynchronize(s);
  const int slot = (int)((step + 1) & 1);
  if (!e) e = download_elems(p, dyn->tau_el[slot], tau_out);
  if (!e) e = download_elems(p, dyn->sigma_el[slot], sigma_out);
  delete ex;
  delete dyn;
  delete dtd;
  if (e) return hip_fail(p, e, "stress");
  return SBIEM_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
int sbiem_batch_create(sbiem_batch** out, sbiem_plan* const* plans, int64_t n) {
  if (!out || !plans || n <= 0) return fail_global(SBIEM_EINVAL, "batch_create: need plans");
  *out = nullptr;
  const int prec = plans[0]->precision;
  std::vector<sbiem_plan*> ps(plans, plans + n);
  std::vector<DtData*> dts;
  std::vector<DynData*> dyns;
  std::vector<FaultDev> descs;
  for (sbiem_plan* p : ps) {
    if (!p) return fail_global(SBIEM_EINVAL, "batch_create: NULL plan");
    if (p->precision != prec) return fail_global(SBIEM_EINVAL, "batch_create: mixed precision");
    if (!p->friction_set || !p->state_set || !p->dtd)
      return fail_global(SBIEM_ENOTREADY, "batch_create: members need friction, state and dt");
    if (p->device != plans[0]->device) return fail_global(SBIEM_EINVAL, "batch_create: one device");
    dts.push_back(p->dtd);
    dyns.push_back(p->dyn);
    descs.push_back(make_fault_desc(p, p->dtd, p->dyn, p->V_pl, p->t0));
  }
  std::string err;
  Exec* ex = nullptr;
  (void)hipSetDevice(plans[0]->device);
  int st = build_exec(ps, dts, dyns, descs, prec, &ex, &err);
  if (st) return fail_global(st, err);
  sbiem_batch* b = new sbiem_batch();
  b->plans = ps;
  b->exec = ex;
  b->stream = plans[0]->stream;
  b->device = plans[0]->device;
  for (sbiem_plan* p : ps) p->batch_refs++;
  *out = b;
  return SBIEM_OK;
}

int sbiem_batch_destroy(sbiem_batch* b) {
  if (!b) return SBIEM_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  for (sbiem_plan* p : b->plans) p->batch_refs--;
  delete b->exec;
  delete b;
  return SBIEM_OK;
}

int sbiem_batch_run(sbiem_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return fail_global(SBIEM_EINVAL, "batch_run: bad arguments");
  hipError_t e = hipSetDevice(b->device);
  // descriptors may have changed (theta mode, loads): refresh
  for (size_t f = 0; f < b->plans.size() && !e; ++f) {
    FaultDev d = make_fault_desc(b->plans[f], b->plans[f]->dtd, b->plans[f]->dyn, b->plans[f]->V_pl,
                                 b->plans[f]->t0);
    if (std::memcmp(&d, &b->exec->host_faults[f], sizeof(d)) != 0) {
      b->exec->host_faults[f] = d;
      e = hipMemcpy(b->exec->d_faults + f, &d, sizeof(d), hipMemcpyHostToDevice);
    }
  }
  const char* what = "refreshing the descriptors";
  if (!e)
    e = run_steps(b->exec, nsteps, b->stream, b->profiling, &b->events, &b->prof_ms,
                  &b->prof_launches, &what);
  if (!e) {
    what = "waiting for the time steps";
    e = hipStreamSynchronize(b->stream);
  }
  if (e)
    return fail_global(SBIEM_EDEVICE, std::string("batch_run: ") + what + ": " + hipGetErrorString(e));
  int first = SBIEM_OK;
  for (sbiem_plan* p : b->plans) {
    int st = check_failure(p);
    if (st && first == SBIEM_OK) first = st;
  }
  return first;
}

int sbiem_tune(sbiem_plan* p, double dt, int64_t steps_per_trial, int32_t* conv_workgroups) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (steps_per_trial < 1) return fail(p, SBIEM_EINVAL, "steps_per_trial must be >= 1");
  if (p->batch_refs > 0) return fail(p, SBIEM_EINVAL, "plan is used by a batch: tune the batch");
  if (int st = ready(p, dt)) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e) return hip_fail(p, e, "hipSetDevice");
  if (!p->exec) {
    if (int st = rebuild_exec(p)) return st;
  }
  if (p->dtd->var) {  // launch by launch: nothing to tune
    if (conv_workgroups) *conv_workgroups = std::min(p->exec->ntasks, 4096);
    return SBIEM_OK;
  }
  int chosen = 0, tile = 0;
  std::string err;
  const int st = tune_tiles(
      {p}, steps_per_trial, p->stream, [&]() { return rebuild_exec(p); },
      [&]() { return p->exec; }, &chosen, &tile, &err);
  if (st == SBIEM_EDEVICE && !err.empty()) return fail(p, st, "tune: " + err);
  if (st) return st;
  if (conv_workgroups) *conv_workgroups = chosen;
  return check_failure(p);
}

int sbiem_batch_tune(sbiem_batch* b, int64_t steps_per_trial, int32_t* conv_workgroups) {
  if (!b || steps_per_trial < 1) return fail_global(SBIEM_EINVAL, "batch_tune: bad arguments");
  hipError_t e = hipSetDevice(b->device);
  if (e) return fail_global(SBIEM_EDEVICE, std::string("batch_tune: hipSetDevice: ") + hipGetErrorString(e));
  int chosen = 0, tile = 0;
  std::string err;
  auto rebuild = [&]() -> int {
    std::vector<DtData*> dts;
    std::vector<DynData*> dyns;
    std::vector<FaultDev> descs;
    for (sbiem_plan* p : b->plans) {
      dts.push_back(p->dtd);
      dyns.push_back(p->dyn);
      descs.push_back(make_fault_desc(p, p->dtd, p->dyn, p->V_pl, p->t0));
    }
    (void)hipStreamSynchronize(b->stream);
    delete b->exec;
    b->exec = nullptr;
    std::string why;
    Exec* ex = nullptr;
    const int st = build_exec(b->plans, dts, dyns, descs, b->plans[0]->precision, &ex, &why);
    if (st) return fail_global(st, "batch_tune: " + why);
    b->exec = ex;
    return (int)SBIEM_OK;
  };
  const int st = tune_tiles(b->plans, steps_per_trial, b->stream, rebuild,
                            [&]() { return b->exec; }, &chosen, &tile, &err);
  if (st == SBIEM_EDEVICE && !err.empty()) return fail_global(st, "batch_tune: " + err);
  if (st) return st;
  if (conv_workgroups) *conv_workgroups = chosen;
  int first = SBIEM_OK;
  for (sbiem_plan* p : b->plans) {
    int st = check_failure(p);
    if (st && first == SBIEM_OK) first = st;
  }
  return first;
}

int sbiem_batch_set_profiling(sbiem_batch* b, int on) {
  if (!b) return fail_global(SBIEM_EINVAL, "NULL batch");
  b->profiling = on != 0;
  b->prof_ms = 0.0;
  b->prof_launches = 0;
  return SBIEM_OK;
}

int sbiem_batch_profile(sbiem_batch* b, double* conv_ms, int64_t* conv_launches,
                        double* conv_bytes_per_launch) {
  if (!b) return fail_global(SBIEM_EINVAL, "NULL batch");
  if (conv_ms) *conv_ms = b->prof_ms;
  if (conv_launches) *conv_launches = b->prof_launches;
  if (conv_bytes_per_launch) *conv_bytes_per_launch = b->exec->conv_bytes;
  b->prof_ms = 0.0;
  b->prof_launches = 0;
  return SBIEM_OK;
}

}  // extern "C"

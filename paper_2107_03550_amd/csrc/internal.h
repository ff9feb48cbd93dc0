// Internal definitions of libsbiem (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sbiem.h"

namespace sbiem {

// Per-mode constants of the traction assembly (mode n = 0..N/2):
//   tau_hat   = mk (B_T + aT vc),  B_T = (1-r) u_hat + w1T hprev_v + S_T
//   sigma_hat = -i ms (B_N + aN gvc), B_N likewise with the curvature spectra
// with mk = -mu |k_n|, ms = s_n mu (0 at n = 0 and n = N/2) and
// aX = (1-r) dt + w0X (the predicted slip dt vc plus the current interval).
struct ModeCoef {
  double mk, ms, aT, aN, w1T, w1N;
  long long ring_off;  // first ring record of the mode
  int Rn;              // ring capacity M_n - 1 (0: no history records)
  int part0;           // index of the mode's second conv partial (the first is
                       // at the mode's own position)
  int nparts;          // number of partials (0: no history records)
  int pad;
};

// ---------------------------------------------------------------------------
// Index maps of the four-step transforms.  N = P Q (powers of two, P <= Q).
// Element i belongs to class b = i mod Q (P elements i = b + Q a); spectral
// index n in [0, N) belongs to class c = n mod P (Q entries n = c + P d).
// Per-element arrays are stored class-major (position b P + a), so one
// element workgroup reads a contiguous block; per-mode arrays (modes
// 0..N/2) are stored at mode_pos(n) = (n mod P) Q/2 + n div P for n < N/2
// and N/2 for the Nyquist mode, so the modes of one class are contiguous.
// ---------------------------------------------------------------------------
__host__ __device__ inline int elem_pos(int i, int log2P, int log2Q) {
  return ((i & ((1 << log2Q) - 1)) << log2P) + (i >> log2Q);
}
__host__ __device__ inline int mode_pos(int n, int log2P, int log2Q) {
  const int half = 1 << (log2P + log2Q - 1);
  if (n >= half) return half;
  return ((n & ((1 << log2P) - 1)) << (log2Q - 1)) + (n >> log2P);
}

// A mode whose window the learned closure cuts (see closure.hip).
struct ClosureMode {
  int fault, pm;      // fault (in the execution context), mode position
  int Rn, Mk;         // kept ring capacity M'_n - 1, kept lags M'_n
  long long ring_off; // first ring record of the mode
  float tcut;         // c_s |k_n| M'_n dt / 100 (network input 0)
  float pad;
  double inv_csk;     // 1 / (c_s |k_n|)
  double dT, dN;      // sums of the discarded weights, lags M'_n .. M_n - 1
};
constexpr int kClosureParams = 6466;  // 33*64 + 64 + 64*64 + 64 + 64*2 + 2
constexpr int kClosureThreads = 512;  // closure inference workgroups (8 waves)
constexpr int kClosureFaults = 64;    // faults whose words a closure workgroup stages in LDS

// ---------------------------------------------------------------------------
// Device-visible description of one fault at one time step.  One array of
// these per execution context (a plan, a batch, a stress evaluation); the
// kernels index it by fault number.
// ---------------------------------------------------------------------------
struct FaultDev {
  int N, log2N, nmodes;     // nmodes = N/2
  int P, Q, log2P, log2Q;   // N = P Q (see the index maps above)
  int ngroups;              // mode workgroups: classes {g, P-g} (g = 0: {0, P/2})
  int ncls;                 // element classes per element workgroup
  int theta_mode;
  int newton_max;           // FP64 Newton iterations of the momentum balance
  double L, mu, r, cs, dt, eta_rad;
  double V_pl, Dc, V_ref, f0, tau_rate, t0, ln_V_ref;

  // per element (FP64, length N, class-major positions)
  const double *a, *b, *sigma_load, *tau_load, *kappa;
  double *slip[2], *V[2], *theta[2], *thd[2];  // committed state at [step & 1]
  double *V1, *thd1;                           // pass-1 solution
  double *tau_el[2], *sigma_el[2];             // last pass of the step at [(step+1) & 1]

  // spectral state (FP64 complex, modes 0..N/2 at mode_pos)
  double2 *u_hat, *g_hat;       // F[slip - V_pl t], F[kappa (slip - V_pl t)]
  double2 *v_hat0, *gv_hat0;    // F[V - V_pl], F[kappa (V - V_pl)] at step start
  double2 *v_hat1, *gv_hat1;    // same for the pass-1 solution
  double2 *hprev_v, *hprev_g;   // rate spectra of the last committed interval
  double2 *B_T, *B_N;           // (1-r) u_hat + w1 hprev + S, pass 1 -> pass 2
  double fwd_scale;             // power of two ~ 1/max|kappa| for the forward packing

  // transform exchange buffers (N complex, convolution precision)
  void* gI;                     // inverse transform after the mode stage: [b][c]
  void* gF;                     // forward transform after the element stage: [c][b]
  int* cells;                   // [0..1] log2 maxima (tau, sigma) of pass 1,
                                // [2..3] of pass 2, [4] balance exponent in use
  int* done;                    // mode workgroups finished in the commit launch

  // per mode (modes 0..N/2 at mode_pos)
  const ModeCoef* coef;
  double4* parts;               // conv partials: (S_T re, im, S_N re, im)
  double4* tails;               // learned-closure tails (same layout), or null

  void* ring;                   // history records: float4 or 2 x double2 per slot
  const double2* wrev;          // FP64 weights per ring slot (see conv kernel)
  const void* twiddle;          // N/4+1 values cos(2 pi t / N), convolution precision

  long long* step;              // committed steps since state/dt were set
  // variable steps and the interval rule (null/0 on the fixed-step engine)
  double kcT, kcN;              // k_c L of the shear and normal windows
  const double* ptab;           // primitive table: per node T = i h, (P^T, C^T, C^T',
                                // P^N, C^N, C^N') in FP64
  int ptab_len;                 // nodes
  double ptab_h;                // node spacing h
  double2* tlog;                // (start, end) time of committed interval l at l mod tlog_cap
  int tlog_cap;
  int* err;                     // first failure status of the pending step (0 = none)
  int* err_count;               // failing elements of that pass
  int* err_index;               // first failing element
};

// A conv tile: one wavefront sums up to kTileSlots ring records of one mode.
// Per-mode constants ride along so that a wave needs no dependent lookups.
struct Tile {
  int fault, mode, p0, len;
  int Rn;          // ring capacity of the mode
  int part;        // fault-local index of the (task, mode) partial sum
  int MT, MN;      // window lengths of the shear and normal kernels (lags >= M^X weigh 0)
  long long ring_off;
  double th;       // FP32 weights: c_s |k_n| dt / 2 / table spacing
  const void* rec; // the mode's first ring record (set per execution context)
  unsigned long long rmagic;  // floor((2^64 - 1) / Rn) + 1: a mod Rn for 32-bit a by multiplication
};

// A conv task: tiles [t0, t1) of one fault, handled by one workgroup.  A task
// holds whole modes, or one piece of a mode longer than a task's tiles; it
// writes one FP64 partial sum per (task, mode) and the spectral kernel adds a
// mode's pieces in order.
struct ConvTask {
  int t0, t1;
  int fault;       // the fault its tiles belong to (index into the launch's faults)
  int nsum;        // packed rows: the task's wave sums (LDS slots); else 0
};
constexpr int kConvThreads = 512;   // 8 wavefronts
constexpr int kTileSlots32 = 512;   // FP32 records per wavefront tile
constexpr int kWaveTiles32 = 2;     // FP32 tiles per wavefront and task
constexpr int kTaskTiles32 = kWaveTiles32 * (kConvThreads / 64);
// FP32 tiles of the short windows the learned closure keeps: half the
// records per tile, twice the tiles per wave (the same 16 rows of 64
// records in flight per wave)
constexpr int kTileSlots32s = 256;
constexpr int kWaveTiles32s = 4;
constexpr int kTaskTiles32s = kWaveTiles32s * (kConvThreads / 64);
// FP32 tile shapes the conv can take (records per tile; 16 rows in flight per
// wave, so every task is 8192 records): 256 (short windows), 512, 1024
constexpr int kTileSlots32l = 1024;
// A wider shape: five rows per tile and four tiles per wave, 20 rows in flight
// per wave (the most the vector registers hold at two workgroups per CU)
constexpr int kTileSlots32w = 320;
constexpr int kWaveTiles32w = 4;
// FP32 tiles per wave of a tile shape (records per tile)
constexpr int conv32_wave_tiles(int tile) {
  return tile == kTileSlots32w ? kWaveTiles32w : 16 / (tile / 64);
}
// The packed FP32 layout: one 64-record row per unit, the rows of one mode
// and of consecutive modes filling each wave's 16 rows (no row past a mode's
// end); a task is 128 rows, whatever the modes.
constexpr int kTileSlots32p = 64;
constexpr int kConvStaticLds = 6144;  // bound on the FP32 conv's static LDS (task sums)
constexpr int kPackRows = 16;                               // rows per wave and task
constexpr int kTaskRows = kPackRows * (kConvThreads / 64);  // rows per task
// A packed row as the conv reads it (48 B: a wave's 16 rows are 768 B, three
// words per lane).  word = len | (flush slot + 1) << 8 | run << 16: the row's
// records, the task's LDS slot of the wave sum that ends at this row (0:
// none), and at the first slot of a partial sum the number of its slots.
struct RowDesc {
  const void* rec;            // the row's first record
  unsigned word;
  int p0;                     // mode-local slot of that record
  int Rn, MT, MN;
  int part;
  double th;
  unsigned long long rmagic;
};
static_assert(sizeof(RowDesc) == 48, "packed row descriptor");
constexpr int kTileSlots64 = 256;   // FP64 records per wavefront tile
constexpr int kTaskTiles64 = 16;
constexpr int kTaskTiles = kTaskTiles32s > kTaskTiles64 ? kTaskTiles32s : kTaskTiles64;  // at most
static_assert(kTaskTiles >= kTaskTiles32 && kTaskTiles >= kTaskTiles32s, "task slots");
constexpr int kModeThreads = 256;   // mode-stage workgroups
constexpr int kElemThreads = 256;   // element-stage workgroups
constexpr double kTableStep = 1.0 / 16.0;  // spacing of the FP32 kernel table in T
constexpr int kMaxLdsBytes = 160 * 1024;
constexpr int kMaxDynLds = kMaxLdsBytes - 4096;  // room for static LDS (reductions)

// Launch arguments of a variable step (on = 0: the fixed-step engine, which
// takes dt and times from the fault descriptor).
struct VarArgs {
  double dt;      // length of the step
  double t_old;   // committed time at the start of the step
  double t_new;   // t_old + dt
  int on;
  int nohist;     // every stored interval is past every window: history sums are 0
};

// Quintic Hermite evaluation of the primitive table at T >= 0 (clamped to
// the last cell): P^T and P^N from the nodes' values, first (C) and second
// (C') derivatives.
__host__ __device__ inline void ptab_eval(const double* __restrict__ tab, int len, double h,
                                          double T, double* PT, double* PN) {
  double x = T / h;
  int i = (int)x;
  if (i > len - 2) i = len - 2;
  if (i < 0) i = 0;
  const double t = x - (double)i;
  const double t2 = t * t, t3 = t2 * t, t4 = t3 * t, t5 = t4 * t;
  const double h0 = 1.0 - 10.0 * t3 + 15.0 * t4 - 6.0 * t5;
  const double h1 = (t - 6.0 * t3 + 8.0 * t4 - 3.0 * t5) * h;
  const double h2 = 0.5 * (t2 - 3.0 * t3 + 3.0 * t4 - t5) * h * h;
  const double h3 = 10.0 * t3 - 15.0 * t4 + 6.0 * t5;
  const double h4 = (-4.0 * t3 + 7.0 * t4 - 3.0 * t5) * h;
  const double h5 = 0.5 * (t3 - 2.0 * t4 + t5) * h * h;
  const double* a = tab + 6 * (size_t)i;
  const double* b = a + 6;
  *PT = h0 * a[0] + h1 * a[1] + h2 * a[2] + h3 * b[0] + h4 * b[1] + h5 * b[2];
  *PN = h0 * a[3] + h1 * a[4] + h2 * a[5] + h3 * b[3] + h4 * b[4] + h5 * b[5];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct DeviceAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
DeviceAllocator& allocator();
void* dev_alloc(size_t bytes);
void dev_free(void* p);

// Extended-precision kernel evaluation (kernel_eval.cpp).
void bessel_jw(long double x, long double* J0, long double* J1, long double* W);
// Sums of the weights dt C^T, dt C^N of lags Mk[i] .. M[i] - 1 of modes n[i]
// (the lags a closure discards), cubic Hermite on T = i h in FP64.
void discarded_weights(double cs, double cp, double L, double dt, const std::vector<int>& n,
                       const std::vector<int>& Mk, const std::vector<int>& M, std::vector<double>* DT,
                       std::vector<double>* DN);
void kernel_values(long double T, long double cs, long double cp, long double* CT,
                   long double* CN, long double* dCT, long double* dCN);
// Primitives P^T, P^N of the kernels at T (integrals over [0, T]).
void kernel_primitives(long double T, long double cs, long double cp, long double* PT,
                       long double* PN);

// Owner of a device allocation list.
struct DevArena {
  std::vector<void*> ptrs;
  void* get(size_t bytes);
  void release_all();
  ~DevArena() { release_all(); }
};

// Tables and ring for one (plan, dt).
struct DtData {
  double dt = 0.0;
  std::vector<int> M;            // M_n, n = 0..N/2
  std::vector<int> Rn;           // ring capacity
  std::vector<long long> ring_off;
  long long ring_slots = 0;
  std::vector<Tile> tiles;       // this fault's tiles (fault field = 0); packed: its rows
  std::vector<int2> row_meta;    // packed rows: (flush slot or -1, run length)
  int tile_slots = 0;            // records per tile (kTileSlots32p: packed rows)
  std::vector<ConvTask> tasks;   // this fault's tasks (tile indices local)
  std::vector<int> part0, nparts;
  int parts_cap = 0;             // partial sums the parts buffer holds
  std::vector<ModeCoef> coef_host;  // host copy of coef (retiling rewrites part0, nparts)
  int table_len = 0;             // FP32 table nodes
  DevArena mem;
  ModeCoef* coef = nullptr;      // at mode_pos
  double4* parts = nullptr;
  void* ring = nullptr;
  double2* wrev = nullptr;
  float4* table = nullptr;       // FP32 kernel table: dt*(C^T, h C^T', C^N, h C^N')
  std::vector<ClosureMode> closure;  // closed modes (fault field 0)
  double4* tails = nullptr;          // closure tails at mode_pos (zero for open modes)
  std::vector<double> th_mode;       // table coordinate step theta_n / h per mode
  std::vector<int> MT, MN;           // window lengths of the shear and normal kernels
  bool var = false;                  // variable-step engine (ring of M_n + 1 intervals)
  double* ptab = nullptr;            // primitive table (variable-step engine)
  int ptab_len = 0;
  double ptab_h = 0.0;
  double2* tlog = nullptr;           // interval times (variable-step engine)
  int tlog_cap = 0;
};

// Device snapshot of the committed state for step doubling (variable-step
// engine): both state buffers, the spectral slip and rate accumulators and
// the step counter; the full step's rate and state for the error measure.
// Up to kMaxCopies device copies (or zero fills: src null) in one launch;
// sizes in 8-byte words.
constexpr int kMaxCopies = 24;
struct CopyList {
  int n = 0;
  const void* src[kMaxCopies] = {};
  void* dst[kMaxCopies] = {};
  long long words[kMaxCopies] = {};
  void add(const void* from, void* to, size_t bytes) {
    src[n] = from;
    dst[n] = to;
    words[n] = (long long)(bytes / 8);
    ++n;
  }
};

struct VarSnap {
  DevArena mem;
  double* el[12] = {};
  double2* sp[6] = {};
  long long* step = nullptr;
  double *Vf = nullptr, *thf = nullptr;
  // [0] error measure bits, [1] maximum slip rate bits, [2] failure status,
  // [3] failing elements << 32 | first failing element
  unsigned long long* eps = nullptr;
  CopyList save, restore, keep_full;  // snapshot save / restore (+ clear eps[0..1]),
                                      // full-step solution -> Vf, thf
};

// Dynamic state of one fault.
struct DynData {
  DevArena mem;
  double *slip[2], *V[2], *theta[2], *thd[2], *V1, *thd1, *tau_el[2], *sigma_el[2];
  double2 *u_hat, *g_hat, *v_hat0, *gv_hat0, *v_hat1, *gv_hat1, *hprev_v, *hprev_g, *B_T,
      *B_N;
  void *gI, *gF;
  int *cells, *done;
  long long* step;
  int *err, *err_count, *err_index;
  // the pass-1 spectra of the next step are in gI/B (set by a step's last
  // launch; cleared whenever the state, dt or frame changes)
  bool primed = false;
};

// Events bracketing conv launches while profiling (two per step, reused).
struct EventPool {
  std::vector<hipEvent_t> ev;
  hipError_t ensure(size_t n);
  ~EventPool();
};

// Execution context: the fault list and conv tiles of one launch sequence.
struct Exec {
  int precision = SBIEM_FP64;
  int nfaults = 0;
  std::vector<FaultDev> host_faults;
  FaultDev* d_faults = nullptr;
  Tile* d_tiles = nullptr;
  int ntiles = 0;
  ConvTask* d_tasks = nullptr;
  int ntasks = 0;
  int2* d_mode_map = nullptr;    // per mode workgroup: fault, group
  int mode_blocks = 0;
  int2* d_elem_map = nullptr;    // per element workgroup: fault, first class
  int elem_blocks = 0;
  size_t mode_lds = 0, elem_lds = 0;
  std::vector<DynData*> dyns;
  const float4* table = nullptr;  // FP32 kernel table (shared by all faults)
  int table_len = 0;
  int conv_grid = 0;
  int tile_rows = kTileSlots32 / 64;  // FP32: 64-record rows per conv tile (8, or 4 for short windows)
  bool stages_first = false;     // enqueue a step's first stage launch before its conv launch
  bool closure_main = false;     // closure network on the stage stream (before the first stage)
  bool cached_loads = false;     // FP32 conv record loads with the default cache policy (else streamed)
  int* conv_ctr = nullptr;        // FP32 conv: dynamic task counter (zeroed by the mode launch after it)
  ClosureMode* closure_modes = nullptr;  // closed modes of every fault (null: no closure)
  int nclosure = 0;
  const void* net_frag[2] = {nullptr, nullptr};  // closure networks (shear, normal)
  const float* net_bias[2] = {nullptr, nullptr};
  double conv_bytes = 0.0;        // algorithmic bytes per conv launch
  DevArena mem;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  int graph_steps = 0;
  hipStream_t graph_stream = nullptr;
  hipStream_t aux = nullptr;     // second stream: the next step's convolution
  hipEvent_t fork = nullptr, join = nullptr;
  ~Exec();
  void drop_graph();
};

}  // namespace sbiem

struct sbiem_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;

  int64_t N = 0;
  int log2N = 0, log2P = 0, log2Q = 0, ncls = 1;
  double L = 0, mu = 0, nu = 0, cs = 0, cp = 0, r = 0;
  int precision = SBIEM_FP64;
  int theta_mode = SBIEM_THETA_PAPER;
  int newton_max = 100;                // FP64 Newton iterations per solve
  int rule = SBIEM_RULE_MIDPOINT;      // history weights
  double kcL[2] = {200.0, 200.0};      // k_c L of the shear and normal windows
  bool adaptive = false;               // variable steps (dt of set_dt = dt_min)
  double t_var = 0.0;                  // committed time on the variable-step engine
  int64_t var_accepted = 0;            // steps accepted by sbiem_adapt since set_state
  // host copy of the committed intervals' end times on the variable-step
  // engine: interval l at l mod tlog_cap, the last one var_b (-1: none)
  std::vector<double> var_tend;
  long long var_b = -1;
  int var_prof_pending = 0;            // evented conv launches not yet read
  double prof_bytes = 0.0;             // algorithmic bytes of the evented var conv launches
  sbiem::VarSnap* snap = nullptr;      // step-doubling snapshot buffers

  bool friction_set = false, state_set = false;
  double Dc = 0, V_ref = 0, f0 = 0, tau_rate = 0, V_pl = 0, t0 = 0;
  int conv_tile = 0;                   // FP32 conv tile records (0: by window length)
  bool conv_tile_set = false;          // set by sbiem_set_conv_tile: tuning keeps it
  std::vector<double> a_host;          // direct effect a as set (natural order)
  std::vector<uint8_t> constrained;    // elements held at V_pl (empty: none)

  sbiem::DevArena mem;                 // per-element constants, twiddles
  double *a = nullptr, *b = nullptr, *sigma_load = nullptr, *tau_load = nullptr,
         *kappa = nullptr;
  void* twiddle = nullptr;             // quarter-wave table, convolution precision
  void* twiddle64 = nullptr;           // the same table in FP64 (slip transforms of set-up paths)
  std::vector<double> kappa_host;
  double fwd_scale = 1.0;              // 2^-ilogb(max|kappa|)

  sbiem::FaultDev* d_desc = nullptr;   // device copy of this fault's descriptor
  sbiem::DtData* dtd = nullptr;        // tables + ring for the stepping dt
  sbiem::DynData* dyn = nullptr;       // stepping state
  sbiem::Exec* exec = nullptr;         // single-fault launch context

  bool profiling = false;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  sbiem::EventPool events;
  int last_fail_count = 0, last_fail_index = -1;
  int batch_refs = 0;

  // learned closure (FP32 convolution only)
  bool closure_on = false;
  double closure_cut = 0.25;
  std::vector<float> closure_params[2];  // shear, normal networks (host copies)
  sbiem::DevArena closure_mem;
  void* net_frag[2] = {nullptr, nullptr};
  float* net_bias[2] = {nullptr, nullptr};
};

struct sbiem_batch {
  std::vector<sbiem_plan*> plans;
  sbiem::Exec* exec = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  bool profiling = false;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  sbiem::EventPool events;
};

namespace sbiem {

// plan.cpp helpers shared with exec.cpp
int fail(sbiem_plan* p, int status, const std::string& msg);
int fail_global(int status, const std::string& msg);
int hip_fail(sbiem_plan* p, hipError_t e, const char* what);

// Natural element order (host) <-> class-major device order.
std::vector<double> to_elem_order(const sbiem_plan* p, const double* x);
hipError_t download_elems(const sbiem_plan* p, const double* dev, double* host);

// Plans stepped by the variable-step engine (adaptive, or FP32 on the
// interval rule).
bool var_engine(const sbiem_plan* p);

// Build the descriptor of a fault for an execution context.
FaultDev make_fault_desc(sbiem_plan* p, DtData* dtd, DynData* dyn, double V_pl, double t0);
// Allocate tables/ring for dt (host side computations + uploads).
int build_dt_data(sbiem_plan* p, double dt, DtData** out);
// Re-cut an FP32 fixed-step plan's conv work into tiles of `tile` records
// (64: packed rows, 256, 320, 512, 1024): tiles, tasks, partial indices and per-mode constants;
// the ring is untouched.  The caller rebuilds the execution context and
// clears `primed` (the pending sums are laid out by tile).
int retile(sbiem_plan* p, int tile);
// Rewrite the plan's device fault descriptor (and its launch context's).
int refresh_desc(sbiem_plan* p);
// Allocate the dynamic state buffers.
int build_dyn_data(sbiem_plan* p, DynData** out);
// Build an execution context over faults (tiles, partials, Newton map).
int build_exec(const std::vector<sbiem_plan*>& plans, const std::vector<DtData*>& dts,
               const std::vector<DynData*>& dyns, const std::vector<FaultDev>& descs,
               int precision, Exec** out, std::string* err);

// kernels.hip launchers
// ahead = 0: sums for the pending step; 1: for the step after it (launched
// beside the pending step's passes, which it does not conflict with)
hipError_t launch_conv(const Exec& ex, int ahead, hipStream_t s);
// mode stage: kind 0 = pass-1 assembly from the stored state (measure != 0:
// only the balance maxima), 1 = pass 2, 2 = commit and next pass 1 (a
// variable step commits only)
hipError_t launch_modes(const Exec& ex, int kind, int measure, hipStream_t s,
                        const VarArgs& va = VarArgs{0.0, 0.0, 0.0, 0, 0});
// element stage: kind 0 = tractions only, 1 = pass 1, 2 = pass 2
hipError_t launch_elems(const Exec& ex, int kind, hipStream_t s,
                        const VarArgs& va = VarArgs{0.0, 0.0, 0.0, 0, 0});
// variable steps: history sums over every stored interval at time va.t_new
// e0, e1 (optional): stamped with the kernel's start and end
hipError_t launch_conv_var(const Exec& ex, const VarArgs& va, hipStream_t s,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// balance cells of every fault to "no maximum yet"
hipError_t launch_reset_cells(const Exec& ex, hipStream_t s);
// out[0] = bits of max_i max(|ln Va - ln Vb|, |ln tha - ln thb|) (equal
// values count 0), out[1] = bits of max_i Vb (both zeroed first unless
// zeroed = true); with err (the fault's failure flags), out[2..3] receive
// them (status; count << 32 | index)
hipError_t launch_err_norm(const double* Va, const double* tha, const double* Vb,
                           const double* thb, int n, unsigned long long* out, hipStream_t s,
                           const int* err = nullptr, bool zeroed = false);
hipError_t launch_copy_many(const CopyList& c, int max_words, hipStream_t s);
// one fault: spectra A (of a) and B (of kappa a) at mode_pos for count real
// signals a (natural element order, stride N); gF holds count * N complex
hipError_t launch_forward(const FaultDev* d_fault, const FaultDev& h_fault, int precision,
                          const double* a, double2* A, double2* B, int count, long long stride_out,
                          void* gF, hipStream_t s);
// stress-only path: fill the ring of a fault from interval spectra
hipError_t launch_fill_ring(const FaultDev* d_fault, int precision, int nmodes,
                            const double2* RV, const double2* RG, int nint, hipStream_t s);
hipError_t launch_rates(const double* hist, double* rates, long long count, long long N, double dt,
                        hipStream_t s);
// closure.hip: tails of every closed mode (for the step the conv sums are for)
hipError_t launch_closure(const Exec& ex, int ahead, hipStream_t s);
// fragment-ordered bfloat16 weights and float32 biases of one network
void closure_pack(const float* params, std::vector<unsigned short>* frag, std::vector<float>* bias);
// kept lags M' = ceil(cut M) of a window of M lags, or M when the mode stays open
int closure_kept(int M, double cut);
// window lengths M_n (steps) of modes n = 0..N/2 for the cut-off k_c L
std::vector<int> window_steps(int64_t N, double L, double cs, double dt, double kcL);
// the conv work lists of a fault's ring (tiles or packed rows, tasks, partial
// sum indices, part0/nparts); returns the number of partial sums
int build_tiles(const sbiem_plan* p, DtData* d, int tile, long double th_unit);
int conv_grid_size(int precision, int ntasks, int table_len, int reserve);
int default_conv_reserve(double conv_bytes);
hipError_t setup_kernel_attributes(int precision);
size_t mode_lds_bytes(int precision, int log2Q);
size_t elem_lds_bytes(int precision, int log2P, int ncls);
// N = P Q with P = 2^floor(log2 N / 2); classes per element workgroup
void split_sizes(int log2N, int* log2P, int* log2Q, int* ncls);

}  // namespace sbiem

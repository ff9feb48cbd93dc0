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
  int part0;    // second conv partial of the mode (the first is parts[n])
  int nparts;   // number of partials (0: no history records)
};

// ---------------------------------------------------------------------------
// Device-visible description of one fault at one time step.  One array of
// these per execution context (a plan, a batch, a stress evaluation); the
// kernels index it by fault number.  Mode index n runs over 0..N/2 in every
// per-mode array (mode 0 carries no elastic term).
// ---------------------------------------------------------------------------
struct FaultDev {
  int N, log2N, nmodes;     // nmodes = N/2
  int theta_mode;
  double L, mu, r, cs, dt, eta_rad;
  double V_pl, Dc, V_ref, f0, tau_rate, t0, ln_V_ref;

  // per element (FP64, length N)
  const double *a, *b, *sigma_load, *tau_load, *kappa;
  double *slip[2], *V[2], *theta[2], *thd[2];  // committed state at [step & 1]
  double *V1, *thd1;                           // pass-1 solution
  double *tau_el[2], *sigma_el[2];             // last pass of the step at [(step+1) & 1]

  // spectral state (FP64 complex, length N/2+1)
  double2 *u_hat, *g_hat;       // F[slip - V_pl t], F[kappa (slip - V_pl t)]
  double2 *v_hat0, *gv_hat0;    // F[V - V_pl], F[kappa (V - V_pl)] at step start
  double2 *v_hat1, *gv_hat1;    // same for the pass-1 solution
  double2 *hprev_v, *hprev_g;   // rate spectra of the last committed interval
  double2 *P_T, *P_N;           // (1-r) u_hat + w1 hprev, set at commit
  double2 *B_T, *B_N;           // P + history sum S, set by pass 1 for pass 2
  int* inv_exp;                 // log2 balancing scale of the inverse packing
  double fwd_scale;             // power of two ~ 1/max|kappa| for the forward packing

  // per mode (length N/2+1)
  const ModeCoef* coef;
  const int* Rn;                // ring capacity M_n - 1 (0 for mode 0)
  const long long* ring_off;    // first ring record of mode n
  const double* theta_h;        // FP32 weights: c_s |k_n| dt / 2 / table spacing
  double4* parts;               // conv partials: (S_T re, im, S_N re, im)

  void* ring;                   // history records: float4 or 2 x double2 per slot
  const double2* wrev;          // FP64 weights per ring slot (see conv kernel)

  void* zbuf;                   // N complex in convolution precision (FFT input)
  const void* twiddle;          // N/4+1 values cos(2 pi t / N), convolution precision

  long long* step;              // committed steps since state/dt were set
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
  int pad0, pad1;
  long long ring_off;
  double th;       // FP32 weights: c_s |k_n| dt / 2 / table spacing
};

// A conv task: tiles [t0, t1) of one fault, handled by one workgroup.  A task
// holds whole modes, or one piece of a mode longer than kTaskTiles tiles; it
// writes one FP64 partial sum per (task, mode) and the spectral kernel adds a
// mode's pieces in order.
struct ConvTask {
  int t0, t1;
};
constexpr int kTaskTiles = 16;  // at most this many tiles per task

constexpr int kTileSlots32 = 512;   // FP32 records per wavefront tile
constexpr int kTileSlots64 = 256;   // FP64 records per wavefront tile
constexpr int kConvThreads = 512;   // 8 wavefronts
constexpr int kSpecThreads = 1024;  // spectral (FFT) kernels
constexpr int kNewtonThreads = 64;
constexpr double kTableStep = 1.0 / 16.0;  // spacing of the FP32 kernel table in T
constexpr int kMaxLdsBytes = 160 * 1024;
constexpr int kMaxDynLds = kMaxLdsBytes - 4096;  // room for static LDS (reductions)

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
void kernel_values(long double T, long double cs, long double cp, long double* CT,
                   long double* CN, long double* dCT, long double* dCN);

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
  std::vector<Tile> tiles;       // this fault's tiles (fault field = 0)
  std::vector<ConvTask> tasks;   // this fault's tasks (tile indices local)
  std::vector<int> part0, nparts;
  int table_len = 0;             // FP32 table nodes
  DevArena mem;
  ModeCoef* coef = nullptr;
  double* theta_h = nullptr;
  int* d_Rn = nullptr;
  long long* d_ring_off = nullptr;
  double4* parts = nullptr;
  void* ring = nullptr;
  double2* wrev = nullptr;
  float4* table = nullptr;       // FP32 kernel table: dt*(C^T, h C^T', C^N, h C^N')
};

// Dynamic state of one fault.
struct DynData {
  DevArena mem;
  double *slip[2], *V[2], *theta[2], *thd[2], *V1, *thd1, *tau_el[2], *sigma_el[2];
  double2 *u_hat, *g_hat, *v_hat0, *gv_hat0, *v_hat1, *gv_hat1, *hprev_v, *hprev_g, *B_T,
      *B_N, *P_T, *P_N;
  int* inv_exp;
  void* zbuf;
  long long* step;
  int *err, *err_count, *err_index;
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
  int2* d_newton_map = nullptr;  // per Newton block: fault, first element
  int newton_blocks = 0;
  int max_N = 0;
  const float4* table = nullptr;  // FP32 kernel table (shared by all faults)
  int table_len = 0;
  int conv_grid = 0;
  double conv_bytes = 0.0;        // algorithmic bytes per conv launch
  DevArena mem;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  int graph_steps = 0;
  hipStream_t graph_stream = nullptr;
  ~Exec();
  void drop_graph();
};

}  // namespace sbiem

struct sbiem_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;

  int64_t N = 0;
  int log2N = 0;
  double L = 0, mu = 0, nu = 0, cs = 0, cp = 0, r = 0;
  int precision = SBIEM_FP64;
  int theta_mode = SBIEM_THETA_PAPER;

  bool friction_set = false, state_set = false;
  double Dc = 0, V_ref = 0, f0 = 0, tau_rate = 0, V_pl = 0, t0 = 0;

  sbiem::DevArena mem;                 // per-element constants, twiddles
  double *a = nullptr, *b = nullptr, *sigma_load = nullptr, *tau_load = nullptr,
         *kappa = nullptr;
  void* twiddle = nullptr;             // quarter-wave table, convolution precision
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

// Build the descriptor of a fault for an execution context.
FaultDev make_fault_desc(sbiem_plan* p, DtData* dtd, DynData* dyn, double V_pl, double t0);
// Allocate tables/ring for dt (host side computations + uploads).
int build_dt_data(sbiem_plan* p, double dt, DtData** out);
// Allocate the dynamic state buffers.
int build_dyn_data(sbiem_plan* p, DynData** out);
// Build an execution context over faults (tiles, partials, Newton map).
int build_exec(const std::vector<sbiem_plan*>& plans, const std::vector<DtData*>& dts,
               const std::vector<DynData*>& dyns, const std::vector<FaultDev>& descs,
               int precision, Exec** out, std::string* err);

// kernels.hip launchers
hipError_t launch_conv(const Exec& ex, hipStream_t s);
hipError_t launch_pass1(const Exec& ex, hipStream_t s);
hipError_t launch_newton(const Exec& ex, int pass, hipStream_t s);
hipError_t launch_pass2(const Exec& ex, hipStream_t s);
hipError_t launch_commit(const Exec& ex, hipStream_t s);
hipError_t launch_step(const Exec& ex, hipStream_t s, bool profile, hipEvent_t e0, hipEvent_t e1);
// one fault: forward FFT of two real FP64 signals packed as z = a + i b
// (a, b device arrays of length N), unpacked spectra n = 0..N/2 into A, B
hipError_t launch_spectra(const FaultDev* d_fault, int precision, int max_N, const double* a,
                          const double* b, double scale_b_by_kappa, double2* A, double2* B,
                          int count, long long stride_in, long long stride_out, hipStream_t s);
// stress-only path: fill the ring of a fault from interval spectra
hipError_t launch_fill_ring(const FaultDev* d_fault, int precision, int nmodes,
                            const double2* RV, const double2* RG, int nint, hipStream_t s);
// P = (1-r) u_hat + w1 hprev for every mode and an unset inverse scale
hipError_t launch_prepare(const FaultDev* d_fault, int nmodes, hipStream_t s);
hipError_t launch_rates(const double* hist, double* rates, long long count, long long N, double dt,
                        hipStream_t s);
int conv_grid_size(int precision, int ntasks, int table_len);
hipError_t setup_kernel_attributes(int precision);

}  // namespace sbiem

// HIP kernels of the sBIEM time step for gfx950 (CDNA4, wave64).
//
// One step (section 3.3) runs over every fault of a context as
//   k_conv     history sums over lags >= 2 of every mode for the NEXT step
//              (HBM-bound stream of the wavenumber-major ring), on a second
//              stream beside the three launches below
//   k_elems<1> inverse-transform finish -> tau^el, sigma^el; pass-1 momentum
//              balance per element (Newton on ln V); forward-transform start
//   k_modes<1> forward-transform finish -> rate spectra of pass 1; pass-2
//              traction assembly; inverse-transform start
//   k_elems<2> the same for pass 2 (writes the next state)
//   k_modes<2> forward-transform finish of V_2; commit (ring push of the
//              interval rate, spectral slip, step counter) and the pass-1
//              assembly of the next step with the sums k_conv produced
// The transforms are four-step FFTs split between element and mode
// workgroups (see the index maps in internal.h).
#include <hip/hip_ext.h>

#include "internal.h"

#include <algorithm>
#include <cstdint>
#include <utility>

#include <hip/hip_runtime.h>

namespace sbiem {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename R> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };

template <typename C> __device__ __forceinline__ C cmk(double x, double y) {
  C c;
  c.x = x;
  c.y = y;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C c; c.x = a.x - b.x; c.y = a.y - b.y; return c; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C c;
  c.x = a.x * b.x - a.y * b.y;
  c.y = a.x * b.y + a.y * b.x;
  return c;
}
template <typename C> __device__ __forceinline__ C cmul_mi(C a) { C c; c.x = a.y; c.y = -a.x; return c; }  // -i a

__device__ __forceinline__ double2 d2(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ double2 d2add(double2 a, double2 b) { return d2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 d2scale(double2 a, double s) { return d2(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// Radix-8/4/2 butterflies and twiddles for LDS Stockham FFTs (forward,
// exp(-2 pi i n k / M)).
// ---------------------------------------------------------------------------
template <typename C> __device__ __forceinline__ void dft2(C* x) {
  C a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  C t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = cmul_mi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  C x1 = cadd(t1, t3), x3 = csub(t1, t3);
  a1 = x1;
  a3 = x3;
}

template <typename C> __device__ __forceinline__ void dft8(C* x) {
  C e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  C o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const double h = 0.70710678118654752440;
  // W8^1 = (1 - i)/sqrt2, W8^2 = -i, W8^3 = (-1 - i)/sqrt2
  C w1, w2, w3;
  w1.x = (o1.x + o1.y) * h;
  w1.y = (o1.y - o1.x) * h;
  w2 = cmul_mi(o2);
  w3.x = (o3.y - o3.x) * h;
  w3.y = -(o3.x + o3.y) * h;
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, w1);
  x[5] = csub(e1, w1);
  x[2] = cadd(e2, w2);
  x[6] = csub(e2, w2);
  x[3] = cadd(e3, w3);
  x[7] = csub(e3, w3);
}

// exp(-2 pi i m / N) for m in [0, N/2) from the quarter-wave table
// q[r] = cos(2 pi r / N), r = 0..N/4 (sin(2 pi r / N) = q[N/4 - r]),
// branch-free.
template <typename C, typename R>
__device__ __forceinline__ C twiddle_half(const R* __restrict__ q, int m, int N) {
  const int Q = N >> 2;
  const bool hi = m >= Q;  // angle in [pi/2, pi)
  const int r = hi ? m - Q : m;
  const R a = q[r], b = q[Q - r];  // cos, sin of the reduced angle
  C w;
  w.x = hi ? -b : a;   // cos
  w.y = hi ? -a : -b;  // -sin
  return w;
}

// LDS index of complex element x: one pad element per 2^ps elements, which
// spreads the power-of-two strides of the Stockham passes over all banks.
__device__ __forceinline__ int lx(int x, int ps) { return x + (x >> ps); }

template <typename R> struct Prec;
template <> struct Prec<float> {
  using C = float2;
  using Rec = float4;  // (v_re, v_im, g_re, g_im)
  static constexpr int kTile = kTileSlots32;
};
struct Rec64 {
  double2 v, g;
};
template <> struct Prec<double> {
  using C = double2;
  using Rec = Rec64;
  static constexpr int kTile = kTileSlots64;
};

// ---------------------------------------------------------------------------
// History convolution for step s (s = the committed-step counter, plus one
// when the launch computes the sums a step ahead).  Slot p of mode n's ring
// holds interval I(p) = b - ((b - p) mod R_n) with b = s - 1 the last
// interval committed before step s; its lag at step s is
// j = 1 + ((b - p) mod R_n).  The slot of lag 1 (p = b mod R_n) is skipped
// here (the mode stage adds it from h_prev): it is the slot that step s - 1
// commits into, so the sums for step s can run while step s - 1 is still in
// its passes.  The weight of slot p is at q = (p - b) mod R_n = (p + o) mod R_n
// with o = (-b) mod R_n: q = 0 is the skipped slot, lag j = R_n - q + 1
// otherwise.
// ---------------------------------------------------------------------------
// Wavefront sum without LDS traffic: DPP exchanges inside each row of 16
// lanes (quad swaps, then half-row and row mirrors leave every lane with its
// row's sum), then row broadcasts: lane 15 of rows 0 and 2 is added into
// rows 1 and 3, lane 31 into rows 2 and 3, and lane 63 holds
// (r2 + r3) + (r0 + r1).  The result is uniform and its summation order
// fixed.  Rows outside a broadcast's row mask add the zero of `old`.
template <int C, int RowMask = 0xF>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), C, RowMask, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_mov<0xB1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);       // row_half_mirror
  v += dpp_mov<0x140>(v);       // row_mirror
  v += dpp_mov<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float4 wave_reduce4(float4 v) {
  return make_float4(wave_sum(v.x), wave_sum(v.y), wave_sum(v.z), wave_sum(v.w));
}
__device__ __forceinline__ Rec64 wave_reduce_r64(Rec64 v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v.v.x += __shfl_xor(v.v.x, off);
    v.v.y += __shfl_xor(v.v.y, off);
    v.g.x += __shfl_xor(v.g.x, off);
    v.g.y += __shfl_xor(v.g.y, off);
  }
  return v;
}

__device__ __forceinline__ long long posmod(long long a, long long m) {
  long long r = a % m;
  return r < 0 ? r + m : r;
}

// a mod m for 0 <= a < 2^52, 0 < m < 2^31 (FP64 quotient estimate, corrected)
__device__ __forceinline__ int mod_pos(long long a, int m) {
  long long q = (long long)((double)a / (double)m);
  long long r = a - q * (long long)m;
  if (r < 0) r += m;
  if (r >= m) r -= m;
  return (int)r;
}

// Offset o = (-b) mod R with b = step - 1 >= -1.
__device__ __forceinline__ int ring_phase(long long step, int Rn) {
  const long long b = step - 1;
  if (b < 0) return 1 % Rn;
  const int r = mod_pos(b, Rn);
  return r == 0 ? 0 : Rn - r;
}

// a mod d for 32-bit a by multiplication with M = floor((2^64 - 1) / d) + 1
// (Lemire, Kaser and Kurz, "Faster remainder by direct computation", 2019):
// the high 64 bits of the 96-bit product (M a mod 2^64) d.  Every operand is
// uniform in the FP32 conv, so this runs on the scalar unit.
__device__ __forceinline__ unsigned fastmod_u32(unsigned a, unsigned long long M, unsigned d) {
  const unsigned long long low = M * a;
  const unsigned lo = (unsigned)low, hi = (unsigned)(low >> 32);
  const unsigned long long t = (unsigned long long)hi * d + __umulhi(lo, d);
  return (unsigned)(t >> 32);
}
// ring_phase with the multiplier of R (steps beyond 2^32 take the FP64 path)
__device__ __forceinline__ int ring_phase_m(long long step, int Rn, unsigned long long M) {
  const long long b = step - 1;
  if (b < 0) return 1 % Rn;
  const int r = b < (1LL << 32) ? (int)fastmod_u32((unsigned)b, M, (unsigned)Rn) : mod_pos(b, Rn);
  return r == 0 ? 0 : Rn - r;
}

// One workgroup per task (a run of tiles of one fault): each wave sums tiles
// of the task, the per-tile FP64 partials go to LDS, and after a barrier the
// first thread of each (task, mode) run adds its tiles in order and stores
// the sum in parts[part].  The spectral kernel adds a mode's parts in order,
// so every sum has a fixed order and results are reproducible.
struct TaskLds {
  double4 part[kTaskTiles];
  int id[kTaskTiles];
};

__device__ __forceinline__ void finish_task(double4* parts, const TaskLds& L, int nt) {
  const int k = threadIdx.x;
  if (k < nt && (k == 0 || L.id[k - 1] != L.id[k])) {
    double4 a = L.part[k];
    for (int j = k + 1; j < nt && L.id[j] == L.id[k]; ++j) {
      const double4 b = L.part[j];
      a.x += b.x;
      a.y += b.y;
      a.z += b.z;
      a.w += b.w;
    }
    // a global-segment store: a flat store counts as a possible LDS access,
    // and the waits for records in flight behind it would then drain them all
    typedef double d4v __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) d4v* gd4p;
    const d4v v = {a.x, a.y, a.z, a.w};
    ((gd4p)(d4v*)parts)[L.id[k]] = v;
  }
}
__device__ __forceinline__ void finish_task(const FaultDev& fd, const TaskLds& L, int nt) {
  finish_task(fd.parts, L, nt);
}

__global__ void __launch_bounds__(kConvThreads)
k_conv64(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles,
         const ConvTask* __restrict__ tasks, int ntasks, int ahead) {
  constexpr int U = kTileSlots64 / 64;
  __shared__ TaskLds L;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wpb = kConvThreads / 64;
  for (int task = blockIdx.x; task < ntasks; task += gridDim.x) {
    const ConvTask tk = tasks[task];
    const int nt = tk.t1 - tk.t0;
    const FaultDev& fd = faults[tiles[tk.t0].fault];
    const int err = *fd.err;
    const long long step = *fd.step + ahead;
    for (int k = wave; k < nt; k += wpb) {
      const Tile tl = tiles[tk.t0 + k];
      Rec64 acc;
      acc.v = d2(0, 0);
      acc.g = d2(0, 0);
      if (err == 0) {
        const int Rn = tl.Rn;
        const int o = ring_phase(step, Rn);
        const Rec64* __restrict__ ring = (const Rec64*)fd.ring + tl.ring_off;
        const double2* __restrict__ w = fd.wrev + tl.ring_off;
        const int end = tl.p0 + tl.len;
        Rec64 h[U];
        double2 wt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int p = tl.p0 + lane + 64 * u;
          int q = p + o;
          q -= (q >= Rn) ? Rn : 0;
          if (p < end) {
            h[u] = ring[p];
            wt[u] = w[q];
          } else {
            h[u].v = d2(0, 0);
            h[u].g = d2(0, 0);
            wt[u] = d2(0, 0);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          acc.v.x = fma(wt[u].x, h[u].v.x, acc.v.x);
          acc.v.y = fma(wt[u].x, h[u].v.y, acc.v.y);
          acc.g.x = fma(wt[u].y, h[u].g.x, acc.g.x);
          acc.g.y = fma(wt[u].y, h[u].g.y, acc.g.y);
        }
      }
      acc = wave_reduce_r64(acc);
      if (lane == 0) {
        L.part[k] = make_double4(acc.v.x, acc.v.y, acc.g.x, acc.g.y);
        L.id[k] = tl.part;
      }
    }
    __syncthreads();
    finish_task(fd, L, nt);
    __syncthreads();
  }
}

// FP32 records with weights interpolated from an LDS table of
// dt*(C^T, h dC^T/dT, C^N, h dC^N/dT) at T = i h (cubic Hermite).  The kernel
// argument of lag j is T = c_s |k_n| (j + 1/2) dt = (2j + 1) theta_n; the
// table coordinate (2j + 1) theta_n / h is formed in FP64 so that the phase
// keeps full accuracy at T ~ 200.
//
// Each wave of a workgroup task owns tiles k = wave + W i, i < K (W waves
// per workgroup); a tile is U rows of 64 records (U K = 16 rows per wave:
// 2 tiles of 8 rows for full windows, 4 of 4 for the short windows of the
// learned closure).  The records of the next task's tiles are requested as
// soon as the registers of the current tile are free, so loads stay in
// flight across the weighting, the wave reductions and the task's barriers.
//
// Everything a task needs besides its records (its tile descriptors, its
// fault's step counter, failure flag and output pointer) is requested one
// task ahead as well: the descriptors stream from HBM once per step, and a
// scalar load's result cannot be awaited apart from other scalar loads, so
// a descriptor fetched right before its records' loads would stall the wave
// for a full memory round trip once per tile.  The K descriptors of a wave's
// next tiles are fetched together after its first tile is weighed (one round
// trip per task), the next task's indices at the end of the task before.

// Per-fault words that a launch only reads (failure flag, step counter) are
// read with scalar loads: the vector-memory counter then tracks record loads
// alone, so waiting for these words never waits for records in flight.
__device__ __forceinline__ int read_word(const int* p) {
  return *(const __attribute__((address_space(4))) int*)p;
}
__device__ __forceinline__ long long read_word(const long long* p) {
  return *(const __attribute__((address_space(4))) long long*)p;
}

// The ring is streamed once per step.  Its loads take the cache policy POL:
// non-temporal by default, which keeps the ring from displacing what the
// stage launches beside the conv reuse; the autotuner also tries the default
// policy, which shortens the step where the ring is far larger than the
// caches (measured: the plain ensemble16-N262144 step 2 % faster, the conv
// launch itself unchanged; rough-N65536, ensemble64 and seamount-N8192 5-7 %
// slower, the closure form 1.3 % slower).  A tile's records
// are read through a buffer resource that spans exactly its len records:
// lanes past the tile's end (and every lane of a wave without a tile, whose
// range is empty) fall outside the range check, read 0 and touch no memory,
// while every pass of the task loop still issues the same number of loads,
// so the wait for a tile's records counts exactly the loads issued after
// them and never drains the next task's loads.  Buffer loads wait on the
// vector-memory counter only, so LDS reads of the table never wait for
// records still in flight.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
constexpr int kLoadStream = 2;            // non-temporal cache policy
constexpr int kLoadCached = 0;            // default cache policy

// The fields of a tile the FP32 conv keeps in scalar registers: those that
// address its records, fetched first, and those that weigh them.
struct TileR {
  const void* rec;
  int p0, len;
  int Rn, part, MT, MN;
  double th;
  unsigned long long rmagic;
};
__device__ __forceinline__ void tile_address(TileR& r, const Tile* tp) {
  r.rec = tp->rec;
  r.p0 = tp->p0;
  r.len = tp->len;
}
__device__ __forceinline__ void tile_weights(TileR& r, const Tile* tp) {
  r.Rn = tp->Rn;
  r.part = tp->part;
  r.MT = tp->MT;
  r.MN = tp->MN;
  r.th = tp->th;
  r.rmagic = tp->rmagic;
}

template <int U, int POL>
__device__ __forceinline__ void conv32_load(const TileR& tl, bool has, int lane, float4 (&h)[U]) {
  const float4* base = (const float4*)tl.rec + (has ? tl.p0 : 0);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, has ? tl.len * 16 : 0, kBufferWord3);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // the whole offset stays in the address register (not the instruction's
    // offset field), where the range check certainly applies
    int off = (lane + 64 * u) * 16;
    asm volatile("" : "+v"(off));
    const f4v t = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, POL));
    h[u] = make_float4(t.x, t.y, t.z, t.w);
  }
}

template <int U>
__device__ __forceinline__ float4 conv32_weigh(const TileR& tl, long long step, int lane,
                                               const float4 (&h)[U], const float4* tab,
                                               int table_len) {
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const int Rn = tl.Rn;
  const int o = ring_phase_m(step, Rn, tl.rmagic);
  const double th = tl.th;
  const int end = tl.p0 + tl.len;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (64 * u >= tl.len) {
      // a row past the tile's end (short modes, most of them under the
      // learned closure): no weights, only mark its registers as read so
      // that every row still waits for exactly its own loads
      asm volatile("" ::"v"(h[u].x), "v"(h[u].y), "v"(h[u].z), "v"(h[u].w));
      continue;
    }
    const int p = tl.p0 + lane + 64 * u;
    int q = p + o;
    q -= (q >= Rn) ? Rn : 0;
    const int j = Rn - q + 1;                       // lag (q = 0: skipped slot)
    const double x = (double)(2 * j + 1) * th;
    const int i = min((int)x, table_len - 2);
    const float f = (float)(x - (double)i);
    const float4 n0 = tab[i], n1 = tab[i + 1];
    const float f2 = f * f, f3 = f2 * f;
    const float h00 = 2.f * f3 - 3.f * f2 + 1.f;
    const float h10 = f3 - 2.f * f2 + f;
    const float h01 = 3.f * f2 - 2.f * f3;
    const float h11 = f3 - f2;
    float wT = h00 * n0.x + h10 * n0.y + h01 * n1.x + h11 * n1.y;
    float wN = h00 * n0.z + h10 * n0.w + h01 * n1.z + h11 * n1.w;
    const bool use = (q != 0) && (p < end);
    wT = (use && j < tl.MT) ? wT : 0.f;   // each kind's own window
    wN = (use && j < tl.MN) ? wN : 0.f;
    acc.x = fmaf(wT, h[u].x, acc.x);
    acc.y = fmaf(wT, h[u].y, acc.y);
    acc.z = fmaf(wN, h[u].z, acc.z);
    acc.w = fmaf(wN, h[u].w, acc.w);
  }
  return acc;
}

template <int U, int K, int POL>
__global__ void __launch_bounds__(kConvThreads)
k_conv32(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles,
         const ConvTask* __restrict__ tasks, int ntasks, const float4* __restrict__ table,
         int table_len, int ahead, int* __restrict__ ctr) {
  extern __shared__ float4 tab[];
  __shared__ TaskLds L;
  __shared__ int s_next;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wpb = kConvThreads / 64;
  // The first two tasks of a workgroup are blockIdx.x and blockIdx.x +
  // gridDim.x; later ones come from an atomic counter (task 2 gridDim.x + c),
  // fetched two ahead of the task being weighed, so a workgroup that starts
  // late simply takes fewer tasks.  The counter is zeroed by the launch that
  // consumes the sums (it runs after this one and before the next).
  int task = blockIdx.x;
  int nxt = blockIdx.x + gridDim.x;
  const int dyn0 = 2 * gridDim.x;
  const ConvTask none{0, 0, 0, 0};
  ConvTask tk = task < ntasks ? tasks[task] : none;
  ConvTask nk = nxt < ntasks ? tasks[nxt] : none;
  static_assert(U * K == 16 || U * K == 20, "16 or 20 rows in flight per wave");
  TileR t[K];
  bool has[K];
  float4 h[K][U];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    has[i] = task < ntasks && wave + wpb * i < tk.t1 - tk.t0;
    const Tile* tp = tiles + (has[i] ? tk.t0 + wave + wpb * i : 0);
    tile_address(t[i], tp);
    tile_weights(t[i], tp);
#pragma unroll
    for (int u = 0; u < U; ++u) h[i][u] = make_float4(0.f, 0.f, 0.f, 0.f);
    conv32_load<U, POL>(t[i], has[i], lane, h[i]);
  }
  // the current task's fault words
  int err = 0;
  long long step = 0;
  double4* parts = nullptr;
  if (task < ntasks) {
    const FaultDev& fd = faults[tk.fault];
    err = read_word(fd.err);
    step = read_word(fd.step) + ahead;
    parts = fd.parts;
  }
  // the table is staged while the first records are in flight
  for (int i = threadIdx.x; i < table_len; i += kConvThreads) tab[i] = table[i];
  __syncthreads();
  while (task < ntasks) {
    const bool more = nxt < ntasks;
    int got = 0;
    if (threadIdx.x == 0 && more) got = atomicAdd(ctr, 1);  // used after the tiles are weighed
    const int nt = tk.t1 - tk.t0;
    TileR un[K];
    int nidx[K];
    bool nh[K];
    int nerr;
    long long nstep;
    double4* nparts;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      // weigh tile i, then reuse its registers for the next task's tile i
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      if (has[i] && !err) acc = conv32_weigh(t[i], step, lane, h[i], tab, table_len);
      __builtin_amdgcn_sched_barrier(0);
      if (i == 0) {
        // the addressing fields of the next task's tiles, all requested
        // before the first wait (a wave without a next tile reads tile 0
        // and never uses it); their weighing fields follow after the last
        // tile of this task, when this task's have been used
#pragma unroll
        for (int j = 0; j < K; ++j) {
          nh[j] = more && wave + wpb * j < nk.t1 - nk.t0;
          nidx[j] = nh[j] ? nk.t0 + wave + wpb * j : 0;
          tile_address(un[j], tiles + nidx[j]);
        }
        const FaultDev& nfd = faults[more ? nk.fault : tk.fault];
        nerr = read_word(nfd.err);
        nstep = read_word(nfd.step) + ahead;
        nparts = nfd.parts;
      }
      conv32_load<U, POL>(un[i], nh[i], lane, h[i]);
      if (has[i]) {
        acc = wave_reduce4(acc);
        if (lane == 0) {
          L.part[wave + wpb * i] = make_double4(acc.x, acc.y, acc.z, acc.w);
          L.id[wave + wpb * i] = t[i].part;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      t[i] = un[i];
      tile_weights(t[i], tiles + nidx[i]);
      has[i] = nh[i];
    }
    if (threadIdx.x == 0) s_next = more ? dyn0 + got : ntasks;  // written and read between the two barriers
    __syncthreads();
    const int after_all = __builtin_amdgcn_readfirstlane(s_next);
    const ConvTask nnk = after_all < ntasks ? tasks[after_all] : none;
    finish_task(parts, L, nt);
    __syncthreads();
    task = nxt;
    nxt = after_all;
    tk = nk;
    nk = nnk;
    err = nerr;
    step = nstep;
    parts = nparts;
  }
}

// Packed rows.  Each wave weighs 16 rows of 64 records per task, the rows of
// one mode and then of the next ones, so no row lies past a mode's end.  A
// row's parameters come with it (RowDesc); a wave's 16 descriptors (768 B)
// are held in three registers, three words per lane, and read out with
// lane reads.  They are requested two tasks ahead, before the records of the
// task in between: in-order completion of vector loads then makes every wait
// for them free, and they never drain records in flight.  Tasks are taken in
// grid order (all tasks have 128 rows, so none is longer than another).
//
// The running wave sum of a partial sum (task, mode) is reduced at the last
// row of the partial sum in the wave and at the wave's last row, into the LDS
// slot the host assigned (slots count the task's wave sums in row order);
// after the barrier the first slot of each run adds its run in order, so every
// sum has a fixed order.
struct PackLds {
  double4 part[kTaskRows];
  int2 meta[kTaskRows];   // (partial sum, run length at a run's first slot)
};
static_assert(sizeof(PackLds) + 64 <= kConvStaticLds && sizeof(TaskLds) + 64 <= kConvStaticLds,
              "static LDS of the FP32 conv kernels");

struct RowBlock {
  int a, b, c;            // words 3 lane, 3 lane + 1, 3 lane + 2 of the wave's rows
};
__device__ __forceinline__ RowBlock load_rows(const RowDesc* rows, int task, int ntasks, int wave,
                                              int lane) {
  const int t = task < ntasks ? task : 0;   // past the last task: never used
  const int* w = (const int*)(rows + (size_t)t * kTaskRows + kPackRows * wave) + 3 * lane;
  return RowBlock{w[0], w[1], w[2]};
}
// word F of row U of a block
template <int U, int F>
__device__ __forceinline__ unsigned row_word(const RowBlock& b) {
  static_assert(U < kPackRows && F < 12, "row descriptor word");
  const int v = F % 3 == 0 ? b.a : (F % 3 == 1 ? b.b : b.c);
  return (unsigned)__builtin_amdgcn_readlane(v, 4 * U + F / 3);
}
typedef const __attribute__((address_space(1))) f4v* gf4p;
template <int U>
__device__ __forceinline__ void row_load(const RowBlock& b, bool live, int lane, const float4* dummy,
                                         float4& h) {
  const unsigned long long rec =
      (unsigned long long)row_word<U, 1>(b) << 32 | (unsigned long long)row_word<U, 0>(b);
  const int len = (int)(row_word<U, 2>(b) & 0xFFu);
  const bool use = live && len > 0;
  // lanes past the row's end re-read its last record (same cache line); an
  // empty row reads the first nodes of the table (cached, never weighed)
  const unsigned long long base = use ? rec : (unsigned long long)(uintptr_t)dummy;
  const int idx = use ? min(lane, len - 1) : (lane & 3);
  // the address is formed in vector registers: a memory instruction reading
  // a scalar register that a lane read has just written needs wait states
  unsigned lo = (unsigned)base, hi = (unsigned)(base >> 32);
  asm volatile("" : "+v"(lo), "+v"(hi));
  const unsigned long long a = ((unsigned long long)hi << 32 | lo) + (unsigned long long)idx * 16u;
  const f4v t = __builtin_nontemporal_load((gf4p)(const float4*)(uintptr_t)a);
  h = make_float4(t.x, t.y, t.z, t.w);
}

// The weights of one row's records (lane: record p0 + lane of the mode's
// ring), added to acc; as in conv32_weigh.
// The ring phase depends on the step and R_n alone: it is recomputed only
// when a row's R_n differs from the previous row's (pRn, po carry it).
template <int U>
__device__ __forceinline__ float4 row_weigh(const RowBlock& b, long long step, int lane,
                                            const float4& hv, const float4* tab, int table_len,
                                            float4 acc, int& pRn, int& po) {
  const int len = (int)(row_word<U, 2>(b) & 0xFFu);
  const int p0 = (int)row_word<U, 3>(b);
  const int Rn = (int)row_word<U, 4>(b);
  const int MT = (int)row_word<U, 5>(b);
  const int MN = (int)row_word<U, 6>(b);
  const double th = __builtin_bit_cast(
      double, (unsigned long long)row_word<U, 9>(b) << 32 | (unsigned long long)row_word<U, 8>(b));
  if (Rn != pRn) {
    const unsigned long long M =
        (unsigned long long)row_word<U, 11>(b) << 32 | (unsigned long long)row_word<U, 10>(b);
    po = ring_phase_m(step, Rn, M);
    pRn = Rn;
  }
  const int o = po;
  const int p = p0 + lane;
  int q = p + o;
  q -= (q >= Rn) ? Rn : 0;
  const int j = Rn - q + 1;                         // lag (q = 0: skipped slot)
  const double x = (double)(2 * j + 1) * th;
  // lanes past the row's end (weight 0) may have j <= 0: keep their node in the table
  const int i = min(max((int)x, 0), table_len - 2);
  const float f = (float)(x - (double)i);
  const float4 n0 = tab[i], n1 = tab[i + 1];
  const float f2 = f * f, f3 = f2 * f;
  const float h00 = 2.f * f3 - 3.f * f2 + 1.f;
  const float h10 = f3 - 2.f * f2 + f;
  const float h01 = 3.f * f2 - 2.f * f3;
  const float h11 = f3 - f2;
  float wT = h00 * n0.x + h10 * n0.y + h01 * n1.x + h11 * n1.y;
  float wN = h00 * n0.z + h10 * n0.w + h01 * n1.z + h11 * n1.w;
  const bool use = (q != 0) && (lane < len);
  wT = (use && j < MT) ? wT : 0.f;
  wN = (use && j < MN) ? wN : 0.f;
  acc.x = fmaf(wT, hv.x, acc.x);
  acc.y = fmaf(wT, hv.y, acc.y);
  acc.z = fmaf(wN, hv.z, acc.z);
  acc.w = fmaf(wN, hv.w, acc.w);
  return acc;
}

__device__ __forceinline__ void finish_packed(double4* parts, const PackLds& L, int nsum) {
  const int k = threadIdx.x;
  if (k < nsum) {
    const int2 m = L.meta[k];
    if (m.y > 0) {
      double4 a = L.part[k];
      for (int j = 1; j < m.y; ++j) {
        const double4 b = L.part[k + j];
        a.x += b.x;
        a.y += b.y;
        a.z += b.z;
        a.w += b.w;
      }
      typedef double d4v __attribute__((ext_vector_type(4)));
      typedef __attribute__((address_space(1))) d4v* gd4p;
      const d4v v = {a.x, a.y, a.z, a.w};
      ((gd4p)(d4v*)parts)[m.x] = v;
    }
  }
}

template <int U>
__device__ __forceinline__ void pack_row(const RowBlock& dc, const RowBlock& dn, bool weigh,
                                         bool more, long long step, int lane, float4 (&h)[kPackRows],
                                         const float4* tab, int table_len, const float4* dummy,
                                         float4& acc, int& pRn, int& po, PackLds& L) {
  const unsigned word = row_word<U, 2>(dc);
  if (weigh && (word & 0xFFu) != 0u)
    acc = row_weigh<U>(dc, step, lane, h[U], tab, table_len, acc, pRn, po);
  else
    asm volatile("" ::"v"(h[U].x), "v"(h[U].y), "v"(h[U].z), "v"(h[U].w));
  __builtin_amdgcn_sched_barrier(0);
  row_load<U>(dn, more, lane, dummy, h[U]);
  const int slot = (int)((word >> 8) & 0xFFu) - 1;
  if (slot >= 0) {
    const float4 r = wave_reduce4(acc);
    if (lane == 0) {
      L.part[slot] = make_double4(r.x, r.y, r.z, r.w);
      L.meta[slot] = make_int2((int)row_word<U, 7>(dc), (int)(word >> 16));
    }
    acc = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

template <int... Us>
__device__ __forceinline__ void pack_rows(std::integer_sequence<int, Us...>, const RowBlock& dc,
                                          const RowBlock& dn, bool weigh, bool more, long long step,
                                          int lane, float4 (&h)[kPackRows], const float4* tab,
                                          int table_len, const float4* dummy, float4& acc,
                                          PackLds& L) {
  int pRn = -1, po = 0;
  (pack_row<Us>(dc, dn, weigh, more, step, lane, h, tab, table_len, dummy, acc, pRn, po, L), ...);
}

template <int... Us>
__device__ __forceinline__ void pack_first(std::integer_sequence<int, Us...>, const RowBlock& d,
                                           bool live, int lane, const float4* dummy,
                                           float4 (&h)[kPackRows]) {
  (row_load<Us>(d, live, lane, dummy, h[Us]), ...);
}

__global__ void __launch_bounds__(kConvThreads)
k_conv32p(const FaultDev* __restrict__ faults, const RowDesc* __restrict__ rows,
          const ConvTask* __restrict__ tasks, int ntasks, const float4* __restrict__ table,
          int table_len, int ahead) {
  extern __shared__ float4 tab[];
  __shared__ PackLds L;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int G = gridDim.x;
  const ConvTask none{0, 0, 0, 0};
  int task = blockIdx.x;
  RowBlock dc = load_rows(rows, task, ntasks, wave, lane);
  RowBlock dn = load_rows(rows, task + G, ntasks, wave, lane);
  float4 h[kPackRows];
  pack_first(std::make_integer_sequence<int, kPackRows>{}, dc, task < ntasks, lane, table, h);
  ConvTask tk = task < ntasks ? tasks[task] : none;
  int err = 0;
  long long step = 0;
  double4* parts = nullptr;
  if (task < ntasks) {
    const FaultDev& fd = faults[tk.fault];
    err = read_word(fd.err);
    step = read_word(fd.step) + ahead;
    parts = fd.parts;
  }
  // the table is staged while the first records are in flight
  for (int i = threadIdx.x; i < table_len; i += kConvThreads) tab[i] = table[i];
  __syncthreads();
  while (task < ntasks) {
    const int nxt = task + G;
    const bool more = nxt < ntasks;
    const RowBlock dnn = load_rows(rows, nxt + G, ntasks, wave, lane);
    const ConvTask nk = more ? tasks[nxt] : none;
    const FaultDev& nfd = faults[more ? nk.fault : tk.fault];
    const int nerr = read_word(nfd.err);
    const long long nstep = read_word(nfd.step) + ahead;
    double4* const nparts = nfd.parts;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    pack_rows(std::make_integer_sequence<int, kPackRows>{}, dc, dn, !err, more, step, lane, h,
              tab, table_len, table, acc, L);
    __syncthreads();
    finish_packed(parts, L, tk.nsum);
    __syncthreads();
    task = nxt;
    tk = nk;
    dc = dn;
    dn = dnn;
    err = nerr;
    step = nstep;
    parts = nparts;
  }
}

// ---------------------------------------------------------------------------
// Four-step transforms across workgroups.  N = P Q; element i = b + Q a
// (class b), spectral index n = c + P d (class c).
//
// Forward, X_n = sum_i x_i w_N^{i n} (w_M = exp(-2 pi i / M)):
//   element stage, class b:  Y_b[c] = w_N^{b c} sum_a x_{b+Qa} w_P^{a c}
//                            -> gF[c Q + b]
//   mode stage, class c:     X_{c+Pd} = sum_b Y_b[c] w_Q^{b d}
// Inverse of a Hermitian-packed spectrum Z, computed as conj(FFT(conj Z))/N:
//   mode stage, class c:     W_c[b] = w_N^{c b} sum_d conj(Z_{c+Pd}) w_Q^{d b}
//                            -> gI[b P + c]
//   element stage, class b:  N conj(x_{b+Qa}) = sum_c W_c[b] w_P^{c a}
// The element stage of the inverse leaves element b + Q a where the forward
// element stage wants it, so the friction solve between them needs no
// exchange; a mode workgroup owns the classes {c, P - c}, which hold every
// index n together with its mirror N - n, so packing and unpacking the two
// real signals of a transform stay inside the workgroup.
// ---------------------------------------------------------------------------

// exp(-2 pi i m / N) for m in [0, N) from the global quarter-wave table.
template <typename C, typename R>
__device__ __forceinline__ C twiddle_full(const R* __restrict__ q, int m, int N) {
  const int h = N >> 1;
  C w = twiddle_half<C, R>(q, m & (h - 1), N);
  if (m >= h) {
    w.x = -w.x;
    w.y = -w.y;
  }
  return w;
}

// Vector stride (complex elements) of an M-point vector with one pad per 8.
__host__ __device__ inline int vstride(int M) { return M + (M >> 3); }

// One Stockham pass with radix 2^LR after sub-transforms of length p, over
// nvec vectors of M = 2^lm points: butterfly j takes x[j + r M/RD], applies
// exp(-2 pi i r k / (p RD)) with k = j mod p and writes the RD outputs to
// (j - k) RD + k + s p.  Out of place (src -> dst), then a barrier.
template <typename C, typename R, int LR>
__device__ __forceinline__ void fft_pass_b(const C* __restrict__ src, C* __restrict__ dst, int nvec,
                                           int lm, int p, const R* __restrict__ q) {
  constexpr int RD = 1 << LR;
  const int M = 1 << lm;
  const int nb = M >> LR;
  const int total = nvec << (lm - LR);
  const int vs = vstride(M);
  const int tws = M / (p * RD);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int v = t >> (lm - LR);
    const int j = t & (nb - 1);
    const C* s = src + v * vs;
    C x[RD];
#pragma unroll
    for (int r = 0; r < RD; ++r) x[r] = s[lx(j + r * nb, 3)];
    const int k = j & (p - 1);
    if (p > 1) {
      const C w1 = twiddle_half<C, R>(q, k * tws, M);
      x[1] = cmul(x[1], w1);
      if (RD >= 4) {
        const C w2 = cmul(w1, w1);
        const C w3 = cmul(w2, w1);
        x[2] = cmul(x[2], w2);
        x[3] = cmul(x[3], w3);
        if (RD == 8) {
          const C w4 = cmul(w2, w2);
          x[4] = cmul(x[4], w4);
          x[5] = cmul(x[5], cmul(w4, w1));
          x[6] = cmul(x[6], cmul(w4, w2));
          x[7] = cmul(x[7], cmul(w4, w3));
        }
      }
    }
    if (RD == 8) dft8(x);
    else if (RD == 4) dft4(x[0], x[1], x[2], x[3]);
    else dft2(x);
    C* d = dst + v * vs;
    const int base = (j - k) * RD + k;
#pragma unroll
    for (int r = 0; r < RD; ++r) d[lx(base + r * p, 3)] = x[r];
  }
  __syncthreads();
}

// Forward FFT of nvec vectors of 2^lm points held in a (natural order,
// padded); b is scratch of the same size; q is the LDS table cos(2 pi r / M),
// r = 0..M/4.  The caller has synchronised after filling a and q.  Returns
// the buffer that holds the transforms (natural order).
template <typename C, typename R>
__device__ __forceinline__ C* fft_batch(C* a, C* b, int nvec, int lm, const R* __restrict__ q) {
  int p = 1, rem = lm;
  C* src = a;
  C* dst = b;
  while (rem > 0) {
    if (rem >= 3) {
      fft_pass_b<C, R, 3>(src, dst, nvec, lm, p, q);
      p <<= 3;
      rem -= 3;
    } else if (rem == 2) {
      fft_pass_b<C, R, 2>(src, dst, nvec, lm, p, q);
      p <<= 2;
      rem -= 2;
    } else {
      fft_pass_b<C, R, 1>(src, dst, nvec, lm, p, q);
      p <<= 1;
      rem -= 1;
    }
    C* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Forward FFT of nvec vectors of M = 64 E points (E = 1, 2, 4), one
// wavefront per vector, held in registers.  With n = l + 64 e (lane l) and
// k = k1 + E k2: E-point DFTs over e give k1, twiddles w_M^{l k1}, then
// 64-point DFTs over the lanes by six radix-2 decimation-in-frequency stages
// that exchange values with lane shuffles (no LDS passes, no barriers between
// stages); lane l ends with k2 = bit-reverse(l).  Same layout as fft_batch
// (a: natural order, padded; the result goes to b); ends with a barrier.
template <typename C, typename R, int E>
__device__ __forceinline__ C* fft_wave(const C* a, C* b, int nvec, const R* __restrict__ q) {
  constexpr int M = 64 * E;
  const int vs = vstride(M);
  const int lane = threadIdx.x & 63;
  const int v = threadIdx.x >> 6;
  if (v < nvec) {
    const C* s = a + v * vs;
    C x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = s[lx(lane + 64 * e, 3)];
    if (E == 2) dft2(x);
    if (E == 4) dft4(x[0], x[1], x[2], x[3]);
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) x[k1] = cmul(x[k1], twiddle_full<C, R>(q, lane * k1, M));
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
      const bool upper = (lane & h) != 0;
      const C w = twiddle_half<C, R>(q, (lane & (h - 1)) * (M / (2 * h)), M);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        C p;
        p.x = __shfl_xor(x[e].x, h);
        p.y = __shfl_xor(x[e].y, h);
        x[e] = upper ? cmul(csub(p, x[e]), w) : cadd(x[e], p);
      }
    }
    const int k2 = (int)(__brev((unsigned)lane) >> 26);
    C* d = b + v * vs;
#pragma unroll
    for (int e = 0; e < E; ++e) d[lx(e + E * k2, 3)] = x[e];
  }
  __syncthreads();
  return b;
}

// The transform of nvec vectors of 2^lm points: register wave FFTs where one
// wavefront per vector fits the workgroup and 64 <= M <= 256, else the LDS
// Stockham passes.
template <typename C, typename R>
__device__ __forceinline__ C* fft_vectors(C* a, C* b, int nvec, int lm, const R* __restrict__ q) {
  if (nvec * 64 <= (int)blockDim.x) {
    if (lm == 6) return fft_wave<C, R, 1>(a, b, nvec, q);
    if (lm == 7) return fft_wave<C, R, 2>(a, b, nvec, q);
    if (lm == 8) return fft_wave<C, R, 4>(a, b, nvec, q);
  }
  return fft_batch<C, R>(a, b, nvec, lm, q);
}

// LDS table cos(2 pi r / M), r = 0..M/4, from the fault's N-point table.
template <typename R>
__device__ __forceinline__ void load_sub_table(R* q, const FaultDev& fd, int lm) {
  const R* __restrict__ g = (const R*)fd.twiddle;
  const int M4 = (1 << lm) >> 2;
  const int stride = fd.N >> lm;
  for (int r = threadIdx.x; r <= M4; r += blockDim.x) q[r] = g[r * stride];
}

// Traction spectra of mode n (section 3.1; current interval rates vc, gvc):
//   tau_hat = mk (B_T + aT vc),  sigma_hat = -i ms (B_N + aN gvc)
__device__ __forceinline__ void traction_mode(const ModeCoef& c, double2 BT, double2 BN, double2 vc,
                                              double2 gvc, double2* tau, double2* sig) {
  const double ATx = BT.x + c.aT * vc.x, ATy = BT.y + c.aT * vc.y;
  const double ANx = BN.x + c.aN * gvc.x, ANy = BN.y + c.aN * gvc.y;
  *tau = d2(c.mk * ATx, c.mk * ATy);
  *sig = d2(c.ms * ANy, -c.ms * ANx);  // -i ms AN
}

// History sum S of a mode: its first conv partial plus any further pieces.
__device__ __forceinline__ double4 history_sum(const FaultDev& fd, const ModeCoef& c, int pm) {
  double4 h = make_double4(0.0, 0.0, 0.0, 0.0);
  if (c.nparts > 0) h = fd.parts[pm];
  for (int j = 1; j < c.nparts; ++j) {
    const double4 b = fd.parts[c.part0 + j - 1];
    h.x += b.x;
    h.y += b.y;
    h.z += b.z;
    h.w += b.w;
  }
  return h;
}

constexpr int kNoExp = -2000;  // "no maximum yet" in the balance cells

__device__ __forceinline__ int ilogb_or_min(double x) {
  return (x > 0.0 && x <= 1.0e300) ? ilogb(x) : kNoExp;
}

// log2 of the balance factor c in Z = tau_hat + i c sigma_hat from the two
// maxima (0 when either is missing).
__device__ __forceinline__ int balance_exp(int te, int se) {
  if (te <= kNoExp || se <= kNoExp) return 0;
  return min(max(te - se, -256), 256);
}

// Workgroup maximum of ilogb(mt), ilogb(ms) folded into two global cells
// (LDS cells red[0..1] were set to kNoExp before the workgroup's first
// barrier; ends with a barrier).
__device__ __forceinline__ void fold_maxima(double mt, double ms, int* red, int* cell) {
  int et = ilogb_or_min(mt), es = ilogb_or_min(ms);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    et = max(et, __shfl_xor(et, off));
    es = max(es, __shfl_xor(es, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&red[0], et);
    atomicMax(&red[1], es);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (red[0] > kNoExp) atomicMax(&cell[0], red[0]);
    if (red[1] > kNoExp) atomicMax(&cell[1], red[1]);
  }
}

// Mode workgroup (fault, group g) of a launch: map, or group = block index.
__device__ __forceinline__ int2 work_item(const int2* __restrict__ map) {
  return map ? map[blockIdx.x] : make_int2(0, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Mode stage.  KIND 0: pass-1 assembly from the stored state (prologue and
// stress path); KIND 1: forward-transform finish of the pass-1 rates, pass-2
// assembly; KIND 2: forward-transform finish of the pass-2 rates, commit
// (ring push of (V_0 + V_1)/2, spectral slip, h_prev, V_0 <- V_2) and the
// pass-1 assembly of the next step; KIND 3: forward-transform finish only,
// spectra to (outA, outB).  Kinds 0-2 end with the first half of the
// inverse transform into gI.
// LDS: buffers A and B (two Q-point vectors each), then the Q-point table.
// Every global load a thread needs for its first slot is issued at the top,
// so the launch waits for memory once.
// ---------------------------------------------------------------------------
struct ModeIn {
  ModeCoef cf;
  double2 v0, gv0, v1, gv1, u, gg, hv, hg, BT, BN;
  double4 S0;  // first conv partial plus the learned-closure tail (if any)
};

// Per-mode arrays of a fault (read from the descriptor once per launch).
struct ModePtrs {
  const ModeCoef* coef;
  double4* parts;
  const double4* tails;
  double2 *u, *g, *v0, *gv0, *v1, *gv1, *hv, *hg, *BT, *BN;
};

__device__ __forceinline__ ModePtrs mode_ptrs(const FaultDev& fd) {
  ModePtrs m;
  m.coef = fd.coef;
  m.parts = fd.parts;
  m.tails = fd.tails;
  m.u = fd.u_hat;
  m.g = fd.g_hat;
  m.v0 = fd.v_hat0;
  m.gv0 = fd.gv_hat0;
  m.v1 = fd.v_hat1;
  m.gv1 = fd.gv_hat1;
  m.hv = fd.hprev_v;
  m.hg = fd.hprev_g;
  m.BT = fd.B_T;
  m.BN = fd.B_N;
  return m;
}

template <int KIND>
__device__ __forceinline__ void load_mode_in(const ModePtrs& f, int pm, ModeIn& m) {
  m.cf = f.coef[pm];
  m.v0 = f.v0[pm];
  m.gv0 = f.gv0[pm];
  if (KIND == 0 || KIND == 2) {
    m.u = f.u[pm];
    m.gg = f.g[pm];
    m.S0 = f.parts[pm];
    if (f.tails) {
      const double4 t = f.tails[pm];
      m.S0.x += t.x;
      m.S0.y += t.y;
      m.S0.z += t.z;
      m.S0.w += t.w;
    }
  }
  if (KIND == 0) {
    m.hv = f.hv[pm];
    m.hg = f.hg[pm];
  }
  if (KIND == 1) {
    m.BT = f.BT[pm];
    m.BN = f.BN[pm];
  }
  if (KIND == 2) {
    m.v1 = f.v1[pm];
    m.gv1 = f.gv1[pm];
  }
}

// Slot t of a mode workgroup: vector v (class cls), entry d, index n.
struct ModeSlot {
  int v, d, cls, n, sn, sm, pm;
  bool mode;  // n <= N/2: the slot's thread handles mode n and its mirror
};

__device__ __forceinline__ ModeSlot mode_slot(int t, int N, int lP, int lQ, int cls0, int cls1, int vs) {
  ModeSlot s;
  const int P = 1 << lP, Q = 1 << lQ;
  s.v = t >> lQ;
  s.d = t & (Q - 1);
  s.cls = s.v ? cls1 : cls0;
  s.n = s.cls + (s.d << lP);
  s.mode = s.n <= (N >> 1);
  const int cm = (P - s.cls) & (P - 1);
  const int dm = ((N - s.n) >> lP) & (Q - 1);
  const int vm = (cm == cls0) ? 0 : 1;
  s.sn = s.v * vs + lx(s.d, 3);
  s.sm = vm * vs + lx(dm, 3);
  s.pm = mode_pos(s.mode ? s.n : 0, lP, lQ);
  return s;
}

// Weight of the current interval (lag span [0, dt]) of mode n in a variable
// step: P^X(c_s |k_n| min(dt, T_w^X)) / (c_s |k_n|), added to (1 - r) dt.
__device__ __forceinline__ void var_lag0(const FaultDev& fd, int n, double dt, double c1,
                                         double* aT, double* aN) {
  *aT = c1 * dt;
  *aN = c1 * dt;
  if (n == 0) return;
  const double kL = 2.0 * M_PI * (double)n;
  const double csk = fd.cs * kL / fd.L;
  const double T = csk * dt;
  const double cutT = fmin(kL, fd.kcT), cutN = fmin(kL, fd.kcN);
  double pt, pn;
  ptab_eval(fd.ptab, fd.ptab_len, fd.ptab_h, fmin(T, cutT), &pt, &pn);
  if (cutN != cutT) {
    double x;
    ptab_eval(fd.ptab, fd.ptab_len, fd.ptab_h, fmin(T, cutN), &x, &pn);
  }
  *aT += pt / csk;
  *aN += pn / csk;
}

template <typename R, int KIND>
__global__ void __launch_bounds__(kModeThreads)
k_modes(const FaultDev* __restrict__ faults, const int2* __restrict__ map, int measure,
        const void* __restrict__ gF_in, double2* __restrict__ outA, double2* __restrict__ outB,
        long long stride_out, int* __restrict__ conv_ctr, VarArgs va) {
  using C = typename Prec<R>::C;
  using Rec = typename Prec<R>::Rec;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int red[2];
  const int2 w = work_item(map);
  const FaultDev& fd = faults[w.x];
  const int g = w.y;
  // ---- every descriptor field the launch uses, read once up front
  const int N = fd.N, P = fd.P, Q = fd.Q, lP = fd.log2P, lQ = fd.log2Q;
  const R* __restrict__ tq = (const R*)fd.twiddle;
  const ModePtrs mp = mode_ptrs(fd);
  const C* __restrict__ src = (const C*)(KIND == 3 ? gF_in : fd.gF);
  C* __restrict__ gI = (C*)fd.gI;
  Rec* __restrict__ ring = (Rec*)fd.ring;
  int* cells = fd.cells;
  int* done = fd.done;
  long long* stepp = fd.step;
  const int ngroups = fd.ngroups;
  const double inv_s = 1.0 / fd.fwd_scale;
  const double dt = va.on ? va.dt : fd.dt, c1 = 1.0 - fd.r;
  int err = 0;
  long long l = 0;
  int e_in = 0;
  if (KIND != 3) {
    err = *fd.err;
    if (KIND == 2) l = *stepp;
    e_in = (KIND == 1) ? balance_exp(cells[0], cells[1]) : balance_exp(cells[2], cells[3]);
  }

  const int vs = vstride(Q);
  const int nslot = 2 * Q;
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + 2 * vs;
  R* q = reinterpret_cast<R*>(bufB + 2 * vs);
  const int cls0 = g == 0 ? 0 : g;
  const int cls1 = g == 0 ? (P >> 1) : P - g;

  // ---- loads of the first slot, the transform input and the tables
  const int t0 = threadIdx.x;
  const ModeSlot s0 = mode_slot(t0 < nslot ? t0 : 0, N, lP, lQ, cls0, cls1, vs);
  ModeIn in0;
  if (KIND != 3 && t0 < nslot && s0.mode) load_mode_in<KIND>(mp, s0.pm, in0);
  C tw0 = cmk<C>(1.0, 0.0);
  if (KIND != 3 && t0 < nslot) tw0 = twiddle_full<C, R>(tq, s0.cls * s0.d, N);
  if (KIND != 0) {
    const C* __restrict__ sp = src + (KIND == 3 ? (size_t)blockIdx.y * N : 0);
    for (int t = threadIdx.x; t < nslot; t += blockDim.x) {
      const int v = t >> lQ, b = t & (Q - 1);
      bufA[v * vs + lx(b, 3)] = sp[(size_t)(v ? cls1 : cls0) * Q + b];
    }
  }
  load_sub_table<R>(q, fd, lQ);
  if (threadIdx.x == 0) {
    red[0] = kNoExp;
    red[1] = kNoExp;
  }
  // the conv launch whose sums this launch consumes has finished: zero its
  // task counter for the next one
  if ((KIND == 0 || KIND == 2) && conv_ctr && blockIdx.x == 0 && threadIdx.x == 0) *conv_ctr = 0;
  if (err) return;
  __syncthreads();
  C* X = bufA;
  if (KIND != 0) X = fft_vectors<C, R>(bufA, bufB, 2, lQ, q);

  const double c = ldexp(1.0, e_in);
  double mt = 0.0, ms = 0.0;
  auto slot_work = [&](const ModeSlot& sl, const ModeIn& in) {
    const int pm = sl.pm;
    double2 A = d2(0, 0), Bv = d2(0, 0);
    if (KIND != 0) {
      const C zn = X[sl.sn], zm = X[sl.sm];
      // A = (Z_n + conj Z_m)/2, B = (Z_n - conj Z_m)/(2i), B rescaled
      A = d2(0.5 * ((double)zn.x + (double)zm.x), 0.5 * ((double)zn.y - (double)zm.y));
      Bv = d2(0.5 * ((double)zn.y + (double)zm.y) * inv_s,
              -0.5 * ((double)zn.x - (double)zm.x) * inv_s);
    }
    if (KIND == 3) {
      outA[(size_t)blockIdx.y * stride_out + pm] = A;
      outB[(size_t)blockIdx.y * stride_out + pm] = Bv;
      return;
    }
    ModeCoef cf = in.cf;
    if (va.on) var_lag0(fd, sl.n, dt, c1, &cf.aT, &cf.aN);
    double4 S = in.S0;
    if (KIND != 1) {
      // no ring records (only a closure tail, none for such modes), or no
      // stored interval inside any window (the conv launch was skipped)
      if (cf.nparts == 0 || va.nohist) S = make_double4(0.0, 0.0, 0.0, 0.0);
      for (int j = 1; j < cf.nparts && !va.nohist; ++j) {  // further pieces of a long window
        const double4 b = mp.parts[cf.part0 + j - 1];
        S.x += b.x;
        S.y += b.y;
        S.z += b.z;
        S.w += b.w;
      }
    }
    double2 tau, sig, BT, BN;
    if (KIND == 0) {
      BT = d2(c1 * in.u.x + cf.w1T * in.hv.x + S.x, c1 * in.u.y + cf.w1T * in.hv.y + S.y);
      BN = d2(c1 * in.gg.x + cf.w1N * in.hg.x + S.z, c1 * in.gg.y + cf.w1N * in.hg.y + S.w);
      traction_mode(cf, BT, BN, in.v0, in.gv0, &tau, &sig);
    } else if (KIND == 1) {
      BT = in.BT;
      BN = in.BN;
      mp.v1[pm] = A;
      mp.gv1[pm] = Bv;
      const double2 vc = d2(0.5 * (in.v0.x + A.x), 0.5 * (in.v0.y + A.y));
      const double2 gvc = d2(0.5 * (in.gv0.x + Bv.x), 0.5 * (in.gv0.y + Bv.y));
      traction_mode(cf, BT, BN, vc, gvc, &tau, &sig);
    } else {  // KIND 2
      // rate of the committed interval: (V_0 + V_1)/2
      const double2 hv = d2(0.5 * (in.v0.x + in.v1.x), 0.5 * (in.v0.y + in.v1.y));
      const double2 hg = d2(0.5 * (in.gv0.x + in.gv1.x), 0.5 * (in.gv0.y + in.gv1.y));
      if (sl.n > 0 && cf.Rn > 0) {
        Rec rec;
        if constexpr (sizeof(R) == 4) {
          rec = make_float4((float)hv.x, (float)hv.y, (float)hg.x, (float)hg.y);
        } else {
          rec.v = hv;
          rec.g = hg;
        }
        ring[cf.ring_off + mod_pos(l, cf.Rn)] = rec;
      }
      const double2 un = d2(in.u.x + dt * hv.x, in.u.y + dt * hv.y);
      const double2 gn = d2(in.gg.x + dt * hg.x, in.gg.y + dt * hg.y);
      mp.u[pm] = un;
      mp.g[pm] = gn;
      mp.hv[pm] = hv;
      mp.hg[pm] = hg;
      mp.v0[pm] = A;
      mp.gv0[pm] = Bv;
      BT = d2(c1 * un.x + cf.w1T * hv.x + S.x, c1 * un.y + cf.w1T * hv.y + S.y);
      BN = d2(c1 * gn.x + cf.w1N * hg.x + S.z, c1 * gn.y + cf.w1N * hg.y + S.w);
      traction_mode(cf, BT, BN, A, Bv, &tau, &sig);
    }
    mt = fmax(mt, fmax(fabs(tau.x), fabs(tau.y)));
    ms = fmax(ms, fmax(fabs(sig.x), fabs(sig.y)));
    if (KIND == 0 && measure) return;
    if (KIND != 1) {
      mp.BT[pm] = BT;
      mp.BN[pm] = BN;
    }
    // conj(Z) at n and at N - n with Z = tau_hat + i c sigma_hat (the two
    // spectra are Hermitian, so Z_{N-n} = conj(tau_hat) + i c conj(sigma_hat))
    const double gx = c * sig.x, gy = c * sig.y;
    X[sl.sn] = cmk<C>(tau.x - gy, -(tau.y + gx));
    if (sl.sm != sl.sn) X[sl.sm] = cmk<C>(tau.x + gy, -(-tau.y + gx));
  };
  // one mode per slot (v, d) with n = cls_v + P d <= N/2; the slot of its
  // mirror N - n is handled by the same thread
  if (t0 < nslot && s0.mode) slot_work(s0, in0);
  for (int t = t0 + blockDim.x; t < nslot; t += blockDim.x) {
    const ModeSlot sl = mode_slot(t, N, lP, lQ, cls0, cls1, vs);
    if (!sl.mode) continue;
    ModeIn in;
    if (KIND != 3) load_mode_in<KIND>(mp, sl.pm, in);
    slot_work(sl, in);
  }
  if (KIND == 3) return;
  __syncthreads();  // X complete; the LDS maxima cells were set before the first barrier
  fold_maxima(mt, ms, red, (KIND == 1 || (KIND == 0 && measure)) ? cells + 2 : cells);
  if (KIND == 0 && measure) return;
  if (g == 0 && threadIdx.x == 0) cells[4] = e_in;
  C* Xo = (X == bufA) ? bufB : bufA;
  C* W = fft_vectors<C, R>(X, Xo, 2, lQ, q);
  for (int t = threadIdx.x; t < nslot; t += blockDim.x) {
    const int v = t >> lQ, b = t & (Q - 1);
    const int cls = v ? cls1 : cls0;
    const C tw = (t == t0) ? tw0 : twiddle_full<C, R>(tq, cls * b, N);
    gI[(size_t)b * P + cls] = cmul(W[v * vs + lx(b, 3)], tw);
  }
  if (KIND == 2) {
    // the last workgroup of the fault to finish advances the step counter
    // (every workgroup has read it above, before its own increment)
    __syncthreads();
    if (threadIdx.x == 0) {
      const int prev = atomicAdd(done, 1);
      if (prev == ngroups - 1) {
        atomicExch(done, 0);
        if (va.on) fd.tlog[l % fd.tlog_cap] = make_double2(va.t_old, va.t_new);
        *stepp = l + 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Momentum balance per element (section 3.3, with radiation damping):
//   tau - eta V = sigma (f0 + a ln(V/V_ref) + b ln(theta V_ref/Dc)),
// eta = mu/(2 c_s), solved for x = ln V.  With K = tau - sigma (psi - a ln V_ref)
// the residual g(x) = K - eta e^x - sigma a x is strictly decreasing, so the
// root is unique; [lo, hi] brackets it:
//   hi = x_rs (where the friction term alone balances tau), lowered to
//        max(ln(tau/eta), x_0) when tau > 0 (x_0: zero friction coefficient),
//   lo = x_rs - eta e^hi / (sigma a).
// A single-precision Newton phase (hardware exp/log, bisection whenever a
// step leaves the bracket) brings x near the root; FP64 Newton steps then
// finish: a Newton step shorter than 1e-9 (|x| >= 1) ends the iteration,
// since the error left after it is below the FP64 resolution of x
// (quadratic convergence, curvature factor <= 1/2).  The single-precision
// bounds carry margins that keep the bracket valid.
// ---------------------------------------------------------------------------
// Constants of the friction update of one fault, read once per launch.
struct FrictionConst {
  double lnVref, eta, f0, Vref_Dc, Dc, dt, t_new_load, V_pl, s;
  int theta_mode, newton_max;
};

__device__ __forceinline__ int solve_rate(double tau, double sig, double theta, double a, double b,
                                          const FrictionConst& k, double Vguess, double* Vout) {
  const double lnVref = k.lnVref, eta = k.eta;
  const double psi = k.f0 + b * log(theta * k.Vref_Dc);
  const double sa = sig * a;
  const double x_rs = lnVref + (tau / sig - psi) / a;
  const double x_0 = lnVref - psi / a;
  double hi = x_rs;
  if (tau > 0.0) {
    const float lt = __logf((float)(tau / eta));
    const double ub = (double)lt + 1e-5 * fmax(1.0, fabs((double)lt));
    hi = fmin(hi, fmax(ub, x_0));
  }
  hi = fmin(hi, 700.0);
  const double ehi = hi < 80.0 ? (double)__expf((float)hi) * (1.0 + 1e-5) : exp(hi);
  double lo = x_rs - eta * ehi / sa;
  if (!(lo <= hi)) return -1;
  const double K = tau - sig * (psi - a * lnVref);  // g(x) = K - eta e^x - sa x

  // single-precision phase
  double x;
  {
    const float Kf = (float)K, ef = (float)eta, saf = (float)sa;
    float flo = (float)lo, fhi = (float)hi;
    float xf = fminf(fmaxf(__logf((float)Vguess), flo), fhi);
    if (!(xf == xf)) xf = 0.5f * (flo + fhi);
    for (int it = 0; it < 40 && xf < 80.f; ++it) {
      const float ex = __expf(xf);
      const float g = Kf - ef * ex - saf * xf;
      const float gp = -ef * ex - saf;
      if (g > 0.f) flo = xf;
      else fhi = xf;
      float xn = xf - __fdividef(g, gp);
      if (!(xn > flo && xn < fhi)) xn = 0.5f * (flo + fhi);
      const float st = fabsf(xn - xf);
      xf = xn;
      if (st <= 1e-6f * fmaxf(1.f, fabsf(xf))) break;
    }
    x = fmin(fmax((double)xf, lo), hi);
  }

  // double-precision phase
  for (int it = 0; it < k.newton_max; ++it) {
    const double ex = exp(x);
    const double g = K - eta * ex - sa * x;
    if (g == 0.0) {
      *Vout = ex;
      return 0;
    }
    const double gp = -eta * ex - sa;
    if (g > 0.0) lo = x;
    else hi = x;
    const double d = g / gp;
    const double scale = fmax(1.0, fabs(x));
    double xn = x - d;
    // a short Newton step is accepted even where it touches the bracket: the
    // root is then within |d| (times a factor near 1) of x
    if (fabs(d) <= 1e-9 * scale) {
      *Vout = exp(xn);
      return 0;
    }
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 4e-16 * scale) {
      *Vout = exp(xn);
      return 0;
    }
    x = xn;
  }
  return -1;
}

__device__ __forceinline__ void report(const FaultDev& fd, int code, int i) {
  atomicCAS(fd.err, 0, code);
  atomicAdd(fd.err_count, 1);
  atomicMin(fd.err_index, i);
}

// Per-element inputs of a pass (loaded at the top of the element stage).
// The committed state is double-buffered by step parity; both buffers are
// loaded so that no address waits for the step counter.
struct ElemIn {
  double V[2], thd[2], th[2], slip[2];
  double V1, thd1;  // pass-1 solution (pass 2 only)
  double tl, sl, a, b, kap;
};

template <int PASS>
__device__ __forceinline__ void load_elem_in(const FaultDev& fd, int pe, ElemIn& e) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    e.V[k] = fd.V[k][pe];
    e.thd[k] = fd.thd[k][pe];
    e.th[k] = fd.theta[k][pe];
    e.slip[k] = PASS == 2 ? fd.slip[k][pe] : 0.0;
  }
  e.V1 = PASS == 2 ? fd.V1[pe] : 0.0;
  e.thd1 = PASS == 2 ? fd.thd1[pe] : 0.0;
  e.tl = fd.tau_load[pe];
  e.sl = fd.sigma_load[pe];
  e.a = fd.a[pe];
  e.b = fd.b[pe];
  e.kap = fd.kappa[pe];
}

// Output pointers of a pass (read once per launch).
struct ElemOut {
  double *V1, *thd1;                     // pass 1
  double *slip, *V, *theta, *thd;        // pass 2: buffer of the next state
  double *tau_el, *sigma_el;
};

// Predictor, momentum balance and aging law of one element (position pe,
// natural index i) in pass PASS; returns V_p - V_pl (0 on failure).
template <int PASS>
__device__ __forceinline__ double friction_element(const FaultDev& fd, const FrictionConst& k,
                                                   const ElemOut& o, int cur, int pe, int i,
                                                   const ElemIn& in, double te, double se) {
  // committed state of this step; the other buffer holds the step before
  // (selects, not indexing: a run-time index would put the arrays in scratch)
  const double V0 = cur ? in.V[1] : in.V[0], Vb = cur ? in.V[0] : in.V[1];
  const double thd0 = cur ? in.thd[1] : in.thd[0], th0 = cur ? in.th[1] : in.th[0];
  const double dt = k.dt;
  if (in.a < 0.0) {
    // constrained element (stored with a negated): slides at exactly V_pl,
    // state frozen, no friction solve and no failure
    if (PASS == 1) {
      o.V1[pe] = k.V_pl;
      o.thd1[pe] = 0.0;
    } else {
      o.slip[pe] = (cur ? in.slip[1] : in.slip[0]) + dt * k.V_pl;
      o.V[pe] = k.V_pl;
      o.theta[pe] = th0;
      o.thd[pe] = 0.0;
    }
    return 0.0;
  }
  double Vc, thdc, guess;
  if (PASS == 1) {
    Vc = V0;
    thdc = thd0;
    // guess: geometric extrapolation from the last two committed rates
    const double r = V0 / Vb;
    guess = (r > 1e-3 && r < 1e3) ? V0 * r : V0;
  } else {
    Vc = 0.5 * (V0 + in.V1);
    thdc = 0.5 * (thd0 + in.thd1);
    guess = in.V1;
  }
  double theta_p;
  if (k.theta_mode == SBIEM_THETA_EXP) {
    const double ss = k.Dc / Vc;
    theta_p = ss + (th0 - ss) * exp(-Vc * dt / k.Dc);
  } else {
    theta_p = th0 + dt * thdc;
  }
  const double tau = in.tl + k.t_new_load + te;
  const double sig = in.sl + se;
  double Vp = Vc;
  if (!(sig > 0.0)) {
    report(fd, SBIEM_EOPEN, i);
    return 0.0;
  }
  if (!(theta_p > 0.0) || !isfinite(theta_p)) {
    report(fd, SBIEM_ESTATE, i);
    return 0.0;
  }
  if (solve_rate(tau, sig, theta_p, in.a, in.b, k, guess, &Vp) != 0 || !isfinite(Vp)) {
    report(fd, SBIEM_ENEWTON, i);
    return 0.0;
  }
  const double thdp = 1.0 - theta_p * Vp / k.Dc;
  if (PASS == 1) {
    o.V1[pe] = Vp;
    o.thd1[pe] = thdp;
  } else {
    o.slip[pe] = (cur ? in.slip[1] : in.slip[0]) + dt * Vc;
    o.V[pe] = Vp;
    o.theta[pe] = theta_p;
    o.thd[pe] = thdp;
  }
  return Vp - k.V_pl;
}

// ---------------------------------------------------------------------------
// Element stage.  A workgroup owns classes b0 .. b0 + ncls - 1 (ncls P
// elements, contiguous at positions b P + a).  KIND 0: second half of the
// inverse transform -> tau^el, sigma^el; KIND 1/2: the same, then the pass's
// momentum balance per element and the first half of the forward transform
// of (V_p - V_pl, s kappa (V_p - V_pl)) into gF; KIND 3: the first half of
// the forward transform of (a, s kappa a) for a real signal a in natural
// order (blockIdx.y selects the signal) into gF_out.
// LDS: buffers A and B (ncls P-point vectors each), then the P-point table.
// ---------------------------------------------------------------------------
template <typename R, int KIND>
__global__ void __launch_bounds__(kElemThreads)
k_elems(const FaultDev* __restrict__ faults, const int2* __restrict__ map,
        const double* __restrict__ in, void* __restrict__ gF_out, VarArgs va) {
  using C = typename Prec<R>::C;
  extern __shared__ unsigned char smem_raw[];
  const int2 w = map ? map[blockIdx.x] : make_int2(0, (int)blockIdx.x * faults[0].ncls);
  const FaultDev& fd = faults[w.x];
  const int b0 = w.y;
  // ---- every descriptor field the launch uses, read once up front
  const int N = fd.N, P = fd.P, Q = fd.Q, lP = fd.log2P, lQ = fd.log2Q;
  const int nv = fd.ncls;
  const R* __restrict__ tq = (const R*)fd.twiddle;
  const double s = fd.fwd_scale;
  const double* __restrict__ kap = fd.kappa;
  C* __restrict__ gF = (C*)(KIND == 3 ? gF_out : fd.gF);
  const C* __restrict__ gIrow = (const C*)fd.gI + (size_t)b0 * P;
  int err = 0, e_used = 0;
  long long l = 0;
  if (KIND != 3) {
    err = *fd.err;
    l = *fd.step;
    e_used = fd.cells[4];
  }
  FrictionConst k;
  ElemOut o;
  const int cur = (int)(l & 1);
  if (KIND == 1 || KIND == 2) {
    k.lnVref = fd.ln_V_ref;
    k.eta = fd.eta_rad;
    k.f0 = fd.f0;
    k.Vref_Dc = fd.V_ref / fd.Dc;
    k.Dc = fd.Dc;
    k.dt = va.on ? va.dt : fd.dt;
    k.t_new_load = fd.tau_rate * (va.on ? va.t_new : fd.t0 + (double)(l + 1) * fd.dt);
    k.V_pl = fd.V_pl;
    k.s = s;
    k.theta_mode = fd.theta_mode;
    k.newton_max = fd.newton_max;
    o.V1 = fd.V1;
    o.thd1 = fd.thd1;
    o.slip = cur ? fd.slip[0] : fd.slip[1];
    o.V = cur ? fd.V[0] : fd.V[1];
    o.theta = cur ? fd.theta[0] : fd.theta[1];
    o.thd = cur ? fd.thd[0] : fd.thd[1];
  }
  const int oslot = (int)((l + 1) & 1);
  o.tau_el = oslot ? fd.tau_el[1] : fd.tau_el[0];
  o.sigma_el = oslot ? fd.sigma_el[1] : fd.sigma_el[0];

  const int E = nv << lP;
  const int vs = vstride(P);
  C* bufA = reinterpret_cast<C*>(smem_raw);
  C* bufB = bufA + nv * vs;
  R* q = reinterpret_cast<R*>(bufB + nv * vs);

  // ---- loads of the first element, the transform input and the tables
  const int t0 = threadIdx.x;
  const int pe0 = b0 * P + (t0 < E ? t0 : 0);
  ElemIn in0;
  if ((KIND == 1 || KIND == 2) && t0 < E) load_elem_in<KIND>(fd, pe0, in0);
  C tw0 = cmk<C>(1.0, 0.0);
  if (KIND != 0 && t0 < E) tw0 = twiddle_full<C, R>(tq, (b0 + (t0 >> lP)) * (t0 & (P - 1)), N);
  if (KIND != 3) {
    for (int t = threadIdx.x; t < E; t += blockDim.x) {
      const int v = t >> lP, cc = t & (P - 1);
      bufA[v * vs + lx(cc, 3)] = gIrow[t];
    }
  } else {
    const double* __restrict__ sig = in + (size_t)blockIdx.y * N;
    for (int t = threadIdx.x; t < E; t += blockDim.x) {
      const int v = t >> lP, a = t & (P - 1);
      const int pe = b0 * P + t;
      const int i = (b0 + v) + (a << lQ);
      const double x = sig[i];
      bufA[v * vs + lx(a, 3)] = cmk<C>(x, s * kap[pe] * x);
    }
  }
  load_sub_table<R>(q, fd, lP);
  if (err) return;
  // the balance cells of the pass just read are no longer needed
  if (b0 == 0 && threadIdx.x == 0) {
    if (KIND == 1) {
      fd.cells[2] = kNoExp;
      fd.cells[3] = kNoExp;
    } else if (KIND == 2) {
      fd.cells[0] = kNoExp;
      fd.cells[1] = kNoExp;
    }
  }
  __syncthreads();
  C* X = bufA;
  if (KIND != 3) {
    X = fft_vectors<C, R>(bufA, bufB, nv, lP, q);
    const double inv = 1.0 / N, invc = inv * ldexp(1.0, -e_used);
    auto element = [&](int t, const ElemIn& e) {
      const int v = t >> lP, a = t & (P - 1);
      const int pe = b0 * P + t;
      const int i = (b0 + v) + (a << lQ);
      const int sx = v * vs + lx(a, 3);
      const C z = X[sx];
      const double te = (double)z.x * inv, se = -(double)z.y * invc;
      o.tau_el[pe] = te;
      o.sigma_el[pe] = se;
      if (KIND == 1 || KIND == 2) {
        const double dv = friction_element<KIND>(fd, k, o, cur, pe, i, e, te, se);
        X[sx] = cmk<C>(dv, s * e.kap * dv);
      }
    };
    if (t0 < E) element(t0, in0);
    for (int t = t0 + blockDim.x; t < E; t += blockDim.x) {
      ElemIn e;
      if (KIND == 1 || KIND == 2) load_elem_in<KIND>(fd, b0 * P + t, e);
      element(t, e);
    }
    if (KIND == 0) return;
    __syncthreads();
  }
  C* Xo = (X == bufA) ? bufB : bufA;
  C* Y = fft_vectors<C, R>(X, Xo, nv, lP, q);
  if (KIND == 3) gF += (size_t)blockIdx.y * N;
  for (int t = threadIdx.x; t < E; t += blockDim.x) {
    const int v = t >> lP, cc = t & (P - 1);
    const int b = b0 + v;
    const C tw = (t == t0) ? tw0 : twiddle_full<C, R>(tq, b * cc, N);
    gF[(size_t)cc * Q + b] = cmul(Y[v * vs + lx(cc, 3)], tw);
  }
}

// ---------------------------------------------------------------------------
// Variable steps (section 3.2).  Slot p of mode n's ring (capacity R_n)
// holds interval I(p) = b - ((b - p) mod R_n), b = step - 1 the last
// committed interval (none while I < 0), whose start and end times are in
// the fault's interval log.  At the step's end time t_new its lag span is
// [tau_a, tau_b] = [t_new - end, t_new - start], and its weight for kind X
//   w^X = [P^X(min(c_s|k_n| tau_b, T^X)) - P^X(min(c_s|k_n| tau_a, T^X))] / (c_s|k_n|)
// with T^X = min(|k_n| L, k_c^X L) the window end in units of c_s|k|t: the
// exact integral of the kernel over the part of the interval inside the
// window.  Every stored interval is summed (lag 1 included: the mode stage
// adds no separate lag-1 term on this engine).  One workgroup per task,
// FP64 accumulation, the same (task, mode) partials as the fixed-step conv.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kConvThreads)
k_conv_var(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles,
           const ConvTask* __restrict__ tasks, int ntasks, VarArgs va) {
  using Rec = typename Prec<R>::Rec;
  constexpr int U = kTileSlots64 / 64;
  __shared__ TaskLds L;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wpb = kConvThreads / 64;
  for (int task = blockIdx.x; task < ntasks; task += gridDim.x) {
    const ConvTask tk = tasks[task];
    const int nt = tk.t1 - tk.t0;
    const FaultDev& fd = faults[tiles[tk.t0].fault];
    const int err = *fd.err;
    const long long b = *fd.step - 1;
    for (int k = wave; k < nt; k += wpb) {
      const Tile tl = tiles[tk.t0 + k];
      double ax = 0.0, ay = 0.0, gx = 0.0, gy = 0.0;
      if (err == 0 && b >= 0) {
        const int Rn = tl.Rn;
        const double kL = 2.0 * M_PI * (double)tl.mode;
        const double csk = fd.cs * kL / fd.L, inv = 1.0 / csk;
        const double cutT = fmin(kL, fd.kcT), cutN = fmin(kL, fd.kcN);
        const Rec* __restrict__ ring = (const Rec*)fd.ring + tl.ring_off;
        const int end = tl.p0 + tl.len;
        // The tile's newest interval sits in its last slot, or in the slot of
        // interval b when the tile holds it; every other slot of the tile
        // holds an older one.  When that interval is past both windows (or
        // none is stored yet) the whole tile weighs 0: one log read instead
        // of one per slot.
        const int pb = mod_pos(b, Rn);
        const long long In = (pb >= tl.p0 && pb < end)
                                 ? b
                                 : b - (long long)mod_pos(b - (end - 1) + (long long)Rn * 4, Rn);
        bool live = In >= 0;
        if (live) {
          const double Tn = csk * (va.t_new - fd.tlog[In % fd.tlog_cap].y);
          live = Tn < cutT || Tn < cutN;
        }
        // (a dead tile still reduces and records its zero partial below)
        //
        // Interval I + 1 starts where I ends (the log holds the same double),
        // so the primitive at the end of slot p's interval is the primitive at
        // the start of slot p + 1's: each lane evaluates P at its interval's
        // start only and takes the end value from the next lane.  Chunks run
        // newest last, so lane 63 takes it from lane 0 of the chunk after;
        // only the tile's last slot and the slot of the newest interval b
        // (whose successor slot holds the oldest one) evaluate it directly.
        // every slot's log entry and record are requested before any is
        // used, so that a wave has all of its tile's loads in flight at once
        double2 ivs[U];
        Rec recs[U];
        bool valids[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int p = tl.p0 + lane + 64 * u;
          bool valid = live && p < end;
          const long long I =
              valid ? b - (long long)mod_pos(b - p + (long long)Rn * 4, Rn) : -1;
          valid = valid && I >= 0;
          valids[u] = valid;
          ivs[u] = valid ? fd.tlog[I % fd.tlog_cap] : make_double2(0.0, 0.0);
          if (valid) recs[u] = ring[p];
        }
        double nxT = 0.0, nxN = 0.0;  // P at lane 0's start in the chunk after
#pragma unroll
        for (int u = U - 1; u >= 0; --u) {
          const int p = tl.p0 + lane + 64 * u;
          const bool valid = valids[u];
          const double2 iv = ivs[u];
          const double Ta = csk * (va.t_new - iv.y), Tb = csk * (va.t_new - iv.x);
          double pTb = 0.0, pNb = 0.0, qNb = 0.0;  // q: the normal kind's own cut
          if (valid) {
            ptab_eval(fd.ptab, fd.ptab_len, fd.ptab_h, fmin(Tb, cutT), &pTb, &pNb);
            if (cutN != cutT) {
              double x;
              ptab_eval(fd.ptab, fd.ptab_len, fd.ptab_h, fmin(Tb, cutN), &x, &qNb);
            } else {
              qNb = pNb;
            }
          }
          // end values from the next slot (lane + 1, or lane 0 of chunk u + 1)
          double pTa = __shfl_down(pTb, 1), qNa = __shfl_down(qNb, 1);
          if (lane == 63) {
            pTa = nxT;
            qNa = nxN;
          }
          nxT = __shfl(pTb, 0);
          nxN = __shfl(qNb, 0);
          const bool inwin = valid && !(Ta >= cutT && Ta >= cutN);
          const bool shared = (lane < 63 || u < U - 1) && p + 1 < end && p != pb;
          if (inwin && !shared) {
            double x;
            ptab_eval(fd.ptab, fd.ptab_len, fd.ptab_h, fmin(Ta, cutT), &pTa, &qNa);
            if (cutN != cutT) ptab_eval(fd.ptab, fd.ptab_len, fd.ptab_h, fmin(Ta, cutN), &x, &qNa);
          }
          if (!inwin) continue;
          const double wT = (pTb - pTa) * inv;
          const double wN = (qNb - qNa) * inv;
          const Rec r = recs[u];
          if constexpr (sizeof(R) == 4) {
            ax = fma(wT, (double)r.x, ax);
            ay = fma(wT, (double)r.y, ay);
            gx = fma(wN, (double)r.z, gx);
            gy = fma(wN, (double)r.w, gy);
          } else {
            ax = fma(wT, r.v.x, ax);
            ay = fma(wT, r.v.y, ay);
            gx = fma(wN, r.g.x, gx);
            gy = fma(wN, r.g.y, gy);
          }
        }
      }
      Rec64 acc;
      acc.v = d2(ax, ay);
      acc.g = d2(gx, gy);
      acc = wave_reduce_r64(acc);
      if (lane == 0) {
        L.part[k] = make_double4(acc.v.x, acc.v.y, acc.g.x, acc.g.y);
        L.id[k] = tl.part;
      }
    }
    __syncthreads();
    finish_task(fd, L, nt);
    __syncthreads();
  }
}

__global__ void k_reset_cells(const FaultDev* __restrict__ faults, int nfaults) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfaults) return;
  int* c = faults[f].cells;
  c[0] = kNoExp;
  c[1] = kNoExp;
  c[2] = kNoExp;
  c[3] = kNoExp;
}

// out[0] = max_i max(|ln Va_i - ln Vb_i|, |ln tha_i - ln thb_i|) and
// out[1] = max_i Vb_i, each folded in as the bit pattern of a non-negative
// double (which orders like its bits).
__global__ void k_err_norm(const double* __restrict__ Va, const double* __restrict__ tha,
                           const double* __restrict__ Vb, const double* __restrict__ thb, int n,
                           unsigned long long* __restrict__ out, const int* __restrict__ err) {
  if (err && blockIdx.x == 0 && threadIdx.x == 0) {
    out[2] = (unsigned long long)(unsigned)err[0];
    out[3] = ((unsigned long long)(unsigned)err[1] << 32) | (unsigned)err[2];
  }
  double m = 0.0, vm = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    vm = fmax(vm, Vb[i]);
    // equal values (constrained elements, where V may be 0) contribute 0
    const double e1 = Va[i] == Vb[i] ? 0.0 : fabs(log(Va[i]) - log(Vb[i]));
    const double e2 = tha[i] == thb[i] ? 0.0 : fabs(log(tha[i]) - log(thb[i]));
    m = fmax(m, fmax(e1, e2));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    vm = fmax(vm, __shfl_xor(vm, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(vm));
  }
}

hipError_t launch_conv_var(const Exec& ex, const VarArgs& va, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  if (ex.ntasks == 0) return hipSuccess;
  const int grid = std::min(ex.ntasks, 4096);
  // with events: stamped by the kernel's own dispatch (its execution alone)
  if (ex.precision == SBIEM_FP32CONV)
    hipExtLaunchKernelGGL(k_conv_var<float>, dim3(grid), dim3(kConvThreads), 0, s, e0, e1, 0,
                          ex.d_faults, ex.d_tiles, ex.d_tasks, ex.ntasks, va);
  else
    hipExtLaunchKernelGGL(k_conv_var<double>, dim3(grid), dim3(kConvThreads), 0, s, e0, e1, 0,
                          ex.d_faults, ex.d_tiles, ex.d_tasks, ex.ntasks, va);
  return hipGetLastError();
}

hipError_t launch_reset_cells(const Exec& ex, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_cells, dim3((ex.nfaults + 63) / 64), dim3(64), 0, s, ex.d_faults,
                     ex.nfaults);
  return hipGetLastError();
}

hipError_t launch_err_norm(const double* Va, const double* tha, const double* Vb,
                           const double* thb, int n, unsigned long long* out, hipStream_t s,
                           const int* err, bool zeroed) {
  if (!zeroed) {
    hipError_t e = hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), s);
    if (e) return e;
  }
  const int blocks = std::max(1, std::min((n + 255) / 256, 1024));
  hipLaunchKernelGGL(k_err_norm, dim3(blocks), dim3(256), 0, s, Va, tha, Vb, thb, n, out, err);
  return hipGetLastError();
}

// Entry blockIdx.y of the list: copy (or zero-fill) its words.
__global__ void __launch_bounds__(256) k_copy_many(CopyList c) {
  const int k = blockIdx.y;
  if (k >= c.n) return;
  const long long w = c.words[k];
  unsigned long long* __restrict__ d = (unsigned long long*)c.dst[k];
  const unsigned long long* __restrict__ sr = (const unsigned long long*)c.src[k];
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < w; i += 256LL * gridDim.x)
    d[i] = sr ? sr[i] : 0ULL;
}

hipError_t launch_copy_many(const CopyList& c, int max_words, hipStream_t s) {
  if (c.n == 0) return hipSuccess;
  const int bx = std::max(1, std::min((max_words + 255) / 256, 64));
  hipLaunchKernelGGL(k_copy_many, dim3(bx, c.n), dim3(256), 0, s, c);
  return hipGetLastError();
}

// Stress path: ring slot p of mode n receives the latest interval
// l <= nint - 2 with l = p (mod R_n) (zero if none); hprev = interval nint-2.
// RV, RG hold the interval spectra at mode_pos, stride N/2 + 1.
template <typename R>
__global__ void k_fill_ring(const FaultDev* __restrict__ fdp, const double2* __restrict__ RV,
                            const double2* __restrict__ RG, int nint) {
  using Rec = typename Prec<R>::Rec;
  const FaultDev& fd = *fdp;
  const int n = blockIdx.x;  // mode
  const int pm = mode_pos(n, fd.log2P, fd.log2Q);
  const int stride = fd.nmodes + 1;
  const long long last = (long long)nint - 2;
  if (threadIdx.x == 0) {
    fd.hprev_v[pm] = last >= 0 ? RV[last * stride + pm] : d2(0, 0);
    fd.hprev_g[pm] = last >= 0 ? RG[last * stride + pm] : d2(0, 0);
  }
  const ModeCoef cf = fd.coef[pm];
  const int Rn = cf.Rn;
  if (n == 0 || Rn == 0) return;
  for (int p = threadIdx.x; p < Rn; p += blockDim.x) {
    double2 v = d2(0, 0), g = d2(0, 0);
    if (last >= 0) {
      const long long ll = last - posmod(last - p, Rn);
      if (ll >= 0) {
        v = RV[ll * stride + pm];
        g = RG[ll * stride + pm];
      }
    }
    Rec rec;
    if constexpr (sizeof(R) == 4) {
      rec = make_float4((float)v.x, (float)v.y, (float)g.x, (float)g.y);
    } else {
      rec.v = v;
      rec.g = g;
    }
    ((Rec*)fd.ring)[cf.ring_off + p] = rec;
  }
}

// rates[l*N + i] = (hist[(l+1)*N + i] - hist[l*N + i]) / dt
__global__ void k_rates(const double* __restrict__ hist, double* __restrict__ rates, long long count,
                        long long N, double inv_dt) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < count;
       k += (long long)gridDim.x * blockDim.x)
    rates[k] = (hist[k + N] - hist[k]) * inv_dt;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void split_sizes(int log2N, int* log2P, int* log2Q, int* ncls) {
  const int lp = log2N / 2;
  *log2P = lp;
  *log2Q = log2N - lp;
  const int P = 1 << lp, Q = 1 << (log2N - lp);
  int n = kElemThreads / P;
  if (n < 1) n = 1;
  if (n > Q) n = Q;
  *ncls = n;
}

size_t mode_lds_bytes(int precision, int log2Q) {
  const size_t c = precision == SBIEM_FP32CONV ? sizeof(float2) : sizeof(double2);
  const size_t r = precision == SBIEM_FP32CONV ? sizeof(float) : sizeof(double);
  const int Q = 1 << log2Q;
  return 4 * (size_t)vstride(Q) * c + (size_t)(Q / 4 + 1) * r;
}

size_t elem_lds_bytes(int precision, int log2P, int ncls) {
  const size_t c = precision == SBIEM_FP32CONV ? sizeof(float2) : sizeof(double2);
  const size_t r = precision == SBIEM_FP32CONV ? sizeof(float) : sizeof(double);
  const int P = 1 << log2P;
  return 2 * (size_t)ncls * vstride(P) * c + (size_t)(P / 4 + 1) * r;
}

template <typename R>
static hipError_t set_attributes() {
  const hipFuncAttribute a = hipFuncAttributeMaxDynamicSharedMemorySize;
  const int bytes = kMaxDynLds;
  hipError_t e = hipFuncSetAttribute((const void*)k_modes<R, 0>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_modes<R, 1>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_modes<R, 2>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_modes<R, 3>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_elems<R, 0>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_elems<R, 1>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_elems<R, 2>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_elems<R, 3>, a, bytes);
  return e;
}

template <int U, int K>
static hipError_t conv32_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_conv32<U, K, kLoadStream>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
  if (!e)
    e = hipFuncSetAttribute((const void*)k_conv32<U, K, kLoadCached>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
  return e;
}

hipError_t setup_kernel_attributes(int precision) {
  static bool done[2] = {false, false};
  const int idx = precision == SBIEM_FP32CONV ? 1 : 0;
  if (done[idx]) return hipSuccess;
  hipError_t e = idx ? set_attributes<float>() : set_attributes<double>();
  if (!e && idx) e = conv32_attributes<8, 2>();
  if (!e && idx) e = conv32_attributes<4, 4>();
  if (!e && idx) e = conv32_attributes<16, 1>();
  if (!e && idx) e = conv32_attributes<5, 4>();
  if (!e && idx)
    e = hipFuncSetAttribute((const void*)k_conv32p, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kMaxLdsBytes - kConvStaticLds);
  if (!e) done[idx] = true;
  return e;
}

int conv_grid_size(int precision, int ntasks, int table_len, int reserve) {
  int need = ntasks;
  if (precision == SBIEM_FP32CONV) {
    // persistent: at most as many workgroups as are resident at once (LDS
    // table and registers allow two per CU), so no workgroup waits for a
    // slot.  Two resident workgroups fill a CU's registers, so the stage
    // launches of the step, which run beside the convolution, find no CU
    // until it ends; `reserve` workgroups fewer leave that many CUs with
    // one, where the stages run in the convolution's shadow.
    const int per_cu = (int)(kMaxLdsBytes / ((size_t)table_len * sizeof(float4) + kConvStaticLds));
    int cap = 256 * (per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu));
    cap = std::max(256, cap - std::max(0, reserve));
    return need < cap ? (need < 1 ? 1 : need) : cap;
  }
  return need < 1 ? 1 : need;
}

int default_conv_reserve(double bytes) {
  // below a few GB of ring per launch the stages' share of the step is large
  // enough for the overlap to pay; above, the convolution's own time
  // dominates and the full grid is faster (sbiem_tune measures instead)
  return bytes < 4e9 ? 64 : 0;
}

// the tiled FP32 conv with the cache policy the context uses
template <int U, int K>
static void launch_conv32(const Exec& ex, int ahead, hipStream_t s, size_t lds) {
  if (!ex.cached_loads)
    hipLaunchKernelGGL((k_conv32<U, K, kLoadStream>), dim3(ex.conv_grid), dim3(kConvThreads), lds,
                       s, ex.d_faults, ex.d_tiles, ex.d_tasks, ex.ntasks, ex.table, ex.table_len,
                       ahead, ex.conv_ctr);
  else
    hipLaunchKernelGGL((k_conv32<U, K, kLoadCached>), dim3(ex.conv_grid), dim3(kConvThreads), lds,
                       s, ex.d_faults, ex.d_tiles, ex.d_tasks, ex.ntasks, ex.table, ex.table_len,
                       ahead, ex.conv_ctr);
}

hipError_t launch_conv(const Exec& ex, int ahead, hipStream_t s) {
  if (ex.ntasks == 0) return hipSuccess;
  if (ex.precision == SBIEM_FP32CONV) {
    const size_t lds = (size_t)ex.table_len * sizeof(float4);
    static_assert(kTileSlots32 == 8 * 64 && kWaveTiles32 == 2, "tile shape");
    static_assert(kTileSlots32s == 4 * 64 && kWaveTiles32s == 4, "short tile shape");
    static_assert(kTileSlots32l == 16 * 64, "long tile shape");
    static_assert(kTileSlots32w == 5 * 64 && conv32_wave_tiles(kTileSlots32w) == 4,
                  "wide tile shape");
    if (ex.tile_rows == 1)
      hipLaunchKernelGGL(k_conv32p, dim3(ex.conv_grid), dim3(kConvThreads), lds, s, ex.d_faults,
                         (const RowDesc*)ex.d_tiles, ex.d_tasks, ex.ntasks, ex.table, ex.table_len,
                         ahead);
    else if (ex.tile_rows == 4)
      launch_conv32<4, 4>(ex, ahead, s, lds);
    else if (ex.tile_rows == 16)
      launch_conv32<16, 1>(ex, ahead, s, lds);
    else if (ex.tile_rows == 5)
      launch_conv32<5, 4>(ex, ahead, s, lds);
    else
      launch_conv32<8, 2>(ex, ahead, s, lds);
  } else {
    hipLaunchKernelGGL(k_conv64, dim3(ex.conv_grid), dim3(kConvThreads), 0, s, ex.d_faults,
                       ex.d_tiles, ex.d_tasks, ex.ntasks, ahead);
  }
  return hipGetLastError();
}

template <typename R>
static void modes_kind(const Exec& ex, int kind, int measure, hipStream_t s, const VarArgs& va) {
  const dim3 grid(ex.mode_blocks), block(kModeThreads);
  const size_t lds = ex.mode_lds;
  const int2* map = ex.nfaults == 1 ? nullptr : ex.d_mode_map;  // one fault: group = block
  switch (kind) {
    case 0:
      k_modes<R, 0><<<grid, block, lds, s>>>(ex.d_faults, map, measure, nullptr, nullptr,
                                              nullptr, 0, ex.conv_ctr, va);
      break;
    case 1:
      k_modes<R, 1><<<grid, block, lds, s>>>(ex.d_faults, map, 0, nullptr, nullptr,
                                              nullptr, 0, nullptr, va);
      break;
    default:
      k_modes<R, 2><<<grid, block, lds, s>>>(ex.d_faults, map, 0, nullptr, nullptr,
                                              nullptr, 0, ex.conv_ctr, va);
      break;
  }
}

hipError_t launch_modes(const Exec& ex, int kind, int measure, hipStream_t s, const VarArgs& va) {
  if (ex.precision == SBIEM_FP32CONV) modes_kind<float>(ex, kind, measure, s, va);
  else modes_kind<double>(ex, kind, measure, s, va);
  return hipGetLastError();
}

template <typename R>
static void elems_kind(const Exec& ex, int kind, hipStream_t s, const VarArgs& va) {
  const dim3 grid(ex.elem_blocks), block(kElemThreads);
  const size_t lds = ex.elem_lds;
  const int2* map = ex.nfaults == 1 ? nullptr : ex.d_elem_map;
  switch (kind) {
    case 0: k_elems<R, 0><<<grid, block, lds, s>>>(ex.d_faults, map, nullptr, nullptr, va); break;
    case 1: k_elems<R, 1><<<grid, block, lds, s>>>(ex.d_faults, map, nullptr, nullptr, va); break;
    default: k_elems<R, 2><<<grid, block, lds, s>>>(ex.d_faults, map, nullptr, nullptr, va); break;
  }
}

hipError_t launch_elems(const Exec& ex, int kind, hipStream_t s, const VarArgs& va) {
  if (ex.precision == SBIEM_FP32CONV) elems_kind<float>(ex, kind, s, va);
  else elems_kind<double>(ex, kind, s, va);
  return hipGetLastError();
}

hipError_t launch_forward(const FaultDev* d_fault, const FaultDev& h, int precision,
                          const double* a, double2* A, double2* B, int count, long long stride_out,
                          void* gF, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 eg((unsigned)(h.Q / h.ncls), (unsigned)count), mg((unsigned)h.ngroups, (unsigned)count);
  const size_t el = elem_lds_bytes(precision, h.log2P, h.ncls), ml = mode_lds_bytes(precision, h.log2Q);
  const VarArgs off{0.0, 0.0, 0.0, 0, 0};
  if (precision == SBIEM_FP32CONV) {
    k_elems<float, 3><<<eg, dim3(kElemThreads), el, s>>>(d_fault, nullptr, a, gF, off);
    k_modes<float, 3><<<mg, dim3(kModeThreads), ml, s>>>(d_fault, nullptr, 0, gF, A, B, stride_out,
                                                          nullptr, off);
  } else {
    k_elems<double, 3><<<eg, dim3(kElemThreads), el, s>>>(d_fault, nullptr, a, gF, off);
    k_modes<double, 3><<<mg, dim3(kModeThreads), ml, s>>>(d_fault, nullptr, 0, gF, A, B, stride_out,
                                                           nullptr, off);
  }
  return hipGetLastError();
}

hipError_t launch_rates(const double* hist, double* rates, long long count, long long N, double dt,
                        hipStream_t s) {
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_rates, dim3((unsigned)blocks), dim3(256), 0, s, hist, rates, count, N, 1.0 / dt);
  return hipGetLastError();
}

hipError_t launch_fill_ring(const FaultDev* d_fault, int precision, int nmodes, const double2* RV,
                            const double2* RG, int nint, hipStream_t s) {
  if (precision == SBIEM_FP32CONV)
    hipLaunchKernelGGL(k_fill_ring<float>, dim3(nmodes + 1), dim3(256), 0, s, d_fault, RV, RG, nint);
  else
    hipLaunchKernelGGL(k_fill_ring<double>, dim3(nmodes + 1), dim3(256), 0, s, d_fault, RV, RG, nint);
  return hipGetLastError();
}

}  // namespace sbiem

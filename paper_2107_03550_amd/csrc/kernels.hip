// HIP kernels of the sBIEM time step for gfx950 (CDNA4, wave64).
//
// One step (section 3.3) is five launches over every fault of a context:
//   k_conv    history sums over lags >= 2 of every mode (HBM-bound stream of
//             the wavenumber-major ring; one wavefront per tile of records)
//   k_pass1   per fault, one workgroup: reduce the conv partials, assemble
//             the traction spectra of pass 1 (section 3.1 + current interval
//             + last interval), inverse FFT in LDS -> tau^el(x), sigma^el(x)
//   k_newton  per element: predictor, momentum balance (Newton on ln V),
//             aging law; writes the FFT input (V_p - V_pl) + i kappa (V_p - V_pl)
//   k_pass2   per fault: forward FFT of the pass-1 rates, pass-2 assembly
//             with V_c = (V_0 + V_1)/2, inverse FFT
//   k_newton  pass 2 (writes the next state)
//   k_commit  per fault: forward FFT of V_2, push (V_0 + V_1)/2 into the ring,
//             advance the spectral slip and the step counter
#include "internal.h"

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
// LDS-resident radix-8/4/2 Stockham FFT (forward, exp(-2 pi i n k / N)).
// Pass with radix RD after sub-transforms of length p: butterfly i takes
// x[i + r N/RD], twiddles by exp(-2 pi i r k / (p RD)) with k = i mod p, and
// writes the RD outputs to (i - k) RD + k + s p.  Every thread first loads
// all inputs of its butterflies, then (after a barrier) writes the outputs,
// so one LDS buffer suffices.
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

template <typename C, typename R, int LR, int MAXPTS>
__device__ __forceinline__ void fft_pass(C* buf, int N, int p, const R* __restrict__ q, int ps) {
  constexpr int RD = 1 << LR;
  constexpr int MAXB = ((MAXPTS >> LR) + kSpecThreads - 1) / kSpecThreads;
  const int nb = N >> LR;
  C x[MAXB][RD];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int i = threadIdx.x + b * kSpecThreads;
    if (i < nb) {
#pragma unroll
      for (int r = 0; r < RD; ++r) x[b][r] = buf[lx(i + r * nb, ps)];
    }
  }
  __syncthreads();
  const int tws = N / (p * RD);
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int i = threadIdx.x + b * kSpecThreads;
    if (i < nb) {
      const int k = i & (p - 1);
      if (p > 1) {
        // w^r = exp(-2 pi i r k / (p RD)) from one lookup and products
        const C w1 = twiddle_half<C, R>(q, k * tws, N);
        x[b][1] = cmul(x[b][1], w1);
        if (RD >= 4) {
          const C w2 = cmul(w1, w1);
          const C w3 = cmul(w2, w1);
          x[b][2] = cmul(x[b][2], w2);
          x[b][3] = cmul(x[b][3], w3);
          if (RD == 8) {
            const C w4 = cmul(w2, w2);
            x[b][4] = cmul(x[b][4], w4);
            x[b][5] = cmul(x[b][5], cmul(w4, w1));
            x[b][6] = cmul(x[b][6], cmul(w4, w2));
            x[b][7] = cmul(x[b][7], cmul(w4, w3));
          }
        }
      }
      if (RD == 8) dft8(x[b]);
      else if (RD == 4) dft4(x[b][0], x[b][1], x[b][2], x[b][3]);
      else dft2(x[b]);
      const int base = (i - k) * RD + k;
#pragma unroll
      for (int s = 0; s < RD; ++s) buf[lx(base + s * p, ps)] = x[b][s];
    }
  }
  __syncthreads();
}

// Forward FFT of buf[0..N) in LDS (q: quarter-wave table in LDS); the caller
// has synchronised after filling both.
template <typename C, typename R, int MAXPTS>
__device__ __forceinline__ void fft_lds(C* buf, int N, int log2N, const R* __restrict__ q, int ps) {
  int p = 1, rem = log2N;
  while (rem >= 3) {
    fft_pass<C, R, 3, MAXPTS>(buf, N, p, q, ps);
    p <<= 3;
    rem -= 3;
  }
  if (rem == 2) fft_pass<C, R, 2, MAXPTS>(buf, N, p, q, ps);
  else if (rem == 1) fft_pass<C, R, 1, MAXPTS>(buf, N, p, q, ps);
}

template <typename R> struct Prec;
template <> struct Prec<float> {
  using C = float2;
  using Rec = float4;  // (v_re, v_im, g_re, g_im)
  static constexpr int kMaxPts = 16384;
  static constexpr int kTile = kTileSlots32;
};
struct Rec64 {
  double2 v, g;
};
template <> struct Prec<double> {
  using C = double2;
  using Rec = Rec64;
  static constexpr int kMaxPts = 8192;
  static constexpr int kTile = kTileSlots64;
};

// LDS bytes of a spectral kernel for N points: padded data + quarter table.
template <typename R>
__host__ __device__ inline size_t spec_lds_bytes(int N, int ps) {
  return (size_t)(N + (N >> ps)) * sizeof(typename Prec<R>::C) + (size_t)(N / 4 + 1) * sizeof(R);
}
// Pad one element in 8 when it fits, else one in 16.
template <typename R>
__host__ __device__ inline int pad_shift(int N) {
  return spec_lds_bytes<R>(N, 3) <= (size_t)kMaxDynLds ? 3 : 4;
}

// ---------------------------------------------------------------------------
// History convolution.  Slot p of mode n's ring holds interval
// I(p) = b - ((b - p) mod R_n) with b = step - 1 the last committed interval;
// its lag at this step is j = 1 + ((b - p) mod R_n).  The slot of lag 1
// (p = b mod R_n) is skipped here (the spectral kernels add it from hprev),
// which also makes this launch independent of the step's own commit.
// The weight of slot p is at q = (p - b) mod R_n = (p + o) mod R_n with
// o = (-b) mod R_n: q = 0 is the skipped slot, lag j = R_n - q + 1 otherwise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 wave_reduce4(float4 v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
    v.z += __shfl_xor(v.z, off);
    v.w += __shfl_xor(v.w, off);
  }
  return v;
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

// One workgroup per task (a run of tiles of one fault): each wave sums tiles
// of the task, the per-tile FP64 partials go to LDS, and after a barrier the
// first thread of each (task, mode) run adds its tiles in order and stores
// the sum in parts[part].  The spectral kernel adds a mode's parts in order,
// so every sum has a fixed order and results are reproducible.
struct TaskLds {
  double4 part[kTaskTiles];
  int id[kTaskTiles];
};

__device__ __forceinline__ void finish_task(const FaultDev& fd, const TaskLds& L, int nt) {
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
    fd.parts[L.id[k]] = a;
  }
}

__global__ void __launch_bounds__(kConvThreads)
k_conv64(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles,
         const ConvTask* __restrict__ tasks, int ntasks) {
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
    const long long step = *fd.step;
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
__global__ void __launch_bounds__(kConvThreads)
k_conv32(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles,
         const ConvTask* __restrict__ tasks, int ntasks, const float4* __restrict__ table,
         int table_len) {
  constexpr int U = kTileSlots32 / 64;
  extern __shared__ float4 tab[];
  __shared__ TaskLds L;
  for (int i = threadIdx.x; i < table_len; i += kConvThreads) tab[i] = table[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wpb = kConvThreads / 64;
  for (int task = blockIdx.x; task < ntasks; task += gridDim.x) {
    const ConvTask tk = tasks[task];
    const int nt = tk.t1 - tk.t0;
    const FaultDev& fd = faults[tiles[tk.t0].fault];
    const int err = *fd.err;
    const long long step = *fd.step;
    for (int k = wave; k < nt; k += wpb) {
      const Tile tl = tiles[tk.t0 + k];
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      if (err == 0) {
        const int Rn = tl.Rn;
        const int o = ring_phase(step, Rn);
        const double th = tl.th;
        const float4* __restrict__ ring = (const float4*)fd.ring + tl.ring_off;
        const int end = tl.p0 + tl.len;
        float4 h[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int p = tl.p0 + lane + 64 * u;
          h[u] = p < end ? ring[p] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
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
          wT = use ? wT : 0.f;
          wN = use ? wN : 0.f;
          acc.x = fmaf(wT, h[u].x, acc.x);
          acc.y = fmaf(wT, h[u].y, acc.y);
          acc.z = fmaf(wN, h[u].z, acc.z);
          acc.w = fmaf(wN, h[u].w, acc.w);
        }
      }
      acc = wave_reduce4(acc);
      if (lane == 0) {
        L.part[k] = make_double4(acc.x, acc.y, acc.z, acc.w);
        L.id[k] = tl.part;
      }
    }
    __syncthreads();
    finish_task(fd, L, nt);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Spectral kernels (one workgroup per fault, N complex in LDS)
// ---------------------------------------------------------------------------
// Block-wide maxima of two non-negative values (all threads get the result).
__device__ __forceinline__ void block_max2(double& a, double& b) {
  constexpr int W = kSpecThreads / 64;
  __shared__ double red[2][W];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off));
    b = fmax(b, __shfl_xor(b, off));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  double ra[W], rb[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    ra[w] = red[0][w];
    rb[w] = red[1][w];
  }
  a = 0.0;
  b = 0.0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    a = fmax(a, ra[w]);
    b = fmax(b, rb[w]);
  }
  __syncthreads();
}

// Power of two closest to x/y (1 when either is zero or not finite).  Two
// real signals packed into one complex transform share its rounding error;
// scaling the smaller one up by an exact power of two keeps each at its own
// relative accuracy.
__device__ __forceinline__ double pow2_ratio(double x, double y) {
  if (!(x > 0.0) || !(y > 0.0) || !isfinite(x) || !isfinite(y)) return 1.0;
  return ldexp(1.0, ilogb(x) - ilogb(y));
}

// LDS layout of the spectral kernels: N complex values (padded), then the
// quarter-wave twiddle table (N/4 + 1 reals) copied from global memory.
template <typename R, int MAXPTS>
__device__ __forceinline__ const R* load_quarter_table(typename Prec<R>::C* buf, const FaultDev& fd) {
  constexpr int K = (MAXPTS / 4) / kSpecThreads + 1;
  R* q = reinterpret_cast<R*>(buf + fd.N + (fd.N >> pad_shift<R>(fd.N)));
  const R* __restrict__ g = (const R*)fd.twiddle;
  const int Q = fd.N >> 2;
  R v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = g[min((int)threadIdx.x + k * kSpecThreads, Q)];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + k * kSpecThreads;
    if (i <= Q) q[i] = v[k];
  }
  return q;
}

// Copy the FFT input z (the Newton kernel has already scaled its curvature
// half by fwd_scale) into LDS; all loads of a thread are issued first.
template <typename R, int MAXPTS>
__device__ __forceinline__ void load_input(typename Prec<R>::C* buf, int N,
                                           const typename Prec<R>::C* __restrict__ z, int ps) {
  using C = typename Prec<R>::C;
  constexpr int K = MAXPTS / kSpecThreads;
  C v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = z[min((int)threadIdx.x + k * kSpecThreads, N - 1)];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + k * kSpecThreads;
    if (i < N) buf[lx(i, ps)] = v[k];
  }
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

// Modes one thread owns in the spectral kernels (n = tid + s T).
template <int MAXPTS>
struct ModesPerThread {
  static constexpr int value = (MAXPTS / 2 + kSpecThreads) / kSpecThreads;
};

constexpr int kInvExpUnset = -100000;

// Exponent bookkeeping of the inverse packing: LDS cells for the block
// maxima of ilogb|tau_hat| and ilogb|sigma_hat|.
struct InvScale {
  int tau_e, sig_e;
};

// log2 of the balancing factor from the two maxima (0 when either is zero).
__device__ __forceinline__ int balance_exp(const InvScale* sc) {
  if (sc->tau_e <= -2000 || sc->sig_e <= -2000) return 0;
  return min(max(sc->tau_e - sc->sig_e, -256), 256);
}

__device__ __forceinline__ int ilogb_or_min(double x) {
  return (x > 0.0 && x <= 1.0e300) ? ilogb(x) : -2000;
}

// Pack Z = tau_hat + i c sigma_hat (c = 2^e, e from the previous pass or, on
// the first pass after a reset, from this pass's maxima) as conj(Z), inverse
// transform in LDS and write tau^el, sigma^el; record this pass's maxima for
// the next pass.  The inverse of Z is conj(FFT(conj Z))/N.
template <typename R, int MAXPTS>
__device__ __forceinline__ void invert_tractions(const FaultDev& fd, typename Prec<R>::C* buf,
                                                 const R* q, const typename Prec<R>::C* tau,
                                                 const typename Prec<R>::C* sig, double mt,
                                                 double ms, InvScale* sc, int e_prev) {
  using C = typename Prec<R>::C;
  constexpr int kPer = ModesPerThread<MAXPTS>::value;
  const int N = fd.N, half = fd.nmodes;
  const int ps = pad_shift<R>(N);
  // this pass's maxima: wave reduction, then an LDS atomic per wave
  int et = ilogb_or_min(mt), es = ilogb_or_min(ms);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    et = max(et, __shfl_xor(et, off));
    es = max(es, __shfl_xor(es, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sc->tau_e, et);
    atomicMax(&sc->sig_e, es);
  }
  int e = e_prev;
  if (e == kInvExpUnset) {  // first pass after a reset: use this pass's maxima
    __syncthreads();
    e = balance_exp(sc);
  }
  const double c = ldexp(1.0, e);
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    const int n = threadIdx.x + sl * kSpecThreads;
    if (n <= half) {
      const double2 t = d2(tau[sl].x, tau[sl].y);
      const double2 g = d2((double)sig[sl].x * c, (double)sig[sl].y * c);
      buf[lx(n, ps)] = cmk<C>(t.x - g.y, -(t.y + g.x));
      if (n > 0 && 2 * n < N) buf[lx(N - n, ps)] = cmk<C>(t.x + g.y, -(-t.y + g.x));
    }
  }
  __syncthreads();
  fft_lds<C, R, MAXPTS>(buf, N, fd.log2N, q, ps);
  const int slot = (int)((*fd.step + 1) & 1);
  double* __restrict__ to = fd.tau_el[slot];
  double* __restrict__ so = fd.sigma_el[slot];
  const double inv = 1.0 / N, invc = 1.0 / (c * N);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const C z = buf[lx(i, ps)];
    to[i] = (double)z.x * inv;
    so[i] = -(double)z.y * invc;
  }
  // the FFT's barriers have ordered every atomicMax above
  if (threadIdx.x == 0)
    *fd.inv_exp = balance_exp(sc);
}

// Unpack the FFT Z of z = a + i s b (a, b real, s the forward scale) into
// A_n, B_n, n = 0..N/2.
template <typename C>
__device__ __forceinline__ void unpack_mode(const C* buf, int N, int n, double inv_s, double2* A,
                                            double2* B, int ps) {
  const C zn = buf[lx(n, ps)];
  const C zm = buf[lx(n == 0 ? 0 : N - n, ps)];
  // A = (Z_n + conj Z_m)/2, B = (Z_n - conj Z_m)/(2i)
  *A = d2(0.5 * ((double)zn.x + (double)zm.x), 0.5 * ((double)zn.y - (double)zm.y));
  const double dx = (double)zn.x - (double)zm.x, dy = (double)zn.y + (double)zm.y;
  *B = d2(0.5 * dy * inv_s, -0.5 * dx * inv_s);
}

__device__ __forceinline__ void init_inv_scale(InvScale* sc) {
  if (threadIdx.x == 0) {
    sc->tau_e = -2000;
    sc->sig_e = -2000;
  }
}

template <typename R, int MAXPTS>
__global__ void __launch_bounds__(kSpecThreads)
k_pass1(const FaultDev* __restrict__ faults) {
  using C = typename Prec<R>::C;
  constexpr int kPer = ModesPerThread<MAXPTS>::value;
  extern __shared__ unsigned char smem_raw[];
  __shared__ InvScale sc;
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = faults[blockIdx.x];
  const int err = *fd.err;
  const int e_prev = *fd.inv_exp;
  if (err) return;
  init_inv_scale(&sc);
  __syncthreads();  // the maxima cells are set before any wave updates them
  const R* q = load_quarter_table<R, MAXPTS>(buf, fd);
  const int half = fd.nmodes;
  C tau[kPer], sig[kPer];
  double mt = 0.0, ms = 0.0;
  // groups of three modes: all loads of a group are issued before its stores
  constexpr int G = (sizeof(R) == 4 && MAXPTS <= 8192) ? 2 : 1;
#pragma unroll
  for (int s0 = 0; s0 < kPer; s0 += G) {
    double4 S[G];
    double2 P[G][2], V[G][2];
    ModeCoef cf[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int n = threadIdx.x + (s0 + k) * kSpecThreads;
      if (s0 + k < kPer && n <= half) {
        cf[k] = fd.coef[n];
        S[k] = fd.parts[n];
        P[k][0] = fd.P_T[n];
        P[k][1] = fd.P_N[n];
        V[k][0] = fd.v_hat0[n];
        V[k][1] = fd.gv_hat0[n];
      }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int sl = s0 + k;
      const int n = threadIdx.x + sl * kSpecThreads;
      if (sl < kPer && n <= half) {
        const ModeCoef& c = cf[k];
        double4 h = c.nparts > 0 ? S[k] : make_double4(0.0, 0.0, 0.0, 0.0);
        for (int j = 1; j < c.nparts; ++j) {  // further pieces of a long window
          const double4 b = fd.parts[c.part0 + j - 1];
          h.x += b.x;
          h.y += b.y;
          h.z += b.z;
          h.w += b.w;
        }
        const double2 BT = d2(P[k][0].x + h.x, P[k][0].y + h.y);
        const double2 BN = d2(P[k][1].x + h.z, P[k][1].y + h.w);
        fd.B_T[n] = BT;
        fd.B_N[n] = BN;
        double2 t, g;
        traction_mode(c, BT, BN, V[k][0], V[k][1], &t, &g);
        tau[sl] = cmk<C>(t.x, t.y);
        sig[sl] = cmk<C>(g.x, g.y);
        mt = fmax(mt, fmax(fabs(t.x), fabs(t.y)));
        ms = fmax(ms, fmax(fabs(g.x), fabs(g.y)));
      }
    }
  }
  invert_tractions<R, MAXPTS>(fd, buf, q, tau, sig, mt, ms, &sc, e_prev);
}

template <typename R, int MAXPTS>
__global__ void __launch_bounds__(kSpecThreads)
k_pass2(const FaultDev* __restrict__ faults) {
  using C = typename Prec<R>::C;
  constexpr int kPer = ModesPerThread<MAXPTS>::value;
  extern __shared__ unsigned char smem_raw[];
  __shared__ InvScale sc;
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = faults[blockIdx.x];
  const int err = *fd.err;
  const int e_prev = *fd.inv_exp;
  if (err) return;
  const int N = fd.N, half = fd.nmodes;
  const int ps = pad_shift<R>(N);
  init_inv_scale(&sc);
  const R* q = load_quarter_table<R, MAXPTS>(buf, fd);
  load_input<R, MAXPTS>(buf, N, (const C*)fd.zbuf, ps);
  __syncthreads();
  fft_lds<C, R, MAXPTS>(buf, N, fd.log2N, q, ps);
  const double inv_s = 1.0 / fd.fwd_scale;
  C tau[kPer], sig[kPer];
  double mt = 0.0, ms = 0.0;
  constexpr int G = (sizeof(R) == 4 && MAXPTS <= 8192) ? 2 : 1;
#pragma unroll
  for (int s0 = 0; s0 < kPer; s0 += G) {
    double2 Bv[G][2], V0[G][2];
    ModeCoef cf[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int n = threadIdx.x + (s0 + k) * kSpecThreads;
      if (s0 + k < kPer && n <= half) {
        cf[k] = fd.coef[n];
        Bv[k][0] = fd.B_T[n];
        Bv[k][1] = fd.B_N[n];
        V0[k][0] = fd.v_hat0[n];
        V0[k][1] = fd.gv_hat0[n];
      }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int sl = s0 + k;
      const int n = threadIdx.x + sl * kSpecThreads;
      if (sl < kPer && n <= half) {
        double2 A, B;
        unpack_mode(buf, N, n, inv_s, &A, &B, ps);
        fd.v_hat1[n] = A;
        fd.gv_hat1[n] = B;
        const double2 vc = d2(0.5 * (V0[k][0].x + A.x), 0.5 * (V0[k][0].y + A.y));
        const double2 gvc = d2(0.5 * (V0[k][1].x + B.x), 0.5 * (V0[k][1].y + B.y));
        double2 t, g;
        traction_mode(cf[k], Bv[k][0], Bv[k][1], vc, gvc, &t, &g);
        tau[sl] = cmk<C>(t.x, t.y);
        sig[sl] = cmk<C>(g.x, g.y);
        mt = fmax(mt, fmax(fabs(t.x), fabs(t.y)));
        ms = fmax(ms, fmax(fabs(g.x), fabs(g.y)));
      }
    }
  }
  __syncthreads();  // every unpack read of buf is done before the packing overwrites it
  invert_tractions<R, MAXPTS>(fd, buf, q, tau, sig, mt, ms, &sc, e_prev);
}

template <typename R, int MAXPTS>
__global__ void __launch_bounds__(kSpecThreads)
k_commit(const FaultDev* __restrict__ faults) {
  using C = typename Prec<R>::C;
  using Rec = typename Prec<R>::Rec;
  constexpr int kPer = ModesPerThread<MAXPTS>::value;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = faults[blockIdx.x];
  const int err = *fd.err;
  const long long l = *fd.step;
  if (err) return;
  const int N = fd.N, half = fd.nmodes;
  const int ps = pad_shift<R>(N);
  const R* q = load_quarter_table<R, MAXPTS>(buf, fd);
  load_input<R, MAXPTS>(buf, N, (const C*)fd.zbuf, ps);
  __syncthreads();
  fft_lds<C, R, MAXPTS>(buf, N, fd.log2N, q, ps);
  const double dt = fd.dt, c1 = 1.0 - fd.r;
  const double inv_s = 1.0 / fd.fwd_scale;
  constexpr int G = (sizeof(R) == 4 && MAXPTS <= 8192) ? 2 : 1;
#pragma unroll
  for (int s0 = 0; s0 < kPer; s0 += G) {
    double2 V0[G][2], V1[G][2], U[G][2];
    double w1[G][2];
    int Rn[G];
    long long off[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int n = threadIdx.x + (s0 + k) * kSpecThreads;
      if (s0 + k < kPer && n <= half) {
        V0[k][0] = fd.v_hat0[n];
        V0[k][1] = fd.gv_hat0[n];
        V1[k][0] = fd.v_hat1[n];
        V1[k][1] = fd.gv_hat1[n];
        U[k][0] = fd.u_hat[n];
        U[k][1] = fd.g_hat[n];
        w1[k][0] = fd.coef[n].w1T;
        w1[k][1] = fd.coef[n].w1N;
        Rn[k] = fd.Rn[n];
        off[k] = fd.ring_off[n];
      }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int n = threadIdx.x + (s0 + k) * kSpecThreads;
      if (s0 + k < kPer && n <= half) {
        double2 A, B;
        unpack_mode(buf, N, n, inv_s, &A, &B, ps);
        // rate of the interval [t, t + dt] in pass 2: (V_0 + V_1)/2
        const double2 hv = d2(0.5 * (V0[k][0].x + V1[k][0].x), 0.5 * (V0[k][0].y + V1[k][0].y));
        const double2 hg = d2(0.5 * (V0[k][1].x + V1[k][1].x), 0.5 * (V0[k][1].y + V1[k][1].y));
        if (n > 0 && Rn[k] > 0) {
          const long long slot = off[k] + (l % Rn[k]);
          Rec rec;
          if constexpr (sizeof(R) == 4) {
            rec = make_float4((float)hv.x, (float)hv.y, (float)hg.x, (float)hg.y);
          } else {
            rec.v = hv;
            rec.g = hg;
          }
          ((Rec*)fd.ring)[slot] = rec;
        }
        const double2 u = d2(U[k][0].x + dt * hv.x, U[k][0].y + dt * hv.y);
        const double2 g = d2(U[k][1].x + dt * hg.x, U[k][1].y + dt * hg.y);
        fd.hprev_v[n] = hv;
        fd.hprev_g[n] = hg;
        fd.u_hat[n] = u;
        fd.g_hat[n] = g;
        fd.P_T[n] = d2(c1 * u.x + w1[k][0] * hv.x, c1 * u.y + w1[k][0] * hv.y);
        fd.P_N[n] = d2(c1 * g.x + w1[k][1] * hg.x, c1 * g.y + w1[k][1] * hg.y);
        fd.v_hat0[n] = A;
        fd.gv_hat0[n] = B;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *fd.step = l + 1;
}

// P = (1-r) u_hat + w1 hprev for every mode of one fault; the inverse
// packing scale is marked unset (the next pass measures it).
__global__ void k_prepare(const FaultDev* __restrict__ fdp) {
  const FaultDev& fd = *fdp;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) *fd.inv_exp = kInvExpUnset;
  if (n > fd.nmodes) return;
  const double c1 = 1.0 - fd.r;
  const double2 u = fd.u_hat[n], g = fd.g_hat[n], hv = fd.hprev_v[n], hg = fd.hprev_g[n];
  const ModeCoef c = fd.coef[n];
  fd.P_T[n] = d2(c1 * u.x + c.w1T * hv.x, c1 * u.y + c.w1T * hv.y);
  fd.P_N[n] = d2(c1 * g.x + c.w1N * hg.x, c1 * g.y + c.w1N * hg.y);
}

// Forward spectra of count real signal pairs (a, kappa*a or b) -> A, B
// (n = 0..N/2).  Block c handles signal c; inputs are FP64 and are balanced
// by their block maxima before rounding to the transform precision.
template <typename R, int MAXPTS>
__global__ void __launch_bounds__(kSpecThreads)
k_spectra(const FaultDev* __restrict__ fdp, const double* __restrict__ a,
          const double* __restrict__ b, int b_is_kappa_a, double2* __restrict__ A,
          double2* __restrict__ B, long long stride_in, long long stride_out) {
  using C = typename Prec<R>::C;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = *fdp;
  const int N = fd.N;
  const int ps = pad_shift<R>(N);
  const R* q = load_quarter_table<R, MAXPTS>(buf, fd);
  const double* ac = a + stride_in * blockIdx.x;
  const double* bc = b ? b + stride_in * blockIdx.x : nullptr;
  double ma = 0.0, mb = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double av = ac[i];
    const double bv = b_is_kappa_a ? fd.kappa[i] * av : (bc ? bc[i] : 0.0);
    ma = fmax(ma, fabs(av));
    mb = fmax(mb, fabs(bv));
  }
  block_max2(ma, mb);
  const double s = pow2_ratio(ma, mb);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double av = ac[i];
    const double bv = b_is_kappa_a ? fd.kappa[i] * av : (bc ? bc[i] : 0.0);
    buf[lx(i, ps)] = cmk<C>(av, bv * s);
  }
  __syncthreads();
  fft_lds<C, R, MAXPTS>(buf, N, fd.log2N, q, ps);
  double2* Ao = A + stride_out * blockIdx.x;
  double2* Bo = B + stride_out * blockIdx.x;
  for (int n = threadIdx.x; n <= fd.nmodes; n += blockDim.x) {
    double2 x, y;
    unpack_mode(buf, N, n, 1.0 / s, &x, &y, ps);
    Ao[n] = x;
    Bo[n] = y;
  }
}

// Stress path: ring slot p of mode n receives the latest interval
// l <= nint - 2 with l = p (mod R_n) (zero if none); hprev = interval nint-2.
template <typename R>
__global__ void k_fill_ring(const FaultDev* __restrict__ fdp, const double2* __restrict__ RV,
                            const double2* __restrict__ RG, int nint) {
  using Rec = typename Prec<R>::Rec;
  const FaultDev& fd = *fdp;
  const int n = blockIdx.x;  // mode
  const int stride = fd.nmodes + 1;
  const long long last = (long long)nint - 2;
  if (threadIdx.x == 0) {
    fd.hprev_v[n] = last >= 0 ? RV[last * stride + n] : d2(0, 0);
    fd.hprev_g[n] = last >= 0 ? RG[last * stride + n] : d2(0, 0);
  }
  const int Rn = fd.Rn[n];
  if (n == 0 || Rn == 0) return;
  for (int p = threadIdx.x; p < Rn; p += blockDim.x) {
    double2 v = d2(0, 0), g = d2(0, 0);
    if (last >= 0) {
      const long long l = last - posmod(last - p, Rn);
      if (l >= 0) {
        v = RV[l * stride + n];
        g = RG[l * stride + n];
      }
    }
    Rec rec;
    if constexpr (sizeof(R) == 4) {
      rec = make_float4((float)v.x, (float)v.y, (float)g.x, (float)g.y);
    } else {
      rec.v = v;
      rec.g = g;
    }
    ((Rec*)fd.ring)[fd.ring_off[n] + p] = rec;
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
// Momentum balance per element (section 3.3 step (3), with radiation damping)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int solve_rate(double tau, double sig, double theta, double a, double b,
                                          const FaultDev& fd, double Vguess, double* Vout) {
  const double lnVref = fd.ln_V_ref;
  const double psi = fd.f0 + b * log(theta * fd.V_ref / fd.Dc);
  const double x_rs = lnVref + (tau / sig - psi) / a;
  const double x_0 = lnVref - psi / a;
  double hi = x_rs;
  if (tau > 0.0) hi = fmin(hi, fmax(log(tau / fd.eta_rad), x_0));
  hi = fmin(hi, 700.0);
  double lo = x_rs - fd.eta_rad * exp(hi) / (sig * a);
  if (!(lo <= hi)) return -1;
  double x = fmin(fmax(log(Vguess), lo), hi);
  for (int it = 0; it < 100; ++it) {
    const double ex = exp(x);
    const double g = tau - fd.eta_rad * ex - sig * (psi + a * (x - lnVref));
    if (g == 0.0) {
      *Vout = ex;
      return 0;
    }
    const double gp = -fd.eta_rad * ex - sig * a;
    if (g > 0.0) lo = x;
    else hi = x;
    double xn = x - g / gp;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 4e-16 * fmax(1.0, fabs(x))) {
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

template <typename R>
__global__ void __launch_bounds__(kNewtonThreads)
k_newton(const FaultDev* __restrict__ faults, const int2* __restrict__ map, int pass) {
  using C = typename Prec<R>::C;
  const int2 m = map[blockIdx.x];
  const FaultDev& fd = faults[m.x];
  const int i = m.y + threadIdx.x;
  const int ii = min(i, fd.N - 1);
  // every load is issued before the first branch
  const int err = *fd.err;
  const long long l = *fd.step;
  const int cur = (int)(l & 1), nxt = cur ^ 1;
  const double V0 = fd.V[cur][ii], thd0 = fd.thd[cur][ii], th0 = fd.theta[cur][ii];
  const double slip0 = fd.slip[cur][ii];
  const double V1 = fd.V1[ii], thd1 = fd.thd1[ii];
  const double tl = fd.tau_load[ii], sl = fd.sigma_load[ii];
  const double te = fd.tau_el[nxt][ii], se = fd.sigma_el[nxt][ii];
  const double a = fd.a[ii], b = fd.b[ii], kap = fd.kappa[ii];
  if (i >= fd.N || err) return;
  const double dt = fd.dt;
  double Vc, thdc;
  if (pass == 1) {
    Vc = V0;
    thdc = thd0;
  } else {
    Vc = 0.5 * (V0 + V1);
    thdc = 0.5 * (thd0 + thd1);
  }
  double theta_p;
  if (fd.theta_mode == SBIEM_THETA_EXP) {
    const double ss = fd.Dc / Vc;
    theta_p = ss + (th0 - ss) * exp(-Vc * dt / fd.Dc);
  } else {
    theta_p = th0 + dt * thdc;
  }
  const double t_new = fd.t0 + (double)(l + 1) * dt;
  const double tau = tl + fd.tau_rate * t_new + te;
  const double sig = sl + se;
  double Vp = Vc;
  if (!(sig > 0.0)) {
    report(fd, SBIEM_EOPEN, i);
    return;
  }
  if (!(theta_p > 0.0) || !isfinite(theta_p)) {
    report(fd, SBIEM_ESTATE, i);
    return;
  }
  if (solve_rate(tau, sig, theta_p, a, b, fd, Vc, &Vp) != 0 || !isfinite(Vp)) {
    report(fd, SBIEM_ENEWTON, i);
    return;
  }
  const double thdp = 1.0 - theta_p * Vp / fd.Dc;
  if (pass == 1) {
    fd.V1[i] = Vp;
    fd.thd1[i] = thdp;
  } else {
    fd.slip[nxt][i] = slip0 + dt * Vc;
    fd.V[nxt][i] = Vp;
    fd.theta[nxt][i] = theta_p;
    fd.thd[nxt][i] = thdp;
  }
  const double dv = Vp - fd.V_pl;
  ((C*)fd.zbuf)[i] = cmk<C>(dv, fd.fwd_scale * kap * dv);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static size_t spec_lds(int precision, int maxN) {
  if (precision == SBIEM_FP32CONV) return spec_lds_bytes<float>(maxN, pad_shift<float>(maxN));
  return spec_lds_bytes<double>(maxN, pad_shift<double>(maxN));
}

// The spectral kernels are instantiated per largest transform size so that
// each thread's per-mode arrays stay in registers.
template <typename R, int M>
struct SpecTag {
  using type = R;
  static constexpr int pts = M;
};

template <typename F>
static hipError_t with_spec_size(int precision, int maxN, F&& f) {
  if (precision == SBIEM_FP32CONV) {
    if (maxN <= 2048) return f(SpecTag<float, 2048>{});
    if (maxN <= 8192) return f(SpecTag<float, 8192>{});
    return f(SpecTag<float, 16384>{});
  }
  if (maxN <= 2048) return f(SpecTag<double, 2048>{});
  return f(SpecTag<double, 8192>{});
}

template <typename T>
static hipError_t set_spec_attributes(T) {
  using R = typename T::type;
  constexpr int M = T::pts;
  const int bytes = kMaxDynLds;
  const hipFuncAttribute a = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipFuncSetAttribute((const void*)k_pass1<R, M>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_pass2<R, M>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_commit<R, M>, a, bytes);
  if (!e) e = hipFuncSetAttribute((const void*)k_spectra<R, M>, a, bytes);
  return e;
}

hipError_t setup_kernel_attributes(int precision) {
  static bool done[2] = {false, false};
  const int idx = precision == SBIEM_FP32CONV ? 1 : 0;
  if (done[idx]) return hipSuccess;
  hipError_t e = hipSuccess;
  for (int maxN : {2048, 8192, 16384}) {
    if (!e) e = with_spec_size(precision, maxN, [](auto t) { return set_spec_attributes(t); });
  }
  if (!e && idx)
    e = hipFuncSetAttribute((const void*)k_conv32, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kMaxDynLds);
  if (!e) done[idx] = true;
  return e;
}

int conv_grid_size(int precision, int ntasks, int table_len) {
  int need = ntasks;
  if (precision == SBIEM_FP32CONV) {
    // persistent: a few workgroups per CU amortise the LDS table load
    const int per_cu = (int)(kMaxLdsBytes / ((size_t)table_len * sizeof(float4) + 1024));
    const int cap = 256 * (per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu));
    return need < cap ? (need < 1 ? 1 : need) : cap;
  }
  return need < 1 ? 1 : need;
}

hipError_t launch_conv(const Exec& ex, hipStream_t s) {
  if (ex.ntasks == 0) return hipSuccess;
  if (ex.precision == SBIEM_FP32CONV) {
    const size_t lds = (size_t)ex.table_len * sizeof(float4);
    hipLaunchKernelGGL(k_conv32, dim3(ex.conv_grid), dim3(kConvThreads), lds, s, ex.d_faults,
                       ex.d_tiles, ex.d_tasks, ex.ntasks, ex.table, ex.table_len);
  } else {
    hipLaunchKernelGGL(k_conv64, dim3(ex.conv_grid), dim3(kConvThreads), 0, s, ex.d_faults,
                       ex.d_tiles, ex.d_tasks, ex.ntasks);
  }
  return hipGetLastError();
}

hipError_t launch_pass1(const Exec& ex, hipStream_t s) {
  const size_t lds = spec_lds(ex.precision, ex.max_N);
  return with_spec_size(ex.precision, ex.max_N, [&](auto t) {
    using T = decltype(t);
    k_pass1<typename T::type, T::pts><<<dim3(ex.nfaults), dim3(kSpecThreads), lds, s>>>(ex.d_faults);
    return hipGetLastError();
  });
}

hipError_t launch_newton(const Exec& ex, int pass, hipStream_t s) {
  if (ex.precision == SBIEM_FP32CONV)
    hipLaunchKernelGGL(k_newton<float>, dim3(ex.newton_blocks), dim3(kNewtonThreads), 0, s,
                       ex.d_faults, ex.d_newton_map, pass);
  else
    hipLaunchKernelGGL(k_newton<double>, dim3(ex.newton_blocks), dim3(kNewtonThreads), 0, s,
                       ex.d_faults, ex.d_newton_map, pass);
  return hipGetLastError();
}

hipError_t launch_pass2(const Exec& ex, hipStream_t s) {
  const size_t lds = spec_lds(ex.precision, ex.max_N);
  return with_spec_size(ex.precision, ex.max_N, [&](auto t) {
    using T = decltype(t);
    k_pass2<typename T::type, T::pts><<<dim3(ex.nfaults), dim3(kSpecThreads), lds, s>>>(ex.d_faults);
    return hipGetLastError();
  });
}

hipError_t launch_commit(const Exec& ex, hipStream_t s) {
  const size_t lds = spec_lds(ex.precision, ex.max_N);
  return with_spec_size(ex.precision, ex.max_N, [&](auto t) {
    using T = decltype(t);
    k_commit<typename T::type, T::pts><<<dim3(ex.nfaults), dim3(kSpecThreads), lds, s>>>(ex.d_faults);
    return hipGetLastError();
  });
}

hipError_t launch_step(const Exec& ex, hipStream_t s, bool profile, hipEvent_t e0, hipEvent_t e1) {
  hipError_t e;
  if (profile && (e = hipEventRecord(e0, s))) return e;
  if ((e = launch_conv(ex, s))) return e;
  if (profile && (e = hipEventRecord(e1, s))) return e;
  if ((e = launch_pass1(ex, s))) return e;
  if ((e = launch_newton(ex, 1, s))) return e;
  if ((e = launch_pass2(ex, s))) return e;
  if ((e = launch_newton(ex, 2, s))) return e;
  return launch_commit(ex, s);
}

hipError_t launch_spectra(const FaultDev* d_fault, int precision, int max_N, const double* a,
                          const double* b, double scale_b_by_kappa, double2* A, double2* B,
                          int count, long long stride_in, long long stride_out, hipStream_t s) {
  const size_t lds = spec_lds(precision, max_N);
  const int kap = scale_b_by_kappa != 0.0 ? 1 : 0;
  return with_spec_size(precision, max_N, [&](auto t) {
    using T = decltype(t);
    k_spectra<typename T::type, T::pts><<<dim3(count), dim3(kSpecThreads), lds, s>>>(
        d_fault, a, b, kap, A, B, stride_in, stride_out);
    return hipGetLastError();
  });
}

hipError_t launch_prepare(const FaultDev* d_fault, int nmodes, hipStream_t s) {
  const int blocks = (nmodes + 1 + 255) / 256;
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, s, d_fault);
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

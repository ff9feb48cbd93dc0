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

template <typename C, int LR, int MAXPTS>
__device__ __forceinline__ void fft_pass(C* buf, int N, int p, const C* __restrict__ tw) {
  constexpr int RD = 1 << LR;
  constexpr int MAXB = ((MAXPTS >> LR) + kSpecThreads - 1) / kSpecThreads;
  const int nb = N >> LR;
  C x[MAXB][RD];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int i = threadIdx.x + b * kSpecThreads;
    if (i < nb) {
#pragma unroll
      for (int r = 0; r < RD; ++r) x[b][r] = buf[i + r * nb];
    }
  }
  __syncthreads();
  const int tws = N / (p * RD);
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int i = threadIdx.x + b * kSpecThreads;
    if (i < nb) {
      const int k = i & (p - 1);
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < RD; ++r) x[b][r] = cmul(x[b][r], tw[r * k * tws]);
      }
      if (RD == 8) dft8(x[b]);
      else if (RD == 4) dft4(x[b][0], x[b][1], x[b][2], x[b][3]);
      else dft2(x[b]);
      const int base = (i - k) * RD + k;
#pragma unroll
      for (int s = 0; s < RD; ++s) buf[base + s * p] = x[b][s];
    }
  }
  __syncthreads();
}

// Forward FFT of buf[0..N) in LDS; caller has synchronised after filling it.
template <typename C, int MAXPTS>
__device__ void fft_lds(C* buf, int N, int log2N, const C* __restrict__ tw) {
  int p = 1, rem = log2N;
  while (rem >= 3) {
    fft_pass<C, 3, MAXPTS>(buf, N, p, tw);
    p <<= 3;
    rem -= 3;
  }
  if (rem == 2) fft_pass<C, 2, MAXPTS>(buf, N, p, tw);
  else if (rem == 1) fft_pass<C, 1, MAXPTS>(buf, N, p, tw);
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

__global__ void __launch_bounds__(kConvThreads)
k_conv64(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles, int ntiles,
         Rec64* __restrict__ partials) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = kConvThreads / 64;
  for (int t = blockIdx.x * wpb + wave; t < ntiles; t += gridDim.x * wpb) {
    const Tile tl = tiles[t];
    const FaultDev& fd = faults[tl.fault];
    Rec64 acc;
    acc.v = d2(0, 0);
    acc.g = d2(0, 0);
    if (*fd.err == 0) {
      const int Rn = fd.Rn[tl.mode];
      const long long off = fd.ring_off[tl.mode];
      const long long b = *fd.step - 1;
      const int o = (int)posmod(-b, Rn);
      const Rec64* __restrict__ ring = (const Rec64*)fd.ring + off;
      const double2* __restrict__ w = fd.wrev + off;
      const int end = tl.p0 + tl.len;
#pragma unroll 4
      for (int p = tl.p0 + lane; p < end; p += 64) {
        int q = p + o;
        q -= (q >= Rn) ? Rn : 0;
        const Rec64 h = ring[p];
        const double2 wt = w[q];
        acc.v.x = fma(wt.x, h.v.x, acc.v.x);
        acc.v.y = fma(wt.x, h.v.y, acc.v.y);
        acc.g.x = fma(wt.y, h.g.x, acc.g.x);
        acc.g.y = fma(wt.y, h.g.y, acc.g.y);
      }
    }
    acc = wave_reduce_r64(acc);
    if (lane == 0) partials[t] = acc;
  }
}

// FP32 records with weights interpolated from an LDS table of
// dt*(C^T, h dC^T/dT, C^N, h dC^N/dT) at T = i h (cubic Hermite).  The kernel
// argument of lag j is T = c_s |k_n| (j + 1/2) dt = (2j + 1) theta_n; the
// table coordinate (2j + 1) theta_n / h is formed in FP64 so that the phase
// keeps full accuracy at T ~ 200.
__global__ void __launch_bounds__(kConvThreads)
k_conv32(const FaultDev* __restrict__ faults, const Tile* __restrict__ tiles, int ntiles,
         float4* __restrict__ partials, const float4* __restrict__ table, int table_len) {
  extern __shared__ float4 tab[];
  for (int i = threadIdx.x; i < table_len; i += kConvThreads) tab[i] = table[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = kConvThreads / 64;
  for (int t = blockIdx.x * wpb + wave; t < ntiles; t += gridDim.x * wpb) {
    const Tile tl = tiles[t];
    const FaultDev& fd = faults[tl.fault];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (*fd.err == 0) {
      const int Rn = fd.Rn[tl.mode];
      const long long off = fd.ring_off[tl.mode];
      const long long b = *fd.step - 1;
      const int o = (int)posmod(-b, Rn);
      const double th = fd.theta_h[tl.mode];
      const float4* __restrict__ ring = (const float4*)fd.ring + off;
      const int end = tl.p0 + tl.len;
#pragma unroll 4
      for (int p = tl.p0 + lane; p < end; p += 64) {
        int q = p + o;
        q -= (q >= Rn) ? Rn : 0;
        const float4 h = ring[p];
        const int j = Rn - q + 1;                       // lag (q = 0: skipped slot)
        const double u = (double)(2 * j + 1) * th;
        const int i = min((int)u, table_len - 2);
        const float f = (float)(u - (double)i);
        const float4 n0 = tab[i], n1 = tab[i + 1];
        const float f2 = f * f, f3 = f2 * f;
        const float h00 = 2.f * f3 - 3.f * f2 + 1.f;
        const float h10 = f3 - 2.f * f2 + f;
        const float h01 = 3.f * f2 - 2.f * f3;
        const float h11 = f3 - f2;
        float wT = h00 * n0.x + h10 * n0.y + h01 * n1.x + h11 * n1.y;
        float wN = h00 * n0.z + h10 * n0.w + h01 * n1.z + h11 * n1.w;
        wT = (q == 0) ? 0.f : wT;
        wN = (q == 0) ? 0.f : wN;
        acc.x = fmaf(wT, h.x, acc.x);
        acc.y = fmaf(wT, h.y, acc.y);
        acc.z = fmaf(wN, h.z, acc.z);
        acc.w = fmaf(wN, h.w, acc.w);
      }
    }
    acc = wave_reduce4(acc);
    if (lane == 0) partials[t] = acc;
  }
}

// ---------------------------------------------------------------------------
// Spectral kernels (one workgroup per fault, N complex in LDS)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void partial_sum(const float4* partials, int a, int b, double2* T,
                                            double2* Nn) {
  double tx = 0, ty = 0, nx = 0, ny = 0;
  for (int t = a; t < b; ++t) {
    const float4 v = partials[t];
    tx += v.x;
    ty += v.y;
    nx += v.z;
    ny += v.w;
  }
  *T = d2(tx, ty);
  *Nn = d2(nx, ny);
}
__device__ __forceinline__ void partial_sum(const Rec64* partials, int a, int b, double2* T,
                                            double2* Nn) {
  double tx = 0, ty = 0, nx = 0, ny = 0;
  for (int t = a; t < b; ++t) {
    const Rec64 v = partials[t];
    tx += v.v.x;
    ty += v.v.y;
    nx += v.g.x;
    ny += v.g.y;
  }
  *T = d2(tx, ty);
  *Nn = d2(nx, ny);
}

// Block-wide maxima of two non-negative values (all threads get the result).
__device__ __forceinline__ void block_max2(double& a, double& b) {
  __shared__ double red[2][kSpecThreads / 64];
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
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    a = fmax(a, red[0][w]);
    b = fmax(b, red[1][w]);
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

// Load z (a + i b) into LDS with b scaled by the returned power of two.
template <typename C>
__device__ double load_balanced(C* buf, int N, const C* __restrict__ z) {
  double mr = 0.0, mi = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const C v = z[i];
    buf[i] = v;
    mr = fmax(mr, fabs((double)v.x));
    mi = fmax(mi, fabs((double)v.y));
  }
  block_max2(mr, mi);
  const double s = pow2_ratio(mr, mi);
  if (s != 1.0)
    for (int i = threadIdx.x; i < N; i += blockDim.x) buf[i].y = buf[i].y * s;
  __syncthreads();
  return s;
}

// Traction spectra of mode n (section 3.1 with the current interval's rate
// spectra vc, gvc and the last committed interval hprev):
//   tau_hat   = -mu |k| [ (1-r)(u + dt vc) + w0T vc + w1T hprev_v + S_T ]
//   sigma_hat = -i s_n mu [ (1-r)(g + dt gvc) + w0N gvc + w1N hprev_g + S_N ]
// Pass 1 uses vc = v_hat0; pass 2 the average of v_hat0 and v_hat1.
__device__ __forceinline__ void traction_mode(const FaultDev& fd, int n, bool pass2, double2* tau,
                                              double2* sig) {
  const int N = fd.N;
  const double c1 = 1.0 - fd.r;
  const double dt = fd.dt;
  double2 vc = fd.v_hat0[n], gvc = fd.gv_hat0[n];
  if (pass2) {
    const double2 v1 = fd.v_hat1[n], g1 = fd.gv_hat1[n];
    vc = d2(0.5 * (vc.x + v1.x), 0.5 * (vc.y + v1.y));
    gvc = d2(0.5 * (gvc.x + g1.x), 0.5 * (gvc.y + g1.y));
  }
  const double2 u = fd.u_hat[n], g = fd.g_hat[n];
  const double2 hv = fd.hprev_v[n], hg = fd.hprev_g[n];
  const double2 sT = fd.S_T[n], sN = fd.S_N[n];
  const double w0T = fd.w0T[n], w0N = fd.w0N[n], w1T = fd.w1T[n], w1N = fd.w1N[n];
  double2 AT, AN;
  AT.x = c1 * (u.x + dt * vc.x) + w0T * vc.x + w1T * hv.x + sT.x;
  AT.y = c1 * (u.y + dt * vc.y) + w0T * vc.y + w1T * hv.y + sT.y;
  AN.x = c1 * (g.x + dt * gvc.x) + w0N * gvc.x + w1N * hg.x + sN.x;
  AN.y = c1 * (g.y + dt * gvc.y) + w0N * gvc.y + w1N * hg.y + sN.y;
  const double mk = -fd.mu * fd.kabs[n];
  *tau = d2(mk * AT.x, mk * AT.y);
  const double sn = (n == 0 || 2 * n == N) ? 0.0 : fd.mu;
  *sig = d2(sn * AN.y, -sn * AN.x);  // -i s mu AN
}

// Assemble Z = tau_hat + i c sigma_hat (c a balancing power of two), inverse
// transform in LDS and write tau^el, sigma^el.  The inverse is the forward
// transform of conj(Z): y = N conj(z).
template <typename R>
__device__ void assemble_and_invert(const FaultDev& fd, bool pass2, typename Prec<R>::C* buf) {
  using C = typename Prec<R>::C;
  const int N = fd.N, half = fd.nmodes;
  double mt = 0.0, ms = 0.0;
  for (int n = threadIdx.x; n <= half; n += blockDim.x) {
    double2 t, g;
    traction_mode(fd, n, pass2, &t, &g);
    mt = fmax(mt, fmax(fabs(t.x), fabs(t.y)));
    ms = fmax(ms, fmax(fabs(g.x), fabs(g.y)));
  }
  block_max2(mt, ms);
  const double c = pow2_ratio(mt, ms);
  for (int n = threadIdx.x; n <= half; n += blockDim.x) {
    double2 t, g;
    traction_mode(fd, n, pass2, &t, &g);
    g = d2(g.x * c, g.y * c);
    buf[n] = cmk<C>(t.x - g.y, -(t.y + g.x));
    if (n > 0 && 2 * n < N) buf[N - n] = cmk<C>(t.x + g.y, -(-t.y + g.x));
  }
  __syncthreads();
  fft_lds<C, Prec<R>::kMaxPts>(buf, N, fd.log2N, (const C*)fd.twiddle);
  const int slot = (int)((*fd.step + 1) & 1);
  double* __restrict__ tau = fd.tau_el[slot];
  double* __restrict__ sig = fd.sigma_el[slot];
  const double inv = 1.0 / N, invc = 1.0 / (c * N);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const C z = buf[i];
    tau[i] = (double)z.x * inv;
    sig[i] = -(double)z.y * invc;
  }
}

// Unpack the FFT Z of z = a + i s b (a, b real, s the balancing scale) into
// A_n, B_n, n = 0..N/2.
template <typename C>
__device__ __forceinline__ void unpack_mode(const C* buf, int N, int n, double inv_s, double2* A,
                                            double2* B) {
  const C zn = buf[n];
  const C zm = buf[n == 0 ? 0 : N - n];
  // A = (Z_n + conj Z_m)/2, B = (Z_n - conj Z_m)/(2i)
  *A = d2(0.5 * ((double)zn.x + (double)zm.x), 0.5 * ((double)zn.y - (double)zm.y));
  const double dx = (double)zn.x - (double)zm.x, dy = (double)zn.y + (double)zm.y;
  *B = d2(0.5 * dy * inv_s, -0.5 * dx * inv_s);
}

template <typename R>
__global__ void __launch_bounds__(kSpecThreads)
k_pass1(const FaultDev* __restrict__ faults, const typename Prec<R>::Rec* __restrict__ partials) {
  using C = typename Prec<R>::C;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = faults[blockIdx.x];
  if (*fd.err) return;
  const int half = fd.nmodes;
  for (int n = threadIdx.x; n <= half; n += blockDim.x) {
    double2 sT = d2(0, 0), sN = d2(0, 0);
    if (n > 0)
      partial_sum(partials, fd.tile_base + fd.tile_start[n], fd.tile_base + fd.tile_start[n + 1],
                  &sT, &sN);
    fd.S_T[n] = sT;
    fd.S_N[n] = sN;
  }
  // each thread reads back only the modes it wrote
  assemble_and_invert<R>(fd, false, buf);
}

template <typename R>
__global__ void __launch_bounds__(kSpecThreads)
k_pass2(const FaultDev* __restrict__ faults) {
  using C = typename Prec<R>::C;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = faults[blockIdx.x];
  if (*fd.err) return;
  const int N = fd.N, half = fd.nmodes;
  const double s = load_balanced(buf, N, (const C*)fd.zbuf);
  fft_lds<C, Prec<R>::kMaxPts>(buf, N, fd.log2N, (const C*)fd.twiddle);
  for (int n = threadIdx.x; n <= half; n += blockDim.x) {
    double2 A, B;
    unpack_mode(buf, N, n, 1.0 / s, &A, &B);
    fd.v_hat1[n] = A;
    fd.gv_hat1[n] = B;
  }
  __syncthreads();  // all LDS reads done before the assembly overwrites buf
  assemble_and_invert<R>(fd, true, buf);
}

template <typename R>
__global__ void __launch_bounds__(kSpecThreads)
k_commit(const FaultDev* __restrict__ faults) {
  using C = typename Prec<R>::C;
  using Rec = typename Prec<R>::Rec;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = faults[blockIdx.x];
  if (*fd.err) return;
  const int N = fd.N, half = fd.nmodes;
  const long long l = *fd.step;
  const double s = load_balanced(buf, N, (const C*)fd.zbuf);
  fft_lds<C, Prec<R>::kMaxPts>(buf, N, fd.log2N, (const C*)fd.twiddle);
  const double dt = fd.dt;
  for (int n = threadIdx.x; n <= half; n += blockDim.x) {
    double2 A, B;
    unpack_mode(buf, N, n, 1.0 / s, &A, &B);
    const double2 a0 = fd.v_hat0[n], b0 = fd.gv_hat0[n];
    const double2 a1 = fd.v_hat1[n], b1 = fd.gv_hat1[n];
    const double2 hv = d2(0.5 * (a0.x + a1.x), 0.5 * (a0.y + a1.y));
    const double2 hg = d2(0.5 * (b0.x + b1.x), 0.5 * (b0.y + b1.y));
    const int Rn = fd.Rn[n];
    if (n > 0 && Rn > 0) {
      const long long slot = fd.ring_off[n] + (l % Rn);
      Rec rec;
      if constexpr (sizeof(R) == 4) {
        rec = make_float4((float)hv.x, (float)hv.y, (float)hg.x, (float)hg.y);
      } else {
        rec.v = hv;
        rec.g = hg;
      }
      ((Rec*)fd.ring)[slot] = rec;
    }
    fd.hprev_v[n] = hv;
    fd.hprev_g[n] = hg;
    const double2 u = fd.u_hat[n], g = fd.g_hat[n];
    fd.u_hat[n] = d2(u.x + dt * hv.x, u.y + dt * hv.y);
    fd.g_hat[n] = d2(g.x + dt * hg.x, g.y + dt * hg.y);
    fd.v_hat0[n] = A;
    fd.gv_hat0[n] = B;
  }
  __syncthreads();
  if (threadIdx.x == 0) *fd.step = l + 1;
}

// Forward spectra of count real signal pairs (a, kappa*a or b) -> A, B
// (n = 0..N/2).  Block c handles signal c; inputs are FP64 and are balanced
// before rounding to the transform precision.
template <typename R>
__global__ void __launch_bounds__(kSpecThreads)
k_spectra(const FaultDev* __restrict__ fdp, const double* __restrict__ a,
          const double* __restrict__ b, int b_is_kappa_a, double2* __restrict__ A,
          double2* __restrict__ B, long long stride_in, long long stride_out) {
  using C = typename Prec<R>::C;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const FaultDev& fd = *fdp;
  const int N = fd.N;
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
    buf[i] = cmk<C>(av, bv * s);
  }
  __syncthreads();
  fft_lds<C, Prec<R>::kMaxPts>(buf, N, fd.log2N, (const C*)fd.twiddle);
  double2* Ao = A + stride_out * blockIdx.x;
  double2* Bo = B + stride_out * blockIdx.x;
  for (int n = threadIdx.x; n <= fd.nmodes; n += blockDim.x) {
    double2 x, y;
    unpack_mode(buf, N, n, 1.0 / s, &x, &y);
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
  const double lnVref = log(fd.V_ref);
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
  if (i >= fd.N) return;
  if (*fd.err) return;
  const long long l = *fd.step;
  const int cur = (int)(l & 1), nxt = cur ^ 1;
  const double dt = fd.dt;
  const double V0 = fd.V[cur][i], thd0 = fd.thd[cur][i], th0 = fd.theta[cur][i];
  double Vc, thdc;
  if (pass == 1) {
    Vc = V0;
    thdc = thd0;
  } else {
    Vc = 0.5 * (V0 + fd.V1[i]);
    thdc = 0.5 * (thd0 + fd.thd1[i]);
  }
  double theta_p;
  if (fd.theta_mode == SBIEM_THETA_EXP) {
    const double ss = fd.Dc / Vc;
    theta_p = ss + (th0 - ss) * exp(-Vc * dt / fd.Dc);
  } else {
    theta_p = th0 + dt * thdc;
  }
  const double t_new = fd.t0 + (double)(l + 1) * dt;
  const double tau = fd.tau_load[i] + fd.tau_rate * t_new + fd.tau_el[nxt][i];
  const double sig = fd.sigma_load[i] + fd.sigma_el[nxt][i];
  double Vp = Vc;
  if (!(sig > 0.0)) {
    report(fd, SBIEM_EOPEN, i);
    return;
  }
  if (!(theta_p > 0.0) || !isfinite(theta_p)) {
    report(fd, SBIEM_ESTATE, i);
    return;
  }
  if (solve_rate(tau, sig, theta_p, fd.a[i], fd.b[i], fd, Vc, &Vp) != 0 || !isfinite(Vp)) {
    report(fd, SBIEM_ENEWTON, i);
    return;
  }
  const double thdp = 1.0 - theta_p * Vp / fd.Dc;
  if (pass == 1) {
    fd.V1[i] = Vp;
    fd.thd1[i] = thdp;
  } else {
    fd.slip[nxt][i] = fd.slip[cur][i] + dt * Vc;
    fd.V[nxt][i] = Vp;
    fd.theta[nxt][i] = theta_p;
    fd.thd[nxt][i] = thdp;
  }
  const double dv = Vp - fd.V_pl;
  ((C*)fd.zbuf)[i] = cmk<C>(dv, fd.kappa[i] * dv);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static size_t spec_lds(int precision, int maxN) {
  return (size_t)maxN * (precision == SBIEM_FP32CONV ? sizeof(float2) : sizeof(double2));
}

hipError_t setup_kernel_attributes(int precision) {
  static bool done[2] = {false, false};
  const int idx = precision == SBIEM_FP32CONV ? 1 : 0;
  if (done[idx]) return hipSuccess;
  const int bytes = kMaxDynLds;
  hipError_t e = hipSuccess;
  if (idx) {
    e = hipFuncSetAttribute((const void*)k_pass1<float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_pass2<float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_commit<float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_spectra<float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_conv32, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  } else {
    e = hipFuncSetAttribute((const void*)k_pass1<double>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_pass2<double>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_commit<double>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (!e) e = hipFuncSetAttribute((const void*)k_spectra<double>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  }
  if (!e) done[idx] = true;
  return e;
}

int conv_grid_size(int precision, int ntiles, int table_len) {
  const int wpb = kConvThreads / 64;
  int need = (ntiles + wpb - 1) / wpb;
  if (precision == SBIEM_FP32CONV) {
    // persistent: a few workgroups per CU amortise the LDS table load
    const int per_cu = (int)(kMaxLdsBytes / ((size_t)table_len * sizeof(float4) + 1024));
    const int cap = 256 * (per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu));
    return need < cap ? (need < 1 ? 1 : need) : cap;
  }
  return need < 1 ? 1 : need;
}

hipError_t launch_conv(const Exec& ex, hipStream_t s) {
  if (ex.ntiles == 0) return hipSuccess;
  if (ex.precision == SBIEM_FP32CONV) {
    const size_t lds = (size_t)ex.table_len * sizeof(float4);
    hipLaunchKernelGGL(k_conv32, dim3(ex.conv_grid), dim3(kConvThreads), lds, s, ex.d_faults,
                       ex.d_tiles, ex.ntiles, (float4*)ex.d_partials, ex.table, ex.table_len);
  } else {
    hipLaunchKernelGGL(k_conv64, dim3(ex.conv_grid), dim3(kConvThreads), 0, s, ex.d_faults,
                       ex.d_tiles, ex.ntiles, (Rec64*)ex.d_partials);
  }
  return hipGetLastError();
}

hipError_t launch_pass1(const Exec& ex, hipStream_t s) {
  const size_t lds = spec_lds(ex.precision, ex.max_N);
  if (ex.precision == SBIEM_FP32CONV)
    hipLaunchKernelGGL(k_pass1<float>, dim3(ex.nfaults), dim3(kSpecThreads), lds, s, ex.d_faults,
                       (const float4*)ex.d_partials);
  else
    hipLaunchKernelGGL(k_pass1<double>, dim3(ex.nfaults), dim3(kSpecThreads), lds, s, ex.d_faults,
                       (const Rec64*)ex.d_partials);
  return hipGetLastError();
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
  if (ex.precision == SBIEM_FP32CONV)
    hipLaunchKernelGGL(k_pass2<float>, dim3(ex.nfaults), dim3(kSpecThreads), lds, s, ex.d_faults);
  else
    hipLaunchKernelGGL(k_pass2<double>, dim3(ex.nfaults), dim3(kSpecThreads), lds, s, ex.d_faults);
  return hipGetLastError();
}

hipError_t launch_commit(const Exec& ex, hipStream_t s) {
  const size_t lds = spec_lds(ex.precision, ex.max_N);
  if (ex.precision == SBIEM_FP32CONV)
    hipLaunchKernelGGL(k_commit<float>, dim3(ex.nfaults), dim3(kSpecThreads), lds, s, ex.d_faults);
  else
    hipLaunchKernelGGL(k_commit<double>, dim3(ex.nfaults), dim3(kSpecThreads), lds, s, ex.d_faults);
  return hipGetLastError();
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
  if (precision == SBIEM_FP32CONV)
    hipLaunchKernelGGL(k_spectra<float>, dim3(count), dim3(kSpecThreads), lds, s, d_fault, a, b,
                       kap, A, B, stride_in, stride_out);
  else
    hipLaunchKernelGGL(k_spectra<double>, dim3(count), dim3(kSpecThreads), lds, s, d_fault, a, b,
                       kap, A, B, stride_in, stride_out);
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

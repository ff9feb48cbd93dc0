// Learned tail closure: the network that stands in for the discarded far
// tail of each truncated window, its training kernels and its C entry points.
//
// Closed modes keep M'_n = ceil(c M_n) ring lags (M'_n >= 18); the tail
//   tail^X_n = sum_{j = M'_n}^{M_n - 1} w^X_{n,j} H^X_n(lag j)
// is predicted per history kind X by a 33 -> 64 -> 64 -> 2 network (erf
// GELU): input T_cut/100 (T_cut = c_s |k_n| M'_n dt) and the 16 oldest kept
// values H(lag M'_n - 16 + k) divided by their RMS r; output y with
// tail = (y_0 + i y_1) r / (c_s |k_n|).  Inference runs on bfloat16 MFMA
// (16x16x16, float32 accumulation); training runs in float32.
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

namespace sbiem {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kIn = 33, kHid = 64, kOut = 2;
constexpr int kOffW1 = 0, kOffB1 = kIn * kHid, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kOut;
static_assert(kOffB3 + kOut == kClosureParams, "parameter layout");

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}
// GELU for inference, whose outputs are rounded to bfloat16: erf from
// Abramowitz & Stegun, formula 7.1.26 (absolute error below 1.5e-7, far
// under half a bfloat16 unit), with the hardware reciprocal and exp2.
__device__ __forceinline__ float gelu_infer(float z) {
  const float x = z * 0.70710678118654752f;
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
  const float erf_ax = fmaf(-poly, e, 1.f);
  return 0.5f * z * (1.f + copysignf(erf_ax, x));
}

// float -> bfloat16 bits, round to nearest even (the conversion instruction,
// two values per instruction where the compiler pairs them)
__device__ __forceinline__ short bf16_bits(float x) {
  return __builtin_bit_cast(short, (__bf16)x);
}
static unsigned short bf16_bits_host(float x) {
  unsigned u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// ---------------------------------------------------------------------------
// Inference.  One wavefront evaluates the network for 16 inputs (columns
// j = lane % 16).  Layers are chained in transposed form, h^T = W^T x^T, so
// the output fragment of a 16-neuron block (rows 4 (lane/16) + r, column
// lane % 16) is already the B-operand fragment of the next layer's K block.
// Weight fragments (A operands, W^T blocks) are stored per lane in the order
// layer 1: 3 nb + kb (nb < 4, kb < 3), layer 2: 12 + 4 ob + kb, layer 3:
// 28 + kb; biases as float32 (b1, b2, b3).
// ---------------------------------------------------------------------------
struct NetDev {
  const v4s* frag;   // [32][64] fragments
  const float* bias; // [130]: b1[64], b2[64], b3[2]
};

// x: the lane's 12 input values (features 16 kb + 4 (lane/16) + e) as
// bfloat16 B fragments; returns y0, y1 (valid in lanes 0..15).
__device__ __forceinline__ void mlp_wave(const v4s* __restrict__ frag, const float* __restrict__ bias,
                                         const v4s (&x)[3], float* y0, float* y1) {
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4;
  const v4s* __restrict__ fr = frag + lane;
  v4s h1[4], h2[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fr[64 * (3 * nb + kb)], x[kb], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[nb][r] = bf16_bits(gelu_infer(acc[r] + bias[16 * nb + 4 * q + r]));
    __builtin_amdgcn_sched_barrier(0);  // one block's weight fragments live at a time
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fr[64 * (12 + 4 * ob + kb)], h1[kb], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[ob][r] = bf16_bits(gelu_infer(acc[r] + bias[64 + 16 * ob + 4 * q + r]));
    __builtin_amdgcn_sched_barrier(0);
  }
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fr[64 * (28 + kb)], h2[kb], acc, 0, 0, 0);
  *y0 = acc[0] + bias[128];
  *y1 = acc[1] + bias[129];
}

// Standalone evaluation: y = net(x) for n inputs (rows of 33 floats).
__global__ void __launch_bounds__(256) k_mlp_eval(NetDev net, const float* __restrict__ X, long long n,
                                                  float* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const long long m = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + (lane & 15);
  const int q = lane >> 4;
  v4s x[3];
#pragma unroll
  for (int kb = 0; kb < 3; ++kb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int f = 16 * kb + 4 * q + e;
      x[kb][e] = bf16_bits((m < n && f < kIn) ? X[m * kIn + f] : 0.f);
    }
  float y0, y1;
  mlp_wave(net.frag, net.bias, x, &y0, &y1);
  if (q == 0 && m < n) {
    Y[2 * m] = y0;
    Y[2 * m + 1] = y1;
  }
}

// ---------------------------------------------------------------------------
// The closure in the step: tails of every closed mode, for the step the
// history sums are computed for (the committed-step counter plus ahead).
// Ring slot of lag j: p = (b - j + 1) mod R with b = that step - 1.
// ---------------------------------------------------------------------------
// The words of one fault that the closure reads (its step counter and error
// word do not change while the closure runs: they are read once per launch).
struct ClosureFault {
  const float4* ring;
  double4* tails;
  long long b;  // the step the tails are for, minus one
  int err, nmodes;
};

__device__ __forceinline__ ClosureFault closure_fault(const FaultDev& fd, int ahead) {
  ClosureFault w;
  w.ring = (const float4*)fd.ring;
  w.tails = fd.tails;
  w.b = *(const __attribute__((address_space(1))) long long*)fd.step + ahead - 1;
  w.err = *(const __attribute__((address_space(1))) int*)fd.err;
  w.nmodes = fd.nmodes;
  return w;
}

__global__ void __launch_bounds__(kClosureThreads) k_closure(const FaultDev* __restrict__ faults,
                                                             int nfaults,
                                                             const ClosureMode* __restrict__ cm,
                                                             int ncm, NetDev netT, NetDev netN,
                                                             int ahead) {
  // both networks and the words of the first kClosureFaults faults staged in
  // LDS once per workgroup; each wave then loops over groups of 16 closed
  // modes
  __shared__ v4s sfrag[2][32 * 64];
  __shared__ float sbias[2][132];
  __shared__ ClosureFault sfault[kClosureFaults];
  for (int i = threadIdx.x; i < 32 * 64; i += kClosureThreads) {
    sfrag[0][i] = netT.frag[i];
    sfrag[1][i] = netN.frag[i];
  }
  for (int i = threadIdx.x; i < 130; i += kClosureThreads) {
    sbias[0][i] = netT.bias[i];
    sbias[1][i] = netN.bias[i];
  }
  const int nstaged = min(nfaults, kClosureFaults);
  for (int i = threadIdx.x; i < nstaged; i += kClosureThreads) sfault[i] = closure_fault(faults[i], ahead);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, j = lane & 15;
  const int ngroups = (ncm + 15) / 16;
  constexpr int wpb = kClosureThreads / 64;
  for (int grp = blockIdx.x * wpb + (threadIdx.x >> 6); grp < ngroups; grp += gridDim.x * wpb) {
    const int m = grp * 16 + j;
    const bool valid = m < ncm;
    const ClosureMode c = cm[valid ? m : 0];
    const ClosureFault fw = c.fault < nstaged ? sfault[c.fault] : closure_fault(faults[c.fault], ahead);
    const int err = fw.err;
    const long long b = fw.b;
    typedef const __attribute__((address_space(1))) v4f* gring;
    const gring ring = (gring)(fw.ring + c.ring_off);
    // ring slot of lag M'_n - 16 (the first input); lag M'_n - 16 + k sits k
    // slots before it (cyclically)
    const int Rn = c.Rn;
    long long p0l = (b - (c.Mk - 16) + 1) % Rn;
    if (p0l < 0) p0l += Rn;
    const int p0 = (int)p0l;
    // the oldest kept record (k = 15), for the constant extrapolation
    const v4f a = ring[p0 >= 15 ? p0 - 15 : p0 - 15 + Rn];
    // raw inputs of this lane: features f = 16 kb + 4 q + e
    float vT[12], vN[12];
    float sT = 0.f, sN = 0.f;
#pragma unroll
    for (int kb = 0; kb < 3; ++kb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int f = 16 * kb + 4 * q + e;
        float t = 0.f, g = 0.f;
        if (f == 0) {
          t = g = c.tcut;
        } else if (f <= 32) {
          const int k = (f - 1) >> 1;
          const int pk = p0 - k;
          const v4f rec = ring[pk >= 0 ? pk : pk + Rn];
          t = (f & 1) ? rec.x : rec.y;   // f odd: real part, even: imaginary part
          g = (f & 1) ? rec.z : rec.w;
          sT += t * t;
          sN += g * g;
        }
        vT[4 * kb + e] = t;
        vN[4 * kb + e] = g;
      }
    // RMS over the 16 values (the four lanes of column j hold them)
    sT += __shfl_xor(sT, 16);
    sT += __shfl_xor(sT, 32);
    sN += __shfl_xor(sN, 16);
    sN += __shfl_xor(sN, 32);
    const float rT = sqrtf(sT * (1.f / 16.f)), rN = sqrtf(sN * (1.f / 16.f));
    const float iT = rT > 0.f ? 1.f / rT : 0.f, iN = rN > 0.f ? 1.f / rN : 0.f;
    v4s xT[3], xN[3];
#pragma unroll
    for (int kb = 0; kb < 3; ++kb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int f = 16 * kb + 4 * q + e;
        xT[kb][e] = bf16_bits(f == 0 ? vT[4 * kb + e] : vT[4 * kb + e] * iT);
        xN[kb][e] = bf16_bits(f == 0 ? vN[4 * kb + e] : vN[4 * kb + e] * iN);
      }
    float yT0, yT1, yN0, yN1;
    mlp_wave(sfrag[0], sbias[0], xT, &yT0, &yT1);
    __builtin_amdgcn_sched_barrier(0);
    mlp_wave(sfrag[1], sbias[1], xN, &yN0, &yN1);
    if (q == 0 && valid && !err) {
      // tail = D a_15 + y r / (c_s |k_n|), a_15 the oldest kept record (lag M'_n - 1)
      const double sT_ = (double)rT * c.inv_csk, sN_ = (double)rN * c.inv_csk;
      // the Nyquist coefficient of a real signal is real
      const double im = c.pm == fw.nmodes ? 0.0 : 1.0;
      fw.tails[c.pm] = make_double4(c.dT * a.x + yT0 * sT_, im * (c.dT * a.y + yT1 * sT_),
                                    c.dN * a.z + yN0 * sN_, im * (c.dN * a.w + yN1 * sN_));
    }
  }
}

// ---------------------------------------------------------------------------
// Training samples from a plain (full-window) ring: one workgroup per
// closable mode; the exact tail uses the convolution's FP32 weights.
// ---------------------------------------------------------------------------
struct SampleMode {
  int n, pm, M, Mk, Rn, pad;
  long long ring_off;
  double th, cs_k;
  double dT, dN;  // sums of the discarded weights
  float tcut, pad2;
};

__global__ void __launch_bounds__(256) k_closure_sample(const FaultDev* __restrict__ fdp,
                                                        const SampleMode* __restrict__ sm,
                                                        const float4* __restrict__ table, int table_len,
                                                        int half, float* __restrict__ X,
                                                        float* __restrict__ Y, double* __restrict__ R) {
  const FaultDev& fd = *fdp;
  const SampleMode s = sm[blockIdx.x];
  const long long b = *fd.step - 1;
  const float4* __restrict__ ring = (const float4*)fd.ring + s.ring_off;
  __shared__ double red[4][256];
  __shared__ float amp[16][4];
  if (threadIdx.x < 16) {
    const int lag = s.Mk - 16 + threadIdx.x;
    long long p = (b - lag + 1) % s.Rn;
    if (p < 0) p += s.Rn;
    const float4 rec = ring[p];
    amp[threadIdx.x][0] = rec.x;
    amp[threadIdx.x][1] = rec.y;
    amp[threadIdx.x][2] = rec.z;
    amp[threadIdx.x][3] = rec.w;
  }
  // exact tail: lags Mk .. M-1 with the Hermite-table weights
  double tT0 = 0, tT1 = 0, tN0 = 0, tN1 = 0;
  for (int lag = s.Mk + threadIdx.x; lag < s.M; lag += blockDim.x) {
    long long p = (b - lag + 1) % s.Rn;
    if (p < 0) p += s.Rn;
    const float4 rec = ring[p];
    const double x = (double)(2 * lag + 1) * s.th;
    const int i = min((int)x, table_len - 2);
    const float f = (float)(x - (double)i);
    const float4 n0 = table[i], n1 = table[i + 1];
    const float f2 = f * f, f3 = f2 * f;
    const float h00 = 2.f * f3 - 3.f * f2 + 1.f, h10 = f3 - 2.f * f2 + f;
    const float h01 = 3.f * f2 - 2.f * f3, h11 = f3 - f2;
    const float wT = h00 * n0.x + h10 * n0.y + h01 * n1.x + h11 * n1.y;
    const float wN = h00 * n0.z + h10 * n0.w + h01 * n1.z + h11 * n1.w;
    tT0 += (double)wT * rec.x;
    tT1 += (double)wT * rec.y;
    tN0 += (double)wN * rec.z;
    tN1 += (double)wN * rec.w;
  }
  red[0][threadIdx.x] = tT0;
  red[1][threadIdx.x] = tT1;
  red[2][threadIdx.x] = tN0;
  red[3][threadIdx.x] = tN1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 2) {
    const int kind = threadIdx.x;
    double ss = 0;
    for (int k = 0; k < 16; ++k) {
      const double a = amp[k][2 * kind], c = amp[k][2 * kind + 1];
      ss += a * a + c * c;
    }
    const double r = sqrt(ss / 16.0);
    const long long row = (long long)kind * (half + 1) + s.n;
    float* x = X + row * kIn;
    x[0] = s.tcut;
    for (int k = 0; k < 16; ++k) {
      x[1 + 2 * k] = r > 0 ? (float)(amp[k][2 * kind] / r) : 0.f;
      x[2 + 2 * k] = r > 0 ? (float)(amp[k][2 * kind + 1] / r) : 0.f;
    }
    // target: (tail - D a_15) c_s |k_n| / r
    const double D = kind ? s.dN : s.dT;
    const double t0 = red[2 * kind][0] - D * amp[15][2 * kind];
    const double t1 = red[2 * kind + 1][0] - D * amp[15][2 * kind + 1];
    Y[2 * row] = r > 0 ? (float)(t0 * s.cs_k / r) : 0.f;
    Y[2 * row + 1] = r > 0 ? (float)(t1 * s.cs_k / r) : 0.f;
    R[row] = r;
  }
}

// ---------------------------------------------------------------------------
// Training (float32).  A workgroup takes 32 samples of the minibatch, runs
// forward and backward with the parameters staged in LDS, and writes its
// partial gradient (and loss) to its own row; a second launch adds the rows
// in a fixed order and applies Adam, so results do not depend on timing.
// ---------------------------------------------------------------------------
constexpr int kTrainS = 32;

__global__ void __launch_bounds__(256) k_train_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                    const float* __restrict__ Yt, long long n, long long start,
                                                    int batch, float* __restrict__ part,
                                                    float* __restrict__ part_loss) {
  __shared__ float w[kClosureParams];
  __shared__ float x[kTrainS][kIn], t[kTrainS][kOut];
  __shared__ float z1[kTrainS][kHid], z2[kTrainS][kHid], dz1[kTrainS][kHid], dz2[kTrainS][kHid];
  __shared__ float dy[kTrainS][kOut], lossv[kTrainS];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kTrainS;
  const int ns = min(kTrainS, batch - s0);
  for (int i = tid; i < kClosureParams; i += blockDim.x) w[i] = P[i];
  for (int i = tid; i < kTrainS * kIn; i += blockDim.x) {
    const int s = i / kIn, f = i % kIn;
    x[s][f] = s < ns ? X[((start + s0 + s) % n) * kIn + f] : 0.f;
  }
  for (int i = tid; i < kTrainS * kOut; i += blockDim.x) {
    const int s = i / kOut, o = i % kOut;
    t[s][o] = s < ns ? Yt[((start + s0 + s) % n) * kOut + o] : 0.f;
  }
  __syncthreads();
  const float* W1 = w + kOffW1;
  const float* B1 = w + kOffB1;
  const float* W2 = w + kOffW2;
  const float* B2 = w + kOffB2;
  const float* W3 = w + kOffW3;
  const float* B3 = w + kOffB3;
  for (int i = tid; i < kTrainS * kHid; i += blockDim.x) {
    const int s = i / kHid, a = i % kHid;
    float z = B1[a];
    for (int f = 0; f < kIn; ++f) z += x[s][f] * W1[f * kHid + a];
    z1[s][a] = z;
  }
  __syncthreads();
  for (int i = tid; i < kTrainS * kHid; i += blockDim.x) {
    const int s = i / kHid, a = i % kHid;
    float z = B2[a];
    for (int c = 0; c < kHid; ++c) z += gelu_f(z1[s][c]) * W2[c * kHid + a];
    z2[s][a] = z;
  }
  __syncthreads();
  if (tid < kTrainS) {
    const int s = tid;
    float l = 0.f;
    for (int o = 0; o < kOut; ++o) {
      float y = B3[o];
      for (int c = 0; c < kHid; ++c) y += gelu_f(z2[s][c]) * W3[c * kOut + o];
      const float d = s < ns ? y - t[s][o] : 0.f;
      dy[s][o] = 2.f * d / (float)batch;
      l += d * d;
    }
    lossv[s] = l;
  }
  __syncthreads();
  for (int i = tid; i < kTrainS * kHid; i += blockDim.x) {
    const int s = i / kHid, a = i % kHid;
    float d = 0.f;
    for (int o = 0; o < kOut; ++o) d += dy[s][o] * W3[a * kOut + o];
    dz2[s][a] = d * gelu_grad_f(z2[s][a]);
  }
  __syncthreads();
  for (int i = tid; i < kTrainS * kHid; i += blockDim.x) {
    const int s = i / kHid, a = i % kHid;
    float d = 0.f;
    for (int c = 0; c < kHid; ++c) d += dz2[s][c] * W2[a * kHid + c];
    dz1[s][a] = d * gelu_grad_f(z1[s][a]);
  }
  __syncthreads();
  float* g = part + (size_t)blockIdx.x * kClosureParams;
  for (int i = tid; i < kClosureParams; i += blockDim.x) {
    float acc = 0.f;
    if (i < kOffB1) {                       // W1[f][a]
      const int f = i / kHid, a = i % kHid;
      for (int s = 0; s < kTrainS; ++s) acc += x[s][f] * dz1[s][a];
    } else if (i < kOffW2) {                // b1[a]
      const int a = i - kOffB1;
      for (int s = 0; s < kTrainS; ++s) acc += dz1[s][a];
    } else if (i < kOffB2) {                // W2[c][a]
      const int c = (i - kOffW2) / kHid, a = (i - kOffW2) % kHid;
      for (int s = 0; s < kTrainS; ++s) acc += gelu_f(z1[s][c]) * dz2[s][a];
    } else if (i < kOffW3) {                // b2[a]
      const int a = i - kOffB2;
      for (int s = 0; s < kTrainS; ++s) acc += dz2[s][a];
    } else if (i < kOffB3) {                // W3[c][o]
      const int c = (i - kOffW3) / kOut, o = (i - kOffW3) % kOut;
      for (int s = 0; s < kTrainS; ++s) acc += gelu_f(z2[s][c]) * dy[s][o];
    } else {                                // b3[o]
      const int o = i - kOffB3;
      for (int s = 0; s < kTrainS; ++s) acc += dy[s][o];
    }
    g[i] = acc;
  }
  if (tid == 0) {
    float l = 0.f;
    for (int s = 0; s < kTrainS; ++s) l += lossv[s];
    part_loss[blockIdx.x] = l;
  }
}

__global__ void __launch_bounds__(256) k_train_adam(float* __restrict__ P, float* __restrict__ Mo,
                                                    float* __restrict__ Vo, const float* __restrict__ part,
                                                    const float* __restrict__ part_loss, int nparts,
                                                    int batch, float lr, float bc1, float bc2,
                                                    double* __restrict__ loss_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    double l = 0.0;
    for (int k = 0; k < nparts; ++k) l += part_loss[k];
    *loss_out = l / batch;
  }
  if (i >= kClosureParams) return;
  float g = 0.f;
  for (int k = 0; k < nparts; ++k) g += part[(size_t)k * kClosureParams + i];
  const float m = 0.9f * Mo[i] + 0.1f * g;
  const float v = 0.999f * Vo[i] + 0.001f * g * g;
  Mo[i] = m;
  Vo[i] = v;
  P[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Fragment-ordered bfloat16 weights and float32 biases of one network.
void closure_pack(const float* p, std::vector<unsigned short>* frag, std::vector<float>* bias) {
  frag->assign(32 * 64 * 4, 0);
  bias->assign(130, 0.f);
  auto put = [&](int fi, int lane, int e, float v) { (*frag)[((size_t)fi * 64 + lane) * 4 + e] = bf16_bits_host(v); };
  for (int lane = 0; lane < 64; ++lane)
    for (int e = 0; e < 4; ++e) {
      const int i = lane % 16, k = 4 * (lane / 16) + e;
      for (int nb = 0; nb < 4; ++nb)
        for (int kb = 0; kb < 3; ++kb) {
          const int f = 16 * kb + k, a = 16 * nb + i;
          put(3 * nb + kb, lane, e, f < kIn ? p[kOffW1 + f * kHid + a] : 0.f);
        }
      for (int ob = 0; ob < 4; ++ob)
        for (int kb = 0; kb < 4; ++kb) {
          const int c = 16 * kb + k, a = 16 * ob + i;
          put(12 + 4 * ob + kb, lane, e, p[kOffW2 + c * kHid + a]);
        }
      for (int kb = 0; kb < 4; ++kb) {
        const int c = 16 * kb + k;
        put(28 + kb, lane, e, i < kOut ? p[kOffW3 + c * kOut + i] : 0.f);
      }
    }
  for (int a = 0; a < kHid; ++a) {
    (*bias)[a] = p[kOffB1 + a];
    (*bias)[64 + a] = p[kOffB2 + a];
  }
  (*bias)[128] = p[kOffB3];
  (*bias)[129] = p[kOffB3 + 1];
}

hipError_t launch_closure(const Exec& ex, int ahead, hipStream_t s) {
  if (!ex.closure_modes || ex.nclosure == 0) return hipSuccess;
  NetDev T{(const v4s*)ex.net_frag[0], ex.net_bias[0]};
  NetDev N{(const v4s*)ex.net_frag[1], ex.net_bias[1]};
  constexpr int wpb = kClosureThreads / 64;
  const int groups = (ex.nclosure + 15) / 16;  // one wave per 16 modes and pass
  // persistent: the workgroups resident at once (three per CU: LDS and registers)
  const int blocks = std::min((groups + wpb - 1) / wpb, 3 * 256);
  hipLaunchKernelGGL(k_closure, dim3(blocks), dim3(kClosureThreads), 0, s, ex.d_faults,
                     ex.nfaults, ex.closure_modes, ex.nclosure, T, N, ahead);
  return hipGetLastError();
}

}  // namespace sbiem

using namespace sbiem;

namespace {
int dev_err(hipError_t e, const char* what) {
  return fail_global(e == hipErrorOutOfMemory ? SBIEM_ENOMEM : SBIEM_EDEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

// Workspace of sbiem_closure_train_noalloc: the per-block gradient rows and
// losses of k_train_grad for a minibatch of at most
// SBIEM_CLOSURE_TRAIN_MAX_BATCH samples, and one double that takes the loss
// when the caller keeps none.  A file-scope device array: each GPU the
// library runs on holds its own copy until the process ends.  Host code
// never uses the array's name as an address: the device address of this
// GPU's copy comes from hipGetSymbolAddress, taken once per device with that
// device current and kept in scratch_dev.  Every launch writes the rows it
// reads next, so nothing needs clearing between calls.
constexpr int kNoAllocParts = SBIEM_CLOSURE_TRAIN_MAX_BATCH / kTrainS;
static_assert(kNoAllocParts * kTrainS == SBIEM_CLOSURE_TRAIN_MAX_BATCH, "whole blocks");
constexpr size_t kScratchLossOff = 0;         // double
constexpr size_t kScratchRowLossOff = 256;    // float[kNoAllocParts]
constexpr size_t kScratchRowsOff = 256 + ((sizeof(float) * kNoAllocParts + 255) / 256) * 256;
constexpr size_t kScratchBytes = kScratchRowsOff + sizeof(float) * (size_t)kNoAllocParts * kClosureParams;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* scratch_dev[kMaxDevices] = {};

// Device address of the current device's workspace (taken on first use).
hipError_t scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e) return e;
    scratch_dev[dev] = (unsigned char*)ptr;
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

int sbiem_closure_eval(const float* params, const float* X, int64_t n, float* Y) {
  if (!params || (n > 0 && (!X || !Y)) || n < 0) return fail_global(SBIEM_EINVAL, "closure_eval: bad arguments");
  if (n == 0) return SBIEM_OK;
  std::vector<unsigned short> frag;
  std::vector<float> bias;
  closure_pack(params, &frag, &bias);
  DevArena mem;
  void* dfrag = mem.get(frag.size() * 2);
  float* dbias = (float*)mem.get(bias.size() * 4);
  float* dX = (float*)mem.get((size_t)n * kIn * 4);
  float* dY = (float*)mem.get((size_t)n * kOut * 4);
  if (!dfrag || !dbias || !dX || !dY) return fail_global(SBIEM_ENOMEM, "closure_eval: device allocation failed");
  hipError_t e = hipMemcpy(dfrag, frag.data(), frag.size() * 2, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dbias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dX, X, (size_t)n * kIn * 4, hipMemcpyHostToDevice);
  if (!e) {
    NetDev net{(const v4s*)dfrag, dbias};
    hipLaunchKernelGGL(k_mlp_eval, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, 0, net, dX, (long long)n, dY);
    e = hipGetLastError();
  }
  if (!e) e = hipMemcpy(Y, dY, (size_t)n * kOut * 4, hipMemcpyDeviceToHost);
  if (e) return dev_err(e, "closure_eval");
  return SBIEM_OK;
}

int sbiem_closure_train(const float* X, const float* Y, int64_t n, int64_t batch, int64_t steps,
                        double lr, float* params, float* adam_m, float* adam_v, int64_t* adam_t,
                        double* losses) {
  if (!X || !Y || !params || !adam_m || !adam_v || !adam_t || n <= 0 || batch <= 0 || steps < 0 ||
      !(lr > 0) || batch > (int64_t)1 << 20)
    return fail_global(SBIEM_EINVAL, "closure_train: bad arguments");
  if (steps == 0) return SBIEM_OK;
  const int nparts = (int)((batch + kTrainS - 1) / kTrainS);
  DevArena mem;
  float* dX = (float*)mem.get((size_t)n * kIn * 4);
  float* dY = (float*)mem.get((size_t)n * kOut * 4);
  float* dP = (float*)mem.get(kClosureParams * 4);
  float* dM = (float*)mem.get(kClosureParams * 4);
  float* dV = (float*)mem.get(kClosureParams * 4);
  float* dpart = (float*)mem.get((size_t)nparts * kClosureParams * 4);
  float* dpl = (float*)mem.get((size_t)nparts * 4);
  double* dloss = (double*)mem.get((size_t)steps * 8);
  if (!dX || !dY || !dP || !dM || !dV || !dpart || !dpl || !dloss)
    return fail_global(SBIEM_ENOMEM, "closure_train: device allocation failed");
  hipError_t e = hipMemcpy(dX, X, (size_t)n * kIn * 4, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dY, Y, (size_t)n * kOut * 4, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dP, params, kClosureParams * 4, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dM, adam_m, kClosureParams * 4, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dV, adam_v, kClosureParams * 4, hipMemcpyHostToDevice);
  int64_t t = *adam_t;
  for (int64_t k = 0; k < steps && !e; ++k) {
    const long long start = (long long)((t * batch) % n);
    hipLaunchKernelGGL(k_train_grad, dim3(nparts), dim3(256), 0, 0, dP, dX, dY, (long long)n, start,
                       (int)batch, dpart, dpl);
    ++t;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(k_train_adam, dim3((kClosureParams + 255) / 256), dim3(256), 0, 0, dP, dM, dV,
                       dpart, dpl, nparts, (int)batch, (float)lr, bc1, bc2, dloss + k);
    e = hipGetLastError();
  }
  if (!e) e = hipMemcpy(params, dP, kClosureParams * 4, hipMemcpyDeviceToHost);
  if (!e) e = hipMemcpy(adam_m, dM, kClosureParams * 4, hipMemcpyDeviceToHost);
  if (!e) e = hipMemcpy(adam_v, dV, kClosureParams * 4, hipMemcpyDeviceToHost);
  if (!e && losses) e = hipMemcpy(losses, dloss, (size_t)steps * 8, hipMemcpyDeviceToHost);
  if (e) return dev_err(e, "closure_train");
  *adam_t = t;
  return SBIEM_OK;
}

int sbiem_closure_sample(sbiem_plan* p, double cut, float* X, float* Y, double* R) {
  if (!p) return fail_global(SBIEM_EINVAL, "NULL plan");
  if (!X || !Y || !R || !(cut > 0.0 && cut < 1.0)) return fail(p, SBIEM_EINVAL, "closure_sample: bad arguments");
  if (p->precision != SBIEM_FP32CONV || p->closure_on)
    return fail(p, SBIEM_EINVAL, "closure_sample: needs a plain SBIEM_FP32CONV plan");
  if (!p->dtd || !p->state_set) return fail(p, SBIEM_ENOTREADY, "closure_sample: set the state and dt first");
  const int half = (int)(p->N / 2);
  const DtData* d = p->dtd;
  std::vector<SampleMode> list;
  std::vector<int> ln, lMk, lM;
  for (int n = 1; n <= half; ++n) {
    const int Mk = closure_kept(d->M[n], cut);
    if (Mk == d->M[n] || d->Rn[n] + 1 != d->M[n]) continue;
    ln.push_back(n);
    lMk.push_back(Mk);
    lM.push_back(d->M[n]);
  }
  std::vector<double> DT, DN;
  discarded_weights(p->cs, p->cp, p->L, d->dt, ln, lMk, lM, &DT, &DN);
  for (size_t i = 0; i < ln.size(); ++i) {
    const int n = ln[i], Mk = lMk[i];
    SampleMode m;
    std::memset(&m, 0, sizeof(m));
    m.n = n;
    m.pm = mode_pos(n, p->log2P, p->log2Q);
    m.M = d->M[n];
    m.Mk = Mk;
    m.Rn = d->Rn[n];
    m.ring_off = d->ring_off[n];
    m.th = d->th_mode[n];
    m.cs_k = p->cs * 2.0 * M_PI * (double)n / p->L;
    m.tcut = (float)(m.cs_k * Mk * d->dt / 100.0);
    m.dT = DT[i];
    m.dN = DN[i];
    list.push_back(m);
  }
  const size_t rows = 2 * (size_t)(half + 1);
  std::memset(X, 0, rows * kIn * sizeof(float));
  std::memset(Y, 0, rows * kOut * sizeof(float));
  std::memset(R, 0, rows * sizeof(double));
  if (list.empty()) return SBIEM_OK;
  hipError_t e = hipSetDevice(p->device);
  DevArena mem;
  SampleMode* dl = (SampleMode*)mem.get(list.size() * sizeof(SampleMode));
  float* dX = (float*)mem.get(rows * kIn * sizeof(float));
  float* dY = (float*)mem.get(rows * kOut * sizeof(float));
  double* dR = (double*)mem.get(rows * sizeof(double));
  if (!dl || !dX || !dY || !dR) return fail(p, SBIEM_ENOMEM, "closure_sample: device allocation failed");
  hipStream_t s = p->stream;
  if (!e) e = hipMemcpyAsync(dl, list.data(), list.size() * sizeof(SampleMode), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(dX, X, rows * kIn * sizeof(float), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(dY, Y, rows * kOut * sizeof(float), hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(dR, R, rows * sizeof(double), hipMemcpyHostToDevice, s);
  if (!e) {
    hipLaunchKernelGGL(k_closure_sample, dim3((unsigned)list.size()), dim3(256), 0, s, p->d_desc, dl,
                       d->table, d->table_len, half, dX, dY, dR);
    e = hipGetLastError();
  }
  if (!e) e = hipMemcpyAsync(X, dX, rows * kIn * sizeof(float), hipMemcpyDeviceToHost, s);
  if (!e) e = hipMemcpyAsync(Y, dY, rows * kOut * sizeof(float), hipMemcpyDeviceToHost, s);
  if (!e) e = hipMemcpyAsync(R, dR, rows * sizeof(double), hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(p, e, "closure_sample");
  return SBIEM_OK;
}

int sbiem_closure_train_noalloc(const float* X, const float* Y, int64_t n, int64_t batch,
                                int64_t steps, double lr, float* params, float* adam_m,
                                float* adam_v, int64_t* adam_t, double* losses, void* hip_stream) {
  if (!X || !Y || !params || !adam_m || !adam_v || !adam_t || n <= 0 || batch <= 0 ||
      steps < 0 || !(lr > 0))
    return fail_global(SBIEM_EINVAL, "closure_train_noalloc: bad arguments");
  if (batch > SBIEM_CLOSURE_TRAIN_MAX_BATCH)
    return fail_global(SBIEM_EINVAL, "closure_train_noalloc: batch " + std::to_string(batch) +
                                         " exceeds the workspace limit of " +
                                         std::to_string(SBIEM_CLOSURE_TRAIN_MAX_BATCH) + " samples");
  if (steps == 0) return SBIEM_OK;
  unsigned char* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e) return dev_err(e, "closure_train_noalloc: workspace address");
  float* rows = (float*)(base + kScratchRowsOff);
  float* row_loss = (float*)(base + kScratchRowLossOff);
  double* sink = (double*)(base + kScratchLossOff);
  hipStream_t s = (hipStream_t)hip_stream;
  const int nparts = (int)((batch + kTrainS - 1) / kTrainS);
  int64_t t = *adam_t;
  for (int64_t k = 0; k < steps && !e; ++k) {
    const long long start = (long long)((t * batch) % n);
    hipLaunchKernelGGL(k_train_grad, dim3(nparts), dim3(256), 0, s, params, X, Y, (long long)n,
                       start, (int)batch, rows, row_loss);
    ++t;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(k_train_adam, dim3((kClosureParams + 255) / 256), dim3(256), 0, s, params,
                       adam_m, adam_v, rows, row_loss, nparts, (int)batch, (float)lr, bc1, bc2,
                       losses ? losses + k : sink);
    e = hipGetLastError();
  }
  if (e) return dev_err(e, "closure_train_noalloc");
  *adam_t = t;
  return SBIEM_OK;
}

}  // extern "C"

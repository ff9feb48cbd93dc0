// Host evaluation of the mode-II kernels in 80-bit extended precision.
//
// The closed forms (section 2.3, eq. Ct; section 2.4) combine terms of size
// ~T^(1/2) into results of size ~T^(-1/2), so W(x) must be accurate to a
// small absolute error at arguments up to ~350.  Neither form of W printed in
// the paper (via Struve functions, or as the tail integral of J1(t)/t) is
// usable as is in finite precision, so:
//   * x < 50: Miller's backward recurrence gives J_0, J_1, ... to full
//     precision, and W(x) = 1 - J1(x) - 2 (J3 + J5 + ...), which follows from
//     the integral of J1(t)/t over [0, x] = J1 + 2 sum_{k>=1} J_{2k+1}
//     (termwise integration of J1(t)/t = (J0 + J2)/2 with
//     int_0^x J_nu = 2 sum_k J_{nu+2k+1});
//   * x >= 50: Hankel's asymptotic expansions for J0, J1 and
//     W = J0 A(x) + J1 B(x) with A = x((pi/2)K1 - 1), B = 1 - x (pi/2) K0,
//     K_nu = H_nu - Y_nu (Struve minus Neumann), whose asymptotic series
//     A ~ 1/x - 3/x^3 + 45/x^5 - ..., B ~ 1/x^2 - 9/x^4 + 225/x^6 - ...
//     are summed to their smallest term (error ~ e^(-x)).
// The derivatives used by the interpolated FP32 weights follow from
// W'(x) = -J1/x, J0' = -J1, J1' = J0 - J1/x:
//   dC^T/dT = 2T (W(eta T) - W(T)) + J1(T)/(2T) - (2/eta) J0(eta T) + 1.5 J0(T)
//   dC^N/dT = 2T (W(T) - W(eta T)) + (2 - (q-2)^2/2)/eta J0(eta T)
//             + (q/2 - 2) J0(T)

#include "internal.h"

#include <cmath>
#include <limits>

namespace sbiem {

namespace {

typedef long double ld;

const ld kPi = 3.141592653589793238462643383279502884L;

void miller(ld x, ld* J0, ld* J1, ld* W) {
  if (x == 0.0L) {
    *J0 = 1.0L;
    *J1 = 0.0L;
    *W = 1.0L;
    return;
  }
  int n0 = (int)(x + 60.0L + 12.0L * cbrtl(x));
  n0 += n0 & 1;  // even start order
  ld jp1 = 0.0L, j = 1e-300L;  // J_{n0+1}, J_{n0} (unnormalised)
  ld norm = 0.0L;              // J0 + 2 sum J_{2k}
  ld odd = 0.0L;               // sum_{k>=1} J_{2k+1}
  ld j0 = 0.0L, j1 = 0.0L;
  for (int n = n0; n >= 1; --n) {
    // here j = J_n, jp1 = J_{n+1}
    if ((n & 1) == 0) norm += 2.0L * j;
    else if (n >= 3) odd += j;
    if (n == 1) j1 = j;
    ld jm1 = (2.0L * n / x) * j - jp1;
    jp1 = j;
    j = jm1;
    if (fabsl(j) > 1e300L) {  // rescale to avoid overflow
      j *= 1e-300L;
      jp1 *= 1e-300L;
      norm *= 1e-300L;
      odd *= 1e-300L;
      j1 *= 1e-300L;
    }
  }
  j0 = j;
  norm += j0;
  *J0 = j0 / norm;
  *J1 = j1 / norm;
  *W = 1.0L - *J1 - 2.0L * odd / norm;
}

void hankel(ld x, ld* J0, ld* J1, ld* W) {
  // P_nu, Q_nu for nu = 0, 1: a_k(nu) = prod_{i=1..k} (4nu^2 - (2i-1)^2) / (k! 8^k)
  ld P[2], Q[2];
  for (int nu = 0; nu < 2; ++nu) {
    ld mu4 = 4.0L * nu * nu;
    ld a = 1.0L, p = 1.0L, q = 0.0L, prev = HUGE_VALL;
    for (int k = 1; k < 200; ++k) {
      a *= (mu4 - (ld)(2 * k - 1) * (2 * k - 1)) / (8.0L * k * x);
      ld t = fabsl(a);
      if (t > prev) break;
      prev = t;
      // term k contributes (-1)^{k/2} a to P (k even) or (-1)^{(k-1)/2} a to Q (k odd)
      if (k & 1) q += ((k / 2) & 1) ? -a : a;
      else p += ((k / 2) & 1) ? -a : a;
      if (t < 1e-24L * fabsl(p)) break;
    }
    P[nu] = p;
    Q[nu] = q;
  }
  ld s = sinl(x), c = cosl(x);
  const ld r2 = 0.70710678118654752440084436210484903928L;
  // chi_0 = x - pi/4, chi_1 = x - 3pi/4
  ld c0 = (c + s) * r2, s0 = (s - c) * r2;
  ld c1 = (s - c) * r2, s1 = -(s + c) * r2;
  ld amp = sqrtl(2.0L / (kPi * x));
  *J0 = amp * (P[0] * c0 - Q[0] * s0);
  *J1 = amp * (P[1] * c1 - Q[1] * s1);
  // A = sum_{k>=1} h_k x^{1-2k}, h_1 = 1, h_{k+1} = h_k (2k+1)(1-2k)
  ld A = 0.0L, h = 1.0L, prevA = HUGE_VALL;
  ld x2 = x * x, xp = 1.0L / x;
  for (int k = 1; k < 200; ++k) {
    ld t = h * xp;
    if (fabsl(t) > prevA) break;
    prevA = fabsl(t);
    A += t;
    if (fabsl(t) < 1e-24L * fabsl(A)) break;
    h *= (ld)(2 * k + 1) * (ld)(1 - 2 * k);
    xp /= x2;
  }
  // B = sum_{k>=1} (-1)^{k+1} g_k x^{-2k}, g_1 = 1, g_{k+1} = g_k (2k+1)^2
  ld B = 0.0L, g = 1.0L, prevB = HUGE_VALL;
  xp = 1.0L / x2;
  for (int k = 1; k < 200; ++k) {
    ld t = g * xp;
    if (t > prevB) break;
    prevB = t;
    B += (k & 1) ? t : -t;
    if (t < 1e-24L * fabsl(B)) break;
    g *= (ld)(2 * k + 1) * (ld)(2 * k + 1);
    xp /= x2;
  }
  *W = *J0 * A + *J1 * B;
}

}  // namespace

void bessel_jw(long double x, long double* J0, long double* J1, long double* W) {
  if (x < 50.0L) miller(x, J0, J1, W);
  else hankel(x, J0, J1, W);
}

void kernel_values(long double T, long double cs, long double cp, long double* CT,
                   long double* CN, long double* dCT, long double* dCN) {
  const ld r = (cs / cp) * (cs / cp);
  const ld q = 1.0L / r;
  const ld eta = cp / cs;
  ld J0a, J1a, Wa, J0b, J1b, Wb;
  bessel_jw(eta * T, &J0a, &J1a, &Wa);
  bessel_jw(T, &J0b, &J1b, &Wb);
  const ld T2 = T * T;
  const ld qm2 = (q - 2.0L) * (q - 2.0L);
  if (CT)
    *CT = (T2 + r) * Wa - (T2 + 1.0L) * Wb - r * J1a + 0.5L * J1b - (T / eta) * J0a + T * J0b;
  if (CN)
    *CN = (qm2 * r / 2.0L - r - T2) * Wa + (1.0L + T2 - q / 2.0L) * Wb +
          (r - qm2 * r / 2.0L) * J1a + (q / 2.0L - 1.0L) * J1b + (T / eta) * J0a - T * J0b;
  if (dCT) {
    ld j1_over = (T > 0.0L) ? J1b / (2.0L * T) : 0.25L;
    *dCT = 2.0L * T * (Wa - Wb) + j1_over - (2.0L / eta) * J0a + 1.5L * J0b;
  }
  if (dCN)
    *dCN = 2.0L * T * (Wb - Wa) + (2.0L - qm2 / 2.0L) / eta * J0a + (q / 2.0L - 2.0L) * J0b;
}

// Primitives P^X(T) = integral of C^X over [0, T] (the interval weights of
// the exact-integral rule and of variable steps), from the elementary
// primitives of each term of C^T and C^N (W'(x) = -J1(x)/x, (x^2 J2)' = x^2 J1, (x J1)' = x J0):
//   P^T = T^3 [W(eta T) - W(T)]/3 + T^2 [J2(eta T)/eta - J2(T)]/3
//         + r T W(eta T) - T W(T) - (1 - J0(T))/2 - r T J1(eta T) + T J1(T)
//   P^N = A T W(eta T) + B T W(T) - T^3 [W(eta T) - W(T)]/3
//         - T^2 [J2(eta T)/eta - J2(T)]/3 + r T J1(eta T) - T J1(T)
// with A = (q-2)^2 r/2 - r and B = 1 - q/2; J2 = 2 J1/x - J0.
void kernel_primitives(long double T, long double cs, long double cp, long double* PT,
                       long double* PN) {
  const ld r = (cs / cp) * (cs / cp);
  const ld q = 1.0L / r;
  const ld eta = cp / cs;
  if (T <= 0.0L) {
    *PT = 0.0L;
    *PN = 0.0L;
    return;
  }
  ld J0a, J1a, Wa, J0b, J1b, Wb;
  bessel_jw(eta * T, &J0a, &J1a, &Wa);
  bessel_jw(T, &J0b, &J1b, &Wb);
  const ld a = eta * T;
  // J2 by the recurrence, or its series where that cancels
  auto j2 = [](ld x, ld j0, ld j1) {
    if (x < 1e-3L) {
      const ld x2 = x * x;
      return x2 / 8.0L * (1.0L - x2 / 12.0L + x2 * x2 / 384.0L);
    }
    return 2.0L * j1 / x - j0;
  };
  const ld J2a = j2(a, J0a, J1a), J2b = j2(T, J0b, J1b);
  const ld T2 = T * T;
  const ld cubic = T2 * T * (Wa - Wb) / 3.0L + T2 * (J2a / eta - J2b) / 3.0L;
  // 1 - J0(T) without cancellation at small T
  const ld one_m_j0 = T < 1e-3L ? T2 / 4.0L * (1.0L - T2 / 16.0L) : 1.0L - J0b;
  *PT = cubic + r * T * Wa - T * Wb - 0.5L * one_m_j0 - r * T * J1a + T * J1b;
  const ld A = (q - 2.0L) * (q - 2.0L) * r / 2.0L - r;
  const ld B = 1.0L - q / 2.0L;
  *PN = A * T * Wa + B * T * Wb - cubic + r * T * J1a - T * J1b;
}

}  // namespace sbiem

// Slip/curvature scaling diagnostic of section 5: the scaled slip gradient
// (1/(f du)) d(du)/dx by second-order centred differences on the periodic
// element grid (x_i = i L/N; along-fault distance equals x to first order in
// the slope).  Elements with |du| <= slip_floor give NaN.
int sbiem_slip_scaling(int64_t N, double L, double f, const double* slip, double slip_floor,
                       double* ratio) {
  if (N < 3 || !(L > 0) || !std::isfinite(L) || !(f != 0) || !std::isfinite(f) || !slip ||
      !ratio || !(slip_floor >= 0))
    return sbiem::fail_global(SBIEM_EINVAL,
                              "slip_scaling: need N >= 3, L > 0, finite f != 0, slip_floor >= 0");
  const double inv2dx = (double)N / (2.0 * L);
  for (int64_t i = 0; i < N; ++i) {
    const double u = slip[i];
    const double up = slip[i + 1 < N ? i + 1 : 0], um = slip[i > 0 ? i - 1 : N - 1];
    ratio[i] = std::fabs(u) > slip_floor ? (up - um) * inv2dx / (f * u)
                                         : std::numeric_limits<double>::quiet_NaN();
  }
  return SBIEM_OK;
}

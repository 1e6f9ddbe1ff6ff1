// Cross-section post-processing (paper Section III): the microscopic-reversibility
// diagnostic of Eq. 19, the symmetrised cross sections of Eq. 20 and rate
// coefficients from them by Maxwell-Boltzmann averaging over a cubic spline
// through the computed collision energies.
//
// Rates, with beta = k_B T, g the level degeneracy and U the symmetrised
// translational energy (mean of initial and final kinetic energies):
//   k_{i->f} = (1/g_i) sqrt(8/(pi mu)) beta^(-3/2) exp(-(E_f - E_i)/(2 beta))
//              * int s(U) U exp(-U/beta) dU,
// s = natural cubic spline through (U_e, sigma~_e) on [U_1, U_n], a linear ramp
// from zero at the threshold |E_f - E_i|/2 up to U_1, sigma~(U_n) beyond U_n.
// The Boltzmann factor is taken relative to the threshold so that nothing
// overflows.  One thread per (temperature, i, f): the spline's second
// derivatives by the tridiagonal (Thomas) elimination, then 8-point
// Gauss-Legendre on pieces no wider than 2 beta (the exponential's quadrature
// error is then below 1e-13 relative), up to 40 beta past the threshold (beyond,
// the weight is below exp(-40)), plus the constant tail beyond in closed form.
#include "internal.h"

#include <math.h>

namespace mqct {

namespace {

__global__ void xs_sym_kernel(int nE, int L, const double* __restrict__ g,
                              const double* __restrict__ sigma, double* __restrict__ sym,
                              double* __restrict__ ratio) {
  const int64_t LL = (int64_t)L * L;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nE * LL) return;
  const int64_t e = idx / LL;
  const int i = (int)((idx - e * LL) / L), f = (int)(idx - e * LL - (int64_t)i * L);
  const double lhs = g[i] * sigma[idx];
  const double rhs = g[f] * sigma[e * LL + (int64_t)f * L + i];
  if (sym) sym[idx] = 0.5 * (lhs + rhs);
  if (ratio) ratio[idx] = rhs != 0.0 ? lhs / rhs : __builtin_nan("");
}

// Gauss-Legendre nodes and weights on [-1, 1], 8 points (symmetric halves)
__constant__ double GL_X[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                               0.9602898564975363};
__constant__ double GL_W[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                               0.1012285362903763};

struct Interp {
  const double* U;
  const double* y;     // sigma~ at the energies, stride ystride
  int64_t ystride;
  const double* M2;    // second derivatives (per thread)
  int n;
  double th;           // threshold
  __device__ double yat(int e) const { return y[e * ystride]; }
  __device__ double operator()(double x) const {
    if (x < th) return 0.0;
    if (x > U[n - 1]) return yat(n - 1);
    if (x < U[0]) return yat(0) * (x - th) / (U[0] - th);   // only reached when th < U[0]
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (U[mid] <= x) lo = mid; else hi = mid;
    }
    const double h = U[hi] - U[lo];
    const double A = (U[hi] - x) / h, B = 1.0 - A;
    return A * yat(lo) + B * yat(hi) +
           ((A * A * A - A) * M2[lo] + (B * B * B - B) * M2[hi]) * h * h / 6.0;
  }
};

constexpr int XS_NE_MAX = 64;

__global__ void __launch_bounds__(128)
xs_rate_kernel(int nE, int L, int nT, const double* __restrict__ U, const double* __restrict__ E,
               const double* __restrict__ g, const double* __restrict__ sym, double mu,
               const double* __restrict__ beta, double* __restrict__ k) {
  const int64_t LL = (int64_t)L * L;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nT * LL) return;
  const int t = (int)(idx / LL);
  const int64_t p = idx - (int64_t)t * LL;
  const int i = (int)(p / L), f = (int)(p - (int64_t)i * L);
  const double b = beta[t];
  const double dE = E[f] - E[i];
  const double th = fabs(dE) * 0.5;
  // natural-spline second derivatives of sigma~_{if}(U_e)
  double M2[XS_NE_MAX], cp[XS_NE_MAX];
  const double* y = sym + p;
  M2[0] = 0.0;
  M2[nE - 1] = 0.0;
  if (nE > 2) {
    // forward sweep on rows 1..n-2: a M_{e-1} + d M_e + c M_{e+1} = r
    double dprev = 0.0, rprev = 0.0, cprev = 0.0;
    for (int e = 1; e < nE - 1; ++e) {
      const double h0 = U[e] - U[e - 1], h1 = U[e + 1] - U[e];
      const double a = h0 / 6.0, c = h1 / 6.0;
      double d = (h0 + h1) / 3.0;
      double r = (y[(e + 1) * LL] - y[e * LL]) / h1 - (y[e * LL] - y[(e - 1) * LL]) / h0;
      if (e > 1) {
        const double w = a / dprev;
        d -= w * cprev;
        r -= w * rprev;
      }
      M2[e] = r;      // holds the reduced right side until the back sweep
      cp[e] = d;
      dprev = d;
      rprev = r;
      cprev = c;
    }
    for (int e = nE - 2; e >= 1; --e) {
      const double c = (U[e + 1] - U[e]) / 6.0;
      const double next = (e == nE - 2) ? 0.0 : M2[e + 1];
      M2[e] = (M2[e] - c * next) / cp[e];
    }
  }
  Interp s{U, y, LL, M2, nE, th};
  // integral of s(U) U exp(-(U - th)/b) from th; pieces no wider than 2 b
  const double lim = th + 40.0 * b;
  double total = 0.0;
  double a0 = th;
  for (int e = -1; e < nE && a0 < lim; ++e) {
    const double b0 = (e + 1 < nE) ? U[e + 1] : lim;     // next breakpoint
    const double hi = fmin(b0, lim);
    if (hi > a0) {
      const int pieces = max(1, (int)ceil((hi - a0) / (2.0 * b)));
      const double w = (hi - a0) / pieces;
      for (int q = 0; q < pieces; ++q) {
        const double c0 = a0 + (q + 0.5) * w, hw = 0.5 * w;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double x1 = c0 - hw * GL_X[j], x2 = c0 + hw * GL_X[j];
          acc += GL_W[j] * (s(x1) * x1 * exp(-(x1 - th) / b) + s(x2) * x2 * exp(-(x2 - th) / b));
        }
        total += acc * hw;
      }
    }
    a0 = fmax(a0, hi);
  }
  // beyond the cut-off s is the constant sigma~(U_n) (when U_n < lim; otherwise the
  // rest weighs less than exp(-40)): its integral in closed form
  const double Un = fmax(U[nE - 1], th);
  if (Un < lim) total += s.yat(nE - 1) * b * (lim + b) * exp(-(lim - th) / b);
  k[idx] = sqrt(8.0 / (M_PI * mu)) * pow(b, -1.5) * exp(-(th + 0.5 * dE) / b) * total / g[i];
}

}  // namespace

hipError_t launch_xs_symmetrize(int nE, int L, const double* g, const double* sigma, double* sym,
                                double* ratio, hipStream_t s) {
  const int64_t n = (int64_t)nE * L * L;
  xs_sym_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(nE, L, g, sigma, sym, ratio);
  return hipGetLastError();
}

hipError_t launch_xs_rates(int nE, int L, int nT, const double* U, const double* E,
                           const double* g, const double* sym, double mu, const double* beta,
                           double* k, hipStream_t s) {
  if (nE < 2 || nE > XS_NE_MAX) return hipErrorInvalidValue;
  const int64_t n = (int64_t)nT * L * L;
  xs_rate_kernel<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(nE, L, nT, U, E, g, sym, mu, beta,
                                                             k);
  return hipGetLastError();
}

}  // namespace mqct

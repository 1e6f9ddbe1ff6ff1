// Coupling-matrix builder for an asymmetric-top rotor + linear rotor (paper
// Section II, Eqs. 12-18).
//
// The potential is expanded over the angular functions tau_t of Eq. 13 with
// radial coefficients v_t(R) (Eq. 12), so the matrix of Eq. 6 between coupled
// states |n m> = |j1 tau1 j2 j m> (Eq. 3) is M(R) = sum_t v_t(R) G_t with
//
//   G_t(n'', n') = F_t(j1' j2' j', j1'' j2'' j'') * K_t(r'', r') * C(j' m lam 0 | j'' m)
//
// for m'' = m' (zero otherwise).  K_t is the rotor-1 factor of Eq. 17 (the sum
// over k1'', k1' of b b [C(j1' k1' lam1 mu1 | j1'' k1'') + s C(j1' k1' lam1 -mu1 |
// j1'' k1'')], s = (-1)^(lam1+mu1+lam2+lam)).  The sums over m1', m1'' and eta of
// Eq. 17, five Clebsch-Gordan coefficients, recouple into one 9j symbol times a
// coefficient in m (Wigner-Eckart theorem for the rank-lam tensor tau_t):
//
//   F_t = sqrt((2j1'+1)(2j2'+1)(2j'+1)(2lam+1)) sqrt((2lam1+1)(2lam2+1)) / (4 pi)
//         * C(j2' 0 lam2 0 | j2'' 0) * {j1' j2' j'; lam1 lam2 lam; j1'' j2'' j''}
//
// which is what makes the build cheap: F depends on the angular momenta only
// (not on m or tau1), K on the rotor-1 states only.  Kernels:
//   cpl_lfact  log-factorials (the Racah sums below run in the log domain);
//   cpl_rotor  K_t for every pair of rotor-1 states;
//   cpl_jlevel F_t for every pair of (j1, j2, j) levels (9j from three 6j);
//   cpl_fill   one thread per output column n' of a row n'': for the columns of
//              the row's m, the coefficients C(j' m lam 0 | j'' m) (recomputed
//              only when lam changes: terms are sorted by lam), then
//              M[k][n''][n'] = sum_t v_t(R_k) G_t for a chunk of knots at a time
//              with v staged in LDS; every other column gets zeros.  The output
//              is written row by row with consecutive lanes on consecutive
//              columns, so the zeros stream at full write bandwidth.
#include "internal.h"

#include <math.h>

namespace mqct {

namespace {

constexpr int LF_N = 256;        // log-factorial table: arguments up to 255
constexpr int FILL_BLOCK = 256;
constexpr int FILL_KC = 32;      // knots per accumulation chunk (registers)
constexpr int FILL_TC = 32;      // terms per LDS stage

__device__ inline bool tri(int a, int b, int c) { return c >= abs(a - b) && c <= a + b; }

// <j1 m1 j2 m2 | J M> by Racah's sum, each term formed in the log domain
__device__ double cg_dev(const double* __restrict__ lf, int j1, int m1, int j2, int m2, int J,
                         int M) {
  if (m1 + m2 != M || !tri(j1, j2, J) || abs(m1) > j1 || abs(m2) > j2 || abs(M) > J) return 0.0;
  const double lpre = 0.5 * (log((double)(2 * J + 1)) + lf[J + j1 - j2] + lf[J - j1 + j2] +
                             lf[j1 + j2 - J] - lf[j1 + j2 + J + 1] + lf[J + M] + lf[J - M] +
                             lf[j1 - m1] + lf[j1 + m1] + lf[j2 - m2] + lf[j2 + m2]);
  const int kmin = max(0, max(j2 - J - m1, j1 - J + m2));
  const int kmax = min(j1 + j2 - J, min(j1 - m1, j2 + m2));
  double s = 0.0;
  for (int k = kmin; k <= kmax; ++k) {
    const double t = exp(lpre - (lf[k] + lf[j1 + j2 - J - k] + lf[j1 - m1 - k] + lf[j2 + m2 - k] +
                                 lf[J - j2 + m1 + k] + lf[J - j1 - m2 + k]));
    s += (k & 1) ? -t : t;
  }
  return s;
}

__device__ inline double ldelta(const double* lf, int a, int b, int c) {
  return lf[a + b - c] + lf[a - b + c] + lf[b + c - a] - lf[a + b + c + 1];
}

// {a b c; d e f} by Racah's sum
__device__ double sixj_dev(const double* __restrict__ lf, int a, int b, int c, int d, int e,
                           int f) {
  if (!tri(a, b, c) || !tri(a, e, f) || !tri(d, b, f) || !tri(d, e, c)) return 0.0;
  const int a1 = a + b + c, a2 = a + e + f, a3 = d + b + f, a4 = d + e + c;
  const int b1 = a + b + d + e, b2 = b + c + e + f, b3 = c + a + f + d;
  const double ld = 0.5 * (ldelta(lf, a, b, c) + ldelta(lf, a, e, f) + ldelta(lf, d, b, f) +
                           ldelta(lf, d, e, c));
  const int tmin = max(max(a1, a2), max(a3, a4)), tmax = min(b1, min(b2, b3));
  double s = 0.0;
  for (int t = tmin; t <= tmax; ++t) {
    const double x = exp(ld + lf[t + 1] - lf[t - a1] - lf[t - a2] - lf[t - a3] - lf[t - a4] -
                         lf[b1 - t] - lf[b2 - t] - lf[b3 - t]);
    s += (t & 1) ? -x : x;
  }
  return s;
}

// {a b c; d e f; g h i} as a sum over x of (2x+1) {a b c; f i x}{d e f; b x h}{g h i; x a d}
__device__ double ninej_dev(const double* __restrict__ lf, int a, int b, int c, int d, int e,
                            int f, int g, int h, int i) {
  const int xmin = max(abs(a - i), max(abs(b - f), abs(d - h)));
  const int xmax = min(a + i, min(b + f, d + h));
  double s = 0.0;
  for (int x = xmin; x <= xmax; ++x)
    s += (2 * x + 1) * sixj_dev(lf, a, b, c, f, i, x) * sixj_dev(lf, d, e, f, b, x, h) *
         sixj_dev(lf, g, h, i, x, a, d);
  return s;
}

__global__ void cpl_lfact(double* __restrict__ lf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < LF_N) lf[i] = lgamma((double)i + 1.0);
}

// K[t][rb][ra]: the rotor-1 factor between rotor-1 states ra (initial) and rb (final)
__global__ void cpl_rotor(CouplingDev d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)d.n1 * d.n1;
  if (i >= (int64_t)d.T * nn) return;
  const int t = (int)(i / nn);
  const int rb = (int)((i - t * nn) / d.n1), ra = (int)(i - t * nn - (int64_t)rb * d.n1);
  const int l1 = d.t_l1[t], mu = d.t_mu[t], l2 = d.t_l2[t], l = d.t_l[t];
  const double s = ((l1 + mu + l2 + l) & 1) ? -1.0 : 1.0;
  const int ja = d.rot_j[ra], jb = d.rot_j[rb];
  const double* ba = d.b + (int64_t)ra * d.b_stride;
  const double* bb = d.b + (int64_t)rb * d.b_stride;
  double acc = 0.0;
  for (int ka = -ja; ka <= ja; ++ka) {
    const double x = ba[ka + ja];
    if (x == 0.0) continue;
    int kb = ka + mu;
    if (abs(kb) <= jb) acc += bb[kb + jb] * x * cg_dev(d.lf, ja, ka, l1, mu, jb, kb);
    kb = ka - mu;
    if (abs(kb) <= jb) acc += s * bb[kb + jb] * x * cg_dev(d.lf, ja, ka, l1, -mu, jb, kb);
  }
  d.Kr[i] = acc;
}

// F[t][Jb][Ja] between (j1, j2, j) levels Ja (initial) and Jb (final)
__global__ void cpl_jlevel(CouplingDev d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)d.nJ * d.nJ;
  if (i >= (int64_t)d.T * nn) return;
  const int t = (int)(i / nn);
  const int Jb = (int)((i - t * nn) / d.nJ), Ja = (int)(i - t * nn - (int64_t)Jb * d.nJ);
  const int l1 = d.t_l1[t], l2 = d.t_l2[t], l = d.t_l[t];
  const int j1a = d.jl_j1[Ja], j2a = d.jl_j2[Ja], ja = d.jl_j[Ja];
  const int j1b = d.jl_j1[Jb], j2b = d.jl_j2[Jb], jb = d.jl_j[Jb];
  double f = 0.0;
  const double c2 = cg_dev(d.lf, j2a, 0, l2, 0, j2b, 0);
  if (c2 != 0.0 && tri(j1a, l1, j1b) && tri(ja, l, jb)) {
    const double nj = ninej_dev(d.lf, j1a, j2a, ja, l1, l2, l, j1b, j2b, jb);
    f = sqrt((double)(2 * j1a + 1) * (2 * j2a + 1) * (2 * ja + 1) * (2 * l + 1)) *
        sqrt((double)(2 * l1 + 1) * (2 * l2 + 1)) * (0.25 / M_PI) * c2 * nj;
  }
  d.F[i] = f;
}

// M[k][nb][na] (and G[t][nb][na] when asked) for one row nb and FILL_BLOCK columns
__global__ void __launch_bounds__(FILL_BLOCK)
cpl_fill(CouplingDev d, int64_t tiles, double* __restrict__ M, double* __restrict__ G) {
  __shared__ double vs[FILL_TC][FILL_KC];
  const int64_t bid = blockIdx.x;
  const int nb = (int)(bid / tiles);
  const int na = (int)(bid - (int64_t)nb * tiles) * FILL_BLOCK + threadIdx.x;
  const int N = d.N, T = d.T, K = d.K;
  const bool in = na < N;
  const int mb = d.chan_m[nb];
  const bool act = in && d.chan_m[na] == mb;
  const int64_t NN = (int64_t)N * N;
  const int64_t pos = (int64_t)nb * N + na;
  if (!__syncthreads_or(act)) {
    if (in) {
      if (M)
        for (int k = 0; k < K; ++k) M[k * NN + pos] = 0.0;
      if (G)
        for (int t = 0; t < T; ++t) G[t * NN + pos] = 0.0;
    }
    return;
  }
  const int Jb = d.chan_J[nb], rb = d.chan_r[nb], jb = d.chan_j[nb];
  const int Ja = act ? d.chan_J[na] : 0, ra = act ? d.chan_r[na] : 0;
  const int ja = act ? d.chan_j[na] : 0;
  const int64_t nJJ = (int64_t)d.nJ * d.nJ, n11 = (int64_t)d.n1 * d.n1;
  const double* Fp = d.F + (int64_t)Jb * d.nJ + Ja;       // + t * nJJ
  const double* Kp = d.Kr + (int64_t)rb * d.n1 + ra;      // + t * n11
  if (in && !act && G)
    for (int t = 0; t < T; ++t) G[t * NN + pos] = 0.0;
  // G alone: one pass over the terms
  const int kpasses = M ? K : 1;
  for (int k0 = 0; k0 < kpasses; k0 += FILL_KC) {
    double acc[FILL_KC];
#pragma unroll
    for (int q = 0; q < FILL_KC; ++q) acc[q] = 0.0;
    int cur = -1;
    double c = 0.0;
    for (int t0 = 0; t0 < T; t0 += FILL_TC) {
      __syncthreads();
      if (M)
        for (int e = threadIdx.x; e < FILL_TC * FILL_KC; e += FILL_BLOCK) {
          const int tt = e / FILL_KC, kk = e - tt * FILL_KC;
          const int t = t0 + tt, k = k0 + kk;
          vs[tt][kk] = (t < T && k < K) ? d.v[(int64_t)t * K + k] : 0.0;
        }
      __syncthreads();
      if (!act) continue;
      const int t1 = min(T, t0 + FILL_TC);
      for (int t = t0; t < t1; ++t) {
        const int l = d.t_l[t];
        if (l != cur) {
          cur = l;
          c = cg_dev(d.lf, ja, mb, l, 0, jb, mb);
        }
        const double g = Fp[t * nJJ] * Kp[t * n11] * c;
        if (G && k0 == 0) G[(int64_t)d.t_user[t] * NN + pos] = g;
        if (M) {
#pragma unroll
          for (int q = 0; q < FILL_KC; ++q) acc[q] = fma(vs[t - t0][q], g, acc[q]);
        }
      }
    }
    if (M && in) {
#pragma unroll
      for (int q = 0; q < FILL_KC; ++q)
        if (k0 + q < K) M[(k0 + q) * NN + pos] = act ? acc[q] : 0.0;
    }
  }
}

}  // namespace

hipError_t launch_coupling(const CouplingDev& d, double* M, double* G, Prof* prof,
                           hipStream_t s) {
  cpl_lfact<<<1, LF_N, 0, s>>>(d.lf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nr = (int64_t)d.T * d.n1 * d.n1;
  cpl_rotor<<<(unsigned)((nr + 255) / 256), 256, 0, s>>>(d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nj = (int64_t)d.T * d.nJ * d.nJ;
  cpl_jlevel<<<(unsigned)((nj + 255) / 256), 256, 0, s>>>(d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t tiles = (d.N + FILL_BLOCK - 1) / FILL_BLOCK;
  const int64_t blocks = tiles * d.N;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipEvent_t e0 = prof ? prof->next() : nullptr, e1 = prof ? prof->next() : nullptr;
  prof_mark(prof, e0, s);
  cpl_fill<<<(unsigned)blocks, FILL_BLOCK, 0, s>>>(d, tiles, M, G);
  prof_mark(prof, e1, s);
  return hipGetLastError();
}

}  // namespace mqct

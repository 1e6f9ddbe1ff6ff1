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
//   cpl_zero   the outputs cleared with 16-byte stores (most elements couple
//              channels of different m and stay zero);
//   cpl_cgm    the coefficients C(j' m lam 0 | j'' m) for every j', j'', m and lam
//              that occur;
//   cpl_fill   one work item per row n'' and 256 of the channels n' that share its
//              m: per lane g_t = F K C gathered for a chunk of terms, then M[k][n''][n']
//              = sum_t v_t(R_k) g_t for a chunk of knots (v by scalar loads).  With
//              channels ordered by m the lanes of a work item write consecutive
//              columns.
#include "internal.h"

#include <math.h>

#include <algorithm>

namespace mqct {

namespace {

constexpr int LF_N = 256;        // log-factorial table: arguments up to 255
constexpr int FILL_BLOCK = 256;
constexpr int FILL_KC = CPL_KNOT_CHUNK;   // knots per accumulation chunk (registers)
constexpr int NXCD = 8;          // accelerator dies of the device, each with its own L2
constexpr int FILL_TC = 8;       // terms whose factors are gathered together

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

// K[rb][ra][t]: the rotor-1 factor between rotor-1 states ra (initial) and rb (final)
__global__ void cpl_rotor(CouplingDev d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)d.n1 * d.n1;
  if (i >= (int64_t)d.T * nn) return;
  const int t = (int)(i % d.T);
  const int64_t pr = i / d.T;
  const int rb = (int)(pr / d.n1), ra = (int)(pr - (int64_t)rb * d.n1);
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

// F[Jb][Ja][t] between (j1, j2, j) levels Ja (initial) and Jb (final)
__global__ void cpl_jlevel(CouplingDev d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)d.nJ * d.nJ;
  if (i >= (int64_t)d.T * nn) return;
  const int t = (int)(i % d.T);
  const int64_t pr = i / d.T;
  const int Jb = (int)(pr / d.nJ), Ja = (int)(pr - (int64_t)Jb * d.nJ);
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

// zero n doubles, one 16-byte store per thread from the first 16-byte boundary
// (single elements before it and after the last pair)
__global__ void __launch_bounds__(256) cpl_zero(double* __restrict__ p, int64_t n) {
  typedef double dv2 __attribute__((ext_vector_type(2)));
  const int64_t head = ((uintptr_t)p & 15) ? 1 : 0;
  const int64_t pairs = (n - head) >> 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < pairs) ((dv2*)(p + head))[i] = dv2{0.0, 0.0};
  if (i == 0) {
    if (head) p[0] = 0.0;
    if ((n - head) & 1) p[n - 1] = 0.0;
  }
}

// C(ja m lam 0 | jb m) for ja, jb <= JM, |m| <= JM, lam <= LM: cgt[((ja * (JM+1) +
// jb) * (2 JM + 1) + m + JM) * (LM + 1) + lam]
__global__ void cpl_cgm(CouplingDev d) {
  const int JM = d.cg_jmax, LM = d.cg_lmax;
  const int64_t total = (int64_t)(JM + 1) * (JM + 1) * (2 * JM + 1) * (LM + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int lam = (int)(i % (LM + 1));
  int64_t r = i / (LM + 1);
  const int m = (int)(r % (2 * JM + 1)) - JM;
  r /= (2 * JM + 1);
  const int jb = (int)(r % (JM + 1)), ja = (int)(r / (JM + 1));
  d.cgt[i] = cg_dev(d.lf, ja, m, lam, 0, jb, m);
}

// Per element (nb, na) of equal m: pointers to its level factors F[Jb][Ja][.],
// rotor-1 factors K[rb][ra][.] and m-coefficients C(ja m . 0 | jb m); g_t is
// F[t] K[t] C[lam_t] for every kernel that forms it.
struct GPtr {
  const double* F;
  const double* Kr;
  const double* C;
};
__device__ __forceinline__ GPtr gptr(const CouplingDev& d, int nb, int na) {
  const int T = d.T, JM = d.cg_jmax, mb = d.chan_m[nb];
  const int Jb = d.chan_J[nb], rb = d.chan_r[nb], jb = d.chan_j[nb];
  const int Ja = d.chan_J[na], ra = d.chan_r[na], ja = d.chan_j[na];
  GPtr p;
  p.F = d.F + ((int64_t)Jb * d.nJ + Ja) * T;
  p.Kr = d.Kr + ((int64_t)rb * d.n1 + ra) * T;
  p.C = d.cgt + (((int64_t)ja * (JM + 1) + jb) * (2 * JM + 1) + mb + JM) * (d.cg_lmax + 1);
  return p;
}
// g_t for the FILL_TC terms from t0 (indices past the last term repeat it)
__device__ __forceinline__ void gather_g(const CouplingDev& d, const GPtr& p, int t0,
                                         double (&gv)[FILL_TC]) {
#pragma unroll
  for (int i = 0; i < FILL_TC; ++i) {
    const int t = min(t0 + i, d.T - 1);
    gv[i] = p.F[t] * p.Kr[t] * p.C[d.t_l[t]];
  }
}

// One work item = (row nb, FILL_BLOCK consecutive entries of the list of channels
// that share nb's m).  M[k][nb][na] (and G[t][nb][na] when asked) for those na.
// Per chunk of FILL_TC terms a lane first gathers the chunk's factors (F, K and
// the m-coefficient, all independent loads), then adds v_t(R_k) g_t into FILL_KC
// knot accumulators; v (rows padded to a multiple of FILL_KC) is the same for
// every lane and is read with uniform (scalar) loads.
__global__ void __launch_bounds__(FILL_BLOCK)
cpl_fill(CouplingDev d, const int2* __restrict__ work, double* __restrict__ M,
         double* __restrict__ G) {
  const int2 w = work[blockIdx.x];
  const int nb = w.x;
  const int g = d.chan_grp[nb];
  const int g0 = d.grp_off[g], cnt = d.grp_off[g + 1] - g0;
  const int q = w.y * FILL_BLOCK + threadIdx.x;
  if (q >= cnt) return;
  const int na = d.grp_list[g0 + q];
  const int N = d.N, T = d.T, K = d.K, KP = d.KP;
  const int64_t NN = (int64_t)N * N;
  const int64_t pos = (int64_t)nb * N + na;
  const GPtr gp = gptr(d, nb, na);
  const double* __restrict__ v = d.v;
  // G alone: one pass over the terms
  const int kpasses = M ? K : 1;
  for (int k0 = 0; k0 < kpasses; k0 += FILL_KC) {
    double acc[FILL_KC];
#pragma unroll
    for (int u = 0; u < FILL_KC; ++u) acc[u] = 0.0;
    for (int t0 = 0; t0 < T; t0 += FILL_TC) {
      double gv[FILL_TC];
      gather_g(d, gp, t0, gv);
      if (G && k0 == 0) {
#pragma unroll
        for (int i = 0; i < FILL_TC; ++i)
          if (t0 + i < T) G[(int64_t)d.t_user[t0 + i] * NN + pos] = gv[i];
      }
      if (M) {
#pragma unroll
        for (int i = 0; i < FILL_TC; ++i) {
          if (t0 + i >= T) break;
          const double* vt = v + (int64_t)(t0 + i) * KP + k0;
#pragma unroll
          for (int u = 0; u < FILL_KC; ++u) acc[u] = fma(vt[u], gv[i], acc[u]);
        }
      }
    }
    if (M) {
#pragma unroll
      for (int u = 0; u < FILL_KC; ++u)
        if (k0 + u < K) M[(k0 + u) * NN + pos] = acc[u];
    }
  }
}

// Screening: an element of equal m is kept when max_s |M(R_s)| > thr over the
// screening radii, M(R_s) = sum_t vs[t][s] g_t.  Kept elements take slots of
// (rows, cols) in the order the per-wave atomics give (one atomic per wave);
// slots past the capacity are counted but not written.
__global__ void __launch_bounds__(FILL_BLOCK)
cpl_screen(CouplingDev d, const int2* __restrict__ work, int S, const double* __restrict__ vs,
           double thr, int64_t capacity, unsigned long long* __restrict__ count,
           int32_t* __restrict__ rows, int32_t* __restrict__ cols) {
  // workgroup ids go to the dies round-robin; give each die one contiguous share
  // of the work list (ordered by the rows' levels) so that its L2 holds the
  // level-factor rows those items read
  const int64_t per = (d.n_work + NXCD - 1) / NXCD;
  const int64_t wi = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (blockIdx.x / NXCD >= per || wi >= d.n_work) return;
  const int2 w = work[wi];
  const int nb = w.x;
  const int g = d.chan_grp[nb];
  const int g0 = d.grp_off[g], cnt = d.grp_off[g + 1] - g0;
  const int q = w.y * FILL_BLOCK + threadIdx.x;
  const bool act = q < cnt;
  const int na = act ? d.grp_list[g0 + q] : nb;
  bool keep = false;
  if (act) {
    // the element is symmetric, so the decision is taken from one ordering of the
    // pair: (n, m) and (m, n) are kept or dropped together
    const GPtr gp = gptr(d, min(nb, na), max(nb, na));
    double acc[CPL_MAX_SCREEN];
#pragma unroll
    for (int u = 0; u < CPL_MAX_SCREEN; ++u) acc[u] = 0.0;
    for (int t0 = 0; t0 < d.T; t0 += FILL_TC) {
      double gv[FILL_TC];
      gather_g(d, gp, t0, gv);
#pragma unroll
      for (int i = 0; i < FILL_TC; ++i) {
        if (t0 + i >= d.T) break;
        const double* vt = vs + (int64_t)(t0 + i) * S;
#pragma unroll
        for (int u = 0; u < CPL_MAX_SCREEN; ++u)
          if (u < S) acc[u] = fma(vt[u], gv[i], acc[u]);
      }
    }
    double mx = 0.0;
#pragma unroll
    for (int u = 0; u < CPL_MAX_SCREEN; ++u)
      if (u < S) mx = fmax(mx, fabs(acc[u]));
    keep = mx > thr;
  }
  const unsigned long long bal = __ballot(keep);
  const int lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == 0 && bal) base = atomicAdd(count, (unsigned long long)__popcll(bal));
  const int lo = __shfl((int)(base & 0xffffffffull), 0, 64);
  const int hi = __shfl((int)(base >> 32), 0, 64);
  base = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  if (keep) {
    const int64_t idx = (int64_t)(base + __popcll(bal & ((1ull << lane) - 1ull)));
    if (idx < capacity) {
      rows[idx] = nb;
      cols[idx] = na;
    }
  }
}

// Values of the kept elements at every knot: values[k * capacity + i] for the
// element (rows[i], cols[i]), one thread per element.
__global__ void __launch_bounds__(256)
cpl_values(CouplingDev d, int64_t n, const int32_t* __restrict__ rows,
           const int32_t* __restrict__ cols, int64_t capacity, double* __restrict__ values) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GPtr gp = gptr(d, rows[i], cols[i]);
  const int T = d.T, K = d.K, KP = d.KP;
  const double* __restrict__ v = d.v;
  for (int k0 = 0; k0 < K; k0 += FILL_KC) {
    double acc[FILL_KC];
#pragma unroll
    for (int u = 0; u < FILL_KC; ++u) acc[u] = 0.0;
    for (int t0 = 0; t0 < T; t0 += FILL_TC) {
      double gv[FILL_TC];
      gather_g(d, gp, t0, gv);
#pragma unroll
      for (int j = 0; j < FILL_TC; ++j) {
        if (t0 + j >= T) break;
        const double* vt = v + (int64_t)(t0 + j) * KP + k0;
#pragma unroll
        for (int u = 0; u < FILL_KC; ++u) acc[u] = fma(vt[u], gv[j], acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < FILL_KC; ++u)
      if (k0 + u < K) values[(int64_t)(k0 + u) * capacity + i] = acc[u];
  }
}

}  // namespace

namespace {

hipError_t launch_factors(const CouplingDev& d, hipStream_t s) {
  cpl_lfact<<<1, LF_N, 0, s>>>(d.lf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t ncg = (int64_t)(d.cg_jmax + 1) * (d.cg_jmax + 1) * (2 * d.cg_jmax + 1) *
                      (d.cg_lmax + 1);
  cpl_cgm<<<(unsigned)((ncg + 255) / 256), 256, 0, s>>>(d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nr = (int64_t)d.T * d.n1 * d.n1;
  cpl_rotor<<<(unsigned)((nr + 255) / 256), 256, 0, s>>>(d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nj = (int64_t)d.T * d.nJ * d.nJ;
  if ((nj + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
  cpl_jlevel<<<(unsigned)((nj + 255) / 256), 256, 0, s>>>(d);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_coupling(const CouplingDev& d, double* M, double* G, Prof* prof,
                           hipStream_t s) {
  hipError_t e = launch_factors(d, s);
  if (e != hipSuccess) return e;
  hipEvent_t e0 = prof ? prof->next() : nullptr, e1 = prof ? prof->next() : nullptr;
  prof_mark(prof, e0, s);
  const int64_t NN = (int64_t)d.N * d.N;
  auto zero = [&](double* p, int64_t n) {
    const int64_t blocks = ((n + 1) / 2 + 255) / 256;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    cpl_zero<<<(unsigned)blocks, 256, 0, s>>>(p, n);
    return hipGetLastError();
  };
  if (M && (e = zero(M, (int64_t)d.K * NN)) != hipSuccess) return e;
  if (G && (e = zero(G, (int64_t)d.T * NN)) != hipSuccess) return e;
  cpl_fill<<<(unsigned)d.n_work, FILL_BLOCK, 0, s>>>(d, d.work, M, G);
  prof_mark(prof, e1, s);
  return hipGetLastError();
}

hipError_t launch_coupling_screen(const CouplingDev& d, int S, const double* vs, double thr,
                                  int64_t capacity, unsigned long long* count, int32_t* rows,
                                  int32_t* cols, hipStream_t s) {
  if (S < 1 || S > CPL_MAX_SCREEN) return hipErrorInvalidValue;
  hipError_t e = launch_factors(d, s);
  if (e != hipSuccess) return e;
  const int64_t blocks = (d.n_work + NXCD - 1) / NXCD * NXCD;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  cpl_screen<<<(unsigned)blocks, FILL_BLOCK, 0, s>>>(d, d.work, S, vs, thr, capacity, count, rows,
                                                      cols);
  return hipGetLastError();
}

hipError_t launch_coupling_values(const CouplingDev& d, int64_t n, const int32_t* rows,
                                  const int32_t* cols, int64_t capacity, double* values,
                                  hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  cpl_values<<<(unsigned)blocks, 256, 0, s>>>(d, n, rows, cols, capacity, values);
  return hipGetLastError();
}

}  // namespace mqct

// Discrete adjoint of fixed-step RK4 for Ehrenfest trajectories: gradients of
// L = sum_b sum_n w_bn P_b(n) (final probabilities) with respect to the
// coefficients theta of a coupling potential that is linear in them,
//   M(R_k) = sum_p theta_p r_p(R_k) G_{t(p)}        (G_t real symmetric),
// the structure of an expansion of the potential over angular functions with
// R-dependent coefficients (paper Section II, Eqs. 12 and 14-18).
//
// Right-hand side (Eqs. 5, 7-10), written with the Hermitian matrices
// H = P* M P, H' = P* M' P, H'' = P* M'' P, P = diag(e^{-iE t}), omega = Phidot:
//   da/dt   = -i (H + omega J) a
//   dR/dt   = P_R / mu,   dPhi/dt = omega = P_Phi / (mu R^2)
//   dP_R/dt = -a^H H' a + P_Phi^2 / (mu R^3)
//   dP_Phi/dt = -i a^H [J, H] a
// With c = P a and g~ = P g, the vector-Jacobian product for a cotangent
// (g, g_R, g_Phi, g_PR, g_PPhi) of (da/dt, dR/dt, dPhi/dt, dP_R/dt, dP_Phi/dt)
// (complex gradients: d/dRe + i d/dIm) is
//   grad_a   = P* [ i M g~ + i omega J g~ - 2 g_PR M' c - 2 i g_PPhi (J M c - M J c) ]
//   grad_R   = Im(g~^H M' c) + omega_R Im(g~^H J c) - 2 g_Phi P_Phi/(mu R^3)
//              + g_PR (-c^H M'' c - 3 P_Phi^2/(mu R^4)) + 2 g_PPhi Im((Jc)^H M' c)
//   grad_PR  = g_R / mu
//   grad_PPhi = Im(g~^H J c)/(mu R^2) + g_Phi/(mu R^2) + 2 g_PR P_Phi/(mu R^3)
//   grad_theta_p = s_p(R) [Im(g~^H G_t c) + 2 g_PPhi Im((Jc)^H G_t c)]
//                  - g_PR s_p'(R) c^H G_t c
// where omega_R = -2 omega / R and s_p is the natural spline of r_p (the
// spline is linear in the knot values, so dM(R)/dtheta_p = s_p(R) G_t).
//
// The RK4 adjoint of y+ = y + h/6 (k1 + 2k2 + 2k3 + k4) propagates lambda
// backward: kbar4 = h/6 lambda, kbar3 = h/3 lambda + h ybar4,
// kbar2 = h/3 lambda + h/2 ybar3, kbar1 = h/6 lambda + h/2 ybar2 with
// ybar_s = VJP at stage state Y_s, and lambda <- lambda + sum_s ybar_s.  Step
// states come from checkpoints every S steps, recomputed segment by segment by
// the same forward code, so they are bitwise the forward states; the forward
// pass stores the last segment's stage states itself.
#include "device.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace mqct {

namespace {

constexpr int AB = 256;           // threads per trajectory
constexpr int ANW = AB / 64;
constexpr int NSC = 4;            // VJP scalars reduced over the workgroup
constexpr int NGMAX = 48;         // angular terms (three bilinear forms each in LDS)

struct AdjArgs {
  const TrajIn* traj;
  const double* dLdP;      // [sum N] weights of the final probabilities
  double* grad_part;       // [B][P] per-trajectory gradient
  double* P_out;           // [sum N] or null
  double* scratch;         // per trajectory: checkpoints + stage states of one segment
  int64_t scratch_stride;  // doubles per trajectory
  int S;                   // checkpoint interval
  const int* goff;         // [nG+1] nonzeros of G_t are goff[t] .. goff[t+1]-1
  const uint32_t* gent;    // row | col << 16
  const double* gval;
  const double* rad;       // [P][K] r_p at the knots
  const double* rad2;      // [P][K] their natural-spline second derivatives
  int P, nG;
  const int* gidx;         // [P]
  const int* order;        // [B] trajectories in the order they are dealt to the dies
  int64_t B;
  int per_die;             // workgroups per die (blocks x, x + 8, ... of die x)
  // angular terms of each wave for the bilinear forms: tord[tbeg[w] .. tbeg[w+1]-1],
  // balanced by their nonzero counts
  int tord[NGMAX];
  int tbeg[ANW + 1];
};

constexpr int GU = 8;      // nonzeros of G_t per lane whose loads are issued together
constexpr int JXB = 4;     // J_x widths up to this have their loads issued together

constexpr int ADIES = 8;   // accelerator dies of the device, each with its own L2

template <bool CPLX, int NR, bool ELL>
struct Adj {
  __device__ static int row(int r) { return threadIdx.x + r * AB; }

  struct St {              // a trajectory state in registers: this lane's rows + classical
    double2 a[NR];
    double y[4];           // R, Phi, P_R, P_Phi
  };

  __device__ static double2 mc(double2 x, double2 y) { return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x); }

  // the four spline coefficients of element (n, m) in interval k: value_k,
  // value_{k+1}, second derivative_k, second derivative_{k+1}.  Column access:
  // M_nm = conj(S[m][n]) for Hermitian tables, S[m][n] for real symmetric ones
  // (m is the stored row, or the slot of sparse tables).
  struct Raw {
    double2 v[4];
  };
  __device__ static Raw raw(const DevSystem& sy, int k, int m, int n) {
    const int64_t ks = sy.knot_stride;
    const int64_t o = (int64_t)k * ks + (int64_t)m * sy.Npad + n;
    Raw r;
    if constexpr (CPLX) {
      const double2* M = (const double2*)sy.M;
      const double2* M2 = (const double2*)sy.M2;
      r.v[0] = M[o]; r.v[1] = M[o + ks]; r.v[2] = M2[o]; r.v[3] = M2[o + ks];
    } else {
      const double* M = (const double*)sy.M;
      const double* M2 = (const double*)sy.M2;
      r.v[0].x = M[o]; r.v[1].x = M[o + ks]; r.v[2].x = M2[o]; r.v[3].x = M2[o + ks];
    }
    return r;
  }
  __device__ static double2 comb(const Raw& r, const double (&w)[4]) {
    double2 z;
    z.x = w[0] * r.v[0].x + w[1] * r.v[1].x + w[2] * r.v[2].x + w[3] * r.v[3].x;
    z.y = CPLX ? -(w[0] * r.v[0].y + w[1] * r.v[1].y + w[2] * r.v[2].y + w[3] * r.v[3].y) : 0.0;
    return z;
  }
  // complex product with a table element that is real for real symmetric tables
  __device__ static double2 mt(double2 M, double2 x) {
    if constexpr (CPLX) return mc(M, x);
    else return make_double2(M.x * x.x, M.x * x.y);
  }

  __device__ static void weights(const Spl& sp, double (&w)[4], double (&d)[4], double (&dd)[4],
                                 double R, const double* x, int K) {
    w[0] = sp.w0; w[1] = sp.w1; w[2] = sp.w2; w[3] = sp.w3;
    d[0] = sp.d0; d[1] = sp.d1; d[2] = sp.d2; d[3] = sp.d3;
    dd[0] = dd[1] = dd[2] = dd[3] = 0.0;
    if (!sp.below && !(R > x[K - 1])) {      // inside the grid: M'' = A M2_k + B M2_{k+1}
      dd[2] = sp.w0;
      dd[3] = sp.w1;
    }
  }

  // J x for this lane's rows from an LDS vector (the row's entries are all
  // requested before the first gather; the sum runs in entry order either way)
  __device__ static double2 jx(const DevSystem& sy, int n, const double2* v) {
    double2 s = make_double2(0.0, 0.0);
    const int W = sy.jx_w;
    if (W <= JXB) {
      int col[JXB];
      double jv[JXB];
#pragma unroll
      for (int q = 0; q < JXB; ++q) {
        col[q] = q < W ? sy.jx_col[(int64_t)n * W + q] : 0;
        jv[q] = q < W ? sy.jx_val[(int64_t)n * W + q] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < JXB; ++q) {
        if (q >= W) break;
        s.x = fma(jv[q], v[col[q]].x, s.x);
        s.y = fma(jv[q], v[col[q]].y, s.y);
      }
      return s;
    }
    for (int q = 0; q < W; ++q) {
      const int col = sy.jx_col[(int64_t)n * W + q];
      const double jv = sy.jx_val[(int64_t)n * W + q];
      s.x = fma(jv, v[col].x, s.x);
      s.y = fma(jv, v[col].y, s.y);
    }
    return s;
  }

  // forward right-hand side: f(t, Y) -> F
  __device__ static void rhs(const DevSystem& sy, double t, const St& Y, St& F, double2* lc,
                             double* red) {
    const int N = sy.N;
    // stored rows per column: all N, or the kept slots of sparse tables (slot j
    // of column n holds stored row ell_col[j][n])
    constexpr bool ell = ELL;
    const int nst = ell ? sy.ell_w : N;
    const double mu = sy.mu, R = Y.y[0], pphi = Y.y[3];
    const Spl sp = spline_at(sy.R, sy.K, R, sy.R_inv_h);
    double w[4], d[4], dd[4];
    weights(sp, w, d, dd, R, sy.R, sy.K);
    const double om = pphi / (mu * R * R);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) {
        double sn, cs;
        sincos(sy.E[n] * t, &sn, &cs);
        lc[n] = mc(make_double2(cs, -sn), Y.a[r]);
      }
    }
    __syncthreads();
    double sums[2] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n >= N) { F.a[r] = make_double2(0.0, 0.0); continue; }
      double2 u = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int j = 0; j < nst; ++j) {
        const int m = ell ? sy.ell_col[(int64_t)j * sy.Npad + n] : j;
        const double2 cm = lc[m];
        const Raw q = raw(sy, sp.k, j, n);
        const double2 a1 = mt(comb(q, w), cm), a2 = mt(comb(q, d), cm);
        u.x += a1.x; u.y += a1.y; v.x += a2.x; v.y += a2.y;
      }
      const double2 c = lc[n];
      const double2 x = jx(sy, n, lc);
      sums[0] += c.x * v.x + c.y * v.y;          // Re(c^H M' c)
      sums[1] += x.x * u.y - x.y * u.x;          // Im((Jc)^H M c)
      const double2 g = make_double2(u.x + om * x.x, u.y + om * x.y);
      double sn, cs;
      sincos(sy.E[n] * t, &sn, &cs);
      const double2 y = mc(make_double2(cs, sn), g);
      F.a[r] = make_double2(y.y, -y.x);          // -i e^{iEt} (u + omega J c)
    }
    block_sum<2, ANW>(sums, red);
    F.y[0] = Y.y[2] / mu;
    F.y[1] = om;
    F.y[2] = -sums[0] + pphi * pphi / (mu * R * R * R);
    F.y[3] = 2.0 * sums[1];
  }

  // vector-Jacobian product at (t, Y) for the cotangent Gc; returns Yb and adds
  // this thread's parameter's share to gth (thread p owns theta_p)
  __device__ static void vjp(const DevSystem& sy, const AdjArgs& A, double t, const St& Y,
                             const St& Gc, St& Yb, double& gth, double2* lc, double2* lg,
                             double2* ljc, double2* lmc, double* red, double* tq) {
    const int N = sy.N;
    // stored rows per column: all N, or the kept slots of sparse tables (slot j
    // of column n holds stored row ell_col[j][n])
    constexpr bool ell = ELL;
    const int nst = ell ? sy.ell_w : N;
    const double mu = sy.mu, R = Y.y[0], pphi = Y.y[3];
    const Spl sp = spline_at(sy.R, sy.K, R, sy.R_inv_h);
    double w[4], d[4], dd[4];
    weights(sp, w, d, dd, R, sy.R, sy.K);
    const double om = pphi / (mu * R * R);
    const double gR = Gc.y[0], gPhi = Gc.y[1], gPR = Gc.y[2], gPPhi = Gc.y[3];
    // the previous product still reads lg, lmc and tq after its last barrier
    __syncthreads();
    double psn[NR], pcs[NR];   // this lane's phase factors, for c, g~ and the result
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      psn[r] = 0.0;
      pcs[r] = 1.0;
      if (n < N) {
        sincos(sy.E[n] * t, &psn[r], &pcs[r]);
        lc[n] = mc(make_double2(pcs[r], -psn[r]), Y.a[r]);
        lg[n] = mc(make_double2(pcs[r], -psn[r]), Gc.a[r]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) ljc[n] = jx(sy, n, lc);
    }
    __syncthreads();
    // bilinear forms of the sparse G_t, one wave per angular term (the terms dealt
    // to the waves by their nonzero counts); each lane sums its nonzeros e, e + 64,
    // ... in order, GU of them requested at a time:
    // tq[3t] = Im(g~^H G_t c), tq[3t+1] = Im((Jc)^H G_t c), tq[3t+2] = Re(c^H G_t c)
    {
      const int lane = threadIdx.x & 63;
      const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      for (int i = A.tbeg[wv]; i < A.tbeg[wv + 1]; ++i) {
        const int tt = A.tord[i];
        double f[3] = {0.0, 0.0, 0.0};
        const int e1 = A.goff[tt + 1];
        for (int e0 = A.goff[tt] + lane; e0 < e1; e0 += 64 * GU) {
          uint32_t nm[GU];
          double gv[GU];
#pragma unroll
          for (int u = 0; u < GU; ++u) {
            const int e = e0 + 64 * u;
            nm[u] = e < e1 ? A.gent[e] : 0u;
            gv[u] = e < e1 ? A.gval[e] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < GU; ++u) {
            if (e0 + 64 * u >= e1) break;
            const int n = nm[u] & 0xffff, m = nm[u] >> 16;
            const double v = gv[u];
            const double2 cm = lc[m], cn = lc[n], gn = lg[n], jn = ljc[n];
            f[0] = fma(v, gn.x * cm.y - gn.y * cm.x, f[0]);
            f[1] = fma(v, jn.x * cm.y - jn.y * cm.x, f[1]);
            f[2] = fma(v, cn.x * cm.x + cn.y * cm.y, f[2]);
          }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) f[i] += __shfl_xor(f[i], off, 64);
        if (lane == 0) {
          tq[3 * tt] = f[0]; tq[3 * tt + 1] = f[1]; tq[3 * tt + 2] = f[2];
        }
      }
    }
    // one pass over the four table slices for the five products
    double sc[NSC] = {0.0, 0.0, 0.0, 0.0};
    double2 Mg[NR], MJc[NR], Mpc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      Mg[r] = MJc[r] = Mpc[r] = make_double2(0.0, 0.0);
      if (n >= N) continue;
      double2 Mc = make_double2(0.0, 0.0), Mppc = make_double2(0.0, 0.0);
#pragma unroll 1
      for (int j = 0; j < nst; ++j) {
        const int m = ell ? sy.ell_col[(int64_t)j * sy.Npad + n] : j;
        const Raw q = raw(sy, sp.k, j, n);
        const double2 Mv = comb(q, w), Md = comb(q, d), Mdd = comb(q, dd);
        const double2 cm = lc[m], gm = lg[m], jm = ljc[m];
        const double2 t1 = mt(Mv, gm), t2 = mt(Mv, cm), t3 = mt(Mv, jm), t4 = mt(Md, cm),
                      t5 = mt(Mdd, cm);
        Mg[r].x += t1.x; Mg[r].y += t1.y;
        Mc.x += t2.x; Mc.y += t2.y;
        MJc[r].x += t3.x; MJc[r].y += t3.y;
        Mpc[r].x += t4.x; Mpc[r].y += t4.y;
        Mppc.x += t5.x; Mppc.y += t5.y;
      }
      const double2 c = lc[n], gt = lg[n], jc = ljc[n];
      sc[0] += gt.x * Mpc[r].y - gt.y * Mpc[r].x;     // Im(g~^H M' c)
      sc[1] += gt.x * jc.y - gt.y * jc.x;             // Im(g~^H J c)
      sc[2] += c.x * Mppc.x + c.y * Mppc.y;           // Re(c^H M'' c)
      sc[3] += jc.x * Mpc[r].y - jc.y * Mpc[r].x;     // Im((Jc)^H M' c)
      lmc[n] = Mc;
    }
    block_sum<NSC, ANW>(sc, red);    // its barrier also publishes lmc and tq
    // grad_a = P* [ i M g~ + i omega J g~ - 2 g_PR M' c - 2 i g_PPhi (J M c - M J c) ]
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n >= N) { Yb.a[r] = make_double2(0.0, 0.0); continue; }
      const double2 jmc = jx(sy, n, lmc);
      const double2 jg = jx(sy, n, lg);
      double2 s;
      s.x = -(Mg[r].y + om * jg.y) - 2.0 * gPR * Mpc[r].x + 2.0 * gPPhi * (jmc.y - MJc[r].y);
      s.y = (Mg[r].x + om * jg.x) - 2.0 * gPR * Mpc[r].y - 2.0 * gPPhi * (jmc.x - MJc[r].x);
      Yb.a[r] = mc(make_double2(pcs[r], psn[r]), s);
    }
    const double R3 = R * R * R;
    const double omR = -2.0 * om / R;
    Yb.y[0] = sc[0] + omR * sc[1] - 2.0 * gPhi * pphi / (mu * R3) +
              gPR * (-sc[2] - 3.0 * pphi * pphi / (mu * R3 * R)) + 2.0 * gPPhi * sc[3];
    Yb.y[1] = 0.0;
    Yb.y[2] = gR / mu;
    Yb.y[3] = sc[1] / (mu * R * R) + gPhi / (mu * R * R) + 2.0 * gPR * pphi / (mu * R3);
    // parameter gradient: thread p owns theta_p
    const int p = threadIdx.x;
    if (p < A.P) {
      const int tt = A.gidx[p];
      const double* rp = A.rad + (int64_t)p * sy.K;
      const double* r2 = A.rad2 + (int64_t)p * sy.K;
      const int k = sp.k;
      const double sv = w[0] * rp[k] + w[1] * rp[k + 1] + w[2] * r2[k] + w[3] * r2[k + 1];
      const double sd = d[0] * rp[k] + d[1] * rp[k + 1] + d[2] * r2[k] + d[3] * r2[k + 1];
      gth += sv * (tq[3 * tt] + 2.0 * gPPhi * tq[3 * tt + 1]) - gPR * sd * tq[3 * tt + 2];
    }
  }

  __device__ static void axpy(St& o, const St& x, double a, const St& y) {   // o = x + a y
#pragma unroll
    for (int r = 0; r < NR; ++r)
      o.a[r] = make_double2(fma(a, y.a[r].x, x.a[r].x), fma(a, y.a[r].y, x.a[r].y));
#pragma unroll
    for (int i = 0; i < 4; ++i) o.y[i] = fma(a, y.y[i], x.y[i]);
  }
  __device__ static void scale(St& o, double a, const St& y) {                // o = a y
#pragma unroll
    for (int r = 0; r < NR; ++r) o.a[r] = make_double2(a * y.a[r].x, a * y.a[r].y);
#pragma unroll
    for (int i = 0; i < 4; ++i) o.y[i] = a * y.y[i];
  }

  __device__ static void save(double* dst, const St& y, int N, int Npad) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) ((double2*)dst)[n] = y.a[r];
    }
    if (threadIdx.x == 0)
      for (int i = 0; i < 4; ++i) dst[2 * Npad + i] = y.y[i];
  }

  __device__ static void load(const double* src, St& y, int N, int Npad) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      y.a[r] = n < N ? ((const double2*)src)[n] : make_double2(0.0, 0.0);
    }
    for (int i = 0; i < 4; ++i) y.y[i] = src[2 * Npad + i];
  }

  // one RK4 step; with `stages` non-null the four stage states are stored there
  // (stride SV doubles), in the order Y1 = y, Y2, Y3, Y4
  __device__ static void rk4(const DevSystem& sy, double t, double h, St& y, double2* lc,
                             double* red, double* stages, int64_t SV) {
    St k, acc, Ys;
    if (stages) save(stages, y, sy.N, sy.Npad);
    rhs(sy, t, y, k, lc, red);
    acc = k;
    axpy(Ys, y, 0.5 * h, k);
    if (stages) save(stages + SV, Ys, sy.N, sy.Npad);
    rhs(sy, t + 0.5 * h, Ys, k, lc, red);
    axpy(acc, acc, 2.0, k);
    axpy(Ys, y, 0.5 * h, k);
    if (stages) save(stages + 2 * SV, Ys, sy.N, sy.Npad);
    rhs(sy, t + 0.5 * h, Ys, k, lc, red);
    axpy(acc, acc, 2.0, k);
    axpy(Ys, y, h, k);
    if (stages) save(stages + 3 * SV, Ys, sy.N, sy.Npad);
    rhs(sy, t + h, Ys, k, lc, red);
    axpy(acc, acc, 1.0, k);
    axpy(y, y, h / 6.0, acc);
  }
};

// PH = 0: forward pass, then the backward sweep, recomputing the segments before
// the last from their checkpoints.  With one segment (nothing to recompute) the
// two passes run as separate launches, each with its own register budget:
// PH = 1 runs the forward pass and stores the end state; PH = 2 starts from it.
constexpr int PH_FUSED = 0, PH_FWD = 1, PH_BWD = 2;

template <bool CPLX, int NR, bool ELL, int PH>
__global__ void __launch_bounds__(AB)
adjoint_kernel(const DevSystem* __restrict__ systems, AdjArgs A) {
  using K = Adj<CPLX, NR, ELL>;
  using St = typename K::St;
  extern __shared__ __align__(16) unsigned char smem[];
  // workgroups are handed to the dies round-robin: die x runs blocks x, x + 8, ...,
  // which take a contiguous share of the ordered trajectories
  const int64_t pos = (int64_t)(blockIdx.x % ADIES) * A.per_die + blockIdx.x / ADIES;
  if (pos >= A.B) return;
  const int b = A.order[pos];
  const TrajIn tj = A.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  double2* lc = (double2*)smem;
  double2* lg = lc + Npad;
  double2* ljc = lg + Npad;
  double2* lmc = ljc + Npad;
  double* red = (double*)(lmc + Npad);     // [ANW][<= NSC]
  double* tq = red + ANW * NSC;            // [3 * NGMAX]
  double* scr = A.scratch + (int64_t)b * A.scratch_stride;
  const int64_t SV = 2 * (int64_t)Npad + 4;
  const int S = A.S;
  const int64_t n = tj.n_steps;
  const int64_t nseg = (n + S - 1) / S;
  double* ck = scr;                                   // [nseg][SV]
  double* seg = scr + (nseg > 0 ? nseg : 1) * SV;     // [S][4][SV] stage states
  double* fin = seg + 4 * (int64_t)S * SV;            // [SV] end state (split passes)
  const double h = tj.dt, t0 = tj.t0;

  St y;
  if constexpr (PH == PH_BWD) {
    K::load(fin, y, N, Npad);
  } else {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int nn = K::row(r);
    y.a[r] = (nn < N && nn == tj.init_channel) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
  }
  {
    const double k = sqrt(2.0 * sy.mu * tj.E_coll);
    const double pphi = tj.b * k;
    y.y[0] = tj.R0; y.y[1] = 0.0;
    y.y[2] = -sqrt(2.0 * sy.mu * tj.E_coll - pphi * pphi / (tj.R0 * tj.R0));
    y.y[3] = pphi;
  }
  // forward pass with checkpoints; the last segment's stage states are stored as
  // they are made, so the backward sweep starts without recomputing it (with one
  // segment, S >= n_steps, nothing is recomputed)
  const int64_t jlast = (nseg - 1) * S;
  for (int64_t j = 0; j < n; ++j) {
    if (j % S == 0) K::save(ck + (j / S) * SV, y, N, Npad);
    K::rk4(sy, t0 + (double)j * h, h, y, lc, red, j >= jlast ? seg + 4 * (j - jlast) * SV : nullptr,
           SV);
  }
  // final probabilities
  if (A.P_out) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int nn = K::row(r);
      if (nn < N) A.P_out[tj.amp_off + nn] = y.a[r].x * y.a[r].x + y.a[r].y * y.a[r].y;
    }
  }
  if constexpr (PH == PH_FWD) {
    K::save(fin, y, N, Npad);
    return;
  }
  }
  // the starting adjoint lambda_a = 2 a dL/dP
  St lam;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int nn = K::row(r);
    if (nn < N) {
      const double wgt = A.dLdP[tj.amp_off + nn];
      lam.a[r] = make_double2(2.0 * wgt * y.a[r].x, 2.0 * wgt * y.a[r].y);
    } else {
      lam.a[r] = make_double2(0.0, 0.0);
    }
  }
  for (int i = 0; i < 4; ++i) lam.y[i] = 0.0;
  double gth = 0.0;
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t j0 = sg * S, j1 = (j0 + S < n) ? j0 + S : n;
    __syncthreads();                     // stage states of the previous segment are consumed
    if constexpr (PH == PH_FUSED) {
      if (sg < nseg - 1) {               // the last segment's states are there already
        K::load(ck + sg * SV, y, N, Npad);
        for (int64_t j = j0; j < j1; ++j)
          K::rk4(sy, t0 + (double)j * h, h, y, lc, red, seg + 4 * (j - j0) * SV, SV);
      }
    }
    __syncthreads();                     // publishes the stored classical coordinates
    for (int64_t j = j1 - 1; j >= j0; --j) {
      const double t = t0 + (double)j * h;
      const double* st = seg + 4 * (j - j0) * SV;
      St Ys, kb, yb, dl;
      // kbar4 = h/6 lambda; kbar3 = h/3 lambda + h ybar4; kbar2 = h/3 lambda + h/2 ybar3;
      // kbar1 = h/6 lambda + h/2 ybar2; lambda += ybar4 + ybar3 + ybar2 + ybar1
      K::scale(kb, h / 6.0, lam);
      K::load(st + 3 * SV, Ys, N, Npad);
      K::vjp(sy, A, t + h, Ys, kb, yb, gth, lc, lg, ljc, lmc, red, tq);
      dl = yb;
      K::scale(kb, h / 3.0, lam);
      K::axpy(kb, kb, h, yb);
      K::load(st + 2 * SV, Ys, N, Npad);
      K::vjp(sy, A, t + 0.5 * h, Ys, kb, yb, gth, lc, lg, ljc, lmc, red, tq);
      K::axpy(dl, dl, 1.0, yb);
      K::scale(kb, h / 3.0, lam);
      K::axpy(kb, kb, 0.5 * h, yb);
      K::load(st + SV, Ys, N, Npad);
      K::vjp(sy, A, t + 0.5 * h, Ys, kb, yb, gth, lc, lg, ljc, lmc, red, tq);
      K::axpy(dl, dl, 1.0, yb);
      K::scale(kb, h / 6.0, lam);
      K::axpy(kb, kb, 0.5 * h, yb);
      K::load(st, Ys, N, Npad);
      K::vjp(sy, A, t, Ys, kb, yb, gth, lc, lg, ljc, lmc, red, tq);
      K::axpy(dl, dl, 1.0, yb);
      K::axpy(lam, lam, 1.0, dl);
    }
  }
  if ((int)threadIdx.x < A.P) A.grad_part[(int64_t)b * A.P + threadIdx.x] = gth;
}

// dL/dtheta_p = sum_b grad_part[b][p], in batch order
__global__ void grad_reduce(const double* __restrict__ part, int64_t B, int P,
                            double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int64_t b = 0; b < B; ++b) s += part[b * P + p];
  out[p] = s;
}

// M[k][n][m] = sum_t V_t(R_k) G_t[n][m], V_t(R_k) = sum_{p: t(p)=t} theta_p r_p(R_k)
__global__ void build_param_tables(const double* __restrict__ G, const double* __restrict__ rad,
                                   const int* __restrict__ gidx, const double* __restrict__ theta,
                                   int P, int nG, int N, int Npad, int K,
                                   double* __restrict__ Mout) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t NN = (int64_t)N * N;
  if (i >= NN * K) return;
  const int64_t k = i / NN;
  const int64_t r = i - k * NN;
  const int64_t nrow = r / N, m = r - nrow * N;
  double s = 0.0;
  for (int p = 0; p < P; ++p) {
    const double v = theta[p] * rad[(int64_t)p * K + k];
    s = fma(v, G[((int64_t)gidx[p] * N + nrow) * Npad + m], s);
  }
  Mout[i] = s;
}

// natural-spline second derivatives of ncol columns y[c][K] (one thread per column)
__global__ void spline_rows(const double* __restrict__ y, const double* __restrict__ x, int K,
                            int ncol, double* __restrict__ y2, double* __restrict__ tmp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double* yc = y + (int64_t)c * K;
  double* o = y2 + (int64_t)c * K;
  double* d = tmp + (int64_t)c * K;
  double* cp = d + (int64_t)ncol * K;
  o[0] = 0.0;
  o[K - 1] = 0.0;
  double dprev = 0.0, cprev = 0.0;
  for (int k = 1; k <= K - 2; ++k) {
    const double hl = x[k] - x[k - 1], hr = x[k + 1] - x[k];
    const double den = (hl + hr) / 3.0 - (k > 1 ? hl / 6.0 * cprev : 0.0);
    const double rhs = (yc[k + 1] - yc[k]) / hr - (yc[k] - yc[k - 1]) / hl;
    const double dk = (rhs - (k > 1 ? hl / 6.0 * dprev : 0.0)) / den;
    cprev = hr / 6.0 / den;
    d[k] = dk;
    cp[k] = cprev;
    dprev = dk;
  }
  double nxt = 0.0;
  for (int k = K - 2; k >= 1; --k) {
    const double v = d[k] - cp[k] * nxt;
    o[k] = v;
    nxt = v;
  }
}

}  // namespace

int64_t adjoint_scratch_doubles(int Npad, int64_t n_steps, int S) {
  const int64_t SV = 2 * (int64_t)Npad + 4;
  const int64_t nseg = (n_steps + S - 1) / S;
  return ((nseg > 0 ? nseg : 1) + 4 * (int64_t)S + 1) * SV;
}

hipError_t launch_adjoint(const DevSystem* d_systems, bool cplx, bool ell, int Npad,
                          const TrajIn* d_traj, const int* order,
                          int64_t B, const double* dLdP, double* grad_part, double* grad_out,
                          double* P_out, double* scratch, int64_t scratch_stride, int S,
                          const int* goff, const int* h_goff, const uint32_t* gent,
                          const double* gval, const double* rad, const double* rad2,
                          const int* gidx, int P, int nG, bool one_segment, hipStream_t s) {
  if (nG > NGMAX || P > AB) return hipErrorInvalidValue;
  const int per = (int)((B + ADIES - 1) / ADIES);
  AdjArgs A{d_traj, dLdP, grad_part, P_out, scratch, scratch_stride, S, goff, gent, gval,
            rad, rad2, P, nG, gidx, order, B, per, {}, {}};
  // angular terms to waves, largest first, each to the wave with the fewest
  // nonzeros so far (the wave with the most sets the time of the forms)
  std::vector<int> byn(nG), of(nG);
  for (int t = 0; t < nG; ++t) byn[t] = t;
  std::stable_sort(byn.begin(), byn.end(), [&](int x, int y) {
    return h_goff[x + 1] - h_goff[x] > h_goff[y + 1] - h_goff[y];
  });
  int64_t load[ANW] = {};
  for (int t : byn) {
    int w = 0;
    for (int v = 1; v < ANW; ++v)
      if (load[v] < load[w]) w = v;
    of[t] = w;
    load[w] += h_goff[t + 1] - h_goff[t];
  }
  int pos = 0;
  for (int w = 0; w < ANW; ++w) {
    A.tbeg[w] = pos;
    for (int t = 0; t < nG; ++t)
      if (of[t] == w) A.tord[pos++] = t;
  }
  A.tbeg[ANW] = pos;
  const unsigned grid = (unsigned)per * ADIES;
  // four double2 vectors, then red [ANW][NSC] and tq [3 NGMAX]
  const size_t lds = (size_t)Npad * 64 + (size_t)ANW * NSC * 8 + (size_t)3 * NGMAX * 8;
  const int nr = (Npad + AB - 1) / AB;
  hipError_t e;
  auto go = [&](auto cp, auto el) {
    constexpr bool C = decltype(cp)::value, E = decltype(el)::value;
    auto run = [&](auto nrt) {
      constexpr int R = decltype(nrt)::value;
      if (one_segment) {
        adjoint_kernel<C, R, E, PH_FWD><<<grid, AB, lds, s>>>(d_systems, A);
        adjoint_kernel<C, R, E, PH_BWD><<<grid, AB, lds, s>>>(d_systems, A);
      } else {
        adjoint_kernel<C, R, E, PH_FUSED><<<grid, AB, lds, s>>>(d_systems, A);
      }
    };
    if (nr <= 1) run(std::integral_constant<int, 1>{});
    else if (nr <= 2) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 4>{});
  };
  if (nr > 4) return hipErrorInvalidValue;
  if (cplx) {
    if (ell) go(std::true_type{}, std::true_type{});
    else go(std::true_type{}, std::false_type{});
  } else {
    if (ell) go(std::false_type{}, std::true_type{});
    else go(std::false_type{}, std::false_type{});
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  grad_reduce<<<(P + 127) / 128, 128, 0, s>>>(grad_part, B, P, grad_out);
  return hipGetLastError();
}

hipError_t launch_build_param_tables(const double* G, const double* rad, const int* gidx,
                                     const double* theta, int P, int nG, int N, int Npad, int K,
                                     double* Mout, hipStream_t s) {
  const int64_t total = (int64_t)N * N * K;
  build_param_tables<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(G, rad, gidx, theta, P, nG,
                                                                     N, Npad, K, Mout);
  return hipGetLastError();
}

hipError_t launch_spline_rows(const double* y, const double* x, int K, int ncol, double* y2,
                              double* tmp, hipStream_t s) {
  spline_rows<<<(ncol + 127) / 128, 128, 0, s>>>(y, x, K, ncol, y2, tmp);
  return hipGetLastError();
}

}  // namespace mqct

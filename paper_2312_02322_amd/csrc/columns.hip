// Coordinate-list coupling tables and the columns schedule: decoupled (AT)
// dynamics of many initial states per classical path on truncated coupling
// matrices -- the paper's production form (Section III: AT-MQCT with 100
// initial states of water per trajectory, on matrices of about 14.6 M kept
// elements for 206,350 states).
//
// Tables: the stored elements in row order (CSR, each row's columns ascending),
// their values and natural-spline second derivatives per knot, [K][nnz]
// (complex interleaved).  A group of columns that shares a path (at most
// COL_MAX) keeps its amplitudes as rows of CT complex FP64 values, [N][CT]
// (CT: the columns padded to even), so the product's gather of a coupled row m
// reads CT contiguous values.
//
// One launch per RK4 stage: a wave takes one row of one group, two columns per
// lane.  A row's elements are read 64 at a time, one per lane, and turned into
// the spline value at the stage's R in FP64; then they are broadcast one by one
// while every lane gathers its columns of the coupled row's phased amplitudes
// c_m = e^{-iE_m t} a_m.  The J_x term, the row's phase, the RK4 update and the
// phased amplitudes of the next stage follow in the same kernel (Eq. 5).  The
// classical path is driven by U(R) alone (AT), so it is integrated once per
// group beforehand (Eqs. 7-9 with the driver's force), one thread per group.
#include "device.h"

#include <math.h>

#include <algorithm>

namespace mqct {

namespace {

constexpr int CB = 512;         // threads of the row kernels
constexpr int CW = CB / 64;
constexpr int ROWS_PER_WAVE = 1;
constexpr int ROWS_PER_WG = CW * ROWS_PER_WAVE;
constexpr int NXCD = 8;         // dies of the device; workgroups are dealt to them round-robin
constexpr int GATHER_UNROLL = 8;

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- loading -----------------------------------------------------------------

// v64[k][e] = values[k][perm[e]] (NC reals per element), counting non-finite values.
__global__ void coo_gather(const double* __restrict__ values, int64_t ld, const int32_t* __restrict__ perm,
                           int64_t nnz, int K, int NC, double* __restrict__ v64,
                           unsigned long long* __restrict__ nonfinite) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int64_t src = perm[e];
  int bad = 0;
  for (int k = 0; k < K; ++k)
    for (int c = 0; c < NC; ++c) {
      const double v = values[((int64_t)k * ld + src) * NC + c];
      bad += !isfinite(v);
      v64[((int64_t)k * nnz + e) * NC + c] = v;
    }
  if (bad) atomicAdd(nonfinite, (unsigned long long)bad);
}

// Natural cubic spline second derivatives of ncol real columns stored knot-major,
// y[k * ncol + col]: Thomas elimination along the grid.  The elimination factors
// depend on the grid only and are formed once per workgroup in LDS; the forward
// sweep's values are held in y2 until the backward sweep overwrites them.
constexpr int SPL_KMAX = 2048;
__global__ void __launch_bounds__(256)
csr_spline(const double* __restrict__ y, const double* __restrict__ x, int K, int64_t ncol,
           double* __restrict__ y2) {
  __shared__ double den[SPL_KMAX], cp[SPL_KMAX];
  if (threadIdx.x == 0) {
    double cprev = 0.0;
    for (int k = 1; k <= K - 2; ++k) {
      const double hl = x[k] - x[k - 1], hr = x[k + 1] - x[k];
      const double dn = (hl + hr) / 3.0 - (k > 1 ? hl / 6.0 * cprev : 0.0);
      den[k] = dn;
      cprev = hr / 6.0 / dn;
      cp[k] = cprev;
    }
  }
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  y2[c] = 0.0;
  y2[(int64_t)(K - 1) * ncol + c] = 0.0;
  double dprev = 0.0;
  for (int k = 1; k <= K - 2; ++k) {
    const double hl = x[k] - x[k - 1], hr = x[k + 1] - x[k];
    const double yl = y[(int64_t)(k - 1) * ncol + c], y0 = y[(int64_t)k * ncol + c],
                 yr = y[(int64_t)(k + 1) * ncol + c];
    const double rhs = (yr - y0) / hr - (y0 - yl) / hl;
    const double dk = (rhs - (k > 1 ? hl / 6.0 * dprev : 0.0)) / den[k];
    y2[(int64_t)k * ncol + c] = dk;
    dprev = dk;
  }
  double nxt = 0.0;
  for (int k = K - 2; k >= 1; --k) {
    const double v = y2[(int64_t)k * ncol + c] - cp[k] * nxt;
    y2[(int64_t)k * ncol + c] = v;
    nxt = v;
  }
}

// The largest |M_e - conj(M_p)| (p: the partner (m, n) of element e = (n, m))
// and the largest |M| over every knot, as the bit patterns of non-negative doubles.
__global__ void csr_partner_check(const double* __restrict__ v64, const int32_t* __restrict__ partner,
                                  int64_t nnz, int K, int NC,
                                  unsigned long long* __restrict__ maxdiff,
                                  unsigned long long* __restrict__ maxabs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dm = 0.0, am = 0.0;
  if (e < nnz) {
    const int64_t p = partner[e];
    for (int k = 0; k < K; ++k) {
      const double* a = v64 + ((int64_t)k * nnz + e) * NC;
      const double* b = v64 + ((int64_t)k * nnz + p) * NC;
      double d = fabs(a[0] - b[0]), m = fabs(a[0]);
      if (NC == 2) {
        d = fmax(d, fabs(a[1] + b[1]));
        m = fmax(m, fabs(a[1]));
      }
      dm = fmax(dm, d);
      am = fmax(am, m);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    dm = fmax(dm, __shfl_xor(dm, off, 64));
    am = fmax(am, __shfl_xor(am, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(maxdiff, (unsigned long long)__double_as_longlong(dm));
    atomicMax(maxabs, (unsigned long long)__double_as_longlong(am));
  }
}

template <typename S>
__global__ void csr_cast(const double* __restrict__ in, int64_t n, S* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (S)in[i];
}

// ---- columns schedule ------------------------------------------------------------

struct ColStage {
  double om;       // dPhi/dt at the stage
  double w[4];     // spline value weights at the stage's R
  int32_t k;       // spline interval
  int32_t pad[5];
};

struct ColArgs {
  const DevSystem* systems;
  const TrajIn* traj;       // records in group order
  const ColGroup* groups;   // [G]
  int G, N, CT;
  int64_t nchunk;           // row chunks of one group
  ColStage* st;             // stage records, group g from groups[g].stage_off
  double* fin;              // [G][8]: R, Phi, P_R, P_Phi, theta, P_theta, E0, E1
  int* gstatus;             // [G]
  double2* A0;              // [G][N][CT] amplitudes at the start of the step
  double2* ACC;             // [G][N][CT] RK4 accumulator
  double2* CUR[2];          // [G][N][CT] stage amplitudes (input, next)
  void* C[2];               // [G][N][CT] phased stage amplitudes in the table precision
  double* part;             // [G][nchunk][CT] partial norms
};

__device__ __forceinline__ int64_t cidx(const ColArgs& a, int g, int n, int col) {
  return ((int64_t)g * a.N + n) * a.CT + col;
}

// Stage times of step j: t_j + cf_s h with t_j = t0 + j h (Eq. 4's time, RK4 stages).
__device__ __forceinline__ double col_cf(int s) { return s == 0 ? 0.0 : (s == 3 ? 1.0 : 0.5); }

// The classical path of every group (AT: Eqs. 7-9 with the driving potential's
// force, no torque), RK4 with the records of every stage; one thread per group.
__global__ void col_path(ColArgs a) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.G) return;
  const ColGroup gr = a.groups[g];
  const TrajIn tj = a.traj[gr.first];
  const DevSystem sy = a.systems[tj.sys];
  const double mu = sy.mu, h = tj.dt;
  double y[4], theta = 0.5 * M_PI, ptheta = 0.0;
  if (tj.flags & TRAJ_HAS_C0) {
    y[0] = tj.c0[0]; theta = tj.c0[1]; y[1] = tj.c0[2]; y[2] = tj.c0[3]; ptheta = tj.c0[4];
    y[3] = tj.c0[5];
  } else {
    const double kk = sqrt(2.0 * mu * tj.E_coll);
    const double pphi = tj.b * kk;
    y[0] = tj.R0; y[1] = 0.0;
    y[2] = -sqrt(2.0 * mu * tj.E_coll - pphi * pphi / (tj.R0 * tj.R0));
    y[3] = pphi;
  }
  int status = 0;
  auto U_of = [&](const Spl& sp) {
    const int k = sp.k;
    return sp.w0 * sy.drv[k] + sp.w1 * sy.drv[k + 1] + sp.w2 * sy.drv2[k] + sp.w3 * sy.drv2[k + 1];
  };
  auto energy = [&](const double (&ys)[4]) {
    const Spl sp = spline_at(sy.R, sy.K, ys[0], sy.R_inv_h);
    return ys[2] * ys[2] / (2.0 * mu) + ys[3] * ys[3] / (2.0 * mu * ys[0] * ys[0]) + U_of(sp);
  };
  auto deriv = [&](const double (&ys)[4], double (&ky)[4], ColStage* rec) {
    const Spl sp = spline_at(sy.R, sy.K, ys[0], sy.R_inv_h);
    if (sp.below) status |= ST_BELOW_GRID;
    const int k = sp.k;
    const double dU = sp.d0 * sy.drv[k] + sp.d1 * sy.drv[k + 1] + sp.d2 * sy.drv2[k] +
                      sp.d3 * sy.drv2[k + 1];
    const double R = ys[0];
    ky[0] = ys[2] / mu;
    ky[1] = ys[3] / (mu * R * R);
    ky[2] = -dU + ys[3] * ys[3] / (mu * R * R * R);
    ky[3] = 0.0;
    ColStage r{};
    r.om = ky[1];
    r.w[0] = sp.w0; r.w[1] = sp.w1; r.w[2] = sp.w2; r.w[3] = sp.w3;
    r.k = k;
    *rec = r;
  };
  const double E0 = energy(y);
  ColStage* rec = a.st + gr.stage_off;
  for (int64_t j = 0; j < gr.n_steps; ++j) {
    double k1[4], k2[4], k3[4], k4[4], ys[4];
    deriv(y, k1, rec + 4 * j);
    for (int i = 0; i < 4; ++i) ys[i] = fma(0.5 * h, k1[i], y[i]);
    deriv(ys, k2, rec + 4 * j + 1);
    for (int i = 0; i < 4; ++i) ys[i] = fma(0.5 * h, k2[i], y[i]);
    deriv(ys, k3, rec + 4 * j + 2);
    for (int i = 0; i < 4; ++i) ys[i] = fma(h, k3[i], y[i]);
    deriv(ys, k4, rec + 4 * j + 3);
    for (int i = 0; i < 4; ++i) {
      const double acc = k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i];
      y[i] = fma(h / 6.0, acc, y[i]);
    }
  }
  // the end state's interval is checked too (the results are evaluated there)
  if (spline_at(sy.R, sy.K, y[0], sy.R_inv_h).below) status |= ST_BELOW_GRID;
  double* f = a.fin + (int64_t)g * 8;
  f[0] = y[0]; f[1] = y[1]; f[2] = y[2]; f[3] = y[3]; f[4] = theta; f[5] = ptheta;
  f[6] = E0; f[7] = energy(y);
  a.gstatus[g] = status;
}

template <typename CS> struct CV;
template <> struct CV<double> {
  using T = double2;
  __device__ static double2 make(double x, double y) { return make_double2(x, y); }
};
template <> struct CV<float> {
  using T = float2;
  __device__ static float2 make(double x, double y) { return make_float2((float)x, (float)y); }
};

// Start amplitudes of every column (a0, or the initial channel), the stage-0
// input and its phased form at t0.
template <typename CS>
__global__ void __launch_bounds__(CB) col_init(ColArgs a, const double* __restrict__ a0_all) {
  const int64_t item = (int64_t)blockIdx.x * CW + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = (int)(item / a.N), n = (int)(item % a.N);
  if (g >= a.G) return;
  const ColGroup gr = a.groups[g];
  const TrajIn t0r = a.traj[gr.first];
  const DevSystem sy = a.systems[t0r.sys];
  double sn, cs;
  sincos(sy.E[n] * t0r.t0, &sn, &cs);
  using C2 = typename CV<CS>::T;
  C2* c = (C2*)a.C[0];
  for (int col = lane; col < a.CT; col += 64) {
    double2 v = make_double2(0.0, 0.0);
    if (col < gr.count) {
      const TrajIn tj = a.traj[gr.first + col];
      if (tj.flags & TRAJ_HAS_A0) v = ((const double2*)a0_all)[tj.amp_off + n];
      else if (n == tj.init_channel) v = make_double2(1.0, 0.0);
    }
    const int64_t o = cidx(a, g, n, col);
    a.A0[o] = v;
    a.CUR[0][o] = v;
    a.ACC[o] = make_double2(0.0, 0.0);
    c[o] = CV<CS>::make(cs * v.x + sn * v.y, cs * v.y - sn * v.x);
  }
}

__device__ __forceinline__ double rl(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// One RK4 stage s of step j for every group still running (see the top of the
// file).  S: table precision; CPLX: complex tables; CS: precision of the phased
// amplitudes (and of the products: FP32 products over one 64-element chunk,
// then FP64 sums).  in = stage parity.
template <typename S, bool CPLX, typename CS>
__global__ void __launch_bounds__(CB)
col_stage(ColArgs a, int64_t j, int s) {
  const int64_t per = (a.G * a.nchunk + NXCD - 1) / NXCD;
  const int64_t pos = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (blockIdx.x / NXCD >= per || pos >= (int64_t)a.G * a.nchunk) return;
  const int g = (int)(pos / a.nchunk);
  const int64_t chunk = pos % a.nchunk;
  const ColGroup gr = a.groups[g];
  if (j >= gr.n_steps) return;
  const TrajIn t0r = a.traj[gr.first];
  const DevSystem sy = a.systems[t0r.sys];
  const ColStage rec = a.st[gr.stage_off + 4 * j + s];
  const double h = t0r.dt;
  const double tj = t0r.t0 + (double)j * h;
  const double t = tj + col_cf(s) * h;
  const double tn = s < 3 ? tj + col_cf(s + 1) * h : t0r.t0 + (double)(j + 1) * h;
  const int in = s & 1, outb = in ^ 1;
  using C2 = typename CV<CS>::T;
  const C2* __restrict__ cin = (const C2*)a.C[in];
  C2* __restrict__ cout = (C2*)a.C[outb];
  const double2* __restrict__ curin = a.CUR[in];
  double2* __restrict__ curout = a.CUR[outb];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c0 = 2 * lane;
  const bool act = c0 < a.CT;
  const int64_t nnz = sy.knot_stride;
  constexpr int NC = CPLX ? 2 : 1;
  const S* __restrict__ V0 = (const S*)sy.M + (int64_t)rec.k * nnz * NC;
  const S* __restrict__ V1 = V0 + nnz * NC;
  const S* __restrict__ D0 = (const S*)sy.M2 + (int64_t)rec.k * nnz * NC;
  const S* __restrict__ D1 = D0 + nnz * NC;
  const double w0 = rec.w[0], w1 = rec.w[1], w2 = rec.w[2], w3 = rec.w[3];
  const C2* cg = cin + (int64_t)g * a.N * a.CT + (act ? c0 : 0);
  for (int r = 0; r < ROWS_PER_WAVE; ++r) {
    const int64_t nl = chunk * ROWS_PER_WG + (int64_t)wave * ROWS_PER_WAVE + r;
    if (nl >= a.N) break;
    const int n = (int)nl;
    const int rs = sy.csr_row[n], re = sy.csr_row[n + 1];
    double y0x = 0.0, y0y = 0.0, y1x = 0.0, y1y = 0.0;
    for (int e0 = rs; e0 < re; e0 += 64) {
      const int e = e0 + lane;
      int m = n;
      double mr = 0.0, mi = 0.0;
      if (e < re) {
        m = sy.csr_col[e];
        mr = w0 * (double)V0[(int64_t)e * NC] + w1 * (double)V1[(int64_t)e * NC] +
             w2 * (double)D0[(int64_t)e * NC] + w3 * (double)D1[(int64_t)e * NC];
        if constexpr (CPLX)
          mi = w0 * (double)V0[(int64_t)e * NC + 1] + w1 * (double)V1[(int64_t)e * NC + 1] +
               w2 * (double)D0[(int64_t)e * NC + 1] + w3 * (double)D1[(int64_t)e * NC + 1];
      }
      const int cnt = min(64, re - e0);
      CS p0x = 0, p0y = 0, p1x = 0, p1y = 0;
      for (int i = 0; i < cnt; i += GATHER_UNROLL) {
        C2 g0[GATHER_UNROLL], g1[GATHER_UNROLL];
        CS br[GATHER_UNROLL], bi[GATHER_UNROLL];
#pragma unroll
        for (int u = 0; u < GATHER_UNROLL; ++u) {
          // entries past the chunk's count read the row's own amplitudes and add zero
          const int l = min(i + u, cnt - 1);
          const int mu = __builtin_amdgcn_readlane(m, l);
          const double vr = i + u < cnt ? rl(mr, l) : 0.0;
          br[u] = (CS)vr;
          if constexpr (CPLX) bi[u] = (CS)(i + u < cnt ? rl(mi, l) : 0.0);
          const C2* src = cg + (int64_t)mu * a.CT;
          if (act) {
            g0[u] = src[0];
            g1[u] = src[1];
          } else {
            g0[u] = CV<CS>::make(0.0, 0.0);
            g1[u] = CV<CS>::make(0.0, 0.0);
          }
        }
#pragma unroll
        for (int u = 0; u < GATHER_UNROLL; ++u) {
          p0x += br[u] * g0[u].x; p0y += br[u] * g0[u].y;
          p1x += br[u] * g1[u].x; p1y += br[u] * g1[u].y;
          if constexpr (CPLX) {
            p0x -= bi[u] * g0[u].y; p0y += bi[u] * g0[u].x;
            p1x -= bi[u] * g1[u].y; p1y += bi[u] * g1[u].x;
          }
        }
      }
      y0x += (double)p0x; y0y += (double)p0y; y1x += (double)p1x; y1y += (double)p1y;
    }
    if (!act) continue;
    double sn, cs;
    sincos(sy.E[n] * t, &sn, &cs);
    double sn2, cs2;
    sincos(sy.E[n] * tn, &sn2, &cs2);
    const double yv[2][2] = {{y0x, y0y}, {y1x, y1y}};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int col = c0 + q;
      if (col >= a.CT) break;
      // J_x a of this row (couples states of equal energy, Eq. 5)
      double xx = 0.0, xy = 0.0;
      for (int w = 0; w < sy.jx_w; ++w) {
        const int jc = sy.jx_col[(int64_t)n * sy.jx_w + w];
        const double jv = sy.jx_val[(int64_t)n * sy.jx_w + w];
        const double2 av = curin[cidx(a, g, jc, col)];
        xx = fma(jv, av.x, xx);
        xy = fma(jv, av.y, xy);
      }
      // da/dt = -i (e^{iE_n t} (M c)_n + Phidot (J_x a)_n)
      const double Gx = cs * yv[q][0] - sn * yv[q][1] + rec.om * xx;
      const double Gy = cs * yv[q][1] + sn * yv[q][0] + rec.om * xy;
      const double fx = Gy, fy = -Gx;
      const int64_t o = cidx(a, g, n, col);
      const double2 av0 = a.A0[o];
      double2 nx;
      if (s == 0) {
        a.ACC[o] = make_double2(fx, fy);
        nx = make_double2(fma(0.5 * h, fx, av0.x), fma(0.5 * h, fy, av0.y));
      } else if (s < 3) {
        const double2 ac = a.ACC[o];
        a.ACC[o] = make_double2(fma(2.0, fx, ac.x), fma(2.0, fy, ac.y));
        const double cfn = s == 1 ? 0.5 * h : h;
        nx = make_double2(fma(cfn, fx, av0.x), fma(cfn, fy, av0.y));
      } else {
        const double2 ac = a.ACC[o];
        nx = make_double2(fma(h / 6.0, ac.x + fx, av0.x), fma(h / 6.0, ac.y + fy, av0.y));
        a.A0[o] = nx;
      }
      curout[o] = nx;
      cout[o] = CV<CS>::make(cs2 * nx.x + sn2 * nx.y, cs2 * nx.y - sn2 * nx.x);
    }
  }
}

// Final probabilities and amplitudes of every column, and partial norms per
// chunk of rows (summed in order by col_fin).
__global__ void __launch_bounds__(CB) col_out(ColArgs a, TrajOut out) {
  const int64_t item = (int64_t)blockIdx.x * CW + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= (int64_t)a.G * a.nchunk) return;
  const int g = (int)(item / a.nchunk);
  const int64_t chunk = item % a.nchunk;
  const ColGroup gr = a.groups[g];
  for (int col = lane; col < a.CT; col += 64) {
    double nrm = 0.0;
    const bool real = col < gr.count;
    const TrajIn tj = a.traj[gr.first + (real ? col : 0)];
    for (int r = 0; r < ROWS_PER_WG; ++r) {
      const int64_t n = chunk * ROWS_PER_WG + r;
      if (n >= a.N) break;
      const double2 v = a.A0[cidx(a, g, (int)n, col)];
      const double p = v.x * v.x + v.y * v.y;
      nrm += p;
      if (real) {
        if (out.P) out.P[tj.amp_off + n] = p;
        if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = v;
      }
    }
    a.part[((int64_t)g * a.nchunk + chunk) * a.CT + col] = nrm;
  }
}

// Per column: the norm (partials summed in row order), the path's end state and
// diagnostics (AT: the driven energy P_R^2/2mu + P_Phi^2/(2 mu R^2) + U(R) and P_Phi).
__global__ void col_fin(ColArgs a, TrajOut out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = (int)(i / COL_MAX), col = (int)(i % COL_MAX);
  if (g >= a.G) return;
  const ColGroup gr = a.groups[g];
  if (col >= gr.count) return;
  const TrajIn tj = a.traj[gr.first + col];
  double nrm = 0.0;
  for (int64_t c = 0; c < a.nchunk; ++c) nrm += a.part[((int64_t)g * a.nchunk + c) * a.CT + col];
  const double* f = a.fin + (int64_t)g * 8;
  const int64_t id = tj.id;
  if (out.classical) {
    double* o = out.classical + id * 6;
    o[0] = f[0]; o[1] = f[4]; o[2] = f[1]; o[3] = f[2]; o[4] = f[5]; o[5] = f[3];
  }
  if (out.t_final) out.t_final[id] = tj.t0 + (double)gr.n_steps * tj.dt;
  if (out.steps) out.steps[id] = gr.n_steps;
  if (out.rejects) out.rejects[id] = 0;
  if (out.status) out.status[id] = a.gstatus[g];
  if (out.norm_err) out.norm_err[id] = nrm - 1.0;
  if (out.energy_err) out.energy_err[id] = (f[7] - f[6]) / fabs(f[6]);
  if (out.angmom_err) out.angmom_err[id] = 0.0;   // no torque: P_Phi is constant
}

}  // namespace

// ---- host ------------------------------------------------------------------------

hipError_t launch_coo_gather(const double* values, int64_t ld, const int32_t* perm, int64_t nnz,
                             int K, int NC, double* v64, unsigned long long* nonfinite,
                             hipStream_t s) {
  coo_gather<<<(unsigned)((nnz + 255) / 256), 256, 0, s>>>(values, ld, perm, nnz, K, NC, v64,
                                                           nonfinite);
  return hipGetLastError();
}

hipError_t launch_csr_spline(const double* y, const double* x, int K, int64_t ncol, double* y2,
                             hipStream_t s) {
  csr_spline<<<(unsigned)((ncol + 255) / 256), 256, 0, s>>>(y, x, K, ncol, y2);
  return hipGetLastError();
}

hipError_t launch_csr_partner_check(const double* v64, const int32_t* partner, int64_t nnz, int K,
                                    int NC, unsigned long long* maxdiff,
                                    unsigned long long* maxabs, hipStream_t s) {
  csr_partner_check<<<(unsigned)((nnz + 255) / 256), 256, 0, s>>>(v64, partner, nnz, K, NC,
                                                                  maxdiff, maxabs);
  return hipGetLastError();
}

hipError_t launch_csr_cast_f32(const double* in, int64_t n, float* out, hipStream_t s) {
  csr_cast<float><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, n, out);
  return hipGetLastError();
}

size_t columns_workspace_bytes(int G, int N, int CT, int64_t stages, bool fp32) {
  const size_t v = (size_t)G * N * CT;
  const int64_t nchunk = (N + ROWS_PER_WG - 1) / ROWS_PER_WG;
  size_t b = 0;
  b += al((size_t)G * sizeof(ColGroup));
  b += al((size_t)std::max<int64_t>(stages, 1) * sizeof(ColStage));
  b += al((size_t)G * 8 * 8) + al((size_t)G * 4);
  b += 4 * al(v * 16);
  b += 2 * al(v * (fp32 ? 8 : 16));
  b += al((size_t)G * nchunk * CT * 8);
  return b;
}

hipError_t run_columns(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                       const std::vector<ColGroup>& groups, int CT, const double* d_a0,
                       TrajOut out, void* wsp, hipStream_t s) {
  const int G = (int)groups.size();
  const int N = hs.N;
  const bool fp32 = dtype_fp32(hs.dtype);
  int64_t stages = 0, nmax = 0;
  for (const ColGroup& g : groups) {
    stages = std::max(stages, g.stage_off + 4 * g.n_steps);
    nmax = std::max(nmax, g.n_steps);
  }
  ColArgs a{};
  a.systems = d_systems;
  a.traj = d_traj;
  a.G = G;
  a.N = N;
  a.CT = CT;
  a.nchunk = (N + ROWS_PER_WG - 1) / ROWS_PER_WG;
  char* p = (char*)wsp;
  auto take = [&](size_t bytes) { void* q = p; p += al(bytes); return q; };
  ColGroup* dg = (ColGroup*)take((size_t)G * sizeof(ColGroup));
  a.groups = dg;
  a.st = (ColStage*)take((size_t)std::max<int64_t>(stages, 1) * sizeof(ColStage));
  a.fin = (double*)take((size_t)G * 8 * 8);
  a.gstatus = (int*)take((size_t)G * 4);
  const size_t v = (size_t)G * N * CT;
  a.A0 = (double2*)take(v * 16);
  a.ACC = (double2*)take(v * 16);
  a.CUR[0] = (double2*)take(v * 16);
  a.CUR[1] = (double2*)take(v * 16);
  a.C[0] = take(v * (fp32 ? 8 : 16));
  a.C[1] = take(v * (fp32 ? 8 : 16));
  a.part = (double*)take((size_t)G * a.nchunk * CT * 8);
  hipError_t e;
  if ((e = hipMemcpyAsync(dg, groups.data(), (size_t)G * sizeof(ColGroup), hipMemcpyHostToDevice,
                          s)) != hipSuccess)
    return e;
  col_path<<<(G + 63) / 64, 64, 0, s>>>(a);
  const unsigned init_grid = (unsigned)(((int64_t)G * N + CW - 1) / CW);
  if (fp32) col_init<float><<<init_grid, CB, 0, s>>>(a, d_a0);
  else col_init<double><<<init_grid, CB, 0, s>>>(a, d_a0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t items = (int64_t)G * a.nchunk;
  const unsigned grid = (unsigned)((items + NXCD - 1) / NXCD * NXCD);
  for (int64_t j = 0; j < nmax; ++j)
    for (int st = 0; st < 4; ++st) {
      if (hs.dtype == R64) col_stage<double, false, double><<<grid, CB, 0, s>>>(a, j, st);
      else if (hs.dtype == C128) col_stage<double, true, double><<<grid, CB, 0, s>>>(a, j, st);
      else if (hs.dtype == R32) col_stage<float, false, float><<<grid, CB, 0, s>>>(a, j, st);
      else col_stage<float, true, float><<<grid, CB, 0, s>>>(a, j, st);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  col_out<<<(unsigned)((items + CW - 1) / CW), CB, 0, s>>>(a, out);
  col_fin<<<(unsigned)(((int64_t)G * COL_MAX + 255) / 256), 256, 0, s>>>(a, out);
  return hipGetLastError();
}

}  // namespace mqct

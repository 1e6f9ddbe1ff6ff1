// Fixed-step RK4 propagation of Ehrenfest mean-field trajectories, one
// workgroup per trajectory with the whole step loop inside the kernel.
//
// Right-hand side (paper Section II, Eqs. 5 and 7-10, collision plane
// Theta = pi/2):
//   c_m   = e^{-i E_m t} a_m                      (Eq. 4 phase, factorised per channel)
//   u     = M(R) c,  v = M'(R) c                  (one pass over the four spline slices
//                                                  M_k, M_{k+1}, M2_k, M2_{k+1})
//   y_n   = e^{+i E_n t} u_n                      (= sum_m M_nm e^{i(E_n - E_m)t} a_m)
//   x     = J_x a
//   da/dt = -i y - i Phidot x                     (Eq. 5, Coriolis generator -i Phidot J_x)
//   dR/dt = P_R/mu,  dPhi/dt = Phidot = P_Phi/(mu R^2)                 (Eqs. 7, 8)
//   dP_R/dt   = -Re(c^H v) + P_Phi^2/(mu R^3)                           (Eq. 9)
//   dP_Phi/dt = 2 Im(x^H y) = -i <[J_x, V]>                             (Eq. 10)
//
// Work split: lane n of the workgroup owns output rows n (16-byte column
// groups of the stored tables).  Because every knot's matrix is Hermitian,
// column n of the stored matrix is conj(row n), so all lanes of a wave stream
// one stored row m contiguously while each keeps its own row sums in registers;
// no cross-lane reduction is needed for the matvec.  c lives in LDS and is read
// as a broadcast.  Only the two mean-field scalars (force, torque) and the
// diagnostics are reduced across the workgroup (wave shuffles, then LDS).
//
// Precision: the FP64 tables use FP64 throughout.  The FP32 tables (R32/C64)
// multiply in FP32 and accumulate in FP32 over chunks of 64 stored rows, then
// add the chunk sums into FP64; phases (E t), spline weights, the classical
// state and every RK accumulator stay FP64.
#include "internal.h"

#include <math.h>

namespace mqct {

namespace {

template <int DT> struct Tr;
template <> struct Tr<C128> {
  using S = double; using L = double2; using CS = double2;
  static constexpr int VEC = 1; static constexpr bool CPLX = true;
};
template <> struct Tr<C64> {
  using S = float; using L = float4; using CS = float2;
  static constexpr int VEC = 2; static constexpr bool CPLX = true;
};
template <> struct Tr<R64> {
  using S = double; using L = double2; using CS = double2;
  static constexpr int VEC = 2; static constexpr bool CPLX = false;
};
template <> struct Tr<R32> {
  using S = float; using L = float4; using CS = float2;
  static constexpr int VEC = 4; static constexpr bool CPLX = false;
};

constexpr int CHUNK = 64;   // stored rows per FP32 partial sum

// Spline interval and weights at R (natural cubic spline on knots x[0..K-1]):
// value = w0 y_k + w1 y_{k+1} + w2 y2_k + w3 y2_{k+1}; derivative with d0..d3.
// Above the last knot the value is held and the slope is zero; below the first
// knot the spline is continued linearly (and the trajectory flagged).
struct Spl {
  int k;
  bool below;
  double w0, w1, w2, w3, d0, d1, d2, d3;
};

__device__ __forceinline__ Spl spline_at(const double* __restrict__ x, int K, double R) {
  Spl s;
  s.below = R < x[0];
  if (R > x[K - 1]) {
    s.k = K - 2;
    s.w0 = 0.0; s.w1 = 1.0; s.w2 = 0.0; s.w3 = 0.0;
    s.d0 = 0.0; s.d1 = 0.0; s.d2 = 0.0; s.d3 = 0.0;
    return s;
  }
  int lo = 0;
  if (!s.below) {
    int hi = K - 2;           // largest k in [0, K-2] with x[k] <= R
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (x[mid] <= R) lo = mid; else hi = mid - 1;
    }
  }
  s.k = lo;
  const double h = x[lo + 1] - x[lo];
  if (s.below) {
    const double dR = R - x[0];
    s.d0 = -1.0 / h; s.d1 = 1.0 / h; s.d2 = -2.0 * h / 6.0; s.d3 = -h / 6.0;
    s.w0 = 1.0 + dR * s.d0; s.w1 = dR * s.d1; s.w2 = dR * s.d2; s.w3 = dR * s.d3;
    return s;
  }
  const double A = (x[lo + 1] - R) / h, B = 1.0 - A;
  s.w0 = A; s.w1 = B;
  s.w2 = (A * A * A - A) * (h * h / 6.0);
  s.w3 = (B * B * B - B) * (h * h / 6.0);
  s.d0 = -1.0 / h; s.d1 = 1.0 / h;
  s.d2 = -(3.0 * A * A - 1.0) * (h / 6.0);
  s.d3 = (3.0 * B * B - 1.0) * (h / 6.0);
  return s;
}

// Buffer resource over one knot slice of a table: the base and size live in
// scalar registers and every lane supplies only a 32-bit byte offset (a knot
// slice is far below 4 GiB).  Reads past `bytes` return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(const void* p, uint32_t bytes) {
  uint64_t v = (uint64_t)p;
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  void* q = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, (int)bytes, 0x00020000);
}

template <typename L>
__device__ __forceinline__ L load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(L, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

__device__ __forceinline__ double uni(double x) {
  // the value is identical in every lane: keep it in scalar registers
  int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

template <int NW>
__device__ __forceinline__ void block_sum6(double (&v)[6], double* red) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) red[w * 8 + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += red[q * 8 + i];
    v[i] = uni(s);
  }
}

// Sums produced by one right-hand-side evaluation.
struct Sums {
  double force;    // Re(c^H v)
  double torque;   // Im((J_x c)^H u)  = Im(x^H y)
  double vexp;     // Re(c^H u) = <V>
  double erot;     // sum E_n |a_n|^2
  double norm;     // sum |a_n|^2
  double jx;       // Re(c^H J_x c) = Re(a^H J_x a)
};

// Complex accumulation of u += conj(val) c and v += conj(der) c for one element
// (complex tables) or u += val c, v += der c (real tables).
template <bool CPLX, typename F, typename F2>
__device__ __forceinline__ void elem(F2& u, F2& v, F s0r, F s0i, F s1r, F s1i, F s2r, F s2i,
                                     F s3r, F s3i, const F (&w)[4], const F (&d)[4], F2 c) {
  if constexpr (CPLX) {
    F vr = w[0] * s0r + w[1] * s1r + w[2] * s2r + w[3] * s3r;
    F vi = w[0] * s0i + w[1] * s1i + w[2] * s2i + w[3] * s3i;
    F dr = d[0] * s0r + d[1] * s1r + d[2] * s2r + d[3] * s3r;
    F di = d[0] * s0i + d[1] * s1i + d[2] * s2i + d[3] * s3i;
    u.x += vr * c.x + vi * c.y;
    u.y += vr * c.y - vi * c.x;
    v.x += dr * c.x + di * c.y;
    v.y += dr * c.y - di * c.x;
  } else {
    F vr = w[0] * s0r + w[1] * s1r + w[2] * s2r + w[3] * s3r;
    F dr = d[0] * s0r + d[1] * s1r + d[2] * s2r + d[3] * s3r;
    u.x += vr * c.x;
    u.y += vr * c.y;
    v.x += dr * c.x;
    v.y += dr * c.y;
  }
}

template <int DT, int BLOCK, int RPT>
struct Kern {
  using T = Tr<DT>;
  using S = typename T::S;
  using L = typename T::L;
  using CS = typename T::CS;
  static constexpr int VEC = T::VEC;
  static constexpr int NR = RPT * VEC;
  static constexpr int NW = BLOCK / 64;
  static constexpr bool FP32 = (DT == C64 || DT == R32);
  static constexpr bool CPLX = T::CPLX;
  static constexpr int NCOMP = CPLX ? 2 : 1;
  static constexpr int UNR = RPT >= 4 ? 1 : 4 / RPT;   // stored rows in flight per lane
  using F = typename std::conditional<FP32, float, double>::type;
  using F2 = typename std::conditional<FP32, float2, double2>::type;

  __device__ static int row(int r) { return (threadIdx.x + (r / VEC) * BLOCK) * VEC + (r % VEC); }

  // The VEC elements of one 16-byte load, as (re, im) pairs.
  __device__ static void split(const L& v, F (&re)[VEC], F (&im)[VEC]) {
    if constexpr (DT == C128) { re[0] = v.x; im[0] = v.y; }
    else if constexpr (DT == C64) { re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w; }
    else if constexpr (DT == R64) { re[0] = v.x; re[1] = v.y; im[0] = im[1] = 0.0; }
    else { re[0] = v.x; re[1] = v.y; re[2] = v.z; re[3] = v.w;
           im[0] = im[1] = im[2] = im[3] = 0.f; }
  }

  // One evaluation of the right-hand side at time ts for the stage amplitudes
  // a = a0 + cf * kk and classical stage state (R, P_R, P_Phi).  Overwrites kk
  // with da/dt; returns the reduced sums.
  __device__ static void eval(const DevSystem& sy, double ts, double R, double pphi, double cf,
                              const double2 (&a0)[NR], double2 (&kk)[NR], Sums& tot,
                              bool& below, CS* lds_c, double2* lds_c64, double* red) {
    const int N = sy.N, Npad = sy.Npad;
    const Spl sp = spline_at(sy.R, sy.K, R);
    below |= sp.below;
    const double phidot = uni(pphi / (sy.mu * R * R));

#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) {
        const double2 cur = make_double2(fma(cf, kk[r].x, a0[r].x), fma(cf, kk[r].y, a0[r].y));
        double sn, cs;
        sincos(sy.E[n] * ts, &sn, &cs);
        const double2 c = make_double2(cs * cur.x + sn * cur.y, cs * cur.y - sn * cur.x);
        if constexpr (FP32) lds_c[n] = make_float2((float)c.x, (float)c.y);
        lds_c64[n] = c;
      }
    }
    __syncthreads();

    // fused spline-evaluate + complex matvec over the four slices
    const int64_t ks = sy.knot_stride;
    const uint32_t sbytes = (uint32_t)(ks * NCOMP * (int64_t)sizeof(S));
    const auto rs0 = slice_rsrc((const S*)sy.M + (int64_t)sp.k * ks * NCOMP, sbytes);
    const auto rs1 = slice_rsrc((const S*)sy.M + (int64_t)(sp.k + 1) * ks * NCOMP, sbytes);
    const auto rs2 = slice_rsrc((const S*)sy.M2 + (int64_t)sp.k * ks * NCOMP, sbytes);
    const auto rs3 = slice_rsrc((const S*)sy.M2 + (int64_t)(sp.k + 1) * ks * NCOMP, sbytes);
    const int ngroups = Npad / VEC;   // 16-byte groups per stored row
    const F w[4] = {(F)uni(sp.w0), (F)uni(sp.w1), (F)uni(sp.w2), (F)uni(sp.w3)};
    const F d[4] = {(F)uni(sp.d0), (F)uni(sp.d1), (F)uni(sp.d2), (F)uni(sp.d3)};

    double2 U[NR], V[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) { U[r] = make_double2(0.0, 0.0); V[r] = make_double2(0.0, 0.0); }

    for (int m0 = 0; m0 < N; m0 += (FP32 ? CHUNK : N)) {
      const int m1 = FP32 ? min(N, m0 + CHUNK) : N;
      F2 pu[NR], pv[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        pu[r].x = pu[r].y = pv[r].x = pv[r].y = (F)0;
      }
#pragma unroll UNR
      for (int m = m0; m < m1; ++m) {
        const CS cm = lds_c[m];
        const uint32_t rowoff = (uint32_t)m * (uint32_t)ngroups * 16u;
        // No lane guard: a lane whose column group lies past the last one reads
        // into the next stored row (or past the slice, which returns zero) and
        // its sums are never used, so the loads of consecutive m stay in flight
        // together.
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const uint32_t off = rowoff + (uint32_t)(threadIdx.x + j * BLOCK) * 16u;
          const L v0 = load16<L>(rs0, off);
          const L v1 = load16<L>(rs1, off);
          const L v2 = load16<L>(rs2, off);
          const L v3 = load16<L>(rs3, off);
          F r0[VEC], i0[VEC], r1[VEC], i1[VEC], r2[VEC], i2[VEC], r3[VEC], i3[VEC];
          split(v0, r0, i0); split(v1, r1, i1); split(v2, r2, i2); split(v3, r3, i3);
#pragma unroll
          for (int q = 0; q < VEC; ++q)
            elem<CPLX, F, F2>(pu[j * VEC + q], pv[j * VEC + q], r0[q], i0[q], r1[q], i1[q],
                              r2[q], i2[q], r3[q], i3[q], w, d, cm);
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        U[r].x += (double)pu[r].x; U[r].y += (double)pu[r].y;
        V[r].x += (double)pv[r].x; V[r].y += (double)pv[r].y;
      }
    }

    // epilogue.  J_x couples only channels of equal energy, so
    // J_x a = e^{iE_n t} (J_x c) row by row, and with y = e^{iE t} u:
    //   Re(c^H v), Im(x^H y) = Im((J_x c)^H u), Re(c^H u), Re(a^H J_x a) = Re(c^H J_x c).
    double sums[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n >= N) { kk[r] = make_double2(0.0, 0.0); continue; }
      const double2 cur = make_double2(fma(cf, kk[r].x, a0[r].x), fma(cf, kk[r].y, a0[r].y));
      double sn, cs;
      sincos(sy.E[n] * ts, &sn, &cs);
      const double2 c = make_double2(cs * cur.x + sn * cur.y, cs * cur.y - sn * cur.x);
      double2 xc = make_double2(0.0, 0.0);
      for (int q = 0; q < sy.jx_w; ++q) {
        const int col = sy.jx_col[(int64_t)n * sy.jx_w + q];
        const double jv = sy.jx_val[(int64_t)n * sy.jx_w + q];
        const double2 cm = lds_c64[col];
        xc.x = fma(jv, cm.x, xc.x);
        xc.y = fma(jv, cm.y, xc.y);
      }
      const double2 u = U[r], v = V[r];
      sums[0] += c.x * v.x + c.y * v.y;
      sums[1] += xc.x * u.y - xc.y * u.x;
      sums[2] += c.x * u.x + c.y * u.y;
      const double pn = cur.x * cur.x + cur.y * cur.y;
      sums[3] += sy.E[n] * pn;
      sums[4] += pn;
      sums[5] += c.x * xc.x + c.y * xc.y;
      // da/dt = -i e^{iE_n t} (u + Phidot J_x c)
      const double gx = u.x + phidot * xc.x, gy = u.y + phidot * xc.y;
      const double yx = cs * gx - sn * gy, yy = cs * gy + sn * gx;
      kk[r] = make_double2(yy, -yx);
    }
    block_sum6<NW>(sums, red);
    tot.force = sums[0]; tot.torque = sums[1]; tot.vexp = sums[2];
    tot.erot = sums[3]; tot.norm = sums[4]; tot.jx = sums[5];
  }
};

// classical state carried by the kernel: R, Phi, P_R, P_Phi (Theta = pi/2 and
// P_Theta = 0 are constants of the planar motion)
template <int DT, int BLOCK, int RPT>
__global__ void __launch_bounds__(BLOCK)
rk4_gemv_kernel(const DevSystem* __restrict__ systems, const TrajIn* __restrict__ trajs,
                const double* __restrict__ a0_all, double2* __restrict__ cfull, TrajOut out) {
  using KK = Kern<DT, BLOCK, RPT>;
  using CS = typename KK::CS;
  constexpr int NR = KK::NR;
  extern __shared__ __align__(16) unsigned char smem[];
  const TrajIn tj = trajs[blockIdx.x];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N;
  const double mu = sy.mu;
  // LDS: c in the matvec precision, c in FP64 (the same array on the FP64
  // path), then the reduction scratch
  CS* lds_c = (CS*)smem;
  double2* lds_c64 = KK::FP32 ? (double2*)(smem + ((sy.Npad * sizeof(CS) + 15) & ~(size_t)15))
                              : (double2*)smem;
  double* red = (double*)(lds_c64 + sy.Npad);
  (void)cfull;

  double2 a0[NR], kk[NR], acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int n = KK::row(r);
    double2 v = make_double2(0.0, 0.0);
    if (n < N) {
      if (tj.flags & TRAJ_HAS_A0) v = ((const double2*)a0_all)[tj.amp_off + n];
      else if (n == tj.init_channel) v = make_double2(1.0, 0.0);
    }
    a0[r] = v;
    kk[r] = make_double2(0.0, 0.0);
  }
  // y = (R, Phi, P_R, P_Phi)
  double y[4], ky[4] = {0.0, 0.0, 0.0, 0.0}, ay[4];
  double theta = 0.5 * M_PI, ptheta = 0.0;
  if (tj.flags & TRAJ_HAS_C0) {
    y[0] = tj.c0[0]; theta = tj.c0[1]; y[1] = tj.c0[2]; y[2] = tj.c0[3]; ptheta = tj.c0[4];
    y[3] = tj.c0[5];
  } else {
    const double k = sqrt(2.0 * mu * tj.E_coll);
    const double pphi = tj.b * k;
    y[0] = tj.R0; y[1] = 0.0;
    y[2] = -sqrt(2.0 * mu * tj.E_coll - pphi * pphi / (tj.R0 * tj.R0));
    y[3] = pphi;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = uni(y[i]);

  const double h = tj.dt, t0 = tj.t0;
  bool below = false;
  int32_t status = 0;
  double E0 = 0.0, J0 = 0.0;
  bool first = true;
  Sums tot;
  int64_t j = 0;
  auto energy = [&](const double* ys, const Sums& s) {
    return ys[2] * ys[2] / (2.0 * mu) + ys[3] * ys[3] / (2.0 * mu * ys[0] * ys[0]) + s.erot +
           s.vexp;
  };
  for (; j < tj.n_steps; ++j) {
    const double t = t0 + (double)j * h;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) ay[i] = 0.0;
    for (int st = 0; st < 4; ++st) {
      const double cf = st == 0 ? 0.0 : (st == 3 ? h : 0.5 * h);
      const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
      double ys[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) ys[i] = fma(cf, ky[i], y[i]);
      KK::eval(sy, t + cf, ys[0], ys[3], cf, a0, kk, tot, below, lds_c, lds_c64, red);
      if (first) {
        E0 = energy(ys, tot);
        J0 = ys[3] - tot.jx;
        first = false;
      }
      const double R = ys[0];
      ky[0] = ys[2] / mu;
      ky[1] = ys[3] / (mu * R * R);
      ky[2] = -tot.force + ys[3] * ys[3] / (mu * R * R * R);
      ky[3] = 2.0 * tot.torque;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[r].x = fma(wgt, kk[r].x, acc[r].x);
        acc[r].y = fma(wgt, kk[r].y, acc[r].y);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) ay[i] = fma(wgt, ky[i], ay[i]);
    }
    const double h6 = h / 6.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      a0[r].x += h6 * acc[r].x;
      a0[r].y += h6 * acc[r].y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = uni(y[i] + h6 * ay[i]);
    if (!isfinite(tot.force) || !isfinite(tot.torque) || !isfinite(tot.norm) ||
        !isfinite(y[0]) || !isfinite(y[2]) || !isfinite(y[3])) {
      status |= ST_NONFINITE;
      ++j;
      break;
    }
  }
  // diagnostics at the final state (one more evaluation; its derivative is unused)
  const double tend = t0 + (double)j * h;
  {
    bool b2 = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = kk[r];
    KK::eval(sy, tend, y[0], y[3], 0.0, a0, acc, tot, b2, lds_c, lds_c64, red);
    if (first) {
      E0 = energy(y, tot);
      J0 = y[3] - tot.jx;
    }
  }
  if (below) status |= ST_BELOW_GRID;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int n = KK::row(r);
    if (n < N) {
      out.P[tj.amp_off + n] = a0[r].x * a0[r].x + a0[r].y * a0[r].y;
      if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = a0[r];
    }
  }
  if (threadIdx.x == 0) {
    const int64_t id = tj.id;
    if (out.classical) {
      double* o = out.classical + id * 6;
      o[0] = y[0]; o[1] = theta; o[2] = y[1]; o[3] = y[2]; o[4] = ptheta; o[5] = y[3];
    }
    if (out.t_final) out.t_final[id] = tend;
    if (out.steps) out.steps[id] = j;
    if (out.rejects) out.rejects[id] = 0;
    if (out.status) out.status[id] = status;
    if (out.norm_err) out.norm_err[id] = tot.norm - 1.0;
    if (out.energy_err) out.energy_err[id] = (energy(y, tot) - E0) / fabs(E0);
    if (out.angmom_err) out.angmom_err[id] = (y[3] - tot.jx) - J0;
  }
}

template <int DT, int BLOCK, int RPT>
hipError_t launch_one(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                      const double* d_a0, TrajOut out, int max_npad, hipStream_t s) {
  using CS = typename Tr<DT>::CS;
  const bool fp32 = DT == C64 || DT == R32;
  size_t lds = (fp32 ? ((max_npad * sizeof(CS) + 15) & ~(size_t)15) : 0) + (size_t)max_npad * 16 +
               (BLOCK / 64) * 8 * sizeof(double);
  auto kern = rk4_gemv_kernel<DT, BLOCK, RPT>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  for (int64_t first = 0; first < n_traj; first += 1 << 30) {
    int64_t cnt = n_traj - first < (1 << 30) ? n_traj - first : (1 << 30);
    kern<<<(unsigned)cnt, BLOCK, lds, s>>>(d_systems, d_traj + first, d_a0, nullptr, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int DT>
hipError_t launch_dt(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                     const double* d_a0, TrajOut out, int max_npad, hipStream_t s) {
  const int groups = max_npad / Tr<DT>::VEC;
  if (groups <= 64) return launch_one<DT, 64, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 128) return launch_one<DT, 128, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 256) return launch_one<DT, 256, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 512) return launch_one<DT, 512, 1>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 1024) return launch_one<DT, 512, 2>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 2048) return launch_one<DT, 512, 4>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  if (groups <= 4096) return launch_one<DT, 512, 8>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_rk4_gemv(const DevSystem* d_systems, const TrajIn* d_traj, int64_t n_traj,
                           const double* d_a0, TrajOut out, int dtype, int max_npad,
                           hipStream_t s) {
  switch (dtype) {
    case C128: return launch_dt<C128>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
    case C64: return launch_dt<C64>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
    case R64: return launch_dt<R64>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
    case R32: return launch_dt<R32>(d_systems, d_traj, n_traj, d_a0, out, max_npad, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mqct

// Right-hand side of the Ehrenfest mean-field equations for one trajectory,
// evaluated by one workgroup (shared by the per-trajectory RK4 kernel and the
// work-list schedule).
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
#pragma once

#include "device.h"

#include <math.h>

#include <type_traits>

namespace mqct {
namespace rhs {

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
  using S = float; using L = float2; using CS = float2;
  static constexpr int VEC = 2; static constexpr bool CPLX = false;
};

constexpr int CHUNK = 64;   // stored rows per FP32 partial sum
constexpr int JXB = 4;      // J_x widths up to this have a row's loads issued together

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
// The operations are written as explicit fused multiply-adds, so that every
// code path that calls this (dense rows, sparse slots in any batching) rounds
// alike and a sparse layout that keeps every nonzero gives the dense results
// bit for bit.
template <typename F>
__device__ __forceinline__ F fmaf_(F a, F b, F c) {
  if constexpr (sizeof(F) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

template <bool CPLX, typename F, typename F2>
__device__ __forceinline__ void elem(F2& u, F2& v, F s0r, F s0i, F s1r, F s1i, F s2r, F s2i,
                                     F s3r, F s3i, const F (&w)[4], const F (&d)[4], F2 c) {
  const F vr = fmaf_(w[3], s3r, fmaf_(w[2], s2r, fmaf_(w[1], s1r, w[0] * s0r)));
  const F dr = fmaf_(d[3], s3r, fmaf_(d[2], s2r, fmaf_(d[1], s1r, d[0] * s0r)));
  if constexpr (CPLX) {
    const F vi = fmaf_(w[3], s3i, fmaf_(w[2], s2i, fmaf_(w[1], s1i, w[0] * s0i)));
    const F di = fmaf_(d[3], s3i, fmaf_(d[2], s2i, fmaf_(d[1], s1i, d[0] * s0i)));
    u.x = fmaf_(vi, c.y, fmaf_(vr, c.x, u.x));
    u.y = fmaf_(-vi, c.x, fmaf_(vr, c.y, u.y));
    v.x = fmaf_(di, c.y, fmaf_(dr, c.x, v.x));
    v.y = fmaf_(-di, c.x, fmaf_(dr, c.y, v.y));
  } else {
    u.x = fmaf_(vr, c.x, u.x);
    u.y = fmaf_(vr, c.y, u.y);
    v.x = fmaf_(dr, c.x, v.x);
    v.y = fmaf_(dr, c.y, v.y);
  }
}


// LDS layout shared by the kernels (bytes):
//   c     [Npad] in the matvec precision (float2 or double2)
//   c64   [Npad] double2 (aliases c on the FP64 path)
//   red0  [16][8] doubles, red1 [16][8] doubles  (two reduction areas)
//   kcl   [8][4] doubles                        (classical stage derivatives of DP5)
//   part  [W][Npad] double4                     (split-row form only: each wave's
//                                                partial (u, v) before they are summed)
__host__ __device__ inline size_t lds_bytes(int npad, bool fp32, int split_waves = 0) {
  size_t c = fp32 ? (((size_t)npad * 8 + 15) & ~(size_t)15) : 0;
  return c + (size_t)npad * 16 + 2 * 16 * 8 * 8 + 8 * 4 * 8 + (size_t)split_waves * npad * 32;
}

template <int DT>
struct Lds {
  typename Tr<DT>::CS* c;
  double2* c64;
  double* red0;
  double* red1;
  double* kcl;
  double4* part;
  __device__ Lds(unsigned char* smem, int npad) {
    constexpr bool fp32 = (DT == C64 || DT == R32);
    c = (typename Tr<DT>::CS*)smem;
    c64 = fp32 ? (double2*)(smem + (((size_t)npad * 8 + 15) & ~(size_t)15)) : (double2*)smem;
    red0 = (double*)(c64 + npad);
    red1 = red0 + 16 * 8;
    kcl = red1 + 16 * 8;
    part = (double4*)(kcl + 8 * 4);
  }
};

// Right-hand side evaluated by one workgroup.  Row-split form (SPLIT = false):
// the BLOCK threads share out the output rows and every thread streams all N
// stored rows.  Split-row form (SPLIT = true): every wave holds all output rows
// (64 lanes x RPT groups) and streams only its 1/W share of the stored rows;
// the W partial sums meet in LDS and are added in a fixed order, so every wave
// ends with the same u and v and carries the trajectory's state redundantly.
// The split form shortens the dependent chain of loads W times: it serves
// trajectories that run alone on the device (latency-bound tails).
template <int DT, int BLOCK, int RPT, bool SPLIT = false>
struct Rhs {
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
  // stored rows in flight per lane (the split-row form streams fewer rows per
  // wave and is latency-bound, so it keeps more in flight)
  static constexpr int UNR = SPLIT ? (RPT >= 8 ? 1 : 8 / RPT) : (RPT >= 4 ? 1 : 4 / RPT);
  // sparse real tables: slots per batch whose row indices and table elements are
  // all requested before the first gather of c (their elements are small enough
  // to hold a batch in registers)
  static constexpr int ELLB = RPT >= 8 ? 1 : 8 / RPT;
  // keep each row's phase factor from the c computation for the epilogue
  static constexpr bool CPH = NR <= 4;
  using F = typename std::conditional<FP32, float, double>::type;
  using F2 = typename std::conditional<FP32, float2, double2>::type;

  static constexpr int ROWW = SPLIT ? 64 : BLOCK;   // threads that share out the rows
  __device__ static int rlane() { return SPLIT ? (int)(threadIdx.x & 63) : (int)threadIdx.x; }
  __device__ static int row(int r) { return (rlane() + (r / VEC) * ROWW) * VEC + (r % VEC); }

  // Sum NV values over the trajectory's rows, identical in every lane.  The
  // row-split form reduces over the workgroup; in the split-row form each wave
  // holds all rows, so a wave reduction suffices.  Both end with a barrier.
  template <int NV>
  __device__ static void reduce(double (&v)[NV], double* red) {
    if constexpr (SPLIT) {
      wave_sum<NV>(v);
      __syncthreads();
    } else {
      block_sum<NV, NW>(v, red);
    }
  }

  // The VEC elements of one 16-byte load, as (re, im) pairs.
  __device__ static void split(const L& v, F (&re)[VEC], F (&im)[VEC]) {
    if constexpr (DT == C128) { re[0] = v.x; im[0] = v.y; }
    else if constexpr (DT == C64) { re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w; }
    else if constexpr (DT == R64) { re[0] = v.x; re[1] = v.y; im[0] = im[1] = 0.0; }
    else { re[0] = v.x; re[1] = v.y; im[0] = im[1] = 0.f; }
  }

  // One evaluation of the right-hand side at time ts for the stage amplitudes
  // cur (this lane's rows) and classical stage values R, P_Phi.  Overwrites
  // cur with da/dt of this lane's rows and returns the workgroup sums in tot.
  // at: decoupled (AT) dynamics -- the trajectory feels the driving potential
  // U(R) instead of the mean field (paper Section III): the sums then carry
  // force = U'(R), torque = 0, and the conserved quantities become
  // P^2/2mu + P_Phi^2/(2 mu R^2) + U(R) (vexp = U, erot = 0) and P_Phi (jx = 0).
  __device__ static void eval(const DevSystem& sy, double ts, double R, double pphi,
                              double2 (&cur)[NR], Sums& tot, bool& below, const Lds<DT>& lds,
                              bool at = false) {
    const int N = sy.N, Npad = sy.Npad;
    const Spl sp = spline_at(sy.R, sy.K, R, sy.R_inv_h);
    below |= sp.below;
    const double phidot = uni(pphi / (sy.mu * R * R));

    double pcos[CPH ? NR : 1], psin[CPH ? NR : 1];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < N) {
        double sn, cs;
        sincos(sy.E[n] * ts, &sn, &cs);
        if constexpr (CPH) {
          pcos[r] = cs;
          psin[r] = sn;
        }
        const double2 c = make_double2(cs * cur[r].x + sn * cur[r].y,
                                       cs * cur[r].y - sn * cur[r].x);
        if constexpr (FP32) lds.c[n] = make_float2((float)c.x, (float)c.y);
        lds.c64[n] = c;
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

    // stored rows this thread streams: N rows of the dense tables, or the
    // ell_w slots of the sparse ones (slot q of column n holds stored row
    // col[q][n], so c is gathered per element instead of broadcast)
    const int nst = sy.ell_w > 0 ? sy.ell_w : N;
    int mb = 0, me = nst;
    if constexpr (SPLIT) {
      const int w = threadIdx.x >> 6;
      mb = (nst * w) / NW;
      me = (nst * (w + 1)) / NW;
    }
    const auto rcol = slice_rsrc(sy.ell_col, (uint32_t)((int64_t)nst * Npad * 4));
    auto stream = [&](auto sparse) {
      constexpr bool ELL = decltype(sparse)::value;
      for (int m0 = mb; m0 < me; m0 += (FP32 ? CHUNK : nst)) {
        const int m1 = FP32 ? min(me, m0 + CHUNK) : me;
        F2 pu[NR], pv[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          pu[r].x = pu[r].y = pv[r].x = pv[r].y = (F)0;
        }
        if constexpr (ELL && !CPLX) {
          // a batch of slots: every row index, then every table element, then
          // the gathers of c and the products (loads retire in order, so an
          // index load issued after a table load would wait for it)
          for (int mb0 = m0; mb0 < m1; mb0 += ELLB) {
            int ci[ELLB][RPT][VEC];
            L tv[ELLB][RPT][4];
#pragma unroll
            for (int u = 0; u < ELLB; ++u) {
              const int m = min(mb0 + u, m1 - 1);
#pragma unroll
              for (int j = 0; j < RPT; ++j) {
                const uint32_t grp = (uint32_t)(rlane() + j * ROWW);
                const uint32_t coff = ((uint32_t)m * (uint32_t)Npad + grp * VEC) * 4u;
                if constexpr (VEC == 2) {
                  const int2 cc = __builtin_bit_cast(
                      int2, __builtin_amdgcn_raw_buffer_load_b64(rcol, coff, 0, 0));
                  ci[u][j][0] = cc.x;
                  ci[u][j][1] = cc.y;
                } else {
                  ci[u][j][0] = (int)__builtin_amdgcn_raw_buffer_load_b32(rcol, coff, 0, 0);
                }
              }
            }
#pragma unroll
            for (int u = 0; u < ELLB; ++u) {
              const int m = min(mb0 + u, m1 - 1);
              const uint32_t rowoff = (uint32_t)m * (uint32_t)ngroups * (uint32_t)sizeof(L);
#pragma unroll
              for (int j = 0; j < RPT; ++j) {
                const uint32_t off =
                    rowoff + (uint32_t)(rlane() + j * ROWW) * (uint32_t)sizeof(L);
                tv[u][j][0] = load16<L>(rs0, off);
                tv[u][j][1] = load16<L>(rs1, off);
                tv[u][j][2] = load16<L>(rs2, off);
                tv[u][j][3] = load16<L>(rs3, off);
              }
            }
#pragma unroll
            for (int u = 0; u < ELLB; ++u) {
              if (mb0 + u >= m1) break;
#pragma unroll
              for (int j = 0; j < RPT; ++j) {
                F r0[VEC], i0[VEC], r1[VEC], i1[VEC], r2[VEC], i2[VEC], r3[VEC], i3[VEC];
                split(tv[u][j][0], r0, i0); split(tv[u][j][1], r1, i1);
                split(tv[u][j][2], r2, i2); split(tv[u][j][3], r3, i3);
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                  const CS cm = lds.c[ci[u][j][q]];
                  elem<CPLX, F, F2>(pu[j * VEC + q], pv[j * VEC + q], r0[q], i0[q], r1[q],
                                    i1[q], r2[q], i2[q], r3[q], i3[q], w, d, cm);
                }
              }
            }
          }
        } else {
#pragma unroll UNR
          for (int m = m0; m < m1; ++m) {
            CS cm;
            if constexpr (!ELL) cm = lds.c[m];
            const uint32_t rowoff = (uint32_t)m * (uint32_t)ngroups * (uint32_t)sizeof(L);
            // No lane guard: a lane whose column group lies past the last one reads
            // into the next stored row (or past the slice, which returns zero) and
            // its sums are never used, so the loads of consecutive m stay in flight
            // together.
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
              const uint32_t grp = (uint32_t)(rlane() + j * ROWW);
              const uint32_t off = rowoff + grp * (uint32_t)sizeof(L);
              const L v0 = load16<L>(rs0, off);
              const L v1 = load16<L>(rs1, off);
              const L v2 = load16<L>(rs2, off);
              const L v3 = load16<L>(rs3, off);
              F r0[VEC], i0[VEC], r1[VEC], i1[VEC], r2[VEC], i2[VEC], r3[VEC], i3[VEC];
              split(v0, r0, i0); split(v1, r1, i1); split(v2, r2, i2); split(v3, r3, i3);
              int cidx[VEC];
              if constexpr (ELL) {
                const uint32_t coff = ((uint32_t)m * (uint32_t)Npad + grp * VEC) * 4u;
                if constexpr (VEC == 2) {
                  const int2 cc = __builtin_bit_cast(int2, __builtin_amdgcn_raw_buffer_load_b64(rcol, coff, 0, 0));
                  cidx[0] = cc.x;
                  cidx[1] = cc.y;
                } else {
                  cidx[0] = (int)__builtin_amdgcn_raw_buffer_load_b32(rcol, coff, 0, 0);
                }
              }
#pragma unroll
              for (int q = 0; q < VEC; ++q) {
                if constexpr (ELL) cm = lds.c[cidx[q]];
                elem<CPLX, F, F2>(pu[j * VEC + q], pv[j * VEC + q], r0[q], i0[q], r1[q], i1[q],
                                  r2[q], i2[q], r3[q], i3[q], w, d, cm);
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          U[r].x += (double)pu[r].x; U[r].y += (double)pu[r].y;
          V[r].x += (double)pv[r].x; V[r].y += (double)pv[r].y;
        }
      }
    };
    if (sy.ell_w > 0) stream(std::true_type{});
    else stream(std::false_type{});

    if constexpr (SPLIT) {
      // every wave's partial sums of all rows, added in wave order
      const int w = threadIdx.x >> 6;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int n = row(r);
        if (n < Npad) lds.part[w * Npad + n] = make_double4(U[r].x, U[r].y, V[r].x, V[r].y);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int n = row(r);
        if (n >= Npad) continue;
        double4 acc = lds.part[n];
        for (int q = 1; q < NW; ++q) {
          const double4 p = lds.part[q * Npad + n];
          acc.x += p.x; acc.y += p.y; acc.z += p.z; acc.w += p.w;
        }
        U[r] = make_double2(acc.x, acc.y);
        V[r] = make_double2(acc.z, acc.w);
      }
    }

    // epilogue.  J_x couples only channels of equal energy, so
    // J_x a = e^{iE_n t} (J_x c) row by row, and with y = e^{iE t} u:
    //   Re(c^H v), Im(x^H y) = Im((J_x c)^H u), Re(c^H u), Re(a^H J_x a) = Re(c^H J_x c).
    double sums[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n >= N) { cur[r] = make_double2(0.0, 0.0); continue; }
      double sn, cs;
      if constexpr (CPH) {
        sn = psin[r];
        cs = pcos[r];
      } else {
        sincos(sy.E[n] * ts, &sn, &cs);
      }
      const double2 c = make_double2(cs * cur[r].x + sn * cur[r].y,
                                     cs * cur[r].y - sn * cur[r].x);
      double2 xc = make_double2(0.0, 0.0);
      const int W = sy.jx_w;
      if (W <= JXB) {
        // the row's entries are all requested before the first gather (the sum
        // runs in entry order either way)
        int jc[JXB];
        double jv[JXB];
#pragma unroll
        for (int q = 0; q < JXB; ++q) {
          jc[q] = q < W ? sy.jx_col[(int64_t)n * W + q] : 0;
          jv[q] = q < W ? sy.jx_val[(int64_t)n * W + q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < JXB; ++q) {
          if (q >= W) break;
          const double2 cm = lds.c64[jc[q]];
          xc.x = fma(jv[q], cm.x, xc.x);
          xc.y = fma(jv[q], cm.y, xc.y);
        }
      } else {
        for (int q = 0; q < W; ++q) {
          const int col = sy.jx_col[(int64_t)n * W + q];
          const double jv = sy.jx_val[(int64_t)n * W + q];
          const double2 cm = lds.c64[col];
          xc.x = fma(jv, cm.x, xc.x);
          xc.y = fma(jv, cm.y, xc.y);
        }
      }
      const double2 u = U[r], v = V[r];
      sums[0] += c.x * v.x + c.y * v.y;
      sums[1] += xc.x * u.y - xc.y * u.x;
      sums[2] += c.x * u.x + c.y * u.y;
      const double pn = cur[r].x * cur[r].x + cur[r].y * cur[r].y;
      sums[3] += sy.E[n] * pn;
      sums[4] += pn;
      sums[5] += c.x * xc.x + c.y * xc.y;
      // da/dt = -i e^{iE_n t} (u + Phidot J_x c)
      const double gx = u.x + phidot * xc.x, gy = u.y + phidot * xc.y;
      const double yx = cs * gx - sn * gy, yy = cs * gy + sn * gx;
      cur[r] = make_double2(yy, -yx);
    }
    reduce<6>(sums, lds.red0);
    tot.force = sums[0]; tot.torque = sums[1]; tot.vexp = sums[2];
    tot.erot = sums[3]; tot.norm = sums[4]; tot.jx = sums[5];
    if (at) {
      const int k = sp.k;
      tot.vexp = uni(sp.w0 * sy.drv[k] + sp.w1 * sy.drv[k + 1] + sp.w2 * sy.drv2[k] +
                     sp.w3 * sy.drv2[k + 1]);
      tot.force = uni(sp.d0 * sy.drv[k] + sp.d1 * sy.drv[k + 1] + sp.d2 * sy.drv2[k] +
                      sp.d3 * sy.drv2[k + 1]);
      tot.torque = 0.0;
      tot.erot = 0.0;
      tot.jx = 0.0;
    }
  }

  // classical derivatives of (R, Phi, P_R, P_Phi), Eqs. 7-10
  __device__ static void classical_rhs(double mu, const double (&ys)[4], const Sums& tot,
                                       double (&ky)[4]) {
    const double R = ys[0];
    ky[0] = ys[2] / mu;
    ky[1] = ys[3] / (mu * R * R);
    ky[2] = -tot.force + ys[3] * ys[3] / (mu * R * R * R);
    ky[3] = 2.0 * tot.torque;
  }

  __device__ static double energy(double mu, const double (&ys)[4], const Sums& s) {
    return ys[2] * ys[2] / (2.0 * mu) + ys[3] * ys[3] / (2.0 * mu * ys[0] * ys[0]) + s.erot +
           s.vexp;
  }

  // initial amplitudes and classical state of a trajectory
  __device__ static void init_state(const DevSystem& sy, const TrajIn& tj,
                                    const double* __restrict__ a0_all, double2 (&a)[NR],
                                    double (&y)[4], double& theta, double& ptheta) {
    const int N = sy.N;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      double2 v = make_double2(0.0, 0.0);
      if (n < N) {
        if (tj.flags & TRAJ_HAS_A0) v = ((const double2*)a0_all)[tj.amp_off + n];
        else if (n == tj.init_channel) v = make_double2(1.0, 0.0);
      }
      a[r] = v;
    }
    theta = 0.5 * M_PI;
    ptheta = 0.0;
    if (tj.flags & TRAJ_HAS_C0) {
      y[0] = tj.c0[0]; theta = tj.c0[1]; y[1] = tj.c0[2]; y[2] = tj.c0[3]; ptheta = tj.c0[4];
      y[3] = tj.c0[5];
    } else {
      // end of Section II / Section III: P_Phi = b k, P_R = -sqrt(k^2 - P_Phi^2/R0^2)
      const double k = sqrt(2.0 * sy.mu * tj.E_coll);
      const double pphi = tj.b * k;
      y[0] = tj.R0; y[1] = 0.0;
      y[2] = -sqrt(2.0 * sy.mu * tj.E_coll - pphi * pphi / (tj.R0 * tj.R0));
      y[3] = pphi;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = uni(y[i]);
  }

  __device__ static void write_out(const DevSystem& sy, const TrajIn& tj, const TrajOut& out,
                                   const double2 (&a)[NR], const double (&y)[4], double theta,
                                   double ptheta, double tend, int64_t steps, int64_t rejects,
                                   int32_t status, const Sums& tot, double E0, double J0) {
    if (!out.P) return;   // timing runs of the autotuner write no results
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = row(r);
      if (n < sy.N) {
        out.P[tj.amp_off + n] = a[r].x * a[r].x + a[r].y * a[r].y;
        if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = a[r];
        if (out.st_amp) out.st_amp[tj.amp_off + n] = a[r];
      }
    }
    if (threadIdx.x == 0) {
      const int64_t id = tj.id;
      if (out.classical) {
        double* o = out.classical + id * 6;
        o[0] = y[0]; o[1] = theta; o[2] = y[1]; o[3] = y[2]; o[4] = ptheta; o[5] = y[3];
      }
      if (out.t_final) out.t_final[id] = tend;
      if (out.steps) out.steps[id] = steps;
      if (out.rejects) out.rejects[id] = rejects;
      if (out.status) out.status[id] = status;
      if (out.norm_err) out.norm_err[id] = tot.norm - 1.0;
      if (out.energy_err) out.energy_err[id] = (energy(sy.mu, y, tot) - E0) / fabs(E0);
      if (out.angmom_err) out.angmom_err[id] = (y[3] - tot.jx) - J0;
    }
  }
};

}  // namespace rhs
}  // namespace mqct

// Device helpers shared by the propagation kernels.
#pragma once

#include "internal.h"

#include <math.h>

namespace mqct {

// Spline interval and weights at R (natural cubic spline on knots x[0..K-1]):
// value = w0 y_k + w1 y_{k+1} + w2 y2_k + w3 y2_{k+1}; derivative with d0..d3.
// Above the last knot the value is held and the slope is zero; below the first
// knot the spline is continued linearly (and the trajectory flagged).
struct Spl {
  int k;
  bool below;
  double w0, w1, w2, w3, d0, d1, d2, d3;
};

// inv_h > 0: the knots are uniform with spacing 1 / inv_h, and the interval is
// found from a guess and at most a step or two of correction instead of a
// binary search (the same k: the largest one in [0, K-2] with x[k] <= R).
__device__ __forceinline__ Spl spline_at(const double* __restrict__ x, int K, double R,
                                         double inv_h = 0.0) {
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
    if (inv_h > 0.0) {
      lo = min(max((int)((R - x[0]) * inv_h), 0), K - 2);
      while (lo > 0 && x[lo] > R) --lo;
      while (lo < K - 2 && x[lo + 1] <= R) ++lo;
    } else {
      int hi = K - 2;           // largest k in [0, K-2] with x[k] <= R
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (x[mid] <= R) lo = mid; else hi = mid - 1;
      }
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
// slice is far below 4 GiB).  Reads past `bytes` return zero.  Lanes load 16
// bytes (8 for real FP32 tables, which serve small systems).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(const void* p, uint32_t bytes) {
  uint64_t v = (uint64_t)p;
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  void* q = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, (int)bytes, 0x00020000);
}

template <typename L>
__device__ __forceinline__ L load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(L) == 16)
    return __builtin_bit_cast(L, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  else
    return __builtin_bit_cast(L, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

__device__ __forceinline__ double uni(double x) {
  // the value is identical in every lane: keep it in scalar registers
  int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Sum NV values over one wave (shuffles), identical in every lane.
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    v[i] = uni(v[i]);
  }
}

// Sum NV values over the workgroup: wave shuffles, then one LDS slot per wave
// (red[w * NV + i], NW * NV doubles) read back in a fixed order
// (deterministic, identical in every lane).  `red` must not be reused by
// another reduction before a barrier separates them.
template <int NV, int NW>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[w * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += red[q * NV + i];
    v[i] = uni(s);
  }
}

// The stored state of a trajectory at the end of a call (one thread): the
// record of mqct_traj_state; y = (R, Phi, P_R, P_Phi).
__device__ __forceinline__ void put_traj_state(const TrajOut& out, const TrajIn& tj, int N,
                                               double t, double t_origin, int64_t n_origin,
                                               double h, const double (&y)[4], double theta,
                                               double ptheta, double E0, double J0,
                                               double R_exit, int64_t steps, int64_t rejects,
                                               int64_t attempts, int32_t status, int32_t flags) {
  if (!out.state) return;
  mqct_traj_state r;
  r.t = t; r.t_origin = t_origin; r.h = h;
  r.classical[0] = y[0]; r.classical[1] = theta; r.classical[2] = y[1];
  r.classical[3] = y[2]; r.classical[4] = ptheta; r.classical[5] = y[3];
  r.E0 = E0; r.J0 = J0; r.R_exit = R_exit;
  r.n_origin = n_origin; r.steps = steps; r.rejects = rejects; r.attempts = attempts;
  r.status = status; r.flags = flags;
  r.system_id = tj.sys; r.N = N;
  out.state[tj.id] = r;
}

// The exit radius a trajectory starts with: the stored one when it continues a
// stored state, else its starting R.
__device__ __forceinline__ double start_exit_radius(const TrajIn& tj, double R_start) {
  return (tj.flags & TRAJ_RESUME) ? tj.R_exit : R_start;
}

}  // namespace mqct

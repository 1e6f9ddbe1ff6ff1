// R-binned lockstep schedule for fixed-step RK4 on matrix cores.
//
// Every trajectory of the batch advances stage by stage in lockstep.  At each
// stage a trajectory at separation R in spline interval k needs four table
// slices, M_k, M_{k+1}, M2_k, M2_{k+1} (the natural cubic spline of the
// coupling matrix, paper Section III).  Grouping trajectories by knot rather
// than by interval ("grid-point-centric" bins) lets knot g serve both the
// trajectories of interval g (as left knot) and of interval g-1 (as right
// knot): each knot's slices M_g, M2_g are then read once per stage and multiply
// all amplitude columns of its bin, a dense table x columns product that runs on
// the MFMA units.  The spline weights differ per column (every trajectory has
// its own R), so they are applied in the product's epilogue.
//
// Complex products as one real product: with a row of the stored table read as
// 2N interleaved reals (re, im, re, im, ...), Re(M c)_n is that row dotted with
// (Re c_0, -Im c_0, Re c_1, -Im c_1, ...) and Im(M c)_n with (Im c_0, Re c_0,
// ...); each trajectory therefore contributes two real columns and the table
// is read exactly as stored.
//
// Per stage: scan (bin offsets and GEMM work list) -> scatter (bin lists) ->
// gemm (per knot and 64-trajectory tile) -> combine (J_x, force, torque,
// derivatives, RK4 accumulation, then the following stage's state: interval,
// weights, phases, c columns and bin counts).  A separate prep kernel sets up
// the first stage and the final diagnostic evaluation.  The right-hand side is
// the same as the per-trajectory kernels' (Eqs. 5 and 7-10).
#include "device.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace mqct {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int TB = 64;     // trajectories per GEMM work item (2 TB real columns), a multiple of 8
constexpr int NT = 256;    // threads of the per-trajectory kernels
constexpr int NWT = NT / 64;

struct BinWS {
  int B, N, Npad, K;
  const TrajIn* traj;     // [B], batch order
  double2* a0;            // [B][Npad] amplitudes at the start of the step
  double2* cur;           // [B][Npad] amplitudes at the current stage, a0 + cf k
  double2* acc;           // [B][Npad] k1 + 2 k2 + 2 k3 + k4
  double2* c64;           // [B][Npad] c = e^{-iEt} a of the stage in the combine, FP64,
                          // when Npad is too large for LDS
  void* cst;              // [B][2][KR] the two real columns of c in the table precision
  void* uv;               // [2][B][Npad][4] in the table precision, left / right knot:
                          // (zA_re, zB_re, zA_im, zB_im), the value (A) and second-
                          // derivative (B) slices times c, before the spline weights
  double* ycl;            // [B][4] R, Phi, P_R, P_Phi at the start of the step
  double* kcl;            // [B][4] classical derivative of the last stage
  double* acl;            // [B][4] classical accumulator
  double* ysb;            // [B][4] classical stage state
  double* wts;            // [B][8] spline weights w0..w3, d0..d3 at the stage
  double* tst;            // [B] stage time
  double* diag;           // [B][4] E0, J0, Theta, P_Theta
  int* kb;                // [B] interval of the stage, -1 when inactive
  int* status;            // [B]
  int* done;              // [B] steps completed when stopped early, else -1
  int* cnt;               // [K] bin sizes
  int* cursor;            // [K]
  int* offset;            // [K]
  int* list;              // [2B] bin entries 2 b + side (0: left knot, 1: right knot)
  int4* items;            // [max_items] (knot, first entry, count, 0)
  int* n_items;           // [1] work items
  unsigned long long* occ;   // [1] occupied knots summed over the stages of the run
};

__device__ __forceinline__ double stage_frac(int st) {
  return st == 0 ? 0.0 : (st == 3 ? 1.0 : 0.5);
}

__global__ void __launch_bounds__(NT)
bin_init(BinWS ws, const DevSystem* __restrict__ systems, const double* __restrict__ a0_all) {
  const int b = blockIdx.x;
  const TrajIn tj = ws.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  for (int n = threadIdx.x; n < Npad; n += NT) {
    double2 v = make_double2(0.0, 0.0);
    if (n < N) {
      if (tj.flags & TRAJ_HAS_A0) v = ((const double2*)a0_all)[tj.amp_off + n];
      else if (n == tj.init_channel) v = make_double2(1.0, 0.0);
    }
    const int64_t o = (int64_t)b * Npad + n;
    ws.a0[o] = v;
    ws.cur[o] = v;
    ws.acc[o] = make_double2(0.0, 0.0);
  }
  if (threadIdx.x == 0) {
    double y[4], theta = 0.5 * M_PI, ptheta = 0.0;
    if (tj.flags & TRAJ_HAS_C0) {
      y[0] = tj.c0[0]; theta = tj.c0[1]; y[1] = tj.c0[2]; y[2] = tj.c0[3]; ptheta = tj.c0[4];
      y[3] = tj.c0[5];
    } else {
      const double k = sqrt(2.0 * sy.mu * tj.E_coll);
      const double pphi = tj.b * k;
      y[0] = tj.R0; y[1] = 0.0;
      y[2] = -sqrt(2.0 * sy.mu * tj.E_coll - pphi * pphi / (tj.R0 * tj.R0));
      y[3] = pphi;
    }
    for (int i = 0; i < 4; ++i) {
      ws.ycl[b * 4 + i] = y[i];
      ws.kcl[b * 4 + i] = 0.0;
      ws.acl[b * 4 + i] = 0.0;
    }
    ws.diag[b * 4 + 2] = theta;
    ws.diag[b * 4 + 3] = ptheta;
    if (tj.flags & TRAJ_RESUME) {
      // a stored state: the references of the diagnostics continue
      ws.diag[b * 4] = tj.E0;
      ws.diag[b * 4 + 1] = tj.J0;
    }
    ws.status[b] = tj.status0;
    ws.done[b] = -1;
  }
}

// The starting separation of a trajectory (its exit radius unless it continues
// a stored state).
__device__ __forceinline__ double start_R(const TrajIn& tj) {
  return (tj.flags & TRAJ_HAS_C0) ? tj.c0[0] : tj.R0;
}

__global__ void bin_zero(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Interval, spline weights, stage state and time of trajectory b at a stage,
// and its entries in the counts of its two knots (one thread).
__device__ __forceinline__ void stage_setup(const BinWS& ws, const DevSystem& sy, int b,
                                            const double (&ys)[4], double t, bool count_below) {
  const Spl sp = spline_at(sy.R, sy.K, ys[0], sy.R_inv_h);
  for (int i = 0; i < 4; ++i) ws.ysb[b * 4 + i] = ys[i];
  double* w = ws.wts + (int64_t)b * 8;
  w[0] = sp.w0; w[1] = sp.w1; w[2] = sp.w2; w[3] = sp.w3;
  w[4] = sp.d0; w[5] = sp.d1; w[6] = sp.d2; w[7] = sp.d3;
  ws.tst[b] = t;
  ws.kb[b] = sp.k;
  atomicAdd(&ws.cnt[sp.k], 1);
  atomicAdd(&ws.cnt[sp.k + 1], 1);
  if (sp.below && count_below) ws.status[b] |= ST_BELOW_GRID;
}

// Element n of the two real columns of c in the table precision (KR = 2 Npad
// reals for complex tables, Npad for real ones): complex tables take
// (Re c_n, -Im c_n) and (Im c_n, Re c_n) at reals 2n, 2n+1; real tables take
// Re c_n and Im c_n.
template <typename S, bool CPLX>
__device__ __forceinline__ void put_cols(const BinWS& ws, int b, int Npad, int n, double2 c) {
  const int64_t KR = (CPLX ? 2 : 1) * (int64_t)Npad;
  S* col0 = (S*)ws.cst + (int64_t)b * 2 * KR;
  S* col1 = col0 + KR;
  const S re = (S)c.x, im = (S)c.y;
  if constexpr (CPLX) {
    col0[2 * n] = re; col0[2 * n + 1] = -im;
    col1[2 * n] = im; col1[2 * n + 1] = re;
  } else {
    col0[n] = re;
    col1[n] = im;
  }
}

// Stage state of every trajectory for the first stage of the run and for the
// final diagnostic evaluation (diag = 1, at the end state): classical stage
// values, interval and weights, the stage amplitudes and c columns, and the
// knot counts.  Both begin a step (st = 0), where the stage amplitudes are a0.
// Every other stage is prepared by the combine of the stage before it.
template <typename S, bool CPLX>
__global__ void __launch_bounds__(NT)
bin_prep(BinWS ws, const DevSystem* __restrict__ systems, int64_t j, int st, int diag) {
  const int b = blockIdx.x;
  const TrajIn tj = ws.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  const int dn = ws.done[b];
  const bool active = diag || (j < tj.n_steps && dn < 0);
  if (!active) {
    if (threadIdx.x == 0) ws.kb[b] = -1;
    return;
  }
  const double h = tj.dt;
  const double cf = diag ? 0.0 : stage_frac(st) * h;
  const int64_t jsteps = diag ? (dn >= 0 ? (int64_t)dn : tj.n_steps) : j;
  const double t = tj.t0 + (double)(tj.step0 + jsteps) * h + cf;
  double ys[4];
  for (int i = 0; i < 4; ++i) ys[i] = fma(cf, ws.kcl[b * 4 + i], ws.ycl[b * 4 + i]);
  if (threadIdx.x == 0) stage_setup(ws, sy, b, ys, t, !diag);
  for (int n = threadIdx.x; n < Npad; n += NT) {
    const int64_t o = (int64_t)b * Npad + n;
    double2 c = make_double2(0.0, 0.0);
    if (n < N) {
      const double2 a = ws.a0[o];
      ws.cur[o] = a;
      double sn, cs;
      sincos(sy.E[n] * t, &sn, &cs);
      c = make_double2(cs * a.x + sn * a.y, cs * a.y - sn * a.x);
    }
    put_cols<S, CPLX>(ws, b, Npad, n, c);
  }
}

// Bin offsets and the GEMM work list; resets the counters for the next stage.
// The work items are listed by their number of 8-trajectory column blocks,
// largest first: the product workgroups of the large items start first and the
// short ones fill the end of the launch.  (The order within one size class is
// that of the slot counters and does not affect any result: every item writes
// its own outputs.)  One workgroup of 1024 threads, two knots per thread.
__global__ void __launch_bounds__(1024) bin_scan(BinWS ws) {
  constexpr int NCLS = TB / 8;                 // column-block classes 1..NCLS
  const int K = ws.K, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ int wsum[16];
  __shared__ int ncls[NCLS + 1], cur[NCLS + 1];
  __shared__ int occupied;
  if (t <= NCLS) ncls[t] = 0;
  if (t == 0) occupied = 0;
  const int g0 = 2 * t, g1 = 2 * t + 1;
  const int c0 = g0 < K ? ws.cnt[g0] : 0, c1 = g1 < K ? ws.cnt[g1] : 0;
  // exclusive prefix of the bin sizes: within the wave, then across waves
  int incl = c0 + c1;
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(incl, d, 64);
    if (lane >= d) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  const int off0 = base + incl - c0 - c1, off1 = off0 + c0;
  if (g0 < K) ws.offset[g0] = off0;
  if (g1 < K) ws.offset[g1] = off1;
  const int cls0 = ((c0 % TB) + 7) >> 3, cls1 = ((c1 % TB) + 7) >> 3;   // 0: no partial item
  if (c0 / TB + c1 / TB) atomicAdd(&ncls[NCLS], c0 / TB + c1 / TB);
  if (cls0) atomicAdd(&ncls[cls0], 1);
  if (cls1) atomicAdd(&ncls[cls1], 1);
  if ((c0 > 0) + (c1 > 0)) atomicAdd(&occupied, (c0 > 0) + (c1 > 0));
  __syncthreads();
  if (t == 0) {
    int io = 0;
    for (int c = NCLS; c >= 1; --c) {
      cur[c] = io;
      io += ncls[c];
    }
    *ws.n_items = io;
    *ws.occ += (unsigned long long)occupied;
  }
  __syncthreads();
  auto emit = [&](int g, int c, int off, int cls) {
    const int nf = c / TB;
    if (nf) {
      const int p = atomicAdd(&cur[NCLS], nf);
      for (int q = 0; q < nf; ++q) ws.items[p + q] = make_int4(g, off + q * TB, TB, 0);
    }
    if (cls) ws.items[atomicAdd(&cur[cls], 1)] = make_int4(g, off + nf * TB, c - nf * TB, 0);
  };
  if (g0 < K) emit(g0, c0, off0, cls0);
  if (g1 < K) emit(g1, c1, off1, cls1);
  if (g0 < K) { ws.cnt[g0] = 0; ws.cursor[g0] = 0; }
  if (g1 < K) { ws.cnt[g1] = 0; ws.cursor[g1] = 0; }
}

__global__ void bin_scatter(BinWS ws) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= ws.B) return;
  const int k = ws.kb[b];
  if (k < 0) return;
  const int p0 = atomicAdd(&ws.cursor[k], 1);
  ws.list[ws.offset[k] + p0] = 2 * b;
  const int p1 = atomicAdd(&ws.cursor[k + 1], 1);
  ws.list[ws.offset[k + 1] + p1] = 2 * b + 1;
}

// K steps of operands in flight, FP32 tables
#ifndef BIN_GEMM_PF32
#define BIN_GEMM_PF32 2
#endif
constexpr int GEMM_PF32 = BIN_GEMM_PF32;
// ring periods per loop iteration: the compiler's waits for the loads are exact
// inside an iteration and conservative only across the loop's back edge
constexpr int GEMM_UF = 1;

template <typename S> struct MF;
template <> struct MF<float> {
  using V = v4f;
  __device__ static V mfma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MF<double> {
  using V = v4d;
  __device__ static V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Four consecutive reals of a stored table row (row >= N lies past the slice
// and reads as zero).
template <typename S>
__device__ __forceinline__ void load4(__amdgpu_buffer_rsrc_t r, uint32_t off, S (&o)[4]) {
  if constexpr (sizeof(S) == 4) {
    const float4 v = load16<float4>(r, off);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else {
    const double2 v0 = load16<double2>(r, off), v1 = load16<double2>(r, off + 16);
    o[0] = v0.x; o[1] = v0.y; o[2] = v1.x; o[3] = v1.y;
  }
}

// One work item (knot g, up to TB trajectories of its bin) x a tile of rows.
// Wave w owns RB 16-row blocks; every lane holds, for each of NX column blocks
// of 16 real columns (8 trajectories), the 16x16 accumulators of both slices
// (v_mfma_*_16x16x4: lane l supplies A[l%16][k] and B[k][l%16] with
// k = l/16; its D values are column l%16, rows 4(l/16)+r for the f32 form
// and l/16+4r for the f64 form).  Along K each lane loads four consecutive
// reals of the table row and of its real column, and the four MFMAs of one
// step take k = k0 + 4(l/16) + i, i = 0..3, on both operands (a permutation
// of K).  NX is the number of column blocks that hold trajectories, so empty
// blocks cost nothing; the operands of the next PF - 1 steps are in flight
// while the MFMAs of step k0 run.
template <int DT, int NX>
__device__ __forceinline__ void gemm_item(const BinWS& ws, const DevSystem& sy, int rb, int g,
                                          int start, int count) {
  constexpr bool FP32 = (DT == C64 || DT == R32);
  constexpr bool CPLX = (DT == C64 || DT == C128);
  using S = typename std::conditional<FP32, float, double>::type;
  using V = typename MF<S>::V;
  constexpr int RB = 2;
  // K steps of operands in flight: the FP32 form has the registers for a deeper ring
  constexpr int PF = FP32 ? GEMM_PF32 : 2;
  constexpr int NCOMP = CPLX ? 2 : 1;
  const int N = sy.N, Npad = sy.Npad;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, c16 = lane & 15, part = c16 & 1;
  const int row0 = rb * (4 * RB * 16) + wave * RB * 16;
  const int64_t ks = sy.knot_stride;
  const uint32_t sbytes = (uint32_t)(ks * NCOMP * (int64_t)sizeof(S));
  const auto rA = slice_rsrc((const S*)sy.M + (int64_t)g * ks * NCOMP, sbytes);
  const auto rB = slice_rsrc((const S*)sy.M2 + (int64_t)g * ks * NCOMP, sbytes);
  const uint32_t rowbytes = (uint32_t)(Npad * NCOMP * sizeof(S));
  const int KR = Npad * NCOMP;   // stored real K extent (zero-padded past N)
  // the products stop at the first 16-multiple past the N * NCOMP stored reals:
  // the steps beyond would add exact zeros
  const int KE = (N * NCOMP + 15) & ~15;

  // this lane's real column in each column block
  const S* col[NX];
#pragma unroll
  for (int cb = 0; cb < NX; ++cb) {
    const int jt = (cb * 16 + c16) >> 1;
    const int e = ws.list[start + (jt < count ? jt : 0)];
    col[cb] = (const S*)ws.cst + ((int64_t)(e >> 1) * 2 + part) * KR + 4 * q;
  }
  V acc[RB][2][NX];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int cb = 0; cb < NX; ++cb) acc[r][s][cb] = V{0, 0, 0, 0};

  // operands of PF K steps in a ring: step k0 + 16 j sits in stage j % PF; the
  // loads for step k0 + 16 (PF - 1) are issued before the products of step k0
  S a[PF][RB][2][4], bv[PF][NX][4];
  auto load = [&](int k0, S (&ao)[RB][2][4], S (&bo)[NX][4]) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const uint32_t off =
          (uint32_t)(row0 + r * 16 + c16) * rowbytes + (uint32_t)(k0 + 4 * q) * sizeof(S);
      load4<S>(rA, off, ao[r][0]);
      load4<S>(rB, off, ao[r][1]);
    }
#pragma unroll
    for (int cb = 0; cb < NX; ++cb) {
      if constexpr (FP32) {
        const float4 v = *(const float4*)(col[cb] + k0);
        bo[cb][0] = v.x; bo[cb][1] = v.y; bo[cb][2] = v.z; bo[cb][3] = v.w;
      } else {
        const double2 v0 = *(const double2*)(col[cb] + k0);
        const double2 v1 = *(const double2*)(col[cb] + k0 + 2);
        bo[cb][0] = v0.x; bo[cb][1] = v0.y; bo[cb][2] = v1.x; bo[cb][3] = v1.y;
      }
    }
  };
  auto mma = [&](const S (&ai)[RB][2][4], const S (&bi)[NX][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int cb = 0; cb < NX; ++cb)
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int s = 0; s < 2; ++s)
            acc[r][s][cb] = MF<S>::mfma(ai[r][s][i], bi[cb][i], acc[r][s][cb]);
  };
  // K steps past the last one reload that step's operands (unused) rather than branch
#pragma unroll
  for (int j = 0; j < PF - 1; ++j) load(min(16 * j, KE - 16), a[j], bv[j]);
  for (int k0 = 0; k0 < KE; k0 += 16 * PF * GEMM_UF) {
#pragma unroll
    for (int j = 0; j < PF * GEMM_UF; ++j) {
      const int kl = k0 + 16 * (j + PF - 1);
      load(kl < KE ? kl : KE - 16, a[(j + PF - 1) % PF], bv[(j + PF - 1) % PF]);
      // keep the loads ahead of the products (and the waits for them behind)
      __builtin_amdgcn_sched_barrier(0);
      if (k0 + 16 * j < KE) mma(a[j % PF], bv[j % PF]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // epilogue: both slices' products of this column (left or right knot); the
  // spline weights are applied in FP64 where the two knots are combined
#pragma unroll
  for (int cb = 0; cb < NX; ++cb) {
    const int jt = (cb * 16 + c16) >> 1;
    if (jt >= count) continue;
    const int e = ws.list[start + jt];
    const int b = e >> 1, side = e & 1;
    using S2 = typename std::conditional<FP32, float2, double2>::type;
    S2* o = (S2*)((S*)ws.uv + ((int64_t)side * ws.B + b) * Npad * 4) + part;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // D rows of lane group q: 4q + i (f32 form), q + 4i (f64 form)
        const int n = row0 + r * 16 + (FP32 ? 4 * q + i : q + 4 * i);
        if (n < N) {
          S2 z;
          z.x = acc[r][0][cb][i];
          z.y = acc[r][1][cb][i];
          o[(int64_t)n * 2] = z;
        }
      }
  }
}

template <int DT, int NX>
__device__ __forceinline__ void gemm_dispatch(const BinWS& ws, const DevSystem& sy, int rb, int g,
                                              int start, int count, int ncb) {
  if constexpr (NX > 1) {
    if (ncb < NX) {
      gemm_dispatch<DT, NX - 1>(ws, sy, rb, g, start, count, ncb);
      return;
    }
  }
  gemm_item<DT, NX>(ws, sy, rb, g, start, count);
}

constexpr int NXCD = 8;    // accelerator dies (each with its own L2) of the device
// Dynamic LDS requested by every product workgroup (unused): more than half of
// a CU's 160 KiB, so one workgroup is resident per CU.  Fewer concurrent items
// keep the table rows and columns streaming through each die's L2 small; with
// the operands of the next K step in flight this ran faster than two or three
// resident workgroups per CU.
constexpr size_t GEMM_LDS_CAP = 96 * 1024;

// Work items are dealt to the dies round-robin (item i to die i mod 8), and the
// row blocks of one item run on one die, one after another: they read the same
// amplitude columns, which then stay in that die's L2.  Workgroups are handed
// to the dies round-robin by id, so die x receives ids x, x + 8, ...: its
// j-th workgroup takes row block j mod nrb of item x + 8 (j / nrb).  The items
// arrive largest first, so every die starts on its long items and ends on its
// short ones.
//
template <int DT>
__global__ void __launch_bounds__(256)
bin_gemm(BinWS ws, const DevSystem* __restrict__ systems, int nrb) {
  const int x = blockIdx.x % NXCD, jj = blockIdx.x / NXCD;
  const int item = x + NXCD * (jj / nrb), rb = jj % nrb;
  if (item >= *ws.n_items) return;
  const int4 it = ws.items[item];
  const DevSystem sy = systems[ws.traj[0].sys];
  if constexpr (DT == R64) {
    // real FP64 tables: at most four column blocks per pass (eight would spill)
    for (int c0 = 0; c0 < it.z; c0 += 32) {
      const int cnt = min(32, it.z - c0);
      gemm_dispatch<DT, 4>(ws, sy, rb, it.x, it.y + c0, cnt, (cnt + 7) >> 3);
    }
  } else {
    gemm_dispatch<DT, TB / 8>(ws, sy, rb, it.x, it.y, it.z, (it.z + 7) >> 3);
  }
}

// Combine the two knots' contributions with the spline weights, add the
// Coriolis term, reduce the mean-field force and torque, and advance the RK4
// accumulators; with next = 1 also prepare the following stage of the step
// sequence (its c columns, interval, weights and knot counts), so that the
// amplitudes are read once per stage.  S, CPLX: the table precision and kind;
// LDSC: c of this stage and its phases e^{-iEt} are held in LDS (Npad <= 2048),
// else c is kept in ws.c64 and the phases are computed again.
template <typename S, bool CPLX, bool LDSC>
__global__ void __launch_bounds__(NT)
bin_combine(BinWS ws, const DevSystem* __restrict__ systems, int64_t j, int st, int diag,
            int next, TrajOut out) {
  extern __shared__ double2 c_lds[];   // [Npad] c, then [Npad] (cos Et, sin Et)
  __shared__ double red[NWT * 8];
  const int b = blockIdx.x;
  if (ws.kb[b] < 0) return;
  const TrajIn tj = ws.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  const double mu = sy.mu, h = tj.dt;
  double ys[4];
  for (int i = 0; i < 4; ++i) ys[i] = ws.ysb[b * 4 + i];
  const double t = ws.tst[b];
  const double R = ys[0];
  const double phidot = ys[3] / (mu * R * R);
  const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
  double2* cb = LDSC ? c_lds : ws.c64 + (int64_t)b * Npad;
  double2* ph = c_lds + Npad;
  double sums[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // c = e^{-iEt} (a0 + cf k) of this stage, for the products with J_x; the
  // rotational energy and the norm
  for (int n = threadIdx.x; n < N; n += NT) {
    const double2 cur = ws.cur[(int64_t)b * Npad + n];
    double sn, cs;
    sincos(sy.E[n] * t, &sn, &cs);
    cb[n] = make_double2(cs * cur.x + sn * cur.y, cs * cur.y - sn * cur.x);
    if constexpr (LDSC) ph[n] = make_double2(cs, sn);
    const double pn = cur.x * cur.x + cur.y * cur.y;
    sums[3] += sy.E[n] * pn;
    sums[4] += pn;
  }
  __syncthreads();
  // the following stage: step jn, stage stn, time tn
  const int stn = st == 3 ? 0 : st + 1;
  const int64_t jn = st == 3 ? j + 1 : j;
  const double cfn = stage_frac(stn) * h;
  const double tn = tj.t0 + (double)(tj.step0 + jn) * h + cfn;
  const bool same_t = tn == t;
  const double* wt = ws.wts + (int64_t)b * 8;
  const double w0 = wt[0], w1 = wt[1], w2 = wt[2], w3 = wt[3];
  const double d0 = wt[4], d1 = wt[5], d2 = wt[6], d3 = wt[7];
  using S4 = typename std::conditional<sizeof(S) == 4, float4, double4>::type;
  const S4* uvl = (const S4*)ws.uv;
  for (int n = threadIdx.x; n < N; n += NT) {
    const int64_t o = (int64_t)b * Npad + n;
    const S4 L = uvl[o], Rr = uvl[(int64_t)ws.B * Npad + o];
    // left knot: weights w0, w2 (d0, d2); right knot: w1, w3 (d1, d3)
    const double2 u = make_double2((w0 * (double)L.x + w2 * (double)L.y) +
                                       (w1 * (double)Rr.x + w3 * (double)Rr.y),
                                   (w0 * (double)L.z + w2 * (double)L.w) +
                                       (w1 * (double)Rr.z + w3 * (double)Rr.w));
    const double2 v = make_double2((d0 * (double)L.x + d2 * (double)L.y) +
                                       (d1 * (double)Rr.x + d3 * (double)Rr.y),
                                   (d0 * (double)L.z + d2 * (double)L.w) +
                                       (d1 * (double)Rr.z + d3 * (double)Rr.w));
    const double2 c = cb[n];
    double2 xc = make_double2(0.0, 0.0);
    for (int qq = 0; qq < sy.jx_w; ++qq) {
      const int col = sy.jx_col[(int64_t)n * sy.jx_w + qq];
      const double jv = sy.jx_val[(int64_t)n * sy.jx_w + qq];
      const double2 cm = cb[col];
      xc.x = fma(jv, cm.x, xc.x);
      xc.y = fma(jv, cm.y, xc.y);
    }
    sums[0] += c.x * v.x + c.y * v.y;
    sums[1] += xc.x * u.y - xc.y * u.x;
    sums[2] += c.x * u.x + c.y * u.y;
    sums[5] += c.x * xc.x + c.y * xc.y;
    if (!diag) {
      const double2 a = ws.a0[o];
      double sn, cs;
      if constexpr (LDSC) {
        const double2 p = ph[n];
        cs = p.x;
        sn = p.y;
      } else {
        sincos(sy.E[n] * t, &sn, &cs);
      }
      const double gx = u.x + phidot * xc.x, gy = u.y + phidot * xc.y;
      const double yx = cs * gx - sn * gy, yy = cs * gy + sn * gx;
      const double2 k = make_double2(yy, -yx);
      double2 ac = st == 0 ? make_double2(0.0, 0.0) : ws.acc[o];
      ac.x = fma(wgt, k.x, ac.x);
      ac.y = fma(wgt, k.y, ac.y);
      double2 base = a;
      if (st == 3) {
        const double h6 = h / 6.0;
        base = make_double2(a.x + h6 * ac.x, a.y + h6 * ac.y);
        ws.a0[o] = base;
      } else {
        ws.acc[o] = ac;
      }
      if (next) {
        // the following stage's amplitudes and c columns
        const double2 curn = make_double2(fma(cfn, k.x, base.x), fma(cfn, k.y, base.y));
        ws.cur[o] = curn;
        double snn = sn, csn = cs;
        if (!same_t) sincos(sy.E[n] * tn, &snn, &csn);
        put_cols<S, CPLX>(ws, b, Npad, n, make_double2(csn * curn.x + snn * curn.y,
                                                       csn * curn.y - snn * curn.x));
      }
    }
  }
  block_sum<6, NWT>(sums, red);
  if (tj.flags & TRAJ_AT) {
    // decoupled (AT) dynamics: the driving potential at the stage's R (same
    // interval and weights as the tables) replaces the mean field
    const int k = ws.kb[b];
    const double* w = ws.wts + (int64_t)b * 8;
    sums[2] = w[0] * sy.drv[k] + w[1] * sy.drv[k + 1] + w[2] * sy.drv2[k] + w[3] * sy.drv2[k + 1];
    sums[0] = w[4] * sy.drv[k] + w[5] * sy.drv[k + 1] + w[6] * sy.drv2[k] + w[7] * sy.drv2[k + 1];
    sums[1] = sums[3] = sums[5] = 0.0;
  }
  const double force = sums[0], torque = sums[1], vexp = sums[2], erot = sums[3];
  const double norm = sums[4], jx = sums[5];
  const double E = ys[2] * ys[2] / (2.0 * mu) + ys[3] * ys[3] / (2.0 * mu * R * R) + erot + vexp;
  if (diag) {
    const int64_t taken = ws.done[b] >= 0 ? (int64_t)ws.done[b] : tj.n_steps;
    const int64_t steps = tj.steps0 + taken;
    for (int n = threadIdx.x; n < N; n += NT) {
      const double2 a = ws.a0[(int64_t)b * Npad + n];
      out.P[tj.amp_off + n] = a.x * a.x + a.y * a.y;
      if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = a;
      if (out.st_amp) out.st_amp[tj.amp_off + n] = a;
    }
    if (threadIdx.x == 0) {
      const int64_t id = tj.id;
      // the references were taken at the first evaluation, or come with a stored state
      const bool ref = taken > 0 || (tj.flags & TRAJ_RESUME);
      const double E0 = ref ? ws.diag[b * 4] : E;
      const double J0 = ref ? ws.diag[b * 4 + 1] : ys[3] - jx;
      if (out.classical) {
        double* o = out.classical + id * 6;
        o[0] = ys[0]; o[1] = ws.diag[b * 4 + 2]; o[2] = ys[1]; o[3] = ys[2];
        o[4] = ws.diag[b * 4 + 3]; o[5] = ys[3];
      }
      if (out.t_final) out.t_final[id] = t;
      if (out.steps) out.steps[id] = steps;
      if (out.rejects) out.rejects[id] = tj.rejects0;
      if (out.status) out.status[id] = ws.status[b];
      if (out.norm_err) out.norm_err[id] = norm - 1.0;
      if (out.energy_err) out.energy_err[id] = (E - E0) / fabs(E0);
      if (out.angmom_err) out.angmom_err[id] = (ys[3] - jx) - J0;
      put_traj_state(out, tj, N, t, tj.t0, tj.step0 + taken, h, ys, ws.diag[b * 4 + 2],
                     ws.diag[b * 4 + 3], E0, J0, start_exit_radius(tj, start_R(tj)), steps,
                     tj.rejects0, tj.attempts0 + taken, ws.status[b], tj.dflags);
    }
    return;
  }
  if (threadIdx.x == 0) {
    if (j == 0 && st == 0 && !(tj.flags & TRAJ_RESUME)) {
      ws.diag[b * 4] = E;
      ws.diag[b * 4 + 1] = ys[3] - jx;
    }
    const double kc[4] = {ys[2] / mu, phidot, -force + ys[3] * ys[3] / (mu * R * R * R),
                          2.0 * torque};
    for (int i = 0; i < 4; ++i) {
      const double ac = (st == 0 ? 0.0 : ws.acl[b * 4 + i]) + wgt * kc[i];
      ws.kcl[b * 4 + i] = kc[i];
      if (st == 3) ws.ycl[b * 4 + i] += h / 6.0 * ac;
      else ws.acl[b * 4 + i] = ac;
    }
    if (st == 3) {
      bool ok = isfinite(force) && isfinite(torque) && isfinite(norm);
      for (int i = 0; i < 4; ++i) ok = ok && isfinite(ws.ycl[b * 4 + i]);
      if (!ok) {
        ws.status[b] |= ST_NONFINITE;
        ws.done[b] = (int)(j + 1);
      }
    }
  }
  if (!next) return;
  // every thread has read this stage's weights and state before thread 0
  // overwrites them with the following stage's
  __syncthreads();
  if (threadIdx.x == 0) {
    if (jn < tj.n_steps && ws.done[b] < 0) {
      double yn[4];
      for (int i = 0; i < 4; ++i) yn[i] = fma(cfn, ws.kcl[b * 4 + i], ws.ycl[b * 4 + i]);
      stage_setup(ws, sy, b, yn, tn, true);
    } else {
      ws.kb[b] = -1;
    }
  }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }


// ---- adaptive Dormand-Prince 5(4) on the binned product ----------------------
//
// Every unfinished trajectory makes one step attempt per round: six stage
// evaluations (the first stage is the last one of the previous accepted step),
// each a binned product as above, then the embedded error estimate and the
// accept/reject decision.  Tableau, error norm, controller, starting step and
// stopping rules are those of the work-list schedule's adaptive stepper (scaled
// RMS over the 2N + 6 real state components; factor min(5, max(0.2,
// 0.9 err^-1/5)), no growth right after a rejection; starting step of Hairer,
// Norsett and Wanner, Solving ODEs I, Sec. II.4; exit after the first accepted
// step with R >= R0 and P_R > 0).  Finished trajectories leave the bins.

__constant__ double D5C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
__constant__ double D5A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
__constant__ double D5E[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920,
                              -17253.0 / 339200, 22.0 / 525, -1.0 / 40};

enum { D5_INIT0 = 0, D5_INIT1 = 1, D5_STAGE = 2, D5_DIAG = 3 };
enum { D5_DONE = 1, D5_LASTREJ = 2 };

struct D5WS {
  double2* ks;            // [B][8][Npad]: stage derivatives k_1..k_7 in slots 0..6, y5 in 7
  double* kc;             // [B][8][4]: the classical ones, y5 of R, Phi, P_R, P_Phi in 7
  double* h;              // [B] step of the next attempt (the starting step while starting)
  double* t;              // [B] time of the current state
  double* rexit;          // [B] exit radius (the starting R)
  double* d1;             // [B] ||f(t0, y0)|| of the starting-step estimate
  long long* steps;       // [B] accepted steps
  long long* rejects;     // [B]
  long long* attempts;    // [B]
  int* flags;             // [B]
  int* active;            // [1] unfinished trajectories after the last counted round
};

// Stage input of every unfinished trajectory (all of them for the final
// evaluation): amplitudes and classical state, the stage time, interval,
// weights, knot counts and c columns.
template <typename S, bool CPLX>
__global__ void __launch_bounds__(NT)
d5_prep(BinWS ws, D5WS d, const DevSystem* __restrict__ systems, int mode, int sg) {
  const int b = blockIdx.x;
  if (mode != D5_DIAG && (d.flags[b] & D5_DONE)) {
    if (threadIdx.x == 0) ws.kb[b] = -1;
    return;
  }
  const TrajIn tj = ws.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  const double h = d.h[b], t0 = d.t[b];
  const double2* ks = d.ks + (int64_t)b * 8 * Npad;
  const double* kc = d.kc + (int64_t)b * 32;
  const double* yc = ws.ycl + (int64_t)b * 4;
  double ys[4];
  double ts = t0;
  if (mode == D5_INIT1) {
    for (int k = 0; k < 4; ++k) ys[k] = fma(h, kc[k], yc[k]);
    ts = t0 + h;
  } else if (mode == D5_STAGE) {
    for (int k = 0; k < 4; ++k) {
      double acc = fma(h * D5A[sg][0], kc[k], yc[k]);
      for (int p = 1; p < sg; ++p) acc = fma(h * D5A[sg][p], kc[p * 4 + k], acc);
      ys[k] = acc;
    }
    ts = t0 + D5C[sg] * h;
  } else {
    for (int k = 0; k < 4; ++k) ys[k] = yc[k];
  }
  if (threadIdx.x == 0) {
    stage_setup(ws, sy, b, ys, ts, mode != D5_DIAG);
    if (mode == D5_STAGE && sg == 6)
      for (int k = 0; k < 4; ++k) d.kc[(int64_t)b * 32 + 28 + k] = ys[k];
  }
  for (int n = threadIdx.x; n < Npad; n += NT) {
    const int64_t o = (int64_t)b * Npad + n;
    double2 c = make_double2(0.0, 0.0);
    if (n < N) {
      double2 cur = ws.a0[o];
      if (mode == D5_INIT1) {
        const double2 k = ks[n];
        cur = make_double2(fma(h, k.x, cur.x), fma(h, k.y, cur.y));
      } else if (mode == D5_STAGE) {
        for (int p = 0; p < sg; ++p) {
          const double2 kp = ks[(int64_t)p * Npad + n];
          const double cc = h * D5A[sg][p];
          cur.x = fma(cc, kp.x, cur.x);
          cur.y = fma(cc, kp.y, cur.y);
        }
        if (sg == 6) d.ks[((int64_t)b * 8 + 7) * Npad + n] = cur;
      }
      ws.cur[o] = cur;
      double sn, cs;
      sincos(sy.E[n] * ts, &sn, &cs);
      c = make_double2(cs * cur.x + sn * cur.y, cs * cur.y - sn * cur.x);
    }
    put_cols<S, CPLX>(ws, b, Npad, n, c);
  }
}

// Right-hand side of the stage from the two knots' products: the amplitude
// derivative into slot `slot`, the classical one into kc; at the first
// evaluation also the conserved quantities' starting values; at the final
// evaluation the results.
template <typename S, bool CPLX, bool LDSC>
__global__ void __launch_bounds__(NT)
d5_combine(BinWS ws, D5WS d, const DevSystem* __restrict__ systems, int mode, int slot,
           TrajOut out) {
  extern __shared__ double2 c_lds[];
  __shared__ double red[NWT * 8];
  const int b = blockIdx.x;
  if (ws.kb[b] < 0) return;
  const TrajIn tj = ws.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  const double mu = sy.mu;
  double ys[4];
  for (int i = 0; i < 4; ++i) ys[i] = ws.ysb[b * 4 + i];
  const double t = ws.tst[b];
  const double R = ys[0];
  const double phidot = ys[3] / (mu * R * R);
  double2* cb = LDSC ? c_lds : ws.c64 + (int64_t)b * Npad;
  double sums[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int n = threadIdx.x; n < N; n += NT) {
    const double2 cur = ws.cur[(int64_t)b * Npad + n];
    double sn, cs;
    sincos(sy.E[n] * t, &sn, &cs);
    cb[n] = make_double2(cs * cur.x + sn * cur.y, cs * cur.y - sn * cur.x);
    const double pn = cur.x * cur.x + cur.y * cur.y;
    sums[3] += sy.E[n] * pn;
    sums[4] += pn;
  }
  __syncthreads();
  const double* wt = ws.wts + (int64_t)b * 8;
  const double w0 = wt[0], w1 = wt[1], w2 = wt[2], w3 = wt[3];
  const double d0 = wt[4], d1 = wt[5], d2 = wt[6], d3 = wt[7];
  using S4 = typename std::conditional<sizeof(S) == 4, float4, double4>::type;
  const S4* uvl = (const S4*)ws.uv;
  double2* kout = d.ks + ((int64_t)b * 8 + slot) * Npad;
  for (int n = threadIdx.x; n < N; n += NT) {
    const int64_t o = (int64_t)b * Npad + n;
    const S4 L = uvl[o], Rr = uvl[(int64_t)ws.B * Npad + o];
    const double2 u = make_double2((w0 * (double)L.x + w2 * (double)L.y) +
                                       (w1 * (double)Rr.x + w3 * (double)Rr.y),
                                   (w0 * (double)L.z + w2 * (double)L.w) +
                                       (w1 * (double)Rr.z + w3 * (double)Rr.w));
    const double2 v = make_double2((d0 * (double)L.x + d2 * (double)L.y) +
                                       (d1 * (double)Rr.x + d3 * (double)Rr.y),
                                   (d0 * (double)L.z + d2 * (double)L.w) +
                                       (d1 * (double)Rr.z + d3 * (double)Rr.w));
    const double2 c = cb[n];
    double2 xc = make_double2(0.0, 0.0);
    for (int qq = 0; qq < sy.jx_w; ++qq) {
      const int col = sy.jx_col[(int64_t)n * sy.jx_w + qq];
      const double jv = sy.jx_val[(int64_t)n * sy.jx_w + qq];
      const double2 cm = cb[col];
      xc.x = fma(jv, cm.x, xc.x);
      xc.y = fma(jv, cm.y, xc.y);
    }
    sums[0] += c.x * v.x + c.y * v.y;
    sums[1] += xc.x * u.y - xc.y * u.x;
    sums[2] += c.x * u.x + c.y * u.y;
    sums[5] += c.x * xc.x + c.y * xc.y;
    if (mode != D5_DIAG) {
      double sn, cs;
      sincos(sy.E[n] * t, &sn, &cs);
      const double gx = u.x + phidot * xc.x, gy = u.y + phidot * xc.y;
      const double yx = cs * gx - sn * gy, yy = cs * gy + sn * gx;
      kout[n] = make_double2(yy, -yx);
    }
  }
  block_sum<6, NWT>(sums, red);
  if (tj.flags & TRAJ_AT) {
    const int k = ws.kb[b];
    sums[2] = w0 * sy.drv[k] + w1 * sy.drv[k + 1] + w2 * sy.drv2[k] + w3 * sy.drv2[k + 1];
    sums[0] = d0 * sy.drv[k] + d1 * sy.drv[k + 1] + d2 * sy.drv2[k] + d3 * sy.drv2[k + 1];
    sums[1] = sums[3] = sums[5] = 0.0;
  }
  const double force = sums[0], torque = sums[1], vexp = sums[2], erot = sums[3];
  const double norm = sums[4], jx = sums[5];
  const double E = ys[2] * ys[2] / (2.0 * mu) + ys[3] * ys[3] / (2.0 * mu * R * R) + erot + vexp;
  if (mode == D5_DIAG) {
    for (int n = threadIdx.x; n < N; n += NT) {
      const double2 a = ws.a0[(int64_t)b * Npad + n];
      out.P[tj.amp_off + n] = a.x * a.x + a.y * a.y;
      if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = a;
      if (out.st_amp) out.st_amp[tj.amp_off + n] = a;
    }
    if (threadIdx.x == 0) {
      const int64_t id = tj.id;
      if (out.classical) {
        double* o = out.classical + id * 6;
        o[0] = ys[0]; o[1] = ws.diag[b * 4 + 2]; o[2] = ys[1]; o[3] = ys[2];
        o[4] = ws.diag[b * 4 + 3]; o[5] = ys[3];
      }
      if (out.t_final) out.t_final[id] = t;
      if (out.steps) out.steps[id] = d.steps[b];
      if (out.rejects) out.rejects[id] = d.rejects[b];
      if (out.status) out.status[id] = ws.status[b];
      if (out.norm_err) out.norm_err[id] = norm - 1.0;
      if (out.energy_err) out.energy_err[id] = (E - ws.diag[b * 4]) / fabs(ws.diag[b * 4]);
      if (out.angmom_err) out.angmom_err[id] = (ys[3] - jx) - ws.diag[b * 4 + 1];
      put_traj_state(out, tj, N, t, t, 0, d.h[b], ys, ws.diag[b * 4 + 2], ws.diag[b * 4 + 3],
                     ws.diag[b * 4], ws.diag[b * 4 + 1], d.rexit[b], d.steps[b], d.rejects[b],
                     d.attempts[b], ws.status[b],
                     (d.flags[b] & D5_LASTREJ) ? MQCT_S_LAST_REJECTED : 0);
    }
    return;
  }
  if (threadIdx.x == 0) {
    if (mode == D5_INIT0 && !(tj.flags & TRAJ_RESUME)) {
      ws.diag[b * 4] = E;
      ws.diag[b * 4 + 1] = ys[3] - jx;
    }
    double* kc = d.kc + (int64_t)b * 32 + slot * 4;
    kc[0] = ys[2] / mu;
    kc[1] = phidot;
    kc[2] = -force + ys[3] * ys[3] / (mu * R * R * R);
    kc[3] = 2.0 * torque;
  }
}

// Starting step, first half (d0 = ||y0||, d1 = ||f(t0, y0)||, h0) and second half
// (d2 = ||f(t0 + h0, y0 + h0 f0) - f0|| / h0, then the step).
__global__ void __launch_bounds__(NT)
d5_start(BinWS ws, D5WS d, const DevSystem* __restrict__ systems, double rtol, double atol,
         int second) {
  __shared__ double red[NWT * 8];
  const int b = blockIdx.x;
  const TrajIn tj = ws.traj[b];
  if (tj.flags & TRAJ_RESUME) return;   // a stored state keeps its step size
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  const double ncomp = 2.0 * N + 6.0;
  const double2* ks = d.ks + (int64_t)b * 8 * Npad;
  double s2[2] = {0.0, 0.0};
  for (int n = threadIdx.x; n < N; n += NT) {
    const double2 a = ws.a0[(int64_t)b * Npad + n], f0 = ks[n];
    const double sx = atol + rtol * fabs(a.x), sy_ = atol + rtol * fabs(a.y);
    if (!second) {
      s2[0] += (a.x / sx) * (a.x / sx) + (a.y / sy_) * (a.y / sy_);
      s2[1] += (f0.x / sx) * (f0.x / sx) + (f0.y / sy_) * (f0.y / sy_);
    } else {
      const double2 f1 = ks[Npad + n];
      const double ex = (f1.x - f0.x) / sx, ey = (f1.y - f0.y) / sy_;
      s2[0] += ex * ex + ey * ey;
    }
  }
  block_sum<2, NWT>(s2, red);
  if (threadIdx.x != 0) return;
  const double* y = ws.ycl + (int64_t)b * 4;
  const double* kc = d.kc + (int64_t)b * 32;
  const double yfull[6] = {y[0], ws.diag[b * 4 + 2], y[1], y[2], ws.diag[b * 4 + 3], y[3]};
  if (!second) {
    const double kf[6] = {kc[0], 0.0, kc[1], kc[2], 0.0, kc[3]};
    for (int k = 0; k < 6; ++k) {
      const double sc = atol + rtol * fabs(yfull[k]);
      s2[0] += (yfull[k] / sc) * (yfull[k] / sc);
      s2[1] += (kf[k] / sc) * (kf[k] / sc);
    }
    const double d0 = sqrt(s2[0] / ncomp), d1 = sqrt(s2[1] / ncomp);
    d.h[b] = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    d.d1[b] = d1;
  } else {
    const double dk[6] = {kc[4] - kc[0], 0.0, kc[5] - kc[1], kc[6] - kc[2], 0.0, kc[7] - kc[3]};
    for (int k = 0; k < 6; ++k) {
      const double sc = atol + rtol * fabs(yfull[k]);
      s2[0] += (dk[k] / sc) * (dk[k] / sc);
    }
    const double h0 = d.h[b], d1 = d.d1[b];
    const double d2 = sqrt(s2[0] / ncomp) / h0;
    const double dm = fmax(d1, d2);
    const double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / 5.0);
    d.h[b] = fmin(100.0 * h0, h1);
  }
}

// Error estimate and decision of one attempt; on acceptance the state moves to
// y5 and k_7 becomes the next attempt's first stage.  Counts the trajectories
// still running.
__global__ void __launch_bounds__(NT)
d5_accept(BinWS ws, D5WS d, const DevSystem* __restrict__ systems, DpCtl ctl,
          long long max_attempts) {
  __shared__ double red[NWT * 8];
  __shared__ int decision;
  const int b = blockIdx.x;
  if (d.flags[b] & D5_DONE) return;
  const TrajIn tj = ws.traj[b];
  const DevSystem sy = systems[tj.sys];
  const int N = sy.N, Npad = sy.Npad;
  const double ncomp = 2.0 * N + 6.0;
  const double h = d.h[b];
  double2* ks = d.ks + (int64_t)b * 8 * Npad;
  double* kc = d.kc + (int64_t)b * 32;
  double* yc = ws.ycl + (int64_t)b * 4;
  double e2[1] = {0.0};
  for (int n = threadIdx.x; n < N; n += NT) {
    double ex = 0.0, ey = 0.0;
    for (int p = 0; p < 7; ++p) {
      const double2 kp = ks[(int64_t)p * Npad + n];
      ex = fma(D5E[p], kp.x, ex);
      ey = fma(D5E[p], kp.y, ey);
    }
    ex *= h; ey *= h;
    const double2 y0 = ws.a0[(int64_t)b * Npad + n], y5 = ks[(int64_t)7 * Npad + n];
    const double sx = ctl.atol + ctl.rtol * fmax(fabs(y0.x), fabs(y5.x));
    const double sy_ = ctl.atol + ctl.rtol * fmax(fabs(y0.y), fabs(y5.y));
    e2[0] += (ex / sx) * (ex / sx) + (ey / sy_) * (ey / sy_);
  }
  block_sum<1, NWT>(e2, red);
  if (threadIdx.x == 0) {
    double ecl = 0.0;
    for (int k = 0; k < 4; ++k) {
      double e = D5E[0] * kc[k];
      for (int p = 1; p < 7; ++p) e = fma(D5E[p], kc[p * 4 + k], e);
      e *= h;
      const double sc = ctl.atol + ctl.rtol * fmax(fabs(yc[k]), fabs(kc[28 + k]));
      ecl += (e / sc) * (e / sc);
    }
    const double en = sqrt((e2[0] + ecl) / ncomp);
    int flags = d.flags[b];
    d.attempts[b] += 1;
    bool done = false, accept = false;
    double hn = h;
    if (!isfinite(en)) {
      ws.status[b] |= ST_NONFINITE;
      done = true;
    } else if (en <= 1.0) {
      accept = true;
      d.t[b] += h;
      for (int k = 0; k < 4; ++k) {
        yc[k] = kc[28 + k];
        kc[k] = kc[24 + k];
      }
      d.steps[b] += 1;
      double fac = en == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(en, -0.2)));
      if (flags & D5_LASTREJ) fac = fmin(1.0, fac);
      flags &= ~D5_LASTREJ;
      if (yc[0] >= d.rexit[b] && yc[2] > 0.0) {
        ws.status[b] |= ST_EXITED;
        done = true;
      } else {
        hn = h * fac;
      }
    } else {
      d.rejects[b] += 1;
      hn = h * fmax(0.2, 0.9 * pow(en, -0.2));
      flags |= D5_LASTREJ;
    }
    if (!done && hn < ctl.h_min) { ws.status[b] |= ST_STEP_UNDERFLOW; done = true; }
    if (!done && d.steps[b] >= ctl.max_steps) { ws.status[b] |= ST_MAX_STEPS; done = true; }
    if (!done && d.attempts[b] >= max_attempts) { ws.status[b] |= ST_MAX_STEPS; done = true; }
    d.h[b] = hn;
    if (done) flags |= D5_DONE;
    else atomicAdd(d.active, 1);
    d.flags[b] = flags;
    decision = accept;
  }
  __syncthreads();
  if (decision) {
    // the accepted state y5 and the first-same-as-last stage
    for (int n = threadIdx.x; n < N; n += NT) {
      ws.a0[(int64_t)b * Npad + n] = ks[(int64_t)7 * Npad + n];
      ks[n] = ks[(int64_t)6 * Npad + n];
    }
  }
}

__global__ void d5_init(BinWS ws, D5WS d) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= ws.B) return;
  const TrajIn& tj = ws.traj[b];
  d.t[b] = tj.t0;
  d.d1[b] = 0.0;
  if (tj.flags & TRAJ_RESUME) {
    // a stored state: step size, rejection flag and counts continue; a
    // trajectory that has stopped for good stays as it is
    d.h[b] = tj.h0;
    d.rexit[b] = tj.R_exit;
    d.steps[b] = tj.steps0;
    d.rejects[b] = tj.rejects0;
    d.attempts[b] = tj.attempts0;
    d.flags[b] = ((tj.dflags & MQCT_S_LAST_REJECTED) ? D5_LASTREJ : 0) |
                 ((tj.flags & TRAJ_FINISHED) ? D5_DONE : 0);
    return;
  }
  d.h[b] = 0.0;
  d.rexit[b] = ws.ycl[(int64_t)b * 4];   // set by bin_init, launched before
  d.steps[b] = 0;
  d.rejects[b] = 0;
  d.attempts[b] = 0;
  d.flags[b] = 0;
}

}  // namespace

size_t binned_workspace_bytes(int B, int Npad, int K, bool fp32) {
  const size_t v = (size_t)B * Npad;
  size_t s = 0;
  s += 4 * al(v * 16);                    // a0, cur, acc, c64
  s += al(v * 2 * 2 * (fp32 ? 4 : 8));    // cst (two real columns, complex worst case)
  s += al(2 * v * 4 * (fp32 ? 4 : 8));    // uv
  s += 4 * al((size_t)B * 32);            // ycl kcl acl ysb
  s += al((size_t)B * 64) + al((size_t)B * 8) + al((size_t)B * 32);   // wts tst diag
  s += 3 * al((size_t)B * 4);             // kb status done
  s += 3 * al((size_t)K * 4);             // cnt cursor offset
  s += al((size_t)2 * B * 4);             // list
  s += al(((size_t)2 * B / TB + K + 1) * 16) + al(16);   // items, n_items
  s += al(16);                                            // occ
  return s;
}

namespace {

// Carves the schedule's buffers out of the workspace; returns the first byte past them.
char* carve(BinWS& ws, const DevSystem& hs, const TrajIn* d_traj, int B, void* wsp) {
  const bool fp32 = dtype_fp32(hs.dtype);
  ws.B = B; ws.N = hs.N; ws.Npad = hs.Npad; ws.K = hs.K;
  ws.traj = d_traj;
  char* p = (char*)wsp;
  auto take = [&](size_t bytes) { void* q = p; p += al(bytes); return q; };
  const size_t v = (size_t)B * hs.Npad;
  ws.a0 = (double2*)take(v * 16);
  ws.cur = (double2*)take(v * 16);
  ws.acc = (double2*)take(v * 16);
  ws.c64 = (double2*)take(v * 16);
  ws.cst = take(v * 2 * 2 * (fp32 ? 4 : 8));
  ws.uv = take(2 * v * 4 * (fp32 ? 4 : 8));
  ws.ycl = (double*)take((size_t)B * 32);
  ws.kcl = (double*)take((size_t)B * 32);
  ws.acl = (double*)take((size_t)B * 32);
  ws.ysb = (double*)take((size_t)B * 32);
  ws.wts = (double*)take((size_t)B * 64);
  ws.tst = (double*)take((size_t)B * 8);
  ws.diag = (double*)take((size_t)B * 32);
  ws.kb = (int*)take((size_t)B * 4);
  ws.status = (int*)take((size_t)B * 4);
  ws.done = (int*)take((size_t)B * 4);
  ws.cnt = (int*)take((size_t)hs.K * 4);
  ws.cursor = (int*)take((size_t)hs.K * 4);
  ws.offset = (int*)take((size_t)hs.K * 4);
  ws.list = (int*)take((size_t)2 * B * 4);
  const int max_items = 2 * B / TB + hs.K + 1;
  ws.items = (int4*)take((size_t)max_items * 16);
  ws.n_items = (int*)take(16);
  ws.occ = (unsigned long long*)take(16);
  return p;
}

// The product of one stage: bin offsets and work list, bin lists, products
// (timed when profiling).
hipError_t stage_product(BinWS& ws, const DevSystem* d_systems, const DevSystem& hs, int B,
                         hipStream_t s, Prof* prof) {
  const int max_items = 2 * B / TB + hs.K + 1;
  const int rows_per_block = 2 * 4 * 16;
  const int nrb = (hs.N + rows_per_block - 1) / rows_per_block;
  const dim3 ggrid((unsigned)((int64_t)(max_items + NXCD - 1) / NXCD * nrb * NXCD));
  bin_scan<<<1, 1024, 0, s>>>(ws);
  bin_scatter<<<(B + 255) / 256, 256, 0, s>>>(ws);
  hipEvent_t e0 = prof ? prof->next() : nullptr, e1 = prof ? prof->next() : nullptr;
  prof_mark(prof, e0, s);
  if (hs.dtype == C64) bin_gemm<C64><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
  else if (hs.dtype == C128) bin_gemm<C128><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
  else if (hs.dtype == R32) bin_gemm<R32><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
  else bin_gemm<R64><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
  prof_mark(prof, e1, s);
  return hipGetLastError();
}

}  // namespace

hipError_t run_binned(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                      int B, int64_t max_steps, const double* d_a0, TrajOut out, void* wsp,
                      hipStream_t s, Prof* prof) {
  BinWS ws;
  carve(ws, hs, d_traj, B, wsp);
  hipError_t e;
  bin_init<<<B, NT, 0, s>>>(ws, d_systems, d_a0);
  bin_zero<<<(hs.K + 255) / 256, 256, 0, s>>>(ws.cnt, hs.K);
  bin_zero<<<(hs.K + 255) / 256, 256, 0, s>>>(ws.cursor, hs.K);
  bin_zero<<<1, 256, 0, s>>>((int*)ws.occ, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  auto prep = [&](int64_t j, int st, int diag) {
    if (hs.dtype == C64) bin_prep<float, true><<<B, NT, 0, s>>>(ws, d_systems, j, st, diag);
    else if (hs.dtype == C128) bin_prep<double, true><<<B, NT, 0, s>>>(ws, d_systems, j, st, diag);
    else if (hs.dtype == R32) bin_prep<float, false><<<B, NT, 0, s>>>(ws, d_systems, j, st, diag);
    else bin_prep<double, false><<<B, NT, 0, s>>>(ws, d_systems, j, st, diag);
  };
  // c of a stage and its phases in LDS when they fit the default 64 KiB
  const bool ldsc = (size_t)hs.Npad * 32 <= 65536;
  const size_t clds = ldsc ? (size_t)hs.Npad * 32 : 0;
  auto combine = [&](auto sc, auto cx, int64_t j, int st, int diag, int next) {
    using S = decltype(sc);
    constexpr bool CX = decltype(cx)::value;
    if (ldsc) bin_combine<S, CX, true><<<B, NT, clds, s>>>(ws, d_systems, j, st, diag, next, out);
    else bin_combine<S, CX, false><<<B, NT, 0, s>>>(ws, d_systems, j, st, diag, next, out);
  };
  auto stage = [&](int64_t j, int st, int diag, int next) -> hipError_t {
    hipError_t pe = stage_product(ws, d_systems, hs, B, s, prof);
    if (pe != hipSuccess) return pe;
    if (hs.dtype == C64) combine(0.0f, std::true_type{}, j, st, diag, next);
    else if (hs.dtype == C128) combine(0.0, std::true_type{}, j, st, diag, next);
    else if (hs.dtype == R32) combine(0.0f, std::false_type{}, j, st, diag, next);
    else combine(0.0, std::false_type{}, j, st, diag, next);
    return hipGetLastError();
  };
  // the first stage is prepared on its own, every later one by the combine of
  // the stage before it, the final diagnostic evaluation on its own again
  if (max_steps > 0) prep(0, 0, 0);
  for (int64_t j = 0; j < max_steps; ++j)
    for (int st = 0; st < 4; ++st)
      if ((e = stage(j, st, 0, !(j == max_steps - 1 && st == 3))) != hipSuccess) return e;
  prep(max_steps, 0, 1);
  if ((e = stage(max_steps, 0, 1, 0)) != hipSuccess) return e;
  // algorithmic table bytes of the timed products: each occupied knot's value
  // and second-derivative slices, read once per stage
  unsigned long long* slot =
      prof ? prof->knot_slot(2.0 * hs.N * (double)hs.Npad * dtype_bytes(hs.dtype)) : nullptr;
  if (slot) e = hipMemcpyAsync(slot, ws.occ, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  return e;
}

size_t binned_dp5_workspace_bytes(int B, int Npad, int K, bool fp32) {
  size_t s = binned_workspace_bytes(B, Npad, K, fp32);
  s += al((size_t)B * 8 * Npad * 16);     // ks
  s += al((size_t)B * 32 * 8);            // kc
  s += 4 * al((size_t)B * 8);             // h t rexit d1
  s += 3 * al((size_t)B * 8);             // steps rejects attempts
  s += al((size_t)B * 4) + al(16);        // flags active
  return s;
}

hipError_t run_binned_dp5(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                          int B, const double* d_a0, TrajOut out, DpCtl ctl,
                          int64_t max_attempts, void* wsp, hipStream_t s, Prof* prof) {
  BinWS ws;
  char* p = carve(ws, hs, d_traj, B, wsp);
  auto take = [&](size_t bytes) { void* q = p; p += al(bytes); return q; };
  D5WS d;
  d.ks = (double2*)take((size_t)B * 8 * hs.Npad * 16);
  d.kc = (double*)take((size_t)B * 32 * 8);
  d.h = (double*)take((size_t)B * 8);
  d.t = (double*)take((size_t)B * 8);
  d.rexit = (double*)take((size_t)B * 8);
  d.d1 = (double*)take((size_t)B * 8);
  d.steps = (long long*)take((size_t)B * 8);
  d.rejects = (long long*)take((size_t)B * 8);
  d.attempts = (long long*)take((size_t)B * 8);
  d.flags = (int*)take((size_t)B * 4);
  d.active = (int*)take(16);
  hipError_t e;
  bin_init<<<B, NT, 0, s>>>(ws, d_systems, d_a0);
  d5_init<<<(B + 255) / 256, 256, 0, s>>>(ws, d);
  bin_zero<<<(hs.K + 255) / 256, 256, 0, s>>>(ws.cnt, hs.K);
  bin_zero<<<(hs.K + 255) / 256, 256, 0, s>>>(ws.cursor, hs.K);
  bin_zero<<<1, 256, 0, s>>>((int*)ws.occ, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const bool ldsc = (size_t)hs.Npad * 16 <= 65536;
  const size_t clds = ldsc ? (size_t)hs.Npad * 16 : 0;
  auto run = [&](auto sc, auto cx) -> hipError_t {
    using S = decltype(sc);
    constexpr bool CX = decltype(cx)::value;
    auto stage = [&](int mode, int sg, int slot) -> hipError_t {
      d5_prep<S, CX><<<B, NT, 0, s>>>(ws, d, d_systems, mode, sg);
      hipError_t pe = stage_product(ws, d_systems, hs, B, s, prof);
      if (pe != hipSuccess) return pe;
      if (ldsc) d5_combine<S, CX, true><<<B, NT, clds, s>>>(ws, d, d_systems, mode, slot, out);
      else d5_combine<S, CX, false><<<B, NT, 0, s>>>(ws, d, d_systems, mode, slot, out);
      return hipGetLastError();
    };
    hipError_t r;
    if ((r = stage(D5_INIT0, 0, 0)) != hipSuccess) return r;
    d5_start<<<B, NT, 0, s>>>(ws, d, d_systems, ctl.rtol, ctl.atol, 0);
    if ((r = stage(D5_INIT1, 0, 1)) != hipSuccess) return r;
    d5_start<<<B, NT, 0, s>>>(ws, d, d_systems, ctl.rtol, ctl.atol, 1);
    // attempt rounds; the count of running trajectories is read every few rounds
    constexpr int CHECK = 8;
    for (int64_t a = 0; a < max_attempts; ++a) {
      for (int sg = 1; sg < 7; ++sg)
        if ((r = stage(D5_STAGE, sg, sg)) != hipSuccess) return r;
      const bool check = (a % CHECK) == CHECK - 1 || a == max_attempts - 1;
      if (check) bin_zero<<<1, 64, 0, s>>>(d.active, 1);
      d5_accept<<<B, NT, 0, s>>>(ws, d, d_systems, ctl, (long long)max_attempts);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if (check) {
        int running = 0;
        if ((r = hipMemcpyAsync(&running, d.active, sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
          return r;
        if ((r = hipStreamSynchronize(s)) != hipSuccess) return r;
        if (running == 0) break;
      }
    }
    return stage(D5_DIAG, 0, 0);
  };
  if (hs.dtype == C64) e = run(0.0f, std::true_type{});
  else if (hs.dtype == C128) e = run(0.0, std::true_type{});
  else if (hs.dtype == R32) e = run(0.0f, std::false_type{});
  else e = run(0.0, std::false_type{});
  if (e != hipSuccess) return e;
  unsigned long long* slot =
      prof ? prof->knot_slot(2.0 * hs.N * (double)hs.Npad * dtype_bytes(hs.dtype)) : nullptr;
  if (slot) e = hipMemcpyAsync(slot, ws.occ, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  return e;
}

}  // namespace mqct

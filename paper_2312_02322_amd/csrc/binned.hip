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
  int* n_items;           // [1]
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
    ws.status[b] = 0;
    ws.done[b] = -1;
  }
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
  const double t = tj.t0 + (double)jsteps * h + cf;
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

constexpr int GEMM_PF32 = 2;   // K steps of operands in flight, FP32 tables (deeper rings measured slower)
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
  const double tn = tj.t0 + (double)jn * h + cfn;
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
    const int64_t steps = ws.done[b] >= 0 ? (int64_t)ws.done[b] : tj.n_steps;
    for (int n = threadIdx.x; n < N; n += NT) {
      const double2 a = ws.a0[(int64_t)b * Npad + n];
      out.P[tj.amp_off + n] = a.x * a.x + a.y * a.y;
      if (out.a_final) ((double2*)out.a_final)[tj.amp_off + n] = a;
    }
    if (threadIdx.x == 0) {
      const int64_t id = tj.id;
      if (out.classical) {
        double* o = out.classical + id * 6;
        o[0] = ys[0]; o[1] = ws.diag[b * 4 + 2]; o[2] = ys[1]; o[3] = ys[2];
        o[4] = ws.diag[b * 4 + 3]; o[5] = ys[3];
      }
      if (out.t_final) out.t_final[id] = t;
      if (out.steps) out.steps[id] = steps;
      if (out.rejects) out.rejects[id] = 0;
      if (out.status) out.status[id] = ws.status[b];
      if (out.norm_err) out.norm_err[id] = norm - 1.0;
      if (out.energy_err) {
        const double E0 = steps > 0 ? ws.diag[b * 4] : E;
        out.energy_err[id] = (E - E0) / fabs(E0);
      }
      if (out.angmom_err) {
        const double J0 = steps > 0 ? ws.diag[b * 4 + 1] : ys[3] - jx;
        out.angmom_err[id] = (ys[3] - jx) - J0;
      }
    }
    return;
  }
  if (threadIdx.x == 0) {
    if (j == 0 && st == 0) {
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

hipError_t run_binned(const DevSystem* d_systems, const DevSystem& hs, const TrajIn* d_traj,
                      int B, int64_t max_steps, const double* d_a0, TrajOut out, void* wsp,
                      hipStream_t s, Prof* prof) {
  const bool fp32 = dtype_fp32(hs.dtype);
  BinWS ws;
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

  const int rows_per_block = 2 * 4 * 16;
  const int nrb = (hs.N + rows_per_block - 1) / rows_per_block;
  const int64_t gblocks = (int64_t)(max_items + NXCD - 1) / NXCD * nrb * NXCD;
  const dim3 ggrid((unsigned)gblocks);
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
    bin_scan<<<1, 1024, 0, s>>>(ws);
    bin_scatter<<<(B + 255) / 256, 256, 0, s>>>(ws);
    hipEvent_t e0 = prof ? prof->next() : nullptr, e1 = prof ? prof->next() : nullptr;
    prof_mark(prof, e0, s);
    if (hs.dtype == C64) bin_gemm<C64><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
    else if (hs.dtype == C128) bin_gemm<C128><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
    else if (hs.dtype == R32) bin_gemm<R32><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
    else bin_gemm<R64><<<ggrid, 256, GEMM_LDS_CAP, s>>>(ws, d_systems, nrb);
    prof_mark(prof, e1, s);
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

}  // namespace mqct

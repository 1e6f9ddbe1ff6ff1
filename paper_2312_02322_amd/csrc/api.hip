// C ABI of libmqct: contexts, system loading and batch launch (include/mqct.h).
#include "internal.h"

#include "../../include/mqct.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <thread>
#include <utility>
#include <vector>

using namespace mqct;

namespace {

// An adaptive batch on the default schedule sends the trajectories of a dense
// system with at least this padded size and count to the binned schedule.
constexpr int SPLIT_MIN_NPAD = 512;
constexpr int64_t SPLIT_MIN_TRAJ = 256;

struct SysHost {
  bool live = false;
  DevSystem dev{};
  void* bufs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t table_bytes = 0;
  // optional linear parametric form of the tables (adjoint)
  int P = 0, nG = 0;
  // G (dense), rad, rad2, gidx, then the nonzeros of G: offsets, row | col << 16, values
  void* pbufs[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<int> h_goff;   // the offsets of the G nonzero lists, on the host
  void* dbuf = nullptr;   // driving potential of AT dynamics and its curvature: [2][K]
  void* ebuf[2] = {nullptr, nullptr};   // sparse tables: slot lists [W][Npad], kept per column [N]
  double R_last = 0.0;    // last knot (the default start radius), kept on the host
};

// Device scratch of mqct_run_noalloc: the trajectory records and start amplitudes
// of one call.  Every GPU the library runs on holds its own copy until the
// process ends; every call on a GPU shares it.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Every device allocation of the library goes through here.  Fault injection
// for the error paths, from the environment (read at every call):
// MQCT_FAULT=alloc fails each allocation as out of device memory;
// MQCT_FAULT=alloc@n fails only the n-th allocation counted from the call that
// first saw that value.
template <typename T>
hipError_t dev_malloc(T** p, size_t bytes) {
  static std::string seen;
  static long count = 0;
  const char* f = getenv("MQCT_FAULT");
  if (f && strncmp(f, "alloc", 5) == 0) {
    if (f[5] == '\0') return hipErrorOutOfMemory;
    if (f[5] == '@') {
      if (seen != f) {
        seen = f;
        count = 0;
      }
      if (++count == atol(f + 6)) return hipErrorOutOfMemory;
    }
  }
  return hipMalloc((void**)p, bytes);
}

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct mqct_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<SysHost> systems;
  DevSystem* d_systems = nullptr;
  size_t d_systems_cap = 0;
  DevBuf traj, a0, outs[10], xs[4], qws, binws;
  hipStream_t cap = nullptr;       // non-default stream on which graphs are captured
  hipStream_t side = nullptr;      // second stream: the binned share of a split adaptive batch
  hipEvent_t side_done = nullptr;  // recorded on `side` when that share has been enqueued
  int* h_counts = nullptr;         // pinned host copy of the work-list counts
  size_t h_counts_cap = 0;
  QueueOpts qopt;                  // work-list schedule options
  QueueCache qcache;               // autotuner decisions
  std::string report;              // last text of mqct_tuning_report
  TrajIn* h_traj = nullptr;        // pinned staging for trajectory records
  size_t h_traj_cap = 0;
  hipEvent_t staged = nullptr;     // recorded after the last upload from h_traj
  Prof prof;                       // optional timing of the dominant step kernel
  unsigned char* scratch = nullptr;   // device address of this GPU's copy of `scratch`
  // state store: the final state of every trajectory of the last run (or what
  // mqct_set_state wrote), records by batch index, amplitudes concatenated
  DevBuf st_rec, st_amp;
  int64_t st_B = 0;
  std::vector<int32_t> st_sys;     // system of each stored trajectory
  std::vector<int64_t> st_off;     // amplitude offsets, [st_B + 1]
};

namespace {

mqct_status fail(mqct_context* c, mqct_status code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

mqct_status hip_fail(mqct_context* c, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(c, MQCT_ERR_OOM, "%s: out of device memory", what);
  return fail(c, MQCT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)              \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

mqct_status ensure(mqct_context* c, DevBuf& b, size_t bytes, const char* what) {
  if (bytes <= b.cap) return MQCT_OK;
  if (b.p) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, what);
    hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = std::max(bytes, (size_t)4096);
  HIP_TRY(c, dev_malloc(&b.p, want), what);
  b.cap = want;
  return MQCT_OK;
}

mqct_status upload_systems(mqct_context* c) {
  std::vector<DevSystem> h(c->systems.size());
  for (size_t i = 0; i < h.size(); ++i) h[i] = c->systems[i].dev;
  size_t bytes = std::max<size_t>(1, h.size()) * sizeof(DevSystem);
  if (bytes > c->d_systems_cap) {
    HIP_TRY(c, hipStreamSynchronize(c->stream), "system table");
    if (c->d_systems) hipFree(c->d_systems);
    c->d_systems = nullptr;
    size_t want = bytes * 2;
    HIP_TRY(c, dev_malloc((void**)&c->d_systems, want), "system table");
    c->d_systems_cap = want;
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_systems, h.data(), h.size() * sizeof(DevSystem),
                            hipMemcpyHostToDevice, c->stream), "system table");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "system table");
  return MQCT_OK;
}

bool finite_arr(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(p[i])) return false;
  return true;
}

void free_params(SysHost& s) {
  for (auto& p : s.pbufs) {
    if (p) hipFree(p);
    p = nullptr;
  }
  s.P = s.nG = 0;
  s.h_goff.clear();
}

void free_system(SysHost& s) {
  for (auto& p : s.bufs) {
    if (p) hipFree(p);
    p = nullptr;
  }
  free_params(s);
  if (s.dbuf) hipFree(s.dbuf);
  s.dbuf = nullptr;
  for (auto& p : s.ebuf) {
    if (p) hipFree(p);
    p = nullptr;
  }
  s.live = false;
}

// J_x (Eq. 5's Coriolis operator) from a coordinate list: range, symmetry and
// equal-energy checks, then the ELL form [N][W] (padding entries point at the
// row itself with value 0).  W = 0 when there is no Coriolis term.
mqct_status build_jx(mqct_context* c, const char* who, int N, const double* E, int nnz,
                     const int32_t* jrow, const int32_t* jcol, const double* jval,
                     std::vector<int32_t>& col, std::vector<double>& val, int& W) {
  if (nnz < 0 || (nnz > 0 && (!jrow || !jcol || !jval)))
    return fail(c, MQCT_ERR_ARG, "%s: bad J_x arrays", who);
  std::vector<std::vector<std::pair<int, double>>> rows(N);
  std::map<std::pair<int, int>, double> jmap;
  for (int q = 0; q < nnz; ++q) {
    int r = jrow[q], cc = jcol[q];
    double v = jval[q];
    if (r < 0 || r >= N || cc < 0 || cc >= N)
      return fail(c, MQCT_ERR_ARG, "%s: J_x index out of range at %d", who, q);
    if (!isfinite(v)) return fail(c, MQCT_ERR_NONFINITE, "%s: non-finite J_x", who);
    if (jmap.count({r, cc})) return fail(c, MQCT_ERR_ARG, "%s: duplicate J_x entry", who);
    jmap[{r, cc}] = v;
    rows[r].push_back({cc, v});
  }
  for (auto& kv : jmap) {
    auto it = jmap.find({kv.first.second, kv.first.first});
    if (it == jmap.end() || fabs(it->second - kv.second) > 1e-12 * (1.0 + fabs(kv.second)))
      return fail(c, MQCT_ERR_ARG, "%s: J_x is not symmetric", who);
  }
  // Eq. 5: the Coriolis term couples m +- 1 within one channel n, i.e. states of
  // equal energy; the kernels rely on that (J_x a = e^{iEt} J_x c row by row).
  double emax = 0.0;
  for (int n = 0; n < N; ++n) emax = std::max(emax, fabs(E[n]));
  for (auto& kv : jmap)
    if (fabs(E[kv.first.first] - E[kv.first.second]) > 1e-12 * emax)
      return fail(c, MQCT_ERR_ARG, "%s: J_x couples channels of different energy", who);
  W = 0;
  for (auto& r : rows) W = std::max<int>(W, (int)r.size());
  if (W > 8) return fail(c, MQCT_ERR_UNSUPPORTED, "%s: J_x has more than 8 nonzeros per row", who);
  col.assign((size_t)N * W, 0);
  val.assign((size_t)N * W, 0.0);
  for (int r = 0; r < N; ++r)
    for (int w = 0; w < W; ++w) {
      const bool have = w < (int)rows[r].size();
      col[(size_t)r * W + w] = have ? rows[r][w].first : r;
      val[(size_t)r * W + w] = have ? rows[r][w].second : 0.0;
    }
  return MQCT_OK;
}

}  // namespace

extern "C" {

mqct_status mqct_create(int32_t device, void* hip_stream, mqct_context** out) {
  if (!out) return MQCT_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MQCT_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return MQCT_ERR_DEVICE;
  mqct_context* c = new mqct_context();
  c->device = device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return MQCT_ERR_DEVICE; }
    c->own_stream = true;
  }
  if (hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess) {
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return MQCT_ERR_DEVICE;
  }
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->side_done, hipEventDisableTiming) != hipSuccess) {
    if (c->cap) hipStreamDestroy(c->cap);
    if (c->side) hipStreamDestroy(c->side);
    hipEventDestroy(c->staged);
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return MQCT_ERR_DEVICE;
  }
  // the address of this device's copy of the static scratch array (the host-side
  // name is not a device address)
  if (hipGetSymbolAddress((void**)&c->scratch, HIP_SYMBOL(scratch)) != hipSuccess) {
    hipEventDestroy(c->side_done);
    hipStreamDestroy(c->side);
    hipStreamDestroy(c->cap);
    hipEventDestroy(c->staged);
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return MQCT_ERR_DEVICE;
  }
  *out = c;
  return MQCT_OK;
}

void mqct_destroy(mqct_context* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto& s : c->systems) free_system(s);
  if (c->d_systems) hipFree(c->d_systems);
  DevBuf* all[] = {&c->traj, &c->a0, &c->xs[0], &c->xs[1], &c->xs[2], &c->xs[3],
                   &c->qws, &c->binws, &c->st_rec, &c->st_amp};
  for (DevBuf* b : all) if (b->p) hipFree(b->p);
  for (auto& b : c->outs) if (b.p) hipFree(b.p);
  if (c->h_traj) hipHostFree(c->h_traj);
  if (c->h_counts) hipHostFree(c->h_counts);
  if (c->side) hipStreamSynchronize(c->side);
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->side) hipStreamDestroy(c->side);
  if (c->side_done) hipEventDestroy(c->side_done);
  if (c->staged) hipEventDestroy(c->staged);
  for (hipEvent_t e : c->prof.ev) hipEventDestroy(e);
  if (c->prof.slots) hipHostFree(c->prof.slots);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
}

const char* mqct_last_error(const mqct_context* c) {
  if (!c) return "no context";
  return c->err.c_str();
}

mqct_status mqct_synchronize(mqct_context* c) {
  if (!c) return MQCT_ERR_ARG;
  HIP_TRY(c, hipSetDevice(c->device), "synchronize");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  return MQCT_OK;
}

mqct_status mqct_system_load(mqct_context* c, const mqct_system_desc* d, int32_t* system_id) {
  if (!c) return MQCT_ERR_ARG;
  if (!d || !system_id) return fail(c, MQCT_ERR_ARG, "system_load: null argument");
  const int N = d->N, K = d->K;
  if (N < 1 || K < 4 || K > 2048)
    return fail(c, MQCT_ERR_ARG, "system_load: need N >= 1 and 4 <= K <= 2048 (N=%d K=%d)", N, K);
  if (!d->R_grid || !d->E || !d->M) return fail(c, MQCT_ERR_ARG, "system_load: null R_grid/E/M");
  if (d->in_dtype != MQCT_R64 && d->in_dtype != MQCT_C128)
    return fail(c, MQCT_ERR_ARG, "system_load: in_dtype must be MQCT_R64 or MQCT_C128");
  if (d->storage < MQCT_R64 || d->storage > MQCT_C64)
    return fail(c, MQCT_ERR_ARG, "system_load: unknown storage type %d", d->storage);
  const bool cplx = d->in_dtype == MQCT_C128;
  if (dtype_complex(d->storage) != cplx)
    return fail(c, MQCT_ERR_ARG, "system_load: storage and input must both be real or both complex");
  if (d->M_mem != MQCT_MEM_HOST && d->M_mem != MQCT_MEM_DEVICE)
    return fail(c, MQCT_ERR_ARG, "system_load: M_mem must be host or device");
  if (!(d->mu > 0.0) || !isfinite(d->mu)) return fail(c, MQCT_ERR_ARG, "system_load: mu must be > 0");
  if (d->layout != MQCT_DENSE && d->layout != MQCT_SPARSE)
    return fail(c, MQCT_ERR_ARG, "system_load: unknown layout %d", d->layout);
  if (!(d->drop_below >= 0.0) || !isfinite(d->drop_below))
    return fail(c, MQCT_ERR_ARG, "system_load: drop_below must be finite and >= 0");
  if (!finite_arr(d->R_grid, K)) return fail(c, MQCT_ERR_NONFINITE, "system_load: non-finite R grid");
  for (int k = 1; k < K; ++k)
    if (!(d->R_grid[k] > d->R_grid[k - 1]))
      return fail(c, MQCT_ERR_ARG, "system_load: R grid not strictly increasing at %d", k);
  if (!finite_arr(d->E, N)) return fail(c, MQCT_ERR_NONFINITE, "system_load: non-finite E");
  // Coriolis operator: coordinate list -> ELL, checked for range and symmetry
  std::vector<int32_t> jx_col_h;
  std::vector<double> jx_val_h;
  int W = 0;
  {
    const mqct_status js = build_jx(c, "system_load", N, d->E, d->jx_nnz, d->jx_row, d->jx_col,
                                    d->jx_val, jx_col_h, jx_val_h, W);
    if (js != MQCT_OK) return js;
  }

  HIP_TRY(c, hipSetDevice(c->device), "system_load");
  const int ncomp = cplx ? 2 : 1;
  const int Npad = (N + 15) / 16 * 16;
  const int64_t in_elems = (int64_t)K * N * N * ncomp;
  const int64_t store_elems = (int64_t)K * N * Npad * ncomp;
  const int es = dtype_fp32(d->storage) ? 4 : 8;

  SysHost sh;
  sh.dev.N = N; sh.dev.K = K; sh.dev.Npad = Npad; sh.dev.dtype = d->storage;
  sh.dev.jx_w = W; sh.dev.mu = d->mu; sh.dev.knot_stride = (int64_t)N * Npad;
  {
    // a uniform grid lets the interval lookup start from a guess one step off at most
    const double hu = (d->R_grid[K - 1] - d->R_grid[0]) / (K - 1);
    bool uniform = true;
    for (int k = 0; k < K && uniform; ++k)
      uniform = fabs(d->R_grid[k] - (d->R_grid[0] + k * hu)) <= 1e-9 * hu;
    sh.dev.R_inv_h = uniform ? 1.0 / hu : 0.0;
  }
  sh.table_bytes = 2 * store_elems * es;

  double* din = nullptr;
  bool own_in = false;
  unsigned long long* stats = nullptr;
  double* tmp = nullptr;
  mqct_status st = MQCT_OK;
  auto cleanup = [&]() {
    if (own_in && din) hipFree(din);
    if (stats) hipFree(stats);
    if (tmp) hipFree(tmp);
  };
  auto dfail = [&](hipError_t e, const char* what) {
    cleanup();
    free_system(sh);
    return hip_fail(c, e, what);
  };
  hipError_t e;
  if (d->M_mem == MQCT_MEM_HOST) {
    if ((e = dev_malloc((void**)&din, in_elems * 8)) != hipSuccess) return dfail(e, "system_load: input");
    own_in = true;
    if ((e = hipMemcpy(din, d->M, in_elems * 8, hipMemcpyHostToDevice)) != hipSuccess)
      return dfail(e, "system_load: upload");
  } else {
    din = (double*)d->M;
  }
  if ((e = dev_malloc((void**)&stats, 3 * sizeof(unsigned long long))) != hipSuccess)
    return dfail(e, "system_load: stats");
  if ((e = hipMemsetAsync(stats, 0, 3 * sizeof(unsigned long long), c->stream)) != hipSuccess)
    return dfail(e, "system_load: stats");
  if ((e = launch_validate(din, N, K, ncomp, stats, c->stream)) != hipSuccess)
    return dfail(e, "system_load: validate");
  unsigned long long hs[3];
  if ((e = hipMemcpyAsync(hs, stats, sizeof hs, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return dfail(e, "system_load: validate");
  double herm, amax;
  memcpy(&herm, &hs[0], 8);
  memcpy(&amax, &hs[1], 8);
  if (hs[2] > 0) {
    cleanup();
    return fail(c, MQCT_ERR_NONFINITE, "system_load: %llu non-finite table entries", hs[2]);
  }
  if (herm > 1e-12 * amax) {
    cleanup();
    return fail(c, MQCT_ERR_NOT_HERMITIAN, "system_load: |M - M^H| = %.3e > 1e-12 max|M| = %.3e",
                herm, 1e-12 * amax);
  }
  // storage, spline curvature, small arrays
  if ((e = dev_malloc(&sh.bufs[0], store_elems * es)) != hipSuccess) return dfail(e, "system_load: tables");
  if ((e = dev_malloc(&sh.bufs[1], store_elems * es)) != hipSuccess) return dfail(e, "system_load: tables");
  if ((e = dev_malloc(&sh.bufs[2], K * 8)) != hipSuccess) return dfail(e, "system_load: grid");
  if ((e = dev_malloc(&sh.bufs[3], N * 8)) != hipSuccess) return dfail(e, "system_load: energies");
  int64_t per_col = (int64_t)N * Npad * ncomp;
  int64_t tmp_doubles = std::min<int64_t>((int64_t)K * per_col, (int64_t)64 << 20);
  tmp_doubles = std::max<int64_t>(tmp_doubles, K);
  if ((e = dev_malloc((void**)&tmp, tmp_doubles * 8)) != hipSuccess) return dfail(e, "system_load: scratch");
  if ((e = hipMemcpy(sh.bufs[2], d->R_grid, K * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return dfail(e, "system_load: grid");
  if ((e = hipMemcpy(sh.bufs[3], d->E, N * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return dfail(e, "system_load: energies");
  if ((e = launch_spline_prepare(din, (const double*)sh.bufs[2], N, K, Npad, ncomp, d->storage,
                                 sh.bufs[0], sh.bufs[1], tmp, tmp_doubles, c->stream)) != hipSuccess)
    return dfail(e, "system_load: spline");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return dfail(e, "system_load: spline");
  if (d->layout == MQCT_SPARSE) {
    // keep the elements above drop_below somewhere on the grid; slot lists per column
    double* amax = nullptr;
    auto efail = [&](hipError_t err, const char* what) {
      if (amax) hipFree(amax);
      return dfail(err, what);
    };
    if ((e = dev_malloc((void**)&amax, (size_t)N * N * 8)) != hipSuccess) return efail(e, "system_load: pattern");
    if ((e = dev_malloc(&sh.ebuf[1], (size_t)N * 4)) != hipSuccess) return efail(e, "system_load: pattern");
    if ((e = launch_ell_pattern(din, N, K, ncomp, d->drop_below, amax, (int*)sh.ebuf[1], c->stream)) != hipSuccess)
      return efail(e, "system_load: pattern");
    std::vector<int> cnt(N);
    if ((e = hipMemcpyAsync(cnt.data(), sh.ebuf[1], (size_t)N * 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
      return efail(e, "system_load: pattern");
    int Wm = 1;
    for (int n = 0; n < N; ++n) Wm = std::max(Wm, cnt[n]);
    void* E = nullptr;
    void* E2 = nullptr;
    const size_t ebytes = (size_t)K * Wm * Npad * ncomp * es;
    if ((e = dev_malloc(&sh.ebuf[0], (size_t)Wm * Npad * 4)) != hipSuccess) return efail(e, "system_load: slots");
    if ((e = launch_ell_fill(amax, N, Npad, Wm, d->drop_below, (int32_t*)sh.ebuf[0], c->stream)) != hipSuccess)
      return efail(e, "system_load: slots");
    if ((e = dev_malloc(&E, ebytes)) != hipSuccess) return efail(e, "system_load: sparse tables");
    if ((e = dev_malloc(&E2, ebytes)) != hipSuccess) { hipFree(E); return efail(e, "system_load: sparse tables"); }
    if ((e = launch_ell_gather(sh.bufs[0], sh.bufs[1], (const int32_t*)sh.ebuf[0], (const int*)sh.ebuf[1],
                               N, Npad, K, Wm, ncomp, d->storage, E, E2, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
      hipFree(E);
      hipFree(E2);
      return efail(e, "system_load: sparse tables");
    }
    hipFree(amax);
    hipFree(sh.bufs[0]);
    hipFree(sh.bufs[1]);
    sh.bufs[0] = E;
    sh.bufs[1] = E2;
    sh.dev.ell_w = Wm;
    sh.dev.ell_col = (const int32_t*)sh.ebuf[0];
    sh.dev.knot_stride = (int64_t)Wm * Npad;
    sh.table_bytes = 2 * (int64_t)ebytes;
  }
  if (W > 0) {
    if ((e = dev_malloc(&sh.bufs[4], jx_col_h.size() * 4)) != hipSuccess) return dfail(e, "system_load: J_x");
    if ((e = dev_malloc(&sh.bufs[5], jx_val_h.size() * 8)) != hipSuccess) return dfail(e, "system_load: J_x");
    if ((e = hipMemcpy(sh.bufs[4], jx_col_h.data(), jx_col_h.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(sh.bufs[5], jx_val_h.data(), jx_val_h.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
      return dfail(e, "system_load: J_x");
  }
  cleanup();
  sh.dev.M = sh.bufs[0];
  sh.dev.M2 = sh.bufs[1];
  sh.dev.R = (const double*)sh.bufs[2];
  sh.dev.E = (const double*)sh.bufs[3];
  sh.dev.jx_col = (const int32_t*)sh.bufs[4];
  sh.dev.jx_val = (const double*)sh.bufs[5];
  sh.R_last = d->R_grid[K - 1];
  sh.live = true;
  int id = -1;
  for (size_t i = 0; i < c->systems.size(); ++i)
    if (!c->systems[i].live) { id = (int)i; break; }
  if (id < 0) { id = (int)c->systems.size(); c->systems.push_back(sh); }
  else c->systems[id] = sh;
  st = upload_systems(c);
  if (st != MQCT_OK) return st;
  *system_id = id;
  return MQCT_OK;
}

mqct_status mqct_system_load_coo(mqct_context* c, const mqct_coo_desc* d, int32_t* system_id) {
  if (!c) return MQCT_ERR_ARG;
  if (!d || !system_id) return fail(c, MQCT_ERR_ARG, "system_load_coo: null argument");
  const int N = d->N, K = d->K;
  if (N < 1 || K < 4 || K > 2048)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: need N >= 1 and 4 <= K <= 2048 (N=%d K=%d)", N, K);
  if (!d->R_grid || !d->E || !d->rows || !d->cols || !d->values)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: null R_grid/E/rows/cols/values");
  if (d->in_dtype != MQCT_R64 && d->in_dtype != MQCT_C128)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: in_dtype must be MQCT_R64 or MQCT_C128");
  if (d->storage < MQCT_R64 || d->storage > MQCT_C64)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: unknown storage type %d", d->storage);
  const bool cplx = d->in_dtype == MQCT_C128;
  if (dtype_complex(d->storage) != cplx)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: storage and input must both be real or both complex");
  if (d->mem != MQCT_MEM_HOST && d->mem != MQCT_MEM_DEVICE)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: mem must be host or device");
  const int64_t nnz = d->n_el;
  if (nnz < 1 || nnz >= ((int64_t)1 << 31) || d->ld < nnz)
    return fail(c, MQCT_ERR_ARG, "system_load_coo: need 1 <= n_el < 2^31 and ld >= n_el");
  if (!(d->mu > 0.0) || !isfinite(d->mu)) return fail(c, MQCT_ERR_ARG, "system_load_coo: mu must be > 0");
  if (!finite_arr(d->R_grid, K)) return fail(c, MQCT_ERR_NONFINITE, "system_load_coo: non-finite R grid");
  for (int k = 1; k < K; ++k)
    if (!(d->R_grid[k] > d->R_grid[k - 1]))
      return fail(c, MQCT_ERR_ARG, "system_load_coo: R grid not strictly increasing at %d", k);
  if (!finite_arr(d->E, N)) return fail(c, MQCT_ERR_NONFINITE, "system_load_coo: non-finite E");
  std::vector<int32_t> jx_col_h;
  std::vector<double> jx_val_h;
  int W = 0;
  {
    const mqct_status js = build_jx(c, "system_load_coo", N, d->E, d->jx_nnz, d->jx_row, d->jx_col,
                                    d->jx_val, jx_col_h, jx_val_h, W);
    if (js != MQCT_OK) return js;
  }
  HIP_TRY(c, hipSetDevice(c->device), "system_load_coo");
  // rows and columns on the host: sorted into CSR order (rows, then columns),
  // duplicates and missing (m, n) partners refused
  std::vector<int32_t> hr(nnz), hc(nnz);
  if (d->mem == MQCT_MEM_HOST) {
    memcpy(hr.data(), d->rows, nnz * 4);
    memcpy(hc.data(), d->cols, nnz * 4);
  } else {
    HIP_TRY(c, hipMemcpy(hr.data(), d->rows, nnz * 4, hipMemcpyDeviceToHost), "system_load_coo: indices");
    HIP_TRY(c, hipMemcpy(hc.data(), d->cols, nnz * 4, hipMemcpyDeviceToHost), "system_load_coo: indices");
  }
  std::vector<std::pair<int64_t, int32_t>> key(nnz);
  for (int64_t i = 0; i < nnz; ++i) {
    if (hr[i] < 0 || hr[i] >= N || hc[i] < 0 || hc[i] >= N)
      return fail(c, MQCT_ERR_ARG, "system_load_coo: element %lld index out of range", (long long)i);
    key[i] = {(int64_t)hr[i] * N + hc[i], (int32_t)i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> perm(nnz), ccol(nnz), rowptr(N + 1, 0), partner(nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    if (e > 0 && key[e].first == key[e - 1].first)
      return fail(c, MQCT_ERR_ARG, "system_load_coo: element (%lld, %lld) given twice",
                  (long long)(key[e].first / N), (long long)(key[e].first % N));
    perm[e] = key[e].second;
    ccol[e] = (int32_t)(key[e].first % N);
    ++rowptr[key[e].first / N + 1];
  }
  for (int n = 0; n < N; ++n) rowptr[n + 1] += rowptr[n];
  for (int n = 0; n < N; ++n)
    for (int32_t e = rowptr[n]; e < rowptr[n + 1]; ++e) {
      const int m = ccol[e];
      const int32_t* lo = ccol.data() + rowptr[m];
      const int32_t* hi = ccol.data() + rowptr[m + 1];
      const int32_t* it = std::lower_bound(lo, hi, n);
      if (it == hi || *it != n)
        return fail(c, MQCT_ERR_ARG, "system_load_coo: element (%d, %d) has no partner (%d, %d)",
                    n, m, m, n);
      partner[e] = (int32_t)(it - ccol.data());
    }
  key.clear();
  key.shrink_to_fit();

  const int NC = cplx ? 2 : 1;
  const int es = dtype_fp32(d->storage) ? 4 : 8;
  const int64_t nreal = nnz * NC;
  SysHost sh;
  sh.dev.N = N; sh.dev.K = K; sh.dev.Npad = (N + 15) / 16 * 16; sh.dev.dtype = d->storage;
  sh.dev.jx_w = W; sh.dev.mu = d->mu; sh.dev.knot_stride = nnz;
  {
    const double hu = (d->R_grid[K - 1] - d->R_grid[0]) / (K - 1);
    bool uniform = true;
    for (int k = 0; k < K && uniform; ++k)
      uniform = fabs(d->R_grid[k] - (d->R_grid[0] + k * hu)) <= 1e-9 * hu;
    sh.dev.R_inv_h = uniform ? 1.0 / hu : 0.0;
  }
  sh.table_bytes = 2 * (int64_t)K * nreal * es;
  double* din = nullptr;
  bool own_in = false;
  double* v64 = nullptr;
  double* c64 = nullptr;
  int32_t* d_perm = nullptr;
  int32_t* d_partner = nullptr;
  unsigned long long* stats = nullptr;
  auto cleanup = [&]() {
    if (own_in && din) hipFree(din);
    for (void* q : {(void*)d_perm, (void*)d_partner, (void*)stats}) if (q) hipFree(q);
    if (v64 && v64 != sh.bufs[0]) hipFree(v64);
    if (c64 && c64 != sh.bufs[1]) hipFree(c64);
  };
  auto dfail = [&](hipError_t e, const char* what) {
    cleanup();
    free_system(sh);
    return hip_fail(c, e, what);
  };
  hipError_t e;
  if (d->mem == MQCT_MEM_HOST) {
    const size_t in_bytes = (size_t)K * d->ld * NC * 8;
    if ((e = dev_malloc((void**)&din, in_bytes)) != hipSuccess) return dfail(e, "system_load_coo: input");
    own_in = true;
    if ((e = hipMemcpy(din, d->values, in_bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return dfail(e, "system_load_coo: upload");
  } else {
    din = (double*)d->values;
  }
  if ((e = dev_malloc((void**)&d_perm, nnz * 4)) != hipSuccess ||
      (e = dev_malloc((void**)&d_partner, nnz * 4)) != hipSuccess ||
      (e = dev_malloc((void**)&stats, 3 * sizeof(unsigned long long))) != hipSuccess ||
      (e = dev_malloc((void**)&v64, (size_t)K * nreal * 8)) != hipSuccess ||
      (e = dev_malloc((void**)&c64, (size_t)K * nreal * 8)) != hipSuccess ||
      (e = dev_malloc(&sh.bufs[2], K * 8)) != hipSuccess ||
      (e = dev_malloc(&sh.bufs[3], N * 8)) != hipSuccess ||
      (e = dev_malloc(&sh.ebuf[0], (size_t)(N + 1) * 4)) != hipSuccess ||
      (e = dev_malloc(&sh.ebuf[1], (size_t)nnz * 4)) != hipSuccess)
    return dfail(e, "system_load_coo: buffers");
  if ((e = hipMemcpy(d_perm, perm.data(), nnz * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_partner, partner.data(), nnz * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(sh.bufs[2], d->R_grid, K * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(sh.bufs[3], d->E, N * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(sh.ebuf[0], rowptr.data(), (size_t)(N + 1) * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(sh.ebuf[1], ccol.data(), (size_t)nnz * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return dfail(e, "system_load_coo: upload");
  if ((e = hipMemsetAsync(stats, 0, 3 * sizeof(unsigned long long), c->stream)) != hipSuccess ||
      (e = launch_coo_gather(din, d->ld, d_perm, nnz, K, NC, v64, stats + 2, c->stream)) != hipSuccess ||
      (e = launch_csr_partner_check(v64, d_partner, nnz, K, NC, stats, stats + 1, c->stream)) != hipSuccess)
    return dfail(e, "system_load_coo: validate");
  unsigned long long hs[3];
  if ((e = hipMemcpyAsync(hs, stats, sizeof hs, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return dfail(e, "system_load_coo: validate");
  if (hs[2] > 0) {
    cleanup();
    free_system(sh);
    return fail(c, MQCT_ERR_NONFINITE, "system_load_coo: %llu non-finite values", hs[2]);
  }
  double dmax, amax;
  memcpy(&dmax, &hs[0], 8);
  memcpy(&amax, &hs[1], 8);
  if (dmax > 1e-12 * amax) {
    cleanup();
    free_system(sh);
    return fail(c, MQCT_ERR_NOT_HERMITIAN, "system_load_coo: |M_nm - conj(M_mn)| = %.3e > 1e-12 "
                "max|M| = %.3e", dmax, 1e-12 * amax);
  }
  // natural-spline second derivatives of every real component, FP64
  if ((e = launch_csr_spline(v64, (const double*)sh.bufs[2], K, nreal, c64, c->stream)) != hipSuccess)
    return dfail(e, "system_load_coo: spline");
  if (es == 8) {
    sh.bufs[0] = v64;
    sh.bufs[1] = c64;
  } else {
    if ((e = dev_malloc(&sh.bufs[0], (size_t)K * nreal * 4)) != hipSuccess ||
        (e = dev_malloc(&sh.bufs[1], (size_t)K * nreal * 4)) != hipSuccess ||
        (e = launch_csr_cast_f32(v64, (int64_t)K * nreal, (float*)sh.bufs[0], c->stream)) != hipSuccess ||
        (e = launch_csr_cast_f32(c64, (int64_t)K * nreal, (float*)sh.bufs[1], c->stream)) != hipSuccess)
      return dfail(e, "system_load_coo: storage");
  }
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return dfail(e, "system_load_coo: spline");
  if (W > 0) {
    if ((e = dev_malloc(&sh.bufs[4], jx_col_h.size() * 4)) != hipSuccess ||
        (e = dev_malloc(&sh.bufs[5], jx_val_h.size() * 8)) != hipSuccess ||
        (e = hipMemcpy(sh.bufs[4], jx_col_h.data(), jx_col_h.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(sh.bufs[5], jx_val_h.data(), jx_val_h.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
      return dfail(e, "system_load_coo: J_x");
  }
  cleanup();
  sh.dev.M = sh.bufs[0];
  sh.dev.M2 = sh.bufs[1];
  sh.dev.R = (const double*)sh.bufs[2];
  sh.dev.E = (const double*)sh.bufs[3];
  sh.dev.jx_col = (const int32_t*)sh.bufs[4];
  sh.dev.jx_val = (const double*)sh.bufs[5];
  sh.dev.csr_row = (const int32_t*)sh.ebuf[0];
  sh.dev.csr_col = (const int32_t*)sh.ebuf[1];
  sh.R_last = d->R_grid[K - 1];
  sh.live = true;
  int id = -1;
  for (size_t i = 0; i < c->systems.size(); ++i)
    if (!c->systems[i].live) { id = (int)i; break; }
  if (id < 0) { id = (int)c->systems.size(); c->systems.push_back(sh); }
  else c->systems[id] = sh;
  const mqct_status st = upload_systems(c);
  if (st != MQCT_OK) return st;
  *system_id = id;
  return MQCT_OK;
}

mqct_status mqct_system_set_driver(mqct_context* c, int32_t id, const double* U) {
  if (!c) return MQCT_ERR_ARG;
  if (id < 0 || id >= (int)c->systems.size() || !c->systems[id].live)
    return fail(c, MQCT_ERR_STATE, "set_driver: unknown system %d", id);
  if (!U) return fail(c, MQCT_ERR_ARG, "set_driver: null U");
  SysHost& sh = c->systems[id];
  const int K = sh.dev.K;
  if (!finite_arr(U, K)) return fail(c, MQCT_ERR_NONFINITE, "set_driver: non-finite U");
  HIP_TRY(c, hipSetDevice(c->device), "set_driver");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "set_driver");
  if (!sh.dbuf) HIP_TRY(c, dev_malloc(&sh.dbuf, (size_t)4 * K * sizeof(double)), "set_driver");
  double* d = (double*)sh.dbuf;   // U [K], U'' [K], then 2K of elimination scratch
  HIP_TRY(c, hipMemcpyAsync(d, U, (size_t)K * sizeof(double), hipMemcpyHostToDevice, c->stream),
          "set_driver");
  HIP_TRY(c, launch_spline_rows(d, sh.dev.R, K, 1, d + K, d + 2 * K, c->stream), "set_driver");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "set_driver");
  sh.dev.drv = d;
  sh.dev.drv2 = d + K;
  return upload_systems(c);
}

mqct_status mqct_system_bytes(mqct_context* c, int32_t id, int64_t* bytes) {
  if (!c) return MQCT_ERR_ARG;
  if (!bytes) return fail(c, MQCT_ERR_ARG, "system_bytes: null output");
  if (id < 0 || id >= (int)c->systems.size() || !c->systems[id].live)
    return fail(c, MQCT_ERR_STATE, "system_bytes: unknown system %d", id);
  *bytes = c->systems[id].table_bytes;
  return MQCT_OK;
}

mqct_status mqct_system_free(mqct_context* c, int32_t id) {
  if (!c) return MQCT_ERR_ARG;
  if (id < 0 || id >= (int)c->systems.size() || !c->systems[id].live)
    return fail(c, MQCT_ERR_STATE, "system_free: unknown system %d", id);
  HIP_TRY(c, hipSetDevice(c->device), "system_free");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "system_free");
  free_system(c->systems[id]);
  c->systems[id].dev = DevSystem{};
  return upload_systems(c);
}

mqct_status mqct_run(mqct_context* c, const mqct_batch_desc* bd, mqct_batch_result* res) {
  if (!c) return MQCT_ERR_ARG;
  if (!bd || !res) return fail(c, MQCT_ERR_ARG, "run: null argument");
  const int64_t B = bd->B;
  if (B < 0) return fail(c, MQCT_ERR_ARG, "run: B < 0");
  if (B == 0) return MQCT_OK;
  if (!bd->system_id) return fail(c, MQCT_ERR_ARG, "run: system_id is required");
  if (!res->P) return fail(c, MQCT_ERR_ARG, "run: result P is required");
  if (res->mem != MQCT_MEM_HOST && res->mem != MQCT_MEM_DEVICE)
    return fail(c, MQCT_ERR_ARG, "run: result mem must be host or device");
  if (bd->integrator != MQCT_RK4 && bd->integrator != MQCT_DP5)
    return fail(c, MQCT_ERR_ARG, "run: unknown integrator %d", bd->integrator);
  if (bd->schedule < MQCT_SCHED_AUTO || bd->schedule > MQCT_SCHED_COLUMNS)
    return fail(c, MQCT_ERR_ARG, "run: unknown schedule %d", bd->schedule);
  // coordinate-list systems run on the columns schedule, and only there
  bool any_csr = false, all_csr = true;
  for (int64_t b = 0; b < B; ++b) {
    const int sid = bd->system_id[b];
    const bool csr = sid >= 0 && sid < (int)c->systems.size() && c->systems[sid].live &&
                     c->systems[sid].dev.csr_row != nullptr;
    any_csr |= csr;
    all_csr &= csr;
  }
  const bool columns = bd->schedule == MQCT_SCHED_COLUMNS ||
                       (bd->schedule == MQCT_SCHED_AUTO && any_csr);
  if (any_csr && !columns)
    return fail(c, MQCT_ERR_UNSUPPORTED, "run: coordinate-list systems run on the columns schedule only");
  if (columns) {
    if (!all_csr)
      return fail(c, MQCT_ERR_UNSUPPORTED, "run: the columns schedule needs a coordinate-list system");
    for (int64_t b = 1; b < B; ++b)
      if (bd->system_id[b] != bd->system_id[0])
        return fail(c, MQCT_ERR_UNSUPPORTED, "run: a columns batch must use a single system");
    if (bd->integrator != MQCT_RK4 || bd->dynamics != MQCT_AT || bd->resume)
      return fail(c, MQCT_ERR_UNSUPPORTED,
                  "run: the columns schedule runs AT dynamics with RK4 (no resume)");
    if (B > INT32_MAX) return fail(c, MQCT_ERR_UNSUPPORTED, "run: B too large for the columns schedule");
  }
  const bool binned = bd->schedule == MQCT_SCHED_BINNED;
  if (binned) {
    for (int64_t b = 1; b < B; ++b)
      if (bd->system_id[b] != bd->system_id[0])
        return fail(c, MQCT_ERR_UNSUPPORTED, "run: a binned batch must use a single system");
    const int sid0 = bd->system_id[0];
    if (sid0 >= 0 && sid0 < (int)c->systems.size() && c->systems[sid0].live &&
        c->systems[sid0].dev.ell_w > 0)
      return fail(c, MQCT_ERR_UNSUPPORTED,
                  "run: the binned schedule multiplies dense tables (system %d is sparse)", sid0);
  }
  const bool dp5 = bd->integrator == MQCT_DP5;
  // DP5 runs on the work-list schedule (trajectory lengths differ) unless the
  // binned schedule is asked for
  const bool queue = (dp5 && !binned) || bd->schedule == MQCT_SCHED_QUEUE;
  if (dp5) {
    if (!(bd->rtol > 0.0) || !(bd->atol > 0.0) || bd->max_steps < 1 || !(bd->h_min >= 0.0))
      return fail(c, MQCT_ERR_ARG, "run: DP5 needs rtol > 0, atol > 0, max_steps >= 1, h_min >= 0");
  } else if ((!bd->dt && bd->resume != 1) || !bd->n_steps) {
    return fail(c, MQCT_ERR_ARG, "run: RK4 needs dt and n_steps (n_steps when resuming)");
  }
  if (bd->resume != 0 && bd->resume != 1)
    return fail(c, MQCT_ERR_ARG, "run: resume must be 0 or 1");
  const bool resume = bd->resume == 1;
  if (!resume && !bd->classical0 && (!bd->E_coll || !bd->b))
    return fail(c, MQCT_ERR_ARG, "run: E_coll and b are required without classical0");
  if (bd->dynamics != MQCT_EHRENFEST && bd->dynamics != MQCT_AT)
    return fail(c, MQCT_ERR_ARG, "run: unknown dynamics %d", bd->dynamics);
  if (!resume && !bd->a0 && !bd->init_channel)
    return fail(c, MQCT_ERR_ARG, "run: init_channel is required without a0");
  // a continued batch: the stored records (read back once) replace the start data
  std::vector<mqct_traj_state> rec;
  if (resume) {
    if (B != c->st_B)
      return fail(c, MQCT_ERR_STATE, "run: resume needs the %lld stored trajectories, got B = %lld",
                  (long long)c->st_B, (long long)B);
    for (int64_t b = 0; b < B; ++b)
      if (bd->system_id[b] != c->st_sys[b])
        return fail(c, MQCT_ERR_STATE, "run: trajectory %lld is stored with system %d, not %d",
                    (long long)b, c->st_sys[b], bd->system_id[b]);
    rec.resize(B);
    HIP_TRY(c, hipSetDevice(c->device), "run");
    HIP_TRY(c, hipMemcpyAsync(rec.data(), c->st_rec.p, B * sizeof(mqct_traj_state),
                              hipMemcpyDeviceToHost, c->stream), "run: stored state");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "run: stored state");
  }

  // trajectory records
  HIP_TRY(c, hipSetDevice(c->device), "run");
  if ((size_t)B > c->h_traj_cap) {
    if (c->h_traj) {
      HIP_TRY(c, hipEventSynchronize(c->staged), "run");
      hipHostFree(c->h_traj);
      c->h_traj = nullptr;
    }
    HIP_TRY(c, hipHostMalloc((void**)&c->h_traj, B * sizeof(TrajIn), 0), "run: staging");
    c->h_traj_cap = B;
  } else {
    HIP_TRY(c, hipEventSynchronize(c->staged), "run");
  }
  int64_t amp_total = 0;
  std::vector<int64_t> order[4];
  std::vector<int> max_npad(4, 0);
  for (int64_t b = 0; b < B; ++b) {
    int sid = bd->system_id[b];
    if (sid < 0 || sid >= (int)c->systems.size() || !c->systems[sid].live)
      return fail(c, MQCT_ERR_STATE, "run: trajectory %lld uses unknown system %d", (long long)b, sid);
    const DevSystem& sy = c->systems[sid].dev;
    TrajIn t{};
    t.id = b;
    t.amp_off = amp_total;
    t.sys = sid;
    t.n_steps = bd->n_steps ? bd->n_steps[b] : 0;
    t.dt = bd->dt ? bd->dt[b] : 0.0;
    t.t0 = bd->t0 ? bd->t0[b] : 0.0;
    if (t.n_steps < 0) return fail(c, MQCT_ERR_ARG, "run: n_steps[%lld] < 0", (long long)b);
    if (!isfinite(t.dt) || !isfinite(t.t0)) return fail(c, MQCT_ERR_ARG, "run: non-finite dt/t0");
    if (resume) {
      const mqct_traj_state& r = rec[b];
      if (r.N != sy.N || r.system_id != sid)
        return fail(c, MQCT_ERR_STATE, "run: stored trajectory %lld does not match its system",
                    (long long)b);
      t.flags |= TRAJ_HAS_A0 | TRAJ_HAS_C0 | TRAJ_RESUME;
      for (int i = 0; i < 6; ++i) t.c0[i] = r.classical[i];
      t.steps0 = r.steps;
      t.rejects0 = r.rejects;
      t.attempts0 = r.attempts;
      t.E0 = r.E0;
      t.J0 = r.J0;
      t.R_exit = r.R_exit;
      t.dflags = r.flags & MQCT_S_LAST_REJECTED;
      t.status0 = r.status & ~MQCT_T_MAX_STEPS;
      if (dp5) {
        // adaptive: continue from t with the stored step size
        t.t0 = r.t;
        t.h0 = r.h;
        if (r.status & (MQCT_T_EXITED | MQCT_T_STEP_UNDERFLOW | MQCT_T_NONFINITE))
          t.flags |= TRAJ_FINISHED;
      } else {
        // fixed steps: t_j = t_origin + j h with j counted on from n_origin
        t.t0 = r.t_origin;
        t.step0 = r.n_origin;
        t.dt = r.h;
      }
      if (!(t.c0[0] > 0.0) || !isfinite(t.t0) || !isfinite(t.dt) || !(dp5 ? t.h0 > 0.0 : t.dt > 0.0))
        return fail(c, MQCT_ERR_STATE, "run: stored trajectory %lld cannot be continued",
                    (long long)b);
      if (bd->dynamics == MQCT_AT && !sy.drv)
        return fail(c, MQCT_ERR_STATE, "run: AT dynamics needs a driving potential for system %d "
                    "(mqct_system_set_driver)", sid);
      if (bd->dynamics == MQCT_AT) t.flags |= TRAJ_AT;
      amp_total += sy.N;
      order[sy.dtype].push_back(b);
      max_npad[sy.dtype] = std::max(max_npad[sy.dtype], sy.Npad);
      c->h_traj[b] = t;
      continue;
    }
    if (bd->a0) {
      t.flags |= TRAJ_HAS_A0;
    } else {
      t.init_channel = bd->init_channel[b];
      if (t.init_channel < 0 || t.init_channel >= sy.N)
        return fail(c, MQCT_ERR_ARG, "run: init_channel[%lld] out of range", (long long)b);
    }
    if (bd->classical0) {
      t.flags |= TRAJ_HAS_C0;
      for (int i = 0; i < 6; ++i) t.c0[i] = bd->classical0[b * 6 + i];
      if (!finite_arr(t.c0, 6) || !(t.c0[0] > 0.0))
        return fail(c, MQCT_ERR_ARG, "run: classical0[%lld] invalid", (long long)b);
    } else {
      t.E_coll = bd->E_coll[b];
      t.b = bd->b[b];
      t.R0 = bd->R0 ? bd->R0[b] : -1.0;
      if (!(t.E_coll > 0.0) || !isfinite(t.E_coll))
        return fail(c, MQCT_ERR_ARG, "run: E_coll[%lld] must be > 0", (long long)b);
      if (t.R0 < 0.0) t.R0 = -1.0;   // resolved below from the grid
    }
    if (bd->dynamics == MQCT_AT) {
      if (!sy.drv)
        return fail(c, MQCT_ERR_STATE, "run: AT dynamics needs a driving potential for system %d "
                    "(mqct_system_set_driver)", sid);
      t.flags |= TRAJ_AT;
    }
    amp_total += sy.N;
    order[sy.dtype].push_back(b);
    max_npad[sy.dtype] = std::max(max_npad[sy.dtype], sy.Npad);
    c->h_traj[b] = t;
  }
  // default R0 = last knot (needs the grid on the host: read it back once per system)
  if (!bd->classical0 && !resume) {
    std::map<int, double> last;
    for (int64_t b = 0; b < B; ++b) {
      TrajIn& t = c->h_traj[b];
      if (t.R0 < 0.0) {
        auto it = last.find(t.sys);
        if (it == last.end()) {
          const DevSystem& sy = c->systems[t.sys].dev;
          double r;
          HIP_TRY(c, hipMemcpy(&r, sy.R + (sy.K - 1), 8, hipMemcpyDeviceToHost), "run: grid");
          it = last.emplace(t.sys, r).first;
        }
        t.R0 = it->second;
      }
      if (!(t.R0 > 0.0) || !isfinite(t.R0) || !(t.b >= 0.0) || !(t.b < t.R0))
        return fail(c, MQCT_ERR_ARG, "run: need 0 <= b < R0 (trajectory %lld)", (long long)b);
    }
  }
  // Order of the records on the device.  Per-trajectory launches need each
  // storage type contiguous.  The work-list schedule needs each class (storage
  // type and padded column count) contiguous, and takes the most expensive
  // trajectories first (cost ~ N^2 x free-flight time 2 R0 / v0), so the
  // longest ones never start last.
  std::vector<TrajIn> sorted;
  sorted.reserve(B);
  std::vector<std::pair<int64_t, int64_t>> ranges(4, {0, 0});
  std::vector<QueueClass> classes;
  struct SideGroup { int sys; int64_t first, n; };
  std::vector<SideGroup> side_groups;   // binned shares of an adaptive batch (records first..)
  auto cost_of = [&](int64_t b) {
    const TrajIn& t = c->h_traj[b];
    const double n = c->systems[t.sys].dev.N;
    double T = 1.0;
    if (!(t.flags & TRAJ_HAS_C0) && t.E_coll > 0.0)
      T = 2.0 * t.R0 / sqrt(2.0 * t.E_coll / c->systems[t.sys].dev.mu);
    else if (t.n_steps > 0)
      T = (double)t.n_steps;
    return n * n * T;
  };
  std::vector<ColGroup> col_groups;
  int col_ct = 2;
  if (columns) {
    // columns that share a path (the same start state or E_coll, b, R0, and the
    // same t0, dt, n_steps), in groups of at most COL_MAX
    std::map<std::vector<uint64_t>, std::vector<int64_t>> paths;
    for (int64_t b = 0; b < B; ++b) {
      const TrajIn& t = c->h_traj[b];
      std::vector<double> v = {t.t0, t.dt, (double)t.n_steps, (double)(t.flags & TRAJ_HAS_C0)};
      if (t.flags & TRAJ_HAS_C0) v.insert(v.end(), t.c0, t.c0 + 6);
      else v.insert(v.end(), {t.E_coll, t.b, t.R0});
      std::vector<uint64_t> k(v.size());
      memcpy(k.data(), v.data(), v.size() * 8);
      paths[k].push_back(b);
    }
    int64_t stage_off = 0;
    for (auto& kv : paths)
      for (size_t i0 = 0; i0 < kv.second.size(); i0 += COL_MAX) {
        ColGroup g{};
        g.first = (int32_t)sorted.size();
        g.count = (int32_t)std::min<size_t>(COL_MAX, kv.second.size() - i0);
        g.n_steps = c->h_traj[kv.second[i0]].n_steps;
        g.stage_off = stage_off;
        stage_off += 4 * g.n_steps;
        for (int q = 0; q < g.count; ++q) sorted.push_back(c->h_traj[kv.second[i0 + q]]);
        col_ct = std::max(col_ct, (g.count + 1) & ~1);
        col_groups.push_back(g);
      }
  } else if (!queue) {
    for (int d = 0; d < 4; ++d) {
      ranges[d].first = (int64_t)sorted.size();
      for (int64_t b : order[d]) sorted.push_back(c->h_traj[b]);
      ranges[d].second = (int64_t)sorted.size();
    }
  } else {
    // An adaptive batch left to the library: the trajectories of a large dense
    // system that holds many of them go to the binned schedule (their stages
    // become table x columns products on the matrix cores), on a second stream
    // beside the work list that takes the rest.
    std::map<int, std::vector<int64_t>> of_system;
    if (dp5 && bd->schedule == MQCT_SCHED_AUTO)
      for (int64_t b = 0; b < B; ++b) of_system[c->h_traj[b].sys].push_back(b);
    std::vector<char> on_side(B, 0);
    for (auto& kv : of_system) {
      const DevSystem& sy = c->systems[kv.first].dev;
      if (sy.ell_w > 0 || sy.Npad < SPLIT_MIN_NPAD || (int64_t)kv.second.size() < SPLIT_MIN_TRAJ ||
          kv.second.size() > (size_t)INT32_MAX)
        continue;
      side_groups.push_back({kv.first, (int64_t)sorted.size(), (int64_t)kv.second.size()});
      for (int64_t b : kv.second) {
        sorted.push_back(c->h_traj[b]);
        on_side[b] = 1;
      }
    }
    std::map<std::pair<int, int>, std::vector<int64_t>> by_class;
    for (int64_t b = 0; b < B; ++b) {
      if (on_side[b]) continue;
      const DevSystem& sy = c->systems[c->h_traj[b].sys].dev;
      by_class[{sy.dtype, sy.Npad}].push_back(b);
    }
    for (auto& kv : by_class) {
      std::vector<std::pair<double, int64_t>> cost;
      for (int64_t b : kv.second) cost.push_back({-cost_of(b), b});
      std::stable_sort(cost.begin(), cost.end());
      QueueClass qc{kv.first.first, kv.first.second, (int64_t)sorted.size(), (int64_t)cost.size()};
      for (auto& pr : cost) sorted.push_back(c->h_traj[pr.second]);
      classes.push_back(qc);
    }
  }
  memcpy(c->h_traj, sorted.data(), B * sizeof(TrajIn));

  mqct_status st;
  if ((st = ensure(c, c->traj, B * sizeof(TrajIn), "run: trajectories")) != MQCT_OK) return st;
  HIP_TRY(c, hipMemcpyAsync(c->traj.p, c->h_traj, B * sizeof(TrajIn), hipMemcpyHostToDevice,
                            c->stream), "run: upload");
  HIP_TRY(c, hipEventRecord(c->staged, c->stream), "run: upload");
  const double* d_a0 = nullptr;
  if (resume) {
    // the stored amplitudes, copied aside: this run overwrites the store
    if ((st = ensure(c, c->a0, amp_total * 16, "run: a0")) != MQCT_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->a0.p, c->st_amp.p, amp_total * 16, hipMemcpyDeviceToDevice,
                              c->stream), "run: stored amplitudes");
    d_a0 = (const double*)c->a0.p;
  } else if (bd->a0) {
    if ((st = ensure(c, c->a0, amp_total * 16, "run: a0")) != MQCT_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->a0.p, bd->a0, amp_total * 16, hipMemcpyHostToDevice, c->stream),
            "run: a0");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "run: a0");
    d_a0 = (const double*)c->a0.p;
  }
  // the state store receives every trajectory's final state
  if ((st = ensure(c, c->st_rec, B * sizeof(mqct_traj_state), "run: state store")) != MQCT_OK)
    return st;
  if ((st = ensure(c, c->st_amp, amp_total * 16, "run: state store")) != MQCT_OK) return st;
  c->st_B = 0;   // valid again once this run is enqueued

  // result arrays: caller's device pointers, or device staging for host results
  TrajOut out{};
  struct Piece { void* host; size_t bytes; int slot; };
  std::vector<Piece> back;
  void* hp[10] = {res->P, res->a_final, res->classical, res->t_final, res->steps,
                  res->rejects, res->status, res->norm_err, res->energy_err, res->angmom_err};
  size_t sz[10] = {(size_t)amp_total * 8, (size_t)amp_total * 16, (size_t)B * 48, (size_t)B * 8,
                   (size_t)B * 8, (size_t)B * 8, (size_t)B * 4, (size_t)B * 8, (size_t)B * 8,
                   (size_t)B * 8};
  void* dp[10];
  for (int i = 0; i < 10; ++i) {
    dp[i] = hp[i];
    if (hp[i] && res->mem == MQCT_MEM_HOST) {
      if ((st = ensure(c, c->outs[i], sz[i], "run: results")) != MQCT_OK) return st;
      dp[i] = c->outs[i].p;
      back.push_back({hp[i], sz[i], i});
    }
  }
  out.P = (double*)dp[0]; out.a_final = (double*)dp[1]; out.classical = (double*)dp[2];
  out.t_final = (double*)dp[3]; out.steps = (int64_t*)dp[4]; out.rejects = (int64_t*)dp[5];
  out.status = (int32_t*)dp[6]; out.norm_err = (double*)dp[7]; out.energy_err = (double*)dp[8];
  out.angmom_err = (double*)dp[9];
  out.state = (mqct_traj_state*)c->st_rec.p;
  out.st_amp = (double2*)c->st_amp.p;

  if (columns) {
    const DevSystem& hs = c->systems[c->h_traj[0].sys].dev;
    const bool f32 = dtype_fp32(hs.dtype);
    // The amplitude columns take 80 or 96 bytes per state and column: a batch
    // whose groups do not fit the cap runs in passes of whole groups (stage
    // records rebased per pass), one after the other in the same workspace.
    size_t cap = (size_t)c->qopt.col_ws;
    if (cap == 0) {
      size_t fr = 0, tot = 0;
      HIP_TRY(c, hipMemGetInfo(&fr, &tot), "run: columns memory query");
      cap = (size_t)(0.8 * (double)(fr + c->binws.cap));
    }
    std::vector<std::vector<ColGroup>> passes;
    size_t wsb = 0;
    for (size_t i = 0; i < col_groups.size();) {
      std::vector<ColGroup> pg;
      int64_t off = 0;
      size_t bytes = 0;
      for (; i < col_groups.size(); ++i) {
        ColGroup g = col_groups[i];
        g.stage_off = off;
        const size_t nb = columns_workspace_bytes((int)pg.size() + 1, hs.N, col_ct, off + 4 * g.n_steps, f32);
        if (nb > cap && !pg.empty()) break;
        if (nb > cap)
          return fail(c, MQCT_ERR_OOM, "run: one path group needs %zu bytes of columns workspace, cap %zu",
                      nb, cap);
        pg.push_back(g);
        off += 4 * g.n_steps;
        bytes = nb;
      }
      wsb = std::max(wsb, bytes);
      passes.push_back(std::move(pg));
    }
    if ((st = ensure(c, c->binws, wsb, "run: columns workspace")) != MQCT_OK) return st;
    out.state = nullptr;    // the columns schedule keeps no stored states
    out.st_amp = nullptr;
    for (const std::vector<ColGroup>& pg : passes) {
      hipError_t e = run_columns(c->d_systems, hs, (const TrajIn*)c->traj.p, pg, col_ct, d_a0, out,
                                 c->binws.p, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "run: columns schedule");
    }
  } else if (binned && dp5) {
    const DevSystem& hs = c->systems[c->h_traj[0].sys].dev;
    if (B > INT32_MAX) return fail(c, MQCT_ERR_UNSUPPORTED, "run: B too large for the binned schedule");
    const DpCtl ctl{bd->rtol, bd->atol, bd->h_min, bd->max_steps};
    const int64_t max_attempts = 4 * bd->max_steps + 256;
    const size_t wsb = binned_dp5_workspace_bytes((int)B, hs.Npad, hs.K, dtype_fp32(hs.dtype));
    if ((st = ensure(c, c->binws, wsb, "run: binned workspace")) != MQCT_OK) return st;
    hipError_t e = run_binned_dp5(c->d_systems, hs, (const TrajIn*)c->traj.p, (int)B, d_a0, out,
                                  ctl, max_attempts, c->binws.p, c->stream, &c->prof);
    if (e != hipSuccess) return hip_fail(c, e, "run: binned DP5");
  } else if (binned) {
    const DevSystem& hs = c->systems[c->h_traj[0].sys].dev;
    int64_t max_steps = 0;
    for (int64_t b = 0; b < B; ++b) max_steps = std::max(max_steps, c->h_traj[b].n_steps);
    const size_t wsb = binned_workspace_bytes((int)B, hs.Npad, hs.K, dtype_fp32(hs.dtype));
    if ((st = ensure(c, c->binws, wsb, "run: binned workspace")) != MQCT_OK) return st;
    hipError_t e = run_binned(c->d_systems, hs, (const TrajIn*)c->traj.p, (int)B, max_steps,
                              d_a0, out, c->binws.p, c->stream, &c->prof);
    if (e != hipSuccess) return hip_fail(c, e, "run: binned launch");
  } else if (!queue) {
    for (int d = 0; d < 4; ++d) {
      int64_t n = ranges[d].second - ranges[d].first;
      if (n == 0) continue;
      if (c->prof.on) {
        // RK4 stages plus the final diagnostic evaluation, four slices each
        for (int64_t q = ranges[d].first; q < ranges[d].second; ++q) {
          const DevSystem& sy = c->systems[c->h_traj[q].sys].dev;
          c->prof.bytes += (4.0 * c->h_traj[q].n_steps + 1.0) * 4.0 * (double)sy.knot_stride *
                           dtype_bytes(sy.dtype);
        }
      }
      hipError_t e = launch_rk4_gemv(c->d_systems, (const TrajIn*)c->traj.p + ranges[d].first, n,
                                     d_a0, out, d, max_npad[d], c->stream, &c->prof);
      if (e == hipErrorInvalidValue)
        return fail(c, MQCT_ERR_UNSUPPORTED, "run: N too large for the per-trajectory schedule");
      if (e != hipSuccess) return hip_fail(c, e, "run: launch");
    }
  } else {
    for (const QueueClass& qc : classes)
      if (qc.npad > 4096 || qc.n > INT32_MAX)
        return fail(c, MQCT_ERR_UNSUPPORTED, "run: N or B too large for the work-list schedule");
    const int method = dp5 ? 1 : 0;
    DpCtl ctl{bd->rtol, bd->atol, bd->h_min, bd->max_steps};
    // RK4: one step per attempt; DP5: accepted steps plus a bound on rejections
    int64_t max_attempts = 0;
    if (dp5) {
      max_attempts = 4 * bd->max_steps + 256;
    } else {
      for (int64_t b = 0; b < B; ++b) max_attempts = std::max(max_attempts, c->h_traj[b].n_steps);
    }
    if (!classes.empty()) {
      if ((st = ensure(c, c->qws, queue_workspace_bytes(classes, method), "run: work-list workspace")) != MQCT_OK)
        return st;
      if (classes.size() > c->h_counts_cap) {
        if (c->h_counts) hipHostFree(c->h_counts);
        c->h_counts = nullptr;
        c->h_counts_cap = 0;
        HIP_TRY(c, hipHostMalloc((void**)&c->h_counts, classes.size() * 4 + 64, 0), "run: counts");
        c->h_counts_cap = classes.size() + 16;
      }
    }
    // the binned shares run on the side stream, driven by a host thread of their
    // own, while this thread drives the work list
    if (!side_groups.empty()) {
      size_t wsb = 0;
      for (const SideGroup& g : side_groups) {
        const DevSystem& hs = c->systems[g.sys].dev;
        wsb = std::max(wsb, binned_dp5_workspace_bytes((int)g.n, hs.Npad, hs.K, dtype_fp32(hs.dtype)));
      }
      if ((st = ensure(c, c->binws, wsb, "run: binned workspace")) != MQCT_OK) return st;
      // records and start amplitudes are on the device before the side starts
      HIP_TRY(c, hipStreamSynchronize(c->stream), "run: upload");
    }
    hipError_t side_err = hipSuccess;
    std::thread side_thread;
    // started when the work list reaches its latency-bound tail (after its
    // autotuner's timing runs), so the binned share has most of the device beside
    // the tail instead of contending with the work list's bulk
    auto start_side = [&]() {
      if (side_groups.empty() || side_thread.joinable()) return;
      side_thread = std::thread([c, ctl, max_attempts, d_a0, out, &side_groups, &side_err]() {
        hipError_t e = hipSetDevice(c->device);
        for (size_t k = 0; k < side_groups.size() && e == hipSuccess; ++k) {
          const SideGroup& g = side_groups[k];
          e = run_binned_dp5(c->d_systems, c->systems[g.sys].dev, (const TrajIn*)c->traj.p + g.first,
                             (int)g.n, d_a0, out, ctl, max_attempts, c->binws.p, c->side, nullptr);
        }
        if (e == hipSuccess) e = hipEventRecord(c->side_done, c->side);
        side_err = e;
      });
    };
    hipError_t e = hipSuccess;
    if (!classes.empty())
      e = run_queue(c->d_systems, (const TrajIn*)c->traj.p, classes, d_a0, out, method, ctl,
                    max_attempts, c->qopt, c->qcache, c->qws.p, c->stream, c->cap, c->h_counts,
                    &c->prof, start_side);
    else
      start_side();
    if (side_thread.joinable()) {
      side_thread.join();
      if (side_err != hipSuccess) return hip_fail(c, side_err, "run: binned share");
      HIP_TRY(c, hipStreamWaitEvent(c->stream, c->side_done, 0), "run: binned share");
    }
    if (e == hipErrorInvalidValue)
      return fail(c, MQCT_ERR_UNSUPPORTED, "run: no workgroup shape for this N and storage type");
    if (e != hipSuccess) return hip_fail(c, e, "run: work-list schedule");
  }
  // the store now describes this batch (records by batch index); a columns batch
  // leaves it empty
  c->st_B = columns ? 0 : B;
  c->st_sys.assign(bd->system_id, bd->system_id + B);
  c->st_off.assign(B + 1, 0);
  for (int64_t b = 0; b < B; ++b)
    c->st_off[b + 1] = c->st_off[b] + c->systems[bd->system_id[b]].dev.N;
  for (auto& p : back)
    HIP_TRY(c, hipMemcpyAsync(p.host, dp[p.slot], p.bytes, hipMemcpyDeviceToHost, c->stream),
            "run: results");
  if (res->mem == MQCT_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream), "run: results");
  return MQCT_OK;
}

mqct_status mqct_run_noalloc(mqct_context* c, const mqct_batch_desc* bd,
                             const mqct_batch_result* res) {
  if (!c) return MQCT_ERR_ARG;
  if (!bd || !res) return fail(c, MQCT_ERR_ARG, "run_noalloc: null argument");
  const int64_t B = bd->B;
  if (B < 0) return fail(c, MQCT_ERR_ARG, "run_noalloc: B < 0");
  if (B == 0) return MQCT_OK;
  if (res->mem != MQCT_MEM_DEVICE || !res->P)
    return fail(c, MQCT_ERR_ARG, "run_noalloc: results must be device arrays (P required)");
  if (bd->integrator != MQCT_RK4 || (bd->schedule != MQCT_SCHED_AUTO &&
                                     bd->schedule != MQCT_SCHED_GEMV) || bd->resume)
    return fail(c, MQCT_ERR_UNSUPPORTED, "run_noalloc: fixed-step RK4 on the per-trajectory "
                "schedule only, without resume");
  if (bd->dynamics != MQCT_EHRENFEST && bd->dynamics != MQCT_AT)
    return fail(c, MQCT_ERR_ARG, "run_noalloc: unknown dynamics %d", bd->dynamics);
  if (!bd->system_id || !bd->dt || !bd->n_steps)
    return fail(c, MQCT_ERR_ARG, "run_noalloc: system_id, dt and n_steps are required");
  if (!bd->classical0 && (!bd->E_coll || !bd->b))
    return fail(c, MQCT_ERR_ARG, "run_noalloc: E_coll and b are required without classical0");
  if (!bd->a0 && !bd->init_channel)
    return fail(c, MQCT_ERR_ARG, "run_noalloc: init_channel is required without a0");
  if (!c->scratch) return fail(c, MQCT_ERR_STATE, "run_noalloc: no scratch address");
  // validation and sizes: one pass over the batch
  int64_t amp_total = 0;
  int max_npad[4] = {0, 0, 0, 0};
  for (int64_t b = 0; b < B; ++b) {
    const int sid = bd->system_id[b];
    if (sid < 0 || sid >= (int)c->systems.size() || !c->systems[sid].live)
      return fail(c, MQCT_ERR_STATE, "run_noalloc: trajectory %lld uses unknown system %d",
                  (long long)b, sid);
    const DevSystem& sy = c->systems[sid].dev;
    if (sy.csr_row)
      return fail(c, MQCT_ERR_UNSUPPORTED, "run_noalloc: system %d is a coordinate-list system", sid);
    if (bd->n_steps[b] < 0 || !isfinite(bd->dt[b]) || (bd->t0 && !isfinite(bd->t0[b])))
      return fail(c, MQCT_ERR_ARG, "run_noalloc: bad n_steps, dt or t0 at %lld", (long long)b);
    if (!bd->a0 && (bd->init_channel[b] < 0 || bd->init_channel[b] >= sy.N))
      return fail(c, MQCT_ERR_ARG, "run_noalloc: init_channel[%lld] out of range", (long long)b);
    if (bd->classical0) {
      if (!finite_arr(bd->classical0 + b * 6, 6) || !(bd->classical0[b * 6] > 0.0))
        return fail(c, MQCT_ERR_ARG, "run_noalloc: classical0[%lld] invalid", (long long)b);
    } else {
      const double R0 = bd->R0 ? bd->R0[b] : c->systems[sid].R_last;
      if (!(bd->E_coll[b] > 0.0) || !isfinite(bd->E_coll[b]) || !(R0 > 0.0) || !isfinite(R0) ||
          !(bd->b[b] >= 0.0) || !(bd->b[b] < R0))
        return fail(c, MQCT_ERR_ARG, "run_noalloc: need E_coll > 0 and 0 <= b < R0 (trajectory "
                    "%lld)", (long long)b);
    }
    if (bd->dynamics == MQCT_AT && !sy.drv)
      return fail(c, MQCT_ERR_STATE, "run_noalloc: AT dynamics needs a driving potential for "
                  "system %d", sid);
    amp_total += sy.N;
    max_npad[sy.dtype] = std::max(max_npad[sy.dtype], sy.Npad);
  }
  const size_t rec_bytes = (size_t)B * sizeof(TrajIn);
  const size_t a0_off = (rec_bytes + 255) & ~(size_t)255;
  const size_t need = bd->a0 ? a0_off + (size_t)amp_total * 16 : rec_bytes;
  if ((size_t)B > NOALLOC_SCRATCH_BYTES / sizeof(TrajIn) || need > NOALLOC_SCRATCH_BYTES)
    return fail(c, MQCT_ERR_ARG, "run_noalloc: the batch needs %zu bytes of scratch, more than "
                "its %zu (at most %zu trajectories without a0)", need, NOALLOC_SCRATCH_BYTES,
                NOALLOC_SCRATCH_BYTES / sizeof(TrajIn));
  HIP_TRY(c, hipSetDevice(c->device), "run_noalloc");
  // the work of an earlier call on the stream may still read the scratch
  HIP_TRY(c, hipStreamSynchronize(c->stream), "run_noalloc");
  // records grouped by storage type, staged through a fixed host buffer and
  // copied into the scratch chunk by chunk (synchronously: the buffer is reused)
  constexpr int CH = 64;
  TrajIn chunk[CH];
  int64_t pos = 0;
  int64_t first[4] = {0, 0, 0, 0}, count[4] = {0, 0, 0, 0};
  for (int d = 0; d < 4; ++d) {
    first[d] = pos;
    int nc = 0;
    int64_t amp_off = 0;
    for (int64_t b = 0; b < B; ++b) {
      const int sid = bd->system_id[b];
      const SysHost& sh = c->systems[sid];
      const int64_t off = amp_off;
      amp_off += sh.dev.N;
      if (sh.dev.dtype != d) continue;
      TrajIn t{};
      t.id = b;
      t.amp_off = off;
      t.sys = sid;
      t.n_steps = bd->n_steps[b];
      t.dt = bd->dt[b];
      t.t0 = bd->t0 ? bd->t0[b] : 0.0;
      if (bd->a0) t.flags |= TRAJ_HAS_A0;
      else t.init_channel = bd->init_channel[b];
      if (bd->classical0) {
        t.flags |= TRAJ_HAS_C0;
        for (int i = 0; i < 6; ++i) t.c0[i] = bd->classical0[b * 6 + i];
      } else {
        t.E_coll = bd->E_coll[b];
        t.b = bd->b[b];
        t.R0 = bd->R0 ? bd->R0[b] : sh.R_last;
      }
      if (bd->dynamics == MQCT_AT) t.flags |= TRAJ_AT;
      chunk[nc++] = t;
      if (nc == CH) {
        HIP_TRY(c, hipMemcpyAsync(c->scratch + (size_t)pos * sizeof(TrajIn), chunk,
                                  CH * sizeof(TrajIn), hipMemcpyHostToDevice, c->stream),
                "run_noalloc: records");
        HIP_TRY(c, hipStreamSynchronize(c->stream), "run_noalloc: records");
        pos += nc;
        nc = 0;
      }
    }
    if (nc) {
      HIP_TRY(c, hipMemcpyAsync(c->scratch + (size_t)pos * sizeof(TrajIn), chunk,
                                nc * sizeof(TrajIn), hipMemcpyHostToDevice, c->stream),
              "run_noalloc: records");
      HIP_TRY(c, hipStreamSynchronize(c->stream), "run_noalloc: records");
      pos += nc;
    }
    count[d] = pos - first[d];
  }
  const double* d_a0 = nullptr;
  if (bd->a0) {
    HIP_TRY(c, hipMemcpyAsync(c->scratch + a0_off, bd->a0, (size_t)amp_total * 16,
                              hipMemcpyHostToDevice, c->stream), "run_noalloc: a0");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "run_noalloc: a0");
    d_a0 = (const double*)(c->scratch + a0_off);
  }
  TrajOut out{};
  out.P = res->P; out.a_final = res->a_final; out.classical = res->classical;
  out.t_final = res->t_final; out.steps = res->steps; out.rejects = res->rejects;
  out.status = res->status; out.norm_err = res->norm_err; out.energy_err = res->energy_err;
  out.angmom_err = res->angmom_err;
  for (int d = 0; d < 4; ++d) {
    if (!count[d]) continue;
    hipError_t e = launch_rk4_gemv(c->d_systems, (const TrajIn*)c->scratch + first[d], count[d],
                                   d_a0, out, d, max_npad[d], c->stream, nullptr);
    if (e == hipErrorInvalidValue)
      return fail(c, MQCT_ERR_UNSUPPORTED, "run_noalloc: N too large for the per-trajectory schedule");
    if (e != hipSuccess) return hip_fail(c, e, "run_noalloc: launch");
  }
  return MQCT_OK;
}

mqct_status mqct_state_count(mqct_context* c, int64_t* count) {
  if (!c) return MQCT_ERR_ARG;
  if (!count) return fail(c, MQCT_ERR_ARG, "state_count: null argument");
  *count = c->st_B;
  return MQCT_OK;
}

mqct_status mqct_get_state(mqct_context* c, int64_t first, int64_t count, mqct_traj_state* state,
                           double* amps) {
  if (!c) return MQCT_ERR_ARG;
  if (!state || first < 0 || count < 0 || first + count > c->st_B)
    return fail(c, MQCT_ERR_ARG, "get_state: range [%lld, %lld) beyond the %lld stored "
                "trajectories (or null state)", (long long)first, (long long)(first + count),
                (long long)c->st_B);
  if (count == 0) return MQCT_OK;
  HIP_TRY(c, hipSetDevice(c->device), "get_state");
  HIP_TRY(c, hipMemcpyAsync(state, (const mqct_traj_state*)c->st_rec.p + first,
                            count * sizeof(mqct_traj_state), hipMemcpyDeviceToHost, c->stream),
          "get_state");
  if (amps) {
    const int64_t a0 = c->st_off[first], a1 = c->st_off[first + count];
    HIP_TRY(c, hipMemcpyAsync(amps, (const double2*)c->st_amp.p + a0, (a1 - a0) * 16,
                              hipMemcpyDeviceToHost, c->stream), "get_state");
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream), "get_state");
  return MQCT_OK;
}

mqct_status mqct_set_state(mqct_context* c, int64_t first, int64_t count,
                           const mqct_traj_state* state, const double* amps) {
  if (!c) return MQCT_ERR_ARG;
  if (!state || !amps || first < 0 || count < 1)
    return fail(c, MQCT_ERR_ARG, "set_state: need count >= 1, first >= 0, state and amps");
  const bool redefine = first == 0 && count != c->st_B;
  if (!redefine && first + count > c->st_B)
    return fail(c, MQCT_ERR_ARG, "set_state: range [%lld, %lld) beyond the %lld stored "
                "trajectories", (long long)first, (long long)(first + count), (long long)c->st_B);
  int64_t amp_n = 0;
  for (int64_t i = 0; i < count; ++i) {
    const mqct_traj_state& r = state[i];
    const int sid = r.system_id;
    if (sid < 0 || sid >= (int)c->systems.size() || !c->systems[sid].live)
      return fail(c, MQCT_ERR_STATE, "set_state: record %lld names unknown system %d",
                  (long long)i, sid);
    if (r.N != c->systems[sid].dev.N)
      return fail(c, MQCT_ERR_ARG, "set_state: record %lld has N = %d, its system %d", (long long)i,
                  r.N, c->systems[sid].dev.N);
    if (!redefine && (sid != c->st_sys[first + i]))
      return fail(c, MQCT_ERR_ARG, "set_state: record %lld changes the stored system", (long long)i);
    const double v[12] = {r.t, r.t_origin, r.h, r.classical[0], r.classical[1], r.classical[2],
                          r.classical[3], r.classical[4], r.classical[5], r.E0, r.J0, r.R_exit};
    if (!finite_arr(v, 12)) return fail(c, MQCT_ERR_NONFINITE, "set_state: record %lld", (long long)i);
    if (!(r.classical[0] > 0.0) || !(r.h >= 0.0) || r.n_origin < 0 || r.steps < 0 ||
        r.rejects < 0 || r.attempts < 0)
      return fail(c, MQCT_ERR_ARG, "set_state: record %lld: need R > 0, h >= 0, counts >= 0",
                  (long long)i);
    amp_n += r.N;
  }
  if (!finite_arr(amps, 2 * amp_n)) return fail(c, MQCT_ERR_NONFINITE, "set_state: amplitudes");
  HIP_TRY(c, hipSetDevice(c->device), "set_state");
  mqct_status st;
  if (redefine) {
    if ((st = ensure(c, c->st_rec, count * sizeof(mqct_traj_state), "set_state")) != MQCT_OK)
      return st;
    if ((st = ensure(c, c->st_amp, amp_n * 16, "set_state")) != MQCT_OK) return st;
    c->st_B = count;
    c->st_sys.resize(count);
    c->st_off.assign(count + 1, 0);
    for (int64_t i = 0; i < count; ++i) {
      c->st_sys[i] = state[i].system_id;
      c->st_off[i + 1] = c->st_off[i] + state[i].N;
    }
  }
  HIP_TRY(c, hipMemcpyAsync((mqct_traj_state*)c->st_rec.p + first, state,
                            count * sizeof(mqct_traj_state), hipMemcpyHostToDevice, c->stream),
          "set_state");
  HIP_TRY(c, hipMemcpyAsync((double2*)c->st_amp.p + c->st_off[first], amps, amp_n * 16,
                            hipMemcpyHostToDevice, c->stream), "set_state");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "set_state");
  return MQCT_OK;
}

mqct_status mqct_system_set_params(mqct_context* c, int32_t id, int32_t P, const double* radial,
                                   const int32_t* gidx, int32_t nG, const double* G) {
  if (!c) return MQCT_ERR_ARG;
  if (id < 0 || id >= (int)c->systems.size() || !c->systems[id].live)
    return fail(c, MQCT_ERR_STATE, "set_params: unknown system %d", id);
  SysHost& sh = c->systems[id];
  const int N = sh.dev.N, K = sh.dev.K, Npad = sh.dev.Npad;
  if (sh.dev.dtype != R64 || sh.dev.csr_row)
    return fail(c, MQCT_ERR_UNSUPPORTED, "set_params: the parametric form needs dense or slot "
                "R64 tables");
  if (P < 1 || P > 256 || nG < 1 || nG > 48 || !radial || !gidx || !G)
    return fail(c, MQCT_ERR_ARG, "set_params: need 1 <= P <= 256, 1 <= nG <= 48 and all arrays");
  for (int p = 0; p < P; ++p)
    if (gidx[p] < 0 || gidx[p] >= nG) return fail(c, MQCT_ERR_ARG, "set_params: gidx out of range");
  if (!finite_arr(radial, (int64_t)P * K) || !finite_arr(G, (int64_t)nG * N * N))
    return fail(c, MQCT_ERR_NONFINITE, "set_params: non-finite input");
  for (int t = 0; t < nG; ++t)
    for (int n = 0; n < N; ++n)
      for (int m = n + 1; m < N; ++m)
        if (G[((int64_t)t * N + n) * N + m] != G[((int64_t)t * N + m) * N + n])
          return fail(c, MQCT_ERR_NOT_HERMITIAN, "set_params: G is not symmetric");
  HIP_TRY(c, hipSetDevice(c->device), "set_params");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "set_params");
  free_params(sh);
  // sparse tables keep the load-time pattern: the model is the truncated one,
  // so its derivative in theta lists only the kept elements of each G_t
  std::vector<char> kept;
  if (sh.dev.ell_w > 0) {
    const int W = sh.dev.ell_w;
    std::vector<int32_t> col((size_t)W * Npad);
    std::vector<int> cnt(N);
    HIP_TRY(c, hipMemcpy(col.data(), sh.dev.ell_col, col.size() * 4, hipMemcpyDeviceToHost),
            "set_params: pattern");
    HIP_TRY(c, hipMemcpy(cnt.data(), sh.ebuf[1], (size_t)N * 4, hipMemcpyDeviceToHost),
            "set_params: pattern");
    kept.assign((size_t)N * N, 0);
    for (int n = 0; n < N; ++n)
      for (int q = 0; q < cnt[n]; ++q) kept[(size_t)col[(size_t)q * Npad + n] * N + n] = 1;
  }
  std::vector<double> Gp((size_t)nG * N * Npad, 0.0);
  std::vector<int> goff(nG + 1, 0);
  std::vector<uint32_t> gent;
  std::vector<double> gval;
  for (int t = 0; t < nG; ++t) {
    for (int n = 0; n < N; ++n)
      for (int m = 0; m < N; ++m) {
        const double v = G[((int64_t)t * N + n) * N + m];
        Gp[((size_t)t * N + n) * Npad + m] = v;
        if (v != 0.0 && (kept.empty() || kept[(size_t)n * N + m])) {
          gent.push_back((uint32_t)n | ((uint32_t)m << 16));
          gval.push_back(v);
        }
      }
    goff[t + 1] = (int)gent.size();
  }
  const size_t nnz = std::max<size_t>(gent.size(), 1);
  double* tmp = nullptr;
  hipError_t e;
  auto bail = [&](hipError_t err) {
    if (tmp) hipFree(tmp);
    free_params(sh);
    return hip_fail(c, err, "set_params");
  };
  if ((e = dev_malloc(&sh.pbufs[0], Gp.size() * 8)) != hipSuccess) return bail(e);
  if ((e = dev_malloc(&sh.pbufs[1], (size_t)P * K * 8)) != hipSuccess) return bail(e);
  if ((e = dev_malloc(&sh.pbufs[2], (size_t)P * K * 8)) != hipSuccess) return bail(e);
  if ((e = dev_malloc(&sh.pbufs[3], (size_t)P * 4)) != hipSuccess) return bail(e);
  if ((e = dev_malloc(&sh.pbufs[4], (size_t)(nG + 1) * 4)) != hipSuccess) return bail(e);
  if ((e = dev_malloc(&sh.pbufs[5], nnz * 4)) != hipSuccess) return bail(e);
  if ((e = dev_malloc(&sh.pbufs[6], nnz * 8)) != hipSuccess) return bail(e);
  if ((e = dev_malloc((void**)&tmp, (size_t)2 * P * K * 8)) != hipSuccess) return bail(e);
  if ((e = hipMemcpy(sh.pbufs[4], goff.data(), (size_t)(nG + 1) * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (!gent.empty() &&
       ((e = hipMemcpy(sh.pbufs[5], gent.data(), gent.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(sh.pbufs[6], gval.data(), gval.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)))
    return bail(e);
  if ((e = hipMemcpy(sh.pbufs[0], Gp.data(), Gp.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(sh.pbufs[1], radial, (size_t)P * K * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(sh.pbufs[3], gidx, (size_t)P * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e);
  if ((e = launch_spline_rows((const double*)sh.pbufs[1], sh.dev.R, K, P, (double*)sh.pbufs[2],
                              tmp, c->stream)) != hipSuccess)
    return bail(e);
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e);
  hipFree(tmp);
  sh.P = P;
  sh.nG = nG;
  sh.h_goff = goff;
  return MQCT_OK;
}

mqct_status mqct_system_set_theta(mqct_context* c, int32_t id, const double* theta) {
  if (!c) return MQCT_ERR_ARG;
  if (id < 0 || id >= (int)c->systems.size() || !c->systems[id].live)
    return fail(c, MQCT_ERR_STATE, "set_theta: unknown system %d", id);
  SysHost& sh = c->systems[id];
  if (sh.P == 0) return fail(c, MQCT_ERR_STATE, "set_theta: no parametric form attached");
  if (!theta || !finite_arr(theta, sh.P)) return fail(c, MQCT_ERR_ARG, "set_theta: bad theta");
  const int N = sh.dev.N, K = sh.dev.K, Npad = sh.dev.Npad;
  HIP_TRY(c, hipSetDevice(c->device), "set_theta");
  double *Min = nullptr, *th = nullptr, *tmp = nullptr;
  const int64_t tmp_doubles = std::max<int64_t>(K, std::min<int64_t>((int64_t)K * N * Npad,
                                                                    (int64_t)64 << 20));
  hipError_t e;
  auto done = [&](hipError_t err) -> mqct_status {
    if (Min) hipFree(Min);
    if (th) hipFree(th);
    if (tmp) hipFree(tmp);
    return err == hipSuccess ? MQCT_OK : hip_fail(c, err, "set_theta");
  };
  if ((e = dev_malloc((void**)&Min, (size_t)K * N * N * 8)) != hipSuccess) return done(e);
  if ((e = dev_malloc((void**)&th, (size_t)sh.P * 8)) != hipSuccess) return done(e);
  if ((e = dev_malloc((void**)&tmp, (size_t)tmp_doubles * 8)) != hipSuccess) return done(e);
  if ((e = hipMemcpyAsync(th, theta, (size_t)sh.P * 8, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return done(e);
  if ((e = launch_build_param_tables((const double*)sh.pbufs[0], (const double*)sh.pbufs[1],
                                     (const int*)sh.pbufs[3], th, sh.P, sh.nG, N, Npad, K, Min,
                                     c->stream)) != hipSuccess)
    return done(e);
  if (sh.dev.ell_w == 0) {
    if ((e = launch_spline_prepare(Min, sh.dev.R, N, K, Npad, 1, sh.dev.dtype, sh.bufs[0],
                                   sh.bufs[1], tmp, tmp_doubles, c->stream)) != hipSuccess)
      return done(e);
    return done(hipStreamSynchronize(c->stream));
  }
  // sparse tables: dense storage first, then the load-time slots (the pattern is
  // fixed when the system is loaded)
  void* D = nullptr;
  void* D2 = nullptr;
  const size_t dbytes = (size_t)K * N * Npad * dtype_bytes(sh.dev.dtype);
  if ((e = dev_malloc(&D, dbytes)) != hipSuccess) return done(e);
  if ((e = dev_malloc(&D2, dbytes)) != hipSuccess) { hipFree(D); return done(e); }
  e = launch_spline_prepare(Min, sh.dev.R, N, K, Npad, 1, sh.dev.dtype, D, D2, tmp, tmp_doubles,
                            c->stream);
  if (e == hipSuccess)
    e = launch_ell_gather(D, D2, sh.dev.ell_col, (const int*)sh.ebuf[1], N, Npad, K, sh.dev.ell_w,
                          1, sh.dev.dtype, sh.bufs[0], sh.bufs[1], c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(D);
  hipFree(D2);
  return done(e);
}

mqct_status mqct_adjoint(mqct_context* c, const mqct_batch_desc* bd, int32_t checkpoint_every,
                         const double* dL_dP, double* dL_dtheta, double* P_out) {
  if (!c) return MQCT_ERR_ARG;
  if (!bd || !dL_dP || !dL_dtheta) return fail(c, MQCT_ERR_ARG, "adjoint: null argument");
  const int64_t B = bd->B;
  if (B < 1 || !bd->system_id || !bd->init_channel || !bd->E_coll || !bd->b || !bd->dt ||
      !bd->n_steps)
    return fail(c, MQCT_ERR_ARG, "adjoint: needs B >= 1, system_id, init_channel, E_coll, b, dt, n_steps");
  if (bd->integrator != MQCT_RK4) return fail(c, MQCT_ERR_UNSUPPORTED, "adjoint: RK4 only");
  if (bd->dynamics != MQCT_EHRENFEST)
    return fail(c, MQCT_ERR_UNSUPPORTED, "adjoint: Ehrenfest dynamics only");
  if (bd->a0 || bd->classical0 || bd->t0 || bd->resume)
    return fail(c, MQCT_ERR_UNSUPPORTED, "adjoint: start states come from init_channel/E_coll/b/R0");
  if (checkpoint_every < 1) return fail(c, MQCT_ERR_ARG, "adjoint: checkpoint_every must be >= 1");
  if (B > INT32_MAX) return fail(c, MQCT_ERR_UNSUPPORTED, "adjoint: B too large");
  const int sid = bd->system_id[0];
  for (int64_t b = 0; b < B; ++b)
    if (bd->system_id[b] != sid) return fail(c, MQCT_ERR_UNSUPPORTED, "adjoint: one system per batch");
  if (sid < 0 || sid >= (int)c->systems.size() || !c->systems[sid].live)
    return fail(c, MQCT_ERR_STATE, "adjoint: unknown system %d", sid);
  SysHost& sh = c->systems[sid];
  if (sh.P == 0) return fail(c, MQCT_ERR_STATE, "adjoint: no parametric form attached");
  const DevSystem& sy = sh.dev;
  if (sy.Npad > 1024) return fail(c, MQCT_ERR_UNSUPPORTED, "adjoint: N > 1024");
  HIP_TRY(c, hipSetDevice(c->device), "adjoint");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "adjoint");
  std::vector<TrajIn> tr(B);
  int64_t maxn = 0, amp = 0;
  double Rlast;
  HIP_TRY(c, hipMemcpy(&Rlast, sy.R + (sy.K - 1), 8, hipMemcpyDeviceToHost), "adjoint");
  for (int64_t b = 0; b < B; ++b) {
    TrajIn t{};
    t.id = b; t.amp_off = amp; t.sys = sid; t.n_steps = bd->n_steps[b]; t.dt = bd->dt[b];
    t.init_channel = bd->init_channel[b]; t.E_coll = bd->E_coll[b]; t.b = bd->b[b];
    t.R0 = bd->R0 ? bd->R0[b] : Rlast;
    if (t.n_steps < 0 || !isfinite(t.dt) || t.init_channel < 0 || t.init_channel >= sy.N ||
        !(t.E_coll > 0.0) || !(t.b >= 0.0) || !(t.b < t.R0))
      return fail(c, MQCT_ERR_ARG, "adjoint: bad trajectory %lld", (long long)b);
    maxn = std::max(maxn, t.n_steps);
    amp += sy.N;
    tr[b] = t;
  }
  // an interval beyond the longest trajectory is one segment: no larger workspace
  const int S = (int)std::min<int64_t>(checkpoint_every, std::max<int64_t>(maxn, 1));
  const int64_t stride = adjoint_scratch_doubles(sy.Npad, maxn, S);
  size_t off = 0;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_traj = off; off += al(B * sizeof(TrajIn));
  const size_t o_ord = off; off += al((size_t)B * 4);
  const size_t o_w = off; off += al((size_t)amp * 8);
  const size_t o_part = off; off += al((size_t)B * sh.P * 8);
  const size_t o_g = off; off += al((size_t)sh.P * 8);
  const size_t o_P = off; off += al((size_t)amp * 8);
  const size_t o_s = off; off += al((size_t)B * stride * 8);
  mqct_status st;
  if ((st = ensure(c, c->binws, off, "adjoint: workspace")) != MQCT_OK) return st;
  char* base = (char*)c->binws.p;
  HIP_TRY(c, hipMemcpyAsync(base + o_traj, tr.data(), B * sizeof(TrajIn), hipMemcpyHostToDevice,
                            c->stream), "adjoint");
  // trajectories of similar paths (same energy and start, neighbouring impact
  // parameters) go to the same die, so the spline slices they read at a time are
  // fewer and stay in that die's L2; every trajectory writes its own results
  std::vector<int> ord(B);
  for (int64_t b = 0; b < B; ++b) ord[b] = (int)b;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    const TrajIn &p = tr[x], &q = tr[y];
    if (p.E_coll != q.E_coll) return p.E_coll < q.E_coll;
    if (p.R0 != q.R0) return p.R0 < q.R0;
    return p.b < q.b;
  });
  HIP_TRY(c, hipMemcpyAsync(base + o_ord, ord.data(), (size_t)B * 4, hipMemcpyHostToDevice,
                            c->stream), "adjoint");
  HIP_TRY(c, hipMemcpyAsync(base + o_w, dL_dP, (size_t)amp * 8, hipMemcpyHostToDevice, c->stream),
          "adjoint");
  hipEvent_t e0 = c->prof.next(), e1 = c->prof.next();
  prof_mark(&c->prof, e0, c->stream);
  HIP_TRY(c, launch_adjoint(c->d_systems, dtype_complex(sy.dtype), sy.ell_w > 0, sy.Npad,
                            (const TrajIn*)(base + o_traj), (const int*)(base + o_ord), B,
                            (const double*)(base + o_w),
                            (double*)(base + o_part), (double*)(base + o_g),
                            (double*)(base + o_P), (double*)(base + o_s), stride, S,
                            (const int*)sh.pbufs[4], sh.h_goff.data(), (const uint32_t*)sh.pbufs[5],
                            (const double*)sh.pbufs[6], (const double*)sh.pbufs[1],
                            (const double*)sh.pbufs[2], (const int*)sh.pbufs[3], sh.P, sh.nG,
                            maxn <= S, c->stream), "adjoint: launch");
  prof_mark(&c->prof, e1, c->stream);
  HIP_TRY(c, hipMemcpyAsync(dL_dtheta, base + o_g, (size_t)sh.P * 8, hipMemcpyDeviceToHost,
                            c->stream), "adjoint");
  if (P_out)
    HIP_TRY(c, hipMemcpyAsync(P_out, base + o_P, (size_t)amp * 8, hipMemcpyDeviceToHost, c->stream),
            "adjoint");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "adjoint");
  return MQCT_OK;
}

mqct_status mqct_set_option(mqct_context* c, int32_t option, int64_t value) {
  if (!c) return MQCT_ERR_ARG;
  switch (option) {
    case MQCT_OPT_GRAPHS: c->qopt.graphs = value != 0; return MQCT_OK;
    case MQCT_OPT_AUTOTUNE: c->qopt.tune = value != 0; return MQCT_OK;
    case MQCT_OPT_CHUNK:
      if (value < 1 || value > 4096) return fail(c, MQCT_ERR_ARG, "set_option: chunk must be 1..4096");
      c->qopt.chunk = (int)value;
      return MQCT_OK;
    case MQCT_OPT_RESET_TUNING: c->qcache.entries.clear(); return MQCT_OK;
    case MQCT_OPT_TAIL:
      if (value < 0 || value > 2) return fail(c, MQCT_ERR_ARG, "set_option: tail must be 0, 1 or 2");
      c->qopt.tail = (int)value;
      return MQCT_OK;
    case MQCT_OPT_PER_LAUNCH:
      if (value < 1 || value > 64) return fail(c, MQCT_ERR_ARG, "set_option: per_launch must be 1..64");
      c->qopt.per_launch = (int)value;
      return MQCT_OK;
    case MQCT_OPT_COL_WORKSPACE:
      if (value < 0) return fail(c, MQCT_ERR_ARG, "set_option: columns workspace cap must be >= 0");
      c->qopt.col_ws = value;
      return MQCT_OK;
  }
  return fail(c, MQCT_ERR_ARG, "set_option: unknown option %d", option);
}

const char* mqct_tuning_report(mqct_context* c) {
  if (!c) return "";
  std::string r = "[";
  char buf[256];
  for (size_t i = 0; i < c->qcache.entries.size(); ++i) {
    const QueueTuneEntry& en = c->qcache.entries[i];
    const QKernelSet& ks = queue_kernels(en.dtype)[en.shape];
    snprintf(buf, sizeof buf,
             "%s{\"dtype\": %d, \"npad\": %d, \"method\": %d, \"block\": %d, \"rows_per_lane\": %d, "
             "\"tuned\": %s, \"candidates\": [",
             i ? ", " : "", en.dtype, en.npad, en.method, ks.block, ks.rpt * (en.dtype == C128 ? 1 : 2),
             en.tuned ? "true" : "false");
    r += buf;
    for (size_t j = 0; j < en.ms.size(); ++j) {
      const QKernelSet& kj = queue_kernels(en.dtype)[en.ms[j].first];
      snprintf(buf, sizeof buf, "%s{\"block\": %d, \"rows_per_lane\": %d, \"ms\": %.6g}",
               j ? ", " : "", kj.block, kj.rpt * (en.dtype == C128 ? 1 : 2), en.ms[j].second);
      r += buf;
    }
    r += "], \"tail\": ";
    if (en.tail_shape >= 0) {
      const QKernelSet& kt = queue_kernels(en.dtype)[en.tail_shape];
      snprintf(buf, sizeof buf, "{\"block\": %d, \"rows_per_lane\": %d, \"split_waves\": %d}",
               kt.block, kt.rpt * (en.dtype == C128 ? 1 : 2), kt.split_waves);
      r += buf;
    } else {
      r += "null";
    }
    r += ", \"tail_candidates\": [";
    for (size_t j = 0; j < en.tail_ms.size(); ++j) {
      const QKernelSet& kj = queue_kernels(en.dtype)[en.tail_ms[j].first];
      snprintf(buf, sizeof buf,
               "%s{\"block\": %d, \"rows_per_lane\": %d, \"split_waves\": %d, \"ms\": %.6g}",
               j ? ", " : "", kj.block, kj.rpt * (en.dtype == C128 ? 1 : 2), kj.split_waves,
               en.tail_ms[j].second);
      r += buf;
    }
    r += "]}";
  }
  r += "]";
  c->report = r;
  return c->report.c_str();
}

mqct_status mqct_xs_symmetrize(mqct_context* c, int32_t mem, int32_t nE, int32_t L,
                               const double* g, const double* sigma, double* sym, double* ratio) {
  if (!c) return MQCT_ERR_ARG;
  if (nE < 1 || L < 1 || !g || !sigma || (!sym && !ratio))
    return fail(c, MQCT_ERR_ARG, "xs_symmetrize: need n_E, L >= 1, g, sigma and an output");
  if (mem != MQCT_MEM_HOST && mem != MQCT_MEM_DEVICE)
    return fail(c, MQCT_ERR_ARG, "xs_symmetrize: mem must be host or device");
  const size_t n = (size_t)nE * L * L;
  if (mem == MQCT_MEM_HOST && (!finite_arr(g, L) || !finite_arr(sigma, (int64_t)n)))
    return fail(c, MQCT_ERR_NONFINITE, "xs_symmetrize: non-finite input");
  HIP_TRY(c, hipSetDevice(c->device), "xs_symmetrize");
  if (mem == MQCT_MEM_DEVICE) {
    HIP_TRY(c, launch_xs_symmetrize(nE, L, g, sigma, sym, ratio, c->stream), "xs_symmetrize");
    return MQCT_OK;
  }
  mqct_status st;
  const size_t need = (L + 3 * n) * 8;
  if ((st = ensure(c, c->xs[1], need, "xs_symmetrize")) != MQCT_OK) return st;
  double* dg = (double*)c->xs[1].p;
  double *ds = dg + L, *dy = ds + n, *dr = dy + n;
  HIP_TRY(c, hipMemcpyAsync(dg, g, L * 8, hipMemcpyHostToDevice, c->stream), "xs_symmetrize");
  HIP_TRY(c, hipMemcpyAsync(ds, sigma, n * 8, hipMemcpyHostToDevice, c->stream), "xs_symmetrize");
  HIP_TRY(c, launch_xs_symmetrize(nE, L, dg, ds, sym ? dy : nullptr, ratio ? dr : nullptr,
                                  c->stream), "xs_symmetrize");
  if (sym) HIP_TRY(c, hipMemcpyAsync(sym, dy, n * 8, hipMemcpyDeviceToHost, c->stream), "xs_symmetrize");
  if (ratio) HIP_TRY(c, hipMemcpyAsync(ratio, dr, n * 8, hipMemcpyDeviceToHost, c->stream), "xs_symmetrize");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "xs_symmetrize");
  return MQCT_OK;
}

mqct_status mqct_rate_coefficients(mqct_context* c, int32_t mem, int32_t nE, int32_t L,
                                   const double* U, const double* E, const double* g,
                                   const double* sym, double mu, int32_t nT, const double* beta,
                                   double* k) {
  if (!c) return MQCT_ERR_ARG;
  if (nE < 2 || nE > 64 || L < 1 || nT < 1 || !U || !E || !g || !sym || !beta || !k)
    return fail(c, MQCT_ERR_ARG, "rate_coefficients: need 2 <= n_E <= 64, L, n_T >= 1 and "
                "every array");
  if (mem != MQCT_MEM_HOST && mem != MQCT_MEM_DEVICE)
    return fail(c, MQCT_ERR_ARG, "rate_coefficients: mem must be host or device");
  if (!(mu > 0.0) || !isfinite(mu)) return fail(c, MQCT_ERR_ARG, "rate_coefficients: mu must be > 0");
  const size_t n = (size_t)nE * L * L, nk = (size_t)nT * L * L;
  if (mem == MQCT_MEM_HOST) {
    if (!finite_arr(U, nE) || !finite_arr(E, L) || !finite_arr(g, L) ||
        !finite_arr(sym, (int64_t)n) || !finite_arr(beta, nT))
      return fail(c, MQCT_ERR_NONFINITE, "rate_coefficients: non-finite input");
    for (int e = 1; e < nE; ++e)
      if (!(U[e] > U[e - 1])) return fail(c, MQCT_ERR_ARG, "rate_coefficients: U must increase");
    for (int i = 0; i < L; ++i)
      if (!(g[i] > 0.0)) return fail(c, MQCT_ERR_ARG, "rate_coefficients: g must be > 0");
    for (int t = 0; t < nT; ++t)
      if (!(beta[t] > 0.0)) return fail(c, MQCT_ERR_ARG, "rate_coefficients: beta must be > 0");
  }
  HIP_TRY(c, hipSetDevice(c->device), "rate_coefficients");
  if (mem == MQCT_MEM_DEVICE) {
    HIP_TRY(c, launch_xs_rates(nE, L, nT, U, E, g, sym, mu, beta, k, c->stream),
            "rate_coefficients");
    return MQCT_OK;
  }
  mqct_status st;
  const size_t need = (nE + 2 * L + n + nT + nk) * 8;
  if ((st = ensure(c, c->xs[2], need, "rate_coefficients")) != MQCT_OK) return st;
  double* dU = (double*)c->xs[2].p;
  double *dE = dU + nE, *dg = dE + L, *dy = dg + L, *db = dy + n, *dk = db + nT;
  HIP_TRY(c, hipMemcpyAsync(dU, U, nE * 8, hipMemcpyHostToDevice, c->stream), "rate_coefficients");
  HIP_TRY(c, hipMemcpyAsync(dE, E, L * 8, hipMemcpyHostToDevice, c->stream), "rate_coefficients");
  HIP_TRY(c, hipMemcpyAsync(dg, g, L * 8, hipMemcpyHostToDevice, c->stream), "rate_coefficients");
  HIP_TRY(c, hipMemcpyAsync(dy, sym, n * 8, hipMemcpyHostToDevice, c->stream), "rate_coefficients");
  HIP_TRY(c, hipMemcpyAsync(db, beta, nT * 8, hipMemcpyHostToDevice, c->stream), "rate_coefficients");
  hipEvent_t e0 = c->prof.next(), e1 = c->prof.next();
  prof_mark(&c->prof, e0, c->stream);
  HIP_TRY(c, launch_xs_rates(nE, L, nT, dU, dE, dg, dy, mu, db, dk, c->stream), "rate_coefficients");
  prof_mark(&c->prof, e1, c->stream);
  HIP_TRY(c, hipMemcpyAsync(k, dk, nk * 8, hipMemcpyDeviceToHost, c->stream), "rate_coefficients");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "rate_coefficients");
  return MQCT_OK;
}

namespace {

// Validation and device set-up shared by the dense and the screened builds: the
// (j1, j2, j) levels, terms sorted by lam, channels grouped by m, the work list
// (per row, tiles of 256 channels of the row's m group), and one device
// workspace holding them with the factor arrays.  On success *buf owns it.
mqct_status coupling_setup(mqct_context* c, const mqct_coupling_desc* d, const char* what,
                           CouplingDev& dev, char** buf) {
  *buf = nullptr;
  if (!d) return fail(c, MQCT_ERR_ARG, "%s: null descriptor", what);
  const int N = d->N, T = d->T, K = d->K, n1 = d->n_rot1, bs = d->b_stride;
  if (N < 1 || T < 1 || K < 1 || n1 < 1 || bs < 1)
    return fail(c, MQCT_ERR_ARG, "%s: need N, T, K, n_rot1, b_stride >= 1", what);
  if (!d->j || !d->m || !d->rot1 || !d->j2 || !d->rot1_j || !d->b || !d->lam1 || !d->mu1 ||
      !d->lam2 || !d->lam || !d->v)
    return fail(c, MQCT_ERR_ARG, "%s: null array", what);
  constexpr int JMAX = 40, LMAX = 20;
  for (int r = 0; r < n1; ++r)
    if (d->rot1_j[r] < 0 || d->rot1_j[r] > JMAX || 2 * d->rot1_j[r] + 1 > bs)
      return fail(c, MQCT_ERR_ARG, "%s: rotor-1 state %d: j1 out of 0..%d or b_stride too small",
                  what, r, JMAX);
  if (!finite_arr(d->b, (int64_t)n1 * bs) || !finite_arr(d->v, (int64_t)T * K))
    return fail(c, MQCT_ERR_NONFINITE, "%s: non-finite b or v", what);
  std::map<std::pair<int, std::pair<int, int>>, int> jl;
  std::vector<int32_t> jl_j1, jl_j2, jl_j, chan_J(N);
  for (int n = 0; n < N; ++n) {
    const int r = d->rot1[n], j2 = d->j2[n], j = d->j[n], m = d->m[n];
    if (r < 0 || r >= n1) return fail(c, MQCT_ERR_ARG, "%s: rot1[%d] out of range", what, n);
    const int j1 = d->rot1_j[r];
    if (j2 < 0 || j2 > JMAX || j < std::abs(j1 - j2) || j > j1 + j2 || std::abs(m) > j)
      return fail(c, MQCT_ERR_ARG, "%s: channel %d: need 0 <= j2 <= %d, |j1-j2| <= j <= j1+j2, "
                  "|m| <= j", what, n, JMAX);
    auto key = std::make_pair(j1, std::make_pair(j2, j));
    auto it = jl.find(key);
    if (it == jl.end()) {
      it = jl.emplace(key, (int)jl_j1.size()).first;
      jl_j1.push_back(j1);
      jl_j2.push_back(j2);
      jl_j.push_back(j);
    }
    chan_J[n] = it->second;
  }
  const int nJ = (int)jl_j1.size();
  std::vector<int32_t> perm(T);
  for (int t = 0; t < T; ++t) {
    const int l1 = d->lam1[t], u = d->mu1[t], l2 = d->lam2[t], l = d->lam[t];
    if (l1 < 0 || l1 > LMAX || l2 < 0 || l2 > LMAX || std::abs(u) > l1 || l < std::abs(l1 - l2) ||
        l > l1 + l2)
      return fail(c, MQCT_ERR_ARG, "%s: term %d: need 0 <= lam1, lam2 <= %d, |mu1| <= lam1, "
                  "|lam1-lam2| <= lam <= lam1+lam2", what, t, LMAX);
    perm[t] = t;
  }
  // terms sorted by lam (kept from the first form of the fill kernel; the order of
  // the sums over t is then the same in every kernel)
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int a, int b) { return d->lam[a] < d->lam[b]; });
  std::vector<int32_t> ints;
  auto put = [&](const int32_t* p, size_t n) {
    const size_t o = ints.size();
    ints.insert(ints.end(), p, p + n);
    return o;
  };
  std::vector<int32_t> tl1(T), tmu(T), tl2(T), tl(T);
  const int KP = (K + CPL_KNOT_CHUNK - 1) / CPL_KNOT_CHUNK * CPL_KNOT_CHUNK;
  std::vector<double> vs((size_t)T * KP, 0.0);
  int cg_lmax = 0, cg_jmax = 0;
  for (int t = 0; t < T; ++t) {
    const int u = perm[t];
    tl1[t] = d->lam1[u]; tmu[t] = d->mu1[u]; tl2[t] = d->lam2[u]; tl[t] = d->lam[u];
    memcpy(&vs[(size_t)t * KP], d->v + (size_t)u * K, (size_t)K * 8);
    cg_lmax = std::max(cg_lmax, tl[t]);
  }
  for (int n = 0; n < N; ++n) cg_jmax = std::max(cg_jmax, (int)d->j[n]);
  std::vector<int32_t> chan_r(d->rot1, d->rot1 + N), chan_j(d->j, d->j + N), chan_m(d->m, d->m + N);
  std::map<int, int> gid;
  for (int n = 0; n < N; ++n) gid.emplace(d->m[n], 0);
  int ng = 0;
  for (auto& kv : gid) kv.second = ng++;
  std::vector<int32_t> chan_grp(N), grp_off(ng + 1, 0), grp_list(N);
  for (int n = 0; n < N; ++n) {
    chan_grp[n] = gid[d->m[n]];
    ++grp_off[chan_grp[n] + 1];
  }
  for (int g = 0; g < ng; ++g) grp_off[g + 1] += grp_off[g];
  {
    std::vector<int32_t> fillp(grp_off.begin(), grp_off.end() - 1);
    for (int n = 0; n < N; ++n) grp_list[fillp[chan_grp[n]]++] = n;
  }
  // rows taken level by level ((j1, j2, j) of the row, then m): consecutive work
  // items then read the same row of level factors
  std::vector<int32_t> order(N);
  for (int n = 0; n < N; ++n) order[n] = n;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return chan_J[a] != chan_J[b] ? chan_J[a] < chan_J[b] : d->m[a] < d->m[b];
  });
  std::vector<int32_t> work;
  for (int n : order) {
    const int cnt = grp_off[chan_grp[n] + 1] - grp_off[chan_grp[n]];
    for (int tile = 0; tile * 256 < cnt; ++tile) {
      work.push_back(n);
      work.push_back(tile);
    }
  }
  const int64_t n_work = (int64_t)work.size() / 2;
  if (n_work > 0x7fffffffLL)
    return fail(c, MQCT_ERR_ARG, "%s: too many channels for one launch", what);
  const size_t o_cJ = put(chan_J.data(), N), o_cr = put(chan_r.data(), N),
               o_cj = put(chan_j.data(), N), o_cm = put(chan_m.data(), N),
               o_j1 = put(jl_j1.data(), nJ), o_j2 = put(jl_j2.data(), nJ),
               o_jj = put(jl_j.data(), nJ), o_rj = put(d->rot1_j, n1),
               o_t1 = put(tl1.data(), T), o_tm = put(tmu.data(), T), o_t2 = put(tl2.data(), T),
               o_tl = put(tl.data(), T), o_tu = put(perm.data(), T),
               o_cg = put(chan_grp.data(), N), o_go = put(grp_off.data(), ng + 1),
               o_gl = put(grp_list.data(), N);
  if (ints.size() & 1) ints.push_back(0);      // the work list is read as int2
  const size_t o_wk = put(work.data(), work.size());
  const size_t ibytes = (ints.size() * 4 + 255) / 256 * 256;
  const size_t n_b = (size_t)n1 * bs, n_v = (size_t)T * KP, n_lf = 256;
  const size_t n_K = (size_t)T * n1 * n1, n_F = (size_t)T * nJ * nJ;
  const size_t n_cg = (size_t)(cg_jmax + 1) * (cg_jmax + 1) * (2 * cg_jmax + 1) * (cg_lmax + 1);
  const size_t total = ibytes + (n_b + n_v + n_lf + n_K + n_F + n_cg) * 8;
  HIP_TRY(c, hipSetDevice(c->device), what);
  char* w = nullptr;
  hipError_t e = dev_malloc((void**)&w, total);
  if (e != hipSuccess) return hip_fail(c, e, what);
  int32_t* di = (int32_t*)w;
  double* dd = (double*)(w + ibytes);
  double *db = dd, *dv = db + n_b, *dlf = dv + n_v, *dK = dlf + n_lf, *dF = dK + n_K,
         *dcg = dF + n_F;
  if ((e = hipMemcpy(di, ints.data(), ints.size() * 4, hipMemcpyHostToDevice)) == hipSuccess &&
      (e = hipMemcpy(db, d->b, n_b * 8, hipMemcpyHostToDevice)) == hipSuccess)
    e = hipMemcpy(dv, vs.data(), n_v * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(w);
    return hip_fail(c, e, what);
  }
  dev = CouplingDev{N, T, K, n1, nJ, bs, di + o_cJ, di + o_cr, di + o_cj, di + o_cm,
                    di + o_j1, di + o_j2, di + o_jj, di + o_rj, db, di + o_t1, di + o_tm,
                    di + o_t2, di + o_tl, di + o_tu, dv, dlf, dK, dF, di + o_cg, di + o_go,
                    di + o_gl, (const int2*)(di + o_wk), n_work, KP, cg_jmax, cg_lmax, dcg};
  *buf = w;
  return MQCT_OK;
}

}  // namespace

mqct_status mqct_coupling_build(mqct_context* c, const mqct_coupling_desc* d, double* M_out,
                                double* G_out) {
  if (!c) return MQCT_ERR_ARG;
  if (!M_out && !G_out) return fail(c, MQCT_ERR_ARG, "coupling_build: no output requested");
  CouplingDev dev;
  char* buf = nullptr;
  mqct_status st = coupling_setup(c, d, "coupling_build", dev, &buf);
  if (st != MQCT_OK) return st;
  hipError_t e = launch_coupling(dev, M_out, G_out, &c->prof, c->stream);
  if (e == hipErrorInvalidValue) {
    hipFree(buf);
    return fail(c, MQCT_ERR_ARG, "coupling_build: output too large for one launch");
  }
  if (e == hipSuccess && c->prof.on)
    c->prof.bytes += ((M_out ? (double)dev.K : 0.0) + (G_out ? (double)dev.T : 0.0)) * dev.N *
                     (double)dev.N * 8.0;
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(buf);
  if (e != hipSuccess) return hip_fail(c, e, "coupling_build");
  return MQCT_OK;
}

mqct_status mqct_coupling_build_sparse(mqct_context* c, const mqct_coupling_desc* d,
                                       int32_t n_screen, const double* v_screen,
                                       double drop_below, int64_t capacity, int32_t* rows,
                                       int32_t* cols, double* values, int64_t* n_kept) {
  if (!c) return MQCT_ERR_ARG;
  if (!n_kept || n_screen < 1 || n_screen > CPL_MAX_SCREEN || !v_screen || capacity < 0 ||
      (capacity > 0 && (!rows || !cols || !values)))
    return fail(c, MQCT_ERR_ARG, "coupling_build_sparse: need 1 <= n_screen <= %d, v_screen, "
                "n_kept, and rows, cols, values when capacity > 0", CPL_MAX_SCREEN);
  if (!(drop_below >= 0.0) || !isfinite(drop_below))
    return fail(c, MQCT_ERR_ARG, "coupling_build_sparse: drop_below must be finite and >= 0");
  *n_kept = 0;
  if (d && d->T >= 1 && !finite_arr(v_screen, (int64_t)d->T * n_screen))
    return fail(c, MQCT_ERR_NONFINITE, "coupling_build_sparse: non-finite v_screen");
  CouplingDev dev;
  char* buf = nullptr;
  mqct_status st = coupling_setup(c, d, "coupling_build_sparse", dev, &buf);
  if (st != MQCT_OK) return st;
  // screening coefficients in the sorted term order, and the kept-element counter
  std::vector<double> vs((size_t)dev.T * n_screen);
  std::vector<int32_t> perm(dev.T);
  HIP_TRY(c, hipMemcpy(perm.data(), dev.t_user, (size_t)dev.T * 4, hipMemcpyDeviceToHost),
          "coupling_build_sparse");
  for (int t = 0; t < dev.T; ++t)
    for (int q = 0; q < n_screen; ++q) vs[(size_t)t * n_screen + q] = v_screen[(size_t)perm[t] * n_screen + q];
  char* sbuf = nullptr;
  hipError_t e = dev_malloc((void**)&sbuf, 256 + vs.size() * 8);
  if (e == hipSuccess) {
    unsigned long long* cnt = (unsigned long long*)sbuf;
    double* dvs = (double*)(sbuf + 256);
    e = hipMemcpy(dvs, vs.data(), vs.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, 8, c->stream);
    hipEvent_t e0 = c->prof.next(), e1 = c->prof.next();
    prof_mark(&c->prof, e0, c->stream);
    if (e == hipSuccess)
      e = launch_coupling_screen(dev, n_screen, dvs, drop_below, capacity, cnt, rows, cols,
                                 c->stream);
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, cnt, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) {
      *n_kept = (int64_t)h;
      if ((int64_t)h <= capacity && h > 0)
        e = launch_coupling_values(dev, (int64_t)h, rows, cols, capacity, values, c->stream);
      prof_mark(&c->prof, e1, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
  }
  if (sbuf) hipFree(sbuf);
  hipFree(buf);
  if (e != hipSuccess) return hip_fail(c, e, "coupling_build_sparse");
  if (*n_kept > capacity)
    return fail(c, MQCT_ERR_ARG, "coupling_build_sparse: %lld elements kept, capacity %lld",
                (long long)*n_kept, (long long)capacity);
  return MQCT_OK;
}

mqct_status mqct_read_bandwidth(mqct_context* c, const void* buf, int64_t bytes, int32_t reps,
                                double* ms_per_pass) {
  if (!c) return MQCT_ERR_ARG;
  if (!buf || !ms_per_pass) return fail(c, MQCT_ERR_ARG, "read_bandwidth: null argument");
  if (bytes < 16 || bytes % 16 != 0 || ((uintptr_t)buf & 15) != 0)
    return fail(c, MQCT_ERR_ARG, "read_bandwidth: bytes must be a positive multiple of 16 "
                                 "and buf 16-byte aligned");
  if (reps < 1) return fail(c, MQCT_ERR_ARG, "read_bandwidth: reps must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device), "read_bandwidth");
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
  // one untimed pass, then reps passes between two events
  HIP_TRY(c, launch_read_probe(buf, bytes, cus, c->stream), "read_bandwidth");
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0), "read_bandwidth");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(c, MQCT_ERR_DEVICE, "read_bandwidth: event");
  }
  hipError_t e = hipEventRecord(e0, c->stream);
  for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = launch_read_probe(buf, bytes, cus, c->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "read_bandwidth");
  *ms_per_pass = (double)ms / reps;
  return MQCT_OK;
}

mqct_status mqct_set_profiling(mqct_context* c, int32_t enable) {
  if (!c) return MQCT_ERR_ARG;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "set_profiling");
  c->prof.on = enable != 0;
  c->prof.reset();
  return MQCT_OK;
}

mqct_status mqct_profile_read(mqct_context* c, double* total_ms, int64_t* launches,
                              double* table_bytes) {
  if (!c) return MQCT_ERR_ARG;
  if (!total_ms || !launches) return fail(c, MQCT_ERR_ARG, "profile_read: null output");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "profile_read");
  double tot = 0.0;
  int64_t n = 0;
  for (size_t i = 0; i + 1 < c->prof.used; i += 2) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->prof.ev[i], c->prof.ev[i + 1]), "profile_read");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  if (table_bytes) {
    double by = c->prof.bytes;
    for (size_t i = 0; i < c->prof.slot_bytes.size(); ++i)
      by += (double)c->prof.slots[i] * c->prof.slot_bytes[i];
    *table_bytes = by;
  }
  c->prof.reset();
  return MQCT_OK;
}

mqct_status mqct_cross_sections(mqct_context* c, int32_t mem, int64_t B, int32_t N,
                                const double* P, const double* b, const int32_t* init_level,
                                const int32_t* level_of_channel, int32_t n_levels,
                                double b_max, double* sigma) {
  if (!c) return MQCT_ERR_ARG;
  if (B < 1 || N < 1 || n_levels < 1 || !P || !b || !init_level || !level_of_channel || !sigma)
    return fail(c, MQCT_ERR_ARG, "cross_sections: bad arguments");
  if (mem != MQCT_MEM_HOST && mem != MQCT_MEM_DEVICE)
    return fail(c, MQCT_ERR_ARG, "cross_sections: mem must be host or device");
  if (!(b_max > 0.0)) return fail(c, MQCT_ERR_ARG, "cross_sections: b_max must be > 0");
  for (int n = 0; n < N; ++n)
    if (level_of_channel[n] < 0 || level_of_channel[n] >= n_levels)
      return fail(c, MQCT_ERR_ARG, "cross_sections: level_of_channel out of range");
  if (mem == MQCT_MEM_HOST)
    for (int64_t i = 0; i < B; ++i)
      if (init_level[i] < 0 || init_level[i] >= n_levels)
        return fail(c, MQCT_ERR_ARG, "cross_sections: init_level out of range");
  HIP_TRY(c, hipSetDevice(c->device), "cross_sections");
  mqct_status st;
  const size_t lsz = (size_t)B * n_levels * 8, ssz = (size_t)n_levels * n_levels * 8;
  if ((st = ensure(c, c->xs[0], lsz + N * 4, "cross_sections")) != MQCT_OK) return st;
  double* lsum = (double*)c->xs[0].p;
  int32_t* dlev = (int32_t*)((char*)c->xs[0].p + lsz);
  HIP_TRY(c, hipMemcpyAsync(dlev, level_of_channel, N * 4, hipMemcpyHostToDevice, c->stream),
          "cross_sections");
  const double *dP = P, *db = b;
  const int32_t* dil = init_level;
  double* dsig = sigma;
  if (mem == MQCT_MEM_HOST) {
    if ((st = ensure(c, c->xs[1], (size_t)B * N * 8 + B * 8 + B * 4 + 64, "cross_sections")) != MQCT_OK)
      return st;
    if ((st = ensure(c, c->xs[2], ssz, "cross_sections")) != MQCT_OK) return st;
    char* base = (char*)c->xs[1].p;
    HIP_TRY(c, hipMemcpyAsync(base, P, (size_t)B * N * 8, hipMemcpyHostToDevice, c->stream), "cross_sections");
    HIP_TRY(c, hipMemcpyAsync(base + (size_t)B * N * 8, b, B * 8, hipMemcpyHostToDevice, c->stream), "cross_sections");
    HIP_TRY(c, hipMemcpyAsync(base + (size_t)B * N * 8 + B * 8, init_level, B * 4,
                              hipMemcpyHostToDevice, c->stream), "cross_sections");
    dP = (const double*)base;
    db = (const double*)(base + (size_t)B * N * 8);
    dil = (const int32_t*)(base + (size_t)B * N * 8 + B * 8);
    dsig = (double*)c->xs[2].p;
  }
  HIP_TRY(c, launch_xsec(B, N, dP, db, dil, dlev, n_levels, b_max, lsum, dsig, c->stream),
          "cross_sections");
  if (mem == MQCT_MEM_HOST) {
    HIP_TRY(c, hipMemcpyAsync(sigma, dsig, ssz, hipMemcpyDeviceToHost, c->stream), "cross_sections");
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream), "cross_sections");
  return MQCT_OK;
}

}  // extern "C"

// Host side of the work-list schedule (kernels: queue_kernels.h).
//
// A batch is split into classes of trajectories that share the storage type
// and padded column count of their systems (systems may differ within a
// class).  Each class has its own work list, its own tuned workgroup shape and
// its own step launches.  The host replays chunks of `chunk` step launches
// followed by one compaction (as a HIP graph captured once per grid size and
// shape), reads the active counts back, and shrinks the grid as trajectories
// retire.  Every launch reads the active count from device memory, so the work
// a replay does always matches the list, whatever grid the graph was built with.
//
// Autotuner, two regimes per class (storage type, Npad, method):
//   bulk  the row-split shapes (64..512 threads, fewest rows per lane covering
//         Npad, lanes within a factor two of the rows), timed after the batch's
//         init on a copy of the state of up to TUNE_SAMPLE trajectories;
//   tail  the split-row shapes (4 or 8 waves that each hold all rows and stream
//         a share of the stored rows) and the bulk choice, timed on a copy of
//         TAIL_SAMPLE trajectories -- few enough that each has the device to
//         itself, as in the last trajectories of a batch.  If a split-row shape
//         wins, the class switches to it once its active count drops to twice
//         the number of compute units.
// Each candidate is timed in two passes of two step launches (results are not
// written); the choices are kept for the context.
#include "rhs.h"

#include <algorithm>
#include <map>

namespace mqct {

const QKernelSet* queue_kernels_r64();
const QKernelSet* queue_kernels_c128();
const QKernelSet* queue_kernels_r32();
const QKernelSet* queue_kernels_c64();

const QKernelSet* queue_kernels(int dtype) {
  switch (dtype) {
    case R64: return queue_kernels_r64();
    case C128: return queue_kernels_c128();
    case R32: return queue_kernels_r32();
    case C64: return queue_kernels_c64();
  }
  return nullptr;
}

namespace {

constexpr int64_t TUNE_SAMPLE = 2048;
constexpr int64_t TAIL_SAMPLE = 32;
constexpr size_t LDS_MAX = 160 * 1024;
constexpr int CT = 1024;   // threads of the compaction kernel

// Compaction of the work list: entries whose trajectory is done are dropped and
// the rest are ordered by their current R (buckets of 1/4 bohr, by counting
// sort; the order within a bucket is whatever the atomics give).  Trajectories
// at nearly the same R read the same table slices, so workgroups that run at the
// same time then share them through the caches.  Each trajectory's arithmetic
// does not depend on its position in the list, so the results are the same for
// any order.
constexpr int QBK = 1024;
__device__ __forceinline__ int r_bucket(double R) {
  const double x = R * 4.0;
  return (x >= 0.0 && x < (double)QBK) ? (int)x : (x >= (double)QBK ? QBK - 1 : 0);
}

__global__ void __launch_bounds__(CT) q_compact(int32_t* list, int32_t* tmp, int32_t* count,
                                               const QState* __restrict__ st) {
  __shared__ int32_t cur[QBK];
  __shared__ int32_t kept;
  const int n = *count;
  for (int b = threadIdx.x; b < QBK; b += CT) cur[b] = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < n; p += CT) {
    const int v = list[p];
    if (!(st[v].flags & Q_DONE)) atomicAdd(&cur[r_bucket(st[v].yc[0])], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < QBK; ++b) {
      const int c = cur[b];
      cur[b] = acc;
      acc += c;
    }
    kept = acc;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < n; p += CT) {
    const int v = list[p];
    if (!(st[v].flags & Q_DONE)) tmp[atomicAdd(&cur[r_bucket(st[v].yc[0])], 1)] = v;
  }
  __syncthreads();
  const int k = kept;
  for (int p = threadIdx.x; p < k; p += CT) list[p] = tmp[p];
  if (threadIdx.x == 0) *count = k;
}

// Work list = all sample slots, count = n (used by the autotuner's copies).
__global__ void q_iota(int32_t* list, int32_t* count, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) list[i] = i;
  if (i == 0) *count = n;
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

size_t class_bytes(int64_t n, int npad, int method) {
  size_t s = al((size_t)n * sizeof(QState)) + al((size_t)n * npad * 16) + 2 * al((size_t)n * 4);
  if (method == 1) s += al((size_t)n * 8 * npad * 16);
  return s;
}

QWS carve(char*& p, int64_t n, int npad, int method, const TrajIn* traj) {
  QWS w{};
  w.n = (int32_t)n;
  w.npad = npad;
  w.traj = traj;
  w.st = (QState*)p; p += al((size_t)n * sizeof(QState));
  w.amp = (double2*)p; p += al((size_t)n * npad * 16);
  w.list = (int32_t*)p; p += al((size_t)n * 4);
  w.list2 = (int32_t*)p; p += al((size_t)n * 4);
  if (method == 1) { w.kst = (double2*)p; p += al((size_t)n * 8 * npad * 16); }
  return w;
}

int vec_of(int dtype) { return dtype == C128 ? 1 : 2; }

// The per-trajectory schedule's shape: the smallest workgroup covering the
// row groups with one group per lane, else 512 threads with more per lane.
int default_shape(int dtype, int npad) {
  const int g = npad / vec_of(dtype);
  if (g <= 64) return 0;
  if (g <= 128) return 2;
  if (g <= 256) return 4;
  if (g <= 512) return 7;
  if (g <= 1024) return 8;
  if (g <= 2048) return 9;
  if (g <= 4096) return 10;
  return -1;
}

size_t shape_lds(int dtype, int npad, int shape) {
  return rhs::lds_bytes(npad, dtype_fp32(dtype), queue_kernels(dtype)[shape].split_waves);
}

// Row-split shapes (split = false) or split-row shapes (split = true) with the
// fewest rows per lane covering Npad, lanes within a factor two of the rows.
std::vector<int> candidates(int dtype, int npad, int method, bool split) {
  const QKernelSet* t = queue_kernels(dtype);
  const int g = npad / vec_of(dtype);
  const int need = std::max(g, 64);
  std::vector<int> c;
  for (int k = 0; k < QUEUE_SHAPES; ++k) {
    if (!t[k].step[method] || (t[k].split_waves > 0) != split) continue;
    if (shape_lds(dtype, npad, k) > LDS_MAX) continue;
    const int lanes = (split ? 64 : t[k].block) * t[k].rpt;
    bool minimal = true;   // fewest rows per lane for this workgroup size
    for (int j = 0; j < QUEUE_SHAPES; ++j)
      if (j != k && t[j].step[method] && (t[j].split_waves > 0) == split &&
          t[j].block == t[k].block && t[j].rpt < t[k].rpt &&
          (split ? 64 : t[j].block) * t[j].rpt >= g)
        minimal = false;
    if (lanes >= g && lanes < 2 * need && minimal) c.push_back(k);
  }
  return c;
}

hipError_t launch(const void* fn, int grid, int block, size_t lds, hipStream_t s, QArgs& a) {
  if (grid <= 0) return hipSuccess;
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3((unsigned)grid), dim3((unsigned)block), args, lds, s);
}

hipError_t prepare_fn(const void* fn, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

struct ClassRun {
  QueueClass c;
  QWS ws;
  int shape = -1;        // shape in use
  int tail_shape = -1;   // split-row shape for the tail (-1: none)
  size_t entry = 0;      // its entry in the context's cache
  int count = 0;         // last active count read back
  int grid = 0;          // grid of the current graph / launches
  bool multi = false;    // several attempts per launch (the tail)
  hipGraphExec_t exec = nullptr;
};

}  // namespace

size_t queue_workspace_bytes(const std::vector<QueueClass>& cls, int method) {
  size_t s = al(cls.size() * 4 + 4) + al(8);
  size_t tune = 0;
  for (const auto& c : cls) {
    s += class_bytes(c.n, c.npad, method);
    tune = std::max(tune, class_bytes(std::min(c.n, TUNE_SAMPLE), c.npad, method));
  }
  return s + tune;
}

hipError_t run_queue(const DevSystem* d_systems, const TrajIn* d_traj,
                     const std::vector<QueueClass>& cls, const double* d_a0, TrajOut out,
                     int method, DpCtl ctl, int64_t max_attempts, const QueueOpts& opt,
                     QueueCache& cache, void* wsp, hipStream_t s, hipStream_t cap, int* h_counts,
                     Prof* prof, const std::function<void()>& on_tail) {
  hipError_t e;
  char* p = (char*)wsp;
  int32_t* d_counts = (int32_t*)p;
  p += al(cls.size() * 4 + 4);
  int32_t* d_tcount = (int32_t*)p;
  p += al(8);
  std::vector<ClassRun> runs(cls.size());
  for (size_t k = 0; k < cls.size(); ++k) {
    ClassRun& r = runs[k];
    r.c = cls[k];
    r.ws = carve(p, r.c.n, r.c.npad, method, d_traj + r.c.first);
    r.ws.count = d_counts + k;
  }
  char* tune_area = p;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);

  auto args_for = [&](const QWS& w) {
    QArgs a;
    a.ws = w;
    a.systems = d_systems;
    a.a0_all = d_a0;
    a.ctl = ctl;
    a.max_attempts = max_attempts;
    a.out = out;
    a.per_launch = std::max(1, opt.per_launch);
    return a;
  };
  auto kset = [&](const ClassRun& r, int shape) -> const QKernelSet& {
    return queue_kernels(r.c.dtype)[shape];
  };
  auto lds_of = [&](const ClassRun& r, int shape) { return shape_lds(r.c.dtype, r.c.npad, shape); };

  // shapes: cached decision, else default (and tuned after init)
  std::vector<size_t> to_tune;
  for (size_t k = 0; k < runs.size(); ++k) {
    ClassRun& r = runs[k];
    bool found = false;
    for (size_t q = 0; q < cache.entries.size(); ++q) {
      const QueueTuneEntry& en = cache.entries[q];
      if (en.dtype == r.c.dtype && en.npad == r.c.npad && en.method == method) {
        r.shape = en.shape;
        r.tail_shape = en.tail_shape;
        r.entry = q;
        found = true;
      }
    }
    if (found) continue;
    const std::vector<int> cand = candidates(r.c.dtype, r.c.npad, method, false);
    if (cand.empty()) return hipErrorInvalidValue;
    const int def = default_shape(r.c.dtype, r.c.npad);
    r.shape = std::find(cand.begin(), cand.end(), def) != cand.end() ? def : cand.back();
    QueueTuneEntry en{r.c.dtype, r.c.npad, method, r.shape, false, {}};
    r.entry = cache.entries.size();
    cache.entries.push_back(en);
    if (opt.tune) to_tune.push_back(k);
  }

  auto init_class = [&](ClassRun& r) -> hipError_t {
    const QKernelSet& ks = kset(r, r.shape);
    QArgs a = args_for(r.ws);
    hipError_t err = prepare_fn(ks.init[method], lds_of(r, r.shape));
    if (err != hipSuccess) return err;
    r.count = (int)r.c.n;
    r.grid = (int)r.c.n;
    return launch(ks.init[method], (int)r.c.n, ks.block, lds_of(r, r.shape), s, a);
  };
  // classes to be tuned start with the default shape, so the candidates are
  // timed on real states
  std::vector<int> init_shape(runs.size(), -1);
  for (size_t k : to_tune) {
    if ((e = init_class(runs[k])) != hipSuccess) return e;
    init_shape[k] = runs[k].shape;
  }

  // time candidate shapes on a copy of the first S trajectories' states
  auto time_shapes = [&](const ClassRun& r, int64_t S, const std::vector<int>& cand,
                         std::vector<double>& best) -> hipError_t {
    char* q = tune_area;
    QWS tw = carve(q, S, r.c.npad, method, r.ws.traj);
    tw.count = d_tcount;
    QArgs a = args_for(tw);
    a.out = TrajOut{};
    best.assign(cand.size(), 1e300);
    hipEvent_t e0, e1;
    hipError_t err;
    if ((err = hipEventCreate(&e0)) != hipSuccess) return err;
    if ((err = hipEventCreate(&e1)) != hipSuccess) { hipEventDestroy(e0); return err; }
    for (int pass = 0; pass < 2 && err == hipSuccess; ++pass) {
      for (size_t ci = 0; ci < cand.size() && err == hipSuccess; ++ci) {
        const QKernelSet& ks = kset(r, cand[ci]);
        const size_t lds = lds_of(r, cand[ci]);
        if ((err = hipMemcpyAsync(tw.st, r.ws.st, (size_t)S * sizeof(QState), hipMemcpyDeviceToDevice, s)) != hipSuccess) break;
        if ((err = hipMemcpyAsync(tw.amp, r.ws.amp, (size_t)S * r.c.npad * 16, hipMemcpyDeviceToDevice, s)) != hipSuccess) break;
        if (method == 1 &&
            (err = hipMemcpyAsync(tw.kst, r.ws.kst, (size_t)S * 8 * r.c.npad * 16, hipMemcpyDeviceToDevice, s)) != hipSuccess)
          break;
        q_iota<<<(unsigned)((S + 255) / 256), 256, 0, s>>>(tw.list, tw.count, (int)S);
        if ((err = prepare_fn(ks.step[method], lds)) != hipSuccess) break;
        if ((err = hipEventRecord(e0, s)) != hipSuccess) break;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep)
          err = launch(ks.step[method], (int)S, ks.block, lds, s, a);
        if (err != hipSuccess) break;
        if ((err = hipEventRecord(e1, s)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (pass == 1) best[ci] = ms / 2.0;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return err;
  };
  for (size_t k : to_tune) {
    ClassRun& r = runs[k];
    QueueTuneEntry& en = cache.entries[r.entry];
    const std::vector<int> cand = candidates(r.c.dtype, r.c.npad, method, false);
    std::vector<double> best;
    if (cand.size() > 1) {
      if ((e = time_shapes(r, std::min(r.c.n, TUNE_SAMPLE), cand, best)) != hipSuccess) return e;
      size_t bi = 0;
      for (size_t ci = 1; ci < cand.size(); ++ci)
        if (best[ci] < best[bi]) bi = ci;
      r.shape = cand[bi];
      en.shape = r.shape;
      en.tuned = true;
      for (size_t ci = 0; ci < cand.size(); ++ci) en.ms.push_back({cand[ci], best[ci]});
    }
    std::vector<int> tc = candidates(r.c.dtype, r.c.npad, method, true);
    if (!tc.empty()) {
      tc.push_back(r.shape);
      if ((e = time_shapes(r, std::min(r.c.n, TAIL_SAMPLE), tc, best)) != hipSuccess) return e;
      size_t bi = 0;
      for (size_t ci = 1; ci < tc.size(); ++ci)
        if (best[ci] < best[bi]) bi = ci;
      r.tail_shape = tc[bi] == r.shape ? -1 : tc[bi];
      en.tail_shape = r.tail_shape;
      for (size_t ci = 0; ci < tc.size(); ++ci) en.tail_ms.push_back({tc[ci], best[ci]});
    }
  }
  // forced split-row form (tests): the widest split-row candidate throughout
  if (opt.tail == 2)
    for (ClassRun& r : runs) {
      const std::vector<int> tc = candidates(r.c.dtype, r.c.npad, method, true);
      r.tail_shape = tc.empty() ? -1 : tc.back();
    }
  // every class starts from an init with its first shape
  for (size_t k = 0; k < runs.size(); ++k)
    if (init_shape[k] != runs[k].shape)
      if ((e = init_class(runs[k])) != hipSuccess) return e;

  // step chunks until every work list is empty
  const int chunk = std::max(1, opt.chunk);
  const int64_t max_rounds = (max_attempts + chunk - 1) / chunk + 2;
  auto enqueue_chunk = [&](ClassRun& r, hipStream_t st) -> hipError_t {
    const QKernelSet& ks = kset(r, r.shape);
    const size_t lds = lds_of(r, r.shape);
    QArgs a = args_for(r.ws);
    hipError_t err;
    const void* fn = r.multi ? ks.step_multi[method] : ks.step[method];
    for (int j = 0; j < chunk; ++j)
      if ((err = launch(fn, r.grid, ks.block, lds, st, a)) != hipSuccess) return err;
    q_compact<<<1, CT, 0, st>>>(r.ws.list, r.ws.list2, r.ws.count, r.ws.st);
    return hipGetLastError();
  };
  auto drop_graph = [](ClassRun& r) {
    if (r.exec) (void)hipGraphExecDestroy(r.exec);
    r.exec = nullptr;
  };
  for (ClassRun& r : runs) {
    if ((e = prepare_fn(kset(r, r.shape).step[method], lds_of(r, r.shape))) != hipSuccess) return e;
    if ((e = prepare_fn(kset(r, r.shape).step_multi[method], lds_of(r, r.shape))) != hipSuccess)
      return e;
    if (r.tail_shape >= 0 &&
        ((e = prepare_fn(kset(r, r.tail_shape).step[method], lds_of(r, r.tail_shape))) != hipSuccess ||
         (e = prepare_fn(kset(r, r.tail_shape).step_multi[method], lds_of(r, r.tail_shape))) !=
             hipSuccess))
      return e;
  }
  e = hipSuccess;
  bool tail_called = false;
  int64_t round = 0;
  for (; round < max_rounds; ++round) {
    bool any = false;
    for (ClassRun& r : runs) {
      if (r.count <= 0) continue;
      any = true;
      // few trajectories left: the latency shape, if the tuner found one
      if (opt.tail && r.tail_shape >= 0 && r.shape != r.tail_shape &&
          (r.count <= 2 * cus || opt.tail == 2)) {
        r.shape = r.tail_shape;
        drop_graph(r);
      }
      // few trajectories left: several attempts per launch
      if (opt.per_launch > 1 && !r.multi && r.count <= 2 * cus) {
        r.multi = true;
        drop_graph(r);
      }
      // shrink the grid once fewer than half of its workgroups have work
      if (r.count * 2 <= r.grid) {
        r.grid = r.count;
        drop_graph(r);
      }
      hipEvent_t ea = prof ? prof->next() : nullptr, eb = prof ? prof->next() : nullptr;
      prof_mark(prof, ea, s);
      if (opt.graphs) {
        if (!r.exec) {
          hipGraph_t g = nullptr;
          if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) break;
          hipError_t ec = enqueue_chunk(r, cap);
          hipError_t ee = hipStreamEndCapture(cap, &g);
          if (ec != hipSuccess || ee != hipSuccess) {
            if (g) hipGraphDestroy(g);
            e = ec != hipSuccess ? ec : ee;
            break;
          }
          e = hipGraphInstantiate(&r.exec, g, nullptr, nullptr, 0);
          hipGraphDestroy(g);
          if (e != hipSuccess) { r.exec = nullptr; break; }
        }
        if ((e = hipGraphLaunch(r.exec, s)) != hipSuccess) break;
      } else {
        if ((e = enqueue_chunk(r, s)) != hipSuccess) break;
      }
      prof_mark(prof, eb, s);
    }
    if (e != hipSuccess || !any) break;
    if ((e = hipMemcpyAsync(h_counts, d_counts, runs.size() * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
      break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    int64_t active = 0;
    for (size_t k = 0; k < runs.size(); ++k) {
      runs[k].count = h_counts[k];
      active += std::max(runs[k].count, 0);
    }
    if (on_tail && !tail_called && active <= 2 * (int64_t)cus) {
      on_tail();
      tail_called = true;
    }
  }
  for (ClassRun& r : runs) drop_graph(r);
  if (on_tail && !tail_called && e == hipSuccess) on_tail();
  if (e != hipSuccess) return e;
  for (const ClassRun& r : runs)
    if (r.count > 0) return hipErrorLaunchTimeOut;   // attempt bound exceeded (cannot happen)
  return hipSuccess;
}

}  // namespace mqct

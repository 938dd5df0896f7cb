// Launch-shape autotuner and the batched driver of libqkrylov.
//
// The autotuner times one Krylov step of a workspace for a small set of launch
// shapes (threads per block and blocks per CU of the row-streaming kernels,
// work-groups per CU of the blocked H-pass) with HIP events on the caller's
// stream, keeps the fastest, and caches it in a JSON file keyed by the
// problem shape.
//
// The batched driver advances several workspaces (different chain lengths,
// different numbers of field sets) together: one step of all of them is
// captured once into a hipGraph -- one branch per workspace, forked from and
// joined back into the caller's stream -- and replayed for every step, with
// the survival probability of every batch item recorded on the device at a
// device-side step counter.  No host round trip and one graph launch per step.
//
// Items start from a basis state (probability |psi[r0]|^2) or from any state
// (r0 < 0: the driver keeps a copy psi0 of the vector given at creation and
// records |<psi0, psi>|^2).  Every step also advances the temporal
// autocorrelation C(t) = (1/t) integral_0^t P(t') dt' of Sec. 4 by the
// trapezoid rule on the step grid, from the creation of the batch on.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "qk_persist.h"
#include "qk_step_bodies.h"

namespace qk {

// ----------------------------------------------------------------- kernels
template <typename T>
__global__ void k_record(const typename Cx<T>::V* __restrict__ psi, uint32_t r0, int B, double* __restrict__ P,
                         const int* __restrict__ counter, int off, int items) {
  record_body<T>(psi, r0, B, P, counter, off, items);
}

__global__ void k_counter(int* counter, int reset) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = reset ? 0 : *counter + 1;
}

// Trapezoid step of the autocorrelation integral (autocorr_body), one block.
__global__ void __launch_bounds__(256)
k_autocorr(const double* __restrict__ P, const int* __restrict__ counter, int items, double dt, double* state,
           double* C) {
  autocorr_body(P, counter, items, dt, state, C);
}

// Deterministic pseudo-random complex entries (an integer hash of the index),
// used as the start vector of timing runs.
template <typename T>
__global__ void k_fill_hash(typename Cx<T>::V* __restrict__ v, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)(i * 2654435761u) ^ 0x9e3779b9u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  const T re = (T)((double)(h & 0xffffu) / 65536.0 - 0.5);
  const T im = (T)((double)(h >> 16) / 65536.0 - 0.5);
  v[i].x = re;
  v[i].y = im;
}

static qk_status launch_record(const qk_krylov* k, const void* psi, int64_t r0, double* P, const int* counter, int off,
                               int items, hipStream_t s) {
  if (k->dtype == QK_C128)
    hipLaunchKernelGGL(k_record<double>, dim3(1), dim3(64), 0, s, (const double2*)psi, (uint32_t)r0, k->batch, P,
                       counter, off, items);
  else
    hipLaunchKernelGGL(k_record<float>, dim3(1), dim3(64), 0, s, (const float2*)psi, (uint32_t)r0, k->batch, P,
                       counter, off, items);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

// ------------------------------------------------------------- autotuner
std::string shape_key(const qk_krylov* k) {
  const qk_ham* H = k->H;
  char buf[256];
  snprintf(buf, sizeof buf, "L%d_N%d_pbc%d_B%d_mode%d_dtype%d_m%d_reorth%d_cus%d", H->basis->L, H->basis->N,
           H->p.pbc, k->batch, H->p.mode, k->dtype, k->m, k->reorth, qk_num_cus());
  return buf;
}

// One entry per line: "key": {"threads": T, "blocks_per_cu": C, "blocked_wgs_per_cu": W, "ms_per_step": X}
static std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;
    const size_t q1 = line.find('"', q0 + 1);
    const size_t b0 = line.find('{', q1);
    const size_t b1 = line.find('}', b0);
    if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) continue;
    m[line.substr(q0 + 1, q1 - q0 - 1)] = line.substr(b0, b1 - b0 + 1);
  }
  return m;
}

static bool parse_shape(const std::string& obj, qk_launch_shape* sh) {
  auto field = [&](const char* name, int* out) {
    const size_t p = obj.find(name);
    if (p == std::string::npos) return false;
    const size_t c = obj.find(':', p);
    if (c == std::string::npos) return false;
    *out = atoi(obj.c_str() + c + 1);
    return true;
  };
  sh->blocked_llo = 0;
  if (!field("\"blocked_llo\"", &sh->blocked_llo)) sh->blocked_llo = 0;   // absent in older caches: keep
  return field("\"threads\"", &sh->threads) && field("\"blocks_per_cu\"", &sh->blocks_per_cu) &&
         field("\"blocked_wgs_per_cu\"", &sh->blocked_wgs_per_cu);
}

static bool write_cache(const char* path, const std::map<std::string, std::string>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

qk_status apply_shape(qk_krylov* k, const qk_launch_shape* sh) {
  const int B = k->batch;
  if (sh->threads < 0 || sh->blocks_per_cu < 0 || sh->blocked_wgs_per_cu < 0) {
    set_error("launch shape fields must be >= 0");
    return QK_EINVAL;
  }
  if (sh->threads > 0 && (sh->threads < B || sh->threads > kMaxBlock)) {
    set_error("threads must be 0 or in [batch, 256]");
    return QK_EINVAL;
  }
  if (sh->blocks_per_cu > 64 || sh->blocked_wgs_per_cu > 64) {
    set_error("per-CU counts must be <= 64");
    return QK_EINVAL;
  }
  if (sh->blocked_llo < 0) {
    set_error("blocked_llo must be >= 0");
    return QK_EINVAL;
  }
  if (sh->blocked_llo > 0 && sh->blocked_llo != k->H->llo) {
    if (k->H->llo <= 0) {
      set_error("this Hamiltonian has no block decomposition");
      return QK_EUNSUPPORTED;
    }
    // the decomposition belongs to the Hamiltonian, which the workspace shares
    const qk_status st = blocked_rebuild(const_cast<qk_ham*>(k->H), sh->blocked_llo);
    if (st != QK_OK) return st;
  }
  k->threads = sh->threads;
  k->blocks_per_cu = sh->blocks_per_cu;
  k->blocked_wgs = sh->blocked_wgs_per_cu;
  k->grid = stream_grid((uint64_t)k->D, B, krylov_threads(k), k->blocks_per_cu);
  return QK_OK;
}

static qk_status time_step(qk_krylov* k, void* v, uint64_t n, double dt, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                           float* ms) {
  const int reps = 2;
  auto fill = [&]() -> qk_status {
    if (k->dtype == QK_C128)
      hipLaunchKernelGGL(k_fill_hash<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (double2*)v, n);
    else
      hipLaunchKernelGGL(k_fill_hash<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (float2*)v, n);
    QK_HIP(hipGetLastError());
    return QK_OK;
  };
  qk_status st = fill();
  if (st == QK_OK) st = launch_krylov_step(k, v, dt, s);   // warm-up
  if (st == QK_OK) st = fill();
  if (st != QK_OK) return st;
  QK_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps && st == QK_OK; ++r) st = launch_krylov_step(k, v, dt, s);
  if (st != QK_OK) return st;
  QK_HIP(hipEventRecord(e1, s));
  QK_HIP(hipEventSynchronize(e1));
  QK_HIP(hipEventElapsedTime(ms, e0, e1));
  *ms /= reps;
  return QK_OK;
}

qk_status krylov_autotune(qk_krylov* k, double dt, const char* cache_path, hipStream_t s, qk_launch_shape* chosen) {
  const std::string key = shape_key(k);
  if (cache_path && *cache_path) {
    const auto m = read_cache(cache_path);
    const auto it = m.find(key);
    qk_launch_shape sh{};
    if (it != m.end() && parse_shape(it->second, &sh)) {
      qk_status st = apply_shape(k, &sh);
      if (st == QK_OK && chosen) *chosen = sh;
      if (st == QK_OK) return st;
    }
  }
  const uint64_t n = (uint64_t)k->D * k->batch;
  const size_t bytes = n * (k->dtype == QK_C128 ? 16 : 8);
  void* v = nullptr;
  QK_HIP(dev_alloc(k->al, &v, bytes));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  const bool prof = k->profiling;
  k->profiling = false;
  qk_status st = he == hipSuccess ? QK_OK : hip_fail(he, "qk_krylov_autotune events");
  qk_launch_shape best{}, cur{};
  float best_ms = 1e30f;
  auto trial = [&](const qk_launch_shape& sh) {
    if (st != QK_OK) return;
    if (apply_shape(k, &sh) != QK_OK) return;   // invalid for this batch size: skip
    float ms = 0.f;
    st = time_step(k, v, n, dt, s, e0, e1, &ms);
    if (st == QK_OK && ms < best_ms) {
      best_ms = ms;
      best = sh;
    }
  };
  const bool blocked = blocked_usable(k->H, k->dtype);
  const int llo0 = k->H->llo;
  // coordinate search: the low-bit count of the block decomposition with the
  // work-groups of the blocked H-pass first, then the shape of the
  // row-streaming kernels
  if (blocked) {
    for (int llo = llo0 - 2; llo <= llo0 + 1; ++llo) {
      if (!blocked_llo_valid(k->H, llo)) continue;
      for (int w : {2, 4, 6, 8}) {
        cur = qk_launch_shape{0, 0, w, llo};
        trial(cur);
      }
    }
  } else {
    trial(qk_launch_shape{0, 0, 0, 0});
  }
  const int wbest = best.blocked_wgs_per_cu, lbest = best.blocked_llo;
  for (int t : {64, 128, 256})
    for (int c : {4, 8, 16}) {
      if (t < k->batch) continue;
      cur = qk_launch_shape{t, c, wbest, lbest};
      trial(cur);
    }
  k->profiling = prof;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dev_free(k->al, v);
  if (st != QK_OK) return st;
  st = apply_shape(k, &best);
  if (st != QK_OK) return st;
  if (chosen) *chosen = best;
  if (cache_path && *cache_path) {
    auto m = read_cache(cache_path);
    char obj[256];
    snprintf(obj, sizeof obj,
             "{\"threads\": %d, \"blocks_per_cu\": %d, \"blocked_wgs_per_cu\": %d, \"blocked_llo\": %d, "
             "\"ms_per_step\": %.4f}",
             best.threads, best.blocks_per_cu, best.blocked_wgs_per_cu, best.blocked_llo, best_ms);
    m[key] = obj;
    if (!write_cache(cache_path, m)) {
      set_error(std::string("could not write the tuning cache ") + cache_path);
      return QK_EINVAL;
    }
  }
  return QK_OK;
}

}  // namespace qk

// ------------------------------------------------------------ batched driver
struct qk_batch {
  qk_allocator al;
  std::vector<qk_krylov*> ks;
  std::vector<void*> psi;
  std::vector<int64_t> r0;
  std::vector<void*> psi0;          // copy of the initial vector of items with r0 < 0 (else NULL)
  std::vector<double*> part;        // overlap partial sums of those items
  std::vector<int> ogrid;           // their overlap grid
  double* d_state = nullptr;        // autocorrelation state: S[items], P_prev[items], t
  std::vector<int> item_off;
  int items = 0;
  int device = 0;
  int* d_counter = nullptr;
  std::vector<hipStream_t> streams;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  hipStream_t cap = nullptr;        // capture stream (the caller's may be the legacy NULL stream)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_dt = NAN;
  double* graph_P = nullptr;
  double* graph_C = nullptr;
  std::vector<uint64_t> graph_sig;  // launch configuration the graph was captured with
  int graph_mode = 0;               // 1: one branch per workspace, 2: the persistent step kernel
  qk::PersistPlan* plan = nullptr;  // work queue of the persistent step (mode 2)
  std::vector<uint64_t> plan_sig;
};

namespace qk {

int batch_items(const qk_batch* b) { return b->items; }

// Survival probability of workspace i's items at the current step counter:
// P[(*counter) * items + offset + b].
static qk_status record_item(qk_batch* b, int i, double* P, hipStream_t s) {
  const qk_krylov* k = b->ks[i];
  if (b->r0[i] >= 0)
    return launch_record(k, b->psi[i], b->r0[i], P, b->d_counter, b->item_off[i], b->items, s);
  return launch_overlap_record(b->psi0[i], b->psi[i], k->dtype, (uint32_t)k->D, k->batch, b->part[i], b->ogrid[i], P,
                               b->d_counter, b->item_off[i], b->items, s);
}
int batch_device(const qk_batch* b) { return b->device; }

void batch_release(qk_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static void batch_release_plan(qk_batch* b) {
  if (b->plan) {
    (void)hipDeviceSynchronize();   // no queued launch may still read the plan
    persist_free(b->plan);
  }
  b->plan = nullptr;
  b->plan_sig.clear();
}

qk_status batch_create(qk_krylov* const* ks, void* const* psi, const int64_t* r0, int n, qk_batch** out) {
  qk_batch* b = new (std::nothrow) qk_batch;
  if (!b) return QK_ENOMEM;
  b->device = ks[0]->device;
  int off = 0;
  for (int i = 0; i < n; ++i) {
    b->ks.push_back(ks[i]);
    b->psi.push_back(psi[i]);
    b->r0.push_back(r0[i]);
    b->item_off.push_back(off);
    off += ks[i]->batch;
  }
  b->items = off;
  b->al = current_allocator();
  hipError_t e = dev_alloc(b->al, (void**)&b->d_counter, sizeof(int));
  if (e == hipSuccess) e = dev_alloc(b->al, (void**)&b->d_state, sizeof(double) * (2 * (size_t)off + 1));
  for (int i = 0; i < n; ++i) {
    void* p0 = nullptr;
    double* pa = nullptr;
    int G = 0;
    if (e == hipSuccess && r0[i] < 0) {
      const size_t vec = (ks[i]->dtype == QK_C128 ? 16 : 8) * (size_t)ks[i]->D * ks[i]->batch;
      G = overlap_grid((uint32_t)ks[i]->D, ks[i]->batch);
      e = dev_alloc(b->al, &p0, vec);
      if (e == hipSuccess) e = dev_alloc(b->al, (void**)&pa, sizeof(double) * (size_t)G * 2 * ks[i]->batch);
      if (e == hipSuccess) e = hipMemcpy(p0, psi[i], vec, hipMemcpyDeviceToDevice);
    }
    b->psi0.push_back(p0);
    b->part.push_back(pa);
    b->ogrid.push_back(G);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);   // default priority
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);   // default priority
    if (e == hipSuccess) b->streams.push_back(st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->joins.push_back(ev);
  }
  if (e != hipSuccess) {
    qk_status st = hip_fail(e, "qk_batch_create");
    batch_destroy(b);
    return st;
  }
  // autocorrelation state: S = 0, t = 0, P_prev = P of the vectors as given
  qk_status st = QK_OK;
  e = hipMemset(b->d_state, 0, sizeof(double) * (2 * (size_t)off + 1));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, nullptr, b->d_counter, 1);
    e = hipGetLastError();
  }
  for (int i = 0; i < n && e == hipSuccess && st == QK_OK; ++i)
    st = record_item(b, i, b->d_state + off, nullptr);
  if (e == hipSuccess && st == QK_OK) e = hipDeviceSynchronize();
  if (e != hipSuccess || st != QK_OK) {
    if (st == QK_OK) st = hip_fail(e, "qk_batch_create");
    batch_destroy(b);
    return st;
  }
  *out = b;
  return QK_OK;
}

void batch_destroy(qk_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  batch_release(b);
  batch_release_plan(b);
  for (auto s : b->streams) (void)hipStreamDestroy(s);
  for (auto e : b->joins) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  dev_free(b->al, b->d_counter);
  dev_free(b->al, b->d_state);
  for (auto p : b->psi0) dev_free(b->al, p);
  for (auto p : b->part) dev_free(b->al, p);
  delete b;
}

// One step of every workspace, each on its own stream forked from `s` and
// joined back, then the autocorrelation advances and the step counter moves on.
static qk_status batch_step(qk_batch* b, double dt, double* P, double* C, hipStream_t s) {
  QK_HIP(hipEventRecord(b->fork, s));
  for (size_t i = 0; i < b->ks.size(); ++i) {
    hipStream_t si = b->streams[i];
    QK_HIP(hipStreamWaitEvent(si, b->fork, 0));
    qk_status st = launch_krylov_step(b->ks[i], b->psi[i], dt, si);
    if (st != QK_OK) return st;
    st = record_item(b, (int)i, P, si);
    if (st != QK_OK) return st;
    QK_HIP(hipEventRecord(b->joins[i], si));
    QK_HIP(hipStreamWaitEvent(s, b->joins[i], 0));
  }
  hipLaunchKernelGGL(k_autocorr, dim3(1), dim3(256), 0, s, P, b->d_counter, b->items, dt, b->d_state, C);
  QK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, b->d_counter, 0);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

// What a captured step depends on besides dt and the output arrays: each
// workspace's launch shape and its Hamiltonian's table generation (a rebuilt
// block decomposition frees the tables the old graph points to).
static std::vector<uint64_t> batch_signature(const qk_batch* b) {
  std::vector<uint64_t> sig;
  for (const qk_krylov* k : b->ks) {
    sig.push_back(k->H->tables_gen);
    sig.push_back((uint64_t)k->H->llo);
    sig.push_back((uint64_t)k->threads);
    sig.push_back((uint64_t)k->blocks_per_cu);
    sig.push_back((uint64_t)k->blocked_wgs);
    sig.push_back((uint64_t)k->grid);
  }
  return sig;
}

// The persistent step's work queue for the current launch shapes (rebuilt
// when a workspace's shape or block decomposition has changed).
static qk_status batch_plan(qk_batch* b, const std::vector<uint64_t>& sig) {
  if (b->plan && b->plan_sig == sig) return QK_OK;
  batch_release(b);   // a captured graph may point at the old plan
  batch_release_plan(b);
  PersistInput in;
  in.al = b->al;
  in.ks = b->ks;
  in.psi = b->psi;
  in.r0 = b->r0;
  for (void* p : b->psi0) in.psi0.push_back(p);
  in.part = b->part;
  in.ogrid = b->ogrid;
  in.item_off = b->item_off;
  qk_status st = persist_plan(in, &b->plan);
  if (st != QK_OK) {
    b->plan = nullptr;
    return st;
  }
  b->plan_sig = sig;
  return QK_OK;
}

qk_status batch_run(qk_batch* b, double dt, int n_steps, int use_graph, double* P, double* C, hipStream_t s) {
  std::vector<bool> prof(b->ks.size());
  for (size_t i = 0; i < b->ks.size(); ++i) {
    prof[i] = b->ks[i]->profiling;
    b->ks[i]->profiling = false;
  }
  auto restore = [&]() {
    for (size_t i = 0; i < b->ks.size(); ++i) b->ks[i]->profiling = prof[i];
  };
  hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, b->d_counter, 1);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) {
    restore();
    return hip_fail(le, "qk_batch_run counter reset");
  }
  qk_status st = QK_OK;
  if (!use_graph) {
    for (int k = 0; k < n_steps && st == QK_OK; ++k) st = batch_step(b, dt, P, C, s);
    restore();
    return st;
  }
  const std::vector<uint64_t> sig = batch_signature(b);
  if (use_graph == 2) {
    st = batch_plan(b, sig);
    if (st != QK_OK) {
      restore();
      return st;
    }
  }
  if (!b->exec || b->graph_mode != use_graph || b->graph_dt != dt || b->graph_P != P || b->graph_C != C ||
      b->graph_sig != sig) {
    batch_release(b);
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      restore();
      return hip_fail(e, "hipStreamBeginCapture");
    }
    if (use_graph == 2)
      st = persist_launch(b->plan, dt, P, C, b->d_counter, b->d_state, b->items, b->cap);
    else
      st = batch_step(b, dt, P, C, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (st != QK_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      restore();
      return st != QK_OK ? st : hip_fail(e, "hipStreamEndCapture");
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      batch_release(b);
      restore();
      return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph_mode = use_graph;
    b->graph_dt = dt;
    b->graph_P = P;
    b->graph_C = C;
    b->graph_sig = sig;
  }
  for (int k = 0; k < n_steps; ++k) {
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) {
      restore();
      return hip_fail(e, "hipGraphLaunch");
    }
  }
  restore();
  return QK_OK;
}

}  // namespace qk

// C ABI of libqkrylov: argument validation, handle management and error
// reporting around the launchers in qk_kernels.hip.  Every entry point
// validates its arguments before touching the device and converts HIP
// failures into QK_EHIP with the runtime's message in qk_last_error().
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qk_device.h"

namespace qk {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

qk_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? QK_ENOMEM : QK_EHIP;
}

// ---------------------------------------------------------- device memory
static std::mutex g_alloc_mu;
static qk_allocator g_alloc;

qk_allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

hipError_t dev_alloc(const qk_allocator& a, void** p, size_t bytes) {
  if (!a.alloc) return hipMalloc(p, bytes);
  *p = a.alloc(bytes, nullptr, a.ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(const qk_allocator& a, void* p) {
  if (!p) return;
  if (a.release) a.release(p, nullptr, a.ctx);
  else (void)hipFree(p);
}

hipError_t dev_alloc_async(const qk_allocator& a, void** p, size_t bytes, hipStream_t s) {
  if (!a.alloc) return hipMallocAsync(p, bytes, s);
  *p = a.alloc(bytes, (void*)s, a.ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t dev_free_async(const qk_allocator& a, void* p, hipStream_t s) {
  if (!p) return hipSuccess;
  if (!a.release) return hipFreeAsync(p, s);
  // a NULL stream tells the callback that no queued work uses the block
  hipError_t e = s ? hipSuccess : hipStreamSynchronize(s);
  a.release(p, (void*)s, a.ctx);
  return e;
}

static qk_status inval(const std::string& msg) {
  g_err = msg;
  return QK_EINVAL;
}

static qk_status check_device(int dev) {
  int cur = -1;
  QK_HIP(hipGetDevice(&cur));
  if (cur != dev) return inval("handle belongs to another device");
  return QK_OK;
}

static size_t elem_bytes(int dtype) { return dtype == QK_C128 ? 16 : 8; }

// [a, a + na) and [b, b + nb) intersect
static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

int krylov_grid(uint64_t D, int B);

// psi (n bytes) intersects the workspace's own vectors (the basis slots, z)
static bool workspace_overlap(const qk_krylov* k, const void* psi, size_t n) {
  const size_t slot = elem_bytes(k->dtype) * (size_t)k->ustride;
  if (ranges_overlap(psi, n, k->d_U, slot * (size_t)k->m)) return true;
  return k->d_Z && ranges_overlap(psi, n, k->d_Z, slot);
}

}  // namespace qk

using namespace qk;

#define QK_API extern "C" __attribute__((visibility("default")))

QK_API int qk_abi_version(void) { return QK_ABI_VERSION; }

QK_API const char* qk_last_error(void) { return g_err.c_str(); }

QK_API qk_status qk_set_allocator(qk_alloc_fn alloc, qk_release_fn release, void* ctx) {
  g_err.clear();
  if ((alloc == nullptr) != (release == nullptr)) return inval("alloc and release must both be set or both be NULL");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.release = release;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return QK_OK;
}

QK_API qk_status qk_fields_quasiperiodic(int32_t L, double h, double beta, const double* phi, int32_t batch,
                                         double* h_out) {
  g_err.clear();
  if (L < 1 || L > QK_MAX_L) return inval("L out of range");
  if (batch < 1) return inval("batch < 1");
  if (!phi || !h_out) return inval("NULL pointer");
  if (!std::isfinite(h) || !std::isfinite(beta)) return inval("non-finite h or beta");
  for (int b = 0; b < batch; ++b) {
    if (!std::isfinite(phi[b])) return inval("non-finite phase");
    for (int i = 1; i <= L; ++i) h_out[(size_t)b * L + (i - 1)] = h * std::cos(2.0 * M_PI * beta * i + phi[b]);
  }
  return QK_OK;
}

// ------------------------------------------------------------------- basis
static int64_t binom64(int n, int k) {
  if (k < 0 || k > n) return 0;
  unsigned __int128 r = 1;
  for (int i = 1; i <= k; ++i) r = r * (unsigned)(n - k + i) / (unsigned)i;   // exact at every step
  return r > (unsigned __int128)INT64_MAX ? INT64_MAX : (int64_t)r;
}

QK_API qk_status qk_basis_build(int32_t L, int32_t n_up, void* stream, qk_basis** out) {
  g_err.clear();
  if (!out) return inval("NULL out");
  *out = nullptr;
  if (L < 2 || L > QK_MAX_L) return inval("L must be in [2, 64]");
  if (n_up <= 0 || n_up >= L) return inval("n_up must be in (0, L)");
  if (binom64(L, n_up) >= (int64_t)0xffffffffll) {
    set_error("sector dimension C(L, n_up) must be below 2^32 - 1");
    return QK_EUNSUPPORTED;
  }
  qk_basis* b = new (std::nothrow) qk_basis;
  if (!b) return QK_ENOMEM;
  b->L = L;
  b->N = n_up;
  b->D = binom64(L, n_up);
  b->wide = L > 32;
  const int K = binom_stride(b);
  const size_t sbytes = b->wide ? sizeof(uint64_t) : sizeof(uint32_t);
  b->al = current_allocator();
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = dev_alloc(b->al, (void**)&b->d_binom, sizeof(uint32_t) * K * K);
  if (e == hipSuccess) e = dev_alloc(b->al, (void**)&b->d_states, sbytes * (size_t)b->D);
  if (e != hipSuccess) {
    qk_status st = hip_fail(e, "qk_basis_build allocation");
    qk_basis_destroy(b);
    return st;
  }
  qk_status st = launch_basis_build(b, (hipStream_t)stream);
  // the handle is complete on return, so calls on any stream (and the
  // stream-less qk_basis_rank) may use its tables at once
  if (st == QK_OK) {
    const hipError_t se = hipStreamSynchronize((hipStream_t)stream);
    if (se != hipSuccess) st = hip_fail(se, "qk_basis_build");
  }
  if (st != QK_OK) {
    qk_basis_destroy(b);
    return st;
  }
  *out = b;
  return QK_OK;
}

QK_API qk_status qk_basis_dim(const qk_basis* b, int64_t* D) {
  g_err.clear();
  if (!b || !D) return inval("NULL pointer");
  *D = b->D;
  return QK_OK;
}

QK_API qk_status qk_basis_shape(const qk_basis* b, int32_t* L, int32_t* n_up) {
  g_err.clear();
  if (!b || !L || !n_up) return inval("NULL pointer");
  *L = b->L;
  *n_up = b->N;
  return QK_OK;
}

QK_API qk_status qk_basis_states(const qk_basis* b, void* dst, void* stream) {
  g_err.clear();
  if (!b || !dst) return inval("NULL pointer");
  qk_status st = check_device(b->device);
  if (st != QK_OK) return st;
  const size_t sbytes = b->wide ? sizeof(uint64_t) : sizeof(uint32_t);
  QK_HIP(hipMemcpyAsync(dst, b->d_states, sbytes * (size_t)b->D, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return QK_OK;
}

QK_API qk_status qk_basis_rank(const qk_basis* b, const uint64_t* states_host, int64_t n, int64_t* idx_host) {
  g_err.clear();
  if (!b) return inval("NULL basis");
  if (n < 0) return inval("n < 0");
  if (n == 0) return QK_OK;
  if (!states_host || !idx_host) return inval("NULL pointer");
  qk_status st = check_device(b->device);
  if (st != QK_OK) return st;
  uint64_t* d_in = nullptr;
  int64_t* d_out = nullptr;
  hipError_t e = dev_alloc(b->al, (void**)&d_in, sizeof(uint64_t) * (size_t)n);
  if (e == hipSuccess) e = dev_alloc(b->al, (void**)&d_out, sizeof(int64_t) * (size_t)n);
  if (e == hipSuccess) e = hipMemcpy(d_in, states_host, sizeof(uint64_t) * (size_t)n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    st = launch_rank(b, d_in, n, d_out, nullptr);
    if (st == QK_OK) e = hipMemcpy(idx_host, d_out, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost);
  }
  dev_free(b->al, d_in);
  dev_free(b->al, d_out);
  if (e != hipSuccess) return hip_fail(e, "qk_basis_rank");
  return st;
}

QK_API void qk_basis_destroy(qk_basis* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  dev_free(b->al, b->d_states);
  dev_free(b->al, b->d_binom);
  delete b;
}

// ------------------------------------------------------------- Hamiltonian
static qk_status check_fields(const double* h, int32_t L, int32_t batch) {
  if (!h) return inval("NULL fields");
  for (int64_t i = 0; i < (int64_t)L * batch; ++i)
    if (!std::isfinite(h[i])) return inval("non-finite field");
  return QK_OK;
}

QK_API qk_status qk_ham_create(const qk_basis* b, const qk_ham_params* p, const double* h_host, int32_t batch,
                               void* stream, qk_ham** out) {
  g_err.clear();
  if (!out) return inval("NULL out");
  *out = nullptr;
  if (!b || !p) return inval("NULL pointer");
  if (batch < 1 || batch > QK_MAX_BATCH) return inval("batch must be in [1, 64]");
  if (!std::isfinite(p->jxy) || !std::isfinite(p->jz)) return inval("non-finite coupling");
  if (p->pbc != 0 && p->pbc != 1) return inval("pbc must be 0 or 1");
  if (p->mode != QK_MATFREE && p->mode != QK_CSR && p->mode != QK_MATFREE_ROWS) return inval("unknown mode");
  if (p->mode == QK_CSR && b->D > (1 << 24)) return inval("CSR form limited to D <= 2^24");
  qk_status st = check_fields(h_host, b->L, batch);
  if (st != QK_OK) return st;
  if (batch * b->L > kFldCap) return inval("batch * L must be at most 2048");
  st = check_device(b->device);
  if (st != QK_OK) return st;
  qk_ham* H = new (std::nothrow) qk_ham;
  if (!H) return QK_ENOMEM;
  H->basis = b;
  H->p = *p;
  H->batch = batch;
  H->device = b->device;
  H->h_host.assign(h_host, h_host + (size_t)b->L * batch);
  hipStream_t s = (hipStream_t)stream;
  const size_t fbytes = sizeof(double) * (size_t)b->L * batch;
  H->al = current_allocator();
  hipError_t e = dev_alloc(H->al, (void**)&H->d_fields, fbytes);
  if (e == hipSuccess) e = hipMemcpyAsync(H->d_fields, h_host, fbytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // h_host may be freed by the caller after return
  if (e != hipSuccess) {
    st = hip_fail(e, "qk_ham_create");
    qk_ham_destroy(H);
    return st;
  }
  if (p->mode == QK_CSR) {
    e = dev_alloc(H->al, (void**)&H->d_rowptr, sizeof(uint32_t) * ((size_t)b->D + 1));
    if (e == hipSuccess) e = dev_alloc(H->al, (void**)&H->d_diag, sizeof(double) * (size_t)b->D * batch);
    if (e != hipSuccess) {
      st = hip_fail(e, "qk_ham_create CSR allocation");
      qk_ham_destroy(H);
      return st;
    }
    st = launch_csr_build(H, s);
    if (st != QK_OK) {
      qk_ham_destroy(H);
      return st;
    }
  }
  H->llo = blocked_llo(b->L, b->N, batch, p->mode);
  if (H->llo > 0) {
    st = launch_blocked_build(H, s);
    if (st != QK_OK) {
      qk_ham_destroy(H);
      return st;
    }
  }
  st = split_build(H, s);
  if (st != QK_OK) {
    qk_ham_destroy(H);
    return st;
  }
  // complete on return, like the basis (the CSR fill is still in flight here)
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    st = hip_fail(e, "qk_ham_create");
    qk_ham_destroy(H);
    return st;
  }
  *out = H;
  return QK_OK;
}

QK_API qk_status qk_ham_set_fields(qk_ham* H, const double* h_host, int32_t batch, void* stream) {
  g_err.clear();
  if (!H) return inval("NULL Hamiltonian");
  if (batch != H->batch) return inval("batch differs from the Hamiltonian's");
  qk_status st = check_fields(h_host, H->basis->L, batch);
  if (st != QK_OK) return st;
  st = check_device(H->device);
  if (st != QK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const size_t fbytes = sizeof(double) * (size_t)H->basis->L * batch;
  QK_HIP(hipMemcpyAsync(H->d_fields, h_host, fbytes, hipMemcpyHostToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  H->h_host.assign(h_host, h_host + (size_t)H->basis->L * batch);
  if (H->llo > 0) {
    st = launch_blocked_fields(H, s);
    if (st != QK_OK) return st;
  }
  st = split_fields(H, s);
  if (st != QK_OK) return st;
  if (H->p.mode == QK_CSR) return launch_csr_diag(H, s);
  return QK_OK;
}

QK_API qk_status qk_ham_get_fields(const qk_ham* H, double* h_host, int32_t batch) {
  g_err.clear();
  if (!H || !h_host) return inval("NULL pointer");
  if (batch != H->batch) return inval("batch differs from the Hamiltonian's");
  std::copy(H->h_host.begin(), H->h_host.end(), h_host);
  return QK_OK;
}

QK_API qk_status qk_ham_shape(const qk_ham* H, int64_t* D, int32_t* batch, int32_t* mode) {
  g_err.clear();
  if (!H || !D || !batch || !mode) return inval("NULL pointer");
  *D = H->basis->D;
  *batch = H->batch;
  *mode = H->p.mode;
  return QK_OK;
}

QK_API qk_status qk_ham_apply(const qk_ham* H, const void* x, void* y, int32_t dtype, void* stream) {
  g_err.clear();
  if (!H || !x || !y) return inval("NULL pointer");
  if (dtype != QK_C128 && dtype != QK_C64) return inval("unknown dtype");
  const size_t bytes = elem_bytes(dtype) * (size_t)H->basis->D * H->batch;
  if (ranges_overlap(x, bytes, y, bytes)) return inval("x and y overlap");
  if (((uintptr_t)x | (uintptr_t)y) % elem_bytes(dtype)) return inval("misaligned vector");
  qk_status st = check_device(H->device);
  if (st != QK_OK) return st;
  return launch_ham_apply(H, x, y, dtype, (hipStream_t)stream);
}

QK_API void qk_ham_destroy(qk_ham* H) {
  if (!H) return;
  (void)hipDeviceSynchronize();
  dev_free(H->al, H->d_fields);
  dev_free(H->al, H->d_rowptr);
  dev_free(H->al, H->d_cols);
  dev_free(H->al, H->d_diag);
  dev_free(H->al, H->d_lo_state);
  dev_free(H->al, H->d_lo_rank);
  dev_free(H->al, H->d_blk);
  split_free(H);
  delete H;
}

// ------------------------------------------------------------------ Krylov
QK_API qk_status qk_krylov_create(const qk_ham* H, int32_t m, int32_t dtype, int32_t reorth, qk_krylov** out) {
  g_err.clear();
  return krylov_create(H, m, dtype, reorth, current_allocator(), out);
}

qk_status qk::krylov_create(const qk_ham* H, int32_t m, int32_t dtype, int32_t reorth, const qk_allocator& al,
                              qk_krylov** out) {
  if (!out) return inval("NULL out");
  *out = nullptr;
  if (!H) return inval("NULL Hamiltonian");
  if (m < 1 || m > QK_MAX_M) return inval("m must be in [1, 64]");
  if (dtype != QK_C128 && dtype != QK_C64) return inval("unknown dtype");
  if (reorth < 0 || reorth > 2) return inval("reorth must be 0, 1 or 2");
  qk_status st = check_device(H->device);
  if (st != QK_OK) return st;
  qk_krylov* k = new (std::nothrow) qk_krylov;
  if (!k) return QK_ENOMEM;
  k->H = H;
  k->m = m;
  k->dtype = dtype;
  k->reorth = reorth;
  k->batch = H->batch;
  k->D = H->basis->D;
  k->device = H->device;
  k->grid = krylov_grid((uint64_t)k->D, k->batch);
  // the two-pass split iteration (built with the Hamiltonian when QK_SPLIT=1)
  // keeps its vectors in the padded layout of the split
  const bool use_split = split_usable(H) && k->batch == 1 && reorth == 0;
  k->ustride = use_split ? split_padded_len(H, dtype) : (uint64_t)k->D * k->batch;
  const size_t vec = elem_bytes(dtype) * (size_t)k->ustride;
  k->al = al;
  hipError_t e = dev_alloc(k->al, &k->d_U, vec * (size_t)m);
  if (e == hipSuccess)
    e = dev_alloc(k->al, (void**)&k->d_partA, sizeof(double) * (size_t)kMaxPartialBlocks * kQA * k->batch);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&k->d_partB, sizeof(double) * (size_t)kMaxPartialBlocks * k->batch);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&k->d_coef, sizeof(double) * kstate_doubles(m, k->batch));
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&k->d_int, sizeof(int32_t) * 2 * k->batch);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&k->d_ptot, sizeof(double) * (size_t)(kQA + 1) * k->batch);
  if (e == hipSuccess) e = hipMemset(k->d_coef, 0, sizeof(double) * kstate_doubles(m, k->batch));
  if (e == hipSuccess) e = hipMemset(k->d_int, 0, sizeof(int32_t) * 2 * k->batch);
  if (e == hipSuccess && reorth == 2) {
    const size_t chunks = (size_t)(m + kReorthChunk - 1) / kReorthChunk;
    e = dev_alloc(k->al, (void**)&k->d_rpart, sizeof(double) * chunks * kReorthGrid * 2 * kReorthChunk * k->batch);
    if (e == hipSuccess) e = dev_alloc(k->al, (void**)&k->d_rcoef, sizeof(double) * (size_t)m * 2 * k->batch);
  }
  if (e == hipSuccess && use_split) {
    e = dev_alloc(k->al, &k->d_Z, vec);
    if (e == hipSuccess) e = dev_alloc(k->al, (void**)&k->d_sp, sizeof(double) * 6 * (size_t)kMaxPartialBlocks);
  }
  if (e != hipSuccess) {
    st = hip_fail(e, "qk_krylov_create allocation");
    qk_krylov_destroy(k);
    return st;
  }
  *out = k;
  return QK_OK;
}

QK_API qk_status qk_krylov_expm_step(qk_krylov* k, void* psi, double dt, void* stream, qk_step_info* info) {
  g_err.clear();
  if (!k || !psi) return inval("NULL pointer");
  if (!std::isfinite(dt)) return inval("dt not finite");
  if ((uintptr_t)psi % elem_bytes(k->dtype)) return inval("misaligned psi");
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  const size_t vec = elem_bytes(k->dtype) * (size_t)k->D * k->batch;
  if (workspace_overlap(k, psi, vec)) return inval("psi overlaps the Krylov workspace");
  hipStream_t s = (hipStream_t)stream;
  st = launch_krylov_step(k, psi, dt, s);
  if (st != QK_OK || !info) return st;
  const int B = k->batch;
  std::vector<int32_t> iv(2 * B);
  std::vector<double> err(B), n0(B);
  const KState ks = make_kstate(k);
  QK_HIP(hipMemcpyAsync(iv.data(), k->d_int, sizeof(int32_t) * 2 * B, hipMemcpyDeviceToHost, s));
  QK_HIP(hipMemcpyAsync(err.data(), ks.err, sizeof(double) * B, hipMemcpyDeviceToHost, s));
  QK_HIP(hipMemcpyAsync(n0.data(), ks.n0, sizeof(double) * B, hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  qk_status worst = QK_OK;
  for (int b = 0; b < B; ++b) {
    info[b].m_used = iv[b];
    info[b].status = iv[B + b];
    info[b].err_est = err[b];
    info[b].beta0 = n0[b];
    if (iv[B + b] != QK_OK) worst = QK_ENUMERIC;
  }
  if (worst != QK_OK) set_error("non-finite Lanczos coefficient");
  return worst;
}

QK_API qk_status qk_krylov_evolve(qk_krylov* k, void* psi, double t, const qk_adapt_params* p, void* stream,
                                  qk_adapt_info* info) {
  g_err.clear();
  if (!k || !psi || !p) return inval("NULL pointer");
  if (!std::isfinite(t) || t < 0.0) return inval("t must be finite and >= 0");
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return inval("tol must be finite and > 0");
  if (!(p->dt_init > 0.0) || !std::isfinite(p->dt_init)) return inval("dt_init must be finite and > 0");
  if (!(p->dt_max > 0.0) || !std::isfinite(p->dt_max)) return inval("dt_max must be finite and > 0");
  if (p->max_steps < 1) return inval("max_steps must be >= 1");
  if ((uintptr_t)psi % elem_bytes(k->dtype)) return inval("misaligned psi");
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  const size_t vec = elem_bytes(k->dtype) * (size_t)k->D * k->batch;
  if (workspace_overlap(k, psi, vec)) return inval("psi overlaps the Krylov workspace");
  hipStream_t s = (hipStream_t)stream;
  const int B = k->batch;
  const KState ks = make_kstate(k);
  std::vector<double> tau(2 * B);
  std::vector<int32_t> iv(2 * B);
  double done = 0.0, dt_try = p->dt_init, err_sum = 0.0, dmin = INFINITY, dmax = 0.0;
  int steps = 0;
  while (t - done > 1e-14 * t) {
    if (steps >= p->max_steps) {
      set_error("adaptive evolution did not reach t within max_steps");
      return QK_ENUMERIC;
    }
    double tau_max = std::min(std::min(dt_try, p->dt_max), t - done);
    st = launch_krylov_adaptive_step(k, psi, tau_max, p->tol, s);
    if (st != QK_OK) return st;
    QK_HIP(hipMemcpyAsync(tau.data(), ks.tau, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s));
    QK_HIP(hipMemcpyAsync(iv.data(), k->d_int, sizeof(int32_t) * 2 * B, hipMemcpyDeviceToHost, s));
    double e0 = 0.0;
    QK_HIP(hipMemcpyAsync(&e0, ks.err, sizeof(double), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b)
      if (iv[B + b] != QK_OK) {
        set_error("non-finite Lanczos coefficient");
        return QK_ENUMERIC;
      }
    double acc = tau[0], nxt = tau[B];
    for (int b = 1; b < B; ++b) {
      acc = std::min(acc, tau[b]);
      nxt = std::min(nxt, tau[B + b]);
    }
    if (!(acc > 0.0)) {
      set_error("adaptive step collapsed to zero");
      return QK_ENUMERIC;
    }
    // the last step lands exactly on t
    done = (acc >= t - done) ? t : done + acc;
    ++steps;
    err_sum += e0;
    dmin = std::min(dmin, acc);
    dmax = std::max(dmax, acc);
    dt_try = nxt > 0.0 ? nxt : acc;
  }
  if (info) {
    info->steps = steps;
    info->dt_min = steps ? dmin : 0.0;
    info->dt_max = dmax;
    info->err_sum = err_sum;
  }
  return QK_OK;
}

QK_API qk_status qk_krylov_coefficients(const qk_krylov* k, int32_t item, double* alpha, double* beta,
                                        int32_t* m_used) {
  g_err.clear();
  if (!k || !alpha || !beta || !m_used) return inval("NULL pointer");
  if (item < 0 || item >= k->batch) return inval("item out of range");
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  const int B = k->batch, m = k->m;
  std::vector<double> a((size_t)m * B), bb((size_t)m * B);
  std::vector<int32_t> iv(2 * B);
  const KState ks = make_kstate(k);
  QK_HIP(hipDeviceSynchronize());
  QK_HIP(hipMemcpy(a.data(), ks.alpha, sizeof(double) * m * B, hipMemcpyDeviceToHost));
  QK_HIP(hipMemcpy(bb.data(), ks.beta, sizeof(double) * m * B, hipMemcpyDeviceToHost));
  QK_HIP(hipMemcpy(iv.data(), k->d_int, sizeof(int32_t) * 2 * B, hipMemcpyDeviceToHost));
  *m_used = iv[item];
  for (int j = 0; j < m; ++j) {
    alpha[j] = a[(size_t)j * B + item];
    beta[j] = bb[(size_t)j * B + item];
  }
  return QK_OK;
}

QK_API qk_status qk_krylov_profile(qk_krylov* k, int32_t enable) {
  g_err.clear();
  if (!k) return inval("NULL workspace");
  if (enable != 0 && enable != 1) return inval("enable must be 0 or 1");
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  if (enable) {
    st = profile_collect(k);
    if (st != QK_OK) return st;
    for (int i = 0; i < QK_NUM_KERNELS; ++i) {
      k->ms_total[i] = 0.0;
      k->launches[i] = 0;
    }
  }
  k->profiling = enable != 0;
  return QK_OK;
}

QK_API qk_status qk_krylov_profile_read(qk_krylov* k, qk_kernel_time* out) {
  g_err.clear();
  if (!k || !out) return inval("NULL pointer");
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  st = profile_collect(k);
  if (st != QK_OK) return st;
  for (int i = 0; i < QK_NUM_KERNELS; ++i) {
    out[i].ms_total = k->ms_total[i];
    out[i].launches = k->launches[i];
  }
  return QK_OK;
}

QK_API void qk_krylov_destroy(qk_krylov* k) {
  if (!k) return;
  (void)hipDeviceSynchronize();
  for (auto& p : k->pending) {
    if (p.start) (void)hipEventDestroy(p.start);
    if (p.end) (void)hipEventDestroy(p.end);
  }
  for (auto e : k->spare) (void)hipEventDestroy(e);
  dev_free(k->al, k->d_U);
  dev_free(k->al, k->d_partA);
  dev_free(k->al, k->d_partB);
  dev_free(k->al, k->d_rpart);
  dev_free(k->al, k->d_rcoef);
  dev_free(k->al, k->d_coef);
  dev_free(k->al, k->d_int);
  dev_free(k->al, k->d_ptot);
  dev_free(k->al, k->d_Z);
  dev_free(k->al, k->d_sp);
  delete k;
}

// ------------------------------------------------------------ launch shapes
QK_API qk_status qk_krylov_set_shape(qk_krylov* k, const qk_launch_shape* shape) {
  g_err.clear();
  if (!k || !shape) return inval("NULL pointer");
  return apply_shape(k, shape);
}

QK_API qk_status qk_krylov_get_shape(const qk_krylov* k, qk_launch_shape* shape) {
  g_err.clear();
  if (!k || !shape) return inval("NULL pointer");
  shape->threads = k->threads;
  shape->blocks_per_cu = k->blocks_per_cu;
  shape->blocked_wgs_per_cu = k->blocked_wgs;
  shape->blocked_llo = k->H->llo;
  return QK_OK;
}

QK_API qk_status qk_krylov_autotune(qk_krylov* k, double dt, const char* cache_path, void* stream,
                                    qk_launch_shape* chosen) {
  g_err.clear();
  if (!k) return inval("NULL workspace");
  if (!std::isfinite(dt)) return inval("dt not finite");
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  return krylov_autotune(k, dt, cache_path, (hipStream_t)stream, chosen);
}

// ----------------------------------------------------------- batched driver
QK_API qk_status qk_batch_create(qk_krylov* const* ks, void* const* psi, const int64_t* r0, int32_t n,
                                 qk_batch** out) {
  g_err.clear();
  if (!out) return inval("NULL out");
  *out = nullptr;
  if (n < 1 || n > 64) return inval("n must be in [1, 64]");
  if (!ks || !psi || !r0) return inval("NULL pointer");
  for (int i = 0; i < n; ++i) {
    if (!ks[i] || !psi[i]) return inval("NULL workspace or vector");
    if (ks[i]->device != ks[0]->device) return inval("workspaces on different devices");
    if (r0[i] >= ks[i]->D) return inval("r0 out of range");
    if ((uintptr_t)psi[i] % elem_bytes(ks[i]->dtype)) return inval("misaligned psi");
    const size_t vec = elem_bytes(ks[i]->dtype) * (size_t)ks[i]->D * ks[i]->batch;
    for (int j = 0; j < n; ++j) {
      if (j != i && ks[j] == ks[i]) return inval("a workspace appears twice");
      const size_t vj = elem_bytes(ks[j]->dtype) * (size_t)ks[j]->D * ks[j]->batch;
      if (workspace_overlap(ks[j], psi[i], vec)) return inval("psi overlaps a workspace");
      if (j != i && ranges_overlap(psi[i], vec, psi[j], vj)) return inval("state vectors overlap");
    }
  }
  qk_status st = check_device(ks[0]->device);
  if (st != QK_OK) return st;
  return batch_create(ks, psi, r0, n, out);
}

QK_API qk_status qk_batch_items(const qk_batch* b, int32_t* items) {
  g_err.clear();
  if (!b || !items) return inval("NULL pointer");
  *items = batch_items(b);
  return QK_OK;
}

QK_API qk_status qk_batch_run_autocorr(qk_batch* b, double dt, int32_t n_steps, int32_t use_graph, double* P_device,
                                       double* C_device, void* stream) {
  g_err.clear();
  if (!b || !P_device) return inval("NULL pointer");
  if (!std::isfinite(dt)) return inval("dt not finite");
  if (n_steps < 0) return inval("n_steps < 0");
  if (use_graph < 0 || use_graph > 2) return inval("use_graph must be 0, 1 or 2");
  qk_status st = check_device(batch_device(b));
  if (st != QK_OK) return st;
  if (n_steps == 0) return QK_OK;
  return batch_run(b, dt, n_steps, use_graph, P_device, C_device, (hipStream_t)stream);
}

QK_API qk_status qk_batch_run(qk_batch* b, double dt, int32_t n_steps, int32_t use_graph, double* P_device,
                              void* stream) {
  return qk_batch_run_autocorr(b, dt, n_steps, use_graph, P_device, nullptr, stream);
}

QK_API void qk_batch_destroy(qk_batch* b) { batch_destroy(b); }

// ----------------------------------------------------------------- gradient
QK_API qk_status qk_grad_return_prob(qk_krylov* k, int64_t r0, double T, int32_t n_steps, int32_t ckpt_every,
                                     double* F_host, double* dFdh_host, void* stream) {
  g_err.clear();
  if (!k || !F_host || !dFdh_host) return inval("NULL pointer");
  if (!std::isfinite(T) || T < 0.0) return inval("T must be finite and >= 0");
  if (n_steps < 1) return inval("n_steps must be >= 1");
  if (ckpt_every < 1) return inval("ckpt_every must be >= 1");
  if (r0 < 0 || r0 >= k->D) return inval("r0 out of range");
  if (k->dtype != QK_C128 || k->batch != 1 || k->m > 32) {
    set_error("the gradient needs a complex128 workspace with batch 1 and m <= 32");
    return QK_EUNSUPPORTED;
  }
  qk_status st = check_device(k->device);
  if (st != QK_OK) return st;
  return grad_return_prob(k, r0, T, n_steps, ckpt_every, F_host, dFdh_host, (hipStream_t)stream);
}

// -------------------------------------------------------------- observable
QK_API qk_status qk_return_prob(const qk_basis* b, int64_t r0, const void* psi0, const void* psi, int32_t dtype,
                                int32_t batch, double* P_device, void* stream) {
  g_err.clear();
  if (!b || !psi || !P_device) return inval("NULL pointer");
  if (dtype != QK_C128 && dtype != QK_C64) return inval("unknown dtype");
  if (batch < 1 || batch > QK_MAX_BATCH) return inval("batch must be in [1, 64]");
  if (!psi0 && (r0 < 0 || r0 >= b->D)) return inval("r0 out of range");
  qk_status st = check_device(b->device);
  if (st != QK_OK) return st;
  return launch_return_prob(b, r0, psi0, psi, dtype, batch, P_device, (hipStream_t)stream);
}

QK_API qk_status qk_return_prob_noalloc(const qk_basis* b, int64_t r0, const void* psi0, const void* psi,
                                        int32_t dtype, int32_t batch, double* P_device, void* stream) {
  g_err.clear();
  if (!b || !psi || !P_device) return inval("NULL pointer");
  if (dtype != QK_C128 && dtype != QK_C64) return inval("unknown dtype");
  if (batch < 1 || batch > QK_MAX_BATCH) return inval("batch must be in [1, 64]");
  if (!psi0 && (r0 < 0 || r0 >= b->D)) return inval("r0 out of range");
  qk_status st = check_device(b->device);
  if (st != QK_OK) return st;
  return launch_return_prob_noalloc(b, r0, psi0, psi, dtype, batch, P_device, (hipStream_t)stream);
}

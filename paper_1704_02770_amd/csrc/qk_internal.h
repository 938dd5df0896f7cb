// Internal declarations of libqkrylov: handle layouts, device-side argument
// blocks and the host launchers that the C ABI layer calls.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "qk.h"

namespace qk {

constexpr int kBinomStride = 33;        // binom[n * 33 + k] = C(n, k), n, k <= 32 (32-bit states)
constexpr int kFldCap = 2048;           // field values the row kernels stage in LDS: batch * L <= kFldCap

// Sector states are 32-bit integers for L <= 32 and 64-bit integers up to
// L = 64; the binomial table of a basis has stride kStride (entries C(n, k),
// n, k < kStride, saturated at 2^32 - 1: every term of a rank is below D).
template <typename S> struct StateT;
template <> struct StateT<uint32_t> {
  static constexpr int kStride = 33;
  static constexpr int kMaxL = 32;
};
template <> struct StateT<uint64_t> {
  static constexpr int kStride = 65;
  static constexpr int kMaxL = 64;
};
constexpr int kNumXcd = 8;              // MI355X: 8 accelerator complex dies, WGs dealt round-robin
constexpr int kMaxBlock = 256;
constexpr int kReorthChunk = 8;         // Krylov vectors per dot-product pass of the full reorthogonalisation
constexpr int kReorthGrid = 512;        // blocks of that pass
constexpr int kMaxPartialBlocks = 4096; // partial-sum slots per reduction (>= any grid used)
// Fewest (row, column) elements a work-group of a Krylov-step pass is given:
// small sectors get fewer, fuller work-groups instead of a chip-filling grid
// of nearly empty ones (and fewer partial sums for the next pass to reduce).
// Measured with plain launches: L = 20 and 22 chains step faster at 512 than
// with the uncapped grids and than at 2048; sectors of L >= 24 are unchanged.
constexpr uint64_t kMinBlockWork = 512;

void set_error(const std::string& msg);
qk_status hip_fail(hipError_t e, const char* what);

#define QK_HIP(call)                                          \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::qk::hip_fail(e_, #call);   \
  } while (0)

// Threads per block for a batch of B problems: B x 2^k <= 256, so that a
// grid-stride loop keeps each thread on one batch column and per-column
// tree reductions halve evenly.
inline int block_threads(int B, int cap = kMaxBlock) {
  if (cap < B) cap = B;
  if (cap > kMaxBlock) cap = kMaxBlock;
  int t = B;
  while (t * 2 <= cap) t *= 2;
  return t;
}

}  // namespace qk

// Allocator of a handle's device memory (qk_set_allocator); all NULL means
// hipMalloc / hipFree.
struct qk_allocator {
  qk_alloc_fn alloc = nullptr;
  qk_release_fn release = nullptr;
  void* ctx = nullptr;
};

namespace qk {
qk_allocator current_allocator();
// memory used on any stream; released only once the device work using it has
// been waited for
hipError_t dev_alloc(const qk_allocator& a, void** p, size_t bytes);
void dev_free(const qk_allocator& a, void* p);
// stream-ordered temporary: used by work queued on s and released right after
// the last of it is queued (hipMallocAsync / hipFreeAsync semantics)
hipError_t dev_alloc_async(const qk_allocator& a, void** p, size_t bytes, hipStream_t s);
hipError_t dev_free_async(const qk_allocator& a, void* p, hipStream_t s);
}  // namespace qk

struct qk_basis {
  qk_allocator al;
  int32_t L = 0, N = 0;
  int64_t D = 0;
  int device = 0;
  bool wide = false;              // L > 32: 64-bit states
  void* d_states = nullptr;       // [D] sorted sector states (uint32_t, or uint64_t when wide)
  uint32_t* d_binom = nullptr;    // [33 * 33] C(n, k), or [65 * 65] when wide
};

struct qk_ham {
  qk_allocator al;
  const qk_basis* basis = nullptr;
  qk_ham_params p{};
  int32_t batch = 1;
  int device = 0;
  double* d_fields = nullptr;     // [batch][L]
  std::vector<double> h_host;     // [batch][L] copy of the fields
  // CSR form (mode == QK_CSR): off-diagonal columns, row pointers, diagonal [D][batch]
  uint32_t* d_rowptr = nullptr;   // [D + 1]
  uint32_t* d_cols = nullptr;     // [nnz]
  double* d_diag = nullptr;       // [D][batch]
  int64_t nnz = 0;
  // blocked matrix-free form (llo > 0): low-bit tables and the block list
  int llo = 0;
  uint16_t* d_lo_state = nullptr; // [2^llo]
  uint16_t* d_lo_rank = nullptr;  // [2^llo]
  void* d_blk = nullptr;          // [nblk] block entries (high bits, first row, ring-partner first row)
  int nblk = 0;
  uint64_t tables_gen = 0;        // incremented whenever the block tables are rebuilt
  // two-pass high/low split (one field set, 18 <= L <= 32): tables of qk_split.hip
  void* split = nullptr;
};

struct qk_krylov {
  qk_allocator al;
  const qk_ham* H = nullptr;
  int32_t m = 0, dtype = 0, reorth = 0, batch = 1;
  int64_t D = 0;
  int device = 0;
  // launch shape (qk_krylov_set_shape / qk_krylov_autotune); 0 = default
  int threads = 0;                // threads per block of the row-streaming kernels (B * 2^k, <= 256)
  int blocks_per_cu = 0;          // blocks per CU of the row-streaming kernels
  int blocked_wgs = 0;            // work-groups per CU of the blocked H-pass
  int grid = 0;                   // blocks of the streaming kernels (multiple of 8)
  void* d_U = nullptr;            // m slots of ustride elements: u_1..u_m
  uint64_t ustride = 0;           // elements per slot: D * batch, or the padded length of the split layout
  double* d_partA = nullptr;      // [grid][2][batch] partial sums of the H-pass
  double* d_partB = nullptr;      // [grid][1][batch] partial sums of the update pass
  double* d_ptot = nullptr;       // [kQA + 1][batch] totals of both (batches of 8 or more)
  double* d_coef = nullptr;       // coefficient block, see qk::KState
  int32_t* d_int = nullptr;       // [2][batch]: m_used, status
  double* d_rpart = nullptr;      // full reorthogonalisation: [chunks][kReorthGrid][2 kReorthChunk][batch] partial dots
  double* d_rcoef = nullptr;      // full reorthogonalisation: [m][2][batch] projection coefficients
  // two-pass split iteration (one field set, no reorthogonalisation)
  void* d_Z = nullptr;            // [ustride] high-pass result z of the current iteration (padded layout)
  double* d_sp = nullptr;         // partial sums: high pass [kMaxPartialBlocks][2], low pass 2 x ([kMaxPartialBlocks] norms, [kMaxPartialBlocks] forms)
  // event timing (qk_krylov_profile)
  bool profiling = false;
  struct Pending { int kind; hipEvent_t start, end; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> spare;
  double ms_total[QK_NUM_KERNELS] = {};
  int64_t launches[QK_NUM_KERNELS] = {};
};

namespace qk {

// Device view of the Lanczos coefficient block of one workspace.
struct KState {
  double* alpha;   // [m][B]
  double* beta;    // [m][B]
  double* sigma;   // [m + 1][B]  1 / norm of stored vector u_j
  double* n0;      // [B]         norm of psi at step start
  double* gre;     // [m][B]      combination coefficients (real)
  double* gim;     // [m][B]      (imaginary)
  double* err;     // [B]
  int32_t* mused;  // [B]
  int32_t* status; // [B]
  double* tau;     // [2][B]      adaptive steps: accepted step, suggested next step
};

inline size_t kstate_doubles(int m, int B) { return (size_t)B * (5 * m + 1 + 2 + 1 + 2); }
KState make_kstate(const qk_krylov* k);
// The same layout over other storage (a saved copy of d_coef and d_int).
KState kstate_at(const qk_krylov* k, double* coef, int32_t* ints);

// Model arguments of the matrix-free rows.
struct ModelArgs {
  int32_t L, N, pbc, B;
  double half_jxy, jz;
  uint64_t lmask;        // low L bits
};
ModelArgs model_args(const qk_ham* H);

// Launchers (all asynchronous on `s`).
qk_status launch_basis_build(qk_basis* b, hipStream_t s);
qk_status launch_rank(const qk_basis* b, const uint64_t* d_in, int64_t n, int64_t* d_out, hipStream_t s);
qk_status launch_csr_build(qk_ham* H, hipStream_t s);
qk_status launch_csr_diag(qk_ham* H, hipStream_t s);
qk_status launch_ham_apply(const qk_ham* H, const void* x, void* y, int dtype, hipStream_t s);
int blocked_llo(int L, int N, int B, int mode);
qk_status launch_blocked_build(qk_ham* H, hipStream_t s);
qk_status launch_blocked_apply(const qk_ham* H, const void* x, void* y, int dtype, hipStream_t s);
qk_status launch_blocked_fields(qk_ham* H, hipStream_t s);
bool blocked_usable(const qk_ham* H, int dtype);
// Valid low-bit counts of the block decomposition for this Hamiltonian
// (empty without block tables), and a rebuild of the tables at another one.
bool blocked_llo_valid(const qk_ham* H, int llo);
qk_status blocked_rebuild(qk_ham* H, int llo);
// two-pass high/low split (qk_split.hip)
qk_status split_build(qk_ham* H, hipStream_t s);   // no-op unless QK_SPLIT=1, one field set, matrix-free, 18 <= L <= 30
qk_status split_fields(qk_ham* H, hipStream_t s);
void split_free(qk_ham* H);
bool split_usable(const qk_ham* H);
int split_llo(int L);
uint64_t split_padded_len(const qk_ham* H, int dtype);   // elements of one workspace vector (padded layout)
qk_status split_line_tables(const qk_ham* H, int dtype, const uint32_t** r0, const uint8_t** n, uint64_t* dpad,
                            int* pe);
qk_status launch_split_apply(const qk_ham* H, const void* x, void* y, int dtype, hipStream_t s);
// qk_krylov_create with the device memory of the workspace from `al`
qk_status krylov_create(const qk_ham* H, int32_t m, int32_t dtype, int32_t reorth, const qk_allocator& al,
                        qk_krylov** out);
// How far one Krylov step goes: the basis and Lanczos coefficients only, or
// the whole step with psi replaced by the combination.
enum class StepUpTo { basis, combination };
qk_status launch_krylov_step(qk_krylov* k, void* psi, double dt, hipStream_t s,
                             StepUpTo upto = StepUpTo::combination);
// One step of at most tau_max whose length the device chooses from the error
// estimate: st.tau[b] receives the accepted step of column b, st.tau[B + b] a
// suggested next step; every column advances by the smallest accepted step.
// Overlap |<psi0, psi>|^2 of every column written at the batched driver's
// record position (counter == NULL: P[b]); part holds G * 2 * B doubles with
// G = overlap_grid(D, B).
int overlap_grid(uint32_t D, int B);
qk_status launch_overlap_record(const void* psi0, const void* psi, int dtype, uint32_t D, int B, double* part, int G,
                                double* P, const int* counter, int off, int items, hipStream_t s);
qk_status launch_krylov_adaptive_step(qk_krylov* k, void* psi, double tau_max, double tol, hipStream_t s);
qk_status grad_return_prob(qk_krylov* k, int64_t r0, double T, int n_steps, int ckpt_every, double* F, double* dFdh,
                           hipStream_t s);
qk_status profile_mark(qk_krylov* k, int kind, bool begin, hipStream_t s);
int stream_grid(uint64_t rows, int B, int threads, int blocks_per_cu);
int krylov_threads(const qk_krylov* k);
int qk_num_cus();
int binom_stride(const qk_basis* b);   // stride of the basis's binomial table
qk_status apply_shape(qk_krylov* k, const qk_launch_shape* sh);
qk_status krylov_autotune(qk_krylov* k, double dt, const char* cache_path, hipStream_t s, qk_launch_shape* chosen);
qk_status batch_create(qk_krylov* const* ks, void* const* psi, const int64_t* r0, int n, qk_batch** out);
void batch_destroy(qk_batch* b);
qk_status batch_run(qk_batch* b, double dt, int n_steps, int use_graph, double* P, double* C, hipStream_t s);
int batch_items(const qk_batch* b);
int batch_device(const qk_batch* b);
qk_status profile_collect(qk_krylov* k);
qk_status launch_return_prob(const qk_basis* b, int64_t r0, const void* psi0, const void* psi, int dtype,
                             int B, double* P, hipStream_t s);
// qk_return_prob with the overlap partials in the library's fixed per-GPU
// scratch array instead of a temporary allocation
qk_status launch_return_prob_noalloc(const qk_basis* b, int64_t r0, const void* psi0, const void* psi, int dtype,
                                     int B, double* P, hipStream_t s);

}  // namespace qk

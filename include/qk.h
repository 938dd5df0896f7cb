/*
 * qk.h -- C ABI of libqkrylov: Krylov-subspace time evolution of a spin-1/2
 * XXZ chain with on-site fields in a fixed particle-number sector, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Brenes, Varma, Scardicchio, Girotto, "Massively parallel
 * implementation and approaches to simulate quantum dynamics using Krylov
 * subspace techniques" (arXiv:1704.02770).  Section / equation / algorithm
 * references below are to that paper.
 *
 * Conventions shared by every entry point
 *   - Model (Sec. 2, Eq. (1), read in spin language):
 *       H = sum_b [ (jxy/2)(S+_a S-_c + S-_a S+_c) + jz S^z_a S^z_c ] + sum_i h_i S^z_i
 *     with S = sigma/2.  Site i (1-based) is bit i-1 of a state integer.  Open
 *     chains have the bonds (0,1)..(L-2,L-1); periodic chains add (L-1,0)
 *     (so a 2-site ring carries its pair twice).  The hopping is +jxy/2.
 *   - Basis (Sec. 2 "Basis representation"; Sec. 3 Algorithm 2): the states
 *     with n_up set bits out of L, in ascending integer order; row r of every
 *     vector belongs to the r-th such integer.  D = C(L, n_up).
 *   - Vectors are device memory holding interleaved complex numbers (real,
 *     imaginary): QK_C128 = 2 x double per element (16 B, 16-B aligned),
 *     QK_C64 = 2 x float (8 B, 8-B aligned).  A batch of B problems that
 *     share one basis is stored row-major [D][B] (batch index fastest).
 *   - Every call that takes `stream` enqueues its device work on that
 *     hipStream_t (NULL = the legacy default stream) and returns without
 *     waiting, unless stated otherwise.  The caller keeps every buffer alive
 *     until that work has completed.
 *   - Errors: every function returns qk_status; arguments are checked before
 *     any device work is enqueued, so an argument error leaves all buffers
 *     untouched.  qk_last_error() returns a thread-local text for the last
 *     failing call on the calling thread.  Nothing aborts or throws across
 *     this boundary.
 *   - Handles (qk_basis, qk_ham, qk_krylov, qk_batch) are created on the current HIP
 *     device, own their device memory (from the allocator registered with
 *     qk_set_allocator, hipMalloc by default), and are released only by the matching
 *     *_destroy (which accepts NULL and synchronises the device first).  A
 *     handle may be used by one stream at a time; calls on a handle from
 *     another device return QK_EINVAL.
 */
#ifndef QK_H
#define QK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QK_ABI_VERSION 2
#define QK_MAX_L 64          /* states are 32-bit integers for L <= 32, 64-bit above */
#define QK_MAX_M 64          /* Krylov dimension limit (one wavefront per projected problem) */
#define QK_MAX_BATCH 64      /* problems per batched handle */

typedef enum {
  QK_OK = 0,
  QK_EINVAL = 1,        /* bad argument; nothing was enqueued */
  QK_ENOMEM = 2,        /* device allocation failed */
  QK_EHIP = 3,          /* a HIP runtime call failed (text in qk_last_error) */
  QK_EUNSUPPORTED = 4,  /* valid request outside what the library implements */
  QK_ENUMERIC = 5       /* non-finite Lanczos coefficient, or an adaptive evolution that could not reach t */
} qk_status;

typedef enum { QK_C128 = 0, QK_C64 = 1 } qk_dtype;
typedef enum { QK_MATFREE = 0, QK_CSR = 1, QK_MATFREE_ROWS = 2 } qk_ham_mode;

/* Version of this header the library was built from (QK_ABI_VERSION). */
int qk_abi_version(void);

/*
 * Device memory of the handles created from now on (their tables and
 * workspaces, and the temporaries of calls on them) comes from alloc(bytes,
 * stream, ctx) and goes back through release(ptr, stream, ctx) -- for
 * instance a framework's caching allocator.  alloc returns NULL on failure
 * (reported as QK_ENOMEM).  stream NULL: the block may be used on any stream,
 * and release comes only once no device work uses it any more.  stream
 * non-NULL (small temporaries of one call): only work queued on that stream
 * uses the block, and release(ptr, stream) comes right after the last of it
 * is queued, as with hipFreeAsync -- the block may then be reused by later
 * work on that stream, or elsewhere once that stream has reached this point.
 * Each handle keeps the pair it was created with, so changing it later does
 * not affect existing handles.  Both NULL restores hipMalloc /
 * hipFree.  Process-wide; safe to call from any thread.  Errors: QK_EINVAL
 * when exactly one of alloc, release is NULL.
 */
typedef void* (*qk_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*qk_release_fn)(void* ptr, void* stream, void* ctx);
qk_status qk_set_allocator(qk_alloc_fn alloc, qk_release_fn release, void* ctx);

/* Thread-local text of the last error on this thread ("" if none).  The
 * pointer stays valid until the next qk_* call on the same thread. */
const char* qk_last_error(void);

/*
 * Quasiperiodic on-site fields of Eq. (1): h_out[b*L + (i-1)] =
 * h * cos(2*pi*beta*i + phi[b]) for i = 1..L and b = 0..batch-1.
 * Host arrays; runs on the host, no device work.  Errors: QK_EINVAL for
 * L outside [1, QK_MAX_L], batch < 1, NULL pointers or non-finite inputs.
 */
qk_status qk_fields_quasiperiodic(int32_t L, double h, double beta, const double* phi,
                                  int32_t batch, double* h_out);

/* ---------------------------------------------------------------- basis */
typedef struct qk_basis qk_basis;

/*
 * Builds the sorted sector basis on the device (Sec. 3, Algorithms 2 and 3:
 * every chunk of rows starts from the unranked first state of its section
 * and advances by the next-bit-permutation), plus the binomial rank table.
 * 2 <= L <= QK_MAX_L, 0 < n_up < L; the dimension C(L, n_up) must be below
 * 2^32 - 1 (QK_EUNSUPPORTED otherwise), which for L > 32 means a low density
 * (the paper's L = 55 runs of Sec. 4).  States are held as 32-bit integers for
 * L <= 32 and as 64-bit integers above.  *out receives the handle; the build
 * runs on `stream` and the call waits for it, so the handle is ready for use
 * on any stream when it returns.  Errors: QK_EINVAL, QK_EUNSUPPORTED,
 * QK_ENOMEM, QK_EHIP.
 */
qk_status qk_basis_build(int32_t L, int32_t n_up, void* stream, qk_basis** out);

/* Sector dimension D = C(L, n_up) (host value, no device work). */
qk_status qk_basis_dim(const qk_basis* b, int64_t* D);

/* L and n_up of a basis (host values). */
qk_status qk_basis_shape(const qk_basis* b, int32_t* L, int32_t* n_up);

/* Copies the D sorted states into caller device memory dst_device: uint32
 * values for L <= 32, uint64 values for L > 32. */
qk_status qk_basis_states(const qk_basis* b, void* dst_device, void* stream);

/*
 * Row index of each of n host states (Sec. 3: lookup of the row of a state;
 * computed on the device by the combinatorial number system, which equals the
 * position in the sorted basis).  idx_host[i] = -1 when states_host[i] does
 * not have n_up set bits below bit L.  Synchronous (waits for its own work on
 * the legacy default stream).  n may be 0.
 */
qk_status qk_basis_rank(const qk_basis* b, const uint64_t* states_host, int64_t n, int64_t* idx_host);

void qk_basis_destroy(qk_basis* b);

/* ---------------------------------------------------------- Hamiltonian */
typedef struct {
  double jxy;      /* hopping: off-diagonal entry jxy/2 (Eq. (1) t = jxy/2) */
  double jz;       /* zz coupling (Eq. (1) V = jz) */
  int32_t pbc;     /* 0 open chain, 1 periodic chain */
  int32_t mode;    /* QK_MATFREE, QK_CSR or QK_MATFREE_ROWS (see qk_ham_create) */
} qk_ham_params;

typedef struct qk_ham qk_ham;

/*
 * Hamiltonian of Eq. (1) on basis `b` (Sec. 3, "Hamiltonian matrix
 * construction") for `batch` field sets h_host[batch][L] (host doubles,
 * copied).  QK_MATFREE generates every row on the fly in the apply kernels;
 * for 18 <= L <= 32 it processes blocks of states sharing their high bits
 * (low-bit tables and a block list are built here; one field set or a
 * batch), otherwise one row per thread from the stored basis.  With the
 * environment variable QK_SPLIT=1 set at this call, a single-field-set
 * Hamiltonian also builds the tables of the two-pass split (high bonds over
 * column slabs, then low bonds with the Lanczos update; vectors in a padded
 * workspace layout), which its reorthogonalisation-free complex workspaces
 * then use: exact, and slower than the one-pass form on MI355X at L = 28, so
 * off by default.  QK_MATFREE_ROWS always uses the
 * one-row-per-thread form (an independent second formulation).  QK_CSR
 * stores the column indices of the off-diagonal entries after an exact
 * counting pass (the exact preallocation of Sec. 3); allowed for D <= 2^24.
 * The tables are built on `stream` and the call waits for them, so the
 * handle is ready for use on any stream when it returns.  The basis must
 * outlive the Hamiltonian.
 * Errors: QK_EINVAL (NULL, batch outside [1, QK_MAX_BATCH], non-finite
 * parameters, CSR too large), QK_ENOMEM, QK_EHIP.
 */
qk_status qk_ham_create(const qk_basis* b, const qk_ham_params* p, const double* h_host,
                        int32_t batch, void* stream, qk_ham** out);

/* Replaces the field sets (same batch count).  Enqueued on `stream`. */
qk_status qk_ham_set_fields(qk_ham* H, const double* h_host, int32_t batch, void* stream);

/* Copies the current field sets into h_host[batch][L] (host doubles); batch
 * must equal the Hamiltonian's (QK_EINVAL otherwise).  Host only, no device work. */
qk_status qk_ham_get_fields(const qk_ham* H, double* h_host, int32_t batch);

/* D, batch and mode of a Hamiltonian (host values). */
qk_status qk_ham_shape(const qk_ham* H, int64_t* D, int32_t* batch, int32_t* mode);

/*
 * y = H x with the Hamiltonian of Eq. (1), row by row as Sec. 3
 * ("Hamiltonian matrix construction") defines it: the diagonal from the zz
 * bonds and the fields, and jxy/2 in the column of the state with the two
 * bits of every anti-aligned bond exchanged (no matrix is stored in the
 * matrix-free modes).  For every batch item (problem k uses field set k):
 * x, y are [D][B] device arrays of `dtype`; x and y must not overlap
 * (QK_EINVAL).  QK_C128 accumulates in double, QK_C64 in float.  Matrix-free
 * Hamiltonians with 18 <= L <= 32 use the blocked kernels; a single-phase
 * vector below 4 GB is addressed with 32-bit byte offsets, a larger one
 * (the half-filled L = 32 chain) with 64-bit element offsets, which needs the
 * 11-bit block decomposition (the default there; QK_EUNSUPPORTED for another
 * one).  The same choice applies to the Lanczos H-pass of every workspace.
 */
qk_status qk_ham_apply(const qk_ham* H, const void* x, void* y, int32_t dtype, void* stream);

void qk_ham_destroy(qk_ham* H);

/* --------------------------------------------------------------- Krylov */
typedef struct {
  int32_t m_used;   /* Krylov dimension actually used (< m after an invariant subspace) */
  int32_t status;   /* QK_OK or QK_ENUMERIC for this problem */
  double err_est;   /* a-posteriori estimate ||psi|| beta_m |[exp(-i dt T)]_{m,1}| */
  double beta0;     /* ||psi|| at the start of the step */
} qk_step_info;

typedef struct qk_krylov qk_krylov;

/*
 * Workspace for Krylov steps of dimension m (1 <= m <= QK_MAX_M) on
 * Hamiltonian H (Sec. 2 "Krylov subspace methods"): m device vectors of
 * D x batch elements of `dtype`, the Lanczos coefficients and the reduction
 * scratch.  reorth: 0 = none (plain three-term recurrence), 1 = local (each
 * new vector is also orthogonalised against v_{j-1}, the alpha term having
 * removed v_j; the dot product is accumulated in double; one extra vector
 * read per iteration), 2 = full (classical Gram-Schmidt applied twice against
 * all previous vectors, dot products and coefficients in double; about
 * 4 (j + 2) extra vector reads at iteration j).  The Hamiltonian must outlive
 * the workspace.
 */
qk_status qk_krylov_create(const qk_ham* H, int32_t m, int32_t dtype, int32_t reorth, qk_krylov** out);

/*
 * One step psi <- exp(-i dt H) psi for every batch item (Sec. 2: psi(t) ~
 * ||psi|| V_m exp(-i dt A_m) e_1 with A_m the projection of H on the Krylov
 * space of psi, built here by the Lanczos recurrence since H is Hermitian).
 * psi is a [D][B] device array of the workspace dtype, updated in place.
 * When the recurrence reaches an invariant subspace it stops early
 * (m_used < m; the result is then exact up to rounding) -- not an error.
 * info_host (NULL or an array of B entries) is filled after the step has
 * completed, which makes the call synchronous; with info_host == NULL the
 * call returns after enqueueing.  Errors: QK_EINVAL (dt not finite, NULL
 * psi), QK_ENUMERIC (only reported when info_host != NULL), QK_EHIP.
 */
qk_status qk_krylov_expm_step(qk_krylov* k, void* psi, double dt, void* stream, qk_step_info* info_host);

/*
 * Adaptive evolution psi <- exp(-i t H) psi with error control, as in the
 * paper's runs (Sec. 4-5 use Expokit / SLEPc's Krylov exponential with a
 * tolerance): each step builds the Krylov basis once, then the device picks
 * the longest step tau <= min(dt_try, dt_max, time left) whose a-posteriori
 * estimate ||psi|| beta_m |[exp(-i tau T_m)]_{m,1}| is at most 1.2 tau tol,
 * shrinking tau by Expokit's rule 0.9 tau (tau tol / err)^(1/(m-1)) on the
 * small tridiagonal only, and proposes the next dt_try by the same rule
 * (at most 10 tau).  tol is an error per unit time: the summed estimates stay
 * below about tol * t.  All batch items advance by the smallest accepted
 * step.  t >= 0; tol > 0; dt_init > 0 (first trial step); dt_max > 0;
 * max_steps >= 1 bounds the accepted steps (QK_ENUMERIC with a message when
 * t is not reached; psi then holds the state after the last accepted step).
 * Synchronous (one small read-back per step).  info_host
 * (may be NULL) receives the number of steps, the smallest and largest
 * accepted step and the sum of the error estimates of batch item 0.
 */
typedef struct {
  double tol;
  double dt_init;
  double dt_max;
  int32_t max_steps;
} qk_adapt_params;
typedef struct {
  int32_t steps;
  double dt_min, dt_max;
  double err_sum;
} qk_adapt_info;
qk_status qk_krylov_evolve(qk_krylov* k, void* psi, double t, const qk_adapt_params* p, void* stream,
                           qk_adapt_info* info_host);

/*
 * Lanczos coefficients of the last completed step for batch item `item`
 * (synchronous): alpha[0..m_used-1], beta[0..m_used-1] (beta[j] = norm of
 * the (j+1)-th residual), *m_used.  Arrays hold at least m entries.
 */
qk_status qk_krylov_coefficients(const qk_krylov* k, int32_t item, double* alpha, double* beta,
                                 int32_t* m_used);

void qk_krylov_destroy(qk_krylov* k);

/*
 * Per-kernel timing of Krylov steps for benchmarks.  With enable = 1 every
 * later qk_krylov_expm_step records a pair of HIP events on its stream around
 * each kernel launch and the running totals restart from zero; enable = 0
 * stops recording.  qk_krylov_profile_read waits for the recorded events and
 * writes, for each kernel kind below, the summed elapsed milliseconds and the
 * number of launches since profiling was enabled (out has QK_NUM_KERNELS
 * entries).  Kernel kinds: the H-pass of a Lanczos iteration (y = H u fused
 * with the three-term update and its dot products; in the two-pass split of
 * large sectors the high-bond pass), the update pass (new vector and its
 * norm; in the split the low-bond pass that also forms the new vector), the
 * projected exponential, the Krylov combination, and the split's pre-pass
 * over a step's initial vector.
 */
enum { QK_KERNEL_LANCZOS_H = 0, QK_KERNEL_LANCZOS_UPDATE = 1, QK_KERNEL_SMALL_EXPM = 2, QK_KERNEL_COMBINE = 3,
       QK_KERNEL_PREPASS = 4, QK_NUM_KERNELS = 5 };
typedef struct {
  double ms_total;
  int64_t launches;
} qk_kernel_time;

qk_status qk_krylov_profile(qk_krylov* k, int32_t enable);
qk_status qk_krylov_profile_read(qk_krylov* k, qk_kernel_time* out);

/* -------------------------------------------------------- launch shapes */
typedef struct {
  int32_t threads;             /* threads per block of the row-streaming kernels
                                  (rounded down to batch * 2^k); 0 = 256 */
  int32_t blocks_per_cu;       /* blocks per compute unit of the row-streaming kernels; 0 = 4 */
  int32_t blocked_wgs_per_cu;  /* work-groups per compute unit of the blocked H-pass;
                                  0 = as many as fit */
  int32_t blocked_llo;         /* low bits of the block decomposition of the blocked
                                  kernels (matrix-free, 18 <= L <= 32): 9..11 for one
                                  phase; for batches 5..11 with the staged block of B
                                  complex128 phases within 64 KB, the work-group's LDS
                                  within the device limit and at most 2^20 blocks;
                                  0 = keep */
} qk_launch_shape;

/* Sets / reads the launch shape of a workspace's kernels.  Results do not
 * depend on the shape beyond the order of floating-point reductions.  A
 * blocked_llo that differs from the Hamiltonian's rebuilds the Hamiltonian's
 * block tables (synchronous, after all device work): every workspace and
 * batch on that Hamiltonian then uses the new decomposition (batches capture
 * their graph again); no work on the Hamiltonian may be in flight on other
 * threads meanwhile.  QK_EINVAL for an unsupported low-bit count,
 * QK_EUNSUPPORTED for a nonzero one on a Hamiltonian without block tables. */
qk_status qk_krylov_set_shape(qk_krylov* k, const qk_launch_shape* shape);
qk_status qk_krylov_get_shape(const qk_krylov* k, qk_launch_shape* shape);

/*
 * Autotuner: times one step of the workspace (time step dt) for a small set
 * of launch shapes with HIP events on `stream`, on a scratch vector the call
 * allocates and frees, and applies the fastest.  With block tables the search
 * covers the low-bit count of the decomposition (three or four candidates
 * around the default) and the blocked H-pass's work-groups per CU, then the
 * row-streaming shape.  With a non-NULL cache_path
 * the result is looked up first and stored afterwards in that JSON file,
 * keyed by (L, n_up, boundary, batch, mode, dtype, m, reorth, compute units).
 * Synchronous.  *chosen (may be NULL) receives the shape.
 */
qk_status qk_krylov_autotune(qk_krylov* k, double dt, const char* cache_path, void* stream, qk_launch_shape* chosen);

/* ------------------------------------------------------- batched driver */
typedef struct qk_batch qk_batch;

/*
 * Groups n (1..64) distinct workspaces -- any chain lengths, field-set counts
 * and Krylov dimensions, one dtype each -- with their state vectors psi[i]
 * (device, [D_i][B_i], updated in place), so that they advance together.
 * r0[i] >= 0: the items start from the basis state of row r0[i] and their
 * survival probability is |psi[r0]|^2; r0[i] < 0: any initial vectors (for
 * instance the random initial states of Sec. 4's disorder averages) -- the
 * batch copies psi[i] as given now and records |<psi0, psi>|^2.  The handles
 * and vectors must outlive the batch.  Synchronous.
 */
qk_status qk_batch_create(qk_krylov* const* ks, void* const* psi, const int64_t* r0, int32_t n, qk_batch** out);

/* Total number of batch items (sum of the workspaces' field-set counts). */
qk_status qk_batch_items(const qk_batch* b, int32_t* items);

/*
 * n_steps Krylov steps of length dt of every workspace (Sec. 2 "Krylov
 * subspace methods"; the ensembles of Sec. 4 "Quasidisordered systems").
 * After step k the survival probability |psi_i[r0_i]|^2 of every item is
 * written to P_device[k * items + offset_i + item] (offsets in workspace
 * order).  use_graph selects how a step is launched:
 *   0  every kernel of every workspace enqueued directly;
 *   1  one step of all workspaces (one graph branch each) captured into a
 *      hipGraph on first use (again when dt, P_device or a launch shape
 *      change) and replayed n_steps times;
 *   2  one persistent kernel per step that advances all workspaces, records
 *      P and advances C(t) (a work queue of every workspace's passes, each
 *      pass waiting on the previous pass of its workspace), captured into a
 *      hipGraph the same way and replayed n_steps times.  It runs the same
 *      kernel bodies on the same grids as 0 and 1, so all three give the same
 *      bits.  Requires one dtype for all workspaces, L <= 32, no split layout,
 *      reorthogonalisation 0 or 1 and 256-thread row-streaming blocks (the
 *      default shape; a batch of B items needs B a power of two), else
 *      QK_EUNSUPPORTED before anything is enqueued.  Its work queue is built
 *      on first use (device memory from the batch's allocator, kept until
 *      the batch is destroyed or a launch shape changes).
 * Asynchronous.
 */
qk_status qk_batch_run(qk_batch* b, double dt, int32_t n_steps, int32_t use_graph, double* P_device, void* stream);

/*
 * qk_batch_run that also writes the temporal autocorrelation of Sec. 4,
 * C(t) = (1/t) integral_0^t P(t') dt', of every item after step k to
 * C_device[k * items + offset_i + item] (C_device may be NULL).  The integral
 * runs from the creation of the batch over every step taken since (in either
 * entry point), by the trapezoid rule on the step grid; t is the total time
 * stepped.  Asynchronous.
 */
qk_status qk_batch_run_autocorr(qk_batch* b, double dt, int32_t n_steps, int32_t use_graph, double* P_device,
                                double* C_device, void* stream);

void qk_batch_destroy(qk_batch* b);

/* ------------------------------------------------------------- gradient */
/*
 * Survival probability F(T) = |<e_r0| exp(-iHT) |e_r0>|^2 (Sec. 4) and its
 * derivative dF/dh_i with respect to every on-site field h_i of Eq. (1),
 * i = 1..L (dFdh_host[i-1]), by the adjoint method: n_steps Krylov steps of
 * dt = T / n_steps forward with every state kept as a checkpoint, then the
 * costate lambda(s) = exp(+iH(T-s)) e_r0 backward; inside each step the time
 * integral of <lambda|Z_i|psi> is taken between the two Krylov bases by
 * Gauss-Legendre quadrature of the projected propagators.  H and e_r0 are
 * real, so the costate is the conjugated forward state, lambda(s) =
 * conj(psi(T - s)), and the costate's Krylov step from lambda_{k+1} has the
 * conjugated basis and the tridiagonal matrix of the forward step from
 * psi_{n_steps-1-k}: no costate is propagated.  When n_steps Krylov bases of
 * the workspace (n_steps * m vectors) and n_steps + 1 states fit in 80 % of
 * the free device memory, the forward pass keeps every basis with its
 * coefficients and every state for the duration of the call, and the
 * backward pass uses them directly (one Krylov step per time step in all);
 * ckpt_every is then not used.  Otherwise (or with the environment
 * variable QK_GRAD_KEEP=0) the forward states are kept every ckpt_every
 * (>= 1) steps, the backward sweep recomputes the states of one segment from
 * its checkpoint (one extra forward pass in total), rebuilds each basis from
 * its state, and takes the mirrored forward steps again from e_r0 in a
 * second workspace; both ways give identical results.  The call also holds
 * up to n_steps / ckpt_every + ckpt_every + 3 state vectors plus, without
 * kept bases, one more workspace, allocated for its duration.  Uses the
 * workspace's Hamiltonian,
 * Krylov dimension and launch shape.  Requires dtype QK_C128, batch 1 and
 * m <= 32 (else QK_EUNSUPPORTED).  Synchronous; F_host and dFdh_host are host
 * pointers.
 */
qk_status qk_grad_return_prob(qk_krylov* k, int64_t r0, double T, int32_t n_steps, int32_t ckpt_every,
                              double* F_host, double* dFdh_host, void* stream);

/* ----------------------------------------------------------- observable */
/*
 * Survival (return) probability of Sec. 4, F = |<psi0|psi>|^2, for every
 * batch item: P_device[k] (device double array of B entries).  With
 * psi0 == NULL the initial state is the basis state of row r0 and
 * F = |psi[r0]|^2; otherwise psi0 is a [D][B] array of `dtype` and the
 * overlap is reduced in double precision through a small stream-ordered
 * temporary.  Asynchronous, except that with a caller allocator and stream
 * NULL the call waits for its own work before handing the temporary back.
 */
qk_status qk_return_prob(const qk_basis* b, int64_t r0, const void* psi0, const void* psi,
                         int32_t dtype, int32_t batch, double* P_device, void* stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as qk_return_prob, from the same kernels, but the partial sums of
 * the general-state overlap live in a fixed array of the library on each GPU
 * (4 MiB, held until the process ends) instead of a temporary, and the call
 * allocates nothing.  Arguments, ownership and errors are those of
 * qk_return_prob; in addition QK_EINVAL if the overlap's partial sums would
 * exceed the fixed array (never for batch <= QK_MAX_BATCH on up to 4096
 * compute units).  All calls on one GPU share that array: calls that overlap
 * in time on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Asynchronous.
 */
qk_status qk_return_prob_noalloc(const qk_basis* b, int64_t r0, const void* psi0, const void* psi,
                                 int32_t dtype, int32_t batch, double* P_device, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QK_H */

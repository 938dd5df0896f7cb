// Blocked matrix-free H x for large sectors (Sec. 3 "Hamiltonian matrix
// construction", Eq. (1)), used by qk_ham_apply and the H-pass of every
// Lanczos iteration.
//
// A state s splits into its high bits a (sites llo+1..L) and low bits b (sites
// 1..llo).  The sorted basis lists all states with the same a contiguously:
// block a holds rows off(a) .. off(a)+len(a)-1, with len(a) = C(llo, N-|a|),
// and the row of s inside its block is the rank of b among the low states of
// the same popcount.  Therefore
//   * a hop on a bond inside the low bits stays in the block and moves the
//     in-block rank by C(p, #set bits of b below p);
//   * a hop on a bond inside the high bits maps block a onto block a' with
//     the same in-block rank, i.e. a fixed row shift for the whole block;
//   * the bond joining the two halves and the ring bond leave the block and
//     are ranked individually.
// One work-group processes one block at a time: it stages x of the block in
// LDS (the low-bond neighbours are read from there), gathers the high-bond
// neighbours as contiguous runs of the other blocks, and writes the block's
// rows.  Work-groups are persistent and sweep the blocks in ascending order
// together, the whole grid one window of consecutive blocks at a time, so the
// partners of the lower high bonds are being read by the whole chip at the
// same moment and are served from the shared last-level cache.  Inside a
// window, runs of `chunk` consecutive blocks go to one XCD, so the partners
// across the lowest high bonds often share that XCD's L2.  The previous
// Lanczos vector and the result are streamed with non-temporal accesses so
// they do not evict the gathered x from the caches.
#include <hipcub/hipcub.hpp>

#include <cstdlib>
#include <type_traits>

#include "qk_blocked_bodies.h"

namespace qk {


// ------------------------------------------------------------ table build
__global__ void k_lo_tables(int llo, const uint32_t* __restrict__ gtab, BlkArgs ba, uint16_t* __restrict__ lo_state,
                            uint16_t* __restrict__ lo_rank) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (1u << llo)) return;
  const int k = __popc(b);
  const uint32_t j = cns_rank(b, gtab);
  lo_state[ba.lo_base[k] + j] = (uint16_t)b;
  lo_rank[b] = (uint16_t)j;
}

__global__ void k_block_flags(int lhi, int llo, int N, uint32_t* __restrict__ flag) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= (1u << lhi)) return;
  const int k = N - __popc(a);
  flag[a] = (k >= 0 && k <= llo) ? 1u : 0u;
}

// First row of block a: the rank of (a, lowest low state of popcount N-|a|).
__device__ __forceinline__ uint32_t block_offset(uint32_t a, int llo, int N, const uint32_t* tab) {
  const int k = N - __popc(a);
  return cns_rank((a << llo) | ((1u << k) - 1u), tab);
}

__global__ void k_block_fill(int lhi, int llo, int N, const uint32_t* __restrict__ flag,
                             const uint32_t* __restrict__ idx, const uint32_t* __restrict__ gtab,
                             BlkEntry* __restrict__ blk) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= (1u << lhi) || !flag[a]) return;
  BlkEntry e;
  e.a = a;
  e.off = block_offset(a, llo, N, gtab);
  const uint32_t a2 = a ^ (1u << (lhi - 1));
  const int k2 = N - __popc(a2);
  e.offw = (k2 >= 0 && k2 <= llo) ? block_offset(a2, llo, N, gtab) : 0u;
  // A hop on the high bond (llo+t, llo+t+1) moves every row of the block by
  // +-C(llo+t, number of set bits of the state below llo+t).
  const int k_lo = N - __popc(a);
  uint32_t n = 0;
  for (int t = 0; t + 1 < lhi; ++t) {
    const uint32_t b0 = (a >> t) & 1u, b1 = (a >> (t + 1)) & 1u;
    if (b0 != b1) {
      const int pcb = k_lo + __popc(a & ((1u << t) - 1u));
      const int c = (int)gtab[(llo + t) * kBinomStride + pcb];
      e.delta[n++] = b0 ? c : -c;
    }
  }
  e.nact = n;
  for (uint32_t i = n; i < (uint32_t)kMaxHi; ++i) e.delta[i] = 0;
  e.dconst = 0.0;
  e.pad[0] = e.pad[1] = 0u;
  blk[idx[a]] = e;
}

// Block part of the diagonal: jz/4 * (number of bonds) - sum_i h_i / 2 plus
// the fields on the set high bits minus jz/2 per anti-aligned high bond.
__global__ void k_block_consts(int nblk, int llo, int lhi, double zz0, double hhalf, double jz,
                               const double* __restrict__ fields, BlkEntry* __restrict__ blk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblk) return;
  const uint32_t a = blk[i].a;
  double f = 0.0;
  for (int t = 0; t < lhi; ++t)
    if ((a >> t) & 1u) f += fields[llo + t];
  blk[i].dconst = zz0 - hhalf + f - 0.5 * jz * (double)blk[i].nact;
}

qk_status launch_block_consts(BlkEntry* blk, int nblk, int llo, int lhi, double zz0, double hhalf, double jz,
                              const double* fields, hipStream_t s) {
  if (nblk <= 0) return QK_OK;
  hipLaunchKernelGGL(k_block_consts, dim3((nblk + 255) / 256), dim3(256), 0, s, nblk, llo, lhi, zz0, hhalf, jz, fields,
                     blk);
  QK_HIP(hipGetLastError());
  return QK_OK;
}


// --------------------------------------------------------- plain launches
template <typename T, int LLO, bool LANCZOS, bool W64 = false>
__global__ void __launch_bounds__(kBlkThreads, blk_min_blocks<T>())
k_blk(BlkArgs ba, const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y,
      const typename Cx<T>::V* __restrict__ ujm1, KState st, LanczosArgs la, const double* __restrict__ partB, int Gp,
      double* __restrict__ partA) {
  extern __shared__ unsigned char smem[];
  blk_body<T, LLO, LANCZOS, W64>(hw_range(), smem, ba, x, y, ujm1, st, la, partB, Gp, partA);
}

template <typename T, bool LANCZOS>
__global__ void __launch_bounds__(kBlkbThreads)
k_blkb(BlkArgs ba, int B, int lb, const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y,
       const typename Cx<T>::V* __restrict__ ujm1, KState st, LanczosArgs la, const double* __restrict__ partB, int Gp,
       double* __restrict__ partA) {
  extern __shared__ unsigned char smem[];
  blkb_body<T, LANCZOS>(hw_range(), smem, ba, B, lb, x, y, ujm1, st, la, partB, Gp, partA);
}


// ================================================================ launchers
static uint64_t binom_host(int n, int k) {
  if (k < 0 || k > n) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

// Launch-shape tunables (defaults; the autotuner and the environment
// variables QK_BLOCKED_LLO / QK_BLOCKED_WGS_PER_CU override them).
static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  const int x = atoi(v);
  return x > 0 ? x : dflt;
}

int blocked_llo(int L, int N, int B, int mode) {
  (void)N;
  if (mode != QK_MATFREE || L < 18 || L > 32) return 0;   // 32-bit states only
  if (B == 1) {
    int llo = env_int("QK_BLOCKED_LLO", 11);
    if (llo < 9) llo = 9;
    if (llo > 11) llo = 11;
    if (llo > L / 2) llo = L / 2;
    return llo;
  }
  // batches: B a power of two; the largest llo whose biggest block of B
  // complex128 phases fits kBlkbBudget bytes of LDS, with at most 2^20 block
  // entries (128 MB of table)
  if (B < 2 || B > QK_MAX_BATCH || (B & (B - 1)) != 0) return 0;
  for (int llo = (L / 2 < 11 ? L / 2 : 11); llo >= 5; --llo) {
    const uint64_t bytes = binom_host(llo, llo / 2) * (uint64_t)B * 16u;
    if (bytes <= kBlkbBudget && L - llo <= 20) return llo;
  }
  return 0;
}

static BlkArgs blk_args(const qk_ham* H) {
  BlkArgs ba{};
  const qk_basis* b = H->basis;
  ba.L = b->L;
  ba.N = b->N;
  ba.pbc = H->p.pbc;
  ba.llo = H->llo;
  ba.lhi = b->L - H->llo;
  ba.maxlen = (int)binom_host(H->llo, H->llo / 2);
  ba.half_jxy = 0.5 * H->p.jxy;
  ba.jz = H->p.jz;
  ba.zz0 = 0.25 * H->p.jz * (H->p.pbc ? b->L : b->L - 1);
  double hs = 0.0;
  for (int i = 0; i < b->L; ++i) hs += H->h_host[i];
  ba.hhalf = 0.5 * hs;
  ba.blk = (const BlkEntry*)H->d_blk;
  ba.lo_state = H->d_lo_state;
  ba.lo_rank = H->d_lo_rank;
  ba.binom = b->d_binom;
  ba.fields = H->d_fields;
  uint32_t acc = 0;
  for (int k = 0; k <= H->llo; ++k) {
    ba.lo_base[k] = acc;
    acc += (uint32_t)binom_host(H->llo, k);
  }
  ba.nblk = H->nblk;
  ba.chunk_log2 = 0;
  return ba;
}

qk_status launch_blocked_build(qk_ham* H, hipStream_t s) {
  const qk_basis* b = H->basis;
  const int llo = H->llo, lhi = b->L - llo;
  const uint32_t nlo = 1u << llo, nhi = 1u << lhi;
  QK_HIP(dev_alloc(H->al, (void**)&H->d_lo_state, sizeof(uint16_t) * nlo));
  QK_HIP(dev_alloc(H->al, (void**)&H->d_lo_rank, sizeof(uint16_t) * nlo));
  BlkArgs ba = blk_args(H);
  hipLaunchKernelGGL(k_lo_tables, dim3((nlo + 255) / 256), dim3(256), 0, s, llo, b->d_binom, ba, H->d_lo_state,
                     H->d_lo_rank);
  QK_HIP(hipGetLastError());
  uint32_t *flag = nullptr, *idx = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  QK_HIP(dev_alloc(H->al, (void**)&flag, sizeof(uint32_t) * nhi));
  hipError_t e = dev_alloc(H->al, (void**)&idx, sizeof(uint32_t) * nhi);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_block_flags, dim3((nhi + 255) / 256), dim3(256), 0, s, lhi, llo, b->N, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, flag, idx, (int)nhi, s);
  if (e == hipSuccess) e = dev_alloc(H->al, &tmp, tmp_bytes + 16);
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, flag, idx, (int)nhi, s);
  uint32_t last_idx = 0, last_flag = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&last_idx, idx + nhi - 1, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&last_flag, flag + nhi - 1, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    H->nblk = (int)(last_idx + last_flag);
    e = dev_alloc(H->al, (void**)&H->d_blk, sizeof(BlkEntry) * (size_t)(H->nblk > 0 ? H->nblk : 1));
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_block_fill, dim3((nhi + 255) / 256), dim3(256), 0, s, lhi, llo, b->N, flag, idx,
                       b->d_binom, (BlkEntry*)H->d_blk);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_block_consts, dim3((H->nblk + 255) / 256), dim3(256), 0, s, H->nblk, llo, lhi, ba.zz0,
                       ba.hhalf, ba.jz, H->d_fields, (BlkEntry*)H->d_blk);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  else (void)hipStreamSynchronize(s);   // nothing queued may still use the temporaries
  dev_free(H->al, tmp);
  dev_free(H->al, flag);
  dev_free(H->al, idx);
  QK_HIP(e);
  return QK_OK;
}

qk_status launch_blocked_fields(qk_ham* H, hipStream_t s) {
  const BlkArgs ba = blk_args(H);
  hipLaunchKernelGGL(k_block_consts, dim3((H->nblk + 255) / 256), dim3(256), 0, s, H->nblk, ba.llo, ba.lhi, ba.zz0,
                     ba.hhalf, ba.jz, H->d_fields, (BlkEntry*)H->d_blk);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

bool blocked_llo_valid(const qk_ham* H, int llo) {
  const int L = H->basis->L, B = H->batch;
  if (H->llo <= 0 || H->p.mode != QK_MATFREE || L < 18 || L > 32 || llo > L / 2) return false;
  if (B == 1) return llo >= 9 && llo <= 11;
  if (llo < 5 || llo > 11 || L - llo > 20 || binom_host(llo, llo / 2) * (uint64_t)B * 16u > 65536u) return false;
  // the batched kernel's dynamic LDS (staged block of B complex128 phases,
  // low tables, fields) must fit one work-group
  const size_t dyn = blkb_smem_bytes((uint32_t)binom_host(llo, llo / 2), B, 16, llo, L);
  int lim = 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, H->device) != hipSuccess) return false;
  return dyn <= (size_t)lim;
}

qk_status blocked_rebuild(qk_ham* H, int llo) {
  if (!blocked_llo_valid(H, llo)) {
    set_error("unsupported low-bit count for this Hamiltonian's block decomposition");
    return QK_EINVAL;
  }
  if (llo == H->llo) return QK_OK;
  QK_HIP(hipDeviceSynchronize());   // no queued kernel may still read the old tables
  const int old = H->llo;
  auto drop = [&]() {
    dev_free(H->al, H->d_lo_state);
    dev_free(H->al, H->d_lo_rank);
    dev_free(H->al, H->d_blk);
    H->d_lo_state = nullptr;
    H->d_lo_rank = nullptr;
    H->d_blk = nullptr;
    H->nblk = 0;
  };
  drop();
  H->llo = llo;
  ++H->tables_gen;
  qk_status st = launch_blocked_build(H, nullptr);
  if (st != QK_OK) {
    // back to the previous decomposition, or to the row-form kernels
    drop();
    H->llo = old;
    if (launch_blocked_build(H, nullptr) != QK_OK) {
      drop();
      H->llo = 0;
    }
  }
  return st;
}

bool blocked_usable(const qk_ham* H, int dtype) {
  // the single-phase kernel addresses vectors below 4 GB with 32-bit byte
  // offsets and larger ones (11 low bits) with 64-bit element offsets
  const uint64_t bytes = (uint64_t)H->basis->D * (dtype == QK_C128 ? 16u : 8u);
  return H->llo > 0 && (H->batch > 1 || bytes < (1ull << 32) || H->llo == 11);
}

// Work-groups of a blocked launch: `wgs` per CU (at most what the kernel can
// hold), at most one per kMinBlockWork elements of the vector, rounded to a
// multiple of the XCD count, and the chunk of consecutive blocks per XCD: 8,
// or the largest power of two dividing the work-groups per XCD.
static int blocked_grid(const qk_ham* H, int occ, int wgs_req, int* chunk_log2) {
  const int cus = qk_num_cus();
  int wgs = wgs_req > 0 ? wgs_req : env_int("QK_BLOCKED_WGS_PER_CU", occ);
  if (wgs > occ) wgs = occ;
  int G = ((cus * wgs) / kNumXcd) * kNumXcd;
  const uint64_t wcap = ((uint64_t)H->basis->D * H->batch + kMinBlockWork - 1) / kMinBlockWork;
  if ((uint64_t)G > wcap) G = (int)(((wcap + kNumXcd - 1) / kNumXcd) * kNumXcd);
  if (G < kNumXcd) G = kNumXcd;
  if (G > kMaxPartialBlocks) G = kMaxPartialBlocks;
  int cl = 3;
  while (cl > 0 && (G / kNumXcd) % (1 << cl) != 0) --cl;
  *chunk_log2 = cl;
  return G;
}

template <typename T, bool LANCZOS>
static void plan_blkb(const qk_ham* H, int wgs_req, BlkPlan* p) {
  using V = typename Cx<T>::V;
  p->ba = blk_args(H);
  const int B = H->batch;
  p->lb = 0;
  while ((1 << p->lb) < B) ++p->lb;
  p->smem = blkb_smem_bytes((uint32_t)p->ba.maxlen, B, sizeof(V), p->ba.llo, p->ba.L);
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_blkb<T, LANCZOS>, kBlkbThreads, p->smem) != hipSuccess ||
      occ < 1)
    occ = 1;
  p->G = blocked_grid(H, occ, wgs_req, &p->ba.chunk_log2);
  p->llo = 0;
  p->w64 = false;
}

template <typename T, int LLO, bool LANCZOS, bool W64>
static void plan_blk(const qk_ham* H, int wgs_req, BlkPlan* p) {
  p->ba = blk_args(H);
  p->smem = blk_smem_bytes<T, LLO>();
  // work-groups per CU the kernel can hold (queried once per instantiation; thread-safe static init)
  static const int occ = [&]() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blk<T, LLO, LANCZOS, W64>, kBlkThreads,
                                                     blk_smem_bytes<T, LLO>()) !=
            hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  p->G = blocked_grid(H, occ, wgs_req, &p->ba.chunk_log2);
  p->lb = 0;
  p->llo = LLO;
  p->w64 = W64;
}

template <typename T, bool LANCZOS>
static qk_status launch_blkb_t(const qk_ham* H, const void* x, void* y, const void* ujm1, const KState* st,
                               const LanczosArgs* la, const double* partB, int Gp, double* partA, int* grid_out,
                               int wgs_req, hipStream_t s) {
  using V = typename Cx<T>::V;
  BlkPlan p;
  plan_blkb<T, LANCZOS>(H, wgs_req, &p);
  KState stv{};
  LanczosArgs lav{};
  if (st) stv = *st;
  if (la) lav = *la;
  hipLaunchKernelGGL((k_blkb<T, LANCZOS>), dim3(p.G), dim3(kBlkbThreads), p.smem, s, p.ba, H->batch, p.lb,
                     (const V*)x, (V*)y, (const V*)ujm1, stv, lav, partB, Gp, partA);
  QK_HIP(hipGetLastError());
  if (grid_out) *grid_out = p.G;
  return QK_OK;
}

template <typename T, int LLO, bool LANCZOS, bool W64>
static qk_status launch_blk_k(const qk_ham* H, const void* x, void* y, const void* ujm1, const KState* st,
                              const LanczosArgs* la, const double* partB, int Gp, double* partA, int* grid_out,
                              int wgs_req, hipStream_t s) {
  using V = typename Cx<T>::V;
  BlkPlan p;
  plan_blk<T, LLO, LANCZOS, W64>(H, wgs_req, &p);
  KState stv{};
  LanczosArgs lav{};
  if (st) stv = *st;
  if (la) lav = *la;
  hipLaunchKernelGGL((k_blk<T, LLO, LANCZOS, W64>), dim3(p.G), dim3(kBlkThreads), p.smem, s, p.ba, (const V*)x,
                     (V*)y, (const V*)ujm1, stv, lav, partB, Gp, partA);
  QK_HIP(hipGetLastError());
  if (grid_out) *grid_out = p.G;
  return QK_OK;
}

// Vectors of 4 GB or more (the half-filled L = 32 chain) take 64-bit element
// offsets; they always have 11 low bits (L >= 22).  QK_BLOCKED_W64=1 selects
// the 64-bit form for smaller vectors too (same arithmetic, so the same bits).
template <typename T, int LLO, bool LANCZOS>
static qk_status launch_blk_t(const qk_ham* H, const void* x, void* y, const void* ujm1, const KState* st,
                              const LanczosArgs* la, const double* partB, int Gp, double* partA, int* grid_out,
                              int wgs_req, hipStream_t s) {
  using V = typename Cx<T>::V;
  const char* fw = getenv("QK_BLOCKED_W64");
  const bool force = fw && fw[0] == '1' && LLO == 11;
  if ((uint64_t)H->basis->D * sizeof(V) < (1ull << 32) && !force)
    return launch_blk_k<T, LLO, LANCZOS, false>(H, x, y, ujm1, st, la, partB, Gp, partA, grid_out, wgs_req, s);
  if constexpr (LLO == 11)
    return launch_blk_k<T, LLO, LANCZOS, true>(H, x, y, ujm1, st, la, partB, Gp, partA, grid_out, wgs_req, s);
  set_error("vectors of 4 GB or more need the 11-bit block decomposition");
  return QK_EUNSUPPORTED;
}

template <typename T, bool LANCZOS>
static qk_status launch_blk_llo(const qk_ham* H, const void* x, void* y, const void* ujm1, const KState* st,
                                const LanczosArgs* la, const double* partB, int Gp, double* partA, int* grid_out,
                                int wgs, hipStream_t s) {
  switch (H->llo) {
    case 9: return launch_blk_t<T, 9, LANCZOS>(H, x, y, ujm1, st, la, partB, Gp, partA, grid_out, wgs, s);
    case 10: return launch_blk_t<T, 10, LANCZOS>(H, x, y, ujm1, st, la, partB, Gp, partA, grid_out, wgs, s);
    case 11: return launch_blk_t<T, 11, LANCZOS>(H, x, y, ujm1, st, la, partB, Gp, partA, grid_out, wgs, s);
    default: set_error("no blocked kernel for this low-bit count"); return QK_EUNSUPPORTED;
  }
}

// The launch plan of the blocked Lanczos H-pass that launch_blocked_lanczos_h
// would use for this workspace shape (kernel, arguments, grid, LDS).
qk_status blocked_lanczos_plan(const qk_ham* H, int dtype, int wgs_req, BlkPlan* p) {
  if (!blocked_usable(H, dtype)) {
    set_error("no blocked H-pass for this Hamiltonian");
    return QK_EUNSUPPORTED;
  }
  if (H->batch > 1) {
    if (dtype == QK_C128) plan_blkb<double, true>(H, wgs_req, p);
    else plan_blkb<float, true>(H, wgs_req, p);
    return QK_OK;
  }
  const bool w64 = (uint64_t)H->basis->D * (dtype == QK_C128 ? 16u : 8u) >= (1ull << 32) ||
                   (getenv("QK_BLOCKED_W64") && getenv("QK_BLOCKED_W64")[0] == '1' && H->llo == 11);
  if (w64) {
    set_error("the persistent step does not take vectors of 4 GB or more");
    return QK_EUNSUPPORTED;
  }
  switch (H->llo * 2 + (dtype == QK_C128 ? 1 : 0)) {
    case 18: plan_blk<float, 9, true, false>(H, wgs_req, p); return QK_OK;
    case 19: plan_blk<double, 9, true, false>(H, wgs_req, p); return QK_OK;
    case 20: plan_blk<float, 10, true, false>(H, wgs_req, p); return QK_OK;
    case 21: plan_blk<double, 10, true, false>(H, wgs_req, p); return QK_OK;
    case 22: plan_blk<float, 11, true, false>(H, wgs_req, p); return QK_OK;
    case 23: plan_blk<double, 11, true, false>(H, wgs_req, p); return QK_OK;
    default: set_error("no blocked kernel for this low-bit count"); return QK_EUNSUPPORTED;
  }
}

qk_status launch_blocked_apply(const qk_ham* H, const void* x, void* y, int dtype, hipStream_t s) {
  if (H->batch > 1) {
    if (dtype == QK_C128)
      return launch_blkb_t<double, false>(H, x, y, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, s);
    return launch_blkb_t<float, false>(H, x, y, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, s);
  }
  if (dtype == QK_C128)
    return launch_blk_llo<double, false>(H, x, y, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, s);
  return launch_blk_llo<float, false>(H, x, y, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, s);
}

qk_status launch_blocked_lanczos_h(const qk_ham* H, int dtype, const void* uj, const void* ujm1, void* w,
                                   const KState& st, const LanczosArgs& la, const double* partB, int Gp,
                                   double* partA, int* grid_out, int wgs_per_cu, hipStream_t s) {
  if (H->batch > 1) {
    if (dtype == QK_C128)
      return launch_blkb_t<double, true>(H, uj, w, ujm1, &st, &la, partB, Gp, partA, grid_out, wgs_per_cu, s);
    return launch_blkb_t<float, true>(H, uj, w, ujm1, &st, &la, partB, Gp, partA, grid_out, wgs_per_cu, s);
  }
  if (dtype == QK_C128)
    return launch_blk_llo<double, true>(H, uj, w, ujm1, &st, &la, partB, Gp, partA, grid_out, wgs_per_cu, s);
  return launch_blk_llo<float, true>(H, uj, w, ujm1, &st, &la, partB, Gp, partA, grid_out, wgs_per_cu, s);
}

}  // namespace qk

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

#include "qk_blocked.h"

namespace qk {

struct BlkArgs {
  int L, N, pbc, llo, lhi, maxlen;
  double half_jxy, jz, zz0, hhalf;         // zz0 = jz/4 * (number of bonds), hhalf = sum_i h_i / 2
  const BlkEntry* blk;
  const uint16_t* lo_state;                // [2^llo] low states grouped by popcount, ascending
  const uint16_t* lo_rank;                 // [2^llo] rank of a low state inside its popcount group
  const uint32_t* binom;                   // [33*33]
  const double* fields;                    // [L]
  uint32_t lo_base[18];                    // first index of each popcount group in lo_state
  int nblk;                                // number of blocks
  int chunk_log2;                          // log2 of the consecutive blocks per XCD in a window
};

constexpr int kBlkThreads = 256;

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

// --------------------------------------------------------- blocked rows
// Largest block, C(LLO, LLO/2) rows.
template <int LLO>
constexpr int blk_max_len() {
  return LLO == 9 ? 126 : LLO == 10 ? 252 : 462;
}

// Bytes of the two x buffers at the start of dynamic LDS; at least the
// kQA x 256 doubles of the reductions that alias them.
template <typename T, int LLO>
constexpr size_t blk_xbytes() {
  constexpr size_t b = sizeof(typename Cx<T>::V) * 2 * (size_t)blk_max_len<LLO>();
  return b > kQA * kBlkThreads * sizeof(double) ? b : kQA * kBlkThreads * sizeof(double);
}

// Element idx of a vector from a uniform base: through a 32-bit byte offset
// (the common case, D * sizeof(V) < 2^32: one VGPR per address), or through
// a 64-bit element offset for larger vectors (W64).
template <bool W64, typename V>
__device__ __forceinline__ const V* elem(const V* base, uint32_t idx) {
  if (W64) return base + (size_t)idx;
  return reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(V));
}
template <bool W64, typename V>
__device__ __forceinline__ V* elem(V* base, uint32_t idx) {
  if (W64) return base + (size_t)idx;
  return reinterpret_cast<V*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(V));
}
template <typename V, bool W64 = false>
__device__ __forceinline__ V ld32(const V* __restrict__ base, uint32_t idx) {
  return *elem<W64>(base, idx);
}
// Non-temporal forms, for data read or written once per pass.
template <typename V, bool W64 = false>
__device__ __forceinline__ V ld32_stream(const V* __restrict__ base, uint32_t idx) {
  using S = decltype(V{}.x);
  typedef S E __attribute__((ext_vector_type(2)));
  const E* p = reinterpret_cast<const E*>(elem<W64>(base, idx));
  const E e = __builtin_nontemporal_load(p);
  return V{e.x, e.y};
}
template <typename V, bool W64 = false>
__device__ __forceinline__ void st32_stream(V* __restrict__ base, uint32_t idx, V v) {
  using S = decltype(V{}.x);
  typedef S E __attribute__((ext_vector_type(2)));
  E* p = reinterpret_cast<E*>(elem<W64>(base, idx));
  const E e = {v.x, v.y};
  __builtin_nontemporal_store(e, p);
}

// LLO low bits (compile-time, so the low-bond loop unrolls).  LANCZOS:
// w = sa * H u_j - sb * u_{j-1} with the dot-product partials of the H-pass;
// otherwise y = H x.  The x values of the next block are loaded into
// registers after the current block's rows and stored into the second LDS
// buffer before the block's barrier (one barrier per block); loading them
// this late rather than at the start of the block keeps them closer in time
// to the neighbouring work-groups' gathers of the same block (1 % faster).
// complex64 rows fit six work-groups per CU in 80 registers (measured 4 %
// faster); complex128 keeps its registers (a cap would spill).
template <typename T>
constexpr int blk_min_blocks() {
  return std::is_same<T, float>::value ? 6 : 1;
}

template <typename T, int LLO, bool LANCZOS, bool W64 = false>
__global__ void __launch_bounds__(kBlkThreads, blk_min_blocks<T>())
k_blk(BlkArgs ba, const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y,
      const typename Cx<T>::V* __restrict__ ujm1, KState st, LanczosArgs la, const double* __restrict__ partB, int Gp,
      double* __restrict__ partA) {
  using V = typename Cx<T>::V;
  constexpr int kMaxLen = blk_max_len<LLO>();
  static_assert(kMaxLen <= 2 * kBlkThreads, "prefetch covers two elements per thread");
  extern __shared__ unsigned char smem[];
  V* xsb = reinterpret_cast<V*>(smem);                                            // [2][kMaxLen]
  uint16_t* lo_state = reinterpret_cast<uint16_t*>(smem + blk_xbytes<T, LLO>());
  uint16_t* lo_rank = lo_state + (1 << LLO);
  __shared__ uint32_t sbin[kBinomStride * kBinomStride];
  __shared__ double flo0[256], flo1[256];
  __shared__ double fld[StateT<uint32_t>::kMaxL];
  __shared__ double tot[1], sa[1], sb[1];
  __shared__ int act[1];
  __shared__ int hds[2][kMaxHi];   // row shifts of the current and the next block
  double* red = reinterpret_cast<double*>(smem);   // aliases the x buffers outside the block loop

  const int tid = threadIdx.x;
  for (int i = tid; i < kBinomStride * kBinomStride; i += kBlkThreads) sbin[i] = ba.binom[i];
  for (int i = tid; i < (1 << LLO); i += kBlkThreads) {
    lo_state[i] = ba.lo_state[i];
    lo_rank[i] = ba.lo_rank[i];
  }
  if (tid < ba.L) fld[tid] = ba.fields[tid];
  __syncthreads();
  {
    // field sums over the low bits, eight bits per table (kBlkThreads == 256 entries)
    const int c = tid;
    double f0 = 0.0, f1 = 0.0;
    for (int i = 0; i < 8; ++i) {
      if ((c >> i) & 1) {
        if (i < LLO) f0 += fld[i];
        if (8 + i < LLO) f1 += fld[8 + i];
      }
    }
    flo0[c] = f0;
    flo1[c] = f1;
  }
  if (LANCZOS) {
    lanczos_h_scalars(1, st, la, partB, Gp, red, tot, sa, sb, act);
  } else {
    if (tid == 0) {
      sa[0] = 1.0;
      sb[0] = 0.0;
      act[0] = 1;
    }
    __syncthreads();
  }
  const T g = (T)ba.half_jxy;
  const double hjz = 0.5 * ba.jz;
  const T ca = (T)sa[0], cb = (T)sb[0];
  const bool prev = LANCZOS && la.j > 0;
  double s1 = 0.0, s2 = 0.0, s3r = 0.0, s3i = 0.0;
  const int lhi = ba.lhi;
  // work-group w runs on XCD w % 8; in every window of gridDim.x blocks the
  // XCD takes chunks of 2^chunk_log2 consecutive blocks (the launcher makes
  // gridDim.x / 8 a multiple of the chunk)
  const int xcd = blockIdx.x % kNumXcd, kx = blockIdx.x / kNumXcd;
  const int cl = ba.chunk_log2;
  const int per = (int)gridDim.x, last = ba.nblk;
  int bi = ((((kx >> cl) * kNumXcd) + xcd) << cl) + (kx & ((1 << cl) - 1));
  const bool run = act[0] != 0;
  __syncthreads();   // `red` (aliasing the x buffers) is no longer read

  if (run && bi < last) {
    const BlkEntry* ep = ba.blk + bi;
    const uint32_t len = sbin[LLO * kBinomStride + (ba.N - __popc(ep->a))];
    const uint32_t off = ep->off;
    for (uint32_t i = tid; i < len; i += kBlkThreads) xsb[i] = ld32<V, W64>(x, off + i);
    if (tid < kMaxHi) hds[0][tid] = ep->delta[tid];
  }
  __syncthreads();
  int cur = 0;
  for (; run && bi < last; bi += per) {
    const BlkEntry* ep = ba.blk + bi;
    const uint32_t a = ep->a, off = ep->off, offw = ep->offw;
    const int nact = (int)ep->nact;
    const double dconst = ep->dconst;
    const int k_lo = ba.N - __popc(a);
    const uint32_t len = sbin[LLO * kBinomStride + k_lo];
    const uint32_t base = ba.lo_base[k_lo];
    const V* xs = xsb + cur * kMaxLen;
    // next block: its x values, loaded and stored after the rows
    const int nbi = bi + per;
    const bool has_next = nbi < last;
    uint32_t nlen = 0;
    V p0 = {0, 0}, p1 = {0, 0};
    int nd = 0;
    const int* hd = hds[cur];
    const uint32_t top = (a >> (lhi - 1)) & 1u;
    for (uint32_t j = tid; j < len; j += kBlkThreads) {
      const uint32_t b = lo_state[base + j];
      const uint32_t r = off + j;
      // global gathers first, so that their latencies overlap: the previous
      // Lanczos vector, the bond joining the halves and the ring bond.  Lanes
      // whose bond is inactive issue no load (their value stays zero), so they
      // add no cache lines to the wave's request.
      const V z = {0, 0};
      V um = z;
      if (prev) um = ld32_stream<V, W64>(ujm1, r);
      const uint32_t bl = (b >> (LLO - 1)) & 1u;
      const bool cx = (bl ^ (a & 1u)) != 0u;
      const uint32_t pcl = (uint32_t)__popc(b & ((1u << (LLO - 1)) - 1u));
      const uint32_t cc = sbin[(LLO - 1) * kBinomStride + pcl];
      V vc = z;
      if (cx) vc = ld32<V, W64>(x, bl ? r + cc : r - cc);
      const bool wx = ba.pbc && ((b & 1u) != top);
      V vw = z;
      if (wx) vw = ld32<V, W64>(x, offw + lo_rank[b ^ 1u]);
      // high bonds: uniform row shifts, contiguous runs of the partner blocks,
      // four loads at a time; slots beyond the block's active bonds are skipped
      // by a uniform test and contribute zero.  The first group is issued
      // before the in-block LDS work and consumed after it.
      const V q0 = (0 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[0]) : z;
      const V q1 = (1 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[1]) : z;
      const V q2 = (2 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[2]) : z;
      const V q3 = (3 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[3]) : z;
      // in-block work from LDS
      const V xr = xs[j];
      const int anti = __popc((b ^ (b >> 1)) & ((1u << (LLO - 1)) - 1u)) + (cx ? 1 : 0) + (wx ? 1 : 0);
      const double d = dconst + flo0[b & 255u] + flo1[b >> 8] - hjz * anti;
      V hs = {0, 0};
      int pc = 0;
#pragma unroll
      for (int p = 0; p < LLO - 1; ++p) {
        const uint32_t b0 = (b >> p) & 1u, b1 = (b >> (p + 1)) & 1u;
        if (b0 != b1) {
          const uint32_t c = sbin[p * kBinomStride + pc];
          const V v = xs[b0 ? j + c : j - c];
          hs.x += v.x;
          hs.y += v.y;
        }
        pc += (int)b0;
      }
      {
        const T w0 = (0 < nact) ? (T)1 : (T)0, w1 = (1 < nact) ? (T)1 : (T)0;
        const T w2 = (2 < nact) ? (T)1 : (T)0, w3 = (3 < nact) ? (T)1 : (T)0;
        hs.x += w0 * q0.x + w1 * q1.x + w2 * q2.x + w3 * q3.x;
        hs.y += w0 * q0.y + w1 * q1.y + w2 * q2.y + w3 * q3.y;
      }
      for (int g0 = 4; g0 < nact; g0 += 4) {
        const V v0 = ld32<V, W64>(x, r + (uint32_t)hd[g0]);
        const V v1 = (g0 + 1 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[g0 + 1]) : z;
        const V v2 = (g0 + 2 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[g0 + 2]) : z;
        const V v3 = (g0 + 3 < nact) ? ld32<V, W64>(x, r + (uint32_t)hd[g0 + 3]) : z;
        const T w1 = (g0 + 1 < nact) ? (T)1 : (T)0;
        const T w2 = (g0 + 2 < nact) ? (T)1 : (T)0;
        const T w3 = (g0 + 3 < nact) ? (T)1 : (T)0;
        hs.x += v0.x + w1 * v1.x + w2 * v2.x + w3 * v3.x;
        hs.y += v0.y + w1 * v1.y + w2 * v2.y + w3 * v3.y;
      }
      hs.x += (cx ? vc.x : (T)0) + (wx ? vw.x : (T)0);
      hs.y += (cx ? vc.y : (T)0) + (wx ? vw.y : (T)0);
      V h;
      h.x = (T)d * xr.x + g * hs.x;
      h.y = (T)d * xr.y + g * hs.y;
      if (LANCZOS) {
        V wv;
        wv.x = ca * h.x - cb * um.x;
        wv.y = ca * h.y - cb * um.y;
        st32_stream<V, W64>(y, r, wv);
        s1 += (double)xr.x * (double)wv.x + (double)xr.y * (double)wv.y;
        s2 += (double)xr.x * (double)xr.x + (double)xr.y * (double)xr.y;
        s3r += (double)um.x * (double)wv.x + (double)um.y * (double)wv.y;
        s3i += (double)um.x * (double)wv.y - (double)um.y * (double)wv.x;
      } else {
        st32_stream<V, W64>(y, r, h);
      }
    }
    if (has_next) {
      const BlkEntry* en = ba.blk + nbi;
      nlen = sbin[LLO * kBinomStride + (ba.N - __popc(en->a))];
      const uint32_t noff = en->off;
      if ((uint32_t)tid < nlen) p0 = ld32<V, W64>(x, noff + tid);
      if ((uint32_t)tid + kBlkThreads < nlen) p1 = ld32<V, W64>(x, noff + tid + kBlkThreads);
      if (tid < kMaxHi) nd = en->delta[tid];
    }
    if (has_next) {
      V* xn = xsb + (cur ^ 1) * kMaxLen;
      if ((uint32_t)tid < nlen) xn[tid] = p0;
      if ((uint32_t)tid + kBlkThreads < nlen) xn[tid + kBlkThreads] = p1;
      if (tid < kMaxHi) hds[cur ^ 1][tid] = nd;
    }
    __syncthreads();
    cur ^= 1;
  }
  if (LANCZOS) {
    double v[kQA] = {s1, s2, s3r, s3i};
    block_partials<kQA>(v, 1, red, partA + (size_t)blockIdx.x * kQA);
  }
}

// ------------------------------------------------ blocked rows, batched
// The same decomposition for B > 1 phases in the [D][B] layout (B a power of
// two): element e = j * B + b of a block is row j, phase b, so a gather of a
// partner run reads B consecutive values per row.  The fields differ per
// phase, so the diagonal is assembled per element from the phase's fields in
// LDS (the block table's constant holds phase 0 only and is not used here).
// llo is a runtime value chosen so that one block of B phases fits the LDS
// buffer; the block is staged once (no double buffer).  Each thread keeps the
// phase tid % B for the whole kernel.  The previous Lanczos vector and the
// result are streamed with non-temporal accesses, as in the one-phase kernel.
constexpr int kBlkbThreads = 256;
constexpr uint64_t kBlkbBudget = 32768;   // LDS bytes of one staged block of B phases (complex128)

__host__ __device__ inline size_t blkb_xbytes(uint32_t maxlen, int B, size_t vbytes) {
  const size_t b = (size_t)maxlen * B * vbytes;
  const size_t r = (size_t)kQA * kBlkbThreads * sizeof(double);
  return ((b > r ? b : r) + 15) & ~(size_t)15;
}

template <typename T, bool LANCZOS>
__global__ void __launch_bounds__(kBlkbThreads)
k_blkb(BlkArgs ba, int B, int lb, const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y,
       const typename Cx<T>::V* __restrict__ ujm1, KState st, LanczosArgs la, const double* __restrict__ partB, int Gp,
       double* __restrict__ partA) {
  using V = typename Cx<T>::V;
  extern __shared__ unsigned char smem[];
  const int llo = ba.llo, L = ba.L, lhi = ba.lhi;
  V* xs = reinterpret_cast<V*>(smem);
  const size_t xb = blkb_xbytes((uint32_t)ba.maxlen, B, sizeof(V));
  uint16_t* lo_state = reinterpret_cast<uint16_t*>(smem + xb);
  uint16_t* lo_rank = lo_state + (1 << llo);
  double* fld = reinterpret_cast<double*>(smem + xb + (((size_t)4 << llo) + 15 & ~(size_t)15));   // [B][L]
  double* hic = fld + (size_t)B * L;   // per phase: block constant of the diagonal
  double* hh = hic + B;                // per phase: sum of the fields / 2
  __shared__ uint32_t sbin[kBinomStride * kBinomStride];
  __shared__ double tot[QK_MAX_BATCH], sa[QK_MAX_BATCH], sb[QK_MAX_BATCH];
  __shared__ int act[QK_MAX_BATCH];
  double* red = reinterpret_cast<double*>(smem);   // aliases xs outside the block loop

  const int tid = threadIdx.x;
  for (int i = tid; i < kBinomStride * kBinomStride; i += kBlkbThreads) sbin[i] = ba.binom[i];
  for (int i = tid; i < (1 << llo); i += kBlkbThreads) {
    lo_state[i] = ba.lo_state[i];
    lo_rank[i] = ba.lo_rank[i];
  }
  for (int i = tid; i < B * L; i += kBlkbThreads) fld[i] = ba.fields[i];
  __syncthreads();
  for (int b = tid; b < B; b += kBlkbThreads) {
    double f = 0.0;
    for (int i = 0; i < L; ++i) f += fld[b * L + i];
    hh[b] = 0.5 * f;
  }
  if (LANCZOS) {
    lanczos_h_scalars(B, st, la, partB, Gp, red, tot, sa, sb, act);
  } else {
    for (int b = tid; b < B; b += kBlkbThreads) {
      sa[b] = 1.0;
      sb[b] = 0.0;
      act[b] = 1;
    }
    __syncthreads();
  }
  const int bc = tid & (B - 1);   // this thread's phase
  const bool mine = act[bc] != 0;
  const T g = (T)ba.half_jxy;
  const double hjz = 0.5 * ba.jz;
  const T ca = (T)sa[bc], cb = (T)sb[bc];
  const bool prev = LANCZOS && la.j > 0;
  const double* fb = fld + (size_t)bc * L;
  double s1 = 0.0, s2 = 0.0, s3r = 0.0, s3i = 0.0;
  const int xcd = blockIdx.x % kNumXcd, kx = blockIdx.x / kNumXcd;
  const int cl = ba.chunk_log2;
  const int last = ba.nblk;
  int bi = ((((kx >> cl) * kNumXcd) + xcd) << cl) + (kx & ((1 << cl) - 1));
  __syncthreads();   // `red` (aliasing xs) is no longer read

  for (; bi < last; bi += (int)gridDim.x) {
    const BlkEntry* ep = ba.blk + bi;
    const uint32_t a = ep->a, off = ep->off, offw = ep->offw;
    const int nact = (int)ep->nact;
    const int k_lo = ba.N - __popc(a);
    const uint32_t len = sbin[llo * kBinomStride + k_lo];
    const uint32_t base = ba.lo_base[k_lo];
    const uint32_t nel = len << lb;
    const size_t eoff = (size_t)off << lb;
    for (uint32_t e = tid; e < nel; e += kBlkbThreads) xs[e] = x[eoff + e];
    if (tid < B) {
      double f = ba.zz0 - 0.5 * ba.jz * (double)nact - hh[tid];
      for (int t = 0; t < lhi; ++t)
        if ((a >> t) & 1u) f += fld[tid * L + llo + t];
      hic[tid] = f;
    }
    __syncthreads();
    const uint32_t top = (a >> (lhi - 1)) & 1u;
    const double dblk = hic[bc];
    if (mine) {
      for (uint32_t e = tid; e < nel; e += kBlkbThreads) {
        const uint32_t j = e >> lb;
        const uint32_t bs = lo_state[base + j];
        const uint32_t r = off + j;
        V um = {0, 0};
        if (prev) um = ld32_stream(ujm1 + ((size_t)r << lb), bc);
        const uint32_t bl = (bs >> (llo - 1)) & 1u;
        const bool cx = (bl ^ (a & 1u)) != 0u;
        const uint32_t pcl = (uint32_t)__popc(bs & ((1u << (llo - 1)) - 1u));
        const uint32_t cc = sbin[(llo - 1) * kBinomStride + pcl];
        const uint32_t rc = cx ? (bl ? r + cc : r - cc) : r;
        const V vc = x[((size_t)rc << lb) + bc];
        const bool wx = ba.pbc && ((bs & 1u) != top);
        const uint32_t rw = wx ? offw + lo_rank[bs ^ 1u] : r;
        const V vw = x[((size_t)rw << lb) + bc];
        const V q0 = x[((size_t)(r + (uint32_t)ep->delta[0]) << lb) + bc];
        const V q1 = x[((size_t)(r + (uint32_t)ep->delta[1]) << lb) + bc];
        const V q2 = x[((size_t)(r + (uint32_t)ep->delta[2]) << lb) + bc];
        const V q3 = x[((size_t)(r + (uint32_t)ep->delta[3]) << lb) + bc];
        const V xr = xs[e];
        const int anti = __popc((bs ^ (bs >> 1)) & ((1u << (llo - 1)) - 1u)) + (cx ? 1 : 0) + (wx ? 1 : 0);
        double d = dblk - hjz * anti;
        for (int i = 0; i < llo; ++i) d += ((bs >> i) & 1u) ? fb[i] : 0.0;
        V hs = {0, 0};
        int pc = 0;
        for (int p = 0; p < llo - 1; ++p) {
          const uint32_t b0 = (bs >> p) & 1u, b1 = (bs >> (p + 1)) & 1u;
          if (b0 != b1) {
            const uint32_t c = sbin[p * kBinomStride + pc];
            const V v = xs[((b0 ? j + c : j - c) << lb) + bc];
            hs.x += v.x;
            hs.y += v.y;
          }
          pc += (int)b0;
        }
        {
          const T w0 = (0 < nact) ? (T)1 : (T)0, w1 = (1 < nact) ? (T)1 : (T)0;
          const T w2 = (2 < nact) ? (T)1 : (T)0, w3 = (3 < nact) ? (T)1 : (T)0;
          hs.x += w0 * q0.x + w1 * q1.x + w2 * q2.x + w3 * q3.x;
          hs.y += w0 * q0.y + w1 * q1.y + w2 * q2.y + w3 * q3.y;
        }
        for (int g0 = 4; g0 < nact; g0 += 4) {
          const V v0 = x[((size_t)(r + (uint32_t)ep->delta[g0]) << lb) + bc];
          const V v1 = x[((size_t)(r + (uint32_t)ep->delta[g0 + 1]) << lb) + bc];
          const V v2 = x[((size_t)(r + (uint32_t)ep->delta[g0 + 2]) << lb) + bc];
          const V v3 = x[((size_t)(r + (uint32_t)ep->delta[g0 + 3]) << lb) + bc];
          const T w1 = (g0 + 1 < nact) ? (T)1 : (T)0;
          const T w2 = (g0 + 2 < nact) ? (T)1 : (T)0;
          const T w3 = (g0 + 3 < nact) ? (T)1 : (T)0;
          hs.x += v0.x + w1 * v1.x + w2 * v2.x + w3 * v3.x;
          hs.y += v0.y + w1 * v1.y + w2 * v2.y + w3 * v3.y;
        }
        hs.x += (cx ? vc.x : (T)0) + (wx ? vw.x : (T)0);
        hs.y += (cx ? vc.y : (T)0) + (wx ? vw.y : (T)0);
        V h;
        h.x = (T)d * xr.x + g * hs.x;
        h.y = (T)d * xr.y + g * hs.y;
        const size_t o = ((size_t)r << lb) + bc;
        if (LANCZOS) {
          V wv;
          wv.x = ca * h.x - cb * um.x;
          wv.y = ca * h.y - cb * um.y;
          st32_stream(y + ((size_t)r << lb), bc, wv);
          s1 += (double)xr.x * (double)wv.x + (double)xr.y * (double)wv.y;
          s2 += (double)xr.x * (double)xr.x + (double)xr.y * (double)xr.y;
          s3r += (double)um.x * (double)wv.x + (double)um.y * (double)wv.y;
          s3i += (double)um.x * (double)wv.y - (double)um.y * (double)wv.x;
        } else {
          st32_stream(y + ((size_t)r << lb), bc, h);
        }
      }
    }
    __syncthreads();   // xs and hic are rewritten by the next block
  }
  if (LANCZOS) {
    double v[kQA] = {s1, s2, s3r, s3i};
    block_partials<kQA>(v, B, red, partA + (size_t)blockIdx.x * kQA * B);
  }
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
  const size_t dyn = blkb_xbytes((uint32_t)binom_host(llo, llo / 2), B, 16) + ((((size_t)4 << llo) + 15) & ~(size_t)15) +
                     sizeof(double) * ((size_t)B * L + 2 * (size_t)B);
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

template <typename T, bool LANCZOS>
static qk_status launch_blkb_t(const qk_ham* H, const void* x, void* y, const void* ujm1, const KState* st,
                               const LanczosArgs* la, const double* partB, int Gp, double* partA, int* grid_out,
                               int wgs_req, hipStream_t s) {
  using V = typename Cx<T>::V;
  BlkArgs ba = blk_args(H);
  const int B = H->batch;
  int lb = 0;
  while ((1 << lb) < B) ++lb;
  const size_t dyn = blkb_xbytes((uint32_t)ba.maxlen, B, sizeof(V)) + ((((size_t)4 << ba.llo) + 15) & ~(size_t)15) +
                     sizeof(double) * ((size_t)B * ba.L + 2 * (size_t)B);
  auto kern = k_blkb<T, LANCZOS>;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlkbThreads, dyn) != hipSuccess || occ < 1) occ = 1;
  const int cus = qk_num_cus();
  int wgs = wgs_req > 0 ? wgs_req : env_int("QK_BLOCKED_WGS_PER_CU", occ);
  if (wgs > occ) wgs = occ;
  int G = ((cus * wgs) / kNumXcd) * kNumXcd;
  if (G < kNumXcd) G = kNumXcd;
  if (G > kMaxPartialBlocks) G = kMaxPartialBlocks;
  int cl = 3;
  while (cl > 0 && (G / kNumXcd) % (1 << cl) != 0) --cl;
  ba.chunk_log2 = cl;
  KState stv{};
  LanczosArgs lav{};
  if (st) stv = *st;
  if (la) lav = *la;
  hipLaunchKernelGGL(kern, dim3(G), dim3(kBlkbThreads), dyn, s, ba, B, lb, (const V*)x, (V*)y, (const V*)ujm1, stv,
                     lav, partB, Gp, partA);
  QK_HIP(hipGetLastError());
  if (grid_out) *grid_out = G;
  return QK_OK;
}

template <typename T, int LLO, bool LANCZOS, bool W64>
static qk_status launch_blk_k(const qk_ham* H, const void* x, void* y, const void* ujm1, const KState* st,
                              const LanczosArgs* la, const double* partB, int Gp, double* partA, int* grid_out,
                              int wgs_req, hipStream_t s) {
  using V = typename Cx<T>::V;
  BlkArgs ba = blk_args(H);
  const size_t dyn = blk_xbytes<T, LLO>() + 2 * sizeof(uint16_t) * ((size_t)1 << LLO);
  auto kern = k_blk<T, LLO, LANCZOS, W64>;
  // work-groups per CU the kernel can hold (queried once per instantiation; thread-safe static init)
  static const int occ = [&]() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlkThreads, dyn) != hipSuccess || n < 1) n = 1;
    return n;
  }();
  const int cus = qk_num_cus();
  int wgs = wgs_req > 0 ? wgs_req : env_int("QK_BLOCKED_WGS_PER_CU", occ);
  if (wgs > occ) wgs = occ;
  int G = ((cus * wgs) / kNumXcd) * kNumXcd;
  if (G < kNumXcd) G = kNumXcd;
  if (G > kMaxPartialBlocks) G = kMaxPartialBlocks;
  // chunk of consecutive blocks per XCD: 8, or the largest power of two
  // dividing the work-groups per XCD
  int cl = 3;
  while (cl > 0 && (G / kNumXcd) % (1 << cl) != 0) --cl;
  ba.chunk_log2 = cl;
  KState stv{};
  LanczosArgs lav{};
  if (st) stv = *st;
  if (la) lav = *la;
  hipLaunchKernelGGL(kern, dim3(G), dim3(kBlkThreads), dyn, s, ba, (const V*)x, (V*)y, (const V*)ujm1, stv, lav,
                     partB, Gp, partA);
  QK_HIP(hipGetLastError());
  if (grid_out) *grid_out = G;
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

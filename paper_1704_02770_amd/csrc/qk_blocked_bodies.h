// Kernel bodies of the blocked matrix-free H x (Sec. 3 "Hamiltonian matrix
// construction", Eq. (1)): the one-phase kernel and the batched [D][B] kernel
// as device functions over a virtual grid (VGrid), so that the plain launches
// of qk_blocked.hip and the persistent step kernel of qk_persist.hip run the
// same code.  The decomposition is described at the top of qk_blocked.hip.
#pragma once

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

// LDS of the one-phase kernel besides the x buffers and the low tables.
struct BlkShared {
  double flo0[256], flo1[256];   // field sums over the low bits, eight bits per table
  double fld[StateT<uint32_t>::kMaxL];
  double tot[1], sa[1], sb[1];
  uint32_t sbin[kBinomStride * kBinomStride];
  int act[1];
  int hds[2][kMaxHi];            // row shifts of the current and the next block
};

// Dynamic LDS of the one-phase kernel: x buffers, low tables, BlkShared.
template <typename T, int LLO>
constexpr size_t blk_smem_bytes() {
  return blk_xbytes<T, LLO>() + 4 * ((size_t)1 << LLO) + sizeof(BlkShared);
}

template <typename T, int LLO, bool LANCZOS, bool W64>
__device__ __forceinline__ void blk_body(VRange rg, unsigned char* smem, const BlkArgs& ba,
                                         const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y,
                                         const typename Cx<T>::V* __restrict__ ujm1, const KState& st,
                                         const LanczosArgs& la, const double* __restrict__ partB, int Gp,
                                         double* __restrict__ partA) {
  using V = typename Cx<T>::V;
  constexpr int kMaxLen = blk_max_len<LLO>();
  static_assert(kMaxLen <= 2 * kBlkThreads, "prefetch covers two elements per thread");
  V* xsb = reinterpret_cast<V*>(smem);                                            // [2][kMaxLen]
  uint16_t* lo_state = reinterpret_cast<uint16_t*>(smem + blk_xbytes<T, LLO>());
  uint16_t* lo_rank = lo_state + (1 << LLO);
  BlkShared& sh = *reinterpret_cast<BlkShared*>(smem + blk_xbytes<T, LLO>() + 4 * ((size_t)1 << LLO));
  uint32_t* sbin = sh.sbin;
  double *flo0 = sh.flo0, *flo1 = sh.flo1, *fld = sh.fld;
  double *tot = sh.tot, *sa = sh.sa, *sb = sh.sb;
  int* act = sh.act;
  int(*hds)[kMaxHi] = sh.hds;
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
    lanczos_h_scalars(1, st, la, partB, Gp, red, tot, sa, sb, act, VGrid{rg.v0, rg.n});
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
  const int lhi = ba.lhi;
  const int cl = ba.chunk_log2;
  const int per = (int)rg.n, last = ba.nblk;
  const bool run = act[0] != 0;
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb) {
    double s1 = 0.0, s2 = 0.0, s3r = 0.0, s3i = 0.0;
    // work-group w runs on XCD w % 8; in every window of rg.n blocks the XCD
    // takes chunks of 2^chunk_log2 consecutive blocks (the launcher makes
    // rg.n / 8 a multiple of the chunk)
    const int xcd = (int)(vb % kNumXcd), kx = (int)(vb / kNumXcd);
    int bi = ((((kx >> cl) * kNumXcd) + xcd) << cl) + (kx & ((1 << cl) - 1));
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
      block_partials<kQA>(v, 1, red, partA + (size_t)vb * kQA);
    }
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

// LDS of the batched kernel besides the staged block, the low tables and the
// per-phase fields.
struct BlkbShared {
  double tot[QK_MAX_BATCH], sa[QK_MAX_BATCH], sb[QK_MAX_BATCH];
  uint32_t sbin[kBinomStride * kBinomStride];
  int act[QK_MAX_BATCH];
};

// Byte offsets of the batched kernel's dynamic LDS: staged block, low tables,
// fields [B][L] with the per-phase block constants and field sums, BlkbShared.
__host__ __device__ inline size_t blkb_fld_offset(uint32_t maxlen, int B, size_t vbytes, int llo) {
  return blkb_xbytes(maxlen, B, vbytes) + ((((size_t)4 << llo) + 15) & ~(size_t)15);
}
__host__ __device__ inline size_t blkb_shared_offset(uint32_t maxlen, int B, size_t vbytes, int llo, int L) {
  return (blkb_fld_offset(maxlen, B, vbytes, llo) + sizeof(double) * ((size_t)B * L + 2 * (size_t)B) + 15) &
         ~(size_t)15;
}
__host__ __device__ inline size_t blkb_smem_bytes(uint32_t maxlen, int B, size_t vbytes, int llo, int L) {
  return blkb_shared_offset(maxlen, B, vbytes, llo, L) + sizeof(BlkbShared);
}

template <typename T, bool LANCZOS>
__device__ __forceinline__ void blkb_body(VRange rg, unsigned char* smem, const BlkArgs& ba, int B, int lb,
                                          const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y,
                                          const typename Cx<T>::V* __restrict__ ujm1, const KState& st,
                                          const LanczosArgs& la, const double* __restrict__ partB, int Gp,
                                          double* __restrict__ partA) {
  using V = typename Cx<T>::V;
  const int llo = ba.llo, L = ba.L, lhi = ba.lhi;
  V* xs = reinterpret_cast<V*>(smem);
  const uint32_t ml = (uint32_t)ba.maxlen;
  uint16_t* lo_state = reinterpret_cast<uint16_t*>(smem + blkb_xbytes(ml, B, sizeof(V)));
  uint16_t* lo_rank = lo_state + (1 << llo);
  double* fld = reinterpret_cast<double*>(smem + blkb_fld_offset(ml, B, sizeof(V), llo));   // [B][L]
  double* hic = fld + (size_t)B * L;   // per phase: block constant of the diagonal
  double* hh = hic + B;                // per phase: sum of the fields / 2
  BlkbShared& sh = *reinterpret_cast<BlkbShared*>(smem + blkb_shared_offset(ml, B, sizeof(V), llo, L));
  uint32_t* sbin = sh.sbin;
  double *tot = sh.tot, *sa = sh.sa, *sb = sh.sb;
  int* act = sh.act;
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
    lanczos_h_scalars(B, st, la, partB, Gp, red, tot, sa, sb, act, VGrid{rg.v0, rg.n});
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
  const int cl = ba.chunk_log2;
  const int last = ba.nblk;
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb) {
    double s1 = 0.0, s2 = 0.0, s3r = 0.0, s3i = 0.0;
    const int xcd = (int)(vb % kNumXcd), kx = (int)(vb / kNumXcd);
    int bi = ((((kx >> cl) * kNumXcd) + xcd) << cl) + (kx & ((1 << cl) - 1));
    __syncthreads();   // `red` (aliasing xs) is no longer read

    for (; bi < last; bi += (int)rg.n) {
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
      block_partials<kQA>(v, B, red, partA + (size_t)vb * kQA * B);
    }
  }
}

// Launch plan of a blocked Lanczos H-pass (host side): arguments, grid and
// dynamic LDS of the one-phase kernel (llo > 0) or the batched kernel (llo = 0).
struct BlkPlan {
  BlkArgs ba;
  int G;        // work-groups, a multiple of 8
  int lb;       // log2 of the batch (batched kernel)
  size_t smem;  // dynamic LDS bytes
  int llo;      // low-bit count of the one-phase kernel, 0 for the batched kernel
  bool w64;     // 64-bit element offsets
};
qk_status blocked_lanczos_plan(const qk_ham* H, int dtype, int wgs_req, BlkPlan* p);

}  // namespace qk

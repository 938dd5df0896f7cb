// Two-pass H x and Lanczos iteration for large sectors (Sec. 3 "Hamiltonian
// matrix construction", Eq. (1); Sec. 2 "Krylov subspace methods").
//
// The bonds of Eq. (1) are split at bit llo2 - 1 of the state:
//   * the high pass applies every bond (p, p+1) with p >= llo2 - 1.  In the
//     split at llo1 = llo2 - 1 these are the bonds inside the high bits a1,
//     and a hop on one of them maps block a1 onto block a1' with the same
//     in-block column, a fixed row shift for the whole block.  Within one
//     low-popcount class k the high bonds therefore act on the matrix
//     X_k[block][column] along its block index only, column by column: the
//     pass walks column slabs of each class, sized so that the slab's values
//     stay resident in one XCD's L2 while the whole XCD works through it, so
//     every gather after the first read of a line hits on chip;
//   * the low pass applies the diagonal and the bonds inside the low llo2
//     bits from LDS, and, on a ring, the wrap bond (L-1, 0), which pairs
//     block a2 with block a2 xor (top bit): both blocks of such a pair are
//     staged in LDS together.
// For a Lanczos iteration the two passes are
//   high:  z = sigma_j H_hi u_j - beta_{j-1} sigma_{j-1} u_{j-1}
//          partials Re<u_j, H_hi u_j>, Re<u_j, u_{j-1}>
//   low:   u_{j+1} = c (z + s H_lo u_j - d u_j)  (H_lo: diagonal, low and wrap bonds)
//          partials |u_{j+1}|^2 and Re<u_{j+1}, H_lo u_{j+1}>
// alpha_j = <v_j, H v_j - beta_{j-1} v_{j-1}> needs Re<u_j, H_lo u_j>, which
// the low pass of the previous iteration computed from the u_j it had just
// written (a second LDS pass over the staged pair, each bond counted once),
// so both passes are single streams: 3 vectors each, 6 per iteration, the
// same as the fused two-pass form, but without re-reading x for the high
// bonds.  A pre-pass gives the same partials for the step's initial vector.
//
// Layout of the workspace's own vectors (the Krylov basis and z): every
// block of the llo1 split starts on a 128-byte line (padded with unused
// elements), so that a slab column range of 128 bytes is one line of every
// block.  The caller's vectors (psi, x, y) keep the sorted-basis layout.
#include <algorithm>
#include <cstddef>
#include <cstdlib>
#include <new>
#include <vector>

#include "qk_blocked.h"

namespace qk {

// ------------------------------------------------------------ table layouts
// One column slab of one low-popcount class of the high pass.
struct SlabDesc {
  uint32_t list0;   // first position of the class in the class-ordered block arrays
  uint32_t nb;      // blocks of the class
  uint16_t j0;      // first column of the slab
  uint16_t ncol;    // columns of the class (block length)
  uint16_t wlog;    // the slab covers columns j0 .. j0 + 2^wlog - 1 (those below ncol)
  uint16_t k;       // the class: popcount of the low bits
};

// One task of the low pass: a block with high top bit 0 and its ring
// partner (entries of the llo2 table; -1 when absent).
struct PairTask {
  int32_t a, b;
};

constexpr int kPadBytes = 128;   // padded blocks start on a 128-byte line

struct SplitTables {
  int llo2 = 0, nhi = 0, nlo = 0, ntask = 0, maxtask = 0;
  uint32_t* coff = nullptr;       // [nhi] first row of each block of the llo1 split, grouped by class
  uint32_t* ca = nullptr;         // [nhi] its high bits
  uint32_t* cpoff[2] = {};        // [nhi] its first element in the padded layout (complex128, complex64)
  SlabDesc* slab[2] = {};         // slab schedules (complex128, complex64)
  uint32_t xcd_slab[2][kNumXcd + 1] = {};
  BlkEntry* lo = nullptr;         // [nlo] blocks of the split at llo2; pad[0..1] = padded first element
  uint16_t* lo_state = nullptr;   // [2^llo2] low states grouped by popcount, ascending
  uint16_t* lo_rank = nullptr;    // [2^llo2] rank of a low state inside its popcount group
  uint32_t* binp[2] = {};         // [33 * 33] padded binomials of the high pass (complex128, complex64)
  PairTask* task = nullptr;       // [ntask]
  uint32_t* line_r0[2] = {};      // per 128-byte line of the padded layout: row of its first element
  uint8_t* line_n[2] = {};        // and its number of used elements
  uint64_t dpad[2] = {};          // padded vector length
  uint64_t nline[2] = {};
  uint32_t lo_base[18] = {};
};

// ---------------------------------------------------------- small helpers
template <typename V>
__device__ __forceinline__ V ldn(const V* p) {
  using S = decltype(V{}.x);
  typedef S E __attribute__((ext_vector_type(2)));
  const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
  return V{e.x, e.y};
}
template <typename V>
__device__ __forceinline__ void stn(V* p, V v) {
  using S = decltype(V{}.x);
  typedef S E __attribute__((ext_vector_type(2)));
  const E e = {v.x, v.y};
  __builtin_nontemporal_store(e, reinterpret_cast<E*>(p));
}

// ================================================================ high pass
constexpr int kHiThreads = 256;
constexpr int kQH = 2;   // partials: Re<u_j, H_hi u_j>, Re<u_j, u_{j-1}>

struct HiArgs {
  const uint32_t* coff;    // sorted-basis first rows, class order
  const uint32_t* cpoff;   // padded first elements, class order
  const uint32_t* ca;
  const SlabDesc* slab;
  const uint32_t* binom;   // row shifts in the sorted layout, or in the padded one when x is padded
  uint32_t xcd_slab[kNumXcd + 1];
  int llo1, lhi1;
  int x_pad, um_pad, z_pad;   // which operands are in the padded layout
  double half_jxy;
};

// Work-group w runs on XCD w % 8 and walks that XCD's run of slabs; the
// XCD's work-groups share each slab's elements, so its lines are read from
// HBM once and the partner gathers of all of them hit the XCD's L2.  A hop
// on the high bond (llo1 + t, llo1 + t + 1) of block a1 moves the row by
// +-C(llo1 + t, number of set bits of the state below bit llo1 + t), the same
// for every column of the block.  In the padded layout the first element of
// block a1 is the same sum of binomials with C'(llo1, k) = C(llo1, k) rounded
// up to whole lines and C'(n, k) = C'(n-1, k) + C'(n-1, k-1) above, so a hop
// moves the element by +-C'(llo1 + t, same count): binom is C or C'.
template <typename T, bool LANCZOS>
__global__ void __launch_bounds__(kHiThreads)
k_split_hi(HiArgs ha, const typename Cx<T>::V* __restrict__ x, const typename Cx<T>::V* __restrict__ um,
           typename Cx<T>::V* __restrict__ z, KState st, LanczosArgs la, const double* __restrict__ partB, int Gp,
           double* __restrict__ partA) {
  using V = typename Cx<T>::V;
  __shared__ double red[kQH * kHiThreads];
  __shared__ uint32_t sbin[kBinomStride * kBinomStride];
  __shared__ double tot[1], sa[1], sb[1];
  __shared__ int act[1];
  for (int i = threadIdx.x; i < kBinomStride * kBinomStride; i += kHiThreads) sbin[i] = ha.binom[i];
  if (LANCZOS) {
    lanczos_h_scalars(1, st, la, partB, Gp, red, tot, sa, sb, act, hw_grid());
  } else {
    if (threadIdx.x == 0) {
      sa[0] = 1.0;
      sb[0] = 0.0;
      act[0] = 1;
    }
    __syncthreads();
  }
  const T g = (T)ha.half_jxy;
  const T ca = (T)sa[0], cb = (T)sb[0];
  const bool prev = LANCZOS && la.j > 0;
  const int llo1 = ha.llo1, nb1 = ha.lhi1 - 1;
  double q = 0.0, rho = 0.0;
  if (act[0]) {
    const int xcd = blockIdx.x % kNumXcd;
    const uint32_t wi = blockIdx.x / kNumXcd, nper = gridDim.x / kNumXcd;
    const uint32_t s_end = ha.xcd_slab[xcd + 1];
    for (uint32_t s = ha.xcd_slab[xcd]; s < s_end; ++s) {
      const SlabDesc d = ha.slab[s];
      const uint32_t wl = d.wlog, total = d.nb << wl, wm = (1u << wl) - 1u;
      for (uint32_t e = wi * kHiThreads + threadIdx.x; e < total; e += nper * kHiThreads) {
        const uint32_t col = (uint32_t)d.j0 + (e & wm);
        const bool on = col < d.ncol;   // lanes past the class's columns only help with the shifts
        const uint32_t pos = d.list0 + (e >> wl);
        const int64_t ru = (int64_t)ha.coff[pos] + col;
        const int64_t rp = (int64_t)ha.cpoff[pos] + col;
        const int64_t rx = ha.x_pad ? rp : ru;
        const uint32_t a1 = ha.ca[pos];
        const V z0 = {0, 0};
        V u = z0, xr = z0;
        if (on) {
          if (prev) u = ldn(um + (ha.um_pad ? rp : ru));
          xr = x[rx];
        }
        // the block's row shifts, computed once per aligned group of 8 lanes
        // (the lanes of one block row, 8 <= 2^wlog): lane l of the group
        // holds the shifts of bonds l, l + 8, l + 16 (0: bond not active)
        const int l8 = (int)(threadIdx.x & 7u);
        int sh[3];
#pragma unroll
        for (int g3 = 0; g3 < 3; ++g3) {
          const int t = l8 + 8 * g3;
          int v = 0;
          if (t < nb1) {
            const uint32_t b0 = (a1 >> t) & 1u, b1 = (a1 >> (t + 1)) & 1u;
            if (b0 != b1) {
              const int pc = d.k + __popc(a1 & ((1u << t) - 1u));
              const int c = (int)sbin[(llo1 + t) * kBinomStride + pc];
              v = b0 ? c : -c;
            }
          }
          sh[g3] = v;
        }
        V hs = z0;
        const int lb = (int)(threadIdx.x & ~7u) & 63;
        for (int t = 0; t < nb1; ++t) {
          const int c = __shfl(sh[t >> 3], lb + (t & 7), 64);
          if (on && c != 0) {
            const V v = x[rx + c];
            hs.x += v.x;
            hs.y += v.y;
          }
        }
        V h;
        h.x = g * hs.x;
        h.y = g * hs.y;
        V* zp = z + (ha.z_pad ? rp : ru);
        if (!on) continue;
        if (LANCZOS) {
          V zv;
          zv.x = ca * h.x - cb * u.x;
          zv.y = ca * h.y - cb * u.y;
          stn(zp, zv);
          q += (double)xr.x * (double)h.x + (double)xr.y * (double)h.y;
          rho += (double)xr.x * (double)u.x + (double)xr.y * (double)u.y;
        } else {
          stn(zp, h);
        }
      }
    }
  }
  if (LANCZOS) {
    double v[kQH] = {q, rho};
    block_partials<kQH>(v, 1, red, partA + (size_t)blockIdx.x * kQH);
  }
}

// ================================================================= low pass
enum { kLoApply = 0, kLoLanczos = 1, kLoForm = 2 };

struct LoArgs {
  int L, N, pbc, lhi;
  double half_jxy, jz;
  const BlkEntry* blk;
  const PairTask* task;
  int ntask;
  const uint16_t* lo_state;
  const uint16_t* lo_rank;
  const uint32_t* binom;
  const double* fields;
  uint32_t lo_base[18];
  int dt;                        // 0: complex128, 1: complex64 (which padded offsets)
  int pad_elems;                 // elements per 128-byte line
  int x_pad, z_pad, out_pad;     // which operands are in the padded layout
};

template <int LLO>
constexpr int lo_threads() {
  return LLO >= 13 ? 1024 : LLO == 12 ? 512 : 256;
}
template <int LLO>
constexpr int lo_maxlen() {   // C(LLO, LLO/2)
  return LLO == 10 ? 252 : LLO == 11 ? 462 : LLO == 12 ? 924 : 1716;
}
template <int LLO>
constexpr int lo_elems() {   // elements per thread for a pair of the largest blocks
  return (2 * lo_maxlen<LLO>() + lo_threads<LLO>() - 1) / lo_threads<LLO>();
}

// The two blocks of a low-pass task (uniform values).
struct LoTask {
  uint32_t offA, lenA, aA, poffA, len0A, offB, lenB, aB, poffB, len0B;
  int kA, kB;
  double dcA, dcB;
};

__device__ __forceinline__ LoTask lo_task(const LoArgs& a, const uint32_t* sbin, int llo, int t) {
  const PairTask pt = a.task[t];
  LoTask ti{};
  if (pt.a >= 0) {
    const BlkEntry* e = a.blk + pt.a;
    ti.aA = e->a;
    ti.offA = e->off;
    ti.poffA = e->pad[a.dt];
    ti.dcA = e->dconst;
    ti.kA = a.N - __popc(ti.aA);
    ti.lenA = sbin[llo * kBinomStride + ti.kA];
    ti.len0A = sbin[(llo - 1) * kBinomStride + ti.kA];
  }
  if (pt.b >= 0) {
    const BlkEntry* e = a.blk + pt.b;
    ti.aB = e->a;
    ti.offB = e->off;
    ti.poffB = e->pad[a.dt];
    ti.dcB = e->dconst;
    ti.kB = a.N - __popc(ti.aB);
    ti.lenB = sbin[llo * kBinomStride + ti.kB];
    ti.len0B = sbin[(llo - 1) * kBinomStride + ti.kB];
  }
  return ti;
}

// Element j of a block: sorted-basis row off + j, or in the padded layout
// its first half (bit llo2 - 1 clear, len0 elements) from poff and its second
// half from the next 128-byte line boundary.
__device__ __forceinline__ size_t lo_row(bool pad, uint32_t off, uint32_t poff, uint32_t len0, uint32_t j, int pe) {
  if (!pad) return (size_t)off + j;
  if (j < len0) return (size_t)poff + j;
  const uint32_t h0 = (len0 + pe - 1) / pe * pe;
  return (size_t)poff + h0 + (j - len0);
}

// Hops inside the low bits of the element at in-block index j with low
// state b, read from the LDS copy xs of its block (segment seg): the state
// b ^ (3 << p) of a hop on bond (p, p+1) sits at index lrk[b ^ (3 << p)] of
// its block (lrk: the ranks of all low states, in LDS).  Every bond issues
// both reads (an inactive one reads the element itself with weight zero),
// so the reads of all bonds are independent.  UP_ONLY sums only hops that
// move a particle from p to p+1 (each bond pair of the block once, for
// quadratic forms).
template <typename T, int LLO, bool UP_ONLY>
__device__ __forceinline__ void lo_hops(const typename Cx<T>::V* xs, const uint16_t* lrk, uint32_t b, uint32_t j,
                                        uint32_t seg, typename Cx<T>::V& hs) {
#pragma unroll
  for (int p = 0; p < LLO - 1; ++p) {
    const uint32_t b0 = (b >> p) & 1u, b1 = (b >> (p + 1)) & 1u;
    const bool act = UP_ONLY ? (b0 && !b1) : (b0 != b1);
    const uint32_t nb = lrk[b ^ (3u << p)];
    const typename Cx<T>::V v = xs[seg + (act ? nb : j)];
    const T w = act ? (T)1 : (T)0;
    hs.x = fma(w, v.x, hs.x);
    hs.y = fma(w, v.y, hs.y);
  }
}

// MODE kLoApply:   out = zin + H_lo x                        (zin may be out)
// MODE kLoLanczos: out = c (zin + s H_lo x - d x), partials |out|^2, Re<out, H_lo out>
// MODE kLoForm:    partials |x|^2, Re<x, H_lo x>             (start of a step)
// Work-groups are persistent over the task list; the global loads of a
// work-group's next task are issued before the current task's LDS work, so
// they are in flight while it computes.
template <typename T, int LLO, int MODE>
__global__ void __launch_bounds__(lo_threads<LLO>())
k_split_lo(LoArgs a, const typename Cx<T>::V* __restrict__ x, const typename Cx<T>::V* zin,
           typename Cx<T>::V* out, KState st, LanczosArgs la, const double* __restrict__ partA, int GA,
           const double* __restrict__ partBin, const double* __restrict__ partQin, int GB,
           double* __restrict__ partBout, double* __restrict__ partQout, int store) {
  using V = typename Cx<T>::V;
  constexpr int NT = lo_threads<LLO>();
  constexpr int E = lo_elems<LLO>();
  constexpr bool ZIN = MODE != kLoForm;
  extern __shared__ unsigned char smem[];
  V* xs = reinterpret_cast<V*>(smem);
  __shared__ double red[2 * NT];
  __shared__ uint32_t sbin[kBinomStride * kBinomStride];
  __shared__ double flo0[256], flo1[256];
  __shared__ double fld[StateT<uint32_t>::kMaxL];
  __shared__ uint16_t lrk[1 << LLO];
  __shared__ double tot[4], sc[3];
  __shared__ int act[1];
  const int tid = threadIdx.x;
  for (int i = tid; i < kBinomStride * kBinomStride; i += NT) sbin[i] = a.binom[i];
  for (int i = tid; i < (1 << LLO); i += NT) lrk[i] = a.lo_rank[i];
  if (tid < a.L) fld[tid] = a.fields[tid];
  __syncthreads();
  if (tid < 256) {
    double f0 = 0.0, f1 = 0.0;
    for (int i = 0; i < 8; ++i) {
      if ((tid >> i) & 1) {
        if (i < LLO) f0 += fld[i];
        if (8 + i < LLO) f1 += fld[8 + i];
      }
    }
    flo0[tid] = f0;
    flo1[tid] = f1;
  }
  if (MODE == kLoLanczos) {
    reduce_partials(partA, GA, kQH, 1, red, tot);        // Re<u_j, H_hi u_j>, Re<u_j, u_{j-1}>
    reduce_partials(partBin, GB, 1, 1, red, tot + 2);    // |u_j|^2
    reduce_partials(partQin, GB, 1, 1, red, tot + 3);    // Re<u_j, H_lo u_j>
    if (tid == 0) {
      const int j = la.j;
      int active = st.mused[0] > j;
      double c = 1.0, dd = 0.0, s = 1.0, alpha = 0.0;
      if (active) {
        const double qH = tot[0], rho = tot[1], S2 = tot[2], qA = tot[3];
        if (j == 0) {
          const double n0 = sqrt(S2);
          alpha = (qH + qA) / S2;
          c = 1.0 / n0;
          dd = alpha;
          if (blockIdx.x == 0) {
            st.n0[0] = n0;
            st.sigma[0] = 1.0 / n0;
          }
          if (!(n0 > 0.0)) {
            active = 0;   // zero vector: nothing to propagate
            if (blockIdx.x == 0) {
              st.mused[0] = 0;
              if (!isfinite(S2)) st.status[0] = QK_ENUMERIC;
            }
          }
        } else {
          const double sj = st.sigma[j], sjm = st.sigma[j - 1], bjm = st.beta[j - 1];
          alpha = sj * sj * (qH + qA) - bjm * sjm * sj * rho;
          dd = alpha * sj;
          s = sj;
        }
        if (active && !isfinite(alpha)) {
          active = 0;
          if (blockIdx.x == 0) {
            st.status[0] = QK_ENUMERIC;
            st.mused[0] = j;
          }
        }
        if (active && blockIdx.x == 0) st.alpha[j] = alpha;
      }
      sc[0] = c;
      sc[1] = dd;
      sc[2] = s;
      act[0] = active;
    }
  } else if (tid == 0) {
    sc[0] = 1.0;
    sc[1] = 0.0;
    sc[2] = 1.0;
    act[0] = 1;
  }
  __syncthreads();
  const T g = (T)a.half_jxy;
  const double hjz = 0.5 * a.jz;
  const T cc = (T)sc[0], cd = (T)sc[1], cs = (T)sc[2];
  const int lhi = a.lhi, pe = a.pad_elems;
  const uint32_t lomask = (1u << (LLO - 1)) - 1u;
  const bool xpad = a.x_pad != 0, zpad = a.z_pad != 0, opad = a.out_pad != 0;
  double nrm = 0.0, qf = 0.0;
  const bool run = act[0] != 0;
  const int G = gridDim.x;
  int t = blockIdx.x;
  V px[E], pz[E];
  LoTask cur{};
  auto rowA = [&](const LoTask& ti, bool pad, uint32_t e) -> size_t {
    return e < ti.lenA ? lo_row(pad, ti.offA, ti.poffA, ti.len0A, e, pe)
                       : lo_row(pad, ti.offB, ti.poffB, ti.len0B, e - ti.lenA, pe);
  };
  // global loads of a task's x (next task, before the current LDS work) and
  // z (the current task's z is consumed by the first phase, so the next
  // task's is loaded after it)
  auto fetch_x = [&](const LoTask& ti) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t e = tid + i * NT;
      if (e < ti.lenA + ti.lenB) px[i] = ldn(x + rowA(ti, xpad, e));
    }
  };
  auto fetch_z = [&](const LoTask& ti) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t e = tid + i * NT;
      if (ZIN && e < ti.lenA + ti.lenB) pz[i] = ldn(zin + rowA(ti, zpad, e));
    }
  };
  if (run && t < a.ntask) {
    cur = lo_task(a, sbin, LLO, t);
    fetch_x(cur);
    fetch_z(cur);
  }
  for (; run && t < a.ntask; t += G) {
    const uint32_t lenA = cur.lenA, n = cur.lenA + cur.lenB;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t e = tid + i * NT;
      if (e < n) xs[e] = px[i];
    }
    __syncthreads();
    const bool more = t + G < a.ntask;
    LoTask nxt{};
    if (more) {
      nxt = lo_task(a, sbin, LLO, t + G);
      fetch_x(nxt);
    }
    V ur[E];
    uint32_t bj[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t e = tid + i * NT;
      if (e < n) {
        const bool sd = e >= lenA;
        const uint32_t j = sd ? e - lenA : e;
        const uint32_t b = a.lo_state[a.lo_base[sd ? cur.kB : cur.kA] + j];
        const uint32_t a2 = sd ? cur.aB : cur.aA;
        const uint32_t top = (a2 >> (lhi - 1)) & 1u;
        const bool wx = a.pbc && ((b & 1u) != top);
        const int anti = __popc((b ^ (b >> 1)) & lomask) + (int)(((b >> (LLO - 1)) ^ a2) & 1u) + (wx ? 1 : 0);
        const double d = (sd ? cur.dcB : cur.dcA) + flo0[b & 255u] + flo1[b >> 8] - hjz * anti;
        const uint32_t seg = sd ? lenA : 0u;
        const V xe = xs[e];
        V hs = {0, 0};
        lo_hops<T, LLO, false>(xs, lrk, b, j, seg, hs);
        if (wx) {
          const V v = xs[(sd ? 0u : lenA) + lrk[b ^ 1u]];
          hs.x += v.x;
          hs.y += v.y;
        }
        V h;
        h.x = (T)d * xe.x + g * hs.x;
        h.y = (T)d * xe.y + g * hs.y;
        if (MODE == kLoApply) {
          V o;
          o.x = pz[i].x + h.x;
          o.y = pz[i].y + h.y;
          stn(out + rowA(cur, opad, e), o);
        } else if (MODE == kLoForm) {
          nrm += (double)xe.x * (double)xe.x + (double)xe.y * (double)xe.y;
          qf += (double)xe.x * (double)h.x + (double)xe.y * (double)h.y;
        } else {
          V un;
          un.x = cc * ((pz[i].x + cs * h.x) - cd * xe.x);
          un.y = cc * ((pz[i].y + cs * h.y) - cd * xe.y);
          if (store) stn(out + rowA(cur, opad, e), un);
          nrm += (double)un.x * (double)un.x + (double)un.y * (double)un.y;
          // the next iteration's form: the diagonal part here, the bonds below
          qf += d * ((double)un.x * (double)un.x + (double)un.y * (double)un.y);
          ur[i] = un;
          bj[i] = (b << 16) | j;
        }
      }
    }
    if (more) fetch_z(nxt);
    if (MODE == kLoLanczos && store) {
      // Re<u_{j+1}, H_lo u_{j+1}> for the next iteration's alpha: each bond
      // pair counted once, from the end whose particle hops up (and the wrap
      // pair from the end with bit 0 set), on the values just written,
      // staged in place of u_j
      __syncthreads();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t e = tid + i * NT;
        if (e < n) xs[e] = ur[i];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t e = tid + i * NT;
        if (e < n) {
          const bool sd = e >= lenA;
          const uint32_t b = bj[i] >> 16, j = bj[i] & 0xffffu;
          const uint32_t a2 = sd ? cur.aB : cur.aA;
          const uint32_t top = (a2 >> (lhi - 1)) & 1u;
          V hs = {0, 0};
          lo_hops<T, LLO, true>(xs, lrk, b, j, sd ? lenA : 0u, hs);
          if (a.pbc && (b & 1u) && !top) {
            const V v = xs[lenA + lrk[b ^ 1u]];   // bit 0 set, top bit clear: the partner is in the second block
            hs.x += v.x;
            hs.y += v.y;
          }
          qf += 2.0 * (double)g * ((double)ur[i].x * (double)hs.x + (double)ur[i].y * (double)hs.y);
        }
      }
    }
    __syncthreads();   // xs is rewritten for the next task
    cur = nxt;
  }
  if (MODE != kLoApply) {
    __shared__ double outv[2];
    double v[2] = {nrm, qf};
    block_partials<2>(v, 1, red, outv);
    if (tid == 0) {
      partBout[blockIdx.x] = outv[0];
      partQout[blockIdx.x] = outv[1];
    }
  }
}

// ============================================== combination, padded basis
// psi <- n0 sum_j g_j v_j with v_0 = psi (sorted-basis layout) and the
// Krylov vectors in the padded layout; one thread per padded element, the
// row of the element from its line's table entry.  FP64 accumulation.
template <typename T>
__global__ void __launch_bounds__(kMaxBlock)
k_combine_pad(typename Cx<T>::V* __restrict__ psi, const typename Cx<T>::V* __restrict__ U, uint64_t dpad,
              const uint32_t* __restrict__ line_r0, const uint8_t* __restrict__ line_n, int pe, KState st) {
  using V = typename Cx<T>::V;
  const int mu = st.mused[0];
  if (!(st.status[0] == QK_OK && mu > 0)) return;   // failed or nothing to propagate: psi unchanged
  constexpr int U8 = 8;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < dpad;
       p += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t ln = p / (uint64_t)pe;
    const uint32_t e = (uint32_t)(p - ln * (uint64_t)pe);
    if (e >= line_n[ln]) continue;
    const size_t r = (size_t)line_r0[ln] + e;
    const V p0 = psi[r];
    double ar = st.gre[0] * (double)p0.x - st.gim[0] * (double)p0.y;
    double ai = st.gre[0] * (double)p0.y + st.gim[0] * (double)p0.x;
    int jj = 1;
    for (; jj + U8 - 1 < mu; jj += U8) {
      V u[U8];
#pragma unroll
      for (int k = 0; k < U8; ++k) u[k] = ldn(U + (uint64_t)(jj - 1 + k) * dpad + p);
#pragma unroll
      for (int k = 0; k < U8; ++k) {
        const double gr = st.gre[jj + k], gi = st.gim[jj + k];
        ar += gr * (double)u[k].x - gi * (double)u[k].y;
        ai += gr * (double)u[k].y + gi * (double)u[k].x;
      }
    }
    for (; jj < mu; ++jj) {
      const V u = ldn(U + (uint64_t)(jj - 1) * dpad + p);
      const double gr = st.gre[jj], gi = st.gim[jj];
      ar += gr * (double)u.x - gi * (double)u.y;
      ai += gr * (double)u.y + gi * (double)u.x;
    }
    V o;
    o.x = (T)ar;
    o.y = (T)ai;
    psi[r] = o;
  }
}

// ================================================================ host side
namespace {

struct HostBinom {
  uint64_t c[65][65];
  HostBinom() {
    for (int n = 0; n <= 64; ++n)
      for (int k = 0; k <= 64; ++k) c[n][k] = (k == 0) ? 1 : (n == 0 ? 0 : c[n - 1][k - 1] + (k <= n - 1 ? c[n - 1][k] : 0));
  }
  uint64_t rank(uint64_t s) const {   // sum_k C(p_k, k) over the set bits p_1 < p_2 < ...
    uint64_t r = 0;
    int k = 1;
    while (s) {
      r += c[__builtin_ctzll(s)][k++];
      s &= s - 1;
    }
    return r;
  }
};

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  const int x = atoi(v);
  return x > 0 ? x : dflt;
}

SplitTables* tables(const qk_ham* H) { return reinterpret_cast<SplitTables*>(H->split); }

template <typename X>
hipError_t upload(const qk_allocator& al, X** dst, const std::vector<X>& src) {
  const size_t bytes = sizeof(X) * (src.empty() ? 1 : src.size());
  hipError_t e = dev_alloc(al, (void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (src.empty()) return hipSuccess;
  return hipMemcpy(*dst, src.data(), sizeof(X) * src.size(), hipMemcpyHostToDevice);
}

}  // namespace

// Low bits of the split for a chain of L sites (QK_SPLIT_LLO overrides):
// blocks of up to C(llo2, llo2/2) rows for the low pass, classes of up to
// C(L - llo2 + 1, (L - llo2 + 1)/2) blocks for the high pass.
int split_llo(int L) {
  int llo = L >= 28 ? 13 : L >= 26 ? 12 : L >= 24 ? 11 : 10;
  llo = env_int("QK_SPLIT_LLO", llo);
  if (llo < 10) llo = 10;
  if (llo > 13) llo = 13;
  if (llo > L - 4) llo = L - 4;
  return llo;
}

void split_free(qk_ham* H) {
  SplitTables* t = tables(H);
  if (!t) return;
  dev_free(H->al, t->coff);
  dev_free(H->al, t->ca);
  for (int dt = 0; dt < 2; ++dt) {
    dev_free(H->al, t->cpoff[dt]);
    dev_free(H->al, t->slab[dt]);
    dev_free(H->al, t->line_r0[dt]);
    dev_free(H->al, t->line_n[dt]);
  }
  dev_free(H->al, t->lo);
  dev_free(H->al, t->lo_state);
  dev_free(H->al, t->lo_rank);
  dev_free(H->al, t->binp[0]);
  dev_free(H->al, t->binp[1]);
  dev_free(H->al, t->task);
  delete t;
  H->split = nullptr;
}

static double split_zz0(const qk_ham* H) { return 0.25 * H->p.jz * (H->p.pbc ? H->basis->L : H->basis->L - 1); }
static double split_hhalf(const qk_ham* H) {
  double hs = 0.0;
  for (int i = 0; i < H->basis->L; ++i) hs += H->h_host[i];
  return 0.5 * hs;
}

qk_status split_fields(qk_ham* H, hipStream_t s) {
  SplitTables* t = tables(H);
  if (!t) return QK_OK;
  const int L = H->basis->L;
  return launch_block_consts(t->lo, t->nlo, t->llo2, L - t->llo2, split_zz0(H), split_hhalf(H), H->p.jz, H->d_fields,
                             s);
}

// The split is built only when QK_SPLIT=1 is set at qk_ham_create: on
// MI355X at L = 28 it is slower than the one-pass blocked kernel (the
// largest class's slab of one 128-byte line per block is 1.65 MB, and with
// the two streamed vectors it does not stay in the XCD's L2), so it is an
// alternative path, kept correct by its own tests.
bool split_enabled() {
  const char* sp = getenv("QK_SPLIT");
  return sp && sp[0] == '1';
}

qk_status split_build(qk_ham* H, hipStream_t s) {
  const qk_basis* bs = H->basis;
  const int L = bs->L, N = bs->N;
  if (!split_enabled()) return QK_OK;
  // its kernels address the padded vectors with 32-bit byte offsets:
  // complex128 vectors of the half-filled L = 30 chain (2.5 GB) are the largest
  if (H->batch != 1 || H->p.mode != QK_MATFREE || L < 18 || L > 30 || bs->wide) return QK_OK;
  static const HostBinom hb;
  SplitTables* t = new (std::nothrow) SplitTables();
  if (!t) {
    set_error("out of host memory");
    return QK_ENOMEM;
  }
  H->split = t;
  const int llo2 = split_llo(L), llo1 = llo2 - 1, lhi1 = L - llo1, lhi2 = L - llo2;
  t->llo2 = llo2;
  const int pe[2] = {kPadBytes / 16, kPadBytes / 8};   // elements per line: complex128, complex64

  // ---- the llo1 split in sorted order: first rows and padded first elements
  const uint64_t n1 = 1ull << lhi1;
  std::vector<uint32_t> off1(n1, 0), poff1[2] = {std::vector<uint32_t>(n1, 0), std::vector<uint32_t>(n1, 0)};
  std::vector<uint32_t> lr0[2];
  std::vector<uint8_t> lnn[2];
  {
    uint64_t acc[2] = {0, 0};
    for (uint64_t a1 = 0; a1 < n1; ++a1) {
      const int k1 = N - __builtin_popcountll(a1);
      const bool ok = k1 >= 0 && k1 <= llo1;
      const uint64_t len = ok ? hb.c[llo1][k1] : 0;
      const uint64_t r0 = ok ? hb.rank((a1 << llo1) | ((1ull << k1) - 1ull)) : 0;
      off1[a1] = (uint32_t)r0;
      for (int dt = 0; dt < 2; ++dt) {
        if (acc[dt] + len + pe[dt] > 0xffffffffull) {
          set_error("padded layout exceeds 32-bit element offsets");
          return QK_EUNSUPPORTED;
        }
        poff1[dt][a1] = (uint32_t)acc[dt];
        for (uint64_t i = 0; i < len; i += (uint64_t)pe[dt]) {
          lr0[dt].push_back((uint32_t)(r0 + i));
          lnn[dt].push_back((uint8_t)std::min<uint64_t>((uint64_t)pe[dt], len - i));
        }
        acc[dt] += (len + pe[dt] - 1) / pe[dt] * pe[dt];
      }
    }
    for (int dt = 0; dt < 2; ++dt) {
      t->dpad[dt] = acc[dt];
      t->nline[dt] = lr0[dt].size();
    }
  }

  // ---- high pass: blocks grouped by class, in each class by descending
  // number of active high bonds (the lanes of a wave then run similar loops)
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> byk(llo1 + 1);   // (active bonds, a1)
  for (uint64_t a1 = 0; a1 < n1; ++a1) {
    const int k1 = N - __builtin_popcountll(a1);
    if (k1 < 0 || k1 > llo1) continue;
    const uint32_t nact = (uint32_t)__builtin_popcountll((a1 ^ (a1 >> 1)) & ((1ull << (lhi1 - 1)) - 1ull));
    byk[k1].push_back({nact, (uint32_t)a1});
  }
  std::vector<uint32_t> coff, ca, cpoff[2];
  std::vector<uint32_t> cstart(llo1 + 2, 0), ccount(llo1 + 1, 0);
  for (int k1 = 0; k1 <= llo1; ++k1) {
    cstart[k1] = (uint32_t)coff.size();
    std::stable_sort(byk[k1].begin(), byk[k1].end(),
                     [](const std::pair<uint32_t, uint32_t>& x, const std::pair<uint32_t, uint32_t>& y) {
                       return x.first > y.first;
                     });
    for (const auto& pr : byk[k1]) {
      coff.push_back(off1[pr.second]);
      ca.push_back(pr.second);
      cpoff[0].push_back(poff1[0][pr.second]);
      cpoff[1].push_back(poff1[1][pr.second]);
    }
    ccount[k1] = (uint32_t)byk[k1].size();
  }
  t->nhi = (int)coff.size();
  // slab schedules: column slabs of each class whose lines fit the budget
  // (QK_SLAB_KB, default 1536 KiB of one XCD's 4 MiB L2), one line (128
  // bytes) of each block at least, consecutive slabs of a class on the same XCD
  const uint64_t budget = (uint64_t)env_int("QK_SLAB_KB", 1536) * 1024u;
  std::vector<SlabDesc> slabs[2];
  for (int dt = 0; dt < 2; ++dt) {
    const uint64_t sz = dt == 0 ? 16 : 8;
    std::vector<uint64_t> elems;
    for (int k1 = 0; k1 <= llo1; ++k1) {
      const uint32_t nb = ccount[k1];
      if (!nb) continue;
      const uint32_t ncol = (uint32_t)hb.c[llo1][k1];
      uint32_t wl = 0;
      while ((1u << wl) * sz < (uint64_t)kPadBytes) ++wl;
      while (wl < 8 && (1u << wl) < ncol && (uint64_t)nb * (2u << wl) * sz <= budget) ++wl;
      for (uint32_t j0 = 0; j0 < ncol; j0 += (1u << wl)) {
        SlabDesc d{};
        d.list0 = cstart[k1];
        d.nb = nb;
        d.j0 = (uint16_t)j0;
        d.ncol = (uint16_t)ncol;
        d.wlog = (uint16_t)wl;
        d.k = (uint16_t)k1;
        slabs[dt].push_back(d);
        elems.push_back((uint64_t)nb * std::min<uint32_t>(1u << wl, ncol - j0));
      }
    }
    uint64_t total = 0;
    for (uint64_t v : elems) total += v;
    uint64_t acc = 0;
    int x = 1;
    t->xcd_slab[dt][0] = 0;
    for (size_t i = 0; i < elems.size() && x < kNumXcd; ++i) {
      acc += elems[i];
      while (x < kNumXcd && acc * kNumXcd >= total * (uint64_t)x) t->xcd_slab[dt][x++] = (uint32_t)(i + 1);
    }
    while (x <= kNumXcd) t->xcd_slab[dt][x++] = (uint32_t)elems.size();
  }

  // ---- low pass: blocks of the split at llo2, their ring pairs, low states
  std::vector<BlkEntry> lo;
  std::vector<int32_t> idx2(1ull << lhi2, -1);
  for (uint64_t a2 = 0; a2 < (1ull << lhi2); ++a2) {
    const int k2 = N - __builtin_popcountll(a2);
    if (k2 < 0 || k2 > llo2) continue;
    BlkEntry e{};
    e.a = (uint32_t)a2;
    e.off = (uint32_t)hb.rank((a2 << llo2) | ((1ull << k2) - 1ull));
    uint32_t n = 0;
    for (int q = 0; q + 1 < lhi2; ++q)
      if (((a2 >> q) ^ (a2 >> (q + 1))) & 1ull) ++n;
    e.nact = n;   // anti-aligned high bonds, for the block part of the diagonal
    // padded first element: that of its first half, the llo1 block 2 a2
    e.pad[0] = poff1[0][2 * a2];
    e.pad[1] = poff1[1][2 * a2];
    idx2[a2] = (int32_t)lo.size();
    lo.push_back(e);
  }
  t->nlo = (int)lo.size();
  const uint64_t topb = 1ull << (lhi2 - 1);
  std::vector<PairTask> task;
  size_t maxlen = 0;
  auto len_of = [&](int32_t i) -> size_t {
    return i < 0 ? 0 : (size_t)hb.c[llo2][N - __builtin_popcount(lo[i].a)];
  };
  for (uint64_t a2 = 0; a2 < (1ull << lhi2); ++a2) {
    PairTask p{-1, -1};
    if (H->p.pbc) {
      // every block belongs to exactly one task: the one of its top-bit-0 pattern
      if (a2 & topb) continue;
      p.a = idx2[a2];
      p.b = idx2[a2 | topb];
      if (p.a < 0 && p.b < 0) continue;
    } else {
      if (idx2[a2] < 0) continue;
      p.a = idx2[a2];
    }
    task.push_back(p);
    maxlen = std::max(maxlen, len_of(p.a) + len_of(p.b));
  }
  t->ntask = (int)task.size();
  t->maxtask = (int)maxlen;
  // low states: the j-th state of popcount k sits at lo_base[k] + j
  std::vector<uint16_t> lstate(1u << llo2), lrank(1u << llo2);
  {
    uint32_t acc = 0;
    for (int k = 0; k <= llo2; ++k) {
      t->lo_base[k] = acc;
      acc += (uint32_t)hb.c[llo2][k];
    }
    for (uint32_t b = 0; b < (1u << llo2); ++b) {
      lrank[b] = (uint16_t)hb.rank(b);
      lstate[t->lo_base[__builtin_popcount(b)] + lrank[b]] = (uint16_t)b;
    }
  }
  // padded binomials C'(n, k), n >= llo1: C(llo1, k) rounded up to whole
  // lines, Pascal's rule above; the padded first element of every block is
  // their CNS sum (checked here against the running offsets)
  std::vector<uint32_t> binp[2] = {std::vector<uint32_t>(kBinomStride * kBinomStride, 0),
                                   std::vector<uint32_t>(kBinomStride * kBinomStride, 0)};
  for (int dt = 0; dt < 2; ++dt) {
    std::vector<uint64_t> cp((size_t)kBinomStride * kBinomStride, 0);
    for (int k = 0; k <= llo1; ++k) cp[llo1 * kBinomStride + k] = (hb.c[llo1][k] + pe[dt] - 1) / pe[dt] * pe[dt];
    for (int n = llo1 + 1; n < kBinomStride; ++n)
      for (int k = 0; k < kBinomStride; ++k)
        cp[n * kBinomStride + k] = cp[(n - 1) * kBinomStride + k] + (k > 0 ? cp[(n - 1) * kBinomStride + k - 1] : 0);
    for (uint64_t a1 = 0; a1 < n1; ++a1) {
      const int k1 = N - __builtin_popcountll(a1);
      if (k1 < 0 || k1 > llo1) continue;
      uint64_t v = 0;
      int i = 1;
      for (uint64_t x = a1; x; x &= x - 1) v += cp[(size_t)(llo1 + __builtin_ctzll(x)) * kBinomStride + k1 + i++];
      if (v != poff1[dt][a1]) {
        set_error("padded offsets disagree with their binomial sums");
        return QK_EUNSUPPORTED;
      }
    }
    for (size_t i = 0; i < cp.size(); ++i) binp[dt][i] = cp[i] > 0xffffffffull ? 0xffffffffu : (uint32_t)cp[i];
  }

  hipError_t e = upload(H->al, &t->coff, coff);
  if (e == hipSuccess) e = upload(H->al, &t->ca, ca);
  for (int dt = 0; dt < 2 && e == hipSuccess; ++dt) {
    e = upload(H->al, &t->cpoff[dt], cpoff[dt]);
    if (e == hipSuccess) e = upload(H->al, &t->slab[dt], slabs[dt]);
    if (e == hipSuccess) e = upload(H->al, &t->line_r0[dt], lr0[dt]);
    if (e == hipSuccess) e = upload(H->al, &t->line_n[dt], lnn[dt]);
  }
  if (e == hipSuccess) e = upload(H->al, &t->lo, lo);
  if (e == hipSuccess) e = upload(H->al, &t->lo_state, lstate);
  if (e == hipSuccess) e = upload(H->al, &t->lo_rank, lrank);
  if (e == hipSuccess) e = upload(H->al, &t->binp[0], binp[0]);
  if (e == hipSuccess) e = upload(H->al, &t->binp[1], binp[1]);
  if (e == hipSuccess) e = upload(H->al, &t->task, task);
  QK_HIP(e);
  qk_status st = split_fields(H, s);
  if (st != QK_OK) return st;
  QK_HIP(hipStreamSynchronize(s));
  return QK_OK;
}

bool split_usable(const qk_ham* H) { return H->split != nullptr; }

uint64_t split_padded_len(const qk_ham* H, int dtype) {
  const SplitTables* t = tables(H);
  return t ? t->dpad[dtype == QK_C128 ? 0 : 1] : 0;
}

static HiArgs hi_args(const qk_ham* H, int dtype, bool x_pad, bool um_pad, bool z_pad) {
  const SplitTables* t = tables(H);
  const int dt = dtype == QK_C128 ? 0 : 1;
  HiArgs a{};
  a.coff = t->coff;
  a.cpoff = t->cpoff[dt];
  a.ca = t->ca;
  a.slab = t->slab[dt];
  a.binom = x_pad ? t->binp[dt] : H->basis->d_binom;
  for (int i = 0; i <= kNumXcd; ++i) a.xcd_slab[i] = t->xcd_slab[dt][i];
  a.llo1 = t->llo2 - 1;
  a.lhi1 = H->basis->L - a.llo1;
  a.x_pad = x_pad;
  a.um_pad = um_pad;
  a.z_pad = z_pad;
  a.half_jxy = 0.5 * H->p.jxy;
  return a;
}

static LoArgs lo_args(const qk_ham* H, int dtype, bool x_pad, bool z_pad, bool out_pad) {
  const SplitTables* t = tables(H);
  LoArgs a{};
  a.L = H->basis->L;
  a.N = H->basis->N;
  a.pbc = H->p.pbc;
  a.lhi = H->basis->L - t->llo2;
  a.half_jxy = 0.5 * H->p.jxy;
  a.jz = H->p.jz;
  a.blk = t->lo;
  a.task = t->task;
  a.ntask = t->ntask;
  a.lo_state = t->lo_state;
  a.lo_rank = t->lo_rank;
  a.binom = H->basis->d_binom;
  a.fields = H->d_fields;
  for (int k = 0; k < 18; ++k) a.lo_base[k] = t->lo_base[k];
  a.dt = dtype == QK_C128 ? 0 : 1;
  a.pad_elems = kPadBytes / (dtype == QK_C128 ? 16 : 8);
  a.x_pad = x_pad;
  a.z_pad = z_pad;
  a.out_pad = out_pad;
  return a;
}

// Work-groups of the high pass: a multiple of the XCD count (QK_SPLIT_HI_WGS
// per CU, default the kernel's occupancy, at most 8).
template <typename T, bool LANCZOS>
static int hi_grid(int wgs_req) {
  static const int occ = []() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_split_hi<T, LANCZOS>, kHiThreads, 0) != hipSuccess || n < 1)
      n = 1;
    return n;
  }();
  int w = wgs_req > 0 ? wgs_req : env_int("QK_SPLIT_HI_WGS", occ < 8 ? occ : 8);
  if (w > occ) w = occ;
  int G = ((qk_num_cus() * w) / kNumXcd) * kNumXcd;
  if (G < kNumXcd) G = kNumXcd;
  if (G > kMaxPartialBlocks) G = kMaxPartialBlocks - kMaxPartialBlocks % kNumXcd;
  return G;
}

template <typename T, bool LANCZOS>
static qk_status launch_hi_t(const HiArgs& ha, const void* x, const void* um, void* z, const KState* st,
                             const LanczosArgs* la, const double* partB, int GB, double* partA, int* grid, int wgs,
                             hipStream_t s) {
  using V = typename Cx<T>::V;
  const int G = hi_grid<T, LANCZOS>(wgs);
  KState stv{};
  LanczosArgs lav{};
  if (st) stv = *st;
  if (la) lav = *la;
  hipLaunchKernelGGL((k_split_hi<T, LANCZOS>), dim3(G), dim3(kHiThreads), 0, s, ha, (const V*)x, (const V*)um, (V*)z,
                     stv, lav, partB, GB, partA);
  QK_HIP(hipGetLastError());
  if (grid) *grid = G;
  return QK_OK;
}

template <typename T, int LLO, int MODE>
static qk_status launch_lo_llo(const qk_ham* H, const LoArgs& la_, const void* x, const void* zin, void* out,
                               const KState* st, const LanczosArgs* la, const double* partA, int GA,
                               const double* partBin, const double* partQin, int GB, double* partBout,
                               double* partQout, int store, int* grid, hipStream_t s) {
  using V = typename Cx<T>::V;
  const SplitTables* t = tables(H);
  const size_t dyn = sizeof(V) * (size_t)(t->maxtask > 0 ? t->maxtask : 1);
  if ((size_t)t->maxtask > (size_t)lo_threads<LLO>() * lo_elems<LLO>()) {
    set_error("low-pass task larger than the kernel's element slots");
    return QK_EUNSUPPORTED;
  }
  auto kern = k_split_lo<T, LLO, MODE>;
  QK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, lo_threads<LLO>(), dyn) != hipSuccess || occ < 1)
    occ = 1;
  int G = qk_num_cus() * occ;
  if (G > t->ntask) G = t->ntask;
  if (G > kMaxPartialBlocks) G = kMaxPartialBlocks;
  if (G < 1) G = 1;
  KState stv{};
  LanczosArgs lav{};
  if (st) stv = *st;
  if (la) lav = *la;
  hipLaunchKernelGGL(kern, dim3(G), dim3(lo_threads<LLO>()), dyn, s, la_, (const V*)x, (const V*)zin, (V*)out, stv,
                     lav, partA, GA, partBin, partQin, GB, partBout, partQout, store);
  QK_HIP(hipGetLastError());
  if (grid) *grid = G;
  return QK_OK;
}

template <typename T, int MODE>
static qk_status launch_lo_t(const qk_ham* H, const LoArgs& la_, const void* x, const void* zin, void* out,
                             const KState* st, const LanczosArgs* la, const double* partA, int GA,
                             const double* partBin, const double* partQin, int GB, double* partBout, double* partQout,
                             int store, int* grid, hipStream_t s) {
  switch (tables(H)->llo2) {
    case 10:
      return launch_lo_llo<T, 10, MODE>(H, la_, x, zin, out, st, la, partA, GA, partBin, partQin, GB, partBout,
                                        partQout, store, grid, s);
    case 11:
      return launch_lo_llo<T, 11, MODE>(H, la_, x, zin, out, st, la, partA, GA, partBin, partQin, GB, partBout,
                                        partQout, store, grid, s);
    case 12:
      return launch_lo_llo<T, 12, MODE>(H, la_, x, zin, out, st, la, partA, GA, partBin, partQin, GB, partBout,
                                        partQout, store, grid, s);
    case 13:
      return launch_lo_llo<T, 13, MODE>(H, la_, x, zin, out, st, la, partA, GA, partBin, partQin, GB, partBout,
                                        partQout, store, grid, s);
    default: set_error("no low-pass kernel for this low-bit count"); return QK_EUNSUPPORTED;
  }
}

// y = H x: the high pass writes y = H_hi x, the low pass adds the rest in place.
qk_status launch_split_apply(const qk_ham* H, const void* x, void* y, int dtype, hipStream_t s) {
  const HiArgs ha = hi_args(H, dtype, false, false, false);
  const LoArgs la = lo_args(H, dtype, false, false, false);
  if (dtype == QK_C128) {
    qk_status st = launch_hi_t<double, false>(ha, x, nullptr, y, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, s);
    if (st != QK_OK) return st;
    return launch_lo_t<double, kLoApply>(H, la, x, y, y, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr,
                                         nullptr, 0, nullptr, s);
  }
  qk_status st = launch_hi_t<float, false>(ha, x, nullptr, y, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, s);
  if (st != QK_OK) return st;
  return launch_lo_t<float, kLoApply>(H, la, x, y, y, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr,
                                      nullptr, 0, nullptr, s);
}

qk_status launch_split_form(const qk_ham* H, int dtype, const void* x, double* partB, double* partQ, int* grid,
                            hipStream_t s) {
  const LoArgs la = lo_args(H, dtype, false, false, false);
  if (dtype == QK_C128)
    return launch_lo_t<double, kLoForm>(H, la, x, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0,
                                        partB, partQ, 0, grid, s);
  return launch_lo_t<float, kLoForm>(H, la, x, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0,
                                     partB, partQ, 0, grid, s);
}

// Iteration j: u_j is the caller's psi (sorted layout) at j = 0 and a padded
// workspace vector after; u_{j-1} likewise; z and u_{j+1} are padded.
qk_status launch_split_hi(const qk_ham* H, int dtype, const void* uj, const void* ujm1, void* z, const KState& st,
                          const LanczosArgs& la, const double* partB, int GB, double* partA, int* grid, int wgs,
                          hipStream_t s) {
  const HiArgs ha = hi_args(H, dtype, la.j > 0, la.j > 1, true);
  if (dtype == QK_C128) return launch_hi_t<double, true>(ha, uj, ujm1, z, &st, &la, partB, GB, partA, grid, wgs, s);
  return launch_hi_t<float, true>(ha, uj, ujm1, z, &st, &la, partB, GB, partA, grid, wgs, s);
}

qk_status launch_split_lo(const qk_ham* H, int dtype, const void* uj, const void* z, void* out, const KState& st,
                          const LanczosArgs& la, const double* partA, int GA, const double* partBin,
                          const double* partQin, int GB, double* partBout, double* partQout, int store, int* grid,
                          hipStream_t s) {
  const LoArgs lo = lo_args(H, dtype, la.j > 0, true, true);
  if (dtype == QK_C128)
    return launch_lo_t<double, kLoLanczos>(H, lo, uj, z, out, &st, &la, partA, GA, partBin, partQin, GB, partBout,
                                           partQout, store, grid, s);
  return launch_lo_t<float, kLoLanczos>(H, lo, uj, z, out, &st, &la, partA, GA, partBin, partQin, GB, partBout,
                                        partQout, store, grid, s);
}

// psi <- combination of psi and the padded Krylov vectors U (one field set).
qk_status launch_split_combine(const qk_ham* H, int dtype, void* psi, const void* U, const KState& st, hipStream_t s) {
  const SplitTables* t = tables(H);
  const int dt = dtype == QK_C128 ? 0 : 1;
  const uint64_t n = t->dpad[dt];
  uint64_t G = (n + kMaxBlock - 1) / kMaxBlock;
  const uint64_t cap = (uint64_t)qk_num_cus() * 8;
  if (G > cap) G = cap;
  if (G < 1) G = 1;
  const int pe = kPadBytes / (dtype == QK_C128 ? 16 : 8);
  if (dtype == QK_C128)
    hipLaunchKernelGGL(k_combine_pad<double>, dim3((unsigned)G), dim3(kMaxBlock), 0, s, (double2*)psi,
                       (const double2*)U, n, t->line_r0[dt], t->line_n[dt], pe, st);
  else
    hipLaunchKernelGGL(k_combine_pad<float>, dim3((unsigned)G), dim3(kMaxBlock), 0, s, (float2*)psi,
                       (const float2*)U, n, t->line_r0[dt], t->line_n[dt], pe, st);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

// Row map of the padded layout for other kernels (the adjoint contraction).
qk_status split_line_tables(const qk_ham* H, int dtype, const uint32_t** r0, const uint8_t** n, uint64_t* dpad,
                            int* pe) {
  const SplitTables* t = tables(H);
  if (!t) return QK_EUNSUPPORTED;
  const int dt = dtype == QK_C128 ? 0 : 1;
  *r0 = t->line_r0[dt];
  *n = t->line_n[dt];
  *dpad = t->dpad[dt];
  *pe = kPadBytes / (dtype == QK_C128 ? 16 : 8);
  return QK_OK;
}

}  // namespace qk

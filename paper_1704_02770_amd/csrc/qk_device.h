// Device-side helpers shared by the HIP kernels of libqkrylov: complex
// vector types, ranking in the sorted basis, the model rows of Eq. (1),
// the XCD-aware tile walk and deterministic block reductions.
#pragma once

#include "qk_internal.h"

namespace qk {

template <typename T> struct Cx;
template <> struct Cx<double> { using V = double2; };
template <> struct Cx<float> { using V = float2; };

// ------------------------------------------------------------------ ranking
__device__ __forceinline__ int popc(uint32_t s) { return __popc(s); }
__device__ __forceinline__ int popc(uint64_t s) { return __popcll(s); }
__device__ __forceinline__ int ctz(uint32_t s) { return __builtin_ctz(s); }
__device__ __forceinline__ int ctz(uint64_t s) { return __builtin_ctzll(s); }

// Position of a state in the sorted basis: with set bits at p_1 < ... < p_N,
// the number of sector states below it is sum_k C(p_k, k) (the counting that
// the sorted order of Sec. 2 implies; the paper finds it by binary lookup).
template <typename S>
__device__ __forceinline__ uint32_t cns_rank(S s, const uint32_t* tab) {
  constexpr int K = StateT<S>::kStride;
  uint32_t r = 0;
  int k = 1;
  while (s) {
    const int p = ctz(s);
    r += tab[p * K + k];
    ++k;
    s &= s - (S)1;
  }
  return r;
}

// The r-th state of the sorted basis (Algorithm 3's first_int()).
template <typename S>
__device__ __forceinline__ S cns_unrank(uint32_t r, int L, int N, const uint32_t* tab) {
  constexpr int K = StateT<S>::kStride;
  S s = 0;
  int k = N;
  for (int p = L - 1; p >= 0 && k > 0; --p) {
    const uint32_t c = tab[p * K + k];
    if (r >= c) {
      s |= (S)1 << p;
      r -= c;
      --k;
    }
  }
  return s;
}

// Next larger integer with the same popcount (Algorithm 2).  The paper's
// exact division of two powers of two is a right shift by ctz(v).
template <typename S>
__device__ __forceinline__ S next_perm(S v) {
  const S t = (v | (v - (S)1)) + (S)1;
  return t | ((((t & ((S)0 - t)) >> ctz(v)) >> 1) - (S)1);
}

// ------------------------------------------------------------- model rows
template <typename S>
__device__ __forceinline__ int anti_bonds(S s, const ModelArgs& a) {
  const S mask = (S)a.lmask;
  if (a.pbc) {
    const S rot = ((s >> 1) | (s << (a.L - 1))) & mask;
    return popc((S)((s ^ rot) & mask));
  }
  return popc((S)((s ^ (s >> 1)) & (mask >> 1)));
}

// Diagonal of Eq. (1): jz/4 * (aligned - anti-aligned bonds) + sum_i h_i (bit_i - 1/2).
template <typename S>
__device__ __forceinline__ double diag_value(S s, const ModelArgs& a, const double* f, double hhalf) {
  const int nb = a.pbc ? a.L : a.L - 1;
  double d = 0.25 * a.jz * (double)(nb - 2 * anti_bonds(s, a)) - hhalf;
  S t = s;
  while (t) {
    d += f[ctz(t)];
    t &= t - (S)1;
  }
  return d;
}

// Calls f(column) for every bond whose bits differ.  A particle hopping
// p -> p+1 raises the rank by C(p, #set bits below p); p+1 -> p lowers it by
// the same amount.  The ring bond (L-1, 0) renumbers every particle and is
// ranked in full.
template <typename S, class F>
__device__ __forceinline__ void for_each_hop(S s, uint32_t r, const ModelArgs& a, const uint32_t* tab, F&& f) {
  constexpr int K = StateT<S>::kStride;
  int pc = 0;
  for (int p = 0; p < a.L - 1; ++p) {
    const uint32_t b0 = (uint32_t)(s >> p) & 1u;
    const uint32_t b1 = (uint32_t)(s >> (p + 1)) & 1u;
    if (b0 != b1) {
      const uint32_t c = tab[p * K + pc];
      f(b0 ? r + c : r - c);
    }
    pc += (int)b0;
  }
  if (a.pbc) {
    const uint32_t b0 = (uint32_t)s & 1u, b1 = (uint32_t)(s >> (a.L - 1)) & 1u;
    if (b0 != b1) f(cns_rank<S>(s ^ ((S)1 | ((S)1 << (a.L - 1))), tab));
  }
}

// Per-block LDS copies of the small tables every row kernel needs.
template <typename S>
struct RowShared {
  uint32_t tab[StateT<S>::kStride * StateT<S>::kStride];
  double fld[kFldCap];
  double hhalf[QK_MAX_BATCH];
};

template <typename S>
__device__ __forceinline__ void load_row_shared(RowShared<S>& sh, const ModelArgs& a, const uint32_t* gtab,
                                                const double* gfields) {
  constexpr int K = StateT<S>::kStride;
  for (int i = threadIdx.x; i < K * K; i += blockDim.x) sh.tab[i] = gtab[i];
  for (int i = threadIdx.x; i < a.B * a.L; i += blockDim.x) sh.fld[i] = gfields[i];
  __syncthreads();
  for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < a.L; ++i) t += sh.fld[b * a.L + i];
    sh.hhalf[b] = 0.5 * t;
  }
  __syncthreads();
}

template <typename S>
struct HamView {
  const S* states;
  const uint32_t* rowptr;
  const uint32_t* cols;
  const double* diag;
  uint32_t D;
};

// (H x)[r, b] and x[r, b].
template <typename T, bool CSR, typename S>
__device__ __forceinline__ typename Cx<T>::V h_row(uint32_t r, int b, const ModelArgs& a, const RowShared<S>& sh,
                                                   const HamView<S>& hv, const typename Cx<T>::V* __restrict__ x,
                                                   typename Cx<T>::V& xr) {
  using V = typename Cx<T>::V;
  const int B = a.B;
  xr = x[(size_t)r * B + b];
  const T g = (T)a.half_jxy;
  V acc;
  if (CSR) {
    const T d = (T)hv.diag[(size_t)r * B + b];
    acc.x = d * xr.x;
    acc.y = d * xr.y;
    V hs = {0, 0};
    for (uint32_t k = hv.rowptr[r]; k < hv.rowptr[r + 1]; ++k) {
      const V xc = x[(size_t)hv.cols[k] * B + b];
      hs.x += xc.x;
      hs.y += xc.y;
    }
    acc.x += g * hs.x;
    acc.y += g * hs.y;
  } else {
    const S s = hv.states[r];
    const T d = (T)diag_value<S>(s, a, sh.fld + b * a.L, sh.hhalf[b]);
    acc.x = d * xr.x;
    acc.y = d * xr.y;
    V hs = {0, 0};
    for_each_hop<S>(s, r, a, sh.tab, [&](uint32_t c) {
      const V xc = x[(size_t)c * B + b];
      hs.x += xc.x;
      hs.y += xc.y;
    });
    acc.x += g * hs.x;
    acc.y += g * hs.y;
  }
  return acc;
}

// The block index and block count a kernel body works with.  A plain launch
// passes (blockIdx.x, gridDim.x); the persistent step kernel (qk_persist.hip)
// passes the tile it has claimed and the tile count of that pass, so a body
// produces the same values, partial sums included, either way.
struct VGrid {
  uint32_t id, n;
};
__device__ __forceinline__ VGrid hw_grid() { return VGrid{blockIdx.x, gridDim.x}; }

// A run of consecutive virtual blocks v0 .. v1-1 of a grid of n, taken by one
// work-group one after another: what a block's results depend on (tables,
// the scalars reduced from the previous pass) is set up once for the run,
// then each virtual block does its own rows and writes its own partial sums.
struct VRange {
  uint32_t v0, v1, n;
};
__device__ __forceinline__ VRange hw_range() { return VRange{blockIdx.x, blockIdx.x + 1, gridDim.x}; }

// XCD-aware tile walk: work-groups are dealt round-robin to the 8 XCDs, so
// block i runs on XCD i % 8.  Each XCD gets one contiguous eighth of the row
// tiles, and its blocks stride through that eighth together, which keeps the
// rows being read on one XCD close together in that XCD's L2.
struct TileWalk {
  uint32_t t, t_end, step;
  __device__ TileWalk(uint32_t ntiles, VGrid g) {
    if (g.n % kNumXcd) {   // a grid that does not split evenly over the XCDs: plain grid stride
      t = g.id;
      t_end = ntiles;
      step = g.n;
      return;
    }
    const uint32_t x = g.id % kNumXcd, k = g.id / kNumXcd, per = g.n / kNumXcd;
    const uint32_t t0 = (uint32_t)(((uint64_t)ntiles * x) / kNumXcd);
    t_end = (uint32_t)(((uint64_t)ntiles * (x + 1)) / kNumXcd);
    t = t0 + k;
    step = per;
  }
};

// ------------------------------------------------------ block reductions
// Sums each of Q values over the threads of the block that share a batch
// column (threadIdx % B; blockDim = B * 2^k) by a fixed tree in LDS and
// writes the Q * B column sums to out_block.
template <int Q>
__device__ __forceinline__ void block_partials(const double (&v)[Q], int B, double* red, double* out_block) {
  // red: LDS scratch of Q * blockDim doubles
  for (int q = 0; q < Q; ++q) red[q * blockDim.x + threadIdx.x] = v[q];
  __syncthreads();
  for (int s = blockDim.x / 2; s >= B; s >>= 1) {
    if (threadIdx.x < (unsigned)s)
      for (int q = 0; q < Q; ++q) red[q * blockDim.x + threadIdx.x] += red[q * blockDim.x + threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)B)
    for (int q = 0; q < Q; ++q) out_block[q * B + threadIdx.x] = red[q * blockDim.x + threadIdx.x];
}

// Reduces partials part[g][q][b] over g < G in a fixed order; every block
// computes identical totals.  out[q * B + b] in LDS, valid after return.
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int G, int Q, int B, double* red,
                                                double* out) {
  const int cols = Q * B;
  const int lanes_per_col = blockDim.x / cols > 0 ? blockDim.x / cols : 1;
  const int c = threadIdx.x % cols;
  const int g0 = threadIdx.x / cols;
  double acc = 0.0;
  if ((int)threadIdx.x < cols * lanes_per_col)
    for (int g = g0; g < G; g += lanes_per_col) acc += part[(size_t)g * cols + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < cols) {
    double t = 0.0;
    for (int l = 0; l < lanes_per_col; ++l) t += red[l * cols + threadIdx.x];
    out[threadIdx.x] = t;
  }
  // columns beyond blockDim (Q * B > blockDim) are reduced serially
  for (int cc = blockDim.x + threadIdx.x; cc < cols; cc += blockDim.x) {
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += part[(size_t)g * cols + cc];
    out[cc] = t;
  }
  __syncthreads();
}

// ------------------------------------------------------- Lanczos passes
// Stored vectors u_j are unnormalised: v_j = sigma_j u_j.  Iteration j:
//   pass A:  w = a_j H u_j - b_j u_{j-1}      (= H v_j - beta_{j-1} v_{j-1}, or H u_0 at j = 0)
//            partials  Re<u_j, w>, |u_j|^2
//   pass B:  u_{j+1} = c_j (w - d_j u_j)       (= w - alpha_j v_j in v-units)
//            partial   |u_{j+1}|^2  -> beta_j
// The scalars come from the previous pass's partials, reduced in each block.
struct LanczosArgs {
  int j, m;
  double breakdown_rtol;
  int reorth;   // 1: the update pass also removes the component along v_{j-1}
};

// Partial sums of the H-pass per batch column: Re<u_j, w>, |u_j|^2 and the
// complex <u_{j-1}, w> used by the local reorthogonalisation.
constexpr int kQA = 4;



// (exp(-i tau T) e_1)_i in lane i of one wavefront, for the real symmetric
// tridiagonal T with diagonal al (lane i), coupling be to component i+1 and bl
// to component i-1 (zero outside the used dimension; `on` marks used lanes).
// T is shifted by the centre mu of its Gershgorin interval, the time is cut
// into substeps with |tau_s| * radius <= 1/2, and each substep sums the Taylor
// series of the exponential applied to the vector until the terms fall below
// 1e-18 of the sum; the phase exp(-i tau mu) is applied at the end.  All 64
// lanes must call it (it uses cross-lane shuffles).
__device__ __forceinline__ void tri_expm_e1(double al, double be, double bl, bool on, int i, double tau, double& er,
                                            double& ei) {
  double lo = on ? al - be - bl : INFINITY, hi = on ? al + be + bl : -INFINITY;
  for (int s = 32; s > 0; s >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, s));
    hi = fmax(hi, __shfl_xor(hi, s));
  }
  const double mu_shift = 0.5 * (lo + hi);
  const double radius = 0.5 * (hi - lo);
  const double ad = on ? al - mu_shift : 0.0;
  // bounded substep count (a non-finite or huge norm cannot stall the wave)
  const double nsd = ceil(fabs(tau) * radius / 0.5);
  const int nsub = (nsd >= 1.0 && nsd <= 100000.0) ? (int)nsd : (nsd > 100000.0 ? 100000 : 1);
  const double ts = tau / nsub;
  double vr = (i == 0) ? 1.0 : 0.0, vi = 0.0;
  for (int sub = 0; sub < nsub; ++sub) {
    double sr = vr, si = vi, tr = vr, ti = vi;
    for (int k = 1; k <= 40; ++k) {
      // t <- (-i ts / k) (T - mu) t
      const double up_r = __shfl_up(tr, 1), up_i = __shfl_up(ti, 1);
      const double dn_r = __shfl_down(tr, 1), dn_i = __shfl_down(ti, 1);
      double yr = ad * tr + (i > 0 ? bl * up_r : 0.0) + (i < 63 ? be * dn_r : 0.0);
      double yi = ad * ti + (i > 0 ? bl * up_i : 0.0) + (i < 63 ? be * dn_i : 0.0);
      if (!on) yr = yi = 0.0;
      const double f = ts / k;
      tr = f * yi;    // (-i f) (yr + i yi) = f yi - i f yr
      ti = -f * yr;
      sr += tr;
      si += ti;
      double tn = fabs(tr) + fabs(ti), sn = fabs(sr) + fabs(si);
      for (int s = 32; s > 0; s >>= 1) {
        tn = fmax(tn, __shfl_xor(tn, s));
        sn = fmax(sn, __shfl_xor(sn, s));
      }
      if (tn <= 1e-18 * sn) break;
    }
    vr = sr;
    vi = si;
  }
  const double cr = cos(tau * mu_shift), ci = -sin(tau * mu_shift);
  er = vr * cr - vi * ci;
  ei = vr * ci + vi * cr;
}

// Scalars of the H-pass of Lanczos iteration j for every batch column b,
// from the update pass of iteration j-1 (its partial sums |u_j|^2):
//   sa[b] = sigma_j, sb[b] = beta_{j-1} sigma_{j-1}, act[b] = column still running.
// Block 0 (of the virtual grid g) records beta_{j-1}, sigma_j, and m_used / status on breakdown or a
// non-finite norm.  Every block reduces the same partials in the same order,
// so all blocks reach the same decisions.
__device__ __forceinline__ void lanczos_h_scalars(int B, const KState& st, const LanczosArgs& la,
                                                  const double* __restrict__ partB, int Gp, double* red, double* tot,
                                                  double* sa, double* sb, int* act, VGrid g) {
  const int j = la.j;
  const bool first = g.id == 0;   // the block that records the shared results
  if (j == 0) {
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
      sa[b] = 1.0;
      sb[b] = 0.0;
      act[b] = 1;
      if (first) {
        st.mused[b] = la.m;
        st.status[b] = QK_OK;
      }
    }
    __syncthreads();
  } else {
    reduce_partials(partB, Gp, 1, B, red, tot);
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
      int active = st.mused[b] > j;
      const double beta = sqrt(tot[b]);
      if (active) {
        double scale = beta;
        for (int i = 0; i < j; ++i) scale = fmax(scale, fabs(st.alpha[i * B + b]));
        for (int i = 0; i + 1 < j; ++i) scale = fmax(scale, st.beta[i * B + b]);
        if (!isfinite(beta)) {
          active = 0;
          if (first) {
            st.status[b] = QK_ENUMERIC;
            st.mused[b] = j;
          }
        } else if (beta <= la.breakdown_rtol * scale) {
          active = 0;  // invariant subspace: the Krylov space stops at dimension j
          if (first) st.mused[b] = j;
        }
        if (first) st.beta[(j - 1) * B + b] = beta;
      }
      if (active) {
        sa[b] = 1.0 / beta;
        sb[b] = beta * st.sigma[(j - 1) * B + b];
        if (first) st.sigma[j * B + b] = 1.0 / beta;
      }
      act[b] = active;
    }
    __syncthreads();
  }

}


qk_status launch_blocked_lanczos_h(const qk_ham* H, int dtype, const void* uj, const void* ujm1, void* w,
                                   const KState& st, const LanczosArgs& la, const double* partB, int Gp,
                                   double* partA, int* grid_out, int wgs_per_cu, hipStream_t s);

// Two-pass split iteration (qk_split.hip): the pre-pass partials |x|^2 and
// Re<x, H_lo x> of a step's initial vector, the high pass
// z = sigma_j H_hi u_j - beta_{j-1} sigma_{j-1} u_{j-1}, and the low pass
// u_{j+1} = c (z + s H_lo u_j - d u_j) with the partials of the next iteration.
qk_status launch_split_form(const qk_ham* H, int dtype, const void* x, double* partB, double* partQ, int* grid,
                            hipStream_t s);
qk_status launch_split_hi(const qk_ham* H, int dtype, const void* uj, const void* ujm1, void* z, const KState& st,
                          const LanczosArgs& la, const double* partB, int GB, double* partA, int* grid, int wgs,
                          hipStream_t s);
qk_status launch_split_lo(const qk_ham* H, int dtype, const void* uj, const void* z, void* out, const KState& st,
                          const LanczosArgs& la, const double* partA, int GA, const double* partBin,
                          const double* partQin, int GB, double* partBout, double* partQout, int store, int* grid,
                          hipStream_t s);
qk_status launch_split_combine(const qk_ham* H, int dtype, void* psi, const void* U, const KState& st, hipStream_t s);

}  // namespace qk

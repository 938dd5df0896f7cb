// Kernel bodies of one Krylov step besides the blocked H-pass (Sec. 2
// "Krylov subspace methods"; rows of Eq. (1); the survival probability of
// Sec. 4): the row-form H-pass, the partial-sum totals, the update pass, the
// projected exponential, the combination and the overlap, as device functions
// over a virtual grid (VGrid), so that the plain launches of qk_kernels.hip
// and the persistent step kernel of qk_persist.hip run the same code.
#pragma once

#include "qk_device.h"

namespace qk {

HamView<uint32_t> ham_view32(const qk_ham* H);   // rows of a Hamiltonian with 32-bit states (host)

// LDS of the row-form H-pass.
template <typename S>
struct LanczosAShared {
  RowShared<S> sh;
  double red[kQA * kMaxBlock];
  double tot[QK_MAX_BATCH], sa[QK_MAX_BATCH], sb[QK_MAX_BATCH];
  int act[QK_MAX_BATCH];
};

// H-pass of Lanczos iteration j in row form (one thread per (row, column)),
// for sectors without block tables: w = sa H u_j - sb u_{j-1} with the
// partial sums of pass A (Sec. 2 "Krylov subspace methods"; rows of Eq. (1)).
template <typename T, bool CSR, typename S>
__device__ __forceinline__ void lanczos_a_body(VRange rg, LanczosAShared<S>& ls,
                                               const typename Cx<T>::V* __restrict__ uj,
                                               const typename Cx<T>::V* __restrict__ ujm1,
                                               typename Cx<T>::V* __restrict__ w, const ModelArgs& a,
                                               const HamView<S>& hv, const uint32_t* __restrict__ gtab,
                                               const double* __restrict__ gfields, const KState& st,
                                               const LanczosArgs& la, const double* __restrict__ partB, int Gp,
                                               double* __restrict__ partA) {
  using V = typename Cx<T>::V;
  RowShared<S>& sh = ls.sh;
  double* red = ls.red;
  double *tot = ls.tot, *sa = ls.sa, *sb = ls.sb;
  int* act = ls.act;
  load_row_shared(sh, a, gtab, gfields);
  const int B = a.B;
  lanczos_h_scalars(B, st, la, partB, Gp, red, tot, sa, sb, act, VGrid{rg.v0, rg.n});

  const int b = threadIdx.x % B;
  const uint32_t R = blockDim.x / B, rl = threadIdx.x / B;
  const uint32_t ntiles = (hv.D + R - 1) / R;
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb) {
    double s1 = 0.0, s2 = 0.0, s3r = 0.0, s3i = 0.0;
    if (act[b]) {
      const T ca = (T)sa[b], cb = (T)sb[b];
      for (TileWalk tw(ntiles, VGrid{vb, rg.n}); tw.t < tw.t_end; tw.t += tw.step) {
        const uint32_t r = tw.t * R + rl;
        if (r >= hv.D) continue;
        V xr;
        const V hx = h_row<T, CSR, S>(r, b, a, sh, hv, uj, xr);
        V wv;
        wv.x = ca * hx.x;
        wv.y = ca * hx.y;
        if (la.j > 0) {
          const V um = ujm1[(size_t)r * B + b];
          wv.x -= cb * um.x;
          wv.y -= cb * um.y;
          s3r += (double)um.x * (double)wv.x + (double)um.y * (double)wv.y;
          s3i += (double)um.x * (double)wv.y - (double)um.y * (double)wv.x;
        }
        w[(size_t)r * B + b] = wv;
        s1 += (double)xr.x * (double)wv.x + (double)xr.y * (double)wv.y;
        s2 += (double)xr.x * (double)xr.x + (double)xr.y * (double)xr.y;
      }
    }
    double v[kQA] = {s1, s2, s3r, s3i};
    block_partials<kQA>(v, B, red, partA + (size_t)vb * kQA * B);
    __syncthreads();   // red is written again by the next virtual block
  }
}

// Non-temporal load of one complex element, for vectors a pass reads once.
// Used only for vectors larger than the last-level cache (kNtBytes): there it
// makes the update pass 9 % and the combination 8 % faster (complex128,
// L = 28); for vectors that the 256 MB cache can hold (L = 24, 26) it is slower.
constexpr size_t kNtBytes = (size_t)256 << 20;
template <typename V>
__device__ __forceinline__ V ld_nt(const V* p) {
  using S = decltype(V{}.x);
  typedef S E __attribute__((ext_vector_type(2)));
  const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
  return V{e.x, e.y};
}

// Totals of per-block partial sums part[g][c] (g < G, c < cols) into tot[c],
// each column summed in a fixed order (32 lanes over g, then a fixed tree
// over the lanes), so every consumer reads one row instead of reducing G rows
// itself.  Used for batches of kPreReduceBatch items or more, where the
// G x cols partials make that per-block reduction the longest part of a pass.
constexpr int kPreReduceBatch = 8;
constexpr int kTotLanes = 32;                  // lanes per column
constexpr int kTotCols = 256 / kTotLanes;      // columns per block
// red: LDS scratch of 256 doubles; 256 threads.
__device__ __forceinline__ void partials_total_body(VRange rg, double* red, const double* __restrict__ part, int G,
                                                    int cols, double* __restrict__ tot) {
  const int tid = threadIdx.x;
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb) {
    const int c = (int)vb * kTotCols + tid / kTotLanes, l = tid % kTotLanes;
    double acc = 0.0;
    if (c < cols)
      for (int g = l; g < G; g += kTotLanes) acc += part[(size_t)g * cols + c];
    red[tid] = acc;
    __syncthreads();
    for (int h = kTotLanes / 2; h > 0; h >>= 1) {
      if (l < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (l == 0 && c < cols) tot[c] = red[tid];
    __syncthreads();   // red is written again by the next virtual block
  }
}

// LDS of the update pass.
struct LanczosBShared {
  double red[kMaxBlock];
  double tot[kQA * QK_MAX_BATCH];
  double sc[QK_MAX_BATCH], sd[QK_MAX_BATCH], ser[QK_MAX_BATCH], sei[QK_MAX_BATCH];
  int act[QK_MAX_BATCH];
};

// Update pass of Lanczos iteration j: u_{j+1} = c_j (w - d_j u_j) [- e_j u_{j-1}]
// in place of w (store != 0), with the partial sums |u_{j+1}|^2.
template <typename T, bool NT>
__device__ __forceinline__ void lanczos_b_body(VRange rg, LanczosBShared& ls,
                                               const typename Cx<T>::V* __restrict__ uj,
                                               const typename Cx<T>::V* __restrict__ ujm1,
                                               typename Cx<T>::V* __restrict__ w, uint32_t D, int B,
                                               const KState& st, const LanczosArgs& la,
                                               const double* __restrict__ partA, int Gp, double* __restrict__ partB,
                                               int store) {
  using V = typename Cx<T>::V;
  double* red = ls.red;
  double* tot = ls.tot;
  double *sc = ls.sc, *sd = ls.sd, *ser = ls.ser, *sei = ls.sei;
  int* act = ls.act;
  const bool first = rg.v0 == 0;   // the block that records the shared results
  const int j = la.j;
  const bool ro = la.reorth && j > 0;
  reduce_partials(partA, Gp, kQA, B, red, tot);
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    int active = st.mused[b] > j;
    if (active) {
      const double S1 = tot[b], S2 = tot[B + b];
      double alpha, c, d;
      if (j == 0) {
        const double n0 = sqrt(S2);
        alpha = S1 / S2;
        c = 1.0 / n0;
        d = alpha;
        if (first) {
          st.n0[b] = n0;
          st.sigma[b] = 1.0 / n0;
        }
        if (!(n0 > 0.0)) {
          active = 0;   // zero vector: nothing to propagate
          if (first) {
            st.mused[b] = 0;
            if (!isfinite(S2)) st.status[b] = QK_ENUMERIC;
          }
        }
      } else {
        const double sj = st.sigma[j * B + b];
        alpha = sj * S1;
        c = 1.0;
        d = alpha * sj;
      }
      if (active && !isfinite(alpha)) {
        active = 0;
        if (first) {
          st.status[b] = QK_ENUMERIC;
          st.mused[b] = j;
        }
      }
      if (active && first) st.alpha[j * B + b] = alpha;
      sc[b] = c;
      sd[b] = d;
      // component of w along v_{j-1}: <v_{j-1}, w> v_{j-1} = sigma_{j-1}^2 <u_{j-1}, w> u_{j-1}
      const double sm = ro ? st.sigma[(j - 1) * B + b] : 0.0;
      ser[b] = sm * sm * tot[2 * B + b];
      sei[b] = sm * sm * tot[3 * B + b];
    }
    act[b] = active;
  }
  __syncthreads();

  const int b = threadIdx.x % B;
  const uint32_t R = blockDim.x / B, rl = threadIdx.x / B;
  const uint32_t ntiles = (D + R - 1) / R;
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb) {
    double s = 0.0;
    if (act[b]) {
      const double c = sc[b], d = sd[b], er = ser[b], ei = sei[b];
      for (TileWalk tw(ntiles, VGrid{vb, rg.n}); tw.t < tw.t_end; tw.t += tw.step) {
        const uint32_t r = tw.t * R + rl;
        if (r >= D) continue;
        const size_t i = (size_t)r * B + b;
        V wv, u;
        if (NT) {
          wv = ld_nt(w + i);
          u = ld_nt(uj + i);
        } else {
          wv = w[i];
          u = uj[i];
        }
        double nx = c * ((double)wv.x - d * (double)u.x);
        double ny = c * ((double)wv.y - d * (double)u.y);
        if (ro) {
          const V um = ujm1[i];
          nx -= er * (double)um.x - ei * (double)um.y;
          ny -= er * (double)um.y + ei * (double)um.x;
        }
        V o;
        o.x = (T)nx;
        o.y = (T)ny;
        if (store) w[i] = o;
        s += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
      }
    }
    double v[1] = {s};
    block_partials<1>(v, B, red, partB + (size_t)vb * B);
    __syncthreads();   // red is written again by the next virtual block
  }
}

// ------------------------------------------ projected exponential (1 wave)
// ||u_m|| of the last update pass (the norm of the residual after m steps;
// only meaningful when the recurrence ran all m steps), reduced by one wave:
// lane i sums rows i, i + 64, ... in order, then lanes i and i + s are added
// for s = 32, 16, ..., 1 (a fixed tree, no LDS and no barrier).
__device__ __forceinline__ double last_residual_norm(const double* __restrict__ partB, int Gp, int B, int b, int i) {
  double acc = 0.0;
  for (int g = i; g < Gp; g += 64) acc += partB[(size_t)g * B + b];
  for (int s = 32; s > 0; s >>= 1) {
    const double o = __shfl_down(acc, s);
    if (i < s) acc += o;
  }
  return sqrt(__shfl(acc, 0));
}

// Tridiagonal entries of column b seen by lane i (zero outside m_used).
struct TriLane {
  double al, be, bl;
  bool on;
};
__device__ __forceinline__ TriLane tri_lane(const KState& st, int B, int b, int mu, int i) {
  TriLane t;
  t.on = i < mu;
  t.al = t.on ? st.alpha[i * B + b] : 0.0;
  t.be = (i + 1 < mu) ? st.beta[i * B + b] : 0.0;     // couples i and i+1
  t.bl = (t.on && i > 0) ? st.beta[(i - 1) * B + b] : 0.0;
  return t;
}

// c = exp(-i tau T) e_1 for the tridiagonal T of the Lanczos recurrence
// (tri_expm_e1), times ||psi|| and the stored-vector scales, plus the
// a-posteriori error estimate ||psi|| beta_m |c_m|.  With tau_dev != NULL the
// step is the smallest of tau_dev[0..B) (the accepted steps of an adaptive
// step, so that all columns stay at the same time).
// Column b by one wavefront (lane i); no barrier, so the waves of a larger
// work-group may take different columns.
__device__ __forceinline__ void small_expm_wave(int b, int i, const KState& st, int m, int B, double tau,
                                                const double* __restrict__ tau_dev, const double* __restrict__ partB,
                                                int Gp) {
  const double beta_last = last_residual_norm(partB, Gp, B, b, i);
  if (tau_dev) {
    tau = tau_dev[0];
    for (int c = 1; c < B; ++c) tau = fmin(tau, tau_dev[c]);
  }
  const int mu = st.mused[b];
  if (st.status[b] != QK_OK || mu <= 0) {
    if (i < m) {
      st.gre[i * B + b] = 0.0;
      st.gim[i * B + b] = 0.0;
    }
    if (i == 0) st.err[b] = 0.0;
    return;
  }
  if (mu == m && i == 0) st.beta[(m - 1) * B + b] = beta_last;
  const TriLane t = tri_lane(st, B, b, mu, i);
  double er, ei;
  tri_expm_e1(t.al, t.be, t.bl, t.on, i, tau, er, ei);
  const double n0 = st.n0[b];
  if (i < m) {
    const double g = t.on ? n0 * st.sigma[i * B + b] : 0.0;
    st.gre[i * B + b] = g * er;
    st.gim[i * B + b] = g * ei;
  }
  const double last = __shfl(sqrt(er * er + ei * ei), mu - 1);
  if (i == 0) st.err[b] = (mu == m) ? n0 * beta_last * last : 0.0;
}


// ------------------------------------------------ Krylov combination
// psi[r, b] = sum_{j < m_used} gamma_j u_j[r, b], u_0 = psi, accumulated in
// double and rounded once.  The [D][B] arrays are walked as flat elements
// i = r * B + b; a thread takes the E consecutive elements of one access
// (E = 2 packs two complex64 values into 16 bytes) and issues the loads of
// kCombineUnroll Krylov vectors before it accumulates them.  With one column
// the coefficients are uniform (scalar loads); with several they are staged
// in LDS.  Columns whose step failed or had nothing to propagate are left
// unchanged.
constexpr int kCombineUnroll = 8;

// cf: LDS of m * B double2 (B > 1; unused for one column).
template <typename T, int E, bool ONE, bool NT>
__device__ __forceinline__ void combine_body(VRange rg, double2* cf, typename Cx<T>::V* __restrict__ psi,
                                             const typename Cx<T>::V* __restrict__ U, uint32_t D, int B, int m,
                                             const KState& st) {
  using V = typename Cx<T>::V;
  struct alignas(sizeof(V) * E) Pack {
    V v[E];
  };
  if (!ONE) {
    for (int i = threadIdx.x; i < m * B; i += blockDim.x) cf[i] = make_double2(st.gre[i], st.gim[i]);
    __syncthreads();
  }
  auto coef = [&](int j, int b) -> double2 {
    if (ONE) return make_double2(st.gre[j], st.gim[j]);
    return cf[j * B + b];
  };
  const uint64_t np = (uint64_t)D * B / E;   // packs per vector (the launcher makes D * B a multiple of E)
  const Pack* Up = reinterpret_cast<const Pack*>(U);
  Pack* Pp = reinterpret_cast<Pack*>(psi);
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb)
  for (uint64_t p = (uint64_t)vb * blockDim.x + threadIdx.x; p < np; p += (uint64_t)rg.n * blockDim.x) {
    int bc[E], mu[E];
    bool ok[E];
    int mumax = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      bc[e] = ONE ? 0 : (int)((p * E + e) % (uint64_t)B);
      mu[e] = st.mused[bc[e]];
      ok[e] = st.status[bc[e]] == QK_OK && mu[e] > 0;
      if (ok[e] && mu[e] > mumax) mumax = mu[e];
    }
    const Pack p0 = Pp[p];
    double ar[E], ai[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double2 g = coef(0, bc[e]);
      ar[e] = g.x * (double)p0.v[e].x - g.y * (double)p0.v[e].y;
      ai[e] = g.x * (double)p0.v[e].y + g.y * (double)p0.v[e].x;
    }
    int jj = 1;
    for (; jj + kCombineUnroll - 1 < mumax; jj += kCombineUnroll) {
      Pack u[kCombineUnroll];
#pragma unroll
      for (int k = 0; k < kCombineUnroll; ++k) {
        // the basis vectors are read once per step: non-temporal 16-byte loads
        // when they exceed the last-level cache
        const Pack* src = Up + (uint64_t)(jj - 1 + k) * np + p;
        if constexpr (NT && sizeof(Pack) == 16) {
          typedef double D2 __attribute__((ext_vector_type(2)));
          const D2 v = __builtin_nontemporal_load(reinterpret_cast<const D2*>(src));
          __builtin_memcpy(&u[k], &v, 16);
        } else {
          u[k] = *src;
        }
      }
#pragma unroll
      for (int k = 0; k < kCombineUnroll; ++k)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (ONE || jj + k < mu[e]) {
            const double2 g = coef(jj + k, bc[e]);
            ar[e] += g.x * (double)u[k].v[e].x - g.y * (double)u[k].v[e].y;
            ai[e] += g.x * (double)u[k].v[e].y + g.y * (double)u[k].v[e].x;
          }
        }
    }
    for (; jj < mumax; ++jj) {
      const Pack u = Up[(uint64_t)(jj - 1) * np + p];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (ONE || jj < mu[e]) {
          const double2 g = coef(jj, bc[e]);
          ar[e] += g.x * (double)u.v[e].x - g.y * (double)u.v[e].y;
          ai[e] += g.x * (double)u.v[e].y + g.y * (double)u.v[e].x;
        }
      }
    }
    Pack o;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      o.v[e].x = ok[e] ? (T)ar[e] : p0.v[e].x;
      o.v[e].y = ok[e] ? (T)ai[e] : p0.v[e].y;
    }
    Pp[p] = o;
  }
}

// ------------------------------------------------ survival probability
// red: LDS of 2 * blockDim doubles.
template <typename T>
__device__ __forceinline__ void overlap_partial_body(VRange rg, double* red, const typename Cx<T>::V* __restrict__ psi0,
                                                     const typename Cx<T>::V* __restrict__ psi, uint32_t D, int B,
                                                     double* __restrict__ part) {
  const int b = threadIdx.x % B;
  const uint32_t R = blockDim.x / B, rl = threadIdx.x / B;
  const uint32_t ntiles = (D + R - 1) / R;
  for (uint32_t vb = rg.v0; vb < rg.v1; ++vb) {
    double sr = 0.0, si = 0.0;
    for (TileWalk tw(ntiles, VGrid{vb, rg.n}); tw.t < tw.t_end; tw.t += tw.step) {
      const uint32_t r = tw.t * R + rl;
      if (r >= D) continue;
      const size_t i = (size_t)r * B + b;
      const typename Cx<T>::V a = psi0[i], c = psi[i];
      sr += (double)a.x * (double)c.x + (double)a.y * (double)c.y;   // conj(a) c
      si += (double)a.x * (double)c.y - (double)a.y * (double)c.x;
    }
    double v[2] = {sr, si};
    block_partials<2>(v, B, red, part + (size_t)vb * 2 * B);
    __syncthreads();   // red is written again by the next virtual block
  }
}

// |<psi0, psi>|^2 per column into P[b], or, with a step counter, into
// P[(*counter) * items + off + b] (the batched driver's record layout).
// red: LDS of blockDim doubles, tot: of 2 * QK_MAX_BATCH doubles; one block.
__device__ __forceinline__ void overlap_final_body(double* red, double* tot, const double* __restrict__ part, int G,
                                                   int B, double* P, const int* __restrict__ counter, int off,
                                                   int items) {
  reduce_partials(part, G, 2, B, red, tot);
  double* out = counter ? P + (size_t)(*counter) * items + off : P;
  for (int b = threadIdx.x; b < B; b += blockDim.x) out[b] = tot[b] * tot[b] + tot[B + b] * tot[B + b];
}

// ------------------------------------------------ batched driver records
// |psi[r0, b]|^2 of every column at the driver's record position
// P[(*counter) * items + off + b]; threads b < B.
template <typename T>
__device__ __forceinline__ void record_body(const typename Cx<T>::V* __restrict__ psi, uint32_t r0, int B,
                                            double* __restrict__ P, const int* __restrict__ counter, int off,
                                            int items) {
  const int b = threadIdx.x;
  if (b >= B) return;
  const typename Cx<T>::V v = psi[(size_t)r0 * B + b];
  P[(size_t)(*counter) * items + off + b] = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// Trapezoid step of the autocorrelation integral for every item: S += dt/2
// (P_prev + P_now), P_prev = P_now, t += dt, C = S / t (written when C is
// not NULL).  One block; `state` = [S(items), P_prev(items), t].
__device__ __forceinline__ void autocorr_body(const double* __restrict__ P, const int* __restrict__ counter, int items,
                                              double dt, double* state, double* C) {
  const int c = *counter;
  double* S = state;
  double* prev = state + items;
  double* tp = state + 2 * (size_t)items;
  const double t = *tp + dt;
  for (int j = threadIdx.x; j < items; j += blockDim.x) {
    const double pn = P[(size_t)c * items + j];
    const double sj = S[j] + 0.5 * dt * (prev[j] + pn);
    S[j] = sj;
    prev[j] = pn;
    if (C) C[(size_t)c * items + j] = (t > 0.0) ? sj / t : pn;
  }
  __syncthreads();
  if (threadIdx.x == 0) *tp = t;
}


}  // namespace qk

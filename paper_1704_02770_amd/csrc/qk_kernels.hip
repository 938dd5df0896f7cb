// HIP kernels of libqkrylov for gfx950 (MI355X).
//
// Method: arXiv:1704.02770.  Basis (Sec. 2 "Basis representation", Sec. 3
// Algorithms 2 and 3), Hamiltonian rows (Sec. 3 "Hamiltonian matrix
// construction", Eq. (1)), Krylov propagation (Sec. 2 "Krylov subspace
// methods") and the survival probability (Sec. 4).
//
// Memory layout: vectors are interleaved complex [D][B] (batch fastest), so a
// row's B values are contiguous and a wavefront of consecutive (row, batch)
// threads streams contiguous memory.  All reductions are deterministic: each
// block writes its partial sums, and the next kernel in the chain reduces all
// partials in a fixed order in every block (no atomics, no cross-XCD fences).
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <mutex>
#include <type_traits>

#include "qk_step_bodies.h"

namespace qk {

// C(n, k) for n, k < K by Pascal's rule, saturated at 2^32 - 1 (entries that
// large are never used: every term of a rank is below D < 2^32).
template <int K>
__global__ void k_binom_table(uint32_t* tab) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int n = 0; n < K; ++n)
    for (int k = 0; k < K; ++k) {
      uint64_t v;
      if (k > n) v = 0;
      else if (k == 0 || k == n) v = 1;
      else v = (uint64_t)tab[(n - 1) * K + k - 1] + tab[(n - 1) * K + k];
      tab[n * K + k] = v > 0xffffffffull ? 0xffffffffu : (uint32_t)v;
    }
}

constexpr int kBasisChunk = 8;
constexpr int kBasisThreads = 256;

// Every thread unranks the first state of its chunk and advances with the
// next bit permutation; the block stages its 2048 states in LDS and writes
// them out coalesced.
template <typename S>
__global__ void __launch_bounds__(kBasisThreads)
k_basis_build(S* __restrict__ states, uint32_t D, int L, int N, const uint32_t* __restrict__ gtab) {
  constexpr int K = StateT<S>::kStride;
  __shared__ uint32_t tab[K * K];
  __shared__ S stage[kBasisThreads * kBasisChunk];
  for (int i = threadIdx.x; i < K * K; i += kBasisThreads) tab[i] = gtab[i];
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kBasisThreads * kBasisChunk;
  const uint64_t start = base + (uint64_t)threadIdx.x * kBasisChunk;
  if (start < D) {
    S s = cns_unrank<S>((uint32_t)start, L, N, tab);
    for (int i = 0; i < kBasisChunk; ++i) {
      stage[threadIdx.x * kBasisChunk + i] = s;
      s = next_perm<S>(s);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBasisThreads * kBasisChunk; i += kBasisThreads) {
    uint64_t r = base + i;
    if (r < D) states[r] = stage[i];
  }
}

template <typename S>
__global__ void k_rank(const uint64_t* __restrict__ in, int64_t n, int64_t* __restrict__ out, int L, int N,
                       const uint32_t* __restrict__ tab) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t s = in[i];
  if ((L < 64 && (s >> L) != 0) || (int)__popcll(s) != N) {
    out[i] = -1;
    return;
  }
  out[i] = (int64_t)cns_rank<S>((S)s, tab);
}

// ----------------------------------------------------------- H x kernels
template <typename T, bool CSR, typename S>
__global__ void __launch_bounds__(kMaxBlock)
k_apply(const typename Cx<T>::V* __restrict__ x, typename Cx<T>::V* __restrict__ y, ModelArgs a, HamView<S> hv,
        const uint32_t* __restrict__ gtab, const double* __restrict__ gfields) {
  __shared__ RowShared<S> sh;
  load_row_shared(sh, a, gtab, gfields);
  const int B = a.B, b = threadIdx.x % B;
  const uint32_t R = blockDim.x / B, rl = threadIdx.x / B;
  const uint32_t ntiles = (hv.D + R - 1) / R;
  for (TileWalk w(ntiles, hw_grid()); w.t < w.t_end; w.t += w.step) {
    const uint32_t r = w.t * R + rl;
    if (r >= hv.D) continue;
    typename Cx<T>::V xr;
    y[(size_t)r * B + b] = h_row<T, CSR, S>(r, b, a, sh, hv, x, xr);
  }
}

template <typename T, bool CSR, typename S>
__global__ void __launch_bounds__(kMaxBlock)
k_lanczos_A(const typename Cx<T>::V* __restrict__ uj, const typename Cx<T>::V* __restrict__ ujm1,
            typename Cx<T>::V* __restrict__ w, ModelArgs a, HamView<S> hv, const uint32_t* __restrict__ gtab,
            const double* __restrict__ gfields, KState st, LanczosArgs la, const double* __restrict__ partB, int Gp,
            double* __restrict__ partA) {
  __shared__ LanczosAShared<S> ls;
  lanczos_a_body<T, CSR, S>(hw_range(), ls, uj, ujm1, w, a, hv, gtab, gfields, st, la, partB, Gp, partA);
}

__global__ void __launch_bounds__(256) k_partials_total(const double* __restrict__ part, int G, int cols,
                                                        double* __restrict__ tot) {
  __shared__ double red[256];
  partials_total_body(hw_range(), red, part, G, cols, tot);
}

template <typename T, bool NT>
__global__ void __launch_bounds__(kMaxBlock)
k_lanczos_B(const typename Cx<T>::V* __restrict__ uj, const typename Cx<T>::V* __restrict__ ujm1,
            typename Cx<T>::V* __restrict__ w, uint32_t D, int B, KState st, LanczosArgs la,
            const double* __restrict__ partA, int Gp, double* __restrict__ partB, int store) {
  __shared__ LanczosBShared ls;
  lanczos_b_body<T, NT>(hw_range(), ls, uj, ujm1, w, D, B, st, la, partA, Gp, partB, store);
}


// ------------------------------------- full reorthogonalisation (reorth = 2)
// Classical Gram-Schmidt applied twice to the new vector w = u_{j+1} against
// v_0..v_j (v_i = sigma_i u_i, u_0 = psi): c_i = sigma_i^2 <u_i, w>, then
// w -= sum_i c_i u_i.  Dot products and coefficients are accumulated in
// double in a fixed order; the last pass leaves |w|^2 in the update pass's
// partial sums, so beta_j is the norm of the reorthogonalised vector.
template <typename T>
__global__ void __launch_bounds__(kMaxBlock)
k_reorth_dots(const typename Cx<T>::V* __restrict__ psi, const typename Cx<T>::V* __restrict__ U,
              const typename Cx<T>::V* __restrict__ w, uint32_t D, int B, int i0, int ni, double* __restrict__ part) {
  using V = typename Cx<T>::V;
  __shared__ double red[2 * kReorthChunk * kMaxBlock];
  const int b = threadIdx.x % B;
  const uint32_t R = blockDim.x / B, rl = threadIdx.x / B;
  const uint32_t ntiles = (D + R - 1) / R;
  const size_t stride = (size_t)D * B;
  double acc[2 * kReorthChunk];
#pragma unroll
  for (int q = 0; q < 2 * kReorthChunk; ++q) acc[q] = 0.0;
  for (TileWalk tw(ntiles, hw_grid()); tw.t < tw.t_end; tw.t += tw.step) {
    const uint32_t r = tw.t * R + rl;
    if (r >= D) continue;
    const size_t i = (size_t)r * B + b;
    const V wv = w[i];
#pragma unroll
    for (int q = 0; q < kReorthChunk; ++q) {
      if (q < ni) {
        const int iv = i0 + q;
        const V u = iv == 0 ? psi[i] : U[(size_t)(iv - 1) * stride + i];
        acc[2 * q] += (double)u.x * (double)wv.x + (double)u.y * (double)wv.y;   // conj(u) w
        acc[2 * q + 1] += (double)u.x * (double)wv.y - (double)u.y * (double)wv.x;
      }
    }
  }
  block_partials<2 * kReorthChunk>(acc, B, red, part + (size_t)blockIdx.x * 2 * kReorthChunk * B);
}

// c_i for i < nv from the partials of every chunk (one block, fixed order);
// zero for columns whose recurrence has stopped.
__global__ void __launch_bounds__(kMaxBlock)
k_reorth_coef(const double* __restrict__ part, int G, int nv, int B, int j, KState st, double* __restrict__ coef) {
  for (int idx = threadIdx.x; idx < nv * 2 * B; idx += blockDim.x) {
    const int i = idx / (2 * B), rem = idx % (2 * B), comp = rem / B, b = rem % B;
    const int chunk = i / kReorthChunk, q = 2 * (i % kReorthChunk) + comp;
    const double* pc = part + (size_t)chunk * kReorthGrid * 2 * kReorthChunk * B;
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += pc[((size_t)g * 2 * kReorthChunk + q) * B + b];
    const double sg = st.sigma[i * B + b];
    coef[idx] = (st.mused[b] > j && st.status[b] == QK_OK) ? sg * sg * t : 0.0;
  }
}

template <typename T>
__global__ void __launch_bounds__(kMaxBlock)
k_reorth_axpy(const typename Cx<T>::V* __restrict__ psi, const typename Cx<T>::V* __restrict__ U,
              typename Cx<T>::V* __restrict__ w, uint32_t D, int B, int nv, const double* __restrict__ coef,
              double* __restrict__ partB) {
  using V = typename Cx<T>::V;
  __shared__ double red[kMaxBlock];
  const int b = threadIdx.x % B;
  const uint32_t R = blockDim.x / B, rl = threadIdx.x / B;
  const uint32_t ntiles = (D + R - 1) / R;
  const size_t stride = (size_t)D * B;
  double s = 0.0;
  for (TileWalk tw(ntiles, hw_grid()); tw.t < tw.t_end; tw.t += tw.step) {
    const uint32_t r = tw.t * R + rl;
    if (r >= D) continue;
    const size_t i = (size_t)r * B + b;
    const V wv = w[i];
    double xr = (double)wv.x, xi = (double)wv.y;
    for (int iv = 0; iv < nv; ++iv) {
      const V u = iv == 0 ? psi[i] : U[(size_t)(iv - 1) * stride + i];
      const double cr = coef[(2 * iv) * B + b], ci = coef[(2 * iv + 1) * B + b];
      xr -= cr * (double)u.x - ci * (double)u.y;
      xi -= cr * (double)u.y + ci * (double)u.x;
    }
    V o;
    o.x = (T)xr;
    o.y = (T)xi;
    w[i] = o;
    s += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
  }
  double v[1] = {s};
  block_partials<1>(v, B, red, partB + (size_t)blockIdx.x * B);
}

__global__ void __launch_bounds__(64)
k_small_expm(KState st, int m, int B, double tau, const double* __restrict__ tau_dev, const double* __restrict__ partB,
             int Gp) {
  small_expm_wave((int)blockIdx.x, (int)threadIdx.x, st, m, B, tau, tau_dev, partB, Gp);
}


// Step-size control of one adaptive step (the rule of Expokit, which the
// paper's runs use through SLEPc): starting from tau_max, the step tau of
// column b is accepted when the estimate err(tau) = ||psi|| beta_m
// |[exp(-i tau T)]_{m,1}| is at most 1.2 tau tol, and otherwise replaced by
// 0.9 tau (tau tol / err)^(1 / (m - 1)), kept within [tau / 10, 0.9 tau].  The
// Krylov basis does not depend on tau, so only the small exponential is
// recomputed.  A recurrence that stopped early spans an invariant subspace
// and accepts tau_max.  st.tau[b] = accepted step, st.tau[B + b] = suggested
// next step (0.9 tau (tau tol / err)^(1/(m-1)), at most 10 tau).
__global__ void __launch_bounds__(64)
k_step_size(KState st, int m, int B, double tau_max, double tol, const double* __restrict__ partB, int Gp) {
  const int b = blockIdx.x;
  const int i = threadIdx.x;
  const double beta_last = last_residual_norm(partB, Gp, B, b, i);
  const int mu = st.mused[b];
  double tau = tau_max, next = tau_max;
  if (st.status[b] == QK_OK && mu == m && m > 1) {
    const TriLane t = tri_lane(st, B, b, mu, i);
    const double n0 = st.n0[b];
    const double xm = 1.0 / (double)(m - 1);
    double err = 0.0;
    for (int it = 0; it < 60; ++it) {
      double er, ei;
      tri_expm_e1(t.al, t.be, t.bl, t.on, i, tau, er, ei);
      err = n0 * beta_last * __shfl(sqrt(er * er + ei * ei), mu - 1);
      if (err <= 1.2 * tau * tol) break;
      double nt = 0.9 * tau * pow(tau * tol / err, xm);
      if (!(nt >= 0.1 * tau)) nt = 0.1 * tau;   // also catches a NaN estimate
      if (nt > 0.9 * tau) nt = 0.9 * tau;
      tau = nt;
    }
    next = (err > 0.0) ? 0.9 * tau * pow(tau * tol / err, xm) : 10.0 * tau;
    if (!(next <= 10.0 * tau)) next = 10.0 * tau;
  }
  if (i == 0) {
    st.tau[b] = tau;
    st.tau[B + b] = next;
  }
}

template <typename T, int E, bool ONE, bool NT>
__global__ void __launch_bounds__(kMaxBlock)
k_combine(typename Cx<T>::V* __restrict__ psi, const typename Cx<T>::V* __restrict__ U, uint32_t D, int B, int m,
          KState st) {
  extern __shared__ double2 cf[];   // [m][B] coefficients when B > 1
  combine_body<T, E, ONE, NT>(hw_range(), cf, psi, U, D, B, m, st);
}


// ------------------------------------------------ survival probability
template <typename T>
__global__ void k_prob_basis_state(const typename Cx<T>::V* __restrict__ psi, uint32_t r0, int B, double* P) {
  const int b = threadIdx.x;
  if (b >= B) return;
  const typename Cx<T>::V v = psi[(size_t)r0 * B + b];
  P[b] = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

template <typename T>
__global__ void __launch_bounds__(kMaxBlock)
k_overlap_partial(const typename Cx<T>::V* __restrict__ psi0, const typename Cx<T>::V* __restrict__ psi, uint32_t D,
                  int B, double* __restrict__ part) {
  __shared__ double red[2 * kMaxBlock];
  overlap_partial_body<T>(hw_range(), red, psi0, psi, D, B, part);
}

// |<psi0, psi>|^2 per column into P[b], or, with a step counter, into
// P[(*counter) * items + off + b] (the batched driver's record layout).
__global__ void __launch_bounds__(kMaxBlock)
k_overlap_final(const double* __restrict__ part, int G, int B, double* P, const int* __restrict__ counter, int off,
                int items) {
  __shared__ double red[kMaxBlock];
  __shared__ double tot[2 * QK_MAX_BATCH];
  overlap_final_body(red, tot, part, G, B, P, counter, off, items);
}


// ------------------------------------------------------------- CSR form
// Counting pass = the exact preallocation of Sec. 3.
template <typename S>
__global__ void __launch_bounds__(kMaxBlock)
k_csr_count(const S* __restrict__ states, uint32_t D, ModelArgs a, uint32_t* __restrict__ cnt) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const S s = states[r];
  uint32_t n = (uint32_t)popc((S)((s ^ (s >> 1)) & ((S)a.lmask >> 1)));
  if (a.pbc) n += (uint32_t)((s ^ (s >> (a.L - 1))) & (S)1);
  cnt[r] = n;
}

template <typename S>
__global__ void __launch_bounds__(kMaxBlock)
k_csr_fill(const S* __restrict__ states, uint32_t D, ModelArgs a, const uint32_t* __restrict__ gtab,
           const uint32_t* __restrict__ rowptr, uint32_t* __restrict__ cols) {
  constexpr int K = StateT<S>::kStride;
  __shared__ uint32_t tab[K * K];
  for (int i = threadIdx.x; i < K * K; i += blockDim.x) tab[i] = gtab[i];
  __syncthreads();
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  uint32_t k = rowptr[r];
  for_each_hop<S>(states[r], r, a, tab, [&](uint32_t c) { cols[k++] = c; });
}

template <typename S>
__global__ void __launch_bounds__(kMaxBlock)
k_csr_diag(const S* __restrict__ states, uint32_t D, ModelArgs a, const double* __restrict__ gfields,
           double* __restrict__ diag) {
  __shared__ double fld[kFldCap];
  __shared__ double hh[QK_MAX_BATCH];
  for (int i = threadIdx.x; i < a.B * a.L; i += blockDim.x) fld[i] = gfields[i];
  __syncthreads();
  for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < a.L; ++i) t += fld[b * a.L + i];
    hh[b] = 0.5 * t;
  }
  __syncthreads();
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const S s = states[r];
  for (int b = 0; b < a.B; ++b) diag[(size_t)r * a.B + b] = diag_value<S>(s, a, fld + b * a.L, hh[b]);
}

// ================================================================ launchers
int qk_num_cus() {
  // compute units of the current device, queried once (thread-safe static init)
  static const int n = []() {
    int dev = 0, c = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      c = prop.multiProcessorCount;
    return c > 0 ? c : 256;
  }();
  return n;
}

// Blocks of a streaming kernel: 4 blocks per CU by default (measured at
// L = 28 against 2, 8 and 16: the update pass 0.324 -> 0.305 ms in complex128,
// 0.168 -> 0.158 ms in complex64), at most one per tile, rounded to a
// multiple of the XCD count.
int stream_grid(uint64_t rows, int B, int threads, int blocks_per_cu) {
  if (threads <= 0) threads = block_threads(B);
  if (blocks_per_cu <= 0) blocks_per_cu = 4;
  const uint64_t R = threads / B;
  uint64_t tiles = (rows + R - 1) / R;
  uint64_t g = (uint64_t)qk_num_cus() * blocks_per_cu;
  if (g > (uint64_t)kMaxPartialBlocks) g = kMaxPartialBlocks;
  if (g > tiles) g = tiles;
  const uint64_t wcap = (rows * (uint64_t)B + kMinBlockWork - 1) / kMinBlockWork;
  if (g > wcap) g = wcap;
  g = ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
  if (g < kNumXcd) g = kNumXcd;
  return (int)g;
}

template <typename S>
static HamView<S> ham_view(const qk_ham* H) {
  HamView<S> v;
  v.states = (const S*)H->basis->d_states;
  v.rowptr = H->d_rowptr;
  v.cols = H->d_cols;
  v.diag = H->d_diag;
  v.D = (uint32_t)H->basis->D;
  return v;
}

HamView<uint32_t> ham_view32(const qk_ham* H) { return ham_view<uint32_t>(H); }

ModelArgs model_args(const qk_ham* H) {
  ModelArgs a;
  a.L = H->basis->L;
  a.N = H->basis->N;
  a.pbc = H->p.pbc;
  a.B = H->batch;
  a.half_jxy = 0.5 * H->p.jxy;
  a.jz = H->p.jz;
  a.lmask = a.L >= 64 ? ~0ull : ((1ull << a.L) - 1ull);
  return a;
}

KState make_kstate(const qk_krylov* k) { return kstate_at(k, k->d_coef, k->d_int); }

KState kstate_at(const qk_krylov* k, double* p, int32_t* ints) {
  const int m = k->m, B = k->batch;
  KState s;
  s.alpha = p;
  s.beta = p + (size_t)m * B;
  s.sigma = p + (size_t)2 * m * B;
  s.n0 = p + (size_t)(3 * m + 1) * B;
  s.gre = p + (size_t)(3 * m + 2) * B;
  s.gim = p + (size_t)(4 * m + 2) * B;
  s.err = p + (size_t)(5 * m + 2) * B;
  s.mused = ints;
  s.status = ints + B;
  s.tau = p + (size_t)(5 * m + 3) * B;
  return s;
}

int binom_stride(const qk_basis* b) { return b->wide ? StateT<uint64_t>::kStride : StateT<uint32_t>::kStride; }

qk_status launch_basis_build(qk_basis* b, hipStream_t s) {
  const uint64_t per = (uint64_t)kBasisThreads * kBasisChunk;
  const uint64_t blocks = ((uint64_t)b->D + per - 1) / per;
  if (b->wide) {
    hipLaunchKernelGGL(k_binom_table<StateT<uint64_t>::kStride>, dim3(1), dim3(1), 0, s, b->d_binom);
    QK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_basis_build<uint64_t>, dim3((unsigned)blocks), dim3(kBasisThreads), 0, s,
                       (uint64_t*)b->d_states, (uint32_t)b->D, b->L, b->N, b->d_binom);
  } else {
    hipLaunchKernelGGL(k_binom_table<StateT<uint32_t>::kStride>, dim3(1), dim3(1), 0, s, b->d_binom);
    QK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_basis_build<uint32_t>, dim3((unsigned)blocks), dim3(kBasisThreads), 0, s,
                       (uint32_t*)b->d_states, (uint32_t)b->D, b->L, b->N, b->d_binom);
  }
  QK_HIP(hipGetLastError());
  return QK_OK;
}

qk_status launch_rank(const qk_basis* b, const uint64_t* d_in, int64_t n, int64_t* d_out, hipStream_t s) {
  if (n == 0) return QK_OK;
  const int64_t blocks = (n + 255) / 256;
  if (b->wide)
    hipLaunchKernelGGL(k_rank<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, d_in, n, d_out, b->L, b->N,
                       b->d_binom);
  else
    hipLaunchKernelGGL(k_rank<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, d_in, n, d_out, b->L, b->N,
                       b->d_binom);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

qk_status launch_csr_diag(qk_ham* H, hipStream_t s) {
  const ModelArgs a = model_args(H);
  const uint32_t D = (uint32_t)H->basis->D;
  if (H->basis->wide)
    hipLaunchKernelGGL(k_csr_diag<uint64_t>, dim3((D + 255) / 256), dim3(256), 0, s,
                       (const uint64_t*)H->basis->d_states, D, a, H->d_fields, H->d_diag);
  else
    hipLaunchKernelGGL(k_csr_diag<uint32_t>, dim3((D + 255) / 256), dim3(256), 0, s,
                       (const uint32_t*)H->basis->d_states, D, a, H->d_fields, H->d_diag);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

qk_status launch_csr_build(qk_ham* H, hipStream_t s) {
  const ModelArgs a = model_args(H);
  const uint32_t D = (uint32_t)H->basis->D;
  // count into rowptr[1..D], then an inclusive scan in place gives the row pointers
  QK_HIP(hipMemsetAsync(H->d_rowptr, 0, sizeof(uint32_t), s));
  if (H->basis->wide)
    hipLaunchKernelGGL(k_csr_count<uint64_t>, dim3((D + 255) / 256), dim3(256), 0, s,
                       (const uint64_t*)H->basis->d_states, D, a, H->d_rowptr + 1);
  else
    hipLaunchKernelGGL(k_csr_count<uint32_t>, dim3((D + 255) / 256), dim3(256), 0, s,
                       (const uint32_t*)H->basis->d_states, D, a, H->d_rowptr + 1);
  QK_HIP(hipGetLastError());
  size_t tmp_bytes = 0;
  QK_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_bytes, H->d_rowptr + 1, H->d_rowptr + 1, (int)D, s));
  void* tmp = nullptr;
  QK_HIP(dev_alloc_async(H->al, &tmp, tmp_bytes + 16, s));
  hipError_t e = hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, H->d_rowptr + 1, H->d_rowptr + 1, (int)D, s);
  QK_HIP(dev_free_async(H->al, tmp, s));
  QK_HIP(e);
  uint32_t nnz = 0;
  QK_HIP(hipMemcpyAsync(&nnz, H->d_rowptr + D, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  H->nnz = nnz;
  QK_HIP(dev_alloc(H->al, (void**)&H->d_cols, sizeof(uint32_t) * (size_t)(nnz > 0 ? nnz : 1)));
  if (H->basis->wide)
    hipLaunchKernelGGL(k_csr_fill<uint64_t>, dim3((D + 255) / 256), dim3(256), 0, s,
                       (const uint64_t*)H->basis->d_states, D, a, H->basis->d_binom, H->d_rowptr, H->d_cols);
  else
    hipLaunchKernelGGL(k_csr_fill<uint32_t>, dim3((D + 255) / 256), dim3(256), 0, s,
                       (const uint32_t*)H->basis->d_states, D, a, H->basis->d_binom, H->d_rowptr, H->d_cols);
  QK_HIP(hipGetLastError());
  return launch_csr_diag(H, s);
}

template <typename T, typename S>
static void launch_apply_rows(const qk_ham* H, const void* x, void* y, hipStream_t s) {
  using V = typename Cx<T>::V;
  const ModelArgs a = model_args(H);
  const HamView<S> hv = ham_view<S>(H);
  const int threads = block_threads(a.B);
  const int grid = stream_grid(hv.D, a.B, threads, 0);
  if (H->p.mode == QK_CSR)
    hipLaunchKernelGGL((k_apply<T, true, S>), dim3(grid), dim3(threads), 0, s, (const V*)x, (V*)y, a, hv,
                       H->basis->d_binom, H->d_fields);
  else
    hipLaunchKernelGGL((k_apply<T, false, S>), dim3(grid), dim3(threads), 0, s, (const V*)x, (V*)y, a, hv,
                       H->basis->d_binom, H->d_fields);
}

qk_status launch_ham_apply(const qk_ham* H, const void* x, void* y, int dtype, hipStream_t s) {
  if (split_usable(H) && H->batch == 1) return launch_split_apply(H, x, y, dtype, s);
  if (blocked_usable(H, dtype)) return launch_blocked_apply(H, x, y, dtype, s);
  const bool wide = H->basis->wide;
  if (dtype == QK_C128) {
    if (wide) launch_apply_rows<double, uint64_t>(H, x, y, s);
    else launch_apply_rows<double, uint32_t>(H, x, y, s);
  } else {
    if (wide) launch_apply_rows<float, uint64_t>(H, x, y, s);
    else launch_apply_rows<float, uint32_t>(H, x, y, s);
  }
  QK_HIP(hipGetLastError());
  return QK_OK;
}

// H-pass of Lanczos iteration j through the row kernels (CSR or matrix-free rows).
// G: launch grid (a multiple of kNumXcd; it also sets the rows of partA the
// launch writes); Gp: rows of partial sums in partB (1 when they were
// totalled beforehand).
template <typename T, typename S>
static void launch_lanczos_rows(const qk_ham* H, const typename Cx<T>::V* uj, const typename Cx<T>::V* ujm1,
                                typename Cx<T>::V* w, const KState& st, const LanczosArgs& la, const double* partB,
                                int Gp, int G, int threads, double* partA, hipStream_t s) {
  const ModelArgs a = model_args(H);
  const HamView<S> hv = ham_view<S>(H);
  if (H->p.mode == QK_CSR)
    hipLaunchKernelGGL((k_lanczos_A<T, true, S>), dim3(G), dim3(threads), 0, s, uj, ujm1, w, a, hv,
                       H->basis->d_binom, H->d_fields, st, la, partB, Gp, partA);
  else
    hipLaunchKernelGGL((k_lanczos_A<T, false, S>), dim3(G), dim3(threads), 0, s, uj, ujm1, w, a, hv,
                       H->basis->d_binom, H->d_fields, st, la, partB, Gp, partA);
}

struct AdaptiveStep {
  double tau_max, tol;
};

template <typename T, bool NT>
static void launch_combine(typename Cx<T>::V* psi, const typename Cx<T>::V* U, uint32_t D, int B, int m,
                           const KState& st, bool pack2, int G, int threads, size_t cfb, hipStream_t s) {
  if (B == 1) {
    if (pack2)
      hipLaunchKernelGGL((k_combine<T, 2, true, NT>), dim3(G), dim3(threads), 0, s, psi, U, D, B, m, st);
    else
      hipLaunchKernelGGL((k_combine<T, 1, true, NT>), dim3(G), dim3(threads), 0, s, psi, U, D, B, m, st);
  } else {
    if (pack2)
      hipLaunchKernelGGL((k_combine<T, 2, false, NT>), dim3(G), dim3(threads), cfb, s, psi, U, D, B, m, st);
    else
      hipLaunchKernelGGL((k_combine<T, 1, false, NT>), dim3(G), dim3(threads), cfb, s, psi, U, D, B, m, st);
  }
}

template <typename T>
static qk_status krylov_step_t(qk_krylov* k, void* psi_v, double dt, hipStream_t s, StepUpTo upto,
                               const AdaptiveStep* ad = nullptr) {
  using V = typename Cx<T>::V;
  const qk_ham* H = k->H;
  const int B = H->batch, threads = krylov_threads(k), G = k->grid, m = k->m;
  const uint32_t D = (uint32_t)H->basis->D;
  const size_t stride = (size_t)k->ustride;   // D * B, or the padded length of the split layout
  V* psi = (V*)psi_v;
  V* U = (V*)k->d_U;
  const KState st = make_kstate(k);
  // streaming kernels read with non-temporal loads once a vector outgrows the last-level cache
  const bool nt = stride * sizeof(V) >= kNtBytes;
  // breakdown threshold relative to the largest coefficient so far
  const double rtol = std::is_same<T, double>::value ? 1e-12 : 1e-5;
#define QK_MARK(kind, begin)                                   \
  do {                                                         \
    if (k->profiling) {                                        \
      qk_status ps_ = profile_mark(k, kind, begin, s);         \
      if (ps_ != QK_OK) return ps_;                            \
    }                                                          \
  } while (0)
  // large batches: partial sums are totalled once per pass (k_partials_total)
  // and consumers read the single row of totals
  const bool pre = B >= kPreReduceBatch;
  double* totA = k->d_ptot;
  double* totB = k->d_ptot + (size_t)kQA * B;
  const double* pB = pre ? totB : k->d_partB;
  int GB = pre ? 1 : G;
  if (k->d_Z) {
    // two-pass split: the pre-pass of the initial vector, then per iteration
    // the high pass (z) and the low pass (u_{j+1}); the low pass's partials
    // alternate between two buffers (one is read while the other is written)
    double* spA = k->d_sp;
    double* spB[2] = {k->d_sp + 2 * (size_t)kMaxPartialBlocks, k->d_sp + 3 * (size_t)kMaxPartialBlocks};
    double* spQ[2] = {k->d_sp + 4 * (size_t)kMaxPartialBlocks, k->d_sp + 5 * (size_t)kMaxPartialBlocks};
    int Glo = 0, Ghi = 0;
    QK_MARK(QK_KERNEL_PREPASS, true);
    {
      qk_status ps = launch_split_form(H, k->dtype, psi, spB[0], spQ[0], &Glo, s);
      if (ps != QK_OK) return ps;
    }
    QK_MARK(QK_KERNEL_PREPASS, false);
    for (int j = 0; j < m; ++j) {
      LanczosArgs la{j, m, rtol, 0};
      const V* uj = j == 0 ? psi : U + (size_t)(j - 1) * stride;
      const V* ujm1 = j == 0 ? nullptr : (j == 1 ? psi : U + (size_t)(j - 2) * stride);
      QK_MARK(QK_KERNEL_LANCZOS_H, true);
      qk_status ps = launch_split_hi(H, k->dtype, uj, ujm1, k->d_Z, st, la, spB[j & 1], Glo, spA, &Ghi,
                                     k->blocked_wgs, s);
      if (ps != QK_OK) return ps;
      QK_MARK(QK_KERNEL_LANCZOS_H, false);
      QK_MARK(QK_KERNEL_LANCZOS_UPDATE, true);
      ps = launch_split_lo(H, k->dtype, uj, k->d_Z, U + (size_t)j * stride, st, la, spA, Ghi, spB[j & 1], spQ[j & 1],
                           Glo, spB[(j + 1) & 1], spQ[(j + 1) & 1], j + 1 < m ? 1 : 0, &Glo, s);
      if (ps != QK_OK) return ps;
      QK_MARK(QK_KERNEL_LANCZOS_UPDATE, false);
    }
    pB = spB[m & 1];
    GB = Glo;
  }
  for (int j = 0; j < (k->d_Z ? 0 : m); ++j) {
    LanczosArgs la{j, m, rtol, k->reorth == 1 ? 1 : 0};
    const V* uj = j == 0 ? psi : U + (size_t)(j - 1) * stride;
    const V* ujm1 = j == 0 ? nullptr : (j == 1 ? psi : U + (size_t)(j - 2) * stride);
    V* w = U + (size_t)j * stride;
    QK_MARK(QK_KERNEL_LANCZOS_H, true);
    int Ga = G;
    if (blocked_usable(H, k->dtype)) {
      qk_status bs = launch_blocked_lanczos_h(H, k->dtype, uj, ujm1, w, st, la, pB, GB, k->d_partA, &Ga,
                                              k->blocked_wgs, s);
      if (bs != QK_OK) return bs;
    } else if (H->basis->wide) {
      launch_lanczos_rows<T, uint64_t>(H, uj, ujm1, w, st, la, pB, GB, G, threads, k->d_partA, s);
    } else {
      launch_lanczos_rows<T, uint32_t>(H, uj, ujm1, w, st, la, pB, GB, G, threads, k->d_partA, s);
    }
    QK_HIP(hipGetLastError());
    QK_MARK(QK_KERNEL_LANCZOS_H, false);
    QK_MARK(QK_KERNEL_LANCZOS_UPDATE, true);
    const double* pA = k->d_partA;
    int GA = Ga;
    if (pre) {
      hipLaunchKernelGGL(k_partials_total, dim3((kQA * B + kTotCols - 1) / kTotCols), dim3(256), 0, s, k->d_partA, Ga,
                         kQA * B, totA);
      QK_HIP(hipGetLastError());
      pA = totA;
      GA = 1;
    }
    if (nt)
      hipLaunchKernelGGL((k_lanczos_B<T, true>), dim3(G), dim3(threads), 0, s, uj, ujm1, w, D, B, st, la, pA, GA,
                         k->d_partB, j + 1 < m ? 1 : 0);
    else
      hipLaunchKernelGGL((k_lanczos_B<T, false>), dim3(G), dim3(threads), 0, s, uj, ujm1, w, D, B, st, la, pA, GA,
                         k->d_partB, j + 1 < m ? 1 : 0);
    QK_HIP(hipGetLastError());
    if (k->reorth == 2 && j + 1 < m) {
      // u_{j+1} against v_0..v_j, twice
      const int nv = j + 1, Gr = G < kReorthGrid ? G : kReorthGrid;
      for (int pass = 0; pass < 2; ++pass) {
        for (int c0 = 0; c0 < nv; c0 += kReorthChunk) {
          const int ni = nv - c0 < kReorthChunk ? nv - c0 : kReorthChunk;
          hipLaunchKernelGGL((k_reorth_dots<T>), dim3(Gr), dim3(threads), 0, s, psi, U, w, D, B, c0, ni,
                             k->d_rpart + (size_t)(c0 / kReorthChunk) * kReorthGrid * 2 * kReorthChunk * B);
          QK_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_reorth_coef, dim3(1), dim3(kMaxBlock), 0, s, k->d_rpart, Gr, nv, B, j, st, k->d_rcoef);
        QK_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_reorth_axpy<T>), dim3(G), dim3(threads), 0, s, psi, U, w, D, B, nv, k->d_rcoef,
                           k->d_partB);
        QK_HIP(hipGetLastError());
      }
    }
    if (pre) {
      hipLaunchKernelGGL(k_partials_total, dim3((B + kTotCols - 1) / kTotCols), dim3(256), 0, s, k->d_partB, G, B,
                         totB);
      QK_HIP(hipGetLastError());
    }
    QK_MARK(QK_KERNEL_LANCZOS_UPDATE, false);
  }
  if (upto == StepUpTo::basis) return QK_OK;   // only the Krylov basis and coefficients were asked for
  QK_MARK(QK_KERNEL_SMALL_EXPM, true);
  if (ad) {
    hipLaunchKernelGGL(k_step_size, dim3(B), dim3(64), 0, s, st, m, B, ad->tau_max, ad->tol, pB, GB);
    QK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_small_expm, dim3(B), dim3(64), 0, s, st, m, B, dt, ad ? (const double*)st.tau : nullptr,
                     pB, GB);
  QK_HIP(hipGetLastError());
  QK_MARK(QK_KERNEL_SMALL_EXPM, false);
  QK_MARK(QK_KERNEL_COMBINE, true);
  if (k->d_Z) {
    qk_status cs = launch_split_combine(H, k->dtype, psi, U, st, s);
    if (cs != QK_OK) return cs;
    QK_MARK(QK_KERNEL_COMBINE, false);
    return QK_OK;
  }
  // complex64 elements go two to a 16-byte access when the vector length and
  // both base addresses allow it
  const bool pack2 = sizeof(V) == 8 && ((uint64_t)D * B) % 2 == 0 && ((uintptr_t)psi % 16) == 0 &&
                     ((uintptr_t)U % 16) == 0;
  const size_t cfb = B > 1 ? sizeof(double2) * (size_t)m * B : 0;
  if (nt)
    launch_combine<T, true>(psi, U, D, B, m, st, pack2, G, threads, cfb, s);
  else
    launch_combine<T, false>(psi, U, D, B, m, st, pack2, G, threads, cfb, s);
  QK_HIP(hipGetLastError());
  QK_MARK(QK_KERNEL_COMBINE, false);
#undef QK_MARK
  return QK_OK;
}

// Event pair around one launch: `begin` records the start event, the
// matching call after the launch records the end event.
qk_status profile_mark(qk_krylov* k, int kind, bool begin, hipStream_t s) {
  hipEvent_t ev;
  if (!k->spare.empty()) {
    ev = k->spare.back();
    k->spare.pop_back();
  } else {
    QK_HIP(hipEventCreate(&ev));
  }
  if (begin) {
    k->pending.push_back({kind, ev, nullptr});
  } else {
    k->pending.back().end = ev;
  }
  QK_HIP(hipEventRecord(ev, s));
  return QK_OK;
}

qk_status profile_collect(qk_krylov* k) {
  for (auto& p : k->pending) {
    if (!p.end) continue;
    QK_HIP(hipEventSynchronize(p.end));
    float ms = 0.f;
    QK_HIP(hipEventElapsedTime(&ms, p.start, p.end));
    k->ms_total[p.kind] += ms;
    k->launches[p.kind] += 1;
    k->spare.push_back(p.start);
    k->spare.push_back(p.end);
  }
  k->pending.clear();
  return QK_OK;
}

qk_status launch_krylov_step(qk_krylov* k, void* psi, double dt, hipStream_t s, StepUpTo upto) {
  if (k->dtype == QK_C128) return krylov_step_t<double>(k, psi, dt, s, upto);
  return krylov_step_t<float>(k, psi, dt, s, upto);
}

qk_status launch_krylov_adaptive_step(qk_krylov* k, void* psi, double tau_max, double tol, hipStream_t s) {
  const AdaptiveStep ad{tau_max, tol};
  if (k->dtype == QK_C128) return krylov_step_t<double>(k, psi, tau_max, s, StepUpTo::combination, &ad);
  return krylov_step_t<float>(k, psi, tau_max, s, StepUpTo::combination, &ad);
}

qk_status launch_return_prob(const qk_basis* b, int64_t r0, const void* psi0, const void* psi, int dtype, int B,
                             double* P, hipStream_t s) {
  const uint32_t D = (uint32_t)b->D;
  if (psi0 == nullptr) {
    if (dtype == QK_C128)
      hipLaunchKernelGGL(k_prob_basis_state<double>, dim3(1), dim3(64), 0, s, (const double2*)psi, (uint32_t)r0, B, P);
    else
      hipLaunchKernelGGL(k_prob_basis_state<float>, dim3(1), dim3(64), 0, s, (const float2*)psi, (uint32_t)r0, B, P);
    QK_HIP(hipGetLastError());
    return QK_OK;
  }
  const int threads = block_threads(B);
  const int G = stream_grid(D, B, threads, 0);
  double* part = nullptr;
  QK_HIP(dev_alloc_async(b->al, (void**)&part, sizeof(double) * (size_t)G * 2 * B, s));
  if (dtype == QK_C128)
    hipLaunchKernelGGL(k_overlap_partial<double>, dim3(G), dim3(threads), 0, s, (const double2*)psi0,
                       (const double2*)psi, D, B, part);
  else
    hipLaunchKernelGGL(k_overlap_partial<float>, dim3(G), dim3(threads), 0, s, (const float2*)psi0,
                       (const float2*)psi, D, B, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_overlap_final, dim3(1), dim3(kMaxBlock), 0, s, part, G, B, P, (const int*)nullptr, 0, 0);
    e = hipGetLastError();
  }
  QK_HIP(dev_free_async(b->al, part, s));
  QK_HIP(e);
  return QK_OK;
}

// --------------------------------------- survival probability without allocation
// Partial sums of the general-state overlap for callers that cannot allocate
// (graph capture, serving loops): one file-scope array per GPU, large enough
// for the widest grid of the overlap pass (kMaxPartialBlocks blocks x 2 x 64
// batch columns, 4 MiB), held until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.  Every
// slot the final reduction reads is written by the partial pass of the same
// call, so nothing has to be cleared; calls that overlap on one GPU share
// the array and race.
constexpr size_t kNoAllocScratchDoubles = (size_t)kMaxPartialBlocks * 2 * QK_MAX_BATCH;
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static qk_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the scratch table");
    return QK_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    QK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = (double*)g_scratch_ptr[dev];
  return QK_OK;
}

qk_status launch_return_prob_noalloc(const qk_basis* b, int64_t r0, const void* psi0, const void* psi, int dtype,
                                     int B, double* P, hipStream_t s) {
  if (psi0 == nullptr) return launch_return_prob(b, r0, psi0, psi, dtype, B, P, s);   // one element, no scratch
  const uint32_t D = (uint32_t)b->D;
  const int threads = block_threads(B);
  const int G = stream_grid(D, B, threads, 0);
  const size_t need = (size_t)G * 2 * B;
  if (need > kNoAllocScratchDoubles) {
    set_error("overlap partials exceed the fixed scratch of the allocation-free entry point");
    return QK_EINVAL;
  }
  double* part = nullptr;
  qk_status st = scratch_address(b->device, &part);
  if (st != QK_OK) return st;
  if (dtype == QK_C128)
    hipLaunchKernelGGL(k_overlap_partial<double>, dim3(G), dim3(threads), 0, s, (const double2*)psi0,
                       (const double2*)psi, D, B, part);
  else
    hipLaunchKernelGGL(k_overlap_partial<float>, dim3(G), dim3(threads), 0, s, (const float2*)psi0,
                       (const float2*)psi, D, B, part);
  QK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_overlap_final, dim3(1), dim3(kMaxBlock), 0, s, part, G, B, P, (const int*)nullptr, 0, 0);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

int overlap_grid(uint32_t D, int B) { return stream_grid(D, B, block_threads(B), 0); }

qk_status launch_overlap_record(const void* psi0, const void* psi, int dtype, uint32_t D, int B, double* part, int G,
                                double* P, const int* counter, int off, int items, hipStream_t s) {
  const int threads = block_threads(B);
  if (dtype == QK_C128)
    hipLaunchKernelGGL(k_overlap_partial<double>, dim3(G), dim3(threads), 0, s, (const double2*)psi0,
                       (const double2*)psi, D, B, part);
  else
    hipLaunchKernelGGL(k_overlap_partial<float>, dim3(G), dim3(threads), 0, s, (const float2*)psi0,
                       (const float2*)psi, D, B, part);
  QK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_overlap_final, dim3(1), dim3(kMaxBlock), 0, s, part, G, B, P, counter, off, items);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

int krylov_threads(const qk_krylov* k) { return block_threads(k->batch, k->threads > 0 ? k->threads : kMaxBlock); }

int krylov_grid(uint64_t D, int B) { return stream_grid(D, B, 0, 0); }

}  // namespace qk

// Derivative of the survival probability F(T) = |A(T)|^2, A(T) =
// <psi0| exp(-iHT) |psi0> (Sec. 4) with respect to every on-site field h_i of
// Eq. (1), by the adjoint (costate) method on top of the Krylov steps.
//
// H depends on h_i through h_i Z_i, Z_i = diag(bit_i - 1/2), so
//     dA/dh_i = -i * integral_0^T <lambda(s)| Z_i |psi(s)> ds,
//     lambda(s) = exp(+iH(T-s)) psi0,
// and dF/dh_i = 2 Re(conj(A) dA/dh_i).  With K time steps t_k = k dt:
//   * the forward pass stores psi_k (checkpoints);
//   * the costate runs backward, lambda_K = psi0 and lambda_k =
//     exp(+iH dt) lambda_{k+1}, i.e. a Krylov step with time step -dt;
//   * inside step k, psi(t_k + tau) = V p(tau) with p(tau) = exp(-i tau T) ||psi_k|| e_1
//     (the Krylov basis V of psi_k) and
//     lambda(t_k + tau) = W q(tau) with q(tau) = exp(+i (dt - tau) T') ||lambda_{k+1}|| e_1
//     (the basis W of the backward step), so
//         integral over the step of <lambda|Z_i|psi>
//           = sum_r z_i(r) sum_{c,d} conj(W_rc) C_cd V_rd,
//         C_cd = integral_0^dt conj(q_c(tau)) p_d(tau) dtau.
//     C is a small m x m matrix, integrated by Gauss-Legendre quadrature of
//     the m-dimensional propagators (an entire function of tau, so the rule
//     converges to rounding error), and the row sum is one pass over the two
//     Krylov bases.
// H is real and psi0 = e_r0 is real, so time reversal gives the costate as
// the conjugated forward state: lambda(s) = conj(psi(T - s)), and with the
// Krylov scheme lambda_{k+1} = conj(psi_{K-1-k}) step by step (a Lanczos run on
// conj(u) with a real H produces the conjugated vectors and the same alpha,
// beta).  The backward step's basis and matrix are therefore those of the
// forward step from psi_{K-1-k}: W = conj(V'), T' = T_{K-1-k}, and
// conj(W_rc) = V'_rc.  The backward sweep reads the forward bases of the
// steps k and K-1-k instead of propagating the costate.
#include <cmath>
#include <cstdlib>
#include <new>
#include <utility>
#include <vector>

#include "qk_device.h"

namespace qk {

constexpr int kGradMaxM = 32;      // Krylov dimension of the gradient (register-held basis rows)
constexpr int kGaussNodes = 24;

struct GaussRule {
  double x[kGaussNodes];   // nodes on [0, 1]
  double w[kGaussNodes];   // weights on [0, 1]
};

// Gauss-Legendre nodes and weights by Newton's method on the Legendre
// polynomial P_n (three-term recurrence), mapped from [-1, 1] to [0, 1].
static GaussRule gauss_legendre() {
  GaussRule g{};
  const int n = kGaussNodes;
  for (int i = 0; i < n; ++i) {
    double x = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    g.x[i] = 0.5 * (x + 1.0);
    g.w[i] = 1.0 / ((1.0 - x * x) * dp * dp);   // 2 / ((1-x^2) P_n'(x)^2) times 1/2
  }
  return g;
}

// C = integral_0^dt conj(q(tau)) p(tau)^T dtau by the Gauss rule: block n
// (one wavefront; lane i owns component i of p and q) evaluates node n and
// writes its weighted term w_n conj(q_c) p_d to Cn[n][c][d] (complex).
__global__ void __launch_bounds__(64)
k_grad_nodes(KState fw, KState bw, double dt, GaussRule gr, double* __restrict__ Cn) {
  __shared__ double Pr[64], Pi[64];
  const int i = threadIdx.x, n = blockIdx.x;
  const int muf = fw.mused[0], mub = bw.mused[0];
  if (fw.status[0] != QK_OK || bw.status[0] != QK_OK || muf <= 0 || mub <= 0) return;   // k_grad_coeffs writes zeros
  const bool onf = i < muf, onb = i < mub;
  const double alf = onf ? fw.alpha[i] : 0.0, bef = (i + 1 < muf) ? fw.beta[i] : 0.0;
  const double blf = (onf && i > 0) ? fw.beta[i - 1] : 0.0;
  const double alb = onb ? bw.alpha[i] : 0.0, beb = (i + 1 < mub) ? bw.beta[i] : 0.0;
  const double blb = (onb && i > 0) ? bw.beta[i - 1] : 0.0;
  const double tau = dt * gr.x[n], wq = dt * gr.w[n];
  double pr, pi, qr, qi;
  tri_expm_e1(alf, bef, blf, onf, i, tau, pr, pi);           // exp(-i tau T) e_1
  tri_expm_e1(alb, beb, blb, onb, i, -(dt - tau), qr, qi);   // exp(+i (dt - tau) T') e_1
  Pr[i] = fw.n0[0] * pr;
  Pi[i] = fw.n0[0] * pi;
  qr *= bw.n0[0];
  qi *= bw.n0[0];
  __syncthreads();
  if (i < mub && i < kGradMaxM) {
    double* out = Cn + (size_t)n * 2 * kGradMaxM * kGradMaxM + 2 * (size_t)i * kGradMaxM;
    for (int d = 0; d < muf && d < kGradMaxM; ++d) {
      // conj(q_i) p_d
      out[2 * d] = wq * (qr * Pr[d] + qi * Pi[d]);
      out[2 * d + 1] = wq * (qr * Pi[d] - qi * Pr[d]);
    }
  }
}

// C~_cd = sigma'_c sigma_d C_cd for the stored (unnormalised) basis vectors:
// the node terms summed in node order (one thread per entry).
__global__ void __launch_bounds__(kGradMaxM * kGradMaxM)
k_grad_coeffs(KState fw, KState bw, const double* __restrict__ Cn, double* __restrict__ Ct) {
  const int e = threadIdx.x, c = e / kGradMaxM, d = e % kGradMaxM;
  const int muf = fw.mused[0], mub = bw.mused[0];
  const bool ok = fw.status[0] == QK_OK && bw.status[0] == QK_OK && c < mub && d < muf;
  double cr = 0.0, ci = 0.0;
  if (ok)
    for (int n = 0; n < kGaussNodes; ++n) {
      cr += Cn[(size_t)n * 2 * kGradMaxM * kGradMaxM + 2 * e];
      ci += Cn[(size_t)n * 2 * kGradMaxM * kGradMaxM + 2 * e + 1];
    }
  const double sc = ok ? bw.sigma[c] * fw.sigma[d] : 0.0;
  Ct[2 * e] = sc * cr;
  Ct[2 * e + 1] = sc * ci;
}

// Per row r: s_r = sum_c v'_c[r] t_c[r], t = C~ u[r], where u is the forward
// basis of step k (u_0 = psi_k) and v' that of the mirrored step K-1-k
// (v'_0 = psi_{K-1-k}), i.e. the conjugated costate basis, further vectors
// from the workspace slots.  t = C~ U
// over all rows is a dense product (m x m times m x rows), done on the FP64
// matrix cores in its real form: the complex C~ becomes the 2m x 2m real
// matrix R with R[2c][2d] = R[2c+1][2d+1] = Re C~_cd, R[2c][2d+1] = -Im C~_cd,
// R[2c+1][2d] = Im C~_cd, and the interleaved (re, im) rows of the basis are
// the other operand.  One wavefront takes tiles of 16 consecutive positions
// (the N of one 16x16x4 FP64 MFMA):
//   * lane (q, n), q = lane / 16, n = lane % 16, loads u_d at position n for
//     d = 4s + q (s = 0..7) as one 16-byte load; its real and imaginary parts
//     are the B operands of K-steps 2s and 2s + 1, so K-step k of quarter q
//     is real column 2(4(k/2) + q) + k%2 of R;
//   * the A operands (R in that K order, per M-block of 16 real rows) are
//     read from LDS, where the block stored them in fragment order;
//   * register v of lane (q, n) of the MFMA's output holds output row
//     4v + q at position n, so R's rows are ordered to make output row 4v + q
//     of M-block b the component v % 2 of t_c, c = 8b + 2q + v / 2: the lane
//     holds t_c for c = 8b + 2q and c + 1 (re, im, re, im), loads v'_c for
//     those c and forms its share of s_n; the four quarters' shares are added
//     across lanes.
// Lane i then adds s_n over the tile's positions whose state has bit i set,
// every lane the total; per block the four waves' sums are added in wave
// order into 2(L_max + 1) partial sums.
constexpr int kGradQ = 2 * (QK_MAX_L + 1);
constexpr int kGcWaves = 4;                    // wavefronts per block
constexpr int kGcN = 16;                       // positions per wavefront tile
constexpr int kGcMb = 2 * kGradMaxM / 16;      // M-blocks of R (16 real rows each)
constexpr int kGcKs = 2 * kGradMaxM / 4;       // K-steps of R (4 real columns each)
constexpr int kGcFrag = kGcMb * kGcKs * 64;    // doubles of R in fragment order
static_assert(kGradMaxM == 32, "fragment layout assumes 32 basis vectors: 8 K-step pairs, 4 M-blocks");

typedef double gc_dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double gc_readlane(double v, int j) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t gc_readlane(uint32_t v, int j) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
}
__device__ __forceinline__ uint64_t gc_readlane(uint64_t v, int j) {
  const uint32_t lo = gc_readlane((uint32_t)v, j), hi = gc_readlane((uint32_t)(v >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

// loads through a global-address-space pointer (plain loads, no flat ones
// that would share the LDS wait counter)
typedef double gc_dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gc_ld(const double2* p) {
  const gc_dbl2 v = *(const __attribute__((address_space(1))) gc_dbl2*)p;
  return make_double2(v.x, v.y);
}
template <typename S>
__device__ __forceinline__ S gc_ld(const S* p) {
  return *(const __attribute__((address_space(1))) S*)p;
}

template <typename S>
__global__ void __launch_bounds__(256, 4)
k_grad_contract(const S* __restrict__ states, uint64_t niter, int L, const double2* __restrict__ psi_k,
                const double2* __restrict__ Uf, const double2* __restrict__ vm0, const double2* __restrict__ Ub,
                size_t stride, const uint32_t* __restrict__ line_r0, const uint8_t* __restrict__ line_n, int pe,
                KState fw, KState bw, const double* __restrict__ Ct, double* __restrict__ part) {
  // niter positions of the workspace vectors (stride elements each): rows of
  // the sorted basis, or, with line tables, elements of the padded layout
  // whose row comes from their line's entry (unused padding is skipped)
  __shared__ double Af[kGcFrag];                // [M-block][K-step][lane]
  __shared__ double red[kGcWaves][kGradQ];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // R in fragment order: lane l of (b, k) holds the R entry of output row
  // i = l % 16 (component (i / 4) % 2 of t_c, c = 8b + 2(i % 4) + i / 8) and
  // of the column of K-step k for quarter l / 16
  for (int e = tid; e < kGcFrag; e += blockDim.x) {
    const int b = e / (kGcKs * 64), k = (e / 64) % kGcKs, l = e % 64, i = l % 16;
    const int c = 8 * b + 2 * (i & 3) + (i >> 3), pc = (i >> 2) & 1;
    const int d = 4 * (k >> 1) + l / 16, pd = k & 1;
    const double cr = Ct[2 * (c * kGradMaxM + d)], ci = Ct[2 * (c * kGradMaxM + d) + 1];
    Af[e] = pc == pd ? cr : (pc == 0 ? -ci : ci);
  }
  const int muf = fw.mused[0] < kGradMaxM ? fw.mused[0] : kGradMaxM;
  const int mub = bw.mused[0] < kGradMaxM ? bw.mused[0] : kGradMaxM;
  __syncthreads();
  const int q = lane >> 4, n = lane & 15;
  // row and validity of position p
  auto locate = [&](uint64_t p, size_t* r) -> bool {
    *r = (size_t)p;
    if (p >= niter) return false;
    if (!line_r0) return true;
    const uint64_t ln = p / (uint64_t)pe;
    const uint32_t e = (uint32_t)(p - ln * (uint64_t)pe);
    *r = (size_t)line_r0[ln] + e;
    return e < line_n[ln];
  };
  const double2 zero = make_double2(0.0, 0.0);
  double ar = 0.0, ai = 0.0, tr = 0.0, ti = 0.0;   // site `lane`, and the total
  const uint64_t ntiles = (niter + kGcN - 1) / kGcN;
  const uint64_t wstep = (uint64_t)gridDim.x * kGcWaves;
  for (uint64_t t = (uint64_t)blockIdx.x * kGcWaves + wv; t < ntiles; t += wstep) {
    // the A fragments are read from LDS per tile: hoisted out of the loop
    // they would need 128 registers per lane
    __asm__ volatile("" ::: "memory");
    const uint64_t p = t * kGcN + (uint64_t)n;
    size_t r;
    const bool valid = locate(p, &r);
    // every lane loads (unused vectors and positions from element 0 of
    // psi_k) and zeroes what it does not use: no branches around the loads
    const size_t rv = valid ? r : 0, pv = valid ? (size_t)p : 0;
    // slot offsets as one per-lane part and one uniform part per load (the
    // uniform part of slot 4s + q - 1 wraps below zero only for d = 0,
    // which reads psi_k instead)
    const size_t lu = (size_t)q * stride + pv, lw = (size_t)(2 * q) * stride + pv;
    double2 u[kGcKs / 2];
#pragma unroll
    for (int s = 0; s < kGcKs / 2; ++s) {
      const int d = 4 * s + q;
      const bool on = valid && d < muf;
      u[s] = gc_ld(d == 0 || !on ? psi_k + rv : Uf + (lu + (size_t)(4 * s - 1) * stride));
      if (!on) u[s] = zero;
    }
    double2 w[2 * kGcMb];
#pragma unroll
    for (int h = 0; h < 2 * kGcMb; ++h) {
      const int c = 8 * (h >> 1) + 2 * q + (h & 1);
      const bool on = valid && c < mub;
      w[h] = gc_ld(!on ? psi_k : (c == 0 ? vm0 + rv : Ub + (lw + (size_t)(8 * (h >> 1) + (h & 1) - 1) * stride)));
      if (!on) w[h] = zero;
    }
    S st = gc_ld(states + rv);
    if (!valid) st = (S)0;
    gc_dbl4 acc[kGcMb];
#pragma unroll
    for (int b = 0; b < kGcMb; ++b) acc[b] = gc_dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kGcKs / 2; ++s) {
#pragma unroll
      for (int b = 0; b < kGcMb; ++b) {
        const double a0 = Af[(b * kGcKs + 2 * s) * 64 + lane], a1 = Af[(b * kGcKs + 2 * s + 1) * 64 + lane];
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, u[s].x, acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, u[s].y, acc[b], 0, 0, 0);
      }
    }
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int b = 0; b < kGcMb; ++b) {
      const double2 w0 = w[2 * b], w1 = w[2 * b + 1];   // v'_c t_c
      sr += w0.x * acc[b][0] - w0.y * acc[b][1];
      si += w0.x * acc[b][1] + w0.y * acc[b][0];
      sr += w1.x * acc[b][2] - w1.y * acc[b][3];
      si += w1.x * acc[b][3] + w1.y * acc[b][2];
    }
    // (q0 + q1) + (q2 + q3): every quarter ends with the same bits
    sr += __shfl_xor(sr, 16);
    si += __shfl_xor(si, 16);
    sr += __shfl_xor(sr, 32);
    si += __shfl_xor(si, 32);
#pragma unroll
    for (int j = 0; j < kGcN; ++j) {
      const double sj = gc_readlane(sr, j), tj = gc_readlane(si, j);
      const S stj = gc_readlane(st, j);
      tr += sj;
      ti += tj;
      const bool on = lane < L && ((stj >> (lane & (8 * (int)sizeof(S) - 1))) & (S)1);
      ar += on ? sj : 0.0;
      ai += on ? tj : 0.0;
    }
  }
  red[wv][2 * lane] = lane < L ? ar : 0.0;
  red[wv][2 * lane + 1] = lane < L ? ai : 0.0;
  if (lane == 0) {
    red[wv][2 * QK_MAX_L] = tr;
    red[wv][2 * QK_MAX_L + 1] = ti;
  }
  __syncthreads();
  if (tid < kGradQ) {
    double v = red[0][tid];
    for (int k = 1; k < kGcWaves; ++k) v += red[k][tid];
    part[(size_t)blockIdx.x * kGradQ + tid] = v;
  }
}

// dA[i] += -i (S_i - S_total / 2), the partial sums of the G contraction
// blocks totalled in a fixed order: kAccLanes lanes per column each add every
// kAccLanes-th block, then one thread adds the lanes in order.
constexpr int kAccLanes = 7;
constexpr int kAccThreads = 1024;
static_assert(kGradQ * kAccLanes <= kAccThreads, "one lane group per column");
__global__ void __launch_bounds__(kAccThreads) k_grad_accum(const double* __restrict__ part, int G, int L,
                                                           double* __restrict__ dA) {
  __shared__ double red[kGradQ * kAccLanes];
  __shared__ double tot[kGradQ];
  const int t = threadIdx.x, c = t / kAccLanes, l = t % kAccLanes;
  if (c < kGradQ) {
    double acc = 0.0;
    for (int g = l; g < G; g += kAccLanes) acc += part[(size_t)g * kGradQ + c];
    red[c * kAccLanes + l] = acc;
  }
  __syncthreads();
  if (t < kGradQ) {
    double s = 0.0;
    for (int k = 0; k < kAccLanes; ++k) s += red[t * kAccLanes + k];
    tot[t] = s;
  }
  __syncthreads();
  if (t < L) {
    const double gr = tot[2 * t] - 0.5 * tot[2 * QK_MAX_L];
    const double gi = tot[2 * t + 1] - 0.5 * tot[2 * QK_MAX_L + 1];
    dA[2 * t] += gi;       // -i (gr + i gi) = gi - i gr
    dA[2 * t + 1] -= gr;
  }
}

__global__ void k_basis_vector(double2* __restrict__ v, uint32_t D, uint32_t r0) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < D) v[r] = make_double2(r == r0 ? 1.0 : 0.0, 0.0);
}

qk_status grad_return_prob(qk_krylov* k, int64_t r0, double T, int n_steps, int ckpt_every, double* F, double* dFdh,
                           hipStream_t s) {
  const qk_ham* H = k->H;
  const uint32_t D = (uint32_t)k->D;
  const int L = H->basis->L;
  const double dt = T / n_steps;
  const size_t vbytes = sizeof(double2) * (size_t)D;
  const int G = 1024;
  // Every forward Krylov basis (and its coefficients) is kept for the
  // duration of the call when all of them fit in 80 % of the free device
  // memory, so the backward pass needs no rebuilding; QK_GRAD_KEEP=0 turns
  // this off.  Otherwise each basis is rebuilt from its checkpoint.
  const size_t ubytes = sizeof(double2) * (size_t)k->ustride * (size_t)k->m;   // one basis
  const size_t cdoubles = kstate_doubles(k->m, 1);
  void* ubank = nullptr;
  double* cbank = nullptr;
  int32_t* ibank = nullptr;
  {
    const char* ev = getenv("QK_GRAD_KEEP");
    size_t fr = 0, tot = 0;
    if (!(ev && ev[0] == '0') && hipMemGetInfo(&fr, &tot) == hipSuccess &&
        ubytes * (size_t)n_steps + vbytes * (size_t)(n_steps + 1) <= fr / 10 * 8) {
      if (dev_alloc(k->al, &ubank, ubytes * (size_t)n_steps) != hipSuccess ||
          dev_alloc(k->al, (void**)&cbank, sizeof(double) * cdoubles * n_steps) != hipSuccess ||
          dev_alloc(k->al, (void**)&ibank, sizeof(int32_t) * 2 * (size_t)n_steps) != hipSuccess) {
        dev_free(k->al, ubank);
        dev_free(k->al, cbank);
        dev_free(k->al, ibank);
        ubank = nullptr;
        cbank = nullptr;
        ibank = nullptr;
        (void)hipGetLastError();
      }
    }
  }
  const bool keep = ubank != nullptr;
  // kept bases need every state psi_t as a checkpoint
  const int c = keep ? 1 : (ckpt_every < 1 ? 1 : (ckpt_every > n_steps ? n_steps : ckpt_every));
  const int nck = n_steps / c + 1;   // checkpoints psi_0, psi_c, psi_2c, ...
  // Without kept bases a second workspace takes the mirrored forward steps
  // (psi_0, psi_1, ... while the backward sweep goes down from K-1), with the
  // launch shape of the first, so that its states and bases have the bits of
  // the forward pass.
  qk_krylov* kb = nullptr;   // workspace of the mirrored steps
  double2* ck = nullptr;     // checkpoints
  double2* seg = nullptr;    // recomputed states of one segment after its checkpoint (c - 1)
  double2* cur = nullptr;    // running forward state
  double2* mir = nullptr;    // psi_{K-1-t} of the mirrored steps
  double2* mnext = nullptr;  // the state after it
  double *Ct = nullptr, *Cn = nullptr, *part = nullptr, *dA = nullptr;
  qk_status st = keep ? QK_OK : krylov_create(H, k->m, QK_C128, k->reorth, k->al, &kb);
  if (st != QK_OK) {
    dev_free(k->al, ubank);
    dev_free(k->al, cbank);
    dev_free(k->al, ibank);
    return st;
  }
  if (kb) {
    kb->threads = k->threads;
    kb->blocks_per_cu = k->blocks_per_cu;
    kb->blocked_wgs = k->blocked_wgs;
    kb->grid = k->grid;
  }
  hipError_t e = dev_alloc(k->al, (void**)&ck, vbytes * (size_t)nck);
  if (e == hipSuccess && c > 1) e = dev_alloc(k->al, (void**)&seg, vbytes * (size_t)(c - 1));
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&cur, vbytes);
  if (e == hipSuccess && !keep) e = dev_alloc(k->al, (void**)&mir, vbytes);
  if (e == hipSuccess && !keep) e = dev_alloc(k->al, (void**)&mnext, vbytes);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&Ct, sizeof(double) * 2 * kGradMaxM * kGradMaxM);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&Cn, sizeof(double) * 2 * kGradMaxM * kGradMaxM * kGaussNodes);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&part, sizeof(double) * (size_t)G * kGradQ);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&dA, sizeof(double) * 2 * L);
  if (e == hipSuccess) e = hipMemsetAsync(dA, 0, sizeof(double) * 2 * L, s);
  const KState fw = make_kstate(k);
  const KState bw = kb ? make_kstate(kb) : fw;
  // the workspaces' vectors in the padded layout of the two-pass split: the
  // contraction walks that layout and finds each element's row in its line
  const uint32_t* lr0 = nullptr;
  const uint8_t* lnn = nullptr;
  int pe = 1;
  uint64_t niter = D;
  if (st == QK_OK && kb && (k->d_Z != nullptr) != (kb->d_Z != nullptr)) {
    set_error("forward and backward workspaces differ in layout");
    st = QK_EUNSUPPORTED;
  }
  if (st == QK_OK && k->d_Z) st = split_line_tables(H, QK_C128, &lr0, &lnn, &niter, &pe);
  const GaussRule gr = gauss_legendre();
  auto chk = [&](const char* what) {
    if (st == QK_OK && e == hipSuccess) e = hipGetLastError();
    if (st == QK_OK && e != hipSuccess) st = hip_fail(e, what);
  };
  chk("qk_grad_return_prob allocation");
  // forward pass, keeping psi_t for t = 0, c, 2c, ...
  if (st == QK_OK) {
    hipLaunchKernelGGL(k_basis_vector, dim3((D + 255) / 256), dim3(256), 0, s, cur, D, (uint32_t)r0);
    chk("k_basis_vector");
  }
  if (st == QK_OK) {
    e = hipMemcpyAsync(ck, cur, vbytes, hipMemcpyDeviceToDevice, s);
    chk("checkpoint copy");
  }
  void* const u_home = k->d_U;
  for (int t = 0; t < n_steps && st == QK_OK; ++t) {
    // with kept bases the step builds its basis directly in the bank
    if (keep) k->d_U = (char*)ubank + (size_t)t * ubytes;
    st = launch_krylov_step(k, cur, dt, s);
    k->d_U = u_home;
    if (st == QK_OK && keep) {
      e = hipMemcpyAsync(cbank + (size_t)t * cdoubles, k->d_coef, sizeof(double) * cdoubles, hipMemcpyDeviceToDevice,
                         s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(ibank + 2 * (size_t)t, k->d_int, sizeof(int32_t) * 2, hipMemcpyDeviceToDevice, s);
      chk("basis bank copy");
    }
    if (st == QK_OK && (t + 1) % c == 0 && (t + 1) / c < nck) {
      e = hipMemcpyAsync(ck + (size_t)((t + 1) / c) * D, cur, vbytes, hipMemcpyDeviceToDevice, s);
      chk("checkpoint copy");
    }
  }
  double2 A = make_double2(0.0, 0.0);
  if (st == QK_OK) {
    e = hipMemcpyAsync(&A, cur + r0, sizeof(double2), hipMemcpyDeviceToHost, s);
    chk("qk_grad_return_prob readback");
  }
  // psi_t inside the segment of checkpoint j: the checkpoint itself or a recomputed state
  auto state_at = [&](int t) -> double2* {
    const int j = t / c, o = t - j * c;
    return o == 0 ? ck + (size_t)j * D : seg + (size_t)(o - 1) * D;
  };
  // backward sweep; the mirrored steps start again from psi_0
  if (st == QK_OK && !keep) {
    hipLaunchKernelGGL(k_basis_vector, dim3((D + 255) / 256), dim3(256), 0, s, mir, D, (uint32_t)r0);
    chk("k_basis_vector");
  }
  for (int t = n_steps - 1; t >= 0 && st == QK_OK; --t) {
    if (t % c == c - 1 || t == n_steps - 1) {
      // entering a segment from its end: recompute its states after the checkpoint
      const int t0 = (t / c) * c;
      for (int u = t0 + 1; u <= t && st == QK_OK; ++u) {
        e = hipMemcpyAsync(state_at(u), state_at(u - 1), vbytes, hipMemcpyDeviceToDevice, s);
        chk("segment copy");
        if (st == QK_OK) st = launch_krylov_step(k, state_at(u), dt, s);
      }
      if (st != QK_OK) break;
    }
    // Krylov basis of psi_t: kept from the forward pass, or rebuilt from the
    // stored state (which is left unchanged)
    const double2* Uf = keep ? (const double2*)((char*)ubank + (size_t)t * ubytes) : (const double2*)k->d_U;
    const KState fwt = keep ? kstate_at(k, cbank + (size_t)t * cdoubles, ibank + 2 * (size_t)t) : fw;
    if (!keep) st = launch_krylov_step(k, state_at(t), dt, s, StepUpTo::basis);
    if (st != QK_OK) break;
    // the costate's step from lambda_{t+1} = conj(psi_{K-1-t}): the forward
    // step of the mirrored index, kept from the forward pass or taken now by
    // the second workspace from the mirrored state (which advances to the next)
    const int tm = n_steps - 1 - t;
    const double2* vm0 = keep ? ck + (size_t)tm * D : mir;
    const double2* Ub = keep ? (const double2*)((char*)ubank + (size_t)tm * ubytes) : (const double2*)kb->d_U;
    const KState bwt = keep ? kstate_at(k, cbank + (size_t)tm * cdoubles, ibank + 2 * (size_t)tm) : bw;
    if (!keep) {
      e = hipMemcpyAsync(mnext, mir, vbytes, hipMemcpyDeviceToDevice, s);
      chk("mirrored state copy");
      if (st == QK_OK) st = launch_krylov_step(kb, mnext, dt, s);
      if (st != QK_OK) break;
    }
    hipLaunchKernelGGL(k_grad_nodes, dim3(kGaussNodes), dim3(64), 0, s, fwt, bwt, dt, gr, Cn);
    chk("k_grad_nodes");
    if (st != QK_OK) break;
    hipLaunchKernelGGL(k_grad_coeffs, dim3(1), dim3(kGradMaxM * kGradMaxM), 0, s, fwt, bwt, (const double*)Cn, Ct);
    chk("k_grad_coeffs");
    if (st != QK_OK) break;
    if (H->basis->wide)
      hipLaunchKernelGGL(k_grad_contract<uint64_t>, dim3(G), dim3(256), 0, s, (const uint64_t*)H->basis->d_states,
                         niter, L, (const double2*)state_at(t), Uf, vm0, Ub, (size_t)k->ustride, lr0, lnn, pe, fwt,
                         bwt, Ct, part);
    else
      hipLaunchKernelGGL(k_grad_contract<uint32_t>, dim3(G), dim3(256), 0, s, (const uint32_t*)H->basis->d_states,
                         niter, L, (const double2*)state_at(t), Uf, vm0, Ub, (size_t)k->ustride, lr0, lnn, pe, fwt,
                         bwt, Ct, part);
    chk("k_grad_contract");
    if (st != QK_OK) break;
    hipLaunchKernelGGL(k_grad_accum, dim3(1), dim3(kAccThreads), 0, s, part, G, L, dA);
    chk("k_grad_accum");
    if (!keep) std::swap(mir, mnext);
  }
  std::vector<double> dAh(2 * L);
  if (st == QK_OK) {
    e = hipMemcpyAsync(dAh.data(), dA, sizeof(double) * 2 * L, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "qk_grad_return_prob readback");
  }
  if (st == QK_OK) {
    *F = A.x * A.x + A.y * A.y;
    for (int i = 0; i < L; ++i) dFdh[i] = 2.0 * (A.x * dAh[2 * i] + A.y * dAh[2 * i + 1]);
  }
  (void)hipStreamSynchronize(s);
  dev_free(k->al, ck);
  dev_free(k->al, seg);
  dev_free(k->al, cur);
  dev_free(k->al, mir);
  dev_free(k->al, mnext);
  dev_free(k->al, Ct);
  dev_free(k->al, Cn);
  dev_free(k->al, part);
  dev_free(k->al, dA);
  dev_free(k->al, ubank);
  dev_free(k->al, cbank);
  dev_free(k->al, ibank);
  qk_krylov_destroy(kb);
  return st;
}

}  // namespace qk

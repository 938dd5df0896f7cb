// Derivative of the survival probability F(T) = |A(T)|^2, A(T) =
// <psi0| exp(-iHT) |psi0> (Sec. 4) with respect to every on-site field h_i of
// Eq. (1), by the adjoint (costate) method on top of the Krylov steps.
//
// H depends on h_i through h_i Z_i, Z_i = diag(bit_i - 1/2), so
//     dA/dh_i = -i * integral_0^T <lambda(s)| Z_i |psi(s)> ds,
//     lambda(s) = exp(+iH(T-s)) psi0,
// and dF/dh_i = 2 Re(conj(A) dA/dh_i).  With time steps t_k = k dt:
//   * the forward pass stores psi_k (checkpoints);
//   * the costate runs backward, lambda_K = psi0 and lambda_k =
//     exp(+iH dt) lambda_{k+1}, i.e. a Krylov step with time step -dt;
//   * inside step k, psi(t_k + tau) = V p(tau) with p(tau) = exp(-i tau T) ||psi_k|| e_1
//     (the Krylov basis V of psi_k, rebuilt from the checkpoint) and
//     lambda(t_k + tau) = W q(tau) with q(tau) = exp(+i (dt - tau) T') ||lambda_{k+1}|| e_1
//     (the basis W of the backward step), so
//         integral over the step of <lambda|Z_i|psi>
//           = sum_r z_i(r) sum_{c,d} conj(W_rc) C_cd V_rd,
//         C_cd = integral_0^dt conj(q_c(tau)) p_d(tau) dtau.
//     C is a small m x m matrix, integrated by Gauss-Legendre quadrature of
//     the m-dimensional propagators (an entire function of tau, so the rule
//     converges to rounding error), and the row sum is one pass over the two
//     Krylov bases.
#include <cmath>
#include <cstdlib>
#include <new>
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

// Per row r: s_r = sum_c conj(u'_c[r]) sum_d C~_cd u_d[r] (u_0 = psi_k,
// u'_0 = lambda_{k+1}, further vectors from the workspace slots).  A block
// takes tiles of kGcRows consecutive positions: it stages u_d of the tile's
// rows for every d in LDS, from registers loaded while the previous tile was
// computed (the contraction reads 2m vectors per row once each, so it is
// bound by how many of those reads are in flight); then thread (g, j) computes t_c = sum_d C~_cd u_d for
// row j and the columns c = g, g + kGcGroups, ... (C~ read from LDS, the
// same address for the 32 threads of a row group), loads its u'_c directly
// and forms its share of s_j; the kGcGroups shares of a row are added in
// group order.  The tile's s_r and states then go to LDS, and thread
// q < 2(L_max+1) adds component q&1 of s_r over the tile's rows whose state
// has bit q>>1 set (q>>1 == L_max: all rows), so each block writes
// 2(L_max+1) partial sums.
constexpr int kGradQ = 2 * (QK_MAX_L + 1);
constexpr int kGcRows = 32;                          // rows per tile
constexpr int kGcGroups = 256 / kGcRows;             // column groups
constexpr int kGcCPer = kGradMaxM / kGcGroups;       // columns per thread

template <typename S>
__global__ void __launch_bounds__(256, 4)
k_grad_contract(const S* __restrict__ states, uint64_t niter, int L, const double2* __restrict__ psi_k,
                const double2* __restrict__ Uf, const double2* __restrict__ lam, const double2* __restrict__ Ub,
                size_t stride, const uint32_t* __restrict__ line_r0, const uint8_t* __restrict__ line_n, int pe,
                KState fw, KState bw, const double* __restrict__ Ct, double* __restrict__ part) {
  // niter positions of the workspace vectors (stride elements each): rows of
  // the sorted basis, or, with line tables, elements of the padded layout
  // whose row comes from their line's entry (unused padding is skipped)
  __shared__ double2 C[kGradMaxM * kGradMaxM];
  __shared__ double2 Us[kGradMaxM * kGcRows];   // [d][row of the tile]
  __shared__ double2 sp[kGcGroups * kGcRows];   // share of s per column group
  __shared__ double2 sbuf[kGcRows];
  __shared__ S sst[kGcRows];
  const int tid = threadIdx.x;
  for (int i = tid; i < kGradMaxM * kGradMaxM; i += blockDim.x) C[i] = make_double2(Ct[2 * i], Ct[2 * i + 1]);
  __syncthreads();
  const int muf = fw.mused[0] < kGradMaxM ? fw.mused[0] : kGradMaxM;
  const int mub = bw.mused[0] < kGradMaxM ? bw.mused[0] : kGradMaxM;
  const int site = tid >> 1, comp = tid & 1;
  const int g = tid / kGcRows, jr = tid % kGcRows;
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
  // staging: element e = d * kGcRows + jj of a tile is u_d at the tile's
  // row jj; thread tid holds elements tid + 256 i.  The next tile's elements
  // are loaded while the current tile is computed.
  constexpr int kPre = kGradMaxM * kGcRows / 256;
  auto fetch = [&](uint64_t base, double2 (&v)[kPre]) {
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int e = tid + 256 * i, d = e / kGcRows, jj = e % kGcRows;
      const uint64_t p = base + (uint64_t)jj;
      size_t r;
      const bool ok = d < muf && locate(p, &r);
      v[i] = !ok ? make_double2(0.0, 0.0) : (d == 0 ? psi_k[r] : Uf[(size_t)(d - 1) * stride + p]);
    }
  };
  double2 pre[kPre];
  const uint64_t step = (uint64_t)gridDim.x * kGcRows;
  if ((uint64_t)blockIdx.x * kGcRows < niter) fetch((uint64_t)blockIdx.x * kGcRows, pre);
  double acc = 0.0;
  for (uint64_t base = (uint64_t)blockIdx.x * kGcRows; base < niter; base += step) {
#pragma unroll
    for (int i = 0; i < kPre; ++i) Us[tid + 256 * i] = pre[i];
    // this thread's row and its costate values u'_c, c = g + kGcGroups k
    const uint64_t p = base + (uint64_t)jr;
    size_t r;
    const bool valid = locate(p, &r);
    double2 w[kGcCPer];
#pragma unroll
    for (int k = 0; k < kGcCPer; ++k) {
      const int c = g + kGcGroups * k;
      w[k] = (valid && c < mub) ? (c == 0 ? lam[r] : Ub[(size_t)(c - 1) * stride + p]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (base + step < niter) fetch(base + step, pre);   // in flight while this tile is computed
    double tr[kGcCPer], ti[kGcCPer];
#pragma unroll
    for (int k = 0; k < kGcCPer; ++k) tr[k] = ti[k] = 0.0;
    for (int d = 0; d < muf; ++d) {
      const double2 u = Us[d * kGcRows + jr];
#pragma unroll
      for (int k = 0; k < kGcCPer; ++k) {
        const double2 cc = C[(g + kGcGroups * k) * kGradMaxM + d];
        tr[k] += cc.x * u.x - cc.y * u.y;
        ti[k] += cc.x * u.y + cc.y * u.x;
      }
    }
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int k = 0; k < kGcCPer; ++k) {
      sr += w[k].x * tr[k] + w[k].y * ti[k];   // conj(w) t
      si += w[k].x * ti[k] - w[k].y * tr[k];
    }
    sp[g * kGcRows + jr] = make_double2(sr, si);
    __syncthreads();
    if (tid < kGcRows) {
      double2 t = sp[tid];
      for (int q = 1; q < kGcGroups; ++q) {
        t.x += sp[q * kGcRows + tid].x;
        t.y += sp[q * kGcRows + tid].y;
      }
      sbuf[tid] = t;
      sst[tid] = valid ? states[r] : (S)0;
    }
    __syncthreads();
    if (tid < kGradQ && (site < L || site == QK_MAX_L)) {
      for (int q = 0; q < kGcRows; ++q) {
        const bool on = site == QK_MAX_L || ((sst[q] >> site) & (S)1);
        const double v = comp ? sbuf[q].y : sbuf[q].x;
        acc += on ? v : 0.0;
      }
    }
    __syncthreads();   // Us, sp and sbuf are written again by the next tile
  }
  if (tid < kGradQ) part[(size_t)blockIdx.x * kGradQ + tid] = acc;
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
  qk_krylov* kb = nullptr;   // workspace of the backward steps
  double2* ck = nullptr;     // checkpoints
  double2* seg = nullptr;    // recomputed states of one segment after its checkpoint (c - 1)
  double2* cur = nullptr;    // running forward state
  double2* lam = nullptr;    // lambda_k
  double2* lamp = nullptr;   // lambda_{k+1}
  double *Ct = nullptr, *Cn = nullptr, *part = nullptr, *dA = nullptr;
  qk_status st = krylov_create(H, k->m, QK_C128, k->reorth, k->al, &kb);
  if (st != QK_OK) {
    dev_free(k->al, ubank);
    dev_free(k->al, cbank);
    dev_free(k->al, ibank);
    return st;
  }
  kb->threads = k->threads;
  kb->blocks_per_cu = k->blocks_per_cu;
  kb->blocked_wgs = k->blocked_wgs;
  kb->grid = k->grid;
  hipError_t e = dev_alloc(k->al, (void**)&ck, vbytes * (size_t)nck);
  if (e == hipSuccess && c > 1) e = dev_alloc(k->al, (void**)&seg, vbytes * (size_t)(c - 1));
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&cur, vbytes);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&lam, vbytes);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&lamp, vbytes);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&Ct, sizeof(double) * 2 * kGradMaxM * kGradMaxM);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&Cn, sizeof(double) * 2 * kGradMaxM * kGradMaxM * kGaussNodes);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&part, sizeof(double) * (size_t)G * kGradQ);
  if (e == hipSuccess) e = dev_alloc(k->al, (void**)&dA, sizeof(double) * 2 * L);
  if (e == hipSuccess) e = hipMemsetAsync(dA, 0, sizeof(double) * 2 * L, s);
  const KState fw = make_kstate(k), bw = make_kstate(kb);
  // the workspaces' vectors in the padded layout of the two-pass split: the
  // contraction walks that layout and finds each element's row in its line
  const uint32_t* lr0 = nullptr;
  const uint8_t* lnn = nullptr;
  int pe = 1;
  uint64_t niter = D;
  if (st == QK_OK && (k->d_Z != nullptr) != (kb->d_Z != nullptr)) {
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
    st = launch_krylov_step(k, cur, dt, s, true);
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
  // backward pass of the costate
  if (st == QK_OK) {
    hipLaunchKernelGGL(k_basis_vector, dim3((D + 255) / 256), dim3(256), 0, s, lam, D, (uint32_t)r0);
    chk("k_basis_vector");
  }
  for (int t = n_steps - 1; t >= 0 && st == QK_OK; --t) {
    if (t % c == c - 1 || t == n_steps - 1) {
      // entering a segment from its end: recompute its states after the checkpoint
      const int t0 = (t / c) * c;
      for (int u = t0 + 1; u <= t && st == QK_OK; ++u) {
        e = hipMemcpyAsync(state_at(u), state_at(u - 1), vbytes, hipMemcpyDeviceToDevice, s);
        chk("segment copy");
        if (st == QK_OK) st = launch_krylov_step(k, state_at(u), dt, s, true);
      }
      if (st != QK_OK) break;
    }
    // Krylov basis of psi_t: kept from the forward pass, or rebuilt from the
    // stored state (which is left unchanged)
    const double2* Uf = keep ? (const double2*)((char*)ubank + (size_t)t * ubytes) : (const double2*)k->d_U;
    const KState fwt = keep ? kstate_at(k, cbank + (size_t)t * cdoubles, ibank + 2 * (size_t)t) : fw;
    if (!keep) st = launch_krylov_step(k, state_at(t), dt, s, false);
    if (st != QK_OK) break;
    // lambda_t = exp(+iH dt) lambda_{t+1}; lamp keeps lambda_{t+1}
    e = hipMemcpyAsync(lamp, lam, vbytes, hipMemcpyDeviceToDevice, s);
    chk("costate copy");
    if (st == QK_OK) st = launch_krylov_step(kb, lam, -dt, s, true);
    if (st != QK_OK) break;
    hipLaunchKernelGGL(k_grad_nodes, dim3(kGaussNodes), dim3(64), 0, s, fwt, bw, dt, gr, Cn);
    chk("k_grad_nodes");
    if (st != QK_OK) break;
    hipLaunchKernelGGL(k_grad_coeffs, dim3(1), dim3(kGradMaxM * kGradMaxM), 0, s, fwt, bw, (const double*)Cn, Ct);
    chk("k_grad_coeffs");
    if (st != QK_OK) break;
    if (H->basis->wide)
      hipLaunchKernelGGL(k_grad_contract<uint64_t>, dim3(G), dim3(256), 0, s, (const uint64_t*)H->basis->d_states,
                         niter, L, (const double2*)state_at(t), Uf, (const double2*)lamp,
                         (const double2*)kb->d_U, (size_t)k->ustride, lr0, lnn, pe, fwt, bw, Ct, part);
    else
      hipLaunchKernelGGL(k_grad_contract<uint32_t>, dim3(G), dim3(256), 0, s, (const uint32_t*)H->basis->d_states,
                         niter, L, (const double2*)state_at(t), Uf, (const double2*)lamp,
                         (const double2*)kb->d_U, (size_t)k->ustride, lr0, lnn, pe, fwt, bw, Ct, part);
    chk("k_grad_contract");
    if (st != QK_OK) break;
    hipLaunchKernelGGL(k_grad_accum, dim3(1), dim3(kAccThreads), 0, s, part, G, L, dA);
    chk("k_grad_accum");
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
  dev_free(k->al, lam);
  dev_free(k->al, lamp);
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

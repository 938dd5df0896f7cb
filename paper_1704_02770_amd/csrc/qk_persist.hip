// Persistent step of the batched driver: one kernel launch advances every
// workspace of a qk_batch by one Krylov step (Sec. 2 "Krylov subspace
// methods"), records the survival probability of every item and advances the
// temporal autocorrelation (Sec. 4), the work of the disorder ensembles of
// Sec. 4 ("Quasidisordered systems") in a single launch that the driver
// captures into a hipGraph and replays once per step.
//
// Work queue.  A step of one workspace is a chain of passes (per Lanczos
// iteration: H-pass, [partial-sum totals], update, [totals]; then the
// projected exponential, the combination and the record).  Every pass keeps
// the grid of its plain launch as a virtual grid, and consecutive virtual
// blocks are grouped into tiles of at least kTileWork (row, column) elements,
// so that small workspaces do not pay a claim and a synchronisation for each
// of the many nearly empty blocks their plain launches are sized with.  The
// passes of all workspaces are laid out in one queue, pass index by pass
// index (workspace 0's first pass, workspace 1's first pass, ..., workspace
// 0's second pass, ...), followed by the batch-wide autocorrelation step.
// The queue is dealt to eight sub-queues, one per XCD: tile t of a pass goes
// to sub-queue t % 8, and work-group w takes its items from sub-queue w % 8
// (the XCD it runs on), so that virtual block v runs on XCD v % 8 as in the
// plain launch, whose block-to-XCD mapping keeps neighbouring blocks in one
// XCD's L2.  Work-groups claim the items of their sub-queue in order with one
// atomic counter per sub-queue; before running a tile, a work-group waits
// until the pass it depends on (the previous pass of the same workspace; for
// the autocorrelation, the record of every workspace) is complete.  Every
// pass depends only on passes that come earlier in every sub-queue, and an
// item is claimed only by a running work-group, so the tiles of the earliest
// unfinished pass have all been claimed by work-groups that can proceed:
// the launch completes whether or not all work-groups are resident at once.
// Different workspaces' passes run side by side on the chip, without a
// launch gap between the passes of one workspace.
//
// Each virtual block runs the same kernel body as the plain launch
// (qk_blocked_bodies.h, qk_step_bodies.h) with the same block index and grid
// size, so the persistent step gives bitwise the same results as the plain
// step.
//
// Completion and visibility across XCDs: when a tile is finished, every wave
// waits until its stores have reached the L2, the work-group synchronises,
// and one thread issues an agent-scope release fence (the L2 writeback that
// makes the tile's results visible to the other XCDs; one per work-group, not
// one per wave, which made the passes up to twice as long) and adds 1 to the
// pass's done counter; the tile completing the pass then issues an acquire
// fence (so that it carries every earlier tile's results) and sets the
// pass's ready flag with a release store.  Waiting work-groups poll only the ready flag (written once per
// launch, on a cache line of its own, so the polls never contend with the
// counter's atomic adds), with a growing sleep between polls; the polling
// thread then issues an agent-scope acquire fence (which invalidates the
// CU's L1 for every wave of the work-group) before the work-group
// synchronises and reads the pass's results.
//
// Counters: the claim counter, the exit counter, the done counters and the
// ready flags are reset by the last work-group to leave the launch (all
// earlier ones have stopped claiming by then), so every launch starts from
// zero without a memset node in the graph.  A work-group whose waits in one
// launch add up to more than a wall-clock bound (five seconds) sets an abort
// flag instead of waiting on: every work-group then stops claiming, the
// launch ends, and the records of that step are NaN.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "qk_blocked_bodies.h"
#include "qk_persist.h"
#include "qk_step_bodies.h"

namespace qk {

// ------------------------------------------------------------ device side
enum PassKind : int {
  PK_HBLK = 0,   // one-phase blocked H-pass (blk_body)
  PK_HBLKB,      // batched blocked H-pass (blkb_body)
  PK_HROW,       // row-form H-pass (lanczos_a_body), matrix-free rows
  PK_HCSR,       // row-form H-pass from the CSR arrays
  PK_TOTA,       // totals of the H-pass partial sums
  PK_UPD,        // update pass
  PK_TOTB,       // totals of the update-pass partial sums
  PK_EXPM,       // projected exponential, one wavefront per column
  PK_COMB,       // combination psi = V c
  PK_REC,        // |psi[r0]|^2 record
  PK_OVLP,       // overlap partial sums (general initial state)
  PK_OVLF,       // overlap total and record
  PK_AUTO,       // autocorrelation step and step counter (batch-wide)
};

struct PSeg {
  int ws;        // workspace, -1 for the batch-wide pass
  int kind;      // PassKind
  int j;         // Lanczos iteration of the H-pass / update / totals
  int vn;        // virtual grid of the pass (the plain launch's grid)
  int per;       // virtual blocks per tile
  int ntiles;    // tiles: ceil(vn / per)
  int dep0;      // first entry of the pass's dependencies in the dependency list
  int ndep;
};

// One workspace of the persistent step (device copy, written at plan time).
struct PWork {
  BlkArgs ba;                 // blocked H-pass
  ModelArgs ma;               // row-form H-pass
  HamView<uint32_t> hv;
  const uint32_t* gtab;
  const double* gfields;
  KState st;
  void* psi;
  void* U;
  const void* psi0;           // initial vector copy (records by overlap), or NULL
  double* partA;
  double* partB;
  double* totA;
  double* totB;
  double* opart;              // overlap partial sums
  uint64_t stride;            // elements per Krylov slot
  double rtol;
  int64_t r0;
  uint32_t D;
  int B, lb, m, reorth;
  int llo;                    // one-phase blocked kernel's low-bit count
  int Ga;                     // H-pass grid
  int G;                      // streaming grid (update, combination)
  int ogrid;                  // overlap grid
  int pre;                    // partial sums totalled once per pass
  int nt;                     // non-temporal streaming loads
  int item_off;
};

// Counters, one 128-byte line each: the claim counter of each XCD's queue,
// exits, abort flag, then the done counter of every pass, then the ready flag
// of every pass.
constexpr int kLine = 32;   // ints per line
constexpr int kCtrClaim = 0, kCtrExit = kNumXcd * kLine, kCtrAbort = kCtrExit + kLine, kCtrDone = kCtrAbort + kLine;
__host__ __device__ inline int ctr_done(int seg) { return kCtrDone + seg * kLine; }
__host__ __device__ inline int ctr_ready(int seg, int nseg) { return kCtrDone + (nseg + seg) * kLine; }
__host__ __device__ inline size_t ctr_ints(int nseg) { return (size_t)kCtrDone + 2 * (size_t)nseg * kLine; }
constexpr int kSegLds = 4096;         // passes whose first items a work-group keeps in LDS (its queue's)
constexpr double kTileWork = 512;     // (row, column) elements a tile covers at least
constexpr double kWaitSeconds = 5.0;  // bound on a work-group's waiting in one launch

__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Operands of pass `j` of workspace w, as the plain step computes them.
template <typename T>
struct PassOps {
  using V = typename Cx<T>::V;
  V *psi, *U, *wv;
  const V *uj, *ujm1;
  LanczosArgs la;
  const double* pB;
  int GB;
  __device__ __forceinline__ PassOps(const PWork& w, int j) {
    psi = (V*)w.psi;
    U = (V*)w.U;
    uj = j == 0 ? psi : U + (size_t)(j - 1) * w.stride;
    ujm1 = j == 0 ? nullptr : (j == 1 ? psi : U + (size_t)(j - 2) * w.stride);
    wv = U + (size_t)j * w.stride;
    la = LanczosArgs{j, w.m, w.rtol, w.reorth == 1 ? 1 : 0};
    pB = w.pre ? w.totB : w.partB;
    GB = w.pre ? 1 : w.G;
  }
};

// One tile (a run of virtual blocks) of each pass kind.
template <typename T, int LLO>
__device__ __forceinline__ void tile_hblk(const PWork& w, int j, VRange rg, unsigned char* smem) {
  const PassOps<T> o(w, j);
  blk_body<T, LLO, true, false>(rg, smem, w.ba, o.uj, o.wv, o.ujm1, w.st, o.la, o.pB, o.GB, w.partA);
}
template <typename T>
__device__ __forceinline__ void tile_hblkb(const PWork& w, int j, VRange rg, unsigned char* smem) {
  const PassOps<T> o(w, j);
  blkb_body<T, true>(rg, smem, w.ba, w.B, w.lb, o.uj, o.wv, o.ujm1, w.st, o.la, o.pB, o.GB, w.partA);
}
template <typename T, bool CSR>
__device__ __forceinline__ void tile_hrow(const PWork& w, int j, VRange rg, unsigned char* smem) {
  const PassOps<T> o(w, j);
  lanczos_a_body<T, CSR, uint32_t>(rg, *reinterpret_cast<LanczosAShared<uint32_t>*>(smem), o.uj, o.ujm1, o.wv, w.ma,
                                   w.hv, w.gtab, w.gfields, w.st, o.la, o.pB, o.GB, w.partA);
}
template <typename T, bool NT>
__device__ __forceinline__ void tile_upd(const PWork& w, int j, VRange rg, unsigned char* smem) {
  const PassOps<T> o(w, j);
  const double* pA = w.pre ? w.totA : w.partA;
  const int GA = w.pre ? 1 : w.Ga;
  lanczos_b_body<T, NT>(rg, *reinterpret_cast<LanczosBShared*>(smem), o.uj, o.ujm1, o.wv, w.D, w.B, w.st, o.la, pA,
                        GA, w.partB, j + 1 < w.m ? 1 : 0);
}
// Columns 4 v .. 4 v + 3, one wavefront each.
__device__ __forceinline__ void tile_expm(const PWork& w, VRange rg, double dt) {
  const double* pB = w.pre ? w.totB : w.partB;
  const int GB = w.pre ? 1 : w.G;
  for (uint32_t v = rg.v0; v < rg.v1; ++v) {
    const int b = (int)v * (kMaxBlock / 64) + (int)(threadIdx.x / 64);
    if (b < w.B) small_expm_wave(b, (int)(threadIdx.x % 64), w.st, w.m, w.B, dt, nullptr, pB, GB);
  }
}
template <typename T>
__device__ __forceinline__ void tile_record(const PWork& w, VRange rg, int kind, unsigned char* smem,
                                            const PArgs& pa) {
  using V = typename Cx<T>::V;
  if (kind == PK_REC) {
    record_body<T>((const V*)w.psi, (uint32_t)w.r0, w.B, pa.P, pa.counter, w.item_off, pa.items);
  } else if (kind == PK_OVLP) {
    overlap_partial_body<T>(rg, reinterpret_cast<double*>(smem), (const V*)w.psi0, (const V*)w.psi, w.D, w.B,
                            w.opart);
  } else {
    double* red = reinterpret_cast<double*>(smem);
    overlap_final_body(red, red + kMaxBlock, w.opart, w.ogrid, w.B, pa.P, pa.counter, w.item_off, pa.items);
  }
}

// Tile `tile` of pass sg: its virtual blocks run as one range (one set-up).
template <typename T>
__device__ __forceinline__ void run_tile(const PSeg& sg, int tile, const PWork& w, const PArgs& pa,
                                         unsigned char* smem) {
  // every branch below is uniform across the work-group; readfirstlane tells
  // the compiler so, which keeps the branches apart (a branch it must treat as
  // divergent is linearised, and the kernel then holds the registers of all
  // its sides at once)
  const int vn = __builtin_amdgcn_readfirstlane(sg.vn), per = __builtin_amdgcn_readfirstlane(sg.per);
  const int v1 = (tile + 1) * per < vn ? (tile + 1) * per : vn;
  const VRange rg{(uint32_t)(tile * per), (uint32_t)v1, (uint32_t)vn};
  const int j = __builtin_amdgcn_readfirstlane(sg.j);
  const int llo = __builtin_amdgcn_readfirstlane(w.llo);
  const int nt = __builtin_amdgcn_readfirstlane(w.nt);
  switch (__builtin_amdgcn_readfirstlane(sg.kind)) {
    case PK_HBLK:
      if (llo == 9) tile_hblk<T, 9>(w, j, rg, smem);
      else if (llo == 10) tile_hblk<T, 10>(w, j, rg, smem);
      else tile_hblk<T, 11>(w, j, rg, smem);
      break;
    case PK_HBLKB: tile_hblkb<T>(w, j, rg, smem); break;
    case PK_HROW: tile_hrow<T, false>(w, j, rg, smem); break;
    case PK_HCSR: tile_hrow<T, true>(w, j, rg, smem); break;
    case PK_TOTA: partials_total_body(rg, reinterpret_cast<double*>(smem), w.partA, w.Ga, kQA * w.B, w.totA); break;
    case PK_UPD:
      if (nt) tile_upd<T, true>(w, j, rg, smem);
      else tile_upd<T, false>(w, j, rg, smem);
      break;
    case PK_TOTB: partials_total_body(rg, reinterpret_cast<double*>(smem), w.partB, w.G, w.B, w.totB); break;
    case PK_EXPM: tile_expm(w, rg, pa.dt); break;
    case PK_COMB:
      // one form for every workspace: the packing, the coefficient staging
      // and the non-temporal loads of the plain launch's variants change how
      // elements are fetched, not how each is summed, so this gives the same
      // bits with one register allocation
      combine_body<T, 1, false, false>(rg, reinterpret_cast<double2*>(smem), (typename Cx<T>::V*)w.psi,
                                       (const typename Cx<T>::V*)w.U, w.D, w.B, w.m, w.st);
      break;
    case PK_REC:
    case PK_OVLP:
    case PK_OVLF: tile_record<T>(w, rg, sg.kind, smem, pa); break;
    default: break;
  }
}

// Four work-groups of 256 threads per CU: the registers of the kernel are
// those of its largest body (capped at 128, a few bytes of spill in
// complex128), and the bodies' LDS (at most about 32 KB) allows four.
template <typename T>
__global__ void __launch_bounds__(kMaxBlock, 4) k_persist(PArgs pa) {
  extern __shared__ unsigned char smem[];
  __shared__ int s_seg, s_tile, s_stop;
  int* ctr = pa.ctr;
  const int xq = (int)(blockIdx.x % kNumXcd);   // this work-group's sub-queue
  const int* xfirst = pa.xfirst + xq;           // stride kNumXcd
  // first item of every pass in this sub-queue, after the bodies' LDS (when
  // it fits), for the search of the pass holding a claimed item
  int* sfirst = pa.nseg <= kSegLds ? reinterpret_cast<int*>(smem + pa.body_smem) : nullptr;
  if (sfirst)
    for (int i = threadIdx.x; i < pa.nseg; i += blockDim.x) sfirst[i] = xfirst[(size_t)i * kNumXcd];
  __syncthreads();
  long long waited = 0;   // wall-clock ticks this work-group has spent waiting (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      int seg = -1, tile = 0, stop = 0;
      if (ld_agent(ctr + kCtrAbort) != 0) {
        stop = 1;   // a wait gave up: claim nothing more
      } else {
        const int item = atomicAdd(ctr + kCtrClaim + xq * kLine, 1);
        if (item >= pa.xitems[xq]) {
          stop = 1;
        } else {
          // the pass holding this item: the last pass whose first item in
          // this sub-queue is <= item (passes with no tile here share their
          // first item with the next pass, so the last one is the holder)
          int lo = 0, hi = pa.nseg - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if ((sfirst ? sfirst[mid] : xfirst[(size_t)mid * kNumXcd]) <= item) lo = mid;
            else hi = mid - 1;
          }
          seg = lo;
          const PSeg sg = pa.seg[lo];
          tile = xq + kNumXcd * (item - (sfirst ? sfirst[lo] : xfirst[(size_t)lo * kNumXcd]));
          // wait for the passes this one depends on: poll their ready flags,
          // sleeping 64 * ns cycles between polls, ns doubling up to 64
          for (int d = 0; d < sg.ndep && !stop; ++d) {
            const int* flag = ctr + ctr_ready(pa.deps[sg.dep0 + d], pa.nseg);
            if (ld_agent(flag) != 0) continue;
            const long long t0 = wall_clock64();
            int ns = 1;
            while (ld_agent(flag) == 0) {
              __builtin_amdgcn_s_sleep(1);
              for (int r = 1; r < ns; ++r) __builtin_amdgcn_s_sleep(1);
              ns = ns < 64 ? 2 * ns : 64;
              const long long dt = wall_clock64() - t0;
              if (waited + dt > pa.wait_ticks || ld_agent(ctr + kCtrAbort) != 0) {
                __hip_atomic_store(ctr + kCtrAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                stop = 1;
                break;
              }
            }
            waited += wall_clock64() - t0;
          }
          if (stop) {
            // this step's records are not valid
            for (int i = 0; i < pa.items; ++i) pa.P[(size_t)(*pa.counter) * pa.items + i] = NAN;
          }
        }
      }
      s_seg = seg;
      s_tile = tile;
      s_stop = stop;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the results of the passes waited for
    }
    __syncthreads();
    // uniform across the work-group: keep them (and every address derived
    // from them) in scalar registers
    const int seg = __builtin_amdgcn_readfirstlane(s_seg), tile = __builtin_amdgcn_readfirstlane(s_tile);
    const int stop = __builtin_amdgcn_readfirstlane(s_stop);
    if (stop) break;
    const PSeg sg = pa.seg[seg];
    if (sg.kind == PK_AUTO) {
      autocorr_body(pa.P, pa.counter, pa.items, pa.dt, pa.state, pa.C);
      __syncthreads();
      if (threadIdx.x == 0) *pa.counter = *pa.counter + 1;
    } else {
      // the workspace arguments never change during a launch: read them
      // through the constant address space (scalar loads, reloaded where
      // needed instead of held in registers), as a plain kernel reads its
      // arguments
      const __attribute__((address_space(4))) PWork* cw =
          (const __attribute__((address_space(4))) PWork*)(uintptr_t)pa.ws;
      run_tile<T>(sg, tile, (const PWork&)cw[sg.ws], pa, smem);
    }
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const int done = __hip_atomic_fetch_add(ctr + ctr_done(seg), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (done == sg.ntiles - 1) {
        // the pass's last tile: its acquire fence pairs with every other
        // tile's release fence through the counter, and the release store of
        // the flag passes all their results on to the waiting work-groups
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(ctr + ctr_ready(seg, pa.nseg), 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  // the last work-group to leave resets the counters for the next launch
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int e = __hip_atomic_fetch_add(ctr + kCtrExit, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (e == (int)gridDim.x - 1) {
      for (int i = 0; i < pa.nseg; ++i) {
        ctr[ctr_done(i)] = 0;
        ctr[ctr_ready(i, pa.nseg)] = 0;
      }
      for (int x = 0; x < kNumXcd; ++x) ctr[kCtrClaim + x * kLine] = 0;
      ctr[kCtrExit] = 0;
    }
  }
}

// -------------------------------------------------------------- host side
struct PersistPlan {
  qk_allocator al;
  int dtype = 0;
  int nseg = 0, grid = 0;
  int xitems[kNumXcd] = {0};
  size_t body_smem = 0;   // LDS of the largest kernel body
  size_t smem = 0;        // dynamic LDS of the launch: bodies, then the pass index
  long long wait_ticks = 0;   // wall-clock ticks of kWaitSeconds
  PWork* d_ws = nullptr;
  PSeg* d_seg = nullptr;
  int* d_deps = nullptr;
  int* d_xfirst = nullptr;
  int* d_ctr = nullptr;
};

void persist_free(PersistPlan* p) {
  if (!p) return;
  dev_free(p->al, p->d_ws);
  dev_free(p->al, p->d_seg);
  dev_free(p->al, p->d_deps);
  dev_free(p->al, p->d_xfirst);
  dev_free(p->al, p->d_ctr);
  delete p;
}

static qk_status unsupported(const char* why) {
  set_error(std::string("persistent batched step: ") + why);
  return QK_EUNSUPPORTED;
}

qk_status persist_plan(const PersistInput& in, PersistPlan** out) {
  const int n = (int)in.ks.size();
  if (n == 0) return unsupported("no workspaces");
  const int dtype = in.ks[0]->dtype;
  std::vector<PWork> ws(n);
  size_t smem = 256 * sizeof(double) + 2 * QK_MAX_BATCH * sizeof(double);   // totals, overlap final
  if (sizeof(LanczosBShared) > smem) smem = sizeof(LanczosBShared);
  if (2 * kMaxBlock * sizeof(double) > smem) smem = 2 * kMaxBlock * sizeof(double);
  for (int i = 0; i < n; ++i) {
    const qk_krylov* k = in.ks[i];
    const qk_ham* H = k->H;
    if (k->dtype != dtype) return unsupported("all workspaces must share one dtype");
    if (H->basis->wide) return unsupported("chains longer than 32 sites");
    if (k->d_Z) return unsupported("the two-pass split layout");
    if (k->reorth == 2) return unsupported("full reorthogonalisation");
    if (krylov_threads(k) != kMaxBlock || block_threads(k->batch) != kMaxBlock)
      return unsupported("row-streaming kernels with fewer than 256 threads per block");
    PWork& w = ws[i];
    std::memset(&w, 0, sizeof(w));
    const int B = k->batch;
    const size_t vb = dtype == QK_C128 ? 16 : 8;
    w.B = B;
    w.m = k->m;
    w.reorth = k->reorth;
    w.D = (uint32_t)H->basis->D;
    w.st = make_kstate(k);
    w.psi = in.psi[i];
    w.U = k->d_U;
    w.stride = k->ustride;
    w.partA = k->d_partA;
    w.partB = k->d_partB;
    w.totA = k->d_ptot;
    w.totB = k->d_ptot + (size_t)kQA * B;
    w.rtol = dtype == QK_C128 ? 1e-12 : 1e-5;
    w.G = k->grid;
    w.pre = B >= kPreReduceBatch;
    w.nt = (size_t)k->ustride * vb >= kNtBytes;
    w.r0 = in.r0[i];
    w.psi0 = in.psi0[i];
    w.opart = in.part[i];
    w.ogrid = in.ogrid[i];
    w.item_off = in.item_off[i];
    if (blocked_usable(H, dtype)) {
      BlkPlan bp;
      qk_status st = blocked_lanczos_plan(H, dtype, k->blocked_wgs, &bp);
      if (st != QK_OK) return st;
      w.ba = bp.ba;
      w.Ga = bp.G;
      w.lb = bp.lb;
      w.llo = bp.llo;
      if (bp.smem > smem) smem = bp.smem;
    } else {
      w.ma = model_args(H);
      w.hv = ham_view32(H);
      w.gtab = H->basis->d_binom;
      w.gfields = H->d_fields;
      w.Ga = k->grid;
      if (sizeof(LanczosAShared<uint32_t>) > smem) smem = sizeof(LanczosAShared<uint32_t>);
    }
    if (sizeof(double2) * (size_t)k->m * B > smem) smem = sizeof(double2) * (size_t)k->m * B;   // combination
  }
  // passes of each workspace in chain order: kind, iteration, virtual grid,
  // (row, column) elements per virtual block
  struct Pass {
    int kind, j, vn;
    double work;
  };
  std::vector<std::vector<Pass>> chain(n);
  for (int i = 0; i < n; ++i) {
    const qk_krylov* k = in.ks[i];
    const PWork& w = ws[i];
    const double elems = (double)w.D * w.B;
    const int hk = blocked_usable(k->H, dtype) ? (k->batch > 1 ? PK_HBLKB : PK_HBLK)
                                               : (k->H->p.mode == QK_CSR ? PK_HCSR : PK_HROW);
    for (int j = 0; j < w.m; ++j) {
      chain[i].push_back({hk, j, w.Ga, elems / w.Ga});
      if (w.pre) chain[i].push_back({PK_TOTA, j, (kQA * w.B + kTotCols - 1) / kTotCols, kTileWork});
      chain[i].push_back({PK_UPD, j, w.G, elems / w.G});
      if (w.pre) chain[i].push_back({PK_TOTB, j, (w.B + kTotCols - 1) / kTotCols, kTileWork});
    }
    chain[i].push_back({PK_EXPM, 0, (w.B + kMaxBlock / 64 - 1) / (kMaxBlock / 64), kTileWork});
    chain[i].push_back({PK_COMB, 0, w.G, elems / w.G});
    if (w.r0 >= 0) {
      chain[i].push_back({PK_REC, 0, 1, kTileWork});
    } else {
      chain[i].push_back({PK_OVLP, 0, w.ogrid, elems / w.ogrid});
      chain[i].push_back({PK_OVLF, 0, 1, kTileWork});
    }
  }
  // queue: pass index by pass index across workspaces, then the autocorrelation
  std::vector<PSeg> segs;
  std::vector<int> deps;
  std::vector<int> last(n, -1);
  size_t longest = 0;
  for (int i = 0; i < n; ++i) longest = chain[i].size() > longest ? chain[i].size() : longest;
  for (size_t p = 0; p < longest; ++p) {
    for (int i = 0; i < n; ++i) {
      if (p >= chain[i].size()) continue;
      const Pass& ps = chain[i][p];
      // virtual blocks per tile: enough for kTileWork elements
      int per = ps.work >= kTileWork ? 1 : (int)std::ceil(kTileWork / (ps.work > 1.0 ? ps.work : 1.0));
      if (per > ps.vn) per = ps.vn;
      const int ntiles = (ps.vn + per - 1) / per;
      PSeg sg{i, ps.kind, ps.j, ps.vn, per, ntiles, (int)deps.size(), 0};
      if (last[i] >= 0) {
        deps.push_back(last[i]);
        sg.ndep = 1;
      }
      last[i] = (int)segs.size();
      segs.push_back(sg);
    }
  }
  {
    PSeg sg{-1, PK_AUTO, 0, 1, 1, 1, (int)deps.size(), n};
    for (int i = 0; i < n; ++i) deps.push_back(last[i]);
    segs.push_back(sg);
  }
  // the XCD sub-queues: tile t of a pass goes to sub-queue t % 8
  std::vector<int> xfirst(segs.size() * kNumXcd);
  int xitems[kNumXcd] = {0};
  for (size_t g = 0; g < segs.size(); ++g)
    for (int x = 0; x < kNumXcd; ++x) {
      xfirst[g * kNumXcd + x] = xitems[x];
      xitems[x] += segs[g].ntiles > x ? (segs[g].ntiles - x + kNumXcd - 1) / kNumXcd : 0;
    }
  PersistPlan* pl = new (std::nothrow) PersistPlan;
  if (!pl) return QK_ENOMEM;
  pl->al = in.al;
  pl->dtype = dtype;
  pl->nseg = (int)segs.size();
  for (int x = 0; x < kNumXcd; ++x) pl->xitems[x] = xitems[x];
  pl->body_smem = (smem + 15) & ~(size_t)15;
  pl->smem = pl->body_smem + (segs.size() <= (size_t)kSegLds ? sizeof(int) * segs.size() : 0);
  auto kern = dtype == QK_C128 ? k_persist<double> : k_persist<float>;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kMaxBlock, pl->smem) != hipSuccess || occ < 1) occ = 1;
  pl->grid = ((qk_num_cus() * occ + kNumXcd - 1) / kNumXcd) * kNumXcd;   // every sub-queue has work-groups
  hipError_t e = dev_alloc(pl->al, (void**)&pl->d_ws, sizeof(PWork) * ws.size());
  if (e == hipSuccess) e = dev_alloc(pl->al, (void**)&pl->d_seg, sizeof(PSeg) * segs.size());
  if (e == hipSuccess) e = dev_alloc(pl->al, (void**)&pl->d_deps, sizeof(int) * (deps.empty() ? 1 : deps.size()));
  if (e == hipSuccess) e = dev_alloc(pl->al, (void**)&pl->d_xfirst, sizeof(int) * xfirst.size());
  if (e == hipSuccess) e = dev_alloc(pl->al, (void**)&pl->d_ctr, sizeof(int) * ctr_ints(pl->nseg));
  if (e == hipSuccess) e = hipMemcpy(pl->d_ws, ws.data(), sizeof(PWork) * ws.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pl->d_seg, segs.data(), sizeof(PSeg) * segs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !deps.empty())
    e = hipMemcpy(pl->d_deps, deps.data(), sizeof(int) * deps.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pl->d_xfirst, xfirst.data(), sizeof(int) * xfirst.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(pl->d_ctr, 0, sizeof(int) * ctr_ints(pl->nseg));
  int khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, in.ks[0]->device);
  pl->wait_ticks = (long long)(kWaitSeconds * 1000.0 * (khz > 0 ? khz : 100000));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    persist_free(pl);
    return hip_fail(e, "persistent step plan");
  }
  *out = pl;
  return QK_OK;
}

qk_status persist_launch(const PersistPlan* pl, double dt, double* P, double* C, int* counter, double* state,
                         int items, hipStream_t s) {
  PArgs pa;
  pa.ws = pl->d_ws;
  pa.seg = pl->d_seg;
  pa.deps = pl->d_deps;
  pa.nseg = pl->nseg;
  pa.xfirst = pl->d_xfirst;
  for (int x = 0; x < kNumXcd; ++x) pa.xitems[x] = pl->xitems[x];
  pa.ctr = pl->d_ctr;
  pa.P = P;
  pa.C = C;
  pa.dt = dt;
  pa.counter = counter;
  pa.state = state;
  pa.items = items;
  pa.body_smem = pl->body_smem;
  pa.wait_ticks = pl->wait_ticks;
  if (pl->dtype == QK_C128)
    hipLaunchKernelGGL(k_persist<double>, dim3(pl->grid), dim3(kMaxBlock), pl->smem, s, pa);
  else
    hipLaunchKernelGGL(k_persist<float>, dim3(pl->grid), dim3(kMaxBlock), pl->smem, s, pa);
  QK_HIP(hipGetLastError());
  return QK_OK;
}

int persist_grid(const PersistPlan* pl) { return pl ? pl->grid : 0; }

}  // namespace qk

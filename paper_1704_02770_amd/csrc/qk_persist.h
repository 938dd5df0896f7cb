// Persistent step of the batched driver (qk_persist.hip): host interface.
#pragma once

#include <vector>

#include "qk_internal.h"

namespace qk {

struct PWork;
struct PSeg;
struct PersistPlan;

// Kernel arguments of one persistent step.
struct PArgs {
  const PWork* ws;     // [workspaces]
  const PSeg* seg;     // [nseg] passes in queue order
  const int* deps;     // dependency list (pass indices)
  const int* xfirst;   // [nseg][8]: first item of each pass in each XCD's queue
  int nseg;
  int xitems[8];       // items in each XCD's queue
  int* ctr;            // claim, exits, abort flag, done counter per pass
  double* P;           // records P[step][items]
  double* C;           // autocorrelation records, or NULL
  double dt;
  int* counter;        // the driver's step counter
  double* state;       // autocorrelation state
  int items;
  size_t body_smem;    // dynamic LDS used by the kernel bodies (the pass index follows)
  long long wait_ticks;   // bound on a work-group's waiting in one launch (wall-clock ticks)
};

// What the plan needs of a qk_batch.
struct PersistInput {
  qk_allocator al;
  std::vector<qk_krylov*> ks;
  std::vector<void*> psi;
  std::vector<int64_t> r0;
  std::vector<const void*> psi0;
  std::vector<double*> part;
  std::vector<int> ogrid;
  std::vector<int> item_off;
};

// Builds the work queue and the device copies of every workspace's
// arguments (QK_EUNSUPPORTED for workspaces the persistent step does not
// cover: mixed dtypes, chains above 32 sites, the split layout, full
// reorthogonalisation, row kernels with fewer than 256 threads per block).
qk_status persist_plan(const PersistInput& in, PersistPlan** out);
void persist_free(PersistPlan* p);
// One step of every workspace in one launch on s.
qk_status persist_launch(const PersistPlan* p, double dt, double* P, double* C, int* counter, double* state,
                         int items, hipStream_t s);
int persist_grid(const PersistPlan* p);

}  // namespace qk

// Host-side plan of the batched engine, shared by the batching form
// (batch.hip) and the request server (server.hip).
#pragma once

#include <vector>

#include "kde_internal.hpp"

namespace kde {

struct BatchPlan {
  int prec = KDE_F64;
  int B = 0;
  double alpha = 0.5;
  std::vector<double> kappas;
  std::vector<kde_batch_set> sets;  // caller order
  std::vector<int> order;           // cost order (largest CV first) -> caller index
  int max_M = 0, max_cells = 1;
  int64_t max_n = 0;
  // pass-size buckets over the cost order: sets [bucket_begin[k], bucket_begin[k+1]) use bucket_bc[k]
  std::vector<int> bucket_begin, bucket_bc;
  size_t ws_need = 0;
  // Launch shape of the phase kernels: true, about as many workgroups as
  // the device keeps resident, each looping over units (one stream owns the
  // device); false, one workgroup per unit, so that kernels of other
  // streams get compute units as workgroups retire (a server's slots).
  bool resident_grids = true;
};

// A captured graph of a plan bound to one workspace.
struct kde_batch_graph {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    exec = nullptr;
    graph = nullptr;
    cap = nullptr;
  }
  ~kde_batch_graph() { reset(); }
};

// Validate and plan (host only).
kde_status batch_plan_make(const kde_batch_set* sets_h, int nsets, int prec, int B, const double* kappas_h,
                           double alpha, BatchPlan& out);
// Bytes of pinned host staging batch_plan_enqueue needs.
size_t batch_staging_bytes(const BatchPlan& b);
// Enqueue the whole plan on `s` without a graph: the descriptors go through
// `staging_h` (pinned host memory of batch_staging_bytes, which must stay
// untouched until the work has completed) by asynchronous copies, then the
// phase kernels are launched. `ws` holds plan.ws_need bytes.
// The sets' numeric status words follow the descriptors in the staging:
// the enqueue ends with their copy to the host, so once the work has
// completed, batch_staged_status(b, staging_h)[k] is set k's word (caller
// order).
kde_status batch_plan_enqueue(const BatchPlan& b, void* ws, hipStream_t s, void* staging_h);
const uint32_t* batch_staged_status(const BatchPlan& b, const void* staging_h);
// Device address of the sets' status words inside workspace `ws`.
uint32_t* batch_status_words(const BatchPlan& b, void* ws);

}  // namespace kde

// ccm_context.h -- the context object behind the opaque ccm_ctx handle.
// Internal to libccm.
#pragma once
#include "ccm_host.h"

namespace ccmh {
// ---------------------------------------------------------------------------
// execution state of one plan
// ---------------------------------------------------------------------------

struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
};

struct Exec {
  Plan plan;
  DevBuf d_ingest, d_embed, d_sample, d_gather, d_rz, d_items, d_plain_items;
  DevBuf d_s64, d_s32, d_emb, d_lib, d_pts, d_pj, d_partial, d_out, d_counter;
  DevBuf d_iota, d_keys, d_keys_out, d_order, d_segoff, d_sort_temp, d_qord, d_start, d_self;
  DevBuf d_orders;
  DevBuf d_tt;       // causal matrix: targets time-major [N][target_stride(M)]
  DevBuf d_tables, d_table;   // distance indexing table jobs and rows
  DevBuf d_nested, d_scratch, d_segs, d_rz_fin;   // nested libraries
  std::vector<int64_t> plain_first;   // per realization: first plain item
  hipGraphExec_t graph = nullptr;
  ~Exec() {
    if (graph) (void)hipGraphExecDestroy(graph);
  }
};

}  // namespace ccmh

struct ccm_ctx {
  int device = 0;
  int num_cus = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::string err;
  bool profiling = false;
  std::vector<ccmh::EvPair> ev_pending, ev_free;
  ccm_profile prof{};
  std::unique_ptr<ccmh::Exec> exec;   // the most recent plan
};

namespace ccmh {

// Run f under the context's lock with HIP errors and exceptions turned into
// status codes (no exception crosses the C ABI).
template <class F>
ccm_status guarded(ccm_ctx* c, F&& f) {
  if (!c) return CCM_E_INVAL;
  std::lock_guard<std::mutex> lock(c->mu);
  c->err.clear();
  try {
    HIPCHK(hipSetDevice(c->device));
    f();
    return CCM_OK;
  } catch (const Fail& e) {
    c->err = e.what;
    return e.status;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return CCM_E_NOMEM;
  } catch (...) {
    c->err = "unexpected error";
    return CCM_E_DEVICE;
  }
}

}  // namespace ccmh

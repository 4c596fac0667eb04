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

// Device addresses of one plan's buffers: an Exec's own allocations, or
// ranges of the static workspace of the no-allocation entry point.
struct PlanBuffers {
  IngestJob* ingest = nullptr;
  EmbedJob* embed = nullptr;
  SampleJob* sample = nullptr;
  GatherJob* gather = nullptr;
  Realization* rz = nullptr;
  Item* items = nullptr;
  Item* plain_items = nullptr;       // CCM_FLAG_PLAIN: each realization's items
  OrderJob* orders = nullptr;
  int32_t* segoff = nullptr;
  double* s64 = nullptr;
  float* s32 = nullptr;
  int32_t* iota = nullptr;
  uint32_t* keys = nullptr;
  uint32_t* keys_out = nullptr;
  int32_t* order = nullptr;
  void* sort_temp = nullptr;
  int32_t* qord = nullptr;
  int32_t* start = nullptr;
  float* emb = nullptr;
  int32_t* lib = nullptr;
  float* pts = nullptr;
  int32_t* pj = nullptr;
  void* partial = nullptr;
  double* out = nullptr;
  int* counter = nullptr;            // one per launch (persistent grids)
  int32_t* self = nullptr;           // causal matrix
  double* tt = nullptr;
  TableJob* tables = nullptr;        // distance indexing tables
  int32_t* table = nullptr;
  NestedJob* nested = nullptr;       // nested libraries
  int32_t* shuffle = nullptr;
  int32_t* segs = nullptr;
  Realization* rz_fin = nullptr;
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
  PlanBuffers buf;
  hipGraphExec_t graph = nullptr;
  ~Exec() {
    if (graph) (void)hipGraphExecDestroy(graph);
  }
};

}  // namespace ccmh

struct ccm_ctx {
  int device = 0;
  int num_cus = 0;
  uint64_t wave_limit = 0;    // see ccm_set_wave_limit
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::string err;
  bool profiling = false;
  std::vector<ccmh::EvPair> ev_pending, ev_free;
  ccm_profile prof{};
  std::unique_ptr<ccmh::Exec> exec;   // the most recent plan
  // pinned staging of the host-array forms' series and results (one
  // buffer, grown as needed; calls on a context are serialised)
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
};

namespace ccmh {

// Queue every launch of plan p on stream st (buffers b; plain_first: each
// realization's first item in b.plain_items, for CCM_FLAG_PLAIN).  With
// evs set, each cross-map launch is bracketed by a pair of HIP events
// (taken from the context's pool), appended to *evs.
void enqueue_plan(ccm_ctx* c, const Plan& p, const PlanBuffers& b,
                  const std::vector<int64_t>& plain_first, hipStream_t st,
                  std::vector<EvPair>* evs);

// The static workspace of the no-allocation entry point on the current
// device: set up once per device (at context creation); false, with a
// message, if the device has none.
bool noalloc_setup(int device, std::string* err);

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

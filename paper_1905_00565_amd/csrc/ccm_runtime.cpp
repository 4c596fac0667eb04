// ccm_runtime.cpp -- host runtime of libccm: device state of a plan, HIP
// graph capture and replay, profiling, and the C ABI declared in
// include/ccm.h (the server is in ccm_server.cpp).
//
// A call is planned once per distinct shape (series length, E and tau grid,
// L list, r, seed, options).  The plan's descriptors and buffers live on the
// device inside an Exec; the launches of a plan are captured into a HIP graph
// and replayed on later calls of the same shape.  Inputs are copied into the
// Exec's own series buffer (host-to-device, or device-to-device for the
// device-pointer forms) and results copied out, so the graph never refers to
// caller memory.
#include "ccm_host.h"
#include "ccm_context.h"
#include "ccm_copy.h"

#include <cstring>
#include <initializer_list>

using namespace ccmh;

namespace {

EvPair take_events(ccm_ctx* c) {
  if (!c->ev_free.empty()) {
    EvPair e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  EvPair e;
  HIPCHK(hipEventCreate(&e.a));
  HIPCHK(hipEventCreate(&e.b));
  return e;
}

void drain_events(ccm_ctx* c) {
  for (EvPair& e : c->ev_pending) {
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    c->prof.kernel_ms += ms;
    c->prof.launches += 1;
    c->ev_free.push_back(e);
  }
  c->ev_pending.clear();
}

// Device buffers and descriptors for a plan (reused when the shape repeats).
Exec* prepare(ccm_ctx* c, const Spec& s) {
  if (c->exec && c->exec->plan.spec == s) return c->exec.get();
  if (c->exec) {
    // work queued earlier on any stream may still read the old buffers
    HIPCHK(hipDeviceSynchronize());
    c->exec.reset();   // free the previous plan's memory first
  }
  auto ex = std::make_unique<Exec>();
  ex->plan = s.M > 0 ? make_plan_matrix(s) : make_plan(s);
  Plan& p = ex->plan;
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  if (p.device_bytes > free_b)
    fail(CCM_E_NOMEM, "plan needs " + std::to_string(p.device_bytes) + " device bytes, " +
                          std::to_string(free_b) + " free");
  upload(ex->d_ingest, p.ingest);
  upload(ex->d_embed, p.embed);
  upload(ex->d_sample, p.sample);
  upload(ex->d_gather, p.gather);
  upload(ex->d_rz, p.rz);
  upload(ex->d_items, p.items);
  if (s.flags & CCM_FLAG_PLAIN) {
    std::vector<Item> pi;
    ex->plain_first.resize(p.rz.size());
    for (size_t r = 0; r < p.rz.size(); ++r) {
      ex->plain_first[r] = (int64_t)pi.size();
      for (int t = 0; t < p.rz[r].n_tiles; ++t) pi.push_back({(int32_t)r, t});
    }
    upload(ex->d_plain_items, pi);
  }
  upload(ex->d_segoff, p.seg_off);
  upload(ex->d_orders, p.orders);
  if (!p.tables.empty()) {
    upload(ex->d_tables, p.tables);
    ex->d_table.ensure(p.n_table * 4);
  }
  if (!p.nested.empty()) {
    upload(ex->d_nested, p.nested);
    ex->d_scratch.ensure(p.n_scratch * 4);
    upload(ex->d_segs, p.segs);
  }
  if (!p.rz_fin.empty()) upload(ex->d_rz_fin, p.rz_fin);
  ex->d_s64.ensure(p.n64 * 8);
  ex->d_s32.ensure(p.n32 * 4);
  ex->d_iota.ensure(p.n_ord * 4);
  ex->d_keys.ensure(p.n_ord * 4);
  ex->d_keys_out.ensure(p.n_ord * 4);
  ex->d_order.ensure(p.n_ord * 4);
  ex->d_sort_temp.ensure(p.sort_temp);
  ex->d_qord.ensure(p.n_qord * 4);
  ex->d_start.ensure(p.n_slots * 4 * kWaves);
  ex->d_emb.ensure(p.n_emb * 4);
  ex->d_lib.ensure(p.n_lib * 4);
  ex->d_pts.ensure(p.n_pts * 4);
  ex->d_pj.ensure(p.n_pj * 4);
  if (s.M > 0) {
    upload(ex->d_self, p.self_of);
    ex->d_tt.ensure((size_t)s.N * target_stride(s.M) * 8);
    ex->d_partial.ensure((size_t)p.n_slots * s.M * multi_sums_bytes());
  } else {
    ex->d_partial.ensure(p.n_slots * sizeof(Moments));
  }
  ex->d_out.ensure(p.n_out * 8);
  ex->d_counter.ensure(std::max<size_t>(64, p.launches.size()) * sizeof(int));
  PlanBuffers& b = ex->buf;
  b.ingest = ex->d_ingest.as<IngestJob>();
  b.embed = ex->d_embed.as<EmbedJob>();
  b.sample = ex->d_sample.as<SampleJob>();
  b.gather = ex->d_gather.as<GatherJob>();
  b.rz = ex->d_rz.as<Realization>();
  b.items = ex->d_items.as<Item>();
  b.plain_items = ex->d_plain_items.as<Item>();
  b.orders = ex->d_orders.as<OrderJob>();
  b.segoff = ex->d_segoff.as<int32_t>();
  b.s64 = ex->d_s64.as<double>();
  b.s32 = ex->d_s32.as<float>();
  b.iota = ex->d_iota.as<int32_t>();
  b.keys = ex->d_keys.as<uint32_t>();
  b.keys_out = ex->d_keys_out.as<uint32_t>();
  b.order = ex->d_order.as<int32_t>();
  b.sort_temp = ex->d_sort_temp.p;
  b.qord = ex->d_qord.as<int32_t>();
  b.start = ex->d_start.as<int32_t>();
  b.emb = ex->d_emb.as<float>();
  b.lib = ex->d_lib.as<int32_t>();
  b.pts = ex->d_pts.as<float>();
  b.pj = ex->d_pj.as<int32_t>();
  b.partial = ex->d_partial.p;
  b.out = ex->d_out.as<double>();
  b.counter = ex->d_counter.as<int>();
  b.self = ex->d_self.as<int32_t>();
  b.tt = ex->d_tt.as<double>();
  b.tables = ex->d_tables.as<TableJob>();
  b.table = ex->d_table.as<int32_t>();
  b.nested = ex->d_nested.as<NestedJob>();
  b.shuffle = ex->d_scratch.as<int32_t>();
  b.segs = ex->d_segs.as<int32_t>();
  b.rz_fin = ex->d_rz_fin.as<Realization>();
  c->exec = std::move(ex);
  return c->exec.get();
}

int persistent_grid(ccm_ctx* c, int n_items) {
  // a few resident workgroups per CU; the queue balances the rest
  const int g = std::max(1, c->num_cus) * 8;
  return std::min(g, n_items);
}

// One cross-map launch over items [first, first + n) of b.items (or of
// b.plain_items), E's kernel variant for the plan's form.
void launch_items(ccm_ctx* c, const Plan& p, const PlanBuffers& b, const Item* items, int n,
                  int E, int grid, int* next, int table_ne, hipStream_t st,
                  std::vector<EvPair>* evs) {
  EvPair ev;
  if (evs) {
    ev = take_events(c);
    HIPCHK(hipEventRecord(ev.a, st));
  }
  const Dump nodump{nullptr, nullptr, nullptr};
  if (p.shared_emax > 0)
    HIPCHK(launch_crossmap_shared(E, p.mode, grid, b.rz, items, n, next, b.emb, b.pts, b.pj,
                                  b.qord, b.start, b.s64, static_cast<Moments*>(b.partial),
                                  p.window, st));
  else if (!p.nested.empty())
    HIPCHK(launch_crossmap_nested(E, p.mode, grid, b.rz, items, n, next, b.emb, b.pts, b.pj,
                                  b.qord, b.start, b.s64, b.segs,
                                  static_cast<Moments*>(b.partial), p.window, st));
  else if (p.spec.M > 0)
    HIPCHK(launch_crossmap_multi(E, p.mode, grid, b.rz, b.self, items, n, next, b.emb, b.pts,
                                 b.pj, b.qord, b.start, b.tt, p.spec.M, b.partial,
                                 p.spec.query_set, p.window, b.table, table_ne, st));
  else
    HIPCHK(launch_crossmap(E, p.mode, grid, b.rz, items, n, next, b.emb, b.pts, b.pj, b.qord,
                           b.start, b.s64, static_cast<Moments*>(b.partial), p.spec.query_set,
                           p.window, nodump, b.table, table_ne, st));
  if (evs) {
    HIPCHK(hipEventRecord(ev.b, st));
    evs->push_back(ev);
  }
}

}  // namespace

namespace ccmh {

void enqueue_plan(ccm_ctx* c, const Plan& p, const PlanBuffers& b,
                  const std::vector<int64_t>& plain_first, hipStream_t st,
                  std::vector<EvPair>* evs) {
  HIPCHK(launch_ingest(b.ingest, (int)p.ingest.size(), p.n64, b.s64, b.s32, st));
  HIPCHK(launch_embed(b.embed, (int)p.embed.size(), p.max_embed, b.s32, b.emb, st));
  if (p.spec.M > 0) HIPCHK(launch_transpose_targets(b.s64, p.spec.M, p.spec.N, b.tt, st));
  HIPCHK(launch_order_keys(b.orders, p.n_sets, b.s32, b.keys, st));
  HIPCHK(launch_iota_segments(b.iota, p.spec.N, p.n_sets, st));
  {
    size_t tb = p.sort_temp;
    HIPCHK(sort_series(b.sort_temp, tb, b.keys, b.keys_out, b.iota, b.order, p.spec.N,
                       p.n_sets, b.segoff, st));
    if (p.kd_levels > 0)
      HIPCHK(refine_orders_kd(b.orders, p.n_sets, p.kd_levels, p.spec.N, b.emb, b.order, b.iota,
                              b.keys, st));
  }
  HIPCHK(launch_query_order(b.embed, (int)p.embed.size(), b.order, b.qord, st));
  for (int E = 1; E <= kMaxE; ++E)
    HIPCHK(launch_table_build(E, b.tables + p.te_first[E], p.te_count[E], p.te_max_ne[E], b.emb,
                              b.table, st));
  const bool plain = (p.spec.flags & CCM_FLAG_PLAIN) != 0;
  const bool persistent = (p.spec.flags & CCM_FLAG_PERSISTENT) != 0;
  const bool nested = !p.nested.empty();
  // each wave draws and gathers its libraries into the shared pools, then
  // runs its cross-map launches (one per E)
  for (size_t wi = 0; wi < p.waves.size(); ++wi) {
    const Wave& w = p.waves[wi];
    if (!plain) {
      if (nested)
        HIPCHK(launch_sample_nested(b.nested + w.sample_first, w.sample_count, b.shuffle, b.lib,
                                    st));
      else
        HIPCHK(launch_sample(b.sample + w.sample_first, w.sample_count, b.lib, st));
      HIPCHK(launch_gather(b.gather + w.gather_first, w.gather_count, w.max_sorted_n_e, b.emb,
                           b.lib, b.order, b.pts, b.pj, b.start, st));
      for (int li = w.launch_first; li < w.launch_first + w.launch_count; ++li) {
        const Launch& L = p.launches[li];
        int grid = L.count;
        int* next = nullptr;
        if (persistent) {
          grid = persistent_grid(c, L.count);
          next = b.counter + li;
          HIPCHK(launch_zero_int(next, 1, st));
        }
        launch_items(c, p, b, b.items + L.first, L.count, L.E, grid, next, p.e_table_ne[L.E],
                     st, evs);
      }
    } else {
      // the unbatched baseline: sampler, gather and cross-map launched per
      // realization
      std::vector<char> sampled(w.sample_count, 0);
      for (int64_t k = p.wave_rz_first[wi]; k < p.wave_rz_first[wi + 1]; ++k) {
        const int32_t r = p.wave_rz[k];
        const Realization& R = p.rz[r];
        const int64_t sj = p.rz_sample[r];
        if (!sampled[sj - w.sample_first]) {
          HIPCHK(launch_sample(b.sample + sj, 1, b.lib, st));
          sampled[sj - w.sample_first] = 1;
        }
        const GatherJob& G = p.gather[p.rz_gather[r]];
        HIPCHK(launch_gather(b.gather + p.rz_gather[r], 1, G.sorted ? G.n_e : 0, b.emb, b.lib,
                             b.order, b.pts, b.pj, b.start, st));
        launch_items(c, p, b, b.plain_items + plain_first[r], R.n_tiles, R.E, R.n_tiles,
                     nullptr, R.table_off >= 0 ? R.n_e : 0, st, evs);
      }
    }
  }
  if (p.spec.M > 0)
    HIPCHK(launch_finalize_multi(b.rz, b.self, (int64_t)p.rz.size(), p.spec.M, b.partial,
                                 (int64_t)p.spec.L.size() * p.spec.r, b.out, st));
  else if (!p.rz_fin.empty())
    HIPCHK(launch_finalize(b.rz_fin, (int64_t)p.rz_fin.size(),
                           static_cast<const Moments*>(b.partial), b.out, st));
  else
    HIPCHK(launch_finalize(b.rz, (int64_t)p.rz.size(), static_cast<const Moments*>(b.partial),
                           b.out, st));
}

}  // namespace ccmh

namespace {

// Capture the plan's launches into an executable graph.
hipGraphExec_t capture(ccm_ctx* c, Exec* ex) {
  hipStream_t cap = c->stream;
  HIPCHK(hipStreamSynchronize(cap));
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_plan(c, ex->plan, ex->buf, ex->plain_first, cap, nullptr);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamEndCapture(cap, &g));
  hipGraphExec_t gx = nullptr;
  hipError_t e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  return gx;
}

// Run a prepared plan on stream st: series already in ex->d_s64.  While
// profiling, the launches are issued directly with an event pair around
// each cross-map launch (events recorded by graph nodes cannot be timed).
void run(ccm_ctx* c, Exec* ex, hipStream_t st) {
  const Plan& p = ex->plan;
  const bool use_graph = !c->profiling && !(p.spec.flags & CCM_FLAG_NO_GRAPH) &&
                         !(p.spec.flags & CCM_FLAG_PLAIN);
  if (use_graph) {
    if (!ex->graph) ex->graph = capture(c, ex);
    HIPCHK(hipGraphLaunch(ex->graph, st));
  } else {
    enqueue_plan(c, ex->plan, ex->buf, ex->plain_first, st,
                 c->profiling ? &c->ev_pending : nullptr);
  }
  if (c->profiling) {
    c->prof.waves += (double)p.waves.size();
    c->prof.pairs += p.pairs;
    c->prof.flops += p.flops;
    c->prof.predictions += p.preds;
    c->prof.realizations += (double)p.n_rho;
    c->prof.table_realizations += (double)p.table_rz;
  }
}


}  // namespace

static Spec make_matrix_spec(int32_t M, int64_t N, int32_t E, int32_t tau, const int64_t* L,
                             int32_t nL, int32_t r, uint64_t seed, const ccm_opts* opts) {
  if (M < 2) fail(CCM_E_INVAL, "M must be >= 2");
  Spec s = make_spec(N, &E, 1, &tau, 1, L, nL, r, seed, opts);
  s.M = M;
  return s;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

ccm_status ccm_create(int device, ccm_ctx** out) {
  if (!out) return CCM_E_INVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return CCM_E_DEVICE;
  ccm_ctx* c = new (std::nothrow) ccm_ctx;
  if (!c) return CCM_E_NOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return CCM_E_DEVICE;
  }
  c->num_cus = prop.multiProcessorCount;
  c->wave_limit = default_wave_limit(prop.totalGlobalMem);
  if (!noalloc_setup(device, &c->err)) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return CCM_E_DEVICE;
  }
  *out = c;
  return CCM_OK;
}

void ccm_destroy(ccm_ctx* c) {
  if (!c) return;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->exec.reset();
    for (auto& e : c->ev_pending) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (auto& e : c->ev_free) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->pinned) (void)hipHostFree(c->pinned);
  }
  delete c;
}

const char* ccm_last_error(const ccm_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

ccm_status ccm_set_wave_limit(ccm_ctx* c, uint64_t bytes) {
  return guarded(c, [&] {
    if (bytes == 0) {
      hipDeviceProp_t prop;
      HIPCHK(hipGetDeviceProperties(&prop, c->device));
      bytes = default_wave_limit(prop.totalGlobalMem);
    }
    c->wave_limit = bytes;
  });
}

namespace {

// The context's pinned staging buffer, at least `bytes` long.  Host arrays
// are copied through it so that the transfers are asynchronous DMA of
// pinned memory rather than staged pageable copies.
double* pinned_stage(ccm_ctx* c, size_t bytes) {
  if (c->pinned_bytes < bytes) {
    if (c->pinned) HIPCHK(hipHostFree(c->pinned));
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    HIPCHK(hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault));
    c->pinned_bytes = bytes;
  }
  return static_cast<double*>(c->pinned);
}

// Series in: n doubles from each of the host arrays, to dst on the device.
void upload_series(ccm_ctx* c, double* dst, std::initializer_list<const double*> src,
                   int64_t n, double* stage) {
  int64_t o = 0;
  for (const double* a : src) {
    std::memcpy(stage + o, a, (size_t)n * 8);
    o += n;
  }
  HIPCHK(hipMemcpyAsync(dst, stage, (size_t)o * 8, hipMemcpyHostToDevice, c->stream));
}

}  // namespace

ccm_status ccm_sweep(ccm_ctx* c, const double* X, const double* Y, int64_t N,
                     const int32_t* E, int32_t nE, const int32_t* tau, int32_t ntau,
                     const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
                     const ccm_opts* opts, double* rho) {
  return guarded(c, [&] {
    if (!rho) fail(CCM_E_INVAL, "rho is NULL");
    Spec s = make_spec(N, E, nE, tau, ntau, L, nL, r, seed, opts);
    s.wave_limit = c->wave_limit;
    check_host_series(X, N, "X");
    check_host_series(Y, N, "Y");
    Exec* ex = prepare(c, s);
    const int64_t n_out = ex->plan.n_out;
    double* h = pinned_stage(c, (size_t)std::max<int64_t>(2 * N, n_out) * 8);
    upload_series(c, ex->d_s64.as<double>(), {X, Y}, N, h);
    run(c, ex, c->stream);
    HIPCHK(hipMemcpyAsync(h, ex->d_out.p, n_out * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(rho, h, (size_t)n_out * 8);
  });
}

ccm_status ccm(ccm_ctx* c, const double* X, const double* Y, int64_t N, int32_t E,
               int32_t tau, const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
               const ccm_opts* opts, double* rho_xy, double* rho_yx, int64_t* L_eff) {
  return guarded(c, [&] {
    if (!rho_xy || !rho_yx) fail(CCM_E_INVAL, "rho output is NULL");
    Spec s = make_spec(N, &E, 1, &tau, 1, L, nL, r, seed, opts);
    s.wave_limit = c->wave_limit;
    check_host_series(X, N, "X");
    check_host_series(Y, N, "Y");
    Exec* ex = prepare(c, s);
    const int64_t half = (int64_t)nL * r;
    double* h = pinned_stage(c, (size_t)std::max<int64_t>(2 * N, 2 * half) * 8);
    upload_series(c, ex->d_s64.as<double>(), {X, Y}, N, h);
    run(c, ex, c->stream);
    HIPCHK(hipMemcpyAsync(h, ex->d_out.p, 2 * half * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(rho_xy, h, (size_t)half * 8);
    std::memcpy(rho_yx, h + half, (size_t)half * 8);
    if (L_eff)
      for (int i = 0; i < nL; ++i) L_eff[i] = ex->plan.L_eff[i];
  });
}

ccm_status ccm_sweep_dev(ccm_ctx* c, const double* X, const double* Y, int64_t N,
                         const int32_t* E, int32_t nE, const int32_t* tau, int32_t ntau,
                         const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
                         const ccm_opts* opts, double* rho, void* stream) {
  return guarded(c, [&] {
    if (!X || !Y || !rho) fail(CCM_E_INVAL, "NULL device pointer");
    Spec s = make_spec(N, E, nE, tau, ntau, L, nL, r, seed, opts);
    s.wave_limit = c->wave_limit;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Exec* ex = prepare(c, s);
    HIPCHK(launch_copy_pair(X, Y, N, ex->d_s64.as<double>(), st));
    run(c, ex, st);
    HIPCHK(hipMemcpyAsync(rho, ex->d_out.p, ex->plan.n_out * 8, hipMemcpyDeviceToDevice, st));
  });
}

ccm_status ccm_dev(ccm_ctx* c, const double* X, const double* Y, int64_t N, int32_t E,
                   int32_t tau, const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
                   const ccm_opts* opts, double* rho_xy, double* rho_yx, int64_t* L_eff,
                   void* stream) {
  return guarded(c, [&] {
    if (!X || !Y || !rho_xy || !rho_yx) fail(CCM_E_INVAL, "NULL device pointer");
    Spec s = make_spec(N, &E, 1, &tau, 1, L, nL, r, seed, opts);
    s.wave_limit = c->wave_limit;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Exec* ex = prepare(c, s);
    HIPCHK(launch_copy_pair(X, Y, N, ex->d_s64.as<double>(), st));
    run(c, ex, st);
    const int64_t half = (int64_t)nL * r;
    HIPCHK(launch_split_pair(ex->d_out.as<double>(), half, rho_xy, rho_yx, st));
    if (L_eff)
      for (int i = 0; i < nL; ++i) L_eff[i] = ex->plan.L_eff[i];
  });
}

ccm_status ccm_matrix(ccm_ctx* c, const double* S, int32_t M, int64_t N, int32_t E,
                      int32_t tau, const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
                      const ccm_opts* opts, double* rho) {
  return guarded(c, [&] {
    if (!rho) fail(CCM_E_INVAL, "rho is NULL");
    Spec s = make_matrix_spec(M, N, E, tau, L, nL, r, seed, opts);
    s.wave_limit = c->wave_limit;
    check_host_series(S, (int64_t)M * N, "S");
    Exec* ex = prepare(c, s);
    const int64_t n_out = ex->plan.n_out;
    double* h = pinned_stage(c, (size_t)std::max<int64_t>((int64_t)M * N, n_out) * 8);
    upload_series(c, ex->d_s64.as<double>(), {S}, (int64_t)M * N, h);
    run(c, ex, c->stream);
    HIPCHK(hipMemcpyAsync(h, ex->d_out.p, n_out * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(rho, h, (size_t)n_out * 8);
  });
}

ccm_status ccm_matrix_dev(ccm_ctx* c, const double* S, int32_t M, int64_t N, int32_t E,
                          int32_t tau, const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
                          const ccm_opts* opts, double* rho, void* stream) {
  return guarded(c, [&] {
    if (!S || !rho) fail(CCM_E_INVAL, "NULL device pointer");
    Spec s = make_matrix_spec(M, N, E, tau, L, nL, r, seed, opts);
    s.wave_limit = c->wave_limit;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Exec* ex = prepare(c, s);
    HIPCHK(hipMemcpyAsync(ex->d_s64.p, S, (size_t)M * N * 8, hipMemcpyDeviceToDevice, st));
    run(c, ex, st);
    HIPCHK(hipMemcpyAsync(rho, ex->d_out.p, ex->plan.n_out * 8, hipMemcpyDeviceToDevice, st));
  });
}

ccm_status ccm_library(ccm_ctx* c, int64_t N_e, int32_t E, int32_t tau, int64_t L_eff,
                       int32_t r_index, uint64_t seed, int32_t* idx_out) {
  return guarded(c, [&] {
    if (!idx_out) fail(CCM_E_INVAL, "idx_out is NULL");
    if (N_e < 1 || L_eff < 1 || L_eff > N_e || N_e > INT32_MAX)
      fail(CCM_E_INVAL, "need 1 <= L_eff <= N_e < 2^31");
    if (E < 1 || E > kMaxE || tau < 1) fail(CCM_E_INVAL, "E in [1, 10] and tau >= 1");
    DevBuf job, out;
    std::vector<SampleJob> j{{seed, N_e, L_eff, 0, E, tau, r_index, 0}};
    upload(job, j);
    out.ensure(L_eff * 4);
    HIPCHK(launch_sample(job.as<SampleJob>(), 1, out.as<int32_t>(), c->stream));
    HIPCHK(hipMemcpyAsync(idx_out, out.p, L_eff * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

ccm_status ccm_nested_library(ccm_ctx* c, int64_t N_e, int32_t E, int32_t tau,
                              int32_t r_index, uint64_t seed, int64_t n_out,
                              int32_t* idx_out) {
  return guarded(c, [&] {
    if (!idx_out) fail(CCM_E_INVAL, "idx_out is NULL");
    if (N_e < 1 || n_out < 1 || n_out > N_e || N_e > INT32_MAX)
      fail(CCM_E_INVAL, "need 1 <= n_out <= N_e < 2^31");
    if (E < 1 || E > kMaxE || tau < 1) fail(CCM_E_INVAL, "E in [1, 10] and tau >= 1");
    DevBuf job, scratch, out;
    NestedJob nj{};
    nj.seed = seed;
    nj.n_e = N_e;
    nj.n_out = n_out;
    nj.E = E;
    nj.tau = tau;
    nj.r_index = r_index;
    std::vector<NestedJob> j{nj};
    upload(job, j);
    scratch.ensure(N_e * 4);
    out.ensure(n_out * 4);
    HIPCHK(launch_sample_nested(job.as<NestedJob>(), 1, scratch.as<int32_t>(),
                                out.as<int32_t>(), c->stream));
    HIPCHK(hipMemcpyAsync(idx_out, out.p, n_out * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

ccm_status ccm_neighbors(ccm_ctx* c, const double* lib_series, const double* target,
                         int64_t N, int32_t E, int32_t tau, const int32_t* lib_idx,
                         int64_t L_eff, const ccm_opts* opts, int32_t* nbr, float* d2,
                         double* pred, double* rho) {
  return guarded(c, [&] {
    if (!lib_idx) fail(CCM_E_INVAL, "lib_idx is NULL");
    if (N < 2 || N > INT32_MAX / 2) fail(CCM_E_INVAL, "N out of range");
    if (E < 1 || E > kMaxE || tau < 1) fail(CCM_E_INVAL, "E in [1, 10] and tau >= 1");
    check_host_series(lib_series, N, "lib_series");
    check_host_series(target, N, "target");
    const int64_t ne = N - (int64_t)(E - 1) * tau;
    if (ne < E + 2) fail(CCM_E_INVAL, "N_e = N - (E-1) tau must be >= E + 2");
    const int32_t excl = opts ? opts->exclusion_radius : 0;
    const int32_t qs = opts ? opts->query_set : 0;
    if (qs != 0 && qs != 1) fail(CCM_E_INVAL, "query_set must be 0 or 1");
    if (L_eff < min_library(E, excl) || L_eff > ne)
      fail(CCM_E_INVAL, "L_eff out of range for this E, tau and exclusion window");
    for (int64_t i = 0; i < L_eff; ++i) {
      if (lib_idx[i] < 0 || lib_idx[i] >= ne) fail(CCM_E_INVAL, "lib_idx out of range");
      if (i > 0 && lib_idx[i] <= lib_idx[i - 1]) fail(CCM_E_INVAL, "lib_idx not ascending");
    }
    const int Q = crossmap_queries_per_lane(E);
    const int64_t nq = qs ? L_eff : ne;
    const int64_t qt = (int64_t)kBlock * Q;
    const int n_tiles = (int)((nq + qt - 1) / qt);
    const int K = E + 1;
    const int32_t sorted = ne <= gather_max_sorted_n_e() ? 1 : 0;

    DevBuf d_s64, d_s32, d_emb, d_lib, d_pts, d_pj, d_rz, d_items, d_ingest, d_embed,
        d_gather, d_partial, d_out, d_nbr, d_d2, d_pred, d_iota, d_keys, d_keys_out, d_order,
        d_segoff, d_temp, d_qord, d_start, d_orders;
    std::vector<int32_t> seg{0, (int32_t)N};
    // the same visiting order as the batched plans
    Plan op;
    op.spec.N = N;
    {
      const int64_t ko = order_set(op, 0, embedding_order(E, tau));
      attach_kd(op, ko, E, 0, ne);
      size_order_sort(op);
    }
    const std::vector<OrderJob>& oj = op.orders;
    size_t temp_bytes = op.sort_temp;
    std::vector<IngestJob> ij{{0, 0, N}};
    std::vector<EmbedJob> ej{{0, 0, 0, 0, ne, N, E, tau}};
    GatherJob g{};
    g.l_eff = L_eff;
    g.n_e = ne;
    g.n_series = N;
    g.E = E;
    g.tau = tau;
    g.qt = (int32_t)qt;
    g.query_set = qs;
    g.sorted = sorted;
    std::vector<GatherJob> gj{g};
    // CCM_FLAG_TABLE: the realization walks a table over the embedding
    // whatever its size (the hook exercises the walk and its fallback).
    const bool tab = opts && (opts->flags & CCM_FLAG_TABLE) && ne <= kTableMaxNe;
    const int32_t tw = (int32_t)std::min<int64_t>(kTableWidth, ne);
    Realization R{};
    R.table_off = tab ? 0 : -1;
    R.table_w = tw;
    R.tgt_off = N;
    R.E = E;
    R.tau = tau;
    R.n_e = (int32_t)ne;
    R.l_eff = (int32_t)L_eff;
    R.n_query = (int32_t)nq;
    R.n_tiles = n_tiles;
    std::vector<Realization> rv{R};
    std::vector<Item> items;
    for (int t = 0; t < n_tiles; ++t) items.push_back({0, t});
    upload(d_segoff, seg);
    upload(d_orders, oj);
    upload(d_ingest, ij);
    upload(d_embed, ej);
    upload(d_gather, gj);
    upload(d_rz, rv);
    upload(d_items, items);
    DevBuf d_tj, d_tab;
    if (tab) {
      TableJob tj{};
      tj.n_e = (int32_t)ne;
      tj.E = E;
      tj.w = tw;
      std::vector<TableJob> tv{tj};
      upload(d_tj, tv);
      d_tab.ensure(ne * table_row_stride(tw) * 4);
    }
    d_s64.ensure(2 * N * 8);
    d_s32.ensure(N * 4);
    d_iota.ensure(N * 4);
    d_keys.ensure(N * 4);
    d_keys_out.ensure(N * 4);
    d_order.ensure(N * 4);
    d_temp.ensure(temp_bytes);
    d_qord.ensure(ne * 4);
    d_start.ensure(n_tiles * 4 * kWaves);
    d_emb.ensure(ne * E * 4);
    d_lib.ensure(L_eff * 4);
    d_pts.ensure(L_eff * E * 4);
    d_pj.ensure(L_eff * 4);
    d_partial.ensure(n_tiles * sizeof(Moments));
    d_out.ensure(8);
    // dump rows are indexed by embedded point
    d_nbr.ensure(ne * K * 4);
    d_d2.ensure(ne * K * 4);
    d_pred.ensure(ne * 8);
    hipStream_t st = c->stream;
    HIPCHK(hipMemcpyAsync(d_s64.p, lib_series, N * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_s64.as<double>() + N, target, N * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_lib.p, lib_idx, L_eff * 4, hipMemcpyHostToDevice, st));
    HIPCHK(launch_ingest(d_ingest.as<IngestJob>(), 1, N, d_s64.as<double>(),
                         d_s32.as<float>(), st));
    HIPCHK(launch_embed(d_embed.as<EmbedJob>(), 1, ne * E, d_s32.as<float>(),
                        d_emb.as<float>(), st));
    HIPCHK(launch_order_keys(d_orders.as<OrderJob>(), 1, d_s32.as<float>(),
                             d_keys.as<uint32_t>(), st));
    HIPCHK(launch_iota_segments(d_iota.as<int32_t>(), N, 1, st));
    HIPCHK(sort_series(d_temp.p, temp_bytes, d_keys.as<uint32_t>(), d_keys_out.as<uint32_t>(),
                       d_iota.as<int32_t>(), d_order.as<int32_t>(), N, 1,
                       d_segoff.as<int32_t>(), st));
    if (op.kd_levels > 0)
      HIPCHK(refine_orders_kd(d_orders.as<OrderJob>(), 1, op.kd_levels, N, d_emb.as<float>(),
                              d_order.as<int32_t>(), d_iota.as<int32_t>(),
                              d_keys.as<uint32_t>(), st));
    HIPCHK(launch_query_order(d_embed.as<EmbedJob>(), 1, d_order.as<int32_t>(),
                              d_qord.as<int32_t>(), st));
    HIPCHK(launch_gather(d_gather.as<GatherJob>(), 1, sorted ? ne : 0, d_emb.as<float>(),
                         d_lib.as<int32_t>(), d_order.as<int32_t>(), d_pts.as<float>(),
                         d_pj.as<int32_t>(), d_start.as<int32_t>(), st));
    if (tab)
      HIPCHK(launch_table_build(E, d_tj.as<TableJob>(), 1, (int)ne, d_emb.as<float>(),
                                d_tab.as<int32_t>(), st));
    Dump dump{d_nbr.as<int32_t>(), d_d2.as<float>(), d_pred.as<double>()};
    HIPCHK(launch_crossmap(E, excl_mode(excl), n_tiles, d_rz.as<Realization>(),
                           d_items.as<Item>(), n_tiles, nullptr, d_emb.as<float>(),
                           d_pts.as<float>(), d_pj.as<int32_t>(), d_qord.as<int32_t>(),
                           d_start.as<int32_t>(), d_s64.as<double>(),
                           d_partial.as<Moments>(), qs, excl > 0 ? excl : 0, dump,
                           d_tab.as<int32_t>(), tab ? (int)ne : 0, st));
    HIPCHK(launch_finalize(d_rz.as<Realization>(), 1, d_partial.as<Moments>(),
                           d_out.as<double>(), st));
    std::vector<int32_t> hn(ne * K);
    std::vector<float> hd(ne * K);
    std::vector<double> hp(ne);
    HIPCHK(hipMemcpyAsync(hn.data(), d_nbr.p, ne * K * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hd.data(), d_d2.p, ne * K * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hp.data(), d_pred.p, ne * 8, hipMemcpyDeviceToHost, st));
    if (rho) HIPCHK(hipMemcpyAsync(rho, d_out.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t q = 0; q < nq; ++q) {
      const int64_t row = qs ? lib_idx[q] : q;
      if (nbr) std::memcpy(nbr + q * K, hn.data() + row * K, K * 4);
      if (d2) std::memcpy(d2 + q * K, hd.data() + row * K, K * 4);
      if (pred) pred[q] = hp[row];
    }
  });
}

ccm_status ccm_profile_enable(ccm_ctx* c, int on) {
  return guarded(c, [&] { c->profiling = on != 0; });
}

ccm_status ccm_profile_read(ccm_ctx* c, ccm_profile* out, int reset) {
  return guarded(c, [&] {
    if (!out) fail(CCM_E_INVAL, "out is NULL");
    drain_events(c);
    *out = c->prof;
    if (reset) c->prof = ccm_profile{};
  });
}

}  // extern "C"

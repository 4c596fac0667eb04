// ccm_server.cpp -- served form: continuous batching of CCM jobs on one GPU.
//
// Jobs (a pair of series plus E, tau, an L grid and r; paper Section 3.1's
// input record, Section 3.3's concurrent pipelines) are submitted from any
// host thread and queued.  A scheduler thread admits them in arrival order
// while their device footprint fits a fixed HBM budget (one preallocated
// arena), runs each admitted job's preparation (ingest, embedding, order,
// library draws, gather) and then feeds the cross-map kernel with *epochs*:
// each epoch takes work items (query tiles) from the admitted jobs, oldest
// first, up to a time budget, so jobs that arrive while others run join the
// next epoch and their work overlaps on the device.  A job's moments live in
// its own slots and are merged in a fixed order when its last item is done,
// so its result does not depend on what it shared epochs with.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "ccm_context.h"

using namespace ccmh;

namespace {

// First-fit allocator over [0, capacity) with coalescing on release.
class RangeAlloc {
 public:
  explicit RangeAlloc(uint64_t cap = 0) { reset(cap); }
  void reset(uint64_t cap) {
    free_.clear();
    cap_ = cap;
    if (cap) free_[0] = cap;
  }
  uint64_t capacity() const { return cap_; }
  bool alloc(uint64_t n, uint64_t align, uint64_t* off) {
    if (n == 0) n = 1;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      const uint64_t start = (it->first + align - 1) / align * align;
      const uint64_t end = it->first + it->second;
      if (start + n <= end) {
        const uint64_t b0 = it->first;
        free_.erase(it);
        if (start > b0) free_[b0] = start - b0;
        if (end > start + n) free_[start + n] = end - (start + n);
        *off = start;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    if (n == 0) n = 1;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  uint64_t cap_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

enum JobState { kPending, kActive, kDone, kCancelled, kFailed };

// Byte layout of one job's region in the arena.  The series and the
// descriptor arrays come first, as one block [0, upload): the job's pinned
// staging block holds the same bytes at the same offsets, so one copy
// uploads them.
struct Layout {
  uint64_t s64, s32, iota, keys, keys_out, order, temp, qord, emb, lib, pts, pj, out, table;
  uint64_t d_ingest, d_embed, d_sample, d_gather, d_segoff, d_orders, d_tables;
  uint64_t upload;   // bytes of the series and descriptor block
  uint64_t bytes;
};

uint64_t up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

Layout layout_of(const Plan& p) {
  Layout l{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = up(o + std::max<uint64_t>(bytes, 1), 256);
    return at;
  };
  l.s64 = take(p.n64 * 8);
  l.d_ingest = take(p.ingest.size() * sizeof(IngestJob));
  l.d_embed = take(p.embed.size() * sizeof(EmbedJob));
  l.d_sample = take(p.sample.size() * sizeof(SampleJob));
  l.d_gather = take(p.gather.size() * sizeof(GatherJob));
  l.d_segoff = take(p.seg_off.size() * 4);
  l.d_orders = take(p.orders.size() * sizeof(OrderJob));
  l.d_tables = take(p.tables.size() * sizeof(TableJob));
  l.upload = o;
  l.s32 = take(p.n32 * 4);
  l.iota = take(p.n_ord * 4);
  l.keys = take(p.n_ord * 4);
  l.keys_out = take(p.n_ord * 4);
  l.order = take(p.n_ord * 4);
  l.temp = take(p.sort_temp);
  l.qord = take(p.n_qord * 4);
  l.emb = take(p.n_emb * 4);
  l.lib = take(p.n_lib * 4);
  l.pts = take(p.n_pts * 4);
  l.pj = take(p.n_pj * 4);
  l.out = take(p.n_out * 8);
  l.table = take(p.n_table * 4);
  l.bytes = o;
  return l;
}

struct Job {
  uint64_t ticket = 0;
  Plan plan;
  Layout lay{};
  // Pinned staging, filled at submit: [0, lay.upload) mirrors the region's
  // series and descriptor block, then the realizations (rebased at
  // admission), then the rho copied back.
  char* staging = nullptr;
  uint64_t staging_rz = 0, staging_rho = 0;
  JobState state = kPending;
  ccm_status status = CCM_OK;
  // resources (valid while active)
  uint64_t region = 0, slot0 = 0, rz0 = 0;
  bool has_region = false, has_slots = false, has_rz = false;
  size_t next_item = 0;          // scheduling cursor into plan.items
  int64_t last_epoch = -1;       // last epoch that ran items of this job
  bool finishing = false;        // finalize queued
  // Set only once the scheduler holds no reference to the job any more (its
  // device work is complete and its resources are released, or it never
  // left the queue): until then ccm_wait keeps waiting and ccm_result
  // answers CCM_E_BUSY, whatever the state says.
  bool retired = false;
  // per epoch stream: an epoch on it has waited for the job's preparation
  // (epochs on the two streams run concurrently, so each stream waits once)
  bool prep_waited[2] = {false, false};
  hipEvent_t prep_ev = nullptr;  // after its upload and preparation kernels
  hipEvent_t done_ev = nullptr;
  double* rho_host = nullptr;    // pinned [n_out], inside staging
  double t_submit = 0, t_admit = 0, t_done = 0;

  Job() = default;
  Job(const Job&) = delete;
  Job& operator=(const Job&) = delete;
  ~Job() {
    if (staging) (void)hipHostFree(staging);
    if (prep_ev) (void)hipEventDestroy(prep_ev);
    if (done_ev) (void)hipEventDestroy(done_ev);
  }
};

// Cost of one work item in VALU lane operations: tile queries x library x (2E+1).
double item_cost(const Realization& R, int tile, int qt) {
  const int q = std::min<int64_t>(qt, (int64_t)R.n_query - (int64_t)tile * qt);
  return (double)q * R.l_eff * (2.0 * R.E + 1.0);
}

}  // namespace

struct ccm_server {
  ccm_ctx* ctx = nullptr;
  int device = 0;
  hipStream_t pstream = nullptr;     // job upload and preparation
  hipStream_t fstream = nullptr;     // job finalize and result copy
  hipStream_t estream[2] = {nullptr, nullptr};   // epochs alternate between these
  double epoch_ms = 20.0;
  int max_jobs = 64;
  // device memory
  DevBuf arena, slots_partial, slots_start, rz_table, items_dev[2];
  size_t items_cap = 0;
  RangeAlloc arena_alloc, slot_alloc, rz_alloc;
  // host staging for epoch items (pinned)
  Item* items_host[2] = {nullptr, nullptr};
  hipEvent_t epoch_ev[2] = {nullptr, nullptr};     // end of each in-flight epoch
  hipEvent_t epoch_ev0[2] = {nullptr, nullptr};    // start of its kernels
  double last_end_host = -1.0;                     // host time the last epoch was seen done
  double epoch_cost[2] = {0.0, 0.0};
  size_t min_items = 8192;                         // keep the GPU full within an epoch
  bool epoch_busy[2] = {false, false};
  int64_t epoch_count = 0;
  double lane_ops_per_ms = 4.0e10;   // throughput estimate, refined online
  // jobs
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;      // admission order
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string fatal;                 // set when the device failed
  std::thread worker;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void free_job_resources(ccm_server* s, Job& j) {
  if (j.has_region) s->arena_alloc.release(j.region, j.lay.bytes);
  if (j.has_slots) s->slot_alloc.release(j.slot0, (uint64_t)j.plan.n_slots);
  if (j.has_rz) s->rz_alloc.release(j.rz0, (uint64_t)j.plan.rz.size());
  j.has_region = j.has_slots = j.has_rz = false;
}

// Try to reserve a job's device resources; false if they do not fit now.
bool reserve(ccm_server* s, Job& j) {
  uint64_t reg = 0, sl = 0, rz = 0;
  if (!s->arena_alloc.alloc(j.lay.bytes, 256, &reg)) return false;
  if (!s->slot_alloc.alloc((uint64_t)j.plan.n_slots, 1, &sl)) {
    s->arena_alloc.release(reg, j.lay.bytes);
    return false;
  }
  if (!s->rz_alloc.alloc((uint64_t)j.plan.rz.size(), 1, &rz)) {
    s->arena_alloc.release(reg, j.lay.bytes);
    s->slot_alloc.release(sl, (uint64_t)j.plan.n_slots);
    return false;
  }
  j.region = reg;
  j.slot0 = sl;
  j.rz0 = rz;
  j.has_region = j.has_slots = j.has_rz = true;
  return true;
}

template <class T>
T* at(const ccm_server* s, uint64_t byte_off) {
  return reinterpret_cast<T*>(static_cast<char*>(s->arena.p) + byte_off);
}

// Fill a job's pinned staging block at submit: series and descriptors at
// their region offsets, then the realizations (region-relative until
// admission).
void stage_job(Job& j, const double* X, const double* Y) {
  const Plan& p = j.plan;
  const Layout& L = j.lay;
  char* b = j.staging;
  auto put = [&](uint64_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(b + off, src, bytes);
  };
  const int64_t N = p.spec.N;
  put(L.s64, X, N * 8);
  put(L.s64 + N * 8, Y, N * 8);
  put(L.d_ingest, p.ingest.data(), p.ingest.size() * sizeof(IngestJob));
  put(L.d_embed, p.embed.data(), p.embed.size() * sizeof(EmbedJob));
  put(L.d_sample, p.sample.data(), p.sample.size() * sizeof(SampleJob));
  put(L.d_gather, p.gather.data(), p.gather.size() * sizeof(GatherJob));
  put(L.d_segoff, p.seg_off.data(), p.seg_off.size() * 4);
  put(L.d_orders, p.orders.data(), p.orders.size() * sizeof(OrderJob));
  put(L.d_tables, p.tables.data(), p.tables.size() * sizeof(TableJob));
  put(j.staging_rz, p.rz.data(), p.rz.size() * sizeof(Realization));
}

// At admission: rebase the staged descriptors to the job's region and slots,
// upload them with two asynchronous copies from the pinned staging, and
// queue the preparation kernels; all on the preparation stream, ending with
// the job's prep_ev.
void start_job(ccm_server* s, Job& j) {
  const Plan& p = j.plan;
  const Layout& L = j.lay;
  const uint64_t R0 = j.region;
  hipStream_t st = s->pstream;
  const int64_t N = p.spec.N;
  // the gather writes scan starts into the server-wide slot space
  GatherJob* gj = reinterpret_cast<GatherJob*>(j.staging + L.d_gather);
  for (size_t k = 0; k < p.gather.size(); ++k) gj[k].start_off += (int64_t)j.slot0 * kWaves;
  // realizations rebased to arena-wide offsets
  Realization* rz = reinterpret_cast<Realization*>(j.staging + j.staging_rz);
  for (size_t k = 0; k < p.rz.size(); ++k) {
    Realization& R = rz[k];
    R.emb_off += (int64_t)((R0 + L.emb) / 4);
    R.pts_off += (int64_t)((R0 + L.pts) / 4);
    R.pj_off += (int64_t)((R0 + L.pj) / 4);
    R.qord_off += (int64_t)((R0 + L.qord) / 4);
    R.tgt_off += (int64_t)((R0 + L.s64) / 8);
    R.slot_base += (int64_t)j.slot0;
    if (R.table_off >= 0) R.table_off += (int64_t)((R0 + L.table) / 4);
  }
  // distance indexing tables, rebased the same way (their extents within
  // the job's embedding and table pools were checked at submit)
  TableJob* tj = reinterpret_cast<TableJob*>(j.staging + L.d_tables);
  for (size_t k = 0; k < p.tables.size(); ++k) {
    tj[k].emb_off += (int64_t)((R0 + L.emb) / 4);
    tj[k].out_off += (int64_t)((R0 + L.table) / 4);
  }
  HIPCHK(hipMemcpyAsync(at<char>(s, R0), j.staging, L.upload, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->rz_table.as<Realization>() + j.rz0, rz,
                        p.rz.size() * sizeof(Realization), hipMemcpyHostToDevice, st));

  HIPCHK(launch_ingest(at<IngestJob>(s, R0 + L.d_ingest), (int)p.ingest.size(), p.n64,
                       at<double>(s, R0 + L.s64), at<float>(s, R0 + L.s32), st));
  HIPCHK(launch_embed(at<EmbedJob>(s, R0 + L.d_embed), (int)p.embed.size(), p.max_embed,
                      at<float>(s, R0 + L.s32), at<float>(s, R0 + L.emb), st));
  for (int E = 1; E <= kMaxE; ++E)
    HIPCHK(launch_table_build(E, at<TableJob>(s, R0 + L.d_tables) + p.te_first[E],
                              p.te_count[E], p.te_max_ne[E], at<float>(s, 0),
                              at<int32_t>(s, 0), st));
  HIPCHK(launch_order_keys(at<OrderJob>(s, R0 + L.d_orders), p.n_sets,
                           at<float>(s, R0 + L.s32), at<uint32_t>(s, R0 + L.keys), st));
  HIPCHK(launch_iota_segments(at<int32_t>(s, R0 + L.iota), N, p.n_sets, st));
  size_t tb = p.sort_temp;
  HIPCHK(sort_series(at<void>(s, R0 + L.temp), tb, at<uint32_t>(s, R0 + L.keys),
                     at<uint32_t>(s, R0 + L.keys_out), at<int32_t>(s, R0 + L.iota),
                     at<int32_t>(s, R0 + L.order), N, p.n_sets,
                     at<int32_t>(s, R0 + L.d_segoff), st));
  if (p.kd_levels > 0)
    HIPCHK(refine_orders_kd(at<OrderJob>(s, R0 + L.d_orders), p.n_sets, p.kd_levels, N,
                            at<float>(s, R0 + L.emb), at<int32_t>(s, R0 + L.order),
                            at<int32_t>(s, R0 + L.iota), at<uint32_t>(s, R0 + L.keys), st));
  HIPCHK(launch_query_order(at<EmbedJob>(s, R0 + L.d_embed), (int)p.embed.size(),
                            at<int32_t>(s, R0 + L.order), at<int32_t>(s, R0 + L.qord), st));
  HIPCHK(launch_sample(at<SampleJob>(s, R0 + L.d_sample), (int64_t)p.sample.size(),
                       at<int32_t>(s, R0 + L.lib), st));
  HIPCHK(launch_gather(at<GatherJob>(s, R0 + L.d_gather), (int64_t)p.gather.size(),
                       p.max_sorted_n_e, at<float>(s, R0 + L.emb), at<int32_t>(s, R0 + L.lib),
                       at<int32_t>(s, R0 + L.order), at<float>(s, R0 + L.pts),
                       at<int32_t>(s, R0 + L.pj), s->slots_start.as<int32_t>(), st));
  HIPCHK(hipEventRecord(j.prep_ev, st));
}

// Queue the merge of a job's moments and the copy of its rho to the host.
void finish_job(ccm_server* s, Job& j) {
  const Plan& p = j.plan;
  // the job's items may be in the latest epoch of either epoch stream
  hipStream_t st = s->fstream;
  for (int b = 0; b < 2; ++b) HIPCHK(hipStreamWaitEvent(st, s->epoch_ev[b], 0));
  HIPCHK(launch_finalize(s->rz_table.as<Realization>() + j.rz0, (int64_t)p.rz.size(),
                         s->slots_partial.as<Moments>(), at<double>(s, j.region + j.lay.out),
                         st));
  HIPCHK(hipMemcpyAsync(j.rho_host, at<double>(s, j.region + j.lay.out), p.n_out * 8,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(j.done_ev, st));
  j.finishing = true;
}

struct GroupKey {
  int E, mode, qs, window;
  bool operator<(const GroupKey& o) const {
    if (E != o.E) return E < o.E;
    if (mode != o.mode) return mode < o.mode;
    if (qs != o.qs) return qs < o.qs;
    return window < o.window;
  }
};

// One scheduler iteration; called with the lock held, may drop it for waits.
void scheduler_loop(ccm_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  int buf = 0;
  while (true) {
    try {
      HIPCHK(hipSetDevice(s->device));
      // 1. retire finished jobs
      for (auto it = s->active.begin(); it != s->active.end();) {
        Job& j = *s->jobs[*it];
        if (j.finishing && hipEventQuery(j.done_ev) == hipSuccess) {
          j.state = (j.state == kCancelled) ? kCancelled : kDone;
          j.t_done = s->now();
          free_job_resources(s, j);
          j.retired = true;
          it = s->active.erase(it);
          s->cv_done.notify_all();
        } else {
          ++it;
        }
      }
      if (s->stop && s->active.empty()) break;
      // 2. admit in arrival order while the footprint fits
      while (!s->stop && !s->pending.empty() && (int)s->active.size() < s->max_jobs) {
        Job& j = *s->jobs[s->pending.front()];
        if (!reserve(s, j)) break;
        s->pending.pop_front();
        j.state = kActive;
        j.t_admit = s->now();
        s->active.push_back(j.ticket);
        start_job(s, j);
      }
      // 3. build an epoch: items of admitted jobs, oldest first, up to the
      // budget.  Two epochs may be in flight: this buffer's previous epoch is
      // waited for (and timed) only now, so the GPU runs the other one while
      // the host prepares this one.
      if (s->epoch_busy[buf]) {
        lk.unlock();
        HIPCHK(hipEventSynchronize(s->epoch_ev[buf]));
        // epochs overlap on two streams: the time an epoch adds is measured
        // end to end (from the previous epoch's completion, or its own start)
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, s->epoch_ev0[buf], s->epoch_ev[buf]));
        const double t_end = s->now();
        if (s->last_end_host >= 0.0) {
          const double gap = (t_end - s->last_end_host) * 1e3;
          if (gap > 0.0 && gap < ms) ms = (float)gap;
        }
        s->last_end_host = t_end;
        lk.lock();
        s->epoch_busy[buf] = false;
        if (ms > 0.5f) {
          const double rate = std::min(2.0e11, std::max(1.0e10, s->epoch_cost[buf] / ms));
          s->lane_ops_per_ms = 0.7 * s->lane_ops_per_ms + 0.3 * rate;
        }
        continue;   // re-check retirements and admissions first
      }
      const double budget = s->epoch_ms * s->lane_ops_per_ms;
      double cost = 0.0;
      std::map<GroupKey, std::vector<Item>> groups;
      std::map<GroupKey, int> group_table_ne;   // largest n_e a group's items walk
      std::vector<Job*> completes, first_epoch;
      size_t n_items = 0;
      for (uint64_t t : s->active) {
        Job& j = *s->jobs[t];
        if (j.finishing || j.state == kCancelled) continue;
        const Plan& p = j.plan;
        if (!j.prep_waited[buf]) {
          first_epoch.push_back(&j);   // its preparation must precede this epoch
          j.prep_waited[buf] = true;
        }
        const int E = p.spec.E[0];
        const int qt = kBlock * crossmap_queries_per_lane(E);
        const GroupKey key{E, p.mode, p.spec.query_set, p.window};
        auto& g = groups[key];
        int& tne = group_table_ne[key];
        tne = std::max(tne, p.e_table_ne[E]);
        while (j.next_item < p.items.size() &&
               (cost < budget || n_items < s->min_items) && n_items < s->items_cap) {
          const Item it = p.items[j.next_item++];
          cost += item_cost(p.rz[it.rz], it.tile, qt);
          g.push_back({(int32_t)(j.rz0 + it.rz), it.tile});
          ++n_items;
        }
        j.last_epoch = g.empty() ? j.last_epoch : s->epoch_count;
        if (j.next_item == p.items.size()) completes.push_back(&j);
        if ((cost >= budget && n_items >= s->min_items) || n_items >= s->items_cap) break;
      }
      // jobs cancelled while active finish once their in-flight preparation
      // and items are done (their region is reused after that)
      for (uint64_t t : s->active) {
        Job& j = *s->jobs[t];
        if (j.state == kCancelled && !j.finishing) {
          HIPCHK(hipStreamWaitEvent(s->fstream, j.prep_ev, 0));
          for (int b = 0; b < 2; ++b)
            HIPCHK(hipStreamWaitEvent(s->fstream, s->epoch_ev[b], 0));
          HIPCHK(hipEventRecord(j.done_ev, s->fstream));
          j.finishing = true;
        }
      }
      if (n_items == 0) {
        bool waiting_done = false;
        for (uint64_t t : s->active) waiting_done |= s->jobs[t]->finishing;
        for (Job* j : completes)
          if (!j->finishing && j->state != kCancelled) finish_job(s, *j);
        if (s->stop && s->active.empty() && s->pending.empty()) break;
        if (waiting_done || !completes.empty()) {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(200));
          lk.lock();
        } else {
          s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
        continue;
      }
      // 4. launch the epoch (items grouped by kernel variant)
      size_t pos = 0;
      for (auto& kv : groups) pos += kv.second.size();
      pos = 0;
      for (auto& kv : groups) {
        std::copy(kv.second.begin(), kv.second.end(), s->items_host[buf] + pos);
        pos += kv.second.size();
      }
      hipStream_t es = s->estream[buf];
      for (Job* j : first_epoch) HIPCHK(hipStreamWaitEvent(es, j->prep_ev, 0));
      HIPCHK(hipMemcpyAsync(s->items_dev[buf].p, s->items_host[buf], pos * sizeof(Item),
                            hipMemcpyHostToDevice, es));
      HIPCHK(hipEventRecord(s->epoch_ev0[buf], es));
      pos = 0;
      float* fa = static_cast<float*>(s->arena.p);
      int32_t* ia = static_cast<int32_t*>(s->arena.p);
      double* da = static_cast<double*>(s->arena.p);
      const Dump nodump{nullptr, nullptr, nullptr};
      for (auto& kv : groups) {
        const int n = (int)kv.second.size();
        if (n == 0) continue;
        HIPCHK(launch_crossmap(kv.first.E, kv.first.mode, n,
                               s->rz_table.as<Realization>(),
                               s->items_dev[buf].as<Item>() + pos, n, nullptr, fa, fa, ia, ia,
                               s->slots_start.as<int32_t>(), da,
                               s->slots_partial.as<Moments>(), kv.first.qs, kv.first.window,
                               nodump, ia, group_table_ne[kv.first], es));
        pos += n;
      }
      HIPCHK(hipEventRecord(s->epoch_ev[buf], es));
      s->epoch_busy[buf] = true;
      s->epoch_cost[buf] = cost;
      for (Job* j : completes)
        if (!j->finishing && j->state != kCancelled) finish_job(s, *j);
      ++s->epoch_count;
      buf ^= 1;
    } catch (const Fail& e) {
      s->fatal = e.what;
      for (uint64_t t : s->active) {
        Job& j = *s->jobs[t];
        j.state = kFailed;
        j.status = e.status;
        j.t_done = s->now();
        free_job_resources(s, j);
        j.retired = true;
      }
      s->active.clear();
      for (uint64_t t : s->pending) {
        Job& j = *s->jobs[t];
        j.state = kFailed;
        j.status = e.status;
        j.retired = true;
      }
      s->pending.clear();
      s->cv_done.notify_all();
      if (s->stop) break;
      s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

}  // namespace

extern "C" {

ccm_status ccm_server_create(ccm_ctx* c, const ccm_server_cfg* cfg, ccm_server** out) {
  if (!c || !out) return CCM_E_INVAL;
  *out = nullptr;
  auto s = std::make_unique<ccm_server>();
  s->ctx = c;
  s->device = c->device;
  s->t0 = std::chrono::steady_clock::now();
  try {
    HIPCHK(hipSetDevice(c->device));
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    uint64_t budget = cfg && cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes
                                                   : std::min<uint64_t>(free_b / 4, 32ull << 30);
    if (budget > free_b / 2) fail(CCM_E_NOMEM, "HBM budget exceeds half the free device memory");
    if (cfg && cfg->max_jobs > 0) s->max_jobs = cfg->max_jobs;
    if (cfg && cfg->epoch_target_ms > 0) s->epoch_ms = cfg->epoch_target_ms;
    budget = std::max<uint64_t>(budget, 1 << 20);
    s->arena.ensure(budget);
    s->arena_alloc.reset(budget);
    const uint64_t slots = std::max<uint64_t>(1 << 20, budget / 2048);
    s->slots_partial.ensure(slots * sizeof(Moments));
    s->slots_start.ensure(slots * 4 * kWaves);
    s->slot_alloc.reset(slots);
    const uint64_t rzc = std::max<uint64_t>(1 << 18, budget / 8192);
    s->rz_table.ensure(rzc * sizeof(Realization));
    s->rz_alloc.reset(rzc);
    s->items_cap = 1 << 20;
    for (int b = 0; b < 2; ++b) {
      s->items_dev[b].ensure(s->items_cap * sizeof(Item));
      HIPCHK(hipHostMalloc((void**)&s->items_host[b], s->items_cap * sizeof(Item),
                           hipHostMallocDefault));
      HIPCHK(hipEventCreate(&s->epoch_ev[b]));
      HIPCHK(hipEventCreate(&s->epoch_ev0[b]));
    }
    HIPCHK(hipStreamCreateWithFlags(&s->pstream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&s->fstream, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
      HIPCHK(hipStreamCreateWithFlags(&s->estream[b], hipStreamNonBlocking));
      HIPCHK(hipEventRecord(s->epoch_ev[b], s->estream[b]));   // waitable from the start
    }
    {
      hipDeviceProp_t prop;
      HIPCHK(hipGetDeviceProperties(&prop, c->device));
      s->min_items = (size_t)std::max(1, prop.multiProcessorCount) * 32;
    }
  } catch (const Fail& e) {
    {
      std::lock_guard<std::mutex> lock(c->mu);
      c->err = e.what;
    }
    for (int b = 0; b < 2; ++b) {
      if (s->items_host[b]) (void)hipHostFree(s->items_host[b]);
      if (s->epoch_ev[b]) (void)hipEventDestroy(s->epoch_ev[b]);
      if (s->epoch_ev0[b]) (void)hipEventDestroy(s->epoch_ev0[b]);
      if (s->estream[b]) (void)hipStreamDestroy(s->estream[b]);
    }
    if (s->pstream) (void)hipStreamDestroy(s->pstream);
    if (s->fstream) (void)hipStreamDestroy(s->fstream);
    return e.status;
  }
  ccm_server* raw = s.release();
  raw->worker = std::thread(scheduler_loop, raw);
  *out = raw;
  return CCM_OK;
}

ccm_status ccm_submit(ccm_server* s, const ccm_job* job, uint64_t* ticket) {
  if (!s || !job || !ticket) return CCM_E_INVAL;
  try {
    auto j = std::make_unique<Job>();
    if (!job->X || !job->Y) fail(CCM_E_INVAL, "NULL series");
    // options that change the draws are not served; the others only choose
    // an execution form, which the server picks itself
    if (job->opts.flags & (CCM_FLAG_NESTED | CCM_FLAG_SHARED_E))
      fail(CCM_E_INVAL, "nested libraries and E-sweep sharing are not served");
    Spec sp = make_spec(job->N, &job->E, 1, &job->tau, 1, job->L, job->nL, job->r, job->seed,
                        &job->opts);
    sp.flags &= CCM_FLAG_TABLE;   // execution forms are the server's; tables keep results
    check_host_series(job->X, job->N, "X");
    check_host_series(job->Y, job->N, "Y");
    j->plan = make_plan(sp);
    // every table lies in the job's pools (its rows, and the embedding its
    // rows are built from), so that rebasing keeps it in the job's region
    const Plan& p = j->plan;
    for (const TableJob& t : p.tables)
      if (t.emb_off < 0 || t.emb_off + (int64_t)t.n_e * t.E > p.n_emb || t.out_off < 0 ||
          t.out_off + (int64_t)t.n_e * table_row_stride(t.w) > p.n_table)
        fail(CCM_E_INVAL, "internal: a table outside the job's pools");
    for (const Realization& R : p.rz)
      if (R.table_off >= 0 && R.table_off >= p.n_table)
        fail(CCM_E_INVAL, "internal: a table offset outside the job's pools");
    j->lay = layout_of(j->plan);
    if (j->lay.bytes > s->arena_alloc.capacity() ||
        (uint64_t)j->plan.n_slots > s->slot_alloc.capacity() ||
        j->plan.rz.size() > s->rz_alloc.capacity())
      fail(CCM_E_NOMEM, "job needs " + std::to_string(j->lay.bytes) +
                            " device bytes, more than the server's budget");
    // pinned staging: the region's upload block, the realizations, the rho
    j->staging_rz = up(j->lay.upload, 256);
    j->staging_rho = up(j->staging_rz + j->plan.rz.size() * sizeof(Realization), 256);
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipHostMalloc((void**)&j->staging, j->staging_rho + j->plan.n_out * 8,
                         hipHostMallocDefault));
    j->rho_host = reinterpret_cast<double*>(j->staging + j->staging_rho);
    stage_job(*j, job->X, job->Y);
    HIPCHK(hipEventCreateWithFlags(&j->prep_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming));
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) fail(CCM_E_BUSY, "server is shutting down");
    j->ticket = s->next_ticket++;
    j->t_submit = s->now();
    *ticket = j->ticket;
    s->pending.push_back(j->ticket);
    s->jobs[j->ticket] = std::move(j);
    s->cv_work.notify_all();
    return CCM_OK;
  } catch (const Fail& e) {
    std::lock_guard<std::mutex> lock(s->ctx->mu);
    s->ctx->err = e.what;
    return e.status;
  } catch (const std::bad_alloc&) {
    return CCM_E_NOMEM;
  }
}

ccm_status ccm_wait(ccm_server* s, uint64_t ticket, int64_t timeout_ns) {
  if (!s) return CCM_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return CCM_E_NOTFOUND;
  Job* j = it->second.get();
  auto done = [&] { return j->retired; };
  if (timeout_ns < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
    return CCM_E_TIMEOUT;
  }
  return j->state == kDone ? CCM_OK : (j->state == kCancelled ? CCM_E_NOTFOUND : j->status);
}

ccm_status ccm_result(ccm_server* s, uint64_t ticket, double* rho_xy, double* rho_yx,
                      ccm_job_stats* stats) {
  if (!s) return CCM_E_INVAL;
  std::unique_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return CCM_E_NOTFOUND;
    // a cancelled job that is still active has device work in flight and
    // is still referenced by the scheduler: it is released only once retired
    if (!it->second->retired) return CCM_E_BUSY;
    j = std::move(it->second);
    s->jobs.erase(it);
  }
  const Plan& p = j->plan;
  const int64_t half = p.n_out / 2;
  if (j->state == kDone) {
    if (rho_xy) std::memcpy(rho_xy, j->rho_host, half * 8);
    if (rho_yx) std::memcpy(rho_yx, j->rho_host + half, half * 8);
  }
  if (stats) {
    stats->t_submit = j->t_submit;
    stats->t_admit = j->t_admit;
    stats->t_done = j->t_done;
    stats->pairs = (uint64_t)p.pairs;
    stats->predictions = (uint64_t)p.preds;
    stats->realizations = (uint64_t)p.rz.size();
    stats->device_bytes = j->lay.bytes;
  }
  (void)hipSetDevice(s->device);
  const ccm_status st = j->state == kDone ? CCM_OK
                        : (j->state == kCancelled ? CCM_E_NOTFOUND : j->status);
  j.reset();   // frees its pinned staging and events
  return st;
}

ccm_status ccm_cancel(ccm_server* s, uint64_t ticket) {
  if (!s) return CCM_E_INVAL;
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return CCM_E_NOTFOUND;
  Job& j = *it->second;
  if (j.state == kPending) {
    s->pending.erase(std::find(s->pending.begin(), s->pending.end(), ticket));
    j.state = kCancelled;
    j.t_done = s->now();
    j.retired = true;
    s->cv_done.notify_all();
  } else if (j.state == kActive) {
    j.state = kCancelled;   // remaining items are skipped; resources freed when idle
  }
  s->cv_work.notify_all();
  return CCM_OK;
}

void ccm_server_destroy(ccm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
    for (uint64_t t : s->pending) {
      s->jobs[t]->state = kCancelled;
      s->jobs[t]->retired = true;
    }
    s->pending.clear();
    for (uint64_t t : s->active) s->jobs[t]->state = kCancelled;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->pstream);
  (void)hipStreamSynchronize(s->fstream);
  for (int b = 0; b < 2; ++b)
    if (s->estream[b]) (void)hipStreamSynchronize(s->estream[b]);
  s->jobs.clear();   // frees each job's pinned staging and events
  for (int b = 0; b < 2; ++b) {
    if (s->items_host[b]) (void)hipHostFree(s->items_host[b]);
    if (s->epoch_ev[b]) (void)hipEventDestroy(s->epoch_ev[b]);
    if (s->epoch_ev0[b]) (void)hipEventDestroy(s->epoch_ev0[b]);
  }
  (void)hipStreamDestroy(s->pstream);
  (void)hipStreamDestroy(s->fstream);
  for (int b = 0; b < 2; ++b)
    if (s->estream[b]) (void)hipStreamDestroy(s->estream[b]);
  delete s;
}

}  // extern "C"

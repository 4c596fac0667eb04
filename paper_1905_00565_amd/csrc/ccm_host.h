// ccm_host.h -- host-side pieces of libccm shared by the runtime and the
// server: error handling, device buffers, call specifications and plans.
// Internal to libccm; the public boundary is include/ccm.h.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ccm.h"
#include "ccm_internal.h"

namespace ccmh {

using namespace ccmk;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

struct Fail {
  ccm_status status;
  std::string what;
};

[[noreturn]] inline void fail(ccm_status st, const std::string& what) { throw Fail{st, what}; }

inline void hip_check(hipError_t e, const char* expr) {
  if (e == hipSuccess) return;
  const ccm_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
                            ? CCM_E_NOMEM
                            : CCM_E_DEVICE;
  fail(st, std::string(expr) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr) hip_check((expr), #expr)

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 256;
    HIPCHK(hipMalloc(&p, n));
    bytes = n;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

template <class T>
void upload(DevBuf& b, const std::vector<T>& v) {
  b.ensure(v.size() * sizeof(T));
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

struct Spec {
  int32_t M = 0;      // 0: a pair of series (X, Y); M >= 2: causal matrix of M series
  int64_t N = 0;
  std::vector<int32_t> E, tau;
  std::vector<int64_t> L;
  int32_t r = 0;
  uint64_t seed = 0;
  int32_t excl = 0;
  int32_t query_set = 0;
  uint32_t flags = 0;
  // Largest device bytes of drawn libraries and gathered library points held
  // at once; the realizations are run in waves that fit (0: one wave).
  uint64_t wave_limit = 0;

  bool operator==(const Spec& o) const {
    return M == o.M && N == o.N && E == o.E && tau == o.tau && L == o.L && r == o.r &&
           seed == o.seed && excl == o.excl && query_set == o.query_set &&
           (flags & ~CCM_FLAG_NO_GRAPH) == (o.flags & ~CCM_FLAG_NO_GRAPH) &&
           wave_limit == o.wave_limit;
  }
};

inline int excl_mode(int32_t excl) {
  if (excl == 0) return kExclSelf;
  if (excl < 0) return kKeepSelf;
  return kWindow;
}

inline int64_t min_library(int32_t E, int32_t excl) {
  const int64_t w = excl < 0 ? 0 : 2 * (int64_t)excl + 1;
  return (int64_t)E + 1 + w;
}

// One cross-map launch: the work items of one E within a wave.
struct Launch {
  int32_t E;
  int32_t first;      // into Plan::items
  int32_t count;
};

// A wave: realizations whose drawn libraries and gathered points are live at
// once.  Its sample (or nested shuffle) jobs and gather jobs are contiguous
// ranges, its launches a contiguous range of Plan::launches; the library,
// gathered-point and shuffle pools are reused by every wave (the plan's
// n_lib, n_pts, n_pj and n_scratch are the largest wave's).
struct Wave {
  int64_t sample_first = 0, sample_count = 0;   // into sample, or nested
  int64_t gather_first = 0, gather_count = 0;
  int64_t max_sorted_n_e = 0;                   // largest n_e of its sorted gathers
  int32_t launch_first = 0, launch_count = 0;
  uint64_t pool_bytes = 0;
};

struct Plan {
  Spec spec;
  int mode = kExclSelf;
  int window = 0;
  std::vector<IngestJob> ingest;
  int64_t n64 = 0, n32 = 0;
  std::vector<EmbedJob> embed;
  int64_t n_emb = 0, max_embed = 0;
  int64_t n_qord = 0;                 // query-order entries (sum of n_e)
  std::vector<OrderJob> orders;       // order sets (each a sort segment of N)
  int32_t n_sets = 0;
  std::vector<int32_t> seg_off;       // segment offsets of the order sort
  int64_t n_ord = 0;                  // n_sets * N
  int32_t kd_levels = 0;              // k-d refinement levels (0: none)
  size_t sort_temp = 0;
  std::vector<SampleJob> sample;
  int64_t n_lib = 0;
  std::vector<GatherJob> gather;
  int64_t n_pts = 0;                  // floats of ordered library coordinates
  int64_t n_pj = 0;                   // ordered library indices
  int64_t max_sorted_n_e = 0;
  std::vector<Realization> rz;
  std::vector<int32_t> self_of;       // matrix: searched series of each realization
  // realization r uses sample job (or nested shuffle) rz_sample[r] and the
  // gather jobs from rz_gather[r] on (one, or one per segment of a chain)
  std::vector<int64_t> rz_sample;
  std::vector<int64_t> rz_gather;
  // waves of realizations (split_waves), and the batched items grouped by
  // wave, then E, longest library first within a group
  std::vector<Wave> waves;
  std::vector<Launch> launches;
  std::vector<int32_t> wave_rz;       // realizations in wave order
  std::vector<int64_t> wave_rz_first; // per wave, into wave_rz (+1 sentinel)
  std::vector<Item> items;
  int64_t n_slots = 0;
  int64_t n_out = 0;
  std::vector<int64_t> L_eff;   // per (iE, itau, iL)
  double pairs = 0, flops = 0, preds = 0;
  size_t device_bytes = 0;
  // distance indexing tables (CCM_FLAG_TABLE), grouped by E
  std::vector<TableJob> tables;
  int64_t n_table = 0;                // int32 entries of every table
  int te_first[kMaxE + 1] = {0};
  int te_count[kMaxE + 1] = {0};
  int te_max_ne[kMaxE + 1] = {0};     // largest table of E (launch grid)
  int e_table_ne[kMaxE + 1] = {0};    // largest n_e walked by E's items (launch LDS)
  int64_t table_rz = 0;               // realizations that walk a table
  // nested libraries (CCM_FLAG_NESTED): rz holds chains, rz_fin one record
  // per rho (slot range of its segment, output index)
  std::vector<NestedJob> nested;
  int64_t n_scratch = 0;              // int32 shuffle positions
  std::vector<int32_t> segs;          // segment bounds of every chain
  std::vector<Realization> rz_fin;
  int64_t n_rho = 0;                  // rho values produced
  // E-sweep sharing (CCM_FLAG_SHARED_E): rz holds one scan per (tau, L, r,
  // direction) at E_max, rz_fin one record per rho
  int32_t shared_emax = 0;
};

// Whether a realization walks a distance indexing table, and the offset of
// that table (created on first use for the embedding at emb_off).
bool use_table(const Plan& p, int E, int64_t ne, int64_t le);
int64_t table_for(Plan& p, int64_t emb_off, int64_t ne, int E);

// The key of an order set: dims and lags as in OrderJob; kd_E > 0 asks for
// the k-d refinement over the E coordinates of the embedding the set is
// attached to (attach_kd).
struct OrderKey {
  int32_t dims;
  int32_t lag[4];
  int32_t kd_E = 0;
};
// Visiting order of the embedding of dimension E with delay tau: the value
// order for E = 1, a Hilbert curve over the two coordinates for E = 2, and
// from E = 3 a k-d order over all E coordinates (one set per embedding).
OrderKey embedding_order(int32_t E, int32_t tau);
// The embedding (at emb_off, n_e points) whose coordinates refine the order
// set at key_off, when the set asks for a k-d refinement; also sets the
// plan's number of refinement levels.
void attach_kd(Plan& p, int64_t key_off, int32_t E, int64_t emb_off, int64_t ne);
// hipcub's scratch for the plan's order sort.
void size_order_sort(Plan& p);
// E-sweep sharing: visiting order of E_max's common points, keyed on the
// newest lag coordinates (the ones every E of the sweep uses): the two
// newest, or for E_max >= 8 (where the long lists of the large E dominate)
// a 4-dimensional curve over the four newest.
OrderKey shared_order(int32_t Emax, int32_t tau);
// Order set of (series, key), created on first use; returns its offset in
// the order pool.
int64_t order_set(Plan& p, int series, const OrderKey& key);

// Validate a sweep (pair of series, E x tau grid) and lay out every
// realization of it.
Plan make_plan(const Spec& s);
// Causal matrix: M series, one (E, tau); libraries per (L, r) shared by every
// series; one realization per (searched series, L, r) predicting all others.
Plan make_plan_matrix(const Spec& s);

// Default wave limit of a device with `total` bytes of memory.
uint64_t default_wave_limit(uint64_t total);

// Host series: finite and |value| <= 1e17 (keeps binary32 d2 finite).
void check_host_series(const double* s, int64_t n, const char* name);

// A call's specification from C-ABI arguments (validation happens when the
// plan is made).
Spec make_spec(int64_t N, const int32_t* E, int32_t nE, const int32_t* tau, int32_t ntau,
               const int64_t* L, int32_t nL, int32_t r, uint64_t seed, const ccm_opts* opts);

}  // namespace ccmh

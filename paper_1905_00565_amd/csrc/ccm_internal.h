// ccm_internal.h -- descriptors shared by the library's host runtime and its
// gfx950 kernels.  Internal to libccm; the public boundary is include/ccm.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmk {

constexpr int kMaxE = 10;          // simplex embedding dimension range is 1..10
constexpr int kBlock = 256;        // threads per workgroup of the cross-map kernel
constexpr int kWaves = kBlock / 64; // wavefronts per workgroup (one scan start each)

// Exclusion handling of the cross-map kernel (compile-time variants).
enum ExclMode : int {
  kExclSelf = 0,    // drop the query itself (rejected when it would be inserted)
  kKeepSelf = 1,    // every library point is a candidate
  kWindow = 2,      // drop candidates with |j - i| <= w (per-pair mask)
};

// One ingest copy: double series -> float series (round to nearest even).
struct IngestJob {
  int64_t src_off;   // doubles into the FP64 series pool
  int64_t dst_off;   // floats into the FP32 series pool
  int64_t n;
};

// One visiting order of a series' embedded points (an "order set"): indices
// i sorted by a key computed from a few values of the series at fixed time
// offsets ("lags") from i -- the time of embedded point i's oldest lag
// coordinate, so one set serves every embedding whose coordinates include
// those times; each embedding keeps the indices below its own n_e.
//   dims == 1: the value S[i + lag[0]];
//   dims == 2: the position on a Hilbert curve over (S[i + lag[0]],
//              S[i + lag[1]]), each scaled to 16 bits by the series' range;
//   dims == 3, 4: the position on the dims-dimensional Hilbert curve over
//              S[i + lag[d]], each scaled to 32 / dims bits.
// An index whose lags run past the series sorts last (it is never an
// embedded point of an embedding that uses the set).
//
// A set with kd_E > 0 belongs to one embedding (kd_E coordinates, kd_n_e
// points at kd_emb_off): after the sort above (dims == 1 on its newest lag
// coordinate, so its first kd_n_e entries are the embedded points), its
// order is refined into a k-d order -- the points are split at the median of
// their widest coordinate, the halves again, for kd_levels levels -- so that
// points close in all E coordinates are close in the order.
struct OrderJob {
  int64_t src_off;   // floats into the FP32 series pool
  int64_t key_off;   // uint32 keys (and the sorted order) of this set
  int64_t n;         // series length
  int32_t dims;
  int32_t lag[4];
  int32_t kd_E;      // 0: no k-d refinement
  int64_t kd_emb_off;  // floats into the embedding pool
  int64_t kd_n_e;
  int32_t kd_levels; // levels of this set's refinement (from its n_e alone)
  int32_t pad;
};

// One embedding of one series.
//   emb[i*E + k] = s[i + (E-1)tau - k tau]           (AoS float [n_e][E])
//   qord[p]      = embedded points in the visiting order of the set
struct EmbedJob {
  int64_t src_off;   // floats into the FP32 series pool
  int64_t dst_off;   // floats into the embedding pool
  int64_t order_off; // int32 into the order pool (its order set, n_series entries)
  int64_t qord_off;  // int32 into the query-order pool (n_e entries)
  int64_t n_e;
  int64_t n_series;
  int32_t E;
  int32_t tau;
};

// One library draw (selection sampling keyed by (seed, E, tau, L_eff, r)).
struct SampleJob {
  uint64_t seed;
  int64_t n_e;
  int64_t l_eff;
  int64_t out_off;   // int32 indices into the library pool
  int32_t E;
  int32_t tau;
  int32_t r_index;
  int32_t pad;
};

// One library gather: the library of one realization laid out in visiting
// order (pts AoS [l_eff][E], pj the embedded index
// of each), plus the library position each query tile starts scanning from.
struct GatherJob {
  int64_t emb_off;   // floats: embedding of the library series
  int64_t lib_off;   // int32: library indices (ascending index order)
  int64_t order_off; // int32: order set of the library embedding
  int64_t pts_off;   // floats: output coordinates
  int64_t pj_off;    // int32: output embedded indices
  int64_t start_off; // int32: output scan start per wavefront of each query tile
  int64_t l_eff;
  int64_t n_e;
  int64_t n_series;
  int32_t E;
  int32_t tau;
  int32_t qt;        // queries per tile
  int32_t query_set; // 0: every embedded point is a query
  int32_t sorted;    // 0: keep ascending index order (no series order)
  int32_t pad;
};

// One realization: a library drawn over one embedding, predicting one target.
struct Realization {
  int64_t emb_off;   // floats: AoS embedding of the library series
  int64_t pts_off;   // floats: ordered library coordinates, AoS [l_eff][E]
  int64_t pj_off;    // int32: ordered library embedded indices
  int64_t qord_off;  // int32: query order of the embedding
  int64_t tgt_off;   // doubles: FP64 target series (time 0)
  int32_t E;
  int32_t tau;
  int32_t n_e;       // embedded points of the library series
  int32_t l_eff;     // library size
  int32_t n_query;   // queries: n_e, or l_eff when only library points are queried
  int32_t n_tiles;   // query tiles (= work items) of this realization
  int64_t slot_base; // first partial-moment slot (one per tile; scan starts kWaves per slot)
  int64_t out_index; // where rho goes in the caller's output
  int64_t table_off; // int32: distance-index rows of the embedding, or -1 (brute force)
  int32_t table_w;   // entries per table row (min(CCM_TABLE_WIDTH, n_e))
  int32_t n_seg;     // nested libraries: segments (library sizes) of this chain, else 0
  int64_t seg_off;   // int32: n_seg + 1 segment bounds (nested libraries)
};

// One nested ordering: the first n_out points of a forward Fisher-Yates
// shuffle of 0..n_e-1 (stream keyed by (seed, E, tau, r_index)), written to
// out; scratch holds the n_e positions being shuffled.
struct NestedJob {
  uint64_t seed;
  int64_t n_e;
  int64_t n_out;
  int64_t out_off;      // int32 into the library pool
  int64_t scratch_off;  // int32 into the shuffle scratch
  int32_t E;
  int32_t tau;
  int32_t r_index;
  int32_t pad;
};

// One distance indexing table: for each embedded point i of one embedding,
// row i = the first w embedded points j (self included) in ascending
// (d2(i, j), j) order, with d2 the kernel's binary32 distance.
struct TableJob {
  int64_t emb_off;   // floats: AoS embedding
  int64_t out_off;   // int32: rows [n_e][w]
  int64_t row0;      // first global row of this table (rows are launched flat)
  int32_t n_e;
  int32_t E;
  int32_t w;
  int32_t pad;
};

// A work item: one query tile of one realization.
struct Item {
  int32_t rz;
  int32_t tile;
};

// Pearson moments of one query tile: count, means, centred sums (Welford).
struct Moments {
  double n, mt, mp, m2t, m2p, c;
};

// Optional per-query dump (test hook), rows indexed by embedded point;
// nbr == nullptr means none.
struct Dump {
  int32_t* nbr;   // [n_e][E+1]
  float* d2;      // [n_e][E+1]
  double* pred;   // [n_e]
};

// Launchers (defined with the kernels).
// Queries per lane of the cross-map kernel of E (a tile holds kBlock times
// as many); the same for batched launches and the per-query hook.
int crossmap_queries_per_lane(int E);
// E-sweep sharing: queries per lane of the scan at E_max (its key registers
// grow as E_max^2, so this falls with E_max).
int shared_queries_per_lane(int emax);
hipError_t launch_ingest(const IngestJob* jobs, int n_jobs, int64_t max_n,
                         const double* src, float* dst, hipStream_t st);
hipError_t launch_embed(const EmbedJob* jobs, int n_jobs, int64_t max_n,
                        const float* s32, float* emb, hipStream_t st);
hipError_t launch_iota_segments(int32_t* out, int64_t n_series, int32_t segs,
                                hipStream_t st);
hipError_t launch_order_keys(const OrderJob* jobs, int n_jobs, const float* s32,
                             uint32_t* keys, hipStream_t st);
hipError_t launch_query_order(const EmbedJob* jobs, int n_jobs,
                              const int32_t* order, int32_t* qord, hipStream_t st);
hipError_t launch_sample(const SampleJob* jobs, int64_t n_jobs, int32_t* out,
                         hipStream_t st);
hipError_t launch_gather(const GatherJob* jobs, int64_t n_jobs, int64_t max_n_e,
                         const float* emb, const int32_t* lib, const int32_t* order,
                         float* pts, int32_t* pj, int32_t* start, hipStream_t st);
hipError_t launch_zero_int(int* p, int n, hipStream_t st);
// d.nbr == nullptr: no per-query export; else (the hook) d.nbr, d.d2 and
// d.pred are all set and the kernel instance that exports them runs.
hipError_t launch_crossmap(int E, int mode, int grid,
                           const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb,
                           const float* pts, const int32_t* pj,
                           const int32_t* qord, const int32_t* start,
                           const double* tgt, Moments* partial, int query_set,
                           int window, Dump d, const int32_t* table, int table_n_e,
                           hipStream_t st);
// Distance indexing tables (Section 3.2), one launch per E: grid
// (max_n_e, n_jobs); rows of job k at table + jobs[k].out_off.
hipError_t launch_table_build(int E, const TableJob* jobs, int n_jobs, int max_n_e,
                              const float* emb, int32_t* table, hipStream_t st);
constexpr int kTableWidth = 1024;           // CCM_TABLE_WIDTH
constexpr int kTableMaxNe = 131072;         // largest embedding given a table (LDS bitmask)
constexpr int table_row_stride(int w) { return (w + 3) & ~3; }
// Nested libraries: the shuffles (one workgroup per job), and the cross map
// of chains (one realization per (E, tau, r, direction) holding every
// library size as a segment; partial slot of segment k, tile t:
// slot_base + k * n_tiles + t; scan starts likewise, kWaves per slot).
hipError_t launch_sample_nested(const NestedJob* jobs, int64_t n_jobs, int32_t* scratch,
                                int32_t* out_pool, hipStream_t st);
hipError_t launch_crossmap_nested(int E, int mode, int grid, const Realization* rzs,
                                  const Item* items, int n_items, int* next,
                                  const float* emb, const float* pts, const int32_t* pj,
                                  const int32_t* qord, const int32_t* start, const double* tgt,
                                  const int32_t* seg, Moments* partial, int window,
                                  hipStream_t st);
// E-sweep sharing: chains over E_max's embedding, one list per E <= emax;
// partial slot of E, tile t: slot_base + (E-1) * n_tiles + t; tiles of
// kBlock * shared_queries_per_lane(emax) queries, scan starts kWaves per tile.
hipError_t launch_crossmap_shared(int emax, int mode, int grid, const Realization* rzs,
                                  const Item* items, int n_items, int* next,
                                  const float* emb, const float* pts, const int32_t* pj,
                                  const int32_t* qord, const int32_t* start, const double* tgt,
                                  Moments* partial, int window, hipStream_t st);
hipError_t launch_finalize(const Realization* rzs, int64_t n_rz,
                           const Moments* partial, double* out, hipStream_t st);

// Causal-matrix form: one neighbour search per realization predicts every
// series; self_of[rz] is the searched series (its own target is skipped).
// partial holds one record of multi_sums_bytes() per (item slot, series).
// Targets come time-major: tt[t * mp + b] = series b at time t, with
// mp = target_stride(m_series) columns (a zero pad column when m is odd).
hipError_t launch_crossmap_multi(int E, int mode, int grid, const Realization* rzs,
                                 const int32_t* self_of, const Item* items, int n_items,
                                 int* next, const float* emb, const float* pts,
                                 const int32_t* pj, const int32_t* qord, const int32_t* start,
                                 const double* tt, int m_series,
                                 void* partial, int query_set, int window,
                                 const int32_t* table, int table_n_e, hipStream_t st);
constexpr int target_stride(int m_series) { return (m_series + 1) & ~1; }
// tt[t * mp + b] = s64[b * n + t] for b < m, 0 in the pad column.
hipError_t launch_transpose_targets(const double* s64, int m_series, int64_t n, double* tt,
                                    hipStream_t st);
hipError_t launch_finalize_multi(const Realization* rzs, const int32_t* self_of,
                                 int64_t n_rz, int m_series, const void* partial,
                                 int64_t out_stride_b, double* out, hipStream_t st);
size_t multi_sums_bytes();

// Order sets (ccm_sort.hip): per segment of n_series keys, the time indices
// sorted by key (stable).  temp_bytes is queried with temp == nullptr.
hipError_t sort_series(void* temp, size_t& temp_bytes, const uint32_t* keys_in,
                       uint32_t* keys_out, const int32_t* idx_in, int32_t* idx_out,
                       int64_t n_series, int32_t segs, const int32_t* seg_offsets,
                       hipStream_t st);

// k-d refinement of the order sets with kd_E > 0 (see OrderJob), on the
// order pool of n_sets segments of n_series entries: `order` holds the
// sorted sets on entry and the refined ones on return; alt and keys (the
// size of the pool) are scratch.  Only kernels of this library run (no
// library sort: the sequence is captured in graphs and replayed).
hipError_t refine_orders_kd(const OrderJob* orders, int32_t n_sets, int levels,
                            int64_t n_series, const float* emb, int32_t* order, int32_t* alt,
                            uint32_t* keys, hipStream_t st);

// Largest embedding whose membership bitmask fits the gather kernel's LDS.
int64_t gather_max_sorted_n_e();

}  // namespace ccmk

// ccm_device.h -- device-side templates of the cross-map kernels (one
// translation unit per embedding dimension instantiates them, see
// ccm_inst.hip): candidate keys, Pearson moments, the fused cross-map item
// and its scan, the distance indexing table, nested libraries, E-sweep
// sharing, and the kernels' entry points.
//
// Arithmetic that must agree bit for bit with the CPU oracle:
//   d2 = sum_k (q_k - p_k)^2 in binary32 as acc = fma(diff, diff, acc),
//   k ascending from acc = +0 (the first term is the plain product, which is
//   the same value), no other contraction (-ffp-contract=off);
//   neighbours are the first E+1 candidates in (d2, j) order.
#pragma once
#include "ccm_internal.h"
#include "ccm_tune.h"

namespace ccmk {

// Exclusive rank of this thread among the flagged threads of its 256-thread
// workgroup, and the workgroup total, in thread order.
__device__ __forceinline__ int block_rank(bool flag, int* s_wave, int& total) {
  const uint64_t m = __builtin_amdgcn_ballot_w64(flag);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int r = __popcll(m & lt);
  if (lane == 0) s_wave[wave] = __popcll(m);
  __syncthreads();
  int before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const int c = s_wave[w];
    if (w < wave) before += c;
    total += c;
  }
  __syncthreads();
  return before + r;
}

// ---------------------------------------------------------------------------
// candidate keys
// ---------------------------------------------------------------------------
//
// A candidate (d2, j) is kept as one 64-bit word: high half the binary32 bits
// of d2, low half its embedded index j.  For d2 >= 0 the bit patterns of
// binary32 order like the values, so the word read as an unsigned integer
// orders exactly like (d2, j) lexicographically.  The same word read as a
// binary64 is a non-negative number (denormal when d2 is 0 or tiny, never
// NaN: the high
// exponent field is at most 0x7f8), and non-negative binary64 values also
// order like their bit patterns -- so the FP64 min/max units keep a sorted
// list of keys, two instructions per slot.  FP64 denormals are preserved in
// the kernel's float mode, which this relies on.

__device__ __forceinline__ double make_key(float d2, int32_t j) {
  return __hiloint2double(__float_as_int(d2), j);
}
__device__ __forceinline__ float key_d2(double k) {
  return __int_as_float(__double2hiint(k));
}
__device__ __forceinline__ int32_t key_j(double k) { return __double2loint(k); }

// Issued directly so the compiler does not quiet-NaN-canonicalise operands
// that can never be NaN (see above).
__device__ __forceinline__ double kmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double kmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Insert c into the ascending list key[0..KS-1], dropping the largest.
// New slot m is the median of (old m-1, c, old m).  A c above the last key
// leaves the list unchanged.
template <int KS>
__device__ __forceinline__ void insert_key(double (&key)[KS], double c) {
#pragma unroll
  for (int m = KS - 1; m >= 1; --m) key[m] = kmin(kmax(key[m - 1], c), key[m]);
  key[0] = kmin(key[0], c);
}

// Empty slot: +inf distance, index above any real one.
__device__ __forceinline__ double empty_key() {
  return __hiloint2double(0x7f800000, -1);
}

template <int E>
__device__ __forceinline__ float sqdist(const float (&q)[E], const float* p) {
  float d = q[0] - p[0];
  float acc = d * d;
#pragma unroll
  for (int k = 1; k < E; ++k) {
    d = q[k] - p[k];
    acc = __builtin_fmaf(d, d, acc);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Pearson moments (Welford / Chan)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void mom_add(Moments& a, double t, double p) {
  a.n += 1.0;
  const double dt = t - a.mt;
  const double dp = p - a.mp;
  a.mt += dt / a.n;
  a.mp += dp / a.n;
  a.m2t += dt * (t - a.mt);
  a.m2p += dp * (p - a.mp);
  a.c += dt * (p - a.mp);
}

__device__ __forceinline__ Moments mom_merge(const Moments& a, const Moments& b) {
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  Moments r;
  r.n = a.n + b.n;
  const double dt = b.mt - a.mt;
  const double dp = b.mp - a.mp;
  const double f = a.n * b.n / r.n;
  r.mt = a.mt + dt * (b.n / r.n);
  r.mp = a.mp + dp * (b.n / r.n);
  r.m2t = a.m2t + b.m2t + dt * dt * f;
  r.m2p = a.m2p + b.m2p + dp * dp * f;
  r.c = a.c + b.c + dt * dp * f;
  return r;
}

// ---------------------------------------------------------------------------
// the fused cross-map item
// ---------------------------------------------------------------------------

// Library candidates per trigger check (tuned per E); the group's
// coordinates (G*E values, uniform across the wavefront) come through the
// scalar cache into SGPRs.
template <int E>
struct Group {
  static constexpr int G = kTuneG[E];
};

// Running list length: the E+1 neighbours.  With self excluded the query
// itself is rejected when it would be inserted, so it never takes a slot.
template <int E, int MODE>
struct Slots {
  static constexpr int KS = E + 1;
};

// G consecutive library candidates (uniform across the wavefront: loaded
// through the scalar cache into SGPRs).
template <int E, int G>
struct Chunk {
  float p[G][E];
  int32_t j[G];
};

template <int E, int G>
__device__ __forceinline__ void load_chunk(Chunk<E, G>& ch, const float* __restrict__ pts,
                                           const int32_t* __restrict__ pj, int c) {
  // one base address per chunk: the G*E coordinates and G indices are
  // contiguous, so the loads merge into a few wide scalar loads with
  // immediate offsets
  const float* __restrict__ p = pts + (int64_t)c * E;
  const int32_t* __restrict__ q = pj + c;
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int k = 0; k < E; ++k) ch.p[g][k] = p[g * E + k];
    ch.j[g] = q[g];
  }
}

// Make the chunk's values available at this point (the wait for its scalar
// loads happens here, before anything issued after it).
template <int E, int G>
__device__ __forceinline__ void settle_chunk(const Chunk<E, G>& ch) {
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int k = 0; k < E; ++k) asm volatile("" ::"s"(ch.p[g][k]));
    asm volatile("" ::"s"(ch.j[g]));
  }
}

// Distances from the lane's queries to the chunk's candidates, then one
// compare per query against its running (KS)-th best; only when some lane
// of the wavefront qualifies are the candidates inserted.
template <int E, int Q, int MODE, int G>
__device__ __forceinline__ void compute_chunk(
    const Chunk<E, G>& ch, const float (&qc)[Q][E], const int (&qi)[Q], int window,
    double (&key)[Q][Slots<E, MODE>::KS]) {
  constexpr int KS = Slots<E, MODE>::KS;
  float d2[G][Q];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      float v = sqdist<E>(qc[m], ch.p[g]);
      if (MODE == kWindow) {
        const int dj = ch.j[g] - qi[m];
        if (dj <= window && dj >= -window) v = __builtin_nanf("");
      }
      d2[g][m] = v;
    }
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    float mn = d2[0][m];
#pragma unroll
    for (int g = 1; g < G; ++g) mn = fminf(mn, d2[g][m]);
    if (__builtin_amdgcn_ballot_w64(mn <= key_d2(key[m][KS - 1]))) {
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (d2[g][m] <= key_d2(key[m][KS - 1]) && (MODE != kExclSelf || ch.j[g] != qi[m]))
          insert_key<KS>(key[m], make_key(d2[g][m], ch.j[g]));
    }
  }
}

// Small E: a cheaper group check with the same outcome.  Each step of the
// binary32 chain adds a non-negative term, and rounding is monotone, so a
// pair's d2 is at least fl(d_k * d_k) for every coordinate k, that is at least
// fl(m * m) with m the largest |d_k|; a group none of whose candidates has
// fl(m * m) <= the running (E+1)-th key has no candidate to insert.  The check
// costs E subtractions, E-1 maxima and half a three-way minimum per pair (at
// E = 1 the bound is d2 itself: fl(d * d) does not decrease with |d|); a group
// that passes recomputes its exact d2 (the same values) and inserts as the
// default check does.
template <int E, int Q, int MODE, int G>
__device__ __forceinline__ void compute_chunk_bound(
    const Chunk<E, G>& ch, const float (&qc)[Q][E], const int (&qi)[Q], int window,
    double (&key)[Q][Slots<E, MODE>::KS]) {
  constexpr int KS = Slots<E, MODE>::KS;
  float a[Q];
#pragma unroll
  for (int m = 0; m < Q; ++m) a[m] = __builtin_inff();
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      float v = fabsf(qc[m][0] - ch.p[g][0]);
#pragma unroll
      for (int k = 1; k < E; ++k) v = fmaxf(v, fabsf(qc[m][k] - ch.p[g][k]));
      if (MODE == kWindow) {
        const int dj = ch.j[g] - qi[m];
        if (dj <= window && dj >= -window) v = __builtin_nanf("");
      }
      a[m] = fminf(a[m], v);
    }
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    if (__builtin_amdgcn_ballot_w64(a[m] * a[m] <= key_d2(key[m][KS - 1]))) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const float d2 = sqdist<E>(qc[m], ch.p[g]);
        bool ok = d2 <= key_d2(key[m][KS - 1]);
        if (MODE == kExclSelf) ok = ok && ch.j[g] != qi[m];
        if (MODE == kWindow) {
          const int dj = ch.j[g] - qi[m];
          ok = ok && (dj > window || dj < -window);
        }
        if (ok) insert_key<KS>(key[m], make_key(d2, ch.j[g]));
      }
    }
  }
}

template <int E, int Q, int MODE, int G>
__device__ __forceinline__ void check_chunk(
    const Chunk<E, G>& ch, const float (&qc)[Q][E], const int (&qi)[Q], int window,
    double (&key)[Q][Slots<E, MODE>::KS]) {
  if constexpr (kBoundCheck[E] != 0)
    compute_chunk_bound<E, Q, MODE, G>(ch, qc, qi, window, key);
  else
    compute_chunk<E, Q, MODE, G>(ch, qc, qi, window, key);
}

template <int E, int Q, int MODE, int G>
__device__ __forceinline__ void scan_group(
    const float* __restrict__ pts, const int32_t* __restrict__ pj, int c,
    const float (&qc)[Q][E], const int (&qi)[Q], int window,
    double (&key)[Q][Slots<E, MODE>::KS]) {
  Chunk<E, G> ch;
  load_chunk<E, G>(ch, pts, pj, c);
  check_chunk<E, Q, MODE, G>(ch, qc, qi, window, key);
}

// Queries of one item and their running candidate lists after the scan of
// the whole library.
template <int E, int Q, int MODE>
struct ScanState {
  float qc[Q][E];
  int qi[Q];
  double key[Q][Slots<E, MODE>::KS];
};

// ---------------------------------------------------------------------------
// distance indexing table (Section 3.2)
// ---------------------------------------------------------------------------
//
// The walk of a query's table row: the first E+1 library members that are
// not excluded, in the row's (d2, j) order, are exactly the E+1 neighbours
// the brute-force scan selects (every candidate before them in the row is
// either outside the library or excluded, and every candidate after them is
// larger in (d2, j)).  Their keys are recomputed from the coordinates with
// the same binary32 chain, so the running lists end identical.  The library
// is a membership bitmask in LDS (built per item), the accepted indices go to
// a per-lane LDS slot array.  Returns false when some lane of the wavefront
// reached the end of a row short of E+1 members (the caller then scans).

struct TableArgs {
  const int32_t* pool;  // int32 rows of every table
  int32_t words;        // bitmask words in dynamic LDS (0: no table in this launch)
  int32_t pad;
};

__device__ __forceinline__ int table_stride(int w) { return (w + 3) & ~3; }

template <int E, int Q, int MODE>
__device__ __forceinline__ bool walk_table(const Realization& R, const int32_t* __restrict__ table,
                                           const uint32_t* __restrict__ bits,
                                           int32_t* __restrict__ acc,
                                           const float* __restrict__ emb, int window,
                                           ScanState<E, Q, MODE>& S) {
  constexpr int K = E + 1;
  const int rs = table_stride(R.table_w);
  bool ok = true;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int qi = S.qi[m];
    int cnt = qi >= 0 ? 0 : K;
    if (qi >= 0) {
      const int4* __restrict__ row =
          reinterpret_cast<const int4*>(table + R.table_off + (int64_t)qi * rs);
      for (int p = 0; p < rs / 4 && cnt < K; ++p) {
        const int4 v = row[p];
        const int js[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = js[u];
          bool keep = cnt < K && j >= 0 && ((bits[j >> 5] >> (j & 31)) & 1u);
          if (MODE == kExclSelf) keep = keep && j != qi;
          if (MODE == kWindow) keep = keep && (j - qi > window || qi - j > window);
          if (keep) {
            acc[cnt * kBlock + threadIdx.x] = j;
            ++cnt;
          }
        }
      }
      if (cnt == K) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const int j = acc[t * kBlock + threadIdx.x];
          S.key[m][t] = make_key(sqdist<E>(S.qc[m], emb + (int64_t)j * E), j);
        }
      }
    }
    ok = ok && cnt == K;
  }
  return !__builtin_amdgcn_ballot_w64(!ok);
}

// Library membership bitmask of realization R in LDS (whole workgroup).
__device__ __forceinline__ void table_bitmask(const Realization& R,
                                              const int32_t* __restrict__ pj_pool,
                                              uint32_t* bits) {
  const int words = (R.n_e + 31) / 32;
  for (int w = threadIdx.x; w < words; w += kBlock) bits[w] = 0u;
  __syncthreads();
  const int32_t* __restrict__ pj = pj_pool + R.pj_off;
  for (int c = threadIdx.x; c < R.l_eff; c += kBlock) {
    const int j = pj[c];
    atomicOr(&bits[j >> 5], 1u << (j & 31));
  }
  __syncthreads();
}

// Queries of this lane for item (R, tile): positions tile*QT + wave*QW +
// m*64 + lane of the query order (every embedded point, or the ordered
// library itself), so that each wavefront holds a run of QW consecutive
// queries.  Their lists start empty.  Returns whether the lane's wavefront
// has any query (uniform across the wavefront).
template <int E, int Q, int MODE>
__device__ __forceinline__ bool scan_queries(const Realization& R, int tile, int wave, int lane,
                                             const float* __restrict__ emb,
                                             const int32_t* __restrict__ pj,
                                             const int32_t* __restrict__ qord, int query_set,
                                             ScanState<E, Q, MODE>& S) {
  constexpr int KS = Slots<E, MODE>::KS;
  constexpr int QT = kBlock * Q;
  constexpr int QW = 64 * Q;
  bool any = false;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int qq = tile * QT + wave * QW + m * 64 + lane;
    const bool valid = qq < R.n_query;
    any |= valid;
    const int i = valid ? (query_set ? pj[qq] : qord[qq]) : 0;
    S.qi[m] = valid ? i : -1;
#pragma unroll
    for (int k = 0; k < E; ++k) S.qc[m][k] = emb[(int64_t)i * E + k];
  }
#pragma unroll
  for (int m = 0; m < Q; ++m)
#pragma unroll
    for (int s = 0; s < KS; ++s) S.key[m][s] = empty_key();
  return __builtin_amdgcn_ballot_w64(any) != 0;
}

// Brute-force scan of the library positions [0, L) (coordinates pts AoS,
// indices pj), outward from s0: a forward group [f, f+G) and a backward
// group [b-G, b) per step while both fit, then the remaining groups of the
// longer side, then single positions at both ends.  Every position is
// visited once; the lists keep the first E+1 candidates in (d2, j) order.
template <int E, int Q, int MODE>
__device__ __forceinline__ void scan_range(const float* __restrict__ pts,
                                           const int32_t* __restrict__ pj, int L, int s0,
                                           int window, ScanState<E, Q, MODE>& S) {
  constexpr int G = Group<E>::G;
  s0 = min(max(s0, 0), L);
  int f = s0, b = s0;
  const int both = min((L - s0) / G, s0 / G);
  // Software pipeline over the scalar loads: a chunk's loads are issued one
  // chunk ahead, and each chunk is waited for before the next is requested
  // (scalar loads return out of order, so a wait covers all that are
  // outstanding).
  if (both > 0) {
    Chunk<E, G> A, B;
    load_chunk<E, G>(A, pts, pj, f);
    for (int k = 0; k < both; ++k) {
      settle_chunk<E, G>(A);
      __builtin_amdgcn_sched_barrier(0);
      load_chunk<E, G>(B, pts, pj, b - G);
      __builtin_amdgcn_sched_barrier(0);
      check_chunk<E, Q, MODE, G>(A, S.qc, S.qi, window, S.key);
      f += G;
      settle_chunk<E, G>(B);
      __builtin_amdgcn_sched_barrier(0);
      load_chunk<E, G>(A, pts, pj, k + 1 < both ? f : f - G);
      __builtin_amdgcn_sched_barrier(0);
      check_chunk<E, Q, MODE, G>(B, S.qc, S.qi, window, S.key);
      b -= G;
    }
  }
  // The one-sided remainder (the longer side), pipelined the same way over
  // consecutive groups of that side; a last request with no group after it
  // re-reads the current group (in bounds, never used).
  if constexpr (kPipeRest[E] != 0) {
    const int nf = (L - f) / G;
    if (nf > 0) {
      Chunk<E, G> A, B;
      load_chunk<E, G>(A, pts, pj, f);
      int k = 0;
      for (; k + 1 < nf; k += 2) {
        settle_chunk<E, G>(A);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk<E, G>(B, pts, pj, f + G);
        __builtin_amdgcn_sched_barrier(0);
        check_chunk<E, Q, MODE, G>(A, S.qc, S.qi, window, S.key);
        f += G;
        settle_chunk<E, G>(B);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk<E, G>(A, pts, pj, k + 2 < nf ? f + G : f);
        __builtin_amdgcn_sched_barrier(0);
        check_chunk<E, Q, MODE, G>(B, S.qc, S.qi, window, S.key);
        f += G;
      }
      if (k < nf) {
        settle_chunk<E, G>(A);
        __builtin_amdgcn_sched_barrier(0);
        check_chunk<E, Q, MODE, G>(A, S.qc, S.qi, window, S.key);
        f += G;
      }
    }
    const int nb = b / G;
    if (nb > 0) {
      Chunk<E, G> A, B;
      load_chunk<E, G>(A, pts, pj, b - G);
      int k = 0;
      for (; k + 1 < nb; k += 2) {
        settle_chunk<E, G>(A);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk<E, G>(B, pts, pj, b - 2 * G);
        __builtin_amdgcn_sched_barrier(0);
        check_chunk<E, Q, MODE, G>(A, S.qc, S.qi, window, S.key);
        b -= G;
        settle_chunk<E, G>(B);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk<E, G>(A, pts, pj, k + 2 < nb ? b - 2 * G : b - G);
        __builtin_amdgcn_sched_barrier(0);
        check_chunk<E, Q, MODE, G>(B, S.qc, S.qi, window, S.key);
        b -= G;
      }
      if (k < nb) {
        settle_chunk<E, G>(A);
        __builtin_amdgcn_sched_barrier(0);
        check_chunk<E, Q, MODE, G>(A, S.qc, S.qi, window, S.key);
        b -= G;
      }
    }
  } else {
    for (; f + G <= L; f += G)
      scan_group<E, Q, MODE, G>(pts, pj, f, S.qc, S.qi, window, S.key);
    for (; b - G >= 0; b -= G)
      scan_group<E, Q, MODE, G>(pts, pj, b - G, S.qc, S.qi, window, S.key);
  }
  for (; f < L; ++f) scan_group<E, Q, MODE, 1>(pts, pj, f, S.qc, S.qi, window, S.key);
  for (; b > 0; --b) scan_group<E, Q, MODE, 1>(pts, pj, b - 1, S.qc, S.qi, window, S.key);
}

template <int E, int Q, int MODE, bool TBL>
__device__ __forceinline__ void scan_library(
    const Realization& R, int tile, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    int query_set, int window, const TableArgs& ta, uint32_t* tlds,
    ScanState<E, Q, MODE>& S) {
  constexpr int KS = Slots<E, MODE>::KS;
  constexpr int QT = kBlock * Q;                    // queries per tile
  constexpr int QW = 64 * Q;                        // queries per wavefront
  // the wavefront index is uniform: say so, so that the scan position and
  // the library addresses stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const float* __restrict__ emb = emb_pool + R.emb_off;
  const float* __restrict__ pts = pts_pool + R.pts_off;
  const int32_t* __restrict__ pj = pj_pool + R.pj_off;
  const int32_t* __restrict__ qord = qord_pool + R.qord_off;
  const int L = R.l_eff;

  // A wavefront with no query (the tail of the last tile) has nothing to scan.
  if (!scan_queries<E, Q, MODE>(R, tile, wave, lane, emb, pj, qord, query_set, S)) return;

  // Table walk (the realization's rows exist): done unless a row ran short.
  // Compiled only into the launches that carry tables.
  if constexpr (TBL) {
    if (R.table_off >= 0 && ta.words > 0) {
      if (walk_table<E, Q, MODE>(R, ta.pool, tlds, reinterpret_cast<int32_t*>(tlds + ta.words),
                                 emb, window, S))
        return;
#pragma unroll
      for (int m = 0; m < Q; ++m)
#pragma unroll
        for (int s = 0; s < KS; ++s) S.key[m][s] = empty_key();
    }
  }

  const int s0 = query_set ? min(tile * QT + wave * QW + QW / 2, L - 1)
                           : start_pool[(R.slot_base + tile) * kWaves + wave];
  scan_range<E, Q, MODE>(pts, pj, L, s0, window, S);
}

// The E+1 neighbours of query m (nearest first): its running list.  Every
// slot holds a real candidate (the library has at least E+1 candidates
// besides the excluded ones).
template <int E, int Q, int MODE>
__device__ __forceinline__ void select_neighbors(const ScanState<E, Q, MODE>& S, int m,
                                                 float (&nd)[E + 1], int32_t (&nj)[E + 1]) {
#pragma unroll
  for (int t = 0; t < E + 1; ++t) {
    nd[t] = key_d2(S.key[m][t]);
    nj[t] = key_j(S.key[m][t]);
  }
}

// Simplex-projection weights (Section 2.1): d = sqrt(d2) in double,
// u = exp(-d / d_1) (or the zero-distance rule when d_1 = 0), w = u / sum u.
template <int K>
__device__ __forceinline__ void simplex_weights(const float (&nd)[K], double (&w)[K]) {
  // the distances are formed inside the loop (sqrt(x) == 0 exactly when
  // x == 0), so no array of them stays live beside the weights
  const double d0 = sqrt((double)nd[0]);
  if (d0 > 0.0) {
#pragma unroll
    for (int t = 0; t < K; ++t) w[t] = exp(-sqrt((double)nd[t]) / d0);
  } else {
#pragma unroll
    for (int t = 0; t < K; ++t) w[t] = nd[t] == 0.0f ? 1.0 : 0.0;
  }
  double su = 0.0;
#pragma unroll
  for (int t = 0; t < K; ++t) su += w[t];
#pragma unroll
  for (int t = 0; t < K; ++t) w[t] = w[t] / su;
}

// DUMP (the test hook): every query's neighbours, squared distances and
// prediction are written out as well.  The hook's instance has the batched
// launches' Q, candidate groups, tiles and merge order; only the export
// after the scan differs.
template <int E, int Q, int MODE, bool DUMP, bool TBL>
__device__ __forceinline__ void crossmap_item(
    const Realization& R, int tile, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tgt_pool, Moments* __restrict__ partial,
    int query_set, int window, const Dump& dump, Moments* red, const TableArgs& ta,
    uint32_t* tlds) {
  constexpr int K = E + 1;                          // neighbours (Section 3.2)
  const int tid = threadIdx.x;
  const double* __restrict__ tgt = tgt_pool + R.tgt_off;
  const int64_t off = (int64_t)(E - 1) * R.tau;     // time of embedded point 0

  if constexpr (TBL)
    if (R.table_off >= 0 && ta.words > 0) table_bitmask(R, pj_pool, tlds);
  ScanState<E, Q, MODE> S;
  scan_library<E, Q, MODE, TBL>(R, tile, emb_pool, pts_pool, pj_pool, qord_pool, start_pool,
                                query_set, window, ta, tlds, S);

  // Simplex projection from the E+1 neighbours, then Pearson moments.
  Moments mo = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    if (S.qi[m] < 0) continue;
    float nd[K];
    int32_t nj[K];
    select_neighbors<E, Q, MODE>(S, m, nd, nj);
    double w[K];
    simplex_weights<K>(nd, w);
    double pred = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) pred += w[t] * tgt[nj[t] + off];
    mom_add(mo, tgt[S.qi[m] + off], pred);
    if (DUMP) {
      const int64_t row = S.qi[m];
#pragma unroll
      for (int t = 0; t < K; ++t) {
        dump.nbr[row * K + t] = nj[t];
        dump.d2[row * K + t] = nd[t];
      }
      dump.pred[row] = pred;
    }
  }

  // Workgroup merge of the moments in a fixed order (deterministic).
  red[tid] = mo;
  __syncthreads();
#pragma unroll
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = mom_merge(red[tid], red[tid + s]);
    __syncthreads();
  }
  if (tid == 0) partial[R.slot_base + tile] = red[0];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// many targets per neighbour search (causal matrix)
// ---------------------------------------------------------------------------
//
// One neighbour search over the manifold of series a serves the prediction of
// every other series b (the library draw does not depend on the series).
// Per target, the tile's observed/predicted pairs are reduced as sums of
// values shifted by the target's first embedded value (n, s_o, s_p, s_oo,
// s_pp, s_op) plus exact min/max of each side (so constant series give NaN
// exactly), first over the wavefront by a fixed butterfly, then over the
// four wavefronts in order.

struct Sums {
  double v[10];   // n, so, sp, soo, spp, sop, min o, max o, min p, max p
};

__device__ __forceinline__ void sums_merge(Sums& a, const Sums& b) {
#pragma unroll
  for (int i = 0; i < 6; ++i) a.v[i] += b.v[i];
  a.v[6] = fmin(a.v[6], b.v[6]);
  a.v[7] = fmax(a.v[7], b.v[7]);
  a.v[8] = fmin(a.v[8], b.v[8]);
  a.v[9] = fmax(a.v[9], b.v[9]);
}

__device__ __forceinline__ void sums_init(Sums& su) {
#pragma unroll
  for (int i = 0; i < 6; ++i) su.v[i] = 0.0;
  su.v[6] = su.v[8] = __builtin_inf();
  su.v[7] = su.v[9] = -__builtin_inf();
}

// One (observed, predicted) pair; the count is added per query set.
__device__ __forceinline__ void sums_add(Sums& su, double o, double pred, double shift) {
  const double a = o - shift, p = pred - shift;
  su.v[1] += a;
  su.v[2] += p;
  su.v[3] = fma(a, a, su.v[3]);
  su.v[4] = fma(p, p, su.v[4]);
  su.v[5] = fma(a, p, su.v[5]);
  // series values and predictions are finite: min/max without the
  // compiler's NaN quieting of the operands
  su.v[6] = kmin(su.v[6], o);
  su.v[7] = kmax(su.v[7], o);
  su.v[8] = kmin(su.v[8], pred);
  su.v[9] = kmax(su.v[9], pred);
}

// Order a wavefront's LDS accesses (its lanes read what other lanes wrote).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of the many-target item: per wavefront, one query set's neighbours
// (w double [K][64], byte offsets of the neighbours' rows 8*nj*mp uint32
// [K][64], of the queries' rows 8*qi*mp uint32 [64]; the row-offset area
// first holds the squared distances' bits while the weights are formed);
// reused afterwards for the wavefronts' per-target sums (Sums [kWaves][64]).
// A byte offset into the table fits in uint32: the planner keeps N*mp*8
// within 4 GiB.
template <int E>
struct MultiLds {
  static constexpr int K = E + 1;
  static constexpr int kWave = 64 * (K * 12 + 4);
  static constexpr int kStage = kWaves * kWave;
  static constexpr int kRed = kWaves * 64 * (int)sizeof(Sums);
  static constexpr int kBytes = kStage > kRed ? kStage : kRed;
};

// The simplex weights of one query set, one neighbour at a time: the same
// operations in the same order as simplex_weights (so the same bits), with a
// single exp in flight (a smaller register peak after the scan).  Lane l's
// squared distances are the float bits d2b[t*64 + l]; weight t goes to
// w[t*64 + l].  The two areas are disjoint, so lanes that take different
// branches cannot overwrite each other's inputs.
template <int K>
__device__ __forceinline__ void stage_weights(const int32_t* __restrict__ d2b,
                                              double* __restrict__ w, int lane) {
  const double d0 = sqrt((double)__int_as_float(d2b[lane]));
  double su = 0.0;
  if (d0 > 0.0) {
#pragma unroll 1
    for (int t = 0; t < K; ++t) {
      const double u = exp(-sqrt((double)__int_as_float(d2b[t * 64 + lane])) / d0);
      w[t * 64 + lane] = u;
      su += u;
    }
  } else {
#pragma unroll 1
    for (int t = 0; t < K; ++t) {
      const double u = __int_as_float(d2b[t * 64 + lane]) == 0.0f ? 1.0 : 0.0;
      w[t * 64 + lane] = u;
      su += u;
    }
  }
#pragma unroll 1
  for (int t = 0; t < K; ++t) w[t * 64 + lane] = w[t * 64 + lane] / su;
}

// One block of 64 targets of the many-target stage (see below): lane b of
// each wavefront accumulates target b0 + b over the wavefront's queries, set
// by set, then the four wavefronts' sums are merged in order.
template <int E, int Q, int MODE>
__device__ __forceinline__ void multi_target_block(const ScanState<E, Q, MODE>& S,
                                                   const Realization& R, int tile,
                                                   const double* __restrict__ T, int b0,
                                                   int m_series, int self, int mp,
                                                   Sums* __restrict__ partial,
                                                   unsigned char* lds) {
  constexpr int K = E + 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* stage = lds + wave * MultiLds<E>::kWave;
  double* __restrict__ sw = reinterpret_cast<double*>(stage);
  int32_t* __restrict__ srow = reinterpret_cast<int32_t*>(stage + 64 * K * 8);
  int32_t* __restrict__ sqrow = reinterpret_cast<int32_t*>(stage + 64 * K * 12);
  Sums* __restrict__ red = reinterpret_cast<Sums*>(lds);
  const int b = b0 + lane;
  const bool act = b < m_series;
  // lane b's value of a row: the row's byte offset plus 8b from the uniform
  // table base (one 32-bit add per load)
  const char* __restrict__ Tc = reinterpret_cast<const char*>(T);
  const uint32_t lb = act ? (uint32_t)b * 8u : 0u;
  const auto at = [&](uint32_t row_bytes) {
    return *reinterpret_cast<const double*>(Tc + (row_bytes + lb));
  };
  const double shift = at(0u);
  Sums su;
  sums_init(su);
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    // valid queries are a prefix of the lanes (the tail of the last tile is
    // invalid)
    const int nq = __popcll(__builtin_amdgcn_ballot_w64(S.qi[m] >= 0));
    {
      float nd[K];
      int32_t nj[K];
      select_neighbors<E, Q, MODE>(S, m, nd, nj);
      sqrow[lane] = (int32_t)((uint32_t)(S.qi[m] * mp) * 8u);
#pragma unroll
      for (int t = 0; t < K; ++t) srow[t * 64 + lane] = __float_as_int(nd[t]);
      stage_weights<K>(srow, sw, lane);
#pragma unroll
      for (int t = 0; t < K; ++t) srow[t * 64 + lane] = (int32_t)((uint32_t)(nj[t] * mp) * 8u);
    }
    wave_sync();
    if (act) {
      su.v[0] += (double)nq;
      // one query per step, its K + 1 loads issued before any is used;
      // pred = w_0 v_0 + ... as a chain of fused multiply-adds
      for (int q = 0; q < nq; ++q) {
        const double o = at((uint32_t)sqrow[q]);   // first: used first
        double v[K];
#pragma unroll
        for (int t = 0; t < K; ++t) v[t] = at((uint32_t)srow[t * 64 + q]);
        double pred = sw[q] * v[0];
#pragma unroll
        for (int t = 1; t < K; ++t) pred = fma(sw[t * 64 + q], v[t], pred);
        sums_add(su, o, pred, shift);
      }
    }
    wave_sync();
  }
  // wavefronts' sums -> LDS (over the staging area), merged in order
  __syncthreads();
  red[wave * 64 + lane] = su;
  __syncthreads();
  if (wave == 0 && act && b != self) {
    Sums tot = red[lane];
#pragma unroll
    for (int wv = 1; wv < kWaves; ++wv) sums_merge(tot, red[wv * 64 + lane]);
    partial[(R.slot_base + tile) * m_series + b] = tot;
  }
  __syncthreads();
}

template <int E, int Q, int MODE, bool TBL>
__device__ __forceinline__ void crossmap_multi_item(
    const Realization& R, int tile, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tt, int m_series, int self,
    Sums* __restrict__ partial, int query_set, int window, unsigned char* lds,
    const TableArgs& ta, uint32_t* tlds) {
  constexpr int K = E + 1;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int mp = target_stride(m_series);
  const int64_t off = (int64_t)(E - 1) * R.tau;

  if constexpr (TBL)
    if (R.table_off >= 0 && ta.words > 0) table_bitmask(R, pj_pool, tlds);
  ScanState<E, Q, MODE> S;
  scan_library<E, Q, MODE, TBL>(R, tile, emb_pool, pts_pool, pj_pool, qord_pool, start_pool,
                                query_set, window, ta, tlds, S);

  // Per-target stage.  Row t of the time-major table holds every series'
  // value at time t.  Lane b of a wavefront owns target b0 + b and walks the
  // wavefront's queries (staged in LDS one query set at a time): each
  // neighbour's row is then read by one coalesced load for all 64 targets.
  // A target's sums are shifted by its first embedded value (time off).
  // With at most 64 targets there is one block, and each query set's running
  // list is dead once its weights are staged (fewer live registers).
  const double* __restrict__ T = tt + off * mp;
  if (m_series <= 64) {
    multi_target_block<E, Q, MODE>(S, R, tile, T, 0, m_series, self, mp, partial, lds);
  } else {
    for (int b0 = 0; b0 < m_series; b0 += 64)
      multi_target_block<E, Q, MODE>(S, R, tile, T, b0, m_series, self, mp, partial, lds);
  }
}

// Build one row of a distance indexing table (one workgroup per row i): the
// first w points j of [0, n_e) in ascending (d2(i, j), j) order.  d2 is the
// cross-map kernel's binary32 distance; its bit pattern orders like its value
// (d2 >= +0), so the w-th smallest value T is found by a three-pass radix
// select on the bits (11, 11 and 10 bits, histograms in LDS), recomputing
// the distances on each pass.  Then every j with d2 < T is kept, plus the
// lowest-index ones with d2 == T up to w in all, and the w keys (d2 bits,
// j) are sorted by a bitonic network in LDS.  Row stride: w rounded up to a
// multiple of 4, padded with -1.
constexpr int kTableMaxW = 1024;

template <int E>
__global__ __launch_bounds__(kBlock) void k_table_build(const TableJob* __restrict__ jobs,
                                                        const float* __restrict__ emb_pool,
                                                        int32_t* __restrict__ table_pool) {
  __shared__ uint32_t hist[2048];
  __shared__ uint64_t keys[kTableMaxW];
  __shared__ uint32_t s_sel[2];
  __shared__ int s_wave[kBlock / 64];
  __shared__ int s_lt;
  const TableJob J = jobs[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= J.n_e) return;                       // uniform: whole workgroup
  const int tid = threadIdx.x;
  const float* __restrict__ emb = emb_pool + J.emb_off;
  float q[E];
#pragma unroll
  for (int k = 0; k < E; ++k) q[k] = emb[(int64_t)i * E + k];
  const int n = J.n_e;
  const int w = J.w;

  uint32_t prefix = 0, mask = 0;
  uint32_t need = (uint32_t)w;                  // rank of T among the matching values
  for (int pass = 0; pass < 3; ++pass) {
    const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
    const int nbins = pass == 2 ? 1024 : 2048;
    for (int b = tid; b < nbins; b += kBlock) hist[b] = 0u;
    __syncthreads();
    for (int j = tid; j < n; j += kBlock) {
      const uint32_t u = __float_as_uint(sqdist<E>(q, emb + (int64_t)j * E));
      if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & (nbins - 1)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      // bin holding the need-th value: lanes own nbins/64 consecutive bins
      const int per = nbins / 64;
      uint32_t loc = 0;
      for (int b = 0; b < per; ++b) loc += hist[tid * per + b];
      uint32_t inc = loc;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (tid >= o) inc += y;
      }
      const uint32_t exc = inc - loc;
      if (exc < need && need <= inc) {
        uint32_t c = exc;
        for (int b = 0; b < per; ++b) {
          const uint32_t h = hist[tid * per + b];
          if (c + h >= need) {
            s_sel[0] = (uint32_t)(tid * per + b);
            s_sel[1] = c;
            break;
          }
          c += h;
        }
      }
    }
    __syncthreads();
    prefix |= s_sel[0] << shift;
    mask |= (uint32_t)(nbins - 1) << shift;
    need -= s_sel[1];
    __syncthreads();
  }
  // prefix = T (all 32 bits fixed); `need` values equal to T are taken,
  // the w - need values below T all are.
  const uint32_t T = prefix;
  if (tid == 0) s_lt = 0;
  __syncthreads();
  int eq_seen = 0;
  for (int base = 0; base < n; base += kBlock) {
    const int j = base + tid;
    const uint32_t u = j < n ? __float_as_uint(sqdist<E>(q, emb + (int64_t)min(j, n - 1) * E))
                             : 0xffffffffu;
    const bool lt = j < n && u < T;
    const bool eq = j < n && u == T;
    if (lt) {
      const int pos = atomicAdd(&s_lt, 1);
      if (pos < w) keys[pos] = ((uint64_t)u << 32) | (uint32_t)j;
    }
    int tot;
    const int r = block_rank(eq, s_wave, tot);
    const int pe = w - (int)need + eq_seen + r;
    if (eq && eq_seen + r < (int)need && pe >= 0 && pe < w)
      keys[pe] = ((uint64_t)u << 32) | (uint32_t)j;
    eq_seen += tot;
  }
  // bitonic sort of keys[0..P), P = the power of two >= w, padded with ~0
  int P = 1;
  while (P < w) P <<= 1;
  for (int x = w + tid; x < P; x += kBlock) keys[x] = ~0ull;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int x = tid; x < P / 2; x += kBlock) {
        const int lo = 2 * x - (x & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = keys[lo], b = keys[hi];
        if ((a > b) == up) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  const int rs = table_stride(w);
  int32_t* __restrict__ row = table_pool + J.out_off + (int64_t)i * rs;
  for (int x = tid; x < rs; x += kBlock) row[x] = x < w ? (int32_t)(keys[x] & 0xffffffffu) : -1;
}

// ---------------------------------------------------------------------------
// nested libraries: one scan per chain, a snapshot per library size
// ---------------------------------------------------------------------------
//
// A chain holds the libraries of one (E, tau, r, direction): the prefixes of
// one ordering, split into segments at the library sizes (segment k holds
// the points between sizes k-1 and k, gathered in visiting order with its
// own scan starts).  The running lists after segments 0..k are exactly the
// first E+1 candidates of the library of size k (a list only ever keeps the
// smallest keys seen), so after each segment every query predicts from them
// and the tile's moments for that size are merged and stored.
template <int E, int Q, int MODE>
__device__ __forceinline__ void nested_item(
    const Realization& R, int tile, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tgt_pool, const int32_t* __restrict__ seg_pool,
    Moments* __restrict__ partial, int window, Moments* red) {
  constexpr int K = E + 1;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const float* __restrict__ emb = emb_pool + R.emb_off;
  const float* __restrict__ pts = pts_pool + R.pts_off;
  const int32_t* __restrict__ pj = pj_pool + R.pj_off;
  const int32_t* __restrict__ qord = qord_pool + R.qord_off;
  const double* __restrict__ tgt = tgt_pool + R.tgt_off;
  const int32_t* __restrict__ seg = seg_pool + R.seg_off;
  const int64_t off = (int64_t)(E - 1) * R.tau;

  ScanState<E, Q, MODE> S;
  const bool any = scan_queries<E, Q, MODE>(R, tile, wave, lane, emb, pj, qord, 0, S);
  for (int k = 0; k < R.n_seg; ++k) {
    const int b0 = seg[k], b1 = seg[k + 1];
    const int64_t slot = R.slot_base + (int64_t)k * R.n_tiles + tile;
    if (any)
      scan_range<E, Q, MODE>(pts + (int64_t)b0 * E, pj + b0, b1 - b0,
                             start_pool[slot * kWaves + wave], window, S);
    Moments mo = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      if (S.qi[m] < 0) continue;
      float nd[K];
      int32_t nj[K];
      select_neighbors<E, Q, MODE>(S, m, nd, nj);
      double w[K];
      simplex_weights<K>(nd, w);
      double pred = 0.0;
#pragma unroll
      for (int t = 0; t < K; ++t) pred += w[t] * tgt[nj[t] + off];
      mom_add(mo, tgt[S.qi[m] + off], pred);
    }
    red[tid] = mo;
    __syncthreads();
#pragma unroll
    for (int s2 = kBlock / 2; s2 > 0; s2 >>= 1) {
      if (tid < s2) red[tid] = mom_merge(red[tid], red[tid + s2]);
      __syncthreads();
    }
    if (tid == 0) partial[slot] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// E-sweep sharing: one scan serves every E <= EMAX
// ---------------------------------------------------------------------------
//
// With the option, every E of a sweep uses the points of E_max's embedding
// (their first E coordinates) and the same libraries.  The binary32 chain of
// a pair after k coordinates is exactly that pair's d2 for E = k (the chain
// runs in the same order from +0), so one pass over the library serves all
// of them; each E keeps its own running list of E+1 keys (lists packed in
// one array: E's list at offset (E-1)(E+2)/2).
//
// Fast path per group of G candidates: the chains, and per (query, E) the
// smallest partial sum of the group; one compare per (query, E) against the
// running E+1-th key decides whether E's list can change.  Only then are the
// group's chains recomputed to E coordinates (the same sequence of binary32
// operations, so the same values) and the candidates inserted, with the
// exclusions checked exactly.

template <int EMAX>
struct SharedLists {
  static constexpr int kTotal = EMAX * (EMAX + 3) / 2;
  static constexpr int off(int e) { return (e - 1) * (e + 2) / 2; }
};

template <int EMAX, int Q>
struct SharedState {
  float qc[Q][EMAX];
  int qi[Q];
  double key[Q][SharedLists<EMAX>::kTotal];
};

template <int KS, int OFF, int TOT>
__device__ __forceinline__ void insert_at(double (&key)[TOT], double c) {
#pragma unroll
  for (int m = KS - 1; m >= 1; --m) key[OFF + m] = kmin(kmax(key[OFF + m - 1], c), key[OFF + m]);
  key[OFF] = kmin(key[OFF], c);
}

// d2 of candidate g to E coordinates.
template <int EMAX, int G, int E>
__device__ __forceinline__ float shared_d2(const Chunk<EMAX, G>& ch, int g,
                                           const float (&q)[EMAX]) {
  float d = q[0] - ch.p[g][0];
  float acc = d * d;
#pragma unroll
  for (int k = 1; k < E; ++k) {
    d = q[k] - ch.p[g][k];
    acc = __builtin_fmaf(d, d, acc);
  }
  return acc;
}

// Slow path of list E: recompute the group's chains to E coordinates and
// insert what enters E's list (exclusions checked exactly).
template <int EMAX, int Q, int MODE, int G, int E>
__device__ __forceinline__ void shared_lists(const Chunk<EMAX, G>& ch, const float (&mn)[Q][EMAX],
                                             int window, SharedState<EMAX, Q>& S) {
  constexpr int TOT = SharedLists<EMAX>::kTotal;
  constexpr int OFF = SharedLists<EMAX>::off(E);
  constexpr int KS = E + 1;
  bool hit = false;
#pragma unroll
  for (int m = 0; m < Q; ++m) hit |= mn[m][E - 1] <= key_d2(S.key[m][OFF + KS - 1]);
  if (__builtin_amdgcn_ballot_w64(hit)) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        const float d2 = shared_d2<EMAX, G, E>(ch, g, S.qc[m]);
        bool ok = d2 <= key_d2(S.key[m][OFF + KS - 1]);
        if (MODE == kExclSelf) ok = ok && ch.j[g] != S.qi[m];
        if (MODE == kWindow) {
          const int dj = ch.j[g] - S.qi[m];
          ok = ok && (dj > window || dj < -window);
        }
        if (ok) insert_at<KS, OFF, TOT>(S.key[m], make_key(d2, ch.j[g]));
      }
  }
  if constexpr (E < EMAX) shared_lists<EMAX, Q, MODE, G, E + 1>(ch, mn, window, S);
}

// Fast path: every chain of the group and, per (query, E), its smallest
// partial sum, then one check per list.
template <int EMAX, int Q, int MODE, int G>
__device__ __forceinline__ void shared_chunk(const Chunk<EMAX, G>& ch, int window,
                                             SharedState<EMAX, Q>& S) {
  float mn[Q][EMAX];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      float d = S.qc[m][0] - ch.p[g][0];
      float acc = d * d;
      if (MODE == kWindow) {
        // an excluded pair never raises a trigger (checked exactly on insert)
        const int dj = ch.j[g] - S.qi[m];
        if (dj <= window && dj >= -window) acc = __builtin_inff();
      }
      mn[m][0] = g == 0 ? acc : fminf(mn[m][0], acc);
#pragma unroll
      for (int k = 1; k < EMAX; ++k) {
        d = S.qc[m][k] - ch.p[g][k];
        acc = __builtin_fmaf(d, d, acc);
        mn[m][k] = g == 0 ? acc : fminf(mn[m][k], acc);
      }
    }
  shared_lists<EMAX, Q, MODE, G, 1>(ch, mn, window, S);
}

template <int EMAX, int Q, int MODE, int G>
__device__ __forceinline__ void shared_group(const float* __restrict__ pts,
                                             const int32_t* __restrict__ pj, int c, int window,
                                             SharedState<EMAX, Q>& S) {
  Chunk<EMAX, G> ch;
  load_chunk<EMAX, G>(ch, pts, pj, c);
  shared_chunk<EMAX, Q, MODE, G>(ch, window, S);
}

// Prediction of list E for each of the lane's queries, the tile's moments
// merged over the workgroup and stored in E's slots; then the next E.
template <int EMAX, int Q, int E>
__device__ __forceinline__ void shared_snapshot(const Realization& R, int tile,
                                                const double* __restrict__ tgt, int64_t off,
                                                const SharedState<EMAX, Q>& S,
                                                Moments* __restrict__ partial, Moments* red) {
  constexpr int K = E + 1;
  constexpr int OFF = SharedLists<EMAX>::off(E);
  const int tid = threadIdx.x;
  Moments mo = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    if (S.qi[m] < 0) continue;
    float nd[K];
    double w[K];
#pragma unroll
    for (int t = 0; t < K; ++t) nd[t] = key_d2(S.key[m][OFF + t]);
    simplex_weights<K>(nd, w);
    double pred = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) pred += w[t] * tgt[key_j(S.key[m][OFF + t]) + off];
    mom_add(mo, tgt[S.qi[m] + off], pred);
  }
  red[tid] = mo;
  __syncthreads();
#pragma unroll
  for (int s2 = kBlock / 2; s2 > 0; s2 >>= 1) {
    if (tid < s2) red[tid] = mom_merge(red[tid], red[tid + s2]);
    __syncthreads();
  }
  if (tid == 0) partial[R.slot_base + (int64_t)(E - 1) * R.n_tiles + tile] = red[0];
  __syncthreads();
  if constexpr (E < EMAX) shared_snapshot<EMAX, Q, E + 1>(R, tile, tgt, off, S, partial, red);
}

template <int EMAX, int MODE>
__device__ __forceinline__ void shared_item(
    const Realization& R, int tile, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tgt_pool, Moments* __restrict__ partial, int window,
    Moments* red) {
  constexpr int TOT = SharedLists<EMAX>::kTotal;
  constexpr int Q = kSharedQ[EMAX];
  constexpr int G = kSharedG[EMAX];
  constexpr int QT = kBlock * Q;
  constexpr int QW = 64 * Q;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const float* __restrict__ emb = emb_pool + R.emb_off;
  const float* __restrict__ pts = pts_pool + R.pts_off;
  const int32_t* __restrict__ pj = pj_pool + R.pj_off;
  const int32_t* __restrict__ qord = qord_pool + R.qord_off;
  const double* __restrict__ tgt = tgt_pool + R.tgt_off;
  const int64_t off = (int64_t)(EMAX - 1) * R.tau;   // time of common point 0
  const int L = R.l_eff;

  SharedState<EMAX, Q> S;
  bool any = false;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int qq = tile * QT + wave * QW + m * 64 + lane;
    const bool valid = qq < R.n_query;
    any |= valid;
    const int i = valid ? qord[qq] : 0;
    S.qi[m] = valid ? i : -1;
#pragma unroll
    for (int k = 0; k < EMAX; ++k) S.qc[m][k] = emb[(int64_t)i * EMAX + k];
#pragma unroll
    for (int s = 0; s < TOT; ++s) S.key[m][s] = empty_key();
  }

  if (__builtin_amdgcn_ballot_w64(any)) {
    int s0 = start_pool[(R.slot_base + tile) * kWaves + wave];
    s0 = min(max(s0, 0), L);
    int f = s0, b = s0;
    const int both = min((L - s0) / G, s0 / G);
    if (both > 0) {
      Chunk<EMAX, G> A, B;
      load_chunk<EMAX, G>(A, pts, pj, f);
      for (int k = 0; k < both; ++k) {
        settle_chunk<EMAX, G>(A);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk<EMAX, G>(B, pts, pj, b - G);
        __builtin_amdgcn_sched_barrier(0);
        shared_chunk<EMAX, Q, MODE, G>(A, window, S);
        f += G;
        settle_chunk<EMAX, G>(B);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk<EMAX, G>(A, pts, pj, k + 1 < both ? f : f - G);
        __builtin_amdgcn_sched_barrier(0);
        shared_chunk<EMAX, Q, MODE, G>(B, window, S);
        b -= G;
      }
    }
    for (; f + G <= L; f += G) shared_group<EMAX, Q, MODE, G>(pts, pj, f, window, S);
    for (; b - G >= 0; b -= G) shared_group<EMAX, Q, MODE, G>(pts, pj, b - G, window, S);
    for (; f < L; ++f) shared_group<EMAX, Q, MODE, 1>(pts, pj, f, window, S);
    for (; b > 0; --b) shared_group<EMAX, Q, MODE, 1>(pts, pj, b - 1, window, S);
  }
  shared_snapshot<EMAX, Q, 1>(R, tile, tgt, off, S, partial, red);
}

// Work items are taken in list order (the host lists them longest first).
// With next == nullptr each workgroup takes items blockIdx.x, +gridDim.x, ...;
// otherwise workgroups pull the next item from an atomic counter that starts
// at zero (a persistent grid).
// Workgroups are dispatched to the chip's 8 XCDs round-robin (workgroup b
// runs on XCD b mod 8), and each XCD has an L2 of its own.  The items of one
// realization are consecutive and all read its library, so each XCD takes
// runs of kXcdRun consecutive items: within every group of 8*kXcdRun
// workgroups, workgroup b takes item  group + (b mod 8)*kXcdRun + (b/8) mod
// kXcdRun.  Workgroups past the last whole group keep their own index; the
// map is a permutation of [0, grid), so the item set is unchanged.
constexpr int kXcds = 8;
#ifndef CCM_XCD_RUN
#define CCM_XCD_RUN 16
#endif
constexpr int kXcdRun = CCM_XCD_RUN;
__device__ __forceinline__ int xcd_item(int b, int grid) {
  constexpr int span = kXcds * kXcdRun;
  const int full = grid / span * span;
  if (b >= full) return b;
  const int base = b / span * span;
  const int r = b - base;
  return base + (r % kXcds) * kXcdRun + r / kXcds;
}

template <int E, int Q, int MODE, bool DUMP, bool TBL>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(kTuneW[E] > 0 ? kTuneW[E] : 1, 8))) void k_crossmap(
    const Realization* __restrict__ rzs, const Item* __restrict__ items,
    int n_items, int* __restrict__ next, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tgt_pool, Moments* __restrict__ partial,
    int query_set, int window, Dump dump, TableArgs ta) {
  __shared__ Moments red[kBlock];
  __shared__ int s_next;
  extern __shared__ uint32_t table_lds[];   // bitmask words, then accepted indices
  int it = xcd_item(blockIdx.x, gridDim.x);
  while (it < n_items) {
    const Item I = items[it];
    const Realization R = rzs[I.rz];
    crossmap_item<E, Q, MODE, DUMP, TBL>(R, I.tile, emb_pool, pts_pool, pj_pool,
                                    qord_pool, start_pool, tgt_pool, partial,
                                    query_set, window, dump, red, ta, table_lds);
    if (next == nullptr) {
      it += gridDim.x;
    } else {
      if (threadIdx.x == 0) s_next = (int)gridDim.x + atomicAdd(next, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_next);
      __syncthreads();
    }
  }
}

// Causal-matrix form: realization rz searches the manifold of series
// R.emb_off's owner (index self_of[rz]) and predicts all m_series series.
template <int E, int Q, int MODE, bool TBL>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(kMultiW[E] > 0 ? kMultiW[E] : 1, 8))) void k_crossmap_multi(
    const Realization* __restrict__ rzs, const int32_t* __restrict__ self_of,
    const Item* __restrict__ items, int n_items, int* __restrict__ next,
    const float* __restrict__ emb_pool, const float* __restrict__ pts_pool,
    const int32_t* __restrict__ pj_pool, const int32_t* __restrict__ qord_pool,
    const int32_t* __restrict__ start_pool, const double* __restrict__ tt,
    int m_series, Sums* __restrict__ partial, int query_set, int window, TableArgs ta) {
  __shared__ __align__(16) unsigned char lds[MultiLds<E>::kBytes];
  __shared__ int s_next;
  extern __shared__ uint32_t table_lds[];   // bitmask words, then accepted indices
  int it = xcd_item(blockIdx.x, gridDim.x);
  while (it < n_items) {
    const Item I = items[it];
    const Realization R = rzs[I.rz];
    crossmap_multi_item<E, Q, MODE, TBL>(R, I.tile, emb_pool, pts_pool, pj_pool, qord_pool,
                                    start_pool, tt, m_series, self_of[I.rz], partial,
                                    query_set, window, lds, ta, table_lds);
    if (next == nullptr) {
      it += gridDim.x;
    } else {
      if (threadIdx.x == 0) s_next = (int)gridDim.x + atomicAdd(next, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_next);
      __syncthreads();
    }
  }
}

// rho[self][b] of every realization from the per-tile sums; NaN on the
// diagonal and when either side is constant.
template <int E, int Q, int MODE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(kNestedW[E] > 0 ? kNestedW[E] : 1, 8))) void k_crossmap_nested(
    const Realization* __restrict__ rzs, const Item* __restrict__ items,
    int n_items, int* __restrict__ next, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tgt_pool, const int32_t* __restrict__ seg_pool,
    Moments* __restrict__ partial, int window) {
  __shared__ Moments red[kBlock];
  __shared__ int s_next;
  int it = xcd_item(blockIdx.x, gridDim.x);
  while (it < n_items) {
    const Item I = items[it];
    const Realization R = rzs[I.rz];
    nested_item<E, Q, MODE>(R, I.tile, emb_pool, pts_pool, pj_pool, qord_pool, start_pool,
                            tgt_pool, seg_pool, partial, window, red);
    if (next == nullptr) {
      it += gridDim.x;
    } else {
      if (threadIdx.x == 0) s_next = (int)gridDim.x + atomicAdd(next, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_next);
      __syncthreads();
    }
  }
}

template <int EMAX, int MODE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(kSharedW[EMAX] > 0 ? kSharedW[EMAX] : 1, 8)))
void k_crossmap_shared(
    const Realization* __restrict__ rzs, const Item* __restrict__ items,
    int n_items, int* __restrict__ next, const float* __restrict__ emb_pool,
    const float* __restrict__ pts_pool, const int32_t* __restrict__ pj_pool,
    const int32_t* __restrict__ qord_pool, const int32_t* __restrict__ start_pool,
    const double* __restrict__ tgt_pool, Moments* __restrict__ partial, int window) {
  __shared__ Moments red[kBlock];
  __shared__ int s_next;
  int it = xcd_item(blockIdx.x, gridDim.x);
  while (it < n_items) {
    const Item I = items[it];
    const Realization R = rzs[I.rz];
    shared_item<EMAX, MODE>(R, I.tile, emb_pool, pts_pool, pj_pool, qord_pool, start_pool,
                            tgt_pool, partial, window, red);
    if (next == nullptr) {
      it += gridDim.x;
    } else {
      if (threadIdx.x == 0) s_next = (int)gridDim.x + atomicAdd(next, 1);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(s_next);
      __syncthreads();
    }
  }
}


// Queries per lane for the hot kernel (tuned per E: fewer when the running
// lists are long so that registers stay within budget).
template <int E>
struct DefaultQ {
  static constexpr int Q = kTuneQ[E];
};

// Dynamic LDS of a cross-map launch whose realizations walk tables over at
// most n_e points: the library bitmask, then E+1 accepted indices per lane.
inline int table_lds_words(int n_e) { return n_e > 0 ? (n_e + 31) / 32 : 0; }
inline size_t table_lds_bytes(int E, int n_e) {
  return n_e > 0 ? (size_t)table_lds_words(n_e) * 4 + (size_t)(E + 1) * kBlock * 4 : 0;
}

}  // namespace ccmk

// ccm_kernels.hip -- gfx950 kernels of the simplex cross-map.
//
// The hot path of convergent cross mapping (paper, Section 3.2): for every
// query point of a shadow manifold, the E+1 nearest vectors of a random
// library subsample, found by brute force over all library vectors; then a
// simplex-projection prediction of the other series (Section 2.1) and the
// Pearson skill of the predictions (Section 2.1), for r subsamples per
// library size L (Introduction).
//
// Kernels, in pipeline order:
//   k_ingest     double series -> float series (round to nearest even)
//   k_embed      lagged-coordinate embedding, AoS float[n_e][E]
//   k_sample     library subsamples: selection sampling driven by SplitMix64
//   k_crossmap   fused distance / top-(E+1) / prediction / Pearson moments,
//                one workgroup per (realization, query tile) work item,
//                optionally persistent with an atomic work queue
//   k_finalize   merge the per-tile moments of each realization -> rho
//
// Arithmetic that must agree bit for bit with the CPU oracle:
//   d2 = sum_k (q_k - p_k)^2 in binary32 as acc = fma(diff, diff, acc),
//   k ascending from acc = +0 (the first term is the plain product, which is
//   the same value), no other contraction (-ffp-contract=off);
//   neighbours are the first E+1 candidates in (d2, j) order.
#include "ccm_internal.h"

namespace ccmk {

// ---------------------------------------------------------------------------
// ingest and embedding
// ---------------------------------------------------------------------------

__global__ void k_ingest(const IngestJob* __restrict__ jobs,
                         const double* __restrict__ src,
                         float* __restrict__ dst) {
  const IngestJob J = jobs[blockIdx.y];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < J.n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[J.dst_off + t] = __double2float_rn(src[J.src_off + t]);
}

// Backward lags: embedded point i sits at time i + (E-1) tau and its
// coordinate k is the series at that time minus k tau.
__global__ void k_embed(const EmbedJob* __restrict__ jobs,
                        const float* __restrict__ s32,
                        float* __restrict__ emb) {
  const EmbedJob J = jobs[blockIdx.y];
  const int64_t n = J.n_e * J.E;
  const float* __restrict__ s = s32 + J.src_off;
  float* __restrict__ o = emb + J.dst_off;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x / J.E;
    const int k = (int)(x - i * J.E);
    o[x] = s[i + (int64_t)(J.E - 1 - k) * J.tau];
  }
}

// ---------------------------------------------------------------------------
// library subsamples
// ---------------------------------------------------------------------------

// SplitMix64 output mix (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Selection sampling (Knuth, TAOCP Vol. 2, Sec. 3.4.2, Algorithm S): visit
// candidates 0..n_e-1 in order and take candidate j with probability
// (needed / remaining); the uniform integer below (n_e - j) is the high word of
// the 64x64-bit product of one SplitMix64 draw with (n_e - j).  The stream of
// a library is keyed by (seed, E, tau, L_eff, r) folded through the mix.
// Once every remaining candidate is needed the rest are taken without draws:
// the test would accept each of them whatever the draw.
__global__ void k_sample(const SampleJob* __restrict__ jobs, int64_t n_jobs,
                         int32_t* __restrict__ out_pool) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= n_jobs) return;
  const SampleJob J = jobs[id];
  uint64_t st = 0;
  st = sm_mix(st ^ J.seed);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.E);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.tau);
  st = sm_mix(st ^ (uint64_t)J.l_eff);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.r_index);
  int32_t* __restrict__ out = out_pool + J.out_off;
  int64_t s = 0;
  int64_t j = 0;
  for (; j < J.n_e && s < J.l_eff; ++j) {
    if (J.l_eff - s == J.n_e - j) break;        // all the rest are needed
    st += 0x9e3779b97f4a7c15ull;
    const uint64_t z = sm_mix(st);
    const uint64_t u = __umul64hi(z, (uint64_t)(J.n_e - j));
    if (u < (uint64_t)(J.l_eff - s)) out[s++] = (int32_t)j;
  }
  for (; s < J.l_eff; ++s, ++j) out[s] = (int32_t)j;
}

// Library coordinates laid out contiguously per realization, so the scan
// streams them through the scalar cache with no dependent index load.
// One workgroup per job.
__global__ void k_gather(const GatherJob* __restrict__ jobs,
                         const float* __restrict__ emb_pool,
                         const int32_t* __restrict__ lib_pool,
                         float* __restrict__ pts_pool) {
  const GatherJob J = jobs[blockIdx.x];
  const float* __restrict__ emb = emb_pool + J.emb_off;
  const int32_t* __restrict__ lib = lib_pool + J.lib_off;
  float* __restrict__ pts = pts_pool + J.pts_off;
  const int64_t n = J.l_eff * J.E;
  for (int64_t x = threadIdx.x; x < n; x += blockDim.x) {
    const int64_t c = x / J.E;
    const int k = (int)(x - c * J.E);
    pts[x] = emb[(int64_t)lib[c] * J.E + k];
  }
}

// ---------------------------------------------------------------------------
// candidate keys
// ---------------------------------------------------------------------------
//
// A candidate (d2, c) is kept as one 64-bit word: high half the binary32 bits
// of d2, low half its position c in the library.  Library indices ascend
// with position, so (d2, c) orders exactly like (d2, j).  For d2 >= 0 the
// bit patterns of binary32 order like the values, so the word read as an
// unsigned integer orders exactly like (d2, c) lexicographically.  The same word read as a binary64 is a
// non-negative number (denormal when d2 is 0 or tiny, never NaN: the high
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

// Library candidates per trigger check; the group's coordinates (G*E values,
// uniform across the wavefront) come through the scalar cache into SGPRs.
template <int E>
struct Group {
  static constexpr int G = E <= 2 ? 8 : (E <= 4 ? 4 : 2);
};

template <int E, int Q, int MODE, int G>
__device__ __forceinline__ void scan_group(
    const float* __restrict__ pts, const int32_t* __restrict__ lib, int c,
    const float (&qc)[Q][E], const int (&qi)[Q], int window,
    double (&key)[Q][MODE == kExclSelf ? E + 2 : E + 1]) {
  constexpr int KS = MODE == kExclSelf ? E + 2 : E + 1;
  float p[G][E];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int k = 0; k < E; ++k) p[g][k] = pts[(int64_t)(c + g) * E + k];
  int32_t jw[G];
  if (MODE == kWindow) {
#pragma unroll
    for (int g = 0; g < G; ++g) jw[g] = lib[c + g];
  }
  float d2[G][Q];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      float v = sqdist<E>(qc[m], p[g]);
      if (MODE == kWindow) {
        const int dj = jw[g] - qi[m];
        if (dj <= window && dj >= -window) v = __builtin_nanf("");
      }
      d2[g][m] = v;
    }
  // One compare per query per group: the group minimum against the current
  // (KS)-th best; only then, and only for lanes that qualify, insert.
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    float mn = d2[0][m];
#pragma unroll
    for (int g = 1; g < G; ++g) mn = fminf(mn, d2[g][m]);
    if (__builtin_amdgcn_ballot_w64(mn <= key_d2(key[m][KS - 1]))) {
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (d2[g][m] <= key_d2(key[m][KS - 1]))
          insert_key<KS>(key[m], make_key(d2[g][m], c + g));
    }
  }
}

template <int E, int Q, int MODE, bool DUMP>
__device__ __forceinline__ void crossmap_item(
    const Realization& R, int tile, const float* __restrict__ emb_pool,
    const int32_t* __restrict__ lib_pool, const float* __restrict__ pts_pool,
    const double* __restrict__ tgt_pool, Moments* __restrict__ partial,
    int query_set, int window, const Dump& dump, Moments* red) {
  constexpr int K = E + 1;                          // neighbours (Section 3.2)
  constexpr int KS = MODE == kExclSelf ? K + 1 : K; // running slots
  constexpr int G = Group<E>::G;
  const int tid = threadIdx.x;
  const float* __restrict__ emb = emb_pool + R.emb_off;
  const int32_t* __restrict__ lib = lib_pool + R.lib_off;
  const float* __restrict__ pts = pts_pool + R.pts_off;
  const double* __restrict__ tgt = tgt_pool + R.tgt_off;
  const int64_t off = (int64_t)(E - 1) * R.tau;     // time of embedded point 0
  const int L = R.l_eff;

  // queries of this lane: tile*QT + m*kBlock + tid
  float qc[Q][E];
  int qi[Q];
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int qq = tile * (kBlock * Q) + m * kBlock + tid;
    const bool valid = qq < R.n_query;
    const int i = valid ? (query_set ? lib[qq] : qq) : 0;
    qi[m] = valid ? i : -1;
#pragma unroll
    for (int k = 0; k < E; ++k) qc[m][k] = emb[(int64_t)i * E + k];
  }

  double key[Q][KS];
#pragma unroll
  for (int m = 0; m < Q; ++m)
#pragma unroll
    for (int s = 0; s < KS; ++s) key[m][s] = empty_key();

  // Brute-force scan of the library in ascending position (= index) order.
  int c = 0;
  for (; c + G <= L; c += G)
    scan_group<E, Q, MODE, G>(pts, lib, c, qc, qi, window, key);
  for (; c < L; ++c)
    scan_group<E, Q, MODE, 1>(pts, lib, c, qc, qi, window, key);

  // Simplex projection from the E+1 neighbours, then Pearson moments.
  Moments mo = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    if (qi[m] < 0) continue;
    // every slot holds a real candidate (the library has at least KS of
    // them); positions are clamped all the same before indexing
    int32_t jj[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int pos = min(max(key_j(key[m][s]), 0), L - 1);
      jj[s] = lib[pos];
    }
    float nd[K];
    int32_t nj[K];
    if (MODE == kExclSelf) {
      // the query itself is at most one of the KS keys; without it the
      // first K of the others are the neighbours
      int pos = KS - 1;
#pragma unroll
      for (int s = KS - 1; s >= 0; --s)
        if (jj[s] == qi[m]) pos = s;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        nd[t] = key_d2(t < pos ? key[m][t] : key[m][t + 1]);
        nj[t] = t < pos ? jj[t] : jj[t + 1];
      }
    } else {
#pragma unroll
      for (int t = 0; t < K; ++t) {
        nd[t] = key_d2(key[m][t]);
        nj[t] = jj[t];
      }
    }
    double dist[K], u[K];
#pragma unroll
    for (int t = 0; t < K; ++t) dist[t] = sqrt((double)nd[t]);
    if (dist[0] > 0.0) {
#pragma unroll
      for (int t = 0; t < K; ++t) u[t] = exp(-dist[t] / dist[0]);
    } else {
#pragma unroll
      for (int t = 0; t < K; ++t) u[t] = dist[t] == 0.0 ? 1.0 : 0.0;
    }
    double su = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) su += u[t];
    double pred = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) pred += (u[t] / su) * tgt[nj[t] + off];
    mom_add(mo, tgt[qi[m] + off], pred);
    if (DUMP) {
      const int64_t qq = (int64_t)tile * (kBlock * Q) + m * kBlock + tid;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        dump.nbr[qq * K + t] = nj[t];
        dump.d2[qq * K + t] = nd[t];
      }
      dump.pred[qq] = pred;
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

// Work items are taken in list order (the host lists them longest first).
// With next == nullptr each workgroup takes items blockIdx.x, +gridDim.x, ...;
// otherwise workgroups pull the next item from an atomic counter that starts
// at zero (a persistent grid).
template <int E, int Q, int MODE, bool DUMP>
__global__ __launch_bounds__(kBlock) void k_crossmap(
    const Realization* __restrict__ rzs, const Item* __restrict__ items,
    int n_items, int* __restrict__ next, const float* __restrict__ emb_pool,
    const int32_t* __restrict__ lib_pool, const float* __restrict__ pts_pool,
    const double* __restrict__ tgt_pool, Moments* __restrict__ partial,
    int query_set, int window, Dump dump) {
  __shared__ Moments red[kBlock];
  __shared__ int s_next;
  int it = blockIdx.x;
  while (it < n_items) {
    const Item I = items[it];
    const Realization R = rzs[I.rz];
    crossmap_item<E, Q, MODE, DUMP>(R, I.tile, emb_pool, lib_pool, pts_pool,
                                    tgt_pool, partial, query_set, window, dump,
                                    red);
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

__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// rho = cov / sqrt(var_t var_p) from the merged moments; NaN when either
// side is constant.
__global__ void k_finalize(const Realization* __restrict__ rzs, int64_t n_rz,
                           const Moments* __restrict__ partial,
                           double* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n_rz) return;
  const Realization R = rzs[r];
  Moments a = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < R.n_tiles; ++t) a = mom_merge(a, partial[R.slot_base + t]);
  double rho = __builtin_nan("");
  if (a.m2t > 0.0 && a.m2p > 0.0) rho = a.c / sqrt(a.m2t * a.m2p);
  out[R.out_index] = rho;
}

// ---------------------------------------------------------------------------
// kernel table
// ---------------------------------------------------------------------------

using CrossmapFn = void (*)(const Realization*, const Item*, int, int*,
                            const float*, const int32_t*, const float*,
                            const double*, Moments*, int, int, Dump);

template <int E, int Q>
struct QSet {
  static CrossmapFn get(int mode, bool dump) {
    if (dump) {
      switch (mode) {
        case kExclSelf: return k_crossmap<E, 1, kExclSelf, true>;
        case kKeepSelf: return k_crossmap<E, 1, kKeepSelf, true>;
        default: return k_crossmap<E, 1, kWindow, true>;
      }
    }
    switch (mode) {
      case kExclSelf: return k_crossmap<E, Q, kExclSelf, false>;
      case kKeepSelf: return k_crossmap<E, Q, kKeepSelf, false>;
      default: return k_crossmap<E, Q, kWindow, false>;
    }
  }
};

// Queries per lane for the hot kernel, per E (fewer when the running lists
// are long so that registers stay within budget).
template <int E>
struct DefaultQ {
  static constexpr int Q = E <= 4 ? 4 : 2;
};

static CrossmapFn crossmap_kernel(int E, int mode, bool dump, int* q_out) {
  int q = 1;
  CrossmapFn f = nullptr;
  switch (E) {
#define CCM_CASE(e)                                           \
  case e:                                                     \
    q = dump ? 1 : DefaultQ<e>::Q;                            \
    f = QSet<e, DefaultQ<e>::Q>::get(mode, dump);             \
    break;
    CCM_CASE(1) CCM_CASE(2) CCM_CASE(3) CCM_CASE(4) CCM_CASE(5)
    CCM_CASE(6) CCM_CASE(7) CCM_CASE(8) CCM_CASE(9) CCM_CASE(10)
#undef CCM_CASE
    default: break;
  }
  if (q_out) *q_out = q;
  return f;
}

// ---------------------------------------------------------------------------
// host-side launchers (the runtime calls only these)
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

int crossmap_queries_per_lane(int E, bool dump) {
  int q = 0;
  crossmap_kernel(E, kExclSelf, dump, &q);
  return q;
}

hipError_t launch_ingest(const IngestJob* jobs, int n_jobs, int64_t max_n,
                         const double* src, float* dst, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  k_ingest<<<dim3(blocks_for(max_n, 256), n_jobs), 256, 0, st>>>(jobs, src, dst);
  return hipGetLastError();
}

hipError_t launch_embed(const EmbedJob* jobs, int n_jobs, int64_t max_n,
                        const float* s32, float* emb, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  k_embed<<<dim3(blocks_for(max_n, 256), n_jobs), 256, 0, st>>>(jobs, s32, emb);
  return hipGetLastError();
}

hipError_t launch_sample(const SampleJob* jobs, int64_t n_jobs, int32_t* out,
                         hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_jobs + 63) / 64);
  k_sample<<<blocks, 64, 0, st>>>(jobs, n_jobs, out);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherJob* jobs, int64_t n_jobs, const float* emb,
                         const int32_t* lib, float* pts, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  k_gather<<<(unsigned)n_jobs, 256, 0, st>>>(jobs, emb, lib, pts);
  return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_zero_int<<<(n + 255) / 256, 256, 0, st>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_crossmap(int E, int mode, bool dump, int grid,
                           const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb,
                           const int32_t* lib, const float* pts,
                           const double* tgt, Moments* partial, int query_set,
                           int window, Dump d, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  CrossmapFn f = crossmap_kernel(E, mode, dump, nullptr);
  if (!f) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f, dim3((unsigned)grid), dim3(kBlock), 0, st, rzs, items,
                     n_items, next, emb, lib, pts, tgt, partial, query_set,
                     window, d);
  return hipGetLastError();
}

hipError_t launch_finalize(const Realization* rzs, int64_t n_rz,
                           const Moments* partial, double* out, hipStream_t st) {
  if (n_rz <= 0) return hipSuccess;
  k_finalize<<<(unsigned)((n_rz + 255) / 256), 256, 0, st>>>(rzs, n_rz, partial, out);
  return hipGetLastError();
}

}  // namespace ccmk

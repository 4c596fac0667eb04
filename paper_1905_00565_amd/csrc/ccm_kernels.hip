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
//   k_ingest       double series -> float series (round to nearest even)
//   k_embed        lagged-coordinate embedding, AoS float[n_e][E]
//   k_order_keys   visiting-order keys of each order set (value, or Hilbert
//                  position over a few lag coordinates)
//   (sort_series)  each order set's embedded indices sorted by key
//   k_query_order  each embedding's points in its set's visiting order
//   k_sample       library subsamples: selection sampling driven by SplitMix64
//   k_gather       each library laid out in visiting order, plus the
//                  position every query tile starts scanning from
//   k_crossmap     fused distance / top-(E+1) / prediction / Pearson moments,
//                  one workgroup per (realization, query tile) work item,
//                  optionally persistent with an atomic work queue
//   k_finalize     merge the per-tile moments of each realization -> rho
//
// Arithmetic that must agree bit for bit with the CPU oracle:
//   d2 = sum_k (q_k - p_k)^2 in binary32 as acc = fma(diff, diff, acc),
//   k ascending from acc = +0 (the first term is the plain product, which is
//   the same value), no other contraction (-ffp-contract=off);
//   neighbours are the first E+1 candidates in (d2, j) order.
// The cross-map kernels themselves are templates in ccm_device.h, compiled
// once per E by ccm_inst.hip; this file holds the kernels that do not depend
// on E and the launchers that dispatch by E.
//
// The order in which candidates are visited is free: selection uses the exact
// (d2, j) key.  Queries are grouped and candidates visited roughly nearest
// first (along a space-filling curve) only so that the running lists settle
// early and the insertion path stays rare; every (query, candidate) pair is
// still evaluated.
#include "ccm_device.h"
#include "ccm_inst.h"
#include "ccm_copy.h"

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

// Time indices 0..n-1 for every series segment (input of the value sort).
__global__ void k_iota_segments(int32_t* __restrict__ out, int64_t n, int64_t total) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x)
    out[x] = (int32_t)(x % n);
}

// Position of (x, y) on the Hilbert curve filling [0, 2^16)^2 (the classic
// quadrant-by-quadrant construction: at each scale the quadrant contributes
// s*s*((3*rx) ^ ry) and the remaining coordinates are reflected/swapped into
// that quadrant's frame).
__device__ __forceinline__ uint32_t hilbert16(uint32_t x, uint32_t y) {
  uint32_t d = 0;
  for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u;
    const uint32_t ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = 0xffffu - x;
        y = 0xffffu - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Order-preserving map of binary32 to uint32.
__device__ __forceinline__ uint32_t ordered_bits(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Index on the n-dimensional Hilbert curve of b bits per axis (n <= 4,
// n * b <= 32): Skilling's transpose form (J. Skilling, "Programming the
// Hilbert curve", AIP Conf. Proc. 707, 2004) -- undo the excess work of the
// recursive reflections and exchanges from the top bit down, Gray-encode
// across axes, then read the index bits axis-interleaved, top bit first.
__device__ __forceinline__ uint32_t hilbert_nd(uint32_t (&x)[4], int n, int b) {
  const uint32_t top = 1u << (b - 1);
  for (uint32_t q = top; q > 1; q >>= 1) {
    const uint32_t low = q - 1;
    for (int i = 0; i < n; ++i) {
      if (x[i] & q) {
        x[0] ^= low;
      } else {
        const uint32_t t = (x[0] ^ x[i]) & low;
        x[0] ^= t;
        x[i] ^= t;
      }
    }
  }
  for (int i = 1; i < n; ++i) x[i] ^= x[i - 1];
  uint32_t t = 0;
  for (uint32_t q = top; q > 1; q >>= 1)
    if (x[n - 1] & q) t ^= q - 1;
  for (int i = 0; i < n; ++i) x[i] ^= t;
  uint32_t h = 0;
  for (int bit = b - 1; bit >= 0; --bit)
    for (int i = 0; i < n; ++i) h = (h << 1) | ((x[i] >> bit) & 1u);
  return h;
}

// Keys of one order set (see OrderJob).  One workgroup per set: the series'
// range first (for the scaling), then one key per time point.
__global__ __launch_bounds__(256) void k_order_keys(const OrderJob* __restrict__ jobs,
                                                    const float* __restrict__ s32,
                                                    uint32_t* __restrict__ keys) {
  __shared__ float s_lo[256], s_hi[256];
  const OrderJob J = jobs[blockIdx.x];
  const float* __restrict__ s = s32 + J.src_off;
  uint32_t* __restrict__ k = keys + J.key_off;
  const int tid = threadIdx.x;
  const int dims = J.dims;
  int64_t lag_max = 0;
  for (int d = 0; d < dims; ++d) lag_max = max(lag_max, (int64_t)J.lag[d]);
  if (dims == 1) {
    for (int64_t t = tid; t < J.n; t += 256)
      k[t] = t + lag_max < J.n ? ordered_bits(s[t + J.lag[0]]) : 0xffffffffu;
    return;
  }
  float lo = __builtin_inff(), hi = -__builtin_inff();
  for (int64_t t = tid; t < J.n; t += 256) {
    lo = fminf(lo, s[t]);
    hi = fmaxf(hi, s[t]);
  }
  s_lo[tid] = lo;
  s_hi[tid] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      s_lo[tid] = fminf(s_lo[tid], s_lo[tid + w]);
      s_hi[tid] = fmaxf(s_hi[tid], s_hi[tid + w]);
    }
    __syncthreads();
  }
  lo = s_lo[0];
  const int bits = dims == 2 ? 16 : 32 / dims;
  const float top = (float)((1u << bits) - 1u);
  const float span = s_hi[0] - lo;
  const float scale = span > 0.f ? top / span : 0.f;
  for (int64_t i = tid; i < J.n; i += 256) {
    if (i + lag_max >= J.n) {
      k[i] = 0xffffffffu;
      continue;
    }
    uint32_t x[4] = {0u, 0u, 0u, 0u};
    for (int d = 0; d < dims; ++d)
      x[d] = (uint32_t)fminf(top, fmaxf(0.f, (s[i + J.lag[d]] - lo) * scale));
    k[i] = dims == 2 ? hilbert16(x[0], x[1]) : hilbert_nd(x, dims, bits);
  }
}

// Smallest and largest value over the 256 threads of a workgroup (every
// thread gets both).
__device__ __forceinline__ void block_minmax(float& lo, float& hi, float* s_lo, float* s_hi) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  lo = fminf(fminf(s_lo[0], s_lo[1]), fminf(s_lo[2], s_lo[3]));
  hi = fmaxf(fmaxf(s_hi[0], s_hi[1]), fmaxf(s_hi[2], s_hi[3]));
}

// One level of the k-d refinement (see OrderJob): workgroup (x, y) splits
// node x of set y -- positions [lo, hi) = [x n_e / 2^level, (x+1) n_e /
// 2^level) of the set's order -- at its median along the coordinate with the
// widest range over the node (the first such coordinate on ties).  The h =
// mid - lo smallest (coordinate, position) entries go to [lo, mid), the rest
// to [mid, hi), each side in its input order, where mid = (2x+1) n_e /
// 2^(level+1) is the next level's boundary between the node's halves.  The
// h-th smallest coordinate T is found by a radix select on its ordered bits
// (four 8-bit passes, histograms in LDS); the entries below T and the first
// ones equal to T make up the lower half (the node's keys are formed once
// into `keys`, scratch of the pool's size).  Sets set0 + blockIdx.y.  Input
// `order`, output `out` (the
// caller has copied every entry to out first, so nodes that do not split
// keep their entries).
__global__ __launch_bounds__(kBlock) void k_kd_split(const OrderJob* __restrict__ orders,
                                                     int set0, int level,
                                                     const float* __restrict__ emb,
                                                     const int32_t* __restrict__ order,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ out) {
  __shared__ float s_lo[kBlock / 64][kMaxE], s_hi[kBlock / 64][kMaxE];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_pick[2];
  __shared__ int s_wave[2][kBlock / 64];
  const OrderJob J = orders[set0 + (int)blockIdx.y];
  if (J.kd_E <= 0 || level >= J.kd_levels) return;
  const int E = J.kd_E;
  const int64_t x = blockIdx.x;
  const int64_t lo = (x * J.kd_n_e) >> level;
  const int64_t hi = ((x + 1) * J.kd_n_e) >> level;
  const int64_t mid = ((2 * x + 1) * J.kd_n_e) >> (level + 1);
  const int64_t h = mid - lo;                       // entries of the lower half
  if (h <= 0 || h >= hi - lo) return;               // nothing moves
  const float* __restrict__ e = emb + J.kd_emb_off;
  const int32_t* __restrict__ o = order + J.key_off;
  int32_t* __restrict__ w = out + J.key_off;
  const int tid = threadIdx.x;

  // the widest coordinate: every coordinate's range in one pass
  float mn[kMaxE], mx[kMaxE];
#pragma unroll
  for (int k = 0; k < kMaxE; ++k) {
    mn[k] = __builtin_inff();
    mx[k] = -__builtin_inff();
  }
  for (int64_t p = lo + tid; p < hi; p += kBlock) {
    const float* __restrict__ v = e + (int64_t)o[p] * E;
#pragma unroll
    for (int k = 0; k < kMaxE; ++k)
      if (k < E) {
        mn[k] = fminf(mn[k], v[k]);
        mx[k] = fmaxf(mx[k], v[k]);
      }
  }
  const int wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < kMaxE; ++k) {
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
      mn[k] = fminf(mn[k], __shfl_xor(mn[k], sh, 64));
      mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], sh, 64));
    }
    if ((tid & 63) == 0) {
      s_lo[wave][k] = mn[k];
      s_hi[wave][k] = mx[k];
    }
  }
  __syncthreads();
  int d = 0;
  float width = -1.f;
  for (int k = 0; k < E; ++k) {
    float a = s_lo[0][k], b = s_hi[0][k];
#pragma unroll
    for (int wv = 1; wv < kBlock / 64; ++wv) {
      a = fminf(a, s_lo[wv][k]);
      b = fmaxf(b, s_hi[wv][k]);
    }
    if (b - a > width) {
      width = b - a;
      d = k;
    }
  }
  // the node's keys, formed once (scratch of the order pool's size)
  uint32_t* __restrict__ kc = keys + J.key_off;
  for (int64_t p = lo + tid; p < hi; p += kBlock) kc[p] = ordered_bits(e[(int64_t)o[p] * E + d]);

  // radix select of the key of rank h - 1 (0-based); each thread reads the
  // keys it wrote
  uint32_t prefix = 0u, mask = 0u;
  uint32_t rank = (uint32_t)(h - 1);
  for (int shift = 24; shift >= 0; shift -= 8) {
    hist[tid] = 0u;
    __syncthreads();
    for (int64_t p = lo + tid; p < hi; p += kBlock) {
      const uint32_t key = kc[p];
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t cum = 0u, b = 0u;
      for (; b < 255u && cum + hist[b] <= rank; ++b) cum += hist[b];
      s_pick[0] = b;
      s_pick[1] = rank - cum;
    }
    __syncthreads();
    prefix |= s_pick[0] << shift;
    mask |= 255u << shift;
    rank = s_pick[1];
    __syncthreads();
  }
  const uint32_t T = prefix;
  const int64_t eq_left = (int64_t)rank + 1;      // entries equal to T in the lower half

  // stable partition, 256 entries at a time
  int64_t at_lo = lo, at_hi = mid, eq_seen = 0;
  for (int64_t base = lo; base < hi; base += kBlock) {
    const int64_t p = base + tid;
    const bool valid = p < hi;
    const int32_t idx = valid ? o[p] : 0;
    const uint32_t key = valid ? kc[p] : 0u;
    const bool is_eq = valid && key == T;
    int n_eq;
    const int r_eq = block_rank(is_eq, s_wave[0], n_eq);
    const bool left = valid && (key < T || (is_eq && eq_seen + r_eq < eq_left));
    int n_left;
    const int r_left = block_rank(left, s_wave[1], n_left);
    if (left) w[at_lo + r_left] = idx;
    else if (valid) w[at_hi + (tid - r_left)] = idx;
    const int64_t n_valid = hi - base < kBlock ? hi - base : kBlock;
    at_lo += n_left;
    at_hi += n_valid - n_left;
    eq_seen += n_eq;
  }
}

__global__ void k_copy_int(const int32_t* __restrict__ src, int32_t* __restrict__ dst,
                           int64_t n) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x)
    dst[x] = src[x];
}

// Embedded points in visiting order: the order set restricted to indices
// below n_e.  One workgroup per embedding.
__global__ __launch_bounds__(kBlock) void k_query_order(
    const EmbedJob* __restrict__ jobs, const int32_t* __restrict__ order_pool,
    int32_t* __restrict__ qord_pool) {
  __shared__ int s_wave[kBlock / 64];
  const EmbedJob J = jobs[blockIdx.x];
  const int32_t* __restrict__ ord = order_pool + J.order_off;
  int32_t* __restrict__ q = qord_pool + J.qord_off;
  int64_t out = 0;
  for (int64_t base = 0; base < J.n_series; base += kBlock) {
    const int64_t k = base + threadIdx.x;
    const int64_t i = k < J.n_series ? ord[k] : J.n_e;
    const bool f = i < J.n_e;
    int total;
    const int r = block_rank(f, s_wave, total);
    if (f) q[out + r] = (int32_t)i;
    out += total;
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
//
// One wavefront per library.  The stream's state advances by the same
// constant for every candidate visited, so candidate j's draw is the output
// mix of (keyed state + (j+1) gamma): the 64 lanes form the draws and their
// integers u_j below (n_e - j) of 64 consecutive candidates at once.  The
// decisions depend on how many were taken before (t_j = needed before j;
// take j when u_j < t_j), but within 64 candidates t_j is at most 63 below
// the step's t_0: u_j < t_0 - 63 is taken and u_j >= t_0 is not whatever
// came before, and only the lanes in between are decided one after another,
// in candidate order, with the count of takes below them.  Then t_j is known
// for every lane, and the first j with t_j = n_e - j (every remaining one
// needed) takes the rest.  Each u_j is below n_e < 2^31.
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

__global__ __launch_bounds__(256) void k_sample(const SampleJob* __restrict__ jobs,
                                                int64_t n_jobs,
                                                int32_t* __restrict__ out_pool) {
  const int lane = threadIdx.x & 63;
  const int64_t id = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (id >= n_jobs) return;                       // the whole wavefront
  const SampleJob J = jobs[id];
  uint64_t st = 0;
  st = sm_mix(st ^ J.seed);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.E);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.tau);
  st = sm_mix(st ^ (uint64_t)J.l_eff);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.r_index);
  int32_t* __restrict__ out = out_pool + J.out_off;
  const int64_t ne = J.n_e, le = J.l_eff;
  const uint64_t below_lane = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int64_t s = 0;                                  // taken so far
  for (int64_t j0 = 0; s < le && j0 < ne; j0 += 64) {
    const int64_t j = j0 + lane;
    const bool valid = j < ne;
    int64_t u = 0;
    if (valid)
      u = (int64_t)__umul64hi(sm_mix(st + (uint64_t)(j + 1) * kGamma), (uint64_t)(ne - j));
    const int64_t t0 = le - s;
    uint64_t take = __builtin_amdgcn_ballot_w64(valid && u + 63 < t0);
    uint64_t open = __builtin_amdgcn_ballot_w64(valid && u + 63 >= t0 && u < t0);
    while (open) {                                // in candidate order
      const int l = __builtin_ctzll(open);
      open &= open - 1ull;
      const int64_t tl = t0 - __popcll(take & ((1ull << l) - 1ull));
      const int64_t ul = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)u, l);
      if (ul < tl) take |= 1ull << l;
    }
    // the first candidate from which every remaining one is needed
    const int64_t tj = t0 - __popcll(take & below_lane);
    const uint64_t full = __builtin_amdgcn_ballot_w64(valid && tj == ne - j);
    int64_t rest = -1;
    if (full) {
      const int l = __builtin_ctzll(full);
      rest = j0 + l;
      take &= (1ull << l) - 1ull;
    }
    if ((take >> lane) & 1ull) out[s + __popcll(take & below_lane)] = (int32_t)j;
    s += __popcll(take);
    if (rest >= 0) {
      for (int64_t k = lane; k < le - s; k += 64) out[s + k] = (int32_t)(rest + k);
      s = le;
    }
  }
}

// Nested libraries (an option of this library): the first n_out points of
// the forward Fisher-Yates shuffle (Durstenfeld 1964; Knuth's Algorithm P,
// TAOCP Vol. 2, Sec. 3.4.2) of 0..n_e-1: step k swaps position k with
// position k + floor(z_k (n_e - k) / 2^64), z_k the k-th SplitMix64 output
// of the stream keyed by (seed, E, tau, r).  One workgroup per job: the
// positions are set to the identity in parallel, then one lane shuffles.
__global__ __launch_bounds__(kBlock) void k_sample_nested(const NestedJob* __restrict__ jobs,
                                                          int32_t* __restrict__ scratch,
                                                          int32_t* __restrict__ out_pool) {
  const NestedJob J = jobs[blockIdx.x];
  int32_t* __restrict__ a = scratch + J.scratch_off;
  for (int64_t i = threadIdx.x; i < J.n_e; i += kBlock) a[i] = (int32_t)i;
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint64_t st = 0;
  st = sm_mix(st ^ J.seed);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.E);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.tau);
  st = sm_mix(st ^ (uint64_t)(int64_t)J.r_index);
  int32_t* __restrict__ out = out_pool + J.out_off;
  for (int64_t k = 0; k < J.n_out; ++k) {
    st += kGamma;
    const uint64_t z = sm_mix(st);
    const int64_t j = k + (int64_t)__umul64hi(z, (uint64_t)(J.n_e - k));
    const int32_t t = a[k];
    a[k] = a[j];
    a[j] = t;
    out[k] = a[k];
  }
}

// The library of one realization, laid out contiguously in visiting order
// (coordinates AoS and embedded indices), so the scan
// streams it through the scalar cache with no dependent index load.  For each
// wavefront of each query tile (a wavefront takes a run of consecutive
// queries in the same order) it records the library position of the run's
// middle query: that wavefront's scan starts there and works outward.  One
// workgroup per job; the library's membership bitmask lives in LDS (dynamic
// size).  Jobs marked unsorted keep ascending index order and start every
// scan at position 0.
__global__ __launch_bounds__(kBlock) void k_gather(
    const GatherJob* __restrict__ jobs, const float* __restrict__ emb_pool,
    const int32_t* __restrict__ lib_pool, const int32_t* __restrict__ order_pool,
    float* __restrict__ pts_pool, int32_t* __restrict__ pj_pool,
    int32_t* __restrict__ start_pool) {
  extern __shared__ uint32_t bits[];
  __shared__ int s_wave[2][kBlock / 64];
  const GatherJob J = jobs[blockIdx.x];
  const float* __restrict__ emb = emb_pool + J.emb_off;
  const int32_t* __restrict__ lib = lib_pool + J.lib_off;
  float* __restrict__ pts = pts_pool + J.pts_off;
  int32_t* __restrict__ pj = pj_pool + J.pj_off;
  int32_t* __restrict__ start = start_pool + J.start_off;
  const int E = J.E;
  const int tid = threadIdx.x;

  if (!J.sorted) {
    for (int64_t x = tid; x < J.l_eff * E; x += kBlock) {
      const int64_t c = x / E;
      const int k = (int)(x - c * E);
      pts[x] = emb[(int64_t)lib[c] * E + k];
    }
    for (int64_t c = tid; c < J.l_eff; c += kBlock) pj[c] = lib[c];
    if (J.query_set == 0) {
      const int64_t n_start = (J.n_e + J.qt - 1) / J.qt * kWaves;
      for (int64_t t = tid; t < n_start; t += kBlock) start[t] = 0;
    }
    return;
  }

  const int64_t nw = (J.n_e + 31) / 32;
  for (int64_t w = tid; w < nw; w += kBlock) bits[w] = 0u;
  __syncthreads();
  for (int64_t c = tid; c < J.l_eff; c += kBlock) {
    const int32_t j = lib[c];
    atomicOr(&bits[j >> 5], 1u << (j & 31));
  }
  __syncthreads();

  const int32_t* __restrict__ ord = order_pool + J.order_off;
  int64_t pf = 0;   // embedded points passed so far (in order)
  int64_t pl = 0;   // library points passed so far (in order)
  for (int64_t base = 0; base < J.n_series; base += kBlock) {
    const int64_t k = base + tid;
    const int64_t t = k < J.n_series ? ord[k] : J.n_e;
    const bool fo = t < J.n_e;
    const int64_t i = fo ? t : 0;
    const bool fl = fo && ((bits[i >> 5] >> (i & 31)) & 1u);
    int tot_o, tot_l;
    const int ro = block_rank(fo, s_wave[0], tot_o);
    const int rl = block_rank(fl, s_wave[1], tot_l);
    if (fl) {
      const int64_t c = pl + rl;
      pj[c] = (int32_t)i;
      for (int kk = 0; kk < E; ++kk) pts[c * E + kk] = emb[i * E + kk];
    }
    if (fo && J.query_set == 0) {
      // wavefront w of tile t takes query positions [s*sub, (s+1)*sub) with
      // s = t*kWaves + w; its scan starts at its middle query
      const int64_t sub = J.qt / kWaves;
      const int64_t p = pf + ro;
      const int64_t sw = p / sub;
      const int64_t anchor = min(sw * sub + sub / 2, J.n_e - 1);
      if (p == anchor) start[sw] = (int32_t)(pl + rl);
    }
    pf += tot_o;
    pl += tot_l;
  }
}

__global__ void k_finalize_multi(const Realization* __restrict__ rzs,
                                 const int32_t* __restrict__ self_of, int64_t n_rz,
                                 int m_series, const Sums* __restrict__ partial,
                                 int64_t out_stride_b, double* __restrict__ out) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= n_rz * m_series) return;
  const int64_t r = x / m_series;
  const int bt = (int)(x - r * m_series);
  const Realization R = rzs[r];
  double rho = __builtin_nan("");
  if (bt != self_of[r]) {
    Sums a;
#pragma unroll
    for (int i = 0; i < 6; ++i) a.v[i] = 0.0;
    a.v[6] = a.v[8] = __builtin_inf();
    a.v[7] = a.v[9] = -__builtin_inf();
    for (int t = 0; t < R.n_tiles; ++t) sums_merge(a, partial[(R.slot_base + t) * m_series + bt]);
    const double n = a.v[0];
    const double vo = n * a.v[3] - a.v[1] * a.v[1];
    const double vp = n * a.v[4] - a.v[2] * a.v[2];
    const double cv = n * a.v[5] - a.v[1] * a.v[2];
    if (a.v[6] < a.v[7] && a.v[8] < a.v[9] && vo > 0.0 && vp > 0.0) rho = cv / sqrt(vo * vp);
  }
  out[R.out_index + bt * out_stride_b] = rho;
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
// host-side launchers (the runtime calls only these)
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}

int shared_queries_per_lane(int emax) {
  return emax >= 1 && emax <= kMaxE ? kSharedQ[emax] : 0;
}

int crossmap_queries_per_lane(int E) { return E >= 1 && E <= kMaxE ? kTuneQ[E] : 0; }

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

hipError_t launch_iota_segments(int32_t* out, int64_t n_series, int32_t segs,
                                hipStream_t st) {
  const int64_t total = n_series * segs;
  if (total <= 0) return hipSuccess;
  k_iota_segments<<<blocks_for(total, 256), 256, 0, st>>>(out, n_series, total);
  return hipGetLastError();
}

hipError_t launch_order_keys(const OrderJob* jobs, int n_jobs, const float* s32,
                             uint32_t* keys, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  k_order_keys<<<n_jobs, 256, 0, st>>>(jobs, s32, keys);
  return hipGetLastError();
}

hipError_t launch_query_order(const EmbedJob* jobs, int n_jobs,
                              const int32_t* order, int32_t* qord, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  k_query_order<<<n_jobs, kBlock, 0, st>>>(jobs, order, qord);
  return hipGetLastError();
}

hipError_t refine_orders_kd(const OrderJob* orders, int32_t n_sets, int levels,
                            int64_t n_series, const float* emb, int32_t* order, int32_t* alt,
                            uint32_t* keys, hipStream_t st) {
  if (n_sets <= 0 || levels <= 0) return hipSuccess;
  const int64_t n = n_series * n_sets;
  int32_t* cur = order;
  int32_t* nxt = alt;
  for (int lv = 0; lv < levels; ++lv) {
    k_copy_int<<<blocks_for(n, 256), 256, 0, st>>>(cur, nxt, n);
    for (int32_t s0 = 0; s0 < n_sets; s0 += 65535) {
      const unsigned ny = (unsigned)std::min<int32_t>(65535, n_sets - s0);
      k_kd_split<<<dim3(1u << lv, ny), kBlock, 0, st>>>(orders, s0, lv, emb, cur, keys, nxt);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (cur != order) k_copy_int<<<blocks_for(n, 256), 256, 0, st>>>(cur, order, n);
  return hipGetLastError();
}


hipError_t launch_sample(const SampleJob* jobs, int64_t n_jobs, int32_t* out,
                         hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_jobs + 3) / 4);   // one wavefront per library
  k_sample<<<blocks, 256, 0, st>>>(jobs, n_jobs, out);
  return hipGetLastError();
}

// Membership bitmasks up to 48 KiB of LDS per workgroup.
static constexpr int64_t kGatherBitmaskWords = 12 * 1024;

int64_t gather_max_sorted_n_e() { return kGatherBitmaskWords * 32; }

hipError_t launch_gather(const GatherJob* jobs, int64_t n_jobs, int64_t max_n_e,
                         const float* emb, const int32_t* lib, const int32_t* order,
                         float* pts, int32_t* pj, int32_t* start, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  // max_n_e covers the jobs marked sorted; larger ones must be unsorted
  int64_t words = (max_n_e + 31) / 32;
  if (words > kGatherBitmaskWords) return hipErrorInvalidValue;
  if (words < 1) words = 1;
  k_gather<<<(unsigned)n_jobs, kBlock, (size_t)words * 4, st>>>(jobs, emb, lib, order,
                                                                 pts, pj, start);
  return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_zero_int<<<(n + 255) / 256, 256, 0, st>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_table_build(int E, const TableJob* jobs, int n_jobs, int max_n_e,
                              const float* emb, int32_t* table, hipStream_t st) {
  if (n_jobs <= 0 || max_n_e <= 0) return hipSuccess;
  switch (E) {
#define CCM_TCASE(e) \
  case e:            \
    return launch_table_build_e<e>(jobs, n_jobs, max_n_e, emb, table, st);
    CCM_TCASE(1) CCM_TCASE(2) CCM_TCASE(3) CCM_TCASE(4) CCM_TCASE(5)
    CCM_TCASE(6) CCM_TCASE(7) CCM_TCASE(8) CCM_TCASE(9) CCM_TCASE(10)
#undef CCM_TCASE
    default:
      return hipErrorInvalidValue;
  }
}

// Two device arrays of n doubles to one buffer, or one buffer to two
// arrays, in a single launch (the device forms' series in and results out).
__global__ void k_copy_pair(const double* __restrict__ a, const double* __restrict__ b,
                            int64_t n, double* __restrict__ dst) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < 2 * n;
       x += (int64_t)gridDim.x * blockDim.x)
    dst[x] = x < n ? a[x] : b[x - n];
}

__global__ void k_split_pair(const double* __restrict__ src, int64_t n, double* __restrict__ a,
                             double* __restrict__ b) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < 2 * n;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < n)
      a[x] = src[x];
    else
      b[x - n] = src[x];
  }
}

hipError_t launch_copy_pair(const double* a, const double* b, int64_t n, double* dst,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_copy_pair<<<blocks_for(2 * n, 256), 256, 0, st>>>(a, b, n, dst);
  return hipGetLastError();
}

hipError_t launch_split_pair(const double* src, int64_t n, double* a, double* b,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_split_pair<<<blocks_for(2 * n, 256), 256, 0, st>>>(src, n, a, b);
  return hipGetLastError();
}

hipError_t launch_sample_nested(const NestedJob* jobs, int64_t n_jobs, int32_t* scratch,
                                int32_t* out_pool, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  k_sample_nested<<<(unsigned)n_jobs, kBlock, 0, st>>>(jobs, scratch, out_pool);
  return hipGetLastError();
}

hipError_t launch_crossmap_nested(int E, int mode, int grid, const Realization* rzs,
                                  const Item* items, int n_items, int* next,
                                  const float* emb, const float* pts, const int32_t* pj,
                                  const int32_t* qord, const int32_t* start, const double* tgt,
                                  const int32_t* seg, Moments* partial, int window,
                                  hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (E) {
#define CCM_NCASE(e)                                                                   \
  case e:                                                                              \
    return launch_nested_e<e>(mode, grid, rzs, items, n_items, next, emb, pts, pj, qord, \
                              start, tgt, seg, partial, window, st);
    CCM_NCASE(1) CCM_NCASE(2) CCM_NCASE(3) CCM_NCASE(4) CCM_NCASE(5)
    CCM_NCASE(6) CCM_NCASE(7) CCM_NCASE(8) CCM_NCASE(9) CCM_NCASE(10)
#undef CCM_NCASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_crossmap_shared(int emax, int mode, int grid, const Realization* rzs,
                                  const Item* items, int n_items, int* next,
                                  const float* emb, const float* pts, const int32_t* pj,
                                  const int32_t* qord, const int32_t* start, const double* tgt,
                                  Moments* partial, int window, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (emax) {
#define CCM_SCASE(e)                                                                     \
  case e:                                                                                \
    return launch_shared_e<e>(mode, grid, rzs, items, n_items, next, emb, pts, pj, qord,  \
                              start, tgt, partial, window, st);
    CCM_SCASE(1) CCM_SCASE(2) CCM_SCASE(3) CCM_SCASE(4) CCM_SCASE(5)
    CCM_SCASE(6) CCM_SCASE(7) CCM_SCASE(8) CCM_SCASE(9) CCM_SCASE(10)
#undef CCM_SCASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_crossmap(int E, int mode, int grid,
                           const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb,
                           const float* pts, const int32_t* pj,
                           const int32_t* qord, const int32_t* start,
                           const double* tgt, Moments* partial, int query_set,
                           int window, Dump d, const int32_t* table, int table_n_e,
                           hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (E) {
#define CCM_CASE(e)                                                                         \
  case e:                                                                                   \
    return launch_crossmap_e<e>(mode, grid, rzs, items, n_items, next, emb, pts, pj, qord,  \
                                start, tgt, partial, query_set, window, d, table, table_n_e, \
                                st);
    CCM_CASE(1) CCM_CASE(2) CCM_CASE(3) CCM_CASE(4) CCM_CASE(5)
    CCM_CASE(6) CCM_CASE(7) CCM_CASE(8) CCM_CASE(9) CCM_CASE(10)
#undef CCM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

__global__ void k_transpose_targets(const double* __restrict__ s64, int m, int mp, int64_t n,
                                    double* __restrict__ tt) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n * mp;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = x / mp;
    const int b = (int)(x - t * mp);
    tt[x] = b < m ? s64[(int64_t)b * n + t] : 0.0;
  }
}

hipError_t launch_transpose_targets(const double* s64, int m_series, int64_t n, double* tt,
                                    hipStream_t st) {
  const int mp = target_stride(m_series);
  k_transpose_targets<<<blocks_for(n * mp, 256), 256, 0, st>>>(s64, m_series, mp, n, tt);
  return hipGetLastError();
}

hipError_t launch_crossmap_multi(int E, int mode, int grid, const Realization* rzs,
                                 const int32_t* self_of, const Item* items, int n_items,
                                 int* next, const float* emb, const float* pts,
                                 const int32_t* pj, const int32_t* qord, const int32_t* start,
                                 const double* tt, int m_series,
                                 void* partial, int query_set, int window,
                                 const int32_t* table, int table_n_e, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (E) {
#define CCM_MCASE(e)                                                                      \
  case e:                                                                                 \
    return launch_multi_e<e>(mode, grid, rzs, self_of, items, n_items, next, emb, pts, pj, \
                             qord, start, tt, m_series, partial, query_set, window, table,  \
                             table_n_e, st);
    CCM_MCASE(1) CCM_MCASE(2) CCM_MCASE(3) CCM_MCASE(4) CCM_MCASE(5)
    CCM_MCASE(6) CCM_MCASE(7) CCM_MCASE(8) CCM_MCASE(9) CCM_MCASE(10)
#undef CCM_MCASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize_multi(const Realization* rzs, const int32_t* self_of,
                                 int64_t n_rz, int m_series, const void* partial,
                                 int64_t out_stride_b, double* out, hipStream_t st) {
  const int64_t n = n_rz * m_series;
  if (n <= 0) return hipSuccess;
  k_finalize_multi<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
      rzs, self_of, n_rz, m_series, static_cast<const Sums*>(partial), out_stride_b, out);
  return hipGetLastError();
}

size_t multi_sums_bytes() { return sizeof(Sums); }

hipError_t launch_finalize(const Realization* rzs, int64_t n_rz,
                           const Moments* partial, double* out, hipStream_t st) {
  if (n_rz <= 0) return hipSuccess;
  k_finalize<<<(unsigned)((n_rz + 255) / 256), 256, 0, st>>>(rzs, n_rz, partial, out);
  return hipGetLastError();
}

}  // namespace ccmk

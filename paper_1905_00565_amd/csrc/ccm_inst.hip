// ccm_inst.hip -- the kernels of one embedding dimension.  The build compiles
// this file once per E = 1..10 with -DCCM_INST_E=E, so the instances of the
// ten dimensions compile in parallel; each object holds the cross-map
// (plain, test-hook and table variants of every exclusion mode), the
// nested-library, E-sweep-sharing (E_max = E) and table-build kernels of its
// E, and their launchers.  The causal-matrix kernels are in
// ccm_inst_multi.hip.
#include "ccm_device.h"
#include "ccm_inst.h"

#ifndef CCM_INST_E
#error "compile with -DCCM_INST_E=<embedding dimension>"
#endif

namespace ccmk {

using CrossmapFn = void (*)(const Realization*, const Item*, int, int*,
                            const float*, const float*, const int32_t*,
                            const int32_t*, const int32_t*, const double*,
                            Moments*, int, int, Dump, TableArgs);

template <int E, int Q, bool DUMP, bool TBL>
static CrossmapFn crossmap_for_mode(int mode) {
  switch (mode) {
    case kExclSelf: return k_crossmap<E, Q, kExclSelf, DUMP, TBL>;
    case kKeepSelf: return k_crossmap<E, Q, kKeepSelf, DUMP, TBL>;
    default: return k_crossmap<E, Q, kWindow, DUMP, TBL>;
  }
}

template <int E>
hipError_t launch_crossmap_e(int mode, int grid, const Realization* rzs, const Item* items,
                             int n_items, int* next, const float* emb, const float* pts,
                             const int32_t* pj, const int32_t* qord, const int32_t* start,
                             const double* tgt, Moments* partial, int query_set, int window,
                             Dump d, const int32_t* table, int table_n_e, hipStream_t st) {
  constexpr int Q = DefaultQ<E>::Q;
  const bool dump = d.nbr != nullptr, tbl = table_n_e > 0;
  const CrossmapFn f = dump ? (tbl ? crossmap_for_mode<E, Q, true, true>(mode)
                                   : crossmap_for_mode<E, Q, true, false>(mode))
                            : (tbl ? crossmap_for_mode<E, Q, false, true>(mode)
                                   : crossmap_for_mode<E, Q, false, false>(mode));
  const TableArgs ta{table, table_lds_words(table_n_e), 0};
  hipLaunchKernelGGL(f, dim3((unsigned)grid), dim3(kBlock), table_lds_bytes(E, table_n_e), st,
                     rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, partial,
                     query_set, window, d, ta);
  return hipGetLastError();
}

template <int E>
hipError_t launch_nested_e(int mode, int grid, const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb, const float* pts,
                           const int32_t* pj, const int32_t* qord, const int32_t* start,
                           const double* tgt, const int32_t* seg, Moments* partial, int window,
                           hipStream_t st) {
  constexpr int Q = DefaultQ<E>::Q;
  switch (mode) {
    case kExclSelf:
      k_crossmap_nested<E, Q, kExclSelf><<<grid, kBlock, 0, st>>>(
          rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, seg, partial, window);
      break;
    case kKeepSelf:
      k_crossmap_nested<E, Q, kKeepSelf><<<grid, kBlock, 0, st>>>(
          rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, seg, partial, window);
      break;
    default:
      k_crossmap_nested<E, Q, kWindow><<<grid, kBlock, 0, st>>>(
          rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, seg, partial, window);
      break;
  }
  return hipGetLastError();
}

template <int EMAX>
hipError_t launch_shared_e(int mode, int grid, const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb, const float* pts,
                           const int32_t* pj, const int32_t* qord, const int32_t* start,
                           const double* tgt, Moments* partial, int window, hipStream_t st) {
  switch (mode) {
    case kExclSelf:
      k_crossmap_shared<EMAX, kExclSelf><<<grid, kBlock, 0, st>>>(
          rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, partial, window);
      break;
    case kKeepSelf:
      k_crossmap_shared<EMAX, kKeepSelf><<<grid, kBlock, 0, st>>>(
          rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, partial, window);
      break;
    default:
      k_crossmap_shared<EMAX, kWindow><<<grid, kBlock, 0, st>>>(
          rzs, items, n_items, next, emb, pts, pj, qord, start, tgt, partial, window);
      break;
  }
  return hipGetLastError();
}

template <int E>
hipError_t launch_table_build_e(const TableJob* jobs, int n_jobs, int max_n_e, const float* emb,
                                int32_t* table, hipStream_t st) {
  const dim3 grid((unsigned)max_n_e, (unsigned)n_jobs);
  k_table_build<E><<<grid, kBlock, 0, st>>>(jobs, emb, table);
  return hipGetLastError();
}

template hipError_t launch_crossmap_e<CCM_INST_E>(int, int, const Realization*, const Item*, int,
                                                  int*, const float*, const float*,
                                                  const int32_t*, const int32_t*,
                                                  const int32_t*, const double*, Moments*, int,
                                                  int, Dump, const int32_t*, int, hipStream_t);
template hipError_t launch_nested_e<CCM_INST_E>(int, int, const Realization*, const Item*, int,
                                                int*, const float*, const float*,
                                                const int32_t*, const int32_t*, const int32_t*,
                                                const double*, const int32_t*, Moments*, int,
                                                hipStream_t);
template hipError_t launch_shared_e<CCM_INST_E>(int, int, const Realization*, const Item*, int,
                                                int*, const float*, const float*,
                                                const int32_t*, const int32_t*, const int32_t*,
                                                const double*, Moments*, int, hipStream_t);
template hipError_t launch_table_build_e<CCM_INST_E>(const TableJob*, int, int, const float*,
                                                     int32_t*, hipStream_t);

}  // namespace ccmk

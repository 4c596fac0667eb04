// ccm_inst_multi.hip -- the causal-matrix (many-target) kernels of one
// embedding dimension, compiled once per E = 1..10 with -DCCM_INST_E=E.
//
// A unit of its own because it is built without machine-level loop-invariant
// hoisting (-mllvm -disable-machine-licm): with it, the compiler lifts the
// FP64 exp's polynomial coefficients of the per-target stage out of the
// persistent item loop into about twenty registers that then stay live
// through the whole neighbour scan, and the scan spills its running lists
// inside the insertion branches.  The cross-map kernels of ccm_inst.hip do
// not gain from the flag and keep the default pipeline.
#include "ccm_device.h"
#include "ccm_inst.h"

#ifndef CCM_INST_E
#error "compile with -DCCM_INST_E=<embedding dimension>"
#endif

namespace ccmk {

template <int E>
hipError_t launch_multi_e(int mode, int grid, const Realization* rzs, const int32_t* self_of,
                          const Item* items, int n_items, int* next, const float* emb,
                          const float* pts, const int32_t* pj, const int32_t* qord,
                          const int32_t* start, const double* tt, int m_series, void* partial,
                          int query_set, int window, const int32_t* table, int table_n_e,
                          hipStream_t st) {
  constexpr int Q = DefaultQ<E>::Q;
  const TableArgs ta{table, table_lds_words(table_n_e), 0};
  const size_t dyn = table_lds_bytes(E, table_n_e);
  using MultiFn = void (*)(const Realization*, const int32_t*, const Item*, int, int*,
                           const float*, const float*, const int32_t*, const int32_t*,
                           const int32_t*, const double*, int, Sums*, int, int, TableArgs);
  MultiFn f;
  const bool tbl = table_n_e > 0;
  switch (mode) {
    case kExclSelf:
      f = tbl ? k_crossmap_multi<E, Q, kExclSelf, true> : k_crossmap_multi<E, Q, kExclSelf, false>;
      break;
    case kKeepSelf:
      f = tbl ? k_crossmap_multi<E, Q, kKeepSelf, true> : k_crossmap_multi<E, Q, kKeepSelf, false>;
      break;
    default:
      f = tbl ? k_crossmap_multi<E, Q, kWindow, true> : k_crossmap_multi<E, Q, kWindow, false>;
      break;
  }
  hipLaunchKernelGGL(f, dim3((unsigned)grid), dim3(kBlock), dyn, st, rzs, self_of, items,
                     n_items, next, emb, pts, pj, qord, start, tt, m_series,
                     static_cast<Sums*>(partial), query_set, window, ta);
  return hipGetLastError();
}

template hipError_t launch_multi_e<CCM_INST_E>(int, int, const Realization*, const int32_t*,
                                               const Item*, int, int*, const float*,
                                               const float*, const int32_t*, const int32_t*,
                                               const int32_t*, const double*, int, void*, int,
                                               int, const int32_t*, int, hipStream_t);

}  // namespace ccmk

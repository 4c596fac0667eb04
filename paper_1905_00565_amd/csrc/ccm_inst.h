// ccm_inst.h -- launchers of the kernels that are compiled once per embedding
// dimension E (or E_max).  Each is defined in ccm_inst.hip and instantiated
// in the translation unit built for that E; the dispatchers in
// ccm_kernels.hip pick one by E.  Arguments as the dispatchers of the same
// name in ccm_internal.h.
#pragma once
#include "ccm_internal.h"

namespace ccmk {

template <int E>
hipError_t launch_crossmap_e(int mode, int grid, const Realization* rzs, const Item* items,
                             int n_items, int* next, const float* emb, const float* pts,
                             const int32_t* pj, const int32_t* qord, const int32_t* start,
                             const double* tgt, Moments* partial, int query_set, int window,
                             Dump d, const int32_t* table, int table_n_e, hipStream_t st);

template <int E>
hipError_t launch_multi_e(int mode, int grid, const Realization* rzs, const int32_t* self_of,
                          const Item* items, int n_items, int* next, const float* emb,
                          const float* pts, const int32_t* pj, const int32_t* qord,
                          const int32_t* start, const double* tt, int m_series, void* partial,
                          int query_set, int window, const int32_t* table, int table_n_e,
                          hipStream_t st);

template <int E>
hipError_t launch_nested_e(int mode, int grid, const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb, const float* pts,
                           const int32_t* pj, const int32_t* qord, const int32_t* start,
                           const double* tgt, const int32_t* seg, Moments* partial, int window,
                           hipStream_t st);

template <int EMAX>
hipError_t launch_shared_e(int mode, int grid, const Realization* rzs, const Item* items,
                           int n_items, int* next, const float* emb, const float* pts,
                           const int32_t* pj, const int32_t* qord, const int32_t* start,
                           const double* tgt, Moments* partial, int window, hipStream_t st);

template <int E>
hipError_t launch_table_build_e(const TableJob* jobs, int n_jobs, int max_n_e, const float* emb,
                                int32_t* table, hipStream_t st);

}  // namespace ccmk

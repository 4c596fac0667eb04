// ccm_tune.h -- launch shape of the cross-map kernel for each embedding
// dimension E (index 0 unused).  Written by paper_1905_00565_amd/autotune.py
// from timings of the E = 1..10, tau = 1..5 sweep on coupled-logistic series
// (N = 10000; r = 250 per (E, tau, L) for the kTune tables, r = 50 for the
// kShared tables); the build may override any table with -DCCM_TUNE_Q={...},
// -DCCM_TUNE_G={...} or -DCCM_TUNE_W={...} (the tuner does, to time
// candidates).
//
//   kTuneQ[E]  queries per lane (a workgroup of 256 lanes holds 256*Q queries)
//   kTuneG[E]  library candidates per trigger check (one group of G distances
//              per query, then one compare against its running E+1-th key)
//   kTuneW[E]  minimum wavefronts per SIMD the compiler must fit (register
//              budget 512/W per lane); 0 leaves it free
#pragma once

#ifndef CCM_TUNE_Q
#define CCM_TUNE_Q {0, 3, 4, 4, 4, 3, 2, 2, 2, 2, 2}
#endif
#ifndef CCM_TUNE_W
#define CCM_TUNE_W {0, 7, 6, 6, 6, 6, 7, 7, 6, 6, 6}
#endif
#ifndef CCM_TUNE_G
#define CCM_TUNE_G {0, 16, 12, 8, 6, 6, 4, 3, 4, 4, 3}
#endif

// E-sweep sharing: the scan at E_max keeps E_max (E_max + 3) / 2 keys per
// query, so its shape is chosen per E_max (index E_max):
//   kSharedQ  queries per lane;  kSharedG  candidates per trigger check;
//   kSharedW  minimum wavefronts per SIMD (0: free)
#ifndef CCM_SHARED_Q
#define CCM_SHARED_Q {0, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1}
#endif
#ifndef CCM_SHARED_G
#define CCM_SHARED_G {0, 8, 8, 8, 8, 6, 6, 4, 4, 4, 4}
#endif
#ifndef CCM_SHARED_W
#define CCM_SHARED_W {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 3}
#endif

// Nested libraries: minimum wavefronts per SIMD of the segmented scan (it
// keeps more state live than the plain scan, so a lower minimum than the
// plain scan's spills less; timed at r = 50 against no minimum and 4, 5 and
// the plain scan's table; 0: free).
#ifndef CCM_NESTED_W
#define CCM_NESTED_W {0, 7, 6, 4, 4, 4, 5, 4, 4, 4, 4}
#endif

// Group check per E (index E): 1 = the largest-coordinate bound (a cheaper
// check with the same outcome), 0 = the exact distances of the group.
#ifndef CCM_BOUND_CHECK
#define CCM_BOUND_CHECK {0, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0}
#endif

// One-sided remainder of the outward scan (index E): 1 = software-pipelined
// like the two-sided part (its scalar loads issued a group ahead), 0 = each
// group loaded when it is checked (at E >= 6 the pipelined form's extra
// scalar registers cost more than the loads it hides).
#ifndef CCM_PIPE_REST
#define CCM_PIPE_REST {0, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0}
#endif

// Causal matrix: minimum wavefronts per SIMD of the many-target kernel (its
// per-target stage holds more state than the plain scan's moments; 0: free).
#ifndef CCM_MULTI_W
#define CCM_MULTI_W {0, 5, 5, 5, 5, 5, 5, 5, 5, 5, 4}
#endif

namespace ccmk {
constexpr int kBoundCheck[11] = CCM_BOUND_CHECK;
constexpr int kPipeRest[11] = CCM_PIPE_REST;
constexpr int kMultiW[11] = CCM_MULTI_W;
constexpr int kNestedW[11] = CCM_NESTED_W;
constexpr int kTuneQ[11] = CCM_TUNE_Q;
constexpr int kTuneG[11] = CCM_TUNE_G;
constexpr int kTuneW[11] = CCM_TUNE_W;
constexpr int kSharedQ[11] = CCM_SHARED_Q;
constexpr int kSharedG[11] = CCM_SHARED_G;
constexpr int kSharedW[11] = CCM_SHARED_W;
}  // namespace ccmk

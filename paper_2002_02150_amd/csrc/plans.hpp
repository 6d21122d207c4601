// plans.hpp -- FFT plans of the supported segment lengths.
//
// N = N1 * N2 with N1 the pass-1 (column) length and N2 the pass-2 (row)
// length; radix-3 lengths (3 * 2^k) put the factor 3 in the length-768 rows.
// Lengths 2^k * 225 (whole minutes at 2048 Hz from 225 s up) add a middle
// pass of length NM = 225 = 15 * 15 between them (N = N1 * NM * N2).
// Work items hold 256 threads for float; the double variants halve the
// columns / rows per item where the LDS buffer would exceed 64 KiB.
#pragma once

#include "fitness_tiles.hpp"

namespace fcas {

// Pass 2 leaves one partial (maximum, sample) per wavefront of each work item:
// TILES2 * T2 / 64 per evaluation, at most kMaxParts2 over all plans.  A
// context sizes its partial buffers by the largest count among the plans its
// maximum segment length admits.
constexpr int kMaxParts2 = 16384;

template <int... R>
using Rad = Radices<R...>;

// clang-format off
#define FCAS_PLAN_LIST(X)                                                                          \
  /*  id     N      N1 E1 rad1          C(f) C(d)  N2  E2 rad2             RW(f) RW(d)  NM EM radM CM(f) CM(d) */ \
  X(0,   2048,     32, 8, (8, 4),       64, 64,   64, 8, (8, 8),          32, 32, 1, 1, (1), 1, 1) \
  X(1,   4096,     64, 8, (8, 8),       32, 32,   64, 8, (8, 8),          32, 32, 1, 1, (1), 1, 1) \
  X(2,   8192,     64, 8, (8, 8),       32, 32,  128, 16, (16, 8),        32, 16, 1, 1, (1), 1, 1) \
  X(3,  16384,    128, 16, (16, 8),     32, 16,  128, 16, (16, 8),        32, 16, 1, 1, (1), 1, 1) \
  X(4,  32768,    128, 16, (16, 8),     32, 16,  256, 16, (16, 16),       16, 8, 1, 1, (1), 1, 1) \
  X(5,  65536,    256, 16, (16, 16),    16, 8,   256, 16, (16, 16),       16, 8, 1, 1, (1), 1, 1) \
  X(6, 131072,    256, 16, (16, 16),    16, 8,   512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(7, 262144,    512, 16, (16, 16, 2), 8, 4,    512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(8,  24576,     32, 8, (8, 4),       64, 64,  768, 24, (8, 8, 4, 3),   8, 4, 1, 1, (1), 1, 1) \
  X(9,  49152,     64, 8, (8, 8),       32, 32,  768, 24, (8, 8, 4, 3),   8, 4, 1, 1, (1), 1, 1) \
  X(10, 98304,    128, 16, (16, 8),     32, 16,  768, 24, (8, 8, 4, 3),   8, 4, 1, 1, (1), 1, 1) \
  X(11, 196608,   256, 16, (16, 16),    16, 8,   768, 24, (8, 8, 4, 3),   8, 4, 1, 1, (1), 1, 1) \
  /* alternatives, picked per device by the autotuner */                                            \
  X(12, 131072,   128, 16, (16, 8),     32, 16, 1024, 16, (16, 16, 4),    4, 2, 1, 1, (1), 1, 1) \
  X(13, 131072,   256, 16, (16, 16),    16, 8,   512, 16, (16, 16, 2),    8, 4, 1, 1, (1), 1, 1) \
  X(14, 131072,   512, 16, (16, 16, 2), 8, 4,    256, 16, (16, 16),       16, 8, 1, 1, (1), 1, 1) \
  X(15, 131072,   256, 8, (8, 8, 4),    8, 8,    512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(16, 262144,   256, 16, (16, 16),    16, 8,  1024, 16, (16, 16, 4),    4, 2, 1, 1, (1), 1, 1) \
  X(17,  65536,   128, 16, (16, 8),     32, 16,  512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(18, 196608,   256, 16, (16, 16),    16, 8,   768, 12, (4, 4, 4, 4, 3), 4, 4, 1, 1, (1), 1, 1) \
  X(19,   8192,   128, 16, (16, 8),     32, 16,   64, 8, (8, 8),          32, 16, 1, 1, (1), 1, 1) \
  X(20, 262144,   256, 8, (8, 8, 4),    8, 8,   1024, 8, (8, 8, 8, 2),    2, 2, 1, 1, (1), 1, 1) \
  X(21, 196608,   256, 8, (8, 8, 4),    8, 8,    768, 12, (4, 4, 4, 4, 3), 4, 4, 1, 1, (1), 1, 1) \
  X(22,  65536,   256, 8, (8, 8, 4),    8, 8,    256, 8, (8, 8, 4),       8, 8, 1, 1, (1), 1, 1) \
  X(23,  65536,   128, 8, (8, 4, 4),    16, 16,  512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(24, 131072,   128, 8, (8, 4, 4),    16, 16, 1024, 8, (8, 8, 8, 2),    2, 2, 1, 1, (1), 1, 1) \
  /* three passes (N = N1 * 225 * N2): 225 s, 30 min and one hour at 2048 Hz;  */                 \
  /* 32 pass-1 columns per work item make 256-byte store segments              */                 \
  X(25,  460800,   32, 8, (8, 4),       64, 64,   64, 8, (8, 8),          32, 32, 225, 15, (15, 15), 16, 8) \
  X(26, 3686400,   64, 8, (8, 8),       32, 32,  256, 8, (8, 8, 4),       8, 8, 225, 15, (15, 15), 16, 8) \
  X(27, 7372800,   64, 8, (8, 8),       32, 32,  512, 8, (8, 8, 8),       4, 4, 225, 15, (15, 15), 16, 8) \
  X(28, 7372800,  128, 8, (8, 4, 4),    16, 16,  256, 8, (8, 8, 4),       8, 8, 225, 15, (15, 15), 16, 8) \
  X(29, 3686400,  256, 8, (8, 8, 4),    8, 8,     64, 8, (8, 8),          32, 32, 225, 15, (15, 15), 16, 8) \
  /* 512-thread pass 1 (twice the columns: 128- or 256-byte store segments)   */                 \
  X(30, 131072,   256, 8, (8, 8, 4),    16, 16,  512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(31, 262144,   256, 8, (8, 8, 4),    16, 16, 1024, 8, (8, 8, 8, 2),    2, 2, 1, 1, (1), 1, 1) \
  X(32,  65536,   128, 8, (8, 4, 4),    32, 32,  512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(33, 196608,   256, 8, (8, 8, 4),    16, 16,  768, 12, (4, 4, 4, 4, 3), 4, 4, 1, 1, (1), 1, 1) \
  X(34, 131072,   128, 8, (8, 4, 4),    16, 16, 1024, 16, (16, 16, 4),    4, 2, 1, 1, (1), 1, 1) \
  X(35, 262144,   512, 8, (8, 8, 8),    8, 8,    512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1) \
  X(36, 262144,   512, 8, (8, 8, 8),    16, 8,   512, 8, (8, 8, 8),       4, 4, 1, 1, (1), 1, 1)
// clang-format on

#define FCAS_UNPAREN(...) __VA_ARGS__

#define FCAS_DECLARE_PLAN(id, n, n1, e1, r1, cf, cd, n2, e2, r2, rwf, rwd, nm, em, rm, cmf, cmd)              \
  using PlanF##id =                                                                                      \
      Plan<n1, e1, Rad<FCAS_UNPAREN r1>, cf, n2, e2, Rad<FCAS_UNPAREN r2>, rwf, nm, em, Rad<FCAS_UNPAREN rm>, cmf>; \
  using PlanD##id =                                                                                      \
      Plan<n1, e1, Rad<FCAS_UNPAREN r1>, cd, n2, e2, Rad<FCAS_UNPAREN r2>, rwd, nm, em, Rad<FCAS_UNPAREN rm>, cmd>; \
  static_assert(PlanF##id::N == n && PlanD##id::N == n, "plan length");                    \
  static_assert(PlanF##id::PARTS2 <= kMaxParts2 && PlanD##id::PARTS2 <= kMaxParts2, "pass-2 partials");

FCAS_PLAN_LIST(FCAS_DECLARE_PLAN)

constexpr int kNumPlans = 37;

struct PlanInfo {
  int64_t n;
  int n1, n2, e1, e2;         // n2: columns of pass 1 (NM N2; the pass-2 length when NM = 1)
  int nm;                     // middle-pass length (1: two passes)
  int cols[2], rows[2];       // [precision]: 0 float, 1 double
  int tiles1[2], tiles2[2];
  int parts2[2];              // pass-2 partials per evaluation
  int threads1[2], threads2[2];
  int tilesm[2], threadsm[2];  // middle pass (0 when NM = 1)
};

#define FCAS_PLAN_INFO(id, n, n1, e1, r1, cf, cd, n2, e2, r2, rwf, rwd, nm, em, rm, cmf, cmd)            \
  {n, n1, PlanF##id::W1, e1, e2, nm, {cf, cd}, {rwf, rwd},                                              \
   {PlanF##id::TILES1, PlanD##id::TILES1}, {PlanF##id::TILES2, PlanD##id::TILES2},                     \
   {PlanF##id::PARTS2, PlanD##id::PARTS2},                                                             \
   {PlanF##id::T1, PlanD##id::T1}, {PlanF##id::T2, PlanD##id::T2},                                     \
   {PlanF##id::TILESM, PlanD##id::TILESM}, {PlanF##id::THREE ? PlanF##id::TM : 0, PlanD##id::THREE ? PlanD##id::TM : 0}},

inline const PlanInfo kPlans[kNumPlans] = {FCAS_PLAN_LIST(FCAS_PLAN_INFO)};

// The default plan of a length: the first listed for it.
inline int plan_for_length(int64_t n) {
  for (int i = 0; i < kNumPlans; ++i)
    if (kPlans[i].n == n) return i;
  return -1;
}

}  // namespace fcas

// eval_kernels.hpp -- gfx950 kernels of fitness_eval_batch (included by the
// per-precision translation units).
#pragma once

#include <hip/hip_runtime.h>

#include "fitness_tiles.hpp"
#include "plans.hpp"

// Build-time overrides of the pass kernels' settings (-1: the per-plan
// choice of PassTune below): software prefetch of the next work item's data
// (1) or a fetch at the start of each item (0), and the occupancy each pass
// kernel is compiled for (waves per SIMD; 1 = no bound below the register
// file's).
#ifndef FCAS_PASS1_PREFETCH
#define FCAS_PASS1_PREFETCH (-1)
#endif
#ifndef FCAS_PASS1_WAVES
#define FCAS_PASS1_WAVES (-1)
#endif
#ifndef FCAS_PASS2_PREFETCH
#define FCAS_PASS2_PREFETCH (-1)
#endif
#ifndef FCAS_PASS2_WAVES
#define FCAS_PASS2_WAVES (-1)
#endif

namespace fcas {

// Settings of the pass kernels of one plan.  Float transforms of 8-element
// threads fit in 128 VGPRs without a prefetch register set: at 4 waves per
// SIMD (their LDS allows 4 work-groups of 4 waves per CU) they run faster
// than at 3 waves with the next item prefetched (measured on the 4 x 131072
// search: pass 1 -7%, pass 2 -10%); the other plans (16-element threads,
// double precision) keep the prefetch at their register-bound occupancy.
template <typename Real, class PL>
struct PassTune {
  static constexpr bool light1 = sizeof(Real) == 4 && PL::E1 == 8;
  static constexpr bool light2 = sizeof(Real) == 4 && PL::E2 == 8;
  static constexpr bool prefetch1 = FCAS_PASS1_PREFETCH >= 0 ? FCAS_PASS1_PREFETCH != 0 : !light1;
  static constexpr bool prefetch2 = FCAS_PASS2_PREFETCH >= 0 ? FCAS_PASS2_PREFETCH != 0 : !light2;
  static constexpr int waves1 = FCAS_PASS1_WAVES >= 0 ? FCAS_PASS1_WAVES : (light1 ? 4 : 3);
  static constexpr int waves2 = FCAS_PASS2_WAVES >= 0 ? FCAS_PASS2_WAVES : (light2 ? 4 : 1);
};

struct PassArgs {
  const SegDesc* segs;
  const EvalDesc* evals;
  const int32_t* list;     // evaluation indices of this plan, in list order
  const int32_t* count;    // number of entries in `list`
  void* ws;                // workspace: cap slots of 2 N complex
  void* part_g;            // [max_batch][part_stride] partial maxima (Real)
  int32_t* part_j;         // [max_batch][part_stride] their samples
  int32_t part_stride;     // partials per evaluation slot (>= the plan's PARTS2)
  int32_t n_det;
  int32_t chunk_begin;     // first list position handled by this launch
  int32_t cap;             // workspace slots (positions per launch)
};

// Number of list positions one launch handles: the chunk [chunk_begin,
// chunk_begin + cap) of the plan's list, cut to the count the set-up kernel
// wrote.
__device__ __forceinline__ int launch_span(const PassArgs& a) {
  const int cnt = *a.count - a.chunk_begin;
  return cnt < 0 ? 0 : (cnt > a.cap ? a.cap : cnt);
}

// ---------------------------------------------------------------------------
// Pass 1: prologue (template phase, delays, projection) + length-N1 column
// FFTs + four-step twiddle, for C columns of one evaluation per work item.
// ---------------------------------------------------------------------------
// Orders the LDS writes of a stage before the reads of the next.  When every
// transform is held by threads of one wavefront (WAVE), the lanes of that wave
// are the only writers and readers of its buffer: waiting for the wave's own
// LDS operations and keeping the compiler from moving accesses across is
// enough.  Otherwise the whole work-group synchronises.
template <bool WAVE>
__device__ __forceinline__ void lds_exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Float transforms exchange both series in one step (LDS buffers buf0 and
// buf1, two synchronisations per stage); double transforms take turns in buf0,
// keeping their LDS within 64 KiB per work-group.
template <typename Real>
constexpr bool kJointExchange = sizeof(Real) == 4;
template <typename Real>
constexpr int kLdsSeries = kJointExchange<Real> ? 2 : 1;

// All stages of the S series (1 or 2) of one transform held in registers;
// JOINT: two series exchange through LDS together (buf0, buf1), else they take
// turns in buf0.
template <typename Real, class PL, int L, int E, class Rad, int I, int Ns, bool HALF, bool WAVE, int PAD,
          bool JOINT = kJointExchange<Real>, int S = 2>
__device__ __forceinline__ void run_stages(cplx<Real> (&v)[S][E], cplx<Real>* buf0, cplx<Real>* buf1,
                                           const cplx<Real>* tw, int t) {
  if constexpr (I < Rad::count) {
    constexpr int R = Rad::value[I];
    constexpr bool LAST = (I == Rad::count - 1);
    static_assert(!JOINT || S == 2, "a joint exchange needs both series");
    if constexpr (JOINT) {
      stage_butterflies<Real, L, E, R, Ns, LAST, HALF && I == 0, PAD>(v[0], buf0, tw, t);
      stage_butterflies<Real, L, E, R, Ns, LAST, HALF && I == 0, PAD>(v[1], buf1, tw, t);
      if constexpr (!LAST) {
        lds_exchange_sync<WAVE>();
        stage_gather<Real, L, E, PAD>(v[0], buf0, t);
        stage_gather<Real, L, E, PAD>(v[1], buf1, t);
        lds_exchange_sync<WAVE>();
      }
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        stage_butterflies<Real, L, E, R, Ns, LAST, HALF && I == 0, PAD>(v[s], buf0, tw, t);
        if constexpr (!LAST) {
          lds_exchange_sync<WAVE>();
          stage_gather<Real, L, E, PAD>(v[s], buf0, t);
          lds_exchange_sync<WAVE>();
        }
      }
    }
    run_stages<Real, PL, L, E, Rad, I + 1, Ns * R, false, WAVE, PAD, JOINT>(v, buf0, buf1, tw, t);
  }
}

// Pass-1 work item -> (list position in the launch, column tile).  Point-major
// (every tile of one point, then the next point) for two-pass plans, whose
// segment data stay in the L2 anyway; tile-major for the long three-pass
// segments (112 MB of data at one hour), so that the work-groups in flight
// take one tile of many points and share its data in the cache instead of
// each point re-reading the whole segment from HBM.  Work-groups are handed
// to the 8 XCDs in turn, so with a grid that is a multiple of 8, items that
// agree mod 8 run on one XCD: the tile-major order then gives XCD x the tiles
// x, x + 8, ... (when 8 divides TILES1), and each XCD's L2 fetches an eighth
// of the segment instead of all of it (pass 1 3% faster at one hour).  Any
// grid gives the same results: only the order of the items changes.
template <class PL>
constexpr bool kTileMajor1 = PL::THREE;

template <class PL>
__device__ __forceinline__ void pass1_decode(int item, int span, int& slot, int& tile) {
  if constexpr (kTileMajor1<PL> && PL::TILES1 % 8 == 0) {
    const int x = item & 7, r = item >> 3;
    const int g = r / span;
    slot = r - g * span;
    tile = x + 8 * g;
  } else if constexpr (kTileMajor1<PL>) {
    tile = item / span;
    slot = item - tile * span;
  } else {
    slot = item / PL::TILES1;
    tile = item - slot * PL::TILES1;
  }
}

// Point (evaluation index) at list position `pos` of the launch, and its
// segment's descriptor: uniform across the work-group, read as scalar loads.
__device__ __forceinline__ int list_entry(const PassArgs& a, int pos) { return *const_view(a.list + pos); }

__device__ __forceinline__ SegDesc segment_of(const PassArgs& a, int e) {
  const int seg = const_view(a.evals + e)->seg;
  return *const_view(a.segs + seg);
}

template <typename Real, class PL, int DT>
__device__ __forceinline__ void pass1_fetch_item(Pass1Data<Real, PL, DT>& d, const PassArgs& a, int item, int span,
                                                 int c, int p) {
  int slot, tile;
  pass1_decode<PL>(item, span, slot, tile);
  const SegDesc sg = segment_of(a, list_entry(a, a.chunk_begin + slot));
  pass1_fetch<Real, PL, DT>(d, sg, tile, c, p);
}

// LDS exchange buffers of the two passes: padded length of one transform and
// elements per work-group.
template <typename Real, class PL>
struct PassLds {
  static constexpr int LP1 = lds_padded_len<kPad1>(PL::N1), LP2 = lds_padded_len<kPad2>(PL::N2);
  static constexpr int X1 = kLdsSeries<Real> * PL::C * LP1, X2 = kLdsSeries<Real> * PL::RW * LP2;
};

// Pass 1 on the items of `a` taken by work-group `block` of `nblocks`
// (tw holds the length-N1 twiddles).
template <typename Real, class PL, int DT>
__device__ __forceinline__ void pass1_body(const PassArgs& a, cplx<Real>* lds, const cplx<Real>* tw, int block,
                                           int nblocks) {
  constexpr int LP = PassLds<Real, PL>::LP1;
  const int tid = threadIdx.x;
  const int span = launch_span(a);
  const int items = span * PL::TILES1;
  const int c = tid % PL::C, p = tid / PL::C;
  cplx<Real>* buf0 = lds + c * LP;
  cplx<Real>* buf1 = kJointExchange<Real> ? lds + (PL::C + c) * LP : buf0;
  if constexpr (DT > 0 && !PassTune<Real, PL>::prefetch1) {
    // each item fetches its own segment data; other waves cover the latency
    for (int item = block; item < items; item += nblocks) {
      int slot, tile;
      pass1_decode<PL>(item, span, slot, tile);
      Pass1Data<Real, PL, DT> d;
      pass1_fetch_item<Real, PL, DT>(d, a, item, span, c, p);
      cplx<Real> v[2][PL::E1];
      pass1_compute<Real, PL, DT>(v, d, pass1_point<Real, DT>(const_view(a.evals + list_entry(a, a.chunk_begin + slot))));
      run_stages<Real, PL, PL::N1, PL::E1, typename PL::Rad1, 0, 1, true, false, kPad1>(v, buf0, buf1, tw, p);
      pass1_store<Real, PL>(v, (cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N, tile, c, p);
    }
  } else if constexpr (DT > 0) {
    // software pipeline: once an item's prologue has consumed its segment
    // data, the next item's are fetched while this one is transformed (one set
    // of prefetch registers)
    Pass1Data<Real, PL, DT> d;
    int item = block;
    if (item < items) pass1_fetch_item<Real, PL, DT>(d, a, item, span, c, p);
    for (; item < items; item += nblocks) {
      int slot, tile;
      pass1_decode<PL>(item, span, slot, tile);
      cplx<Real> v[2][PL::E1];
      pass1_compute<Real, PL, DT>(v, d, pass1_point<Real, DT>(const_view(a.evals + list_entry(a, a.chunk_begin + slot))));
      // the fetch is unconditional (the last item re-reads its own data) so
      // that every path through the loop has the same loads in flight and the
      // compiler's wait counts never drain the prefetch early
      const int next = item + nblocks;
      pass1_fetch_item<Real, PL, DT>(d, a, next < items ? next : item, span, c, p);
      run_stages<Real, PL, PL::N1, PL::E1, typename PL::Rad1, 0, 1, true, false, kPad1>(v, buf0, buf1, tw, p);
      pass1_store<Real, PL>(v, (cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N, tile, c, p);
    }
  } else {
    for (int item = block; item < items; item += nblocks) {
      int slot, tile;
      pass1_decode<PL>(item, span, slot, tile);
      const int e = a.list[a.chunk_begin + slot];
      const EvalDesc& ev = a.evals[e];
      const SegDesc& sg = a.segs[ev.seg];
      cplx<Real> v[2][PL::E1];
      pass1_prologue<Real, PL, 0>(v, ev, sg, a.n_det, tile, c, p);
      run_stages<Real, PL, PL::N1, PL::E1, typename PL::Rad1, 0, 1, true, false, kPad1>(v, buf0, buf1, tw, p);
      cplx<Real>* ws = (cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N;
      pass1_store<Real, PL>(v, ws, tile, c, p);
    }
  }
}

template <typename Real, int L, int T>
__device__ __forceinline__ void init_twiddles(cplx<Real>* tw) {
  for (int m = threadIdx.x; m < L; m += T) tw[m] = twiddle<Real>(m, L);
  __syncthreads();
}

template <typename Real, class PL, int DT>
__global__ void __launch_bounds__(PL::T1)
    __attribute__((amdgpu_waves_per_eu(PassTune<Real, PL>::waves1))) k_pass1(PassArgs a) {
  __shared__ cplx<Real> lds[PassLds<Real, PL>::X1];
  __shared__ cplx<Real> tw[PL::N1];
  init_twiddles<Real, PL::N1, PL::T1>(tw);
  pass1_body<Real, PL, DT>(a, lds, tw, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Middle pass of the three-pass plans: length-NM transforms over the pass-1
// output, in place (see Plan).  Each work item takes CM adjacent columns of
// one pass-1 row, so every load and store instruction moves CM * 8 bytes of
// contiguous row per transform element (128 bytes at CM = 16).
// ---------------------------------------------------------------------------
// Exchange mode, series per work item and software prefetch of the middle
// pass.  Measured on the hour-long plans: the series taking turns in LDS (half
// the LDS) runs 1.75x faster than both at once; a second register set for
// prefetching then gains nothing, and neither does one series per work item
// (117 instead of 240 VGPRs, twice the waves per SIMD, 4% slower): the pass
// moves its 32 N bytes per point at the rate of a device copy.
constexpr bool kPassmJoint = false;
constexpr int kPassmSeries = 2;         // series per work item (1: each series its own item)
constexpr bool kPassmPrefetch = false;
template <typename Real>
constexpr bool kPassmJointFor = kPassmJoint && kJointExchange<Real> && kPassmSeries == 2;

// Work item -> (list position in the launch, first series, tile); the items
// of one point run series by series, tiles in order.
template <class PL>
__device__ __forceinline__ void passm_decode(int item, int& slot, int& s0, int& tile) {
  constexpr int PER_SERIES = PL::TILESM, PER_SLOT = (2 / kPassmSeries) * PL::TILESM;
  slot = item / PER_SLOT;
  const int r = item - slot * PER_SLOT;
  const int g = r / PER_SERIES;
  s0 = g * kPassmSeries;
  tile = r - g * PER_SERIES;
}

template <typename Real, class PL>
__device__ __forceinline__ void passm_fetch_item(cplx<Real> (&v)[kPassmSeries][PL::EM], const PassArgs& a,
                                                 int item, int c, int p) {
  int slot, s0, tile;
  passm_decode<PL>(item, slot, s0, tile);
  passm_fetch<Real, PL>(v, (const cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N, tile, c, p, s0);
}

template <typename Real, class PL>
__device__ __forceinline__ void passm_item(cplx<Real> (&v)[kPassmSeries][PL::EM], const PassArgs& a, int item,
                                           cplx<Real>* buf0, cplx<Real>* buf1, const cplx<Real>* tw, int c, int p) {
  int slot, s0, tile;
  passm_decode<PL>(item, slot, s0, tile);
  passm_twiddle_in<Real, PL>(v, tile, c, p);
  run_stages<Real, PL, PL::NM, PL::EM, typename PL::RadM, 0, 1, false, false, kPadM, kPassmJointFor<Real>>(
      v, buf0, buf1, tw, p);
  passm_twiddle_out<Real, PL>(v, tile, c, p);
  passm_store<Real, PL>(v, (cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N, tile, c, p, s0);
}

// Middle pass on the items of `a` taken by work-group `block` of `nblocks`;
// with kPassmPrefetch the next item's loads are in flight while one is
// transformed (two register sets).  Items cover disjoint workspace elements,
// so a prefetch never reads what another item stores.
template <typename Real, class PL>
__device__ __forceinline__ void passm_body(const PassArgs& a, cplx<Real>* lds, const cplx<Real>* tw, int block,
                                           int nblocks) {
  constexpr int LP = lds_padded_len<kPadM>(PL::NM);
  const int tid = threadIdx.x;
  const int items = launch_span(a) * (2 / kPassmSeries) * PL::TILESM;
  const int c = tid % PL::CM, p = tid / PL::CM;
  cplx<Real>* buf0 = lds + c * LP;
  cplx<Real>* buf1 = kPassmJointFor<Real> ? lds + (PL::CM + c) * LP : buf0;
  if constexpr (kPassmPrefetch) {
    cplx<Real> va[kPassmSeries][PL::EM], vb[kPassmSeries][PL::EM];
    int item = block;
    if (item < items) passm_fetch_item<Real, PL>(va, a, item, c, p);
    while (item < items) {
      const int next = item + nblocks;
      if (next < items) passm_fetch_item<Real, PL>(vb, a, next, c, p);
      passm_item<Real, PL>(va, a, item, buf0, buf1, tw, c, p);
      if (next >= items) break;
      item = next + nblocks;
      if (item < items) passm_fetch_item<Real, PL>(va, a, item, c, p);
      passm_item<Real, PL>(vb, a, next, buf0, buf1, tw, c, p);
    }
  } else {
    for (int item = block; item < items; item += nblocks) {
      cplx<Real> v[kPassmSeries][PL::EM];
      passm_fetch_item<Real, PL>(v, a, item, c, p);
      passm_item<Real, PL>(v, a, item, buf0, buf1, tw, c, p);
    }
  }
}

template <typename Real, class PL>
__global__ void __launch_bounds__(PL::TM) k_passm(PassArgs a) {
  static_assert(PL::THREE, "two-pass plans have no middle pass");
  __shared__ cplx<Real> lds[(kPassmJointFor<Real> ? 2 : 1) * PL::CM * lds_padded_len<kPadM>(PL::NM)];
  __shared__ cplx<Real> tw[PL::NM];
  init_twiddles<Real, PL::NM, PL::TM>(tw);
  passm_body<Real, PL>(a, lds, tw, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Pass 2: length-N2 row FFTs, |a_0|^2 + |a_1|^2 and its maximum over the rows
// of one work item -> one partial (value, sample) per wavefront.  When every
// row transform lies inside one wavefront the items need no work-group
// barrier; rows longer than a wavefront's share synchronise the work-group.
// ---------------------------------------------------------------------------
template <typename Real, class PL>
__device__ __forceinline__ void pass2_item(cplx<Real> (&v)[2][PL::E2], const PassArgs& a, int item,
                                           cplx<Real>* buf0, cplx<Real>* buf1, const cplx<Real>* tw, int r, int p,
                                           int lane, int wave) {
  constexpr int NW = PL::T2 / 64;
  const int slot = item / PL::TILES2;
  const int tile = item - slot * PL::TILES2;
  const int e = list_entry(a, a.chunk_begin + slot);
  // row transforms held by one wavefront exchange through LDS without a
  // work-group barrier
  constexpr bool WAVE = (64 % PL::P2) == 0;
  if constexpr (!PL::THREE) pass2_twiddle<Real, PL>(v, tile, r, p);
  run_stages<Real, PL, PL::N2, PL::E2, typename PL::Rad2, 0, 1, false, WAVE, kPad2>(v, buf0, buf1, tw, p);
  const SegDesc sg = segment_of(a, e);
  Real g;
  int j;
  pass2_best<Real, PL>(v, tile, r, p, g, j, sg.j_lo, sg.j_hi);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const Real go = __shfl_xor(g, off, 64);
    const int jo = __shfl_xor(j, off, 64);
    if (better(go, jo, g, j)) {
      g = go;
      j = jo;
    }
  }
  if (lane == 0) {
    const int64_t o = (int64_t)e * a.part_stride + tile * NW + wave;
    ((Real*)a.part_g)[o] = g;
    a.part_j[o] = j;
  }
}

template <typename Real, class PL>
__device__ __forceinline__ void pass2_fetch_item(cplx<Real> (&v)[2][PL::E2], const PassArgs& a, int item, int r,
                                                 int p) {
  const int slot = item / PL::TILES2;
  pass2_fetch<Real, PL>(v, (const cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N, item - slot * PL::TILES2, r, p);
}

// Pass 2 on the items of `a` taken by work-group `block` of `nblocks` (tw holds
// the length-N2 twiddles).
template <typename Real, class PL>
__device__ __forceinline__ void pass2_body(const PassArgs& a, cplx<Real>* lds, const cplx<Real>* tw, int block,
                                           int nblocks) {
  constexpr int LP = PassLds<Real, PL>::LP2;
  const int tid = threadIdx.x;
  const int items = launch_span(a) * PL::TILES2;
  const int p = tid % PL::P2, r = tid / PL::P2;
  cplx<Real>* buf0 = lds + r * LP;
  cplx<Real>* buf1 = kJointExchange<Real> ? lds + (PL::RW + r) * LP : buf0;
  const int lane = tid & 63, wave = tid >> 6;
  // software pipeline over two register sets: the rows of the next item are
  // fetched while this one is transformed
  // (the fetches are unconditional, a missing next item replaced by one
  // already fetched, so that every path has the same loads in flight and the
  // compiler's wait counts only wait for the set being transformed)
  if constexpr (!PassTune<Real, PL>::prefetch2) {
    // one register set: each item's rows are loaded when it starts
    for (int item = block; item < items; item += nblocks) {
      cplx<Real> v[2][PL::E2];
      pass2_fetch_item<Real, PL>(v, a, item, r, p);
      pass2_item<Real, PL>(v, a, item, buf0, buf1, tw, r, p, lane, wave);
    }
    return;
  }
  cplx<Real> va[2][PL::E2], vb[2][PL::E2];
  int item = block;
  if (item < items) pass2_fetch_item<Real, PL>(va, a, item, r, p);
  while (item < items) {
    const int next = item + nblocks;
    pass2_fetch_item<Real, PL>(vb, a, next < items ? next : item, r, p);
    pass2_item<Real, PL>(va, a, item, buf0, buf1, tw, r, p, lane, wave);
    if (next >= items) break;
    item = next + nblocks;
    pass2_fetch_item<Real, PL>(va, a, item < items ? item : next, r, p);
    pass2_item<Real, PL>(vb, a, next, buf0, buf1, tw, r, p, lane, wave);
  }
}

template <typename Real, class PL>
__global__ void __launch_bounds__(PL::T2)
    __attribute__((amdgpu_waves_per_eu(PassTune<Real, PL>::waves2))) k_pass2(PassArgs a) {
  __shared__ cplx<Real> lds[PassLds<Real, PL>::X2];
  __shared__ cplx<Real> tw[PL::N2];
  init_twiddles<Real, PL::N2, PL::T2>(tw);
  pass2_body<Real, PL>(a, lds, tw, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Finalize: one wavefront per point reduces its pass-2 partials.
// ---------------------------------------------------------------------------
// Gamma^2 and j* of point e from its partials, by the 64 lanes of one
// wavefront (lane 0 writes them); -inf / -1 outside the rectangle, NaN / -2
// for a bad segment.
template <typename Real>
__device__ __forceinline__ void finalize_point(const EvalDesc& ev, const Real* __restrict__ part_g,
                                               const int32_t* __restrict__ part_j, int part_stride,
                                               const int32_t* __restrict__ plan_parts2, int e, int lane,
                                               double* __restrict__ fitness, int32_t* __restrict__ argmax) {
  const int status = ev.status;
  if (status != 1) {
    if (lane == 0) {
      fitness[e] = status == 0 ? -INFINITY : NAN;
      argmax[e] = status == 0 ? -1 : -2;
    }
    return;
  }
  const int nt = plan_parts2[ev.plan];
  Real g = (Real)-1;
  int j = 0x7fffffff;
  for (int t = lane; t < nt; t += 64) {
    const Real go = part_g[(int64_t)e * part_stride + t];
    const int jo = part_j[(int64_t)e * part_stride + t];
    if (better(go, jo, g, j)) {
      g = go;
      j = jo;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const Real go = __shfl_xor(g, off, 64);
    const int jo = __shfl_xor(j, off, 64);
    if (better(go, jo, g, j)) {
      g = go;
      j = jo;
    }
  }
  if (lane == 0) {
    fitness[e] = (double)g;
    argmax[e] = j;
  }
}

// The same by a group of 8 lanes (lane g of the group, groups aligned to 8
// lanes, every lane of the group calling it): the largest (g, then smallest j)
// of the partials is unique, so any grouping of the reduction gives the same
// result as finalize_point.
template <typename Real>
__device__ __forceinline__ void finalize_group(const EvalDesc& ev, const Real* __restrict__ part_g,
                                               const int32_t* __restrict__ part_j, int part_stride,
                                               const int32_t* __restrict__ plan_parts2, int e, int g,
                                               double* __restrict__ fitness, int32_t* __restrict__ argmax) {
  const int status = ev.status;
  if (status != 1) {
    if (g == 0) {
      fitness[e] = status == 0 ? -INFINITY : NAN;
      argmax[e] = status == 0 ? -1 : -2;
    }
    return;
  }
  const int nt = plan_parts2[ev.plan];
  Real bg = (Real)-1;
  int bj = 0x7fffffff;
  // batches of 16 loads per lane in flight before any is compared
  constexpr int B = 16;
  for (int t0 = g; t0 < nt; t0 += 8 * B) {
    Real gv[B];
    int jv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int t = t0 + 8 * u;
      gv[u] = t < nt ? part_g[(int64_t)e * part_stride + t] : (Real)-1;
      jv[u] = t < nt ? part_j[(int64_t)e * part_stride + t] : 0x7fffffff;
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (better(gv[u], jv[u], bg, bj)) {
        bg = gv[u];
        bj = jv[u];
      }
  }
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) {
    const Real go = __shfl_xor(bg, off, 8);
    const int jo = __shfl_xor(bj, off, 8);
    if (better(go, jo, bg, bj)) {
      bg = go;
      bj = jo;
    }
  }
  if (g == 0) {
    fitness[e] = (double)bg;
    argmax[e] = bj;
  }
}

template <typename Real>
__global__ void __launch_bounds__(256) k_finalize(const EvalDesc* __restrict__ evals,
                                                  const SegDesc* __restrict__ segs, const Real* __restrict__ part_g,
                                                  const int32_t* __restrict__ part_j, int n, int part_stride,
                                                  const int32_t* __restrict__ plan_parts2,
                                                  int32_t* __restrict__ counts,
                                                  unsigned long long* __restrict__ evaluated,
                                                  double* __restrict__ fitness, int32_t* __restrict__ argmax) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // running total of points evaluated (inside the rectangle); the passes of
    // this call are done with the list counts, which start the next call at 0
    unsigned long long t = 0;
    for (int p = 0; p < kNumPlans; ++p) {
      t += (unsigned long long)counts[p];
      counts[p] = 0;
    }
    atomicAdd(evaluated, t);
  }
  if (e >= n) return;
  finalize_point<Real>(evals[e], part_g, part_j, part_stride, plan_parts2, e, lane, fitness, argmax);
}

}  // namespace fcas

namespace fcas {

// ---------------------------------------------------------------------------
// Fused persistent schedule: both passes of every evaluation of one plan in
// a single launch.  Work items (TILES1 pass-1 tiles and TILES2 pass-2 tiles per
// evaluation) form a software pipeline in which pass-1 tiles of evaluation
// e + L interleave with pass-2 tiles of evaluation e:
//   [P1(0) .. P1(L-1)] [P1(L) P2(0)] [P1(L+1) P2(1)] ... [P2(cnt-L) .. P2(cnt-1)]
// Work-group w takes items w, w + G, w + 2G, ... (G <= resident work-groups),
// so ALU-bound pass-1 tiles and bandwidth-bound pass-2 tiles run side by side
// and only S = `slots` evaluations occupy the workspace (S > L), small enough
// to stay in the memory-side cache.  A pass-2 tile waits for its evaluation's
// pass-1 tiles; a pass-1 tile waits for the pass-2 tiles of the evaluation that
// last used its slot.  Both are earlier in the sequence, so the wait always
// ends; each wait is also bounded (on overflow an error flag is set and the
// item proceeds).
// ---------------------------------------------------------------------------
struct FusedArgs {
  PassArgs p;
  int32_t* done1;    // [max_batch] pass-1 tiles finished, per list position
  int32_t* done2;    // [max_batch] pass-2 tiles finished, per list position
  int32_t* err;      // error flags (bit 1: a wait exceeded its bound)
  int32_t lag;       // L
  int32_t slots;     // S
  int32_t max_spin;  // polls before a wait gives up
};

__device__ __forceinline__ void wait_count(const int32_t* ctr, int target, int max_spin, int32_t* err) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > max_spin) {
        __hip_atomic_fetch_or(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void signal_count(int32_t* ctr) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename Real, class PL>
__global__ void __launch_bounds__(PL::T1) k_fused(FusedArgs f) {
  static_assert(PL::T1 == PL::T2, "the fused schedule needs equal work-item sizes");
  static_assert(!PL::THREE, "the fused schedule covers two-pass plans");
  constexpr int LP1 = lds_padded_len<kPad1>(PL::N1), LP2 = lds_padded_len<kPad2>(PL::N2);
  constexpr int LDSN = 2 * ((PL::C * LP1 > PL::RW * LP2) ? PL::C * LP1 : PL::RW * LP2);
  constexpr int NW = PL::T2 / 64;
  constexpr int T1 = PL::TILES1, T2 = PL::TILES2, T = T1 + T2;
  __shared__ cplx<Real> lds[LDSN];
  __shared__ cplx<Real> tw1[PL::N1];
  __shared__ cplx<Real> tw2[PL::N2];
  const PassArgs& a = f.p;
  const int tid = threadIdx.x;
  for (int m = tid; m < PL::N1; m += PL::T1) tw1[m] = twiddle<Real>(m, PL::N1);
  for (int m = tid; m < PL::N2; m += PL::T1) tw2[m] = twiddle<Real>(m, PL::N2);
  __syncthreads();
  const int cnt = *a.count;
  const int L = f.lag < cnt ? f.lag : cnt;
  const int total = cnt * T;
  const int lane = tid & 63, wave = tid >> 6;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    int kind, ep, tile;
    fused_decode(item, cnt, L, T1, T2, kind, ep, tile);
    const int slot = ep % f.slots;
    cplx<Real>* ws = (cplx<Real>*)a.ws + (int64_t)slot * 2 * PL::N;
    const int e = a.list[ep];
    if (kind == 1) {
      if (ep >= f.slots) wait_count(f.done2 + (ep - f.slots), T2, f.max_spin, f.err);
      const EvalDesc& ev = a.evals[e];
      const SegDesc& sg = a.segs[ev.seg];
      const int c = tid % PL::C, p = tid / PL::C;
      cplx<Real> v[2][PL::E1];
      pass1_prologue<Real, PL>(v, ev, sg, a.n_det, tile, c, p);
      run_stages<Real, PL, PL::N1, PL::E1, typename PL::Rad1, 0, 1, true, false, kPad1>(v, lds + c * LP1, lds + (PL::C + c) * LP1,
                                                                          tw1, p);
      pass1_store<Real, PL>(v, ws, tile, c, p);
      signal_count(f.done1 + ep);
    } else {
      wait_count(f.done1 + ep, T1, f.max_spin, f.err);
      const int p = tid % PL::P2, r = tid / PL::P2;
      cplx<Real> v[2][PL::E2];
      pass2_load<Real, PL>(v, ws, tile, r, p);
      run_stages<Real, PL, PL::N2, PL::E2, typename PL::Rad2, 0, 1, false, false, kPad2>(v, lds + r * LP2, lds + (PL::RW + r) * LP2, tw2,
                                                                   p);
      const SegDesc& sg = a.segs[a.evals[e].seg];
      Real g;
      int j;
      pass2_best<Real, PL>(v, tile, r, p, g, j, sg.j_lo, sg.j_hi);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const Real go = __shfl_xor(g, off, 64);
        const int jo = __shfl_xor(j, off, 64);
        if (better(go, jo, g, j)) { g = go; j = jo; }
      }
      if (lane == 0) {
        const int64_t o = (int64_t)e * a.part_stride + tile * NW + wave;
        ((Real*)a.part_g)[o] = g;
        a.part_j[o] = j;
      }
      signal_count(f.done2 + ep);
    }
  }
}

}  // namespace fcas

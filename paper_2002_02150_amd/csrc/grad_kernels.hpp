// grad_kernels.hpp -- fixed-sample adjoint of the coherent fitness.
#pragma once

#include <hip/hip_runtime.h>

#include "eval_kernels.hpp"

namespace fcas {

// Per point and detector, six complex sums over the in-band bins at j*:
// [0] z^i, [1..4] sum a_k b_k^{5,3,2,1}, [5] sum a_k k.
constexpr int kAdjSums = 6;
constexpr int kAdjMinBlocks = 2048;   // adjoint blocks wanted for small batches
constexpr int kAdjMaxParts = 64;      // most parts one (point, detector) sum is split into

struct GradBuffers {
  double* sums = nullptr;   // [n][n_det][parts][kAdjSums][2]
  int max_batch = 0;
  int n_det = 0;
};

int grad_parts(int n, int n_det);
int alloc_grad_buffers(GradBuffers& g, int max_batch, int n_det);
void free_grad_buffers(GradBuffers& g);
hipError_t launch_gradient(int precision, const GradBuffers& g, const NetDesc* net, const SegDesc* segs,
                           const EvalDesc* evals, const double* theta, const int32_t* argmax, int n, int n_det,
                           double* grad, hipStream_t s);

hipError_t launch_polish_trials(const double* theta, const double* grad, const int32_t* seg, const NetDesc* net,
                                int n, int trials, double step_frac, double* cand, int32_t* cand_seg, hipStream_t s);
hipError_t launch_polish_select(double* theta, double* fitness, int32_t* argmax, const double* cand,
                                const double* cand_f, const int32_t* cand_j, int n, int trials, hipStream_t s);

}  // namespace fcas

// sk_batch.hpp -- many independent sketches in one pass: the persistent form
// of the sketch kernel and the batched split reduction.
//
// The inspector of a batch is the item-flattened inspector of sk_inspect.hpp.
// The persistent kernel's workgroups take work units (item, S-row tile,
// column range, row-block split) from a list sorted longest-first, one atomic
// counter being the only shared state; each unit runs the same code as a
// workgroup of the single-sketch grid, so an item's result is bitwise the
// same as its single-sketch call with the same tuning.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_mfma.hpp"
#include "sk_sketch.hpp"

namespace sk {

struct BatchOut {
  SketchParams P;  // the sketch kernel's parameters for this item
  int32_t slices;  // partial slices (1: the kernel writes A_hat directly)
  float* Ahat;     // final output (d x n, leading dimension ld)
  int64_t ld;
  const float* part;
  int64_t d, n;
  int64_t o_out;   // exclusive prefix of d * n over items with slices > 1
};

template <int64_t BatchOut::*F>
__device__ __forceinline__ int find_out(const BatchOut* __restrict__ it, int count, int64_t t) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].*F <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// persistent sketch kernel: work[u] = {item, unit}; unit = (crange * tiles +
// tile) * splits + split, the same numbering as the single-sketch grid
template <int DIST, int DL, int Q, int CS, int WGS>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(4))) void k_sketch_persistent(
    const BatchOut* __restrict__ it, const int2* __restrict__ work, int total,
    int32_t* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_unit;
  while (true) {
    if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1);
    __syncthreads();
    const int u = __builtin_amdgcn_readfirstlane(s_unit);  // uniform: parameters in SGPRs
    __syncthreads();
    if (u >= total) break;
    const int2 w = work[u];
    const SketchParams P = it[w.x].P;
    const int split = w.y % P.splits;
    const int rest = w.y / P.splits;
    sketch_unit<DIST, DL, Q, CS, WGS>(P, split, rest % P.tiles, rest / P.tiles, smem);
    __syncthreads();  // LDS of this unit is consumed before the next one starts
  }
}

// persistent form of the matrix-core kernel (+-1 S in BF16 / FP8)
template <int FMT>
__global__ __launch_bounds__(MF_THREADS) void k_sketch_mfma_persistent(
    const BatchOut* __restrict__ it, const int2* __restrict__ work, int total,
    int32_t* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_unit;
  while (true) {
    if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1);
    __syncthreads();
    const int u = __builtin_amdgcn_readfirstlane(s_unit);  // uniform: parameters in SGPRs
    __syncthreads();
    if (u >= total) break;
    const int2 w = work[u];
    const SketchParams P = it[w.x].P;
    const int split = w.y % P.splits;
    const int rest = w.y / P.splits;
    mfma_unit<FMT>(P, split, rest % P.tiles, rest / P.tiles, smem);
    __syncthreads();
  }
}

__global__ void k_batch_reduce(const BatchOut* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_out<&BatchOut::o_out>(it, count, g);
  const BatchOut& I = it[i];
  const int64_t t = g - I.o_out;
  const int64_t d = I.d, n = I.n;
  const int64_t k = t / d, r = t - k * d;
  // eight loads in flight, added in slice order
  const float* __restrict__ p = I.part + t;
  const int64_t stride = d * n;
  float s = p[0];
  int q = 1;
  for (; q + 8 <= I.slices; q += 8) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
  }
  for (; q < I.slices; ++q) s += p[(int64_t)q * stride];
  I.Ahat[r + k * I.ld] = s;
}

}  // namespace sk

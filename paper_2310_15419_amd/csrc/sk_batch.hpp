// sk_batch.hpp -- many independent sketches in one pass: a batched inspector
// and one persistent launch of the sketch kernel.
//
// Every batched inspector kernel runs over a flattened index space that
// concatenates the items; a thread finds its item by binary search over the
// items' prefix offsets, then does exactly what the single-sketch kernel does
// for that item.  Per-item exclusive scans are one scan over the
// concatenation followed by subtraction of each item's value at its region
// start.  The persistent kernel's workgroups take work units (item, S-row
// tile, column range, row-block split) from a list sorted longest-first, one
// atomic counter being the only shared state; each unit runs the same code
// as a workgroup of the single-sketch grid, so an item's result is bitwise
// the same as its single-sketch call with the same tuning.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"
#include "sk_sketch.hpp"

namespace sk {

struct BatchItem {
  // input
  int64_t m, n, nnz;
  const int64_t* colptr;
  const int32_t* rowidx;
  const void* vals;
  int32_t vtype;
  int32_t slices;       // partial slices (1: the kernel writes A_hat directly)
  float* Ahat;          // final output (d x n, leading dimension ld)
  int64_t ld;
  int64_t nb_max;
  int32_t* ridx;        // this item's region of the concatenated occupancy / rank array
  int32_t* pos;
  int32_t* seg_region;  // this item's region of the concatenated segment array
  float* part;
  int32_t ridx_base;    // value of the global scan at the region start
  int32_t seg_base;
  // exclusive prefix offsets of this item in each flattened index space
  int64_t o_valid;  // max(nnz, n + 1)
  int64_t o_ridx;   // m + 1 (region of the concatenated occupancy array)
  int64_t o_m;      // m
  int64_t o_pos;    // (nb_max + 1) * n
  int64_t o_cnt;    // nb_max * n
  int64_t o_seg;    // nb_max * n + 1 (region of the concatenated segment array)
  int64_t o_nnz;    // nnz
  int64_t o_out;    // d * n when slices > 1, else 0
  int64_t o_items_pad;
  SketchParams P;   // the sketch kernel's parameters for this item
};

// offsets are at fixed positions in BatchItem: select by member pointer
template <int64_t BatchItem::*F>
__device__ __forceinline__ int find_item(const BatchItem* __restrict__ it, int count, int64_t t) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].*F <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_batch_validate_mark(const BatchItem* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_item<&BatchItem::o_valid>(it, count, g);
  const BatchItem& I = it[i];
  const int64_t t = g - I.o_valid;
  Header* hdr = const_cast<Header*>(I.P.hdr);
  int bad = 0;
  if (t <= I.n) {
    const int64_t c = I.colptr[t];
    if (t == 0 && c != 0) bad |= ST_COLPTR;
    if (t == I.n && c != I.nnz) bad |= ST_COLPTR;
    if (t < I.n && I.colptr[t + 1] < c) bad |= ST_COLPTR;
    if (c < 0 || c > I.nnz) bad |= ST_COLPTR;
  }
  if (t < I.nnz) {
    const int32_t r = I.rowidx[t];
    if (r < 0 || r >= I.m) bad |= ST_RANGE;
    else I.ridx[r] = 1;
    if (t > 0) {
      const int64_t k = column_of(I.colptr, I.n, t);
      if (I.colptr[k] < t && I.rowidx[t - 1] >= r) bad |= ST_UNSORTED;
    }
  }
  if (bad) atomicOr(&hdr->status, bad);
}

// region bases after a global scan: which = 0 (ranks) or 1 (segments)
__global__ void k_batch_bases(BatchItem* __restrict__ it, int count, int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (which == 0) it[i].ridx_base = it[i].ridx[0];
  else it[i].seg_base = it[i].seg_region[0];
}

__global__ void k_batch_rebase(const BatchItem* __restrict__ it, int count, int64_t total,
                               int which) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  if (which == 0) {
    const int i = find_item<&BatchItem::o_ridx>(it, count, g);
    it[i].ridx[g - it[i].o_ridx] -= it[i].ridx_base;
  } else {
    const int i = find_item<&BatchItem::o_seg>(it, count, g);
    it[i].seg_region[g - it[i].o_seg] -= it[i].seg_base;
  }
}

__global__ void k_batch_rowlist(const BatchItem* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_item<&BatchItem::o_m>(it, count, g);
  const BatchItem& I = it[i];
  const int64_t r = g - I.o_m;
  int32_t* rowlist = const_cast<int32_t*>(I.P.rowlist);
  if (I.ridx[r + 1] > I.ridx[r]) rowlist[I.ridx[r]] = (int32_t)r;
  if (r == 0) {
    Header* hdr = const_cast<Header*>(I.P.hdr);
    const int64_t R = I.ridx[I.m];
    hdr->nonempty = R;
    const int64_t nb = (R + I.P.m_b - 1) / I.P.m_b;
    hdr->nblocks = nb < I.nb_max ? nb : I.nb_max;
  }
}

__global__ void k_batch_block_pos(const BatchItem* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_item<&BatchItem::o_pos>(it, count, g);
  const BatchItem& I = it[i];
  if (I.P.hdr->status) return;
  const int64_t t = g - I.o_pos;
  const int64_t b = t / I.n, k = t - b * I.n;
  int64_t lo = I.colptr[k], hi = I.colptr[k + 1];
  if (b < I.P.hdr->nblocks) {
    const int32_t fr = I.P.rowlist[b * I.P.m_b];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (I.rowidx[mid] < fr) lo = mid + 1;
      else hi = mid;
    }
  } else {
    lo = hi;
  }
  I.pos[t] = (int32_t)lo;
}

__global__ void k_batch_block_cnt(const BatchItem* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_item<&BatchItem::o_cnt>(it, count, g);
  const BatchItem& I = it[i];
  const int64_t t = g - I.o_cnt;
  I.seg_region[t] = I.P.hdr->status ? 0 : I.pos[t + I.n] - I.pos[t];
}

__global__ void k_batch_scatter(const BatchItem* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_item<&BatchItem::o_nnz>(it, count, g);
  const BatchItem& I = it[i];
  if (I.P.hdr->status) return;
  const int64_t p = g - I.o_nnz;
  const int32_t r = I.rowidx[p];
  const int32_t c = I.ridx[r];
  const int32_t b = c / I.P.m_b;
  const int32_t l = c - b * I.P.m_b;
  const int64_t k = column_of(I.colptr, I.n, p);
  const int64_t bk = (int64_t)b * I.n + k;
  const int64_t dest = (int64_t)I.seg_region[bk] + (p - (int64_t)I.pos[bk]);
  uint2* ent = const_cast<uint2*>(I.P.ent);
  ent[dest] = make_uint2((uint32_t)l * (uint32_t)(I.P.ldS * 4),
                         __float_as_uint(load_value(I.vals, I.vtype, p)));
}

// persistent sketch kernel: work[u] = {item, unit}; unit = (crange * tiles +
// tile) * splits + split, the same numbering as the single-sketch grid
template <int DIST, int DL, int Q, int CS, int WGS>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(4))) void k_sketch_persistent(
    const BatchItem* __restrict__ it, const int2* __restrict__ work, int total,
    int32_t* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_unit;
  while (true) {
    if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1);
    __syncthreads();
    const int u = s_unit;
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

__global__ void k_batch_reduce(const BatchItem* __restrict__ it, int count, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int i = find_item<&BatchItem::o_out>(it, count, g);
  const BatchItem& I = it[i];
  const int64_t t = g - I.o_out;
  const int64_t d = I.P.d, n = I.n;
  const int64_t k = t / d, r = t - k * d;
  float s = I.part[t];
  for (int q = 1; q < I.slices; ++q) s += I.part[(int64_t)q * d * n + t];
  I.Ahat[r + k * I.ld] = s;
}

}  // namespace sk

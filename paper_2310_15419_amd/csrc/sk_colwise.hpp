// sk_colwise.hpp -- the sketch in the loop order of Algorithm 3 (variant
// kji): for every column k of A and every nonzero a_jk of it, the segment
// S[r : r + d, j] is generated anew and a_jk S[:, j] is added into
// A_hat[:, k].  Nothing is reused across columns (every nonzero pays its own
// generator calls: Sec. III-A's cost of the kji order), no inspector runs
// (the CSC input is used as given), and the cost does not depend on where the
// nonzeros sit (Table VI's observation).  It is the GPU counterpart of the
// paper's Algorithm 3 beside the S-tile kernel (the counterpart of Algorithm
// 4's reuse).
//
// A wave owns A_hat[tile rows, k]: its 64 lanes hold DL consecutive S rows
// each (DL = 4: one generator call per lane per nonzero for (-1,1) and the
// Gaussian; DL = 32: one word of a call per lane for +-1).  The nonzeros of
// column k are the same for the whole wave, so their row indices and values
// are scalar loads.  Every A_hat entry is one lane's sum in row order of the
// column: no atomics, a fixed summation order.
//
// Heavy columns: a column with more than C nonzeros is cut into chunks of C
// consecutive nonzeros, each walked by its own waves into a partial sum; a
// second kernel adds a column's partials in chunk order.  Work items are
// chunks (a light column is one chunk and writes A_hat directly), located
// by a search over the scanned chunk counts.  C is a power of two chosen
// from the shape so that the partials fit a fixed budget.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"
#include "sk_rng.hpp"

namespace sk {

struct ColwiseParams {
  const int64_t* colptr;
  const int32_t* rowidx;
  const void* vals;
  int32_t vtype;
  const Header* hdr;  // validation status of A (set by the validation pass)
  int64_t n, d, row0;
  uint64_t seed;
  void* out;          // float (FP32 form) or double (FP64 form)
  int64_t ld;
  int32_t tiles;      // S-row tiles of 64 * DL rows
  int32_t chunk;      // C: nonzeros per chunk of a heavy column
  const int32_t* cbase;  // [n + 1]: first chunk of each column (scanned)
  const int32_t* hbase;  // [n + 1]: first partial slot of each column (heavy only)
  void* part;         // partial sums of heavy columns' chunks, d per slot
};

// chunks of column k: one for a light column (at most C nonzeros, or any
// column of a matrix that failed validation), ceil(len / C) for a heavy one
__device__ __forceinline__ int32_t colwise_chunks(const int64_t* colptr, int64_t k, int32_t C,
                                                  int status) {
  if (status) return 1;
  const int64_t len = colptr[k + 1] - colptr[k];
  return len > C ? (int32_t)((len + C - 1) / C) : 1;
}

// per column: chunks, heavy chunks (partial slots) and the heavy flag, for
// three scans
__global__ void k_colwise_counts(const int64_t* __restrict__ colptr, int64_t n, int32_t C,
                                 const Header* __restrict__ hdr, int32_t* __restrict__ cb,
                                 int32_t* __restrict__ hb, int32_t* __restrict__ hk) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t c = colwise_chunks(colptr, k, C, hdr->status);
  cb[k] = c;
  hb[k] = c > 1 ? c : 0;
  hk[k] = c > 1 ? 1 : 0;
}

// the heavy columns in order (hk scanned: column k is heavy when its rank
// moves)
__global__ void k_colwise_heavy_list(const int32_t* __restrict__ hk, int64_t n,
                                     int32_t* __restrict__ hcol) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (hk[k + 1] > hk[k]) hcol[hk[k]] = (int32_t)k;
}

// the column holding chunk c: the k with cbase[k] <= c < cbase[k + 1]
// (every column has at least one chunk, so the bounds increase strictly)
__device__ __forceinline__ int64_t colwise_column(const int32_t* cbase, int64_t n, int64_t c) {
  int64_t lo = 0, hi = n;  // cbase[lo] <= c < cbase[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (cbase[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

// a_jk in FP64 (FP32 and BF16 values widen exactly)
__device__ __forceinline__ double load_value_f64(const void* vals, int vtype, int64_t p) {
  if (vtype == 0) return in_global((const double*)vals)[p];
  return (double)load_value(vals, vtype, p);
}

constexpr int CW_WAVES = 4;  // waves (tiles of one column) per workgroup

// S(gi + t, j) for t < DL (gi: the lane's first global S row)
template <int DIST, int DL>
__device__ __forceinline__ void colwise_values(uint64_t seed, uint64_t gi, uint64_t j,
                                               float (&s)[DL]) {
  if constexpr (DIST == DIST_RADEMACHER) {
    static_assert(DL == 32, "+-1: one 32-bit word per lane");
    // rows gi .. gi + 31: bits of one word when gi is a multiple of 32, else
    // the tail of one word and the head of the next (perhaps the next call's)
    const uint64_t g = gi >> 7;
    const int w = (int)((gi >> 5) & 3);
    const int b = (int)(gi & 31);
    const Words x = gen_words(seed, g, j);
    uint32_t bits = word_at(x, w);
    if (b) {
      const uint32_t hi = w < 3 ? word_at(x, w + 1) : gen_words(seed, g + 1, j).x0;
      bits = (bits >> b) | (hi << (32 - b));
    }
#pragma unroll
    for (int t = 0; t < 32; ++t)
      s[t] = __uint_as_float((((bits >> t) & 1u) << 31) | 0x3F800000u);
  } else {
    static_assert(DL == 4, "(-1,1) and Gaussian: one call (four rows) per lane");
    const uint64_t g = gi >> 2;
    const int sh = (int)(gi & 3);
    float v[4];
    quad_values<DIST>(seed, g, j, v);
    if (sh == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) s[t] = v[t];
    } else {
      float u[4];
      quad_values<DIST>(seed, g + 1, j, u);
#pragma unroll
      for (int t = 0; t < 4; ++t) s[t] = t + sh < 4 ? v[t + sh] : u[t + sh - 4];
    }
  }
}

// ACC = float: the product form (A's values rounded to FP32, FP32 sums).
// ACC = double: the FP64 form for the SVD form of sketch-and-precondition,
// where singular values down to 1e-12 sigma_max must survive the sketch: the
// same S entries (exact in FP64), A's values in FP64, FP64 sums.
template <int DIST, int DL, typename ACC = float>
__global__ __launch_bounds__(64 * CW_WAVES) void k_sketch_colwise(ColwiseParams P) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tgroups = (P.tiles + CW_WAVES - 1) / CW_WAVES;
  const int64_t c = blockIdx.x / tgroups;  // the chunk
  const int64_t tile = (blockIdx.x - c * tgroups) * CW_WAVES + wave;
  if (tile >= P.tiles || c >= P.cbase[P.n]) return;
  const int64_t k = colwise_column(P.cbase, P.n, c);
  const int64_t r = c - P.cbase[k];                 // chunk within the column
  const bool heavy = P.cbase[k + 1] - P.cbase[k] > 1;
  const int64_t i0 = tile * (64 * DL) + (int64_t)lane * DL;  // the lane's first row
  ACC acc[DL];
#pragma unroll
  for (int t = 0; t < DL; ++t) acc[t] = (ACC)0;
  const int status = P.hdr->status;
  if (status == 0 && i0 < P.d) {
    const uint64_t gi = (uint64_t)(P.row0 + i0);
    const int64_t p0 = P.colptr[k] + (heavy ? r * P.chunk : 0);
    const int64_t pe = P.colptr[k + 1];
    const int64_t p1 = heavy && p0 + P.chunk < pe ? p0 + P.chunk : pe;
    for (int64_t p = p0; p < p1; ++p) {
      const uint64_t j = (uint64_t)(uint32_t)P.rowidx[p];
      float s[DL];
      colwise_values<DIST, DL>(P.seed, gi, j, s);
      if constexpr (sizeof(ACC) == 4) {
        const float a = load_value(P.vals, P.vtype, p);
#pragma unroll
        for (int t = 0; t < DL; ++t) acc[t] = __builtin_fmaf(a, s[t], acc[t]);
      } else {
        const double a = load_value_f64(P.vals, P.vtype, p);
#pragma unroll
        for (int t = 0; t < DL; ++t) acc[t] = __builtin_fma(a, (double)s[t], acc[t]);
      }
    }
  }
  if (heavy) {  // the chunk's partial sum (a matrix that failed validation has no heavy column)
    ACC* part = (ACC*)P.part + (P.hbase[k] + r) * P.d;
#pragma unroll
    for (int t = 0; t < DL; ++t)
      if (i0 + t < P.d) part[i0 + t] = acc[t];
    return;
  }
  ACC* out = (ACC*)P.out;
  const ACC nan = (ACC)__builtin_nan("");
#pragma unroll
  for (int t = 0; t < DL; ++t)
    if (i0 + t < P.d) out[i0 + t + k * P.ld] = status ? nan : acc[t];
}

// A_hat[:, k] of each heavy column k: its chunks' partials added in chunk
// order.  Grid: heavy-column capacity x row blocks of 256.
template <typename ACC>
__global__ void k_colwise_reduce(const int32_t* __restrict__ hk, const int32_t* __restrict__ hcol,
                                 const int32_t* __restrict__ cbase,
                                 const int32_t* __restrict__ hbase, int64_t n, int64_t d,
                                 const ACC* __restrict__ part, ACC* __restrict__ out, int64_t ld) {
  const int64_t rblocks = (d + 255) / 256;
  const int64_t h = blockIdx.x / rblocks;
  const int64_t i = (blockIdx.x - h * rblocks) * 256 + threadIdx.x;
  if (h >= hk[n] || i >= d) return;
  const int64_t k = hcol[h];
  const int64_t nch = cbase[k + 1] - cbase[k];
  const ACC* src = part + (int64_t)hbase[k] * d + i;
  ACC s = (ACC)0;
  for (int64_t r = 0; r < nch; ++r) s += src[r * d];
  out[i + k * ld] = s;
}

}  // namespace sk

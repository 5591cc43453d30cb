// sk_dense.hpp -- row blocks of A dense enough to run as a dense contraction
// on the matrix cores.
//
// The sparse kernel spends a few VALU instructions per nonzero on top of the
// multiply-add; a row block whose density reaches a threshold is cheaper as
// A_hat_tile += S_tile * A_blk with A_blk densified, on MFMA (the paper's
// large-density regime of the cost model, Sec. III-A-2, where reuse of the
// S tile across columns is near its maximum).  Steps:
//   k_dense_select  picks the dense blocks in increasing block order
//                   (deterministic list, capped by the workspace capacity);
//                   their rows are concatenated in that order
//   k_densify       writes the dense rows as a row-major (rows x n) matrix
//   k_dense_mfma    one workgroup per 64 x 64 output tile; per 32-row K chunk
//                   of the dense rows it regenerates S (64 S rows x 32 A
//                   rows) into LDS, loads the dense A chunk, and runs
//                   v_mfma_f32_32x32x2f32 per wave (each wave a 32 x 32
//                   quarter); the tile is written to its own slice of the
//                   split partials, so the final reduction stays fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"
#include "sk_rng.hpp"

namespace sk {

typedef float floatx16 __attribute__((ext_vector_type(16)));

struct DenseHeader {
  int32_t nd;       // dense blocks selected
  int32_t rows;     // their rows, concatenated in block order
  int32_t pad[14];
};

// single workgroup: dense blocks in block order, taken while the dense-row
// capacity lasts; dflag[b] = slot + 1 or 0, doff[slot] = first dense row
__global__ __launch_bounds__(256) void k_dense_select(const int32_t* __restrict__ seg, int64_t nv,
                                                      int64_t n, const int32_t* __restrict__ bstart,
                                                      int32_t min_pct, int64_t kd_max,
                                                      const Header* __restrict__ hdr,
                                                      int32_t* __restrict__ dflag,
                                                      int32_t* __restrict__ dlist,
                                                      int32_t* __restrict__ doff,
                                                      DenseHeader* __restrict__ dh) {
  __shared__ int32_t sh_f[256];
  __shared__ int32_t sh_r[256];
  const int tid = threadIdx.x;
  const int64_t nb = hdr->status ? 0 : hdr->nblocks;
  int32_t base_f = 0, base_r = 0;
  bool full = false;
  for (int64_t b0 = 0; b0 < nb; b0 += 256) {
    const int64_t b = b0 + tid;
    int flag = 0, rb = 0;
    if (b < nb) {
      rb = bstart[b + 1] - bstart[b];
      const int64_t cnt = (int64_t)seg[(b + 1) * nv] - (int64_t)seg[b * nv];
      // density >= min_pct %  <=>  100 cnt >= min_pct rb n
      flag = (!full && 100 * cnt >= (int64_t)min_pct * rb * n) ? 1 : 0;
    }
    if (!__syncthreads_or(flag)) {  // (usual: no dense block here, nothing taken)
      if (b < nb) dflag[b] = 0;
      continue;
    }
    sh_f[tid] = flag;
    sh_r[tid] = flag ? rb : 0;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive scans
      const int32_t af = tid >= off ? sh_f[tid - off] : 0;
      const int32_t ar = tid >= off ? sh_r[tid - off] : 0;
      __syncthreads();
      sh_f[tid] += af;
      sh_r[tid] += ar;
      __syncthreads();
    }
    const int32_t slot = base_f + sh_f[tid] - flag;
    const int64_t row_end = (int64_t)base_r + sh_r[tid];  // inclusive of this block
    const bool take = flag && row_end <= kd_max;
    if (b < nb) {
      dflag[b] = take ? slot + 1 : 0;
      if (take) {
        dlist[slot] = (int32_t)b;
        doff[slot] = (int32_t)(row_end - rb);
      }
    }
    // the taken blocks are a prefix of the flagged ones: count them
    const int taken = __syncthreads_count(take ? 1 : 0);
    const bool overflow = __syncthreads_or(flag && !take);
    int32_t rows_taken = 0;
    if (tid == 0) sh_f[0] = 0;
    __syncthreads();
    if (take) atomicAdd(&sh_f[0], rb);
    __syncthreads();
    rows_taken = sh_f[0];
    __syncthreads();
    base_f += taken;
    base_r += rows_taken;
    if (overflow) full = true;
  }
  if (tid == 0) {
    dh->nd = base_f;
    dh->rows = base_r;
  }
}

// zero the dense rows in use (grid-stride)
__global__ void k_dense_zero(float* __restrict__ D, int64_t n, const DenseHeader* __restrict__ dh) {
  const int64_t total = (int64_t)dh->rows * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    D[i] = 0.0f;
}

// drows[t] = the A row of dense row t (t < rows); one thread per dense row
__global__ void k_dense_rows(const int32_t* __restrict__ rowlist, const int32_t* __restrict__ bstart,
                             const int32_t* __restrict__ dlist, const int32_t* __restrict__ doff,
                             const DenseHeader* __restrict__ dh, int32_t* __restrict__ drows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= dh->rows) return;
  int lo = 0, hi = dh->nd - 1;  // last slot with doff <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (doff[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  drows[t] = rowlist[bstart[dlist[lo]] + (t - doff[lo])];
}

// D[doff[slot] + l][k] = a for every entry of dense block dlist[slot]; one
// thread per (slot, virtual column) walks the column's segment and writes
// real column k (vbase == nullptr: virtual == real).
__global__ void k_densify(const int32_t* __restrict__ seg, const uint2* __restrict__ ent, int64_t nv,
                          int64_t n, const int32_t* __restrict__ vbase, int32_t row_bytes,
                          const int32_t* __restrict__ dlist, const int32_t* __restrict__ doff,
                          const DenseHeader* __restrict__ dh, float* __restrict__ D) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slot = t / nv, v = t - slot * nv;
  if (slot >= dh->nd) return;
  if (vbase && v >= vbase[n]) return;
  const int64_t k = vbase ? real_column(vbase, n, v) : v;
  const int64_t b = dlist[slot];
  float* Dt = D + (int64_t)doff[slot] * n;
  const int32_t p0 = seg[b * nv + v], p1 = seg[b * nv + v + 1];
  for (int32_t p = p0; p < p1; ++p) {
    const uint2 e = ent[p];
    const int32_t l = (int32_t)(e.x / (uint32_t)row_bytes);
    Dt[(int64_t)l * n + k] = __uint_as_float(e.y);
  }
}

struct DenseParams {
  const int32_t* drows;  // A row of each dense row
  const DenseHeader* dh;
  const Header* hdr;
  const float* D;        // dense rows x n, row-major
  int64_t n, d, row0;
  uint64_t seed;
  float* out;  // the dense slice of the split partials (d x n, ld = d)
};

constexpr int DT_M = 64, DT_N = 64, DT_K = 32;

// S[grow0 + i][rows[kk]] for i < 64, kk < 32 (kk >= nk: zero) into
// Ss[i * (DT_K + 1) + kk]
template <int DIST>
__device__ __forceinline__ void dense_fill_s(float* __restrict__ Ss, const int32_t* __restrict__ rows,
                                             int nk, uint64_t grow0, uint64_t seed) {
  const int tid = threadIdx.x;
  if (DIST == DIST_RADEMACHER) {
    // one generator call per (row, 128-row group the 64 tile rows touch: one,
    // or two when the tile straddles a group boundary); each word of a call
    // holds 32 consecutive rows' signs
    const uint64_t g0 = grow0 >> 7;
    const int ng = (int)(((grow0 + DT_M - 1) >> 7) - g0 + 1);
    if (tid < ng * DT_K) {
      const int kk = tid / ng, gi = tid - kk * ng;
      const uint64_t g = g0 + (uint64_t)gi;
      Words x{0u, 0u, 0u, 0u};
      if (kk < nk) x = gen_words(seed, g, (uint64_t)(uint32_t)rows[kk]);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t bits = word_at(x, w);
        const int64_t r_w = (int64_t)(g * 128u) + 32 * w;
        for (int u = 0; u < 32; ++u) {
          const int64_t i = r_w + u - (int64_t)grow0;
          if (i >= 0 && i < DT_M)
            Ss[i * (DT_K + 1) + kk] = kk < nk ? ((bits >> u) & 1u ? -1.0f : 1.0f) : 0.0f;
        }
      }
    }
  } else {
    // 64 S rows span 16 generator groups (17 when grow0 is not 4-aligned)
    const int shift = (int)(grow0 & 3u);
    const int ng = shift ? 17 : 16;
    const uint64_t g0 = grow0 >> 2;
    for (int idx = tid; idx < ng * DT_K; idx += 256) {
      const int kk = idx / ng, gi = idx - kk * ng;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (kk < nk) quad_values<DIST>(seed, g0 + gi, (uint64_t)(uint32_t)rows[kk], v);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int i = gi * 4 + w - shift;
        if (i >= 0 && i < DT_M) Ss[i * (DT_K + 1) + kk] = v[w];
      }
    }
  }
}

template <int DIST>
__global__ __launch_bounds__(256) void k_dense_mfma(DenseParams P) {
  __shared__ float Ss[DT_M * (DT_K + 1)];
  __shared__ float Ds[DT_K * (DT_N + 4)];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t ntiles = (P.n + DT_N - 1) / DT_N;
  const int64_t tm = blockIdx.x / ntiles, tn = blockIdx.x - tm * ntiles;
  const int64_t i0 = tm * DT_M, j0 = tn * DT_N;
  const uint64_t grow0 = (uint64_t)(P.row0 + i0);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

  const int64_t K = P.hdr->status ? 0 : P.dh->rows;
  for (int64_t k0 = 0; k0 < K; k0 += DT_K) {
    const int nk = (int)(K - k0 < DT_K ? K - k0 : DT_K);
    __syncthreads();
    dense_fill_s<DIST>(Ss, P.drows + k0, nk, grow0, P.seed);
    const float* Dt = P.D + k0 * P.n;
    for (int idx = tid; idx < DT_K * DT_N; idx += 256) {
      const int kk = idx / DT_N, jj = idx - kk * DT_N;
      const int64_t j = j0 + jj;
      Ds[kk * (DT_N + 4) + jj] = (kk < nk && j < P.n) ? Dt[(int64_t)kk * P.n + j] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < DT_K; kq += 2) {
      const int kk = kq + (lane >> 5);
      const float a = Ss[(wm + (lane & 31)) * (DT_K + 1) + kk];
      const float bv = Ds[kk * (DT_N + 4) + wn + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc, 0, 0, 0);
    }
  }
  // D[i][j]: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4
  const int64_t j = j0 + wn + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (i < P.d && j < P.n) P.out[i + j * P.d] = acc[r];
  }
}

}  // namespace sk

// sk_mfma.hpp -- the sketch on the matrix cores for +-1 S in BF16 or FP8.
//
// A +-1 entry is exact in BF16 and in FP8 (E4M3), so S A can run as a dense
// contraction on MFMA with FP32 accumulation; the only rounding is that of A's
// values (BF16: 8-bit significand; FP8: the value split as hi + lo, two E4M3
// numbers, about 8 significant bits together) and of the FP32 sums.  Row
// blocks are densified on the fly in LDS: nothing dense is written to HBM.
//
// One work unit owns an output tile A_hat[i0 : i0 + 64, c0 : c0 + 128] for a
// run of row blocks (a split), four waves each holding a 32 x 64 quarter as
// two 32 x 32 MFMA accumulators.  Per block of at most MF_MB rows:
//   1. S tile (64 S rows x the block's rows) from the generator's sign bits,
//      stored as +-1 in the operand format,
//   2. the block's entries in the unit's 128 columns scattered into a zeroed
//      dense tile (column-major, the block's rows contiguous),
//   3. for every 16 rows: v_mfma_f32_32x32x16 (bf16 or fp8) per accumulator.
// Both operands use the same lane -> K mapping, so each instruction forms the
// right dot products whatever the hardware's K order inside a lane group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"
#include "sk_rng.hpp"
#include "sk_sketch.hpp"

namespace sk {

enum : int { MF_BF16 = 1, MF_FP8 = 2 };

constexpr int MF_MB = 128;     // rows per block (K extent of one dense tile)
constexpr int MF_TM = 64;      // S rows per unit
constexpr int MF_TN = 128;     // columns per unit
constexpr int MF_THREADS = 256;

typedef float mf_floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));

template <int FMT>
struct MfmaLds;

template <>
struct MfmaLds<MF_BF16> {
  static constexpr int LDK = MF_MB + 8;  // elements per tile row (16-byte aligned, skewed)
  uint16_t S[MF_TM][LDK];
  uint16_t A[MF_TN][LDK];
  int32_t seg[MF_TN + 1];
};

template <>
struct MfmaLds<MF_FP8> {
  static constexpr int LDK = MF_MB + 16;
  uint8_t S[MF_TM][LDK];
  uint8_t Ahi[MF_TN][LDK];
  uint8_t Alo[MF_TN][LDK];
  int32_t seg[MF_TN + 1];
};

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // finite inputs
}

// first k in [lo, hi) with seg[k + 1] > p (seg non-decreasing)
__device__ __forceinline__ int seg_column(const int32_t* seg, int cols, int32_t p) {
  int lo = 0, hi = cols - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (seg[mid + 1] > p) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

template <int FMT>
__device__ __forceinline__ void mfma_unit(const SketchParams& P, int split, int tile, int crange,
                                          unsigned char* __restrict__ smem) {
  MfmaLds<FMT>& L = *reinterpret_cast<MfmaLds<FMT>*>(smem);
  constexpr int LDK = MfmaLds<FMT>::LDK;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int mh = wave & 1, nh = wave >> 1;
  const int64_t i0 = (int64_t)tile * MF_TM;
  const int64_t c0 = (int64_t)crange * MF_TN;
  const int cols = (int)(P.n - c0 < MF_TN ? P.n - c0 : MF_TN);
  const uint64_t grow0 = (uint64_t)(P.row0 + i0);

  mf_floatx16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;

  const int status = P.hdr->status;
  if (status == 0) {
    const int64_t nb = P.hdr->nblocks;
    const int64_t T = P.bcost[nb];
    auto first_at = [&](int64_t x) {
      int64_t lo = 0, hi = nb;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (P.bcost[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    const int64_t b_lo = first_at((split * T + P.splits - 1) / P.splits);
    const int64_t b_hi =
        split + 1 == P.splits ? nb : first_at(((split + 1) * T + P.splits - 1) / P.splits);
    uint32_t one_fp8 = 0, neg_fp8 = 0;
    if constexpr (FMT == MF_FP8) {
      one_fp8 = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(1.0f, 1.0f, 0, false) & 0xFFu;
      neg_fp8 = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(-1.0f, -1.0f, 0, false) & 0xFFu;
    }
    for (int64_t b = b_lo; b < b_hi; ++b) {
      const int32_t r0 = P.bstart[b];
      const int rb = P.bstart[b + 1] - r0;
      const int32_t* segb = P.seg + b * P.n + c0;
      __syncthreads();  // the previous block's tiles are consumed
      // zero the dense tile, stage the unit's segment bounds
      if constexpr (FMT == MF_BF16) {
        uint32_t* z = reinterpret_cast<uint32_t*>(&L.A[0][0]);
        for (int i = tid; i < MF_TN * LDK / 2; i += MF_THREADS) z[i] = 0u;
      } else {
        uint32_t* z = reinterpret_cast<uint32_t*>(&L.Ahi[0][0]);
        for (int i = tid; i < 2 * MF_TN * LDK / 4; i += MF_THREADS) z[i] = 0u;
      }
      for (int k = tid; k <= cols; k += MF_THREADS) L.seg[k] = segb[k];
      // S tile: 64 rows x rb block rows; rows beyond rb are zero
      {
        const int l = tid >> 1, half = tid & 1;
        if (l < MF_MB) {
          uint32_t bits = 0;
          const bool live = l < rb;
          if (live) bits = sign_bits32(P.seed, grow0 + 32u * half, (uint64_t)(uint32_t)P.rowlist[r0 + l]);
#pragma unroll 8
          for (int u = 0; u < 32; ++u) {
            const bool neg = (bits >> u) & 1u;
            if constexpr (FMT == MF_BF16)
              L.S[32 * half + u][l] = live ? (neg ? 0xBF80u : 0x3F80u) : 0u;
            else
              L.S[32 * half + u][l] = live ? (uint8_t)(neg ? neg_fp8 : one_fp8) : (uint8_t)0;
          }
        }
      }
      __syncthreads();
      // scatter the entries of the unit's columns (row offset in e.x)
      const int32_t p0 = L.seg[0], p1 = L.seg[cols];
      for (int32_t p = p0 + tid; p < p1; p += MF_THREADS) {
        const uint2 e = P.ent[p];
        const int c = seg_column(L.seg, cols, p);
        const float a = __uint_as_float(e.y);
        if constexpr (FMT == MF_BF16) {
          L.A[c][e.x] = bf16_rne(a);
        } else {
          const uint32_t hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, a, 0, false) & 0xFFu;
          const float back = __builtin_amdgcn_cvt_f32_fp8((int)hi, 0);
          const uint32_t lo =
              (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a - back, a - back, 0, false) & 0xFFu;
          L.Ahi[c][e.x] = (uint8_t)hi;
          L.Alo[c][e.x] = (uint8_t)lo;
        }
      }
      __syncthreads();
      // K loop: 16 rows per instruction
      const int kq = 8 * (lane >> 5);
      const int mrow = 32 * mh + (lane & 31);
      for (int k0 = 0; k0 < rb; k0 += 16) {
        if constexpr (FMT == MF_BF16) {
          const mf_bf16x8 a = *reinterpret_cast<const mf_bf16x8*>(&L.S[mrow][k0 + kq]);
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const int ncol = 64 * nh + 32 * t + (lane & 31);
            const mf_bf16x8 bv = *reinterpret_cast<const mf_bf16x8*>(&L.A[ncol][k0 + kq]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[t], 0, 0, 0);
          }
        } else {
          const long a = *reinterpret_cast<const long*>(&L.S[mrow][k0 + kq]);
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const int ncol = 64 * nh + 32 * t + (lane & 31);
            const long bh = *reinterpret_cast<const long*>(&L.Ahi[ncol][k0 + kq]);
            const long bl = *reinterpret_cast<const long*>(&L.Alo[ncol][k0 + kq]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, bh, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, bl, acc[t], 0, 0, 0);
          }
        }
      }
    }
  }
  // C[i][j]: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4
  float* __restrict__ out = P.out + (int64_t)split * P.split_stride;
  const float nan = __uint_as_float(0x7FC00000u);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t j = c0 + 64 * nh + 32 * t + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t i = i0 + 32 * mh + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (i < P.d && j < P.n) out[i + j * P.ld] = status ? nan : acc[t][r];
    }
  }
}

template <int FMT>
__global__ __launch_bounds__(MF_THREADS) void k_sketch_mfma(SketchParams P) {
  __shared__ __align__(16) unsigned char smem[sizeof(MfmaLds<FMT>)];
  const int bid = blockIdx.x;
  const int split = bid % P.splits;
  const int rest = bid / P.splits;
  mfma_unit<FMT>(P, split, rest % P.tiles, rest / P.tiles, smem);
}

}  // namespace sk

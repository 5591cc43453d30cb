// sk_mfma.hpp -- the sketch on the matrix cores for +-1 S in BF16 or FP8.
//
// A +-1 entry is exact in BF16 and in FP8 (E4M3), so S A can run as a dense
// contraction on MFMA with FP32 accumulation; the only rounding is that of A's
// values (BF16: 8-bit significand; FP8: the value split as hi + lo, two E4M3
// numbers, about 8 significant bits together) and of the FP32 sums.  Row
// blocks are densified on the fly in LDS: nothing dense is written to HBM.
//
// One work unit owns an output tile A_hat[i0 : i0 + 128, c0 : c0 + 256] for
// a run of row blocks (a split); eight waves each hold a 32 x 128 part as four
// 32 x 32 MFMA accumulators.  Per block of at most MF_MB rows:
//   1. the S tile (128 S rows x the block's rows) as sign bits, one ballot
//      per S row; expanded to +-1 operands through a 256-entry table,
//   2. the block's entries in the unit's 256 columns scattered into a zeroed
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

constexpr int MF_MB = 128;      // rows per block (K extent of one dense tile)
constexpr int MF_TM = 128;      // S rows per unit
constexpr int MF_TN = 256;      // columns per unit
constexpr int MF_THREADS = 512; // eight waves: four S-row quarters x two column halves

typedef float mf_floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));

// S is held as bits (bit k % 8 of byte [i][k / 8]: S row i, block row k;
// set = -1) and expanded to MFMA operands through a table of the 256 byte
// values -> eight +-1 operands.
template <int FMT>
struct MfmaLds;

template <>
struct MfmaLds<MF_BF16> {
  static constexpr int LDK = MF_MB + 8;  // elements per dense-tile row (16-byte rows, skewed)
  uint16_t A[MF_TN][LDK];
  uint4 lut[256];                        // eight bf16 +-1
  uint8_t S[MF_TM][MF_MB / 8];
  int32_t seg[MF_TN + 1];
};

template <>
struct MfmaLds<MF_FP8> {
  static constexpr int LDK = MF_MB + 16;
  uint8_t Ahi[MF_TN][LDK];
  uint8_t Alo[MF_TN][LDK];
  uint2 lut[256];                        // eight fp8 +-1
  uint8_t S[MF_TM][MF_MB / 8];
  int32_t seg[MF_TN + 1];
};

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // finite inputs
}

// first k in [0, cols) with seg[k + 1] > p (seg non-decreasing)
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
  const int mq = wave & 3, nh = wave >> 2;  // S-row quarter, column half
  const int64_t i0 = (int64_t)tile * MF_TM;
  const int64_t c0 = (int64_t)crange * MF_TN;
  const int cols = (int)(P.n - c0 < MF_TN ? P.n - c0 : MF_TN);
  const uint64_t grow0 = (uint64_t)(P.row0 + i0);

  mf_floatx16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;

  // operand table: byte -> eight +-1 values (bit set: -1)
  if (tid < 256) {
    if constexpr (FMT == MF_BF16) {
      uint32_t w[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint32_t lo = (tid >> (2 * h)) & 1u ? 0xBF80u : 0x3F80u;
        const uint32_t hi = (tid >> (2 * h + 1)) & 1u ? 0xBF80u : 0x3F80u;
        w[h] = lo | (hi << 16);
      }
      L.lut[tid] = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
      const uint32_t one = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(1.0f, 1.0f, 0, false) & 0xFFu;
      const uint32_t neg = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(-1.0f, -1.0f, 0, false) & 0xFFu;
      uint32_t w[2] = {0u, 0u};
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e >> 2] |= ((tid >> e) & 1u ? neg : one) << (8 * (e & 3));
      L.lut[tid] = make_uint2(w[0], w[1]);
    }
  }

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
    // Software pipeline over the blocks: while block b runs on the matrix
    // cores, the entries and rows of block b + 1 and the segment bounds of
    // block b + 2 are in flight to registers.
    const int krow = 64 * nh + lane;  // the block row whose S bits this thread makes
    struct Bounds {
      int32_t r0, rb, segv, p0, p1;
    };
    auto load_bounds = [&](int64_t b) {
      Bounds x;
      x.r0 = P.bstart[b];
      x.rb = P.bstart[b + 1] - x.r0;
      const int32_t* segb = P.seg + b * P.n + c0;
      x.segv = tid <= cols ? segb[tid] : 0;
      x.p0 = segb[0];
      x.p1 = segb[cols];
      return x;
    };
    constexpr int ET = 4;  // entries per thread carried in registers
    uint2 ent[ET];
    int32_t row = 0;
    auto load_payload = [&](const Bounds& x) {
#pragma unroll
      for (int q = 0; q < ET; ++q) {
        const int32_t p = x.p0 + tid + q * MF_THREADS;
        ent[q] = p < x.p1 ? P.ent[p] : make_uint2(0u, 0u);
      }
      row = krow < x.rb ? P.rowlist[x.r0 + krow] : 0;
    };
    Bounds cur{}, nxt{};
    if (b_lo < b_hi) {
      cur = load_bounds(b_lo);
      load_payload(cur);
    }
    if (b_lo + 1 < b_hi) nxt = load_bounds(b_lo + 1);
    for (int64_t b = b_lo; b < b_hi; ++b) {
      const int rb = cur.rb;
      __syncthreads();  // the previous block's tiles are consumed
      // zero the dense tile, stage the unit's segment bounds
      {
        uint4* z = reinterpret_cast<uint4*>(smem);
        constexpr int n16 = (FMT == MF_BF16 ? MF_TN * LDK * 2 : 2 * MF_TN * LDK) / 16;
        for (int i = tid; i < n16; i += MF_THREADS) z[i] = make_uint4(0u, 0u, 0u, 0u);
      }
      if (tid <= cols) L.seg[tid] = cur.segv;
      // S bits: wave w takes S rows 32 (w & 3) .. + 31 and block rows
      // 64 (w >> 2) .. + 63 (one per lane); one ballot per S row gives the
      // 64 bits of that row for the wave's block rows
      {
        uint32_t bits = 0;
        if (krow < rb) bits = sign_bits32(P.seed, grow0 + 32u * mq, (uint64_t)(uint32_t)row);
        for (int u = 0; u < 32; ++u) {
          const uint64_t srow = __ballot((bits >> u) & 1u);
          if (lane == u) *reinterpret_cast<uint64_t*>(&L.S[32 * mq + u][8 * nh]) = srow;
        }
      }
      __syncthreads();
      // scatter the entries of the unit's columns (row offset in e.x): those
      // carried in registers, then any beyond them straight from memory
      auto put = [&](const uint2 e, int32_t p) {
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
      };
#pragma unroll
      for (int q = 0; q < ET; ++q) {
        const int32_t p = cur.p0 + tid + q * MF_THREADS;
        if (p < cur.p1) put(ent[q], p);
      }
      for (int32_t p = cur.p0 + tid + ET * MF_THREADS; p < cur.p1; p += MF_THREADS) put(P.ent[p], p);
      // prefetch: entries and rows of block b + 1, bounds of block b + 2
      if (b + 1 < b_hi) load_payload(nxt);
      Bounds nn{};
      if (b + 2 < b_hi) nn = load_bounds(b + 2);
      __syncthreads();
      // K loop: 16 block rows per instruction; rows past rb are zero in A
      const int kq = 8 * (lane >> 5);
      const int mrow = 32 * mq + (lane & 31);
      for (int k0 = 0; k0 < rb; k0 += 16) {
        const int sb = L.S[mrow][(k0 + kq) >> 3];
        if constexpr (FMT == MF_BF16) {
          const uint4 sv = L.lut[sb];
          const mf_bf16x8 a = *reinterpret_cast<const mf_bf16x8*>(&sv);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int ncol = 128 * nh + 32 * t + (lane & 31);
            const mf_bf16x8 bv = *reinterpret_cast<const mf_bf16x8*>(&L.A[ncol][k0 + kq]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[t], 0, 0, 0);
          }
        } else {
          const uint2 sv = L.lut[sb];
          const long a = (long)(((uint64_t)sv.y << 32) | sv.x);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int ncol = 128 * nh + 32 * t + (lane & 31);
            const long bh = *reinterpret_cast<const long*>(&L.Ahi[ncol][k0 + kq]);
            const long bl = *reinterpret_cast<const long*>(&L.Alo[ncol][k0 + kq]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, bh, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, bl, acc[t], 0, 0, 0);
          }
        }
      }
      cur = nxt;
      nxt = nn;
    }
  }
  // C[i][j]: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4
  float* __restrict__ out = P.out + (int64_t)split * P.split_stride;
  const float nan = __uint_as_float(0x7FC00000u);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t j = c0 + 128 * nh + 32 * t + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t i = i0 + 32 * mq + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
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

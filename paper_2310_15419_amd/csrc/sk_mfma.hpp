// sk_mfma.hpp -- the sketch on the matrix cores for +-1 S in BF16 or FP8.
//
// A +-1 entry is exact in BF16 and in FP8 (E4M3), so S A can run as a dense
// contraction on MFMA with FP32 accumulation; the only rounding is that of A's
// values (BF16: 8-bit significand; FP8: the value split as hi + lo, two E4M3
// numbers, about 8 significant bits together) and of the FP32 sums.  Row
// blocks are densified on the fly in LDS: nothing dense is written to HBM.
//
// One work unit owns an output tile A_hat[i0 : i0 + 128, c0 : c0 + 256] for
// a run of row blocks (a split).  Eight waves run the matrix cores, each
// holding four 32 x 32 accumulators (a 32 x 128 part in BF16, 64 x 64 in
// FP8, where each operand read from LDS then feeds two instructions); eight
// more waves, in
// two groups that take turns, build the next block's tiles in a second copy
// meanwhile, so building and multiplying overlap:
//   1. the S tile (128 S rows x the block's rows) as sign bits: one
//      generator call per block row gives its 128 bits (four words), which a
//      bit transpose across the lanes turns into words per S row; each
//      matrix-core lane reads its S row's two words once per block and makes
//      every +-1 operand from them with a shift and a mask,
//   2. the block's entries in the unit's 256 columns scattered into the
//      dense tile (column-major, the block's rows contiguous), after zeros
//      over the entries the copy held before,
//   3. for every 16 rows: v_mfma_f32_32x32x16 (bf16 or fp8) per accumulator.
// One workgroup barrier per block hands the copies over.
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
constexpr int MF_CONSUMERS = 8; // waves on the matrix cores
constexpr int MF_PRODUCERS = 8; // waves building tiles: two groups (even, odd blocks) of
                                // four, 64 columns each
constexpr int MF_THREADS = 64 * (MF_CONSUMERS + MF_PRODUCERS);
constexpr int MF_EQ = 8;        // entries per producer lane kept in registers

typedef float mf_floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));

// Two copies of the per-block tiles (the one the matrix cores read and the
// one being built).  S is held per S row: W[h][i][u] holds the signs (bit
// set: -1) of S row i in the block rows a matrix-core lane of half h needs
// for steps 4u .. 4u + 3 (block rows 16 s + 8 h + e, e < 8), at the bit
// positions mf_bit_pos gives, so that each operand word is one shift and
// one mask away.
template <int FMT>
struct MfmaLds;

// Bit position in a W word of element e (block row 16 s + 8 h + e) of step
// s = 4 u + j: BF16 operands are pairs of 16-bit values, sign bits 15 and 31,
// taken with a left shift by (e / 2 + 4 j); FP8 operands are four bytes,
// sign bits 7, 15, 23, 31, taken with a shift by (e / 4 + 2 j).
template <int FMT>
__device__ __forceinline__ int mf_bit_pos(int j, int e) {
  if constexpr (FMT == MF_BF16) return 15 + 16 * (e & 1) - (e >> 1) - 4 * j;
  else return 7 + 8 * (e & 3) - (e >> 2) - 2 * j;
}

// (j, e) of bit position r (the inverse of mf_bit_pos)
template <int FMT>
__device__ __forceinline__ void mf_bit_owner(int r, int& j, int& e) {
  if constexpr (FMT == MF_BF16) {
    const int lo = 15 - (r & 15);
    j = lo >> 2;
    e = ((r >> 4) & 1) | ((lo & 3) << 1);
  } else {
    const int lo = 7 - (r & 7);
    j = lo >> 1;
    e = ((r >> 3) & 3) | ((lo & 1) << 2);
  }
}

// x of lane l ^ D (within each 32-lane half).  D = 1, 2, 8 are single DPP
// moves (quad permutations; a rotation by 8 within a 16-lane row), D = 4
// takes one of two row rotations (a row rotation by r brings lane l - r mod
// 16), D = 16 goes through the LDS crossbar; only the last has LDS latency.
template <int D>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, int lane) {
  const int v = (int)x;
  if constexpr (D == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  if constexpr (D == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  if constexpr (D == 8) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
  if constexpr (D == 4) {
    const int dn = __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, false);  // from l - 4
    const int up = __builtin_amdgcn_mov_dpp(v, 0x12C, 0xF, 0xF, false);  // from l + 4
    return (uint32_t)((lane & 4) ? dn : up);
  }
  if constexpr (D == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x1F | (16 << 10));
}

// One stage of a 32 x 32 bit transpose across the lanes of each 32-lane
// half: lanes l and l ^ D swap the D x D blocks off the diagonal (M selects
// the bit positions with bit D clear).
template <int D, uint32_t M>
__device__ __forceinline__ uint32_t transpose_stage(uint32_t x, int lane) {
  const uint32_t p = lane_xor<D>(x, lane);
  const bool upper = (lane & D) != 0;
  const uint32_t z = __builtin_amdgcn_alignbit(p, p, upper ? D : 32 - D);  // rotate by -/+ D
  const uint32_t keep = upper ? ~M : M;
  return (x & keep) | (z & ~keep);
}

// After it, lane t's bit r is lane r's bit t (within each 32-lane half).
__device__ __forceinline__ uint32_t transpose32(uint32_t x, int lane) {
  x = transpose_stage<16, 0x0000FFFFu>(x, lane);
  x = transpose_stage<8, 0x00FF00FFu>(x, lane);
  x = transpose_stage<4, 0x0F0F0F0Fu>(x, lane);
  x = transpose_stage<2, 0x33333333u>(x, lane);
  return transpose_stage<1, 0x55555555u>(x, lane);
}

template <>
struct MfmaLds<MF_BF16> {
  static constexpr int LDK = MF_MB + 8;  // elements per dense-tile row (16-byte rows, skewed)
  uint16_t A[2][MF_TN][LDK];
  uint32_t W[2][2][MF_TM][2];
};

template <>
struct MfmaLds<MF_FP8> {
  static constexpr int LDK = MF_MB + 8;  // bytes per row: 34 dwords, so 32 lanes' 8-byte reads cover all banks
  uint8_t Ahi[2][MF_TN][LDK];
  uint8_t Alo[2][MF_TN][LDK];
  uint32_t W[2][2][MF_TM][2];
};

// (Parameters read from memory, as the batched kernel's are, arrive as
// generic pointers; the unit addresses its arrays through in_global.)

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // finite inputs
}

// Sign bits of the 128 consecutive S rows i..i+127 of column j, word t
// holding rows i + 32t .. i + 32t + 31 (bit set <=> -1): one generator call
// when i is a multiple of 128, else two, joined at the offset.
__host__ __device__ __forceinline__ Words sign_bits128(uint64_t seed, uint64_t i, uint64_t j) {
  const uint64_t g = i >> 7;
  const int s = (int)(i & 127);
  const Words a = gen_words(seed, g, j);
  if (s == 0) return a;
  const Words c = gen_words(seed, g + 1, j);
  const int q = s >> 5, r = s & 31;
  // words q .. q + 4 of the 256-bit concatenation a, c (q is 0..3)
  const uint32_t v0 = q == 0 ? a.x0 : q == 1 ? a.x1 : q == 2 ? a.x2 : a.x3;
  const uint32_t v1 = q == 0 ? a.x1 : q == 1 ? a.x2 : q == 2 ? a.x3 : c.x0;
  const uint32_t v2 = q == 0 ? a.x2 : q == 1 ? a.x3 : q == 2 ? c.x0 : c.x1;
  const uint32_t v3 = q == 0 ? a.x3 : q == 1 ? c.x0 : q == 2 ? c.x1 : c.x2;
  const uint32_t v4 = q == 0 ? c.x0 : q == 1 ? c.x1 : q == 2 ? c.x2 : c.x3;
  auto join = [r](uint32_t lo, uint32_t hi) { return r ? (lo >> r) | (hi << (32 - r)) : lo; };
  return Words{join(v0, v1), join(v1, v2), join(v2, v3), join(v3, v4)};
}

template <int FMT>
__device__ __forceinline__ void mfma_unit(const SketchParams& P, int split, int tile, int crange,
                                          unsigned char* __restrict__ smem) {
  MfmaLds<FMT>& L = *reinterpret_cast<MfmaLds<FMT>*>(smem);
  constexpr int LDK = MfmaLds<FMT>::LDK;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const bool consumer = wave < MF_CONSUMERS;
  // consumers: a wave holds RA x TB accumulators of 32 x 32, S-row group rg
  // (32 RA rows) and column group cg (32 TB columns); BF16 takes one S
  // operand per step across four column tiles (its operand VALU is the
  // larger cost), FP8 two S operands across two (its LDS reads are)
  constexpr int RA = FMT == MF_BF16 ? 1 : 2, TB = 4 / RA;
  const int rg = wave % (4 / RA), cg = (wave / (4 / RA)) % (8 / TB);
  // producers: group (the parity of the blocks it builds) and wave in it
  const int grp = __builtin_amdgcn_readfirstlane((wave - MF_CONSUMERS) >> 2);
  const int pw = __builtin_amdgcn_readfirstlane(wave & 3);
  const int64_t i0 = (int64_t)tile * MF_TM;
  const int64_t c0 = (int64_t)crange * MF_TN;
  const int cols = (int)(P.n - c0 < MF_TN ? P.n - c0 : MF_TN);
  const uint64_t grow0 = (uint64_t)(P.row0 + i0);
  const auto* hdr = in_global(P.hdr);
  const auto* bcost = in_global(P.bcost);
  const auto* bstart = in_global(P.bstart);
  const auto* seg = in_global(P.seg);
  const auto* rowlist = in_global(P.rowlist);
  const auto* ent64 = in_global(reinterpret_cast<const uint64_t*>(P.ent));
  auto ent = [ent64](int64_t p) {
    const uint64_t v = ent64[p];
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
  };

  const int status = hdr->status;
  int64_t b_lo = 0, b_hi = 0;
  if (status == 0) {
    const int64_t nb = hdr->nblocks;
    const int64_t T = bcost[nb];
    auto first_at = [&](int64_t x) {
      int64_t lo = 0, hi = nb;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (bcost[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    b_lo = first_at((split * T + P.splits - 1) / P.splits);
    b_hi = split + 1 == P.splits ? nb : first_at(((split + 1) * T + P.splits - 1) / P.splits);
  }

  if (!consumer) {
    // A producer wave builds its share of a copy for one block: waves 0 and
    // 1 the S words of 64 block rows each (one half h of the W layout, one
    // generator call per row), and every wave the dense
    // tile of its 64 columns: zeros where that copy's previous block had
    // entries (or everywhere, when they were not all kept), then the
    // block's entries.  A wave's LDS writes to its share all come from that
    // wave, in program order, so the producers never wait on each other.
    //
    // Group g builds the blocks of parity g, always into copy g, so it has
    // two blocks' time on the matrix cores between a build and the next:
    // right after a build it issues the loads of its next block's rows and
    // entries (in registers across the barriers) and of the bounds of the
    // block after that, and memory latency (longer than one block's time)
    // is covered.  Every build issues the same loads (indices held in range
    // rather than branched around), so the wait before a build covers only
    // loads two steps old.
    const int cw0 = 64 * pw;
    const int ncw = cols - cw0 < 64 ? cols - cw0 : 64;  // <= 0: past the last column
    const int cs0 = ncw > 0 ? cw0 : 0, cs1 = ncw > 0 ? cw0 + ncw : 0;
    // the group's S bits come from its waves 0 and 1: wave hh makes half
    // hh of the W layout, and lane r of its 32-lane half u generates block
    // row krow, whose sign lands at bit r of word u after the transpose
    // (one distinct generator call per lane)
    const bool signs = pw < 2;
    const int hh = pw & 1, wu = lane >> 5;
    int krow;
    {
      int j, e;
      mf_bit_owner<FMT>(lane & 31, j, e);
      krow = 16 * (4 * wu + j) + 8 * hh + e;
    }
    const int64_t nblk = b_hi - b_lo;
    struct Bounds {
      int32_t r0, rb, p0, p1;
    };
    struct Payload {
      int32_t row, rb, p0, p1;
      uint2 e[MF_EQ];
    };
    struct Placed {     // where a copy's block put this lane's entries
      int32_t count;    // the wave's entries; -1: not all kept (clear everything)
      uint32_t at[MF_EQ];
    };
    // bounds of block b_lo + i (any i >= 0: past the end, those of the last
    // block, unused)
    auto load_bounds = [&](int64_t i) {
      const int64_t b = b_lo + (i < nblk ? i : nblk - 1);
      Bounds x;
      x.r0 = bstart[b];
      x.rb = bstart[b + 1];
      const auto* segb = seg + b * P.n + c0;
      x.p0 = segb[cs0];
      x.p1 = segb[cs1];
      return x;
    };
    // rowlist is padded past its last group, so r0 + krow stays in range;
    // an entry index is clamped to a valid one (the array has at least two)
    auto load_payload = [&](const Bounds& x) {
      // (the wave-uniform bounds move to scalar registers, so the next
      // bounds can load straight into the vector registers just read)
      Payload y;
      y.rb = __builtin_amdgcn_readfirstlane(x.rb - x.r0);
      y.p0 = __builtin_amdgcn_readfirstlane(x.p0);
      y.p1 = __builtin_amdgcn_readfirstlane(x.p1);
      y.row = rowlist[x.r0 + krow];
      const int32_t last = x.p1 > 0 ? x.p1 - 1 : 0;
#pragma unroll
      for (int q = 0; q < MF_EQ; ++q) {
        const int32_t p = x.p0 + lane + 64 * q;
        y.e[q] = ent(p < last ? p : last);
      }
      return y;
    };
    // an entry holds its row in the block (low 16 bits) and its tile column
    // (high 16 bits); its element index in a copy is column * LDK + row
    auto slot = [](uint32_t ex) {
      return (uint32_t)(((ex >> 16) & (MF_TN - 1)) * LDK + (ex & (MF_MB - 1)));
    };
    auto put = [&](int buf, uint32_t at, float a) {
      if constexpr (FMT == MF_BF16) {
        (&L.A[buf][0][0])[at] = bf16_rne(a);
      } else {
        const uint32_t hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, a, 0, false) & 0xFFu;
        const float back = __builtin_amdgcn_cvt_f32_fp8((int)hi, 0);
        const uint32_t lo =
            (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a - back, a - back, 0, false) & 0xFFu;
        (&L.Ahi[buf][0][0])[at] = (uint8_t)hi;
        (&L.Alo[buf][0][0])[at] = (uint8_t)lo;
      }
    };
    auto zero = [&](int buf, uint32_t at) {
      if constexpr (FMT == MF_BF16) {
        (&L.A[buf][0][0])[at] = 0;
      } else {
        (&L.Ahi[buf][0][0])[at] = 0;
        (&L.Alo[buf][0][0])[at] = 0;
      }
    };
    // 128 signs of block row krow from one generator call; transposing its
    // four words across the half wave leaves lane t with S rows 32 q + t
    // (word q) over the half's 32 block rows
    auto sign_words = [&](const Payload& y) {
      Words w{0u, 0u, 0u, 0u};
      if (krow < y.rb) w = sign_bits128(P.seed, grow0, (uint64_t)(uint32_t)y.row);
      return make_uint4(transpose32(w.x0, lane), transpose32(w.x1, lane),
                        transpose32(w.x2, lane), transpose32(w.x3, lane));
    };
    auto build = [&](int buf, const Payload& y, const uint4 t, Placed& pl) {
      if (signs) {
        const int i = lane & 31;
        L.W[buf][hh][i][wu] = t.x;
        L.W[buf][hh][32 + i][wu] = t.y;
        L.W[buf][hh][64 + i][wu] = t.z;
        L.W[buf][hh][96 + i][wu] = t.w;
      }
      if (ncw <= 0) return;  // past the last column: never stored
      if (pl.count >= 0) {
#pragma unroll
        for (int q = 0; q < MF_EQ; ++q)
          if (lane + 64 * q < pl.count) zero(buf, pl.at[q]);
      } else {
        constexpr int w16 = (FMT == MF_BF16 ? 64 * LDK * 2 : 64 * LDK) / 16;
        if constexpr (FMT == MF_BF16) {
          uint4* z = reinterpret_cast<uint4*>(&L.A[buf][cw0][0]);
          for (int i = lane; i < w16; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
        } else {
          uint4* z = reinterpret_cast<uint4*>(&L.Ahi[buf][cw0][0]);
          uint4* z2 = reinterpret_cast<uint4*>(&L.Alo[buf][cw0][0]);
          for (int i = lane; i < w16; i += 64) {
            z[i] = make_uint4(0u, 0u, 0u, 0u);
            z2[i] = make_uint4(0u, 0u, 0u, 0u);
          }
        }
      }
      // the zeros are written before any store of the block's entries
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int32_t cnt = y.p1 - y.p0;
      pl.count = cnt <= 64 * MF_EQ ? cnt : -1;
#pragma unroll
      for (int q = 0; q < MF_EQ; ++q) {
        pl.at[q] = slot(y.e[q].x);
        if (lane + 64 * q < cnt) put(buf, pl.at[q], __uint_as_float(y.e[q].y));
      }
      for (int32_t p = y.p0 + lane + 64 * MF_EQ; p < y.p1; p += 64) {
        const uint2 e = ent(p);
        put(buf, slot(e.x), __uint_as_float(e.y));
      }
    };

    // Block k (relative to b_lo) is built before barrier k and consumed
    // between barriers k and k + 1; the two roles run separate loops with
    // the same barriers, and a role is the same for a whole wave.  A group
    // makes the sign words of its next block in the window in which it
    // builds nothing, so only the stores and the dense tile remain for the
    // window in which it builds.
    Placed pl{-1, {}};  // copy grp: its last block's entries
    Payload Y{};        // the group's next block
    Bounds Bn{};        // the block after that
    uint4 T{};          // sign words of the group's next block (waves 0, 1)
    if (grp < nblk) {
      Y = load_payload(load_bounds(grp));
      Bn = load_bounds(grp + 2);
      if (grp == 0 && signs) T = sign_words(Y);
    }
    for (int64_t k = 0; k <= nblk; ++k) {
      if ((int)(k & 1) == grp) {
        if (k < nblk) {
          build(grp, Y, T, pl);
          Y = load_payload(Bn);    // block k + 2
          Bn = load_bounds(k + 4);
        }
      } else if (k + 1 < nblk && signs) {
        T = sign_words(Y);         // block k + 1
      }
      __syncthreads();  // block k is built; block k - 1 consumed
    }
    return;
  }

  // acc[TB a + t]: S rows 32 (RA rg + a) + (0..31) x columns 32 (TB cg + t) + (0..31)
  mf_floatx16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
  // a +-1 operand: eight block rows of one S row as BF16 (sign bit 15 of
  // each half) or FP8 (sign bit 7 of each byte) values, from that row's two
  // W words by a shift and a mask
  const int kq = 8 * (lane >> 5);
  const int srow = 32 * RA * rg + (lane & 31);  // + 32 a
  const int ncol = 32 * TB * cg + (lane & 31);  // + 32 t
  uint32_t one8 = 0;
  if constexpr (FMT == MF_FP8)
    one8 = ((uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(1.0f, 1.0f, 0, false) & 0xFFu) * 0x01010101u;
  __syncthreads();  // copy 0 holds block b_lo
  for (int64_t b = b_lo; b < b_hi; ++b) {
    const int buf = (int)((b - b_lo) & 1);
    // the matrix cores on block b: 16 block rows per instruction (rows past
    // the block's end are zero in the dense tile and their S words are
    // zero, so they add nothing); steps 4 u + j take word u of each S row
    // (u unrolled, so the word is picked at compile time)
    uint2 wv[RA];
#pragma unroll
    for (int a = 0; a < RA; ++a)
      wv[a] = *reinterpret_cast<const uint2*>(&L.W[buf][kq >> 3][srow + 32 * a][0]);
    if constexpr (FMT == MF_BF16) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k0 = 16 * (4 * u + j);
          mf_bf16x8 sa[RA], bv[TB];
#pragma unroll
          for (int a = 0; a < RA; ++a) {
            const uint32_t w = u ? wv[a].y : wv[a].x;
            // elements 2h, 2h + 1: 0x3F80 (+1) with sign bits 15 and 31
            auto pair = [&](int h) { return ((w << (h + 4 * j)) & 0x80008000u) | 0x3F803F80u; };
            const uint4 sv = make_uint4(pair(0), pair(1), pair(2), pair(3));
            sa[a] = *reinterpret_cast<const mf_bf16x8*>(&sv);
          }
#pragma unroll
          for (int t = 0; t < TB; ++t)
            bv[t] = *reinterpret_cast<const mf_bf16x8*>(&L.A[buf][ncol + 32 * t][k0 + kq]);
#pragma unroll
          for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int t = 0; t < TB; ++t)
              acc[TB * a + t] =
                  __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa[a], bv[t], acc[TB * a + t], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll 2
        for (int j = 0; j < 4; ++j) {
          const int k0 = 16 * (4 * u + j);
          long sa[RA], bh[TB], bl[TB];
#pragma unroll
          for (int a = 0; a < RA; ++a) {
            const uint32_t w = u ? wv[a].y : wv[a].x;
            // four elements per word: the +1 byte with sign bits 7, 15, 23, 31
            auto quad = [&](int g) { return ((w << (g + 2 * j)) & 0x80808080u) | one8; };
            sa[a] = (long)(((uint64_t)quad(1) << 32) | quad(0));
          }
#pragma unroll
          for (int t = 0; t < TB; ++t) {
            bh[t] = *reinterpret_cast<const long*>(&L.Ahi[buf][ncol + 32 * t][k0 + kq]);
            bl[t] = *reinterpret_cast<const long*>(&L.Alo[buf][ncol + 32 * t][k0 + kq]);
          }
#pragma unroll
          for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int t = 0; t < TB; ++t) {
              acc[TB * a + t] =
                  __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(sa[a], bh[t], acc[TB * a + t], 0, 0, 0);
              acc[TB * a + t] =
                  __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(sa[a], bl[t], acc[TB * a + t], 0, 0, 0);
            }
        }
    }
    __syncthreads();  // block b consumed; the other copy holds block b + 1
  }
  // C[i][j]: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4
  auto* out = in_global(P.out) + (int64_t)split * P.split_stride;
  const float nan = __uint_as_float(0x7FC00000u);
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      const int64_t j = c0 + ncol + 32 * t;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t i = i0 + 32 * RA * rg + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < P.d && j < P.n) out[i + j * P.ld] = status ? nan : acc[TB * a + t][r];
      }
    }
}

template <int FMT>
__global__ __launch_bounds__(MF_THREADS) void k_sketch_mfma(SketchParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int bid = blockIdx.x;
  const int split = bid % P.splits;
  const int rest = bid / P.splits;
  mfma_unit<FMT>(P, split, rest % P.tiles, rest / P.tiles, smem);
}

}  // namespace sk

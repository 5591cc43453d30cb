// sk_sketch.hpp -- the fused sketch kernel A_hat = S A on the blocked layout.
//
// One workgroup owns an output tile A_hat[i0 : i0 + d_b, column range] for a
// range of row blocks (a "split" of the nonempty rows).  Per row block it
//   1. regenerates the S tile S[i0 : i0 + d_b, rows of the block] into LDS,
//      one generator call per (row, 4 S rows), or per (row, 128 S rows) for
//      the +-1 distribution -- every S entry is generated once per tile and
//      reused by every column that has a nonzero in that row (the reuse of
//      Algorithm 4, Sec. II-B; generation count of Sec. III-B),
//   2. stages the block's entries (ordered by column, then row) into LDS,
//   3. accumulates: lanes are grouped Q at a time; a group owns CS columns
//      and, inside the tile, Q*DL consecutive S rows (DL per lane).  For each
//      of its columns it walks the column's entries in row order (the kji
//      order of Algorithm 3 restricted to the block) and does
//      acc[col][r] += a * S_tile[row][r] in FP32 registers.
// Columns are owned by exactly one group, so there are no atomics; every sum
// has a fixed order for a fixed tuning, and splits are combined by a
// fixed-order reduction.  The outer grid is Algorithm 1's blocking over the
// S rows (tiles) plus a split of the inner dimension.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"
#include "sk_rng.hpp"

namespace sk {

struct SketchParams {
  const int32_t* rowlist;
  const int32_t* bstart;  // first nonempty row of each block (nblocks + 1)
  const int32_t* seg;
  const uint2* ent;
  const Header* hdr;
  const int32_t* dflag;  // per block: nonzero when the block runs on the dense path
  const int32_t* bcost;  // exclusive prefix of the block costs (nblocks + 1)
  int64_t n, d, row0;
  uint64_t seed;
  int32_t m_b;      // rows per block at most (S-tile capacity)
  int32_t e_max;    // entries staged per pass (even; LDS holds e_max + 2)
  int32_t d_b;      // S rows per tile = dt * Q * DL (power of two)
  int32_t ldS;      // S tile row stride in floats (d_b plus optional padding,
                    // a multiple of 4 so rows stay 16-byte aligned)
  int32_t log2_cpr; // log2(d_b / rows per generator chunk)
  int32_t dt;       // S-row subtiles per workgroup
  int32_t cg;       // column groups per subtile
  int32_t tiles;    // ceil(d / d_b)
  int32_t splits;   // row-range splits
  int32_t col_per_wg; // columns one workgroup covers (cg * CS)
  int32_t split_slow; // workgroup index -> unit: 0 the split fastest, then
                      // the tile, then the column range; 1 the split slowest
  float* out;       // A_hat (splits == 1) or the split partials
  int64_t ld;       // leading dimension of out
  int64_t split_stride;
  // non-null: n counts virtual columns (all in one column range) and the
  // kernel adds each real column's virtual columns before writing out
  // (nreal columns); null: out holds the n (virtual) columns
  const int32_t* vbase;
  int64_t nreal;
  // GEN_STORED only: S itself, column-major with leading dimension s_ld
  // (S(i, j) at s_pre[i + j * s_ld]; s_ld and the address multiples of 4)
  const float* s_pre;
  int64_t s_ld;
};

// ---------------------------------------------------------------- S tile
// S_lds[l * ldS + t] = S(grow0 + t, rows[l]) for l < rb, t < d_b, by the PT
// threads ptid = 0 .. PT-1, U generator calls in flight per thread.  COUNT:
// add the number of generator calls made to *calls (the call-count check's
// instantiation; the product has no atomics).
template <int DIST, int PT, int U, bool COUNT, int GEN = GEN_PHILOX>
__device__ __forceinline__ void produce_tile(float* __restrict__ S_lds, const SketchParams& P,
                                             const int32_t* __restrict__ rows, int rb,
                                             uint64_t grow0, int ptid,
                                             unsigned long long* calls) {
  uint32_t ncalls = 0;
  const int d_b = P.d_b;
  if (DIST == DIST_RADEMACHER) {
    // one call per (row, 128-row group the tile touches): its four words give
    // 128 consecutive S rows, bit b of word w being row 128 g + 32 w + b.
    // Tile row t of group gi sits at bit position t + off - 128 gi.
    const uint64_t g0 = grow0 >> 7;
    const int off = (int)(grow0 & 127u);
    const int ng = (off + d_b + 127) >> 7;
    const int total = rb * ng;
    for (int idx = ptid; idx < total; idx += PT) {
      const int l = idx / ng;
      const int gi = idx - l * ng;
      const Words x = words_of<GEN>(P.seed, g0 + (uint64_t)gi, (uint64_t)(uint32_t)rows[l]);
      ++ncalls;
      float* row = S_lds + l * P.ldS;
      const int t_lo = 128 * gi - off > 0 ? 128 * gi - off : 0;
      const int t_hi = 128 * (gi + 1) - off < d_b ? 128 * (gi + 1) - off : d_b;
      if (((off | d_b) & 3) == 0) {
        // four rows per store: sign bit into the sign of 1.0f
        for (int t = t_lo; t < t_hi; t += 4) {
          const int bp = t + off - 128 * gi;
          const uint32_t w = word_at(x, bp >> 5) >> (bp & 31);
          float4 v;
          v.x = __uint_as_float(((w << 31) & 0x80000000u) | 0x3F800000u);
          v.y = __uint_as_float(((w << 30) & 0x80000000u) | 0x3F800000u);
          v.z = __uint_as_float(((w << 29) & 0x80000000u) | 0x3F800000u);
          v.w = __uint_as_float(((w << 28) & 0x80000000u) | 0x3F800000u);
          *reinterpret_cast<float4*>(row + t) = v;
        }
      } else {
        for (int t = t_lo; t < t_hi; ++t) {
          const int bp = t + off - 128 * gi;
          const uint32_t w = word_at(x, bp >> 5) >> (bp & 31);
          row[t] = __uint_as_float(((w << 31) & 0x80000000u) | 0x3F800000u);
        }
      }
    }
  } else if ((grow0 & 3u) == 0) {
    // aligned: chunk ch of row l is generator group grow0/4 + ch
    const uint64_t g0 = grow0 >> 2;
    const int lg = P.log2_cpr;
    const int cmask = (1 << lg) - 1;
    const int total = rb << lg;
    for (int base = ptid; base < total; base += U * PT) {
      int32_t jr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * PT;
        jr[u] = idx < total ? rows[idx >> lg] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * PT;
        if (idx < total) {
          float4 v4;
          if (GEN == GEN_STORED) {
            v4 = *reinterpret_cast<const float4*>(P.s_pre + (int64_t)(uint32_t)jr[u] * P.s_ld +
                                                  (int64_t)grow0 + (idx & cmask) * 4);
          } else {
            float v[4];
            quad_values<DIST, GEN>(P.seed, g0 + (uint64_t)(idx & cmask),
                                   (uint64_t)(uint32_t)jr[u], v);
            v4 = make_float4(v[0], v[1], v[2], v[3]);
          }
          ++ncalls;
          *reinterpret_cast<float4*>(S_lds + (idx >> lg) * P.ldS + (idx & cmask) * 4) = v4;
        }
      }
    }
  } else {
    // misaligned tile start: d_b/4 + 1 generator groups per row, each
    // generated once, its rows inside the tile kept
    const int ng = (d_b >> 2) + 1;
    const uint64_t g0 = grow0 >> 2;
    const int shift = (int)(grow0 & 3u);
    const int tot = rb * ng;
    for (int idx = ptid; idx < tot; idx += PT) {
      const int l = idx / ng;
      const int gi = idx - l * ng;
      float v[4];
      if (GEN == GEN_STORED) {
        const float* col = P.s_pre + (int64_t)(uint32_t)rows[l] * P.s_ld;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int64_t i = (int64_t)(g0 + (uint64_t)gi) * 4 + w;
          v[w] = i >= (int64_t)grow0 && i < (int64_t)grow0 + d_b ? col[i] : 0.0f;
        }
      } else {
        quad_values<DIST, GEN>(P.seed, g0 + (uint64_t)gi, (uint64_t)(uint32_t)rows[l], v);
      }
      ++ncalls;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int t = gi * 4 + w - shift;
        if (t >= 0 && t < d_b) S_lds[l * P.ldS + t] = v[w];
      }
    }
  }
  if (COUNT && ncalls) atomicAdd(calls, (unsigned long long)ncalls);
}

// DL consecutive S values of one tile row (rows start 16-byte aligned).
template <int DL>
__device__ __forceinline__ void load_rows(const float* __restrict__ p, float (&s)[DL]) {
  static_assert(DL % 4 == 0 || DL == 1 || DL == 2, "DL");
  if constexpr (DL % 4 == 0) {
#pragma unroll
    for (int t = 0; t < DL; t += 4) {
      const float4 v = *reinterpret_cast<const float4*>(p + t);
      s[t] = v.x; s[t + 1] = v.y; s[t + 2] = v.z; s[t + 3] = v.w;
    }
  } else if constexpr (DL == 2) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    s[0] = v.x; s[1] = v.y;
  } else {
    s[0] = p[0];
  }
}

// Stage entries [s0a, s1) (s0a even) of the blocked layout into E_lds with
// direct global->LDS loads, 16 bytes (two entries) per lane.  Completion is
// tracked by the vector-memory counter; the caller waits and synchronises.
template <int WGS>
__device__ __forceinline__ void stage_entries(uint2* __restrict__ E_lds,
                                              const uint2* __restrict__ ent, int32_t s0a,
                                              int32_t s1) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nchunk = (s1 - s0a + 1) >> 1;  // 16-byte chunks
  for (int c0 = wave * 64; c0 < nchunk; c0 += WGS) {
    if (c0 + lane < nchunk) {
      const uint2* src = ent + s0a + 2 * (c0 + lane);
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1)))*)src,
          (void __attribute__((address_space(3)))*)(E_lds + 2 * c0), 16, 0, 0);
    }
  }
}

// One work unit: S-row tile `tile`, column range `crange`, row-block split
// `split` of one sketch.  Used by the plain grid and by the persistent batched
// kernel.
// FOLD: the columns are virtual (P.vbase) and the unit adds each real
// column's pieces before writing (a separate instantiation, so the plain
// kernels keep their own register allocation)
template <int DIST, int DL, int Q, int CS, int WGS, bool FOLD = false, bool COUNT = false,
          int GEN = GEN_PHILOX>
__device__ __forceinline__ void sketch_unit(const SketchParams& P, int split, int tile, int crange,
                                            unsigned char* __restrict__ smem) {
  // LDS: S tile (m_b x ldS floats) | entries (e_max + 2) | segment bounds of
  // the unit's columns (col_per_wg + 1)
  float* S_lds = reinterpret_cast<float*>(smem);
  uint2* E_lds = reinterpret_cast<uint2*>(smem + (size_t)P.m_b * P.ldS * sizeof(float));
  int32_t* seg_lds = reinterpret_cast<int32_t*>(E_lds + P.e_max + 2);

  const int tid = threadIdx.x;
  const int64_t i_tile = (int64_t)tile * P.d_b;
  const uint64_t grow0 = (uint64_t)(P.row0 + i_tile);

  const int grp = tid / Q;
  const int q = tid - grp * Q;
  const int dsub = grp / P.cg;
  const int cgi = grp - dsub * P.cg;
  const bool active = dsub < P.dt;
  const int rofs = dsub * (Q * DL) + q * DL;
  const int64_t kbase = (int64_t)crange * P.col_per_wg + (int64_t)cgi * CS;
  // entries hold the byte offset of their row in the S tile
  const unsigned char* Sl = smem + rofs * (int)sizeof(float);

  float acc[CS][DL];
#pragma unroll
  for (int c = 0; c < CS; ++c)
#pragma unroll
    for (int t = 0; t < DL; ++t) acc[c][t] = 0.0f;

  const int status = P.hdr->status;
  if (status == 0) {
    const int64_t nb = P.hdr->nblocks;
    // this split's blocks: an equal share of the total estimated cost
    const int64_t T = P.bcost[nb];
    auto first_at = [&](int64_t x) {  // first b in [0, nb] with bcost[b] >= x
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
    // segment bounds of the unit's columns in block b: loaded one block ahead
    // (a few values per thread) so their latency hides behind the previous
    // block's accumulation, then staged in LDS for the column walk
    constexpr int KS = ((WGS / Q) * CS + 1 + WGS - 1) / WGS;
    const int64_t cw0 = (int64_t)crange * P.col_per_wg;
    const int64_t ncw = P.n - cw0 < P.col_per_wg ? P.n - cw0 : P.col_per_wg;
    int32_t sreg[KS];
    int32_t beg_n = 0, end_n = 0, dense_n = 0, r0_n = 0, r1_n = 0;
    auto load_bounds = [&](int64_t b) {
      const int32_t* segb = P.seg + b * P.n;
      beg_n = segb[0];
      end_n = segb[P.n];
      r0_n = P.bstart[b];
      r1_n = P.bstart[b + 1];
      dense_n = P.dflag ? P.dflag[b] : 0;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int64_t i = tid + k * WGS;
        sreg[k] = segb[cw0 + (i < ncw ? i : ncw)];
      }
    };
    const int cl = cgi * CS;  // the group's first column inside the unit
    if (b_lo < b_hi) load_bounds(b_lo);
    for (int64_t b = b_lo; b < b_hi; ++b) {
      if (dense_n) {  // the block runs on the dense (matrix core) path
        if (b + 1 < b_hi) load_bounds(b + 1);
        continue;
      }
      const int32_t row_beg = r0_n;
      const int rb = r1_n - r0_n;
      const int32_t blk_beg = beg_n;
      const int32_t blk_end = end_n;
      // entry positions are kept relative to the first pass's staging start,
      // in bytes (8 per entry) for the column bounds in LDS
      const int32_t base0 = blk_beg & ~1;
      __syncthreads();  // the previous block's tile, entries and bounds are consumed
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int i = tid + k * WGS;
        if (i <= P.col_per_wg) seg_lds[i] = (sreg[k] - base0) * (int32_t)sizeof(uint2);
      }
      // pass: entries [sp, s1) are processed; staging starts at the even s0a
      // (all relative to base0)
      int32_t sp = blk_beg - base0;
      int32_t s0a = 0;
      int32_t s1 = (blk_end - base0 < P.e_max) ? blk_end - base0 : P.e_max;
      stage_entries<WGS>(E_lds, P.ent + base0, s0a, s1);
      // fewer generator calls in flight when the accumulators are many
      produce_tile<DIST, WGS, (DL * CS >= 64 ? 2 : 4), COUNT, GEN>(
          S_lds, P, P.rowlist + row_beg, rb, grow0, tid,
          reinterpret_cast<unsigned long long*>(const_cast<int64_t*>(&P.hdr->reserved[0])));
      bool first_pass = true;
      while (true) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (first_pass && b + 1 < b_hi) load_bounds(b + 1);
        first_pass = false;
        if (active) {
          // the column segments clipped to this pass's entries [sp, s1), as
          // byte offsets; the staged entries start at s0a
          const int32_t sp_b = sp * (int32_t)sizeof(uint2);
          const int32_t s1_b = s1 * (int32_t)sizeof(uint2);
          const unsigned char* const e_base =
              reinterpret_cast<const unsigned char*>(E_lds) - s0a * (int32_t)sizeof(uint2);
#pragma unroll
          for (int c = 0; c < CS; ++c) {
            const int32_t pc0 = seg_lds[cl + c], pc1 = seg_lds[cl + c + 1];
            const int32_t lo = pc0 > sp_b ? pc0 : sp_b;
            const int32_t hi = pc1 < s1_b ? pc1 : s1_b;
            // walk by LDS pointer: one add and one compare per two entries
            const uint2* ep = reinterpret_cast<const uint2*>(e_base + lo);
            const uint2* const ep_last = reinterpret_cast<const uint2*>(e_base + hi) - 1;
            for (; ep < ep_last; ep += 2) {
              const uint2 e0 = ep[0];
              const uint2 e1 = ep[1];
              float x0[DL], x1[DL];
              load_rows<DL>(reinterpret_cast<const float*>(Sl + e0.x), x0);
              load_rows<DL>(reinterpret_cast<const float*>(Sl + e1.x), x1);
              const float a0 = __uint_as_float(e0.y);
              const float a1 = __uint_as_float(e1.y);
#pragma unroll
              for (int t = 0; t < DL; ++t) acc[c][t] = __builtin_fmaf(a0, x0[t], acc[c][t]);
#pragma unroll
              for (int t = 0; t < DL; ++t) acc[c][t] = __builtin_fmaf(a1, x1[t], acc[c][t]);
            }
            if (ep == ep_last) {
              const uint2 e0 = *ep;
              float x0[DL];
              load_rows<DL>(reinterpret_cast<const float*>(Sl + e0.x), x0);
              const float a0 = __uint_as_float(e0.y);
#pragma unroll
              for (int t = 0; t < DL; ++t) acc[c][t] = __builtin_fmaf(a0, x0[t], acc[c][t]);
            }
          }
        }
        if (s1 >= blk_end - base0) break;
        // more entries than one pass holds: stage the next pass
        sp = s1;
        s0a = sp & ~1;
        s1 = (blk_end - base0 - s0a < P.e_max) ? blk_end - base0 : s0a + P.e_max;
        __syncthreads();
        stage_entries<WGS>(E_lds, P.ent + base0, s0a, s1);
      }
    }
  }
  float* __restrict__ out = P.out + (int64_t)split * P.split_stride;
  const float nan = __uint_as_float(0x7FC00000u);
  if constexpr (!FOLD) {
    if (active) {
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        const int64_t k = kbase + c;
        if (k < P.n && k < (int64_t)(crange + 1) * P.col_per_wg) {
#pragma unroll
          for (int t = 0; t < DL; ++t) {
            const int64_t i = i_tile + rofs + t;
            // (the scaled mode's S is 2^24 S: one exact rescaling here)
            const float v = GEN == GEN_SCALED ? acc[c][t] * 0x1.0p-24f : acc[c][t];
            if (i < P.d) out[i + k * P.ld] = status ? nan : v;
          }
        }
      }
    }
  } else {
  if (!P.vbase) return;  // (the host launches this form only with virtual columns)
  // Heavy columns split into virtual columns, all in this workgroup's one
  // column range: add each real column's virtual columns (in order) through
  // LDS, one of every lane's DL rows at a time, and write the real columns.
  float* __restrict__ V = reinterpret_cast<float*>(smem);  // row slots x col_per_wg
  const int slots = P.dt * Q;
  const int cpw = P.col_per_wg;
  const int slot = dsub * Q + q;  // rofs = slot * DL
#pragma unroll
  for (int t = 0; t < DL; ++t) {
    __syncthreads();  // the tiles (or the previous row) are no longer read
    if (active) {
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        const int lc = cgi * CS + c;
        if (lc < cpw) V[slot * cpw + lc] = acc[c][t];
      }
    }
    __syncthreads();
    for (int64_t x = tid; x < (int64_t)slots * P.nreal; x += WGS) {
      const int64_t k = x / slots;
      const int r = (int)(x - k * slots);
      const int64_t i = i_tile + (int64_t)r * DL + t;
      if (i >= P.d) continue;
      const int32_t v0 = P.vbase[k], v1 = P.vbase[k + 1];
      float sum = 0.0f;
      for (int32_t v = v0; v < v1; ++v) sum += V[r * cpw + v];
      out[i + k * P.ld] = status ? nan : sum;
    }
  }
  }
}

template <int DIST, int DL, int Q, int CS, int WGS, bool FOLD = false, bool COUNT = false,
          int GEN = GEN_PHILOX>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(4))) void k_sketch(
    SketchParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  // Units in one of two orders.  With the split slowest, each split's units
  // run together, spread over the whole chip, so a split whose blocks cost
  // more than their estimate (uneven blocks) slows one stretch of the launch
  // on every CU instead of a few CUs at its end (skewed workload, 4 splits:
  // 3.45 ms per step against 4.34 with the split fastest).  With balanced
  // row blocks the estimates hold, and the split fastest is faster (plain
  // workload, 6 splits: kernel 14.38 ms against 14.80: with the split
  // slowest every CU reads the same split's blocks at once).
  int split;
  int64_t rest;
  if (P.split_slow) {
    const int64_t units = (int64_t)P.tiles * ((P.n + P.col_per_wg - 1) / P.col_per_wg);
    split = (int)(blockIdx.x / units);
    rest = blockIdx.x - (int64_t)split * units;
  } else {
    split = (int)(blockIdx.x % P.splits);
    rest = blockIdx.x / P.splits;
  }
  sketch_unit<DIST, DL, Q, CS, WGS, FOLD, COUNT, GEN>(P, split, (int)(rest % P.tiles),
                                                      (int)(rest / P.tiles), smem);
}

// Generator throughput (the measured cost h of the ablation): each thread
// makes `calls` generator calls for distinct counters (group c, column =
// global thread index) and folds every output into one word, written once,
// so that nothing is stored but nothing can be skipped either.
template <int DIST, int GEN>
__global__ __launch_bounds__(256) void k_rng_throughput(int64_t calls, uint64_t seed,
                                                        uint32_t* __restrict__ sink) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int64_t c = 0; c < calls; ++c) {
    if (DIST == DIST_RADEMACHER) {
      const Words x = words_of<GEN>(seed, (uint64_t)c, j);
      acc ^= x.x0 ^ x.x1 ^ x.x2 ^ x.x3;
    } else {
      float v[4];
      quad_values<DIST, GEN>(seed, (uint64_t)c, j, v);
      acc ^= __float_as_uint(v[0]) ^ __float_as_uint(v[1]) ^ __float_as_uint(v[2]) ^
             __float_as_uint(v[3]);
    }
  }
  sink[j] = acc;
}

// A_hat[i, k] = sum over sparse slices of the virtual columns of k, then the
// dense slice (if any); fixed order.  vbase == nullptr: virtual == real.
__global__ void k_reduce_virtual(const float* __restrict__ part, int splits, int64_t d, int64_t n,
                                 int64_t nv, const int32_t* __restrict__ vbase,
                                 const float* __restrict__ dense_slice, float* __restrict__ out,
                                 int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d * n) return;
  const int64_t k = t / d, i = t - k * d;
  float s = 0.0f;
  // the slice column(s) of real column k
  const int64_t col = vbase ? vbase[k] : k;
  const int64_t ncol = vbase ? vbase[k + 1] - col : 1;
  if (ncol == 1) {
    // one value per split: eight loads in flight, added in split order
    const float* __restrict__ p = part + i + col * d;
    const int64_t stride = d * nv;
    int q = 0;
    for (; q + 8 <= splits; q += 8) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = q + u == 0 ? x[u] : s + x[u];
    }
    for (; q < splits; ++q) {
      const float x = p[(int64_t)q * stride];
      s = q == 0 ? x : s + x;
    }
  } else {
    const int64_t v0 = col, v1 = col + ncol;
    bool first = true;
    for (int q = 0; q < splits; ++q) {
      const float* sl = part + (int64_t)q * d * nv;
      for (int64_t v = v0; v < v1; ++v) {
        const float x = sl[i + v * d];
        s = first ? x : s + x;
        first = false;
      }
    }
  }
  if (dense_slice) s += dense_slice[i + k * d];
  out[i + k * ld] = s;
}


// S[r + c*ld] = S(row0 + r, col0 + c): one thread per (generator group,
// column); rows outside [row0, row0 + d) are skipped.
template <int DIST>
__global__ void k_materialize(int64_t row0, int64_t d, int64_t col0, int64_t ncols,
                              uint64_t seed, float* __restrict__ S, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int rpg = DIST == DIST_RADEMACHER ? 32 : 4;  // rows per thread
  const int64_t gfirst = row0 / rpg;
  const int64_t groups = (row0 + d - 1) / rpg - gfirst + 1;
  if (t >= groups * ncols) return;
  const int64_t c = t / groups, gi = t - c * groups;
  const uint64_t j = (uint64_t)(col0 + c);
  const int64_t gr = (gfirst + gi) * rpg;  // first global row of the group
  float* col = S + c * ld;
  if (DIST == DIST_RADEMACHER) {
    const uint32_t bits = sign_bits32(seed, (uint64_t)gr, j);
    for (int u = 0; u < 32; ++u) {
      const int64_t r = gr + u - row0;
      if (r >= 0 && r < d) col[r] = (bits >> u) & 1u ? -1.0f : 1.0f;
    }
  } else {
    float v[4];
    quad_values<DIST>(seed, (uint64_t)(gr >> 2), j, v);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = gr + u - row0;
      if (r >= 0 && r < d) col[r] = v[u];
    }
  }
}

}  // namespace sk

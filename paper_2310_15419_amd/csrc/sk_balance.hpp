// sk_balance.hpp -- balanced row blocks for the S-tile kernel.
//
// The S-tile kernel walks, for every row block, each column's entries in that
// block with one group of lanes per column, and the groups of a wave run in
// lockstep: a wave takes as long as its column with the most entries in the
// block.  With rows cut into blocks in row order, the count of column k in a
// block is close to Poisson, and the lockstep costs about twice the useful
// multiply-adds when a block holds a few entries per column (the plain-scale
// workload: 3.7 on average, lockstep padding 2.19).
//
// Any assignment of rows to blocks gives the same A_hat up to rounding (S is a
// function of the row index, not of the block), so the rows can be grouped to
// even out the counts.  Positions (the nonempty rows in row order) are cut
// into super-blocks of sb consecutive blocks of m_b rows; inside a
// super-block, rows are dealt to its sb blocks greedily in position order,
// each to the block where the sum over its columns of the squared current
// counts is least (a block that is full takes no more).  Rows are decided in
// batches of up to 128 against the counts before the batch; a batch keeps its
// rows up to the first one whose block would overflow, and the next batch
// starts there, so no block overflows.  Inside a block the rows keep their
// order.  A super-block that
// is not full, or that holds a row with more than BAL_ROW_MAX entries (dense
// rows belong together, for the dense path), keeps its order.
//
// The blocked layout is then built by the usual inspector from A' = A with
// rows renumbered by their new positions (rows sorted inside each column,
// values in FP32), and the row list maps the new positions back to the rows
// of A, whose indices are the generator's counters.  On the plain-scale
// workload this takes the padding from 2.19 to about 1.5.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"

namespace sk {

constexpr int BAL_SB_MAX = 16;        // blocks per super-block
constexpr int BAL_THREADS = 1024;     // the assignment's workgroup
constexpr int BAL_BATCH = 128;        // rows decided together (eight lanes each)
constexpr int BAL_CHUNK = 8192;       // column ids staged in LDS at once (a multiple of BAL_THREADS)
constexpr int BAL_CHUNK_ROWS = 2048;  // rows staged at once
constexpr int BAL_ROW_MAX = 64;       // longer rows keep their super-block in order
constexpr int BAL_SBM_MAX = 16384;    // positions per super-block
static_assert(BAL_CHUNK % BAL_THREADS == 0, "column-id staging: whole rounds of the workgroup");
constexpr int BAL_N_MAX = 2048;       // columns (the count table: sb x n 16-bit counters)

struct BalParams {
  const Header* hdr;
  int64_t m, n, nnz, r_max;
  const int64_t* colptr;
  const int32_t* rowidx;
  const void* vals;
  int32_t vtype;
  int32_t m_b, sb, sbm;     // rows per block, blocks per super-block, sb * m_b
  const int32_t* ridx;      // position of each nonempty row of A
  const int32_t* rowlist;   // the nonempty rows of A in order
  const int32_t* rowcnt;    // their entry counts
  int32_t* rowoff;          // r_max + 1: exclusive prefix of rowcnt (scanned)
  uint16_t* ccol;           // nnz: the column ids of each row, rows in position order
  int32_t* newidx;          // m: new position of each nonempty row
  int32_t* orig;            // r_max: the row of A at each new position
  int32_t* cnt2;            // r_max: the entry count at each new position
  int32_t* rowidx2;         // nnz: A' row indices (new positions)
  float* vals2;             // nnz: A' values
};

__device__ __forceinline__ int bal_status(const BalParams& B) {
  return in_global(const_cast<Header*>(B.hdr))->status;
}

// rowoff[p] = entries of position p (scanned afterwards)
__global__ void k_bal_prep(BalParams B) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.r_max) return;
  const int64_t R = bal_status(B) ? 0 : in_global(const_cast<Header*>(B.hdr))->nonempty;
  B.rowoff[p] = p < R ? B.rowcnt[p] : 0;
}

// Per-slab partial row counts (several column slabs) to exclusive prefixes
// over the slabs, in place: where slab j's columns of a row start inside the
// row's column list.  (The partials are consumed by then.)
__global__ void k_bal_slab_prefix(BalParams B, int32_t* __restrict__ rpart) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B.m || bal_status(B)) return;
  const int64_t slabs = rt_slabs(B.n);
  const int64_t tile = r / RT_ROWS, j = r - tile * RT_ROWS;
  int32_t* p = rpart + tile * slabs * RT_ROWS + j;
  int32_t run = 0;
  for (int64_t s = 0; s < slabs; ++s) {
    const int32_t c = p[s * RT_ROWS];
    p[s * RT_ROWS] = run;
    run += c;
  }
}

// The column ids of every row (a transpose of the pattern), by the walk of
// the row-count pass: one workgroup per (tile of RT_ROWS rows, slab of
// RT_COLS columns); an entry's slot among its row's entries of the slab is
// the value an LDS counter had before the entry's increment, added to the
// row's base (its list's start plus the slab's offset in it), staged in LDS
// for the tile.  The order inside a row does not matter (only sums over it
// are taken).  A row's list is written by every slab's workgroup, two bytes
// at a time; the workgroups are dealt to the chip's eight L2 slices (XCDs)
// round-robin by their index, so the slabs of a tile get indices equal
// modulo 8 (runs of 8 tiles, the tile fastest): a list's cache lines are
// then completed in one L2 rather than written in pieces from eight.
__global__ __launch_bounds__(1024) void k_bal_csr(BalParams B, const int32_t* __restrict__ rpart) {
  __shared__ int32_t cnt[RT_ROWS];
  __shared__ int32_t base_l[RT_ROWS];
  if (bal_status(B)) return;
  const int64_t slabs = rt_slabs(B.n);
  const int64_t tiles = (B.m + RT_ROWS - 1) / RT_ROWS;
  const int64_t x = blockIdx.x;
  const int64_t run = x / (8 * slabs), within = x - run * 8 * slabs;
  const int64_t nt = tiles - run * 8 < 8 ? tiles - run * 8 : 8;  // tiles of this run
  if (within >= nt * slabs) return;  // (no such pair: x is past the last one)
  const int64_t tile = run * 8 + within % nt, slab = within / nt;
  const int64_t w = tile * slabs + slab;  // the pair's index in the row-count pass
  const int64_t r0 = tile * RT_ROWS;
  if (r0 >= B.m) return;
  const int64_t r1 = r0 + RT_ROWS < B.m ? r0 + RT_ROWS : B.m;
  const auto* rowidx = in_global(B.rowidx);
  {
    const auto* ridx = in_global(B.ridx);
    const auto* rowoff = in_global(B.rowoff);
    const int32_t* sofs = slabs > 1 ? rpart + w * RT_ROWS : nullptr;
    // (a row without entries reads the next position's offset: in range, unused)
    for (int j = threadIdx.x; j < RT_ROWS; j += blockDim.x) {
      cnt[j] = 0;
      base_l[j] = r0 + j < r1 ? rowoff[ridx[r0 + j]] + (sofs ? in_global(sofs)[j] : 0) : 0;
    }
  }
  __syncthreads();
  const int64_t k = slab * RT_COLS + (threadIdx.x >> 2);
  if (k >= B.n) return;
  const int64_t c0 = in_global(B.colptr)[k], c1 = in_global(B.colptr)[k + 1];
  int64_t lo = c0, hi = c1;  // first entry with row >= r0
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rowidx[mid] < r0) lo = mid + 1;
    else hi = mid;
  }
  // entries p, p + 4, ... eight per round (independent loads), up to the
  // first row past the tile
  for (int64_t p = lo + (threadIdx.x & 3); p < c1; p += 32) {
    int32_t r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = p + 4 * u < c1 ? rowidx[p + 4 * u] : (int32_t)r1;
    bool past = false;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (r[u] >= r1) {
        past = true;
      } else {
        const int32_t slot = atomicAdd(&cnt[r[u] - r0], 1);
        B.ccol[base_l[r[u] - r0] + slot] = (uint16_t)k;
      }
    }
    if (past) break;
  }
}

// The count table: row j (j = 0..7) holds, for every column c, the counters
// of blocks j and j + 8 in the low and high halves of word c, so a lane's two
// candidate blocks are one read; rows of an odd number of words, so that the
// eight lanes of a row (rows 0..7), reading one column together, fall in
// different LDS banks.  (A counter stays below 2^14 = BAL_SBM_MAX.)
__host__ __device__ inline int64_t bal_pair_words(int64_t n) { return n | 1; }

// min of (cost << 4 | block) over the 8 lanes of a segment (ties: the lower
// block); DPP inside the 16-lane rows, called with all lanes active
__device__ __forceinline__ uint32_t seg8_min(uint32_t key) {
  // (the 8-lane halves of a row: quad swaps, then the half-row mirrored)
  uint32_t o;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  key = o < key ? o : key;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  key = o < key ? o : key;
  o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x141, 0xF, 0xF, false);  // row_half_mirror
  key = o < key ? o : key;
  return key;
}


// One workgroup per super-block: the greedy assignment, then the new
// positions (block b of the super-block takes positions s0 + b m_b + slot,
// slots in position order).  LDS: the count table (16-bit counters, blocks j
// and j + 8 in one word), the staged column ids and row offsets, the block
// of each position.
__global__ __launch_bounds__(BAL_THREADS) void k_bal_assign(BalParams B) {
  extern __shared__ __align__(16) uint32_t bal_lds[];
  __shared__ int32_t fill[BAL_SB_MAX];
  __shared__ uint8_t pick_l[BAL_BATCH];
  __shared__ int32_t wtot[BAL_THREADS / 64][BAL_SB_MAX];
  __shared__ int32_t wsum[BAL_SB_MAX];
  __shared__ int32_t flag;
  __shared__ int32_t chunk_end;
  if (bal_status(B)) return;
  const int64_t R = in_global(const_cast<Header*>(B.hdr))->nonempty;
  const int64_t s0 = (int64_t)blockIdx.x * B.sbm;
  if (s0 >= R) return;
  const int tid = threadIdx.x;
  const int sbm = B.sbm, sb = B.sb, m_b = B.m_b;
  const int64_t nh = bal_pair_words(B.n);
  uint32_t* cntw = bal_lds;                                    // 8 * nh
  uint16_t* col_l = reinterpret_cast<uint16_t*>(cntw + 8 * nh);  // BAL_CHUNK
  int32_t* off_l = reinterpret_cast<int32_t*>(col_l + BAL_CHUNK);  // BAL_CHUNK_ROWS + 1
  uint8_t* blk_l = reinterpret_cast<uint8_t*>(off_l + BAL_CHUNK_ROWS + 1);  // sbm
  const auto* rowlist = in_global(B.rowlist);
  const auto* rowcnt = in_global(B.rowcnt);
  const auto* rowoff = in_global(B.rowoff);
  int32_t* cnt2 = B.cnt2;
  const int64_t rows = R - s0 < sbm ? R - s0 : sbm;
  // the super-block's rows in order (new position = old position)
  auto keep_order = [&]() {
    for (int64_t q = tid; q < rows; q += BAL_THREADS) {
      const int32_t r = rowlist[s0 + q];
      const int32_t c = rowcnt[s0 + q];
      B.newidx[r] = (int32_t)(s0 + q);
      B.orig[s0 + q] = r;
      cnt2[s0 + q] = c;
    }
  };

  if (tid == 0) flag = rows < sbm ? 1 : 0;
  __syncthreads();
  for (int64_t q = tid; q < rows && !flag; q += BAL_THREADS)
    if (rowcnt[s0 + q] > BAL_ROW_MAX) flag = 1;  // (benign race: any writer sets 1)
  __syncthreads();
  if (flag) {
    keep_order();
    return;
  }
  for (int64_t j = tid; j < 8 * nh; j += BAL_THREADS) cntw[j] = 0;
  if (tid < BAL_SB_MAX) fill[tid] = 0;
  __syncthreads();

  const int i = tid >> 3;    // row of the batch
  const int l = tid & 7;     // lane of the row: candidate blocks l and l + 8
  const int b0 = l, b1 = l + 8;
  const int lane = tid & 63;
  const uint64_t le = ~uint64_t(0) >> (63 - lane);  // lanes 0..lane
  int64_t p = s0;
  while (p < s0 + sbm) {
    // stage rows [p, pc): at most BAL_CHUNK_ROWS rows and BAL_CHUNK column ids
    // (the offsets first, then the last row end within BAL_CHUNK; a row has
    // at most BAL_ROW_MAX entries, so one row always fits)
    const int64_t pmax = p + BAL_CHUNK_ROWS < s0 + sbm ? p + BAL_CHUNK_ROWS : s0 + sbm;
    // (each thread's loads issued together, then stored)
    const int32_t o_p = rowoff[p];
    if (tid == 0) chunk_end = 1;
    {
      constexpr int K = (BAL_CHUNK_ROWS + BAL_THREADS) / BAL_THREADS;  // covers BAL_CHUNK_ROWS + 1
      int32_t x[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int64_t j = tid + k * BAL_THREADS;
        x[k] = j <= pmax - p ? rowoff[p + j] : 0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int64_t j = tid + k * BAL_THREADS;
        if (j <= pmax - p) off_l[j] = x[k] - o_p;
      }
    }
    __syncthreads();
    for (int64_t j = tid + 1; j <= pmax - p; j += BAL_THREADS)
      if (off_l[j] <= BAL_CHUNK) atomicMax(&chunk_end, (int)j);
    __syncthreads();
    const int64_t pc = p + chunk_end;
    const int32_t ncol = off_l[chunk_end];
    {
      constexpr int K = BAL_CHUNK / BAL_THREADS;
      uint16_t x[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = tid + k * BAL_THREADS;
        x[k] = j < ncol ? B.ccol[o_p + j] : (uint16_t)0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = tid + k * BAL_THREADS;
        if (j < ncol) col_l[j] = x[k];
      }
    }
    __syncthreads();
    int64_t q = p;
    while (q < pc) {
      // every row of the batch picks, against the counts before the batch,
      // its cheapest block among those with room; the batch keeps its rows
      // up to the first one whose block would take more rows than its room
      // (that row and the later ones start the next batch; the first row
      // always fits, so every batch decides at least one row)
      const int nb = pc - q < BAL_BATCH ? (int)(pc - q) : BAL_BATCH;
      // room of blocks b0 and b1 (every segment of 8 lanes holds the same),
      // and the least room of a block that has room (in vector registers:
      // every wave needs it)
      const int f0 = b0 < sb ? m_b - fill[b0] : 0;
      const int f1 = b1 < sb ? m_b - fill[b1] : 0;
      const uint32_t r0 = f0 > 0 ? (uint32_t)f0 : 0xFFFFFFFFu;
      const uint32_t r1 = f1 > 0 ? (uint32_t)f1 : 0xFFFFFFFFu;
      const uint32_t least = (uint32_t)__builtin_amdgcn_readfirstlane((int)seg8_min(r0 < r1 ? r0 : r1));
      uint32_t key = ~uint32_t(0);
      int32_t o0 = 0, o1 = 0;
      if (i < nb) {
        o0 = off_l[q - p + i];
        o1 = off_l[q - p + i + 1];
        const bool ok0 = f0 > 0, ok1 = f1 > 0;
        // (saturating sums: a tie among huge costs is harmless)
        uint32_t cost0 = 0, cost1 = 0;
        const uint32_t* row = cntw + b0 * nh;  // blocks b0 (low half) and b1 (high)
#pragma unroll 4
        for (int32_t e = o0; e < o1; ++e) {
          const uint32_t w = row[col_l[e]];
          const uint32_t x0 = w & 0xFFFFu, x1 = w >> 16;
          cost0 = __builtin_elementwise_add_sat(cost0, x0 * x0);
          cost1 = __builtin_elementwise_add_sat(cost1, x1 * x1);
        }
        const uint32_t k0 = ok0 ? ((cost0 < 0x07FFFFFFu ? cost0 : 0x07FFFFFFu) << 4) | (uint32_t)b0
                                : ~uint32_t(0);
        const uint32_t k1 = ok1 ? ((cost1 < 0x07FFFFFFu ? cost1 : 0x07FFFFFFu) << 4) | (uint32_t)b1
                                : ~uint32_t(0);
        key = k0 < k1 ? k0 : k1;
      }
      key = seg8_min(key);
      const int pick = (int)(key & 0xF);
      if (i < nb && l == 0) pick_l[i] = (uint8_t)pick;
      __syncthreads();  // every cost read the counts and rooms before this batch; the picks are in
      int acc = nb;
      if ((uint32_t)nb > least) {
        // the accepted prefix: lane L looks at batch rows L and 64 + L
        const int p_lo = lane < nb ? pick_l[lane] : 0xFF;
        const int p_hi = 64 + lane < nb ? pick_l[64 + lane] : 0xFF;
        bool bad_lo = false, bad_hi = false;
#pragma unroll
        for (int bb = 0; bb < BAL_SB_MAX; ++bb) {
          const int rb = __builtin_amdgcn_readlane(bb < 8 ? f0 : f1, bb & 7);  // room of block bb
          const uint64_t m_lo = __ballot(p_lo == bb), m_hi = __ballot(p_hi == bb);
          bad_lo |= p_lo == bb && __popcll(m_lo & le) > rb;
          bad_hi |= p_hi == bb && __popcll(m_lo) + __popcll(m_hi & le) > rb;
        }
        const uint64_t x_lo = __ballot(bad_lo), x_hi = __ballot(bad_hi);
        // (at least one row, so that the loop ends whatever the rooms: a row
        // that found no room overfills a block, and the check after the
        // loop then keeps the super-block in order)
        acc = x_lo ? __builtin_ctzll(x_lo) : (x_hi ? 64 + __builtin_ctzll(x_hi) : nb);
        acc = acc > 0 ? acc : 1;
      }
      if (i < acc && pick < sb) {
        for (int32_t e = o0 + l; e < o1; e += 8) {
          const int c = col_l[e];
          atomicAdd(&cntw[(pick & 7) * nh + c], pick >= 8 ? 0x10000u : 1u);
        }
        if (l == 0) {
          blk_l[q - s0 + i] = (uint8_t)pick;
          atomicAdd(&fill[pick], 1);
        }
      }
      __syncthreads();
      q += acc;
    }
    p = pc;
  }
  // (every block holds exactly m_b rows; should that ever fail, the
  // super-block keeps its order, so the renumbering stays a permutation)
  if (tid == 0) {
    int bad = 0;
    for (int bb = 0; bb < BAL_SB_MAX; ++bb) bad |= fill[bb] != (bb < sb ? m_b : 0);
    flag = bad;
  }
  __syncthreads();
  if (flag) {
    keep_order();
    return;
  }
  // slots: rank of each position among the super-block's positions of its
  // block, in position order
  const int wave = tid >> 6;
  int32_t base[BAL_SB_MAX];
#pragma unroll
  for (int bb = 0; bb < BAL_SB_MAX; ++bb) base[bb] = 0;
  for (int64_t c0 = 0; c0 < sbm; c0 += BAL_THREADS) {
    const int64_t q = c0 + tid;
    const int my = q < sbm ? blk_l[q] : -1;
    const uint64_t lt = (lane ? ~uint64_t(0) >> (64 - lane) : uint64_t(0));
    int rank = 0;
#pragma unroll
    for (int bb = 0; bb < BAL_SB_MAX; ++bb) {
      const uint64_t mk = __ballot(my == bb);
      if (my == bb) rank = __popcll(mk & lt);
      if (lane == 0) wtot[wave][bb] = __popcll(mk);
    }
    __syncthreads();
    if (tid < BAL_SB_MAX) {  // per block: exclusive prefix over the waves, total last
      int t = 0;
      for (int w = 0; w < BAL_THREADS / 64; ++w) {
        const int x = wtot[w][tid];
        wtot[w][tid] = t;
        t += x;
      }
      wsum[tid] = t;
    }
    __syncthreads();
    if (my >= 0) {
      int32_t bs = 0;
#pragma unroll
      for (int bb = 0; bb < BAL_SB_MAX; ++bb)
        if (bb == my) bs = base[bb];
      const int slot = bs + wtot[wave][my] + rank;
      if (my < sb && slot < m_b) {  // (always: no block takes more than m_b rows)
        const int64_t np = s0 + (int64_t)my * m_b + slot;
        const int32_t r = rowlist[s0 + q];
        const int32_t c = rowcnt[s0 + q];
        B.newidx[r] = (int32_t)np;
        B.orig[np] = r;
        cnt2[np] = c;
      }
    }
#pragma unroll
    for (int bb = 0; bb < BAL_SB_MAX; ++bb) base[bb] += wsum[bb];
    __syncthreads();
  }
}

__host__ __device__ inline size_t bal_assign_lds(int64_t n, int sb, int sbm) {
  const size_t words = (size_t)8 * bal_pair_words(n);
  return words * 4 + BAL_CHUNK * 2 + (BAL_CHUNK_ROWS + 1) * 4 + (size_t)sbm;
}

// A' = A with rows renumbered: one wave per (column, BAL_BUILD_G consecutive
// super-blocks).  The column's entries in a super-block's rows are one run,
// and their new positions stay inside the super-block's range, so A' keeps
// A's column pointers; a run is reordered by a stable partition on the new
// block, which sorts it by new position (a block keeps its rows in order).
// The first run's start is searched; each run's end is found by its walk
// (the first row at or past the next super-block's first row), and is the
// next run's start.  A run that fits one chunk of 64 is placed from the
// registers of its walk.
constexpr int BAL_BUILD_G = 8;
__global__ __launch_bounds__(256) void k_bal_build(BalParams B) {
  if (bal_status(B)) return;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t R = in_global(const_cast<Header*>(B.hdr))->nonempty;
  const int64_t nsb = (R + B.sbm - 1) / B.sbm;
  const int64_t ngrp = (nsb + BAL_BUILD_G - 1) / BAL_BUILD_G;
  const int64_t sg = g / B.n, k = g - sg * B.n;
  if (sg >= ngrp) return;  // wave-uniform
  const auto* rowlist = in_global(B.rowlist);
  const auto* rowidx = in_global(B.rowidx);
  const auto* newidx = in_global(B.newidx);
  const int64_t c0 = in_global(B.colptr)[k], c1 = in_global(B.colptr)[k + 1];
  const uint64_t lt = lane ? ~uint64_t(0) >> (64 - lane) : uint64_t(0);
  auto value = [&](int64_t e) {
    if (B.vtype == 0) return (float)in_global(static_cast<const double*>(B.vals))[e];
    if (B.vtype == 1) return in_global(static_cast<const float*>(B.vals))[e];
    return __uint_as_float((uint32_t)in_global(static_cast<const uint16_t*>(B.vals))[e] << 16);
  };
  // first entry of the column with row >= r: an 8-way search (each step
  // probes 8 evenly spaced entries, lanes 0..7: few cache lines per step;
  // the answer stays in [lo, hi]), then one window of 64
  auto first_at = [&](int64_t r) {
    int64_t lo = c0, hi = c1;
    while (hi - lo > 64) {
      const int64_t step = (hi - lo + 7) >> 3;
      const int64_t q = lo + (int64_t)(lane + 1) * step - 1;
      const int below = __popcll(__ballot(lane < 8 && q < hi && rowidx[q < hi ? q : lo] < r));
      const int64_t nhi = lo + (int64_t)(below + 1) * step - 1;
      lo += (int64_t)below * step;
      if (nhi < hi) hi = nhi;
    }
    const int64_t q = lo + lane;
    return lo + __popcll(__ballot(q < hi && rowidx[q < hi ? q : lo] < r));
  };
  // new block of new position np inside the super-block at base: (np - base)
  // / m_b from a float reciprocal, corrected by one step (the quotient's
  // operands are below 2^14 = BAL_SBM_MAX, exact in FP32)
  const float inv_mb = 1.0f / (float)B.m_b;
  int64_t base = 0;
  auto blk_of = [&](int32_t np) {
    const int x = (int)(np - base);
    int q = (int)((float)x * inv_mb);
    if (q * B.m_b > x) --q;
    else if ((q + 1) * B.m_b <= x) ++q;
    return q;
  };
  const int64_t s_end = (sg + 1) * BAL_BUILD_G < nsb ? (sg + 1) * BAL_BUILD_G : nsb;
  int64_t lo = first_at(rowlist[sg * BAL_BUILD_G * B.sbm]);
  for (int64_t s = sg * BAL_BUILD_G; s < s_end; ++s) {
    base = s * B.sbm;
    const int64_t rhi = base + B.sbm < R ? (int64_t)rowlist[base + B.sbm] : B.m;
    // walk: entries per new block, and the run's end
    int32_t off[BAL_SB_MAX];
#pragma unroll
    for (int bb = 0; bb < BAL_SB_MAX; ++bb) off[bb] = 0;
    int32_t np0 = 0;
    int my0 = -1;
    float v0 = 0.0f;
    int64_t hi = lo;
    for (int64_t e0 = lo;; e0 += 64) {
      const int64_t e = e0 + lane;
      const int32_t r = e < c1 ? rowidx[e] : INT32_MAX;
      const bool in = r < rhi;  // (rows are sorted: a prefix of the lanes)
      const int cnt = __popcll(__ballot(in));
      const int32_t np = in ? newidx[r] : 0;
      const int my = in ? blk_of(np) : -1;
#pragma unroll
      for (int bb = 0; bb < BAL_SB_MAX; ++bb) off[bb] += __popcll(__ballot(my == bb));
      if (e0 == lo) {
        np0 = np;
        my0 = my;
        v0 = in ? value(e) : 0.0f;
      }
      if (cnt < 64) {
        hi = e0 + cnt;
        break;
      }
    }
    int32_t acc = 0;
#pragma unroll
    for (int bb = 0; bb < BAL_SB_MAX; ++bb) {
      const int32_t t = off[bb];
      off[bb] = acc;
      acc += t;
    }
    // place, stable within a block
    for (int64_t e0 = lo; e0 < hi; e0 += 64) {
      const int64_t e = e0 + lane;
      int32_t np;
      int my;
      float v;
      if (e0 == lo) {
        np = np0; my = my0; v = v0;
      } else {
        const bool in = e < hi;
        const int32_t r = in ? rowidx[e] : 0;
        np = in ? newidx[r] : 0;
        my = in ? blk_of(np) : -1;
        v = in ? value(e) : 0.0f;
      }
      int64_t dst = 0;
#pragma unroll
      for (int bb = 0; bb < BAL_SB_MAX; ++bb) {
        const uint64_t mk = __ballot(my == bb);
        if (my == bb) dst = lo + off[bb] + __popcll(mk & lt);
        off[bb] += __popcll(mk);
      }
      if (my >= 0) {
        B.rowidx2[dst] = np;
        B.vals2[dst] = v;
      }
    }
    lo = hi;
  }
}

// The nonempty-row arrays of A' without counting: its rows 0..R-1 are the
// new positions, all nonempty (entry counts from the assignment, in cnt2),
// the rows from R on are empty.  (rowlist is the identity here: the block
// positions of the inspector compare A' rows; k_bal_remap maps it back.)
__global__ void k_bal_rows2(BalParams B, int32_t* __restrict__ ridx, int32_t* __restrict__ rcnt,
                            int32_t* __restrict__ rowlist, int32_t* __restrict__ rowcnt) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > B.m || bal_status(B)) return;
  const int64_t R = in_global(const_cast<Header*>(B.hdr))->nonempty;
  ridx[r] = (int32_t)(r < R ? r : R);
  if (r == B.m) return;
  const int32_t c = r < R ? B.cnt2[r] : 0;
  rcnt[r] = c;
  if (r < R) {
    rowlist[r] = (int32_t)r;
    rowcnt[r] = c;
  }
}

// the row list of A' (positions 0..R-1 in order) back to the rows of A
__global__ void k_bal_remap(const Header* __restrict__ hdr, const int32_t* __restrict__ orig,
                            int64_t r_max, int32_t* __restrict__ rowlist) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= r_max || hdr->status) return;
  if (c < hdr->nonempty) rowlist[c] = orig[c];
}

}  // namespace sk

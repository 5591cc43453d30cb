// sk_inspect.hpp -- device kernels of the inspector: validation of the CSC
// input, compaction of the nonempty rows of A, and the blocked layout of A
// that the sketch kernels consume.
//
// The paper's Algorithm 4 needs a blocked representation built from the CSC
// input (Sec. III-B: the conversion costs O(ceil(n/b_n) m + nnz) and is cheap
// next to the multiplication, Table IV).  Here the blocks run the other way:
// a row block is a run of consecutive *nonempty* rows of A (empty rows need
// no S column at all, Sec. III-B), and inside a block the entries are ordered
// by column, then row, so one S tile of the block's rows is reused by every
// column that has nonzeros there.
//
// Blocks are balanced by entries: the nonempty rows are cut into groups of
// m_b (the S-tile capacity), and each group is cut further, greedily in row
// order, so that no block holds more than e_cap entries (the LDS staging
// capacity) unless one row alone does.  Rows of very different weight (a few
// dense rows among many light ones) then never make a block that needs many
// staging passes.
//
// Every kernel here runs over a flattened index space that concatenates the
// items of a batch (a single sketch is a batch of one): a workgroup finds
// the items of its first and last index by a search over the items' prefix
// offsets (all its threads share one item in the usual case; else each
// thread searches).  Per-item exclusive
// scans are one scan over the concatenated regions, followed by subtraction
// of each item's value at its region start.
//
// Layout produced per item (all int32; nnz, m and the block grid fit int32):
//   ridx[r]            position of row r among the nonempty rows; ridx[m] = R
//   rowlist[c], rowcnt[c]  the c-th nonempty row and its entry count
//   bfl[c]             number of block starts among rows < c (so row c is in
//                      block bfl[c + 1] - 1); bfl[R] = number of blocks
//   bstart[b]          first nonempty row of block b; bstart[nblocks] = R
//   vbase[k]           first virtual column of column k (heavy-column
//                      splitting; absent when off)
//   pos[b*nv + v]      first position of (virtual) column v whose row is >=
//                      the first row of block b (b = 0..nb_max)
//   seg[b*nv + v]      start of block b / column v's segment in `ent`;
//                      block b spans [seg[b*nv], seg[(b+1)*nv])
//   ent[p]             {byte offset of the entry's row in the S tile (row
//                      inside the block times the tile's row bytes), FP32
//                      bits of the value}
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace sk {

// Accesses through a generic pointer are flat instructions, which count as
// LDS traffic in the wait counters too (an LDS wait then also waits for every
// load in flight).  Pointers read from memory (item descriptors, the batched
// kernels' parameters) are generic, so the hot loops address their arrays as
// global memory explicitly.
template <typename T>
using global_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ global_t<T>* in_global(T* p) {
  return (global_t<T>*)p;
}
// (HIP's vector types cannot be read or written through such pointers; pairs
// go through 64-bit words, quadruples through a native vector type)
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int2 load_pair(const int2* p, int64_t i) {
  const uint64_t x = in_global(reinterpret_cast<const uint64_t*>(p))[i];
  return make_int2((int32_t)(uint32_t)x, (int32_t)(uint32_t)(x >> 32));
}
__device__ __forceinline__ void store_pair(uint2* p, int64_t i, uint32_t lo, uint32_t hi) {
  in_global(reinterpret_cast<uint64_t*>(p))[i] = (uint64_t)lo | ((uint64_t)hi << 32);
}

// status bits written by the validation kernel
enum : int { ST_RANGE = 1, ST_UNSORTED = 2, ST_COLPTR = 4, ST_CAPACITY = 8 };

struct Header {       // one per item, in the workspace
  int32_t status;     // OR of ST_* bits
  int32_t pad;
  int64_t nonempty;   // R
  int64_t nblocks;
  int64_t reserved[5];
};

struct Item {
  // input (device memory)
  int64_t m, n, nnz;
  const int64_t* colptr;
  const int32_t* rowidx;
  const void* vals;
  int32_t vtype;
  // plan
  int32_t m_b;        // rows per row group (S-tile capacity)
  int32_t e_cap;      // entries per block (staging capacity)
  int32_t row_bytes;  // S-tile row stride in bytes
  int32_t bp_chunk;   // blocks per thread of the block-position search
  int32_t col_tag;    // 0 or a power of two: an entry's row offset also carries
                      // (column mod col_tag) << 16 (the matrix-core kernel's tile
                      // column)
  int64_t nv;         // (virtual) columns of the layout
  int64_t nb_max;     // block capacity
  int64_t r_max;      // nonempty-row capacity, min(m, max(nnz, 1))
  // workspace (device memory)
  Header* hdr;
  int32_t* ridx;      // m + 1, region of a concatenated array
  int32_t* rcnt;      // m
  int32_t* rpart;     // partial row counts per (row tile, column slab): tiles *
                      // slabs * RT_ROWS (nullptr when the item has one slab)
  int32_t* rowlist;   // r_max + m_b + 1 (padded for whole-group reads)
  int32_t* rowcnt;    // r_max
  int32_t* bfl;       // r_max + 1, region of a concatenated array
  int32_t* bstart;    // nb_max + 1
  int32_t* vbase;     // n + 1, region of a concatenated array; nullptr: no splitting
  int32_t* pos;       // (nb_max + 1) * nv: first position of each (block,
                      // column) inside the column's entries
  int32_t* seg;       // nb_max * nv + 1, region of a concatenated array
  uint2* ent;         // nnz + 2
  int2* rowinfo;      // m: {block, row offset in the S tile in bytes} of row r
  int32_t* bcost;     // nb_max + 1, region of a concatenated array: block costs,
                      // then their exclusive prefix (splits cut it evenly)
  const int32_t* dflag;  // per block: nonzero on the dense path (may be null)
  // block cost model: (rows w_row + entries w_ent + w_blk) >> cost_shift
  int32_t w_row, w_ent, w_blk, cost_shift;
  // value of each concatenated scan at this item's region start
  int32_t base_ridx, base_bfl, base_vbase, base_seg, base_cost;
  // exclusive prefix offsets of this item in each flattened index space
  int64_t o_valid;    // max(nnz, n + 1)
  int64_t o_ridx;     // m + 1
  int64_t o_m;        // m
  int64_t o_grp;      // row groups, ceil(r_max / m_b)
  int64_t o_bfl;      // r_max + 1
  int64_t o_rmax;     // r_max
  int64_t o_col;      // n
  int64_t o_vb;       // n + 1
  int64_t o_pos;      // ceil((nb_max + 1) / bp_chunk) * nv
  int64_t o_cnt;      // nb_max * nv
  int64_t o_seg;      // nb_max * nv + 1
  int64_t o_nnz;      // nnz
  int64_t o_blk;      // nb_max + 1
  int64_t o_rt;       // (row tile, column slab) pairs of the counting pass
};

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ float load_value(const void* vals, int vtype, int64_t p) {
  if (vtype == 0) return (float)in_global((const double*)vals)[p];  // RNE
  if (vtype == 1) return in_global((const float*)vals)[p];
  const uint16_t h = in_global((const uint16_t*)vals)[p];          // bf16 -> fp32 exact
  return __uint_as_float((uint32_t)h << 16);
}

// ------------------------------------------------------------- scan (int32)
// In-place exclusive scan of a[0..count) in chunks of SCAN_CHUNK; the grand
// total goes to a[count].  Three passes: the chunk sums (a read), their scan
// (one workgroup), and the chunk-local scans from those offsets (a read and a
// write).  Block scans are wave scans by lane shuffles plus one exchange of
// the wave totals through LDS.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// exclusive scan of one value per thread over the workgroup; the total to
// every thread.  sh: SCAN_THREADS / 64 ints, free again on return.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t& total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int32_t inc = wave_inclusive_scan(v);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int32_t before = 0;
  total = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / 64; ++i) {
    const int32_t t = sh[i];
    before += i < w ? t : 0;
    total += t;
  }
  __syncthreads();
  return before + inc - v;
}

// a thread's SCAN_ITEMS consecutive values (zero past count); VEC: a is
// 16-byte aligned, so a whole run is two 16-byte loads
template <bool VEC>
__device__ __forceinline__ void scan_load(const int32_t* __restrict__ a, int64_t base,
                                          int64_t count, int32_t (&v)[SCAN_ITEMS]) {
  if (VEC && base + SCAN_ITEMS <= count) {
    const int4 x = *reinterpret_cast<const int4*>(a + base);
    const int4 y = *reinterpret_cast<const int4*>(a + base + 4);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) v[i] = base + i < count ? a[base + i] : 0;
  }
}

template <bool VEC>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int32_t* __restrict__ a,
                                                              int64_t count,
                                                              int32_t* __restrict__ sums) {
  __shared__ int32_t sh[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  scan_load<VEC>(a, base, count, v);
  int32_t run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) run += v[i];
  int32_t total;
  block_exclusive_scan(run, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// chunk-local exclusive scans, offset by the scanned chunk sums
template <bool VEC>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(int32_t* __restrict__ a,
                                                             int64_t count,
                                                             const int32_t* __restrict__ sums) {
  __shared__ int32_t sh[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  scan_load<VEC>(a, base, count, v);
  int32_t run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) run += v[i];
  int32_t total;
  int32_t off = block_exclusive_scan(run, sh, total) + sums[blockIdx.x];
  int32_t o[SCAN_ITEMS];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    o[i] = off;
    off += v[i];
  }
  if (VEC && base + SCAN_ITEMS <= count) {
    *reinterpret_cast<int4*>(a + base) = make_int4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<int4*>(a + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
      if (base + i < count) a[base + i] = o[i];
  }
}

// one workgroup: exclusive scan of sums[0..nchunks), total -> *grand
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(int32_t* __restrict__ sums,
                                                            int64_t nchunks,
                                                            int32_t* __restrict__ grand) {
  __shared__ int32_t sh[SCAN_THREADS / 64];
  int32_t carry = 0;
  for (int64_t base = 0; base < nchunks; base += SCAN_CHUNK) {
    const int64_t b0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      v[i] = (b0 + i) < nchunks ? sums[b0 + i] : 0;
      run += v[i];
    }
    int32_t total;
    int32_t off = block_exclusive_scan(run, sh, total) + carry;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      if ((b0 + i) < nchunks) sums[b0 + i] = off;
      off += v[i];
    }
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}



// item owning flattened index t of the space whose offsets are field F
template <int64_t Item::*F>
__device__ __forceinline__ int find_item(const Item* __restrict__ it, int count, int64_t t) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].*F <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The largest q in [lo, hi] with key(q) <= x (lo when there is none), found
// by the 32 lanes of a half wave together: each step loads 32 evenly spaced
// keys at once and keeps the stretch between the last one at or below x and
// the next, so a search over n keys takes about log32(n) load round trips.
// The keys ascend (where they do not, as in malformed input, the result is
// still some q in [lo, hi]).  Every lane of the half wave passes the same
// arguments.
template <class Key>
__device__ __forceinline__ int64_t halfwave_last_le(int64_t lo, int64_t hi, int64_t x, Key key) {
  const int l = threadIdx.x & 31;
  const int half = threadIdx.x & 32;  // this half's bits in a ballot
  while (hi > lo) {
    const int64_t step = (hi - lo + 32) / 32;  // ceil of (hi - lo + 1) / 32
    const int64_t q = lo + l * step;
    const bool le = q <= hi && (l == 0 || key(q) <= x);  // (lane 0: lo, kept)
    const uint32_t m = (uint32_t)(__ballot(le) >> half);
    const int c = m == 0xFFFFFFFFu ? 32 : __builtin_ctz(~m);  // probes before the first above x
    const int64_t nlo = lo + (int64_t)(c - 1) * step;
    const int64_t nhi = lo + (int64_t)c * step - 1;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

// The items of a workgroup's first and last indices (s_item[0], s_item[1]);
// when they are the same (the usual case) the item is uniform, so its
// descriptor is read with scalar loads rather than once per lane.
template <int64_t Item::*F>
__device__ __forceinline__ void workgroup_items(const Item* __restrict__ it, int count,
                                                int64_t total, int64_t g0, int64_t span,
                                                int* s_item) {
  const int64_t glast = (g0 + span < total ? g0 + span : total) - 1;
  if (threadIdx.x < 64) {  // half wave h finds the item of index h ? glast : g0
    const int h = threadIdx.x >> 5;
    const int i = (int)halfwave_last_le(0, count - 1, h ? glast : g0,
                                        [&](int64_t q) { return it[q].*F; });
    if ((threadIdx.x & 31) == 0) s_item[h] = i;
  }
  __syncthreads();
}

// Indices per thread of k_items in a batch: 8 (strided by the workgroup
// size, so the accesses stay coalesced), which spreads a workgroup's item
// lookup over 2048 of them; an op whose per-index work is long sets
// kPerThread.  A single item has no lookup and takes one per thread.
constexpr int KI_THREADS = 256;
template <class Op, class = void>
struct per_thread {
  static constexpr int value = 8;
};
template <class Op>
struct per_thread<Op, std::void_t<decltype(Op::kPerThread)>> {
  static constexpr int value = Op::kPerThread;
};

// Op::run(item, index inside the item) for every flattened index, PER per
// thread.
template <int64_t Item::*F, class Op, int PER>
__global__ __launch_bounds__(KI_THREADS) void k_items(const Item* __restrict__ it, int count,
                                                      int64_t total) {
  const int64_t g0 = (int64_t)blockIdx.x * (KI_THREADS * PER);
  if (count == 1) {
    const Item I = it[0];  // a copy: the op's stores cannot change it
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int64_t g = g0 + threadIdx.x + j * KI_THREADS;
      if (g < total) Op::run(I, g);
    }
    return;
  }
  __shared__ int s_item[2];
  workgroup_items<F>(it, count, total, g0, KI_THREADS * PER, s_item);
  if (s_item[0] == s_item[1]) {
    const Item I = it[__builtin_amdgcn_readfirstlane(s_item[0])];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int64_t g = g0 + threadIdx.x + j * KI_THREADS;
      if (g < total) Op::run(I, g - I.*F);
    }
  } else {
    for (int j = 0; j < PER; ++j) {
      const int64_t g = g0 + threadIdx.x + j * KI_THREADS;
      if (g >= total) break;
      const int i = find_item<F>(it, count, g);
      Op::run(it[i], g - it[i].*F);
    }
  }
}

// An entry-indexed space (field F holds each item's offset), IC_PER indices
// per thread (strided by the workgroup size, so loads stay coalesced);
// Op::run also gets the column of the entry, found by a search limited to the
// columns of the workgroup's first and last entries (a few columns,
// typically) instead of one over all of colptr.  The workgroup's searches
// for those bounds (on 32 lanes each) are the latency every index waits on,
// so they cover 1024 of them.
constexpr int IC_THREADS = 256;
constexpr int IC_PER = 4;

// An op with run_many takes a thread's IC_PER indices at once (all loads
// before any store, so their memory latencies overlap).
template <class Op, class = void>
struct takes_many : std::false_type {};
template <class Op>
struct takes_many<Op, std::void_t<decltype(&Op::template run_many<IC_PER>)>> : std::true_type {};

template <int64_t Item::*F, class Op>
__global__ __launch_bounds__(IC_THREADS) void k_items_cols(const Item* __restrict__ it, int count,
                                                           int64_t total) {
  __shared__ int s_item[2];
  __shared__ int64_t s_col[2];
  const int64_t g0 = (int64_t)blockIdx.x * (IC_THREADS * IC_PER);
  const int64_t span = IC_THREADS * IC_PER;
  const int64_t glast = (g0 + span < total ? g0 + span : total) - 1;
  if (threadIdx.x < 64) {  // half wave h: the item and column of index h ? glast : g0
    const int h = threadIdx.x >> 5;
    const int64_t gg = h ? glast : g0;
    const int i = count == 1 ? 0
                             : (int)halfwave_last_le(0, count - 1, gg,
                                                     [&](int64_t q) { return it[q].*F; });
    const Item& I = it[i];
    int64_t t = gg - I.*F;
    if (t >= I.nnz) t = I.nnz - 1;
    const auto* colptr = in_global(I.colptr);
    const int64_t col =
        t >= 0 ? halfwave_last_le(0, I.n - 1, t, [&](int64_t q) { return colptr[q]; }) : 0;
    if ((threadIdx.x & 31) == 0) {
      s_item[h] = i;
      s_col[h] = col;
    }
  }
  __syncthreads();
  // the column of entry t, searched between the given bounds
  auto column = [](const Item& I, int64_t t, int64_t lo, int64_t hi) {
    int64_t k = 0;
    if (t < I.nnz) {
      const auto* colptr = in_global(I.colptr);
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (colptr[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
      k = lo;
    }
    return k;
  };
  if (s_item[0] == s_item[1]) {  // one item: uniform descriptor, narrow search
    // (a copy, in scalar registers: the op's stores cannot change it)
    const Item I = it[__builtin_amdgcn_readfirstlane(s_item[0])];
    if constexpr (takes_many<Op>::value) {
      // indices past the end stand in as the workgroup's last one (same
      // item), so every load is valid; their results are not stored
      int64_t t[IC_PER], k[IC_PER];
      bool ok[IC_PER];
#pragma unroll
      for (int j = 0; j < IC_PER; ++j) {
        const int64_t g = g0 + threadIdx.x + j * IC_THREADS;
        ok[j] = g < total;
        t[j] = (ok[j] ? g : glast) - I.*F;
        k[j] = column(I, t[j], s_col[0], s_col[1]);
      }
      Op::template run_many<IC_PER>(I, t, k, ok);
    } else {
#pragma unroll
      for (int j = 0; j < IC_PER; ++j) {
        const int64_t g = g0 + threadIdx.x + j * IC_THREADS;
        if (g >= total) break;
        const int64_t t = g - I.*F;
        Op::run(I, t, column(I, t, s_col[0], s_col[1]));
      }
    }
  } else {
    for (int j = 0; j < IC_PER; ++j) {
      const int64_t g = g0 + threadIdx.x + j * IC_THREADS;
      if (g >= total) break;
      const Item& I = it[find_item<F>(it, count, g)];
      const int64_t t = g - I.*F;
      Op::run(I, t, column(I, t, 0, I.n - 1));
    }
  }
}

// Validate, mark occupied rows and count entries per row.  One thread per
// nonzero (and per colptr entry); k is the column of nonzero t.
struct OpValidate {
  static __device__ void run(const Item& I, int64_t t, int64_t k) {
    int bad = 0;
    const auto* colptr = in_global(I.colptr);
    const auto* rowidx = in_global(I.rowidx);
    if (t <= I.n) {
      const int64_t c = colptr[t];
      if (t == 0 && c != 0) bad |= ST_COLPTR;
      if (t == I.n && c != I.nnz) bad |= ST_COLPTR;
      if (t < I.n && colptr[t + 1] < c) bad |= ST_COLPTR;
      if (c < 0 || c > I.nnz) bad |= ST_COLPTR;
    }
    if (t < I.nnz) {
      const int32_t r = rowidx[t];
      if (r < 0 || r >= I.m) bad |= ST_RANGE;
      if (t > 0 && colptr[k] < t && rowidx[t - 1] >= r) bad |= ST_UNSORTED;
    }
    if (bad) atomicOr(&I.hdr->status, bad);
  }
  // the same for N indices: every load first (indices clamped into range,
  // results of the clamped ones unused), then the checks, one status update
  template <int N>
  static __device__ void run_many(const Item& I, const int64_t (&t)[N], const int64_t (&k)[N],
                                  const bool (&ok)[N]) {
    const auto* colptr = in_global(I.colptr);
    const auto* rowidx = in_global(I.rowidx);
    int64_t c[N], c1[N], ck[N];
    int32_t r[N], rp[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int64_t tc = t[j] < I.n ? t[j] : I.n;
      c[j] = colptr[tc];
      c1[j] = colptr[tc < I.n ? tc + 1 : I.n];
      ck[j] = colptr[k[j]];
      r[j] = rp[j] = 0;
      if (I.nnz > 0) {
        const int64_t te = t[j] < I.nnz ? t[j] : I.nnz - 1;
        r[j] = rowidx[te];
        rp[j] = rowidx[te > 0 ? te - 1 : 0];
      }
    }
    int bad = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (!ok[j]) continue;
      if (t[j] <= I.n) {
        if (t[j] == 0 && c[j] != 0) bad |= ST_COLPTR;
        if (t[j] == I.n && c[j] != I.nnz) bad |= ST_COLPTR;
        if (t[j] < I.n && c1[j] < c[j]) bad |= ST_COLPTR;
        if (c[j] < 0 || c[j] > I.nnz) bad |= ST_COLPTR;
      }
      if (t[j] < I.nnz) {
        if (r[j] < 0 || r[j] >= I.m) bad |= ST_RANGE;
        if (t[j] > 0 && ck[j] < t[j] && rp[j] >= r[j]) bad |= ST_UNSORTED;
      }
    }
    if (bad) atomicOr(&I.hdr->status, bad);
  }
};

// Entries per row without global atomics: one workgroup per (tile of
// RT_ROWS rows, slab of RT_COLS columns) of one item.  Rows are sorted
// inside each column, so the entries of a column that fall in the tile are
// one run, found by a binary search; four lanes walk it (every fourth entry)
// and count the rows with LDS atomics.  Column slabs spread a tile whose rows
// are dense (many columns share them) over several workgroups; with more
// than one slab the counts go to per-slab partials, summed by OpRowReduce.
// (On malformed input the counts are meaningless, and the validation status
// stops everything after.)
constexpr int RT_ROWS = 8192;
constexpr int RT_COLS = 256;

__host__ __device__ inline int64_t rt_slabs(int64_t n) {
  return n > RT_COLS ? (n + RT_COLS - 1) / RT_COLS : 1;
}

__global__ __launch_bounds__(1024) void k_row_counts(const Item* __restrict__ it, int count,
                                                      int64_t total) {
  __shared__ int32_t cnt[RT_ROWS];
  const int64_t g = blockIdx.x;
  if (g >= total) return;
  const int i = count == 1 ? 0 : find_item<&Item::o_rt>(it, count, g);
  const Item& I = it[i];
  const int64_t slabs = rt_slabs(I.n);
  const int64_t w = g - I.o_rt;
  const int64_t tile = w / slabs, slab = w - tile * slabs;
  const int64_t r0 = tile * RT_ROWS;
  const int64_t r1 = r0 + RT_ROWS < I.m ? r0 + RT_ROWS : I.m;
  for (int j = threadIdx.x; j < RT_ROWS; j += blockDim.x) cnt[j] = 0;
  __syncthreads();
  const int64_t k = slab * RT_COLS + (threadIdx.x >> 2);
  const auto* rowidx = in_global(I.rowidx);
  const int64_t c0 = k < I.n ? in_global(I.colptr)[k] : 0;
  const int64_t c1 = k < I.n ? in_global(I.colptr)[k + 1] : 0;
  if (k < I.n && c0 >= 0 && c1 <= I.nnz && c1 >= c0) {  // (malformed: flagged by the validation)
    int64_t lo = c0, hi = c1;  // first entry with row >= r0
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (rowidx[mid] < r0) lo = mid + 1;
      else hi = mid;
    }
    // entries p, p + 4, ... below `end`, eight per load round (independent
    // loads, so their latencies overlap), up to the first row past the tile
    auto run = [&](int64_t p, int64_t end) {
      for (; p < end; p += 32) {
        int32_t r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = p + 4 * u < end ? rowidx[p + 4 * u] : (int32_t)r1;
        bool past = false;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (r[u] >= r1 || r[u] < r0) past = true;  // (below r0 only on malformed input)
          else atomicAdd(&cnt[r[u] - r0], 1);
        }
        if (past) break;
      }
    };
    // the lanes of a wave start at staggered points of their runs (then wrap
    // round to the head), so where columns share rows they add to
    // different counters at a time
    const int64_t s0 = lo + (threadIdx.x & 3);
    const int64_t st = s0 + 4 * ((threadIdx.x >> 2) & 7);
    const int64_t mid = st < c1 ? st : c1;
    run(mid, c1);
    run(s0, mid);
  }
  __syncthreads();
  if (slabs == 1) {
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const int32_t c = cnt[r - r0];
      I.rcnt[r] = c;
      I.ridx[r] = c > 0 ? 1 : 0;
    }
  } else {
    int32_t* __restrict__ out = I.rpart + w * RT_ROWS;
    for (int64_t j = threadIdx.x; j < r1 - r0; j += blockDim.x) out[j] = cnt[j];
  }
}

// rows of an item with several column slabs: counts and occupancy flags
// from the slabs' partial counts (in a fixed order)
struct OpRowReduce {
  static __device__ void run(const Item& I, int64_t r) {
    if (!I.rpart) return;
    const int64_t slabs = rt_slabs(I.n);
    const int64_t tile = r / RT_ROWS, j = r - tile * RT_ROWS;
    const int32_t* __restrict__ p = I.rpart + tile * slabs * RT_ROWS + j;
    int32_t c = 0;
    for (int64_t s = 0; s < slabs; ++s) c += p[s * RT_ROWS];
    I.rcnt[r] = c;
    I.ridx[r] = c > 0 ? 1 : 0;
  }
};

// region bases after a concatenated scan
enum : int { SCAN_RIDX = 0, SCAN_BFL = 1, SCAN_VBASE = 2, SCAN_SEG = 3, SCAN_COST = 4 };

__global__ void k_item_bases(Item* __restrict__ it, int count, int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  Item& I = it[i];
  if (which == SCAN_RIDX) I.base_ridx = I.ridx[0];
  else if (which == SCAN_BFL) I.base_bfl = I.bfl[0];
  else if (which == SCAN_VBASE) I.base_vbase = I.vbase ? I.vbase[0] : 0;
  else if (which == SCAN_SEG) I.base_seg = I.seg[0];
  else I.base_cost = I.bcost[0];
}

template <int WHICH>
struct OpRebase {
  static __device__ void run(const Item& I, int64_t t) {
    if (WHICH == SCAN_RIDX) I.ridx[t] -= I.base_ridx;
    else if (WHICH == SCAN_BFL) I.bfl[t] -= I.base_bfl;
    else if (WHICH == SCAN_VBASE) { if (I.vbase) I.vbase[t] -= I.base_vbase; }
    else if (WHICH == SCAN_SEG) I.seg[t] -= I.base_seg;
    else I.bcost[t] -= I.base_cost;
  }
};

// nonempty-row list with entry counts; R to the header
struct OpRowlist {
  static __device__ void run(const Item& I, int64_t r) {
    const int32_t c = I.ridx[r];
    if (I.ridx[r + 1] > c) {
      I.rowlist[c] = (int32_t)r;
      I.rowcnt[c] = I.rcnt[r];
    }
    if (r == 0) I.hdr->nonempty = I.ridx[I.m];
  }
};

// Block starts inside row group g (rows [g m_b, min(R, (g+1) m_b))): greedy
// in row order, a new block starts at the first row that would take the open
// block past e_cap entries; a row that alone exceeds e_cap is a block of its
// own.  One wave per group, 64 rows per step: a wave-wide prefix sum of the
// row counts, then one ballot per block start found in the step.
__global__ __launch_bounds__(256) void k_partition(const Item* __restrict__ it, int count,
                                                   int64_t total_groups) {
  const int64_t g_all = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (g_all >= total_groups) return;  // wave-uniform
  const int i = count == 1 ? 0 : find_item<&Item::o_grp>(it, count, g_all);
  const Item& I = it[i];
  if (I.hdr->status) return;
  const int64_t R = I.hdr->nonempty;
  const int64_t c0 = (g_all - I.o_grp) * I.m_b;
  if (c0 >= R) return;
  const int64_t c1 = c0 + I.m_b < R ? c0 + I.m_b : R;
  const int32_t E = I.e_cap;
  if (lane == 0) I.bfl[c0] = 1;
  int32_t cur = 0;  // entries of the open block
  for (int64_t cb = c0; cb < c1; cb += 64) {
    const int nvalid = (int)(c1 - cb < 64 ? c1 - cb : 64);
    const int32_t x = lane < nvalid ? I.rowcnt[cb + lane] : 0;
    int32_t pre = x;  // inclusive prefix over the lanes
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(pre, off, 64);
      if (lane >= off) pre += y;
    }
    int base = 0;       // first lane not yet placed in a closed block
    int32_t pbase = 0;  // prefix before lane `base`
    while (true) {
      const bool over = lane >= base && lane < nvalid && cur + (pre - pbase) > E;
      const uint64_t mask = __ballot(over);
      if (mask == 0) {
        cur += __shfl(pre, nvalid - 1, 64) - pbase;
        break;
      }
      const int f = __ffsll((unsigned long long)mask) - 1;
      const int32_t pre_f = __shfl(pre, f, 64);
      const int32_t x_f = __shfl(x, f, 64);
      if (f == base && cur == 0) {
        // row f alone exceeds the cap: it closes its own block
        if (lane == 0 && cb + f + 1 < c1) I.bfl[cb + f + 1] = 1;
        base = f + 1;
        pbase = pre_f;
      } else {
        if (lane == 0) I.bfl[cb + f] = 1;
        base = f;
        pbase = pre_f - x_f;
      }
      cur = 0;
    }
  }
}

// block start rows from the scanned flags; block count to the header
struct OpBstart {
  static __device__ void run(const Item& I, int64_t c) {
    if (I.hdr->status) return;
    const int64_t R = I.hdr->nonempty;
    if (c < R) {
      const int32_t b = I.bfl[c];
      if (I.bfl[c + 1] != b && b < I.nb_max) I.bstart[b] = (int32_t)c;
    }
    if (c == 0) {
      const int64_t nb = I.bfl[R];
      if (nb > I.nb_max) atomicOr(&I.hdr->status, ST_CAPACITY);
      const int64_t nbc = nb < I.nb_max ? nb : I.nb_max;
      I.hdr->nblocks = nbc;
      I.bstart[nbc] = (int32_t)R;
    }
  }
};

// ---------------------------------------------------- heavy-column splitting
// A column with many more entries than average would make its owning lane
// the straggler of every block.  Column k is split into s_k interleaved
// virtual columns (entry t of the column goes to virtual column
// vbase[k] + t mod s_k, position t / s_k), s_k = ceil(cnt_k / L) with
// L = ceil(nnz / (nv - n)): the virtual column count stays within the
// planned capacity nv.  The sketch runs on virtual columns; the final
// reduction adds them back up.

// vbase[k] = s_k (scanned afterwards)
struct OpColsplit {
  static __device__ void run(const Item& I, int64_t k) {
    if (!I.vbase) return;
    int64_t s = 1;
    const int64_t spare = I.nv - I.n;
    if (!I.hdr->status && spare > 0 && I.nnz > 0) {
      const int64_t L = (I.nnz + spare - 1) / spare;
      const int64_t c = I.colptr[k + 1] - I.colptr[k];
      s = c > L ? (c + L - 1) / L : 1;
    }
    I.vbase[k] = (int32_t)s;
  }
};

// real column of virtual column v (v < vbase[n])
__device__ __forceinline__ int64_t real_column(const int32_t* __restrict__ vbase, int64_t n,
                                               int64_t v) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (vbase[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// pos[b*nv + v], b = 0..nb_max, in units of the (virtual) column's own
// positions: how many of its entries lie above block b (all of them for
// b >= nblocks).  One thread per (virtual column, run of bp_chunk blocks);
// every step loads its values together, so a thread waits on few memory
// round trips:
//   - the first rows of the run's blocks,
//   - the first block's position by an 8-way search (8 probes per step, the
//     range shrinking 9-fold) until the range fits one window,
//   - each block's position by counting, in a window of 16 consecutive
//     entries, those above its first row; the window moves down the column
//     while a block's first row lies below all of it.
constexpr int BP_MAX_CHUNK = 16;  // bp_chunk at most
constexpr int BP_P = 8;          // probes per search step
constexpr int BP_W = 16;         // entries per window
struct OpBlockPos {
  static constexpr int kPerThread = 1;
  static __device__ void run(const Item& I, int64_t t) {
    if (in_global(I.hdr)->status) return;
    const auto* vbase = in_global(I.vbase);
    const auto* colptr = in_global(I.colptr);
    const auto* rowlist = in_global(I.rowlist);
    const auto* bstart = in_global(I.bstart);
    auto* pos = in_global(I.pos);
    const int64_t bc = t / I.nv, v = t - bc * I.nv;
    const int chunk = I.bp_chunk;
    const int64_t b0 = bc * chunk;
    int64_t k = v, s = 1, r = 0;
    if (vbase) {
      if (v >= vbase[I.n]) {
        for (int j = 0; j < chunk && b0 + j <= I.nb_max; ++j) pos[(b0 + j) * I.nv + v] = 0;
        return;
      }
      k = real_column(I.vbase, I.n, v);
      s = vbase[k + 1] - vbase[k];
      r = v - vbase[k];
    }
    const int64_t c0 = colptr[k], cnt = colptr[k + 1] - c0;
    const int64_t T = cnt > r ? (cnt - r + s - 1) / s : 0;  // entries of v
    const auto* rows = in_global(I.rowidx) + c0 + r;        // entry j of v: rows[j * s]
    const int64_t nbk = in_global(I.hdr)->nblocks;
    const int64_t jn64 = I.nb_max + 1 - b0;
    const int jn = jn64 < chunk ? (int)jn64 : chunk;  // blocks of the run with a pos row
    // first row of each block (past the last block: above every row)
    int32_t fr[BP_MAX_CHUNK];
#pragma unroll
    for (int j = 0; j < BP_MAX_CHUNK; ++j) {
      const int64_t b = b0 + j;
      fr[j] = (j < jn && b < nbk) ? rowlist[bstart[b]] : INT32_MAX;
    }
    // the first entry at or below fr[0] lies in [lo, hi]
    int64_t lo = 0, hi = T;
    while (hi - lo > BP_W) {
      // probes lo + step, ..., lo + 8 step, all below hi
      const int64_t step = (hi - lo) / (BP_P + 1);
      int32_t x[BP_P];
#pragma unroll
      for (int i = 0; i < BP_P; ++i) x[i] = rows[(lo + (i + 1) * step) * s];
      int c = 0;  // probes above fr[0] (a prefix: the rows ascend)
#pragma unroll
      for (int i = 0; i < BP_P; ++i) c += x[i] < fr[0] ? 1 : 0;
      const int64_t nlo = c > 0 ? lo + c * step + 1 : lo;
      const int64_t nhi = c < BP_P ? lo + (c + 1) * step : hi;
      lo = nlo;
      hi = nhi;
    }
    // Windows start at entry wl <= lo (every entry before lo lies above
    // fr[0] <= fr[j]); a slot before the column's first entry counts as
    // above every block, one past its last as below all.  Where v is a real
    // column and the row indices are 16-byte aligned, wl is rounded down to
    // an aligned index, so that a window inside the column is four 16-byte
    // loads.
    const bool wide = s == 1 && (reinterpret_cast<uintptr_t>(I.rowidx) & 15u) == 0;
    int64_t wl = wide ? lo - ((c0 + lo) & 3) : lo;
    int32_t w[BP_W];
    auto load_window = [&]() {
      if (wide && wl >= 0 && wl + BP_W <= T) {
        const auto* q = in_global(reinterpret_cast<const i32x4*>(I.rowidx + c0 + wl));
#pragma unroll
        for (int i = 0; i < BP_W / 4; ++i) {
          const i32x4 x = q[i];
          w[4 * i] = x.x; w[4 * i + 1] = x.y; w[4 * i + 2] = x.z; w[4 * i + 3] = x.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < BP_W; ++i) {
          const int64_t e = wl + i;
          w[i] = e < 0 ? INT32_MIN : (e < T ? rows[e * s] : INT32_MAX);
        }
      }
    };
    load_window();
    for (int j = 0; j < jn; ++j) {
      int32_t f = fr[0];
#pragma unroll
      for (int q = 1; q < BP_MAX_CHUNK; ++q) f = j == q ? fr[q] : f;
      while (true) {
        int c = 0;
#pragma unroll
        for (int i = 0; i < BP_W; ++i) c += w[i] < f ? 1 : 0;
        if (c < BP_W) {
          pos[(b0 + j) * I.nv + v] = (int32_t)(wl + c);
          break;
        }
        wl += BP_W;  // all 16 slots lie above f, so wl + 16 <= T
        load_window();
      }
    }
  }
};

// seg[b*nv + v] = entries of (b, v), b < nb_max (scanned afterwards)
struct OpBlockCnt {
  static __device__ void run(const Item& I, int64_t t) {
    I.seg[t] = I.hdr->status ? 0 : I.pos[t + I.nv] - I.pos[t];
  }
};

// rowinfo[r] = {block of row r, its offset in the S tile in bytes}
struct OpRowInfo {
  static __device__ void run(const Item& I, int64_t r) {
    if (I.hdr->status) return;
    const int32_t c = I.ridx[r];
    if (I.ridx[r + 1] == c) return;  // empty row
    const int32_t b = I.bfl[c + 1] - 1;
    I.rowinfo[r] = make_int2(b, (c - I.bstart[b]) * I.row_bytes);
  }
};

// ent[seg[b nv + v] + position in v - pos[b nv + v]] = {row offset in the S
// tile, value}: one thread per entry (for blocks whose column segments are
// long, where the per-segment gather below would walk them one by one)
struct OpScatter {
  // (v, position in v) of entry p of column k; a position inside one
  // column fits 32 bits (pos holds int32)
  static __device__ __forceinline__ void virt(const Item& I, int64_t p, int64_t k, int64_t c0,
                                              int64_t& v, int64_t& q) {
    v = k;
    q = p - c0;
    if (I.vbase) {
      const auto* vbase = in_global(I.vbase);
      const uint32_t s = (uint32_t)(vbase[k + 1] - vbase[k]);
      const uint32_t q32 = (uint32_t)q;
      const uint32_t qs = q32 / s;
      v = vbase[k] + (q32 - qs * s);
      q = qs;
    }
  }
  static __device__ __forceinline__ uint32_t tagged(const Item& I, int2 ri, int64_t k) {
    uint32_t x = (uint32_t)ri.y;
    if (I.col_tag) x |= ((uint32_t)k & (uint32_t)(I.col_tag - 1)) << 16;
    return x;
  }
  static __device__ void run(const Item& I, int64_t p, int64_t k) {
    if (in_global(I.hdr)->status) return;
    const int2 ri = load_pair(I.rowinfo, in_global(I.rowidx)[p]);
    int64_t v, q;
    virt(I, p, k, in_global(I.colptr)[k], v, q);
    const int64_t bv = (int64_t)ri.x * I.nv + v;
    const int64_t dest = (int64_t)in_global(I.seg)[bv] - in_global(I.pos)[bv] + q;
    store_pair(I.ent, dest, tagged(I, ri, k), __float_as_uint(load_value(I.vals, I.vtype, p)));
  }
  // the same for N entries, stage by stage: rows and values, the rows'
  // block and offset, the (block, column) positions, then the stores
  template <int N>
  static __device__ void run_many(const Item& I, const int64_t (&p)[N], const int64_t (&k)[N],
                                  const bool (&ok)[N]) {
    if (in_global(I.hdr)->status) return;
    const auto* rowidx = in_global(I.rowidx);
    const auto* colptr = in_global(I.colptr);
    const auto* pos = in_global(I.pos);
    int32_t row[N];
    float a[N];
    int64_t v[N], q[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      row[j] = rowidx[p[j]];
      a[j] = load_value(I.vals, I.vtype, p[j]);
      virt(I, p[j], k[j], colptr[k[j]], v[j], q[j]);
    }
    int2 ri[N];
#pragma unroll
    for (int j = 0; j < N; ++j) ri[j] = load_pair(I.rowinfo, row[j]);
    int32_t base[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int64_t bv = (int64_t)ri[j].x * I.nv + v[j];
      base[j] = in_global(I.seg)[bv] - pos[bv];
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (ok[j]) store_pair(I.ent, (int64_t)base[j] + q[j], tagged(I, ri[j], k[j]), __float_as_uint(a[j]));
  }
};

// ent, one thread per (block b, virtual column v): the segment
// [seg[b nv + v], seg[b nv + v + 1]) takes the column's entries from its
// position pos[b nv + v] on (entry t of column k lies in virtual column
// vbase[k] + t mod s_k at position t / s_k), each as {row offset in the S
// tile, value}.  Thread index -> (b, v) in bands of GA_TB blocks, the block
// fastest: the eight lanes of a column read its consecutive segments, which
// lie one after another in the column (a segment is a few entries, far
// shorter than a cache line), and a workgroup writes 32 columns' segments of
// each of its blocks, which lie one after another in ent.
constexpr int GA_TB = 8;
struct OpGather {
  static constexpr int kPerThread = 1;
  static __device__ __forceinline__ uint32_t tagged(const Item& I, int2 ri, int64_t k) {
    uint32_t x = (uint32_t)ri.y;
    if (I.col_tag) x |= ((uint32_t)k & (uint32_t)(I.col_tag - 1)) << 16;
    return x;
  }
  static __device__ void run(const Item& I, int64_t x) {
    if (in_global(I.hdr)->status) return;
    // (b, v) of thread index x in [0, nb_max nv): band of GA_TB blocks (the
    // last one possibly shorter), then column, then block
    const int64_t band = x / ((int64_t)GA_TB * I.nv);
    const int64_t rem = x - band * GA_TB * I.nv;
    const int64_t b_lo = band * GA_TB;
    const int64_t rows = I.nb_max - b_lo < GA_TB ? I.nb_max - b_lo : GA_TB;
    const int64_t v = rows == GA_TB ? rem / GA_TB : rem / rows;
    const int64_t t = (b_lo + (rem - v * rows)) * I.nv + v;
    const auto* seg = in_global(I.seg);
    const int32_t s0 = seg[t], s1 = seg[t + 1];
    if (s1 <= s0) return;
    const int32_t q0 = in_global(I.pos)[t];
    int64_t k = v, j = 0, sk = 1;
    if (I.vbase) {
      const auto* vb = in_global(I.vbase);
      k = real_column(I.vbase, I.n, v);
      j = v - vb[k];
      sk = vb[k + 1] - vb[k];
    }
    const int64_t c0 = in_global(I.colptr)[k];
    const auto* rowidx = in_global(I.rowidx);
    const int32_t cnt = s1 - s0;
    // four entries a round: their loads together, then the row offsets
    for (int32_t i0 = 0; i0 < cnt; i0 += 4) {
      int32_t r[4];
      float a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t i = i0 + u < cnt ? i0 + u : i0;
        const int64_t p = c0 + (int64_t)(q0 + i) * sk + j;
        r[u] = rowidx[p];
        a[u] = load_value(I.vals, I.vtype, p);
      }
      int2 ri[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) ri[u] = load_pair(I.rowinfo, r[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u < cnt) store_pair(I.ent, (int64_t)s0 + i0 + u, tagged(I, ri[u], k), __float_as_uint(a[u]));
    }
  }
};

// Estimated cost of block b for one tile (b < nblocks; 0 past the end, so
// the scanned prefix ends at the total).  The sketch kernel gives each split
// a contiguous run of blocks holding an equal share of the total, so cheap
// blocks (dense ones, which the matrix cores take) do not leave splits idle.
struct OpBlockCost {
  static __device__ void run(const Item& I, int64_t b) {
    int32_t c = 0;
    if (!I.hdr->status && b < I.hdr->nblocks) {
      int64_t w = I.w_blk;
      if (!(I.dflag && I.dflag[b])) {
        const int64_t rb = I.bstart[b + 1] - I.bstart[b];
        const int64_t e = (int64_t)I.seg[(b + 1) * I.nv] - I.seg[b * I.nv];
        w += rb * I.w_row + e * I.w_ent;
      }
      w >>= I.cost_shift;
      c = (int32_t)(w < 1 ? 1 : (w > 0x3FFFFFFF ? 0x3FFFFFFF : w));
    }
    I.bcost[b] = c;
  }
};

}  // namespace sk

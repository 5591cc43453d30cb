// sk_inspect.hpp -- device kernels of the inspector: validation of the CSC
// input, compaction of the nonempty rows of A, and the blocked layout of A
// that the sketch kernels consume.
//
// The paper's Algorithm 4 needs a blocked representation built from the CSC
// input (Sec. III-B: the conversion costs O(ceil(n/b_n) m + nnz) and is cheap
// next to the multiplication, Table IV).  Here the blocks run the other way:
// a row block is a run of m_b consecutive *nonempty* rows of A (empty rows
// need no S column at all, Sec. III-B), and inside a block the entries are
// ordered by column, then row, so one S tile of the block's rows is reused by
// every column that has nonzeros there.
//
// Layout produced (all int32; nnz, m and the block grid must fit in int32):
//   ridx[r]            position of row r among the nonempty rows (exclusive
//                      scan of the occupancy flags); ridx[m] = R
//   rowlist[c]         the c-th nonempty row
//   pos[b*n + k]       first CSC position of column k with row >= first row
//                      of block b (b = 0..nb_max, the last one = colptr[k+1])
//   seg[b*n + k]       position of block b / column k's segment in `ent`;
//                      seg[nb_max*n] = nnz.  Block b spans
//                      [seg[b*n], seg[(b+1)*n]).
//   ent[p]             {byte offset of the entry's row in the S tile (row
//                      inside the block times the tile's row bytes), FP32
//                      bits of the value}
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// status bits written by the validation kernel
enum : int { ST_RANGE = 1, ST_UNSORTED = 2, ST_COLPTR = 4 };

struct Header {       // first bytes of the workspace
  int32_t status;     // OR of ST_* bits
  int32_t pad;
  int64_t nonempty;   // R
  int64_t nblocks;    // ceil(R / m_b)
  int64_t reserved[5];
};

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// largest k in [0, n) with colptr[k] <= p (colptr assumed non-decreasing;
// stays in range even when it is not)
__device__ __forceinline__ int64_t column_of(const int64_t* __restrict__ colptr, int64_t n,
                                             int64_t p) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (colptr[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float load_value(const void* vals, int vtype, int64_t p) {
  if (vtype == 0) return (float)((const double*)vals)[p];  // RNE
  if (vtype == 1) return ((const float*)vals)[p];
  const uint16_t h = ((const uint16_t*)vals)[p];          // bf16 -> fp32 exact
  return __uint_as_float((uint32_t)h << 16);
}

// Validate and mark occupied rows.  One thread per nonzero (and per colptr
// entry).
__global__ void k_validate_mark(const int64_t* __restrict__ colptr,
                                const int32_t* __restrict__ rowidx, int64_t m, int64_t n,
                                int64_t nnz, int32_t* __restrict__ flags,
                                Header* __restrict__ hdr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (t <= n) {
    const int64_t c = colptr[t];
    if (t == 0 && c != 0) bad |= ST_COLPTR;
    if (t == n && c != nnz) bad |= ST_COLPTR;
    if (t < n && colptr[t + 1] < c) bad |= ST_COLPTR;
    if (c < 0 || c > nnz) bad |= ST_COLPTR;
  }
  if (t < nnz) {
    const int32_t r = rowidx[t];
    if (r < 0 || r >= m) {
      bad |= ST_RANGE;
    } else {
      flags[r] = 1;
    }
    if (t > 0) {
      const int64_t k = column_of(colptr, n, t);
      if (colptr[k] < t && rowidx[t - 1] >= r) bad |= ST_UNSORTED;
    }
  }
  if (bad) atomicOr(&hdr->status, bad);
}

// ------------------------------------------------------------- scan (int32)
// In-place exclusive scan of a[0..count) in chunks of SCAN_CHUNK; the grand
// total goes to a[count].  Three passes: chunk-local scans (+ chunk sums),
// scan of the chunk sums (one workgroup), add the chunk offsets.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t& total) {
  // sh: SCAN_THREADS ints
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    const int32_t add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  total = sh[SCAN_THREADS - 1];
  const int32_t excl = sh[tid] - v;
  __syncthreads();
  return excl;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_chunks(int32_t* __restrict__ a,
                                                              int64_t count,
                                                              int32_t* __restrict__ sums) {
  __shared__ int32_t sh[SCAN_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t run = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int64_t idx = base + i;
    v[i] = idx < count ? a[idx] : 0;
    run += v[i];
  }
  int32_t total;
  int32_t off = block_exclusive_scan(run, sh, total);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int64_t idx = base + i;
    if (idx < count) a[idx] = off;
    off += v[i];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// one workgroup: exclusive scan of sums[0..nchunks), total -> *grand
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(int32_t* __restrict__ sums,
                                                            int64_t nchunks,
                                                            int32_t* __restrict__ grand) {
  __shared__ int32_t sh[SCAN_THREADS];
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

__global__ void k_scan_add(int32_t* __restrict__ a, int64_t count,
                           const int32_t* __restrict__ sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] += sums[i / SCAN_CHUNK];
}

// nonempty-row list and block count.  ridx = scanned flags, ridx[m] = R.
__global__ void k_rowlist(const int32_t* __restrict__ ridx, int64_t m,
                          int32_t* __restrict__ rowlist, int32_t m_b, int64_t nb_max,
                          Header* __restrict__ hdr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m && ridx[r + 1] > ridx[r]) rowlist[ridx[r]] = (int32_t)r;
  if (r == 0) {
    const int64_t R = ridx[m];
    hdr->nonempty = R;
    int64_t nb = (R + m_b - 1) / m_b;
    hdr->nblocks = nb < nb_max ? nb : nb_max;
  }
}

// pos[b*n + k], b = 0..nb_max: first position of column k whose row is >= the
// first row of block b (b >= nblocks: the end of the column).
__global__ void k_block_pos(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                            int64_t m, int64_t n, const int32_t* __restrict__ rowlist,
                            int32_t m_b, int64_t nb_max, const Header* __restrict__ hdr,
                            int32_t* __restrict__ pos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (nb_max + 1) * n) return;
  if (hdr->status) return;
  const int64_t b = t / n, k = t - b * n;
  int64_t lo = colptr[k], hi = colptr[k + 1];
  if (b < hdr->nblocks) {
    const int32_t fr = rowlist[b * m_b];
    while (lo < hi) {  // lower bound of fr in rowidx[lo, hi)
      const int64_t mid = (lo + hi) >> 1;
      if (rowidx[mid] < fr) lo = mid + 1;
      else hi = mid;
    }
  } else {
    lo = hi;
  }
  pos[t] = (int32_t)lo;
}

// seg[b*n + k] = count of (b, k), b < nb_max (scanned afterwards)
__global__ void k_block_cnt(const int32_t* __restrict__ pos, int64_t n, int64_t nb_max,
                            const Header* __restrict__ hdr, int32_t* __restrict__ seg) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb_max * n) return;
  seg[t] = hdr->status ? 0 : pos[t + n] - pos[t];
}

// ent[seg[b n + k] + (p - pos[b n + k])] = {row in block * row_bytes, value}
__global__ void k_scatter(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                          const void* __restrict__ vals, int vtype, int64_t n, int64_t nnz,
                          const int32_t* __restrict__ ridx, const int32_t* __restrict__ pos,
                          const int32_t* __restrict__ seg, int32_t m_b, int32_t row_bytes,
                          const Header* __restrict__ hdr, uint2* __restrict__ ent) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  if (hdr->status) return;
  const int32_t r = rowidx[p];
  const int32_t c = ridx[r];
  const int32_t b = c / m_b;
  const int32_t l = c - b * m_b;
  const int64_t k = column_of(colptr, n, p);
  const int64_t bk = (int64_t)b * n + k;
  const int64_t dest = (int64_t)seg[bk] + (p - (int64_t)pos[bk]);
  ent[dest] = make_uint2((uint32_t)l * (uint32_t)row_bytes,
                         __float_as_uint(load_value(vals, vtype, p)));
}


// ---------------------------------------------------- heavy-column splitting
// A column with many more entries than average would make its owning lane
// the straggler of every block.  Column k is split into s_k interleaved
// virtual columns (entry t of the column goes to virtual column
// vbase[k] + t mod s_k, position t / s_k), s_k = ceil(cnt_k / L) with
// L = ceil(nnz / spare): the virtual column count stays within the planned
// capacity n_v.  The sketch runs on virtual columns; the final reduction adds
// them back up.

// vbase[k] = s_k (scanned afterwards); one thread per column
__global__ void k_colsplit_count(const int64_t* __restrict__ colptr, int64_t n, int64_t nnz,
                                 int64_t spare, const Header* __restrict__ hdr,
                                 int32_t* __restrict__ vbase) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int64_t s = 1;
  if (!hdr->status && spare > 0 && nnz > 0) {
    const int64_t L = (nnz + spare - 1) / spare;
    const int64_t c = colptr[k + 1] - colptr[k];
    s = c > L ? (c + L - 1) / L : 1;
  }
  vbase[k] = (int32_t)s;
}

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

// pos[b*nv + v] (in units of the virtual column's own positions), b = 0..nb_max
__global__ void k_block_pos_v(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                              int64_t n, int64_t nv, const int32_t* __restrict__ vbase,
                              const int32_t* __restrict__ rowlist, int32_t m_b, int64_t nb_max,
                              const Header* __restrict__ hdr, int32_t* __restrict__ pos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (nb_max + 1) * nv) return;
  if (hdr->status) return;
  const int64_t b = t / nv, v = t - b * nv;
  const int64_t vtot = vbase[n];
  if (v >= vtot) {
    pos[t] = 0;
    return;
  }
  const int64_t k = real_column(vbase, n, v);
  const int64_t s = vbase[k + 1] - vbase[k], r = v - vbase[k];
  const int64_t c0 = colptr[k], cnt = colptr[k + 1] - c0;
  const int64_t T = cnt > r ? (cnt - r + s - 1) / s : 0;  // entries of this virtual column
  int64_t lo = 0, hi = T;
  if (b < hdr->nblocks) {
    const int32_t fr = rowlist[b * m_b];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (rowidx[c0 + r + mid * s] < fr) lo = mid + 1;
      else hi = mid;
    }
  } else {
    lo = hi;
  }
  pos[t] = (int32_t)lo;
}

__global__ void k_scatter_v(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                            const void* __restrict__ vals, int vtype, int64_t n, int64_t nv,
                            int64_t nnz, const int32_t* __restrict__ vbase,
                            const int32_t* __restrict__ ridx, const int32_t* __restrict__ pos,
                            const int32_t* __restrict__ seg, int32_t m_b, int32_t row_bytes,
                            const Header* __restrict__ hdr, uint2* __restrict__ ent) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  if (hdr->status) return;
  const int32_t r = rowidx[p];
  const int32_t c = ridx[r];
  const int32_t b = c / m_b;
  const int32_t l = c - b * m_b;
  const int64_t k = column_of(colptr, n, p);
  const int64_t s = vbase[k + 1] - vbase[k];
  const int64_t tall = p - colptr[k];
  const int64_t v = vbase[k] + tall % s;
  const int64_t bv = (int64_t)b * nv + v;
  const int64_t dest = (int64_t)seg[bv] + (tall / s - (int64_t)pos[bv]);
  ent[dest] = make_uint2((uint32_t)l * (uint32_t)row_bytes,
                         __float_as_uint(load_value(vals, vtype, p)));
}

}  // namespace sk

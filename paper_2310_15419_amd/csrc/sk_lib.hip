// sk_lib.hip -- host side of libsketch.so: argument checks, the plan (tile
// shapes from the problem shape only, so a given request always runs the same
// summation order), the workspace layout, and the launches of the inspector,
// sketch and reduction kernels.  Every step of the computation runs in the
// kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "sk_dense.hpp"
#include "sk_inspect.hpp"
#include "sk_rng.hpp"
#include "sk_sketch.hpp"
#include "sketch.h"

using namespace sk;

namespace {

constexpr int64_t kAlign = 256;
constexpr int kLdsPerCu = 160 * 1024;  // LDS bytes per CU (gfx950)

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << (r + 1)) <= v) ++r;
  return r;
}

// ------------------------------------------------------------ kernel table
using SketchKernel = void (*)(SketchParams);

struct Variant {
  int dl, q, cs, wgs;
  SketchKernel k[3];  // per distribution
};

#define SK_VARIANT(DL, Q, CS, WGS)                                                         \
  Variant {                                                                                \
    DL, Q, CS, WGS, {                                                                      \
      k_sketch<DIST_RADEMACHER, DL, Q, CS, WGS>, k_sketch<DIST_UNIFORM, DL, Q, CS, WGS>, \
          k_sketch<DIST_GAUSSIAN, DL, Q, CS, WGS>                                          \
    }                                                                                      \
  }

const Variant kVariants[] = {
    SK_VARIANT(4, 4, 8, 1024),   // 1: d_b = 16 per subtile, 2048 columns per workgroup
    SK_VARIANT(4, 4, 16, 1024),  // 2: 4096 columns
    SK_VARIANT(8, 4, 8, 1024),   // 3: d_b = 32 per subtile
    SK_VARIANT(8, 2, 4, 1024),   // 4: pairs of lanes per column group
    SK_VARIANT(16, 1, 2, 1024),  // 5: one lane per column group
    SK_VARIANT(4, 4, 2, 1024),   // 6: few columns, many S rows per workgroup
    SK_VARIANT(16, 1, 4, 512),   // 7: two workgroups per CU, one lane per column group
    SK_VARIANT(8, 2, 8, 512),    // 8: two workgroups per CU, lane pairs
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

struct Plan {
  int variant;  // index into kVariants
  int32_t m_b, e_max, d_b, ldS, dt, cg, tiles, splits, col_per_wg, ncr, log2_cpr;
  int64_t nb_max;
  size_t lds;
  int32_t dense_pct;  // densify at >= this % density; 0: no dense path
  int64_t nd_max;     // capacity in dense blocks
  int32_t slices;     // partial slices: splits (+1 for the dense path)
};

struct Layout {
  int64_t hdr, ridx, sums, rowlist, pos, seg, ent, dflag, dlist, dhdr, dense, part, total;
};

constexpr int kDenseAutoPct = 40;                 // FP32 operands
constexpr int64_t kDenseMaxBytes = int64_t(4) << 30;

bool plan_for(int64_t m, int64_t n, int64_t nnz, int64_t d, int dist, const sk_tuning* tune,
              Plan& P) {
  int v = tune && tune->variant > 0 ? tune->variant - 1 : -1;
  if (v >= kNumVariants) return false;
  if (v < 0) {
    // auto: enough columns per workgroup, then the most S rows per lane
    if (n <= 512) v = 5;
    else if (n <= 2048) v = 0;
    else v = 1;
  }
  const Variant& V = kVariants[v];
  const int groups = V.wgs / V.q;
  P.variant = v;
  int64_t cg = (n + V.cs - 1) / V.cs;
  int ncr = 1;
  if (cg > groups) {  // more columns than one workgroup covers: split the columns
    ncr = (int)((cg + groups - 1) / groups);
    cg = (int64_t)groups;
  }
  P.cg = (int32_t)cg;
  P.ncr = ncr;
  P.col_per_wg = (int32_t)(cg * V.cs);
  // S-row subtiles: a power of two, no more than the groups allow, d_b <= 128,
  // and not far beyond d
  int dt = 1;
  while (dt * 2 * cg <= groups && dt * 2 * V.q * V.dl <= 128 &&
         (int64_t)dt * V.q * V.dl < d)
    dt *= 2;
  P.dt = dt;
  P.d_b = dt * V.q * V.dl;
  P.ldS = P.d_b + 4;
  P.tiles = (int32_t)((d + P.d_b - 1) / P.d_b);
  const int rows_per_chunk = dist == DIST_RADEMACHER ? std::min(32, P.d_b) : 4;
  P.log2_cpr = ilog2(P.d_b / rows_per_chunk);
  // rows per block from the LDS budget (1024-thread workgroups: one per CU;
  // 512-thread workgroups: two per CU): S tile row + the block's entries
  const int budget = (V.wgs >= 1024 ? kLdsPerCu : kLdsPerCu / 2) - 1024;
  const int64_t rmax = std::max<int64_t>(1, std::min(m, nnz));
  const double per_row = std::max(1.0, (double)nnz / (double)rmax);
  int64_t m_b = tune && tune->rows_per_block > 0
                    ? tune->rows_per_block
                    : (int64_t)((double)budget / (P.ldS * 4.0 + 8.0 * per_row));
  m_b = std::max<int64_t>(1, std::min<int64_t>(m_b, 8192));
  while (m_b > 1 && m_b * P.ldS * 4 + 8 * 64 > budget) m_b /= 2;
  P.m_b = (int32_t)m_b;
  P.e_max = (int32_t)(((budget - m_b * P.ldS * 4) / 8 - 2) & ~int64_t(1));
  if (P.e_max < 2) return false;
  P.lds = (size_t)m_b * P.ldS * 4 + (size_t)(P.e_max + 2) * 8;
  P.nb_max = std::max<int64_t>(1, (rmax + m_b - 1) / m_b);
  int64_t splits;
  if (tune && tune->splits > 0) {
    splits = tune->splits;
  } else {
    const int64_t wgs_now = (int64_t)P.tiles * ncr;
    splits = (2048 + wgs_now - 1) / wgs_now;
    if (splits >= 8) splits = (splits + 7) / 8 * 8;  // whole XCDs per split
    splits = std::min<int64_t>(splits, 64);
  }
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, P.nb_max));
  P.splits = (int32_t)splits;
  // dense row blocks: only if at least one block could reach the threshold
  int pct = tune && tune->dense_min_pct > 0 ? tune->dense_min_pct : kDenseAutoPct;
  P.dense_pct = 0;
  P.nd_max = 0;
  if (pct <= 100 && (double)nnz * 100.0 >= (double)pct * (double)m_b * (double)n) {
    int64_t ndm = (int64_t)((double)nnz * 100.0 / ((double)pct * (double)m_b * (double)n)) + 1;
    ndm = std::min<int64_t>(ndm, P.nb_max);
    ndm = std::min<int64_t>(ndm, kDenseMaxBytes / (4 * (int64_t)m_b * n));
    if (ndm > 0) {
      P.dense_pct = pct;
      P.nd_max = ndm;
    }
  }
  P.slices = P.splits + (P.dense_pct ? 1 : 0);
  return true;
}

Layout layout_for(int64_t m, int64_t n, int64_t nnz, int64_t d, const Plan& P) {
  Layout L{};
  int64_t off = 0;
  L.hdr = off;     off = align_up(off + (int64_t)sizeof(Header));
  L.ridx = off;    off = align_up(off + 4 * (m + 1));
  const int64_t big = std::max<int64_t>({m, (P.nb_max + 1) * n, nnz, 1});
  L.sums = off;    off = align_up(off + 4 * (big / SCAN_CHUNK + 2));
  L.rowlist = off; off = align_up(off + 4 * (std::min(m, std::max<int64_t>(nnz, 1)) + P.m_b + 1));
  L.pos = off;     off = align_up(off + 4 * (P.nb_max + 1) * n);
  L.seg = off;     off = align_up(off + 4 * (P.nb_max * n + 1));
  L.ent = off;     off = align_up(off + 8 * (nnz + 2));  // +2: 16-byte staging tail
  L.dflag = off;   off = align_up(off + 4 * P.nb_max);
  L.dlist = off;   off = align_up(off + 4 * std::max<int64_t>(P.nd_max, 1));
  L.dhdr = off;    off = align_up(off + (int64_t)sizeof(DenseHeader));
  L.dense = off;   off = align_up(off + 4 * P.nd_max * P.m_b * n);
  L.part = off;
  if (P.slices > 1) off = align_up(off + 4 * (int64_t)P.slices * d * n);
  L.total = off;
  return L;
}

sk_status check_csc(const sk_csc* A) {
  if (!A || !A->colptr) return SK_EINVAL;
  if (A->m < 1 || A->n < 1 || A->nnz < 0) return SK_EINVAL;
  if (A->nnz > 0 && (!A->rowidx || !A->vals)) return SK_EINVAL;
  if (A->m >= INT32_MAX || A->nnz >= INT32_MAX) return SK_EUNSUPPORTED;
  if (A->vtype < SK_F64 || A->vtype > SK_BF16) return SK_EINVAL;
  return SK_OK;
}

int blocks_for(int64_t count, int threads) {
  const int64_t b = (count + threads - 1) / threads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, INT32_MAX));
}

sk_status launch_ok() {
  return hipGetLastError() == hipSuccess ? SK_OK : SK_EHIP;
}

// in-place exclusive scan of a[0..count), total to a[count]
sk_status scan_i32(int32_t* a, int64_t count, int32_t* sums, hipStream_t st) {
  const int64_t nchunks = (count + SCAN_CHUNK - 1) / SCAN_CHUNK;
  if (nchunks == 0) {
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, a, int64_t(1), 0);
    return launch_ok();
  }
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nchunks), dim3(SCAN_THREADS), 0, st, a,
                     count, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, st, sums, nchunks, a + count);
  hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(count, 256)), dim3(256), 0, st, a, count, sums);
  return launch_ok();
}

}  // namespace

extern "C" {

const char* sk_status_string(int s) {
  switch (s) {
    case SK_OK: return "ok";
    case SK_EINVAL: return "invalid argument";
    case SK_EUNSORTED: return "row indices not strictly increasing within a column";
    case SK_ERANGE: return "row index out of range";
    case SK_EWORKSPACE: return "workspace missing or too small";
    case SK_EHIP: return "HIP runtime error";
    case SK_EUNSUPPORTED: return "unsupported request";
    case SK_ECOLPTR: return "column pointers malformed";
    default: return "unknown status";
  }
}

int sk_variant_count(void) { return kNumVariants; }

sk_status sk_sketch_workspace(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                              const sk_tuning* tune, size_t* bytes) {
  if (!bytes) return SK_EINVAL;
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || dist < 0 || dist > 2 || prec < 0 || prec > 2) return SK_EINVAL;
  Plan P;
  if (!plan_for(A->m, A->n, A->nnz, d, dist, tune, P)) return SK_EINVAL;
  *bytes = (size_t)layout_for(A->m, A->n, A->nnz, d, P).total;
  return SK_OK;
}

sk_status sk_sketch(const sk_csc* A, int64_t row0, int64_t d, int32_t dist, uint64_t seed,
                    int32_t prec, const sk_tuning* tune, float* Ahat, int64_t ld, void* ws,
                    size_t ws_bytes, void* hip_stream) {
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || row0 < 0 || !Ahat || ld < d || dist < 0 || dist > 2) return SK_EINVAL;
  if (prec < 0 || prec > 2) return SK_EINVAL;
  if (prec != SK_PREC_F32 && dist != SK_RADEMACHER) return SK_EUNSUPPORTED;
  Plan P;
  if (!plan_for(A->m, A->n, A->nnz, d, dist, tune, P)) return SK_EINVAL;
  if ((int64_t)(P.nb_max + 1) * A->n >= INT32_MAX) return SK_EUNSUPPORTED;
  const Layout L = layout_for(A->m, A->n, A->nnz, d, P);
  if (!ws || ws_bytes < (size_t)L.total) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t m = A->m, n = A->n, nnz = A->nnz;
  const int phases = tune && tune->phases ? tune->phases : 7;
  char* w = (char*)ws;
  Header* hdr = (Header*)(w + L.hdr);
  int32_t* ridx = (int32_t*)(w + L.ridx);
  int32_t* sums = (int32_t*)(w + L.sums);
  int32_t* rowlist = (int32_t*)(w + L.rowlist);
  int32_t* pos = (int32_t*)(w + L.pos);
  int32_t* seg = (int32_t*)(w + L.seg);
  uint2* ent = (uint2*)(w + L.ent);
  int32_t* dflag = (int32_t*)(w + L.dflag);
  int32_t* dlist = (int32_t*)(w + L.dlist);
  DenseHeader* dhdr = (DenseHeader*)(w + L.dhdr);
  float* dense = (float*)(w + L.dense);
  float* part = (float*)(w + L.part);

  if (phases & 1) {
  // a1: validate + mark nonempty rows
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, (int32_t*)hdr,
                     (int64_t)(sizeof(Header) / 4), 0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(m + 1, 256)), dim3(256), 0, st, ridx, m + 1,
                     0);
  const int64_t vthreads = std::max<int64_t>(nnz, n + 1);
  hipLaunchKernelGGL(k_validate_mark, dim3(blocks_for(vthreads, 256)), dim3(256), 0, st,
                     A->colptr, A->rowidx, m, n, nnz, ridx, hdr);
  // a2: inspector -- compaction of nonempty rows, blocked layout
  if ((s = scan_i32(ridx, m, sums, st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_rowlist, dim3(blocks_for(m, 256)), dim3(256), 0, st, ridx, m, rowlist,
                     P.m_b, P.nb_max, hdr);
  // pad the row list so every block reads a full m_b rows
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(256), 0, st,
                     rowlist + std::min(m, std::max<int64_t>(nnz, 1)), (int64_t)P.m_b + 1, 0);
  const int64_t npos = (P.nb_max + 1) * n;
  hipLaunchKernelGGL(k_block_pos, dim3(blocks_for(npos, 256)), dim3(256), 0, st, A->colptr,
                     A->rowidx, m, n, rowlist, P.m_b, P.nb_max, hdr, pos);
  const int64_t nseg = P.nb_max * n;
  hipLaunchKernelGGL(k_block_cnt, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, pos, n,
                     P.nb_max, hdr, seg);
  if ((s = scan_i32(seg, nseg, sums, st)) != SK_OK) return s;
  if (nnz > 0)
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, A->colptr,
                       A->rowidx, A->vals, A->vtype, n, nnz, ridx, pos, seg, P.m_b, P.ldS * 4,
                       hdr, ent);
  if ((s = launch_ok()) != SK_OK) return s;
  // a5 (selection): dense row blocks, densified
  if (P.dense_pct) {
    hipLaunchKernelGGL(k_dense_select, dim3(1), dim3(256), 0, st, seg, n, P.m_b, P.dense_pct,
                       (int32_t)P.nd_max, hdr, dflag, dlist, dhdr);
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks_for(P.nd_max * P.m_b * n, 256 * 16)),
                       dim3(256), 0, st, dense, P.nd_max * P.m_b * n, 0.0f);
    hipLaunchKernelGGL(k_densify, dim3(blocks_for(P.nd_max * n, 256)), dim3(256), 0, st, seg,
                       ent, n, P.m_b, P.ldS * 4, dlist, dhdr, dense);
    if ((s = launch_ok()) != SK_OK) return s;
  }
  }

  // a3 + a4: S tiles and sparse accumulation
  const Variant& V = kVariants[P.variant];
  SketchParams K{};
  K.rowlist = rowlist; K.seg = seg; K.ent = ent; K.hdr = hdr;
  K.dflag = P.dense_pct ? dflag : nullptr;
  K.n = n; K.d = d; K.row0 = row0; K.seed = seed;
  K.m_b = P.m_b; K.e_max = P.e_max; K.d_b = P.d_b; K.ldS = P.ldS; K.log2_cpr = P.log2_cpr;
  K.dt = P.dt; K.cg = P.cg; K.tiles = P.tiles; K.splits = P.splits;
  K.col_per_wg = P.col_per_wg;
  if (P.slices > 1) { K.out = part; K.ld = d; K.split_stride = d * n; }
  else { K.out = Ahat; K.ld = ld; K.split_stride = 0; }
  const int64_t grid = (int64_t)P.tiles * P.ncr * P.splits;
  if (grid >= INT32_MAX) return SK_EUNSUPPORTED;
  SketchKernel kern = V.k[dist];
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)P.lds) != hipSuccess)
    return SK_EHIP;
  if (phases & 2) {
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(V.wgs), P.lds, st, K);
    if ((s = launch_ok()) != SK_OK) return s;
  }
  // a5: dense row blocks on the matrix cores, into the last partial slice
  if ((phases & 2) && P.dense_pct) {
    DenseParams DP{};
    DP.rowlist = rowlist; DP.dlist = dlist; DP.dh = dhdr; DP.hdr = hdr; DP.D = dense;
    DP.n = n; DP.d = d; DP.row0 = row0; DP.seed = seed; DP.m_b = P.m_b;
    DP.out = part + (int64_t)P.splits * d * n;
    const int64_t dgrid = ((d + DT_M - 1) / DT_M) * ((n + DT_N - 1) / DT_N);
    if (dgrid >= INT32_MAX) return SK_EUNSUPPORTED;
    if (dist == SK_RADEMACHER)
      hipLaunchKernelGGL(k_dense_mfma<DIST_RADEMACHER>, dim3((unsigned)dgrid), dim3(256), 0, st, DP);
    else if (dist == SK_UNIFORM)
      hipLaunchKernelGGL(k_dense_mfma<DIST_UNIFORM>, dim3((unsigned)dgrid), dim3(256), 0, st, DP);
    else
      hipLaunchKernelGGL(k_dense_mfma<DIST_GAUSSIAN>, dim3((unsigned)dgrid), dim3(256), 0, st, DP);
    if ((s = launch_ok()) != SK_OK) return s;
  }
  // a6: fixed-order reduction of the partial slices
  if ((phases & 4) && P.slices > 1)
    hipLaunchKernelGGL(k_reduce_splits, dim3(blocks_for(d * n, 256)), dim3(256), 0, st, part,
                       P.slices, d, n, Ahat, ld);
  return launch_ok();
}

sk_status sk_sketch_status(const void* ws, void* hip_stream, int64_t* nonempty_rows,
                           int64_t* row_blocks) {
  if (!ws) return SK_EINVAL;
  Header h;
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess) return SK_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SK_EHIP;
  if (nonempty_rows) *nonempty_rows = h.nonempty;
  if (row_blocks) *row_blocks = h.nblocks;
  if (h.status & ST_COLPTR) return SK_ECOLPTR;
  if (h.status & ST_RANGE) return SK_ERANGE;
  if (h.status & ST_UNSORTED) return SK_EUNSORTED;
  return SK_OK;
}

sk_status sk_materialize_s(int64_t row0, int64_t d, int64_t col0, int64_t ncols, int32_t dist,
                           uint64_t seed, float* S, int64_t ld, void* hip_stream) {
  if (d < 1 || ncols < 1 || row0 < 0 || col0 < 0 || !S || ld < d || dist < 0 || dist > 2)
    return SK_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const int rpc = dist == SK_RADEMACHER ? 32 : 4;
  const int64_t threads = ((row0 + d - 1) / rpc - row0 / rpc + 1) * ncols;
  const int b = blocks_for(threads, 256);
  if (dist == SK_RADEMACHER)
    hipLaunchKernelGGL(k_materialize<DIST_RADEMACHER>, dim3(b), dim3(256), 0, st, row0, d, col0,
                       ncols, seed, S, ld);
  else if (dist == SK_UNIFORM)
    hipLaunchKernelGGL(k_materialize<DIST_UNIFORM>, dim3(b), dim3(256), 0, st, row0, d, col0,
                       ncols, seed, S, ld);
  else
    hipLaunchKernelGGL(k_materialize<DIST_GAUSSIAN>, dim3(b), dim3(256), 0, st, row0, d, col0,
                       ncols, seed, S, ld);
  return launch_ok();
}

void sk_rng_tables(float* log_c, float* sin_c, float* cos_c, float* misc) {
  std::memcpy(log_c, kTables.log_c, sizeof kTables.log_c);
  std::memcpy(sin_c, kTables.sin_c, sizeof kTables.sin_c);
  std::memcpy(cos_c, kTables.cos_c, sizeof kTables.cos_c);
  misc[0] = kTables.ln2_hi;
  misc[1] = kTables.ln2_lo;
  misc[2] = kTables.sqrt2;
}

}  // extern "C"

// sk_lib.hip -- host side of libsketch.so: argument checks, the plan (tile
// shapes from the problem shape only, so a given request always runs the same
// summation order), the workspace layout, and the launches of the inspector,
// sketch and reduction kernels.  Every step of the computation runs in the
// kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>
#include <cstdint>
#include <cstring>

#include "sk_batch.hpp"
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

using PersistentKernel = void (*)(const BatchItem*, const int2*, int, int32_t*);

struct Variant {
  int dl, q, cs, wgs;
  SketchKernel k[3];      // per distribution
  PersistentKernel p[3];  // persistent (batched) form, per distribution
};

#define SK_VARIANT(DL, Q, CS, WGS)                                                           \
  Variant {                                                                                  \
    DL, Q, CS, WGS,                                                                          \
        {k_sketch<DIST_RADEMACHER, DL, Q, CS, WGS>, k_sketch<DIST_UNIFORM, DL, Q, CS, WGS>,  \
         k_sketch<DIST_GAUSSIAN, DL, Q, CS, WGS>},                                           \
        {k_sketch_persistent<DIST_RADEMACHER, DL, Q, CS, WGS>,                               \
         k_sketch_persistent<DIST_UNIFORM, DL, Q, CS, WGS>,                                  \
         k_sketch_persistent<DIST_GAUSSIAN, DL, Q, CS, WGS>}                                 \
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
  double cost;        // autotuner's cost estimate (CU-cycles)
  int64_t nv;         // virtual columns (== n without heavy-column splitting)
};

struct Layout {
  int64_t hdr, ridx, sums, rowlist, vbase, pos, seg, ent, dflag, dlist, dhdr, dense, part, total;
};

constexpr int kDenseAutoPct = 40;                 // FP32 operands
constexpr int64_t kDenseMaxBytes = int64_t(4) << 30;

// ------------------------------------------------------------ autotuner
// Cost model of one sketch under a plan, in CU-cycles (one VALU wave
// instruction ~ one CU-cycle: four SIMDs, four cycles each).  Terms: S
// generation (one generator call per nonempty row per chunk of S rows per
// tile), the multiply-adds with the lane-lockstep padding of the column walk
// (a wave waits for its longest column segment: E[max of W Poisson(lambda)]
// over lambda), staging the block entries once per tile, and a fixed cost per
// (tile, block).
double plan_cost(const Plan& P, const Variant& V, int64_t m, int64_t n, int64_t nnz, int64_t d,
                 int dist) {
  if (nnz <= 0) return 0.0;
  const double R = (double)m * (1.0 - std::exp(-(double)nnz / (double)m));
  const double tiles = (double)P.tiles * P.ncr;
  const double d_eff = (double)P.tiles * P.d_b;
  const int rpc = dist == DIST_RADEMACHER ? std::min(32, P.d_b) : 4;
  const double call_ops = dist == DIST_GAUSSIAN ? 200.0 : (dist == DIST_UNIFORM ? 75.0 : 70.0);
  const double rng = R * (double)P.ncr * (d_eff / rpc) * call_ops / 64.0;
  const double lambda = std::max(1e-3, (double)P.m_b * ((double)nnz / R) / (double)n);
  const double W = 64.0 / V.q;
  const double emax = std::max(lambda + std::sqrt(2.0 * lambda * std::log(W)), std::min(1.0, W * lambda));
  const double pad = emax / lambda;
  const double fma = (double)nnz * d_eff * (V.dl + 3.0) / V.dl / 64.0 * pad;
  const double stage = (double)nnz * tiles * 8.0 / 128.0;
  const double nb = std::ceil(R / P.m_b);
  const double blocks = nb * tiles * 1000.0;
  return rng + fma + stage + blocks;
}

// Plan for one sketch.  `forced_variant` >= 0 pins the kernel shape (batched
// launches share one); `unit_cycles` > 0 sizes the row-range splits so that
// one work unit costs about that much (batched), else splits fill the GPU.
bool plan_for(int64_t m, int64_t n, int64_t nnz, int64_t d, int dist, const sk_tuning* tune,
              Plan& P, int forced_variant = -1, double unit_cycles = 0.0) {
  int v = forced_variant >= 0 ? forced_variant : (tune && tune->variant > 0 ? tune->variant - 1 : -1);
  if (v >= kNumVariants) return false;
  if (forced_variant >= 0 && tune && tune->variant > 0 && tune->variant - 1 != forced_variant)
    return false;
  if (v < 0) {
    // auto: enough columns per workgroup, then the most S rows per lane
    if (n <= 512) v = 5;
    else if (n <= 2048) v = 0;
    else v = 1;
  }
  const Variant& V = kVariants[v];
  const int groups = V.wgs / V.q;
  P.variant = v;
  // heavy-column splitting (single sketches only): reserve up to n spare
  // virtual columns inside one workgroup's column capacity
  const int split_mode = tune ? tune->col_split : 0;
  bool split = forced_variant < 0 && (split_mode == 2 || (split_mode == 0 && n >= 512));
  const int64_t capacity = (int64_t)groups * V.cs;
  P.nv = n;
  if (split && capacity > n) P.nv = std::min<int64_t>(capacity, 2 * n);
  int64_t cg = (P.nv + V.cs - 1) / V.cs;
  int ncr = 1;
  if (cg > groups) {  // more columns than one workgroup covers: split the columns
    ncr = (int)((cg + groups - 1) / groups);
    cg = (int64_t)groups;
  }
  P.cg = (int32_t)cg;
  P.ncr = ncr;
  P.col_per_wg = (int32_t)(cg * V.cs);
  const int budget = (V.wgs >= 1024 ? kLdsPerCu : kLdsPerCu / 2) - 1024;
  const int64_t rmax = std::max<int64_t>(1, std::min(m, nnz));
  const double per_row = std::max(1.0, (double)nnz / (double)rmax);

  // candidate S-row subtile counts: powers of two that the column groups
  // allow, d_b <= 128, not far beyond d
  int dt_max = 1;
  while (dt_max * 2 * cg <= groups && dt_max * 2 * V.q * V.dl <= 128 &&
         (int64_t)dt_max * V.q * V.dl < d)
    dt_max *= 2;
  int dt_fixed = 0;
  if (tune && tune->tile_rows > 0) {
    const int unit = V.q * V.dl;
    if (tune->tile_rows % unit) return false;
    dt_fixed = tune->tile_rows / unit;
    if ((dt_fixed & (dt_fixed - 1)) || dt_fixed * cg > groups) return false;
  }
  double best = -1.0;
  Plan bestP = P;
  for (int dt = 1; dt <= (dt_fixed ? dt_fixed : dt_max); dt *= 2) {
    if (dt_fixed && dt != dt_fixed) continue;
    Plan Q = P;
    Q.dt = dt;
    Q.d_b = dt * V.q * V.dl;
    Q.ldS = Q.d_b + 4;
    Q.tiles = (int32_t)((d + Q.d_b - 1) / Q.d_b);
    const int rows_per_chunk = dist == DIST_RADEMACHER ? std::min(32, Q.d_b) : 4;
    Q.log2_cpr = ilog2(Q.d_b / rows_per_chunk);
    // rows per block from the LDS budget (1024-thread workgroups: one per CU;
    // 512-thread workgroups: two per CU): S tile row + the block's entries
    int64_t m_b = tune && tune->rows_per_block > 0
                      ? tune->rows_per_block
                      : (int64_t)((double)budget / (Q.ldS * 4.0 + 8.0 * per_row));
    m_b = std::max<int64_t>(1, std::min<int64_t>(m_b, 8192));
    while (m_b > 1 && m_b * Q.ldS * 4 + 8 * 64 > budget) m_b /= 2;
    Q.m_b = (int32_t)m_b;
    Q.e_max = (int32_t)(((budget - m_b * Q.ldS * 4) / 8 - 2) & ~int64_t(1));
    if (Q.e_max < 2) continue;
    Q.lds = (size_t)m_b * Q.ldS * 4 + (size_t)(Q.e_max + 2) * 8;
    Q.nb_max = std::max<int64_t>(1, (rmax + m_b - 1) / m_b);
    const double c = plan_cost(Q, V, m, P.nv, nnz, d, dist);
    if (best < 0 || c < best) {
      best = c;
      bestP = Q;
    }
  }
  if (best < 0) return false;
  P = bestP;
  int64_t splits;
  if (tune && tune->splits > 0) {
    splits = tune->splits;
  } else if (unit_cycles > 0) {
    splits = (int64_t)std::ceil(best / ((double)P.tiles * P.ncr * unit_cycles));
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
  const int64_t m_b = P.m_b;
  if (unit_cycles <= 0 && pct <= 100 &&
      (double)nnz * 100.0 >= (double)pct * (double)m_b * (double)n) {
    int64_t ndm = (int64_t)((double)nnz * 100.0 / ((double)pct * (double)m_b * (double)n)) + 1;
    ndm = std::min<int64_t>(ndm, P.nb_max);
    ndm = std::min<int64_t>(ndm, kDenseMaxBytes / (4 * (int64_t)m_b * n));
    if (ndm > 0) {
      P.dense_pct = pct;
      P.nd_max = ndm;
    }
  }
  P.slices = P.splits + (P.dense_pct ? 1 : 0);
  P.cost = best;
  return true;
}

Layout layout_for(int64_t m, int64_t n, int64_t nnz, int64_t d, const Plan& P) {
  Layout L{};
  int64_t off = 0;
  L.hdr = off;     off = align_up(off + (int64_t)sizeof(Header));
  L.ridx = off;    off = align_up(off + 4 * (m + 1));
  const int64_t big = std::max<int64_t>({m, (P.nb_max + 1) * P.nv, nnz, 1});
  L.sums = off;    off = align_up(off + 4 * (big / SCAN_CHUNK + 2));
  L.rowlist = off; off = align_up(off + 4 * (std::min(m, std::max<int64_t>(nnz, 1)) + P.m_b + 1));
  L.vbase = off;   off = align_up(off + 4 * (n + 1));
  L.pos = off;     off = align_up(off + 4 * (P.nb_max + 1) * P.nv);
  L.seg = off;     off = align_up(off + 4 * (P.nb_max * P.nv + 1));
  L.ent = off;     off = align_up(off + 8 * (nnz + 2));  // +2: 16-byte staging tail
  L.dflag = off;   off = align_up(off + 4 * P.nb_max);
  L.dlist = off;   off = align_up(off + 4 * std::max<int64_t>(P.nd_max, 1));
  L.dhdr = off;    off = align_up(off + (int64_t)sizeof(DenseHeader));
  L.dense = off;   off = align_up(off + 4 * P.nd_max * P.m_b * n);
  L.part = off;
  if (P.slices > 1 || P.nv != n)
    off = align_up(off + 4 * ((int64_t)P.splits * d * P.nv + (P.dense_pct ? d * n : 0)));
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


// ------------------------------------------------------------------ batch
struct BatchPlan {
  int variant = 0;
  std::vector<Plan> plans;
  std::vector<int64_t> rowlist, pos, ent, part;
  int64_t hdrs = 0, items = 0, work = 0, counters = 0, ridx_all = 0, seg_all = 0, sums = 0;
  int64_t total = 0;
  int64_t t_valid = 0, t_ridx = 0, t_m = 0, t_pos = 0, t_cnt = 0, t_seg = 0, t_nnz = 0, t_out = 0;
  int64_t units[3] = {0, 0, 0};
  size_t lds[3] = {0, 0, 0};
};

constexpr int kBatchUnitsPerSlot = 8;  // work units per persistent workgroup, for balance

sk_status batch_plan(int32_t count, const sk_csc* A, const int64_t* d, const int32_t* dist,
                     int32_t prec, const sk_tuning* tune, BatchPlan& B) {
  if (count < 1 || !A || !d || !dist) return SK_EINVAL;
  if (prec != SK_PREC_F32) return SK_EUNSUPPORTED;
  int64_t nmax = 0;
  for (int i = 0; i < count; ++i) {
    sk_status s = check_csc(&A[i]);
    if (s != SK_OK) return s;
    if (d[i] < 1 || dist[i] < 0 || dist[i] > 2) return SK_EINVAL;
    nmax = std::max(nmax, A[i].n);
  }
  B.variant = nmax <= 512 ? 5 : (nmax <= 2048 ? 0 : 1);
  B.plans.resize(count);
  double total_cost = 0.0;
  for (int i = 0; i < count; ++i) {
    const sk_tuning* t = tune ? &tune[i] : nullptr;
    if (!plan_for(A[i].m, A[i].n, A[i].nnz, d[i], dist[i], t, B.plans[i], B.variant, 0.0))
      return SK_EINVAL;
    total_cost += B.plans[i].cost;
  }
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
  const double unit = std::max(1.0, total_cost / ((double)cus * kBatchUnitsPerSlot));
  for (int i = 0; i < count; ++i) {
    const sk_tuning* t = tune ? &tune[i] : nullptr;
    if (!plan_for(A[i].m, A[i].n, A[i].nnz, d[i], dist[i], t, B.plans[i], B.variant, unit))
      return SK_EINVAL;
    const Plan& P = B.plans[i];
    if ((int64_t)(P.nb_max + 1) * A[i].n >= INT32_MAX) return SK_EUNSUPPORTED;
  }
  // layout: shared arrays first, then per-item regions
  int64_t off = 0;
  B.hdrs = off;     off = align_up(off + (int64_t)sizeof(Header) * count);
  B.items = off;    off = align_up(off + (int64_t)sizeof(BatchItem) * count);
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    const int64_t u = (int64_t)P.tiles * P.ncr * P.splits;
    B.units[dist[i]] += u;
    B.lds[dist[i]] = std::max(B.lds[dist[i]], P.lds);
    const int64_t m = A[i].m, n = A[i].n, nnz = A[i].nnz;
    B.t_valid += std::max<int64_t>(nnz, n + 1);
    B.t_ridx += m + 1;
    B.t_m += m;
    B.t_pos += (P.nb_max + 1) * n;
    B.t_cnt += P.nb_max * n;
    B.t_seg += P.nb_max * n + 1;
    B.t_nnz += nnz;
    if (P.slices > 1) B.t_out += d[i] * n;
  }
  const int64_t nunits = B.units[0] + B.units[1] + B.units[2];
  if (nunits >= INT32_MAX || B.t_ridx >= INT32_MAX || B.t_seg >= INT32_MAX) return SK_EUNSUPPORTED;
  B.work = off;     off = align_up(off + 8 * std::max<int64_t>(nunits, 1));
  B.counters = off; off = align_up(off + 4 * 4);
  B.ridx_all = off; off = align_up(off + 4 * (B.t_ridx + 1));
  B.seg_all = off;  off = align_up(off + 4 * (B.t_seg + 1));
  B.sums = off;     off = align_up(off + 4 * (std::max(B.t_ridx, B.t_seg) / SCAN_CHUNK + 2));
  B.rowlist.resize(count); B.pos.resize(count); B.ent.resize(count); B.part.resize(count);
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    const int64_t m = A[i].m, n = A[i].n, nnz = A[i].nnz;
    B.rowlist[i] = off; off = align_up(off + 4 * (std::min(m, std::max<int64_t>(nnz, 1)) + P.m_b + 1));
    B.pos[i] = off;     off = align_up(off + 4 * (P.nb_max + 1) * n);
    B.ent[i] = off;     off = align_up(off + 8 * (nnz + 2));
    B.part[i] = off;
    if (P.slices > 1) off = align_up(off + 4 * (int64_t)P.slices * d[i] * n);
  }
  B.total = off;
  return SK_OK;
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
  if ((int64_t)(P.nb_max + 1) * P.nv >= INT32_MAX) return SK_EUNSUPPORTED;
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
  int32_t* vbase = (int32_t*)(w + L.vbase);
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
  const int64_t nv = P.nv;
  const int64_t npos = (P.nb_max + 1) * nv;
  const int64_t nseg = P.nb_max * nv;
  if (nv != n) {
    // heavy columns become s_k interleaved virtual columns (entry t of
    // column k goes to virtual column vbase[k] + t mod s_k)
    hipLaunchKernelGGL(k_colsplit_count, dim3(blocks_for(n, 256)), dim3(256), 0, st, A->colptr,
                       n, nnz, nv - n, hdr, vbase);
    if ((s = scan_i32(vbase, n, sums, st)) != SK_OK) return s;
    hipLaunchKernelGGL(k_block_pos_v, dim3(blocks_for(npos, 256)), dim3(256), 0, st, A->colptr,
                       A->rowidx, n, nv, vbase, rowlist, P.m_b, P.nb_max, hdr, pos);
  } else {
    hipLaunchKernelGGL(k_block_pos, dim3(blocks_for(npos, 256)), dim3(256), 0, st, A->colptr,
                       A->rowidx, m, n, rowlist, P.m_b, P.nb_max, hdr, pos);
  }
  hipLaunchKernelGGL(k_block_cnt, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, pos, nv,
                     P.nb_max, hdr, seg);
  if ((s = scan_i32(seg, nseg, sums, st)) != SK_OK) return s;
  if (nnz > 0 && nv != n)
    hipLaunchKernelGGL(k_scatter_v, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, A->colptr,
                       A->rowidx, A->vals, A->vtype, n, nv, nnz, vbase, ridx, pos, seg, P.m_b,
                       P.ldS * 4, hdr, ent);
  else if (nnz > 0)
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, A->colptr,
                       A->rowidx, A->vals, A->vtype, n, nnz, ridx, pos, seg, P.m_b, P.ldS * 4,
                       hdr, ent);
  if ((s = launch_ok()) != SK_OK) return s;
  // a5 (selection): dense row blocks, densified
  if (P.dense_pct) {
    hipLaunchKernelGGL(k_dense_select, dim3(1), dim3(256), 0, st, seg, nv, n, P.m_b,
                       P.dense_pct, (int32_t)P.nd_max, hdr, dflag, dlist, dhdr);
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks_for(P.nd_max * P.m_b * n, 256 * 16)),
                       dim3(256), 0, st, dense, P.nd_max * P.m_b * n, 0.0f);
    hipLaunchKernelGGL(k_densify, dim3(blocks_for(P.nd_max * nv, 256)), dim3(256), 0, st, seg,
                       ent, nv, n, nv != n ? vbase : nullptr, P.m_b, P.ldS * 4, dlist, dhdr,
                       dense);
    if ((s = launch_ok()) != SK_OK) return s;
  }
  }

  // a3 + a4: S tiles and sparse accumulation
  const Variant& V = kVariants[P.variant];
  SketchParams K{};
  K.rowlist = rowlist; K.seg = seg; K.ent = ent; K.hdr = hdr;
  K.dflag = P.dense_pct ? dflag : nullptr;
  K.n = P.nv; K.d = d; K.row0 = row0; K.seed = seed;
  K.m_b = P.m_b; K.e_max = P.e_max; K.d_b = P.d_b; K.ldS = P.ldS; K.log2_cpr = P.log2_cpr;
  K.dt = P.dt; K.cg = P.cg; K.tiles = P.tiles; K.splits = P.splits;
  K.col_per_wg = P.col_per_wg;
  const bool staged = P.slices > 1 || P.nv != n;  // partials, then the reduction
  if (staged) { K.out = part; K.ld = d; K.split_stride = d * P.nv; }
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
    DP.out = part + (int64_t)P.splits * d * P.nv;
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
  if ((phases & 4) && staged)
    hipLaunchKernelGGL(k_reduce_virtual, dim3(blocks_for(d * n, 256)), dim3(256), 0, st, part,
                       P.splits, d, n, P.nv, P.nv != n ? vbase : nullptr,
                       P.dense_pct ? part + (int64_t)P.splits * d * P.nv : nullptr, Ahat, ld);
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

sk_status sk_sketch_batched_workspace(int32_t count, const sk_csc* A, const int64_t* d,
                                      const int32_t* dist, int32_t prec, const sk_tuning* tune,
                                      size_t* bytes) {
  if (!bytes) return SK_EINVAL;
  BatchPlan B;
  sk_status s = batch_plan(count, A, d, dist, prec, tune, B);
  if (s != SK_OK) return s;
  *bytes = (size_t)B.total;
  return SK_OK;
}

sk_status sk_sketch_batched(int32_t count, const sk_csc* A, const int64_t* d, const int32_t* dist,
                            const uint64_t* seed, int32_t prec, const sk_tuning* tune,
                            float* const* Ahat, const int64_t* ld, void* ws, size_t ws_bytes,
                            void* hip_stream) {
  if (!seed || !Ahat || !ld) return SK_EINVAL;
  BatchPlan B;
  sk_status s = batch_plan(count, A, d, dist, prec, tune, B);
  if (s != SK_OK) return s;
  for (int i = 0; i < count; ++i)
    if (!Ahat[i] || ld[i] < d[i]) return SK_EINVAL;
  if (!ws || ws_bytes < (size_t)B.total) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* w = (char*)ws;
  Header* hdrs = (Header*)(w + B.hdrs);
  BatchItem* d_items = (BatchItem*)(w + B.items);
  int2* d_work = (int2*)(w + B.work);
  int32_t* counters = (int32_t*)(w + B.counters);
  int32_t* ridx_all = (int32_t*)(w + B.ridx_all);
  int32_t* seg_all = (int32_t*)(w + B.seg_all);
  int32_t* sums = (int32_t*)(w + B.sums);
  const Variant& V = kVariants[B.variant];

  // item descriptors (host), copied to the workspace
  std::vector<BatchItem> items(count);
  int64_t o_valid = 0, o_ridx = 0, o_m = 0, o_pos = 0, o_cnt = 0, o_seg = 0, o_nnz = 0, o_out = 0;
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    BatchItem& I = items[i];
    std::memset(&I, 0, sizeof I);
    const int64_t m = A[i].m, n = A[i].n, nnz = A[i].nnz;
    I.m = m; I.n = n; I.nnz = nnz;
    I.colptr = A[i].colptr; I.rowidx = A[i].rowidx; I.vals = A[i].vals; I.vtype = A[i].vtype;
    I.slices = P.slices; I.Ahat = Ahat[i]; I.ld = ld[i]; I.nb_max = P.nb_max;
    I.ridx = ridx_all + o_ridx;
    I.pos = (int32_t*)(w + B.pos[i]);
    I.seg_region = seg_all + o_seg;
    I.part = (float*)(w + B.part[i]);
    I.o_valid = o_valid; o_valid += std::max<int64_t>(nnz, n + 1);
    I.o_ridx = o_ridx;   o_ridx += m + 1;
    I.o_m = o_m;         o_m += m;
    I.o_pos = o_pos;     o_pos += (P.nb_max + 1) * n;
    I.o_cnt = o_cnt;     o_cnt += P.nb_max * n;
    I.o_seg = o_seg;     o_seg += P.nb_max * n + 1;
    I.o_nnz = o_nnz;     o_nnz += nnz;
    I.o_out = o_out;     if (P.slices > 1) o_out += d[i] * n;
    SketchParams& K = I.P;
    K.rowlist = (int32_t*)(w + B.rowlist[i]);
    K.seg = I.seg_region;
    K.ent = (uint2*)(w + B.ent[i]);
    K.hdr = hdrs + i;
    K.dflag = nullptr;
    K.n = n; K.d = d[i]; K.row0 = 0; K.seed = seed[i];
    K.m_b = P.m_b; K.e_max = P.e_max; K.d_b = P.d_b; K.ldS = P.ldS; K.log2_cpr = P.log2_cpr;
    K.dt = P.dt; K.cg = P.cg; K.tiles = P.tiles; K.splits = P.splits; K.col_per_wg = P.col_per_wg;
    if (P.slices > 1) { K.out = I.part; K.ld = d[i]; K.split_stride = d[i] * n; }
    else { K.out = Ahat[i]; K.ld = ld[i]; K.split_stride = 0; }
  }
  // work list: grouped by distribution, longest units first (LPT)
  struct U { double cost; int32_t item, unit; int32_t dist; };
  std::vector<U> units;
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    const int32_t nu = P.tiles * P.ncr * P.splits;
    for (int32_t u = 0; u < nu; ++u) units.push_back({P.cost / nu, i, u, dist[i]});
  }
  std::stable_sort(units.begin(), units.end(), [](const U& a, const U& b) {
    if (a.dist != b.dist) return a.dist < b.dist;
    return a.cost > b.cost;
  });
  std::vector<int2> work(std::max<size_t>(units.size(), 1));
  for (size_t k = 0; k < units.size(); ++k) work[k] = make_int2(units[k].item, units[k].unit);
  // host vectors are staged by the runtime before these calls return
  if (hipMemcpyAsync(d_items, items.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return SK_EHIP;
  if (hipMemcpyAsync(d_work, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return SK_EHIP;

  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(count * (int64_t)sizeof(Header) / 4, 256)),
                     dim3(256), 0, st, (int32_t*)hdrs, count * (int64_t)sizeof(Header) / 4, 0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, counters, int64_t(4), 0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(B.t_ridx + 1, 256 * 8)), dim3(256), 0, st,
                     ridx_all, B.t_ridx + 1, 0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(B.t_seg + 1, 256 * 8)), dim3(256), 0, st,
                     seg_all, B.t_seg + 1, 0);
  // a1 + a2 for every item at once
  hipLaunchKernelGGL(k_batch_validate_mark, dim3(blocks_for(B.t_valid, 256)), dim3(256), 0, st,
                     d_items, count, B.t_valid);
  if ((s = scan_i32(ridx_all, B.t_ridx, sums, st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_batch_bases, dim3(blocks_for(count, 256)), dim3(256), 0, st, d_items, count,
                     0);
  hipLaunchKernelGGL(k_batch_rebase, dim3(blocks_for(B.t_ridx, 256)), dim3(256), 0, st, d_items,
                     count, B.t_ridx, 0);
  hipLaunchKernelGGL(k_batch_rowlist, dim3(blocks_for(B.t_m, 256)), dim3(256), 0, st, d_items,
                     count, B.t_m);
  hipLaunchKernelGGL(k_batch_block_pos, dim3(blocks_for(B.t_pos, 256)), dim3(256), 0, st, d_items,
                     count, B.t_pos);
  hipLaunchKernelGGL(k_batch_block_cnt, dim3(blocks_for(B.t_cnt, 256)), dim3(256), 0, st, d_items,
                     count, B.t_cnt);
  if ((s = scan_i32(seg_all, B.t_seg, sums, st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_batch_bases, dim3(blocks_for(count, 256)), dim3(256), 0, st, d_items, count,
                     1);
  hipLaunchKernelGGL(k_batch_rebase, dim3(blocks_for(B.t_seg, 256)), dim3(256), 0, st, d_items,
                     count, B.t_seg, 1);
  if (B.t_nnz > 0)
    hipLaunchKernelGGL(k_batch_scatter, dim3(blocks_for(B.t_nnz, 256)), dim3(256), 0, st, d_items,
                       count, B.t_nnz);
  if ((s = launch_ok()) != SK_OK) return s;
  // a7: one persistent launch per distribution present
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
  int64_t first = 0;
  for (int dd = 0; dd < 3; ++dd) {
    if (B.units[dd] == 0) continue;
    PersistentKernel kern = V.p[dd];
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)B.lds[dd]) != hipSuccess)
      return SK_EHIP;
    const int per_cu = V.wgs >= 1024 ? 1 : 2;
    const int64_t grid = std::min<int64_t>(B.units[dd], (int64_t)cus * per_cu);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(V.wgs), B.lds[dd], st, d_items,
                       d_work + first, (int)B.units[dd], counters + dd);
    if ((s = launch_ok()) != SK_OK) return s;
    first += B.units[dd];
  }
  // a6 for every item with split partials
  if (B.t_out > 0)
    hipLaunchKernelGGL(k_batch_reduce, dim3(blocks_for(B.t_out, 256)), dim3(256), 0, st, d_items,
                       count, B.t_out);
  return launch_ok();
}

sk_status sk_sketch_batched_plan(int32_t count, const sk_csc* A, const int64_t* d,
                                 const int32_t* dist, int32_t prec, const sk_tuning* tune,
                                 sk_tuning* chosen) {
  if (!chosen) return SK_EINVAL;
  BatchPlan B;
  sk_status s = batch_plan(count, A, d, dist, prec, tune, B);
  if (s != SK_OK) return s;
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    std::memset(&chosen[i], 0, sizeof chosen[i]);
    chosen[i].rows_per_block = P.m_b;
    chosen[i].splits = P.splits;
    chosen[i].variant = P.variant + 1;
    chosen[i].dense_min_pct = 101;
    chosen[i].tile_rows = P.d_b;
    chosen[i].col_split = 1;
  }
  return SK_OK;
}

sk_status sk_sketch_batched_status(const void* ws, int32_t count, void* hip_stream,
                                   int32_t* statuses) {
  if (!ws || count < 1 || !statuses) return SK_EINVAL;
  std::vector<Header> h(count);
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(h.data(), ws, sizeof(Header) * count, hipMemcpyDeviceToHost, st) != hipSuccess)
    return SK_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SK_EHIP;
  sk_status worst = SK_OK;
  for (int i = 0; i < count; ++i) {
    sk_status si = SK_OK;
    if (h[i].status & ST_COLPTR) si = SK_ECOLPTR;
    else if (h[i].status & ST_RANGE) si = SK_ERANGE;
    else if (h[i].status & ST_UNSORTED) si = SK_EUNSORTED;
    statuses[i] = si;
    if (si != SK_OK) worst = si;
  }
  return worst;
}

sk_status sk_autotune(const sk_csc* A, int64_t d, int32_t dist, sk_tuning* out) {
  if (!out) return SK_EINVAL;
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || dist < 0 || dist > 2) return SK_EINVAL;
  Plan P;
  if (!plan_for(A->m, A->n, A->nnz, d, dist, nullptr, P)) return SK_EINVAL;
  std::memset(out, 0, sizeof *out);
  out->rows_per_block = P.m_b;
  out->splits = P.splits;
  out->variant = P.variant + 1;
  out->dense_min_pct = P.dense_pct ? P.dense_pct : 101;
  out->tile_rows = P.d_b;
  out->col_split = P.nv != A->n ? 2 : 1;
  return SK_OK;
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

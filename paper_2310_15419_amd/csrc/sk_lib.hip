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
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "sk_balance.hpp"
#include "sk_batch.hpp"
#include "sk_colwise.hpp"
#include "sk_dense.hpp"
#include "sk_inspect.hpp"
#include "sk_mfma.hpp"
#include "sk_rng.hpp"
#include "sk_sap.hpp"
#include "sk_sketch.hpp"
#include "sk_svd.hpp"
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

using PersistentKernel = void (*)(const BatchOut*, const int2*, int, int32_t*);

struct Variant {
  int dl, q, cs, wgs;
  SketchKernel k[3];      // per distribution
  SketchKernel kf[3];     // per distribution, adding virtual columns in the kernel
  SketchKernel kc[3];     // per distribution, counting the generator calls
  PersistentKernel p[3];  // persistent (batched) form, per distribution (none: null)
};

#define SK_VARIANT(DL, Q, CS, WGS)                                                           \
  Variant {                                                                                  \
    DL, Q, CS, WGS,                                                                          \
        {k_sketch<DIST_RADEMACHER, DL, Q, CS, WGS>, k_sketch<DIST_UNIFORM, DL, Q, CS, WGS>,  \
         k_sketch<DIST_GAUSSIAN, DL, Q, CS, WGS>},                                           \
        {k_sketch<DIST_RADEMACHER, DL, Q, CS, WGS, true>,                                    \
         k_sketch<DIST_UNIFORM, DL, Q, CS, WGS, true>,                                       \
         k_sketch<DIST_GAUSSIAN, DL, Q, CS, WGS, true>},                                     \
        {k_sketch<DIST_RADEMACHER, DL, Q, CS, WGS, false, true>,                             \
         k_sketch<DIST_UNIFORM, DL, Q, CS, WGS, false, true>,                                \
         k_sketch<DIST_GAUSSIAN, DL, Q, CS, WGS, false, true>},                              \
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
    SK_VARIANT(4, 8, 16, 1024),  // 9: eight lanes per group (one 128-byte S window per read)
    SK_VARIANT(4, 4, 16, 512),   // 10: two workgroups per CU, 2048 columns each
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Generator-ablation forms of two kernel shapes (index 2: the shape of
// columns in the thousands; index 5: a few hundred columns): junk generator
// per distribution, S read from memory, and the (-1,1) scaled integers.
struct AblationKernels {
  int variant;
  SketchKernel junk[3];
  SketchKernel stored;
  SketchKernel scaled;
};

#define SK_ABLATION(V, DL, Q, CS, WGS)                                                        \
  AblationKernels {                                                                          \
    V,                                                                                       \
        {k_sketch<DIST_RADEMACHER, DL, Q, CS, WGS, false, false, GEN_JUNK>,                  \
         k_sketch<DIST_UNIFORM, DL, Q, CS, WGS, false, false, GEN_JUNK>,                     \
         k_sketch<DIST_GAUSSIAN, DL, Q, CS, WGS, false, false, GEN_JUNK>},                   \
        k_sketch<DIST_UNIFORM, DL, Q, CS, WGS, false, false, GEN_STORED>,                    \
        k_sketch<DIST_UNIFORM, DL, Q, CS, WGS, false, false, GEN_SCALED>                     \
  }

const AblationKernels kAblation[] = {SK_ABLATION(2, 8, 4, 8, 1024), SK_ABLATION(5, 4, 4, 2, 1024),
                                     SK_ABLATION(8, 4, 8, 16, 1024)};

// the ablation kernel of a plan's shape for a generator mode (null: none)
SketchKernel ablation_kernel(int variant, int gen, int dist) {
  for (const AblationKernels& a : kAblation) {
    if (a.variant != variant) continue;
    if (gen == GEN_JUNK) return a.junk[dist];
    if (gen == GEN_STORED) return a.stored;
    if (gen == GEN_SCALED && dist == DIST_UNIFORM) return a.scaled;
  }
  return nullptr;
}

struct Plan {
  int variant;  // index into kVariants
  int32_t m_b, e_max, d_b, ldS, dt, cg, tiles, splits, col_per_wg, ncr, log2_cpr;
  int64_t r_max;      // nonempty-row capacity
  int64_t ngroups;    // row groups of m_b rows
  int64_t nb_max;     // block capacity
  int64_t nv;         // virtual columns (== n without heavy-column splitting)
  size_t lds;
  int32_t dense_pct;  // densify at >= this % density; 0: no dense path
  int64_t kd_max;     // dense-row capacity
  int32_t slices;     // partial slices: splits (+1 for the dense path)
  double cost;        // autotuner's cost estimate (CU-cycles)
  int32_t row_bytes;  // row offset unit of the entries (S-tile row bytes; 1 on MFMA)
  int32_t mfma;       // 0: sparse FP32 kernel; MF_BF16 / MF_FP8: matrix-core kernel
  int32_t bal_sb;     // balanced row blocks: blocks per super-block (0: rows in order)
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
  // S rows per generator call (+-1: 128, one call per 128-row group a tile touches)
  const int rpc = dist == DIST_RADEMACHER ? std::min(128, P.d_b) : 4;
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
  if (tune && (tune->row_pad < 0 || tune->row_pad % 4)) return false;
  if (forced_variant >= 0 && tune && tune->variant > 0 && tune->variant - 1 != forced_variant)
    return false;
  if (v < 0) {
    // auto: enough columns per workgroup, then the most S rows per lane.
    // Between 512 and 2048 columns: four lanes per column group (shape 3)
    // when rows hold several nonzeros; pairs of lanes with half the columns
    // per group (shape 4) when they hold about one (nnz / nonempty rows < 2
    // for uniform positions): a block's column segments then hold zero or
    // one entry and a lane's per-column setup, not its multiply-adds, is the
    // cost, which shape 4 halves (measured on MI355X: the 4e6 x 1000
    // power-law matrix 4.4 against 5.3 ms, the 2e6 x 2000 one with ten
    // nonzeros per row 21.6 against 18.1 ms).  Rows of four or more
    // nonzeros get balanced row blocks (below) unless the caller keeps the
    // rows in order; with the lockstep padding then lower, eight lanes per
    // group and sixteen columns (shape 9) take the lead (the 2e6 x 2000
    // workload: 16.8 against 17.3 ms)
    const double r_uni = std::max(1.0, (double)m * -std::expm1(-(double)nnz / (double)m));
    const double per_uni = (double)nnz / r_uni;
    if (n <= 512) v = 5;
    else if (n <= 2048)
      v = per_uni < 2.0 ? 3 : (per_uni >= 4.0 && !(tune && tune->balance == 1) ? 8 : 2);
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
  // LDS per workgroup minus the static part and the staged segment bounds
  const int seg_bytes = (P.col_per_wg + 1) * 4;
  const int budget = (V.wgs >= 1024 ? kLdsPerCu : kLdsPerCu / 2) - 1024 - seg_bytes;
  const int64_t rmax = std::max<int64_t>(1, std::min(m, nnz));
  // entries per nonempty row if the positions were uniform (the expected
  // number of nonempty rows is m (1 - exp(-nnz / m)))
  const double r_est = std::max(1.0, (double)m * -std::expm1(-(double)nnz / (double)m));
  const double per_row = std::max(1.0, (double)nnz / r_est);

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
    Q.ldS = Q.d_b + (tune && tune->row_pad > 0 ? std::min(tune->row_pad, 64) : 0);
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
    auto e_of = [&](int64_t mb) {
      return (int64_t)(((budget - mb * Q.ldS * 4) / 8 - 2) & ~int64_t(1));
    };
    // leave room for the spread of a group's entry count around its mean, so
    // a typical group stays one block
    if (!(tune && tune->rows_per_block > 0))
      while (m_b > 64 && (double)e_of(m_b) < m_b * per_row + 3.0 * std::sqrt(m_b * per_row) + 2.0)
        m_b -= std::max<int64_t>(1, m_b / 64);
    Q.m_b = (int32_t)m_b;
    Q.e_max = (int32_t)e_of(m_b);
    if (Q.e_max < 2) continue;
    Q.lds = (size_t)m_b * Q.ldS * 4 + (size_t)(Q.e_max + 2) * 8 + (size_t)seg_bytes;
    Q.r_max = rmax;
    Q.ngroups = (rmax + m_b - 1) / m_b;
    // groups, plus at most two blocks per e_max entries from the entry cuts
    Q.nb_max = Q.ngroups + (2 * std::max<int64_t>(nnz, 1) + Q.e_max - 1) / Q.e_max + 1;
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
    // Few splits, in whole rounds of workgroups: every split writes a full
    // partial slice (d x columns FP32) that the reduction reads back, so
    // more splits cost traffic that grows with d n, not with the work
    // (measured on MI355X: 2-6 splits beat 16-24 on the 2e6 x 2000 uniform
    // and the 4e6 x 1000 power-law workloads; on a Table I shape with
    // d = 3n the 16 partial slices took most of the time).  The splits are
    // cost-balanced, so the workgroups run about equally long and a launch
    // of x rounds of resident workgroups (one of 1024 threads or two of 512
    // per CU) keeps x / ceil(x) of the chip busy: 375 workgroups on 256 CUs
    // measured 24 ms where 250 took 18.  Take the fewest splits (up to 16)
    // with that fraction >= 0.9, else the best one.  (MI355X's 256 CUs as a
    // constant: the plan, and so the summation order, follows from the
    // shape alone.)
    const int64_t wgs_now = (int64_t)P.tiles * ncr;
    const double resident = 256.0 * (V.wgs >= 1024 ? 1 : 2);
    splits = 1;
    double best_util = -1.0;
    for (int64_t sp = 1; sp <= 16; ++sp) {
      const double x = (double)(wgs_now * sp) / resident;
      const double util = x / std::ceil(x);
      if (util >= 0.9) { splits = sp; break; }
      if (util > best_util + 1e-9) { best_util = util; splits = sp; }
    }
  }
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, P.nb_max));
  P.splits = (int32_t)splits;
  // dense row blocks: only if some row could reach the threshold; capacity
  // in dense rows (a dense block of rb rows holds >= pct % of rb * n entries)
  int pct = tune && tune->dense_min_pct > 0 ? tune->dense_min_pct : kDenseAutoPct;
  P.dense_pct = 0;
  P.kd_max = 0;
  if (unit_cycles <= 0 && pct <= 100 && (double)nnz * 100.0 >= (double)pct * (double)n) {
    int64_t kd = (int64_t)((double)nnz * 100.0 / ((double)pct * (double)n));
    kd = std::min<int64_t>(kd, rmax);
    kd = std::min<int64_t>(kd, kDenseMaxBytes / (4 * n));
    if (kd > 0) {
      P.dense_pct = pct;
      P.kd_max = kd;
    }
  }
  P.slices = P.splits + (P.dense_pct ? 1 : 0);
  P.cost = best;
  P.row_bytes = P.ldS * 4;
  P.mfma = 0;
  // balanced row blocks (single sketches): where a block holds a few entries
  // per column, so that the lockstep of the column walk costs most (measured
  // on MI355X, the 2e6 x 2000 workload with ten nonzeros per row and 3.7
  // entries per (block, column): kernel 17.6 -> 15.2-15.5 ms with 16-32
  // blocks per super-block)
  P.bal_sb = 0;
  const int bal_mode = tune ? tune->balance : 0;
  if (unit_cycles <= 0 && bal_mode != 1 && n <= BAL_N_MAX && P.m_b >= 1) {
    const int sb = (int)std::min<int64_t>(BAL_SB_MAX, BAL_SBM_MAX / P.m_b);
    const double lam = (double)P.m_b * per_row / (double)n;  // entries per (block, column)
    const bool auto_on = n >= 512 && sb >= 8 && r_est >= 4.0 * sb * P.m_b && per_row >= 4.0 &&
                         lam >= 1.0 && lam <= 16.0;
    if (sb >= 2 && (bal_mode == 2 || (bal_mode == 0 && auto_on))) P.bal_sb = sb;
  }
  // with balanced blocks the splits' workgroups run about equally long, and
  // about three rounds of them beat one (measured on MI355X, the 2e6 x 2000
  // workload: 6 splits 16.17 ms per step, 4 splits 16.26, 2 splits 16.27):
  // the fewest splits from the whole-rounds choice on that span at least 2.5
  // rounds with a whole-round fraction >= 0.9
  if (P.bal_sb && !(tune && tune->splits > 0) && unit_cycles <= 0) {
    const double resident = 256.0 * (V.wgs >= 1024 ? 1 : 2);
    const int64_t units = (int64_t)P.tiles * P.ncr;
    for (int64_t sp = P.splits; sp <= 16 && sp <= P.nb_max; ++sp) {
      const double x = (double)(units * sp) / resident;
      if (x >= 2.5 && x / std::ceil(x) >= 0.9) {
        P.splits = (int32_t)sp;
        break;
      }
    }
    P.slices = P.splits + (P.dense_pct ? 1 : 0);
  }
  return true;
}

// --------------------------------------------------------- precision path
// +-1 S on the matrix cores in BF16 or FP8 when the matrix is dense enough
// for the dense contraction (d m n MACs at MFMA rate) to beat the sparse
// kernel (nnz d FMAs at the VALU rate, with its gather and padding costs).
// The threshold is a density in percent (the measured crossover of the two
// kernels on MI355X); dense_min_pct overrides it.
constexpr double kMfmaAutoPct[3] = {0.0, 1.5, 3.0};  // unused, BF16, FP8
// In a batch the matrix-core items share one launch with the others and pay
// no per-item launch, so the crossover is lower (measured on the 512-item
// workload: 1% beats 1.5% in BF16 and 3% in FP8).  Whole percents: a batch
// reports them as its items' tuning.
constexpr int kMfmaBatchPct[3] = {0, 1, 1};

int mfma_format(int64_t m, int64_t n, int64_t nnz, int dist, int prec, const sk_tuning* tune,
                bool batch = false) {
  if (prec == SK_PREC_F32 || dist != SK_RADEMACHER) return 0;
  const double pct = tune && tune->dense_min_pct > 0 ? (double)tune->dense_min_pct
                     : batch                          ? (double)kMfmaBatchPct[prec]
                                                      : kMfmaAutoPct[prec];
  if (pct > 100.0) return 0;
  const double density = 100.0 * (double)nnz / ((double)m * (double)n);
  if (density < pct) return 0;
  return prec == SK_PREC_BF16 ? MF_BF16 : MF_FP8;
}

bool plan_mfma(int64_t m, int64_t n, int64_t nnz, int64_t d, int fmt, const sk_tuning* tune,
               Plan& P, double unit_cycles = 0.0) {
  P = Plan{};
  P.variant = 0;
  P.mfma = fmt;
  P.m_b = MF_MB;
  P.e_max = 1 << 30;  // blocks are cut by rows only
  P.row_bytes = 1;
  P.d_b = MF_TM;
  P.ldS = 0;
  P.dt = 1;
  P.cg = 0;
  P.log2_cpr = 0;
  P.tiles = (int32_t)((d + MF_TM - 1) / MF_TM);
  P.ncr = (int32_t)((n + MF_TN - 1) / MF_TN);
  P.col_per_wg = MF_TN;
  P.nv = n;
  P.r_max = std::max<int64_t>(1, std::min(m, nnz));
  P.ngroups = (P.r_max + P.m_b - 1) / P.m_b;
  P.nb_max = P.ngroups + 1;
  P.lds = fmt == MF_BF16 ? sizeof(MfmaLds<MF_BF16>) : sizeof(MfmaLds<MF_FP8>);
  P.dense_pct = 0;
  P.kd_max = 0;
  // cost per unit and block in CU-cycles: the larger of the MFMA issue (four
  // accumulators per wave, 16 rows per instruction at 32 cycles, two waves
  // per SIMD; twice for FP8's hi + lo) and the next block's build that
  // overlaps it (the dense-tile clear and the scatter), plus the barrier
  const double R = (double)m * -std::expm1(-(double)nnz / (double)m);
  const double blocks = std::ceil(R / P.m_b);
  const double mf = (double)P.m_b / 16.0 * 4.0 * 2.0 * 32.0 * (fmt == MF_FP8 ? 2.0 : 1.0) / 4.0;
  const double build = 600.0 + (double)nnz / std::max(1.0, blocks) / P.ncr / 8.0;
  const double per_unit_block = std::max(mf, build) + 100.0;
  P.cost = blocks * per_unit_block * (double)P.tiles * P.ncr;
  int64_t splits;
  if (tune && tune->splits > 0) {
    splits = tune->splits;
  } else if (unit_cycles > 0) {
    splits = (int64_t)std::ceil(P.cost / ((double)P.tiles * P.ncr * unit_cycles));
  } else {
    const int64_t units = (int64_t)P.tiles * P.ncr;
    splits = (2 * 256 * 2 + units - 1) / units;  // about two rounds of two units per CU
    splits = std::min<int64_t>(splits, 64);
  }
  P.splits = (int32_t)std::max<int64_t>(1, std::min<int64_t>(splits, P.nb_max));
  P.slices = P.splits;
  return true;
}

// Predicted time of the Algorithm 3 loop-order kernel (sk_colwise.hpp), in
// microseconds: every nonzero pays, per tile of 64 DL rows, one lane's
// generator call(s), transform and DL multiply-adds (measured issue costs on
// MI355X: a Philox4x32-10 call about 48 full-rate slots, the (-1,1)
// transform about 2 per value, a Gaussian call with Box-Muller about 180),
// spread over the 1024 SIMDs; fewer waves than four per SIMD leave the
// dependent generator chains exposed.  Columns are taken as balanced (the
// plan sees only the shape).
double kji_time_us(int64_t n, int64_t nnz, int64_t d, int dist) {
  const int dl = dist == DIST_RADEMACHER ? 32 : 4;
  const double per_entry = dist == DIST_RADEMACHER ? 48.0 + 32.0 * 3.0
                           : dist == DIST_UNIFORM  ? 48.0 + 4.0 * 2.2 + 8.0
                                                   : 180.0 + 8.0;
  const double tiles = std::ceil((double)d / (64.0 * dl));
  const double clk = (double)nnz * tiles * per_entry * 4.0 / 1024.0;  // per SIMD
  const double waves = std::min<double>((double)n, std::max(1.0, (double)nnz)) * tiles;
  const double eff = std::min(1.0, waves / 4096.0);
  return clk / eff / 2400.0 + 5.0;
}

// Predicted time of the S-tile kernel's plan: its cost model (CU-cycles on
// 256 CUs at 2.4 GHz) times a factor fitted to measured runs, plus the fixed
// cost of the validation, inspector and reduction launches (measured
// 0.11-0.15 ms on small inputs).  The model counts issue slots; the column
// walk's LDS bank conflicts and the lockstep padding it leaves out make the
// measured time 1.7-2.1x the count on matrices with uniform nonzero
// positions (the Table I stand-ins, Table VI's B and the 2e6 x 2000
// uniform case), hence the factor 2.
constexpr double kTileCostFactor = 2.0;
constexpr double kTileFixedUs = 150.0;
double tile_time_us(const Plan& P) {
  return kTileCostFactor * P.cost / (256.0 * 2400.0) + kTileFixedUs;
}

// the plan a request runs with: the matrix-core path or the sparse kernel
bool plan_any(int64_t m, int64_t n, int64_t nnz, int64_t d, int dist, int prec,
              const sk_tuning* tune, Plan& P, int forced_variant = -1, double unit_cycles = 0.0,
              bool batch = false) {
  const int fmt = mfma_format(m, n, nnz, dist, prec, tune, batch);
  if (fmt) return plan_mfma(m, n, nnz, d, fmt, tune, P, unit_cycles);
  return plan_for(m, n, nnz, d, dist, tune, P, forced_variant, unit_cycles);
}

// Workspace of one sketch.  The header sits at offset 0 (the status call
// reads it there).
// partial row counts of an item with several column slabs (ints)
int64_t rpart_ints(int64_t m, int64_t n) {
  const int64_t slabs = rt_slabs(n);
  return slabs > 1 ? (m + RT_ROWS - 1) / RT_ROWS * slabs * RT_ROWS : 0;
}

struct Layout {
  int64_t rpart;
  int64_t hdr, item, ridx, rcnt, rowlist, rowcnt, bfl, bstart, vbase, pos, seg, ent, bcost, sums,
      rowinfo;
  int64_t dflag, dlist, doff, dhdr, drows, dense, part, total;
  int64_t bal_rowoff, bal_ccol, bal_newidx, bal_orig, bal_cnt2, bal_rowidx, bal_vals;
};

int64_t scan_sums_len(int64_t longest) { return longest / SCAN_CHUNK + 2; }

Layout layout_for(int64_t m, int64_t n, int64_t nnz, int64_t d, const Plan& P) {
  Layout L{};
  int64_t off = 0;
  const int64_t nd_cap = std::max<int64_t>(1, std::min(P.nb_max, P.kd_max));
  L.hdr = off;     off = align_up(off + (int64_t)sizeof(Header));
  L.item = off;    off = align_up(off + (int64_t)sizeof(Item));
  // scanned arrays hold one more element: the scan's grand total
  L.ridx = off;    off = align_up(off + 4 * (m + 2));
  L.rcnt = off;    off = align_up(off + 4 * m);
  L.rowlist = off; off = align_up(off + 4 * (P.r_max + P.m_b + 1));
  L.rowcnt = off;  off = align_up(off + 4 * P.r_max);
  L.bfl = off;     off = align_up(off + 4 * (P.r_max + 2));
  L.bstart = off;  off = align_up(off + 4 * (P.nb_max + 1));
  L.vbase = off;   if (P.nv != n) off = align_up(off + 4 * (n + 2));
  L.pos = off;     off = align_up(off + 4 * (P.nb_max + 1) * P.nv);
  L.seg = off;     off = align_up(off + 4 * (P.nb_max * P.nv + 2));
  L.ent = off;     off = align_up(off + 8 * (nnz + 2));  // +2: 16-byte staging tail
  L.bcost = off;   off = align_up(off + 4 * (P.nb_max + 2));
  L.rowinfo = off; off = align_up(off + 8 * m);
  L.rpart = off;   off = align_up(off + 4 * rpart_ints(m, n));
  const int64_t longest = std::max<int64_t>({m + 1, P.r_max + 1, n + 1, P.nb_max * P.nv + 1});
  L.sums = off;    off = align_up(off + 4 * scan_sums_len(longest));
  L.dflag = off;   off = align_up(off + 4 * P.nb_max);
  L.dlist = off;   off = align_up(off + 4 * nd_cap);
  L.doff = off;    off = align_up(off + 4 * nd_cap);
  L.dhdr = off;    off = align_up(off + (int64_t)sizeof(DenseHeader));
  L.drows = off;   off = align_up(off + 4 * std::max<int64_t>(P.kd_max, 1));
  L.dense = off;   off = align_up(off + 4 * P.kd_max * n);
  if (P.bal_sb) {  // balanced row blocks: the row pattern, the renumbering and A'
    L.bal_rowoff = off; off = align_up(off + 4 * (P.r_max + 2));
    L.bal_ccol = off;   off = align_up(off + 2 * std::max<int64_t>(nnz, 1));
    L.bal_newidx = off; off = align_up(off + 4 * m);
    L.bal_orig = off;   off = align_up(off + 4 * P.r_max);
    L.bal_cnt2 = off;   off = align_up(off + 4 * P.r_max);
    L.bal_rowidx = off; off = align_up(off + 4 * std::max<int64_t>(nnz, 1));
    L.bal_vals = off;   off = align_up(off + 4 * std::max<int64_t>(nnz, 1));
  }
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

// ------------------------------------------------- kernel choice and cache
enum { KERNEL_AUTO = 0, KERNEL_TILE = 1, KERNEL_KJI = 2 };

// The model takes the Algorithm 3 kernel only when it predicts it twice as
// fast: the model sees the shape alone and takes the nonzero positions as
// uniform, while structure it cannot see (most nonzeros in a few rows, as in
// Table VI's A or a dense row block) gives the S-tile kernel reuse of S
// that the estimate misses (measured: 2x on A, 1.5x on a 4e6 x 1000 matrix
// with a dense 2000-row block).  The measured tuner decides the rest.
constexpr double kKjiMargin = 2.0;

// any field that only the S-tile kernel has
bool tile_fields_set(const sk_tuning* t) {
  return t && (t->rows_per_block || t->splits || t->variant || t->dense_min_pct || t->phases ||
               t->tile_rows || t->col_split || t->row_pad || t->count_rng || t->rng_mode ||
               t->balance);
}

// KERNEL_TILE or KERNEL_KJI for a request (FP32 only for the latter); an
// out-of-range tune->kernel is returned as is (the caller rejects it)
int choose_kernel(const sk_csc* A, int64_t d, int dist, int prec, const sk_tuning* tune) {
  if (tune && tune->kernel != KERNEL_AUTO) return tune->kernel;
  if (prec != SK_PREC_F32 || tile_fields_set(tune)) return KERNEL_TILE;
  Plan P;
  if (!plan_for(A->m, A->n, A->nnz, d, dist, tune, P)) return KERNEL_TILE;
  return kji_time_us(A->n, A->nnz, d, dist) * kKjiMargin < tile_time_us(P) ? KERNEL_KJI
                                                                              : KERNEL_TILE;
}

// Plan cache: the tuning sk_autotune_measure found best, per shape class
// (distribution, precision and the half-octave classes of m, n, nnz and d).
// The only process-wide mutable state besides the no-allocation scratch
// array; guarded by one mutex.
struct ShapeKey {
  int32_t dist, prec, m, n, nnz, d;
  bool operator<(const ShapeKey& o) const {
    return std::tie(dist, prec, m, n, nnz, d) < std::tie(o.dist, o.prec, o.m, o.n, o.nnz, o.d);
  }
};

int32_t size_class(int64_t v) {
  return (int32_t)std::lround(2.0 * std::log2((double)std::max<int64_t>(v, 1)));
}

ShapeKey shape_key(const sk_csc* A, int64_t d, int dist, int prec) {
  return ShapeKey{dist, prec, size_class(A->m), size_class(A->n), size_class(A->nnz),
                  size_class(d)};
}

std::mutex g_plan_mu;
std::map<ShapeKey, sk_tuning> g_plans;

// The tuning a request runs with: the caller's if given, else the cached one
// of its shape class, else none (the model's choice).  A cached entry holds
// only the searched fields (kernel, kernel shape, splits), so it plans for
// any matrix of the class.
const sk_tuning* effective_tuning(const sk_csc* A, int64_t d, int dist, int prec,
                                  const sk_tuning* tune, sk_tuning& buf) {
  if (tune) return tune;
  std::lock_guard<std::mutex> g(g_plan_mu);
  if (g_plans.empty()) return nullptr;
  const auto it = g_plans.find(shape_key(A, d, dist, prec));
  if (it == g_plans.end()) return nullptr;
  buf = it->second;
  return &buf;
}

// Workspace of the Algorithm 3 kernel: the validation record, the chunk
// bookkeeping of heavy columns and their partial sums (8 bytes each, so one
// layout serves the FP32 and the FP64 form).  C, the chunk length, is the
// smallest power of two from 512 on that keeps the partials (at most
// 2 nnz / C chunks of d values) within kColwisePartBytes.
constexpr int64_t kColwisePartBytes = int64_t(256) << 20;

struct ColwiseLayout {
  int64_t hdr, item, cb, hb, hk, hcol, sums, part, total;
  int64_t chunk, chunks_max, heavy_max, slots_max;
};

ColwiseLayout colwise_layout(int64_t n, int64_t nnz, int64_t d) {
  ColwiseLayout L{};
  int64_t C = 512;
  while (2 * ((nnz + C - 1) / C) * d * 8 > kColwisePartBytes && C < (int64_t(1) << 30)) C *= 2;
  L.chunk = C;
  L.chunks_max = n + (nnz + C - 1) / C;  // every column one chunk, heavy ones ceil(len / C)
  L.heavy_max = nnz / C + 1;             // a heavy column has more than C nonzeros
  L.slots_max = 2 * ((nnz + C - 1) / C) + 1;
  int64_t off = 0;
  L.hdr = off;   off = align_up(off + (int64_t)sizeof(Header));
  L.item = off;  off = align_up(off + (int64_t)sizeof(Item));
  L.cb = off;    off = align_up(off + 4 * (n + 2));
  L.hb = off;    off = align_up(off + 4 * (n + 2));
  L.hk = off;    off = align_up(off + 4 * (n + 2));
  L.hcol = off;  off = align_up(off + 4 * (L.heavy_max + 1));
  L.sums = off;  off = align_up(off + 4 * scan_sums_len(n + 1));
  L.part = off;  off = align_up(off + 8 * L.slots_max * d);
  L.total = off;
  return L;
}

size_t colwise_bytes(const sk_csc* A, int64_t d) {
  return (size_t)colwise_layout(A->n, A->nnz, d).total;
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
  if (nchunks <= 4) {  // short: one workgroup scans it in place (one launch, not three)
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, st, a, count, a + count);
    return launch_ok();
  }
  const bool vec = ((uintptr_t)a & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(k_scan_reduce<true>, dim3((unsigned)nchunks), dim3(SCAN_THREADS), 0, st, a,
                       count, sums);
  else
    hipLaunchKernelGGL(k_scan_reduce<false>, dim3((unsigned)nchunks), dim3(SCAN_THREADS), 0, st,
                       a, count, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, st, sums, nchunks, a + count);
  if (vec)
    hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)nchunks), dim3(SCAN_THREADS), 0, st, a,
                       count, sums);
  else
    hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)nchunks), dim3(SCAN_THREADS), 0, st, a,
                       count, sums);
  return launch_ok();
}


// ------------------------------------------------------------- inspector
// Flattened index-space sizes of a batch of items (a single sketch is a
// batch of one), and the concatenated arrays the per-item scans run over.
struct InspectSizes {
  int64_t valid = 0, ridx = 0, m = 0, grp = 0, bfl = 0, rmax = 0, col = 0, vb = 0, pos = 0,
          cnt = 0, seg = 0, nnz = 0, blk = 0, rt = 0;
  bool slabs = false;  // some item counts its rows in several column slabs
};

// offsets of item I in each index space; sizes accumulate into Z
void item_offsets(Item& I, InspectSizes& Z) {
  I.o_valid = Z.valid; Z.valid += std::max<int64_t>(I.nnz, I.n + 1);
  I.o_ridx = Z.ridx;   Z.ridx += I.m + 1;
  I.o_m = Z.m;         Z.m += I.m;
  I.o_grp = Z.grp;     Z.grp += (I.r_max + I.m_b - 1) / I.m_b;
  I.o_bfl = Z.bfl;     Z.bfl += I.r_max + 1;
  I.o_rmax = Z.rmax;   Z.rmax += I.r_max;
  I.o_col = Z.col;     Z.col += I.n;
  I.o_vb = Z.vb;       if (I.vbase) Z.vb += I.n + 1;
  I.o_pos = Z.pos;     Z.pos += (I.nb_max + I.bp_chunk) / I.bp_chunk * I.nv;
  I.o_cnt = Z.cnt;     Z.cnt += I.nb_max * I.nv;
  I.o_seg = Z.seg;     Z.seg += I.nb_max * I.nv + 1;
  I.o_nnz = Z.nnz;     Z.nnz += I.nnz;
  I.o_blk = Z.blk;     Z.blk += I.nb_max + 1;
  I.o_rt = Z.rt;       Z.rt += (I.m + RT_ROWS - 1) / RT_ROWS * rt_slabs(I.n);
  if (rt_slabs(I.n) > 1) Z.slabs = true;
}

struct InspectArrays {
  int32_t* ridx;   // Z.ridx (+1 for the scan total)
  int32_t* rcnt;   // Z.m
  int32_t* bfl;    // Z.bfl (+1)
  int32_t* vbase;  // Z.vb (+1), may be null when no item splits
  int32_t* seg;    // Z.seg (+1)
  int32_t* bcost;  // Z.blk (+1)
  int32_t* sums;   // scan_sums_len(longest)
};

template <int64_t Item::*F, class Op>
void launch_items(Item* it, int count, int64_t total, hipStream_t st) {
  if (total <= 0) return;
  if (count == 1) {
    hipLaunchKernelGGL((k_items<F, Op, 1>), dim3(blocks_for(total, KI_THREADS)), dim3(KI_THREADS),
                       0, st, it, count, total);
  } else {
    constexpr int per = per_thread<Op>::value;
    hipLaunchKernelGGL((k_items<F, Op, per>), dim3(blocks_for(total, KI_THREADS * per)),
                       dim3(KI_THREADS), 0, st, it, count, total);
  }
}

template <int64_t Item::*F, class Op>
void launch_items_cols(Item* it, int count, int64_t total, hipStream_t st) {
  if (total > 0)
    hipLaunchKernelGGL((k_items_cols<F, Op>), dim3(blocks_for(total, IC_THREADS * IC_PER)),
                       dim3(IC_THREADS), 0, st, it, count, total);
}

// exclusive scan of a concatenated array, then per-region rebasing
template <int WHICH, int64_t Item::*F>
sk_status scan_regions(int32_t* all, int64_t total, Item* it, int count, int32_t* sums,
                       hipStream_t st) {
  sk_status s = scan_i32(all, total, sums, st);
  if (s != SK_OK || count == 1) return s;
  hipLaunchKernelGGL(k_item_bases, dim3(blocks_for(count, 256)), dim3(256), 0, st, it, count, WHICH);
  launch_items<F, OpRebase<WHICH>>(it, count, total, st);
  return launch_ok();
}

// a1 + a2 for every item: validation, nonempty rows, entry-balanced row
// blocks, heavy-column splitting, segments and the entries' gather.  The
// items' headers must be zero.
// a1 and the nonempty rows
sk_status inspect_rows(Item* it, int count, const InspectSizes& Z, const InspectArrays& W,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(Z.ridx + 1, 256 * 8)), dim3(256), 0, st,
                     W.ridx, Z.ridx + 1, 0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(Z.bfl + 1, 256 * 8)), dim3(256), 0, st,
                     W.bfl, Z.bfl + 1, 0);
  launch_items_cols<&Item::o_valid, OpValidate>(it, count, Z.valid, st);
  if (Z.rt > 0)
    hipLaunchKernelGGL(k_row_counts, dim3((unsigned)Z.rt), dim3(1024), 0, st, it, count, Z.rt);
  if (Z.slabs) launch_items<&Item::o_m, OpRowReduce>(it, count, Z.m, st);
  sk_status s;
  if ((s = scan_regions<SCAN_RIDX, &Item::o_ridx>(W.ridx, Z.ridx, it, count, W.sums, st)) != SK_OK)
    return s;
  launch_items<&Item::o_m, OpRowlist>(it, count, Z.m, st);
  return launch_ok();
}

// the row blocks, segments and entries after inspect_rows; `gather`: the
// entries by (block, column) segment (short segments), else by entry
sk_status inspect_blocks(Item* it, int count, const InspectSizes& Z, const InspectArrays& W,
                         hipStream_t st, bool gather) {
  sk_status s;
  hipLaunchKernelGGL(k_partition, dim3(blocks_for(Z.grp * 64, 256)), dim3(256), 0, st, it, count,
                     Z.grp);
  if ((s = scan_regions<SCAN_BFL, &Item::o_bfl>(W.bfl, Z.bfl, it, count, W.sums, st)) != SK_OK)
    return s;
  launch_items<&Item::o_rmax, OpBstart>(it, count, Z.rmax, st);
  if (Z.vb > 0) {
    launch_items<&Item::o_col, OpColsplit>(it, count, Z.col, st);
    if ((s = scan_regions<SCAN_VBASE, &Item::o_vb>(W.vbase, Z.vb, it, count, W.sums, st)) !=
        SK_OK)
      return s;
  }
  launch_items<&Item::o_pos, OpBlockPos>(it, count, Z.pos, st);
  launch_items<&Item::o_cnt, OpBlockCnt>(it, count, Z.cnt, st);
  if ((s = scan_regions<SCAN_SEG, &Item::o_seg>(W.seg, Z.seg, it, count, W.sums, st)) != SK_OK)
    return s;
  launch_items<&Item::o_m, OpRowInfo>(it, count, Z.m, st);
  if (gather) launch_items<&Item::o_cnt, OpGather>(it, count, Z.cnt, st);
  else launch_items_cols<&Item::o_nnz, OpScatter>(it, count, Z.nnz, st);
  return launch_ok();
}

sk_status run_inspector(Item* it, int count, const InspectSizes& Z, const InspectArrays& W,
                        hipStream_t st, bool gather = false) {
  sk_status s = inspect_rows(it, count, Z, W, st);
  return s != SK_OK ? s : inspect_blocks(it, count, Z, W, st, gather);
}

// The entries' gather walks a (block, column) segment in one thread: it pays
// where segments are short (the plain-scale workload: 3.7 entries, 0.46 ->
// 0.31 ms), not where few blocks hold long ones (small items: one thread
// per entry is faster).  Estimated from the plan: entries per (row group,
// column).
bool gather_pays(const Plan& P, int64_t nnz) {
  return (double)nnz <= 8.0 * (double)std::max<int64_t>(P.ngroups, 1) * (double)P.nv;
}

// block costs and their prefix (after the dense selection, if any)
sk_status run_block_costs(Item* it, int count, const InspectSizes& Z, const InspectArrays& W,
                          hipStream_t st) {
  launch_items<&Item::o_blk, OpBlockCost>(it, count, Z.blk, st);
  return scan_regions<SCAN_COST, &Item::o_blk>(W.bcost, Z.blk, it, count, W.sums, st);
}

// the device copy of a single item, written from a kernel argument (no host
// staging of the descriptor)
__global__ void k_put_item(Item I, Item* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = I;
}

Item make_item(const sk_csc* A, const Plan& P, int dist) {
  Item I;
  std::memset(&I, 0, sizeof I);
  I.m = A->m; I.n = A->n; I.nnz = A->nnz;
  I.colptr = A->colptr; I.rowidx = A->rowidx; I.vals = A->vals; I.vtype = A->vtype;
  I.m_b = P.m_b; I.e_cap = P.e_max; I.row_bytes = P.row_bytes;
  // block-position search: blocks per thread from the expected entries per
  // (column, block) (measured: 16 at ~3.7 entries, 8 at ~4-6, 1-2 at ~14)
  {
    const double per = (double)A->nnz / std::max(1.0, (double)A->n * (double)P.ngroups);
    I.bp_chunk = per <= 4.0 ? 16 : (per <= 6.0 ? 8 : (per <= 24.0 ? 2 : 1));
  }
  I.nv = P.nv; I.nb_max = P.nb_max; I.r_max = P.r_max;
  if (P.mfma) {  // blocks of equal height; the cost follows the rows
    static_assert((MF_TN & (MF_TN - 1)) == 0, "the tile-column tag is taken by a mask");
    I.col_tag = MF_TN;
    I.w_row = 16;
    I.w_ent = 1;
    I.w_blk = 16 * 300;
    I.cost_shift = 0;
    const double bound = (double)P.r_max * I.w_row + (double)A->nnz * I.w_ent +
                         (double)(P.nb_max + 1) * I.w_blk;
    while (bound / (double)(int64_t(1) << I.cost_shift) > (double)(1 << 29)) ++I.cost_shift;
    return I;
  }
  // block cost weights in 1/16 wave instructions per tile: S generation per
  // row, multiply-adds (with the lockstep padding) and staging per entry, a
  // fixed cost per block
  const Variant& V = kVariants[P.variant];
  const int rpc = dist == DIST_RADEMACHER ? std::min(128, P.d_b) : 4;
  const double call_ops = dist == DIST_GAUSSIAN ? 200.0 : (dist == DIST_UNIFORM ? 75.0 : 70.0);
  I.w_row = (int32_t)std::max(1.0, std::round(16.0 * (P.d_b / rpc) * call_ops / 64.0));
  I.w_ent = (int32_t)std::max(
      1.0, std::round(16.0 * (P.d_b * (V.dl + 3.0) / V.dl * 2.0 / 64.0 + 0.25)));
  I.w_blk = 16 * 400;
  const double bound = (double)P.r_max * I.w_row + (double)A->nnz * I.w_ent +
                       (double)(P.nb_max + 1) * I.w_blk;
  I.cost_shift = 0;
  while (bound / (double)(int64_t(1) << I.cost_shift) > (double)(1 << 29)) ++I.cost_shift;
  return I;
}

SketchParams make_params(const Plan& P, const Item& I, int64_t d, int64_t row0, uint64_t seed) {
  SketchParams K{};
  K.rowlist = I.rowlist; K.bstart = I.bstart; K.seg = I.seg; K.ent = I.ent; K.hdr = I.hdr;
  K.bcost = I.bcost;
  K.dflag = nullptr;
  K.n = P.nv; K.d = d; K.row0 = row0; K.seed = seed;
  K.m_b = P.m_b; K.e_max = P.e_max; K.d_b = P.d_b; K.ldS = P.ldS; K.log2_cpr = P.log2_cpr;
  K.dt = P.dt; K.cg = P.cg; K.tiles = P.tiles; K.splits = P.splits;
  K.col_per_wg = P.col_per_wg;
  K.split_slow = P.bal_sb ? 0 : 1;
  K.vbase = nullptr;
  K.nreal = P.nv;
  return K;
}

// The sparse kernel adds virtual columns itself when they all lie in one
// column range, one row of every lane's S rows fits the LDS at once, and
// the split is substantial (at least n/4 extra virtual columns: heavy
// columns with many pieces make the separate reduction's longest sums; with
// few pieces that reduction is cheap and the kernel's folded writes, one
// row of DL per pass, cost more)
bool folds_virtual(const Plan& P, int64_t n) {
  if (P.mfma || P.nv <= n || P.nv - n < (n + 3) / 4 || P.ncr != 1) return false;
  const Variant& V = kVariants[P.variant];
  return (int64_t)(P.d_b / V.dl) * P.col_per_wg * 4 <= (int64_t)P.lds;
}

// ------------------------------------------------------------------ batch
struct BatchPlan {
  int variant = 0;
  std::vector<Plan> plans;
  std::vector<int64_t> rowlist, rowcnt, bstart, pos, ent, part, rowinfo, rpart;
  InspectSizes Z;
  int64_t hdrs = 0, items = 0, outs = 0, work = 0, counters = 0;
  int64_t ridx_all = 0, rcnt_all = 0, bfl_all = 0, seg_all = 0, bcost_all = 0, sums = 0;
  int64_t total = 0, t_out = 0;
  // work-unit kinds: 0..2 the sparse kernel per distribution, 3 / 4 the
  // matrix-core kernel in BF16 / FP8
  int64_t units[5] = {0, 0, 0, 0, 0};
  size_t lds[5] = {0, 0, 0, 0, 0};
};

int unit_kind(const Plan& P, int dist) { return P.mfma ? 2 + P.mfma : dist; }

// compute units of the caller's current device (256 on MI355X when it cannot
// be queried, e.g. planning on a host without a GPU)
int current_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return 256;
  return cus;
}

constexpr int kBatchUnitsPerSlot = 8;  // work units per persistent workgroup, for balance

sk_status batch_plan(int32_t count, const sk_csc* A, const int64_t* d, const int32_t* dist,
                     int32_t prec, const sk_tuning* tune, BatchPlan& B) {
  if (count < 1 || !A || !d || !dist) return SK_EINVAL;
  if (prec < 0 || prec > 2) return SK_EINVAL;
  int64_t nmax = 0;
  for (int i = 0; i < count; ++i) {
    sk_status s = check_csc(&A[i]);
    if (s != SK_OK) return s;
    if (d[i] < 1 || dist[i] < 0 || dist[i] > 2) return SK_EINVAL;
    if (prec != SK_PREC_F32 && dist[i] != SK_RADEMACHER) return SK_EUNSUPPORTED;
    nmax = std::max(nmax, A[i].n);
  }
  B.variant = nmax <= 512 ? 5 : (nmax <= 2048 ? 2 : 1);
  B.plans.resize(count);
  double total_cost = 0.0;
  for (int i = 0; i < count; ++i) {
    const sk_tuning* t = tune ? &tune[i] : nullptr;
    if (!plan_any(A[i].m, A[i].n, A[i].nnz, d[i], dist[i], prec, t, B.plans[i], B.variant, 0.0,
                  true))
      return SK_EINVAL;
    total_cost += B.plans[i].cost;
  }
  const int cus = current_cus();
  const double unit = std::max(1.0, total_cost / ((double)cus * kBatchUnitsPerSlot));
  for (int i = 0; i < count; ++i) {
    const sk_tuning* t = tune ? &tune[i] : nullptr;
    if (!plan_any(A[i].m, A[i].n, A[i].nnz, d[i], dist[i], prec, t, B.plans[i], B.variant, unit,
                  true))
      return SK_EINVAL;
    const Plan& P = B.plans[i];
    if ((int64_t)(P.nb_max + 1) * P.nv >= INT32_MAX) return SK_EUNSUPPORTED;
  }
  // layout: headers first (the status call reads them there), shared arrays,
  // then per-item regions
  int64_t off = 0;
  B.hdrs = off;     off = align_up(off + (int64_t)sizeof(Header) * count);
  B.items = off;    off = align_up(off + (int64_t)sizeof(Item) * count);
  B.outs = off;     off = align_up(off + (int64_t)sizeof(BatchOut) * count);
  B.Z = InspectSizes{};
  B.t_out = 0;
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    Item I = make_item(&A[i], P, dist[i]);
    item_offsets(I, B.Z);
    const int kind = unit_kind(P, dist[i]);
    B.units[kind] += (int64_t)P.tiles * P.ncr * P.splits;
    B.lds[kind] = std::max(B.lds[kind], P.lds);
    if (P.slices > 1) B.t_out += d[i] * A[i].n;
  }
  const InspectSizes& Z = B.Z;
  const int64_t nunits = B.units[0] + B.units[1] + B.units[2] + B.units[3] + B.units[4];
  if (nunits >= INT32_MAX || Z.ridx >= INT32_MAX || Z.seg >= INT32_MAX || Z.bfl >= INT32_MAX)
    return SK_EUNSUPPORTED;
  B.work = off;     off = align_up(off + 8 * std::max<int64_t>(nunits, 1));
  B.counters = off; off = align_up(off + 4 * 8);
  B.ridx_all = off; off = align_up(off + 4 * (Z.ridx + 1));
  B.rcnt_all = off; off = align_up(off + 4 * std::max<int64_t>(Z.m, 1));
  B.bfl_all = off;  off = align_up(off + 4 * (Z.bfl + 1));
  B.seg_all = off;  off = align_up(off + 4 * (Z.seg + 1));
  B.bcost_all = off; off = align_up(off + 4 * (Z.blk + 1));
  B.sums = off;
  off = align_up(off + 4 * scan_sums_len(std::max({Z.ridx, Z.bfl, Z.seg, Z.blk})));
  B.rowlist.resize(count); B.rowcnt.resize(count); B.bstart.resize(count);
  B.pos.resize(count); B.ent.resize(count); B.part.resize(count); B.rowinfo.resize(count);
  B.rpart.resize(count);
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    const int64_t n = A[i].n, nnz = A[i].nnz;
    B.rowlist[i] = off; off = align_up(off + 4 * (P.r_max + P.m_b + 1));
    B.rowcnt[i] = off;  off = align_up(off + 4 * P.r_max);
    B.bstart[i] = off;  off = align_up(off + 4 * (P.nb_max + 1));
    B.pos[i] = off;     off = align_up(off + 4 * (P.nb_max + 1) * n);
    B.ent[i] = off;     off = align_up(off + 8 * (nnz + 2));
    B.rowinfo[i] = off; off = align_up(off + 8 * A[i].m);
    B.rpart[i] = off;   off = align_up(off + 4 * rpart_ints(A[i].m, n));
    B.part[i] = off;
    if (P.slices > 1) off = align_up(off + 4 * (int64_t)P.slices * d[i] * n);
  }
  B.total = off;
  return SK_OK;
}

// ------------------------------------------------------------------ SAP
static_assert(offsetof(LsqrState, rnorm) == offsetof(sk_sap_info, rnorm) &&
                  offsetof(LsqrState, test3) == offsetof(sk_sap_info, test3) &&
                  offsetof(LsqrState, itn) == offsetof(sk_sap_info, iterations) &&
                  offsetof(LsqrState, done) == offsetof(sk_sap_info, done) &&
                  offsetof(LsqrState, rank) == offsetof(sk_sap_info, rank) &&
                  offsetof(LsqrState, sweeps) == offsetof(sk_sap_info, sweeps) &&
                  sizeof(sk_sap_info) <= offsetof(LsqrState, alpha),
              "solver info prefix");

struct SapLayout {
  int64_t state, sk_ws, sk_bytes, ahat, q, tau, tq, r, rinv, rinvt, vsv, sig, smax, jctl, v64,
      rcnt, rowptr, cursor, ccol, cval, lidx, lrows, sums, cbase, cpart, u, partial, partial2, v,
      w, y, tn, sn, t2, total;
  bool svd;
  int64_t nchunk_max, nblk_m, nlong_max, nblk_long;
};

sk_status sap_layout(const sk_csc* A, const sk_sap_params* p, SapLayout& L) {
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (!p) return SK_EINVAL;
  const int64_t m = A->m, n = A->n, nnz = A->nnz, d = p->d;
  if (n > m || d < n || n > SAP_MAX_N || p->dist < 0 || p->dist > 2 || p->iter_lim < 1 ||
      (p->method != SK_SAP_QR && p->method != SK_SAP_SVD))
    return SK_EINVAL;
  L.svd = p->method == SK_SAP_SVD;
  // the sketch's own workspace: the FP32 sketch's plan (the kernel choice and
  // any cached tuning of the shape class), or the FP64 Algorithm 3 kernel's
  // validation record for the SVD form
  size_t sk_bytes = 0;
  if (L.svd) {
    if (p->prec != SK_PREC_F32) return SK_EUNSUPPORTED;
    sk_bytes = colwise_bytes(A, d);
  } else if ((s = sk_sketch_workspace(A, d, p->dist, p->prec, nullptr, &sk_bytes)) != SK_OK) {
    return s;
  }
  int64_t off = 0;
  L.state = off;   off = align_up(off + (int64_t)sizeof(LsqrState));
  L.sk_ws = off;   L.sk_bytes = (int64_t)sk_bytes; off = align_up(off + L.sk_bytes);
  L.ahat = off;    off = align_up(off + 4 * d * n);
  L.q = off;       off = align_up(off + 8 * d * n);
  L.tau = off;     off = align_up(off + 8 * n);
  L.tq = off;      off = align_up(off + 8 * QR_NB * QR_NB);
  L.r = off;       off = align_up(off + 8 * n * n);
  L.rinv = off;    off = align_up(off + 8 * n * n);
  L.rinvt = off;   off = align_up(off + 8 * n * n);
  const int64_t nsv = L.svd ? n : 0;  // the Jacobi SVD's arrays (R^T orthogonalised)
  L.vsv = off;     off = align_up(off + 8 * nsv * nsv);
  L.sig = off;     off = align_up(off + 8 * nsv);
  L.smax = off;    off = align_up(off + 8);
  L.jctl = off;    off = align_up(off + (int64_t)sizeof(JacobiCtl));
  L.v64 = off;     off = align_up(off + 8 * std::max<int64_t>(nnz, 1));
  L.rcnt = off;    off = align_up(off + 4 * m);
  L.rowptr = off;  off = align_up(off + 4 * (m + 2));
  L.cursor = off;  off = align_up(off + 4 * m);
  L.ccol = off;    off = align_up(off + 4 * std::max<int64_t>(nnz, 1));
  L.cval = off;    off = align_up(off + 8 * std::max<int64_t>(nnz, 1));
  L.nlong_max = nnz / (SAP_LONG + 1) + 1;  // rows with more than SAP_LONG entries
  L.nblk_long = (L.nlong_max + 3) / 4;     // four waves per workgroup
  L.lidx = off;    off = align_up(off + 4 * (m + 2));
  L.lrows = off;   off = align_up(off + 4 * L.nlong_max);
  L.sums = off;    off = align_up(off + 4 * scan_sums_len(std::max<int64_t>(m + 1, n + 1)));
  L.nchunk_max = n + nnz / SAP_CHUNK + 1;
  L.cbase = off;   off = align_up(off + 4 * (n + 2));
  L.cpart = off;   off = align_up(off + 8 * L.nchunk_max);
  L.nblk_m = (m + SAP_THREADS - 1) / SAP_THREADS;
  L.u = off;       off = align_up(off + 8 * m);
  L.partial = off; off = align_up(off + 8 * L.nblk_m);
  L.partial2 = off; off = align_up(off + 8 * L.nblk_long);
  L.v = off;       off = align_up(off + 8 * n);
  L.w = off;       off = align_up(off + 8 * n);
  L.y = off;       off = align_up(off + 8 * n);
  L.tn = off;      off = align_up(off + 8 * n);
  L.sn = off;      off = align_up(off + 8 * n);
  L.t2 = off;      off = align_up(off + 8 * n);
  L.total = off;
  return SK_OK;
}

sk_status qr_launch(int64_t d, int64_t n, double* A, int64_t lda, double* R, int64_t ldr,
                    double* tau, double* T, hipStream_t st) {
  for (int64_t j0 = 0; j0 < n;) {
    // panels of at most QR_REG_ROWS rows are factored in registers, eight
    // columns at a time
    const bool in_regs = d - j0 <= QR_REG_ROWS;
    const int nb = (int)std::min<int64_t>(in_regs ? QR_NB_REG : QR_NB, n - j0);
    if (in_regs)
      hipLaunchKernelGGL(k_qr_panel_regs, dim3(1), dim3(QR_PT), 0, st, A,
                         lda, d, j0, nb, tau, T);
    else
      hipLaunchKernelGGL(k_qr_panel, dim3(1), dim3(SAP_THREADS), 0, st, A, lda, d, j0, nb, tau,
                         T);
    const int64_t trail = n - j0 - nb;
    if (trail > 0)
      hipLaunchKernelGGL(k_qr_update, dim3((unsigned)trail), dim3(SAP_THREADS), 0, st, A, lda, d,
                         n, j0, nb, T);
    j0 += nb;
  }
  hipLaunchKernelGGL(k_qr_extract_r, dim3(blocks_for(n * n, 256)), dim3(256), 0, st, A, lda, n, R,
                     ldr);
  return launch_ok();
}

sk_status trinv_launch(int64_t n, const double* R, int64_t ldr, double* Ri, int64_t ldi,
                       hipStream_t st) {
  if (hipFuncSetAttribute((const void*)k_trinv_upper, hipFuncAttributeMaxDynamicSharedMemorySize,
                          16 * SAP_MAX_N) != hipSuccess)
    return SK_EHIP;
  hipLaunchKernelGGL(k_trinv_upper, dim3((unsigned)n), dim3(SAP_THREADS), (size_t)(16 * n), st, R,
                     ldr, n, Ri, ldi);
  return launch_ok();
}

// one LSQR iteration's launches (every kernel returns at once after the stop)
// One-sided Jacobi on G (rows x n, in place) with V = I accumulated: sweeps
// of the round-robin order, enqueued in batches; between batches the host
// reads the converged flag (a sweep without rotations) and stops.  Relative
// orthogonality tolerance sqrt(rows) * 2^-52.
constexpr int kJacobiMaxSweeps = 40;
constexpr int kJacobiBatch = 4;

// tmp: n doubles of scratch (the column norms for the rounding floor)
sk_status jacobi_svd(int64_t rows, int64_t n, double* G, double* V, JacobiCtl* ctl, double* tmp,
                     hipStream_t st) {
  const bool withv = V != nullptr;  // else no V is accumulated
  if (withv) hipLaunchKernelGGL(k_eye, dim3(blocks_for(n * n, 256)), dim3(256), 0, st, V, n);
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)n), dim3(SVD_THREADS), 0, st, (const double*)G,
                     rows, tmp);
  hipLaunchKernelGGL(k_jacobi_reset, dim3(1), dim3(SVD_THREADS), 0, st, (const double*)tmp, n,
                     ctl);
  const int64_t npad = n + (n & 1);
  const double tol = std::sqrt((double)rows) * 0x1.0p-52;
  const bool reg = rows <= (int64_t)SVD_THREADS * SVD_RPT;  // n <= rows
  // without V: the block form when 2W columns of G fit in LDS and there are
  // at least two blocks, from n = 768 on (measured: n = 1000 107 ms against
  // 134 ms pairwise; n = 500 38 against 32 ms, too few block pairs to fill
  // the chip)
  int W = 0;
  if (!withv && n >= 768)
    for (int w : {8, 4, 2})
      if ((int64_t)2 * w * rows * 8 + 2048 <= kLdsPerCu && (n + w - 1) / w >= 2) {
        W = w;
        break;
      }
  const int64_t nblk = W ? (n + W - 1) / W : 0;
  const int64_t nbpad = nblk + (nblk & 1);
  const size_t blk_lds = W ? (size_t)(2 * W * rows * 8) : 0;
  using BlockKernel = void (*)(double*, int64_t, int64_t, int64_t, int64_t, int64_t, double,
                               JacobiCtl*);
  const BlockKernel bk = W == 8 ? k_jacobi_block<8> : W == 4 ? k_jacobi_block<4>
                                                             : k_jacobi_block<2>;
  if (W && hipFuncSetAttribute((const void*)bk, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)blk_lds) != hipSuccess)
    return SK_EHIP;
  for (int sweep = 0; sweep < kJacobiMaxSweeps;) {
    for (int b = 0; b < kJacobiBatch && sweep < kJacobiMaxSweeps; ++b, ++sweep) {
      if (W) {
        for (int64_t step = 0; step < nbpad - 1; ++step)
          hipLaunchKernelGGL(bk, dim3((unsigned)(nbpad / 2)), dim3(1024), blk_lds, st, G, rows, n,
                             nblk, nbpad, step, tol, ctl);
      } else {
        for (int64_t step = 0; step < npad - 1; ++step)
          hipLaunchKernelGGL(withv ? (reg ? k_jacobi_step<true, true> : k_jacobi_step<false, true>)
                                   : (reg ? k_jacobi_step<true, false> : k_jacobi_step<false, false>),
                             dim3((unsigned)(npad / 2)), dim3(SVD_THREADS), 0, st, G, rows, V, n,
                             npad, step, tol, ctl);
      }
      hipLaunchKernelGGL(k_jacobi_sweep_end, dim3(1), dim3(64), 0, st, ctl);
    }
    sk_status s = launch_ok();
    if (s != SK_OK) return s;
    JacobiCtl h;
    if (hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SK_EHIP;
    if (h.converged) break;
  }
  return SK_OK;
}

void lsqr_iteration(const sk_csc* A, const SapLayout& L, char* w, hipStream_t st) {
  const int64_t m = A->m, n = A->n;
  LsqrState* state = (LsqrState*)(w + L.state);
  const double* Ri = (const double*)(w + L.rinv);
  double* v = (double*)(w + L.v);
  double* tn = (double*)(w + L.tn);
  double* u = (double*)(w + L.u);
  double* partial = (double*)(w + L.partial);
  double* partial2 = (double*)(w + L.partial2);
  hipLaunchKernelGGL(L.svd ? k_gemv_upper<false> : k_gemv_upper<true>,
                     dim3(blocks_for(n * 64, 256)), dim3(256), 0, st,
                     (const double*)(w + L.rinvt), n, v, tn, state);
  hipLaunchKernelGGL(k_lsqr_av<false>, dim3((unsigned)L.nblk_m), dim3(SAP_THREADS), 0, st,
                     (const int32_t*)(w + L.rowptr), (const int32_t*)(w + L.ccol),
                     (const double*)(w + L.cval), m, tn, (const double*)nullptr, u, partial,
                     state);
  hipLaunchKernelGGL(k_lsqr_av_long, dim3((unsigned)L.nblk_long), dim3(SAP_THREADS), 0, st,
                     (const int32_t*)(w + L.rowptr), (const int32_t*)(w + L.ccol),
                     (const double*)(w + L.cval), (const int32_t*)(w + L.lidx), m,
                     (const int32_t*)(w + L.lrows), tn, u, partial2, state);
  hipLaunchKernelGGL(k_lsqr_beta<false>, dim3(1), dim3(1024), 0, st, partial, L.nblk_m,
                     (const double*)partial2, L.nblk_long, state);
  hipLaunchKernelGGL(k_lsqr_atu, dim3(blocks_for(L.nchunk_max * 64, 256)), dim3(256), 0, st,
                     A->colptr, A->rowidx, (const double*)(w + L.v64), n,
                     (const int32_t*)(w + L.cbase), u, (double*)(w + L.cpart), state,
                     (const Header*)(w + L.sk_ws));
  hipLaunchKernelGGL(k_lsqr_colsum, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                     (const int32_t*)(w + L.cbase), n, (const double*)(w + L.cpart),
                     (double*)(w + L.sn), state);
  hipLaunchKernelGGL(L.svd ? k_gemv_upper_t<false> : k_gemv_upper_t<true>,
                     dim3(blocks_for(n * 64, 256)), dim3(256), 0, st, Ri, n, n,
                     (const double*)(w + L.sn), (double*)(w + L.t2), state);
  hipLaunchKernelGGL(k_lsqr_update<false>, dim3(1), dim3(1024), 0, st, n,
                     (const double*)(w + L.t2), v, (double*)(w + L.w), (double*)(w + L.y), state);
}
}  // namespace

// ------------------------------------------------- allocation-free form
// Workspace of sk_sketch_noalloc: a fixed device array, one copy per device
// (the loader gives each GPU its own), held until the process ends.  Host
// code never passes the array's name to a kernel: that name is a host-side
// stand-in, not a device address.  The device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SK_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

sk_status scratch_for_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SK_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return SK_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SK_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SK_OK;
}
}  // namespace

namespace {
// The Algorithm 3 (kji) kernel after the validation pass (arguments checked
// by the caller); ACC = double: the FP64 form.
template <typename ACC = float>
sk_status colwise_impl(const sk_csc* A, int64_t row0, int64_t d, int32_t dist, uint64_t seed,
                       ACC* Ahat, int64_t ld, void* ws, size_t ws_bytes, hipStream_t st) {
  const ColwiseLayout CL = colwise_layout(A->n, A->nnz, d);
  if (!ws || ws_bytes < (size_t)CL.total) return SK_EWORKSPACE;
  const int dl = dist == SK_RADEMACHER ? 32 : 4;
  const int64_t tiles = (d + 64 * dl - 1) / (64 * dl);
  const int64_t tgroups = (tiles + CW_WAVES - 1) / CW_WAVES;
  const int64_t grid = CL.chunks_max * tgroups;
  const int64_t rgrid = CL.heavy_max * ((d + 255) / 256);
  if (grid >= INT32_MAX || rgrid >= INT32_MAX || CL.chunks_max >= INT32_MAX / 2)
    return SK_EUNSUPPORTED;
  char* w = (char*)ws;
  Header* hdr = (Header*)(w + CL.hdr);
  Item* d_item = (Item*)(w + CL.item);
  int32_t* cb = (int32_t*)(w + CL.cb);
  int32_t* hb = (int32_t*)(w + CL.hb);
  int32_t* hk = (int32_t*)(w + CL.hk);
  int32_t* hcol = (int32_t*)(w + CL.hcol);
  int32_t* sums = (int32_t*)(w + CL.sums);
  // validation only: the CSC input is used as given
  Item I;
  std::memset(&I, 0, sizeof I);
  I.m = A->m; I.n = A->n; I.nnz = A->nnz;
  I.colptr = A->colptr; I.rowidx = A->rowidx; I.vals = A->vals; I.vtype = A->vtype;
  I.hdr = hdr;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, (int32_t*)hdr,
                     (int64_t)(sizeof(Header) / 4), 0);
  hipLaunchKernelGGL(k_put_item, dim3(1), dim3(64), 0, st, I, d_item);
  launch_items_cols<&Item::o_valid, OpValidate>(d_item, 1, std::max<int64_t>(A->nnz, A->n + 1),
                                                st);
  // chunks of the heavy columns
  const int64_t n = A->n;
  hipLaunchKernelGGL(k_colwise_counts, dim3(blocks_for(n, 256)), dim3(256), 0, st, A->colptr, n,
                     (int32_t)CL.chunk, (const Header*)hdr, cb, hb, hk);
  sk_status s;
  if ((s = scan_i32(cb, n, sums, st)) != SK_OK) return s;
  if ((s = scan_i32(hb, n, sums, st)) != SK_OK) return s;
  if ((s = scan_i32(hk, n, sums, st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_colwise_heavy_list, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                     (const int32_t*)hk, n, hcol);
  ColwiseParams P{};
  P.colptr = A->colptr; P.rowidx = A->rowidx; P.vals = A->vals; P.vtype = A->vtype;
  P.hdr = hdr; P.n = n; P.d = d; P.row0 = row0; P.seed = seed; P.out = Ahat; P.ld = ld;
  P.tiles = (int32_t)tiles;
  P.chunk = (int32_t)CL.chunk;
  P.cbase = cb;
  P.hbase = hb;
  P.part = w + CL.part;
  if (dist == SK_RADEMACHER)
    hipLaunchKernelGGL((k_sketch_colwise<DIST_RADEMACHER, 32, ACC>), dim3((unsigned)grid),
                       dim3(64 * CW_WAVES), 0, st, P);
  else if (dist == SK_UNIFORM)
    hipLaunchKernelGGL((k_sketch_colwise<DIST_UNIFORM, 4, ACC>), dim3((unsigned)grid),
                       dim3(64 * CW_WAVES), 0, st, P);
  else
    hipLaunchKernelGGL((k_sketch_colwise<DIST_GAUSSIAN, 4, ACC>), dim3((unsigned)grid),
                       dim3(64 * CW_WAVES), 0, st, P);
  hipLaunchKernelGGL(k_colwise_reduce<ACC>, dim3((unsigned)rgrid), dim3(256), 0, st,
                     (const int32_t*)hk, (const int32_t*)hcol, (const int32_t*)cb,
                     (const int32_t*)hb, n, d, (const ACC*)(w + CL.part), Ahat, ld);
  return launch_ok();
}

// The sketch with generator mode `gen` (GEN_PHILOX for the product; the
// others are the distribution-cost ablation's, on the shapes that have them,
// without the dense path or the folded virtual columns).
// a2 with balanced row blocks: the nonempty rows of A, their renumbering
// (sk_balance.hpp), A' with its nonempty rows set directly, the blocked
// layout of A' and the row list mapped back to the rows of A (the
// generator's counters)
sk_status balanced_inspector(const sk_csc* A, const Plan& P, const Item& I, const Layout& L,
                             char* w, Item* d_item, const InspectSizes& Z, const InspectArrays& W,
                             hipStream_t st) {
  sk_status s;
  if ((s = inspect_rows(d_item, 1, Z, W, st)) != SK_OK) return s;
  BalParams B{};
  B.hdr = I.hdr;
  B.m = A->m; B.n = A->n; B.nnz = A->nnz; B.r_max = P.r_max;
  B.colptr = A->colptr; B.rowidx = A->rowidx; B.vals = A->vals; B.vtype = A->vtype;
  B.m_b = P.m_b; B.sb = P.bal_sb; B.sbm = P.bal_sb * P.m_b;
  B.ridx = I.ridx; B.rowlist = I.rowlist; B.rowcnt = I.rowcnt;
  B.rowoff = (int32_t*)(w + L.bal_rowoff);
  B.ccol = (uint16_t*)(w + L.bal_ccol);
  B.newidx = (int32_t*)(w + L.bal_newidx);
  B.orig = (int32_t*)(w + L.bal_orig);
  B.cnt2 = (int32_t*)(w + L.bal_cnt2);
  B.rowidx2 = (int32_t*)(w + L.bal_rowidx);
  B.vals2 = (float*)(w + L.bal_vals);
  hipLaunchKernelGGL(k_bal_prep, dim3(blocks_for(P.r_max, 256)), dim3(256), 0, st, B);
  if ((s = scan_i32(B.rowoff, P.r_max, W.sums, st)) != SK_OK) return s;
  if (I.rpart)
    hipLaunchKernelGGL(k_bal_slab_prefix, dim3(blocks_for(A->m, 256)), dim3(256), 0, st, B,
                       I.rpart);
  if (A->nnz > 0 && Z.rt > 0)
    hipLaunchKernelGGL(k_bal_csr, dim3((unsigned)Z.rt), dim3(1024), 0, st, B,
                       (const int32_t*)I.rpart);
  const size_t lds = bal_assign_lds(A->n, B.sb, B.sbm);
  if (hipFuncSetAttribute((const void*)k_bal_assign, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return SK_EHIP;
  const int64_t nsb = (P.r_max + B.sbm - 1) / B.sbm;
  hipLaunchKernelGGL(k_bal_assign, dim3((unsigned)nsb), dim3(BAL_THREADS), lds, st, B);
  const int64_t ngrp = (nsb + BAL_BUILD_G - 1) / BAL_BUILD_G;
  hipLaunchKernelGGL(k_bal_build, dim3(blocks_for(ngrp * A->n * 64, 256)), dim3(256), 0, st, B);
  if ((s = launch_ok()) != SK_OK) return s;
  Item I2 = I;  // A' (validated through A)
  I2.rowidx = B.rowidx2;
  I2.vals = B.vals2;
  I2.vtype = SK_F32;
  hipLaunchKernelGGL(k_put_item, dim3(1), dim3(64), 0, st, I2, d_item);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(Z.bfl + 1, 256 * 8)), dim3(256), 0, st,
                     W.bfl, Z.bfl + 1, 0);
  hipLaunchKernelGGL(k_bal_rows2, dim3(blocks_for(A->m + 1, 256)), dim3(256), 0, st, B, I.ridx,
                     I.rcnt, I.rowlist, I.rowcnt);
  if ((s = inspect_blocks(d_item, 1, Z, W, st, gather_pays(P, A->nnz))) != SK_OK) return s;
  hipLaunchKernelGGL(k_bal_remap, dim3(blocks_for(P.r_max, 256)), dim3(256), 0, st, I.hdr,
                     B.orig, P.r_max, I.rowlist);
  return launch_ok();
}

sk_status sketch_impl(const sk_csc* A, int64_t row0, int64_t d, int32_t dist, uint64_t seed,
                      int32_t prec, const sk_tuning* tune, float* Ahat, int64_t ld, void* ws,
                      size_t ws_bytes, void* hip_stream, int gen, const float* s_pre,
                      int64_t s_ld) {
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || row0 < 0 || !Ahat || ld < d || dist < 0 || dist > 2) return SK_EINVAL;
  if (prec < 0 || prec > 2) return SK_EINVAL;
  if (prec != SK_PREC_F32 && dist != SK_RADEMACHER) return SK_EUNSUPPORTED;
  sk_tuning cached;
  if (gen == GEN_PHILOX) tune = effective_tuning(A, d, dist, prec, tune, cached);
  const int kernel = gen == GEN_PHILOX ? choose_kernel(A, d, dist, prec, tune)
                     : tune && tune->kernel == KERNEL_KJI ? KERNEL_KJI
                                                          : KERNEL_TILE;
  if (kernel == KERNEL_KJI) {
    // the Algorithm 3 kernel has FP32 S only, no ablation or counting forms
    if (gen != GEN_PHILOX || prec != SK_PREC_F32 || (tune && tune->count_rng))
      return SK_EUNSUPPORTED;
    return colwise_impl(A, row0, d, dist, seed, Ahat, ld, ws, ws_bytes, (hipStream_t)hip_stream);
  }
  if (kernel != KERNEL_TILE) return SK_EINVAL;
  Plan P;
  if (!plan_any(A->m, A->n, A->nnz, d, dist, prec, tune, P)) return SK_EINVAL;
  if ((int64_t)(P.nb_max + 1) * P.nv >= INT32_MAX) return SK_EUNSUPPORTED;
  if (gen != GEN_PHILOX) {
    if (P.mfma || !ablation_kernel(P.variant, gen, dist) || (tune && tune->count_rng))
      return SK_EUNSUPPORTED;
    P.dense_pct = 0;
    P.kd_max = 0;
    P.slices = P.splits;
  }
  const Layout L = layout_for(A->m, A->n, A->nnz, d, P);
  if (!ws || ws_bytes < (size_t)L.total) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n = A->n;
  const int phases = tune && tune->phases ? tune->phases : 15;
  char* w = (char*)ws;
  Item I = make_item(A, P, dist);
  I.hdr = (Header*)(w + L.hdr);
  I.ridx = (int32_t*)(w + L.ridx);
  I.rcnt = (int32_t*)(w + L.rcnt);
  I.rowlist = (int32_t*)(w + L.rowlist);
  I.rowcnt = (int32_t*)(w + L.rowcnt);
  I.bfl = (int32_t*)(w + L.bfl);
  I.bstart = (int32_t*)(w + L.bstart);
  I.vbase = P.nv != n ? (int32_t*)(w + L.vbase) : nullptr;
  I.pos = (int32_t*)(w + L.pos);
  I.seg = (int32_t*)(w + L.seg);
  I.ent = (uint2*)(w + L.ent);
  I.bcost = (int32_t*)(w + L.bcost);
  I.rowinfo = (int2*)(w + L.rowinfo);
  I.rpart = rpart_ints(A->m, n) ? (int32_t*)(w + L.rpart) : nullptr;
  I.dflag = P.dense_pct ? (int32_t*)(w + L.dflag) : nullptr;
  InspectSizes Z;
  item_offsets(I, Z);
  Item* d_item = (Item*)(w + L.item);
  int32_t* dflag = (int32_t*)(w + L.dflag);
  int32_t* dlist = (int32_t*)(w + L.dlist);
  int32_t* doff = (int32_t*)(w + L.doff);
  DenseHeader* dhdr = (DenseHeader*)(w + L.dhdr);
  int32_t* drows = (int32_t*)(w + L.drows);
  float* dense = (float*)(w + L.dense);
  float* part = (float*)(w + L.part);
  const int64_t nv = P.nv;

  if (phases & 1) {
    // a1 + a2: validation and the blocked layout
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, (int32_t*)I.hdr,
                       (int64_t)(sizeof(Header) / 4), 0);
    hipLaunchKernelGGL(k_put_item, dim3(1), dim3(64), 0, st, I, d_item);
    // pad the row list so a block can read past its last row
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(256), 0, st, I.rowlist + P.r_max,
                       (int64_t)P.m_b + 1, 0);
    const InspectArrays W{I.ridx, I.rcnt, I.bfl, I.vbase, I.seg, I.bcost, (int32_t*)(w + L.sums)};
    if (P.bal_sb) {
      if ((s = balanced_inspector(A, P, I, L, w, d_item, Z, W, st)) != SK_OK) return s;
    } else if ((s = run_inspector(d_item, 1, Z, W, st, gather_pays(P, A->nnz))) != SK_OK) {
      return s;
    }
    // a5 (selection): dense row blocks, their rows concatenated and densified
    if (P.dense_pct) {
      hipLaunchKernelGGL(k_dense_select, dim3(1), dim3(256), 0, st, I.seg, nv, n, I.bstart,
                         P.dense_pct, P.kd_max, I.hdr, dflag, dlist, doff, dhdr);
      hipLaunchKernelGGL(k_dense_zero, dim3(blocks_for(P.kd_max * n, 256 * 16)), dim3(256), 0, st,
                         dense, n, dhdr);
      hipLaunchKernelGGL(k_dense_rows, dim3(blocks_for(P.kd_max, 256)), dim3(256), 0, st,
                         I.rowlist, I.bstart, dlist, doff, dhdr, drows);
      const int64_t nd_cap = std::max<int64_t>(1, std::min(P.nb_max, P.kd_max));
      hipLaunchKernelGGL(k_densify, dim3(blocks_for(nd_cap * nv, 256)), dim3(256), 0, st, I.seg,
                         I.ent, nv, n, I.vbase, P.row_bytes, dlist, doff, dhdr, dense);
      if ((s = launch_ok()) != SK_OK) return s;
    }
    if ((s = run_block_costs(d_item, 1, Z, W, st)) != SK_OK) return s;
  }

  // a3 + a4: S tiles and sparse accumulation (or the whole contraction on
  // the matrix cores for +-1 S in BF16/FP8)
  SketchParams K = make_params(P, I, d, row0, seed);
  K.s_pre = s_pre;
  K.s_ld = s_ld;
  K.dflag = P.dense_pct ? dflag : nullptr;
  // virtual columns: added in the kernel (then it writes the n real
  // columns) or in the reduction
  // the call-counting instantiation leaves virtual columns to the reduction
  const bool counting = tune && tune->count_rng && !P.mfma;
  const bool fold = !counting && gen == GEN_PHILOX && I.vbase != nullptr && folds_virtual(P, n);
  if (fold) { K.vbase = I.vbase; K.nreal = n; }
  const int64_t wcols = fold ? n : nv;  // columns of one partial slice
  const bool staged = P.slices > 1 || wcols != n;  // partials, then the reduction
  if (staged) { K.out = part; K.ld = d; K.split_stride = d * wcols; }
  else { K.out = Ahat; K.ld = ld; K.split_stride = 0; }
  const int64_t grid = (int64_t)P.tiles * P.ncr * P.splits;
  if (grid >= INT32_MAX) return SK_EUNSUPPORTED;
  if (P.mfma) {
    const void* kern = P.mfma == MF_BF16 ? (const void*)k_sketch_mfma<MF_BF16>
                                         : (const void*)k_sketch_mfma<MF_FP8>;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds) !=
        hipSuccess)
      return SK_EHIP;
    if (phases & 2) {
      if (P.mfma == MF_BF16)
        hipLaunchKernelGGL(k_sketch_mfma<MF_BF16>, dim3((unsigned)grid), dim3(MF_THREADS), P.lds,
                           st, K);
      else
        hipLaunchKernelGGL(k_sketch_mfma<MF_FP8>, dim3((unsigned)grid), dim3(MF_THREADS), P.lds,
                           st, K);
      if ((s = launch_ok()) != SK_OK) return s;
    }
  } else {
    const Variant& V = kVariants[P.variant];
    SketchKernel kern = gen != GEN_PHILOX ? ablation_kernel(P.variant, gen, dist)
                        : counting        ? V.kc[dist]
                        : fold            ? V.kf[dist]
                                          : V.k[dist];
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)P.lds) != hipSuccess)
      return SK_EHIP;
    if (phases & 2) {
      hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(V.wgs), P.lds, st, K);
      if ((s = launch_ok()) != SK_OK) return s;
    }
  }
  // a5: dense row blocks on the matrix cores, into the last partial slice
  if ((phases & 8) && P.dense_pct) {
    DenseParams DP{};
    DP.drows = drows; DP.dh = dhdr; DP.hdr = I.hdr; DP.D = dense;
    DP.n = n; DP.d = d; DP.row0 = row0; DP.seed = seed;
    DP.out = part + (int64_t)P.splits * d * wcols;
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
  // a6: fixed-order reduction of the partial slices (and virtual columns)
  if ((phases & 4) && staged)
    hipLaunchKernelGGL(k_reduce_virtual, dim3(blocks_for(d * n, 256)), dim3(256), 0, st, part,
                       P.splits, d, n, wcols, fold ? nullptr : I.vbase,
                       P.dense_pct ? part + (int64_t)P.splits * d * wcols : nullptr, Ahat, ld);
  return launch_ok();
}

// ------------------------------------------------------ measured tuner
// Splits tried for the chosen S-tile shapes, and the most partial-slice
// memory a candidate may take.
constexpr int kSplitCands[] = {1, 2, 4, 6, 8, 12, 16, 20, 24, 32, 48, 64};
constexpr int64_t kTunePartMax = int64_t(4) << 30;

sk_tuning searched(int kernel, int variant, int splits) {
  sk_tuning t;
  std::memset(&t, 0, sizeof t);
  t.kernel = kernel;
  t.variant = variant;
  t.splits = splits;
  return t;
}

// stage one: the Algorithm 3 kernel (FP32) and each S-tile kernel shape at
// the model's splits (the matrix-core path has one shape)
std::vector<sk_tuning> tune_stage_one(const sk_csc* A, int dist, int prec) {
  std::vector<sk_tuning> c;
  if (prec == SK_PREC_F32) c.push_back(searched(KERNEL_KJI, 0, 0));
  if (mfma_format(A->m, A->n, A->nnz, dist, prec, nullptr)) {
    c.push_back(searched(KERNEL_TILE, 0, 0));
    return c;
  }
  for (int v = 1; v <= kNumVariants; ++v) c.push_back(searched(KERNEL_TILE, v, 0));
  return c;
}

// stage two: the splits of one S-tile shape (variant 0: the matrix cores)
std::vector<sk_tuning> tune_stage_two(const sk_csc* A, int64_t d, int dist, int prec,
                                      int variant) {
  std::vector<sk_tuning> c;
  for (int sp : kSplitCands) {
    const sk_tuning t = searched(KERNEL_TILE, variant, sp);
    Plan P;
    if (!plan_any(A->m, A->n, A->nnz, d, dist, prec, &t, P)) continue;
    if (P.splits != sp) continue;  // clamped to the block count
    if ((int64_t)P.splits * d * P.nv * 4 > kTunePartMax) continue;
    c.push_back(t);
  }
  return c;
}

// stage three: the winner with the balanced row blocks switched the other
// way (on where its plan has them off, off where on), when that plan exists
bool tune_stage_three(const sk_csc* A, int64_t d, int dist, int prec, const sk_tuning& win,
                      sk_tuning* flip) {
  if (win.kernel != KERNEL_TILE || win.variant == 0) return false;
  Plan P;
  if (!plan_any(A->m, A->n, A->nnz, d, dist, prec, &win, P) || P.mfma) return false;
  sk_tuning t = win;
  t.balance = P.bal_sb ? 1 : 2;
  Plan P2;
  if (!plan_any(A->m, A->n, A->nnz, d, dist, prec, &t, P2)) return false;
  if ((P2.bal_sb != 0) == (P.bal_sb != 0)) return false;  // (the rule refuses the switch)
  *flip = t;
  return true;
}

// every candidate the stages may run (for the workspace bound): the S-tile
// candidates also with the balanced row blocks on and off
std::vector<sk_tuning> tune_candidates_all(const sk_csc* A, int64_t d, int dist, int prec) {
  std::vector<sk_tuning> c = tune_stage_one(A, dist, prec);
  const size_t first = c.size();
  for (size_t i = 0; i < first; ++i)
    if (c[i].kernel == KERNEL_TILE)
      for (const sk_tuning& t : tune_stage_two(A, d, dist, prec, c[i].variant)) c.push_back(t);
  const size_t all = c.size();
  for (size_t i = 0; i < all; ++i) {
    if (c[i].kernel != KERNEL_TILE || c[i].variant == 0) continue;
    for (int b = 1; b <= 2; ++b) {
      sk_tuning t = c[i];
      t.balance = b;
      c.push_back(t);
    }
  }
  return c;
}

// The time of one sketch with tuning t, in ms: one untimed call, then the
// fastest of up to three timed ones (one only when it is already slower
// than `cutoff_ms`), each bracketed by events on the stream.
sk_status time_call(const sk_csc* A, int64_t d, int dist, uint64_t seed, int prec,
                    const sk_tuning& t, float* Ahat, int64_t ld, void* ws, size_t ws_bytes,
                    hipStream_t st, double cutoff_ms, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SK_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SK_EHIP;
  }
  double best = INFINITY;
  sk_status s = sketch_impl(A, 0, d, dist, seed, prec, &t, Ahat, ld, ws, ws_bytes, st,
                            GEN_PHILOX, nullptr, 0);
  for (int r = 0; s == SK_OK && r < 3; ++r) {
    if (hipEventRecord(e0, st) != hipSuccess) { s = SK_EHIP; break; }
    s = sketch_impl(A, 0, d, dist, seed, prec, &t, Ahat, ld, ws, ws_bytes, st, GEN_PHILOX,
                    nullptr, 0);
    if (s != SK_OK) break;
    float f = 0.0f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&f, e0, e1) != hipSuccess) {
      s = SK_EHIP;
      break;
    }
    best = std::min(best, (double)f);
    if (best > cutoff_ms) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return s;
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
  if (prec != SK_PREC_F32 && dist != SK_RADEMACHER) return SK_EUNSUPPORTED;
  sk_tuning cached;
  const int gen = tune ? tune->rng_mode : GEN_PHILOX;
  if (gen == GEN_PHILOX) tune = effective_tuning(A, d, dist, prec, tune, cached);
  const int kernel = gen == GEN_PHILOX ? choose_kernel(A, d, dist, prec, tune)
                     : tune && tune->kernel == KERNEL_KJI ? KERNEL_KJI
                                                          : KERNEL_TILE;
  if (kernel == KERNEL_KJI) {
    if (gen != GEN_PHILOX || prec != SK_PREC_F32 || (tune && tune->count_rng))
      return SK_EUNSUPPORTED;
    *bytes = colwise_bytes(A, d);
    return SK_OK;
  }
  if (kernel != KERNEL_TILE) return SK_EINVAL;
  Plan P;
  if (!plan_any(A->m, A->n, A->nnz, d, dist, prec, tune, P)) return SK_EINVAL;
  *bytes = (size_t)layout_for(A->m, A->n, A->nnz, d, P).total;
  return SK_OK;
}

sk_status sk_sketch(const sk_csc* A, int64_t row0, int64_t d, int32_t dist, uint64_t seed,
                    int32_t prec, const sk_tuning* tune, float* Ahat, int64_t ld, void* ws,
                    size_t ws_bytes, void* hip_stream) {
  return sketch_impl(A, row0, d, dist, seed, prec, tune, Ahat, ld, ws, ws_bytes, hip_stream,
                     tune ? tune->rng_mode : GEN_PHILOX, nullptr, 0);
}

sk_status sk_sketch_stored(const sk_csc* A, int64_t d, const float* S, int64_t lds,
                           const sk_tuning* tune, float* Ahat, int64_t ld, void* ws,
                           size_t ws_bytes, void* hip_stream) {
  if (!S || d < 1 || lds < (d + 127) / 128 * 128 || (reinterpret_cast<uintptr_t>(S) & 15))
    return SK_EINVAL;
  if (tune && tune->rng_mode) return SK_EINVAL;
  return sketch_impl(A, 0, d, SK_UNIFORM, 0, SK_PREC_F32, tune, Ahat, ld, ws, ws_bytes,
                     hip_stream, GEN_STORED, S, lds);
}

// ------------------------------------------- Algorithm 3 (kji) order
sk_status sk_sketch_colwise_workspace(const sk_csc* A, int64_t d, size_t* bytes) {
  if (!bytes) return SK_EINVAL;
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1) return SK_EINVAL;
  *bytes = colwise_bytes(A, d);
  return SK_OK;
}

sk_status sk_sketch_colwise(const sk_csc* A, int64_t row0, int64_t d, int32_t dist,
                            uint64_t seed, float* Ahat, int64_t ld, void* ws, size_t ws_bytes,
                            void* hip_stream) {
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || row0 < 0 || !Ahat || ld < d || dist < 0 || dist > 2) return SK_EINVAL;
  return colwise_impl(A, row0, d, dist, seed, Ahat, ld, ws, ws_bytes, (hipStream_t)hip_stream);
}

sk_status sk_sketch_colwise_f64(const sk_csc* A, int64_t row0, int64_t d, int32_t dist,
                                uint64_t seed, double* Ahat, int64_t ld, void* ws,
                                size_t ws_bytes, void* hip_stream) {
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || row0 < 0 || !Ahat || ld < d || dist < 0 || dist > 2) return SK_EINVAL;
  return colwise_impl<double>(A, row0, d, dist, seed, Ahat, ld, ws, ws_bytes,
                              (hipStream_t)hip_stream);
}

sk_status sk_rng_throughput(int32_t dist, int32_t gen, int64_t calls, int32_t blocks,
                            uint64_t seed, uint32_t* sink, void* hip_stream) {
  if (dist < 0 || dist > 2 || (gen != GEN_PHILOX && gen != GEN_JUNK) || calls < 1 ||
      blocks < 1 || !sink)
    return SK_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  using RK = void (*)(int64_t, uint64_t, uint32_t*);
  const RK table[2][3] = {
      {k_rng_throughput<DIST_RADEMACHER, GEN_PHILOX>, k_rng_throughput<DIST_UNIFORM, GEN_PHILOX>,
       k_rng_throughput<DIST_GAUSSIAN, GEN_PHILOX>},
      {k_rng_throughput<DIST_RADEMACHER, GEN_JUNK>, k_rng_throughput<DIST_UNIFORM, GEN_JUNK>,
       k_rng_throughput<DIST_GAUSSIAN, GEN_JUNK>}};
  hipLaunchKernelGGL(table[gen][dist], dim3(blocks), dim3(256), 0, st, calls, seed, sink);
  return launch_ok();
}

sk_status sk_sketch_noalloc(const sk_csc* A, int64_t row0, int64_t d, int32_t dist,
                            uint64_t seed, int32_t prec, const sk_tuning* tune, float* Ahat,
                            int64_t ld, void* hip_stream) {
  size_t need = 0;
  sk_status s = sk_sketch_workspace(A, d, dist, prec, tune, &need);
  if (s != SK_OK) return s;
  if (need > (size_t)SK_NOALLOC_SCRATCH_BYTES) return SK_EWORKSPACE;
  void* ws = nullptr;
  if ((s = scratch_for_current_device(&ws)) != SK_OK) return s;
  // sk_sketch itself allocates nothing and clears what must start at zero
  // (the header, the scanned flags) with fill kernels on the stream
  return sk_sketch(A, row0, d, dist, seed, prec, tune, Ahat, ld, ws, need, hip_stream);
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
  if (h.status & ST_CAPACITY) return SK_EUNSUPPORTED;  // block capacity (a planning bound) exceeded
  return SK_OK;
}

sk_status sk_sketch_rng_calls(const void* ws, void* hip_stream, uint64_t* calls) {
  if (!ws || !calls) return SK_EINVAL;
  Header h;
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess) return SK_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SK_EHIP;
  *calls = (uint64_t)h.reserved[0];
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
  Item* d_items = (Item*)(w + B.items);
  BatchOut* d_outs = (BatchOut*)(w + B.outs);
  int2* d_work = (int2*)(w + B.work);
  int32_t* counters = (int32_t*)(w + B.counters);
  const InspectArrays W{(int32_t*)(w + B.ridx_all), (int32_t*)(w + B.rcnt_all),
                        (int32_t*)(w + B.bfl_all), nullptr, (int32_t*)(w + B.seg_all),
                        (int32_t*)(w + B.bcost_all), (int32_t*)(w + B.sums)};
  const Variant& V = kVariants[B.variant];

  // item descriptors (host), copied to the workspace
  std::vector<Item> items(count);
  std::vector<BatchOut> outs(count);
  InspectSizes Z;
  int64_t o_ridx = 0, o_m = 0, o_bfl = 0, o_seg = 0, o_blk = 0, o_out = 0;
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    Item& I = items[i];
    I = make_item(&A[i], P, dist[i]);
    I.hdr = hdrs + i;
    I.ridx = W.ridx + o_ridx;  o_ridx += I.m + 1;
    I.rcnt = W.rcnt + o_m;     o_m += I.m;
    I.bfl = W.bfl + o_bfl;     o_bfl += I.r_max + 1;
    I.seg = W.seg + o_seg;     o_seg += I.nb_max * I.nv + 1;
    I.bcost = W.bcost + o_blk; o_blk += I.nb_max + 1;
    I.dflag = nullptr;
    I.rowlist = (int32_t*)(w + B.rowlist[i]);
    I.rowcnt = (int32_t*)(w + B.rowcnt[i]);
    I.bstart = (int32_t*)(w + B.bstart[i]);
    I.vbase = nullptr;
    I.pos = (int32_t*)(w + B.pos[i]);
    I.ent = (uint2*)(w + B.ent[i]);
    I.rowinfo = (int2*)(w + B.rowinfo[i]);
    I.rpart = rpart_ints(I.m, I.n) ? (int32_t*)(w + B.rpart[i]) : nullptr;
    item_offsets(I, Z);
    BatchOut& O = outs[i];
    std::memset(&O, 0, sizeof O);
    O.slices = P.slices; O.Ahat = Ahat[i]; O.ld = ld[i];
    O.part = (float*)(w + B.part[i]);
    O.d = d[i]; O.n = I.n;
    O.o_out = o_out;  if (P.slices > 1) o_out += d[i] * I.n;
    SketchParams& K = O.P;
    K = make_params(P, I, d[i], 0, seed[i]);
    if (P.slices > 1) { K.out = (float*)O.part; K.ld = d[i]; K.split_stride = d[i] * I.n; }
    else { K.out = Ahat[i]; K.ld = ld[i]; K.split_stride = 0; }
  }
  // work list: grouped by distribution, longest units first (LPT)
  struct U { double cost; int32_t item, unit; int32_t dist; };
  std::vector<U> units;
  for (int i = 0; i < count; ++i) {
    const Plan& P = B.plans[i];
    const int32_t nu = P.tiles * P.ncr * P.splits;
    for (int32_t u = 0; u < nu; ++u) units.push_back({P.cost / nu, i, u, unit_kind(P, dist[i])});
  }
  std::stable_sort(units.begin(), units.end(), [](const U& a, const U& b) {
    if (a.dist != b.dist) return a.dist < b.dist;
    return a.cost > b.cost;
  });
  std::vector<int2> work(std::max<size_t>(units.size(), 1));
  for (size_t k = 0; k < units.size(); ++k) work[k] = make_int2(units[k].item, units[k].unit);
  // host vectors are staged by the runtime before these calls return
  if (hipMemcpyAsync(d_items, items.data(), sizeof(Item) * count, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return SK_EHIP;
  if (hipMemcpyAsync(d_outs, outs.data(), sizeof(BatchOut) * count, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return SK_EHIP;
  if (hipMemcpyAsync(d_work, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return SK_EHIP;

  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(count * (int64_t)sizeof(Header) / 4, 256)),
                     dim3(256), 0, st, (int32_t*)hdrs, count * (int64_t)sizeof(Header) / 4, 0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, counters, int64_t(8), 0);
  // a1 + a2 for every item at once
  if ((s = run_inspector(d_items, count, Z, W, st)) != SK_OK) return s;
  if ((s = run_block_costs(d_items, count, Z, W, st)) != SK_OK) return s;
  // a7: one persistent launch per kind of work unit present
  const int cus = current_cus();
  int64_t first = 0;
  for (int kind = 0; kind < 5; ++kind) {
    if (B.units[kind] == 0) continue;
    if (kind < 3) {
      PersistentKernel kern = V.p[kind];
      if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)B.lds[kind]) != hipSuccess)
        return SK_EHIP;
      const int per_cu = V.wgs >= 1024 ? 1 : 2;
      const int64_t grid = std::min<int64_t>(B.units[kind], (int64_t)cus * per_cu);
      hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(V.wgs), B.lds[kind], st, d_outs,
                         d_work + first, (int)B.units[kind], counters + kind);
    } else {
      // one workgroup per CU: the two tile copies take most of the LDS
      const int64_t grid = std::min<int64_t>(B.units[kind], (int64_t)cus);
      const bool bf = kind == 2 + MF_BF16;
      const void* kern = bf ? (const void*)k_sketch_mfma_persistent<MF_BF16>
                            : (const void*)k_sketch_mfma_persistent<MF_FP8>;
      if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)B.lds[kind]) != hipSuccess)
        return SK_EHIP;
      if (bf)
        hipLaunchKernelGGL(k_sketch_mfma_persistent<MF_BF16>, dim3((unsigned)grid),
                           dim3(MF_THREADS), B.lds[kind], st, d_outs, d_work + first,
                           (int)B.units[kind], counters + kind);
      else
        hipLaunchKernelGGL(k_sketch_mfma_persistent<MF_FP8>, dim3((unsigned)grid),
                           dim3(MF_THREADS), B.lds[kind], st, d_outs, d_work + first,
                           (int)B.units[kind], counters + kind);
    }
    if ((s = launch_ok()) != SK_OK) return s;
    first += B.units[kind];
  }
  // a6 for every item with split partials
  if (B.t_out > 0)
    hipLaunchKernelGGL(k_batch_reduce, dim3(blocks_for(B.t_out, 256)), dim3(256), 0, st, d_outs,
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
    chosen[i].variant = P.mfma ? 0 : P.variant + 1;
    // sparse items: no dense blocks (and no matrix-core path); matrix-core
    // items: the threshold that picked it (the caller's, else the batch's),
    // so a single call with this tuning takes the same path
    chosen[i].dense_min_pct =
        P.mfma ? (tune && tune[i].dense_min_pct > 0 ? tune[i].dense_min_pct : kMfmaBatchPct[prec])
               : 101;
    chosen[i].tile_rows = P.mfma ? 0 : P.d_b;
    chosen[i].col_split = 1;
    chosen[i].balance = 1;  // (a batch keeps every item's rows in order)
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
    else if (h[i].status & ST_CAPACITY) si = SK_EUNSUPPORTED;
    statuses[i] = si;
    if (si != SK_OK) worst = si;
  }
  return worst;
}

sk_status sk_plan_info(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                       const sk_tuning* tune, double* info, int32_t ninfo) {
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || dist < 0 || dist > 2 || prec < 0 || prec > 2 || !info || ninfo < 1)
    return SK_EINVAL;
  sk_tuning cached;
  tune = effective_tuning(A, d, dist, prec, tune, cached);
  Plan P;
  if (!plan_any(A->m, A->n, A->nnz, d, dist, prec, tune, P)) return SK_EINVAL;
  const double v[6] = {tile_time_us(P), kji_time_us(A->n, A->nnz, d, dist),
                       (double)choose_kernel(A, d, dist, prec, tune), P.cost,
                       (double)(P.variant + 1), (double)(P.mfma ? 0 : P.bal_sb)};
  for (int i = 0; i < ninfo && i < 6; ++i) info[i] = v[i];
  return SK_OK;
}

sk_status sk_autotune(const sk_csc* A, int64_t d, int32_t dist, sk_tuning* out) {
  if (!out) return SK_EINVAL;
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || dist < 0 || dist > 2) return SK_EINVAL;
  sk_tuning cached;
  const sk_tuning* tune = effective_tuning(A, d, dist, SK_PREC_F32, nullptr, cached);
  std::memset(out, 0, sizeof *out);
  if (choose_kernel(A, d, dist, SK_PREC_F32, tune) == KERNEL_KJI) {
    out->kernel = KERNEL_KJI;
    return SK_OK;
  }
  Plan P;
  if (!plan_for(A->m, A->n, A->nnz, d, dist, tune, P)) return SK_EINVAL;
  out->kernel = KERNEL_TILE;
  out->rows_per_block = P.m_b;
  out->splits = P.splits;
  out->variant = P.variant + 1;
  out->dense_min_pct = P.dense_pct ? P.dense_pct : 101;
  out->tile_rows = P.d_b;
  out->col_split = P.nv != A->n ? 2 : 1;
  out->balance = P.bal_sb ? 2 : 1;
  return SK_OK;
}

sk_status sk_autotune_workspace(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                                size_t* bytes) {
  if (!bytes) return SK_EINVAL;
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || dist < 0 || dist > 2 || prec < 0 || prec > 2) return SK_EINVAL;
  if (prec != SK_PREC_F32 && dist != SK_RADEMACHER) return SK_EUNSUPPORTED;
  size_t most = 0;
  for (const sk_tuning& t : tune_candidates_all(A, d, dist, prec)) {
    size_t b = 0;
    if (sk_sketch_workspace(A, d, dist, prec, &t, &b) == SK_OK) most = std::max(most, b);
  }
  *bytes = most;
  return SK_OK;
}

sk_status sk_autotune_measure(const sk_csc* A, int64_t d, int32_t dist, uint64_t seed,
                              int32_t prec, float* Ahat, int64_t ld, void* ws, size_t ws_bytes,
                              void* hip_stream, sk_tuning* out, double* best_ms) {
  if (!out) return SK_EINVAL;
  sk_status s = check_csc(A);
  if (s != SK_OK) return s;
  if (d < 1 || !Ahat || ld < d || dist < 0 || dist > 2 || prec < 0 || prec > 2) return SK_EINVAL;
  size_t need = 0;
  if ((s = sk_autotune_workspace(A, d, dist, prec, &need)) != SK_OK) return s;
  if (!ws || ws_bytes < need) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  // stage one: the two kernels, and every S-tile kernel shape at the
  // model's splits
  std::vector<std::pair<double, sk_tuning>> timed;
  double best = INFINITY;
  for (const sk_tuning& t : tune_stage_one(A, dist, prec)) {
    double ms = 0.0;
    s = time_call(A, d, dist, seed, prec, t, Ahat, ld, ws, ws_bytes, st, 1.5 * best, &ms);
    if (s == SK_EUNSUPPORTED || s == SK_EINVAL) continue;  // not a form this request has
    if (s != SK_OK) return s;
    // an invalid A: report it and cache nothing; a plan whose block bound
    // the matrix exceeds: not a candidate
    s = sk_sketch_status(ws, st, nullptr, nullptr);
    if (s == SK_EUNSUPPORTED) continue;
    if (s != SK_OK) return s;
    timed.emplace_back(ms, t);
    best = std::min(best, ms);
  }
  if (timed.empty()) return SK_EUNSUPPORTED;
  // stage two: the splits of the three fastest S-tile shapes
  std::vector<std::pair<double, sk_tuning>> tiles;
  for (const auto& e : timed)
    if (e.second.kernel == KERNEL_TILE) tiles.push_back(e);
  std::sort(tiles.begin(), tiles.end(),
            [](const auto& a, const auto& b) { return a.first < b.first; });
  for (size_t i = 0; i < tiles.size() && i < 3; ++i) {
    for (const sk_tuning& t : tune_stage_two(A, d, dist, prec, tiles[i].second.variant)) {
      double ms = 0.0;
      s = time_call(A, d, dist, seed, prec, t, Ahat, ld, ws, ws_bytes, st, 1.5 * best, &ms);
      if (s == SK_EUNSUPPORTED || s == SK_EINVAL) continue;
      if (s != SK_OK) return s;
      s = sk_sketch_status(ws, st, nullptr, nullptr);
      if (s == SK_EUNSUPPORTED) continue;
      if (s != SK_OK) return s;
      timed.emplace_back(ms, t);
      best = std::min(best, ms);
    }
  }
  auto faster = [](const auto& a, const auto& b) { return a.first < b.first; };
  // stage three: the winner with the balanced row blocks switched
  sk_tuning flip;
  if (tune_stage_three(A, d, dist, prec, std::min_element(timed.begin(), timed.end(), faster)->second,
                       &flip)) {
    double ms = 0.0;
    s = time_call(A, d, dist, seed, prec, flip, Ahat, ld, ws, ws_bytes, st, 1.5 * best, &ms);
    if (s == SK_OK) s = sk_sketch_status(ws, st, nullptr, nullptr);
    if (s == SK_OK) timed.emplace_back(ms, flip);
    else if (s != SK_EUNSUPPORTED && s != SK_EINVAL) return s;
  }
  const auto win = std::min_element(timed.begin(), timed.end(), faster);
  *out = win->second;
  if (best_ms) *best_ms = win->first;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_plans[shape_key(A, d, dist, prec)] = win->second;
  }
  // leave the sketch of the chosen tuning in A_hat
  return sketch_impl(A, 0, d, dist, seed, prec, out, Ahat, ld, ws, ws_bytes, hip_stream,
                     GEN_PHILOX, nullptr, 0);
}

int sk_plan_cache_lookup(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                         sk_tuning* out) {
  if (!A || !out) return SK_EINVAL;
  std::lock_guard<std::mutex> g(g_plan_mu);
  const auto it = g_plans.find(shape_key(A, d, dist, prec));
  if (it == g_plans.end()) return 0;
  *out = it->second;
  return 1;
}

void sk_plan_cache_clear(void) {
  std::lock_guard<std::mutex> g(g_plan_mu);
  g_plans.clear();
}

// ------------------------------------------------------------------ SAP
sk_status sk_qr_f64_workspace(int64_t d, int64_t n, size_t* bytes) {
  if (!bytes || n < 1 || d < n) return SK_EINVAL;
  *bytes = (size_t)(align_up(8 * n) + 8 * QR_NB * QR_NB);
  return SK_OK;
}

sk_status sk_qr_f64(int64_t d, int64_t n, double* A, int64_t lda, double* R, int64_t ldr,
                    void* ws, size_t ws_bytes, void* hip_stream) {
  if (n < 1 || d < n || !A || lda < d || !R || ldr < n) return SK_EINVAL;
  size_t need = 0;
  sk_qr_f64_workspace(d, n, &need);
  if (!ws || ws_bytes < need) return SK_EWORKSPACE;
  double* tau = (double*)ws;
  double* T = (double*)((char*)ws + align_up(8 * n));
  return qr_launch(d, n, A, lda, R, ldr, tau, T, (hipStream_t)hip_stream);
}

sk_status sk_trinv_f64(int64_t n, const double* R, int64_t ldr, double* Rinv, int64_t ldi,
                       void* hip_stream) {
  if (n < 1 || n > SAP_MAX_N || !R || !Rinv || ldr < n || ldi < n) return SK_EINVAL;
  return trinv_launch(n, R, ldr, Rinv, ldi, (hipStream_t)hip_stream);
}

sk_status sk_svd_f64_workspace(int64_t rows, int64_t n, size_t* bytes) {
  if (!bytes || n < 1 || rows < n || n > SAP_MAX_N || n >= INT32_MAX / 2) return SK_EINVAL;
  *bytes = (size_t)align_up((int64_t)sizeof(JacobiCtl));
  return SK_OK;
}

sk_status sk_svd_f64(int64_t rows, int64_t n, double* G, double* V, double* sigma,
                     int32_t* sweeps, void* ws, size_t ws_bytes, void* hip_stream) {
  size_t need = 0;
  sk_status s = sk_svd_f64_workspace(rows, n, &need);
  if (s != SK_OK) return s;
  if (!G || !V || !sigma) return SK_EINVAL;
  if (!ws || ws_bytes < need) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  JacobiCtl* ctl = (JacobiCtl*)ws;
  if ((s = jacobi_svd(rows, n, G, V, ctl, sigma, st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)n), dim3(SVD_THREADS), 0, st, (const double*)G,
                     rows, sigma);
  if ((s = launch_ok()) != SK_OK) return s;
  if (sweeps) {
    JacobiCtl h;
    if (hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SK_EHIP;
    *sweeps = h.converged ? h.sweeps : -h.sweeps;
  }
  return SK_OK;
}

sk_status sk_sap_workspace(const sk_csc* A, const sk_sap_params* p, size_t* bytes) {
  if (!bytes) return SK_EINVAL;
  SapLayout L;
  sk_status s = sap_layout(A, p, L);
  if (s != SK_OK) return s;
  *bytes = (size_t)L.total;
  return SK_OK;
}

sk_status sk_sap_begin(const sk_csc* A, const double* b, const sk_sap_params* p, void* ws,
                       size_t ws_bytes, void* hip_stream) {
  SapLayout L;
  sk_status s = sap_layout(A, p, L);
  if (s != SK_OK) return s;
  if (!b) return SK_EINVAL;
  if (!ws || ws_bytes < (size_t)L.total) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  char* w = (char*)ws;
  const int64_t m = A->m, n = A->n, nnz = A->nnz, d = p->d;
  LsqrState* state = (LsqrState*)(w + L.state);
  const double ctol = p->conlim > 0.0 ? 1.0 / p->conlim : 0.0;
  hipLaunchKernelGGL(k_lsqr_set, dim3(1), dim3(64), 0, st, state, p->atol, p->btol, ctol,
                     p->iter_lim, (int32_t)n);
  // the sketch: FP32 and widened to FP64 for the QR form; FP64 throughout
  // for the SVD form (an FP32 sketch's rounding would leave singular values
  // near 1e-7 sigma_max where A has none, far above the drop threshold)
  double* q = (double*)(w + L.q);
  if (L.svd) {
    if ((s = colwise_impl<double>(A, 0, d, p->dist, p->seed, q, d, w + L.sk_ws,
                                  (size_t)L.sk_bytes, st)) != SK_OK)
      return s;
  } else {
    float* ahat = (float*)(w + L.ahat);
    if ((s = sk_sketch(A, 0, d, p->dist, p->seed, p->prec, nullptr, ahat, d, w + L.sk_ws,
                       (size_t)L.sk_bytes, hip_stream)) != SK_OK)
      return s;
    hipLaunchKernelGGL(k_widen, dim3(blocks_for(d * n, 256)), dim3(256), 0, st, ahat, d, d, n, q,
                       d);
  }
  // R and R^{-1}
  double* R = (double*)(w + L.r);
  double* Ri = (double*)(w + L.rinv);
  if ((s = qr_launch(d, n, q, d, R, n, (double*)(w + L.tau), (double*)(w + L.tq), st)) != SK_OK)
    return s;
  if (L.svd) {
    // Sec. V-E-1: N = V_r diag(1 / sigma_r) from the SVD of R (that of the
    // sketch), through one-sided Jacobi on R^T (no V to carry)
    double* Gt = (double*)(w + L.vsv);
    hipLaunchKernelGGL(k_transpose, dim3(blocks_for(n * n, 256)), dim3(256), 0, st,
                       (const double*)R, n, Gt);
    double* sig = (double*)(w + L.sig);
    if ((s = jacobi_svd(n, n, Gt, nullptr, (JacobiCtl*)(w + L.jctl), sig, st)) != SK_OK) return s;
    hipLaunchKernelGGL(k_col_norms, dim3((unsigned)n), dim3(SVD_THREADS), 0, st,
                       (const double*)Gt, n, sig);
    hipLaunchKernelGGL(k_svd_rank, dim3(1), dim3(SVD_THREADS), 0, st, (const double*)sig, n,
                       (const JacobiCtl*)(w + L.jctl), (double*)(w + L.smax), state);
    hipLaunchKernelGGL(k_svd_precond, dim3(blocks_for(n * n, 256)), dim3(256), 0, st,
                       (const double*)Gt, (const double*)sig, (const double*)(w + L.smax), n,
                       Ri);
  } else if ((s = trinv_launch(n, R, n, Ri, n, st)) != SK_OK) {
    return s;
  }
  hipLaunchKernelGGL(k_transpose, dim3(blocks_for(n * n, 256)), dim3(256), 0, st, (const double*)Ri,
                     n, (double*)(w + L.rinvt));
  // FP64 values, row counts, row-major copy (only of input the sketch's
  // validation passed: its header sits at the start of its workspace)
  const Header* skh = (const Header*)(w + L.sk_ws);
  int32_t* rcnt = (int32_t*)(w + L.rcnt);
  int32_t* rowptr = (int32_t*)(w + L.rowptr);
  int32_t* cursor = (int32_t*)(w + L.cursor);
  double* v64 = (double*)(w + L.v64);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(m, 256 * 8)), dim3(256), 0, st, rcnt, m, 0);
  if (nnz > 0)
    hipLaunchKernelGGL(k_csc_f64_count, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, A->rowidx,
                       A->vals, A->vtype, nnz, v64, rcnt, skh);
  hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(m, 256)), dim3(256), 0, st, rcnt, m, rowptr);
  if ((s = scan_i32(rowptr, m, (int32_t*)(w + L.sums), st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(m, 256)), dim3(256), 0, st, rowptr, m, cursor);
  if (nnz > 0) {
    hipLaunchKernelGGL(k_csr_scatter, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, A->colptr,
                       A->rowidx, v64, n, nnz, cursor, (int32_t*)(w + L.ccol),
                       (double*)(w + L.cval), skh);
  }
  // long rows: listed, sorted by a workgroup each; short rows by a thread
  int32_t* lidx = (int32_t*)(w + L.lidx);
  hipLaunchKernelGGL(k_long_flags, dim3(blocks_for(m, 256)), dim3(256), 0, st, rowptr, m, lidx);
  if ((s = scan_i32(lidx, m, (int32_t*)(w + L.sums), st)) != SK_OK) return s;
  hipLaunchKernelGGL(k_long_list, dim3(blocks_for(m, 256)), dim3(256), 0, st, lidx, m,
                     (int32_t*)(w + L.lrows));
  if (nnz > 0) {
    hipLaunchKernelGGL(k_csr_sort_rows, dim3(blocks_for(m, 256)), dim3(256), 0, st, rowptr, m,
                       (int32_t*)(w + L.ccol), (double*)(w + L.cval));
    hipLaunchKernelGGL(k_csr_sort_long, dim3((unsigned)L.nlong_max), dim3(SAP_THREADS), 0, st,
                       rowptr, lidx, m, (const int32_t*)(w + L.lrows), (int32_t*)(w + L.ccol),
                       (double*)(w + L.cval));
  }
  int32_t* cbase = (int32_t*)(w + L.cbase);
  hipLaunchKernelGGL(k_col_chunks, dim3(blocks_for(n, 256)), dim3(256), 0, st, A->colptr, n, cbase,
                     skh);
  if ((s = scan_i32(cbase, n, (int32_t*)(w + L.sums), st)) != SK_OK) return s;
  // LSQR start: beta u = b, alpha v = (A R^{-1})^T u, w = v, y = 0
  double* u = (double*)(w + L.u);
  double* partial = (double*)(w + L.partial);
  hipLaunchKernelGGL(k_lsqr_av<true>, dim3((unsigned)L.nblk_m), dim3(SAP_THREADS), 0, st,
                     (const int32_t*)nullptr, (const int32_t*)nullptr, (const double*)nullptr, m,
                     (const double*)nullptr, b, u, partial, state);
  hipLaunchKernelGGL(k_lsqr_beta<true>, dim3(1), dim3(1024), 0, st, partial, L.nblk_m,
                     (const double*)nullptr, int64_t(0), state);
  hipLaunchKernelGGL(k_lsqr_atu, dim3(blocks_for(L.nchunk_max * 64, 256)), dim3(256), 0, st,
                     A->colptr, A->rowidx, (const double*)v64, n, (const int32_t*)cbase, u,
                     (double*)(w + L.cpart), state, skh);
  hipLaunchKernelGGL(k_lsqr_colsum, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                     (const int32_t*)cbase, n, (const double*)(w + L.cpart), (double*)(w + L.sn),
                     state);
  hipLaunchKernelGGL(L.svd ? k_gemv_upper_t<false> : k_gemv_upper_t<true>,
                     dim3(blocks_for(n * 64, 256)), dim3(256), 0, st,
                     (const double*)Ri, n, n, (const double*)(w + L.sn), (double*)(w + L.t2),
                     state);
  hipLaunchKernelGGL(k_lsqr_update<true>, dim3(1), dim3(1024), 0, st, n,
                     (const double*)(w + L.t2), (double*)(w + L.v), (double*)(w + L.w),
                     (double*)(w + L.y), state);
  hipLaunchKernelGGL(k_lsqr_input_check, dim3(1), dim3(64), 0, st, state, skh);
  return launch_ok();
}

sk_status sk_sap_iterate(const sk_csc* A, const sk_sap_params* p, int32_t iters, void* ws,
                         size_t ws_bytes, void* hip_stream) {
  SapLayout L;
  sk_status s = sap_layout(A, p, L);
  if (s != SK_OK) return s;
  if (iters < 0) return SK_EINVAL;
  if (!ws || ws_bytes < (size_t)L.total) return SK_EWORKSPACE;
  for (int32_t k = 0; k < iters; ++k) lsqr_iteration(A, L, (char*)ws, (hipStream_t)hip_stream);
  return launch_ok();
}

sk_status sk_sap_finish(const sk_csc* A, const sk_sap_params* p, double* x, void* ws,
                        size_t ws_bytes, void* hip_stream) {
  SapLayout L;
  sk_status s = sap_layout(A, p, L);
  if (s != SK_OK) return s;
  if (!x) return SK_EINVAL;
  if (!ws || ws_bytes < (size_t)L.total) return SK_EWORKSPACE;
  char* w = (char*)ws;
  const int64_t n = A->n;
  hipLaunchKernelGGL(L.svd ? k_gemv_upper_final<false> : k_gemv_upper_final<true>,
                     dim3(blocks_for(n, 256)), dim3(256), 0,
                     (hipStream_t)hip_stream, (const double*)(w + L.rinv), n, n,
                     (const double*)(w + L.y), x);
  return launch_ok();
}

sk_status sk_sap_read_info(const sk_csc* A, const sk_sap_params* p, const void* ws,
                           size_t ws_bytes, void* hip_stream, sk_sap_info* info) {
  SapLayout L;
  sk_status s = sap_layout(A, p, L);
  if (s != SK_OK) return s;
  if (!info) return SK_EINVAL;
  if (!ws || ws_bytes < (size_t)L.total) return SK_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(info, (const char*)ws + L.state, sizeof *info, hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return SK_EHIP;
  return sk_sketch_status((const char*)ws + L.sk_ws, hip_stream, nullptr, nullptr);
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

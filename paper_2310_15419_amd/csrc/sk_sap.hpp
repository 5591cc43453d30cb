// sk_sap.hpp -- device kernels of the sketch-and-precondition least-squares
// solve (paper Sec. V-E): QR of the sketch A_hat = S A gives R, and LSQR runs
// on the preconditioned operator A R^{-1}; x = R^{-1} y.  Everything is FP64
// (the sketch itself is accumulated in FP32 and widened), since the
// orthogonalisation and the Krylov recurrences need the precision.
//
//   QR      blocked Householder, panels of QR_NB columns: one workgroup
//           factors a panel (reflectors stored below the diagonal as in
//           LAPACK, plus the triangular factor T of the compact WY form
//           I - V T V^T), then every trailing column gets
//           C <- C - V T^T (V^T C) from its own workgroup.
//   R^{-1}  upper triangular inverse, one workgroup per column (column-
//           oriented back substitution); LSQR then applies R^{-1} and R^{-T}
//           as plain matrix-vector products.
//   CSR     a row-major copy of A for A z (deterministic: counts, scan,
//           scatter, then each row sorted by column), and FP64 values of the
//           CSC for A^T u, whose heavy columns are cut into chunks summed in
//           a fixed order.
//   LSQR    the recurrences of Paige and Saunders' LSQR (the same quantities
//           and stopping tests as their published algorithm) with all
//           scalars on the device; every kernel returns at once after the
//           solve has stopped, so the host can enqueue iterations in chunks
//           and poll.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_inspect.hpp"

namespace sk {

constexpr int QR_NB = 16;          // panel width
constexpr int SAP_THREADS = 256;
constexpr int SAP_CHUNK = 2048;    // entries per A^T u chunk

// ---------------------------------------------------------------- helpers
// v from another lane by a DPP move (the two halves of a double apart);
// lanes outside row_mask get 0
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}

// Sum over the 64 lanes of a wave (all active), every lane gets it: pairs
// and quads by quad permutations, 8- and 16-lane rows by mirrors, then
// lane 15 of each row into the next (rows 1, 3) and lane 31 into rows 2, 3,
// so lane 63 holds the total.  DPP moves stay in the VALU, so no step waits
// on the LDS crossbar.  (The order of the additions is fixed.)
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm 1,0,3,2
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm 2,3,0,1
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));  // in every lane
}

// sum over the workgroup (blockDim.x a multiple of 64, <= 1024); every
// thread gets the result.  sh: 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += sh[w];  // fixed order
  return s;
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int64_t count, int32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

// FP32 sketch (d x n, ld) -> FP64 (d x n, ldq)
__global__ void k_widen(const float* __restrict__ src, int64_t ld, int64_t d, int64_t n,
                        double* __restrict__ dst, int64_t ldq) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d * n) return;
  const int64_t j = t / d, i = t - j * d;
  dst[i + j * ldq] = (double)src[i + j * ld];
}

// ------------------------------------------------------------------- QR
// Factor columns [j0, j0 + nb) of A (d x n, column-major, lda), rows >= j0.
// Reflector k (global column c = j0 + k): H = I - tau v v^T with v[c] = 1 and
// v[r] (r > c) stored in A[r, c]; A[c, c] becomes beta.  T (ldt = QR_NB) is
// the upper triangular factor with H_0 ... H_{nb-1} = I - V T V^T.
// One workgroup; partial dot products of the panel columns in registers.
__global__ __launch_bounds__(SAP_THREADS) void k_qr_panel(double* __restrict__ A, int64_t lda,
                                                           int64_t d, int64_t j0, int nb,
                                                           double* __restrict__ tau,
                                                           double* __restrict__ T) {
  __shared__ double sh[16];
  __shared__ double s_dot[QR_NB][SAP_THREADS / 64];
  __shared__ double s_w[QR_NB];
  __shared__ double s_t[QR_NB][QR_NB];  // T[i][j] (the panel's T, kept here)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int k = 0; k < nb; ++k) {
    const int64_t c = j0 + k;
    double* col = A + c * lda;
    // ||A[c+1:, c]||^2
    double ss = 0.0;
    for (int64_t r = c + 1 + tid; r < d; r += SAP_THREADS) ss += col[r] * col[r];
    const double sigma = block_sum(ss, sh);
    const double alpha = col[c];
    double t_k, beta, scale;
    if (sigma == 0.0) {
      t_k = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t_k = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v below the diagonal
    for (int64_t r = c + 1 + tid; r < d; r += SAP_THREADS) col[r] *= scale;
    __syncthreads();
    if (tid == 0) {
      col[c] = beta;
      tau[c] = t_k;
    }
    // dots of v with every other panel column: j < k gives V_j^T v (for T),
    // j > k gives v^T A[:, j] (for the update)
    double part[QR_NB];
#pragma unroll
    for (int j = 0; j < QR_NB; ++j) part[j] = 0.0;
    for (int64_t r = c + 1 + tid; r < d; r += SAP_THREADS) {
      const double vr = col[r];
#pragma unroll
      for (int j = 0; j < QR_NB; ++j)
        if (j < nb && j != k) part[j] += A[r + (j0 + j) * lda] * vr;
    }
#pragma unroll
    for (int j = 0; j < QR_NB; ++j) {
      const double s = wave_sum(part[j]);
      if (lane == 0) s_dot[j][wave] = s;
    }
    __syncthreads();
    if (tid < nb && tid != k) {
      double s = 0.0;
      for (int w = 0; w < SAP_THREADS / 64; ++w) s += s_dot[tid][w];
      // the row-c term: v[c] = 1
      s_w[tid] = s + A[c + (j0 + tid) * lda];
    }
    __syncthreads();
    // apply H to the panel columns right of c
    for (int j = k + 1; j < nb; ++j) {
      const double wj = t_k * s_w[j];
      double* cj = A + (j0 + j) * lda;
      for (int64_t r = c + 1 + tid; r < d; r += SAP_THREADS) cj[r] -= wj * col[r];
      if (tid == 0) cj[c] -= wj;
    }
    // T[0:k, k] = -tau_k T[0:k, 0:k] z, z_j = V_j^T v (j < k); T[k, k] =
    // tau_k.  Thread i < k takes T[i][k] (T's earlier columns of row i were
    // written by the same thread).
    if (tid < k) {
      double s = 0.0;
      for (int j = tid; j < k; ++j) s += s_t[tid][j] * s_w[j];
      s_t[tid][k] = -t_k * s;
    }
    if (tid == 0) s_t[k][k] = t_k;
    __syncthreads();
  }
  // T (ldt = QR_NB): the upper triangle, zeros below
  if (tid < QR_NB * nb) {
    const int i = tid % QR_NB, j = tid / QR_NB;
    T[i + j * QR_NB] = i <= j ? s_t[i][j] : 0.0;
  }
}

// The same factorisation for a panel of rows j0..d-1 (at most QR_REG_ROWS)
// and nb <= QR_NB_REG columns, by one workgroup of QR_PT threads that keep
// the panel in registers: thread t holds rows t, t + QR_PT, ... of every
// panel column for the whole panel.  Only the partial sums, the T factor and
// row k (published by its owner, thread k) go through LDS.  A column takes
// three barriers: its norm (summed from the previous column's update), its
// dot products with the other panel columns (taken while the reflector is
// scaled), and their totals; the update of the later columns computes the
// next column's norm on the way.
constexpr int QR_NB_REG = 8;
constexpr int QR_PT = 1024;        // threads of the panel workgroup (measured: 256 and 512 slower)
constexpr int QR_REG_ROWS = 3 * QR_PT;  // panel rows held: 3 per thread
__global__ __launch_bounds__(QR_PT) void k_qr_panel_regs(double* __restrict__ A, int64_t lda,
                                                        int64_t d, int64_t j0, int nb,
                                                        double* __restrict__ tau,
                                                        double* __restrict__ T) {
  constexpr int RPT = (QR_REG_ROWS + QR_PT - 1) / QR_PT;
  static_assert(QR_NB_REG <= QR_PT, "row k of the panel is owned by thread k");
  __shared__ double s_norm[QR_PT / 64];
  __shared__ double s_dot[QR_NB_REG][QR_PT / 64];
  __shared__ double s_w[QR_NB_REG];
  __shared__ double s_row[QR_NB_REG];           // row k of the panel's columns
  __shared__ double s_t[QR_NB_REG][QR_NB_REG];  // T[i][j] (the panel's T, kept here)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int rows = (int)(d - j0);
  // x[j][q]: row tid + QR_PT q of panel column j
  double x[QR_NB_REG][RPT];
#pragma unroll
  for (int j = 0; j < QR_NB_REG; ++j)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + QR_PT * q;
      x[j][q] = j < nb && r < rows ? A[j0 + r + (j0 + j) * lda] : 0.0;
    }
  {
    // per-wave partial sums of squares of column 0 below its diagonal, and
    // row 0 published
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + QR_PT * q;
      if (r > 0 && r < rows) ss += x[0][q] * x[0][q];
    }
    ss = wave_sum(ss);
    if (lane == 0) s_norm[wave] = ss;
    if (tid == 0)
#pragma unroll
      for (int j = 0; j < QR_NB_REG; ++j) s_row[j] = x[j][0];
  }
#pragma unroll
  for (int k = 0; k < QR_NB_REG; ++k) {
    if (k >= nb) break;
    __syncthreads();  // norm partials and row k are final
    double sigma = 0.0;
    for (int w = 0; w < QR_PT / 64; ++w) sigma += s_norm[w];  // fixed order
    const double alpha = s_row[k];
    double t_k, beta, scale;
    if (sigma == 0.0) {
      t_k = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t_k = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v = the scaled column below row k, and its dots with the other columns
    double part[QR_NB_REG];
#pragma unroll
    for (int j = 0; j < QR_NB_REG; ++j) part[j] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + QR_PT * q;
      if (r > k && r < rows) {
        const double vr = x[k][q] * scale;
        x[k][q] = vr;
#pragma unroll
        for (int j = 0; j < QR_NB_REG; ++j)
          if (j < nb && j != k) part[j] += x[j][q] * vr;
      }
    }
#pragma unroll
    for (int j = 0; j < QR_NB_REG; ++j) {
      const double sj = wave_sum(part[j]);
      if (lane == 0) s_dot[j][wave] = sj;
    }
    __syncthreads();
    if (tid < nb && tid != k) {
      double sj = 0.0;
      for (int w = 0; w < QR_PT / 64; ++w) sj += s_dot[tid][w];
      s_w[tid] = sj + s_row[tid];  // row c: v[c] = 1
    }
    __syncthreads();
    // columns j > k: a_j -= t_k w_j v (row k: v = 1), and the partial norm
    // of column k + 1 below its diagonal
    double ss = 0.0;
#pragma unroll
    for (int j = 0; j < QR_NB_REG; ++j) {
      if (j > k && j < nb) {
        const double wj = t_k * s_w[j];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = tid + QR_PT * q;
          if (r > k && r < rows) {
            const double y = x[j][q] - wj * x[k][q];
            x[j][q] = y;
            if (j == k + 1 && r > k + 1) ss += y * y;
          } else if (r == k) {
            x[j][q] -= wj;
          }
        }
      }
    }
    if (tid == k) x[k][0] = beta;  // (row k of column k: R's diagonal)
    if (k + 1 < nb) {
      ss = wave_sum(ss);
      if (lane == 0) s_norm[wave] = ss;
      if (tid == k + 1)
#pragma unroll
        for (int j = 0; j < QR_NB_REG; ++j) s_row[j] = x[j][0];
    }
    // T column k: thread i < k takes T[i][k] (T's earlier columns of row i
    // were written by the same thread)
    if (tid < k) {
      double si = 0.0;
      for (int j = tid; j < k; ++j) si += s_t[tid][j] * s_w[j];
      s_t[tid][k] = -t_k * si;
    }
    if (tid == 0) {
      tau[j0 + k] = t_k;
      s_t[k][k] = t_k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < QR_NB_REG; ++j)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + QR_PT * q;
      if (j < nb && r < rows) A[j0 + r + (j0 + j) * lda] = x[j][q];
    }
  // T (ldt = QR_NB): the upper triangle, zeros below
  if (tid < QR_NB * nb) {
    const int i = tid % QR_NB, j = tid / QR_NB;
    T[i + j * QR_NB] = i <= j ? s_t[i][j] : 0.0;
  }
}

// C <- C - V T^T (V^T C) for the trailing columns j >= j0 + nb, rows >= j0;
// one workgroup per trailing column.  Rows go in chunks of QU_R per thread
// (strided by the workgroup): a chunk's column values, then each
// reflector's values in the chunk, are loaded together, so a pass waits on
// a few memory round trips rather than one per row step; with one chunk
// (d - j0 <= QU_R * SAP_THREADS) the column stays in registers between the
// passes.
constexpr int QU_R = 8;
__global__ __launch_bounds__(SAP_THREADS) void k_qr_update(double* __restrict__ A, int64_t lda,
                                                            int64_t d, int64_t n, int64_t j0,
                                                            int nb, const double* __restrict__ T) {
  __shared__ double s_dot[QR_NB][SAP_THREADS / 64];
  __shared__ double s_w[QR_NB];
  __shared__ double s_w2[QR_NB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t j = j0 + nb + blockIdx.x;
  if (j >= n) return;
  double* cj = A + j * lda;
  constexpr int64_t CH = (int64_t)QU_R * SAP_THREADS;  // rows per chunk
  // V_i has 1 at row j0 + i, zeros above, A[r, j0 + i] below
  auto vval = [&](int i, int64_t r) {
    const int64_t ri = j0 + i;
    return r > ri ? A[r + ri * lda] : (r == ri ? 1.0 : 0.0);
  };
  double c[QU_R];
  // W = V^T C[:, j]
  double part[QR_NB];
#pragma unroll
  for (int i = 0; i < QR_NB; ++i) part[i] = 0.0;
  for (int64_t r0 = j0; r0 < d; r0 += CH) {
#pragma unroll
    for (int q = 0; q < QU_R; ++q) {
      const int64_t r = r0 + tid + (int64_t)q * SAP_THREADS;
      c[q] = r < d ? cj[r] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) {
      if (i < nb) {
        double v[QU_R];
#pragma unroll
        for (int q = 0; q < QU_R; ++q) {
          const int64_t r = r0 + tid + (int64_t)q * SAP_THREADS;
          v[q] = r < d ? vval(i, r) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QU_R; ++q) part[i] += v[q] * c[q];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QR_NB; ++i) {
    const double s = wave_sum(part[i]);
    if (lane == 0) s_dot[i][wave] = s;
  }
  __syncthreads();
  if (tid < nb) {
    double s = 0.0;
    for (int w = 0; w < SAP_THREADS / 64; ++w) s += s_dot[tid][w];
    s_w[tid] = s;
  }
  __syncthreads();
  // W2 = T^T W
  if (tid < nb) {
    double s = 0.0;
    for (int i = 0; i <= tid; ++i) s += T[i + tid * QR_NB] * s_w[i];
    s_w2[tid] = s;
  }
  __syncthreads();
  // C -= V W2
  double w2[QR_NB];
#pragma unroll
  for (int i = 0; i < QR_NB; ++i) w2[i] = i < nb ? s_w2[i] : 0.0;
  const bool one_chunk = d - j0 <= CH;
  for (int64_t r0 = j0; r0 < d; r0 += CH) {
    if (!one_chunk) {
#pragma unroll
      for (int q = 0; q < QU_R; ++q) {
        const int64_t r = r0 + tid + (int64_t)q * SAP_THREADS;
        c[q] = r < d ? cj[r] : 0.0;
      }
    }
    double acc[QU_R];
#pragma unroll
    for (int q = 0; q < QU_R; ++q) acc[q] = 0.0;
#pragma unroll
    for (int i = 0; i < QR_NB; ++i) {
      if (i < nb) {
        double v[QU_R];
#pragma unroll
        for (int q = 0; q < QU_R; ++q) {
          const int64_t r = r0 + tid + (int64_t)q * SAP_THREADS;
          v[q] = r < d ? vval(i, r) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QU_R; ++q) acc[q] += v[q] * w2[i];
      }
    }
#pragma unroll
    for (int q = 0; q < QU_R; ++q) {
      const int64_t r = r0 + tid + (int64_t)q * SAP_THREADS;
      if (r < d) cj[r] = c[q] - acc[q];
    }
  }
}

// R (n x n, ldr) = upper triangle of the factored A
__global__ void k_qr_extract_r(const double* __restrict__ A, int64_t lda, int64_t n,
                               double* __restrict__ R, int64_t ldr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int64_t j = t / n, i = t - j * n;
  R[i + j * ldr] = i <= j ? A[i + j * lda] : 0.0;
}

// Rinv = R^{-1} (upper triangular); one workgroup per column j: solve
// R x = e_j by column-oriented back substitution with the right-hand side
// and R's diagonal in LDS (n <= SAP_MAX_N); each step's column of R is
// loaded the step before.
constexpr int SAP_MAX_N = 8192;
constexpr int TRI_Q = 4;  // rows per thread held in registers (n <= 1024 all of them)
__global__ __launch_bounds__(SAP_THREADS) void k_trinv_upper(const double* __restrict__ R,
                                                              int64_t ldr, int64_t n,
                                                              double* __restrict__ Ri,
                                                              int64_t ldi) {
  extern __shared__ double rhs[];  // 2 n doubles: the right-hand side, then R's diagonal
  double* diag = rhs + n;
  const int tid = threadIdx.x;
  const int64_t j = blockIdx.x;
  if (j >= n) return;
  for (int64_t i = tid; i < n; i += SAP_THREADS) {
    rhs[i] = i == j ? 1.0 : 0.0;
    diag[i] = i <= j ? R[i + i * ldr] : 1.0;
  }
  // the thread's rows of column c (rows < c) into v; up to TRI_Q rows per
  // thread are held in registers, the rest (n > TRI_Q * SAP_THREADS) read
  // when used
  auto load_col = [&](int64_t c, double (&v)[TRI_Q]) {
#pragma unroll
    for (int q = 0; q < TRI_Q; ++q) {
      const int64_t r = tid + (int64_t)SAP_THREADS * q;
      v[q] = r < c ? R[r + c * ldr] : 0.0;
    }
  };
  auto step = [&](int64_t i, const double (&v)[TRI_Q]) {
    const double xi = rhs[i] / diag[i];
    __syncthreads();  // every thread has read rhs[i]
    if (tid == 0) rhs[i] = xi;
#pragma unroll
    for (int q = 0; q < TRI_Q; ++q) {
      const int64_t r = tid + (int64_t)SAP_THREADS * q;
      if (r < i) rhs[r] -= xi * v[q];
    }
    const double* ci = R + i * ldr;
    for (int64_t r = tid + (int64_t)SAP_THREADS * TRI_Q; r < i; r += SAP_THREADS)
      rhs[r] -= xi * ci[r];
    __syncthreads();
  };
  __syncthreads();
  // two register buffers in turn: a column's loads are issued one step
  // before it is used, and no copy of in-flight registers is made
  double ca[TRI_Q], cb[TRI_Q];
  load_col(j, ca);
  for (int64_t i = j; i >= 0; i -= 2) {
    load_col(i - 1, cb);
    step(i, ca);
    if (i == 0) break;
    load_col(i - 2, ca);
    step(i - 1, cb);
  }
  double* out = Ri + j * ldi;
  for (int64_t i = tid; i < n; i += SAP_THREADS) out[i] = i <= j ? rhs[i] : 0.0;
}


// ------------------------------------------------------------- A copies
// The kernels that index by A's structure run only on input the sketch's
// validation passed (hdr: the sketch's header, final by then on the stream).

// FP64 values of the CSC, and per-row entry counts (rcnt zeroed before)
__global__ void k_csc_f64_count(const int32_t* __restrict__ rowidx, const void* __restrict__ vals,
                                int vtype, int64_t nnz, double* __restrict__ v64,
                                int32_t* __restrict__ rcnt, const Header* __restrict__ hdr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz || hdr->status) return;
  double a;
  if (vtype == 0) a = ((const double*)vals)[p];
  else if (vtype == 1) a = (double)((const float*)vals)[p];
  else a = (double)__uint_as_float((uint32_t)((const uint16_t*)vals)[p] << 16);
  v64[p] = a;
  atomicAdd(&rcnt[rowidx[p]], 1);
}

// scatter into CSR rows (cursor = copy of rowptr); order inside a row is
// fixed afterwards by k_csr_sort_rows
__global__ void k_csr_scatter(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                              const double* __restrict__ v64, int64_t n, int64_t nnz,
                              int32_t* __restrict__ cursor, int32_t* __restrict__ ccol,
                              double* __restrict__ cval, const Header* __restrict__ hdr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz || hdr->status) return;
  int64_t lo = 0, hi = n - 1;  // column of p
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (colptr[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  const int32_t q = atomicAdd(&cursor[rowidx[p]], 1);
  ccol[q] = (int32_t)lo;
  cval[q] = v64[p];
}

// Rows with more than SAP_LONG entries are "long": their products run on a
// whole wave and they are sorted by a workgroup; the rest by one thread.
constexpr int SAP_LONG = 32;
constexpr int SAP_SORT_MAX = 8192;  // entries of a long row sorted in LDS (n <= SAP_MAX_N)

// lflag[r] = row r is long (scanned afterwards into its index in lrows)
__global__ void k_long_flags(const int32_t* __restrict__ rowptr, int64_t m,
                             int32_t* __restrict__ lflag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) lflag[r] = rowptr[r + 1] - rowptr[r] > SAP_LONG ? 1 : 0;
}

__global__ void k_long_list(const int32_t* __restrict__ lidx, int64_t m, int32_t* __restrict__ lrows) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m && lidx[r + 1] > lidx[r]) lrows[lidx[r]] = (int32_t)r;
}

// sort each short CSR row by column (insertion sort; columns are unique)
__global__ void k_csr_sort_rows(const int32_t* __restrict__ rowptr, int64_t m,
                                int32_t* __restrict__ ccol, double* __restrict__ cval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int32_t a = rowptr[r], b = rowptr[r + 1];
  if (b - a > SAP_LONG) return;
  for (int32_t i = a + 1; i < b; ++i) {
    const int32_t c = ccol[i];
    const double v = cval[i];
    int32_t k = i - 1;
    while (k >= a && ccol[k] > c) {
      ccol[k + 1] = ccol[k];
      cval[k + 1] = cval[k];
      --k;
    }
    ccol[k + 1] = c;
    cval[k + 1] = v;
  }
}

// one workgroup per long row: bitonic sort of (column, value) in LDS
__global__ __launch_bounds__(SAP_THREADS) void k_csr_sort_long(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ lidx, int64_t m,
    const int32_t* __restrict__ lrows, int32_t* __restrict__ ccol, double* __restrict__ cval) {
  __shared__ int32_t kc[SAP_SORT_MAX];
  __shared__ int32_t kp[SAP_SORT_MAX];  // position in the row (to move the values)
  const int64_t li = blockIdx.x;
  if (li >= lidx[m]) return;
  const int32_t r = lrows[li];
  const int32_t a = rowptr[r], len = rowptr[r + 1] - a;
  int np2 = 1;
  while (np2 < len) np2 <<= 1;
  for (int i = threadIdx.x; i < np2; i += SAP_THREADS) {
    kc[i] = i < len ? ccol[a + i] : 0x7FFFFFFF;
    kp[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < np2; i += SAP_THREADS) {
        const int jx = i ^ stride;
        if (jx > i) {
          const bool up = (i & size) == 0;
          const int32_t ci = kc[i], cj = kc[jx];
          if ((ci > cj) == up) {
            kc[i] = cj; kc[jx] = ci;
            const int32_t t = kp[i]; kp[i] = kp[jx]; kp[jx] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  // gather the values in the new order, then write both back
  double v[SAP_SORT_MAX / SAP_THREADS];
  int cnt = 0;
  for (int i = threadIdx.x; i < len; i += SAP_THREADS) v[cnt++] = cval[a + kp[i]];
  __syncthreads();
  cnt = 0;
  for (int i = threadIdx.x; i < len; i += SAP_THREADS) {
    cval[a + i] = v[cnt++];
    ccol[a + i] = kc[i];
  }
}

// chunks of at most SAP_CHUNK entries per column: cbase[k] = chunks of k
// (scanned afterwards)
__global__ void k_col_chunks(const int64_t* __restrict__ colptr, int64_t n,
                             int32_t* __restrict__ cbase, const Header* __restrict__ hdr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t c = hdr->status ? 0 : colptr[k + 1] - colptr[k];
  cbase[k] = (int32_t)(c > 0 ? (c + SAP_CHUNK - 1) / SAP_CHUNK : 1);
}

// ------------------------------------------------------------------ LSQR
// The first fields are the public solver info (sk_sap_info in the C header,
// same layout); the rest is private.
struct LsqrState {
  int32_t itn, istop, done, iter_lim;
  double rnorm, arnorm, anorm, acond, xnorm, bnorm, test1, test2, test3;
  int32_t rank, sweeps;  // preconditioner rank; Jacobi sweeps of the SVD form
  // private
  double alpha, beta, rhobar, phibar;
  double ddnorm, res2, xxnorm, z, cs2, sn2;
  double atol, btol, ctol;
  double pad[3];
};

// Rt = R^T (n x n, column-major both)
__global__ void k_transpose(const double* __restrict__ R, int64_t n, double* __restrict__ Rt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int64_t j = t / n, i = t - j * n;
  Rt[j + i * n] = R[i + j * n];
}

// The preconditioner products of LSQR.  M is R^{-1} (upper triangular: the
// QR form, UPPER) or N = V_r diag(1 / sigma_r) (dense: the SVD form).
// t = M v from the transposed copy Mt = M^T (row i of M is column i of Mt,
// contiguous): one wave per row
template <bool UPPER>
__global__ void k_gemv_upper(const double* __restrict__ Rit, int64_t n,
                             const double* __restrict__ v, double* __restrict__ t,
                             const LsqrState* __restrict__ st) {
  if (st->done) return;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const double* row = Rit + i * n;
  double acc = 0.0;
#pragma unroll 4
  for (int64_t j = (UPPER ? i : 0) + lane; j < n; j += 64) acc += row[j] * v[j];
  acc = wave_sum(acc);
  if (lane == 0) t[i] = acc;
}

// t = M^T s: one wave per column j (t[j] = sum_i M[i, j] s[i], i <= j when
// M is upper triangular)
template <bool UPPER>
__global__ void k_gemv_upper_t(const double* __restrict__ Ri, int64_t ldi, int64_t n,
                               const double* __restrict__ s, double* __restrict__ t,
                               const LsqrState* __restrict__ st) {
  if (st->done) return;
  const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (j >= n) return;
  double acc = 0.0;
  const int64_t i_end = UPPER ? j + 1 : n;
#pragma unroll 4
  for (int64_t i = lane; i < i_end; i += 64) acc += Ri[i + j * ldi] * s[i];
  acc = wave_sum(acc);
  if (lane == 0) t[j] = acc;
}

// u is kept unnormalised (the normalised vector is u / beta):
// u <- A z - alpha (u / beta), or u <- b at the start; partial sums of u^2
// per workgroup
template <bool INIT>
__global__ __launch_bounds__(SAP_THREADS) void k_lsqr_av(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ ccol,
    const double* __restrict__ cval, int64_t m, const double* __restrict__ z,
    const double* __restrict__ b, double* __restrict__ u, double* __restrict__ partial,
    const LsqrState* __restrict__ st) {
  __shared__ double sh[16];
  if (st->done) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0;
  if (r < m) {
    if (INIT) {
      val = b[r];
      u[r] = val;
    } else if (rowptr[r + 1] - rowptr[r] <= SAP_LONG) {  // long rows: k_lsqr_av_long
      double s = 0.0;
      for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) s += cval[p] * z[ccol[p]];
      const double beta = st->beta;
      val = s - st->alpha * (beta > 0.0 ? u[r] / beta : 0.0);
      u[r] = val;
    }
  }
  const double tot = block_sum(val * val, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// the long rows of u <- A z - alpha (u / beta): one wave per long row;
// partial sums of their u^2 per workgroup (4 waves)
__global__ __launch_bounds__(SAP_THREADS) void k_lsqr_av_long(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ ccol,
    const double* __restrict__ cval, const int32_t* __restrict__ lidx, int64_t m,
    const int32_t* __restrict__ lrows, const double* __restrict__ z, double* __restrict__ u,
    double* __restrict__ partial, const LsqrState* __restrict__ st) {
  __shared__ double sh[16];
  if (st->done) return;
  const int64_t li = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  double val = 0.0;
  if (li < lidx[m]) {
    const int32_t r = lrows[li];
    double s = 0.0;
#pragma unroll 4
    for (int32_t p = rowptr[r] + lane; p < rowptr[r + 1]; p += 64) s += cval[p] * z[ccol[p]];
    s = wave_sum(s);
    if (lane == 0) {
      const double beta = st->beta;
      val = s - st->alpha * (beta > 0.0 ? u[r] / beta : 0.0);
      u[r] = val;
    }
  }
  const double tot = block_sum(val * val, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// beta = sqrt(sum of both partial arrays) (fixed order), one workgroup
template <bool INIT>
__global__ __launch_bounds__(1024) void k_lsqr_beta(const double* __restrict__ partial,
                                                     int64_t np, const double* __restrict__ partial2,
                                                     int64_t np2, LsqrState* __restrict__ st) {
  __shared__ double sh[16];
  if (st->done) return;
  double s = 0.0;
#pragma unroll 4
  for (int64_t i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  if (!INIT) {
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < np2; i += blockDim.x) s += partial2[i];
  }
  const double tot = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double beta = sqrt(tot);
    st->beta = beta;
    if (INIT) st->bnorm = beta;
  }
}

// chunk sums of A^T (u / beta): chunk q of column k covers entries
// [colptr[k] + q SAP_CHUNK, ...); one wave per chunk
__global__ void k_lsqr_atu(const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                           const double* __restrict__ v64, int64_t n,
                           const int32_t* __restrict__ cbase, const double* __restrict__ u,
                           double* __restrict__ cpart, const LsqrState* __restrict__ st,
                           const Header* __restrict__ hdr) {
  if (st->done) return;
  const bool valid = hdr->status == 0;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (g >= cbase[n]) return;
  // column of chunk g (both half waves search for the same g)
  const int64_t k = halfwave_last_le(0, n - 1, g, [&](int64_t q) { return (int64_t)cbase[q]; });
  const int64_t p0 = colptr[k] + (g - cbase[k]) * SAP_CHUNK;
  const int64_t p1 = p0 + SAP_CHUNK < colptr[k + 1] ? p0 + SAP_CHUNK : colptr[k + 1];
  double acc = 0.0;
  if (valid) {
#pragma unroll 4
    for (int64_t p = p0 + lane; p < p1; p += 64) acc += v64[p] * u[rowidx[p]];
  }
  acc = wave_sum(acc);
  if (lane == 0) cpart[g] = acc / (st->beta > 0.0 ? st->beta : 1.0);
}

// s[k] = sum of k's chunk sums (in order)
__global__ void k_lsqr_colsum(const int32_t* __restrict__ cbase, int64_t n,
                              const double* __restrict__ cpart, double* __restrict__ s,
                              const LsqrState* __restrict__ st) {
  if (st->done) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int32_t g = cbase[k]; g < cbase[k + 1]; ++g) acc += cpart[g];
  s[k] = acc;
}

// One workgroup: v' = t - beta v (t = R^{-T} A^T u), alpha = ||v'||, v = v'/alpha,
// then the LSQR scalar recurrences and the updates of x and w.  INIT: the
// start of the iteration (v' = t, w = v, x = 0).
template <bool INIT>
__global__ __launch_bounds__(1024) void k_lsqr_update(int64_t n, const double* __restrict__ t,
                                                       double* __restrict__ v,
                                                       double* __restrict__ w,
                                                       double* __restrict__ x,
                                                       LsqrState* __restrict__ st) {
  __shared__ double sh[16];
  if (st->done) return;
  const double beta = st->beta;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double vi = INIT ? t[i] : t[i] - beta * v[i];
    v[i] = vi;
    ss += vi * vi;
  }
  const double alpha = sqrt(block_sum(ss, sh));
  const double inv_a = alpha > 0.0 ? 1.0 / alpha : 0.0;
  if (INIT) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const double vi = v[i] * inv_a;
      v[i] = vi;
      w[i] = vi;
      x[i] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      st->alpha = alpha;
      st->rhobar = alpha;
      st->phibar = st->beta;
      st->rnorm = st->beta;
      st->arnorm = alpha * st->beta;
      st->anorm = 0.0; st->acond = 0.0; st->ddnorm = 0.0; st->res2 = 0.0;
      st->xnorm = 0.0; st->xxnorm = 0.0; st->z = 0.0; st->cs2 = -1.0; st->sn2 = 0.0;
      st->itn = 0;
      st->istop = 0;
      if (st->arnorm == 0.0) st->done = 1;
    }
    return;
  }
  // scalar recurrences (every thread computes them; thread 0 stores)
  const double anorm = sqrt(st->anorm * st->anorm + st->alpha * st->alpha + beta * beta);
  const double rhobar1 = st->rhobar;
  const double phibar0 = st->phibar;
  const double rho = sqrt(rhobar1 * rhobar1 + beta * beta);
  const double cs = rhobar1 / rho, sn = beta / rho;
  const double theta = sn * alpha;
  const double rhobar = -cs * alpha;
  const double phi = cs * phibar0;
  const double phibar = sn * phibar0;
  const double tau = sn * phi;
  const double t1 = phi / rho, t2 = -theta / rho;
  double dd = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double vi = v[i] * inv_a;
    const double wi = w[i];
    const double dk = wi / rho;
    dd += dk * dk;
    x[i] += t1 * wi;
    w[i] = vi + t2 * wi;
    v[i] = vi;
  }
  const double ddnorm = st->ddnorm + block_sum(dd, sh);
  if (threadIdx.x == 0) {
    const double delta = st->sn2 * rho;
    const double gambar = -st->cs2 * rho;
    const double rhs = phi - delta * st->z;
    const double zbar = rhs / gambar;
    const double xnorm = sqrt(st->xxnorm + zbar * zbar);
    const double gamma = sqrt(gambar * gambar + theta * theta);
    const double cs2 = gambar / gamma, sn2 = theta / gamma;
    const double z = rhs / gamma;
    const double xxnorm = st->xxnorm + z * z;
    const double acond = anorm * sqrt(ddnorm);
    const double rnorm = sqrt(phibar * phibar + st->res2);
    const double arnorm = alpha * fabs(tau);
    const double bnorm = st->bnorm;
    const double test1 = rnorm / bnorm;
    const double test2 = arnorm / (anorm * rnorm);
    const double test3 = 1.0 / acond;
    const double tt1 = test1 / (1.0 + anorm * xnorm / bnorm);
    const double rtol = st->btol + st->atol * anorm * xnorm / bnorm;
    const int itn = st->itn + 1;
    int istop = 0;
    if (itn >= st->iter_lim) istop = 7;
    if (1.0 + test3 <= 1.0) istop = 6;
    if (1.0 + test2 <= 1.0) istop = 5;
    if (1.0 + tt1 <= 1.0) istop = 4;
    if (test3 <= st->ctol) istop = 3;
    if (test2 <= st->atol) istop = 2;
    if (test1 <= rtol) istop = 1;
    st->alpha = alpha; st->rhobar = rhobar; st->phibar = phibar; st->anorm = anorm;
    st->acond = acond; st->ddnorm = ddnorm; st->xnorm = xnorm; st->xxnorm = xxnorm;
    st->z = z; st->cs2 = cs2; st->sn2 = sn2; st->rnorm = rnorm; st->arnorm = arnorm;
    st->test1 = test1; st->test2 = test2; st->test3 = test3;
    st->itn = itn;
    st->istop = istop;
    if (istop) st->done = 1;
  }
}

// x = M y (after the solve); not gated by the stop flag
template <bool UPPER>
__global__ void k_gemv_upper_final(const double* __restrict__ Ri, int64_t ldi, int64_t n,
                                   const double* __restrict__ y, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = UPPER ? i : 0; j < n; ++j) s += Ri[i + j * ldi] * y[j];
  x[i] = s;
}

// LSQR stop code of a request whose A failed the sketch's device validation
constexpr int32_t LSQR_ISTOP_INPUT = 8;

// a request whose A failed validation stops before its first iteration (the
// info prefix then tells an asynchronous reader without another call)
__global__ void k_lsqr_input_check(LsqrState* __restrict__ st, const Header* __restrict__ skh) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && skh->status) {
    st->istop = LSQR_ISTOP_INPUT;
    st->done = 1;
  }
}

__global__ void k_lsqr_set(LsqrState* __restrict__ st, double atol, double btol, double ctol,
                           int32_t iter_lim, int32_t rank) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    LsqrState s{};
    s.atol = atol; s.btol = btol; s.ctol = ctol; s.iter_lim = iter_lim; s.rank = rank;
    *st = s;
  }
}

}  // namespace sk

// sk_svd.hpp -- the SVD form of sketch-and-precondition (Sec. V-E-1): the
// singular values and right singular vectors of the sketch A_hat = S A, with
// the singular values below sigma_max / 1e12 dropped, give the
// preconditioner N = V_r diag(1 / sigma_r) in place of R^{-1}.
//
// A_hat is first reduced by the Householder QR the QR form already runs
// (A_hat = Q R, same singular values and right singular vectors), then a
// matrix is orthogonalised by one-sided (Hestenes) Jacobi rotations: columns
// p and q of G are rotated until G^T G is diagonal to a relative tolerance;
// the same rotations applied to V (initially I) give G = U diag(sigma) with
// G = G0 V.  The least-squares path orthogonalises G0 = R^T and needs no V
// (see k_svd_precond); the general entry point accumulates V.  One-sided Jacobi works on G itself, never on G^T G, so singular
// values down to rounding level of sigma_max come out with small relative
// error -- the property that matters for choosing what to drop.
//
// Parallel order: the round-robin (circle) tournament on the n columns
// (padded to even): n_pad - 1 steps per sweep, each with n_pad / 2 disjoint
// pairs, one workgroup per pair.  A sweep with no rotation ends the
// iteration: a device flag that every later step reads first, so sweeps
// enqueued past convergence cost only their launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_sap.hpp"

namespace sk {

constexpr int SVD_THREADS = 256;
constexpr double SVD_DROP = 1e-12;  // Sec. V-E-1: drop sigma < sigma_max * 1e-12

// Jacobi control block: rotations in the current sweep, the converged flag,
// sweeps done, and the squared rounding floor of G's column norms
struct JacobiCtl {
  int32_t rotations, converged, sweeps, pad;
  double floor2;
};

// Rows per thread held in registers by a step (rows <= SVD_THREADS * this;
// taller G runs the looping form)
constexpr int SVD_RPT = 8;

__global__ void k_eye(double* __restrict__ V, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int64_t j = t / n, i = t - j * n;
  V[t] = i == j ? 1.0 : 0.0;
}

// Reset the control block; floor2 = (2^-52 |G|_F)^2 from the column norms
// (|G|_F^2 = sum of the squared column norms).  A column whose norm is at
// that floor holds only rounding noise: its singular value is below
// 2^-52 |G|_F <= 2^-52 sqrt(n) sigma_max, far under the drop threshold, and
// rotating it against the others would only stir that noise (the pair test
// is relative, and noise never passes it), so steps leave such pairs alone.
// A rotation against a column of norm f turns the other column by an angle
// of at most f / (its norm), so what is left undone is rounding-sized.
__global__ __launch_bounds__(SVD_THREADS) void k_jacobi_reset(const double* __restrict__ cnorm,
                                                              int64_t n,
                                                              JacobiCtl* __restrict__ c) {
  __shared__ double sh[16];
  double a = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += SVD_THREADS) a = __builtin_fma(cnorm[j], cnorm[j], a);
  const double f = block_sum(a, sh);
  if (threadIdx.x == 0) {
    JacobiCtl z{};
    z.floor2 = f * 0x1.0p-104;
    *c = z;
  }
}

// Sums of three values over the workgroup (fixed order), every thread gets them
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int nw = SVD_THREADS / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (lane == 0) {
    sh[wave] = a;
    sh[nw + wave] = b;
    sh[2 * nw + wave] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
  for (int w = 0; w < nw; ++w) {
    a += sh[w];
    b += sh[nw + w];
    c += sh[2 * nw + w];
  }
}

// the rotation (cs, sn) that zeroes the (p, q) entry of G^T G, or false when
// the pair is orthogonal to the tolerance or at the rounding floor:
// t = tan(theta) is the smaller root of t^2 + 2 zeta t - 1 = 0 with
// zeta = (beta - alpha) / (2 gamma)
__device__ __forceinline__ bool jacobi_rotation(double alpha, double beta, double gamma,
                                                double tol, double floor2, double& cs,
                                                double& sn) {
  // also false for a zero column (gamma = 0) and for NaN input
  if (!(fabs(gamma) > tol * sqrt(alpha) * sqrt(beta))) return false;
  if (!(fmin(alpha, beta) > floor2)) return false;
  const double zeta = (beta - alpha) / (2.0 * gamma);
  const double t = fabs(zeta) > 1e150 ? 0.5 / zeta
                                      : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  cs = 1.0 / sqrt(1.0 + t * t);
  sn = cs * t;
  return true;
}

// the pair (p, q) of workgroup b in step `step` of the circle order
__device__ __forceinline__ void jacobi_pair(int64_t npad, int64_t step, int64_t b, int64_t& p,
                                            int64_t& q) {
  const int64_t L = npad - 1;
  if (b == 0) {
    p = step;
    q = L;
  } else {
    p = (step + b) % L;
    q = (step - b + L) % L;
  }
  if (p > q) { const int64_t t = p; p = q; q = t; }
}

// One step of a sweep: workgroup b rotates its pair (p, q) of the circle
// order in G (rows x n, column-major, rows >= n) and V (n x n), unless G's
// columns p and q are already orthogonal to the tolerance,
// |g_p . g_q| <= tol |g_p| |g_q|, or one of them is at the rounding floor.
// REG: the two columns of G and of V stay in registers between the sums and
// the update (rows, n <= SVD_THREADS * SVD_RPT), V's loads issued with G's.
// WITHV = false: no V is accumulated (V unused).
template <bool REG, bool WITHV = true>
__global__ __launch_bounds__(SVD_THREADS) void k_jacobi_step(double* __restrict__ G,
                                                             int64_t rows,
                                                             double* __restrict__ V, int64_t n,
                                                             int64_t npad, int64_t step,
                                                             double tol,
                                                             JacobiCtl* __restrict__ ctl) {
  if (ctl->converged) return;
  int64_t p, q;
  jacobi_pair(npad, step, blockIdx.x, p, q);
  if (q >= n) return;  // the padding column (odd n)
  __shared__ double sh[3 * SVD_THREADS / 64];
  double* gp = G + p * rows;
  double* gq = G + q * rows;
  double* vp = WITHV ? V + p * n : nullptr;
  double* vq = WITHV ? V + q * n : nullptr;
  const int tid = threadIdx.x;
  double a = 0.0, c = 0.0, g = 0.0, cs, sn;
  if constexpr (REG) {
    double x[SVD_RPT], y[SVD_RPT], u[SVD_RPT], w[SVD_RPT];
#pragma unroll
    for (int k = 0; k < SVD_RPT; ++k) {
      const int64_t i = tid + (int64_t)k * SVD_THREADS;
      x[k] = i < rows ? gp[i] : 0.0;
      y[k] = i < rows ? gq[i] : 0.0;
      u[k] = WITHV && i < n ? vp[i] : 0.0;
      w[k] = WITHV && i < n ? vq[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < SVD_RPT; ++k) {
      a = __builtin_fma(x[k], x[k], a);
      c = __builtin_fma(y[k], y[k], c);
      g = __builtin_fma(x[k], y[k], g);
    }
    block_sum3(a, c, g, sh);
    if (!jacobi_rotation(a, c, g, tol, ctl->floor2, cs, sn)) return;
#pragma unroll
    for (int k = 0; k < SVD_RPT; ++k) {
      const int64_t i = tid + (int64_t)k * SVD_THREADS;
      if (i < rows) {
        gp[i] = cs * x[k] - sn * y[k];
        gq[i] = sn * x[k] + cs * y[k];
      }
      if (WITHV && i < n) {
        vp[i] = cs * u[k] - sn * w[k];
        vq[i] = sn * u[k] + cs * w[k];
      }
    }
  } else {
    for (int64_t i = tid; i < rows; i += SVD_THREADS) {
      const double x = gp[i], y = gq[i];
      a = __builtin_fma(x, x, a);
      c = __builtin_fma(y, y, c);
      g = __builtin_fma(x, y, g);
    }
    block_sum3(a, c, g, sh);
    if (!jacobi_rotation(a, c, g, tol, ctl->floor2, cs, sn)) return;
    for (int64_t i = tid; i < rows; i += SVD_THREADS) {
      const double x = gp[i], y = gq[i];
      gp[i] = cs * x - sn * y;
      gq[i] = sn * x + cs * y;
    }
    if (WITHV) {
      for (int64_t i = tid; i < n; i += SVD_THREADS) {
        const double x = vp[i], y = vq[i];
        vp[i] = cs * x - sn * y;
        vq[i] = sn * x + cs * y;
      }
    }
  }
  if (tid == 0) atomicAdd(&ctl->rotations, 1);
}

// Block form (no V): the columns are grouped into blocks of W; one step of
// the round-robin order over blocks gives each workgroup a pair of blocks,
// whose 2W columns it copies into LDS (2W x rows doubles), orthogonalises
// among themselves by one inner round-robin sweep (2W - 1 inner steps of W
// disjoint column pairs, 1024 / W threads per pair), and writes back.  A
// sweep over the block pairs checks every column pair at least once, so a
// sweep with no rotation anywhere is converged as in the pairwise form; it
// needs nblocks - 1 launches instead of n - 1.  The same test and rotation
// as the pairwise step.
template <int W>
__global__ __launch_bounds__(1024) void k_jacobi_block(double* __restrict__ G, int64_t rows,
                                                       int64_t n, int64_t nblk, int64_t nbpad,
                                                       int64_t step, double tol,
                                                       JacobiCtl* __restrict__ ctl) {
  if (ctl->converged) return;
  constexpr int TPP = 1024 / W;  // threads per column pair
  constexpr int WPP = TPP / 64;  // waves per column pair
  extern __shared__ __align__(16) double colbuf[];  // 2W columns of `rows`
  __shared__ double red[W][WPP][3];
  __shared__ int rot_count;
  int64_t bp, bq;
  jacobi_pair(nbpad, step, blockIdx.x, bp, bq);
  if (bq >= nblk) return;  // the padding block
  const int tid = threadIdx.x;
  if (tid == 0) rot_count = 0;
  auto gcol = [&](int c) -> int64_t { return c < W ? bp * W + c : bq * W + (c - W); };
  for (int64_t x = tid; x < (int64_t)2 * W * rows; x += 1024) {
    const int c = (int)(x / rows);
    const int64_t i = x - (int64_t)c * rows;
    const int64_t gc = gcol(c);
    colbuf[x] = gc < n ? G[gc * rows + i] : 0.0;
  }
  __syncthreads();
  const int pr = tid / TPP;  // this thread's pair in an inner step
  const int lt = tid - pr * TPP;
  const int wv = lt >> 6;
  const double floor2 = ctl->floor2;
  int rotated = 0;
  for (int s = 0; s < 2 * W - 1; ++s) {
    int64_t p, q;
    jacobi_pair(2 * W, s, pr, p, q);
    double* x = colbuf + p * rows;
    double* y = colbuf + q * rows;
    double a = 0.0, c = 0.0, g = 0.0;
    // the thread's rows of both columns stay in registers for the update
    // when rows <= TPP * RPT (else they are read again)
    constexpr int RPT = 8;
    double ur[RPT], vr[RPT];
    const bool regs = rows <= (int64_t)TPP * RPT;
    if (regs) {
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int64_t i = lt + (int64_t)k * TPP;
        ur[k] = i < rows ? x[i] : 0.0;
        vr[k] = i < rows ? y[i] : 0.0;
        a = __builtin_fma(ur[k], ur[k], a);
        c = __builtin_fma(vr[k], vr[k], c);
        g = __builtin_fma(ur[k], vr[k], g);
      }
    } else {
      for (int64_t i = lt; i < rows; i += TPP) {
        const double u = x[i], v = y[i];
        a = __builtin_fma(u, u, a);
        c = __builtin_fma(v, v, c);
        g = __builtin_fma(u, v, g);
      }
    }
    a = wave_sum(a);
    c = wave_sum(c);
    g = wave_sum(g);
    if ((lt & 63) == 0) {
      red[pr][wv][0] = a;
      red[pr][wv][1] = c;
      red[pr][wv][2] = g;
    }
    __syncthreads();
    a = c = g = 0.0;
    for (int k = 0; k < WPP; ++k) {  // fixed order
      a += red[pr][k][0];
      c += red[pr][k][1];
      g += red[pr][k][2];
    }
    double cs, sn;
    if (jacobi_rotation(a, c, g, tol, floor2, cs, sn)) {
      if (regs) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int64_t i = lt + (int64_t)k * TPP;
          if (i < rows) {
            x[i] = cs * ur[k] - sn * vr[k];
            y[i] = sn * ur[k] + cs * vr[k];
          }
        }
      } else {
        for (int64_t i = lt; i < rows; i += TPP) {
          const double u = x[i], v = y[i];
          x[i] = cs * u - sn * v;
          y[i] = sn * u + cs * v;
        }
      }
      rotated += lt == 0;
    }
    __syncthreads();  // the next inner step reads other threads' rows
  }
  if (rotated) atomicAdd(&rot_count, rotated);
  __syncthreads();
  if (rot_count == 0) return;  // nothing moved: G is unchanged
  for (int64_t x = tid; x < (int64_t)2 * W * rows; x += 1024) {
    const int c = (int)(x / rows);
    const int64_t i = x - (int64_t)c * rows;
    const int64_t gc = gcol(c);
    if (gc < n) G[gc * rows + i] = colbuf[x];
  }
  if (tid == 0) atomicAdd(&ctl->rotations, rot_count);
}

// end of a sweep: converged when it rotated nothing
__global__ void k_jacobi_sweep_end(JacobiCtl* __restrict__ ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || ctl->converged) return;
  ctl->sweeps += 1;
  if (ctl->rotations == 0) ctl->converged = 1;
  ctl->rotations = 0;
}

// sigma_j = |g_j| (one workgroup per column; fixed summation order)
__global__ __launch_bounds__(SVD_THREADS) void k_col_norms(const double* __restrict__ G,
                                                           int64_t rows,
                                                           double* __restrict__ sigma) {
  __shared__ double sh[16];
  const int64_t j = blockIdx.x;
  const double* g = G + j * rows;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += SVD_THREADS) a = __builtin_fma(g[i], g[i], a);
  const double s = block_sum(a, sh);
  if (threadIdx.x == 0) sigma[j] = sqrt(s);
}

// sigma_max, the kept count r and the sweep count into the solver state
// (one workgroup; the maximum is order-independent, the count exact)
__global__ __launch_bounds__(SVD_THREADS) void k_svd_rank(const double* __restrict__ sigma,
                                                          int64_t n, const JacobiCtl* __restrict__ ctl,
                                                          double* __restrict__ smax_out,
                                                          LsqrState* __restrict__ st) {
  __shared__ double shm[SVD_THREADS];
  __shared__ int shc[SVD_THREADS];
  double mx = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += SVD_THREADS) mx = fmax(mx, sigma[j]);
  shm[threadIdx.x] = mx;
  __syncthreads();
  for (int s = SVD_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + s]);
    __syncthreads();
  }
  const double smax = shm[0];
  const double cut = smax * SVD_DROP;
  int cnt = 0;
  for (int64_t j = threadIdx.x; j < n; j += SVD_THREADS)
    cnt += (smax > 0.0 && sigma[j] >= cut) ? 1 : 0;
  shc[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = SVD_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) shc[threadIdx.x] += shc[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *smax_out = smax;
    st->rank = shc[0];
    st->sweeps = ctl->sweeps;
  }
}

// N = sum over the kept j of v_j e_j^T / sigma_j, zero columns for the dropped
// ones (their LSQR coordinates then stay zero: x lies in the span of the kept
// right singular vectors, the row space of A up to the dropped part).  The
// sketch-and-precondition path orthogonalises G = R^T (no V accumulated):
// then R^T V' = G = U' diag(sigma), so R = V' diag(sigma) U'^T and R's right
// singular vectors are v_j = g_j / sigma_j, giving N's column j = g_j / sigma_j^2.
__global__ void k_svd_precond(const double* __restrict__ G, const double* __restrict__ sigma,
                              const double* __restrict__ smax, int64_t n,
                              double* __restrict__ N) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int64_t j = t / n;
  const double s = sigma[j], mx = *smax;
  N[t] = (mx > 0.0 && s >= mx * SVD_DROP) ? (G[t] / s) / s : 0.0;
}

}  // namespace sk

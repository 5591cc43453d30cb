/*
 * sk_oracle.c -- plain, slow, obviously-correct CPU oracle for the sketch
 * A_hat = S * A  (paper: Sec. I-A, eq. (1); S is d x m with i.i.d. entries,
 * A is a tall m x n sparse matrix in CSC).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes, in the paper's order:
 *   1. S entries from a counter-based generator (Sec. IV-B-1: a CBRNG whose
 *      counter is the (row, column) position of the entry) -- Philox4x32-10
 *      from its published definition (Salmon, Moraes, Dror, Shaw, SC'11).
 *   2. The transform of the generator's 32-bit words to the three
 *      distributions of Sec. I-A (uniform +-1, uniform (-1,1), Gaussian) as
 *      discussed in Sec. III-C.  Each entry is the FP32 value the GPU library
 *      produces, widened exactly to FP64.
 *   3. S materialised explicitly (whole, or in column panels), then
 *      A_hat[:, k] += a_jk * S[:, j] for every nonzero, columns k outer and
 *      the nonzeros of a column in row order inner -- the loop order of
 *      Algorithm 3 (variant kji), in FP64.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - counter = (g, j_lo, j_hi, 0), key = (seed_lo, seed_hi); g is the group
 *     of S rows one generator call covers, j the S column (= the A row).
 *   - +-1: one call covers 128 rows: row 128g + 32w + b takes bit b of word w,
 *     bit 0 -> +1, bit 1 -> -1.
 *   - (-1,1): one call covers 4 rows: row 4g + w takes word w,
 *     t = (int32)x >> 8 (arithmetic), s = (2t + 1) * 2^-24  (open interval,
 *     exact in FP32).  The paper's "signed int / 2^31" would include -1.
 *   - Gaussian: Box-Muller on word pairs (x0,x1) -> rows 4g, 4g+1 and
 *     (x2,x3) -> rows 4g+2, 4g+3, with a fixed FP32 op sequence for ln, sqrt
 *     and the quarter-turn sine/cosine (coefficients from the Taylor series,
 *     rounded to FP32).
 *
 * Compile with -ffp-contract=off and without fast-math: the FP32 Gaussian
 * sequence below must round exactly as written.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_RADEMACHER 0
#define OR_UNIFORM 1
#define OR_GAUSSIAN 2

/* ---------------------------------------------------------------- Philox */
/* One Philox4x32 round: two 32x32->64 products, then the fixed word
 * permutation with the round key xor'ed into the high halves. */
static void or_philox_round(uint32_t x[4], uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x[1] ^ k0;
    const uint32_t y1 = lo1;
    const uint32_t y2 = hi0 ^ x[3] ^ k1;
    const uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

/* Philox4x32-10: ten rounds, the key advanced by the Weyl constants between
 * consecutive rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        or_philox_round(x, k0, k1);
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* The generator call that covers S rows of group g in S column j. */
static void or_block(uint64_t seed, uint64_t g, uint64_t j, uint32_t out[4])
{
    const uint32_t ctr[4] = {(uint32_t)g, (uint32_t)j, (uint32_t)(j >> 32), 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------ transforms */
/* (-1,1): t = top 24 bits of the word read as signed, s = (2t+1) 2^-24. */
static float or_uniform_from_word(uint32_t w)
{
    const int32_t t = ((int32_t)w) >> 8;
    return (float)(2 * t + 1) * 0x1.0p-24f;
}

/* Coefficient tables, built at load time from their mathematical definition
 * (FP64 evaluation, one rounding to FP32). */
static float OR_LOG_C[5];      /* 1/3, 1/5, 1/7, 1/9, 1/11              */
static float OR_SIN_C[7];      /* (-1)^k (pi/2)^(2k+1) / (2k+1)!, k=0..6 */
static float OR_COS_C[8];      /* (-1)^k (pi/2)^(2k)   / (2k)!,   k=0..7 */
static float OR_LN2_HI, OR_LN2_LO, OR_SQRT2;
static int or_tables_ready = 0;

static void or_build_tables(void)
{
    if (or_tables_ready) return;
    for (int k = 0; k < 5; ++k) OR_LOG_C[k] = (float)(1.0 / (double)(2 * k + 3));
    const double half_pi = 1.57079632679489661923;
    /* term_n = (pi/2)^n / n!, accumulated as a running product */
    double term = 1.0;
    for (int n = 0; n <= 14; ++n) {
        if (n > 0) term = term * half_pi / (double)n;
        const double sgn = ((n / 2) % 2) ? -1.0 : 1.0;
        if (n % 2 == 0) OR_COS_C[n / 2] = (float)(sgn * term);
        else if (n <= 13) OR_SIN_C[n / 2] = (float)(sgn * term);
    }
    /* ln 2 split: a high part with 15 significant bits (so (e-24)*hi is
     * exact for |e-24| < 2^9) and the rounded remainder. */
    const double ln2 = 0.69314718055994530942;
    OR_LN2_HI = (float)(22713.0 / 32768.0);
    OR_LN2_LO = (float)(ln2 - 22713.0 / 32768.0);
    OR_SQRT2 = (float)1.41421356237309504880;
    or_tables_ready = 1;
}

/* ln(u1) with u1 = ((x >> 8) + 1) * 2^-24 in (0, 1].
 * u1 = f * 2^(e-24), f in [sqrt(1/2), sqrt(2)];  ln f = 2 atanh(s),
 * s = (f-1)/(f+1), series 2s(1 + s^2/3 + s^4/5 + ... + s^10/11). */
static float or_ln_u1(uint32_t x)
{
    const uint32_t k = (x >> 8) + 1u;               /* 1 .. 2^24 */
    int e = 31 - __builtin_clz(k);                  /* floor(log2 k) */
    float f = ldexpf((float)k, -e);                 /* exact, in [1,2) */
    if (f > OR_SQRT2) { f = f * 0.5f; e = e + 1; }
    const float s = (f - 1.0f) / (f + 1.0f);
    const float z = s * s;
    float q = OR_LOG_C[4];
    q = fmaf(q, z, OR_LOG_C[3]);
    q = fmaf(q, z, OR_LOG_C[2]);
    q = fmaf(q, z, OR_LOG_C[1]);
    q = fmaf(q, z, OR_LOG_C[0]);
    const float t = 2.0f * s;
    const float lnf = fmaf(t * z, q, t);
    const float ef = (float)(e - 24);
    return fmaf(ef, OR_LN2_HI, fmaf(ef, OR_LN2_LO, lnf));
}

/* cos and sin of (pi/2) * phi for phi in [0, 1), Taylor polynomials. */
static void or_quarter_sincos(float phi, float *c, float *s)
{
    const float w = phi * phi;
    float ps = OR_SIN_C[6];
    for (int k = 5; k >= 0; --k) ps = fmaf(ps, w, OR_SIN_C[k]);
    float pc = OR_COS_C[7];
    for (int k = 6; k >= 0; --k) pc = fmaf(pc, w, OR_COS_C[k]);
    *s = ps * phi;
    *c = pc;
}

/* Box-Muller on one word pair: z0 = r cos(2 pi u2), z1 = r sin(2 pi u2). */
static void or_gauss_pair(uint32_t xe, uint32_t xo, float *z0, float *z1)
{
    const float lnu = or_ln_u1(xe);
    const float r = sqrtf(-2.0f * lnu);
    const uint32_t t2 = xo >> 8;                     /* 24-bit angle */
    const uint32_t q = t2 >> 22;                     /* quadrant */
    const float phi = (float)(t2 & 0x3FFFFFu) * 0x1.0p-22f;
    float c, s, ct, st;
    or_quarter_sincos(phi, &c, &s);
    switch (q) {
    case 0: ct = c; st = s; break;
    case 1: ct = -s; st = c; break;
    case 2: ct = -c; st = -s; break;
    default: ct = s; st = -c; break;
    }
    *z0 = r * ct;
    *z1 = r * st;
}

/* Rows per generator call for each distribution. */
static int64_t or_rows_per_call(int dist) { return dist == OR_RADEMACHER ? 128 : 4; }

/* Fill rows [g*rpc, g*rpc + rpc) of S column j from one generator call. */
static void or_fill_group(int dist, uint64_t seed, uint64_t g, uint64_t j, float *v)
{
    uint32_t x[4];
    or_block(seed, g, j, x);
    if (dist == OR_RADEMACHER) {
        for (int w = 0; w < 4; ++w)
            for (int b = 0; b < 32; ++b)
                v[32 * w + b] = ((x[w] >> b) & 1u) ? -1.0f : 1.0f;
    } else if (dist == OR_UNIFORM) {
        for (int w = 0; w < 4; ++w) v[w] = or_uniform_from_word(x[w]);
    } else {
        or_gauss_pair(x[0], x[1], &v[0], &v[1]);
        or_gauss_pair(x[2], x[3], &v[2], &v[3]);
    }
}

/* --------------------------------------------------------------- public */
void or_tables(float *log_c5, float *sin_c7, float *cos_c8, float *misc3)
{
    or_build_tables();
    memcpy(log_c5, OR_LOG_C, sizeof OR_LOG_C);
    memcpy(sin_c7, OR_SIN_C, sizeof OR_SIN_C);
    memcpy(cos_c8, OR_COS_C, sizeof OR_COS_C);
    misc3[0] = OR_LN2_HI; misc3[1] = OR_LN2_LO; misc3[2] = OR_SQRT2;
}

/* Gaussian pair for given words (exposed for the transform pins). */
void or_gauss_words(int64_t count, const uint32_t *xe, const uint32_t *xo, float *z0, float *z1)
{
    or_build_tables();
    for (int64_t p = 0; p < count; ++p) or_gauss_pair(xe[p], xo[p], &z0[p], &z1[p]);
}

/* One S entry (global row i, column j). */
double or_s_entry(int dist, uint64_t seed, int64_t i, int64_t j)
{
    or_build_tables();
    const int64_t rpc = or_rows_per_call(dist);
    float v[128];
    or_fill_group(dist, seed, (uint64_t)(i / rpc), (uint64_t)j, v);
    return (double)v[i % rpc];
}

/* S[r + c*ld] = S(row0 + r, col0 + c), r < d, c < ncols. */
void or_materialize_s(int dist, uint64_t seed, int64_t row0, int64_t d, int64_t col0,
                      int64_t ncols, double *S, int64_t ld, int nthreads)
{
    or_build_tables();
    const int64_t rpc = or_rows_per_call(dist);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t c = 0; c < ncols; ++c) {
        float v[128];
        const uint64_t j = (uint64_t)(col0 + c);
        int64_t r = 0;
        while (r < d) {
            const int64_t i = row0 + r;
            const int64_t g = i / rpc;
            or_fill_group(dist, seed, (uint64_t)g, j, v);
            const int64_t first = i - g * rpc;
            for (int64_t q = first; q < rpc && r < d; ++q, ++r) S[r + c * ld] = (double)v[q];
        }
    }
}

/* A_hat (d x n, column-major, leading dimension ld) = S[row0:row0+d, :] * A.
 * A is CSC: colptr[n+1] (int64), rowidx[nnz] (int32, sorted within a
 * column), vals[nnz] (FP64).  S is materialised in column panels of `panel`
 * columns (panel <= 0 or >= m: the whole S at once).  For every column k the
 * nonzeros are visited in row order, so the FP64 sum order of each entry is
 * the same for every panel width.  Returns 0, or -1 on a malformed input. */
int or_sketch(int64_t m, int64_t n, const int64_t *colptr, const int32_t *rowidx,
              const double *vals, int64_t row0, int64_t d, int dist, uint64_t seed,
              int64_t panel, int nthreads, double *Ahat, int64_t ld)
{
    or_build_tables();
    if (m < 1 || n < 1 || d < 1 || ld < d) return -1;
    for (int64_t k = 0; k < n; ++k) {
        if (colptr[k + 1] < colptr[k]) return -1;
        for (int64_t p = colptr[k]; p < colptr[k + 1]; ++p) {
            if (rowidx[p] < 0 || rowidx[p] >= m) return -1;
            if (p > colptr[k] && rowidx[p] <= rowidx[p - 1]) return -1;
        }
    }
    if (panel <= 0 || panel > m) panel = m;
    for (int64_t k = 0; k < n; ++k)
        for (int64_t i = 0; i < d; ++i) Ahat[i + k * ld] = 0.0;

    double *S = (double *)malloc((size_t)d * (size_t)panel * sizeof(double));
    int64_t *cur = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!S || !cur) { free(S); free(cur); return -2; }
    for (int64_t k = 0; k < n; ++k) cur[k] = colptr[k];

    for (int64_t j0 = 0; j0 < m; j0 += panel) {
        const int64_t pw = (m - j0 < panel) ? (m - j0) : panel;
        or_materialize_s(dist, seed, row0, d, j0, pw, S, d, nthreads);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t k = 0; k < n; ++k) {
            double *out = Ahat + k * ld;
            int64_t p = cur[k];
            const int64_t pend = colptr[k + 1];
            while (p < pend && rowidx[p] < j0 + pw) {
                const double a = vals[p];
                const double *sc = S + (int64_t)(rowidx[p] - j0) * d;
                for (int64_t i = 0; i < d; ++i) out[i] += a * sc[i];
                ++p;
            }
            cur[k] = p;
        }
    }
    free(S);
    free(cur);
    return 0;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

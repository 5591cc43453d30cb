// sk_rng.hpp -- the on-the-fly generator of S for the sketch A_hat = S A.
//
// S is never stored: each entry is a pure function of (seed, S row, S column)
// through a counter-based generator, so any tile can be regenerated anywhere
// (paper Sec. IV-B-1: a CBRNG whose counters are the entry's row and column
// indices; Sec. IV-C: results independent of the blocking and thread count).
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed,
// counter = (g, j_lo, j_hi, 0) where j is the S column (= A row) and g the
// group of S rows one call covers.
//
// Transforms (Sec. III-C; the paper leaves the bit-level mapping open):
//   +-1    : 128 rows per call, row 128g + 32w + b <- bit b of word w,
//            bit 0 -> +1, bit 1 -> -1.
//   (-1,1) : 4 rows per call, row 4g + w <- word w: t = (int32)w >> 8,
//            s = (2t+1) 2^-24 (open interval, exact in FP32).
//   N(0,1) : 4 rows per call, Box-Muller on (w0,w1) -> rows 4g, 4g+1 and
//            (w2,w3) -> rows 4g+2, 4g+3 with a fixed FP32 op sequence
//            (u1 = ((w>>8)+1) 2^-24, ln via 2 atanh series after a range
//            reduction to [sqrt(1/2), sqrt(2)], angle 2 pi (w'>>8) 2^-24 by
//            quadrant + Taylor sine/cosine of a quarter turn).
// Every FP32 operation rounds exactly once as written (explicit fmaf; the
// library is compiled without FP contraction and with IEEE div/sqrt), so the
// values are reproducible bit for bit on any IEEE FP32 implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

enum : int { DIST_RADEMACHER = 0, DIST_UNIFORM = 1, DIST_GAUSSIAN = 2 };

// ----------------------------------------------------- coefficient tables
// Built at compile time from their definitions: FP64 evaluation, one
// rounding to FP32.
struct RngTables {
  float log_c[5];   // 1/(2k+3), k = 0..4   (atanh series after the 1)
  float sin_c[7];   // (-1)^k (pi/2)^(2k+1)/(2k+1)!
  float cos_c[8];   // (-1)^k (pi/2)^(2k)/(2k)!
  float ln2_hi, ln2_lo, sqrt2;
};

constexpr double kHalfPi = 1.5707963267948966192313216916398;
constexpr double kLn2 = 0.69314718055994530941723212145818;

constexpr double quarter_turn_term(int n) {  // (pi/2)^n / n!
  double t = 1.0;
  for (int i = 1; i <= n; ++i) t = t * kHalfPi / (double)i;
  return t;
}

constexpr RngTables make_tables() {
  RngTables T{};
  for (int k = 0; k < 5; ++k) T.log_c[k] = (float)(1.0 / (double)(2 * k + 3));
  for (int k = 0; k < 7; ++k)
    T.sin_c[k] = (float)((k % 2 ? -1.0 : 1.0) * quarter_turn_term(2 * k + 1));
  for (int k = 0; k < 8; ++k)
    T.cos_c[k] = (float)((k % 2 ? -1.0 : 1.0) * quarter_turn_term(2 * k));
  // ln 2 = hi + lo with hi = 22713 / 2^15 (15 significant bits, so that
  // e * hi is exact for the small integer exponents used here)
  T.ln2_hi = (float)(22713.0 / 32768.0);
  T.ln2_lo = (float)(kLn2 - 22713.0 / 32768.0);
  T.sqrt2 = (float)1.4142135623730950488016887242097;
  return T;
}

constexpr RngTables kTables = make_tables();

// ----------------------------------------------------------------- Philox
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

struct Words { uint32_t x0, x1, x2, x3; };

// a ^ b ^ k in one instruction on the device: gfx950's three-input bitwise
// operation with truth table 0x96 (the parity of the three input bits).  The
// key word k is the same in every lane and is read from a scalar register.
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
#else
  return a ^ b ^ k;
#endif
}

__host__ __device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                   uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return Words{c0, c1, c2, c3};
}

// words for S-row group g of S column j
__host__ __device__ __forceinline__ Words gen_words(uint64_t seed, uint64_t g, uint64_t j) {
  return philox10((uint32_t)g, (uint32_t)j, (uint32_t)(j >> 32), 0u, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

__host__ __device__ __forceinline__ uint32_t word_at(const Words& x, int w) {
  return w == 0 ? x.x0 : (w == 1 ? x.x1 : (w == 2 ? x.x2 : x.x3));
}

// ------------------------------------------------------------- transforms
__host__ __device__ __forceinline__ float uniform_of(uint32_t w) {
  const int32_t t = ((int32_t)w) >> 8;
  return (float)(2 * t + 1) * 0x1.0p-24f;
}

__host__ __device__ __forceinline__ uint32_t bits_of(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  return v.u;
}

__host__ __device__ __forceinline__ float float_of(uint32_t u) {
  union { uint32_t u; float f; } v;
  v.u = u;
  return v.f;
}

__host__ __device__ __forceinline__ float pow2_neg(int e) {  // 2^-e, 0 <= e <= 126
  union { uint32_t u; float f; } v;
  v.u = (uint32_t)(127 - e) << 23;
  return v.f;
}

__host__ __device__ __forceinline__ int floor_log2(uint32_t k) {  // k >= 1
#if defined(__HIP_DEVICE_COMPILE__)
  return 31 - __clz((int)k);
#else
  return 31 - __builtin_clz(k);
#endif
}

// ln u1, u1 = ((w >> 8) + 1) 2^-24
__host__ __device__ __forceinline__ float ln_u1(uint32_t w) {
  const uint32_t k = (w >> 8) + 1u;
  int e = floor_log2(k);
  float f = (float)k * pow2_neg(e);  // exact, in [1, 2)
  if (f > kTables.sqrt2) {
    f = f * 0.5f;
    e = e + 1;
  }
  const float s = (f - 1.0f) / (f + 1.0f);
  const float z = s * s;
  float q = kTables.log_c[4];
  q = __builtin_fmaf(q, z, kTables.log_c[3]);
  q = __builtin_fmaf(q, z, kTables.log_c[2]);
  q = __builtin_fmaf(q, z, kTables.log_c[1]);
  q = __builtin_fmaf(q, z, kTables.log_c[0]);
  const float t = 2.0f * s;
  const float lnf = __builtin_fmaf(t * z, q, t);
  const float ef = (float)(e - 24);
  return __builtin_fmaf(ef, kTables.ln2_hi, __builtin_fmaf(ef, kTables.ln2_lo, lnf));
}

// (z0, z1) = r (cos 2 pi u2, sin 2 pi u2), u2 = (wo >> 8) 2^-24
__host__ __device__ __forceinline__ void box_muller(uint32_t we, uint32_t wo, float& z0,
                                                    float& z1) {
  const float r = __builtin_sqrtf(-2.0f * ln_u1(we));
  const uint32_t t2 = wo >> 8;
  const uint32_t quad = t2 >> 22;
  const float phi = (float)(t2 & 0x3FFFFFu) * 0x1.0p-22f;
  const float w = phi * phi;
  float ps = kTables.sin_c[6];
#pragma unroll
  for (int k = 5; k >= 0; --k) ps = __builtin_fmaf(ps, w, kTables.sin_c[k]);
  float pc = kTables.cos_c[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) pc = __builtin_fmaf(pc, w, kTables.cos_c[k]);
  const float sn = ps * phi;
  const float cs = pc;
  // rotation by quad quarter turns, branch-free (selection and sign flips are
  // exact): odd quadrants swap (cos, sin); cos is negated in quadrants 1 and
  // 2, sin in quadrants 2 and 3.
  const bool odd = (quad & 1u) != 0;
  const uint32_t ct_bits = bits_of(odd ? sn : cs) ^ (((quad ^ (quad >> 1)) & 1u) << 31);
  const uint32_t st_bits = bits_of(odd ? cs : sn) ^ (((quad >> 1) & 1u) << 31);
  z0 = r * float_of(ct_bits);
  z1 = r * float_of(st_bits);
}

// ------------------------------------------- distribution-cost ablation
// Generator modes of the ablation of the paper's cost model (Sec. III-A: the
// cost h of one random number; Sec. V: the sketch with a "junk" generator):
//   GEN_PHILOX -- the product generator;
//   GEN_JUNK   -- a counter hash of one multiply-add and three xors per call,
//                 NOT a usable random source: it only measures the sketch
//                 without the generator's cost;
//   GEN_STORED -- S read from memory (a materialised S, the stored-S SpMM);
//   GEN_SCALED -- (-1,1) only: S kept as the odd integers (2t + 1) of the
//                 uniform transform, A_hat scaled by 2^-24 once at the end
//                 (the paper's (S f)(A / f) integer-scaling trick; every FP32
//                 rounding scales exactly, so A_hat is unchanged).
enum : int { GEN_PHILOX = 0, GEN_JUNK = 1, GEN_STORED = 2, GEN_SCALED = 3 };

__host__ __device__ __forceinline__ Words junk_words(uint64_t g, uint64_t j) {
  const uint32_t b = (uint32_t)j * 0x9E3779B9u + (uint32_t)g;
  return Words{b, b ^ 0x6C8E9CF5u, b ^ 0xB5297A4Du, b ^ 0x1B56C4E9u};
}

template <int GEN>
__host__ __device__ __forceinline__ Words words_of(uint64_t seed, uint64_t g, uint64_t j) {
  if (GEN == GEN_JUNK) return junk_words(g, j);
  return gen_words(seed, g, j);
}

// 2^24 times the uniform value of word w: the odd integer 2t + 1 with
// t = (int32)w >> 8 (bit 7 of w is the low bit of w >> 7, replaced by 1)
__host__ __device__ __forceinline__ float uniform_scaled_of(uint32_t w) {
  return (float)((((int32_t)w) >> 7) | 1);
}

// Four consecutive S rows 4g..4g+3 of column j (uniform or Gaussian).
template <int DIST, int GEN = GEN_PHILOX>
__host__ __device__ __forceinline__ void quad_values(uint64_t seed, uint64_t g, uint64_t j,
                                                     float v[4]) {
  const Words x = words_of<GEN>(seed, g, j);
  if (DIST == DIST_UNIFORM && GEN == GEN_SCALED) {
    v[0] = uniform_scaled_of(x.x0);
    v[1] = uniform_scaled_of(x.x1);
    v[2] = uniform_scaled_of(x.x2);
    v[3] = uniform_scaled_of(x.x3);
  } else if (DIST == DIST_UNIFORM) {
    v[0] = uniform_of(x.x0);
    v[1] = uniform_of(x.x1);
    v[2] = uniform_of(x.x2);
    v[3] = uniform_of(x.x3);
  } else {
    box_muller(x.x0, x.x1, v[0], v[1]);
    box_muller(x.x2, x.x3, v[2], v[3]);
  }
}

// Sign bits of 32 consecutive S rows i..i+31 of column j (+-1 distribution):
// bit t set <=> S(i + t, j) = -1.
__host__ __device__ __forceinline__ uint32_t sign_bits32(uint64_t seed, uint64_t i, uint64_t j) {
  const uint64_t g = i >> 7;
  const int w = (int)((i >> 5) & 3);
  const int b = (int)(i & 31);
  const Words x = gen_words(seed, g, j);
  const uint32_t lo = word_at(x, w);
  if (b == 0) return lo;
  uint32_t hi;
  if (w < 3) {
    hi = word_at(x, w + 1);
  } else {
    hi = gen_words(seed, g + 1, j).x0;
  }
  return (lo >> b) | (hi << (32 - b));
}

}  // namespace sk

// Modular arithmetic for RNS limbs on gfx950 (and the host).
//
// Residues are uint64 in [0, q) in memory.  Each prime is one of three
// width classes, chosen per limb and uniform across a workgroup:
//   narrow  q < 2^30 : residues fit 32-bit words with headroom (4q < 2^32);
//                      reductions use 32-bit multiplies (v_mul_hi_u32,
//                      v_mad_u64_u32) and min-based conditional subtraction;
//   f64     q < 2^42 : inside the transform kernels residues are exact
//                      integers held in FP64 registers, signed and only
//                      lazily reduced; products use the exact FMA splitting
//                      below (all full-rate FP64 instructions on gfx950);
//   wide    q < 2^62 : 128-bit products from __umul64hi.
// Products with a fixed operand (twiddles, inverses) use Shoup's method with a
// precomputed companion w' = floor(w * 2^32 / q) (narrow) or
// floor(w * 2^64 / q) (wide).  Products of two data operands use Barrett
// reduction with s = bitlen(q) and mu = floor(2^(2s) / q): the quotient
// estimate floor(floor(x / 2^(s-1)) * mu / 2^(s+1)) is at most 2 below the
// true quotient, so two conditional subtractions finish.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace he {

typedef uint64_t u64;
typedef uint32_t u32;

struct ModConst {
  u64 q;
  u64 mu64;    // floor((2^64 - 1) / q): Barrett for any 64-bit input
  u64 bmu;     // floor(2^(2s) / q): Barrett for products of residues
  u32 s;       // bit length of q
  u32 narrow;  // q < 2^30
  u64 n_inv;   // N^-1 mod q
  u64 n_inv_sh;
  u64 r64;     // 2^64 mod q (folds the high word of a 128-bit sum)
  u64 r64_sh;
  u32 cls;     // width class (CLS_*)
  u32 r32_sh;  // narrow: Shoup companion of 2^32 mod q (else 0)
  double qd;       // q as a double (exact for q < 2^53)
  double qinv;     // 1 / q rounded to double
  double n_inv_q;  // n_inv / q rounded to double (f64 Shoup-style companion)
};

enum { CLS_N32 = 0, CLS_F64 = 1, CLS_U64 = 2 };
constexpr u64 F64_LIMIT = (u64)1 << 42;

__host__ __device__ inline u64 mulhi64(u64 a, u64 b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (u64)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline u64 add_mod(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}

__host__ __device__ inline u64 sub_mod(u64 a, u64 b, u64 q) {
  return a >= b ? a - b : a + (q - b);
}

constexpr u64 NARROW_LIMIT = (u64)1 << 30;
__host__ __device__ inline bool is_narrow(u64 q) { return q < NARROW_LIMIT; }
__host__ __device__ inline int width_class(u64 q) {
  return q < NARROW_LIMIT ? CLS_N32 : (q < F64_LIMIT ? CLS_F64 : CLS_U64);
}

// ---- f64 class ---------------------------------------------------------------
// Values are integers |a| < 2^46 held exactly in doubles.  For a multiplier
// w < q with wq ~ w / q (rounded, or formed as fl(w * fl(1/q))) the product
// a * w is split exactly as h + l with h = fl(a w) and l = fma(a, w, -h);
// the quotient estimate t = rint(a * wq) is within 1/2 + 2^-5 of a w / q
// (relative error of a * wq below 3 * 2^-53 and |a w / q| < 2^46), so
// r = (h - t q) + l lies in (-0.54 q, 0.54 q).  h - t q is an integer below 2^44 in magnitude, hence
// fma(-t, q, h) is exact, and so is the final sum with |l| <= ulp(h) / 2.
// The result is congruent to a w mod q but only "centred", not canonical.
__host__ __device__ inline double f64_mulc(double a, double w, double wq, double q) {
  const double h = a * w;
  const double l = fma(a, w, -h);
  const double t = rint(a * wq);
  return fma(-t, q, h) + l;
}
// a * b mod q (centred) for two data operands: wq computed on the fly.
__host__ __device__ inline double f64_mulmod(double a, double b, double q, double qinv) {
  return f64_mulc(a, b, b * qinv, q);
}
// Centred representative in [-q/2 - 2^-6 q, q/2 + 2^-6 q] of any |a| < 2^46.
__host__ __device__ inline double f64_centre(double a, double q, double qinv) {
  return fma(-rint(a * qinv), q, a);
}
// Canonical residue in [0, q) of any |a| < 2^46.
__host__ __device__ inline double f64_canon(double a, double q, double qinv) {
  const double r = f64_centre(a, q, qinv);
  return r < 0.0 ? r + q : r;
}
// Exact conversions between integers in [0, 2^52) and doubles: with the
// exponent of 2^52 fixed, the mantissa field of 2^52 + v is v itself.
__host__ __device__ inline double f64_from_u64(u64 v) {
  union { u64 u; double d; } x;
  x.u = v | 0x4330000000000000ull;
  return x.d - 4503599627370496.0;
}
__host__ __device__ inline u64 f64_to_u64(double v) {  // v an integer in [0, 2^52)
  union { u64 u; double d; } x;
  x.d = v + 4503599627370496.0;
  return x.u & 0x000FFFFFFFFFFFFFull;
}

// a * w mod q with Shoup companion wsh; a < 2^32 (narrow) or any a (wide).
__host__ __device__ inline u64 mul_shoup(u64 a, u64 w, u64 wsh, u64 q, bool narrow) {
  if (narrow) {
    u32 a32 = (u32)a;
    u32 qh = (u32)(((u64)a32 * (u32)wsh) >> 32);
    u32 r = a32 * (u32)w - qh * (u32)q;
    return r >= (u32)q ? r - (u32)q : r;
  }
  u64 qh = mulhi64(a, wsh);
  u64 r = a * w - qh * q;
  return r >= q ? r - q : r;
}

// a * b mod q for residues a, b < q.
__host__ __device__ inline u64 mul_mod(u64 a, u64 b, const ModConst& m) {
  const u64 q = m.q;
  const u32 s = m.s;
  if (m.narrow) {
    const u64 x = (u64)(u32)a * (u32)b;              // < 2^60
    const u32 t = (u32)(x >> (s - 1));               // < 2^(s+1) <= 2^31
    const u32 qh = (u32)(((u64)t * (u32)m.bmu) >> (s + 1));  // quotient estimate
    u32 r = (u32)x - qh * (u32)q;                    // true remainder < 3q < 2^32
    r = r >= (u32)q ? r - (u32)q : r;
    r = r >= (u32)q ? r - (u32)q : r;
    return r;
  }
  u64 lo = a * b, hi = mulhi64(a, b);                // x < 2^(2s)
  u64 t = (hi << (65 - s)) | (lo >> (s - 1));        // x >> (s-1) < 2^(s+1)
  u64 plo = t * m.bmu, phi = mulhi64(t, m.bmu);
  u64 qh = (phi << (63 - s)) | (plo >> (s + 1));     // (t * mu) >> (s+1)
  u64 r = lo - qh * q;                               // < 3q, exact mod 2^64
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  return r;
}

// v mod q for any 64-bit v.
__host__ __device__ inline u64 reduce64(u64 v, const ModConst& m) {
  u64 qh = mulhi64(v, m.mu64);
  u64 r = v - qh * m.q;
  return r >= m.q ? r - m.q : r;
}

// A 64-bit sum of products of narrow residues reduced to [0, 2q) in 32-bit
// arithmetic (q < 2^30): the high word through r = 2^32 mod q by a Shoup
// product (companion m.r32_sh), the low word by Barrett with floor(2^32 / q)
// (the high word of m.mu64); each part lands in [0, 2q), their sum below 4q.
// ModDown reads the ciphertext-prime rows of u in this form (its subtraction
// and Shoup product take inputs below 2q); the P row stays canonical.
__host__ __device__ inline u32 reduce64_lazy32(u64 a, const ModConst& m) {
  const u32 q = (u32)m.q;
  const u32 mu32 = (u32)(m.mu64 >> 32);
  const u32 r32 = 0u - mu32 * q;  // 2^32 - floor(2^32 / q) q
  const u32 hi = (u32)(a >> 32), lo = (u32)a;
  const u32 x = hi * r32 - (u32)(((u64)hi * m.r32_sh) >> 32) * q;
  const u32 y = lo - (u32)(((u64)lo * mu32) >> 32) * q;
  const u32 s = x + y;
  const u32 t = s - 2 * q;
  return t < s ? t : s;
}

// Centred representative of v (a residue mod qs, qs odd) reduced mod m.
__host__ __device__ inline u64 lift_centered(u64 v, u64 qs, const ModConst& m) {
  if (v <= (qs - 1) / 2) return reduce64(v, m);
  u64 r = reduce64(qs - v, m);
  return r ? m.q - r : 0;
}

// Signed integer (|x| < 2^63) reduced mod m.
__host__ __device__ inline u64 from_signed(int64_t x, const ModConst& m) {
  if (x >= 0) return reduce64((u64)x, m);
  u64 r = reduce64((u64)(-(x + 1)) + 1, m);  // |x| without overflow at INT64_MIN+1
  return r ? m.q - r : 0;
}

// Compile-time width class variants (the class is uniform per workgroup).
template <bool NARROW>
__host__ __device__ inline u64 mul_mod_t(u64 a, u64 b, const ModConst& m) {
  const u64 q = m.q;
  const u32 s = m.s;
  if constexpr (NARROW) {
    const u64 x = (u64)(u32)a * (u32)b;
    const u32 t = (u32)(x >> (s - 1));
    const u32 qh = (u32)(((u64)t * (u32)m.bmu) >> (s + 1));
    u32 r = (u32)x - qh * (u32)q;
#if defined(__HIP_DEVICE_COMPILE__)
    r = min(r, r - (u32)q);
    r = min(r, r - (u32)q);
#else
    r = r >= (u32)q ? r - (u32)q : r;
    r = r >= (u32)q ? r - (u32)q : r;
#endif
    return r;
  } else {
    u64 lo = a * b, hi = mulhi64(a, b);
    u64 t = (hi << (65 - s)) | (lo >> (s - 1));
    u64 plo = t * m.bmu, phi = mulhi64(t, m.bmu);
    u64 qh = (phi << (63 - s)) | (plo >> (s + 1));
    u64 r = lo - qh * q;
    if (r >= q) r -= q;
    if (r >= q) r -= q;
    return r;
  }
}

// Lazily accumulated sums of products, reduced once.
//  narrow: sum of up to 16 products (< 2^60 each) in one u64;
//  wide:   sum of up to 15 products (< 2^124 each) in a 128-bit (hi, lo) pair.
struct Acc128 {
  u64 lo, hi;
};
__host__ __device__ inline void mac128(Acc128& a, u64 x, u64 y) {
  const u64 plo = x * y, phi = mulhi64(x, y);
  const u64 lo = a.lo + plo;
  a.hi += phi + (lo < plo ? 1 : 0);
  a.lo = lo;
}
// (hi * 2^64 + lo) mod q
__host__ __device__ inline u64 reduce128(const Acc128& a, const ModConst& m) {
  const u64 h = reduce64(a.hi, m);
  const u64 l = reduce64(a.lo, m);
  return add_mod(mul_shoup(h, m.r64, m.r64_sh, m.q, m.narrow), l, m.q);
}

}  // namespace he

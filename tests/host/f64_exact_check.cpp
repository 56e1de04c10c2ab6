// Host check of the FP64 width class of the library's modular arithmetic
// (paper_2102_03494_amd/csrc/modarith.h): residues mod primes below 2^42
// held as exact integers in doubles.  Every result is compared with exact
// 128-bit integer arithmetic.
//
// Claims checked, at random inputs concentrated at the extreme magnitudes:
//   f64_mulc(a, w, w/q, q)   for |a| < 2^46, 0 <= w < q: an integer congruent
//                            to a w mod q with |r| < 0.54 q;
//   f64_mulmod(a, b, q, 1/q) the same with the companion formed on the fly;
//   f64_centre(a, q, 1/q)    for |a| < 2^46: congruent to a, |r| <= (1/2 + 2^-6) q;
//   f64_canon                in [0, q);
//   f64_from_u64 / f64_to_u64 round trip on [0, 2^52);
//   lazy sums: up to 15 centred products summed unreduced stay below 8.2 q
//   (< 2^46 for q < 2^42), so f64_canon of the sum is the exact residue;
//   forward-transform growth: a chain of 14 Cooley-Tukey stages on unreduced
//   values (x + w y, x - w y with the product from f64_mulc) stays below
//   8.6 q, inside the 2^46 input range of the next product.
// Prints "OK <cases>" and exits 0, or the first failures and exits 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

#include "../../paper_2102_03494_amd/csrc/modarith.h"

using namespace he;
typedef __int128 i128;

static int failures = 0;
static long long cases = 0;

static void fail(const char* what, double a, double w, double q, double r) {
  if (failures++ < 10) std::printf("FAIL %s: a=%.0f w=%.0f q=%.0f r=%.17g\n", what, a, w, q, r);
}

static bool is_int(double x) { return std::nearbyint(x) == x; }

static i128 mod_exact(i128 x, i128 q) {
  i128 r = x % q;
  return r < 0 ? r + q : r;
}

static bool is_prime(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull}) if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) d >>= 1, ++s;
  auto mulm = [&](uint64_t a, uint64_t b) { return (uint64_t)((unsigned __int128)a * b % n); };
  for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    uint64_t x = 1, b = a % n, e = d;
    while (e) {
      if (e & 1) x = mulm(x, b);
      b = mulm(b, b);
      e >>= 1;
    }
    if (x == 1 || x == n - 1) continue;
    bool ok = false;
    for (int i = 1; i < s && !ok; ++i) {
      x = mulm(x, x);
      ok = x == n - 1;
    }
    if (!ok) return false;
  }
  return true;
}

// Largest prime below 2^bits that is 1 mod 2^15 (an NTT prime for N up to 2^14).
static uint64_t ntt_prime(int bits) {
  const uint64_t step = 1ull << 15;
  for (uint64_t q = ((1ull << bits) / step) * step + 1; q > step; q -= step)
    if (q < (1ull << bits) && is_prime(q)) return q;
  return 0;
}

int main() {
  std::mt19937_64 rng(2102034941ull);
  const int bits_list[] = {30, 31, 36, 40, 41, 42};
  const double A_MAX = 70368744177664.0;  // 2^46
  for (int bits : bits_list) {
    const uint64_t qi = ntt_prime(bits);
    const double q = (double)qi, qinv = 1.0 / q;
    // magnitudes: uniform, and within 2^20 of the limits
    auto rand_a = [&](int mode) -> double {
      const int64_t lim = (int64_t)1 << 46;
      int64_t v;
      if (mode == 0) v = (int64_t)(rng() % (uint64_t)(2 * lim - 1)) - (lim - 1);
      else v = (lim - 1) - (int64_t)(rng() % (1u << 20));
      if (mode != 0 && (rng() & 1)) v = -v;
      return (double)v;
    };
    auto rand_w = [&](int mode) -> double {
      uint64_t v = rng() % qi;
      if (mode == 2) v = qi - 1 - (rng() % 1024);
      return (double)v;
    };
    for (int it = 0; it < 1500000; ++it) {
      const int mode = it % 3;
      const double a = rand_a(mode), w = rand_w(mode);
      ++cases;
      // f64_mulc with the rounded companion w / q
      const double r1 = f64_mulc(a, w, w / q, q);
      const double r2 = f64_mulmod(a, w, q, qinv);
      for (double r : {r1, r2}) {
        if (!is_int(r) || std::fabs(r) >= 0.54 * q ||
            mod_exact((i128)r, (i128)qi) != mod_exact((i128)(int64_t)a * (i128)(int64_t)w, (i128)qi))
          fail("mulc", a, w, q, r);
      }
      // centre and canonical representative of any |a| < 2^46
      const double c = f64_centre(a, q, qinv);
      if (!is_int(c) || std::fabs(c) > (0.5 + 1.0 / 64) * q ||
          mod_exact((i128)c, (i128)qi) != mod_exact((i128)(int64_t)a, (i128)qi))
        fail("centre", a, 0, q, c);
      const double k = f64_canon(a, q, qinv);
      if (!(k >= 0 && k < q) || (i128)k != mod_exact((i128)(int64_t)a, (i128)qi)) fail("canon", a, 0, q, k);
    }
    // lazy inner-product sums: 15 centred products of transform outputs
    // (|value| < 8.6 q) and canonical key residues, reduced once
    for (int it = 0; it < 200000; ++it) {
      double s = 0;
      i128 exact = 0;
      for (int j = 0; j < 15; ++j) {
        const double lim = std::floor(8.6 * q);
        double a = std::floor((double)(rng() % (uint64_t)(2 * lim)) - lim);
        if (it % 2) a = (j & 1) ? lim - 1 : -(lim - 1);
        const double w = (double)(it % 2 ? qi - 1 - (rng() % 16) : rng() % qi);
        const double p = f64_mulmod(a, w, q, qinv);
        s += p;
        exact += (i128)(int64_t)a * (i128)(int64_t)w;
      }
      ++cases;
      if (std::fabs(s) >= 8.2 * q || std::fabs(s) >= A_MAX) fail("lazy-sum bound", s, 0, q, s);
      const double k = f64_canon(s, q, qinv);
      if ((i128)k != mod_exact(exact, (i128)qi)) fail("lazy-sum residue", s, 0, q, k);
    }
    // growth through 14 forward stages on one path of the butterfly network,
    // the adversarial case: both inputs at the current bound, same sign
    for (int it = 0; it < 20000; ++it) {
      double x = (double)(rng() % qi), y = (double)(rng() % qi);
      i128 xe = (i128)(int64_t)x;
      for (int st = 0; st < 14; ++st) {
        const double w = (double)(rng() % qi);
        const double p = f64_mulc(y, w, w * qinv, q);
        const i128 pe = (i128)(int64_t)y * (i128)(int64_t)w;
        const bool take_sum = (rng() & 1) != 0;
        const double nx = take_sum ? x + p : x - p;
        xe = take_sum ? xe + pe : xe - pe;
        y = take_sum ? x - p : x + p;  // the sibling, carried as the next stage's partner
        x = nx;
        ++cases;
        if (std::fabs(x) >= 8.6 * q || std::fabs(y) >= 8.6 * q || !is_int(x)) fail("forward growth", x, w, q, y);
        if (mod_exact((i128)(int64_t)x, (i128)qi) != mod_exact(xe, (i128)qi)) fail("forward residue", x, w, q, x);
        xe = (i128)(int64_t)x;  // re-anchor (y's exact value is checked through its own path)
      }
    }
  }
  // exact conversions on [0, 2^52)
  for (int it = 0; it < 1000000; ++it) {
    const uint64_t v = rng() & ((1ull << 52) - 1);
    ++cases;
    if (f64_to_u64(f64_from_u64(v)) != v || f64_from_u64(v) != (double)v) fail("convert", (double)v, 0, 0, 0);
  }
  if (failures) {
    std::printf("FAILED %d of %lld cases\n", failures, cases);
    return 1;
  }
  std::printf("OK %lld\n", cases);
  return 0;
}

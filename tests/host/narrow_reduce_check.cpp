// Host check of reduce64_lazy32 (paper_2102_03494_amd/csrc/modarith.h), the
// reduction of a 64-bit sum of narrow products that ModUp stores for ModDown:
// for narrow primes q < 2^30 and any 64-bit a, the result must be below 2q
// and congruent to a mod q.  Compared with exact 64-bit remainders over
// random sums, sums of up to 16 products of residues below 2q and q, and the
// extreme words (0, 2^64 - 1, multiples of q and their neighbours).
// Prints "OK <cases>" and exits 0, or the first failures and exits 1.
#include <cstdint>
#include <cstdio>
#include <random>

#include "../../paper_2102_03494_amd/csrc/modarith.h"

using namespace he;

static int failures = 0;
static long long cases = 0;

static void check(uint64_t a, const ModConst& m) {
  ++cases;
  const uint32_t r = reduce64_lazy32(a, m);
  if (r >= 2 * m.q || r % m.q != a % m.q) {
    if (failures++ < 10)
      std::printf("FAIL a=%llu q=%llu r=%u\n", (unsigned long long)a, (unsigned long long)m.q, r);
  }
}

int main() {
  std::mt19937_64 rng(20261203);
  // primes below 2^30 of several sizes, including the largest 30-bit ones
  const uint64_t primes[] = {1073692673ull, 1073643521ull, 1073479681ull, 1073430529ull, 1073741789ull,
                             998244353ull, 469762049ull, 167772161ull, 12289ull, 7681ull, 97ull};
  for (uint64_t q : primes) {
    ModConst m{};
    m.q = q;
    m.mu64 = ~(uint64_t)0 / q;
    const uint64_t r32 = ((uint64_t)1 << 32) % q;
    m.r32_sh = (uint32_t)((r32 << 32) / q);
    for (uint64_t a : {(uint64_t)0, ~(uint64_t)0, ~(uint64_t)0 - 1, q, q - 1, q + 1, 2 * q, 2 * q - 1,
                       ((uint64_t)1 << 32), ((uint64_t)1 << 32) - 1, (~(uint64_t)0 / q) * q,
                       (~(uint64_t)0 / q) * q - 1})
      check(a, m);
    for (int it = 0; it < 1000000; ++it) check(rng(), m);
    for (int it = 0; it < 1000000; ++it) {
      uint64_t a = 0;
      const int k = 1 + (int)(rng() % 16);
      for (int j = 0; j < k; ++j) a += (rng() % (2 * q)) * (rng() % q);
      check(a, m);
    }
    for (int it = 0; it < 200000; ++it) {  // near multiples of q and of 2^32
      const uint64_t k = rng() % (~(uint64_t)0 / q);
      check(k * q + (rng() % 5) - 2, m);
      check((rng() << 32) + (rng() % 4) - 2, m);
    }
  }
  if (failures) {
    std::printf("%d failures in %lld cases\n", failures, cases);
    return 1;
  }
  std::printf("OK %lld\n", cases);
  return 0;
}

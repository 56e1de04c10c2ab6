// Host-side parameter generation and the client FP64 encoder/decoder.
//
// Primes: the largest prime q < 2^b with q = 1 (mod 2N), then the next one
// below it for further primes of the same size (deterministic Miller-Rabin
// with the first twelve prime bases, exact for 64-bit inputs).
// Root: psi = x^((q-1)/(2N)) for x the smallest quadratic non-residue mod q,
// so psi^N = -1 and psi has order 2N.
// Twiddles: fwd[k] = psi^brv(k), inv[k] = psi^-brv(k) (log2 N-bit reversal),
// each with its Shoup companion.
//
// CKKS slot encoding (client side): slot j <-> zeta^(5^j mod 2N), zeta =
// exp(i pi / N); for real slots z the real coefficients are
// m_k = (2/N) Re sum_j z_j zeta^(-k 5^j), evaluated here with an iterative
// radix-2 complex FFT of length 2N; the plaintext is round-half-away(scale m).
#include <cmath>
#include <complex>
#include <vector>

#include "host_params.h"

namespace he {

typedef unsigned __int128 u128;

static u64 mulmod_host(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 powmod(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod_host(r, a, q);
    a = mulmod_host(a, a, q);
    e >>= 1;
  }
  return r;
}

bool is_prime_u64(u64 n) {
  static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (u64 p : bases) {
    if (n % p == 0) return n == p;
  }
  u64 d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (u64 a : bases) {
    u64 x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod_host(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

// Largest prime below `start` congruent to 1 mod two_n (0 if none).
static u64 prime_below(u64 start, u64 two_n) {
  u64 q = ((start - 1) / two_n) * two_n + 1;
  if (q >= start) q -= two_n;
  while (q > two_n) {
    if (is_prime_u64(q)) return q;
    q -= two_n;
  }
  return 0;
}

int gen_moduli(int n, int n_q, const int* q_bits, int p_bits, u64* out) {
  if (n < 1024 || n > 65536 || (n & (n - 1))) return -1;
  if (n_q < 1 || n_q >= 16) return -1;
  const u64 two_n = 2 * (u64)n;
  u64 last_of_size[64] = {0};
  for (int i = 0; i <= n_q; ++i) {
    int b = (i < n_q) ? q_bits[i] : p_bits;
    if (b < 20 || b > 61) return -1;
    u64 start = last_of_size[b] ? last_of_size[b] : ((u64)1 << b);
    u64 q = prime_below(start, two_n);
    if (!q) return -1;
    last_of_size[b] = q;
    out[i] = q;
  }
  return 0;
}

// Inverse modulo a prime q (Fermat); not valid for composite moduli.
u64 inv_mod(u64 a, u64 q) { return powmod(a, q - 2, q); }

u64 root_2n(u64 q, int n) {
  u64 x = 2;
  while (powmod(x, (q - 1) / 2, q) != q - 1) ++x;
  return powmod(x, (q - 1) / (2 * (u64)n), q);
}

static u32 bitlen(u64 q) {
  u32 s = 0;
  while (s < 64 && (q >> s)) ++s;
  return s;
}

u64 shoup_companion(u64 w, u64 q) {
  if (is_narrow(q)) return (u64)(((u128)w << 32) / q);
  return (u64)(((u128)w << 64) / q);
}

ModConst make_modconst(u64 q, int n) {
  ModConst m;
  m.q = q;
  m.mu64 = (u64)(~(u64)0) / q;
  m.s = bitlen(q);
  m.bmu = (u64)(((u128)1 << (2 * m.s)) / q);
  m.narrow = is_narrow(q) ? 1u : 0u;
  m.n_inv = inv_mod((u64)n % q, q);
  m.n_inv_sh = shoup_companion(m.n_inv, q);
  m.r64 = (u64)(((u128)1 << 64) % q);
  m.r64_sh = shoup_companion(m.r64, q);
  m.cls = (u32)width_class(q);
  m.r32_sh = is_narrow(q) ? (u32)shoup_companion(((u64)1 << 32) % q, q) : 0u;
  m.qd = (double)q;
  m.qinv = 1.0 / (double)q;
  m.n_inv_q = (double)m.n_inv / (double)q;
  return m;
}

void make_twiddles(u64 q, int n, u64* fwd, u64* fwd_sh, u64* inv, u64* inv_sh) {
  int logn = 0;
  while ((1 << logn) < n) ++logn;
  u64 psi = root_2n(q, n);
  u64 psi_inv = inv_mod(psi, q);
  std::vector<u64> pw(n), pwi(n);
  pw[0] = pwi[0] = 1;
  for (int i = 1; i < n; ++i) {
    pw[i] = mulmod_host(pw[i - 1], psi, q);
    pwi[i] = mulmod_host(pwi[i - 1], psi_inv, q);
  }
  for (int k = 0; k < n; ++k) {
    u32 r = 0;
    for (int b = 0; b < logn; ++b) r |= ((k >> b) & 1u) << (logn - 1 - b);
    fwd[k] = pw[r];
    inv[k] = pwi[r];
    fwd_sh[k] = shoup_companion(fwd[k], q);
    inv_sh[k] = shoup_companion(inv[k], q);
  }
}

// ---- client encoder ---------------------------------------------------------

static void fft_inplace(std::vector<std::complex<double>>& a, bool inverse) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {  // bit-reversal permutation
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    double ang = 2.0 * M_PI / (double)len * (inverse ? 1.0 : -1.0);
    for (size_t i = 0; i < n; i += len) {
      for (size_t k = 0; k < len / 2; ++k) {
        std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
        std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

int encode_coeffs(int n, const double* z, int n_values, double scale, int64_t* out) {
  if (n < 2 || (n & (n - 1)) || n_values < 0 || n_values > n / 2) return -1;
  const size_t two_n = 2 * (size_t)n;
  std::vector<std::complex<double>> v(two_n, 0.0);
  u64 e = 1;
  for (int j = 0; j < n / 2; ++j) {
    double zj = j < n_values ? z[j] : 0.0;
    v[e] += zj;
    v[two_n - e] += zj;  // conjugate of a real value
    e = e * 5 % two_n;
  }
  fft_inplace(v, false);  // sum_e v[e] exp(-2 pi i k e / 2N)
  for (int k = 0; k < n; ++k) {
    double x = scale * (v[k].real() / (double)n);
    double r = std::floor(std::fabs(x) + 0.5);
    if (r >= 4611686018427387904.0) return -1;  // 2^62
    out[k] = (int64_t)(x < 0 ? -r : r);
  }
  return 0;
}

int decode_coeffs(int n, const double* m, int n_values, double* z) {
  if (n < 2 || (n & (n - 1)) || n_values < 0 || n_values > n / 2) return -1;
  const size_t two_n = 2 * (size_t)n;
  std::vector<std::complex<double>> w(two_n, 0.0);
  for (int k = 0; k < n; ++k) w[k] = m[k];
  fft_inplace(w, true);  // sum_k m_k exp(+2 pi i k e / 2N)
  u64 e = 1;
  for (int j = 0; j < n_values; ++j) {
    z[j] = w[e].real();
    e = e * 5 % two_n;
  }
  return 0;
}

}  // namespace he

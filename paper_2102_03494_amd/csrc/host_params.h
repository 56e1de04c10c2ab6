// Host-side number theory, table generation and the client encoder.
#pragma once
#include <stdint.h>

#include "modarith.h"

namespace he {

u64 powmod(u64 a, u64 e, u64 q);
u64 inv_mod(u64 a, u64 q);
bool is_prime_u64(u64 n);
u64 root_2n(u64 q, int n);
u64 shoup_companion(u64 w, u64 q);
ModConst make_modconst(u64 q, int n);
int gen_moduli(int n, int n_q, const int* q_bits, int p_bits, u64* out);
void make_twiddles(u64 q, int n, u64* fwd, u64* fwd_sh, u64* inv, u64* inv_sh);
int encode_coeffs(int n, const double* z, int n_values, double scale, int64_t* out);
int decode_coeffs(int n, const double* m, int n_values, double* z);

}  // namespace he

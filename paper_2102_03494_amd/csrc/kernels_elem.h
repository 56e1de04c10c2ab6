// Elementwise and bookkeeping kernels of the library that do not depend on
// the ring size (job tables, additions, integer-scalar MACs, the square
// tensor, client-side helpers).  Included by the C-ABI unit only.
#pragma once
#include "kernels.h"

namespace he {

// Job table of a uniform batch: ciphertext b at base + b * stride.
__global__ void k_make_jobs(KsJob* jobs, int count, const u64* d_base, size_t d_stride, const u64* c_base,
                            size_t c_stride, u64* out_base, size_t out_stride, const u64* key, u32 g, u32 ginv,
                            int level, int flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  KsJob jb;
  jb.d = d_base + (size_t)b * d_stride;
  jb.c = c_base + (size_t)b * c_stride;
  jb.out = out_base + (size_t)b * out_stride;
  jb.key = key;
  jb.g = g;
  jb.ginv = ginv;
  jb.level = level;
  jb.flags = flags;
  jobs[b] = jb;
}

// Job tables of all steps of a rotate-and-sum chain over `count` ciphertexts
// updated in place (ciphertext b at base + b * stride): step j's table at
// jobs + j * count.  With `packed`, every step writes its output packed and
// every step but the first reads packed input (the first too with
// in_packed0).  grid (ceil(count / 256), steps).
__global__ void k_make_chain_jobs(KsJob* jobs, int count, u64* base, size_t stride, size_t c1_off, int level,
                                  ChainKeys ck, int packed, int in_packed0) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (b >= count) return;
  u64* x = base + (size_t)b * stride;
  KsJob jb;
  jb.d = x + c1_off;
  jb.c = x;
  jb.out = x;
  jb.key = ck.key[j];
  jb.g = ck.g[j];
  jb.ginv = ck.ginv[j];
  jb.level = level;
  jb.flags = packed ? (JOB_OUT_PACKED | ((j > 0 || in_packed0) ? JOB_IN_PACKED : 0)) : 0;
  jobs[(size_t)j * count + b] = jb;
}

// Jobs of hoisted rotations of n_in ciphertexts (ciphertext i at
// in + i in_stride): jobs[i m + r] rotates ciphertext i by rotation r of hk
// into out + i out_stride + r 2 level n.  With digits_only, jobs[i] is ciphertext
// i's decomposition job (no permutation; key hk.key[0] marks it as
// switching).  grid (ceil(n_in / 256), m).
__global__ void k_make_hoist_jobs(KsJob* jobs, int n_in, int m, const u64* in, size_t in_stride, u64* out,
                                  size_t out_stride, int level, int n, HoistKeys hk, int digits_only) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n_in) return;
  const u64* x = in + (size_t)i * in_stride;
  KsJob jb;
  jb.d = x + (size_t)level * n;
  jb.c = x;
  jb.level = level;
  jb.flags = 0;
  if (digits_only) {
    jb.out = nullptr;
    jb.key = hk.key[0];
    jb.g = jb.ginv = 1u;
    jobs[i] = jb;
    return;
  }
  jb.out = out + (size_t)i * out_stride + (size_t)r * 2 * level * n;
  jb.key = hk.key[r];
  jb.g = hk.g[r];
  jb.ginv = hk.ginv[r];
  jobs[(size_t)i * m + r] = jb;
}

// The masking step of the homomorphic Im2Col (Him2colMap).
__global__ void __launch_bounds__(256)
k_him2col_mask(const u64* __restrict__ z, const u64* __restrict__ rot, const u64* __restrict__ masks, int mask_limbs,
               u64* __restrict__ out, int level, int n, Him2colMap hm, Mods mods) {
  const int i = blockIdx.x * 256 + (int)threadIdx.x;
  const int t = blockIdx.y;
  const size_t bk = blockIdx.z;
  const int kk = hm.d2 * hm.c_in;
  const size_t b = bk / kk;
  const int k = (int)(bk % kk);
  const int tap = k / hm.c_in, c = k % hm.c_in;
  const int m = c / hm.per, blk = c % hm.per;
  const size_t cs = (size_t)2 * level * n;
  const int id = hm.idx[tap];
  const u64* src = id < 0 ? z + ((b * hm.m_cts + m) * hm.per + blk) * cs
                          : rot + ((b * hm.nvalid + (size_t)m * hm.per + blk) * hm.nrot + id) * cs;
  const ModConst mc = mods.m[t];
  const u64 mv = masks[((size_t)tap * mask_limbs + t) * n + i];
  u64* o = out + (bk * 2 * level + t) * n + i;
  o[0] = mul_mod(src[(size_t)t * n + i], mv, mc);
  o[(size_t)level * n] = mul_mod(src[((size_t)level + t) * n + i], mv, mc);
}

// Switching keys made by a client, [L][2][L+1][N] canonical 64-bit residues
// per key, into the library's stored form (rows of narrow moduli packed as N
// 32-bit words at the start of the row); residues not below their modulus
// set *bad.  grid (N / 256, L + 1, 2 L); src and dst do not overlap.
__global__ void k_key_pack(u64* __restrict__ dst, const u64* __restrict__ src, int big_l, int n, Mods mods,
                           int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t row = ((size_t)blockIdx.z * (big_l + 1) + t) * n;
  const ModConst m = mods.m[t];
  const u64 v = src[row + i];
  if (v >= m.q) atomicOr(bad, 1);
  if (m.narrow)
    reinterpret_cast<u32*>(dst + row)[i] = (u32)v;
  else
    dst[row + i] = v;
}

// CP -> DP combine, summing step: out[m] = sum_{o in block m} rot[o], block
// m = [m B, min(O_c, (m+1) B)); grid (N / 256, level, n_dense).
__global__ void k_block_sum(u64* __restrict__ out, const u64* __restrict__ rot, int o_c, int per_dense, int n_dense,
                            int level, int n, Mods mods) {
  // blockIdx.z = item * n_dense + m: out[z] = sum of item's ciphertexts
  // m * per_dense .. (m + 1) * per_dense - 1 (rot holds o_c per item)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t z = blockIdx.z;
  const size_t item = z / n_dense;
  const int mblk = (int)(z - item * n_dense);
  const u64 q = mods.m[t].q;
  const int o_end = min(o_c, (mblk + 1) * per_dense);
  rot += item * o_c * 2 * level * (size_t)n;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    u64 acc = 0;
    for (int o = mblk * per_dense; o < o_end; ++o) acc = add_mod(acc, rot[(((size_t)o * 2 + c) * level + t) * n + i], q);
    out[((z * 2 + c) * level + t) * n + i] = acc;
  }
}

// Batched MulPC over a ragged batch: out_b = ct_b * pt_b (slot-wise), every
// item with its own level; jobs give (d = ct, c = pt, out).  grid
// (N / 256, Lmax, count); limbs above an item's level exit.
__global__ void k_batch_mul_plain(const KsJob* __restrict__ jobs, int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const KsJob jb = jobs[blockIdx.z];
  if (t >= jb.level) return;
  const ModConst m = mods.m[t];
  const u64 pv = jb.c[(size_t)t * n + i];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const size_t off = ((size_t)c * jb.level + t) * n + i;
    jb.out[off] = mul_mod(jb.d[off], pv, m);
  }
}

// out[z] = a[z] + b[z] (ciphertext-sized items).
__global__ void k_add(u64* out, const u64* a, const u64* b, int level, int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t z = blockIdx.z;
  const u64 q = mods.m[t].q;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const size_t off = ((z * 2 + c) * level + t) * (size_t)n + i;
    out[off] = add_mod(a[off], b[off], q);
  }
}

// Integer-scalar MAC (ConvPack, Table II): out[o] = sum_k w[k][o] * in[k],
// with w given per limb as residues + Shoup companions: wres[(k*o_c + o)*level + t].
// blockIdx.z = layer * o_c + o over independent layers: layer l reads
// in + l in_stride and its table at wres / wsh + l tab_stride; out[z].
__global__ void k_scalar_mac(u64* __restrict__ out, const u64* __restrict__ in, int K, int o_c,
                             const u64* __restrict__ wres, const u64* __restrict__ wsh, int level, int n,
                             size_t in_stride, size_t tab_stride, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t z = blockIdx.z;
  const size_t layer = z / o_c;
  const size_t o = z - layer * o_c;
  in += layer * in_stride;
  wres += layer * tab_stride;
  wsh += layer * tab_stride;
  const ModConst m = mods.m[t];
  u64 s0 = 0, s1 = 0;
  for (int k = 0; k < K; ++k) {
    const size_t wi = ((size_t)k * o_c + o) * level + t;
    const u64 w = wres[wi], ws = wsh[wi];
    s0 = add_mod(s0, mul_shoup(in[(((size_t)k * 2 + 0) * level + t) * n + i], w, ws, m.q, m.narrow), m.q);
    s1 = add_mod(s1, mul_shoup(in[(((size_t)k * 2 + 1) * level + t) * n + i], w, ws, m.q, m.narrow), m.q);
  }
  out[((z * 2 + 0) * level + t) * n + i] = s0;
  out[((z * 2 + 1) * level + t) * n + i] = s1;
}

// Square tensor: d0 = c0^2, d1 = 2 c0 c1 (both into d01 = [count][2][level][N])
// and d2 = c1^2 into [count][level][N].
__global__ void k_tensor_sq(u64* __restrict__ d01, u64* __restrict__ d2, const u64* __restrict__ in,
                            int level, int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t z = blockIdx.z;
  const ModConst m = mods.m[t];
  const u64 c0 = in[((z * 2 + 0) * level + t) * n + i];
  const u64 c1 = in[((z * 2 + 1) * level + t) * n + i];
  const u64 x01 = mul_mod(c0, c1, m);
  d01[((z * 2 + 0) * level + t) * n + i] = mul_mod(c0, c0, m);
  d01[((z * 2 + 1) * level + t) * n + i] = add_mod(x01, x01, m.q);
  d2[(z * level + t) * n + i] = mul_mod(c1, c1, m);
}

// out[t] = coeffs mod modulus (first_mod + t), coefficient domain.
__global__ void k_from_signed(u64* out, const int64_t* coeffs, int first_mod, int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  out[(size_t)t * n + i] = from_signed(coeffs[i], mods.m[first_mod + t]);
}

// Encryption: c0 = pt + ehat - a*s, c1 = a.
__global__ void k_encrypt(u64* ct, const u64* pt, const u64* a, const u64* ehat, const u64* s, int level,
                          int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const ModConst m = mods.m[t];
  const size_t k = (size_t)t * n + i;
  const u64 av = a[k];
  ct[k] = sub_mod(add_mod(pt[k], ehat[k], m.q), mul_mod(av, s[k], m), m.q);
  ct[(size_t)level * n + k] = av;
}

__global__ void k_decrypt(u64* out, const u64* ct, const u64* s, int level, int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const ModConst m = mods.m[t];
  const size_t k = (size_t)t * n + i;
  out[k] = add_mod(ct[k], mul_mod(ct[(size_t)level * n + k], s[k], m), m.q);
}

}  // namespace he

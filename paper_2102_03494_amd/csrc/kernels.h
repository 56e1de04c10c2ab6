// HIP kernels of the homomorphic convolution path (gfx950).
//
// Data layout (device, caller-owned): a ciphertext is [2][level][N] uint64
// residues in the NTT domain, limb-major, so each limb is one contiguous
// 8N-byte run and every kernel reads and writes whole limbs with unit-stride
// (coalesced) accesses.  Kernels that need a transform hold one limb per
// workgroup in LDS (ntt_lds.h); elementwise kernels use one thread per
// coefficient.  The width class of each prime (narrow < 2^30, wide < 2^62) is
// uniform per workgroup; each transform kernel branches once on it into a
// body compiled for that class (32-bit words for narrow limbs).
//
// Key switching of a batch of ciphertexts (rotation or relinearisation) runs
// as four kernels, each batched over every ciphertext of the call:
//   k_ks_digits    INTT of each limb of sigma_g(c1)  -> coefficient digits
//   k_ks_modup_ip  per target modulus: centred lift of each digit, NTT, and
//                  the inner product with the key, accumulated in registers
//                  (the lifted digits never go to memory)
//   k_intt_last    INTT of the P limb of (u0, u1)
//   k_drop_last    per target prime: centred lift of that limb, NTT,
//                  (u - lift) * P^-1, fused with the operation's epilogue
//                  (rotation, rotate-and-add, relinearisation, or plain store)
// Rescale is k_intt_last + k_drop_last with the last ciphertext prime as the
// divisor.
#pragma once
#include "modarith.h"
#include "ntt_lds.h"

namespace he {

#define HE_MAXM 16

struct Mods {
  ModConst m[HE_MAXM];
};

struct ConstTable {  // one constant per modulus index with its Shoup companion
  u64 v[HE_MAXM];
  u64 sh[HE_MAXM];
};

// Twiddle tables [n_mods][4][N] (fwd, fwd_shoup, inv, inv_shoup): 64-bit for
// every modulus, 32-bit copies for the narrow ones.
struct Tables {
  const u64* tw64;
  const u32* tw32;
};

template <int LOGN, bool NARROW>
__device__ __forceinline__ Tw<NARROW> tw_of(const Tables& tb, int mi, int which) {
  constexpr size_t N = (size_t)1 << LOGN;
  if constexpr (NARROW)
    return {tb.tw32 + ((size_t)mi * 4 + which) * N, tb.tw32 + ((size_t)mi * 4 + which + 1) * N};
  else
    return {tb.tw64 + ((size_t)mi * 4 + which) * N, tb.tw64 + ((size_t)mi * 4 + which + 1) * N};
}

// An opaque copy of the thread index (see ntt_lds.h): defined where it is
// used so that address arithmetic is not hoisted out of enclosing loops.
__device__ __forceinline__ int opaque_tid() {
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  return tid;
}

template <int LOGN, bool NARROW>
__device__ __forceinline__ void fwd_lds(u64* lds, const Tables& tb, int mi, u64 q) {
  ntt_fwd_lds<LOGN, NARROW>(lds, tw_of<LOGN, NARROW>(tb, mi, 0), (word_t<NARROW>)q, opaque_tid());
}

template <int LOGN, bool NARROW>
__device__ __forceinline__ void inv_lds(u64* lds, const Tables& tb, int mi, u64 q) {
  ntt_inv_lds<LOGN, NARROW>(lds, tw_of<LOGN, NARROW>(tb, mi, 2), (word_t<NARROW>)q, opaque_tid());
}

template <bool NARROW>
__device__ __forceinline__ u64 addm(u64 a, u64 b, u64 q) {
  if constexpr (NARROW) return add32((u32)a, (u32)b, (u32)q);
  else return add_mod(a, b, q);
}
template <bool NARROW>
__device__ __forceinline__ u64 subm(u64 a, u64 b, u64 q) {
  if constexpr (NARROW) return sub32((u32)a, (u32)b, (u32)q);
  else return sub_mod(a, b, q);
}
template <bool NARROW>
__device__ __forceinline__ u64 shoupm(u64 a, u64 w, u64 wsh, u64 q) {
  if constexpr (NARROW) return shoup32((u32)a, (u32)w, (u32)wsh, (u32)q);
  else return mul_shoup(a, w, wsh, q, false);
}

// Coalesced limb load into LDS, optionally through the Galois permutation
// sigma_g: afterwards lds[i] = src[galois_src(i, g)].  ginv = g^-1 mod 2N
// (the scatter position of source entry idx is galois_src(idx, ginv)).
template <int LOGN, bool NARROW>
__device__ __forceinline__ void load_limb_perm(u64* lds, const u64* __restrict__ src, u32 ginv) {
  constexpr int T = NttGeom<LOGN>::T;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int idx = (int)threadIdx.x + r * T;
    const u64 v = src[idx];
    const int dst = (ginv == 1u) ? idx : galois_src<LOGN>(idx, ginv);
    lds_put<NARROW>(lds, dst, v);
  }
}

// Store the LDS limb, optionally scaled by N^-1 (after an inverse transform).
template <int LOGN, bool NARROW>
__device__ __forceinline__ void store_limb(u64* __restrict__ dst, const u64* lds, const ModConst& m, bool scale) {
  constexpr int T = NttGeom<LOGN>::T;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (int)threadIdx.x + r * T;
    u64 v = lds_get<NARROW>(lds, i);
    if (scale) v = shoupm<NARROW>(v, m.n_inv, m.n_inv_sh, m.q);
    dst[i] = v;
  }
}

// ---------------------------------------------------------------------------
// Standalone transforms: blockIdx.x = limb, blockIdx.y = polynomial.
template <int LOGN, bool FWD, bool NARROW>
__device__ __forceinline__ void ntt_body(u64* lds, u64* p, int mi, const ModConst& m, const Tables& tb) {
  load_limb_perm<LOGN, NARROW>(lds, p, 1u);
  if (FWD) fwd_lds<LOGN, NARROW>(lds, tb, mi, m.q); else inv_lds<LOGN, NARROW>(lds, tb, mi, m.q);
  store_limb<LOGN, NARROW>(p, lds, m, !FWD);
}

template <int LOGN, bool FWD>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_ntt(u64* data, int n_limbs, int first_mod, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  const int limb = blockIdx.x;
  const int mi = first_mod + limb;
  const ModConst m = mods.m[mi];
  u64* p = data + ((size_t)blockIdx.y * n_limbs + limb) * N;
  if (m.narrow) ntt_body<LOGN, FWD, true>(lds, p, mi, m, tb);
  else ntt_body<LOGN, FWD, false>(lds, p, mi, m, tb);
}

// ---------------------------------------------------------------------------
// Key switch, step 1: coefficient-domain digits of sigma_g(c1).
// blockIdx.x = digit j (< level), blockIdx.y = ciphertext b.
// c1 points at limb 0 of component 1 of ciphertext 0; cstride = elements
// between ciphertexts.  dcoef = [count][level][N].
template <int LOGN, bool NARROW>
__device__ __forceinline__ void digits_body(u64* lds, const u64* src, u32 ginv, u64* out, int j, const ModConst& m,
                                            const Tables& tb) {
  load_limb_perm<LOGN, NARROW>(lds, src, ginv);
  inv_lds<LOGN, NARROW>(lds, tb, j, m.q);
  store_limb<LOGN, NARROW>(out, lds, m, true);
}

template <int LOGN>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_ks_digits(const u64* __restrict__ c1, size_t cstride, u32 ginv, u64* __restrict__ dcoef, int level,
            Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  const int j = blockIdx.x;
  const size_t b = blockIdx.y;
  const ModConst m = mods.m[j];
  const u64* src = c1 + b * cstride + (size_t)j * N;
  u64* out = dcoef + (b * level + j) * N;
  if (m.narrow) digits_body<LOGN, true>(lds, src, ginv, out, j, m, tb);
  else digits_body<LOGN, false>(lds, src, ginv, out, j, m, tb);
}

// Key switch, step 2: ModUp + inner product for one target modulus t in
// [0, level]: t < level is q_t, t == level is P (modulus index big_l);
// blockIdx.y = ciphertext b.
// key = [big_l][2][big_l+1][N]; u = [count][2][level+1][N].
template <int LOGN, bool NARROW>
__device__ __forceinline__ void modup_ip_body(u64* lds, const u64* __restrict__ dcoef, const u64* __restrict__ c1,
                                              size_t cstride, u32 ginv, const u64* __restrict__ key,
                                              u64* __restrict__ u, int level, int big_l, int t, const Mods& mods,
                                              const Tables& tb) {
  typedef word_t<NARROW> W;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN>::T;
  const size_t b = blockIdx.y;
  const int mi = (t < level) ? t : big_l;
  const ModConst m = mods.m[mi];
  W acc0[16], acc1[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0;
  for (int j = 0; j < level; ++j) {
    if (j == t) {
      // the digit reduced mod its own prime is the (permuted) input limb itself
      load_limb_perm<LOGN, NARROW>(lds, c1 + b * cstride + (size_t)j * N, ginv);
      __syncthreads();
    } else {
      const u64 qj = mods.m[j].q;
      const u64* d = dcoef + (b * level + j) * N;
      const int tid = opaque_tid();
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = tid + r * T;
        lds_put<NARROW>(lds, i, lift_centered(d[i], qj, m));
      }
      fwd_lds<LOGN, NARROW>(lds, tb, mi, m.q);
    }
    const u64* kb = key + (((size_t)j * 2 + 0) * (big_l + 1) + mi) * N;
    const u64* ka = key + (((size_t)j * 2 + 1) * (big_l + 1) + mi) * N;
    const int tid = opaque_tid();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = tid + r * T;
      const u64 dv = lds_get<NARROW>(lds, i);
      // narrow key residues fit the low word of their u64 slot
      const u64 kbv = NARROW ? (u64)reinterpret_cast<const u32*>(kb)[2 * i] : kb[i];
      const u64 kav = NARROW ? (u64)reinterpret_cast<const u32*>(ka)[2 * i] : ka[i];
      acc0[r] = (W)addm<NARROW>(acc0[r], mul_mod_t<NARROW>(dv, kbv, m), m.q);
      acc1[r] = (W)addm<NARROW>(acc1[r], mul_mod_t<NARROW>(dv, kav, m), m.q);
      if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the load hoisting
    }
    __syncthreads();
  }
  u64* u0 = u + ((b * 2 + 0) * (level + 1) + t) * N;
  u64* u1 = u + ((b * 2 + 1) * (level + 1) + t) * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (int)threadIdx.x + r * T;
    u0[i] = acc0[r];
    u1[i] = acc1[r];
  }
}

// Target moduli of one width class: blockIdx.x indexes tl.t[] (values in
// [0, level], level meaning P).  Each class is its own kernel so the 32-bit
// body gets a register allocation of its own.
struct TargetList {
  int n;
  int t[HE_MAXM];
};

template <int LOGN, bool NARROW>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_ks_modup_ip(const u64* __restrict__ dcoef, const u64* __restrict__ c1, size_t cstride, u32 ginv,
              const u64* __restrict__ key, u64* __restrict__ u, int level, int big_l, TargetList tl, Mods mods,
              Tables tb) {
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  modup_ip_body<LOGN, NARROW>(lds, dcoef, c1, cstride, ginv, key, u, level, big_l, tl.t[blockIdx.x], mods, tb);
}

// INTT of one limb of each polynomial: blockIdx.x = polynomial p.
// src + p * pstride + limb * N  ->  rcoef[p] (coefficient domain).
template <int LOGN>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_intt_last(const u64* __restrict__ src, size_t pstride, int limb, int mi, u64* __restrict__ rcoef, Mods mods,
            Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  const size_t p = blockIdx.x;
  const ModConst m = mods.m[mi];
  const u64* s = src + p * pstride + (size_t)limb * N;
  u64* out = rcoef + p * N;
  if (m.narrow) digits_body<LOGN, true>(lds, s, 1u, out, mi, m, tb);
  else digits_body<LOGN, false>(lds, s, 1u, out, mi, m, tb);
}

enum { EPI_STORE = 0, EPI_ROT = 1, EPI_ROTSUM = 2, EPI_RELIN = 3 };

struct EpiArgs {
  u64* out;              // output base (component 0, limb 0 of ciphertext 0)
  size_t out_pstride;    // elements between output polynomials (2 per ciphertext)
  const u64* c0;         // EPI_ROT: source ciphertexts (component 0 used); EPI_RELIN: d0/d1 base
  size_t c0_pstride;     // elements between source polynomials
  u32 g;                 // Galois element (EPI_ROT / EPI_ROTSUM)
  u32 ginv;              // its inverse mod 2N
  const u32* gpairs;     // optional per-ciphertext (g, g^-1) pairs (hoisted rotations)
};

// Drop the last limb: for polynomial p (blockIdx.y) and kept prime t
// (blockIdx.x): val = (src[p][t] - NTT(lift(rcoef[p]))) * div^-1 mod q_t,
// followed by the epilogue.  The divisor modulus is mods.m[div_mi].
template <int LOGN, int EPI, bool NARROW>
__device__ __forceinline__ void drop_last_body(u64* lds, const u64* __restrict__ src, size_t pstride,
                                               const u64* __restrict__ rcoef, int div_mi,
                                               const ConstTable& inv, EpiArgs ea, const Mods& mods,
                                               const Tables& tb) {
  typedef word_t<NARROW> W;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN>::T;
  const int t = blockIdx.x;
  const size_t p = blockIdx.y;
  const ModConst m = mods.m[t];
  const u64 qd = mods.m[div_mi].q;
  const u64* rc = rcoef + p * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (int)threadIdx.x + r * T;
    lds_put<NARROW>(lds, i, lift_centered(rc[i], qd, m));
  }
  fwd_lds<LOGN, NARROW>(lds, tb, t, m.q);
  const u64* s = src + p * pstride + (size_t)t * N;
  W val[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (int)threadIdx.x + r * T;
    val[r] = (W)shoupm<NARROW>(subm<NARROW>(s[i], lds_get<NARROW>(lds, i), m.q), inv.v[t], inv.sh[t], m.q);
  }
  const int comp = (int)(p & 1);
  u64* o = ea.out + p * ea.out_pstride + (size_t)t * N;
  if constexpr (EPI == EPI_STORE) {
#pragma unroll
    for (int r = 0; r < 16; ++r) o[(int)threadIdx.x + r * T] = val[r];
  } else if constexpr (EPI == EPI_RELIN) {
    const u64* d = ea.c0 + p * ea.c0_pstride + (size_t)t * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = (int)threadIdx.x + r * T;
      o[i] = addm<NARROW>(d[i], val[r], m.q);
    }
  } else {  // EPI_ROT / EPI_ROTSUM
    if (comp == 0) {
      const u32 ginv = ea.gpairs ? ea.gpairs[2 * (p >> 1) + 1] : ea.ginv;
      __syncthreads();  // everyone is done reading the lifted limb
      const u64* c0 = ea.c0 + p * ea.c0_pstride + (size_t)t * N;
      W own[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int idx = (int)threadIdx.x + r * T;
        const u64 v = c0[idx];
        own[r] = (W)v;
        lds_put<NARROW>(lds, galois_src<LOGN>(idx, ginv), v);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = (int)threadIdx.x + r * T;
        u64 x = addm<NARROW>(lds_get<NARROW>(lds, i), val[r], m.q);  // sigma_g(c0) + u0
        if constexpr (EPI == EPI_ROTSUM) x = addm<NARROW>(x, own[r], m.q);
        o[i] = x;
      }
    } else {
      if constexpr (EPI == EPI_ROTSUM) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = (int)threadIdx.x + r * T;
          o[i] = addm<NARROW>(o[i], val[r], m.q);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) o[(int)threadIdx.x + r * T] = val[r];
      }
    }
  }
}

template <int LOGN, int EPI>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_drop_last(const u64* __restrict__ src, size_t pstride, const u64* __restrict__ rcoef, int div_mi,
            ConstTable inv, EpiArgs ea, Mods mods, Tables tb) {
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  if (mods.m[blockIdx.x].narrow)
    drop_last_body<LOGN, EPI, true>(lds, src, pstride, rcoef, div_mi, inv, ea, mods, tb);
  else
    drop_last_body<LOGN, EPI, false>(lds, src, pstride, rcoef, div_mi, inv, ea, mods, tb);
}

// ---------------------------------------------------------------------------
// Hoisted rotations of one ciphertext.
// ModUp once: dhat[j][t] = NTT(lift(digit_j) mod m_t) for j < level,
// t <= level (t == level is P).  blockIdx.x = t, blockIdx.y = j.
template <int LOGN, bool NARROW>
__device__ __forceinline__ void modup_store_body(u64* lds, const u64* __restrict__ dcoef, const u64* __restrict__ c1,
                                                 u64* __restrict__ dhat, int level, int big_l, const Mods& mods,
                                                 const Tables& tb) {
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN>::T;
  const int t = blockIdx.x;
  const int j = blockIdx.y;
  const int mi = (t < level) ? t : big_l;
  const ModConst m = mods.m[mi];
  u64* out = dhat + ((size_t)j * (level + 1) + t) * N;
  if (j == t) {
    const u64* src = c1 + (size_t)j * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) out[(int)threadIdx.x + r * T] = src[(int)threadIdx.x + r * T];
    return;
  }
  const u64 qj = mods.m[j].q;
  const u64* d = dcoef + (size_t)j * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (int)threadIdx.x + r * T;
    lds_put<NARROW>(lds, i, lift_centered(d[i], qj, m));
  }
  fwd_lds<LOGN, NARROW>(lds, tb, mi, m.q);
  store_limb<LOGN, NARROW>(out, lds, m, false);
}

template <int LOGN>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_modup_store(const u64* __restrict__ dcoef, const u64* __restrict__ c1, u64* __restrict__ dhat, int level, int big_l,
              Mods mods, Tables tb) {
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  const int mi = ((int)blockIdx.x < level) ? (int)blockIdx.x : big_l;
  if (mods.m[mi].narrow)
    modup_store_body<LOGN, true>(lds, dcoef, c1, dhat, level, big_l, mods, tb);
  else
    modup_store_body<LOGN, false>(lds, dcoef, c1, dhat, level, big_l, mods, tb);
}

// Inner product of the shared lifted digits, permuted per rotation, with
// that rotation's key: u[r][c][t][i] = sum_j dhat[j][t][src_{g_r}(i)] *
// key_r[j][c][m_t][i].  grid (N / 256, level + 1, m).
template <int LOGN>
__global__ void k_ip_perm(const u64* __restrict__ dhat, const u64* const* __restrict__ keys,
                          const u32* __restrict__ gpairs, u64* __restrict__ u, int level, int big_l, Mods mods) {
  constexpr int N = 1 << LOGN;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t r = blockIdx.z;
  const int mi = (t < level) ? t : big_l;
  const ModConst m = mods.m[mi];
  const u32 g = gpairs[2 * r];
  const int src = galois_src<LOGN>(i, g);
  const u64* key = keys[r];
  u64 s0 = 0, s1 = 0;
  for (int j = 0; j < level; ++j) {
    const u64 dv = dhat[((size_t)j * (level + 1) + t) * N + src];
    s0 = add_mod(s0, mul_mod(dv, key[(((size_t)j * 2 + 0) * (big_l + 1) + mi) * N + i], m), m.q);
    s1 = add_mod(s1, mul_mod(dv, key[(((size_t)j * 2 + 1) * (big_l + 1) + mi) * N + i], m), m.q);
  }
  u[((r * 2 + 0) * (level + 1) + t) * N + i] = s0;
  u[((r * 2 + 1) * (level + 1) + t) * N + i] = s1;
}

// ---------------------------------------------------------------------------
// Elementwise kernels: blockIdx.x * blockDim.x + threadIdx.x = coefficient,
// blockIdx.y = limb, blockIdx.z = item.

__device__ __forceinline__ u32 pow_mod_2n(u32 base, u32 e, u32 mask2n) {
  u32 r = 1, b = base;
  while (e) {
    if (e & 1u) r = (r * b) & mask2n;
    b = (b * b) & mask2n;
    e >>= 1;
  }
  return r;
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

// DensePack MulPC (Table I): output out_base + blockIdx.y (index o*S + p),
// limb blockIdx.x; out[blockIdx.y] = sum_m x_m * sigma_{g_p}(F[o][class][m]).
struct DPGeom {
  int h, w, c_in, d, stride, pad, o_c;
  int out_h, out_w, n_row_cls, n_col_cls, m_cts;
  int row_cls[64], col_cls[64];  // class id of every output row / column
};

template <int LOGN, bool NARROW>
__device__ __forceinline__ void dp_hma_body(const u64* __restrict__ x, const u64* __restrict__ filt,
                                            u64* __restrict__ out, int level, int out_base, const DPGeom& geo,
                                            const ModConst& m, u64* lds) {
  typedef word_t<NARROW> W;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN>::T;
  const int t = blockIdx.x;
  const int oi = out_base + (int)blockIdx.y;  // absolute output index o*S + p
  const int spatial = geo.out_h * geo.out_w;
  const int o = oi / spatial;
  const int pidx = oi % spatial;
  const int i = pidx / geo.out_w, j = pidx % geo.out_w;
  const int cls = geo.row_cls[i] * geo.n_col_cls + geo.col_cls[j];
  const int slots = N / 2;
  const int anchor = (geo.stride * i - geo.pad) * geo.w + (geo.stride * j - geo.pad);
  // rotation right by anchor: g = 5^(-anchor mod slots); its inverse is 5^(anchor mod slots)
  int a_mod = anchor % slots;
  if (a_mod < 0) a_mod += slots;
  const u32 mask2n = (2u << LOGN) - 1u;
  const u32 ginv = pow_mod_2n(5u, (u32)a_mod, mask2n);
  W acc0[16], acc1[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0;
  const int n_cls = geo.n_row_cls * geo.n_col_cls;
  for (int mc = 0; mc < geo.m_cts; ++mc) {
    const u64* f = filt + ((((size_t)o * n_cls + cls) * geo.m_cts + mc) * level + t) * N;
    load_limb_perm<LOGN, NARROW>(lds, f, ginv);
    __syncthreads();
    const u64* x0 = x + (((size_t)mc * 2 + 0) * level + t) * N;
    const u64* x1 = x + (((size_t)mc * 2 + 1) * level + t) * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int k = (int)threadIdx.x + r * T;
      const u64 fv = lds_get<NARROW>(lds, k);
      acc0[r] = (W)addm<NARROW>(acc0[r], mul_mod_t<NARROW>(x0[k], fv, m), m.q);
      acc1[r] = (W)addm<NARROW>(acc1[r], mul_mod_t<NARROW>(x1[k], fv, m), m.q);
    }
    __syncthreads();
  }
  u64* o0 = out + (((size_t)blockIdx.y * 2 + 0) * level + t) * N;  // chunk-relative
  u64* o1 = out + (((size_t)blockIdx.y * 2 + 1) * level + t) * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = (int)threadIdx.x + r * T;
    o0[k] = acc0[r];
    o1[k] = acc1[r];
  }
}

template <int LOGN>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_dp_hma(const u64* __restrict__ x, const u64* __restrict__ filt, u64* __restrict__ out, int level, int out_base,
         DPGeom geo, Mods mods) {
  __shared__ u64 lds[NttGeom<LOGN>::LDS];
  const ModConst m = mods.m[blockIdx.x];
  if (m.narrow) dp_hma_body<LOGN, true>(x, filt, out, level, out_base, geo, m, lds);
  else dp_hma_body<LOGN, false>(x, filt, out, level, out_base, geo, m, lds);
}

// Sum of permuted-plaintext products into one accumulator per blockIdx.z:
// acc[z] (+)= sum_{k<K} cts[z*K + k] * sigma_{g_k}(pts[k * pt_stride]), with
// g_k = gal[k] (or g_k = g_step^k when gal == nullptr).
template <int LOGN>
__global__ void k_hma_perm(u64* __restrict__ acc, const u64* __restrict__ cts, int K,
                           const u64* __restrict__ pts, int pt_stride, int pt_limbs,
                           const int32_t* __restrict__ gal, u32 g_step, int level, int accumulate, Mods mods) {
  constexpr int N = 1 << LOGN;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t z = blockIdx.z;
  const ModConst m = mods.m[t];
  const u32 mask2n = (2u << LOGN) - 1u;
  u64* a0 = acc + ((z * 2 + 0) * level + t) * N;
  u64* a1 = acc + ((z * 2 + 1) * level + t) * N;
  u64 s0 = accumulate ? a0[i] : 0, s1 = accumulate ? a1[i] : 0;
  u32 g = 1;
  for (int k = 0; k < K; ++k) {
    const u32 gk = gal ? (u32)gal[k] : g;
    const int src = (gk == 1u) ? i : galois_src<LOGN>(i, gk);
    const u64 pv = pts[((size_t)k * pt_stride * pt_limbs + t) * N + src];
    const size_t cbase = (z * K + k) * 2;
    s0 = add_mod(s0, mul_mod(cts[((cbase + 0) * level + t) * N + i], pv, m), m.q);
    s1 = add_mod(s1, mul_mod(cts[((cbase + 1) * level + t) * N + i], pv, m), m.q);
    g = (g * g_step) & mask2n;
  }
  a0[i] = s0;
  a1[i] = s1;
}

// Integer-scalar MAC (ConvPack, Table II): out[o] = sum_k w[k][o] * in[k],
// with w given per limb as residues + Shoup companions: wres[(k*o_c + o)*level + t].
__global__ void k_scalar_mac(u64* __restrict__ out, const u64* __restrict__ in, int K, int o_c,
                             const u64* __restrict__ wres, const u64* __restrict__ wsh, int level, int n,
                             Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t o = blockIdx.z;
  const ModConst m = mods.m[t];
  u64 s0 = 0, s1 = 0;
  for (int k = 0; k < K; ++k) {
    const size_t wi = ((size_t)k * o_c + o) * level + t;
    const u64 w = wres[wi], ws = wsh[wi];
    s0 = add_mod(s0, mul_shoup(in[(((size_t)k * 2 + 0) * level + t) * n + i], w, ws, m.q, m.narrow), m.q);
    s1 = add_mod(s1, mul_shoup(in[(((size_t)k * 2 + 1) * level + t) * n + i], w, ws, m.q, m.narrow), m.q);
  }
  out[((o * 2 + 0) * level + t) * n + i] = s0;
  out[((o * 2 + 1) * level + t) * n + i] = s1;
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

// ---------------------------------------------------------------------------
// Client-side helpers (key generation, encryption, decryption).

// out[t] = coeffs mod modulus (first_mod + t), coefficient domain.
__global__ void k_from_signed(u64* out, const int64_t* coeffs, int first_mod, int n, Mods mods) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  out[(size_t)t * n + i] = from_signed(coeffs[i], mods.m[first_mod + t]);
}

// Switching key rows: for digit j (blockIdx.z) and modulus t (blockIdx.y):
// b = e_hat - a*s + [t == j] (P mod q_t) * s', with s' = sigma_g(s) (g odd)
// or s^2 (g == 0).  ehat = NTT(e_j mod m_t) = [L][L+1][N] precomputed.
template <int LOGN>
__global__ void k_keygen(u64* key, const u64* s, const u64* a, const u64* ehat, u32 g, int big_l,
                         ConstTable p_mod, Mods mods) {
  constexpr int N = 1 << LOGN;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const int j = blockIdx.z;
  const ModConst m = mods.m[t];
  const size_t row = ((size_t)j * (big_l + 1) + t) * N;
  const u64 sv = s[(size_t)t * N + i];
  const u64 av = a[row + i];
  u64 b = sub_mod(ehat[row + i], mul_mod(av, sv, m), m.q);
  if (t == j) {
    u64 sp;
    if (g == 0) sp = mul_mod(sv, sv, m);
    else sp = s[(size_t)t * N + galois_src<LOGN>(i, g)];
    b = add_mod(b, mul_shoup(sp, p_mod.v[t], p_mod.sh[t], m.q, m.narrow), m.q);
  }
  key[(((size_t)j * 2 + 0) * (big_l + 1) + t) * N + i] = b;
  key[(((size_t)j * 2 + 1) * (big_l + 1) + t) * N + i] = av;
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

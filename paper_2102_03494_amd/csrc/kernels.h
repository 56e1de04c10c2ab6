// HIP kernels of the homomorphic convolution path (gfx950).
//
// Data layout (device, caller-owned): a ciphertext is [2][level][N] uint64
// residues in the NTT domain, limb-major, so each limb is one contiguous
// 8N-byte run and every kernel reads and writes whole limbs with unit-stride
// (coalesced) accesses.  Kernels that need a transform hold one limb per
// workgroup in LDS (ntt_lds.h); elementwise kernels use one thread per
// coefficient.  The width class of each prime (modarith.h: narrow < 2^30,
// f64 < 2^42, wide < 2^62) is uniform per workgroup; each transform kernel
// branches once on it into a body compiled for that class (32-bit words for
// narrow limbs, exact integers in doubles for f64 limbs).
//
// Key switching of a batch of ciphertexts (rotation or relinearisation) runs
// as four kernels, each batched over every ciphertext of the call:
//   k_ks_digits    INTT of each limb of sigma_g(c1)  -> coefficient digits
//   k_ks_modup_ip  per target modulus: centred lift of each digit, NTT, and
//                  the inner product with the key, accumulated in registers
//                  (the lifted digits never go to memory); the P target is
//                  split over `pg` groups of digits, each its own workgroup
//   k_intt_last    sum of the P partials, INTT of the P limb of (u0, u1)
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

// Twiddle tables [n_mods][4][N] (fwd, fwd companion, inv, inv companion):
// 64-bit with Shoup companions for every modulus, 32-bit copies for the
// narrow ones, and doubles (w, w / q) for the f64 ones.
struct Tables {
  const u64* tw64;
  const u32* tw32;
  const double* twf;
  // half-ring forward tables [n_mods][2 halves][2 (w, companion)][N/2]
  const u64* twh64;
  const u32* twh32;
  const double* twhf;
};

template <int LOGN, int CLS>
__device__ __forceinline__ Tw<CLS> tw_of(const Tables& tb, int mi, int which) {
  constexpr size_t N = (size_t)1 << LOGN;
  const size_t o = ((size_t)mi * 4 + which) * N;
  if constexpr (CLS == CLS_N32) return {tb.tw32 + o, tb.tw32 + o + N};
  else if constexpr (CLS == CLS_F64) return {tb.twf + o, tb.twf + o + N};
  else return {tb.tw64 + o, tb.tw64 + o + N};
}

// Forward twiddles of half h of a ring of 2^LOGN points after its first stage:
// the table of an N/2-point transform (index 2^s' + k' of its stage s', block
// k') holding the full transform's twiddles of the blocks inside half h.
template <int LOGN, int CLS>
__device__ __forceinline__ Tw<CLS> tw_half_of(const Tables& tb, int mi, int h) {
  constexpr size_t NH = (size_t)1 << (LOGN - 1);
  const size_t o = ((size_t)mi * 2 + h) * 2 * NH;
  if constexpr (CLS == CLS_N32) return {tb.twh32 + o, tb.twh32 + o + NH};
  else if constexpr (CLS == CLS_F64) return {tb.twhf + o, tb.twhf + o + NH};
  else return {tb.twh64 + o, tb.twh64 + o + NH};
}

// Transform kernels are templated on the width class CLS: the host launches
// one instance per class present among the primes a launch touches (in every
// configuration here that is one launch), and workgroups whose prime is of
// another class exit at once.  One class per kernel keeps its register
// allocation to what that class needs.

// An opaque copy of the thread index (see ntt_lds.h): defined where it is
// used so that address arithmetic is not hoisted out of enclosing loops.
__device__ __forceinline__ int opaque_tid() {
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  return tid;
}

// Residue i of a limb row stored as 64-bit words, or packed as 32-bit words
// (narrow primes).
__device__ __forceinline__ u64 ld_res(const u64* row, int i, bool packed) {
  return packed ? (u64) reinterpret_cast<const u32*>(row)[i] : row[i];
}
__device__ __forceinline__ void st_res(u64* row, int i, u64 v, bool packed) {
  if (packed) reinterpret_cast<u32*>(row)[i] = (u32)v;
  else row[i] = v;
}

template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void fwd_lds(u64* lds, const Tables& tb, int mi, const ModConst& m) {
  ntt_fwd_lds<LOGN, CLS, E>(lds, tw_of<LOGN, CLS>(tb, mi, 0), mview<CLS>(m), opaque_tid());
}

template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void inv_lds(u64* lds, const Tables& tb, int mi, const ModConst& m) {
  ntt_inv_lds<LOGN, CLS, E>(lds, tw_of<LOGN, CLS>(tb, mi, 2), mview<CLS>(m), opaque_tid());
}

// Entries per thread of the ModUp + inner-product kernels: 8 (twice the
// threads of a transform workgroup, half the registers per thread, so twice
// the waves per SIMD) while N / 8 threads fit a workgroup.
template <int LOGN>
constexpr int modup_e() {
  return LOGN <= 13 ? 8 : 16;
}
template <int LOGN>
constexpr int modup_threads() {
  return NttGeom<LOGN, modup_e<LOGN>()>::T;
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
// IN_LOOP: the call sits in a loop whose trips share ginv; the permuted
// indices are then formed at each call instead of being hoisted out of the
// loop and held in registers (or spilled) across it.
template <int LOGN, int CLS, int E = 16, bool IN_LOOP = false>
__device__ __forceinline__ void load_limb_perm(u64* lds, const u64* __restrict__ src, u32 ginv, bool packed = false) {
  constexpr int T = NttGeom<LOGN, E>::T;
  const int tid = IN_LOOP ? opaque_tid() : (int)threadIdx.x;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int idx = tid + r * T;
    const u64 v = ld_res(src, idx, packed);
    const int dst = (ginv == 1u) ? idx : galois_src<LOGN>(idx, ginv);
    lds_put<CLS>(lds, dst, v);
  }
}

// Store the LDS limb as canonical residues, optionally scaled by N^-1 (after
// an inverse transform).  PACK: a narrow limb goes out as N 32-bit words at
// the start of its row (the layout of coefficient-domain scratch rows, which
// lift_limb reads); otherwise every residue takes a 64-bit word.
template <int LOGN, int CLS, bool PACK = false, int E = 16>
__device__ __forceinline__ void store_limb(u64* __restrict__ dst, const u64* lds, const ModConst& m, bool scale) {
  constexpr int T = NttGeom<LOGN, E>::T;
  const int i0 = lds_idx((int)threadIdx.x);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = (int)threadIdx.x + r * T;
    const int li = lds_step(i0, r, T);
    if constexpr (CLS == CLS_F64) {
      double v = lds_getw_at<CLS>(lds, li);
      if (scale) v = f64_mulc(v, f64_from_u64(m.n_inv), m.n_inv_q, m.qd);
      dst[i] = to_canon<CLS>(v, m);
    } else {
      u64 v = to_canon<CLS>(lds_getw_at<CLS>(lds, li), m);
      if (scale) v = shoupm<CLS == CLS_N32>(v, m.n_inv, m.n_inv_sh, m.q);
      if constexpr (PACK && CLS == CLS_N32) reinterpret_cast<u32*>(dst)[i] = (u32)v;
      else dst[i] = v;
    }
  }
}

// Centred lift into LDS of one limb of residues mod qs (odd), the 16 entries
// tid + r T of this thread, in the word of target m's class.  All loads are
// issued before any is used, and the method is chosen once (it is uniform
// per workgroup):
//   narrow target, narrow source with qs < 2 q_t: one conditional add (both
//     halves of the centred range then land in [0, q_t));
//   f64 target, source below 2^43: the signed value itself (the transforms
//     take it unreduced);
//   narrow target, source below 2^43: an exact FP64 reduction of the signed
//     value;
//   otherwise: lift_centered (64-bit Barrett).
// A narrow source row is packed: N 32-bit words (store_limb<.., true>).
template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void lift_limb(u64* lds, const u64* __restrict__ src, u64 qs, const ModConst& m, int tid) {
  constexpr int T = NttGeom<LOGN, E>::T;
  const int i0 = lds_idx(tid);
  if (qs < NARROW_LIMIT) {
    const u32* s32 = reinterpret_cast<const u32*>(src);
    u32 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = s32[tid + r * T];
    const u32 half = (u32)((qs - 1) / 2);
    if constexpr (CLS == CLS_N32) {
      if (qs < 2 * m.q) {
        const u32 add = (u32)(m.q - qs);
#pragma unroll
        for (int r = 0; r < E; ++r) lds_putw_at<CLS>(lds, lds_step(i0, r, T), v[r] > half ? v[r] + add : v[r]);
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r) lds_putw_at<CLS>(lds, lds_step(i0, r, T), (u32)lift_centered(v[r], qs, m));
      }
    } else if constexpr (CLS == CLS_F64) {
      const double qsd = (double)(u32)qs;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const double x = (double)v[r];
        lds_putw_at<CLS>(lds, lds_step(i0, r, T), v[r] > half ? x - qsd : x);
      }
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) lds_putw_at<CLS>(lds, lds_step(i0, r, T), lift_centered(v[r], qs, m));
    }
  } else {
    u64 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = src[tid + r * T];
    const u64 half = (qs - 1) / 2;
    if constexpr (CLS == CLS_F64) {
      if (qs < ((u64)1 << 43)) {
        const double qsd = f64_from_u64(qs);
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const double x = f64_from_u64(v[r]);
          lds_putw_at<CLS>(lds, lds_step(i0, r, T), v[r] > half ? x - qsd : x);
        }
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r)
          lds_putw_at<CLS>(lds, lds_step(i0, r, T), f64_from_u64(lift_centered(v[r], qs, m)));
      }
    } else if constexpr (CLS == CLS_N32) {
      if (qs < ((u64)1 << 43)) {
        const double qsd = f64_from_u64(qs);
#pragma unroll
        for (int r = 0; r < E; ++r) {
          double x = f64_from_u64(v[r]);
          if (v[r] > half) x -= qsd;
          lds_putw_at<CLS>(lds, lds_step(i0, r, T), (u32)f64_canon(x, m.qd, m.qinv));
        }
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r) lds_putw_at<CLS>(lds, lds_step(i0, r, T), (u32)lift_centered(v[r], qs, m));
      }
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) lds_putw_at<CLS>(lds, lds_step(i0, r, T), lift_centered(v[r], qs, m));
    }
  }
}

// ---------------------------------------------------------------------------
// Standalone transforms: blockIdx.x = limb, blockIdx.y = polynomial.
template <int LOGN, bool FWD, int CLS>
__device__ __forceinline__ void ntt_body(u64* lds, u64* p, int mi, const ModConst& m, const Tables& tb) {
  load_limb_perm<LOGN, CLS>(lds, p, 1u);
  if (FWD) fwd_lds<LOGN, CLS>(lds, tb, mi, m); else inv_lds<LOGN, CLS>(lds, tb, mi, m);
  store_limb<LOGN, CLS>(p, lds, m, !FWD);
}

template <int LOGN, bool FWD, int CLS>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_ntt(u64* data, int n_limbs, int first_mod, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const int limb = blockIdx.x;
  const int mi = first_mod + limb;
  const ModConst m = mods.m[mi];
  u64* p = data + ((size_t)blockIdx.y * n_limbs + limb) * N;
  if ((int)m.cls != CLS) return;
  ntt_body<LOGN, FWD, CLS>(lds, p, mi, m, tb);
}

// ---------------------------------------------------------------------------
// Inverse transform of one limb into the coefficient domain (scaled by N^-1),
// optionally through the Galois permutation on the way into LDS.
template <int LOGN, int CLS>
__device__ __forceinline__ void digits_body(u64* lds, const u64* src, u32 ginv, u64* out, int j, const ModConst& m,
                                            const Tables& tb, bool packed = false) {
  load_limb_perm<LOGN, CLS>(lds, src, ginv, packed);
  inv_lds<LOGN, CLS>(lds, tb, j, m);
  store_limb<LOGN, CLS, true>(out, lds, m, true);
}

// ---------------------------------------------------------------------------
// Batched key switching and rescaling over per-ciphertext job descriptors.
//
// One job per ciphertext: the polynomial to switch (`d`, NTT domain,
// [level][N]), the ciphertext whose c0 the epilogue uses (`c`), the output,
// the switching key (nullptr: identity job, the epilogue copies `c` to
// `out`), the Galois element applied before switching and its inverse, and
// the job's level.  Jobs of one launch may have different levels, keys and
// Galois elements (ragged batches, several layers or requests at once);
// workspace rows are laid out with the launch's largest level Lmax and the
// number pg of P groups:
//   dcoef [count][Lmax][N]        coefficient-domain digits (narrow rows packed,
//                                 N 32-bit words)
//   u     [count][2][Lmax+pg][N]  inner products: q_t at row t < level, the
//                                 partial sum of P group k at row Lmax + k
//                                 (rows of narrow primes packed)
//   rc    [count][2][N]           coefficient-domain last limb (ModDown/rescale;
//                                 packed when narrow)
// Switching keys are [L][2][L+1][N] 64-bit words (digit j, component b/a,
// modulus); a row of a narrow modulus holds N packed 32-bit residues.
// Workgroup placement of the key-switch kernels.  The dispatcher hands
// workgroup i of a 1-D grid to XCD i mod 8, and each XCD has its own L2.  The
// kernels below run on grids of per * round8(count) workgroups mapped
// job-major per XCD: all `per` workgroups of job b run on XCD b mod 8, one
// after another, so the targets of a ciphertext share its digits in one L2 and
// what one kernel writes for a job (digits, inner products, the P limb) the
// next reads from that L2.  Slots past `count` exit.
struct XcdSlot {
  int job;  // job index (may be >= count: exit)
  int sub;  // workgroup within the job, 0 .. per-1
};
__device__ __forceinline__ XcdSlot xcd_slot(int per) {
  const unsigned i = blockIdx.x;
  const unsigned local = i >> 3;
  return XcdSlot{(int)((local / per) * 8 + (i & 7u)), (int)(local % per)};
}
__host__ __device__ inline unsigned xcd_grid(int per, int count) { return (unsigned)per * ((count + 7) & ~7); }

struct KsJob {
  const u64* d;    // polynomial to switch / ciphertext to rescale
  const u64* c;    // EPI_ROT*: source ciphertext (c0 at c); EPI_RELIN: (d0, d1)
  u64* out;        // output ciphertext
  const u64* key;  // [big_l][2][big_l+1][N]; nullptr = identity
  u32 g, ginv;     // Galois element (1 = none) and its inverse mod 2N
  int level;
  int flags;       // JOB_IN_PACKED / JOB_OUT_PACKED
};

// Packed ciphertexts: every limb (all narrow primes) as N 32-bit residues at
// the start of its 64-bit row, in the usual [2][level][N] layout.  The
// internal accumulator of a rotate-and-sum chain is kept so between steps:
// d and c of a job are packed (JOB_IN_PACKED), out is written packed
// (JOB_OUT_PACKED).  ModUp reads the flag of each job; the digit, P-INTT
// and ModDown/rescale kernels take the launch's flags as a template
// parameter (all jobs of a launch share them).
enum { JOB_IN_PACKED = 1, JOB_OUT_PACKED = 2 };

// Key switch, step 1: coefficient-domain digits of sigma_g(d).
// grid xcd_grid(Lmax, count): workgroup = (job b, digit j).
template <int LOGN, int CLS, bool PIN = false>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_ks_digits(const KsJob* __restrict__ jobs, int count, u64* __restrict__ dcoef, int lmax, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const XcdSlot sl = xcd_slot(lmax);
  if (sl.job >= count) return;
  const int j = sl.sub;
  const size_t b = sl.job;
  const KsJob jb = jobs[b];
  if (jb.key == nullptr || j >= jb.level) return;
  const ModConst m = mods.m[j];
  const u64* src = jb.d + (size_t)j * N;
  u64* out = dcoef + (b * lmax + j) * N;
  if ((int)m.cls != CLS) return;
  digits_body<LOGN, CLS>(lds, src, jb.ginv, out, j, m, tb, PIN);
}

// P groups: with pg groups a job at `level` gives group k the digits
// [k G, min((k + 1) G, level)), G = ceil(level / pg); groups past the last
// digit are empty and have no partial.
__host__ __device__ inline int pgroup_size(int level, int pg) { return (level + pg - 1) / pg; }
__host__ __device__ inline int pgroup_count(int level, int pg) {
  const int g = pgroup_size(level, pg);
  return (level + g - 1) / g;
}

// The whole P limb of one inner-product polynomial, held as this thread's E
// accumulators (entries tid + r T, as modup_ip_body sums them), to its
// coefficient-domain copy for ModDown: canonical residues, INTT, N^-1, packed
// store at out (what k_intt_last computes from a u row).
template <int LOGN, int CLS, int E, typename A>
__device__ __forceinline__ void p_limb_to_coeffs(u64* lds, const A (&acc)[E], u64* out, int mi, const ModConst& m,
                                                 const Tables& tb) {
  constexpr int T = NttGeom<LOGN, E>::T;
  __syncthreads();  // the LDS buffer is free
#pragma unroll
  for (int r = 0; r < E; ++r) {
    u64 v;
    if constexpr (CLS == CLS_N32) v = reduce64(acc[r], m);
    else if constexpr (CLS == CLS_F64) v = to_canon<CLS>(acc[r], m);
    else v = acc[r];
    lds_put<CLS>(lds, (int)threadIdx.x + r * T, v);
  }
  inv_lds<LOGN, CLS, E>(lds, tb, mi, m);
  store_limb<LOGN, CLS, true, E>(out, lds, m, true);
}

// Key switch, step 2: ModUp + inner product for one target: a ciphertext
// prime t over all digits, or one group of digits [j0, j1) for P.
// Accumulates sum_j NTT(lift(digit_j) mod m) * key[j][.][m] in registers and
// writes it to u row `row` (canonical residues).
template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void modup_ip_body(u64* lds, const u64* __restrict__ dcoef, const KsJob& jb, size_t b,
                                              u64* __restrict__ u, u64* __restrict__ rc_p, int lmax, int urows,
                                              int big_l, int t, int mi, int j0, int j1, int row, const Mods& mods,
                                              const Tables& tb) {
  // accumulators: 64-bit sums of products of canonical narrow residues
  // (each < 2^60, at most 15 digits), centred doubles (f64), residues (wide)
  typedef std::conditional_t<CLS == CLS_N32, u64, word_t<CLS>> A;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN, E>::T;
  const ModConst m = mods.m[mi];
  const u64* key = jb.key;
  A acc0[E], acc1[E];
#pragma unroll
  for (int r = 0; r < E; ++r) acc0[r] = acc1[r] = 0;
  for (int j = j0; j < j1; ++j) {
    if (j == t) {
      // the digit reduced mod its own prime is the (permuted) input limb itself
      load_limb_perm<LOGN, CLS, E, true>(lds, jb.d + (size_t)j * N, jb.ginv, (jb.flags & JOB_IN_PACKED) != 0);
      __syncthreads();
    } else {
      lift_limb<LOGN, CLS, E>(lds, dcoef + (b * lmax + j) * N, mods.m[j].q, m, opaque_tid());
      fwd_lds<LOGN, CLS, E>(lds, tb, mi, m);
    }
    const u64* kb = key + (((size_t)j * 2 + 0) * (big_l + 1) + mi) * N;
    const u64* ka = key + (((size_t)j * 2 + 1) * (big_l + 1) + mi) * N;
    const int tid = opaque_tid();
    const int i0 = lds_idx(tid);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = tid + r * T;
      const int li = lds_step(i0, r, T);
      if constexpr (CLS == CLS_N32) {
        const u32 dv = (u32)to_canon<CLS>(lds_getw_at<CLS>(lds, li), m);
        // narrow key rows are packed 32-bit residues
        acc0[r] += (u64)dv * reinterpret_cast<const u32*>(kb)[i];
        acc1[r] += (u64)dv * reinterpret_cast<const u32*>(ka)[i];
      } else if constexpr (CLS == CLS_F64) {
        const double dv = lds_getw_at<CLS>(lds, li);
        // centred products, summed unreduced (|sum| < 8.2 q for <= 15 digits)
        acc0[r] += f64_mulmod(dv, f64_from_u64(kb[i]), m.qd, m.qinv);
        acc1[r] += f64_mulmod(dv, f64_from_u64(ka[i]), m.qd, m.qinv);
      } else {
        const u64 dv = lds_getw_at<CLS>(lds, li);
        acc0[r] = add_mod(acc0[r], mul_mod_t<false>(dv, kb[i], m), m.q);
        acc1[r] = add_mod(acc1[r], mul_mod_t<false>(dv, ka[i], m), m.q);
      }
      if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the load hoisting
    }
    __syncthreads();
  }
  if (rc_p) {
    p_limb_to_coeffs<LOGN, CLS, E>(lds, acc0, rc_p, mi, m, tb);
    p_limb_to_coeffs<LOGN, CLS, E>(lds, acc1, rc_p + N, mi, m, tb);
    return;
  }
  const bool lazy = mi != big_l;  // ciphertext-prime rows in [0, 2q) (reduce64_lazy32)
  u64* u0 = u + ((b * 2 + 0) * urows + row) * N;
  u64* u1 = u + ((b * 2 + 1) * urows + row) * N;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = (int)threadIdx.x + r * T;
    if constexpr (CLS == CLS_N32) {  // packed row
      reinterpret_cast<u32*>(u0)[i] = lazy ? reduce64_lazy32(acc0[r], m) : (u32)reduce64(acc0[r], m);
      reinterpret_cast<u32*>(u1)[i] = lazy ? reduce64_lazy32(acc1[r], m) : (u32)reduce64(acc1[r], m);
    } else if constexpr (CLS == CLS_F64) {
      u0[i] = to_canon<CLS>(acc0[r], m);
      u1[i] = to_canon<CLS>(acc1[r], m);
    } else {
      u0[i] = acc0[r];
      u1[i] = acc1[r];
    }
  }
}

// Asynchronous copy of one 32-bit word per lane from global memory into LDS
// (global_load_lds_dword): lane l of the calling wave writes wave_dst[l], so
// wave_dst must be the same for all lanes of the wave.  The copy is counted
// by the wave's vector-memory counter; wait_vm() waits for all of them.
__device__ __forceinline__ void copy_to_lds(const u32* src, u32* wave_dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)wave_dst, 4, 0, 0);
}
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Largest ring with a staged narrow ModUp (its staging array and transform
// buffer fit a CU's LDS), and the staging array's size in 32-bit words: the
// key rows of one digit (2 N), or the transform buffer of the ring's other
// class when the kernel serves two.
constexpr int STAGE_MAX_LOGN = 13;
template <int LOGN>
constexpr int stage_words() {
  return (2 << LOGN) > 2 * lds_words<LOGN, CLS_U64>() ? (2 << LOGN) : 2 * lds_words<LOGN, CLS_U64>();
}

// ModUp + inner product for a narrow target (as modup_ip_body), with the key
// rows of digit j (both components, packed 32-bit) copied asynchronously
// into the staging array S = [key b | key a] before the digit itself is
// loaded: both loads are in flight together, and the products read the key
// from LDS.  (Vector-memory loads complete in issue order, so the twiddle
// loads of the transform would wait for copies issued after the digit; the
// copies go first.)  Each lane reads back only the words it copied, so a
// wave waits for its own copies and needs no barrier for them.
template <int LOGN, int E>
__device__ __forceinline__ void modup_ip_narrow_staged(u64* lds, u32* S, const u64* __restrict__ dcoef,
                                                       const KsJob& jb, size_t b, u64* __restrict__ u,
                                                       u64* __restrict__ rc_p, int lmax, int urows, int big_l, int t,
                                                       int mi, int j0, int j1, int row, const Mods& mods,
                                                       const Tables& tb) {
  constexpr int CLS = CLS_N32;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN, E>::T;
  const ModConst m = mods.m[mi];
  const u64* key = jb.key;
  const int tid = opaque_tid();
  const int wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;  // first thread of the wave
  const int i0 = lds_idx(tid);
  u64 acc0[E], acc1[E];
#pragma unroll
  for (int r = 0; r < E; ++r) acc0[r] = acc1[r] = 0;
  for (int j = j0; j < j1; ++j) {
    const u32* kb = reinterpret_cast<const u32*>(key + (((size_t)j * 2 + 0) * (big_l + 1) + mi) * N);
    const u32* ka = reinterpret_cast<const u32*>(key + (((size_t)j * 2 + 1) * (big_l + 1) + mi) * N);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      copy_to_lds(kb + tid + r * T, S + r * T + wave0);
      copy_to_lds(ka + tid + r * T, S + N + r * T + wave0);
    }
    __builtin_amdgcn_sched_barrier(0);  // the copies are issued before the digit's loads
    if (j == t) {
      // the digit reduced mod its own prime is the (permuted) input limb itself
      load_limb_perm<LOGN, CLS, E, true>(lds, jb.d + (size_t)j * N, jb.ginv, (jb.flags & JOB_IN_PACKED) != 0);
      lds_barrier();
    } else {
      lift_limb<LOGN, CLS, E>(lds, dcoef + (b * lmax + j) * N, mods.m[j].q, m, tid);
      fwd_lds<LOGN, CLS, E>(lds, tb, mi, m);
    }
    wait_vm();
    if (j1 - j0 <= 8) {
      // transform outputs (< 4q) brought below 2q only: each product is below
      // 2^61, so the 64-bit sums of up to 8 digits cannot overflow
      const u32 q2 = 2u * (u32)m.q;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const u32 v = lds_getw_at<CLS>(lds, lds_step(i0, r, T));
        const u32 dv = min(v, v - q2);
        acc0[r] += (u64)dv * S[r * T + tid];
        acc1[r] += (u64)dv * S[N + r * T + tid];
      }
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const u32 dv = (u32)to_canon<CLS>(lds_getw_at<CLS>(lds, lds_step(i0, r, T)), m);
        acc0[r] += (u64)dv * S[r * T + tid];
        acc1[r] += (u64)dv * S[N + r * T + tid];
      }
    }
    lds_barrier();  // the copies of the next digit overwrite S
  }
  if (rc_p) {
    p_limb_to_coeffs<LOGN, CLS, E>(lds, acc0, rc_p, mi, m, tb);
    p_limb_to_coeffs<LOGN, CLS, E>(lds, acc1, rc_p + N, mi, m, tb);
    return;
  }
  const bool lazy = mi != big_l;  // ciphertext-prime rows in [0, 2q) (reduce64_lazy32)
  u64* u0 = u + ((b * 2 + 0) * urows + row) * N;
  u64* u1 = u + ((b * 2 + 1) * urows + row) * N;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = (int)threadIdx.x + r * T;
    reinterpret_cast<u32*>(u0)[i] = lazy ? reduce64_lazy32(acc0[r], m) : (u32)reduce64(acc0[r], m);
    reinterpret_cast<u32*>(u1)[i] = lazy ? reduce64_lazy32(acc1[r], m) : (u32)reduce64(acc1[r], m);
  }
}

// Target x of workgroup `sub` of job jb in the ModUp grid: ciphertext prime
// x (x < lmax) over all digits, or group x - lmax of P's digits, whose
// partial goes to u row x.  False: the workgroup has nothing to do.
struct ModupTarget {
  int t, mi, j0, j1, row;
};
// The P groups come first in a job's run of workgroups (sub < pg): a P
// workgroup is the longest of its job (costlier width class, and with one
// group also the INTT of the P limb), so it starts before the short ones.
__device__ __forceinline__ bool modup_target(const KsJob& jb, int sub, int lmax, int pg, int big_l, ModupTarget& o) {
  const int level = jb.level;
  const int x = sub < pg ? lmax + sub : sub - pg;
  if (x < lmax) {
    if (x >= level) return false;
    o.t = o.mi = o.row = x;
    o.j0 = 0;
    o.j1 = level;
  } else {
    const int g = pgroup_size(level, pg);
    o.j0 = (x - lmax) * g;
    if (o.j0 >= level) return false;
    o.j1 = min(o.j0 + g, level);
    o.t = -1;
    o.mi = big_l;
    o.row = x;
  }
  return true;
}

// grid xcd_grid(Lmax + pg, count): workgroup (job b, x), x < Lmax is
// ciphertext prime x, x = Lmax + k is group k of P's digits.  Each width class is its
// own kernel (so each body gets a register allocation of its own); blocks of
// the other classes, primes above a job's level and empty P groups exit at
// once.  Narrow targets of rings up to 2^STAGE_MAX_LOGN take the staged body.
template <int LOGN, int CLS>
__global__ void __launch_bounds__(modup_threads<LOGN>())
k_ks_modup_ip(const KsJob* __restrict__ jobs, int count, const u64* __restrict__ dcoef, u64* __restrict__ u,
              u64* __restrict__ rc, int lmax, int pg, int big_l, Mods mods, Tables tb) {
  constexpr int EM = modup_e<LOGN>();
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const XcdSlot sl = xcd_slot(lmax + pg);
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const KsJob jb = jobs[b];
  if (jb.key == nullptr) return;
  ModupTarget o;
  if (!modup_target(jb, sl.sub, lmax, pg, big_l, o)) return;
  // with one P group (rc given) its workgroup also finishes the P limb
  u64* rc_p = (rc != nullptr && o.t < 0) ? rc + b * 2 * ((size_t)1 << LOGN) : nullptr;
  if ((int)mods.m[o.mi].cls != CLS) return;
  if constexpr (CLS == CLS_N32 && LOGN <= STAGE_MAX_LOGN) {
    __shared__ __align__(16) u32 S[stage_words<LOGN>()];
    modup_ip_narrow_staged<LOGN, EM>(lds, S, dcoef, jb, b, u, rc_p, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1,
                                     o.row, mods, tb);
  } else {
    modup_ip_body<LOGN, CLS, EM>(lds, dcoef, jb, b, u, rc_p, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1, o.row,
                                 mods, tb);
  }
}

// The same for a ring whose primes span two width classes A and B: one
// launch in which each workgroup runs the body of its target's class,
// instead of one kernel per class on two streams joined by events.
template <int LOGN, int CA, int CB>
__global__ void __launch_bounds__(modup_threads<LOGN>())
k_ks_modup_ip2(const KsJob* __restrict__ jobs, int count, const u64* __restrict__ dcoef, u64* __restrict__ u,
               u64* __restrict__ rc, int lmax, int pg, int big_l, Mods mods, Tables tb) {
  constexpr int EM = modup_e<LOGN>();
  const XcdSlot sl = xcd_slot(lmax + pg);
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const KsJob jb = jobs[b];
  if (jb.key == nullptr) return;
  ModupTarget o;
  if (!modup_target(jb, sl.sub, lmax, pg, big_l, o)) return;
  // with one P group (rc given) its workgroup also finishes the P limb
  u64* rc_p = (rc != nullptr && o.t < 0) ? rc + b * 2 * ((size_t)1 << LOGN) : nullptr;
  const bool is_a = (int)mods.m[o.mi].cls == CA;
  if constexpr (CA == CLS_N32 && LOGN <= STAGE_MAX_LOGN) {
    // narrow targets: transform buffer lds + staging S; class-B targets use
    // S as their transform buffer
    __shared__ u64 lds[lds_words<LOGN, CA>()];
    __shared__ __align__(16) u32 S[stage_words<LOGN>()];
    if (is_a)
      modup_ip_narrow_staged<LOGN, EM>(lds, S, dcoef, jb, b, u, rc_p, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1,
                                       o.row, mods, tb);
    else
      modup_ip_body<LOGN, CB, EM>(reinterpret_cast<u64*>(S), dcoef, jb, b, u, rc_p, lmax, lmax + pg, big_l, o.t,
                                  o.mi, o.j0, o.j1, o.row, mods, tb);
  } else {
    constexpr int LW = lds_words<LOGN, CA>() > lds_words<LOGN, CB>() ? lds_words<LOGN, CA>() : lds_words<LOGN, CB>();
    __shared__ u64 lds[LW];
    if (is_a)
      modup_ip_body<LOGN, CA, EM>(lds, dcoef, jb, b, u, rc_p, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1, o.row,
                                  mods, tb);
    else
      modup_ip_body<LOGN, CB, EM>(lds, dcoef, jb, b, u, rc_p, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1, o.row,
                                  mods, tb);
  }
}

// ---------------------------------------------------------------------------
// Half-ring ModUp for the largest rings.  A workgroup that holds a whole
// N = 2^14 limb has N / 16 = 1024 threads and so at most 128 registers each,
// too few for the two 16-entry accumulators beside a radix-16 pass (it
// spills).  Here a target's work is split over two workgroups, one per half
// of the NTT-domain output: the transform's first stage pairs entries i and
// i + N/2 with the same twiddle, and after it each half is an independent
// N/2-point transform whose output lands in that half (bit-reversed order
// keeps blocks in place).  So the workgroup of half h reads both halves of
// the coefficient-domain digit, forms its half of the first stage while it
// lifts (x + w y for h = 0, x - w y for h = 1), runs the N/2-point transform
// with the half's twiddles (tw_half_of) at 8 entries per thread, and keeps
// 8 accumulators per output polynomial.  The cost: each digit is read twice
// (the second read from L2) and each first-stage product computed twice.

// Centred lift of one source residue v (mod qs, odd) into the word of the
// target class (as lift_limb, per value).
template <int CLS>
__device__ __forceinline__ word_t<CLS> lift_word(u64 v, u64 qs, const ModConst& m) {
  const u64 half = (qs - 1) / 2;
  if constexpr (CLS == CLS_F64) {
    if (qs < ((u64)1 << 43)) {
      const double x = f64_from_u64(v);
      return v > half ? x - f64_from_u64(qs) : x;
    }
    return f64_from_u64(lift_centered(v, qs, m));
  } else if constexpr (CLS == CLS_N32) {
    if (qs < 2 * m.q) return (u32)(v > half ? v + (m.q - qs) : v);
    return (u32)lift_centered(v, qs, m);
  } else {
    return lift_centered(v, qs, m);
  }
}

// Half h of the first forward stage of the lifted digit into LDS: local
// entry k < N/2 gets x_k + w x_{k+N/2} (h = 0) or x_k - w x_{k+N/2} (h = 1),
// x the centred lift of the source row (packed 32-bit words when qs is
// narrow) and w = tw[1].  All loads are issued before any is used.
template <int LOGN, int CLS, int E>
__device__ __forceinline__ void lift_half(u64* lds, const u64* __restrict__ src, u64 qs, const ModConst& m, int h,
                                          word_t<CLS> w1, word_t<CLS> w1sh, int tid) {
  typedef word_t<CLS> W;
  typedef Arith<CLS> A;
  constexpr int NH = 1 << (LOGN - 1);
  constexpr int T = NH / E;
  const MV<CLS> q = mview<CLS>(m);
  const int i0 = lds_idx(tid);
  u64 x[E], y[E];
  if (qs < NARROW_LIMIT) {
    const u32* s32 = reinterpret_cast<const u32*>(src);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      x[r] = s32[tid + r * T];
      y[r] = s32[NH + tid + r * T];
    }
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      x[r] = src[tid + r * T];
      y[r] = src[NH + tid + r * T];
    }
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const W a = A::fwd_x(lift_word<CLS>(x[r], qs, m), q);
    const W b = A::mulc(lift_word<CLS>(y[r], qs, m), w1, w1sh, q);
    lds_putw_at<CLS>(lds, lds_step(i0, r, T), h ? A::sub(a, b, q) : A::add(a, b, q));
  }
}

// NTT-domain limb src through the Galois permutation, half h into LDS:
// lds[k] = src[galois_src(h N/2 + k, g)] for k < N/2.  The permutation maps a
// half onto one half (the half of 2 brv(i) + 1 mod 4, which a factor g = 1
// mod 4 keeps and g = 3 mod 4 swaps), so the workgroup reads that source
// half coalesced and scatters it into LDS.
template <int LOGN, int CLS, int E>
__device__ __forceinline__ void load_half_perm(u64* lds, const u64* __restrict__ src, u32 ginv, bool packed, int h) {
  constexpr int NH = 1 << (LOGN - 1);
  constexpr int T = NH / E;
  const int sh = h ^ (int)((ginv >> 1) & 1u);  // source half
  const int tid = opaque_tid();  // indices formed at each call, not held across the caller's digit loop
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int idx = sh * NH + tid + r * T;
    const u64 v = ld_res(src, idx, packed);
    const int dst = ((ginv == 1u) ? idx : galois_src<LOGN>(idx, ginv)) - h * NH;
    lds_put<CLS>(lds, dst, v);
  }
}

// ModUp + inner product of half h of one target (as modup_ip_body, which it
// mirrors entry for entry): output entries h N/2 + k, k < N/2, of u row `row`.
template <int LOGN, int CLS>
__device__ __forceinline__ void modup_ip_half_body(u64* lds, const u64* __restrict__ dcoef, const KsJob& jb, size_t b,
                                                   u64* __restrict__ u, int lmax, int urows, int big_l, int t, int mi,
                                                   int j0, int j1, int row, int h, const Mods& mods,
                                                   const Tables& tb) {
  typedef std::conditional_t<CLS == CLS_N32, u64, word_t<CLS>> A;
  constexpr int E = 8;
  constexpr int N = 1 << LOGN;
  constexpr int NH = N / 2;
  constexpr int T = NH / E;
  const ModConst m = mods.m[mi];
  const u64* key = jb.key;
  const Tw<CLS> tw0 = tw_of<LOGN, CLS>(tb, mi, 0);
  const word_t<CLS> w1 = tw0.w[1];
  const word_t<CLS> w1sh = CLS == CLS_F64 ? word_t<CLS>(0) : tw0.sh[1];
  const Tw<CLS> twh = tw_half_of<LOGN, CLS>(tb, mi, h);
  const size_t hoff = (size_t)h * NH;
  A acc0[E], acc1[E];
#pragma unroll
  for (int r = 0; r < E; ++r) acc0[r] = acc1[r] = 0;
  for (int j = j0; j < j1; ++j) {
    if (j == t) {
      load_half_perm<LOGN, CLS, E>(lds, jb.d + (size_t)j * N, jb.ginv, (jb.flags & JOB_IN_PACKED) != 0, h);
      __syncthreads();
    } else {
      lift_half<LOGN, CLS, E>(lds, dcoef + (b * lmax + j) * N, mods.m[j].q, m, h, w1, w1sh, opaque_tid());
      ntt_fwd_lds<LOGN - 1, CLS, E>(lds, twh, mview<CLS>(m), opaque_tid());
    }
    const u64* kb = key + (((size_t)j * 2 + 0) * (big_l + 1) + mi) * N + hoff;
    const u64* ka = key + (((size_t)j * 2 + 1) * (big_l + 1) + mi) * N + hoff;
    const int tid = opaque_tid();
    const int i0 = lds_idx(tid);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = tid + r * T;
      const int li = lds_step(i0, r, T);
      if constexpr (CLS == CLS_N32) {
        const u32 dv = (u32)to_canon<CLS>(lds_getw_at<CLS>(lds, li), m);
        // narrow key rows are packed 32-bit residues (the half starts at word N/2)
        acc0[r] += (u64)dv * reinterpret_cast<const u32*>(kb - hoff)[hoff + i];
        acc1[r] += (u64)dv * reinterpret_cast<const u32*>(ka - hoff)[hoff + i];
      } else if constexpr (CLS == CLS_F64) {
        const double dv = lds_getw_at<CLS>(lds, li);
        acc0[r] += f64_mulmod(dv, f64_from_u64(kb[i]), m.qd, m.qinv);
        acc1[r] += f64_mulmod(dv, f64_from_u64(ka[i]), m.qd, m.qinv);
      } else {
        const u64 dv = lds_getw_at<CLS>(lds, li);
        acc0[r] = add_mod(acc0[r], mul_mod_t<false>(dv, kb[i], m), m.q);
        acc1[r] = add_mod(acc1[r], mul_mod_t<false>(dv, ka[i], m), m.q);
      }
    }
    __syncthreads();
  }
  const bool lazy = mi != big_l;  // ciphertext-prime rows in [0, 2q) (reduce64_lazy32)
  u64* u0 = u + ((b * 2 + 0) * urows + row) * N;
  u64* u1 = u + ((b * 2 + 1) * urows + row) * N;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = (int)hoff + (int)threadIdx.x + r * T;
    if constexpr (CLS == CLS_N32) {  // packed row
      reinterpret_cast<u32*>(u0)[i] = lazy ? reduce64_lazy32(acc0[r], m) : (u32)reduce64(acc0[r], m);
      reinterpret_cast<u32*>(u1)[i] = lazy ? reduce64_lazy32(acc1[r], m) : (u32)reduce64(acc1[r], m);
    } else if constexpr (CLS == CLS_F64) {
      u0[i] = to_canon<CLS>(acc0[r], m);
      u1[i] = to_canon<CLS>(acc1[r], m);
    } else {
      u0[i] = acc0[r];
      u1[i] = acc1[r];
    }
  }
}

// Narrow targets of the half-ring ModUp (as modup_ip_half_body), with the key
// half-rows of digit j (both components, packed 32-bit) copied
// asynchronously into the staging array S = [key b | key a] before the
// digit is loaded, as modup_ip_narrow_staged does for a whole limb: both
// loads are in flight together and the products read the key from LDS.
template <int LOGN>
__device__ __forceinline__ void modup_ip_half_narrow_staged(u64* lds, u32* S, const u64* __restrict__ dcoef,
                                                            const KsJob& jb, size_t b, u64* __restrict__ u,
                                                            int lmax, int urows, int big_l, int t, int mi, int j0,
                                                            int j1, int row, int h, const Mods& mods,
                                                            const Tables& tb) {
  constexpr int CLS = CLS_N32;
  constexpr int E = 8;
  constexpr int N = 1 << LOGN;
  constexpr int NH = N / 2;
  constexpr int T = NH / E;
  const ModConst m = mods.m[mi];
  const u64* key = jb.key;
  const Tw<CLS> tw0 = tw_of<LOGN, CLS>(tb, mi, 0);
  const u32 w1 = tw0.w[1];
  const u32 w1sh = tw0.sh[1];
  const Tw<CLS> twh = tw_half_of<LOGN, CLS>(tb, mi, h);
  const int hoff = h * NH;
  const int tid = opaque_tid();
  const int wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;
  const int i0 = lds_idx(tid);
  u64 acc0[E], acc1[E];
#pragma unroll
  for (int r = 0; r < E; ++r) acc0[r] = acc1[r] = 0;
  for (int j = j0; j < j1; ++j) {
    const u32* kb = reinterpret_cast<const u32*>(key + (((size_t)j * 2 + 0) * (big_l + 1) + mi) * N) + hoff;
    const u32* ka = reinterpret_cast<const u32*>(key + (((size_t)j * 2 + 1) * (big_l + 1) + mi) * N) + hoff;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      copy_to_lds(kb + tid + r * T, S + r * T + wave0);
      copy_to_lds(ka + tid + r * T, S + NH + r * T + wave0);
    }
    __builtin_amdgcn_sched_barrier(0);  // the copies are issued before the digit's loads
    if (j == t) {
      load_half_perm<LOGN, CLS, E>(lds, jb.d + (size_t)j * N, jb.ginv, (jb.flags & JOB_IN_PACKED) != 0, h);
      lds_barrier();
    } else {
      lift_half<LOGN, CLS, E>(lds, dcoef + (b * lmax + j) * N, mods.m[j].q, m, h, w1, w1sh, tid);
      ntt_fwd_lds<LOGN - 1, CLS, E>(lds, twh, mview<CLS>(m), opaque_tid());
    }
    wait_vm();
    if (j1 - j0 <= 8) {
      // transform outputs (< 4q) brought below 2q only: each product is below
      // 2^61, so the 64-bit sums of up to 8 digits cannot overflow
      const u32 q2 = 2u * (u32)m.q;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const u32 v = lds_getw_at<CLS>(lds, lds_step(i0, r, T));
        const u32 dv = min(v, v - q2);
        acc0[r] += (u64)dv * S[r * T + tid];
        acc1[r] += (u64)dv * S[NH + r * T + tid];
      }
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const u32 dv = (u32)to_canon<CLS>(lds_getw_at<CLS>(lds, lds_step(i0, r, T)), m);
        acc0[r] += (u64)dv * S[r * T + tid];
        acc1[r] += (u64)dv * S[NH + r * T + tid];
      }
    }
    lds_barrier();  // the copies of the next digit overwrite S
  }
  const bool lazy = mi != big_l;  // ciphertext-prime rows in [0, 2q) (reduce64_lazy32)
  u64* u0 = u + ((b * 2 + 0) * urows + row) * N;
  u64* u1 = u + ((b * 2 + 1) * urows + row) * N;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = hoff + (int)threadIdx.x + r * T;
    reinterpret_cast<u32*>(u0)[i] = lazy ? reduce64_lazy32(acc0[r], m) : (u32)reduce64(acc0[r], m);
    reinterpret_cast<u32*>(u1)[i] = lazy ? reduce64_lazy32(acc1[r], m) : (u32)reduce64(acc1[r], m);
  }
}

// Staging array of the half-ring ModUp in 32-bit words: the key half-rows of
// one digit (2 N/2), or the half-ring transform buffer of the other class.
template <int LOGN>
constexpr int stage_words_half() {
  return (2 << (LOGN - 1)) > 2 * lds_words<LOGN - 1, CLS_U64>() ? (2 << (LOGN - 1))
                                                                   : 2 * lds_words<LOGN - 1, CLS_U64>();
}

// Rings from 2^HALF_MODUP_MIN_LOGN up run ModUp in halves unless the
// context's "modup_halves" knob says otherwise; smaller rings (from 2^11)
// run it in halves when the knob asks for it.
constexpr int HALF_MODUP_MIN_LOGN = 13;
constexpr int HALF_MODUP_ANY_LOGN = 11;
template <int LOGN>
constexpr int modup_half_threads() {
  return (1 << (LOGN - 1)) / 8;
}

// grid xcd_grid(2 (Lmax + pg), count): workgroup (job b, 2 x + h): target x
// as in k_ks_modup_ip2 (P groups first), half h.  Each workgroup runs the
// body of its target's class (CA or CB; CA == CB for a one-class ring).  The
// P limb's coefficient-domain copy is always left to k_intt_last.
template <int LOGN, int CA, int CB>
__global__ void __launch_bounds__(modup_half_threads<LOGN>())
k_ks_modup_half(const KsJob* __restrict__ jobs, int count, const u64* __restrict__ dcoef, u64* __restrict__ u,
                int lmax, int pg, int big_l, Mods mods, Tables tb) {
  const XcdSlot sl = xcd_slot(2 * (lmax + pg));
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const KsJob jb = jobs[b];
  if (jb.key == nullptr) return;
  ModupTarget o;
  if (!modup_target(jb, sl.sub >> 1, lmax, pg, big_l, o)) return;
  const int h = sl.sub & 1;
  const int cls = (int)mods.m[o.mi].cls;
  if constexpr (CA == CLS_N32) {
    // narrow targets: transform buffer lds + key staging S; targets of the
    // other class use S as their transform buffer
    __shared__ u64 lds[lds_words<LOGN - 1, CLS_N32>()];
    __shared__ __align__(16) u32 S[stage_words_half<LOGN>()];
    if (cls == CA)
      modup_ip_half_narrow_staged<LOGN>(lds, S, dcoef, jb, b, u, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1,
                                        o.row, h, mods, tb);
    else if constexpr (CB != CA)
      if (cls == CB)
        modup_ip_half_body<LOGN, CB>(reinterpret_cast<u64*>(S), dcoef, jb, b, u, lmax, lmax + pg, big_l, o.t, o.mi,
                                     o.j0, o.j1, o.row, h, mods, tb);
  } else {
    constexpr int LW = lds_words<LOGN - 1, CA>() > lds_words<LOGN - 1, CB>() ? lds_words<LOGN - 1, CA>()
                                                                              : lds_words<LOGN - 1, CB>();
    __shared__ u64 lds[LW];
    if (cls == CA)
      modup_ip_half_body<LOGN, CA>(lds, dcoef, jb, b, u, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1, o.row, h,
                                   mods, tb);
    else if constexpr (CB != CA)
      if (cls == CB)
        modup_ip_half_body<LOGN, CB>(lds, dcoef, jb, b, u, lmax, lmax + pg, big_l, o.t, o.mi, o.j0, o.j1, o.row, h,
                                     mods, tb);
  }
}

enum { MODE_P = 0, MODE_LAST = 1 };

// Coefficient-domain copy of the P limb of u: the sum of its group partials
// (rows lmax .. lmax + groups - 1, each canonical mod P), INTT, N^-1.
template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void intt_p_body(u64* lds, const u64* __restrict__ urow, int groups, u64* out, int mi,
                                            const ModConst& m, const Tables& tb) {
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN, E>::T;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = (int)threadIdx.x + r * T;
    u64 v;
    if constexpr (CLS == CLS_N32) {  // packed rows
      v = reinterpret_cast<const u32*>(urow)[i];
      for (int k = 1; k < groups; ++k) v = add_mod(v, reinterpret_cast<const u32*>(urow + (size_t)k * N)[i], m.q);
    } else {
      v = urow[i];
      for (int k = 1; k < groups; ++k) v = add_mod(v, urow[(size_t)k * N + i], m.q);
    }
    lds_put<CLS>(lds, i, v);
  }
  inv_lds<LOGN, CLS, E>(lds, tb, mi, m);
  store_limb<LOGN, CLS, true, E>(out, lds, m, true);
}

// The P INTT of k_intt_last (MODE_P) with 8 entries per thread: at N <= 8192
// an f64 or wide P limb takes 64-bit LDS words, two workgroups per CU, so
// twice the threads per workgroup double the waves that hide the passes'
// latency.  grid xcd_grid(2, count), N / 8 threads.
template <int LOGN>
constexpr int p8_threads() {
  return NttGeom<LOGN, 8>::T;
}
template <int LOGN, int CLS>
__global__ void __launch_bounds__(p8_threads<LOGN>())
k_intt_p8(const KsJob* __restrict__ jobs, int count, const u64* __restrict__ u, int lmax, int pg, int big_l,
          u64* __restrict__ rcoef, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const XcdSlot sl = xcd_slot(2);
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const int comp = sl.sub;
  const KsJob jb = jobs[b];
  if (jb.key == nullptr) return;
  const ModConst m = mods.m[big_l];
  if ((int)m.cls != CLS) return;
  intt_p_body<LOGN, CLS, 8>(lds, u + ((b * 2 + comp) * (lmax + pg) + lmax) * N, pgroup_count(jb.level, pg),
                            rcoef + (2 * b + comp) * N, big_l, m, tb);
}

// INTT of the limb that is divided out: for polynomial p = 2 b + comp,
//   MODE_P:    the P limb of u, i.e. the sum of its group partials (ModDown
//              after a key switch; u rows per polynomial lmax + pg);
//   MODE_LAST: the last limb of the ciphertext jobs[b].d (rescale).
template <int LOGN, int MODE, int CLS, bool PIN = false>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_intt_last(const KsJob* __restrict__ jobs, int count, const u64* __restrict__ u, int lmax, int pg, int big_l,
            u64* __restrict__ rcoef, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const XcdSlot sl = xcd_slot(2);  // grid xcd_grid(2, count): workgroup (job b, polynomial comp)
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const int comp = sl.sub;
  const size_t p = 2 * b + comp;
  const KsJob jb = jobs[b];
  u64* out = rcoef + p * N;
  if (MODE == MODE_P) {
    if (jb.key == nullptr) return;
    const u64* s = u + ((b * 2 + comp) * (lmax + pg) + lmax) * N;
    const int groups = pgroup_count(jb.level, pg);
    const ModConst m = mods.m[big_l];
    if ((int)m.cls != CLS) return;
    intt_p_body<LOGN, CLS>(lds, s, groups, out, big_l, m, tb);
  } else {
    const u64* s = jb.d + ((size_t)comp * jb.level + jb.level - 1) * N;
    const int mi = jb.level - 1;
    const ModConst m = mods.m[mi];
    if ((int)m.cls != CLS) return;
    digits_body<LOGN, CLS>(lds, s, 1u, out, mi, m, tb, PIN);
  }
}

// Largest ring whose ModDown also writes the next step's digits: at
// N = 16384 the transform in the epilogue would make the kernel spill (its
// 1024 threads get 128 registers each), so the digit kernel runs instead.
constexpr int NEXT_DIGITS_MAX_LOGN = 13;

// The next rotate-and-add step's digits, produced by this step's ModDown:
// dcoef rows [count][lmax][N] of the next step, written for limb t by the
// workgroup that computes limb t of the new c1, through the next step's
// Galois element (ginv = its inverse).  dcoef == nullptr: none.
struct NextDigits {
  u64* dcoef;
  u32 ginv;
  int lmax;
};

// Coefficient-domain digit of limb t from an NTT-domain limb the caller has
// put into LDS through the Galois permutation: INTT, N^-1, packed store
// (what k_ks_digits computes from memory).
template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void digits_from_lds(u64* lds, u64* out, int t, const ModConst& m, const Tables& tb) {
  inv_lds<LOGN, CLS, E>(lds, tb, t, m);  // begins with a barrier
  store_limb<LOGN, CLS, true, E>(out, lds, m, true);
}

// Entries per thread of the ModDown / rescale kernel: 16 (with 8, as ModUp
// uses, its 1024-thread workgroups measured slower: one workgroup per CU at
// the same four waves per SIMD).
template <int LOGN>
constexpr int drop_e() {
  return 16;
}
template <int LOGN>
constexpr int drop_threads() {
  return NttGeom<LOGN, drop_e<LOGN>()>::T;
}

enum { EPI_STORE = 0, EPI_ROT = 1, EPI_ROTSUM = 2, EPI_RELIN = 3 };


// Drop the last limb, for polynomial p = 2 b + comp (blockIdx.y) and kept
// prime t (blockIdx.x):  val = (src_t - NTT(lift(rc_p))) * div^-1 mod q_t,
// with (src, div) = (u row t, P) in MODE_P and (d limb t, q_{level-1}) in
// MODE_LAST, followed by the epilogue into jobs[b].out:
//   EPI_STORE   out = val
//   EPI_ROT     out = (sigma_g(c0) + val, val)        (identity job: out = c)
//   EPI_ROTSUM  out = c + (sigma_g(c0) + val, val)    (identity job: out = 2c)
//   EPI_RELIN   out = (d0 + val, d1 + val), (d0, d1) = c
// inv_tab[div][t] holds q_div^-1 mod q_t (div = big_l for P) and its Shoup
// companion at inv_tab[HE_MAXM * HE_MAXM + ...].  u has `urows` rows per
// polynomial.
template <int LOGN, int MODE, int EPI, int CLS, int PK = 0, int E = 16>
__device__ __forceinline__ void drop_last_body(u64* lds, const KsJob& jb, size_t b, int comp, int t,
                                               const u64* __restrict__ u, int urows, int big_l,
                                               const u64* __restrict__ rcoef, const u64* __restrict__ inv_tab,
                                               const Mods& mods, const Tables& tb, const NextDigits& nd) {
  constexpr bool NW = CLS == CLS_N32;  // canonical values in 32-bit words
  typedef std::conditional_t<NW, u32, u64> V;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN, E>::T;
  const int level = jb.level;
  const int keep = (MODE == MODE_P) ? level : level - 1;
  const int div_mi = (MODE == MODE_P) ? big_l : level - 1;
  const ModConst m = mods.m[t];
  u64* o = jb.out + ((size_t)comp * keep + t) * N;
  constexpr bool in_p = (PK & JOB_IN_PACKED) != 0;
  constexpr bool out_p = (PK & JOB_OUT_PACKED) != 0;
  if (MODE == MODE_P && jb.key == nullptr) {  // identity job
    const u64* cs = jb.c + ((size_t)comp * level + t) * N;
    if constexpr (in_p != out_p) {
      // in place with a change of format, the whole row is read before any of it is written
      u64 xv[E];
#pragma unroll
      for (int r = 0; r < E; ++r) {
        xv[r] = ld_res(cs, (int)threadIdx.x + r * T, in_p);
        if constexpr (EPI == EPI_ROTSUM) xv[r] = addm<NW>(xv[r], xv[r], m.q);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) st_res(o, (int)threadIdx.x + r * T, xv[r], out_p);
    } else {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int i = (int)threadIdx.x + r * T;
        u64 x = ld_res(cs, i, in_p);
        if constexpr (EPI == EPI_ROTSUM) x = addm<NW>(x, x, m.q);
        st_res(o, i, x, out_p);
      }
    }
    return;
  }
  lift_limb<LOGN, CLS, E>(lds, rcoef + (b * 2 + comp) * N, mods.m[div_mi].q, m, (int)threadIdx.x);
  fwd_lds<LOGN, CLS, E>(lds, tb, t, m);
  const u64* s = (MODE == MODE_P) ? u + ((b * 2 + comp) * urows + t) * N
                                  : jb.d + ((size_t)comp * level + t) * N;
  const u64 iv = inv_tab[div_mi * HE_MAXM + t];
  const u64 ivs = inv_tab[HE_MAXM * HE_MAXM + div_mi * HE_MAXM + t];
  V val[E];
  const int i0 = lds_idx((int)threadIdx.x);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = (int)threadIdx.x + r * T;
    const int li = lds_step(i0, r, T);
    // u rows of narrow primes are packed; ciphertext limbs as the job says
    const u64 sv = (MODE == MODE_P) ? (NW ? (u64)reinterpret_cast<const u32*>(s)[i] : s[i]) : ld_res(s, i, in_p);
    if constexpr (CLS == CLS_F64) {
      const double dlt = f64_from_u64(sv) - lds_getw_at<CLS>(lds, li);
      val[r] = to_canon<CLS>(f64_mulmod(dlt, f64_from_u64(iv), m.qd, m.qinv), m);
    } else {
      val[r] = (V)shoupm<NW>(subm<NW>(sv, to_canon<CLS>(lds_getw_at<CLS>(lds, li), m), m.q), iv, ivs, m.q);
    }
  }
  if constexpr (EPI == EPI_STORE) {
#pragma unroll
    for (int r = 0; r < E; ++r) st_res(o, (int)threadIdx.x + r * T, val[r], out_p);
  } else if constexpr (EPI == EPI_RELIN) {
    const u64* dd = jb.c + ((size_t)comp * level + t) * N;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = (int)threadIdx.x + r * T;
      st_res(o, i, addm<NW>(ld_res(dd, i, in_p), val[r], m.q), out_p);
    }
  } else {  // EPI_ROT / EPI_ROTSUM
    const u64* cs = jb.c + ((size_t)comp * level + t) * N;
    if (comp == 0) {
      // sigma_g(c0) through LDS, in canonical 32-bit (narrow) or 64-bit words
      constexpr int PC = NW ? CLS_N32 : CLS_U64;
      __syncthreads();  // everyone is done reading the lifted limb
      V own[E];
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int idx = (int)threadIdx.x + r * T;
        const u64 v = ld_res(cs, idx, in_p);
        own[r] = (V)v;
        lds_put<PC>(lds, galois_src<LOGN>(idx, jb.ginv), v);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int i = (int)threadIdx.x + r * T;
        u64 x = addm<NW>((u64)lds_getw_at<PC>(lds, lds_step(i0, r, T)), val[r], m.q);  // sigma_g(c0) + u0
        if constexpr (EPI == EPI_ROTSUM) x = addm<NW>(x, own[r], m.q);
        st_res(o, i, x, out_p);
      }
    } else {
      if constexpr (EPI == EPI_ROTSUM) {
        V xs[E];
#pragma unroll
        for (int r = 0; r < E; ++r) xs[r] = (V)addm<NW>(ld_res(cs, (int)threadIdx.x + r * T, in_p), val[r], m.q);
        // in place with a change of format the whole row is read before any of it is written;
        // with the next step's digits the LDS buffer (read above) is free after the barrier
        if (in_p != out_p || nd.dcoef != nullptr) __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int idx = (int)threadIdx.x + r * T;
          st_res(o, idx, xs[r], out_p);
          if (nd.dcoef != nullptr) lds_put<CLS>(lds, nd.ginv == 1u ? idx : galois_src<LOGN>(idx, nd.ginv), (u64)xs[r]);
        }
        if constexpr (LOGN <= NEXT_DIGITS_MAX_LOGN) {
          if (nd.dcoef != nullptr) digits_from_lds<LOGN, CLS, E>(lds, nd.dcoef + (b * nd.lmax + t) * N, t, m, tb);
        }
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r) st_res(o, (int)threadIdx.x + r * T, val[r], out_p);
      }
    }
  }
}

// grid xcd_grid(2 Kmax, count), Kmax the largest number of kept limbs:
// workgroup (job b, polynomial comp, kept prime t).  nd: with EPI_ROTSUM,
// the c1 workgroups also write the next step's digits.
template <int LOGN, int MODE, int EPI, int CLS, int PK = 0>
__global__ void __launch_bounds__(drop_threads<LOGN>())
k_drop_last(const KsJob* __restrict__ jobs, int count, int kmax, const u64* __restrict__ u, int urows, int big_l,
            const u64* __restrict__ rcoef, const u64* __restrict__ inv_tab, Mods mods, Tables tb, NextDigits nd) {
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const XcdSlot sl = xcd_slot(2 * kmax);
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const int comp = sl.sub / kmax;
  const int t = sl.sub - comp * kmax;
  const KsJob jb = jobs[b];
  const int keep = (MODE == MODE_P) ? jb.level : jb.level - 1;
  if (t >= keep) return;
  if ((int)mods.m[t].cls != CLS) return;
  drop_last_body<LOGN, MODE, EPI, CLS, PK, drop_e<LOGN>()>(lds, jb, b, comp, t, u, urows, big_l, rcoef, inv_tab,
                                                          mods, tb, nd);
}

// ModDown (MODE_P) in halves: workgroup (job b, polynomial comp, kept prime
// t, half h) computes the entries h N/2 .. (h + 1) N/2 - 1 of the output
// limb exactly as drop_last_body does for the whole limb.  The lifted P
// limb's first forward stage is fused into the lift (lift_half) and the rest
// is an N/2-point transform with the half's twiddles, as in
// k_ks_modup_half; a rotation's sigma_g(c0) comes from one source half
// (load_half_perm).  Every Galois element here is a power of 5 (1 mod 4),
// which maps each half onto itself, so an in-place rotate-and-add reads and
// writes only its own half.  Unpacked ciphertexts, no next-step digits.  With
// 8 entries per thread a 16384-point ring gets 1024-thread workgroups with
// half the LDS of the whole-limb kernel: two per CU, twice its waves.
// grid xcd_grid(4 Kmax, count).
constexpr int HALF_MODDOWN_MIN_LOGN = 14;  // default: halves from N = 16384
template <int LOGN>
constexpr int drop_half_threads() {
  return (1 << (LOGN - 1)) / 8;
}
template <int LOGN, int EPI, int CLS>
__global__ void __launch_bounds__(drop_half_threads<LOGN>())
k_drop_half(const KsJob* __restrict__ jobs, int count, int kmax, const u64* __restrict__ u, int urows, int big_l,
            const u64* __restrict__ rcoef, const u64* __restrict__ inv_tab, Mods mods, Tables tb) {
  constexpr int E = 8;
  constexpr bool NW = CLS == CLS_N32;
  typedef std::conditional_t<NW, u32, u64> V;
  constexpr int N = 1 << LOGN;
  constexpr int NH = N / 2;
  constexpr int T = NH / E;
  constexpr int PC = NW ? CLS_N32 : CLS_U64;  // word of sigma_g(c0) in LDS
  __shared__ u64 lds[lds_words<LOGN - 1, CLS>()];
  const XcdSlot sl = xcd_slot(4 * kmax);
  if (sl.job >= count) return;
  const size_t b = sl.job;
  const int h = sl.sub & 1;
  const int comp = (sl.sub >> 1) / kmax;
  const int t = (sl.sub >> 1) - comp * kmax;
  const KsJob jb = jobs[b];
  const int level = jb.level;
  if (t >= level) return;
  const ModConst m = mods.m[t];
  if ((int)m.cls != CLS) return;
  const int hoff = h * NH;
  u64* o = jb.out + ((size_t)comp * level + t) * N;
  const u64* cs = jb.c + ((size_t)comp * level + t) * N;
  if (jb.key == nullptr) {  // identity job
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = hoff + (int)threadIdx.x + r * T;
      u64 x = cs[i];
      if constexpr (EPI == EPI_ROTSUM) x = addm<NW>(x, x, m.q);
      o[i] = x;
    }
    return;
  }
  const Tw<CLS> tw0 = tw_of<LOGN, CLS>(tb, t, 0);
  lift_half<LOGN, CLS, E>(lds, rcoef + (b * 2 + comp) * N, mods.m[big_l].q, m, h, tw0.w[1],
                          CLS == CLS_F64 ? word_t<CLS>(0) : tw0.sh[1], opaque_tid());
  ntt_fwd_lds<LOGN - 1, CLS, E>(lds, tw_half_of<LOGN, CLS>(tb, t, h), mview<CLS>(m), opaque_tid());
  const u64* s = u + ((b * 2 + comp) * urows + t) * N;
  const u64 iv = inv_tab[big_l * HE_MAXM + t];
  const u64 ivs = inv_tab[HE_MAXM * HE_MAXM + big_l * HE_MAXM + t];
  const int tid = opaque_tid();
  const int i0 = lds_idx(tid);
  V val[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = hoff + tid + r * T;
    const int li = lds_step(i0, r, T);
    const u64 sv = NW ? (u64)reinterpret_cast<const u32*>(s)[i] : s[i];  // narrow u rows are packed
    if constexpr (CLS == CLS_F64) {
      const double dlt = f64_from_u64(sv) - lds_getw_at<CLS>(lds, li);
      val[r] = to_canon<CLS>(f64_mulmod(dlt, f64_from_u64(iv), m.qd, m.qinv), m);
    } else {
      val[r] = (V)shoupm<NW>(subm<NW>(sv, to_canon<CLS>(lds_getw_at<CLS>(lds, li), m), m.q), iv, ivs, m.q);
    }
  }
  if constexpr (EPI == EPI_STORE) {
#pragma unroll
    for (int r = 0; r < E; ++r) o[hoff + tid + r * T] = val[r];
  } else if constexpr (EPI == EPI_RELIN) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = hoff + tid + r * T;
      o[i] = addm<NW>(cs[i], val[r], m.q);
    }
  } else if (comp == 0) {  // EPI_ROT / EPI_ROTSUM: sigma_g(c0) through LDS
    V own[E];
    if constexpr (EPI == EPI_ROTSUM) {
#pragma unroll
      for (int r = 0; r < E; ++r) own[r] = (V)cs[hoff + tid + r * T];
    }
    __syncthreads();  // everyone is done reading the transform
    load_half_perm<LOGN, PC, E>(lds, cs, jb.ginv, false, h);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      u64 x = addm<NW>((u64)lds_getw_at<PC>(lds, lds_step(i0, r, T)), val[r], m.q);  // sigma_g(c0) + u0
      if constexpr (EPI == EPI_ROTSUM) x = addm<NW>(x, own[r], m.q);
      o[hoff + tid + r * T] = x;
    }
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = hoff + tid + r * T;
      o[i] = (EPI == EPI_ROTSUM) ? addm<NW>(cs[i], val[r], m.q) : (u64)val[r];
    }
  }
}

// ---------------------------------------------------------------------------
// Hoisted rotations of one ciphertext.
// ModUp once: dhat[j][t] = NTT(lift(digit_j) mod m_t) for j < level,
// t <= level (t == level is P).  blockIdx.x = t, blockIdx.y = j.
template <int LOGN, int CLS>
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
  lift_limb<LOGN, CLS>(lds, dcoef + (size_t)j * N, mods.m[j].q, m, (int)threadIdx.x);
  fwd_lds<LOGN, CLS>(lds, tb, mi, m);
  store_limb<LOGN, CLS>(out, lds, m, false);
}

// grid dim3(level + 1, level, count): ciphertext z = blockIdx.z of a batch,
// its c1 at jobs[z].d, its digits at dcoef + z level N (k_ks_digits' layout)
// and its lifted digits stored at dhat + z level (level + 1) N.
template <int LOGN, int CLS>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_modup_store(const u64* __restrict__ dcoef, const KsJob* __restrict__ jobs, u64* __restrict__ dhat, int level,
              int big_l, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[lds_words<LOGN, CLS>()];
  const int mi = ((int)blockIdx.x < level) ? (int)blockIdx.x : big_l;
  if ((int)mods.m[mi].cls != CLS) return;
  const size_t z = blockIdx.z;
  modup_store_body<LOGN, CLS>(lds, dcoef + z * level * N, jobs[z].d, dhat + z * level * (level + 1) * N, level, big_l,
                              mods, tb);
}

// Inner product of the shared lifted digits, permuted per rotation, with
// that rotation's key: u[r][c][t][i] = sum_j dhat[j][t][src_{g_r}(i)] *
// key_r[j][c][m_t][i], with (key_r, g_r) from jobs[r]; with add_c0, row t <
// level of u_0 also gets P sigma_{g_r}(c0) (c0 from jobs[r].c).  The products are
// summed at full width (64-bit for narrow primes, 128-bit otherwise) and
// reduced once.  grid (N / 256, level + 1, m).  Batches of ciphertexts:
// job r belongs to ciphertext (job_base + r) / per_ct, whose lifted digits
// start dstride words after the previous one's.
template <int LOGN>
__global__ void k_ip_perm(const u64* __restrict__ dhat, const KsJob* __restrict__ jobs, u64* __restrict__ u,
                          int level, int big_l, Mods mods, int job_base, int per_ct, size_t dstride,
                          int add_c0) {
  constexpr int N = 1 << LOGN;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const size_t r = blockIdx.z;
  dhat += (size_t)((job_base + (int)r) / per_ct) * dstride;
  const int mi = (t < level) ? t : big_l;
  const ModConst m = mods.m[mi];
  const KsJob jb = jobs[r];
  const int src = galois_src<LOGN>(i, jb.g);
  const u64* key = jb.key;
  u64 s0, s1;
  if (m.narrow) {  // products < 2^60, at most 15 digits: one 64-bit sum each
    u64 a0 = 0, a1 = 0;
    for (int j = 0; j < level; ++j) {
      const u64 dv = dhat[((size_t)j * (level + 1) + t) * N + src];
      a0 += (u64)(u32)dv * reinterpret_cast<const u32*>(key + (((size_t)j * 2 + 0) * (big_l + 1) + mi) * N)[i];
      a1 += (u64)(u32)dv * reinterpret_cast<const u32*>(key + (((size_t)j * 2 + 1) * (big_l + 1) + mi) * N)[i];
    }
    s0 = reduce64(a0, m);
    s1 = reduce64(a1, m);
  } else {  // 128-bit sums of the full products, reduced once
    Acc128 a0{0, 0}, a1{0, 0};
    for (int j = 0; j < level; ++j) {
      const u64 dv = dhat[((size_t)j * (level + 1) + t) * N + src];
      mac128(a0, dv, key[(((size_t)j * 2 + 0) * (big_l + 1) + mi) * N + i]);
      mac128(a1, dv, key[(((size_t)j * 2 + 1) * (big_l + 1) + mi) * N + i]);
    }
    s0 = reduce128(a0, m);
    s1 = reduce128(a1, m);
  }
  if (add_c0 && t < level)  // + P sigma_g(c0): the rotation's c0 term, ahead of a deferred ModDown
    s0 = add_mod(s0, mul_mod(jb.c[(size_t)t * N + src], reduce64(mods.m[big_l].q, m), m), m.q);
  u64* u0 = u + ((r * 2 + 0) * (level + 1) + t) * N;
  u64* u1 = u + ((r * 2 + 1) * (level + 1) + t) * N;
  if (m.narrow) {  // packed rows
    reinterpret_cast<u32*>(u0)[i] = (u32)s0;
    reinterpret_cast<u32*>(u1)[i] = (u32)s1;
  } else {
    u0[i] = s0;
    u1[i] = s1;
  }
}

// Hoisted rotations with ModDown fused into the inner product, so the
// 2 (level + 1) inner-product rows of a rotation never go to memory.  The
// permutation sigma_g of the shared lifted digits is applied through LDS: a
// workgroup loads a digit row coalesced into LDS and each thread reads its
// entries at the permuted positions, instead of gathering them from memory.
//
// Lazy sums of products per width class: narrow 64-bit sums of products of
// canonical residues (< 2^60 each, at most 15 digits), f64 unreduced sums of
// centred products (below 8.2 q for at most 15 digits), wide residues.
template <int CLS>
struct IpAcc {
  typedef std::conditional_t<CLS == CLS_N32, u64, word_t<CLS>> A;
  static __device__ __forceinline__ void mac(A& acc, u64 dv, u64 k, const ModConst& m) {
    if constexpr (CLS == CLS_N32) acc += (u64)(u32)dv * (u32)k;
    else if constexpr (CLS == CLS_F64) acc += f64_mulmod(f64_from_u64(dv), f64_from_u64(k), m.qd, m.qinv);
    else acc = add_mod(acc, mul_mod_t<false>(dv, k, m), m.q);
  }
  static __device__ __forceinline__ u64 canon(A acc, const ModConst& m) {
    if constexpr (CLS == CLS_N32) return reduce64(acc, m);
    else if constexpr (CLS == CLS_F64) return to_canon<CLS>(acc, m);
    else return acc;
  }
};

// Key residue i of row (digit j, component comp, modulus mi): narrow rows are
// packed 32-bit words.
__device__ __forceinline__ u64 key_at(const u64* key, int big_l, int j, int comp, int mi, int i, int n, bool narrow) {
  const u64* row = key + (((size_t)j * 2 + comp) * (big_l + 1) + mi) * n;
  return narrow ? (u64) reinterpret_cast<const u32*>(row)[i] : row[i];
}

// The rotation's P row of the inner product, for one polynomial comp, into
// the coefficient domain: for each digit the P row of dhat is loaded into
// LDS and read through sigma_g; the sum goes back to LDS, INTT, N^-1,
// stored (packed when narrow) at rcoef.  grid xcd_grid(2, m): workgroup
// (rotation r, polynomial comp).
template <int LOGN, int CLS>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_hoist_p_intt(const u64* __restrict__ dhat, const KsJob* __restrict__ jobs, int m_rot, int level, int big_l,
               u64* __restrict__ rcoef, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN>::T;
  constexpr int E = 16;
  __shared__ u64 lds[NttGeom<LOGN>::LDS];  // 64-bit residues of the digit rows, then the transform
  const XcdSlot sl = xcd_slot(2);
  if (sl.job >= m_rot) return;
  const size_t r = sl.job;
  const int comp = sl.sub;
  const KsJob jb = jobs[r];
  const ModConst m = mods.m[big_l];
  if ((int)m.cls != CLS) return;
  typedef IpAcc<CLS> IP;
  typename IP::A acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0;
  for (int j = 0; j < level; ++j) {
    const u64* row = dhat + ((size_t)j * (level + 1) + level) * N;
#pragma unroll
    for (int e = 0; e < E; ++e) lds_putw<CLS_U64>(lds, (int)threadIdx.x + e * T, row[(int)threadIdx.x + e * T]);
    __syncthreads();
#pragma unroll 4
    for (int e = 0; e < E; ++e) {
      const int i = (int)threadIdx.x + e * T;
      const u64 dv = lds_getw<CLS_U64>(lds, galois_src<LOGN>(i, jb.g));
      IP::mac(acc[e], dv, key_at(jb.key, big_l, j, comp, big_l, i, N, m.narrow), m);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < E; ++e) lds_put<CLS>(lds, (int)threadIdx.x + e * T, IP::canon(acc[e], m));
  inv_lds<LOGN, CLS>(lds, tb, big_l, m);
  store_limb<LOGN, CLS, true>(rcoef + (r * 2 + comp) * N, lds, m, true);
}

// ModDown of the hoisted rotation into ciphertext prime t, half h of the
// NTT-domain output, polynomial comp: the inner product of the t rows with
// key component comp (digit half-rows through LDS and sigma_g, the key read
// coalesced) is kept in registers; then the P limb's coefficients (rcoef)
// are lifted to q_t with the transform's first stage fused (lift_half), the
// N/2-point transform runs, and out = (ip - that) P^-1 (+ sigma_g(c0) for
// c0).  grid xcd_grid(4 level, m): workgroup (rotation r, (comp level + t)
// 2 + h).
template <int LOGN, int CLS>
__global__ void __launch_bounds__(modup_half_threads<LOGN>())
k_hoist_drop(const u64* __restrict__ dhat, const KsJob* __restrict__ jobs, int m_rot, int level, int big_l,
             const u64* __restrict__ rcoef, const u64* __restrict__ inv_tab, Mods mods, Tables tb) {
  constexpr int N = 1 << LOGN;
  constexpr int NH = N / 2;
  constexpr int E = 8;
  constexpr int T = NH / E;
  constexpr bool NW = CLS == CLS_N32;
  __shared__ u64 lds[NttGeom<LOGN - 1, E>::LDS];
  const XcdSlot sl = xcd_slot(4 * level);
  if (sl.job >= m_rot) return;
  const size_t b = sl.job;
  const int h = sl.sub & 1;
  const int comp = (sl.sub >> 1) / level;
  const int t = (sl.sub >> 1) - comp * level;
  const KsJob jb = jobs[b];
  const ModConst m = mods.m[t];
  if ((int)m.cls != CLS) return;
  typedef IpAcc<CLS> IP;
  const int hoff = h * NH;
  const int sh = h ^ (int)((jb.g >> 1) & 1u);  // the source half of sigma_g's output half h
  typename IP::A acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0;
  for (int j = 0; j < level; ++j) {
    const u64* row = dhat + ((size_t)j * (level + 1) + t) * N + (size_t)sh * NH;
    // the key entries of this digit are loaded together with the digit row
    // (both in flight before the barrier)
    u64 kv[E], dv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) kv[e] = key_at(jb.key, big_l, j, comp, t, hoff + (int)threadIdx.x + e * T, N, m.narrow);
#pragma unroll
    for (int e = 0; e < E; ++e) dv[e] = row[(int)threadIdx.x + e * T];
#pragma unroll
    for (int e = 0; e < E; ++e) lds_putw<CLS_U64>(lds, (int)threadIdx.x + e * T, dv[e]);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = hoff + (int)threadIdx.x + e * T;
      IP::mac(acc[e], lds_getw<CLS_U64>(lds, galois_src<LOGN>(i, jb.g) - sh * NH), kv[e], m);
    }
    __syncthreads();
  }
  const Tw<CLS> tw0 = tw_of<LOGN, CLS>(tb, t, 0);
  const word_t<CLS> w1 = tw0.w[1];
  const word_t<CLS> w1sh = CLS == CLS_F64 ? word_t<CLS>(0) : tw0.sh[1];
  lift_half<LOGN, CLS, E>(lds, rcoef + (b * 2 + comp) * N, mods.m[big_l].q, m, h, w1, w1sh, (int)threadIdx.x);
  ntt_fwd_lds<LOGN - 1, CLS, E>(lds, tw_half_of<LOGN, CLS>(tb, t, h), mview<CLS>(m), opaque_tid());
  const u64 iv = inv_tab[big_l * HE_MAXM + t];
  const u64 ivs = inv_tab[HE_MAXM * HE_MAXM + big_l * HE_MAXM + t];
  const int i0 = lds_idx((int)threadIdx.x);
  u64 val[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int li = lds_step(i0, e, T);
    const u64 ipv = IP::canon(acc[e], m);
    if constexpr (CLS == CLS_F64) {
      const double dlt = f64_from_u64(ipv) - lds_getw_at<CLS>(lds, li);
      val[e] = to_canon<CLS>(f64_mulmod(dlt, f64_from_u64(iv), m.qd, m.qinv), m);
    } else {
      val[e] = shoupm<NW>(subm<NW>(ipv, to_canon<CLS>(lds_getw_at<CLS>(lds, li), m), m.q), iv, ivs, m.q);
    }
  }
  u64* o = jb.out + ((size_t)comp * level + t) * N;
  if (comp == 0) {
    // sigma_g(c0) of this half through LDS (64-bit canonical words)
    __syncthreads();
    load_half_perm<LOGN, CLS_U64, E>(lds, jb.c + (size_t)t * N, jb.ginv, false, h);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
      o[hoff + (int)threadIdx.x + e * T] = addm<NW>(lds_getw_at<CLS_U64>(lds, lds_step(i0, e, T)), val[e], m.q);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) o[hoff + (int)threadIdx.x + e * T] = val[e];
  }
}

// Keys and Galois elements of the steps of a rotate-and-sum chain.
constexpr int MAX_CHAIN = 16;
struct ChainKeys {
  const u64* key[MAX_CHAIN];
  u32 g[MAX_CHAIN], ginv[MAX_CHAIN];
};

// Keys and Galois elements of the rotations hoisted over one decomposition.
constexpr int MAX_HOIST = 64;
struct HoistKeys {
  const u64* key[MAX_HOIST];
  u32 g[MAX_HOIST], ginv[MAX_HOIST];
};

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

// DensePack MulPC (Table I): output out_base + blockIdx.y (index o*S + p),
// limb blockIdx.x; out[blockIdx.y] = sum_m x_m * sigma_{g_p}(F[o][class][m]),
// narrow limbs packed as 32-bit words when out_packed (KsJob's packed rows).
struct DPGeom {
  int h, w, c_in, d, stride, pad, o_c;
  int out_h, out_w, n_row_cls, n_col_cls, m_cts;
  int row_cls[64], col_cls[64];  // class id of every output row / column
  // several independent layers of this geometry in one launch: output index
  // oi = layer * per_layer + o * S + p; layer l reads x + l x_stride and its
  // base filters at filt + l f_stride (u64 elements)
  int per_layer;
  size_t x_stride, f_stride;
};

template <int LOGN, bool NARROW>
__device__ __forceinline__ void dp_hma_body(const u64* __restrict__ x, const u64* __restrict__ filt,
                                            u64* __restrict__ out, int level, int out_base, const DPGeom& geo,
                                            const ModConst& m, u64* lds, int out_packed) {
  typedef std::conditional_t<NARROW, u32, u64> W;
  constexpr int N = 1 << LOGN;
  constexpr int T = NttGeom<LOGN>::T;
  const int t = blockIdx.x;
  const int oall = out_base + (int)blockIdx.y;  // absolute output index over all layers
  const int layer = oall / geo.per_layer;
  const int oi = oall - layer * geo.per_layer;  // o*S + p within the layer
  x += (size_t)layer * geo.x_stride;
  filt += (size_t)layer * geo.f_stride;
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
    load_limb_perm<LOGN, NARROW ? CLS_N32 : CLS_U64, 16, true>(lds, f, ginv);
    __syncthreads();
    const u64* x0 = x + (((size_t)mc * 2 + 0) * level + t) * N;
    const u64* x1 = x + (((size_t)mc * 2 + 1) * level + t) * N;
    const int tid = opaque_tid();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int k = tid + r * T;
      const u64 fv = lds_get<NARROW ? CLS_N32 : CLS_U64>(lds, k, m);
      acc0[r] = (W)addm<NARROW>(acc0[r], mul_mod_t<NARROW>(x0[k], fv, m), m.q);
      acc1[r] = (W)addm<NARROW>(acc1[r], mul_mod_t<NARROW>(x1[k], fv, m), m.q);
    }
    __syncthreads();
  }
  u64* o0 = out + (((size_t)blockIdx.y * 2 + 0) * level + t) * N;  // chunk-relative
  u64* o1 = out + (((size_t)blockIdx.y * 2 + 1) * level + t) * N;
  if (NARROW && out_packed) {  // packed row (as a rotate-and-sum chain keeps its accumulator)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int k = (int)threadIdx.x + r * T;
      reinterpret_cast<u32*>(o0)[k] = (u32)acc0[r];
      reinterpret_cast<u32*>(o1)[k] = (u32)acc1[r];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = (int)threadIdx.x + r * T;
    o0[k] = acc0[r];
    o1[k] = acc1[r];
  }
}

// One instance per width class (limbs of other classes exit at once): the
// narrow one declares half the LDS, so twice the workgroups fit a CU.
template <int LOGN, int CLS>
__global__ void __launch_bounds__(NttGeom<LOGN>::T)
k_dp_hma(const u64* __restrict__ x, const u64* __restrict__ filt, u64* __restrict__ out, int level, int out_base,
         DPGeom geo, Mods mods, int out_packed) {
  constexpr bool NARROW = CLS == CLS_N32;
  __shared__ u64 lds[lds_words<LOGN, NARROW ? CLS_N32 : CLS_U64>()];
  const ModConst m = mods.m[blockIdx.x];
  if ((int)m.cls != CLS) return;
  dp_hma_body<LOGN, NARROW>(x, filt, out, level, out_base, geo, m, lds, out_packed);
}

// Sum of permuted-plaintext products into one accumulator per blockIdx.z:
// acc[z] (+)= sum_{k<K} cts[z*K + k] * sigma_{g_k}(pts[k * pt_stride]), with
// g_k = gal[k] (or g_k = g_step^k when gal == nullptr).  grid (N / 64,
// level, n_acc), 256 threads: 64 coefficients x 4 slices of the k loop
// (slice s takes k = s, s + 4, ...), whose partial sums meet in LDS.
// Narrow primes sum up to 15 products (< 2^60 each) before one reduction.
constexpr int HMA_SLICES = 4;
template <int LOGN>
__global__ void __launch_bounds__(256)
k_hma_perm(u64* __restrict__ acc, const u64* __restrict__ cts, int K, const u64* __restrict__ pts, int pt_stride,
           int pt_limbs, const int32_t* __restrict__ gal, u32 g_step, int level, int accumulate, Mods mods) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 part[2][HMA_SLICES][64];
  const int lane = (int)threadIdx.x & 63;
  const int sl = (int)threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int t = blockIdx.y;
  const size_t z = blockIdx.z;
  const ModConst m = mods.m[t];
  const u32 mask2n = (2u << LOGN) - 1u;
  u32 g = 1, g_stride = 1;  // g_step^sl, g_step^HMA_SLICES
  for (int e = 0; e < HMA_SLICES; ++e) {
    if (e < sl) g = (g * g_step) & mask2n;
    g_stride = (g_stride * g_step) & mask2n;
  }
  u64 s0 = 0, s1 = 0;
  if (m.narrow) {
    u64 l0 = 0, l1 = 0;
    int n_lazy = 0;
    for (int k = sl; k < K; k += HMA_SLICES) {
      const u32 gk = gal ? (u32)gal[k] : g;
      const int src = (gk == 1u) ? i : galois_src<LOGN>(i, gk);
      const u32 pv = (u32)pts[((size_t)k * pt_stride * pt_limbs + t) * N + src];
      const size_t cbase = (z * K + k) * 2;
      l0 += (u64)(u32)cts[((cbase + 0) * level + t) * N + i] * pv;
      l1 += (u64)(u32)cts[((cbase + 1) * level + t) * N + i] * pv;
      if (++n_lazy == 15) {
        s0 = add_mod(s0, reduce64(l0, m), m.q);
        s1 = add_mod(s1, reduce64(l1, m), m.q);
        l0 = l1 = 0;
        n_lazy = 0;
      }
      g = (g * g_stride) & mask2n;
    }
    s0 = add_mod(s0, reduce64(l0, m), m.q);
    s1 = add_mod(s1, reduce64(l1, m), m.q);
  } else {
    for (int k = sl; k < K; k += HMA_SLICES) {
      const u32 gk = gal ? (u32)gal[k] : g;
      const int src = (gk == 1u) ? i : galois_src<LOGN>(i, gk);
      const u64 pv = pts[((size_t)k * pt_stride * pt_limbs + t) * N + src];
      const size_t cbase = (z * K + k) * 2;
      s0 = add_mod(s0, mul_mod(cts[((cbase + 0) * level + t) * N + i], pv, m), m.q);
      s1 = add_mod(s1, mul_mod(cts[((cbase + 1) * level + t) * N + i], pv, m), m.q);
      g = (g * g_stride) & mask2n;
    }
  }
  part[0][sl][lane] = s0;
  part[1][sl][lane] = s1;
  __syncthreads();
  if (sl >= 2) return;  // slice c sums polynomial c
  const int c = sl;
  u64* a = acc + ((z * 2 + c) * level + t) * N;
  u64 v = accumulate ? a[i] : 0;
#pragma unroll
  for (int e = 0; e < HMA_SLICES; ++e) v = add_mod(v, part[c][e][lane], m.q);
  a[i] = v;
}

// Tap-style DensePack MulPC: out[b][o] = sum_{m < M} sum_{k < d^2}
// F[o][m][k] * X(b, m, k), where X(b, m, k) is the input x[b][m] for the tap
// with shift 0 (idx[k] < 0) and its hoisted rotation
// rot[(b M + m) nrot + idx[k]] otherwise.  F: [O][M][d^2][pt_limbs][N];
// x, rot, out: ciphertexts [2][level][N].  grid (N / 64, level,
// n_b ceil(O / TAP_OT)), 256 threads: 64 coefficients x TAP_SLICES slices
// of the (m, k) sum (slice s takes terms s, s + TAP_SLICES, ...), each
// thread holding up to TAP_OT outputs of its coefficient (per term 2
// ciphertext words and one plaintext word per output are read); the slices'
// partial sums meet in LDS.  Narrow primes sum 15 products (< 2^60 each)
// before one reduction.
constexpr int TAP_OT = 8;
constexpr int TAP_SLICES = 4;
struct TapMap {
  int d2, m_cts, o_c, nrot;
  signed char idx[64];
};
template <int LOGN>
__global__ void __launch_bounds__(256)
k_tap_hma(const u64* __restrict__ x, const u64* __restrict__ rot, const u64* __restrict__ filt, u64* __restrict__ out,
          int level, int pt_limbs, TapMap tm, Mods mods) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 part[TAP_SLICES][2 * TAP_OT][64];
  const int lane = (int)threadIdx.x & 63;
  const int sl = (int)threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int t = blockIdx.y;
  const int n_ot = (tm.o_c + TAP_OT - 1) / TAP_OT;
  const size_t b = blockIdx.z / n_ot;
  const int o0 = (int)(blockIdx.z % n_ot) * TAP_OT;
  const int no = min(TAP_OT, tm.o_c - o0);
  const ModConst m = mods.m[t];
  const size_t cstride = (size_t)2 * level * N;
  const size_t fo = (size_t)tm.m_cts * tm.d2 * pt_limbs * N;  // from one output's plaintexts to the next
  const u64* fbase = filt + (size_t)o0 * fo + (size_t)t * N + i;
  const int terms = tm.m_cts * tm.d2;
  u64 s0[TAP_OT], s1[TAP_OT];
#pragma unroll
  for (int r = 0; r < TAP_OT; ++r) s0[r] = s1[r] = 0;
  if (m.narrow) {
    u64 l0[TAP_OT], l1[TAP_OT];
#pragma unroll
    for (int r = 0; r < TAP_OT; ++r) l0[r] = l1[r] = 0;
    int n_lazy = 0;
    for (int e = sl; e < terms; e += TAP_SLICES) {
      const int mc = e / tm.d2, k = e - mc * tm.d2;
      const size_t ct = b * tm.m_cts + mc;
      const int id = tm.idx[k];
      const u64* src = (id < 0 ? x + ct * cstride : rot + (ct * tm.nrot + id) * cstride) + (size_t)t * N + i;
      const u64 a0 = (u32)src[0], a1 = (u32)src[(size_t)level * N];
      const u64* f = fbase + (size_t)e * pt_limbs * N;
#pragma unroll
      for (int r = 0; r < TAP_OT; ++r)
        if (r < no) {
          const u64 fv = (u32)f[r * fo];
          l0[r] += a0 * fv;
          l1[r] += a1 * fv;
        }
      if (++n_lazy == 15) {
#pragma unroll
        for (int r = 0; r < TAP_OT; ++r) {
          s0[r] = add_mod(s0[r], reduce64(l0[r], m), m.q);
          s1[r] = add_mod(s1[r], reduce64(l1[r], m), m.q);
          l0[r] = l1[r] = 0;
        }
        n_lazy = 0;
      }
    }
#pragma unroll
    for (int r = 0; r < TAP_OT; ++r) {
      s0[r] = add_mod(s0[r], reduce64(l0[r], m), m.q);
      s1[r] = add_mod(s1[r], reduce64(l1[r], m), m.q);
    }
  } else {
    for (int e = sl; e < terms; e += TAP_SLICES) {
      const int mc = e / tm.d2, k = e - mc * tm.d2;
      const size_t ct = b * tm.m_cts + mc;
      const int id = tm.idx[k];
      const u64* src = (id < 0 ? x + ct * cstride : rot + (ct * tm.nrot + id) * cstride) + (size_t)t * N + i;
      const u64 a0 = src[0], a1 = src[(size_t)level * N];
      const u64* f = fbase + (size_t)e * pt_limbs * N;
#pragma unroll
      for (int r = 0; r < TAP_OT; ++r)
        if (r < no) {
          const u64 fv = f[r * fo];
          s0[r] = add_mod(s0[r], mul_mod(a0, fv, m), m.q);
          s1[r] = add_mod(s1[r], mul_mod(a1, fv, m), m.q);
        }
    }
  }
#pragma unroll
  for (int r = 0; r < TAP_OT; ++r) {
    part[sl][r][lane] = s0[r];
    part[sl][TAP_OT + r][lane] = s1[r];
  }
  __syncthreads();
  // 2 TAP_OT x 64 sums of TAP_SLICES partials; consecutive threads take consecutive coefficients
  for (int e = (int)threadIdx.x; e < 2 * TAP_OT * 64; e += 256) {
    const int l = e & 63, v = e >> 6;
    const int c = v / TAP_OT, r = v - c * TAP_OT;
    if (r >= no) continue;
    u64 acc = part[0][v][l];
#pragma unroll
    for (int q = 1; q < TAP_SLICES; ++q) acc = add_mod(acc, part[q][v][l], m.q);
    out[(((b * tm.o_c + o0 + r) * 2 + c) * level + t) * N + blockIdx.x * 64 + l] = acc;
  }
}

// Tap-style DensePack MulPC over (Q, P) ahead of one ModDown per output:
// U[b][o] = sum_{m < M} [ sum_{k: idx[k] >= 0} F[o][m][k] * u[(b M + m) nrot
// + idx[k]] + F[o][m][k0] * P x[b][m] ], u the hoisted key inner products
// with P sigma(c0) already in (k_ip_perm with add_c0), P x on the Q limbs
// only.  Limb t < level reads F's limb t (F: [O][M][d^2][pt_limbs][N]); limb
// level is P and reads fp ([O][M][d^2][N]).  u and U rows in the key-switch
// layout: [2][level + 1][N] per ciphertext, narrow rows packed.  grid
// (N / 64, level + 1, n_b ceil(O / TAP_OT)), 256 threads as k_tap_hma.
template <int LOGN>
__global__ void __launch_bounds__(256)
k_tap_hma_qp(const u64* __restrict__ x, const u64* __restrict__ u, const u64* __restrict__ filt,
             const u64* __restrict__ fp, u64* __restrict__ out, int level, int pt_limbs, int big_l, TapMap tm,
             Mods mods) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 part[TAP_SLICES][2 * TAP_OT][64];
  const int lane = (int)threadIdx.x & 63;
  const int sl = (int)threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int t = blockIdx.y;
  const bool is_p = t == level;
  const int n_ot = (tm.o_c + TAP_OT - 1) / TAP_OT;
  const size_t b = blockIdx.z / n_ot;
  const int o0 = (int)(blockIdx.z % n_ot) * TAP_OT;
  const int no = min(TAP_OT, tm.o_c - o0);
  const ModConst m = mods.m[is_p ? big_l : t];
  const u64 pm = is_p ? 0 : reduce64(mods.m[big_l].q, m);  // P mod q_t
  const size_t cstride = (size_t)2 * level * N;
  const size_t ustride = (size_t)2 * (level + 1) * N;
  const int fl = is_p ? 1 : pt_limbs;  // limbs per plaintext in the array read
  const size_t fo = (size_t)tm.m_cts * tm.d2 * fl * N;
  const u64* fbase = (is_p ? fp : filt + (size_t)t * N) + (size_t)o0 * fo + i;
  const int terms = tm.m_cts * tm.d2;
  u64 s0[TAP_OT], s1[TAP_OT];
#pragma unroll
  for (int r = 0; r < TAP_OT; ++r) s0[r] = s1[r] = 0;
  if (m.narrow) {
    u64 l0[TAP_OT], l1[TAP_OT];
#pragma unroll
    for (int r = 0; r < TAP_OT; ++r) l0[r] = l1[r] = 0;
    int n_lazy = 0;
    for (int e = sl; e < terms; e += TAP_SLICES) {
      const int mc = e / tm.d2, k = e - mc * tm.d2;
      const size_t ct = b * tm.m_cts + mc;
      const int id = tm.idx[k];
      u64 a0, a1;
      if (id >= 0) {  // packed rows: N 32-bit residues at the start of each 64-bit row
        const u64* row0 = u + (ct * tm.nrot + id) * ustride + (size_t)t * N;
        a0 = reinterpret_cast<const u32*>(row0)[i];
        a1 = reinterpret_cast<const u32*>(row0 + (size_t)(level + 1) * N)[i];
      } else {
        if (is_p) continue;
        const u64* src = x + ct * cstride + (size_t)t * N + i;
        a0 = mul_mod(src[0], pm, m);
        a1 = mul_mod(src[(size_t)level * N], pm, m);
      }
      const u64* f = fbase + (size_t)e * fl * N;
#pragma unroll
      for (int r = 0; r < TAP_OT; ++r)
        if (r < no) {
          const u64 fv = (u32)f[r * fo];
          l0[r] += a0 * fv;
          l1[r] += a1 * fv;
        }
      if (++n_lazy == 15) {
#pragma unroll
        for (int r = 0; r < TAP_OT; ++r) {
          s0[r] = add_mod(s0[r], reduce64(l0[r], m), m.q);
          s1[r] = add_mod(s1[r], reduce64(l1[r], m), m.q);
          l0[r] = l1[r] = 0;
        }
        n_lazy = 0;
      }
    }
#pragma unroll
    for (int r = 0; r < TAP_OT; ++r) {
      s0[r] = add_mod(s0[r], reduce64(l0[r], m), m.q);
      s1[r] = add_mod(s1[r], reduce64(l1[r], m), m.q);
    }
  } else {
    for (int e = sl; e < terms; e += TAP_SLICES) {
      const int mc = e / tm.d2, k = e - mc * tm.d2;
      const size_t ct = b * tm.m_cts + mc;
      const int id = tm.idx[k];
      u64 a0, a1;
      if (id >= 0) {
        const u64* ur = u + (ct * tm.nrot + id) * ustride + (size_t)t * N + i;
        a0 = ur[0];
        a1 = ur[(size_t)(level + 1) * N];
      } else {
        if (is_p) continue;
        const u64* src = x + ct * cstride + (size_t)t * N + i;
        a0 = mul_mod(src[0], pm, m);
        a1 = mul_mod(src[(size_t)level * N], pm, m);
      }
      const u64* f = fbase + (size_t)e * fl * N;
#pragma unroll
      for (int r = 0; r < TAP_OT; ++r)
        if (r < no) {
          const u64 fv = f[r * fo];
          s0[r] = add_mod(s0[r], mul_mod(a0, fv, m), m.q);
          s1[r] = add_mod(s1[r], mul_mod(a1, fv, m), m.q);
        }
    }
  }
#pragma unroll
  for (int r = 0; r < TAP_OT; ++r) {
    part[sl][r][lane] = s0[r];
    part[sl][TAP_OT + r][lane] = s1[r];
  }
  __syncthreads();
  for (int e = (int)threadIdx.x; e < 2 * TAP_OT * 64; e += 256) {
    const int l = e & 63, v = e >> 6;
    const int c = v / TAP_OT, r = v - c * TAP_OT;
    if (r >= no) continue;
    u64 acc = part[0][v][l];
#pragma unroll
    for (int q = 1; q < TAP_SLICES; ++q) acc = add_mod(acc, part[q][v][l], m.q);
    u64* row = out + ((b * tm.o_c + o0 + r) * 2 + c) * (level + 1) * N + (size_t)t * N;
    if (m.narrow)
      reinterpret_cast<u32*>(row)[blockIdx.x * 64 + l] = (u32)acc;
    else
      row[blockIdx.x * 64 + l] = acc;
  }
}

// Homomorphic Im2Col, the masking step: out[b][k] (k = tap I_c + c,
// c = m B + blk) = mask_tap * X, X the block-shifted ciphertext
// z[b][m][blk] for the zero-shift tap (idx < 0) and its tap rotation
// rot[b][(m B + blk) nrot + idx[tap]] otherwise (nvalid block-shifted
// ciphertexts per input).  masks: [d^2][mask_limbs][N].  grid (N / 256,
// level, n_b K).
struct Him2colMap {
  int d2, c_in, per, m_cts, nrot, nvalid;
  signed char idx[64];
};
// ---------------------------------------------------------------------------
// Client-side helpers (key generation, encryption, decryption).

// Switching key rows: for digit j (blockIdx.z) and modulus t (blockIdx.y):
// b = e_hat - a*s + [t == j] (P mod q_t) * s', with s' = sigma_g(s) (g odd)
// or s^2 (g == 0).  ehat = NTT(e_j mod m_t) = [L][L+1][N] precomputed.
// With `pack`, rows of narrow moduli are written in the library's stored
// form (N 32-bit words), else every row as canonical 64-bit residues.
template <int LOGN>
__global__ void k_keygen(u64* key, const u64* s, const u64* a, const u64* ehat, u32 g, int big_l,
                         ConstTable p_mod, Mods mods, int pack) {
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
  u64* kb = key + (((size_t)j * 2 + 0) * (big_l + 1) + t) * N;
  u64* ka = key + (((size_t)j * 2 + 1) * (big_l + 1) + t) * N;
  if (pack && m.narrow) {  // packed 32-bit residues
    reinterpret_cast<u32*>(kb)[i] = (u32)b;
    reinterpret_cast<u32*>(ka)[i] = (u32)av;
  } else {
    kb[i] = b;
    ka[i] = av;
  }
}

}  // namespace he

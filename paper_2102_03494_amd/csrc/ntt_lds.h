// LDS-staged negacyclic NTT / INTT of one limb per workgroup (gfx950).
//
// Transform (the convention of the whole library): forward maps coefficients
// a_j to ahat[i] = a(psi^(2 brv(i) + 1)), i.e. evaluations at the odd powers
// of psi in bit-reversed order.  It is computed as log2 N Cooley-Tukey
// stages; stage s (m = 2^s groups, half-width t = N / 2^(s+1)) maps
// (a[j], a[j+t]) -> (a[j] + w a[j+t], a[j] - w a[j+t]) with
// w = psi^brv(m + j / (2t)).  The inverse runs the Gentleman-Sande mirror
// (stages in reverse order, (a[j], a[j+t]) -> (a[j] + a[j+t],
// (a[j] - a[j+t]) w^-1)) and scales by N^-1.
//
// `tid` is the thread index; callers that run several transforms in a loop
// pass it through an opaque copy made inside the loop, so that the compiler
// recomputes the LDS/twiddle addresses of each pass instead of keeping all of
// them live across iterations (which otherwise doubles register use).
//
// Work split: a workgroup of T = N / 16 threads holds the limb in LDS (one
// word of padding every 32 entries to spread LDS banks).  Stages are grouped
// into passes of up to 4; in a pass every thread loads 16 entries (one or
// more radix-2^k groups) into registers, runs the k stages there and writes
// them back, with one barrier per pass: 3-4 LDS round trips per transform
// instead of log2 N.  Callers stage data into LDS (coalesced, with any fused
// pre-processing such as a Galois permutation or a centred lift) and read the
// result back out of LDS in a coalesced pattern.
//
// Word size: limbs of a narrow prime (q < 2^30) are held as 32-bit words in
// registers and LDS and use 32-bit twiddle tables, so every butterfly is pure
// 32-bit integer work (three 32-bit multiplies for the Shoup product, min-based
// conditional subtractions); wide primes use 64-bit words.
#pragma once
#include <type_traits>

#include "modarith.h"

namespace he {

template <bool NARROW>
using word_t = std::conditional_t<NARROW, u32, u64>;

__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 5); }

template <int LOGN>
struct NttGeom {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 16;           // entries per thread per pass
  static constexpr int T = N / E;        // threads per workgroup
  static constexpr int LDS = N + (N >> 5);  // u64 words reserved (narrow limbs use half)
};

// LDS accessors in the word size of the width class.
template <bool NARROW>
__device__ __forceinline__ void lds_put(u64* lds, int i, u64 v) {
  if constexpr (NARROW) reinterpret_cast<u32*>(lds)[lds_idx(i)] = (u32)v;
  else lds[lds_idx(i)] = v;
}
template <bool NARROW>
__device__ __forceinline__ u64 lds_get(const u64* lds, int i) {
  if constexpr (NARROW) return reinterpret_cast<const u32*>(lds)[lds_idx(i)];
  else return lds[lds_idx(i)];
}

// ---- butterfly arithmetic ------------------------------------------------------
__device__ __forceinline__ u32 add32(u32 a, u32 b, u32 q) {
  const u32 s = a + b;          // < 2q < 2^32
  return min(s, s - q);         // s - q wraps above s when s < q
}
__device__ __forceinline__ u32 sub32(u32 a, u32 b, u32 q) {
  const u32 d = a + (q - b);    // in (0, 2q)
  return min(d, d - q);
}
__device__ __forceinline__ u32 shoup32(u32 a, u32 w, u32 wsh, u32 q) {
  const u32 qh = __umulhi(a, wsh);
  const u32 r = a * w - qh * q;  // in [0, 2q)
  return min(r, r - q);
}

template <bool NARROW>
struct Arith;

template <>
struct Arith<true> {
  typedef u32 W;
  static __device__ __forceinline__ W add(W a, W b, W q) { return add32(a, b, q); }
  static __device__ __forceinline__ W sub(W a, W b, W q) { return sub32(a, b, q); }
  static __device__ __forceinline__ W mulc(W a, W w, W wsh, W q) { return shoup32(a, w, wsh, q); }
};

template <>
struct Arith<false> {
  typedef u64 W;
  static __device__ __forceinline__ W add(W a, W b, W q) { return add_mod(a, b, q); }
  static __device__ __forceinline__ W sub(W a, W b, W q) { return sub_mod(a, b, q); }
  static __device__ __forceinline__ W mulc(W a, W w, W wsh, W q) { return mul_shoup(a, w, wsh, q, false); }
};

// Twiddle table view: narrow primes read the 32-bit tables.
template <bool NARROW>
struct Tw {
  const word_t<NARROW>* w;
  const word_t<NARROW>* sh;
};

// One forward pass: stages s0 .. s0+K-1.
template <int LOGN, int K, bool NARROW>
__device__ __forceinline__ void fwd_pass(u64* lds_raw, int s0, Tw<NARROW> tw, word_t<NARROW> q, int tid) {
  typedef word_t<NARROW> W;
  typedef Arith<NARROW> A;
  W* lds = reinterpret_cast<W*>(lds_raw);
  constexpr int N = 1 << LOGN;
  constexpr int R = 1 << K;
  constexpr int T = NttGeom<LOGN>::T;
  constexpr int G = 16 / R;
  const int B0 = N >> s0;
  const int Wd = B0 >> K;
  const int logW = LOGN - s0 - K;
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int g = gi * T + tid;
    const int blk = g >> logW;
    const int off = g & (Wd - 1);
    const int base = blk * B0 + off;
    W v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[lds_idx(base + r * Wd)];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int half = R >> (u + 1);
      const int m = 1 << (s0 + u);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & half) continue;
        const int ti = m + (blk << u) + (r >> (K - u));
        const W x = v[r];
        const W y = A::mulc(v[r + half], tw.w[ti], tw.sh[ti], q);
        v[r] = A::add(x, y, q);
        v[r + half] = A::sub(x, y, q);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) lds[lds_idx(base + r * Wd)] = v[r];
  }
}

// One inverse pass: stages s0+K-1 down to s0.
template <int LOGN, int K, bool NARROW>
__device__ __forceinline__ void inv_pass(u64* lds_raw, int s0, Tw<NARROW> tw, word_t<NARROW> q, int tid) {
  typedef word_t<NARROW> W;
  typedef Arith<NARROW> A;
  W* lds = reinterpret_cast<W*>(lds_raw);
  constexpr int N = 1 << LOGN;
  constexpr int R = 1 << K;
  constexpr int T = NttGeom<LOGN>::T;
  constexpr int G = 16 / R;
  const int B0 = N >> s0;
  const int Wd = B0 >> K;
  const int logW = LOGN - s0 - K;
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int g = gi * T + tid;
    const int blk = g >> logW;
    const int off = g & (Wd - 1);
    const int base = blk * B0 + off;
    W v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[lds_idx(base + r * Wd)];
#pragma unroll
    for (int u = K - 1; u >= 0; --u) {
      const int half = R >> (u + 1);
      const int m = 1 << (s0 + u);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & half) continue;
        const int ti = m + (blk << u) + (r >> (K - u));
        const W x = v[r];
        const W y = v[r + half];
        v[r] = A::add(x, y, q);
        v[r + half] = A::mulc(A::sub(x, y, q), tw.w[ti], tw.sh[ti], q);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) lds[lds_idx(base + r * Wd)] = v[r];
  }
}

// Forward transform of the limb held in LDS (all threads of the workgroup).
template <int LOGN, bool NARROW>
__device__ __forceinline__ void ntt_fwd_lds(u64* lds, Tw<NARROW> tw, word_t<NARROW> q, int tid) {
  constexpr int FULL = LOGN / 4;
  constexpr int REM = LOGN % 4;
  __syncthreads();
#pragma unroll
  for (int p = 0; p < FULL; ++p) {
    fwd_pass<LOGN, 4, NARROW>(lds, 4 * p, tw, q, tid);
    __syncthreads();
  }
  if constexpr (REM > 0) {
    fwd_pass<LOGN, REM, NARROW>(lds, 4 * FULL, tw, q, tid);
    __syncthreads();
  }
}

// Inverse transform of the limb held in LDS, without the N^-1 factor (the
// caller folds it into its store).
template <int LOGN, bool NARROW>
__device__ __forceinline__ void ntt_inv_lds(u64* lds, Tw<NARROW> tw, word_t<NARROW> q, int tid) {
  constexpr int FULL = LOGN / 4;
  constexpr int REM = LOGN % 4;
  __syncthreads();
  if constexpr (REM > 0) {
    inv_pass<LOGN, REM, NARROW>(lds, 4 * FULL, tw, q, tid);
    __syncthreads();
  }
#pragma unroll
  for (int p = FULL - 1; p >= 0; --p) {
    inv_pass<LOGN, 4, NARROW>(lds, 4 * p, tw, q, tid);
    __syncthreads();
  }
}

// NTT-domain index permutation of the automorphism X -> X^g:
// out[i] = in[galois_src(i)], 2 brv(src) + 1 = (2 brv(i) + 1) g mod 2N.
template <int LOGN>
__device__ __forceinline__ int galois_src(int i, u32 g) {
  const u32 mask2n = (2u << LOGN) - 1u;
  const u32 e = ((2u * (__brev((u32)i) >> (32 - LOGN)) + 1u) * g) & mask2n;
  return (int)(__brev((e - 1u) >> 1) >> (32 - LOGN));
}

}  // namespace he

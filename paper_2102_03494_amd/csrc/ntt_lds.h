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
// instead of log2 N.  A forward transform whose last 1 or 2 stages do not
// fill a pass runs them on the last full pass's registers with lane
// exchanges inside a quad (DPP) instead of one more LDS pass.  Callers stage data into LDS (coalesced, with any fused
// pre-processing such as a Galois permutation or a centred lift) and read the
// result back out of LDS in a coalesced pattern.
//
// Word size per width class (modarith.h): narrow limbs are 32-bit words in
// registers and LDS with 32-bit twiddle tables and Harvey's lazy butterflies
// (forward values kept in [0, 4q), inverse values in [0, 2q), which 4q < 2^32
// allows; three 32-bit multiplies per Shoup product, min-based conditional
// subtractions); f64 limbs are exact
// integers in doubles, left unreduced through the forward butterflies
// (|value| grows by at most 0.54 q per stage, below 8.6 q after 14 stages)
// and centred after each inverse sum; wide limbs are 64-bit words.
#pragma once
#include <type_traits>

#include "modarith.h"

namespace he {

template <int CLS>
struct Word {
  typedef u64 W;
};
template <>
struct Word<CLS_N32> {
  typedef u32 W;
};
template <>
struct Word<CLS_F64> {
  typedef double W;
};
template <int CLS>
using word_t = typename Word<CLS>::W;

__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 5); }

// lds_idx(i0 + r * stride) from lds_idx(i0), for stride a power of two and
// i0 mod stride + (r * stride) mod 32 < 32 (true for the element sets of a
// butterfly pass, where i0 mod 32 < stride or stride >= 32, and for the
// coalesced sets tid + r * T with 32 | T).  The added part is a compile-time
// constant once r and stride are, so it folds into the LDS instruction's
// immediate offset.
__device__ __forceinline__ int lds_step(int idx0, int r, int stride) { return idx0 + r * stride + ((r * stride) >> 5); }

// Workgroup barrier for LDS traffic only: each wave waits for its own LDS
// operations, then all waves meet.  __syncthreads also waits for the wave's
// outstanding global-to-LDS copies; this one lets copies into another LDS
// array stay in flight across the passes of a transform.  The memory clobber
// keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Transform workgroup geometry: E entries per thread per pass (16, or 8 for
// twice the threads with half the registers each), T = N / E threads, and
// radix-E register passes (log2 E stages between barriers).
template <int LOGN, int E_ = 16>
struct NttGeom {
  static_assert(E_ == 16 || E_ == 8, "16 or 8 entries per thread");
  static constexpr int N = 1 << LOGN;
  static constexpr int E = E_;              // entries per thread per pass
  static constexpr int T = N / E;           // threads per workgroup
  static constexpr int KMAX = E == 16 ? 4 : 3;  // stages per register pass
  static constexpr int LDS = N + (N >> 5);  // 64-bit words reserved (narrow limbs use half)
};

// 64-bit words of LDS a transform workgroup of class CLS declares: narrow
// limbs are 32-bit words, so half (more workgroups fit a CU).
template <int LOGN, int CLS>
constexpr int lds_words() {
  return CLS == CLS_N32 ? NttGeom<LOGN>::LDS / 2 : NttGeom<LOGN>::LDS;
}

// Modulus as seen by the butterflies of one class.
template <int CLS>
struct MV {
  u64 q;
};
template <>
struct MV<CLS_N32> {
  u32 q;
};
template <>
struct MV<CLS_F64> {
  double q, qinv;
};
template <int CLS>
__device__ __forceinline__ MV<CLS> mview(const ModConst& m) {
  if constexpr (CLS == CLS_N32) return MV<CLS>{(u32)m.q};
  else if constexpr (CLS == CLS_F64) return MV<CLS>{m.qd, m.qinv};
  else return MV<CLS>{m.q};
}

// Canonical residue (u64 in [0, q)) <-> word of the class.
template <int CLS>
__device__ __forceinline__ word_t<CLS> to_word(u64 v) {
  if constexpr (CLS == CLS_F64) return f64_from_u64(v);
  else return (word_t<CLS>)v;
}
// Canonical residue of a transform output (narrow: from [0, 4q)).
template <int CLS>
__device__ __forceinline__ u64 to_canon(word_t<CLS> v, const ModConst& m) {
  if constexpr (CLS == CLS_F64) {
    return f64_to_u64(f64_canon(v, m.qd, m.qinv));
  } else if constexpr (CLS == CLS_N32) {
    const u32 q = (u32)m.q;
    v = min(v, v - 2 * q);
    return (u64)min(v, v - q);
  } else {
    return (u64)v;
  }
}

// LDS accessors in the word size of the class: raw words, and canonical
// residues in and out.
template <int CLS>
__device__ __forceinline__ void lds_putw(u64* lds, int i, word_t<CLS> v) {
  reinterpret_cast<word_t<CLS>*>(lds)[lds_idx(i)] = v;
}
template <int CLS>
__device__ __forceinline__ word_t<CLS> lds_getw(const u64* lds, int i) {
  return reinterpret_cast<const word_t<CLS>*>(lds)[lds_idx(i)];
}
// The same at an already padded index (lds_idx / lds_step).
template <int CLS>
__device__ __forceinline__ void lds_putw_at(u64* lds, int idx, word_t<CLS> v) {
  reinterpret_cast<word_t<CLS>*>(lds)[idx] = v;
}
template <int CLS>
__device__ __forceinline__ word_t<CLS> lds_getw_at(const u64* lds, int idx) {
  return reinterpret_cast<const word_t<CLS>*>(lds)[idx];
}
template <int CLS>
__device__ __forceinline__ void lds_put(u64* lds, int i, u64 v) {
  lds_putw<CLS>(lds, i, to_word<CLS>(v));
}
template <int CLS>
__device__ __forceinline__ u64 lds_get(const u64* lds, int i, const ModConst& m) {
  return to_canon<CLS>(lds_getw<CLS>(lds, i), m);
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

// Butterfly pieces.  Forward (Cooley-Tukey): x = fwd_x(a), y = mulc(b),
// outputs (add(x, y), sub(x, y)).  Inverse (Gentleman-Sande): outputs
// (add_inv(a, b), mulc(sub_inv(a, b))).  mulc is the product with a table
// constant (w, companion wsh).
template <int CLS>
struct Arith;

template <>
struct Arith<CLS_N32> {  // Harvey: forward in [0, 4q), inverse in [0, 2q)
  typedef u32 W;
  static __device__ __forceinline__ W fwd_x(W a, MV<CLS_N32> m) { return min(a, a - 2 * m.q); }
  static __device__ __forceinline__ W add(W a, W b, MV<CLS_N32>) { return a + b; }
  static __device__ __forceinline__ W sub(W a, W b, MV<CLS_N32> m) { return a - b + 2 * m.q; }
  static __device__ __forceinline__ W add_inv(W a, W b, MV<CLS_N32> m) {
    const W s = a + b;
    return min(s, s - 2 * m.q);
  }
  static __device__ __forceinline__ W sub_inv(W a, W b, MV<CLS_N32> m) { return a - b + 2 * m.q; }
  // lazy Shoup product in [0, 2q) of any a < 2^32
  static __device__ __forceinline__ W mulc(W a, W w, W wsh, MV<CLS_N32> m) {
    return a * w - __umulhi(a, wsh) * m.q;
  }
};

template <>
struct Arith<CLS_F64> {
  typedef double W;
  static __device__ __forceinline__ W fwd_x(W a, MV<CLS_F64>) { return a; }
  static __device__ __forceinline__ W add(W a, W b, MV<CLS_F64>) { return a + b; }
  static __device__ __forceinline__ W sub(W a, W b, MV<CLS_F64>) { return a - b; }
  static __device__ __forceinline__ W add_inv(W a, W b, MV<CLS_F64> m) { return f64_centre(a + b, m.q, m.qinv); }
  static __device__ __forceinline__ W sub_inv(W a, W b, MV<CLS_F64>) { return a - b; }
  // the companion w / q is formed on the fly (one multiply instead of a
  // second table load and two registers per twiddle)
  static __device__ __forceinline__ W mulc(W a, W w, W, MV<CLS_F64> m) { return f64_mulc(a, w, w * m.qinv, m.q); }
};

template <>
struct Arith<CLS_U64> {
  typedef u64 W;
  static __device__ __forceinline__ W fwd_x(W a, MV<CLS_U64>) { return a; }
  static __device__ __forceinline__ W add(W a, W b, MV<CLS_U64> m) { return add_mod(a, b, m.q); }
  static __device__ __forceinline__ W sub(W a, W b, MV<CLS_U64> m) { return sub_mod(a, b, m.q); }
  static __device__ __forceinline__ W add_inv(W a, W b, MV<CLS_U64> m) { return add_mod(a, b, m.q); }
  static __device__ __forceinline__ W sub_inv(W a, W b, MV<CLS_U64> m) { return sub_mod(a, b, m.q); }
  static __device__ __forceinline__ W mulc(W a, W w, W wsh, MV<CLS_U64> m) {
    return mul_shoup(a, w, wsh, m.q, false);
  }
};

// Twiddle table view in the class's word type: w and its Shoup companion
// (integer classes; the f64 class reads w only).
template <int CLS>
struct Tw {
  const word_t<CLS>* w;
  const word_t<CLS>* sh;
};

// Lane exchange inside a quad through DPP (xor 1: quad_perm [1,0,3,2];
// xor 2: [2,3,0,1]); every lane of the wave must be active.
template <int X>
__device__ __forceinline__ u32 quad_xor32(u32 v) {
  static_assert(X == 1 || X == 2, "quad lanes only");
  return (u32)__builtin_amdgcn_update_dpp(0, (int)v, X == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int X, typename W>
__device__ __forceinline__ W quad_xor(W v) {
  if constexpr (sizeof(W) == 4) {
    return (W)quad_xor32<X>((u32)v);
  } else {
    const u64 b = __builtin_bit_cast(u64, v);
    const u64 r = ((u64)quad_xor32<X>((u32)(b >> 32)) << 32) | quad_xor32<X>((u32)b);
    return __builtin_bit_cast(W, r);
  }
}

// One forward pass: stages s0 .. s0+K-1.  With TAIL (1 or 2, the pass that
// ends K stages before the last), the last TAIL stages follow in registers:
// after the pass a thread's entries are j = blk B0 + off + 2^TAIL r with
// off = lane mod 2^TAIL, so each remaining butterfly pairs the same r of
// lanes off and off ^ t (t = 1, 2), exchanged within the quad through DPP
// instead of another LDS round trip and barrier.  The lane of the lower
// entry sends fwd_x(x), the upper lane w y; both form the usual x + w y /
// x - w y, so the results are those of the LDS pass.
template <int LOGN, int K, int CLS, int E = 16, int TAIL = 0>
__device__ __forceinline__ void fwd_pass(u64* lds_raw, int s0, Tw<CLS> tw, MV<CLS> q, int tid) {
  typedef word_t<CLS> W;
  typedef Arith<CLS> A;
  W* lds = reinterpret_cast<W*>(lds_raw);
  constexpr int N = 1 << LOGN;
  constexpr int R = 1 << K;
  constexpr int T = NttGeom<LOGN, E>::T;
  constexpr int G = E / R;
  const int B0 = N >> s0;
  const int Wd = B0 >> K;
  const int logW = LOGN - s0 - K;
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int g = gi * T + tid;
    const int blk = g >> logW;
    const int off = g & (Wd - 1);
    const int base = blk * B0 + off;
    const int b0 = lds_idx(base);
    W v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[lds_step(b0, r, Wd)];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int half = R >> (u + 1);
      const int m = 1 << (s0 + u);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & half) continue;
        const int ti = m + (blk << u) + (r >> (K - u));
        const W x = A::fwd_x(v[r], q);
        const W y = A::mulc(v[r + half], tw.w[ti], CLS == CLS_F64 ? W(0) : tw.sh[ti], q);
        v[r] = A::add(x, y, q);
        v[r + half] = A::sub(x, y, q);
      }
    }
    if constexpr (TAIL > 0) {
      static_assert(TAIL <= 2 && G == 1, "a tail follows a full pass with one group per thread");
#pragma unroll
      for (int u = 0; u < TAIL; ++u) {
        const int t = 1 << (TAIL - 1 - u);  // lane (and entry) distance of this stage's pairs
        const int m = 1 << (s0 + K + u);
        const bool upper = (off & t) != 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int j = base + Wd * r;
          const int ti = m + (j >> (TAIL - u));
          const W x = A::fwd_x(v[r], q);
          const W y = A::mulc(v[r], tw.w[ti], CLS == CLS_F64 ? W(0) : tw.sh[ti], q);
          const W send = upper ? y : x;
          const W recv = (TAIL - 1 - u) == 0 ? quad_xor<1>(send) : quad_xor<2>(send);
          v[r] = upper ? A::sub(recv, y, q) : A::add(x, recv, q);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) lds[lds_step(b0, r, Wd)] = v[r];
  }
}

// One inverse pass: stages s0+K-1 down to s0.  f64 sums are centred only at
// the pass's last stage (and, in a first radix-16 pass, whose input is
// canonical in [0, q), also after its second stage): a pass's input then
// stays below 0.54 q in magnitude (q in the first pass), so sums stay below
// 8.7 q and the products' inputs within the forward transform's range.
template <int LOGN, int K, int CLS, int E = 16, bool FIRST = false>
__device__ __forceinline__ void inv_pass(u64* lds_raw, int s0, Tw<CLS> tw, MV<CLS> q, int tid) {
  typedef word_t<CLS> W;
  typedef Arith<CLS> A;
  W* lds = reinterpret_cast<W*>(lds_raw);
  constexpr int N = 1 << LOGN;
  constexpr int R = 1 << K;
  constexpr int T = NttGeom<LOGN, E>::T;
  constexpr int G = E / R;
  const int B0 = N >> s0;
  const int Wd = B0 >> K;
  const int logW = LOGN - s0 - K;
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int g = gi * T + tid;
    const int blk = g >> logW;
    const int off = g & (Wd - 1);
    const int base = blk * B0 + off;
    const int b0 = lds_idx(base);
    W v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[lds_step(b0, r, Wd)];
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
        if constexpr (CLS == CLS_F64) {
          const bool centre = u == 0 || (FIRST && K == 4 && u == 2);
          v[r] = centre ? A::add_inv(x, y, q) : A::add(x, y, q);
        } else {
          v[r] = A::add_inv(x, y, q);
        }
        v[r + half] = A::mulc(A::sub_inv(x, y, q), tw.w[ti], CLS == CLS_F64 ? W(0) : tw.sh[ti], q);
      }
      // f64: load the next stage's twiddles after this stage, so only one
      // stage's are live (measured faster for the f64 inverse transform)
      if constexpr (CLS == CLS_F64) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) lds[lds_step(b0, r, Wd)] = v[r];
  }
}

// Forward transform of the limb held in LDS (all threads of the workgroup).
template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void ntt_fwd_lds(u64* lds, Tw<CLS> tw, MV<CLS> q, int tid) {
  constexpr int KM = NttGeom<LOGN, E>::KMAX;
  constexpr int FULL = LOGN / KM;
  constexpr int REM = LOGN % KM;
  lds_barrier();
  if constexpr (REM > 0 && REM <= 2 && FULL > 0) {
    // the last REM stages ride on the last full pass (lane exchanges, no LDS pass)
#pragma unroll
    for (int p = 0; p < FULL - 1; ++p) {
      fwd_pass<LOGN, KM, CLS, E>(lds, KM * p, tw, q, tid);
      lds_barrier();
    }
    fwd_pass<LOGN, KM, CLS, E, REM>(lds, KM * (FULL - 1), tw, q, tid);
    lds_barrier();
  } else {
#pragma unroll
    for (int p = 0; p < FULL; ++p) {
      fwd_pass<LOGN, KM, CLS, E>(lds, KM * p, tw, q, tid);
      lds_barrier();
    }
    if constexpr (REM > 0) {
      fwd_pass<LOGN, REM, CLS, E>(lds, KM * FULL, tw, q, tid);
      lds_barrier();
    }
  }
}

// Inverse transform of the limb held in LDS, without the N^-1 factor (the
// caller folds it into its store).
template <int LOGN, int CLS, int E = 16>
__device__ __forceinline__ void ntt_inv_lds(u64* lds, Tw<CLS> tw, MV<CLS> q, int tid) {
  constexpr int KM = NttGeom<LOGN, E>::KMAX;
  constexpr int FULL = LOGN / KM;
  constexpr int REM = LOGN % KM;
  lds_barrier();
  if constexpr (REM > 0) {
    inv_pass<LOGN, REM, CLS, E, true>(lds, KM * FULL, tw, q, tid);
    lds_barrier();
  } else {
    inv_pass<LOGN, KM, CLS, E, true>(lds, KM * (FULL - 1), tw, q, tid);
    lds_barrier();
  }
#pragma unroll
  for (int p = (REM > 0 ? FULL : FULL - 1) - 1; p >= 0; --p) {
    inv_pass<LOGN, KM, CLS, E>(lds, KM * p, tw, q, tid);
    lds_barrier();
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

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
// Work split: a workgroup of T = N / 16 threads holds the limb in LDS (one
// u64 of padding every 32 entries to spread LDS banks).  Stages are grouped
// into passes of up to 4; in a pass every thread loads 16 entries (one or
// more radix-2^k groups) into registers, runs the k stages there and writes
// them back, with one barrier per pass: 3-4 LDS round trips per transform
// instead of log2 N.  Callers stage data into LDS (coalesced, with any fused
// pre-processing such as a Galois permutation or a centred lift) and read the
// result back out of LDS in a coalesced pattern.
#pragma once
#include "modarith.h"

namespace he {

__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 5); }

template <int LOGN>
struct NttGeom {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 16;           // entries per thread per pass
  static constexpr int T = N / E;        // threads per workgroup
  static constexpr int LDS = N + (N >> 5);
};

// One forward pass: stages s0 .. s0+K-1.
template <int LOGN, int K, bool NARROW>
__device__ __forceinline__ void fwd_pass(u64* lds, int s0, const u64* __restrict__ tw,
                                         const u64* __restrict__ twsh, u64 q) {
  constexpr int N = 1 << LOGN;
  constexpr int R = 1 << K;
  constexpr int T = NttGeom<LOGN>::T;
  constexpr int G = 16 / R;
  const int B0 = N >> s0;
  const int W = B0 >> K;
  const int logW = LOGN - s0 - K;
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int g = gi * T + (int)threadIdx.x;
    const int blk = g >> logW;
    const int off = g & (W - 1);
    const int base = blk * B0 + off;
    u64 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[lds_idx(base + r * W)];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int half = R >> (u + 1);
      const int m = 1 << (s0 + u);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & half) continue;
        const int ti = m + (blk << u) + (r >> (K - u));
        const u64 x = v[r];
        const u64 y = mul_shoup(v[r + half], tw[ti], twsh[ti], q, NARROW);
        v[r] = add_mod(x, y, q);
        v[r + half] = sub_mod(x, y, q);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) lds[lds_idx(base + r * W)] = v[r];
  }
}

// One inverse pass: stages s0+K-1 down to s0.
template <int LOGN, int K, bool NARROW>
__device__ __forceinline__ void inv_pass(u64* lds, int s0, const u64* __restrict__ tw,
                                         const u64* __restrict__ twsh, u64 q) {
  constexpr int N = 1 << LOGN;
  constexpr int R = 1 << K;
  constexpr int T = NttGeom<LOGN>::T;
  constexpr int G = 16 / R;
  const int B0 = N >> s0;
  const int W = B0 >> K;
  const int logW = LOGN - s0 - K;
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int g = gi * T + (int)threadIdx.x;
    const int blk = g >> logW;
    const int off = g & (W - 1);
    const int base = blk * B0 + off;
    u64 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[lds_idx(base + r * W)];
#pragma unroll
    for (int u = K - 1; u >= 0; --u) {
      const int half = R >> (u + 1);
      const int m = 1 << (s0 + u);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & half) continue;
        const int ti = m + (blk << u) + (r >> (K - u));
        const u64 x = v[r];
        const u64 y = v[r + half];
        v[r] = add_mod(x, y, q);
        v[r + half] = mul_shoup(sub_mod(x, y, q), tw[ti], twsh[ti], q, NARROW);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) lds[lds_idx(base + r * W)] = v[r];
  }
}

// Forward transform of the limb held in LDS (all threads of the workgroup).
template <int LOGN, bool NARROW>
__device__ __forceinline__ void ntt_fwd_lds(u64* lds, const u64* tw, const u64* twsh, u64 q) {
  constexpr int FULL = LOGN / 4;
  constexpr int REM = LOGN % 4;
  __syncthreads();
#pragma unroll
  for (int p = 0; p < FULL; ++p) {
    fwd_pass<LOGN, 4, NARROW>(lds, 4 * p, tw, twsh, q);
    __syncthreads();
  }
  if constexpr (REM > 0) {
    fwd_pass<LOGN, REM, NARROW>(lds, 4 * FULL, tw, twsh, q);
    __syncthreads();
  }
}

// Inverse transform of the limb held in LDS, without the N^-1 factor (the
// caller folds it into its store).
template <int LOGN, bool NARROW>
__device__ __forceinline__ void ntt_inv_lds(u64* lds, const u64* tw, const u64* twsh, u64 q) {
  constexpr int FULL = LOGN / 4;
  constexpr int REM = LOGN % 4;
  __syncthreads();
  if constexpr (REM > 0) {
    inv_pass<LOGN, REM, NARROW>(lds, 4 * FULL, tw, twsh, q);
    __syncthreads();
  }
#pragma unroll
  for (int p = FULL - 1; p >= 0; --p) {
    inv_pass<LOGN, 4, NARROW>(lds, 4 * p, tw, twsh, q);
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

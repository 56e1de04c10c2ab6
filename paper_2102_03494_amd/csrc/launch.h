// Definitions of the launch wrappers declared in ctx.h: each picks the
// kernel instances of its ring size and width classes and enqueues them.
#pragma once
#include "ctx.h"

namespace he {


template <int LOGN>
void LNtt<LOGN>::run(he_ctx* c, u64* d, int n_polys, int n_limbs, int first_mod, bool fwd, hipStream_t s) {
  dim3 grid(n_limbs, n_polys);
  Prof pr(c, "ntt", s);
  const unsigned mask = cls_mask(c, first_mod, n_limbs);
  if (fwd)
    HE_FOR_CLASSES(mask, (k_ntt<LOGN, true, CLS><<<grid, NttGeom<LOGN>::T, 0, s>>>(d, n_limbs, first_mod, c->mods,
                                                                                    c->tb())));
  else
    HE_FOR_CLASSES(mask, (k_ntt<LOGN, false, CLS><<<grid, NttGeom<LOGN>::T, 0, s>>>(d, n_limbs, first_mod, c->mods,
                                                                                     c->tb())));
}

// Key switch of a job batch: digits -> ModUp + inner product -> INTT of P (in
// the ModUp launch when P is one group).
// ModUp is one launch when the ring's primes span one or two width classes
// (each workgroup runs its target's class); with all three, the kernel of
// each class runs on its own stream (the caller's for the first, the side
// stream for the others), joined before the P INTT.
template <int LOGN>
void LKsCore<LOGN>::run(he_ctx* c, const KsJob* jobs, int count, int lmax, int pg, u64* dcoef, u64* u, u64* rc,
                  hipStream_t s, int pk, bool digits_done) {
  constexpr int T = NttGeom<LOGN>::T;
  const int n_cls = (int)c->has_cls[0] + (int)c->has_cls[1] + (int)c->has_cls[2];
  // rings run in halves leave the P limb to k_intt_last
  const int hs = c->halves_set[lmax];
  const bool want_halves = hs < 0 ? LOGN >= HALF_MODUP_MIN_LOGN : hs != 0;
  const bool halves = LOGN >= HALF_MODUP_ANY_LOGN && want_halves && n_cls <= 2;
  // with one P group, ModUp's P workgroups also write the coefficient-domain
  // P limb (rc), and no separate INTT launch is needed
  u64* rc1 = (pg == 1 && !halves) ? rc : nullptr;
  {
    Prof pr(c, "ks_digits", s);
    if (digits_done) {
      // the previous step's ModDown wrote them
    } else if (pk & JOB_IN_PACKED)
      HE_FOR_CLASSES(c->q_mask, (k_ks_digits<LOGN, CLS, true><<<xcd_grid(lmax, count), T, 0, s>>>(
                                    jobs, count, dcoef, lmax, c->mods, c->tb())));
    else
      HE_FOR_CLASSES(c->q_mask, (k_ks_digits<LOGN, CLS, false><<<xcd_grid(lmax, count), T, 0, s>>>(
                                    jobs, count, dcoef, lmax, c->mods, c->tb())));
  }
  const unsigned grid = xcd_grid(lmax + pg, count);
  constexpr int TM = modup_threads<LOGN>();  // ModUp workgroup size
  static const char* names[3] = {"ks_modup_ip", "ks_modup_ip_f64", "ks_modup_ip_wide"};
  if constexpr (LOGN >= HALF_MODUP_ANY_LOGN) {
    if (halves) {  // one launch, two workgroups (halves) per target
      Prof stage(c, "ks_modup_stage", s);
      const unsigned hgrid = xcd_grid(2 * (lmax + pg), count);
      constexpr int TH = modup_half_threads<LOGN>();
#define HE_HALF(A, B) \
  k_ks_modup_half<LOGN, A, B><<<hgrid, TH, 0, s>>>(jobs, count, dcoef, u, lmax, pg, c->big_l, c->mods, c->tb())
      if (n_cls == 1) {
        if (c->has_cls[CLS_N32]) HE_HALF(CLS_N32, CLS_N32);
        else if (c->has_cls[CLS_F64]) HE_HALF(CLS_F64, CLS_F64);
        else HE_HALF(CLS_U64, CLS_U64);
      } else if (!c->has_cls[CLS_U64]) {
        HE_HALF(CLS_N32, CLS_F64);
      } else if (!c->has_cls[CLS_F64]) {
        HE_HALF(CLS_N32, CLS_U64);
      } else {
        HE_HALF(CLS_F64, CLS_U64);
      }
#undef HE_HALF
    }
  }
  if (halves) {
    // ModUp done above
  } else if (n_cls == 2) {  // one launch, each workgroup in its target's class
    Prof stage(c, "ks_modup_stage", s);
    if (!c->has_cls[CLS_U64])
      k_ks_modup_ip2<LOGN, CLS_N32, CLS_F64><<<grid, TM, 0, s>>>(jobs, count, dcoef, u, rc1, lmax, pg, c->big_l,
                                                                 c->mods, c->tb());
    else if (!c->has_cls[CLS_F64])
      k_ks_modup_ip2<LOGN, CLS_N32, CLS_U64><<<grid, TM, 0, s>>>(jobs, count, dcoef, u, rc1, lmax, pg, c->big_l,
                                                                 c->mods, c->tb());
    else
      k_ks_modup_ip2<LOGN, CLS_F64, CLS_U64><<<grid, TM, 0, s>>>(jobs, count, dcoef, u, rc1, lmax, pg, c->big_l,
                                                                 c->mods, c->tb());
  } else {
  const bool forked = n_cls > 1;
  {
    Prof stage(c, "ks_modup_stage", s);  // wall time of all classes together
    if (forked) {  // the side stream starts after the digits, not after the first ModUp kernel
      (void)hipEventRecord(c->fork_ev, s);
      (void)hipStreamWaitEvent(c->side, c->fork_ev, 0);
    }
    bool first = true;
    for (int cls = 0; cls < 3; ++cls) {
      if (!c->has_cls[cls]) continue;
      const hipStream_t st = first ? s : c->side;
      first = false;
      Prof pr(c, names[cls], st);
      if (cls == CLS_N32)
        k_ks_modup_ip<LOGN, CLS_N32><<<grid, TM, 0, st>>>(jobs, count, dcoef, u, rc1, lmax, pg, c->big_l, c->mods,
                                                          c->tb());
      else if (cls == CLS_F64)
        k_ks_modup_ip<LOGN, CLS_F64><<<grid, TM, 0, st>>>(jobs, count, dcoef, u, rc1, lmax, pg, c->big_l, c->mods,
                                                          c->tb());
      else
        k_ks_modup_ip<LOGN, CLS_U64><<<grid, TM, 0, st>>>(jobs, count, dcoef, u, rc1, lmax, pg, c->big_l, c->mods,
                                                          c->tb());
    }
    if (forked) {
      (void)hipEventRecord(c->join_ev, c->side);
      (void)hipStreamWaitEvent(s, c->join_ev, 0);
    }
  }
  }
  if (rc1) return;
  Prof pr(c, "intt_last", s);
  if constexpr (LOGN <= 13) {
    if (c->p_cls != CLS_N32) {  // 64-bit LDS words: 8 entries per thread, twice the waves
      HE_FOR_CLASSES(1u << c->p_cls, (k_intt_p8<LOGN, CLS><<<xcd_grid(2, count), p8_threads<LOGN>(), 0, s>>>(
                                         jobs, count, u, lmax, pg, c->big_l, rc, c->mods, c->tb())));
      return;
    }
  }
  HE_FOR_CLASSES(1u << c->p_cls, (k_intt_last<LOGN, MODE_P, CLS><<<xcd_grid(2, count), T, 0, s>>>(
                                     jobs, count, u, lmax, pg, c->big_l, rc, c->mods, c->tb())));
}

// ModDown (MODE_P, u with `urows` rows per polynomial) or rescale
// (MODE_LAST) of a job batch with the given epilogue.
template <int LOGN>
void LDrop<LOGN>::run(he_ctx* c, int mode, int epi, const KsJob* jobs, int count, int lmax, int urows, const u64* u,
                  const u64* rc, hipStream_t s, int pk, NextDigits nd) {
  constexpr int T = drop_threads<LOGN>();
  const int keep = mode == MODE_P ? lmax : lmax - 1;
  const unsigned grid = xcd_grid(2 * keep, count);
  Prof pr(c, "drop_last", s);
  if constexpr (LOGN >= HALF_MODUP_ANY_LOGN) {
    // ModDown in halves (k_drop_half): unpacked ciphertexts, no next-step digits
    const bool halves = c->moddown_halves < 0 ? LOGN >= HALF_MODDOWN_MIN_LOGN : c->moddown_halves != 0;
    if (halves && mode == MODE_P && pk == 0 && nd.dcoef == nullptr) {
      const unsigned hgrid = xcd_grid(4 * keep, count);
      constexpr int TH = drop_half_threads<LOGN>();
#define HE_DROP_HALF(EP)                                                                                        \
  HE_FOR_CLASSES(c->q_mask, (k_drop_half<LOGN, EP, CLS><<<hgrid, TH, 0, s>>>(jobs, count, keep, u, urows, c->big_l, \
                                                                             rc, c->d_inv, c->mods, c->tb())))
      if (epi == EPI_ROT) HE_DROP_HALF(EPI_ROT);
      else if (epi == EPI_ROTSUM) HE_DROP_HALF(EPI_ROTSUM);
      else if (epi == EPI_RELIN) HE_DROP_HALF(EPI_RELIN);
      else HE_DROP_HALF(EPI_STORE);
#undef HE_DROP_HALF
      return;
    }
  }
#define HE_DROP(MD, EP, PK)                                                                                    \
HE_FOR_CLASSES(c->q_mask, (k_drop_last<LOGN, MD, EP, CLS, PK><<<grid, T, 0, s>>>(jobs, count, keep, u, urows,  \
                                                                                 c->big_l, rc, c->d_inv, c->mods, \
                                                                                 c->tb(), nd)))
  // packed variants exist where a rotate-and-sum chain uses them: its steps
  // (ROTSUM, output packed, input packed after the first) and its rescale
  if (mode == MODE_LAST) {
    if (pk & JOB_IN_PACKED) HE_DROP(MODE_LAST, EPI_STORE, JOB_IN_PACKED);
    else HE_DROP(MODE_LAST, EPI_STORE, 0);
  } else if (epi == EPI_ROT) {
    HE_DROP(MODE_P, EPI_ROT, 0);
  } else if (epi == EPI_ROTSUM) {
    if (pk == (JOB_IN_PACKED | JOB_OUT_PACKED)) HE_DROP(MODE_P, EPI_ROTSUM, JOB_IN_PACKED | JOB_OUT_PACKED);
    else if (pk == JOB_OUT_PACKED) HE_DROP(MODE_P, EPI_ROTSUM, JOB_OUT_PACKED);
    else HE_DROP(MODE_P, EPI_ROTSUM, 0);
  } else if (epi == EPI_RELIN) {
    HE_DROP(MODE_P, EPI_RELIN, 0);
  } else {
    HE_DROP(MODE_P, EPI_STORE, 0);
  }
#undef HE_DROP
}

template <int LOGN>
void LIntt1<LOGN>::run(he_ctx* c, const KsJob* jobs, int count, int lmax, u64* rc, hipStream_t s, int pk) {
  Prof pr(c, "intt_last", s);
  if (pk & JOB_IN_PACKED)
    HE_FOR_CLASSES(c->q_mask, (k_intt_last<LOGN, MODE_LAST, CLS, true><<<xcd_grid(2, count), NttGeom<LOGN>::T, 0,
                                                                         s>>>(jobs, count, nullptr, lmax, 1,
                                                                              c->big_l, rc, c->mods, c->tb())));
  else
    HE_FOR_CLASSES(c->q_mask, (k_intt_last<LOGN, MODE_LAST, CLS, false><<<xcd_grid(2, count), NttGeom<LOGN>::T, 0,
                                                                          s>>>(jobs, count, nullptr, lmax, 1,
                                                                               c->big_l, rc, c->mods, c->tb())));
}

template <int LOGN>
void LDpHma<LOGN>::run(he_ctx* c, const u64* x, const u64* filt, u64* out, int level, int out_base, int n_out,
                  const DPGeom& geo, hipStream_t s, bool out_packed) {
  Prof pr(c, "dp_hma", s);
  HE_FOR_CLASSES(c->q_mask, (k_dp_hma<LOGN, CLS><<<dim3(level, n_out), NttGeom<LOGN>::T, 0, s>>>(
                                 x, filt, out, level, out_base, geo, c->mods, (int)out_packed)));
}

template <int LOGN>
void LHmaPerm<LOGN>::run(he_ctx* c, u64* acc, const u64* cts, int K, const u64* pts, int pt_stride, int pt_limbs,
                  const int32_t* gal, u32 g_step, int level, int accumulate, int n_acc, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  Prof pr(c, "hma_perm", s);
  k_hma_perm<LOGN><<<dim3(N / 64, level, n_acc), 256, 0, s>>>(acc, cts, K, pts, pt_stride, pt_limbs, gal, g_step,
                                                                level, accumulate, c->mods);
}

template <int LOGN>
void LKeygen<LOGN>::run(he_ctx* c, u64* key, const u64* sk, const u64* a, const u64* ehat, u32 g, ConstTable pm,
                  hipStream_t s, int pack) {
  constexpr int N = 1 << LOGN;
  k_keygen<LOGN><<<dim3(N / 256, c->big_l + 1, c->big_l), 256, 0, s>>>(key, sk, a, ehat, g, c->big_l, pm,
                                                                        c->mods, pack);
}

// Hoisted rotations: digits of c1 and the lifted digits, computed once per
// ciphertext (jobs1: one decomposition job per ciphertext) ...
template <int LOGN>
void LHoistUp<LOGN>::run(he_ctx* c, const KsJob* jobs1, int count, int level, u64* dcoef, u64* dhat, hipStream_t s) {
  constexpr int T = NttGeom<LOGN>::T;
  HE_FOR_CLASSES(c->q_mask, (k_ks_digits<LOGN, CLS><<<xcd_grid(level, count), T, 0, s>>>(jobs1, count, dcoef, level,
                                                                                           c->mods, c->tb())));
  Prof pr(c, "modup_store", s);
  HE_FOR_CLASSES(c->q_mask | (1u << c->p_cls),
                 (k_modup_store<LOGN, CLS><<<dim3(level + 1, level, count), T, 0, s>>>(dcoef, jobs1, dhat, level,
                                                                                       c->big_l, c->mods, c->tb())));
}

// ... then, per chunk of rotations: inner product with each key, ModDown.
// Rotation r of the chunk uses the lifted digits of ciphertext
// (job_base + r) / per_ct, dstride words apart; the fused form (u null)
// serves one ciphertext.
template <int LOGN>
void LHoisted<LOGN>::run(he_ctx* c, const KsJob* jobs, int m, int level, const u64* dhat, u64* u, u64* rc, hipStream_t s,
                         int job_base, int per_ct, size_t dstride, int part, int add_c0) {
  constexpr int T = NttGeom<LOGN>::T;
  constexpr int N = 1 << LOGN;
  if (u == nullptr) {
    // fused: the P row of each rotation's inner product to the coefficient
    // domain, then ModDown with the other rows computed where they are used
    {
      Prof pr(c, "hoist_p_intt", s);
      HE_FOR_CLASSES(1u << c->p_cls, (k_hoist_p_intt<LOGN, CLS><<<xcd_grid(2, m), T, 0, s>>>(
                                         dhat, jobs, m, level, c->big_l, rc, c->mods, c->tb())));
    }
    Prof pr(c, "hoist_drop", s);
    HE_FOR_CLASSES(c->q_mask, (k_hoist_drop<LOGN, CLS><<<xcd_grid(4 * level, m), modup_half_threads<LOGN>(), 0, s>>>(
                                  dhat, jobs, m, level, c->big_l, rc, c->d_inv, c->mods, c->tb())));
    return;
  }
  if (part != 2) {
    Prof pr(c, "ip_perm", s);
    k_ip_perm<LOGN><<<dim3(N / 256, level + 1, m), 256, 0, s>>>(dhat, jobs, u, level, c->big_l, c->mods, job_base,
                                                                 per_ct, dstride, add_c0);
  }
  if (part == 1) return;
  {  // u rows per polynomial: level + 1, P at row level (one P group)
    Prof pr(c, "intt_last", s);
    HE_FOR_CLASSES(1u << c->p_cls, (k_intt_last<LOGN, MODE_P, CLS><<<xcd_grid(2, m), T, 0, s>>>(
                                       jobs, m, u, level, 1, c->big_l, rc, c->mods, c->tb())));
  }
  LDrop<LOGN>::run(c, MODE_P, EPI_ROT, jobs, m, level, level + 1, u, rc, s);
}

template <int LOGN>
void LModDown<LOGN>::run(he_ctx* c, const KsJob* jobs, int count, int level, const u64* u, u64* rc, hipStream_t s) {
  constexpr int T = NttGeom<LOGN>::T;
  {
    Prof pr(c, "intt_last", s);
    HE_FOR_CLASSES(1u << c->p_cls, (k_intt_last<LOGN, MODE_P, CLS><<<xcd_grid(2, count), T, 0, s>>>(
                                       jobs, count, u, level, 1, c->big_l, rc, c->mods, c->tb())));
  }
  LDrop<LOGN>::run(c, MODE_P, EPI_STORE, jobs, count, level, level + 1, u, rc, s);
}

template <int LOGN>
void LTapHmaQp<LOGN>::run(he_ctx* c, const u64* x, const u64* u, const u64* filt, const u64* fp, u64* out, int level,
                          int pt_limbs, const TapMap& tm, int n_b, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  Prof pr(c, "tap_hma", s);
  const int n_ot = (tm.o_c + TAP_OT - 1) / TAP_OT;
  k_tap_hma_qp<LOGN><<<dim3(N / 64, level + 1, n_b * n_ot), 256, 0, s>>>(x, u, filt, fp, out, level, pt_limbs,
                                                                        c->big_l, tm, c->mods);
}

template <int LOGN>
void LTapHma<LOGN>::run(he_ctx* c, const u64* x, const u64* rot, const u64* filt, u64* out, int level, int pt_limbs,
                        const TapMap& tm, int n_b, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  Prof pr(c, "tap_hma", s);
  const int n_ot = (tm.o_c + TAP_OT - 1) / TAP_OT;
  k_tap_hma<LOGN><<<dim3(N / 64, level, n_b * n_ot), 256, 0, s>>>(x, rot, filt, out, level, pt_limbs, tm, c->mods);
}

}  // namespace he

#define HE_INSTANTIATE_LAUNCHERS(LOGN)    \
  namespace he {                          \
  template struct LNtt<LOGN>;             \
  template struct LKsCore<LOGN>;          \
  template struct LDrop<LOGN>;            \
  template struct LIntt1<LOGN>;           \
  template struct LDpHma<LOGN>;           \
  template struct LHmaPerm<LOGN>;         \
  template struct LKeygen<LOGN>;          \
  template struct LHoistUp<LOGN>;         \
  template struct LHoisted<LOGN>;         \
  template struct LTapHma<LOGN>;          \
  template struct LTapHmaQp<LOGN>;        \
  template struct LModDown<LOGN>;         \
  }
